// Launch sequence of the sine-transform preconditioner (one precision per
// build of this file: FL_T = float or double).
#include "fl_internal.hpp"

// Sine kernels are specialised per length (dst_lf): each specialisation holds
// only its own FFT; other lengths take the run-time plan (LF = 0).
template <typename T, int DPRO, int DEPI>
static fl_status launch_dst_rows(int lf, dim3 g, dim3 b, size_t sm, hipStream_t s, const Prob& pb, Iter it, int chk) {
  switch (lf) {
    case 2050: LAUNCH((k_dst_rows<T, DPRO, DEPI, 2050>), g, b, sm, s, pb, it, chk); break;
    case 1026: LAUNCH((k_dst_rows<T, DPRO, DEPI, 1026>), g, b, sm, s, pb, it, chk); break;
    case 770: LAUNCH((k_dst_rows<T, DPRO, DEPI, 770>), g, b, sm, s, pb, it, chk); break;
    case 258: LAUNCH((k_dst_rows<T, DPRO, DEPI, 258>), g, b, sm, s, pb, it, chk); break;
    case 130: LAUNCH((k_dst_rows<T, DPRO, DEPI, 130>), g, b, sm, s, pb, it, chk); break;
    case kRaderLF: LAUNCH((k_dst_rows<T, DPRO, DEPI, kRaderLF>), g, b, sm, s, pb, it, chk); break;
    case -512: LAUNCH((k_dst_rows<T, DPRO, DEPI, -512>), g, b, sm, s, pb, it, chk); break;
    case -256: LAUNCH((k_dst_rows<T, DPRO, DEPI, -256>), g, b, sm, s, pb, it, chk); break;
    case -1024: LAUNCH((k_dst_rows<T, DPRO, DEPI, -1024>), g, b, sm, s, pb, it, chk); break;
    default: LAUNCH((k_dst_rows<T, DPRO, DEPI, 0>), g, b, sm, s, pb, it, chk); break;
  }
  return FL_OK;
}

template <typename T, bool SCALE>
static fl_status launch_dst_cols(int lf, dim3 g, dim3 b, size_t sm, hipStream_t s, const Prob& pb, const DGeom& dg,
                                 int chk, int tplf = 0) {
  if (lf == 2050 && tplf == 128) {
    LAUNCH((k_dst_cols<T, SCALE, 2050, 128>), g, b, sm, s, pb, dg, chk);
    return FL_OK;
  }
  switch (lf) {
    case 2050: LAUNCH((k_dst_cols<T, SCALE, 2050>), g, b, sm, s, pb, dg, chk); break;
    case 1026: LAUNCH((k_dst_cols<T, SCALE, 1026>), g, b, sm, s, pb, dg, chk); break;
    case 770: LAUNCH((k_dst_cols<T, SCALE, 770>), g, b, sm, s, pb, dg, chk); break;
    case 258: LAUNCH((k_dst_cols<T, SCALE, 258>), g, b, sm, s, pb, dg, chk); break;
    case 130: LAUNCH((k_dst_cols<T, SCALE, 130>), g, b, sm, s, pb, dg, chk); break;
    case kRaderLF: LAUNCH((k_dst_cols<T, SCALE, kRaderLF>), g, b, sm, s, pb, dg, chk); break;
    case -512: LAUNCH((k_dst_cols<T, SCALE, -512>), g, b, sm, s, pb, dg, chk); break;
    case -256: LAUNCH((k_dst_cols<T, SCALE, -256>), g, b, sm, s, pb, dg, chk); break;
    case -1024: LAUNCH((k_dst_cols<T, SCALE, -1024>), g, b, sm, s, pb, dg, chk); break;
    default: LAUNCH((k_dst_cols<T, SCALE, 0>), g, b, sm, s, pb, dg, chk); break;
  }
  return FL_OK;
}

// ---------------------------------------------------------------------------
// preconditioner (p0 I + p1 pcs T)^{-1}
// ---------------------------------------------------------------------------
template <typename T, int DPRO, int DEPI> fl_status precond_seq(fl_op op, Prob pb, Iter it, int chk) {
  hipStream_t s = op->stream;
  const int d = op->d;
  long rows = rows_of(op, pb.nrhs);
  const long rlines = pb.ax[d - 1].dst_direct ? (rows + 1) / 2 : rows;  // FFT lines
  pb.ax[d - 1].dst.tpl = tune_tpl(pb.ax[d - 1].dst.tpl, pb.ax[d - 1].dst.L, rlines);
  const Axis& AL = pb.ax[d - 1];
  int nt = block_for(AL.dst.tpl), G = nt / AL.dst.tpl;
  size_t sm = (size_t)G * Line<T>::stride(AL.dst.L) * sizeof(cx<T>) * (AL.dst_direct ? 2 : 1);
  dim3 gr((rlines + G - 1) / G);
  if (d == 1) {
    return launch_dst_rows<T, DPRO, DEPI>(dst_lf(AL), gr, dim3(nt), sm, s, pb, it, chk);
  }
  Prob p1 = pb;
  p1.out = pb.T1;
  STCHK((launch_dst_rows<T, DPRO, DEPI_STORE>(dst_lf(AL), gr, dim3(nt), sm, s, p1, it, chk)));
  auto cols = [&](DGeom g, bool scale) -> fl_status {
    Prob pc = pb;
    Axis& A = pc.ax[g.axis];
    const int per = A.dst_direct ? 2 : 1;  // real lines per FFT line
    const int lf = dst_lf(A), tplf = (lf == 2050 && A.dcol_tplf == 128) ? 128 : 0;
    A.dst.tpl = tplf ? tplf : tune_tpl(A.dst.tpl, A.dst.L, g.gs * g.ngroup / per);
    int ntc = block_for(A.dst.tpl), Gf = ntc / A.dst.tpl, Gc = Gf * per;
    long grid = g.ngroup * ((g.gs + Gc - 1) / Gc);
    size_t smc = (size_t)Gf * Line<T>::stride(A.dst.L) * sizeof(cx<T>) * per;
    if (scale) return launch_dst_cols<T, true>(lf, dim3(grid), dim3(ntc), smc, s, pc, g, chk, tplf);
    return launch_dst_cols<T, false>(lf, dim3(grid), dim3(ntc), smc, s, pc, g, chk, tplf);
  };
  const long nr = pb.nrhs;
  if (d == 2) {
    const long n0 = op->n[0], n1 = op->n[1];
    STCHK(cols(DGeom{0, n1, nr, n1, n0 * n1}, true));
  } else {
    const long n0 = op->n[0], n1 = op->n[1], n2 = op->n[2];
    DGeom g1 = {1, n2, nr * n0, n2, n1 * n2};
    DGeom g0 = {0, n1 * n2, nr, n1 * n2, n0 * n1 * n2};
    STCHK(cols(g1, false));
    STCHK(cols(g0, true));
    STCHK(cols(g1, false));
  }
  Prob p3 = pb;
  p3.in = pb.T1;
  return launch_dst_rows<T, DPRO_PLAIN, DEPI>(dst_lf(AL), gr, dim3(nt), sm, s, p3, it, chk);
}


template fl_status precond_seq<FL_T, DPRO_PLAIN, DEPI_FINAL>(fl_op, Prob, Iter, int);
template fl_status precond_seq<FL_T, DPRO_PLAIN, DEPI_Z>(fl_op, Prob, Iter, int);
template fl_status precond_seq<FL_T, DPRO_UPD, DEPI_Z>(fl_op, Prob, Iter, int);
template fl_status precond_seq<FL_T, DPRO_UPD, DEPI_FINAL>(fl_op, Prob, Iter, int);

// One pass of the preconditioner on the op's workspace, launched with the same
// lane tuning as precond_seq: 3 first sine pass (in -> T1), 4 scaled column
// pass on T1, 5 last sine pass (T1 -> out).
template <typename T> fl_status launch_precond_pass(fl_op op, Prob pb, int pass) {
  hipStream_t s = op->stream;
  const int d = op->d;
  Iter it = {0, 0};
  if (d == 1) return fail(FL_E_UNSUPPORTED, "single passes are defined for d >= 2");
  long rows = rows_of(op, 1);
  if (pass == 3 || pass == 5) {
    const long rlines = pb.ax[d - 1].dst_direct ? (rows + 1) / 2 : rows;
    pb.ax[d - 1].dst.tpl = tune_tpl(pb.ax[d - 1].dst.tpl, pb.ax[d - 1].dst.L, rlines);
    const Axis& AL = pb.ax[d - 1];
    int nt = block_for(AL.dst.tpl), G = nt / AL.dst.tpl;
    size_t sm = (size_t)G * Line<T>::stride(AL.dst.L) * sizeof(cx<T>) * (AL.dst_direct ? 2 : 1);
    Prob p1 = pb;
    if (pass == 3) {
      p1.out = pb.T1;
      STCHK((launch_dst_rows<T, DPRO_PLAIN, DEPI_STORE>(dst_lf(AL), dim3((rlines + G - 1) / G), dim3(nt), sm, s, p1,
                                                        it, 0)));
    } else {
      p1.in = pb.T1;
      STCHK((launch_dst_rows<T, DPRO_PLAIN, DEPI_FINAL>(dst_lf(AL), dim3((rlines + G - 1) / G), dim3(nt), sm, s, p1,
                                                        it, 0)));
    }
    return FL_OK;
  }
  if (pass == 4) {
    DGeom g;
    if (d == 2) g = DGeom{0, (long)op->n[1], 1, (long)op->n[1], (long)op->n[0] * op->n[1]};
    else {
      long n12 = (long)op->n[1] * op->n[2];
      g = DGeom{0, n12, 1, n12, (long)op->n[0] * n12};
    }
    const int per = pb.ax[0].dst_direct ? 2 : 1;
    const int lf = dst_lf(pb.ax[0]), tplf = (lf == 2050 && pb.ax[0].dcol_tplf == 128) ? 128 : 0;
    pb.ax[0].dst.tpl = tplf ? tplf : tune_tpl(pb.ax[0].dst.tpl, pb.ax[0].dst.L, g.gs * g.ngroup / per);
    const Axis& A = pb.ax[0];
    int nt = block_for(A.dst.tpl), Gf = nt / A.dst.tpl, G = Gf * per;
    long grid = g.ngroup * ((g.gs + G - 1) / G);
    STCHK((launch_dst_cols<T, true>(lf, dim3(grid), dim3(nt),
                                    (size_t)Gf * Line<T>::stride(A.dst.L) * sizeof(cx<T>) * per, s, pb, g, 0, tplf)));
    return FL_OK;
  }
  return fail(FL_E_INVALID, "preconditioner pass must be 3, 4 or 5");
}
template fl_status launch_precond_pass<FL_T>(fl_op, Prob, int);

