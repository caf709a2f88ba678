// Launch sequence of the operator application (one precision per build of
// this file: FL_T = float or double).
#include "fl_internal.hpp"

// The symbol column pass: lengths 1024 and 2048 (grids of 512 and 1024) can run
// a specialised kernel with fewer lanes per column (64 or 128), i.e. 4 or 2
// adjacent columns per block; the autotuner sets A.col_tplf (0 = the run-time
// plan, which every other length follows).
template <typename T> static fl_status launch_col_conv(const Prob& pc, const ColGeom& cg, Iter it, int chk,
                                                        hipStream_t s) {
  const Axis& A = pc.ax[cg.axis];
  int lf = 0, tplf = 0;
  if (A.fft.fixed && (A.P == 2048 || A.P == 1024) && (A.col_tplf == 64 || A.col_tplf == 128 || A.col_tplf == 256)) {
    lf = A.P;
    tplf = A.col_tplf;
    // FP64 at 2048 with 64 lanes would need 4 x 37 KB of LDS: keep 128 or more
    if (lf == 2048 && sizeof(T) == 8 && tplf == 64) tplf = 128;
    if (lf == 1024) tplf = 64;
  } else if (fft_lf(A) == 8192 || fft_lf(A) == 512 || fft_lf(A) == 256) {
    lf = A.P;  // compile-time lanes
    tplf = lf == 512 ? col_tpl<T>(A, pc.d) : c_fixed_tpl(lf);
  }
  Prob pl = pc;
  if (!lf) pl.ax[cg.axis].fft.tpl = tune_tpl(A.fft.tpl, A.P, cg.gs * cg.ngroup);
  const int tpl = lf ? tplf : pl.ax[cg.axis].fft.tpl;
  const int nt = block_for(tpl), G = nt / tpl;
  const long grid = cg.ngroup * ((cg.gs + G - 1) / G);
  const size_t sm = (size_t)G * Line<T>::stride(A.P) * sizeof(cx<T>);
  if (lf == 8192)
    LAUNCH((k_colpass<T, COL_CONV, 8192, c_fixed_tpl(8192)>), dim3(grid), dim3(nt), sm, s, pl, cg, it, chk);
  else if (lf == 2048 && tplf == 256)
    LAUNCH((k_colpass<T, COL_CONV, 2048, 256>), dim3(grid), dim3(nt), sm, s, pl, cg, it, chk);
  else if (lf == 2048 && tplf == 64)
    LAUNCH((k_colpass<T, COL_CONV, 2048, 64>), dim3(grid), dim3(nt), sm, s, pl, cg, it, chk);
  else if (lf == 2048)
    LAUNCH((k_colpass<T, COL_CONV, 2048, 128>), dim3(grid), dim3(nt), sm, s, pl, cg, it, chk);
  else if (lf == 1024)
    LAUNCH((k_colpass<T, COL_CONV, 1024, 64>), dim3(grid), dim3(nt), sm, s, pl, cg, it, chk);
  else if (lf == 512)
    if (tplf == kCol3DLanes512)
      LAUNCH((k_colpass<T, COL_CONV, 512, kCol3DLanes512>), dim3(grid), dim3(nt), sm, s, pl, cg, it, chk);
    else
      LAUNCH((k_colpass<T, COL_CONV, 512, c_fixed_tpl(512)>), dim3(grid), dim3(nt), sm, s, pl, cg, it, chk);
  else if (lf == 256)
    LAUNCH((k_colpass<T, COL_CONV, 256, c_fixed_tpl(256)>), dim3(grid), dim3(nt), sm, s, pl, cg, it, chk);
  else
    LAUNCH((k_colpass<T, COL_CONV>), dim3(grid), dim3(nt), sm, s, pl, cg, it, chk);
  return FL_OK;
}

// Row passes with the length specialisation of the last axis (fft_lf).
template <typename T, int PRO>
static fl_status launch_rowfwd(int lf, dim3 g, dim3 b, size_t sm, hipStream_t s, const Prob& pb, Iter it) {
  if (lf == 8192) {  // application-only grids: the plain application
    if constexpr (PRO == PRO_PLAIN) {
      LAUNCH((k_rowfwd<T, PRO, 8192>), g, b, sm, s, pb, it);
      return FL_OK;
    }
    return fail(FL_E_UNSUPPORTED, "lines of 8192 points support the plain application only");
  }
  switch (lf) {
    case 2048: LAUNCH((k_rowfwd<T, PRO, 2048>), g, b, sm, s, pb, it); break;
    case 1024: LAUNCH((k_rowfwd<T, PRO, 1024>), g, b, sm, s, pb, it); break;
    case 512: LAUNCH((k_rowfwd<T, PRO, 512>), g, b, sm, s, pb, it); break;
    case 256: LAUNCH((k_rowfwd<T, PRO, 256>), g, b, sm, s, pb, it); break;
    default: LAUNCH((k_rowfwd<T, PRO>), g, b, sm, s, pb, it); break;
  }
  return FL_OK;
}
template <typename T, int EPI>
static fl_status launch_rowinv(int lf, dim3 g, dim3 b, size_t sm, hipStream_t s, const Prob& pb, Iter it, int chk) {
  if (lf == 8192) {
    if constexpr (EPI == EPI_PLAIN) {
      LAUNCH((k_rowinv<T, EPI, 8192>), g, b, sm, s, pb, it, chk);
      return FL_OK;
    }
    return fail(FL_E_UNSUPPORTED, "lines of 8192 points support the plain application only");
  }
  switch (lf) {
    case 2048: LAUNCH((k_rowinv<T, EPI, 2048>), g, b, sm, s, pb, it, chk); break;
    case 1024: LAUNCH((k_rowinv<T, EPI, 1024>), g, b, sm, s, pb, it, chk); break;
    case 512: LAUNCH((k_rowinv<T, EPI, 512>), g, b, sm, s, pb, it, chk); break;
    case 256: LAUNCH((k_rowinv<T, EPI, 256>), g, b, sm, s, pb, it, chk); break;
    default: LAUNCH((k_rowinv<T, EPI>), g, b, sm, s, pb, it, chk); break;
  }
  return FL_OK;
}

// ---------------------------------------------------------------------------
// operator application (M or shift0 I + shift1 M)
// ---------------------------------------------------------------------------
template <typename T, int PRO, int EPI> fl_status apply_seq(fl_op op, const Prob& pb, Iter it, int chk) {
  hipStream_t s = op->stream;
  const int d = op->d;
  if (d == 1) {
    Prob p1 = pb;
    long pairs = (pb.nrhs + 1) / 2;
    p1.ax[0].fft.tpl = tune_tpl(pb.ax[0].fft.tpl, pb.ax[0].P, pairs);
    const Axis& A = p1.ax[0];
    int nt = block_for(A.fft.tpl), G = nt / A.fft.tpl;
    LAUNCH(k_conv1d<T, PRO, EPI>, dim3((pairs + G - 1) / G), dim3(nt), (size_t)G * Line<T>::stride(A.P) * sizeof(cx<T>), s, p1, it);
    return FL_OK;
  }
  long rows = rows_of(op, pb.nrhs), pairs = (rows + 1) / 2;
  Prob pr = pb;  // row passes: lanes per line tuned to the number of row pairs
  pr.ax[d - 1].fft.tpl = tune_tpl(pb.ax[d - 1].fft.tpl, pb.ax[d - 1].P, pairs);
  const Axis& AL = pr.ax[d - 1];
  {
    int nt = block_for(AL.fft.tpl), G = nt / AL.fft.tpl;
    STCHK((launch_rowfwd<T, PRO>(fft_lf(AL), dim3((pairs + G - 1) / G), dim3(nt),
                                  (size_t)G * Line<T>::stride(AL.P) * sizeof(cx<T>), s, pr, it)));
  }
  auto col = [&](ColGeom cg, int mode) -> fl_status {
    Prob pc = pb;
    Axis& A = pc.ax[cg.axis];
    if (mode == COL_CONV) return launch_col_conv<T>(pc, cg, it, chk, s);
    A.fft.tpl = tune_tpl(A.fft.tpl, A.P, cg.gs * cg.ngroup);
    const int lf = fft_lf(A);
    const int tpl = lf == 512 ? col_tpl<T>(A, d) : A.fft.tpl;
    int nt = block_for(tpl), G = nt / tpl;
    long grid = cg.ngroup * ((cg.gs + G - 1) / G);
    size_t sm = (size_t)G * Line<T>::stride(A.P) * sizeof(cx<T>);
    if (mode == COL_FWD) {
      if (lf == 512 && tpl == kCol3DLanes512)
        LAUNCH((k_colpass<T, COL_FWD, 512, kCol3DLanes512>), dim3(grid), dim3(nt), sm, s, pc, cg, it, chk);
      else if (lf == 512) LAUNCH((k_colpass<T, COL_FWD, 512, c_fixed_tpl(512)>), dim3(grid), dim3(nt), sm, s, pc, cg, it, chk);
      else if (lf == 256) LAUNCH((k_colpass<T, COL_FWD, 256, c_fixed_tpl(256)>), dim3(grid), dim3(nt), sm, s, pc, cg, it, chk);
      else LAUNCH(k_colpass<T, COL_FWD>, dim3(grid), dim3(nt), sm, s, pc, cg, it, chk);
    }
    if (mode == COL_INV) {
      if (lf == 512 && tpl == kCol3DLanes512)
        LAUNCH((k_colpass<T, COL_INV, 512, kCol3DLanes512>), dim3(grid), dim3(nt), sm, s, pc, cg, it, chk);
      else if (lf == 512) LAUNCH((k_colpass<T, COL_INV, 512, c_fixed_tpl(512)>), dim3(grid), dim3(nt), sm, s, pc, cg, it, chk);
      else if (lf == 256) LAUNCH((k_colpass<T, COL_INV, 256, c_fixed_tpl(256)>), dim3(grid), dim3(nt), sm, s, pc, cg, it, chk);
      else LAUNCH(k_colpass<T, COL_INV>, dim3(grid), dim3(nt), sm, s, pc, cg, it, chk);
    }
    return FL_OK;
  };
  const long nr = pb.nrhs;
  if (d == 2) {
    const long H1 = op->H[1], n0 = op->n[0];
    ColGeom cg = {0, (int)n0, (int)n0, H1, nr, H1, n0 * H1, H1, n0 * H1, 1, 1};
    STCHK(col(cg, COL_CONV));
  } else {
    const long n0 = op->n[0], n1 = op->n[1], P1 = op->P[1], H2 = op->H[2];
    ColGeom f = {1, (int)n1, (int)P1, H2, nr * n0, H2, n1 * H2, H2, P1 * H2, 1, 2};
    ColGeom c = {0, (int)n0, (int)n0, P1 * H2, nr, P1 * H2, n0 * P1 * H2, P1 * H2, n0 * P1 * H2, 2, 2};
    ColGeom i = {1, (int)P1, (int)n1, H2, nr * n0, H2, P1 * H2, H2, n1 * H2, 2, 1};
    STCHK(col(f, COL_FWD));
    STCHK(col(c, COL_CONV));
    STCHK(col(i, COL_INV));
  }
  {
    int nt = block_for(AL.fft.tpl), G = nt / AL.fft.tpl;
    STCHK((launch_rowinv<T, EPI>(fft_lf(AL), dim3((pairs + G - 1) / G), dim3(nt),
                                  (size_t)G * Line<T>::stride(AL.P) * sizeof(cx<T>), s, pr, it, chk)));
  }
  return FL_OK;
}


template fl_status apply_seq<FL_T, PRO_PLAIN, EPI_PLAIN>(fl_op, const Prob&, Iter, int);
template fl_status apply_seq<FL_T, PRO_PLAIN, EPI_RESID>(fl_op, const Prob&, Iter, int);
template fl_status apply_seq<FL_T, PRO_PUPD, EPI_PQ>(fl_op, const Prob&, Iter, int);
template fl_status apply_seq<FL_T, PRO_PLAIN, EPI_PQ>(fl_op, const Prob&, Iter, int);

// One pass of the application on the op's workspace (inputs pb.in, output
// pb.out, work W1/W2), launched with the same lane tuning as apply_seq.
template <typename T> fl_status launch_apply_pass(fl_op op, Prob pb, int pass) {
  hipStream_t s = op->stream;
  const int d = op->d;
  long rows = rows_of(op, 1), pairs = (rows + 1) / 2;
  Iter it = {0, 0};
  if (d == 1) return fail(FL_E_UNSUPPORTED, "single passes are defined for d >= 2");
  if (pass == 0 || pass == 2) {
    pb.ax[d - 1].fft.tpl = tune_tpl(pb.ax[d - 1].fft.tpl, pb.ax[d - 1].P, pairs);
    const Axis& AL = pb.ax[d - 1];
    int nt = block_for(AL.fft.tpl), G = nt / AL.fft.tpl;
    size_t sm = (size_t)G * Line<T>::stride(AL.P) * sizeof(cx<T>);
    if (pass == 0) STCHK((launch_rowfwd<T, PRO_PLAIN>(fft_lf(AL), dim3((pairs + G - 1) / G), dim3(nt), sm, s, pb, it)));
    else STCHK((launch_rowinv<T, EPI_PLAIN>(fft_lf(AL), dim3((pairs + G - 1) / G), dim3(nt), sm, s, pb, it, 0)));
    return FL_OK;
  }
  if (pass == 1) {
    ColGeom cg;
    if (d == 2) {
      const long H1 = op->H[1], n0 = op->n[0];
      cg = {0, (int)n0, (int)n0, H1, 1, H1, n0 * H1, H1, n0 * H1, 1, 1};
    } else {
      const long n0 = op->n[0], P1 = op->P[1], H2 = op->H[2];
      cg = {0, (int)n0, (int)n0, P1 * H2, 1, P1 * H2, n0 * P1 * H2, P1 * H2, n0 * P1 * H2, 2, 2};
    }
    return launch_col_conv<T>(pb, cg, it, 0, s);
  }
  return fail(FL_E_INVALID, "apply pass must be 0, 1 or 2");
}
template fl_status launch_apply_pass<FL_T>(fl_op, Prob, int);

