// Batched Krylov driver: many problems (uneven grids, different alpha, or many
// right-hand sides of one operator) advanced together.  Every kernel of an
// iteration is a single launch over all problems (blockIdx.y = problem, each
// problem with its own block count); a problem that has converged leaves its
// blocks idle.  The iteration is captured once as a hipGraph and replayed;
// the host polls one contiguous array of per-problem scalars.
//
// This file is compiled once per precision (FL_T) for the launch sequences,
// and once with FL_BATCH_HOST for the C entry points.
#include "fl_internal.hpp"
#include "fl_batch.hpp"
#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>

// ---------------------------------------------------------------------------
// per-precision launch sequences
// ---------------------------------------------------------------------------
#ifndef FL_BATCH_HOST

template <typename T> static size_t lds_fft(int L, int G) { return (size_t)G * Line<T>::stride(L) * sizeof(cx<T>); }

template <typename T> fl_status bt_setup(BatchT& bt, const BatchDesc& B, const std::vector<Prob>& base) {
  const int np = B.np, d = B.d;
  bt.np = np;
  bt.d = d;
  bt.elem = sizeof(T);
  // per problem (problem order): block counts, geometry, LDS and the length
  // specialisation of every pass
  struct One {
    int nb_rowfwd, nb_dstrow, nb_upd, nb_col[3], nb_dcol[2];
    ColGeom cg[3];
    DGeom dg[2];
    long N;
    size_t sm_row, sm_dstrow, sm_col[3], sm_dcol[2];
    int key[6];  // lf_rowfft, lf_col[0..2], lf_row, lf_dcol[0] (lf_dcol[1] = lf_dcol[0] in 3D)
    int lf_dcol1;
  };
  std::vector<One> pr(np);
  for (int p = 0; p < np; ++p) {
    One& o = pr[p];
    memset(&o, 0, sizeof(One));
    const Prob& pb = base[p];
    const int* n = B.n[p].data();
    long rows = 1, N = 1;
    for (int a = 0; a < d - 1; ++a) rows *= n[a];
    for (int a = 0; a < d; ++a) N *= n[a];
    o.N = N;
    o.nb_upd = (int)std::min<long>(2048, (N + 255) / 256);
    const Axis& AL = pb.ax[d - 1];
    const long pairs = (rows + 1) / 2;
    {
      const int G = 256 / AL.fft.tpl;
      o.nb_rowfwd = (int)((pairs + G - 1) / G);
      o.sm_row = lds_fft<T>(AL.P, G);
    }
    if (d == 2) {
      const long H1 = pb.ax[1].H, n0 = n[0];
      o.cg[0] = ColGeom{0, (int)n0, (int)n0, H1, 1, H1, n0 * H1, H1, n0 * H1, 1, 1};
    } else if (d == 3) {
      const long n0 = n[0], n1 = n[1], P1 = pb.ax[1].P, H2 = pb.ax[2].H;
      o.cg[0] = ColGeom{1, (int)n1, (int)P1, H2, n0, H2, n1 * H2, H2, P1 * H2, 1, 2};
      o.cg[1] = ColGeom{0, (int)n0, (int)n0, P1 * H2, 1, P1 * H2, n0 * P1 * H2, P1 * H2, n0 * P1 * H2, 2, 2};
      o.cg[2] = ColGeom{1, (int)P1, (int)n1, H2, n0, H2, P1 * H2, H2, n1 * H2, 2, 1};
    }
    o.key[0] = fft_lf(AL);
    const int ncol = d == 3 ? 3 : (d == 2 ? 1 : 0);
    for (int r = 0; r < ncol; ++r) {
      const ColGeom& c = o.cg[r];
      const Axis& A = pb.ax[c.axis];
      const int lfa = fft_lf(A);
      o.key[1 + r] = (lfa == 1024 || lfa == 512 || lfa == 256) ? lfa : 0;
      const int G = 256 / A.fft.tpl;  // batched launches keep the plan's lanes (measured faster there)
      o.nb_col[r] = (int)(c.ngroup * ((c.gs + G - 1) / G));
      o.sm_col[r] = lds_fft<T>(A.P, G);
    }
    // sine transforms
    {
      const long rl = AL.dst_direct ? (rows + 1) / 2 : rows;
      const int G = 256 / AL.dst.tpl;
      o.nb_dstrow = (int)((rl + G - 1) / G);
      o.sm_dstrow = lds_fft<T>(AL.dst.L, G) * (AL.dst_direct ? 2 : 1);
    }
    if (d == 2) {
      o.dg[0] = DGeom{0, (long)n[1], 1, (long)n[1], (long)n[0] * n[1]};
    } else if (d == 3) {
      o.dg[0] = DGeom{1, (long)n[2], (long)n[0], (long)n[2], (long)n[1] * n[2]};
      o.dg[1] = DGeom{0, (long)n[1] * n[2], 1, (long)n[1] * n[2], (long)n[0] * n[1] * n[2]};
    }
    o.key[4] = dst_lf(AL);
    const int ndc = d == 3 ? 2 : (d == 2 ? 1 : 0);
    for (int r = 0; r < ndc; ++r) {
      const DGeom& g = o.dg[r];
      const Axis& A = pb.ax[g.axis];
      if (r == 0) o.key[5] = dst_lf(A);
      else o.lf_dcol1 = dst_lf(A);
      const int per = A.dst_direct ? 2 : 1;
      const int Gf = 256 / A.dst.tpl, G = Gf * per;
      o.nb_dcol[r] = (int)(g.ngroup * ((g.gs + G - 1) / G));
      o.sm_dcol[r] = lds_fft<T>(A.dst.L, Gf) * per;
    }
  }
  // group order: problems with equal specialisations next to each other
  // (stable, so a uniform batch keeps problem order)
  auto key_of = [&](int p) {
    std::array<int, 7> k;
    for (int i = 0; i < 6; ++i) k[i] = pr[p].key[i];
    k[6] = pr[p].lf_dcol1;
    return k;
  };
  bt.order.resize(np);
  for (int p = 0; p < np; ++p) bt.order[p] = p;
  std::stable_sort(bt.order.begin(), bt.order.end(), [&](int a, int b) { return key_of(a) < key_of(b); });
  auto mk = [&](std::vector<int>& v) { v.assign(np, 0); };
  mk(bt.nb_rowfwd); mk(bt.nb_rowinv); mk(bt.nb_dstrow); mk(bt.nb_upd);
  for (auto& v : bt.nb_col) mk(v);
  for (auto& v : bt.nb_dcol) mk(v);
  bt.cg.assign(3 * np, ColGeom{});
  bt.dg.assign(2 * np, DGeom{});
  bt.N.assign(np, 0);
  bt.groups.clear();
  for (int q = 0; q < np; ++q) {
    const int p = bt.order[q];
    const One& o = pr[p];
    bt.nb_rowfwd[q] = bt.nb_rowinv[q] = o.nb_rowfwd;
    bt.nb_dstrow[q] = o.nb_dstrow;
    bt.nb_upd[q] = o.nb_upd;
    for (int r = 0; r < 3; ++r) {
      bt.nb_col[r][q] = o.nb_col[r];
      bt.cg[r * np + q] = o.cg[r];
    }
    for (int r = 0; r < 2; ++r) {
      bt.nb_dcol[r][q] = o.nb_dcol[r];
      bt.dg[r * np + q] = o.dg[r];
    }
    bt.N[q] = o.N;
    if (q == 0 || key_of(p) != key_of(bt.order[q - 1])) {
      BatchGroup g;
      g.g0 = q;
      g.lf_rowfft = o.key[0];
      for (int r = 0; r < 3; ++r) g.lf_col[r] = o.key[1 + r];
      g.lf_row = o.key[4];
      g.lf_dcol[0] = o.key[5];
      g.lf_dcol[1] = o.lf_dcol1;
      bt.groups.push_back(g);
    }
    BatchGroup& g = bt.groups.back();
    ++g.gn;
    g.nb_rowfwd = std::max(g.nb_rowfwd, o.nb_rowfwd);
    g.nb_rowinv = g.nb_rowfwd;
    g.nb_dstrow = std::max(g.nb_dstrow, o.nb_dstrow);
    g.sm_row = std::max(g.sm_row, o.sm_row);
    g.sm_dstrow = std::max(g.sm_dstrow, o.sm_dstrow);
    for (int r = 0; r < 3; ++r) {
      g.nb_col[r] = std::max(g.nb_col[r], o.nb_col[r]);
      g.sm_col[r] = std::max(g.sm_col[r], o.sm_col[r]);
    }
    for (int r = 0; r < 2; ++r) {
      g.nb_dcol[r] = std::max(g.nb_dcol[r], o.nb_dcol[r]);
      g.sm_dcol[r] = std::max(g.sm_dcol[r], o.sm_dcol[r]);
    }
  }
  return FL_OK;
}

static int vmax(const std::vector<int>& v) {
  int m = 0;
  for (int x : v) m = std::max(m, x);
  return m;
}

// Batched operator application with prologue PRO / epilogue EPI over the Prob
// array `pbs` (device, group order): one launch per group and pass.
template <typename T, int PRO, int EPI> fl_status bt_apply(BatchT& bt, const Prob* pbs, Iter it, int chk,
                                                          hipStream_t s) {
  const int np = bt.np, d = bt.d;
  for (const BatchGroup& G : bt.groups) {
    const Prob* pg = pbs + G.g0;
    if (d == 1) {
      LAUNCH(k_conv1d_b<T, PRO, EPI>, dim3(G.nb_rowfwd, G.gn), dim3(256), G.sm_row, s, pg, it,
             (const int*)bt.d_nb_rowfwd + G.g0);
      continue;
    }
    const int* nbf = (const int*)bt.d_nb_rowfwd + G.g0;
    const dim3 gf(G.nb_rowfwd, G.gn);
    switch (G.lf_rowfft) {
      case 2048: LAUNCH((k_rowfwd_b<T, PRO, 2048>), gf, dim3(256), G.sm_row, s, pg, it, nbf); break;
      case 1024: LAUNCH((k_rowfwd_b<T, PRO, 1024>), gf, dim3(256), G.sm_row, s, pg, it, nbf); break;
      case 512: LAUNCH((k_rowfwd_b<T, PRO, 512>), gf, dim3(256), G.sm_row, s, pg, it, nbf); break;
      case 256: LAUNCH((k_rowfwd_b<T, PRO, 256>), gf, dim3(256), G.sm_row, s, pg, it, nbf); break;
      default: LAUNCH((k_rowfwd_b<T, PRO>), gf, dim3(256), G.sm_row, s, pg, it, nbf); break;
    }
  }
  auto col = [&](const BatchGroup& G, int r, int mode) -> fl_status {
    const Prob* pg = pbs + G.g0;
    // grid width a multiple of 8, so that the XCD-aware tile mapping holds
    // for every problem (blocks beyond a problem's count exit)
    const dim3 g((G.nb_col[r] + 7) & ~7, G.gn);
    const ColGeom* cg = (const ColGeom*)bt.d_cg + r * np + G.g0;
    const int* nb = (const int*)bt.d_nb_col[r] + G.g0;
    const size_t sm = G.sm_col[r];
#define FL_COLB(M)                                                                                   \
  switch (G.lf_col[r]) {                                                                             \
    case 1024: LAUNCH((k_colpass_b<T, M, 1024>), g, dim3(256), sm, s, pg, cg, it, chk, nb); break;  \
    case 512: LAUNCH((k_colpass_b<T, M, 512>), g, dim3(256), sm, s, pg, cg, it, chk, nb); break;    \
    case 256: LAUNCH((k_colpass_b<T, M, 256>), g, dim3(256), sm, s, pg, cg, it, chk, nb); break;    \
    default: LAUNCH((k_colpass_b<T, M>), g, dim3(256), sm, s, pg, cg, it, chk, nb); break;          \
  }
    if (mode == COL_FWD) { FL_COLB(COL_FWD) }
    else if (mode == COL_CONV) { FL_COLB(COL_CONV) }
    else { FL_COLB(COL_INV) }
#undef FL_COLB
    return FL_OK;
  };
  if (d == 1) return FL_OK;
  for (const BatchGroup& G : bt.groups) {
    if (d == 2) {
      STCHK(col(G, 0, COL_CONV));
    } else {
      STCHK(col(G, 0, COL_FWD));
      STCHK(col(G, 1, COL_CONV));
      STCHK(col(G, 2, COL_INV));
    }
  }
  for (const BatchGroup& G : bt.groups) {
    const Prob* pg = pbs + G.g0;
    const int* nbi = (const int*)bt.d_nb_rowinv + G.g0;
    const dim3 gi(G.nb_rowinv, G.gn);
    switch (G.lf_rowfft) {
      case 2048: LAUNCH((k_rowinv_b<T, EPI, 2048>), gi, dim3(256), G.sm_row, s, pg, it, chk, nbi); break;
      case 1024: LAUNCH((k_rowinv_b<T, EPI, 1024>), gi, dim3(256), G.sm_row, s, pg, it, chk, nbi); break;
      case 512: LAUNCH((k_rowinv_b<T, EPI, 512>), gi, dim3(256), G.sm_row, s, pg, it, chk, nbi); break;
      case 256: LAUNCH((k_rowinv_b<T, EPI, 256>), gi, dim3(256), G.sm_row, s, pg, it, chk, nbi); break;
      default: LAUNCH((k_rowinv_b<T, EPI>), gi, dim3(256), G.sm_row, s, pg, it, chk, nbi); break;
    }
  }
  return FL_OK;
}

// Batched preconditioner.  pfirst: Prob array of the first pass (reads `in`,
// writes `out` = T1); plast: Prob array of the last pass (reads `in` = T1).
// Sine-kernel launches with the length specialisation of each group.
template <typename T, int DPRO, int DEPI>
static fl_status bt_dst_rows(int lf, dim3 g, size_t sm, hipStream_t s, const Prob* pbs, Iter it, int chk, const int* nb) {
  switch (lf) {
    case 2050: LAUNCH((k_dst_rows_b<T, DPRO, DEPI, 2050>), g, dim3(256), sm, s, pbs, it, chk, nb); break;
    case 1026: LAUNCH((k_dst_rows_b<T, DPRO, DEPI, 1026>), g, dim3(256), sm, s, pbs, it, chk, nb); break;
    case 770: LAUNCH((k_dst_rows_b<T, DPRO, DEPI, 770>), g, dim3(256), sm, s, pbs, it, chk, nb); break;
    case 258: LAUNCH((k_dst_rows_b<T, DPRO, DEPI, 258>), g, dim3(256), sm, s, pbs, it, chk, nb); break;
    case 130: LAUNCH((k_dst_rows_b<T, DPRO, DEPI, 130>), g, dim3(256), sm, s, pbs, it, chk, nb); break;
    case kRaderLF: LAUNCH((k_dst_rows_b<T, DPRO, DEPI, kRaderLF>), g, dim3(256), sm, s, pbs, it, chk, nb); break;
    case -512: LAUNCH((k_dst_rows_b<T, DPRO, DEPI, -512>), g, dim3(256), sm, s, pbs, it, chk, nb); break;
    case -256: LAUNCH((k_dst_rows_b<T, DPRO, DEPI, -256>), g, dim3(256), sm, s, pbs, it, chk, nb); break;
    case -1024: LAUNCH((k_dst_rows_b<T, DPRO, DEPI, -1024>), g, dim3(256), sm, s, pbs, it, chk, nb); break;
    default: LAUNCH((k_dst_rows_b<T, DPRO, DEPI>), g, dim3(256), sm, s, pbs, it, chk, nb); break;
  }
  return FL_OK;
}
template <typename T, bool SCALE>
static fl_status bt_dst_cols(int lf, dim3 g, size_t sm, hipStream_t s, const Prob* pbs, const DGeom* dgs, int chk,
                        const int* nb) {
  switch (lf) {
    case 2050: LAUNCH((k_dst_cols_b<T, SCALE, 2050>), g, dim3(256), sm, s, pbs, dgs, chk, nb); break;
    case 1026: LAUNCH((k_dst_cols_b<T, SCALE, 1026>), g, dim3(256), sm, s, pbs, dgs, chk, nb); break;
    case 770: LAUNCH((k_dst_cols_b<T, SCALE, 770>), g, dim3(256), sm, s, pbs, dgs, chk, nb); break;
    case 258: LAUNCH((k_dst_cols_b<T, SCALE, 258>), g, dim3(256), sm, s, pbs, dgs, chk, nb); break;
    case 130: LAUNCH((k_dst_cols_b<T, SCALE, 130>), g, dim3(256), sm, s, pbs, dgs, chk, nb); break;
    case kRaderLF: LAUNCH((k_dst_cols_b<T, SCALE, kRaderLF>), g, dim3(256), sm, s, pbs, dgs, chk, nb); break;
    case -512: LAUNCH((k_dst_cols_b<T, SCALE, -512>), g, dim3(256), sm, s, pbs, dgs, chk, nb); break;
    case -256: LAUNCH((k_dst_cols_b<T, SCALE, -256>), g, dim3(256), sm, s, pbs, dgs, chk, nb); break;
    case -1024: LAUNCH((k_dst_cols_b<T, SCALE, -1024>), g, dim3(256), sm, s, pbs, dgs, chk, nb); break;
    default: LAUNCH((k_dst_cols_b<T, SCALE>), g, dim3(256), sm, s, pbs, dgs, chk, nb); break;
  }
  return FL_OK;
}

template <typename T, int DPRO, int DEPI> fl_status bt_precond(BatchT& bt, const Prob* pfirst, const Prob* plast,
                                                              Iter it, int chk, hipStream_t s) {
  const int np = bt.np, d = bt.d;
  const DGeom* dg = (const DGeom*)bt.d_dg;
  if (d == 1) {
    for (const BatchGroup& G : bt.groups)
      STCHK((bt_dst_rows<T, DPRO, DEPI>(G.lf_row, dim3(G.nb_dstrow, G.gn), G.sm_dstrow, s, pfirst + G.g0, it, chk,
                                         (const int*)bt.d_nb_dstrow + G.g0)));
    return FL_OK;
  }
  for (const BatchGroup& G : bt.groups)
    STCHK((bt_dst_rows<T, DPRO, DEPI_STORE>(G.lf_row, dim3(G.nb_dstrow, G.gn), G.sm_dstrow, s, pfirst + G.g0, it,
                                             chk, (const int*)bt.d_nb_dstrow + G.g0)));
  auto cols = [&](const BatchGroup& G, int r, bool scale) -> fl_status {
    const dim3 g((G.nb_dcol[r] + 7) & ~7, G.gn);
    const int* nb = (const int*)bt.d_nb_dcol[r] + G.g0;
    const DGeom* dgr = dg + r * np + G.g0;
    if (scale) return bt_dst_cols<T, true>(G.lf_dcol[r], g, G.sm_dcol[r], s, plast + G.g0, dgr, chk, nb);
    return bt_dst_cols<T, false>(G.lf_dcol[r], g, G.sm_dcol[r], s, plast + G.g0, dgr, chk, nb);
  };
  if (d == 2) {
    for (const BatchGroup& G : bt.groups) STCHK(cols(G, 0, true));
  } else {
    for (const BatchGroup& G : bt.groups) STCHK(cols(G, 0, false));
    for (const BatchGroup& G : bt.groups) STCHK(cols(G, 1, true));
    for (const BatchGroup& G : bt.groups) STCHK(cols(G, 0, false));
  }
  for (const BatchGroup& G : bt.groups)
    STCHK((bt_dst_rows<T, DPRO_PLAIN, DEPI>(G.lf_row, dim3(G.nb_dstrow, G.gn), G.sm_dstrow, s, plast + G.g0, it, chk,
                                             (const int*)bt.d_nb_dstrow + G.g0)));
  return FL_OK;
}

template <typename T> fl_status bt_iteration(BatchT& bt, int pc, int k, hipStream_t s) {
  Iter it = {k & 1, k == 0 ? 1 : 0};
  const Prob* pi = (const Prob*)bt.d_iter;
  STCHK((bt_apply<T, PRO_PUPD, EPI_PQ>(bt, pc ? pi : (const Prob*)bt.d_iter_nopc, it, 1, s)));
  if (pc) {
    STCHK((bt_precond<T, DPRO_UPD, DEPI_Z>(bt, pi, pi, it, 1, s)));
  } else {
    LAUNCH(k_update_b<T>, dim3(vmax(bt.nb_upd), bt.np), dim3(256), 0, s, pi, it, (const long*)bt.d_N,
           (const int*)bt.d_nb_upd);
  }
  return FL_OK;
}

template <typename T> fl_status bt_initial_precond(BatchT& bt, int pc, hipStream_t s) {
  if (pc) {
    STCHK((bt_precond<T, DPRO_PLAIN, DEPI_Z>(bt, (const Prob*)bt.d_pc0, (const Prob*)bt.d_iter, Iter{1, 0}, 0, s)));
  }
  return FL_OK;
}

template <typename T> fl_status bt_resid(BatchT& bt, const Prob* pbs, hipStream_t s) {
  return bt_apply<T, PRO_PLAIN, EPI_RESID>(bt, pbs, Iter{0, 0}, 0, s);
}

template <typename T> fl_status bt_apply_plain(BatchT& bt, const Prob* pbs, hipStream_t s) {
  return bt_apply<T, PRO_PLAIN, EPI_PLAIN>(bt, pbs, Iter{0, 0}, 0, s);
}

template fl_status bt_setup<FL_T>(BatchT&, const BatchDesc&, const std::vector<Prob>&);
template fl_status bt_iteration<FL_T>(BatchT&, int, int, hipStream_t);
template fl_status bt_initial_precond<FL_T>(BatchT&, int, hipStream_t);
template fl_status bt_resid<FL_T>(BatchT&, const Prob*, hipStream_t);
template fl_status bt_apply_plain<FL_T>(BatchT&, const Prob*, hipStream_t);

#else  // FL_BATCH_HOST
static int vmax(const std::vector<int>& v) {
  int m = 0;
  for (int x : v) m = std::max(m, x);
  return m;
}
// ---------------------------------------------------------------------------
// host logic and C entry points
// ---------------------------------------------------------------------------

struct ProbBufs {
  void *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *f = nullptr;
  void *W1 = nullptr, *W2 = nullptr, *T1 = nullptr;
};

struct Batch {
  BatchDesc desc;
  std::vector<fl_op> ops;
  std::vector<ProbBufs> b64, b32;
  Scalars* sc64 = nullptr;
  Scalars* sc32 = nullptr;
  double* part64 = nullptr;
  double* part32 = nullptr;
  long pstride = 0;
  BatchT t64, t32;
  std::vector<void*> owned;
  std::vector<Scalars> hsc;
  Scalars* hpin = nullptr;
  int pc = FL_PC_FD;
  void* d_true = nullptr;
  hipGraphExec_t g[2] = {nullptr, nullptr}, g2[2] = {nullptr, nullptr};  // poll and 2 iterations
  int gpc[2] = {-1, -1}, gpoll[2] = {0, 0};
  int last_its[2] = {0, 0};  // iterations of the last solve per graph slot (all problems)
  double* d_tol = nullptr;      // per-problem tolerances (device, FP64 group order)
  std::vector<double> tolq;     // its host staging
  void* d_rhs = nullptr;        // explicit-part role of theta steps (theta < 1)
  std::vector<double> tolv;     // the same on the host
  // what the batch was built for (a later call with the same key reuses it)
  std::vector<const uint8_t*> kmasks;
  std::vector<double> ks1, kp1;
  double ks0 = 0, kp0 = 0, ktheta = -1;
  int kmixed = 0, kpc = -1;
  ~Batch() {
    for (void* p : owned) (void)hipFree(p);
    for (auto& e : g) if (e) (void)hipGraphExecDestroy(e);
    for (auto& e : g2) if (e) (void)hipGraphExecDestroy(e);
    if (hpin) (void)hipHostFree(hpin);
  }
  fl_status alloc(void** p, size_t bytes) {
    STCHK(dalloc(p, bytes));
    owned.push_back(*p);
    return FL_OK;
  }
};

template <typename T> static fl_status alloc_bufs(Batch& bt, std::vector<ProbBufs>& bufs, bool with_f) {
  const int np = bt.desc.np, d = bt.desc.d;
  bufs.assign(np, ProbBufs{});
  for (int p = 0; p < np; ++p) {
    fl_op op = bt.ops[p];
    const long N = op->N;
    ProbBufs& b = bufs[p];
    for (void** v : {&b.x, &b.r, &b.z, &b.p, &b.q}) STCHK(bt.alloc(v, N * sizeof(T)));
    if (with_f) STCHK(bt.alloc(&b.f, N * sizeof(T)));
    long rows = rows_of(op, 1);
    STCHK(bt.alloc(&b.W1, (size_t)rows * op->H[d - 1] * sizeof(cx<T>)));
    if (d == 3) STCHK(bt.alloc(&b.W2, (size_t)op->n[0] * op->P[1] * op->H[2] * sizeof(cx<T>)));
    STCHK(bt.alloc(&b.T1, N * sizeof(T)));
  }
  return FL_OK;
}

template <typename T> static Prob make_prob(Batch& bt, int p, const ProbBufs& b, Scalars* sc, double* part,
                                            double s0, double s1, double p0, double p1, const uint8_t* mask) {
  Prob pb = base_prob<T>(bt.ops[p], 1);
  if (bt.pc == FL_PC_SPECTRAL) {  // table built in make_batch
    pb.tau = bt.ops[p]->tau[tix<T>()];
    pb.pcs = 1.0;
  }
  pb.s0 = s0;
  pb.s1 = s1;
  pb.p0 = p0;
  pb.p1 = p1;
  if (bt.pc == FL_PC_MTILDE) (void)set_precond<T>(bt.ops[p], pb, FL_PC_MTILDE);
  pb.W1 = b.W1;
  pb.W2 = b.W2;
  pb.T1 = b.T1;
  pb.mask = mask;
  pb.x = b.x;
  pb.r = b.r;
  pb.z = b.z;
  pb.p = b.p;
  pb.q = b.q;
  pb.sc = sc + p;
  pb.part = part + (size_t)p * NSITE * bt.pstride;
  pb.pstride = bt.pstride;
  return pb;
}

static fl_status upload_vec(Batch& bt, const void* h, size_t bytes, void** d) {
  STCHK(bt.alloc(d, bytes));
  HIPCHK(hipMemcpy(*d, h, bytes, hipMemcpyHostToDevice));
  return FL_OK;
}

// A per-problem vector (problem order) in the device arrays' group order.
template <typename V> static std::vector<V> in_group_order(const BatchT& t, const std::vector<V>& v) {
  std::vector<V> out(v.size());
  for (size_t q = 0; q < t.order.size(); ++q) out[q] = v[t.order[q]];
  return out;
}

// Device arrays of the launch geometry and of the Prob roles for one precision.
template <typename T> static fl_status build_roles(Batch& bt, BatchT& t, std::vector<ProbBufs>& bufs, Scalars* sc,
                                                   double* part, const std::vector<double>& s0,
                                                   const std::vector<double>& s1, const std::vector<double>& p0,
                                                   const std::vector<double>& p1, const uint8_t* const* masks) {
  const int np = bt.desc.np;
  std::vector<Prob> iter(np), iter_nopc(np), pc0(np), res(np);
  for (int p = 0; p < np; ++p) {
    const uint8_t* m = masks ? masks[p] : nullptr;
    Prob pb = make_prob<T>(bt, p, bufs[p], sc, part, s0[p], s1[p], p0[p], p1[p], m);
    iter[p] = pb;
    iter[p].in = pb.T1;
    iter[p].out = pb.T1;
    iter_nopc[p] = pb;
    iter_nopc[p].z = pb.r;  // z aliases r without a preconditioner
    pc0[p] = pb;
    pc0[p].in = pb.r;
    pc0[p].out = pb.T1;
    res[p] = pb;  // residual r = f - A x: in = x, aux = f, out = r
    res[p].in = pb.x;
    res[p].aux = bufs[p].f;
    res[p].out = pb.r;
  }
  STCHK((bt_setup<T>(t, bt.desc, iter)));
  STCHK(upload_vec(bt, in_group_order(t, iter).data(), np * sizeof(Prob), &t.d_iter));
  STCHK(upload_vec(bt, in_group_order(t, iter_nopc).data(), np * sizeof(Prob), &t.d_iter_nopc));
  STCHK(upload_vec(bt, in_group_order(t, pc0).data(), np * sizeof(Prob), &t.d_pc0));
  STCHK(upload_vec(bt, in_group_order(t, res).data(), np * sizeof(Prob), &t.d_res));
  t.h_iter = iter;
  t.h_res = res;
  STCHK(upload_vec(bt, t.cg.data(), t.cg.size() * sizeof(ColGeom), &t.d_cg));
  STCHK(upload_vec(bt, t.dg.data(), t.dg.size() * sizeof(DGeom), &t.d_dg));
  STCHK(upload_vec(bt, t.nb_rowfwd.data(), np * sizeof(int), &t.d_nb_rowfwd));
  STCHK(upload_vec(bt, t.nb_rowinv.data(), np * sizeof(int), &t.d_nb_rowinv));
  STCHK(upload_vec(bt, t.nb_dstrow.data(), np * sizeof(int), &t.d_nb_dstrow));
  STCHK(upload_vec(bt, t.nb_upd.data(), np * sizeof(int), &t.d_nb_upd));
  for (int r = 0; r < 3; ++r) STCHK(upload_vec(bt, t.nb_col[r].data(), np * sizeof(int), &t.d_nb_col[r]));
  for (int r = 0; r < 2; ++r) STCHK(upload_vec(bt, t.nb_dcol[r].data(), np * sizeof(int), &t.d_nb_dcol[r]));
  STCHK(upload_vec(bt, t.N.data(), np * sizeof(long), &t.d_N));
  return FL_OK;
}

static fl_status read_all(Batch& bt, Scalars* dsc, hipStream_t s) {
  const int np = bt.desc.np;
  HIPCHK(hipMemcpyAsync(bt.hpin, dsc, np * sizeof(Scalars), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  bt.hsc.assign(bt.hpin, bt.hpin + np);
  return FL_OK;
}

// per-problem vector launches (setup and refinement; not in the iteration)
template <typename T> static fl_status per_dot(Batch& bt, BatchT& t, int p, const void* a, const void* b, int target,
                                               hipStream_t s) {
  const Prob& pb = t.h_iter[p];
  const long N = bt.ops[p]->N;
  LAUNCH(k_dot<T>, dim3(std::min<long>(1024, nblocks_vec(N))), dim3(256), 0, s, pb, a, b, (int)S_DOT, N);
  LAUNCH(k_finalize<>, dim3(1), dim3(256), 0, s, pb, (int)S_DOT, target);
  return FL_OK;
}

// Batched Krylov solve on precision T: r holds the initial residuals, x the
// initial iterates, sc[p].ff the squared rhs norms (and sc[p].rr the squared
// residual norms if use_rr).
template <typename T> static fl_status bt_krylov(Batch& bt, BatchT& t, Scalars* dsc, int pc, double tol,
                                                 const double* d_tols, int maxit, int use_rr, int graph, int poll,
                                                 hipStream_t s, int gslot) {
  const int np = bt.desc.np;
  LAUNCH(k_init_b<>, dim3(1, np), dim3(64), 0, s, (const Prob*)t.d_iter, tol, d_tols, maxit, use_rr);
  if (pc) {
    STCHK(bt_initial_precond<T>(t, pc, s));
  } else {
    for (int p = 0; p < np; ++p) {
      const Prob& pb = t.h_iter[p];
      const long N = bt.ops[p]->N;
      LAUNCH(k_dot<T>, dim3(std::min<long>(1024, nblocks_vec(N))), dim3(256), 0, s, pb, (const void*)pb.r,
             (const void*)pb.r, (int)S_RZ0, N);
    }
  }
  if (poll <= 0) poll = 8;
  if (poll & 1) ++poll;
  STCHK(bt_iteration<T>(t, pc, 0, s));
  bool use_graph = graph && s != nullptr;
  auto capture = [&](int len, hipGraphExec_t* ex) -> fl_status {
    hipGraph_t g;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    fl_status st = FL_OK;
    for (int j = 0; j < len && st == FL_OK; ++j) st = bt_iteration<T>(t, pc, 1 + j, s);
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st != FL_OK) return st;
    HIPCHK(e);
    const hipError_t ei = hipGraphInstantiate(ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(ei);
    return FL_OK;
  };
  if (use_graph && (!bt.g[gslot] || bt.gpc[gslot] != pc || bt.gpoll[gslot] != poll)) {
    for (hipGraphExec_t* e : {&bt.g[gslot], &bt.g2[gslot]})
      if (*e) {
        (void)hipGraphExecDestroy(*e);
        *e = nullptr;
      }
    STCHK(capture(poll, &bt.g[gslot]));
    bt.gpc[gslot] = pc;
    bt.gpoll[gslot] = poll;
    bt.last_its[gslot] = 0;
  }
  // The first stretch after iteration 0 covers the iteration count of the
  // previous solve of this batch (time steps repeat it closely) with graphs of
  // `poll` and of 2 iterations launched back to back: each iteration of a
  // batch past its stop still dispatches every pass of every group, so
  // stopping near the count saves those no-op launches.
  int k = 1;
  if (use_graph && bt.last_its[gslot] > 1) {
    int left = std::min(bt.last_its[gslot] - 1, maxit);
    if (left % poll != 0 && !bt.g2[gslot] && poll > 2) STCHK(capture(2, &bt.g2[gslot]));
    while (left > 0) {
      const bool whole = left >= poll || poll == 2;
      HIPCHK(hipGraphLaunch(whole ? bt.g[gslot] : bt.g2[gslot], s));
      left -= whole ? poll : 2;
      k += whole ? poll : 2;
    }
  }
  for (;;) {
    STCHK(read_all(bt, dsc, s));
    bool all = true;
    int mx = 0;
    for (auto& sc : bt.hsc) {
      all = all && sc.done;
      mx = std::max(mx, std::max(sc.itc[0], sc.itc[1]));
    }
    if (all) {
      bt.last_its[gslot] = mx;
      break;
    }
    if (mx >= maxit + 2 * poll) return fail(FL_E_HIP, "batched iteration bookkeeping lost");
    if (use_graph) {
      HIPCHK(hipGraphLaunch(bt.g[gslot], s));
      k += poll;
    } else {
      for (int j = 0; j < poll; ++j, ++k) STCHK(bt_iteration<T>(t, pc, k, s));
    }
  }
  return FL_OK;
}

// Build a batch (allocations, geometry, roles) for problems with the given
// shifts (s0 I + s1 M, preconditioner p0 I + p1 pcs T).
static fl_status make_batch(Batch& bt, int nprob, const fl_op* ops, const uint8_t* const* masks,
                            const std::vector<double>& s1, const std::vector<double>& p1, double s0, double p0,
                            const fl_solve_opts* o) {
  if (nprob < 1 || !ops) return fail(FL_E_INVALID, "nprob must be >= 1");
  const bool mixed = o && o->mixed;
  bt.pc = o ? o->pc : FL_PC_FD;
  // masked problems of a batch take the box inverse restricted to the domain
  // (the exact inverse on a mask is built per op by the single-problem calls)
  if (bt.pc == FL_PC_FD_BOX) bt.pc = FL_PC_FD;
  if (bt.pc == FL_PC_LEARNED || bt.pc == FL_PC_AUTO)
    return fail(FL_E_UNSUPPORTED, "batched solves take FL_PC_NONE, FD, FD_BOX, MTILDE or SPECTRAL");
  if (bt.pc != FL_PC_NONE && bt.pc != FL_PC_FD && bt.pc != FL_PC_SPECTRAL && bt.pc != FL_PC_MTILDE)
    return fail(FL_E_INVALID, "unknown preconditioner");
  if (bt.pc == FL_PC_SPECTRAL)
    for (int p = 0; p < nprob; ++p)
      if (ops[p]) STCHK(build_tau(ops[p]));
  const int d = ops[0]->d;
  bt.desc.np = nprob;
  bt.desc.d = d;
  bt.desc.n.assign(nprob, {1, 1, 1});
  bt.ops.assign(ops, ops + nprob);
  hipStream_t s = ops[0]->stream;
  long maxrows = 0;
  for (int p = 0; p < nprob; ++p) {
    if (!ops[p]) return fail(FL_E_INVALID, "NULL op in batch");
    if (ops[p]->d != d) return fail(FL_E_UNSUPPORTED, "a batch must share the dimension d");
    if (ops[p]->stream != s) return fail(FL_E_INVALID, "a batch must share one stream");
    for (int a = 0; a < 3; ++a) bt.desc.n[p][a] = ops[p]->n[a];
    maxrows = std::max(maxrows, rows_of(ops[p], 1));
  }
  bt.pstride = std::max<long>(4096, maxrows + 1);
  STCHK(alloc_bufs<double>(bt, bt.b64, true));
  STCHK(bt.alloc((void**)&bt.sc64, nprob * sizeof(Scalars)));
  STCHK(bt.alloc((void**)&bt.part64, (size_t)nprob * NSITE * bt.pstride * sizeof(double)));
  HIPCHK(hipMemset(bt.sc64, 0, nprob * sizeof(Scalars)));
  std::vector<double> s0v(nprob, s0), p0v(nprob, p0);
  STCHK(build_roles<double>(bt, bt.t64, bt.b64, bt.sc64, bt.part64, s0v, s1, p0v, p1, masks));
  if (mixed) {
    STCHK(alloc_bufs<float>(bt, bt.b32, false));
    STCHK(bt.alloc((void**)&bt.sc32, nprob * sizeof(Scalars)));
    STCHK(bt.alloc((void**)&bt.part32, (size_t)nprob * NSITE * bt.pstride * sizeof(double)));
    HIPCHK(hipMemset(bt.sc32, 0, nprob * sizeof(Scalars)));
    STCHK(build_roles<float>(bt, bt.t32, bt.b32, bt.sc32, bt.part32, s0v, s1, p0v, p1, masks));
  }
  if (hipHostMalloc((void**)&bt.hpin, nprob * sizeof(Scalars)) != hipSuccess) return fail(FL_E_NOMEM, "pinned");
  STCHK(bt.alloc((void**)&bt.d_tol, nprob * sizeof(double)));
  bt.tolv.assign(nprob, 0.0);
  bt.tolq.assign(nprob, 0.0);
  bt.kmasks.assign(nprob, nullptr);
  if (masks)
    for (int p = 0; p < nprob; ++p) bt.kmasks[p] = masks[p];
  bt.ks1 = s1;
  bt.kp1 = p1;
  bt.ks0 = s0;
  bt.kp0 = p0;
  bt.kmixed = mixed ? 1 : 0;
  bt.kpc = o ? o->pc : FL_PC_FD;
  return FL_OK;
}

// The batch of the last batched call, kept for the next call with the same
// problems (ops, masks, shifts, precision and preconditioner): its vectors,
// work arrays, descriptor tables and captured graphs are reused, so repeated
// calls allocate nothing.  fl_op_destroy of any member releases it.
static std::mutex g_batch_mu;
static std::unique_ptr<Batch> g_batch;

static bool batch_matches(const Batch& bt, int nprob, const fl_op* ops, const uint8_t* const* masks,
                          const std::vector<double>& s1, const std::vector<double>& p1, double s0, double p0,
                          const fl_solve_opts* o, double theta) {
  if (bt.desc.np != nprob || (int)bt.ops.size() != nprob) return false;
  for (int p = 0; p < nprob; ++p) {
    if (bt.ops[p] != ops[p]) return false;
    if (bt.kmasks[p] != (masks ? masks[p] : nullptr)) return false;
  }
  return bt.ks1 == s1 && bt.kp1 == p1 && bt.ks0 == s0 && bt.kp0 == p0 && bt.kmixed == ((o && o->mixed) ? 1 : 0) &&
         bt.kpc == (o ? o->pc : FL_PC_FD) && bt.ktheta == theta;
}

static fl_status batch_get(Batch** out, int nprob, const fl_op* ops, const uint8_t* const* masks,
                           const std::vector<double>& s1, const std::vector<double>& p1, double s0, double p0,
                           const fl_solve_opts* o, double theta) {
  if (g_batch && batch_matches(*g_batch, nprob, ops, masks, s1, p1, s0, p0, o, theta)) {
    *out = g_batch.get();
    return FL_OK;
  }
  g_batch.reset();
  std::unique_ptr<Batch> bt(new Batch());
  STCHK(make_batch(*bt, nprob, ops, masks, s1, p1, s0, p0, o));
  bt->ktheta = theta;
  g_batch = std::move(bt);
  *out = g_batch.get();
  return FL_OK;
}

void batch_forget_op(fl_op op) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  if (g_batch && std::find(g_batch->ops.begin(), g_batch->ops.end(), op) != g_batch->ops.end()) {
    (void)hipStreamSynchronize(op->stream);
    g_batch.reset();
  }
}

// Solve A_p x_p = f_p for every problem: f in b64[p].f, x in b64[p].x (initial
// guess when use_x0).  FP64 PCG, or FP32 PCG with FP64 refinement.
static fl_status batch_solve(Batch& bt, const double* tols, const fl_solve_opts* o, int use_x0,
                             std::vector<fl_info>& out) {
  const int np = bt.desc.np;
  hipStream_t s = bt.ops[0]->stream;
  const int pc = o ? o->pc : FL_PC_FD;
  const int mixed = o ? o->mixed : 0;
  const int graph = o ? o->graph : 1;
  const int poll = (o && o->poll_every > 0) ? o->poll_every : 8;
  long Nmax = 0;
  for (auto op : bt.ops) Nmax = std::max(Nmax, op->N);
  const int maxit = (o && o->maxit > 0) ? o->maxit : std::max(1000, (int)(10 * std::sqrt((double)Nmax)));
  out.assign(np, fl_info{});
  for (int p = 0; p < np; ++p) bt.tolv[p] = tols[p];
  // group order of the FP64 arrays (the only role k_init_b reads them with)
  for (int q = 0; q < np; ++q) bt.tolq[q] = tols[bt.t64.order[q]];
  HIPCHK(hipMemcpyAsync(bt.d_tol, bt.tolq.data(), np * sizeof(double), hipMemcpyHostToDevice, s));
  // ff (one launch over all problems: aux of the residual role is f) and the
  // initial residuals; the host reads ff with the next scalar read
  for (int p = 0; p < np; ++p) {
    ProbBufs& b = bt.b64[p];
    const long N = bt.ops[p]->N;
    if (!use_x0) LAUNCH(k_fill<double>, dim3(nblocks_vec(N)), dim3(256), 0, s, (double*)b.x, 0.0, N);
  }
  const dim3 gv(vmax(bt.t64.nb_upd), np);
  LAUNCH((k_dot_b<double, DOT_AUX>), gv, dim3(256), 0, s, (const Prob*)bt.t64.d_res, (int)S_DOT,
         (const long*)bt.t64.d_N, (const int*)bt.t64.d_nb_upd);
  LAUNCH(k_finalize_b<>, dim3(1, np), dim3(256), 0, s, (const Prob*)bt.t64.d_iter, (int)S_DOT, (int)FIN_FF);
  // r = f - A x and r.r on the device; read: also bring every scalar to the host
  auto residuals = [&](std::vector<double>& rr, bool read) -> fl_status {
    STCHK(bt_resid<double>(bt.t64, (const Prob*)bt.t64.d_res, s));
    LAUNCH(k_finalize_b<>, dim3(1, np), dim3(256), 0, s, (const Prob*)bt.t64.d_iter, (int)S_DOT, (int)FIN_RR);
    if (!read) return FL_OK;
    STCHK(read_all(bt, bt.sc64, s));
    rr.resize(np);
    for (int p = 0; p < np; ++p) rr[p] = bt.hsc[p].rr;
    return FL_OK;
  };
  std::vector<double> rr, ff(np);
  // the mixed loop ends with the true FP64 residuals of the returned x in rr:
  // its last evaluation precedes every exit, and finished problems keep x
  bool have_final = false;
  if (!mixed) {
    if (use_x0) {
      STCHK(residuals(rr, false));  // the Krylov start takes r.r on the device
    } else {
      for (int p = 0; p < np; ++p)
        HIPCHK(hipMemcpyAsync(bt.b64[p].r, bt.b64[p].f, bt.ops[p]->N * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    STCHK(bt_krylov<double>(bt, bt.t64, bt.sc64, pc, 0.0, bt.d_tol, maxit, use_x0, graph, poll, s, 0));
    for (int p = 0; p < np; ++p) ff[p] = bt.hsc[p].ff;
    for (int p = 0; p < np; ++p) {
      const Scalars& sc = bt.hsc[p];
      out[p].iters = std::max(sc.itc[0], sc.itc[1]);
      out[p].rel_res_recur = ff[p] > 0 ? std::sqrt(sc.rr / ff[p]) : 0.0;
      out[p].status = sc.done == 1 ? FL_OK : sc.done == 2 ? FL_E_NOCONV : FL_E_BREAKDOWN;
    }
  } else {
    have_final = true;
    const double itol = (o && o->inner_tol > 0) ? o->inner_tol : 1e-4;
    const int max_outer = (o && o->max_outer > 0) ? o->max_outer : 12;
    std::vector<char> active(np, 1);
    for (int p = 0; p < np; ++p) out[p].status = FL_E_NOCONV;
    for (int outer = 0;; ++outer) {
      STCHK(residuals(rr, true));
      if (outer == 0)
        for (int p = 0; p < np; ++p) ff[p] = bt.hsc[p].ff;
      bool any = false;
      for (int p = 0; p < np; ++p) {
        if (!active[p]) continue;
        if (ff[p] == 0.0 || std::sqrt(rr[p] / ff[p]) <= bt.tolv[p]) {
          active[p] = 0;
          out[p].status = FL_OK;
        } else if (!std::isfinite(rr[p])) {
          active[p] = 0;
          out[p].status = FL_E_BREAKDOWN;
        } else {
          any = true;
        }
      }
      if (!any || outer >= max_outer) break;
      // inner right-hand sides r32 = r64/||r64|| (zero for finished problems)
      for (int p = 0; p < np; ++p) {
        const long N = bt.ops[p]->N;
        const double sc = active[p] ? 1.0 / std::sqrt(rr[p]) : 0.0;
        LAUNCH((k_axpby<double, float>), dim3(nblocks_vec(N)), dim3(256), 0, s, (const double*)bt.b64[p].r,
               (float*)bt.b32[p].r, sc, 0.0, N);
        LAUNCH(k_fill<float>, dim3(nblocks_vec(N)), dim3(256), 0, s, (float*)bt.b32[p].x, 0.0f, N);
        STCHK(per_dot<float>(bt, bt.t32, p, bt.b32[p].r, bt.b32[p].r, FIN_FF, s));
        if (active[p]) out[p].outer_iters = outer + 1;
      }
      STCHK(bt_krylov<float>(bt, bt.t32, bt.sc32, pc, itol, nullptr, maxit, 0, graph, poll, s, 1));
      for (int p = 0; p < np; ++p) {
        const Scalars& sc = bt.hsc[p];
        if (!active[p]) continue;
        out[p].iters += std::max(sc.itc[0], sc.itc[1]);
        out[p].rel_res_recur = sc.ff > 0 ? std::sqrt(sc.rr / sc.ff) : 0.0;
        const long N = bt.ops[p]->N;
        LAUNCH((k_axpby<float, double>), dim3(nblocks_vec(N)), dim3(256), 0, s, (const float*)bt.b32[p].x,
               (double*)bt.b64[p].x, std::sqrt(rr[p]), 1.0, N);
      }
    }
  }
  // true residuals (FP64) into q
  if (have_final) {
    for (int p = 0; p < np; ++p) out[p].rel_res_true = ff[p] > 0 ? std::sqrt(rr[p] / ff[p]) : 0.0;
  } else {
    if (!bt.d_true) {  // residual role writing q, built once per batch
      std::vector<Prob> tr = bt.t64.h_res;
      for (int p = 0; p < np; ++p) tr[p].out = bt.b64[p].q;
      STCHK(upload_vec(bt, in_group_order(bt.t64, tr).data(), np * sizeof(Prob), &bt.d_true));
    }
    STCHK(bt_resid<double>(bt.t64, (const Prob*)bt.d_true, s));
    LAUNCH(k_finalize_b<>, dim3(1, np), dim3(256), 0, s, (const Prob*)bt.t64.d_iter, (int)S_DOT, (int)FIN_RR);
    STCHK(read_all(bt, bt.sc64, s));
    for (int p = 0; p < np; ++p) out[p].rel_res_true = ff[p] > 0 ? std::sqrt(bt.hsc[p].rr / ff[p]) : 0.0;
  }
  return FL_OK;
}

extern "C" {

fl_status fl_solve_batched(int nprob, const fl_op* ops, const double* const* f, const uint8_t* const* masks,
                           const double* tol, const fl_solve_opts* opts, double* const* u, fl_info* infos) {
  auto t0 = std::chrono::steady_clock::now();
  if (nprob < 1 || !ops || !f || !u || !infos || !tol) return fail(FL_E_INVALID, "NULL argument");
  for (int p = 0; p < nprob; ++p) {
    if (!ops[p] || !f[p] || !u[p]) return fail(FL_E_INVALID, "NULL problem entry");
    if (!(tol[p] > 0.0)) return fail(FL_E_INVALID, "tol must be positive");
    STCHK(need_solver_grid(ops[p]));
  }
  std::lock_guard<std::mutex> lk(g_batch_mu);
  Batch* bp = nullptr;
  std::vector<double> s1(nprob, 1.0), p1(nprob, 1.0);
  STCHK(batch_get(&bp, nprob, ops, masks, s1, p1, 0.0, 0.0, opts, -1.0));
  Batch& bt = *bp;
  hipStream_t s = ops[0]->stream;
  const int use_x0 = opts ? opts->use_x0 : 0;
  for (int p = 0; p < nprob; ++p) {
    HIPCHK(hipMemcpyAsync(bt.b64[p].f, f[p], ops[p]->N * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (use_x0) HIPCHK(hipMemcpyAsync(bt.b64[p].x, u[p], ops[p]->N * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  std::vector<fl_info> out;
  STCHK(batch_solve(bt, tol, opts, use_x0, out));
  for (int p = 0; p < nprob; ++p)
    HIPCHK(hipMemcpyAsync(u[p], bt.b64[p].x, ops[p]->N * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  fl_status worst = FL_OK;
  for (int p = 0; p < nprob; ++p) {
    infos[p] = out[p];
    infos[p].ms = ms;
    if (out[p].status != FL_OK) worst = (fl_status)out[p].status;
  }
  if (worst != FL_OK) return fail(worst, "a batched problem did not reach the tolerance");
  return FL_OK;
}

fl_status fl_step_batched(int nprob, const fl_op* ops, double* const* u, const double* dt, double theta, int nsteps,
                          double tol, const fl_solve_opts* opts, fl_info* infos) {
  auto t0 = std::chrono::steady_clock::now();
  if (nprob < 1 || !ops || !u || !dt || !infos) return fail(FL_E_INVALID, "NULL argument");
  if (!(theta > 0.0 && theta <= 1.0) || !(tol > 0.0) || nsteps < 0) return fail(FL_E_INVALID, "theta, tol or nsteps");
  for (int p = 0; p < nprob; ++p) {
    if (!ops[p] || !u[p] || !(dt[p] > 0.0)) return fail(FL_E_INVALID, "bad problem entry");
    STCHK(need_solver_grid(ops[p]));
  }
  std::lock_guard<std::mutex> lk(g_batch_mu);
  Batch* bp = nullptr;
  std::vector<double> s1(nprob), p1(nprob);
  for (int p = 0; p < nprob; ++p) s1[p] = p1[p] = theta * dt[p];
  STCHK(batch_get(&bp, nprob, ops, nullptr, s1, p1, 1.0, 1.0, opts, theta));
  Batch& bt = *bp;
  hipStream_t s = ops[0]->stream;
  const std::vector<double> tols(nprob, tol);
  // explicit part (I - (1-theta) dt M) u for theta < 1: a second role with that
  // shift, uploaded once per batch
  std::vector<Prob> rhs;
  void* d_rhs = bt.d_rhs;
  if (theta < 1.0 && !d_rhs) {
    rhs = bt.t64.h_res;
    for (int p = 0; p < nprob; ++p) {
      rhs[p].s0 = 1.0;
      rhs[p].s1 = -(1.0 - theta) * dt[p];
      rhs[p].in = bt.b64[p].x;
      rhs[p].out = bt.b64[p].f;
    }
    STCHK(upload_vec(bt, in_group_order(bt.t64, rhs).data(), nprob * sizeof(Prob), &d_rhs));
    bt.d_rhs = d_rhs;
  }
  for (int p = 0; p < nprob; ++p) {
    HIPCHK(hipMemcpyAsync(bt.b64[p].x, u[p], ops[p]->N * sizeof(double), hipMemcpyDeviceToDevice, s));
    infos[p] = fl_info{};
  }
  fl_status worst = FL_OK;
  for (int k = 0; k < nsteps; ++k) {
    // right-hand side b = u^k (backward Euler) or (I - (1-theta) dt M) u^k; warm start x = u^k
    if (theta < 1.0) {
      STCHK(bt_apply_plain<double>(bt.t64, (const Prob*)d_rhs, s));
    } else {  // f = x for every problem, one launch (in and aux of the residual role)
      LAUNCH(k_copy_in_aux_b<double>, dim3(vmax(bt.t64.nb_upd), nprob), dim3(256), 0, s,
             (const Prob*)bt.t64.d_res, (const long*)bt.t64.d_N, (const int*)bt.t64.d_nb_upd);
    }
    std::vector<fl_info> out;
    STCHK(batch_solve(bt, tols.data(), opts, 1, out));
    for (int p = 0; p < nprob; ++p) {
      infos[p].iters += out[p].iters;
      infos[p].outer_iters += out[p].outer_iters;
      infos[p].rel_res_true = std::max(infos[p].rel_res_true, out[p].rel_res_true);
      infos[p].rel_res_recur = out[p].rel_res_recur;
      if (out[p].status != FL_OK) {
        infos[p].status = out[p].status;
        worst = (fl_status)out[p].status;
      }
    }
  }
  for (int p = 0; p < nprob; ++p)
    HIPCHK(hipMemcpyAsync(u[p], bt.b64[p].x, ops[p]->N * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int p = 0; p < nprob; ++p) infos[p].ms = ms;
  if (worst != FL_OK) return fail(worst, "a batched step did not reach the tolerance");
  return FL_OK;
}

}  // extern "C"
#endif  // FL_BATCH_HOST
