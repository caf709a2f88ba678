// Batched driver: launch geometry of many problems advanced together.
#pragma once
#include <array>
#include <vector>

#include "fl_internal.hpp"

struct BatchDesc {
  int np = 0, d = 0;
  std::vector<std::array<int, 3>> n;  // grid of every problem
};

// Problems of a batch whose passes share their length specialisations: one
// launch per pass covers positions g0 .. g0 + gn - 1 of the device arrays,
// with the kernels compiled for those lengths (0: the run-time plan), the
// group's largest block counts and LDS sizes.
struct BatchGroup {
  int g0 = 0, gn = 0;
  int lf_rowfft = 0, lf_col[3] = {0, 0, 0};  // FFT row / column kernels
  int lf_row = 0, lf_dcol[2] = {0, 0};       // sine row / column kernels
  int nb_rowfwd = 0, nb_rowinv = 0, nb_dstrow = 0, nb_col[3] = {0, 0, 0}, nb_dcol[2] = {0, 0};
  size_t sm_row = 0, sm_dstrow = 0, sm_col[3] = {0, 0, 0}, sm_dcol[2] = {0, 0};
};

// Geometry and device descriptor arrays of a batch for one precision.  The
// device arrays (Prob roles, geometry, block counts, sizes, tolerances) hold
// the problems in group order: position q is problem order[q].  A launch per
// group has gridDim.y = gn; nb_* hold each problem's own block count (blocks
// beyond it exit at once).  Host-side copies (h_iter, h_res) stay in problem
// order.
struct BatchT {
  int np = 0, d = 0, elem = 0;
  std::vector<int> order;
  std::vector<BatchGroup> groups;
  std::vector<int> nb_rowfwd, nb_rowinv, nb_dstrow, nb_upd;  // group order
  std::vector<int> nb_col[3], nb_dcol[2];
  std::vector<ColGeom> cg;  // [3][np]: column passes of the application
  std::vector<DGeom> dg;    // [2][np]: column passes of the sine transform
  std::vector<long> N;
  // Prob roles (device arrays of np entries, host copies)
  //  iter: Krylov iteration (in = out = T1);  iter_nopc: z aliases r;
  //  pc0:  first preconditioner pass of the start (in = r);
  //  res:  residual r = f - A x (in = x, aux = f, out = r)
  void *d_iter = nullptr, *d_iter_nopc = nullptr, *d_pc0 = nullptr, *d_res = nullptr;
  std::vector<Prob> h_iter, h_res;
  void *d_cg = nullptr, *d_dg = nullptr, *d_N = nullptr;
  void *d_nb_rowfwd = nullptr, *d_nb_rowinv = nullptr, *d_nb_dstrow = nullptr, *d_nb_upd = nullptr;
  void* d_nb_col[3] = {nullptr, nullptr, nullptr};
  void* d_nb_dcol[2] = {nullptr, nullptr};
};

// Per-precision launch sequences (fl_batch.hip built with FL_T).
template <typename T> fl_status bt_setup(BatchT& bt, const BatchDesc& B, const std::vector<Prob>& base);
template <typename T> fl_status bt_iteration(BatchT& bt, int pc, int k, hipStream_t s);
template <typename T> fl_status bt_initial_precond(BatchT& bt, int pc, hipStream_t s);
template <typename T> fl_status bt_resid(BatchT& bt, const Prob* pbs, hipStream_t s);
template <typename T> fl_status bt_apply_plain(BatchT& bt, const Prob* pbs, hipStream_t s);
