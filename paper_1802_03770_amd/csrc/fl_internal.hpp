// Internal declarations shared by the translation units of the library.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fraclap.h"
#include "fl_kernels.hpp"

using namespace fl;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
extern thread_local std::string g_err;
inline fl_status fail(fl_status s, const std::string& m) {
  g_err = m;
  return s;
}
#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) return fail(FL_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define STCHK(x)                     \
  do {                               \
    fl_status s_ = (x);              \
    if (s_ != FL_OK) return s_;      \
  } while (0)

template <typename K, typename... A>
inline hipError_t launch(K* k, dim3 g, dim3 b, size_t smem, hipStream_t s, A... args) {
  if (g.x == 0 || g.y == 0) return hipSuccess;
  if (smem > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k, g, b, smem, s, args...);
  return hipGetLastError();
}
#define LAUNCH(...) HIPCHK(launch(__VA_ARGS__))

// ---------------------------------------------------------------------------
// operator object
// ---------------------------------------------------------------------------
struct Workspace {
  long cap_rhs = 0;        // apply/precond batch capacity
  void* W1 = nullptr;
  void* W2 = nullptr;
  void* T1 = nullptr;
  bool solver = false;     // Krylov vectors allocated
  void *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *f = nullptr;
  Scalars* sc = nullptr;
  double* part = nullptr;
  long npart = 0;
  // graph of `gK` PCG iterations starting at an odd iteration
  hipGraphExec_t gexec = nullptr;
  int gK = 0, gpc = -1, gcap = 0;
  double gs0 = 0, gs1 = 0, gp0 = 0, gp1 = 0;
  const uint8_t* gmask = nullptr;
  // graphs of flexible-CG iterations with the learned preconditioner: k >= 1
  // per slot of the host scalar ring (lexec[k & 1]) and the first iteration
  // (lexec[2]), valid for the network generation lgen and the solver Prob
  // whose bytes are lkey
  hipGraphExec_t lexec[3] = {nullptr, nullptr, nullptr};
  unsigned long long lgen = 0;
  std::vector<unsigned char> lkey;
};

// Capacitance correction that makes the sine-diagonalised preconditioner
// exact on an occluded domain (fl_capacity.hip).  One per op, keyed by the
// mask (pointer and checksum of its points) and the box operator
// p0 I + p1 pcs T it inverts.
constexpr long kCapMax = 8192;  // largest number of exterior points next to the domain
struct CapCache {
  bool valid = false;
  unsigned long long key = 0;
  const uint8_t* mask = nullptr;
  double p0 = 0, p1 = 0, pcs = 0;
  long k = 0;                          // |Gamma|
  int* idx = nullptr;                  // [k] grid indices of Gamma (device)
  void* cinv[2] = {nullptr, nullptr};  // [k][k] inverse capacitance matrix, FP64 / FP32
  void* Y[2] = {nullptr, nullptr};     // [cap][N] first box solve
  void* S[2] = {nullptr, nullptr};     // [cap][N] zero but on Gamma (mu)
  void* G[2] = {nullptr, nullptr};     // [cap][k] gathered first solve on Gamma
  long cap[2] = {0, 0};
};

struct fl_op_s {
  int d = 0;
  double alpha = 0, h = 0, c = 20;
  int dst_mode = 0;         // 0 autotune, 1 direct when possible, 2 chirp-z
  bool apply_only = false;  // an axis padded to 8192: the application only (2D)
  int col_lanes = 0;        // 0 autotune, -1 run-time plan, 64 / 128 forced
  int sine_col_lanes = 0;   // 0 autotune, -1 plan, 128 forced
  int dst_form[2][3] = {};  // chosen per precision and axis: 1 direct, 2 chirp-z, 3 prime form
  int n[3] = {1, 1, 1}, P[3] = {2, 2, 2}, H[3] = {1, 1, 1};
  long N = 0, NH = 0;
  hipStream_t stream = nullptr;
  double cst[8] = {0};
  double* d_cst = nullptr;
  double* wf = nullptr;     // folded weights [H...] FP64
  void* lam[2] = {nullptr, nullptr};  // folded symbol FP64 / FP32
  void* tau[2] = {nullptr, nullptr};  // sine-basis diagonal [n...] FP64 / FP32 (built on first use)
  Axis ax[2][3];            // per dtype
  std::vector<void*> tables;
  Workspace ws[2];
  CapCache cap;
  Scalars* hsc = nullptr;   // pinned host mirror of a Scalars
  ~fl_op_s();
};

template <typename T> constexpr int tix() { return sizeof(T) == 8 ? 0 : 1; }

// Count of device allocations the library has made (fl_device_allocations).
extern std::atomic<long long> g_dallocs;

inline fl_status dalloc(void** p, size_t bytes) {
  g_dallocs.fetch_add(1, std::memory_order_relaxed);
  if (hipMalloc(p, std::max<size_t>(bytes, 16)) != hipSuccess) {
    *p = nullptr;
    return fail(FL_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return FL_OK;
}

template <typename T> inline fl_status upload(fl_op op, const std::vector<T>& h, const void** out) {
  void* p;
  STCHK(dalloc(&p, h.size() * sizeof(T)));
  op->tables.push_back(p);
  HIPCHK(hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  *out = p;
  return FL_OK;
}

// block size for a line-FFT kernel with `tpl` lanes per line
inline int block_for(int) { return 256; }

// Length specialisation of the sine kernels along an axis: the direct lengths
// 2(n+1) of the common grids (n = 64, 128, 384, 512, 1024), or minus the FFT
// length of a chirp-z plan of length 256, 512 or 1024; 0 = the run-time plan.
inline int dst_lf(const Axis& A) {
  if (A.dst_rader) return kRaderLF;  // the prime form has no run-time version
  if (!A.dst.fixed) return 0;
  if (A.dst_direct) {
    switch (A.dst.L) {
      case 2050: case 1026: case 770: case 258: case 130: return A.dst.L;
      default: return 0;
    }
  }
  switch (A.dst.L) {
    case 1024: case 512: case 256: return -A.dst.L;
    default: return 0;
  }
}

// Length specialisation of the FFT row and column kernels of the application:
// the padded lengths 256..2048 of the common grids (lanes c_fixed_tpl(P));
// 0 = the run-time plan.
// Entry points beyond the application refuse application-only ops.
inline fl_status need_solver_grid(fl_op op) {
  if (op->apply_only)
    return fail(FL_E_UNSUPPORTED, "grids padded to 8192 points along an axis support fl_apply only");
  return FL_OK;
}

inline int fft_lf(const Axis& A) {
  if (!A.fft.fixed) return 0;
  switch (A.P) {
    case 8192: case 2048: case 1024: case 512: case 256: return A.P;
    default: return 0;
  }
}

// Lanes per column of a single-problem column pass of the application along
// axis A of a d-dimensional grid: the plan's, but kCol3DLanes512 for FP32 3D
// lines of 512 (FP64 needs too many registers for it: 841 against 786 us).
template <typename T> inline int col_tpl(const Axis& A, int d) {
  return (sizeof(T) == 4 && d == 3 && fft_lf(A) == 512) ? kCol3DLanes512 : A.fft.tpl;
}

// More lanes per line (fewer elements per lane) when a pass has too few lines
// to give every CU two workgroups; the plan's tpl is the minimum.
inline int tune_tpl(int tpl0, int L, long nlines) {
  if (c_is_fixed(L)) return tpl0;  // specialised lengths keep their compile-time lane count
  int tpl = tpl0;
  while (tpl < 256 && (nlines * tpl) / 256 < 512 && L / tpl >= 8) tpl *= 2;
  return tpl;
}

// ---------------------------------------------------------------------------
// problem descriptors
// ---------------------------------------------------------------------------
template <typename T> inline Prob base_prob(fl_op op, long nrhs) {
  Prob pb;
  memset(&pb, 0, sizeof(pb));
  pb.d = op->d;
  pb.nrhs = (int)nrhs;
  for (int a = 0; a < 3; ++a) pb.ax[a] = op->ax[tix<T>()][a];
  pb.lam = op->lam[tix<T>()];
  pb.s0 = 0.0;
  pb.s1 = 1.0;
  pb.pcs = op->cst[0] * std::fabs(op->cst[2]) * std::pow(op->h, -op->alpha);
  pb.p0 = 0.0;
  pb.p1 = 1.0;
  return pb;
}

inline long rows_of(fl_op op, long nrhs) {
  long r = nrhs;
  for (int a = 0; a < op->d - 1; ++a) r *= op->n[a];
  return r;
}

// A captured iteration graph holds the workspace pointers by value: every
// reallocation below invalidates it.
inline void drop_graph(Workspace& w) {
  if (w.gexec) {
    (void)hipGraphExecDestroy(w.gexec);
    w.gexec = nullptr;
  }
  for (hipGraphExec_t& g : w.lexec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  w.lkey.clear();
}

template <typename T> inline fl_status ensure_ws(fl_op op, long nrhs, bool solver) {
  Workspace& w = op->ws[tix<T>()];
  const long N = op->N;
  if (w.cap_rhs < nrhs) {
    drop_graph(w);
    for (void** p : {&w.W1, &w.W2, &w.T1})
      if (*p) { hipFree(*p); *p = nullptr; }
    long rows = rows_of(op, nrhs);
    STCHK(dalloc(&w.W1, (size_t)rows * op->H[op->d - 1] * sizeof(cx<T>)));
    if (op->d == 3) STCHK(dalloc(&w.W2, (size_t)nrhs * op->n[0] * op->P[1] * op->H[2] * sizeof(cx<T>)));
    STCHK(dalloc(&w.T1, (size_t)nrhs * N * sizeof(T)));
    w.cap_rhs = nrhs;
    long np = std::max<long>(4096, rows + 1);  // partials per site
    if (w.npart < np) {
      if (w.part) hipFree(w.part);
      STCHK(dalloc((void**)&w.part, NSITE * np * sizeof(double)));
      w.npart = np;
    }
  }
  if (!w.sc) {
    STCHK(dalloc((void**)&w.sc, sizeof(Scalars)));
    HIPCHK(hipMemset(w.sc, 0, sizeof(Scalars)));
  }
  if (solver && !w.solver) {
    drop_graph(w);
    for (void** p : {&w.x, &w.r, &w.z, &w.p, &w.q, &w.f}) STCHK(dalloc(p, (size_t)N * sizeof(T)));
    w.solver = true;
  }
  return FL_OK;
}

template <typename T> inline Prob solver_prob(fl_op op, const uint8_t* mask, double s0, double s1, double p0,
                                              double p1) {
  Workspace& w = op->ws[tix<T>()];
  Prob pb = base_prob<T>(op, 1);
  pb.s0 = s0;
  pb.s1 = s1;
  pb.p0 = p0;
  pb.p1 = p1;
  pb.W1 = w.W1;
  pb.W2 = w.W2;
  pb.T1 = w.T1;
  pb.mask = mask;
  pb.x = w.x;
  pb.r = w.r;
  pb.z = w.z;
  pb.p = w.p;
  pb.q = w.q;
  pb.sc = w.sc;
  pb.part = w.part;
  pb.pstride = w.npart;
  return pb;
}

inline long nblocks_vec(long n) { return (n + 255) / 256; }

// Sine-basis diagonal table of the operator (built once per op, in fl_host.hip).
fl_status build_tau(fl_op op);

// Select the preconditioner of a solver Prob: the FD Laplacian keeps pcs =
// C|B|h^-alpha; the sine-basis diagonal sets the table and pcs = 1.
// M~ = q0 I + q1 T with q0 = C h^-alpha (Z - 2d), q1 = C h^-alpha (1 - B): the
// shifted system p0 I + p1 M~ has sine eigenvalues (p0 + p1 q0) + p1 q1 sum_a eig_a.
template <typename T> inline fl_status set_precond(fl_op op, Prob& pb, int pc) {
  if (pc == FL_PC_SPECTRAL) {
    STCHK(build_tau(op));
    pb.tau = op->tau[tix<T>()];
    pb.pcs = 1.0;
  } else if (pc == FL_PC_MTILDE) {
    const double Ch = op->cst[7];
    pb.tau = nullptr;
    pb.p0 = pb.p0 + pb.p1 * Ch * (op->cst[1] - 2.0 * op->d);
    pb.pcs = Ch * (1.0 - op->cst[2]);
  } else {
    pb.tau = nullptr;
  }
  return FL_OK;
}

// Preconditioners that are made exact on an occluded domain.
inline bool pc_exact_on_mask(int pc) { return pc == FL_PC_FD || pc == FL_PC_MTILDE; }
// Anything that applies the sine-transform preconditioner (not plain CG).
inline bool pc_is_sine(int pc) {
  return pc == FL_PC_FD || pc == FL_PC_SPECTRAL || pc == FL_PC_MTILDE || pc == FL_PC_FD_BOX;
}

// Learned preconditioner (fl_net.hip): scratch on op's grid, then flexible CG
// on the workspace Prob pb (r: initial residual, x: initial iterate).  status:
// 1 converged, 2 iteration cap, 3 breakdown; fell_back: the FD preconditioner
// took over.
fl_status learned_prepare(fl_op op, fl_net net, size_t elem);
template <typename T>
fl_status learned_fcg(fl_op op, fl_net net, const Prob& pb, double tol, int maxit, double ff, double rr0, int graph,
                      int* iters, double* rr_out, int* status, int* fell_back);

// Exact preconditioner on occluded domains (fl_capacity.hip): the mask
// checksum into *dst (device), the build or reuse of the correction for the
// box operator of pbox, its per-precision buffers, and the corrected
// preconditioner sequence (same epilogues as precond_seq).
fl_status cap_hash_launch(fl_op op, const uint8_t* mask, unsigned long long* dst);
fl_status cap_prepare(fl_op op, const uint8_t* mask, const Prob& pbox, unsigned long long key, bool* active);
void cap_destroy(fl_op op);
template <typename T> fl_status cap_buffers(fl_op op, long nrhs);
template <typename T, int DPRO, int DEPI> fl_status cap_precond_seq(fl_op op, const Prob& pb, Iter it, int chk);

// Release the cached batch of the batched driver if it holds this op
// (fl_batch.hip; called by fl_op_destroy).
void batch_forget_op(fl_op op);

// Launch sequences (defined per precision in fl_apply.hip / fl_precond.hip).
template <typename T, int PRO, int EPI> fl_status apply_seq(fl_op op, const Prob& pb, Iter it, int chk);
template <typename T, int DPRO, int DEPI> fl_status precond_seq(fl_op op, Prob pb, Iter it, int chk);
// One pass of the application (0 rows fwd, 1 symbol column pass, 2 rows inverse)
// or of the preconditioner (3 first sine pass, 4 scaled column pass, 5 last).
template <typename T> fl_status launch_apply_pass(fl_op op, Prob pb, int pass);
template <typename T> fl_status launch_precond_pass(fl_op op, Prob pb, int pass);

