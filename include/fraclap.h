/* fraclap.h -- C ABI of the MI355X (gfx950) fractional Laplacian solver.
 *
 * Method: Minden & Ying, "A simple solver for the fractional Laplacian in
 * multiple dimensions".  The operator is the singularity-subtracted
 * trapezoidal discretisation of (-Delta)^{alpha/2} (Sec. 2, eqs. fl,
 * int1constants, a3, window) on a regular grid of n_1 x ... x n_d interior
 * points with spacing h (Sec. 3.1, eq. linearelliptic):
 *
 *   (M u)_i = sum_j w_{i-j} u_j,  w_m = C h^{-alpha} omega_m,
 *   omega_0 = Z - 2 d B, omega_{+-e_k} = -1 + B, omega_m = -|m|^{-(d+alpha)},
 *
 * with Z the lattice sum A_1 h^{d+alpha}, B = h^{d+alpha-2}(A_2 + A_3) and
 * C = C_{alpha,d}.  M is applied as a zero-padded FFT convolution
 * (Sec. 3.1, "Forward operator and application with FFT"); solves use CG
 * preconditioned by the finite-difference Laplacian C h^d L applied with
 * sine transforms (Sec. 3.1, "Preconditioning"); time steps use the implicit
 * scheme of Sec. 3.2 (eq. timestepping) with theta in (0, 1].
 *
 * Conventions for every call:
 *  - Arrays are DEVICE pointers owned by the caller, C-contiguous row-major
 *    [batch][n_1]...[n_d] (last axis fastest).  The library never frees
 *    caller memory.
 *  - An fl_op owns its weights, symbol, transform tables and workspaces.  It
 *    allocates in fl_make_weights and on the first call of each kind/size;
 *    later calls of the same shape do not allocate.
 *  - Work is ordered on the op's HIP stream (given at creation; NULL = the
 *    null stream).  fl_apply / fl_precond return after enqueueing; fl_solve,
 *    fl_step and the batched calls return after the final device poll with
 *    `info` filled.
 *  - A nonzero status is returned on any failure and nothing aborts;
 *    fl_last_error() gives a thread-local message.  FL_E_NOCONV still leaves
 *    the best iterate in the output and fills `info`.
 *  - An op is not thread safe: use one op per host thread / stream.
 */
#ifndef FRACLAP_H
#define FRACLAP_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fl_op_s* fl_op;
typedef struct fl_net_s* fl_net;

typedef enum {
  FL_OK = 0,
  FL_E_INVALID = -1,     /* bad argument (d, alpha, h, sizes, tol, null pointer) */
  FL_E_NOMEM = -2,       /* device allocation failed */
  FL_E_HIP = -3,         /* HIP runtime error */
  FL_E_NOCONV = -4,      /* iteration cap reached before the tolerance */
  FL_E_BREAKDOWN = -5,   /* p.q <= 0 or a non-finite value in the recurrence */
  FL_E_UNSUPPORTED = -6  /* valid request this build does not implement */
} fl_status;

typedef enum { FL_F64 = 0, FL_F32 = 1 } fl_dtype;

typedef enum {
  FL_PC_NONE = 0,     /* plain CG */
  FL_PC_FD = 1,       /* finite-difference Laplacian preconditioner (Sec. 3.1) */
  FL_PC_LEARNED = 2,  /* not in the paper: flexible CG with z = B (r + s N(r/s, alpha)), N the network
                         opts->net (of the op's dimension), B the FL_PC_SPECTRAL inverse, s = RMS(r); the FD
                         preconditioner is the fallback (d = 2 or 3, no mask) */
  FL_PC_SPECTRAL = 3, /* not in the paper: the sine basis of the FD preconditioner with the
                         operator's own diagonal in that basis as eigenvalues, i.e. the best
                         approximation of M diagonalised by the type-I sine transform */
  FL_PC_MTILDE = 4,   /* M~ (Sec. 3.1, the alternative the paper mentions): M restricted to the
                         sparsity pattern of L, M~ = C h^-alpha [(Z - 2d) I + (1 - B) T], T the
                         (2d+1)-point Laplacian; sine transforms on the box, exact on a mask */
  FL_PC_FD_BOX = 5,   /* on a mask: P_Omega (C h^d L_box)^{-1} P_Omega, the box inverse restricted to
                         the domain (not the paper's operator; on the box the same as FL_PC_FD) */
  FL_PC_AUTO = 6      /* the paper's rule (Sec. 4.1, 4.2): no preconditioner for alpha < 1, FL_PC_FD
                         otherwise */
} fl_precond_kind;

typedef struct {
  double delta_over_h;  /* window radius c in grid points (Sec. 4.1 uses 20); <= 0 -> 20 */
  int dst_mode;         /* sine-transform plan per axis: 0 = autotune (time the preconditioner with both
                           forms when the op is built and keep the faster, per precision); 1 = direct odd
                           extension of length 2(n+1) when it factors over radices <= 43, the prime form
                           when n + 1 = 257 (Rader's identity: a real DFT of length 257 as a cyclic
                           convolution of length 256), else chirp-z; 2 = chirp-z with a 5-smooth length
                           >= 2n-1 */
  int col_lanes;        /* symbol column pass at lengths 1024 and 2048: 0 = autotune, -1 = run-time plan,
                           64, 128 or 256 (length 2048) = lanes per column of the specialised kernel */
  int sine_col_lanes;   /* sine column pass at direct length 2050: 0 = autotune, -1 = plan, 128 = forced */
  int reserved[3];
} fl_weights_opts;

typedef struct {
  int pc;            /* fl_precond_kind */
  int mixed;         /* 0: FP64 PCG; 1: FP32 inner PCG + FP64 iterative refinement */
  int maxit;         /* iteration cap (FP64 PCG) or inner cap (mixed); <= 0 -> default */
  double inner_tol;  /* mixed: relative tolerance of each inner FP32 solve; <= 0 -> 1e-4 */
  int use_x0;        /* 1: u holds the initial guess on entry */
  int graph;         /* 1: replay the Krylov iteration as a captured hipGraph (FL_PC_LEARNED: one
                        graph launch per iteration, the graphs kept with the op's workspace
                        until its Prob or the network's buffers change) */
  int poll_every;    /* iterations between host polls of the convergence flag (<= 0 -> 8) */
  int max_outer;     /* mixed: cap on refinement steps (<= 0 -> 12) */
  fl_net net;        /* FL_PC_LEARNED: the trained network (same stream as the op); else ignored */
} fl_solve_opts;

typedef struct {
  int iters;         /* Krylov iterations (sum over inner solves when mixed) */
  int outer_iters;   /* refinement steps (mixed) */
  int status;        /* fl_status of the solve */
  int fell_back;     /* FL_PC_LEARNED: 1 if the FD preconditioner took over in some inner solve */
  double rel_res_true;   /* ||f - M u||_2 / ||f||_2 recomputed in FP64 at exit */
  double rel_res_recur;  /* last recurrence residual of the (inner) Krylov loop */
  double ms;             /* wall time of the call, milliseconds */
} fl_info;

/* Build M for dimension d in {1,2,3}, 0 < alpha < 2, spacing h > 0 and grid
 * n[0..d-1] (each >= 1): constants C, Z, B (FP64, one workgroup), the folded
 * weight array, the symbol lambda = DFT of the circulant embedding of the
 * weights (padded length per axis: smallest even 2^a 3^b 5^c >= 2 n_k; lags
 * >= n_k of the embedding are zero), FP64 and FP32 copies, and the transform
 * tables.  Paper: Sec. 2.7 (constants), Sec. 3.1 (M and its FFT application).
 * `opts` may be NULL.  On success *out owns all device memory of the op.
 * Padded lengths up to 4096 are supported everywhere; a padded length of 8192
 * (n_k = 4081 .. 4096, e.g. the 4095^2 fine grid of the smooth 2D example of
 * Sec. 4.2) only in 2D and only for fl_apply: on such an op every other
 * computing call returns FL_E_UNSUPPORTED.  Other lengths above 4096 fail here
 * with FL_E_UNSUPPORTED. */
fl_status fl_make_weights(int d, double alpha, double h, const int64_t* n, const fl_weights_opts* opts,
                          void* hip_stream, fl_op* out);

/* Host FP64 copy of the scalar constants:
 * out[0..7] = C, Z, B, a2, h^{d+alpha-2} A_3, omega_0, omega_e, C h^{-alpha}. */
fl_status fl_op_constants(fl_op op, double out[8]);

/* Padded circulant lengths P_k (out[0..d-1]). */
fl_status fl_op_padded(fl_op op, int64_t* out);

/* Plans chosen for the op (16 entries), per precision p (0 FP64, 1 FP32):
 * out[3 p + a] = 1 (direct), 2 (chirp-z) or 3 (prime form) sine transform along axis a < d,
 * out[6 + 3 p + a] = its FFT length, out[12 + p] = lanes per column of the
 * symbol column pass (0: run-time plan; 64 or 128: specialised kernel),
 * out[14 + p] = lanes per FFT line of the sine column pass (0: plan; 128). */
fl_status fl_op_plan(fl_op op, int64_t* out);

/* Device-to-device copy of the folded arrays, shape [P_1/2+1]...[P_d/2+1]:
 * which = 0: weights w_m (FP64, zero for m_k >= n_k); 1: symbol lambda (FP64);
 * 2: symbol lambda (FP32).  dst must hold prod(P_k/2+1) elements.
 * which = 3 / 4: the sine-basis diagonal tau (FP64 / FP32, shape [n_1]..[n_d],
 * index k_a - 1; see fl_precond_spectral), prod(n_k) elements. */
fl_status fl_op_export(fl_op op, int which, void* dst);

/* Mu = M u for `batch` stacked inputs (dtype FL_F64 or FL_F32, both arrays of
 * that type).  mask (uint8 [n...], 1 = inside, may be NULL) gives the occluded
 * operator P_Omega M P_Omega.  shift0/shift1: computes (shift0 I + shift1 M) u
 * (pass 0, 1 for M itself).  Paper Sec. 3.1, "Forward operator". */
fl_status fl_apply(fl_op op, const void* u, void* Mu, int dtype, int64_t batch, const uint8_t* mask,
                   double shift0, double shift1);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as fl_apply, with the complex work arrays in a fixed device array of
 * 64 MiB that the library holds on each device (not in the op's workspace),
 * and no allocation of any kind.  The scratch must hold the half spectrum of
 * the last axis, rows x (P_d/2+1) complex values of dtype, plus in 3D batch x
 * n_1 x P_2 x (P_3/2+1) complex values (e.g. a 1024 x 1024 FP64 grid needs
 * 16.8 MB, 128^3 FP32 51 MB); larger requests return FL_E_INVALID before any
 * work is enqueued.  Every call on a device shares that array: calls that
 * overlap in time on one device (other streams, other ops, other host
 * threads) race and must be serialised by the caller.  Arguments, layout and
 * stream ordering as fl_apply; call it with the op's device current. */
fl_status fl_apply_noalloc(fl_op op, const void* u, void* Mu, int dtype, int64_t batch, const uint8_t* mask,
                           double shift0, double shift1);

/* z = (p0 I + p1 C h^d L)^{-1} r, sine transforms along every axis.  p0 = 0,
 * p1 = 1 is the elliptic preconditioner; p0 = 1, p1 = theta dt the time-step
 * one.  Paper Sec. 3.1 ("Preconditioning") and Sec. 3.2.
 * With a mask (uint8 [n...], 1 = inside the domain Omega) the inverse is the
 * exact one on Omega, (p0 I + p1 C h^d L)_Omega^{-1} with zero data outside
 * Omega (the paper's L_Omega^{-1}, Sec. 4.4, there by sparse Cholesky): the
 * box inverse corrected by a capacitance matrix on the k exterior points next
 * to Omega (two box solves and a k x k product per application).  The
 * correction is built on the first call for a mask (k box solves in FP64 and
 * a k x k inversion; checksum of the mask's points and the pointer identify
 * it) and reused while mask and (p0, p1) stay the same; k <= 8192, else
 * FL_E_UNSUPPORTED.  z is zero outside Omega. */
fl_status fl_precond(fl_op op, const void* r, void* z, int dtype, int64_t batch, const uint8_t* mask,
                     double p0, double p1);

/* The preconditioner of any kind: FL_PC_FD (as fl_precond), FL_PC_SPECTRAL
 * (as fl_precond_spectral), FL_PC_MTILDE ((p0 I + p1 M~)^{-1}, exact on a mask
 * as for FL_PC_FD) or FL_PC_FD_BOX (P_Omega (p0 I + p1 C h^d L_box)^{-1}
 * P_Omega).  Same layout and errors as fl_precond. */
fl_status fl_precond_any(fl_op op, int kind, const void* r, void* z, int dtype, int64_t batch,
                          const uint8_t* mask, double p0, double p1);

/* As fl_precond with the sine-basis diagonal of M in place of the FD
 * Laplacian: z = (p0 I + p1 Q diag(tau) Q^T)^{-1} r, where Q is the
 * orthonormal type-I sine transform on the box and tau_k = (Q^T M Q)_kk,
 * computed once per op in FP64 (about 2 n^{d+1} flops) on first use.  Not in
 * the paper: it keeps the paper's fast sine-transform solve (Sec. 3.1) and
 * replaces the Laplacian's eigenvalues by the operator's own.  Same layout,
 * masking and errors as fl_precond. */
fl_status fl_precond_spectral(fl_op op, const void* r, void* z, int dtype, int64_t batch, const uint8_t* mask,
                              double p0, double p1);

/* Solve M u = f (FP64 f and u, single right-hand side) to relative residual
 * tol (recurrence residual in the loop; the true FP64 residual is reported).
 * Paper Sec. 3.1 (eq. matelliptic) and Sec. 4 (stopping test).  With a mask
 * the system is P_Omega M P_Omega u = P_Omega f on Omega (f is restricted to
 * Omega; u is zero outside it), Sec. 4.4; FL_PC_FD and FL_PC_MTILDE then use
 * the exact inverse on Omega (see fl_precond). */
fl_status fl_solve(fl_op op, const double* f, const uint8_t* mask, double tol, const fl_solve_opts* opts,
                   double* u, fl_info* info);

/* One implicit step: (I + theta dt M) u^{k+1} = (I - (1-theta) dt M) u^k
 *                    + dt (theta f^{k+1} + (1-theta) f^k),
 * preconditioner I + theta dt C h^d L, warm start u^k.  u: u^k in, u^{k+1}
 * out (FP64).  f_k, f_k1 may be NULL (zero forcing).  theta in (0, 1]
 * (0.5 Crank-Nicolson as in Sec. 3.2, 1 backward Euler). */
fl_status fl_step(fl_op op, double* u, double dt, double theta, const double* f_k, const double* f_k1,
                  const uint8_t* mask, double tol, const fl_solve_opts* opts, fl_info* info);

/* Solve nprob independent systems ops[i] u[i] = f[i] (Sec. 3, the same PCG
 * as fl_solve) together: every kernel of an iteration is one launch over all
 * problems (blockIdx.y = problem), and the iteration is replayed as one
 * captured hipGraph; a converged problem stops doing work while the others
 * continue.  Uneven grids and alphas are allowed and problems may share an op
 * (several right-hand sides of one operator).
 *   ops[i]   : all of the same dimension d and created on the same stream
 *              (otherwise FL_E_UNSUPPORTED / FL_E_INVALID)
 *   f[i]     : device FP64, ops[i]'s grid, row-major, read only
 *   masks    : NULL, or an array whose entries are NULL (box) or device uint8
 *              masks of ops[i]'s grid
 *   opts     : as for fl_solve (pc, mixed, maxit, inner_tol, use_x0, graph,
 *              poll_every, max_outer); NULL = defaults
 *   u[i]     : device FP64, initial guess when opts->use_x0, solution out
 *   infos[i] : each problem's iterations, status and residuals; ms is the
 *              wall time of the whole batch
 *   tol[i]   : host array, the relative residual tolerance of each problem (> 0)
 * Per-problem Krylov vectors, work arrays and descriptor tables are allocated
 * on the first call for a set of problems and kept for the next batched call
 * with the same ops, masks, shifts, precision and preconditioner (one such
 * set at a time, for fl_solve_batched and fl_step_batched together), which
 * then allocates nothing; a call for another set, or fl_op_destroy of a
 * member, releases them.  Returns the status of a failing problem (and its
 * infos entry says which) when any problem misses its tolerance.
 * Masked problems take the box preconditioner restricted to the mask
 * (FL_PC_FD and FL_PC_FD_BOX are the same here). */
fl_status fl_solve_batched(int nprob, const fl_op* ops, const double* const* f, const uint8_t* const* masks,
                           const double* tol, const fl_solve_opts* opts, double* const* u, fl_info* infos);

/* Advance nprob problems by nsteps implicit theta steps each (Sec. 3.2, the
 * same step as fl_step with zero forcing and no mask), every step one batched
 * solve with warm start u^k.  dt[i] > 0 per problem; u[i] device FP64 in/out;
 * theta in (0, 1].  infos[i]: iters and outer_iters summed over the steps,
 * rel_res_true the largest over the steps. */
fl_status fl_step_batched(int nprob, const fl_op* ops, double* const* u, const double* dt, double theta,
                          int nsteps, double tol, const fl_solve_opts* opts, fl_info* infos);

/* ---- learned preconditioner (not in the paper) ----
 * A multilevel convolutional network N(x, alpha) on a 2D grid H x W (d = 2)
 * or a 3D grid D x H x W (d = 3), every side a multiple of 8: 3 x 3 (x 3)
 * convolutions with 32 channels on 4 levels (average pooling over 2 x 2 (x 2)
 * blocks, nearest upsampling, additive skips, ReLU), BF16 activations with
 * FP32 accumulation, FP32 master parameters.  Parameter vector (FP32,
 * fl_net_nparams(d) entries): per layer W[tap][ci][co] then b[co], with
 * K = 3^d taps, tap = 9 kz + 3 ky + kx (kz absent in 2D) over the offsets,
 * layers cin (2 -> 32; input channels x and alpha - 1), d1, d2, d3, b3, u2,
 * u1, u0 (32 -> 32), out (32 -> 1).  Inside flexible CG (FL_PC_LEARNED) the
 * preconditioner is z = B (r + s N(r/s, alpha)), B the FL_PC_SPECTRAL inverse
 * and s the RMS of r; the op's grid is zero-padded to multiples of 8 for the
 * network.  All arrays are device arrays on the net's stream; grids are
 * [batch][D][H][W] with D = 1 for a 2D network. */

/* New network for d = 2 or 3 with zero parameters (call fl_net_set_params
 * before use). */
fl_status fl_net_create(int d, void* hip_stream, fl_net* out);
/* Number of FP32 parameters of a network for d (65633 for d = 2, 196385 for
 * d = 3; 0 otherwise). */
int64_t fl_net_nparams(int d);
/* Copy in / out the FP32 parameter vector; set also clears the Adam moments. */
fl_status fl_net_set_params(fl_net net, const float* params);
fl_status fl_net_get_params(fl_net net, float* params);
/* y = N(x, alpha[b]) for batch grids x[b] (FP32 [batch][D][H][W]); alpha is a
 * host array of batch values. */
fl_status fl_net_forward(fl_net net, const float* x, const double* alpha, float* y, int batch, int D, int H, int W);
/* grad = d/dtheta sum(gy * N(x, alpha)) (FP32, fl_net_nparams(d) entries). */
fl_status fl_net_grad(fl_net net, const float* x, const double* alpha, const float* gy, float* grad, int batch,
                      int D, int H, int W);
/* `steps` Adam steps (lr, beta1 0.9, beta2 0.999, eps 1e-8) on the loss
 * mean over the minibatch of ||N(R_i, A_i) - T_i||^2 / (D H W); minibatch k
 * takes pairs idx[k*batch .. k*batch+batch-1] (host array, each < npairs).
 * R, T: FP32 [npairs][D][H][W]; A: FP32 [npairs] (device).  losses (host,
 * `steps` entries) receives the loss of each minibatch before its update. */
fl_status fl_net_train(fl_net net, const float* R, const float* T, const float* A, int npairs, int D, int H, int W,
                       const int* idx, int steps, int batch, double lr, float* losses);
/* Training pairs from errors e_k = e[k * e_stride] - e_sub[k] (FP64 grids of
 * the op, d = 2 or 3; e_stride 0 repeats one array, e_sub may be NULL):
 * r = M e, s = RMS(r), R = r / s and T = (D e - r) / s with D = Q diag(tau) Q^T
 * (the operator diagonal in the sine basis), written zero-padded into the
 * Dp x Hp x Wp grid (R, T: FP32 [count][Dp][Hp][Wp]; d = 2: Dp = 1,
 * Hp >= n_0, Wp >= n_1; d = 3: Dp >= n_0, Hp >= n_1, Wp >= n_2). */
fl_status fl_learned_pairs(fl_op op, const double* e, int64_t e_stride, const double* e_sub, int count, float* R,
                           float* T, int Dp, int Hp, int Wp);
/* Measurement aid: average duration (ms, HIP events on the net's stream) of
 * `reps` launches on a 1 x D x H x W input: which = 0 the whole forward pass,
 * 1 the level-0 32 -> 32 convolution (MFMA, skip-add staging), 2 the input
 * layer, 3 the output layer. */
fl_status fl_net_profile(fl_net net, int which, int D, int H, int W, int reps, double* avg_ms);
fl_status fl_net_destroy(fl_net net);

/* Measurement aid: average duration (ms, HIP events on the op's stream) of
 * `reps` back-to-back launches of one pass on the op's zero-filled workspace.
 * pass: 0 row FFT forward, 1 symbol column pass (axis 0), 2 row FFT inverse,
 * 3 first sine pass, 4 scaled sine column pass, 5 last sine pass,
 * 6 whole application of M, 7 whole preconditioner.  Single passes need d >= 2. */
fl_status fl_profile_pass(fl_op op, int dtype, int pass, int reps, double* avg_ms);

/* Release every device resource of the op. */
fl_status fl_op_destroy(fl_op op);

/* Thread-local description of the last failure ("" if none). */
const char* fl_last_error(void);

/* Measurement aid: the number of device allocations (hipMalloc) the library
 * has made in this process, over all ops, nets and batches. */
int64_t fl_device_allocations(void);

#ifdef __cplusplus
}
#endif
#endif /* FRACLAP_H */
