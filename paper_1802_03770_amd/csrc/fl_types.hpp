// Descriptors shared by the host driver and the kernels.
//
// Every kernel body takes one `Prob` (a problem: one operator, one right-hand
// side) and a block index inside that problem.  A single-problem launch passes
// the Prob by value; a batched launch (many right-hand sides and/or many
// operators of uneven size) passes a device array of Probs and uses blockIdx.y
// as the problem index, blocks beyond a problem's own count exiting at once.
#pragma once
#include <stdint.h>

#include "fl_fft.hpp"

namespace fl {

// Per-axis data.  Axis 0 is the slowest (outermost) axis, axis d-1 the
// contiguous one.  n: grid points; P: padded circulant length (even);
// H = P/2 + 1 (folded / half-spectrum length).
struct Axis {
  int n, P, H;
  FFTPlan fft;      // complex FFT of length P (operator application)
  // type-I sine transform of length n by the chirp-z (Bluestein) identity:
  //   sum_{j=1..n} x_j sin(pi j k/(n+1)) = Im( ch_k sum_j (x_j ch_j) conj(ch_{k-j}) ),
  //   ch_m = e^{i pi m^2 / (2(n+1))}, convolution of length Lb >= 2n-1.
  FFTPlan dst;      // complex FFT of length Lb (chirp-z) or 2(n+1) (direct)
  int col_tplf;     // lanes per line of the specialised symbol column pass (lengths
                    // 1024, 2048): 0 = run-time plan, else 64 or 128 (autotuned)
  int dcol_tplf;    // lanes per FFT line of the sine column pass at direct length
                    // 2050: 0 = the plan's lanes, else 128 (autotuned)
  int dst_direct;   // 1: two real lines packed as x + i y in an odd extension of
                    //    length 2(n+1); FFT gives -2i S_x + 2 S_y
                    // 0: one line per FFT line by the chirp-z identity
  int dst_rader;    // 1 (with dst_direct = 1): the prime form, n + 1 = 257: two real
                    //    lines packed as x + i y, transformed by a real DFT of length
                    //    n + 1 taken by Rader's identity (FFT length 256)
  const void* chirp;  // cx<T>[n+1]; prime form: T[128] sin(pi g^-p / (n+1))
  const void* bhat;   // cx<T>[Lb]  = FFT_Lb(conj chirp, circularly placed) / Lb;
                      // prime form: cx<T>[256] = FFT_256(e^{-2 pi i g^m / (n+1)}) / 256
  const void* rtab;   // prime form: int[128] g^-p mod (n+1), int[129] log_g k
  const void* eig;    // T[n]       = 4 sin^2(pi k / (2 (n+1))), k = 1..n
};

// Device-resident scalars of one Krylov solve (always FP64).  Reductions are
// finished by their consumer: a producing kernel writes one partial per block
// into part[site * pstride + block] and its block count into cnt[site]; every
// block of the consuming kernel sums the partials in the same fixed order.
struct Scalars {
  double pq;      // p.q (reporting)
  double rr;      // r.r at stop / of the last finalised residual
  double ff;      // f.f
  double thr;     // stop when rr <= thr  (thr = tol^2 ff)
  double rr0;     // r.r at start
  double aux[3];  // finalised dot products
  int done;       // 0 running, 1 converged, 2 iteration cap, 3 breakdown
  int itc[2];     // iteration counter ring (written by parity)
  int maxit;
  int cnt[8];     // partial counts per site
  unsigned long long mhash;  // checksum of a domain mask (identifies the mask a correction was built for)
};

enum Site { S_PQ = 0, S_RR = 1, S_RZ0 = 2, S_RZ1 = 3, S_DOT = 4, S_AUX = 5, NSITE = 6 };

struct Prob {
  int d;          // 1, 2, 3
  int nrhs;       // right-hand sides of this problem stacked along the batch axis (apply only)
  Axis ax[3];
  const void* lam;  // folded symbol, T, shape [H_0][H_1]...  (P_a/2+1 per axis)
  double s0, s1;    // operator symbol is s0 + s1 * lambda  (identity shift for time steps)
  double pcs;       // C |B| h^-alpha (FD Laplacian) or 1 (sine-basis diagonal)
  double p0, p1;    // preconditioner eigenvalue p0 + p1 * pcs * (sum_a eig_a  or  tau[k])
  const void* tau;  // null: FD Laplacian eigenvalues; else the operator's own diagonal in the
                    // sine basis, T, [n_0][n_1][n_2] indexed by k_a - 1
  int pmul;         // 1: multiply by the eigenvalue instead of dividing (the operator
                    //    diagonalised by the sine transform, not its inverse)
  // buffers
  const void* in;   // real input  [nrhs][n...]
  void* out;        // real output
  const void* aux;  // second real input (residual rhs f, or p for the p.q dot)
  void* W1;         // complex work [nrhs][n_0..n_{d-2}][H_{d-1}]
  void* W2;         // complex work, 3D only: [nrhs][n_0][P_1][H_2]
  void* T1;         // real work for the sine transforms  [nrhs][n...]
  const uint8_t* mask;  // optional domain mask (1 inside), [n...]
  const void* corr;     // optional correction added to the masked input of the first sine pass, [nrhs][n...]
  int nomask_out;       // 1: the last sine pass leaves its output unmasked
  // Krylov vectors (solver launches)
  void* x;
  void* r;
  void* z;
  void* p;
  void* q;
  Scalars* sc;
  double* part;     // partial sums: NSITE sites of pstride entries
  long pstride;     // >= blocks of any reduction launch
};

}  // namespace fl
