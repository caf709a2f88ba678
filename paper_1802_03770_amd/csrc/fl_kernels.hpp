// HIP kernels for gfx950: operator construction, FFT application of the BTTB
// operator, the sine-transform (fast Poisson) preconditioner, and the fused
// Krylov vector work.  All kernel bodies act on one problem (`Prob`) and are
// wrapped twice: a single-problem kernel taking the Prob by value, and a
// batched kernel taking a device array of Probs (blockIdx.y = problem).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "fl_fft.hpp"
#include "fl_types.hpp"

namespace fl {

struct Iter {
  int parity;  // iteration parity: selects the r.z slots and the counter slot
  int first;   // first iteration: p = z, no stop test
};

// ---------------------------------------------------------------------------
// reductions (wave64 shuffle tree, then LDS across waves)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the block; the result is returned to every thread.
__device__ __forceinline__ double block_sum_all(double v) {
  __shared__ double red[16];
  __shared__ double tot;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x < 64) {
    double s = threadIdx.x < nw ? red[threadIdx.x] : 0.0;
    s = wave_sum(s);
    if (threadIdx.x == 0) tot = s;
  }
  __syncthreads();
  return tot;
}

// Producer side: block partial of site `site`; block 0 records the count.
__device__ __forceinline__ void put_partial(const Prob& pb, int site, double v, int nblk, int blk) {
  double s = block_sum_all(v);
  if (threadIdx.x == 0) {
    pb.part[site * pb.pstride + blk] = s;
    if (blk == 0) pb.sc->cnt[site] = nblk;
  }
}

// Consumer side: the grand total of a site (same fixed order in every block).
__device__ __forceinline__ double get_total(const Prob& pb, int site) {
  const int n = pb.sc->cnt[site];
  const double* p = pb.part + site * pb.pstride;
  double v = 0.0;
  // eight partials' loads in flight before they are added (same order; a
  // 256^3 pass leaves several thousand partials)
  const int st = blockDim.x;
  int i = threadIdx.x;
  for (; i + 7 * st < n; i += 8 * st) {
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = p[i + u * st];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += a[u];
  }
  for (; i < n; i += st) v += p[i];
  return block_sum_all(v);
}

__device__ __forceinline__ int fold(int k, int P) { return k <= P / 2 ? k : P - k; }

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).  Map
// block b to tile t so that the blocks one XCD runs concurrently take adjacent
// tiles (strided column passes then share 128-byte lines inside one L2).  A
// batched launch (gridDim.y problems) keeps the XCD of block b equal to b mod 8
// when gridDim.x is a multiple of 8, so the same mapping holds per problem.
__device__ __forceinline__ long xcd_tile(long b, long nb) {
  if ((gridDim.y != 1 && (gridDim.x & 7) != 0) || nb < 16) return b;
  const long q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// Rows of the real array: every index except the last axis, rhs outermost.
__device__ __forceinline__ long nrows_of(const Prob& pb) {
  long r = pb.nrhs;
  for (int a = 0; a < pb.d - 1; ++a) r *= pb.ax[a].n;
  return r;
}
__device__ __forceinline__ long nper_of(const Prob& pb) {
  long r = 1;
  for (int a = 0; a < pb.d; ++a) r *= pb.ax[a].n;
  return r;
}

#ifdef FL_MISC_KERNELS
// ---------------------------------------------------------------------------
// Operator construction (FP64)
// ---------------------------------------------------------------------------
// Upper incomplete gamma Gamma(a, x), x > 0, any real a, by Legendre's
// continued fraction evaluated with the modified Lentz method (accurate for
// x >~ 1; here x >= pi).
__device__ double upper_gamma_cf(double a, double x) {
  const double tiny = 1e-300;
  double b = x + 1.0 - a, c = 1.0 / tiny, dd = 1.0 / b, f = dd;
  for (int i = 1; i < 500; ++i) {
    double an = -i * (i - a);
    b += 2.0;
    dd = an * dd + b;
    if (fabs(dd) < tiny) dd = tiny;
    c = b + an / c;
    if (fabs(c) < tiny) c = tiny;
    dd = 1.0 / dd;
    double del = dd * c;
    f *= del;
    if (fabs(del - 1.0) < 1e-17) break;
  }
  return exp(-x + a * log(x)) * f;
}

__device__ double window_poly(double t) {
  if (t >= 1.0) return 0.0;
  double t2 = t * t, t4 = t2 * t2;
  return 1.0 + t4 * (-35.0 + t * (84.0 + t * (-70.0 + 20.0 * t)));
}

// One workgroup.  out[0..7] = C, Z, B, a2, h^{s-2}A3, omega0, omega_e, C h^-alpha.
//   C      = alpha 2^{alpha-1} Gamma((d+alpha)/2) / (pi^{d/2} Gamma(1 - alpha/2))
//   Z      = sum_{j != 0} |j|^{-(d+alpha)}  (theta split with parameter 1, |j|_inf <= 5)
//   a2     = sum_{0<|j|<c} W(|j|/c) j_1^2 |j|^{-(d+alpha)}
//   A3s    = -(1/2)(|S^{d-1}|/d) c^{2-alpha} Pw(alpha)
//   B      = a2/2 + A3s
__global__ void k_constants(int d, double alpha, double h, double c, double* out) {
  const double PI = 3.141592653589793238462643383279502884;
  const double s = d + alpha, sig = 0.5 * s;
  const int R = 5, W = 2 * R + 1;
  int tot = 1;
  for (int a = 0; a < d; ++a) tot *= W;
  double z = 0.0;
  for (int t = threadIdx.x; t < tot; t += blockDim.x) {
    int rem = t;
    double r2 = 0.0;
    for (int a = 0; a < d; ++a) {
      int j = rem % W - R;
      rem /= W;
      r2 += (double)j * j;
    }
    if (r2 == 0.0) continue;
    double q = PI * r2;
    z += pow(q, -sig) * upper_gamma_cf(sig, q) + pow(q, 0.5 * alpha) * upper_gamma_cf(-0.5 * alpha, q);
  }
  z = block_sum_all(z);
  // ball sum for a2
  const int Rc = (int)ceil(c), Wc = 2 * Rc + 1;
  int totc = 1;
  for (int a = 0; a < d; ++a) totc *= Wc;
  double a2 = 0.0;
  for (int t = threadIdx.x; t < totc; t += blockDim.x) {
    int rem = t;
    double r2 = 0.0, j1 = 0.0;
    for (int a = 0; a < d; ++a) {
      int j = rem % Wc - Rc;
      rem /= Wc;
      r2 += (double)j * j;
      if (a == 0) j1 = j;
    }
    if (r2 == 0.0) continue;
    double r = sqrt(r2);
    if (r >= c) continue;
    a2 += window_poly(r / c) * j1 * j1 * pow(r2, -0.5 * s);
  }
  a2 = block_sum_all(a2);
  if (threadIdx.x == 0) {
    double Z = (z + (2.0 / alpha) - 1.0 / sig) * pow(PI, sig) / tgamma(sig);
    double C = alpha * pow(2.0, alpha - 1.0) * tgamma(0.5 * (d + alpha)) /
               (pow(PI, 0.5 * d) * tgamma(1.0 - 0.5 * alpha));
    double area = 2.0 * pow(PI, 0.5 * d) / tgamma(0.5 * d);
    double pw = 1.0 / (2.0 - alpha) - 35.0 / (6.0 - alpha) + 84.0 / (7.0 - alpha) - 70.0 / (8.0 - alpha) +
                20.0 / (9.0 - alpha);
    double a3s = -0.5 * area / d * pow(c, 2.0 - alpha) * pw;
    double B = 0.5 * a2 + a3s;
    out[0] = C;
    out[1] = Z;
    out[2] = B;
    out[3] = a2;
    out[4] = a3s;
    out[5] = Z - 2.0 * d * B;
    out[6] = -1.0 + B;
    out[7] = C * pow(h, -alpha);
  }
}

// Folded circulant generator on [0, H_0) x ... : C h^-alpha omega_m where every
// m_a < n_a, zero elsewhere.  omega_0 = Z - 2dB, omega_{e_k} = -1 + B,
// omega_m = -|m|^{-(d+alpha)} otherwise.
__global__ void k_weights(int d, double alpha, int n0, int n1, int n2, int H0, int H1, int H2,
                          const double* cst, double* wf) {
  long tot = (long)H0 * H1 * H2;
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= tot) return;
  int m2 = i % H2, m1 = (i / H2) % H1, m0 = i / ((long)H1 * H2);
  double v = 0.0;
  if (m0 < n0 && m1 < n1 && m2 < n2) {
    long r2 = (long)m0 * m0 + (long)m1 * m1 + (long)m2 * m2;
    if (r2 == 0)
      v = cst[5];
    else if (r2 == 1)
      v = cst[6];
    else
      v = -pow((double)r2, -0.5 * (d + alpha));
    v *= cst[7];
  }
  wf[i] = v;
}

// Real-even DFT (type-I cosine transform of the folded line) along one axis
// of the folded array, in place.  Two lines are packed as x + i y, extended
// evenly to length P and transformed; x' = Re, y' = Im.  Lines along axis a:
// index = o * (H_a * inner) + m * inner + c, c in [0, inner).
// LF > 0: the compile-time FFT of that length (8192, whose line the run-time
// stages cannot hold).
template <int LF = 0>
__global__ __launch_bounds__(256) void k_dct1_axis(double* wf, int H, int P, long inner, long nlines, FFTPlan pl) {
  extern __shared__ __align__(16) char smem[];
  const int tpl = LF > 0 ? c_fixed_tpl(LF) : pl.tpl, G = blockDim.x / tpl, g = threadIdx.x / tpl,
            lane = threadIdx.x % tpl;
  Line<double> buf = line_at<double>(smem, g, P);
  long pair = (long)blockIdx.x * G + g;
  long la = 2 * pair, lb = la + 1;
  bool va = la < nlines, vb = lb < nlines;
  long ba = va ? (la / inner) * (long)H * inner + (la % inner) : 0;
  long bb = vb ? (lb / inner) * (long)H * inner + (lb % inner) : 0;
  for (int i = lane; i < P; i += tpl) {
    int m = fold(i, P);
    double xa = va ? wf[ba + (long)m * inner] : 0.0;
    double xb = vb ? wf[bb + (long)m * inner] : 0.0;
    buf[i] = {xa, xb};
  }
  __syncthreads();
  if constexpr (LF > 0)
    fft_fixed<double, LF, false>(buf, buf, (const cx<double>*)pl.tw, lane);
  else
    fft_line<double, false>(buf, pl, lane);
  for (int k = lane; k < H; k += tpl) {
    if (va) wf[ba + (long)k * inner] = buf[k].x;
    if (vb) wf[bb + (long)k * inner] = buf[k].y;
  }
}

// ---------------------------------------------------------------------------
// Sine-basis diagonal of the operator (FP64): m_k = sum_m w_m prod_a G_a(k_a, m_a)
// ---------------------------------------------------------------------------
// G(k, m) = c_m sum_{i=1}^{n-m} q_k(i) q_k(i+m) with the orthonormal sine
// vectors q_k, in closed form; row k-1, column m; c_0 = 1, c_m = 2.
__global__ void k_sine_corr(double* G, int n) {
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)n * n) return;
  const int k = (int)(idx / n) + 1, m = (int)(idx % n);
  const double th = M_PI * k / (n + 1);
  const double sgn = (k & 1) ? -1.0 : 1.0;  // cos((n+1) theta) = (-1)^k
  const double sm = 0.5 * ((n - m) * cos(m * th) - sgn * sin((n - m) * th) / sin(th));
  G[idx] = (2.0 / (n + 1)) * sm * (m == 0 ? 1.0 : 2.0);
}

// X[i0][i1][i2] = wf[i0][i1][i2] on the n-block of the folded [H0][H1][H2] weights.
__global__ void k_weight_block(const double* wf, double* X, int n0, int n1, int n2, int H1, int H2) {
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long N = (long)n0 * n1 * n2;
  if (idx >= N) return;
  const int i2 = (int)(idx % n2);
  const long t = idx / n2;
  const int i1 = (int)(t % n1), i0 = (int)(t / n1);
  X[idx] = wf[((long)i0 * H1 + i1) * H2 + i2];
}

// Strided batched FP64 product C_b[i][j] = sum_m A_b[i][m] B_b[m][j] (64 x 64
// output tile per block, fixed summation order).
__global__ __launch_bounds__(256) void k_gemm_f64(int M, int N, int K, const double* A, long sai, long sam, long sab,
                                                  const double* B, long sbm, long sbj, long sbb, double* C, long sci,
                                                  long scj, long scb) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  A += blockIdx.z * sab;
  B += blockIdx.z * sbb;
  C += blockIdx.z * scb;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int r = e / 16, ka = e % 16;
      As[ka][r] = (i0 + r < M && k0 + ka < K) ? A[(long)(i0 + r) * sai + (long)(k0 + ka) * sam] : 0.0;
      const int c = e % 64, kb = e / 64;
      Bs[kb][c] = (k0 + kb < K && j0 + c < N) ? B[(long)(k0 + kb) * sbm + (long)(j0 + c) * sbj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][ty + 16 * q];
        b[q] = Bs[kk][tx + 16 * q];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = fma(a[p], b[q], acc[p][q]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + ty + 16 * p, j = j0 + tx + 16 * q;
      if (i < M && j < N) C[(long)i * sci + (long)j * scj] = acc[p][q];
    }
}
#endif  // FL_MISC_KERNELS

template <typename TO, typename TI>
__global__ void k_cast(const TI* in, TO* out, long n, double scale) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) out[i] = (TO)((double)in[i] * scale);
}

// ---------------------------------------------------------------------------
// Krylov bookkeeping shared by the first kernel of every iteration
// ---------------------------------------------------------------------------
// Stop test of iteration k (k >= 1) on the r.r left by iteration k-1's update,
// and beta = rz_k / rz_{k-1}.  Returns true when the solve is over; block 0
// records the status.  Every block takes the same decision (same sums).
__device__ __forceinline__ bool iter_head(const Prob& pb, const Iter& it, int blk, double* beta) {
  *beta = 0.0;
  if (it.first) return false;
  Scalars* sc = pb.sc;
  const double rr = get_total(pb, S_RR);
  const int itn = sc->itc[it.parity ^ 1] + 1;  // updates completed so far
  int st = 0;
  if (!isfinite(rr)) st = 3;
  else if (rr <= sc->thr) st = 1;
  else if (itn >= sc->maxit) st = 2;
  if (blk == 0 && threadIdx.x == 0) {
    sc->itc[it.parity] = itn;
    sc->rr = rr;
    if (st) sc->done = st;
  }
  if (st) return true;
  const double rzn = get_total(pb, S_RZ0 + it.parity), rzo = get_total(pb, S_RZ0 + (it.parity ^ 1));
  *beta = rzn / rzo;
  return false;
}

// ---------------------------------------------------------------------------
// Operator application: forward row pass (last axis, real -> half spectrum)
// ---------------------------------------------------------------------------
enum { PRO_PLAIN = 0, PRO_PUPD = 1 };
enum { EPI_PLAIN = 0, EPI_RESID = 1, EPI_PQ = 2 };

// Prologue value of the operator input at element e (row-major over the
// stacked arrays).  PUPD: p <- z + beta p, stored.
template <typename T, int PRO>
__device__ __forceinline__ T load_input(const Prob& pb, long e, long nper, double beta, bool first) {
  if (PRO == PRO_PUPD) {
    T zv = ((const T*)pb.z)[e];
    T pv = first ? zv : (T)(zv + (T)beta * ((T*)pb.p)[e]);
    ((T*)pb.p)[e] = pv;
    return pv;
  } else {
    T v = ((const T*)pb.in)[e];
    if (pb.mask) v *= (T)pb.mask[e % nper];
    return v;
  }
}

// Roots of unity of a compile-time length L copied to LDS by the whole block
// when they take at most 8 KB (lengths up to 1024 in FP32, 512 in FP64), so
// the FFT stages read them without a round trip to memory; else the table in
// memory.  Readable after the caller's next barrier.  Larger tables would cost
// the long lines an occupancy step, and at 1024^2 the passes measured no gain.
template <typename T, int L> __host__ __device__ constexpr bool tw_in_lds() {
  return L > 0 && L * (int)sizeof(cx<T>) <= 8192;
}
template <typename T, int L>
__device__ __forceinline__ const cx<T>* tw_stage(const cx<T>* tw) {
  __shared__ cx<T> t[tw_in_lds<T, L>() ? L : 1];
  if constexpr (tw_in_lds<T, L>()) {
    for (int m = threadIdx.x; m < L; m += blockDim.x) t[m] = tw[m];
    return t;
  } else {
    return tw;
  }
}

// Staging loops load a chunk of a thread's elements into registers before
// writing any of them to LDS: a load consumed in its own loop iteration makes
// the wavefront wait for it before the next is issued, which serialised the
// memory round trips of a line.
constexpr int kStageChunk = 8;

// Row line FFT: LF = 0 follows the run-time plan; LF > 0 is a kernel
// specialised for that padded length (lanes c_fixed_tpl(LF)).  Padded lengths
// are at least twice the grid's: the forward transform's input is zero from
// LF/2 on (ZIN) and the inverse's output is cropped below LF/2 (ZOUT), which
// the specialised kernels use to skip that half at the first (last) stage.
template <typename T, bool INV, int LF, bool ZIN = false, bool ZOUT = false>
__device__ __forceinline__ void row_fft(Line<T> buf, const FFTPlan& pl, const cx<T>* tw, int lane) {
  if constexpr (LF > 0) fft_fixed<T, LF, INV, ZIN, ZOUT>(buf, buf, tw, lane);
  else fft_line<T, INV>(buf, pl, lane);
}

// Entries of a zero-padded line of compile-time length LF that are staged in
// LDS: the lower half when the first stage skips the upper one.
__host__ __device__ constexpr int c_staged_len(int LF) { return LF > 0 && c_zin_pruned(LF) ? LF / 2 : LF; }
// Elements of a row line per lane and chunk: no more than the staged part holds.
__host__ __device__ constexpr int c_row_chunk(int LF) {
  return (c_staged_len(LF) + c_fixed_tpl(LF) - 1) / c_fixed_tpl(LF) < kStageChunk
             ? (c_staged_len(LF) + c_fixed_tpl(LF) - 1) / c_fixed_tpl(LF) : kStageChunk;
}

template <typename T, int PRO, int LF = 0>
__device__ __forceinline__ void rowfwd_body(const Prob& pb, const Iter& it, int blk) {
  double beta = 0.0;
  if (PRO == PRO_PUPD) {
    if (pb.sc->done) return;
    if (iter_head(pb, it, blk, &beta)) return;
  }
  extern __shared__ __align__(16) char smem[];
  const Axis& A = pb.ax[pb.d - 1];
  const int n = A.n, P = LF > 0 ? LF : A.P, H = A.H, tpl = LF > 0 ? c_fixed_tpl(LF) : A.fft.tpl;
  const int G = blockDim.x / tpl, g = threadIdx.x / tpl, lane = threadIdx.x % tpl;
  Line<T> buf = line_at<T>(smem, g, P);
  const long rows = nrows_of(pb), nper = nper_of(pb);
  const long ra = 2 * ((long)blk * G + g), rb = ra + 1;
  const bool va = ra < rows, vb = rb < rows;
  const cx<T>* tw = tw_stage<T, LF>((const cx<T>*)A.fft.tw);
  // entries staged: all P, or the lower half that the pruned first stage reads
  // (n <= P/2 either way, so the direction update still covers every entry)
  const int PS = LF > 0 ? c_staged_len(LF) : P;
  constexpr int CH = LF > 0 ? c_row_chunk(LF) : kStageChunk;
  // A chunk of a thread's elements of rows a and b: every load first (z and
  // p of the direction update, or the input with its mask), then the
  // arithmetic, the update's stores and the LDS writes.
  for (int i0 = lane; i0 < PS; i0 += CH * tpl) {
    T v[2][CH];
    if (PRO == PRO_PUPD) {
      const T* z = (const T*)pb.z;
      T* p = (T*)pb.p;
      T zs[2][CH], ps[2][CH];
#pragma unroll
      for (int u = 0; u < CH; ++u)
#pragma unroll
        for (int sr = 0; sr < 2; ++sr) {
          const int i = i0 + u * tpl;
          const bool ok = (sr ? vb : va) && i < n;
          const long e = ok ? (sr ? rb : ra) * n + i : 0;  // clamped: unconditional loads
          const T zv = z[e], pv = p[e];
          zs[sr][u] = ok ? zv : (T)0;
          ps[sr][u] = (ok && !it.first) ? pv : (T)0;
        }
#pragma unroll
      for (int u = 0; u < CH; ++u)
#pragma unroll
        for (int sr = 0; sr < 2; ++sr) {
          const int i = i0 + u * tpl;
          const bool ok = (sr ? vb : va) && i < n;
          const T pv = it.first ? zs[sr][u] : (T)(zs[sr][u] + (T)beta * ps[sr][u]);
          if (ok) p[(sr ? rb : ra) * n + i] = pv;
          v[sr][u] = ok ? pv : (T)0;
        }
    } else {
      const T* in = (const T*)pb.in;
#pragma unroll
      for (int u = 0; u < CH; ++u)
#pragma unroll
        for (int sr = 0; sr < 2; ++sr) {
          const int i = i0 + u * tpl;
          const bool ok = (sr ? vb : va) && i < n;
          const T t = in[ok ? (sr ? rb : ra) * n + i : 0];  // clamped: unconditional load
          v[sr][u] = ok ? t : (T)0;
        }
      if (pb.mask) {
        T ms[2][CH];
#pragma unroll
        for (int u = 0; u < CH; ++u)
#pragma unroll
          for (int sr = 0; sr < 2; ++sr) {
            const int i = i0 + u * tpl;
            const bool ok = (sr ? vb : va) && i < n;
            ms[sr][u] = ok ? (T)pb.mask[((sr ? rb : ra) * n + i) % nper] : (T)0;
          }
#pragma unroll
        for (int u = 0; u < CH; ++u)
#pragma unroll
          for (int sr = 0; sr < 2; ++sr) v[sr][u] *= ms[sr][u];
      }
    }
#pragma unroll
    for (int u = 0; u < CH; ++u)
      if (i0 + u * tpl < PS) buf[i0 + u * tpl] = {v[0][u], v[1][u]};
  }
  __syncthreads();
  row_fft<T, false, LF, true, false>(buf, A.fft, tw, lane);
  cx<T>* W = (cx<T>*)pb.W1;
  for (int k = lane; k < H; k += tpl) {
    cx<T> zk = buf[k], zm = buf[(P - k) % P];
    // X_a = (Z_k + conj Z_{P-k})/2 ; X_b = -i (Z_k - conj Z_{P-k})/2
    cx<T> xa = {(T)0.5 * (zk.x + zm.x), (T)0.5 * (zk.y - zm.y)};
    cx<T> xb = {(T)0.5 * (zk.y + zm.y), (T)0.5 * (zm.x - zk.x)};
    if (va) W[ra * H + k] = xa;
    if (vb) W[rb * H + k] = xb;
  }
}

// Strided complex line pass.  Lines c = c0 + j (j < G) of group grp; element i
// of a line is at base + grp*gstride + i*estride + c.
struct ColGeom {
  int axis;      // transformed axis
  int nin, nout; // elements loaded / stored per line
  long gs;       // lines per group (adjacent in memory)
  long ngroup;   // number of groups (outer index incl. rhs)
  long ein, gin, eout, gout;
  int src, dst;  // 1 = W1, 2 = W2
};

enum { COL_FWD = 0, COL_CONV = 1, COL_INV = 2 };

// Lanes per column of the single-problem FP32 3D column passes at 512 points:
// 32, i.e. eight adjacent columns per workgroup (64-byte rows; the axis-0
// convolution at 256^3 took 245 us against 285 us with 64 lanes).  2D grids of
// that length have too few columns for it, FP64 too many registers, and the
// batched launches, whose grids hold every problem's blocks, measured faster
// with the plan's 64.
constexpr int kCol3DLanes512 = 32;

// Column line FFT: LF = 0 follows the run-time plan; LF > 0 is a kernel
// specialised for that length with TPLF lanes per line (fewer lanes than the
// row passes use, so that a block holds several adjacent columns).  ZIN/ZOUT
// as for the rows: a transform of a zero-padded column skips the upper half of
// its input, one whose output is cropped to the grid skips that of its output.
template <typename T, bool INV, int LF, int TPLF, bool ZIN = false, bool ZOUT = false>
__device__ __forceinline__ void col_fft(Line<T> buf, const FFTPlan& pl, const cx<T>* tw, int lane) {
  if constexpr (LF > 0)
    cstages<T, LF, TPLF, INV, 0, 1, ZIN, ZOUT>(buf, buf, tw, lane);
  else
    fft_line<T, INV>(buf, pl, lane);
}

template <typename T, int MODE, int LF = 0, int TPLF = 0>
__device__ __forceinline__ void colpass_body(const Prob& pb, const ColGeom& cg, const Iter& it, bool check_done,
                                             int blk0, int nblk) {
  if (check_done && pb.sc->done) return;
  const long blk = xcd_tile(blk0, nblk);
  extern __shared__ __align__(16) char smem[];
  const Axis& A = pb.ax[cg.axis];
  const int L = LF > 0 ? LF : A.P, tpl = LF > 0 ? TPLF : A.fft.tpl;
  const int G = blockDim.x / tpl, g = threadIdx.x / tpl, lane = threadIdx.x % tpl;
  const long tiles = (cg.gs + G - 1) / G;
  const long grp = blk / tiles, c0 = (blk % tiles) * G;
  if (grp >= cg.ngroup) return;  // uniform across the block
  const cx<T>* src = (const cx<T>*)(cg.src == 1 ? pb.W1 : pb.W2) + grp * cg.gin + c0;
  cx<T>* dst = (cx<T>*)(cg.dst == 1 ? pb.W1 : pb.W2) + grp * cg.gout + c0;
  const int gv = (int)min((long)G, cg.gs - c0);  // valid lines in this tile
  // Coalesced staging: consecutive threads take consecutive lines of one
  // element row.  With G * tpl threads, thread t always serves line t % G
  // and elements t / G + m tpl, so the strided loops below step a pointer
  // and a 32-bit index instead of dividing a flat index every element.
  const int jt = threadIdx.x % G, i0 = threadIdx.x / G;
  const bool jv = jt < gv;
  Line<T> lnt = line_at<T>(smem, jt, L);
  const cx<T>* tw = tw_stage<T, LF>((const cx<T>*)A.fft.tw);  // read after the barrier below
  // Symbol values of this thread's line and frequencies k = i0 + q tpl: for
  // the compile-time lengths up to 1024 (at most 8 per thread) they are
  // loaded here, with the line itself, so that one round trip serves both.
  constexpr int NPF = (MODE == COL_CONV && LF > 0 && LF <= 1024 && TPLF > 0 && LF / TPLF <= (sizeof(T) == 4 ? 16 : 8))
                          ? LF / TPLF : 0;
  const T* lt = nullptr;
  long tailsz = 0;
  T lpf[NPF > 0 ? NPF : 1];
  if (MODE == COL_CONV) {
    tailsz = (pb.d == 2) ? pb.ax[1].H : (long)pb.ax[1].H * pb.ax[2].H;
    const long c = c0 + jt;
    long tail = c;  // index contribution of the axes after axis 0
    if (pb.d != 2) {
      const int H2 = pb.ax[2].H, P1 = pb.ax[1].P;
      tail = (long)fold((int)(c / H2), P1) * H2 + c % H2;
    }
    lt = (const T*)pb.lam + tail;
    if constexpr (NPF > 0) {
      if (jv) {
#pragma unroll
        for (int q = 0; q < NPF; ++q) lpf[q] = lt[(long)fold(i0 + q * TPLF, LF) * tailsz];
      }
    }
  }
  {
    // The forward transforms of COL_FWD and COL_CONV take a zero-padded column
    // (nin <= L/2): with a pruned first stage only its lower half is staged.
    constexpr bool ZS = MODE != COL_INV && LF > 0 && c_zin_pruned(LF);
    constexpr int LS = ZS ? LF / 2 : LF;
    const int Ls = LF > 0 ? LS : L;
    const cx<T>* sp = src + (long)i0 * cg.ein + jt;
    const long sst = (long)tpl * cg.ein;
    const int nin = cg.nin;
    constexpr int CH = (LF > 0 && TPLF > 0 && LF / TPLF <= 16) ? (LS + TPLF - 1) / TPLF : kStageChunk;
    for (int i = i0; i < Ls; i += CH * tpl, sp += CH * sst) {
      cx<T> v[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        v[u] = {0, 0};
        if (i + u * tpl < nin && jv) v[u] = sp[u * sst];
      }
#pragma unroll
      for (int u = 0; u < CH; ++u)
        if (i + u * tpl < Ls) lnt[i + u * tpl] = v[u];
    }
  }
  __syncthreads();
  Line<T> buf = line_at<T>(smem, g, L);
  col_fft<T, MODE == COL_INV, LF, TPLF, MODE != COL_INV, MODE == COL_INV>(buf, A.fft, tw, lane);
  if (MODE == COL_CONV) {
    // symbol s0 + s1 lambda on the folded octant, times 1/prod(P); consecutive
    // threads take consecutive lines of one frequency (adjacent symbol entries)
    double norm = 1.0;
    for (int a = 0; a < pb.d; ++a) norm *= pb.ax[a].P;
    const T s0 = (T)(pb.s0 / norm), s1 = (T)(pb.s1 / norm);
    if (jv) {
      if constexpr (NPF > 0) {
#pragma unroll
        for (int q = 0; q < NPF; ++q) {
          const int k = i0 + q * TPLF;
          lnt[k] = cscale(lnt[k], s0 + s1 * lpf[q]);
        }
      } else {
        // a chunk's symbol values loaded before any of them is used
        for (int k0 = i0; k0 < L; k0 += kStageChunk * tpl) {
          T lv[kStageChunk];
#pragma unroll
          for (int u = 0; u < kStageChunk; ++u) {
            const int k = k0 + u * tpl;
            lv[u] = k < L ? lt[(long)fold(k, L) * tailsz] : (T)0;
          }
#pragma unroll
          for (int u = 0; u < kStageChunk; ++u) {
            const int k = k0 + u * tpl;
            if (k < L) lnt[k] = cscale(lnt[k], s0 + s1 * lv[u]);
          }
        }
      }
    }
    __syncthreads();
    col_fft<T, true, LF, TPLF, false, true>(buf, A.fft, tw, lane);
  }
  if (jv) {
    cx<T>* dp = dst + (long)i0 * cg.eout + jt;
    const long dst_step = (long)tpl * cg.eout;
    for (int i = i0; i < cg.nout; i += tpl, dp += dst_step) *dp = lnt[i];
  }
}

// Inverse row pass: half spectrum -> real rows, crop to n, epilogue.
//  EPI_PLAIN: out = y;  EPI_RESID: out = aux - y, |out|^2 partials (site S_DOT);
//  EPI_PQ: q = y, p.q partials (site S_PQ).
template <typename T, int EPI, int LF = 0>
__device__ __forceinline__ void rowinv_body(const Prob& pb, const Iter& it, bool check_done, int nblk, int blk) {
  if (check_done && pb.sc->done) return;
  extern __shared__ __align__(16) char smem[];
  const Axis& A = pb.ax[pb.d - 1];
  const int n = A.n, P = LF > 0 ? LF : A.P, H = A.H, tpl = LF > 0 ? c_fixed_tpl(LF) : A.fft.tpl;
  const int G = blockDim.x / tpl, g = threadIdx.x / tpl, lane = threadIdx.x % tpl;
  Line<T> buf = line_at<T>(smem, g, P);
  const long rows = nrows_of(pb), nper = nper_of(pb);
  const long ra = 2 * ((long)blk * G + g), rb = ra + 1;
  const bool va = ra < rows, vb = rb < rows;
  const cx<T>* W = (const cx<T>*)pb.W1;
  const cx<T>* tw = tw_stage<T, LF>((const cx<T>*)A.fft.tw);
  for (int k0 = lane; k0 < P; k0 += kStageChunk * tpl) {
    cx<T> xa[kStageChunk], xb[kStageChunk];
#pragma unroll
    for (int u = 0; u < kStageChunk; ++u) {
      const int k = k0 + u * tpl, kk = k < H ? k : P - k;
      xa[u] = {0, 0};
      xb[u] = {0, 0};
      if (k < P) {
        if (va) xa[u] = W[ra * H + kk];
        if (vb) xb[u] = W[rb * H + kk];
      }
    }
#pragma unroll
    for (int u = 0; u < kStageChunk; ++u) {
      const int k = k0 + u * tpl, kk = k < H ? k : P - k;
      if (k >= P) continue;
      cx<T> a = xa[u], b = xb[u];
      if (kk == 0 || 2 * kk == P) { a.y = 0; b.y = 0; }
      if (k >= H) { a.y = -a.y; b.y = -b.y; }
      buf[k] = {a.x - b.y, a.y + b.x};
    }
  }
  __syncthreads();
  row_fft<T, true, LF, false, true>(buf, A.fft, tw, lane);
  double acc = 0.0;
  // per chunk: the epilogue's loads (aux or p, mask) first, then the stores
  for (int i0 = lane; i0 < n; i0 += kStageChunk * tpl) {
    // unconditional loads from clamped in-range indices, then a select
    T ld[2][kStageChunk], ms[2][kStageChunk];
    if (EPI != EPI_PLAIN) {
      const T* src = EPI == EPI_RESID ? (const T*)pb.aux : (const T*)pb.p;
#pragma unroll
      for (int u = 0; u < kStageChunk; ++u)
#pragma unroll
        for (int sr = 0; sr < 2; ++sr) {
          const int i = i0 + u * tpl;
          const bool ok = (sr ? vb : va) && i < n;
          const T t = src[ok ? (sr ? rb : ra) * n + i : 0];
          ld[sr][u] = ok ? t : (T)0;
        }
    }
    if (pb.mask) {
#pragma unroll
      for (int u = 0; u < kStageChunk; ++u)
#pragma unroll
        for (int sr = 0; sr < 2; ++sr) {
          const int i = i0 + u * tpl;
          const bool ok = (sr ? vb : va) && i < n;
          const T t = (T)pb.mask[ok ? ((sr ? rb : ra) * n + i) % nper : 0];
          ms[sr][u] = ok ? t : (T)1;
        }
    }
#pragma unroll
    for (int u = 0; u < kStageChunk; ++u) {
      const int i = i0 + u * tpl;
      if (i >= n) continue;
      const cx<T> y = buf[i];
#pragma unroll
      for (int sr = 0; sr < 2; ++sr) {
        if (!(sr ? vb : va)) continue;
        const long e = (sr ? rb : ra) * n + i;
        T v = sr ? y.y : y.x;
        if (pb.mask) v *= ms[sr][u];
        if (EPI == EPI_PLAIN) {
          ((T*)pb.out)[e] = v;
        } else if (EPI == EPI_RESID) {
          const T rv = ld[sr][u] - v;
          ((T*)pb.out)[e] = rv;
          acc += (double)rv * (double)rv;
        } else {  // EPI_PQ: q = M p, accumulate p.q
          ((T*)pb.q)[e] = v;
          acc += (double)ld[sr][u] * (double)v;
        }
      }
    }
  }
  if (EPI == EPI_RESID) put_partial(pb, S_DOT, acc, nblk, blk);
  if (EPI == EPI_PQ) put_partial(pb, S_PQ, acc, nblk, blk);
}

// 1D: whole convolution of two packed lines in one pass (real symbol keeps
// x + i y separable: conv(x) = Re, conv(y) = Im).
template <typename T, int PRO, int EPI>
__device__ __forceinline__ void conv1d_body(const Prob& pb, const Iter& it, int nblk, int blk) {
  double beta = 0.0;
  if (PRO == PRO_PUPD) {
    if (pb.sc->done) return;
    if (iter_head(pb, it, blk, &beta)) return;
  }
  extern __shared__ __align__(16) char smem[];
  const Axis& A = pb.ax[0];
  const int n = A.n, P = A.P, tpl = A.fft.tpl;
  const int G = blockDim.x / tpl, g = threadIdx.x / tpl, lane = threadIdx.x % tpl;
  Line<T> buf = line_at<T>(smem, g, P);
  const long rows = pb.nrhs, nper = n;
  const long ra = 2 * ((long)blk * G + g), rb = ra + 1;
  const bool va = ra < rows, vb = rb < rows;
  for (int i = lane; i < P; i += tpl) {
    T xa = 0, xb = 0;
    if (i < n) {
      if (va) xa = load_input<T, PRO>(pb, ra * n + i, nper, beta, it.first);
      if (vb) xb = load_input<T, PRO>(pb, rb * n + i, nper, beta, it.first);
    }
    buf[i] = {xa, xb};
  }
  __syncthreads();
  fft_line<T, false>(buf, A.fft, lane);
  {
    const T* lam = (const T*)pb.lam;
    const T s0 = (T)(pb.s0 / P), s1 = (T)(pb.s1 / P);
    for (int k = lane; k < P; k += tpl) buf[k] = cscale(buf[k], s0 + s1 * lam[fold(k, P)]);
  }
  __syncthreads();
  fft_line<T, true>(buf, A.fft, lane);
  double acc = 0.0;
  for (int i = lane; i < n; i += tpl) {
    cx<T> y = buf[i];
    for (int s = 0; s < 2; ++s) {
      if (!(s ? vb : va)) continue;
      long e = (s ? rb : ra) * n + i;
      T v = s ? y.y : y.x;
      if (pb.mask) v *= (T)pb.mask[e % nper];
      if (EPI == EPI_PLAIN) {
        ((T*)pb.out)[e] = v;
      } else if (EPI == EPI_RESID) {
        T rv = ((const T*)pb.aux)[e] - v;
        ((T*)pb.out)[e] = rv;
        acc += (double)rv * (double)rv;
      } else {
        ((T*)pb.q)[e] = v;
        acc += (double)((const T*)pb.p)[e] * (double)v;
      }
    }
  }
  if (EPI == EPI_RESID) put_partial(pb, S_DOT, acc, nblk, blk);
  if (EPI == EPI_PQ) put_partial(pb, S_PQ, acc, nblk, blk);
}

// ---------------------------------------------------------------------------
// Sine transforms (type I)
// ---------------------------------------------------------------------------
// Chirp-z form, one real line per FFT line.  In: buf[j].x = x_j (j < n).
// Out: buf[k].x = sum_j x_j sin(pi (j+1)(k+1)/(n+1)).  CL > 0: the FFT length
// is the compile-time CL (lanes c_fixed_tpl(CL)), else the run-time plan.
template <typename T, int CL = 0>
__device__ __forceinline__ void dst_line(Line<T> buf, const Axis& A, int lane, int tpl) {
  const int n = A.n, Lb = CL > 0 ? CL : A.dst.L;
  const cx<T>* ch = (const cx<T>*)A.chirp;
  const cx<T>* bh = (const cx<T>*)A.bhat;
  for (int j = lane; j < Lb; j += tpl) {
    cx<T> v = {0, 0};
    if (j < n) v = cscale(ch[j + 1], buf[j].x);
    buf[j] = v;
  }
  __syncthreads();
  if constexpr (CL > 0) fft_fixed<T, CL, false>(buf, buf, (const cx<T>*)A.dst.tw, lane);
  else fft_line<T, false>(buf, A.dst, lane);
  for (int k = lane; k < Lb; k += tpl) buf[k] = cmul(buf[k], bh[k]);
  __syncthreads();
  if constexpr (CL > 0) fft_fixed<T, CL, true>(buf, buf, (const cx<T>*)A.dst.tw, lane);
  else fft_line<T, true>(buf, A.dst, lane);
  for (int k = lane; k < n; k += tpl) {
    cx<T> y = cmul(ch[k + 1], buf[k]);
    buf[k] = {y.y, 0};
  }
  __syncthreads();
}

// Direct form of a packed pair: the line holds the odd extension
// (0, x_1.., x_n, 0, -x_n.., -x_1) of x_a + i x_b, length M = 2(n+1).  After the
// FFT, S_a[k] = -Im Z_k / 2 and S_b[k] = Re Z_k / 2 for k = 1..n.
template <typename T>
__device__ __forceinline__ void sine_pair_put(Line<T> buf, int M, int k, T a, T b) {
  buf[k] = {a, b};
  buf[M - k] = {-a, -b};
}
template <typename T>
__device__ __forceinline__ cx<T> sine_pair_get(Line<T> buf, int k) {
  cx<T> z = buf[k];
  return {(T)-0.5 * z.y, (T)0.5 * z.x};
}

// Sine-transform line FFT: LF = 0 follows the run-time plan (any direct or
// chirp-z form); LF > 0 is a kernel specialised for the direct form of that
// length, which then contains no other path (and no other register demand);
// LF < 0 is a kernel specialised for the chirp-z form with FFT length -LF,
// which never takes the direct form.
template <typename T, bool INV, int LF, int TPLF = 0>
__device__ __forceinline__ Line<T> dst_fft(Line<T> a, Line<T> b, const FFTPlan& pl, int lane) {
  if constexpr (LF > 0) {
    cstages<T, LF, (TPLF > 0 ? TPLF : c_fixed_tpl(LF)), INV, 0, 1>(a, b, (const cx<T>*)pl.tw, lane);
    return a;
  } else if constexpr (LF < 0) {
    return a;
  } else {
    return fft_line_wide<T, INV>(a, b, pl, lane);
  }
}

// Length code of the prime form's kernels (N = n + 1 = 257, FFT length 256);
// odd, so it never equals a direct length 2(n+1).
constexpr int kRaderLF = 257;

// Elements per chunk of a sine pass's staging loop: a thread's whole share
// where the length is compile-time (n = LF/2 - 1 direct, 256 prime form; per
// thread n / lanes in a row pass, 2n / lanes in a column pass, whose lanes hold
// two columns), at most CMAX; 4 otherwise.
__host__ __device__ constexpr int dst_chunk(int LF, int lanes, bool cols, int CMAX) {
  const int n = LF == 257 ? 256 : (LF > 0 ? LF / 2 - 1 : 0);
  if (n == 0 || lanes == 0) return CMAX < 4 ? CMAX : 4;
  const int c = ((cols ? 2 * n : n) + lanes - 1) / lanes;
  return c < 1 ? 1 : (c > CMAX ? CMAX : c);
}

// Transform of a packed pair in either two-line form: the prime form when
// LF == kRaderLF (result in a), else the direct odd extension.
template <typename T> using RaderPF = RaderRegs<T, kRaderLF - 1>;
template <typename T, int LF, int TPLF = 0>
__device__ __forceinline__ Line<T> dst_pair(Line<T> a, Line<T> b, const Axis& A, const cx<T>* tw,
                                            const RaderPF<T>& rr, int lane) {
  if constexpr (LF == kRaderLF) {
    rader_sine<T, kRaderLF - 1>(a, b, A.n, rr, tw, lane);
    return a;
  } else {
    return dst_fft<T, false, LF, TPLF>(a, b, A.dst, lane);
  }
}
// Element k (1..n) of a packed pair: in place in the prime form, through the
// odd extension in the direct form.
template <typename T, bool RAD>
__device__ __forceinline__ void pair_put(Line<T> buf, int M, int k, T a, T b) {
  if constexpr (RAD) buf[k] = {a, b};
  else sine_pair_put(buf, M, k, a, b);
}
template <typename T, bool RAD>
__device__ __forceinline__ cx<T> pair_get(Line<T> buf, int k) {
  if constexpr (RAD) return buf[k];
  else return sine_pair_get(buf, k);
}

enum { DPRO_PLAIN = 0, DPRO_UPD = 1 };
enum { DEPI_STORE = 0, DEPI_FINAL = 1, DEPI_Z = 2 };

// Row sine pass along the last axis.  d == 1 performs the whole inverse
// (transform, divide by the eigenvalue, transform, normalise) in this pass.
//  DPRO_UPD: alpha = rz/pq; x += alpha p, r -= alpha q; r.r partials (S_RR);
//            the new r is transformed.
//  DEPI_STORE: out = result (a first pass of a multi-axis transform)
//  DEPI_FINAL: out = norm * result
//  DEPI_Z:     z = norm * result, r.z partials into slot parity ^ 1.
template <typename T, int DPRO, int DEPI, int LF = 0>
__device__ __forceinline__ void dst_rows_body(const Prob& pb, const Iter& it, bool check_done, int nblk, int blk) {
  if (check_done && pb.sc->done) return;
  double alpha = 0.0;
  if (DPRO == DPRO_UPD) {
    const double pq = get_total(pb, S_PQ);
    if (!(pq > 0.0) || !isfinite(pq)) {  // breakdown: every block sees the same pq
      if (blk == 0 && threadIdx.x == 0) {
        pb.sc->pq = pq;
        pb.sc->done = 3;
      }
      return;
    }
    alpha = get_total(pb, S_RZ0 + it.parity) / pq;
  }
  extern __shared__ __align__(16) char smem[];
  const Axis& A = pb.ax[pb.d - 1];
  constexpr int CL = LF < 0 ? -LF : 0;  // chirp-z FFT length of a chirp specialisation
  constexpr bool RAD = LF == kRaderLF;   // prime form
  const int n = A.n, Lf = RAD ? kRaderLF - 1 : (CL > 0 ? CL : A.dst.L);
  const int tpl = RAD ? c_fixed_tpl(kRaderLF - 1) : (CL > 0 ? c_fixed_tpl(CL) : A.dst.tpl);
  const bool direct = LF > 0 ? true : (LF < 0 ? false : A.dst_direct);
  const int G = blockDim.x / tpl, g = threadIdx.x / tpl, lane = threadIdx.x % tpl;
  const cx<T>* dtw = (const cx<T>*)A.dst.tw;  // prime form: staged in LDS, read after the next barrier
  RaderPF<T> rr;                               // prime form: this lane's table entries
  if constexpr (RAD) {
    dtw = tw_stage<T, kRaderLF - 1>(dtw);
    rader_load(rr, (const int*)A.rtab, (const T*)A.chirp, (const cx<T>*)A.bhat, lane);
  }
  // direct: a ping-pong pair of lines per FFT line
  Line<T> buf = line_at<T>(smem, direct ? 2 * g : g, Lf);
  Line<T> buf2 = line_at<T>(smem, 2 * g + 1, Lf);
  const long rows = nrows_of(pb), nper = nper_of(pb);
  const long ra = ((long)blk * G + g) * (direct ? 2 : 1), rb = ra + 1;
  const bool va = ra < rows, vb = direct && rb < rows;
  double acc = 0.0;
  // A chunk of a thread's elements (rows a and b of the pair): every load
  // first (x, p, r, q of the update, or the input with its mask and
  // correction), then the arithmetic, the update's stores and the LDS writes.
  constexpr int CK = dst_chunk(LF, RAD ? c_fixed_tpl(kRaderLF - 1) : (LF > 0 ? c_fixed_tpl(LF) : 0), false,
                               DPRO == DPRO_UPD ? 4 : 8);
  for (int i0 = lane; i0 < n; i0 += CK * tpl) {
    T v[2][CK];
    if (DPRO == DPRO_UPD) {
      T* x = (T*)pb.x;
      T* r = (T*)pb.r;
      const T* p = (const T*)pb.p;
      const T* q = (const T*)pb.q;
      T xs[2][CK], ps[2][CK], rs[2][CK], qs[2][CK];
#pragma unroll
      for (int u = 0; u < CK; ++u)
#pragma unroll
        for (int sr = 0; sr < 2; ++sr) {
          const int i = i0 + u * tpl;
          const bool ok = (sr ? vb : va) && i < n;
          const long e = ok ? (sr ? rb : ra) * n + i : 0;  // clamped: unconditional loads
          const T xv = x[e], pv = p[e], rv = r[e], qv = q[e];
          xs[sr][u] = ok ? xv : (T)0;
          ps[sr][u] = ok ? pv : (T)0;
          rs[sr][u] = ok ? rv : (T)0;
          qs[sr][u] = ok ? qv : (T)0;
        }
#pragma unroll
      for (int u = 0; u < CK; ++u)
#pragma unroll
        for (int sr = 0; sr < 2; ++sr) {
          const int i = i0 + u * tpl;
          const bool ok = (sr ? vb : va) && i < n;
          const long e = (sr ? rb : ra) * n + i;
          v[sr][u] = 0;
          if (ok) {
            x[e] = xs[sr][u] + (T)alpha * ps[sr][u];
            const T rv = rs[sr][u] - (T)alpha * qs[sr][u];
            r[e] = rv;
            acc += (double)rv * (double)rv;
            v[sr][u] = rv;
          }
        }
    } else {
      const T* in = (const T*)pb.in;
#pragma unroll
      for (int u = 0; u < CK; ++u)
#pragma unroll
        for (int sr = 0; sr < 2; ++sr) {
          const int i = i0 + u * tpl;
          const bool ok = (sr ? vb : va) && i < n;
          const T t = in[ok ? (sr ? rb : ra) * n + i : 0];  // clamped: unconditional load
          v[sr][u] = ok ? t : (T)0;
        }
      // the domain mask acts on grid functions only: the input of the first
      // pass (or of the single 1D pass), never on a transformed intermediate
      if ((DEPI == DEPI_STORE || pb.d == 1) && pb.mask) {
        T ms[2][CK];
#pragma unroll
        for (int u = 0; u < CK; ++u)
#pragma unroll
          for (int sr = 0; sr < 2; ++sr) {
            const int i = i0 + u * tpl;
            const bool ok = (sr ? vb : va) && i < n;
            const T t = (T)pb.mask[ok ? ((sr ? rb : ra) * n + i) % nper : 0];
            ms[sr][u] = ok ? t : (T)1;
          }
#pragma unroll
        for (int u = 0; u < CK; ++u)
#pragma unroll
          for (int sr = 0; sr < 2; ++sr) v[sr][u] *= ms[sr][u];
      }
      if ((DEPI == DEPI_STORE || pb.d == 1) && pb.corr) {
        T cs[2][CK];
#pragma unroll
        for (int u = 0; u < CK; ++u)
#pragma unroll
          for (int sr = 0; sr < 2; ++sr) {
            const int i = i0 + u * tpl;
            const bool ok = (sr ? vb : va) && i < n;
            const T t = ((const T*)pb.corr)[ok ? (sr ? rb : ra) * n + i : 0];
            cs[sr][u] = ok ? t : (T)0;
          }
#pragma unroll
        for (int u = 0; u < CK; ++u)
#pragma unroll
          for (int sr = 0; sr < 2; ++sr) v[sr][u] += cs[sr][u];
      }
    }
#pragma unroll
    for (int u = 0; u < CK; ++u) {
      const int i = i0 + u * tpl;
      if (i >= n) continue;
      if (direct) pair_put<T, RAD>(buf, Lf, i + 1, v[0][u], v[1][u]);
      else buf[i] = {v[0][u], (T)0};
    }
  }
  if (direct && lane == 0) {
    buf[0] = {0, 0};
    buf[n + 1] = {0, 0};
  }
  if (DPRO == DPRO_UPD) put_partial(pb, S_RR, acc, nblk, blk);
  __syncthreads();
  Line<T> res = buf;  // line holding the transform result
  if (direct) {
    res = dst_pair<T, LF>(buf, buf2, A, dtw, rr, lane);
  } else {
    if constexpr (LF <= 0) dst_line<T, CL>(buf, A, lane, tpl);
  }
  if (pb.d == 1) {
    const T* ev = (const T*)A.eig;
    if (direct) {
      const T* tau = (const T*)pb.tau;
      for (int k = lane + 1; k <= n; k += tpl) {
        cx<T> sv = pair_get<T, RAD>(res, k);
        T e = (T)(pb.p0 + pb.p1 * pb.pcs * (double)(tau ? tau[k - 1] : ev[k - 1]));
        pair_put<T, RAD>(res, Lf, k, pb.pmul ? sv.x * e : sv.x / e, pb.pmul ? sv.y * e : sv.y / e);
      }
      if (lane == 0) {
        res[0] = {0, 0};
        res[n + 1] = {0, 0};
      }
      __syncthreads();
      res = dst_pair<T, LF>(res, res.p == buf.p ? buf2 : buf, A, dtw, rr, lane);
    } else {
      const T* tau = (const T*)pb.tau;
      for (int k = lane; k < n; k += tpl)
      {
        const T e = (T)(pb.p0 + pb.p1 * pb.pcs * (double)(tau ? tau[k] : ev[k]));
        buf[k].x = pb.pmul ? buf[k].x * e : buf[k].x / e;
      }
      __syncthreads();
      if constexpr (LF <= 0) dst_line<T, CL>(buf, A, lane, tpl);
    }
  }
  double norm = 1.0;
  if (pb.d == 1 || DEPI != DEPI_STORE)
    for (int a = 0; a < pb.d; ++a) norm *= 2.0 / (pb.ax[a].n + 1);
  double acc2 = 0.0;
  const bool mask_out = pb.mask && !pb.nomask_out && (DEPI != DEPI_STORE || pb.d == 1);
  constexpr int CKE = dst_chunk(LF, RAD ? c_fixed_tpl(kRaderLF - 1) : (LF > 0 ? c_fixed_tpl(LF) : 0), false, 8);
  // per chunk: the epilogue's loads (r, mask) first, then the stores
  for (int i0 = lane; i0 < n; i0 += CKE * tpl) {
    // unconditional loads from clamped in-range indices, then a select
    T rs[2][CKE], ms[2][CKE];
    if (DEPI == DEPI_Z) {
#pragma unroll
      for (int u = 0; u < CKE; ++u)
#pragma unroll
        for (int sr = 0; sr < 2; ++sr) {
          const int i = i0 + u * tpl;
          const bool ok = (sr ? vb : va) && i < n;
          const T t = ((const T*)pb.r)[ok ? (sr ? rb : ra) * n + i : 0];
          rs[sr][u] = ok ? t : (T)0;
        }
    }
    if (mask_out) {
#pragma unroll
      for (int u = 0; u < CKE; ++u)
#pragma unroll
        for (int sr = 0; sr < 2; ++sr) {
          const int i = i0 + u * tpl;
          const bool ok = (sr ? vb : va) && i < n;
          const T t = (T)pb.mask[ok ? ((sr ? rb : ra) * n + i) % nper : 0];
          ms[sr][u] = ok ? t : (T)1;
        }
    }
#pragma unroll
    for (int u = 0; u < CKE; ++u) {
      const int i = i0 + u * tpl;
      if (i >= n) continue;
      const cx<T> sv = direct ? pair_get<T, RAD>(res, i + 1) : buf[i];
#pragma unroll
      for (int sr = 0; sr < 2; ++sr) {
        if (!(sr ? vb : va)) continue;
        const long e = (sr ? rb : ra) * n + i;
        T v = (sr ? sv.y : sv.x) * (T)norm;
        if (mask_out) v *= ms[sr][u];
        if (DEPI != DEPI_Z) {
          ((T*)pb.out)[e] = v;
        } else {
          ((T*)pb.z)[e] = v;
          acc2 += (double)rs[sr][u] * (double)v;
        }
      }
    }
  }
  if (DEPI == DEPI_Z) put_partial(pb, S_RZ0 + (it.parity ^ 1), acc2, nblk, blk);
}

// Strided real sine pass on T1 (in place).  SCALE: transform along axis 0,
// divide by p0 + p1 pcs (e_0 + e_1 [+ e_2]), transform again.
struct DGeom {
  int axis;
  long gs, ngroup, estride, gstride;
};

template <typename T>
__device__ __forceinline__ double eig_tail(const Prob& pb, long c) {
  if (pb.d == 2) return (double)((const T*)pb.ax[1].eig)[c];
  const int n2 = pb.ax[2].n;
  return (double)((const T*)pb.ax[1].eig)[c / n2] + (double)((const T*)pb.ax[2].eig)[c % n2];
}

template <typename T, bool SCALE, int LF = 0, int TPLF = 0>
__device__ __forceinline__ void dst_cols_body(const Prob& pb, const DGeom& dg, bool check_done, int blk0, int nblk) {
  if (check_done && pb.sc->done) return;
  const long blk = xcd_tile(blk0, nblk);
  extern __shared__ __align__(16) char smem[];
  const Axis& A = pb.ax[dg.axis];
  constexpr int CL = LF < 0 ? -LF : 0;  // chirp-z FFT length of a chirp specialisation
  constexpr bool RAD = LF == kRaderLF;   // prime form
  const int n = A.n, Lf = RAD ? kRaderLF - 1 : (LF > 0 ? LF : (CL > 0 ? CL : A.dst.L));
  const int tpl = RAD ? c_fixed_tpl(kRaderLF - 1)
                      : ((LF > 0 && TPLF > 0) ? TPLF : (CL > 0 ? c_fixed_tpl(CL) : A.dst.tpl));
  const bool direct = LF > 0 ? true : (LF < 0 ? false : A.dst_direct);
  const int GF = blockDim.x / tpl, g = threadIdx.x / tpl, lane = threadIdx.x % tpl;
  const cx<T>* dtw = (const cx<T>*)A.dst.tw;  // prime form: staged in LDS, read after the next barrier
  RaderPF<T> rr;                               // prime form: this lane's table entries
  if constexpr (RAD) {
    dtw = tw_stage<T, kRaderLF - 1>(dtw);
    rader_load(rr, (const int*)A.rtab, (const T*)A.chirp, (const cx<T>*)A.bhat, lane);
  }
  const int G = direct ? 2 * GF : GF;  // real lines per block
  const long tiles = (dg.gs + G - 1) / G;
  const long grp = blk / tiles, c0 = (blk % tiles) * G;
  if (grp >= dg.ngroup) return;
  T* base = (T*)pb.T1 + grp * dg.gstride + c0;
  const int gv = (int)min((long)G, dg.gs - c0);
  // Thread t serves real line t % G, elements t / G + m (blockDim / G), when
  // the block has at least as many threads as real lines; a block of more
  // lines than threads (one lane per FFT line of a short direct form) walks a
  // flat index instead.
  const bool wide = G > (int)blockDim.x;
  constexpr int CKC = dst_chunk(LF, RAD ? c_fixed_tpl(kRaderLF - 1) : (LF > 0 ? (TPLF > 0 ? TPLF : c_fixed_tpl(LF)) : 0),
                                true, 8);
  const int jt = wide ? 0 : threadIdx.x % G, i0 = wide ? 0 : threadIdx.x / G;
  const int ist = wide ? 1 : blockDim.x / G;
  const bool jv = jt < gv;
  if (wide) {
    for (int e = threadIdx.x; e < G * n; e += blockDim.x) {
      const int j = e % G, i = e / G;
      T v = 0;
      if (j < gv) v = base[(long)i * dg.estride + j];
      if (direct) {
        Line<T> ln = line_at<T>(smem, 2 * (j >> 1), Lf);
        ((T*)&ln[i + 1])[j & 1] = v;
        if constexpr (!RAD) ((T*)&ln[Lf - 1 - i])[j & 1] = -v;
      } else {
        line_at<T>(smem, j, Lf)[i] = {v, 0};
      }
    }
    if (direct)
      for (int q = threadIdx.x; q < GF; q += blockDim.x) {
        Line<T> lq = line_at<T>(smem, 2 * q, Lf);
        lq[0] = {0, 0};
        lq[n + 1] = {0, 0};
      }
  } else if (direct) {
    // real line j is component (j & 1) of FFT line j >> 1 (ping-pong lines 2q, 2q+1)
    Line<T> ln = line_at<T>(smem, 2 * (jt >> 1), Lf);
    const T* bp = base + (long)i0 * dg.estride + jt;
    const long bst = (long)ist * dg.estride;
    for (int i = i0; i < n; i += CKC * ist, bp += CKC * bst) {
      T v[CKC];
#pragma unroll
      for (int u = 0; u < CKC; ++u) {
        v[u] = 0;
        if (jv && i + u * ist < n) v[u] = bp[u * bst];
      }
#pragma unroll
      for (int u = 0; u < CKC; ++u) {
        const int ii = i + u * ist;
        if (ii >= n) continue;
        ((T*)&ln[ii + 1])[jt & 1] = v[u];
        if constexpr (!RAD) ((T*)&ln[Lf - 1 - ii])[jt & 1] = -v[u];
      }
    }
    for (int q = threadIdx.x; q < GF; q += blockDim.x) {
      Line<T> lq = line_at<T>(smem, 2 * q, Lf);
      lq[0] = {0, 0};
      lq[n + 1] = {0, 0};
    }
  } else {
    Line<T> ln = line_at<T>(smem, jt, Lf);
    const T* bp = base + (long)i0 * dg.estride + jt;
    const long bst = (long)ist * dg.estride;
    for (int i = i0; i < n; i += CKC * ist, bp += CKC * bst) {
      T v[CKC];
#pragma unroll
      for (int u = 0; u < CKC; ++u) {
        v[u] = 0;
        if (jv && i + u * ist < n) v[u] = bp[u * bst];
      }
#pragma unroll
      for (int u = 0; u < CKC; ++u)
        if (i + u * ist < n) ln[i + u * ist] = {v[u], 0};
    }
  }
  __syncthreads();
  Line<T> buf = line_at<T>(smem, direct ? 2 * g : g, Lf);
  Line<T> buf2 = line_at<T>(smem, 2 * g + 1, Lf);
  Line<T> res = buf;
  if (direct) {
    res = dst_pair<T, LF, TPLF>(buf, buf2, A, dtw, rr, lane);
  } else {
    if constexpr (LF <= 0) dst_line<T, CL>(buf, A, lane, tpl);
  }
  if (SCALE) {
    const T* ev = (const T*)A.eig;
    // sine-basis diagonal: mode (k, c) of the axis-0 pass is table entry (k-1) gs + c
    const T* tau = (const T*)pb.tau;
    if (direct) {
      const long ca = c0 + 2 * g, cb = ca + 1;
      const bool oka = ca < dg.gs, okb = cb < dg.gs;
      const double ta = (oka && !tau) ? eig_tail<T>(pb, ca) : 0.0;
      const double tb = (okb && !tau) ? eig_tail<T>(pb, cb) : 0.0;
      constexpr int CKS = dst_chunk(LF, RAD ? c_fixed_tpl(kRaderLF - 1) : (LF > 0 ? (TPLF > 0 ? TPLF : c_fixed_tpl(LF)) : 0),
                                    false, RAD ? 2 : 4);
      // per chunk: the diagonal's entries (table or eigenvalues) loaded first
      for (int k0 = lane + 1; k0 <= n; k0 += CKS * tpl) {
        // unconditional loads from clamped in-range indices, then a select:
        // no branch around a load, so no wait between them
        T da[CKS], db[CKS];
        if (tau) {
#pragma unroll
          for (int u = 0; u < CKS; ++u) {
            const int k = k0 + u * tpl;
            const bool ua = oka && k <= n, ub = okb && k <= n;
            const T va_ = tau[ua ? (long)(k - 1) * dg.gs + ca : 0];
            const T vb_ = tau[ub ? (long)(k - 1) * dg.gs + cb : 0];
            da[u] = ua ? va_ : (T)1;
            db[u] = ub ? vb_ : (T)1;
          }
        } else {
#pragma unroll
          for (int u = 0; u < CKS; ++u) {
            const int k = k0 + u * tpl;
            const T e = ev[k <= n ? k - 1 : 0];
            da[u] = k <= n ? e : (T)0;
          }
        }
#pragma unroll
        for (int u = 0; u < CKS; ++u) {
          const int k = k0 + u * tpl;
          if (k > n) continue;
          const cx<T> sv = pair_get<T, RAD>(res, k);
          double la, lb;
          if (tau) {
            la = (double)da[u];
            lb = (double)db[u];
          } else {
            const double ek = (double)da[u];
            la = ek + ta;
            lb = ek + tb;
          }
          T ea = (T)(pb.p0 + pb.p1 * pb.pcs * la);
          T eb = (T)(pb.p0 + pb.p1 * pb.pcs * lb);
          pair_put<T, RAD>(res, Lf, k, pb.pmul ? sv.x * ea : sv.x / ea, pb.pmul ? sv.y * eb : sv.y / eb);
        }
      }
      if (lane == 0) {
        res[0] = {0, 0};
        res[n + 1] = {0, 0};
      }
      __syncthreads();
      res = dst_pair<T, LF, TPLF>(res, res.p == buf.p ? buf2 : buf, A, dtw, rr, lane);
    } else {
      const long c = c0 + g;
      const bool ok = c < dg.gs;
      const double etail = (ok && !tau) ? eig_tail<T>(pb, c) : 0.0;
      for (int k = lane; k < n; k += tpl) {
        const double lv = tau ? (ok ? (double)tau[(long)k * dg.gs + c] : 1.0) : (double)ev[k] + etail;
        const T e = (T)(pb.p0 + pb.p1 * pb.pcs * lv);
        buf[k].x = pb.pmul ? buf[k].x * e : buf[k].x / e;
      }
      __syncthreads();
      if constexpr (LF <= 0) dst_line<T, CL>(buf, A, lane, tpl);
    }
  }
  // every FFT line of the block ends in the same member of its ping-pong pair
  const int rsel = direct ? (res.p == buf.p ? 0 : 1) : 0;
  __syncthreads();
  if (wide) {
    for (int e = threadIdx.x; e < G * n; e += blockDim.x) {
      const int j = e % G, i = e / G;
      if (j >= gv) continue;
      T v;
      if (direct) {
        const cx<T> sv = pair_get<T, RAD>(line_at<T>(smem, 2 * (j >> 1) + rsel, Lf), i + 1);
        v = (j & 1) ? sv.y : sv.x;
      } else {
        v = line_at<T>(smem, j, Lf)[i].x;
      }
      base[(long)i * dg.estride + j] = v;
    }
  } else if (jv) {
    T* bp = base + (long)i0 * dg.estride + jt;
    const long bst = (long)ist * dg.estride;
    if (direct) {
      Line<T> ln = line_at<T>(smem, 2 * (jt >> 1) + rsel, Lf);
      for (int i = i0; i < n; i += ist, bp += bst) {
        const cx<T> sv = pair_get<T, RAD>(ln, i + 1);
        *bp = (jt & 1) ? sv.y : sv.x;
      }
    } else {
      Line<T> ln = line_at<T>(smem, jt, Lf);
      for (int i = i0; i < n; i += ist, bp += bst) *bp = ln[i].x;
    }
  }
}

// ---------------------------------------------------------------------------
// Vector kernels
// ---------------------------------------------------------------------------
// dot(a, b) partials (FP64 accumulation) into `site`.
template <typename T>
__device__ __forceinline__ void dot_body(const Prob& pb, const void* a, const void* b, int site, long n, int nblk,
                                         int blk) {
  double acc = 0.0;
  const T* x = (const T*)a;
  const T* y = (const T*)b;
  const long st = (long)nblk * blockDim.x;
  long i = (long)blk * blockDim.x + threadIdx.x;
  // eight elements' loads in flight before their products (same order)
  for (; i + 7 * st < n; i += 8 * st) {
    T xs[8], ys[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      xs[u] = x[i + u * st];
      ys[u] = y[i + u * st];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += (double)xs[u] * (double)ys[u];
  }
  for (; i < n; i += st) acc += (double)x[i] * (double)y[i];
  put_partial(pb, site, acc, nblk, blk);
}

// One workgroup: total of `site` into a scalar slot.
enum { FIN_FF = 0, FIN_RR = 1, FIN_AUX0 = 2, FIN_AUX1 = 3 };
__device__ __forceinline__ void finalize_body(const Prob& pb, int site, int target) {
  double t = get_total(pb, site);
  if (threadIdx.x == 0) {
    if (target == FIN_FF) pb.sc->ff = t;
    else if (target == FIN_RR) pb.sc->rr = t;
    else if (target == FIN_AUX0) pb.sc->aux[0] = t;
    else pb.sc->aux[1] = t;
  }
}

// Plain CG update (no preconditioner, z aliases r): alpha = r.r / p.q;
// x += alpha p, r -= alpha q; r.r partials into S_RR and into the r.z slot.
template <typename T>
__device__ __forceinline__ void update_body(const Prob& pb, const Iter& it, long n, int nblk, int blk) {
  if (pb.sc->done) return;
  const double pq = get_total(pb, S_PQ);
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (blk == 0 && threadIdx.x == 0) {
      pb.sc->pq = pq;
      pb.sc->done = 3;
    }
    return;
  }
  const double alpha = get_total(pb, S_RZ0 + it.parity) / pq;
  T* x = (T*)pb.x;
  T* r = (T*)pb.r;
  const T* p = (const T*)pb.p;
  const T* q = (const T*)pb.q;
  double acc = 0.0;
  const long st = (long)nblk * blockDim.x;
  long i = (long)blk * blockDim.x + threadIdx.x;
  // four elements' loads before their stores (same order)
  for (; i + 3 * st < n; i += 4 * st) {
    T xs[4], ps[4], rs[4], qs[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      xs[u] = x[i + u * st];
      ps[u] = p[i + u * st];
      rs[u] = r[i + u * st];
      qs[u] = q[i + u * st];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[i + u * st] = xs[u] + (T)alpha * ps[u];
      const T rv = rs[u] - (T)alpha * qs[u];
      r[i + u * st] = rv;
      acc += (double)rv * (double)rv;
    }
  }
  for (; i < n; i += st) {
    x[i] += (T)alpha * p[i];
    T rv = r[i] - (T)alpha * q[i];
    r[i] = rv;
    acc += (double)rv * (double)rv;
  }
  double s = block_sum_all(acc);
  if (threadIdx.x == 0) {
    pb.part[S_RR * pb.pstride + blk] = s;
    pb.part[(S_RZ0 + (it.parity ^ 1)) * pb.pstride + blk] = s;
    if (blk == 0) {
      pb.sc->cnt[S_RR] = nblk;
      pb.sc->cnt[S_RZ0 + (it.parity ^ 1)] = nblk;
    }
  }
}

// Start of a Krylov solve: thr = tol^2 ff, counters cleared, done when the
// initial residual already meets the tolerance.  use_rr: the initial residual
// norm is in rr (warm start); otherwise r = f and rr = ff.
__device__ __forceinline__ void init_body(const Prob& pb, double tol, int maxit, int use_rr) {
  if (threadIdx.x != 0) return;
  Scalars* s = pb.sc;
  if (!use_rr) s->rr = s->ff;
  s->thr = tol * tol * s->ff;
  s->rr0 = s->rr;
  s->itc[0] = 0;
  s->itc[1] = 0;
  s->maxit = maxit;
  s->done = (s->rr <= s->thr) ? 1 : 0;
  if (!(s->ff > 0.0)) s->done = 1;  // zero right-hand side: x = 0 is exact
}

// y = a * x + b * y elementwise (any of the two real types), n elements.
template <typename TX, typename TY>
__global__ void k_axpby(const TX* x, TY* y, double a, double b, long n) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) y[i] = (TY)(a * (double)x[i] + (b == 0.0 ? 0.0 : b * (double)y[i]));
}
template <typename T> __global__ void k_fill(T* y, T v, long n) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}

// ---------------------------------------------------------------------------
// kernel wrappers
// ---------------------------------------------------------------------------
#define FL_BOUNDS __launch_bounds__(256)

template <typename T, int PRO, int LF = 0> __global__ FL_BOUNDS void k_rowfwd(Prob pb, Iter it) {
  rowfwd_body<T, PRO, LF>(pb, it, blockIdx.x);
}
template <typename T, int PRO, int LF = 0>
__global__ FL_BOUNDS void k_rowfwd_b(const Prob* pbs, Iter it, const int* nb) {
  if ((int)blockIdx.x >= nb[blockIdx.y]) return;
  rowfwd_body<T, PRO, LF>(pbs[blockIdx.y], it, blockIdx.x);
}
template <typename T, int MODE, int LF = 0, int TPLF = 0>
__global__ FL_BOUNDS void k_colpass(Prob pb, ColGeom cg, Iter it, int chk) {
  colpass_body<T, MODE, LF, TPLF>(pb, cg, it, chk, blockIdx.x, gridDim.x);
}
template <typename T, int MODE, int LF = 0, int TPLF = (LF > 0 ? c_fixed_tpl(LF) : 0)>
__global__ FL_BOUNDS void k_colpass_b(const Prob* pbs, const ColGeom* cgs, Iter it, int chk, const int* nb) {
  if ((int)blockIdx.x >= nb[blockIdx.y]) return;
  colpass_body<T, MODE, LF, TPLF>(pbs[blockIdx.y], cgs[blockIdx.y], it, chk, blockIdx.x,
                                                             nb[blockIdx.y]);
}
template <typename T, int EPI, int LF = 0> __global__ FL_BOUNDS void k_rowinv(Prob pb, Iter it, int chk) {
  rowinv_body<T, EPI, LF>(pb, it, chk, gridDim.x, blockIdx.x);
}
template <typename T, int EPI, int LF = 0>
__global__ FL_BOUNDS void k_rowinv_b(const Prob* pbs, Iter it, int chk, const int* nb) {
  if ((int)blockIdx.x >= nb[blockIdx.y]) return;
  rowinv_body<T, EPI, LF>(pbs[blockIdx.y], it, chk, nb[blockIdx.y], blockIdx.x);
}
template <typename T, int PRO, int EPI> __global__ FL_BOUNDS void k_conv1d(Prob pb, Iter it) {
  conv1d_body<T, PRO, EPI>(pb, it, gridDim.x, blockIdx.x);
}
template <typename T, int PRO, int EPI>
__global__ FL_BOUNDS void k_conv1d_b(const Prob* pbs, Iter it, const int* nb) {
  if ((int)blockIdx.x >= nb[blockIdx.y]) return;
  conv1d_body<T, PRO, EPI>(pbs[blockIdx.y], it, nb[blockIdx.y], blockIdx.x);
}
template <typename T, int DPRO, int DEPI, int LF = 0> __global__ FL_BOUNDS void k_dst_rows(Prob pb, Iter it, int chk) {
  dst_rows_body<T, DPRO, DEPI, LF>(pb, it, chk, gridDim.x, blockIdx.x);
}
template <typename T, int DPRO, int DEPI, int LF = 0>
__global__ FL_BOUNDS void k_dst_rows_b(const Prob* pbs, Iter it, int chk, const int* nb) {
  if ((int)blockIdx.x >= nb[blockIdx.y]) return;
  dst_rows_body<T, DPRO, DEPI, LF>(pbs[blockIdx.y], it, chk, nb[blockIdx.y], blockIdx.x);
}
template <typename T, bool SCALE, int LF = 0, int TPLF = 0>
__global__ FL_BOUNDS void k_dst_cols(Prob pb, DGeom dg, int chk) {
  dst_cols_body<T, SCALE, LF, TPLF>(pb, dg, chk, blockIdx.x, gridDim.x);
}
template <typename T, bool SCALE, int LF = 0>
__global__ FL_BOUNDS void k_dst_cols_b(const Prob* pbs, const DGeom* dgs, int chk, const int* nb) {
  if ((int)blockIdx.x >= nb[blockIdx.y]) return;
  dst_cols_body<T, SCALE, LF>(pbs[blockIdx.y], dgs[blockIdx.y], chk, blockIdx.x, nb[blockIdx.y]);
}
template <typename T> __global__ FL_BOUNDS void k_dot(Prob pb, const void* a, const void* b, int site, long n) {
  dot_body<T>(pb, a, b, site, n, gridDim.x, blockIdx.x);
}
// (small solver kernels are templates so that every translation unit that
// launches them carries its own instance)
template <int = 0> __global__ FL_BOUNDS void k_finalize(Prob pb, int site, int target) {
  finalize_body(pb, site, target);
}
// Batched forms over a device Prob array (blockIdx.y = problem): the total of
// a site into a scalar slot; r.r (or aux.aux) partials; aux = in (the
// right-hand side of a backward-Euler step from the state).
template <int = 0> __global__ FL_BOUNDS void k_finalize_b(const Prob* pbs, int site, int target) {
  finalize_body(pbs[blockIdx.y], site, target);
}
enum { DOT_AUX = 0, DOT_R = 1 };
template <typename T, int WHICH>
__global__ FL_BOUNDS void k_dot_b(const Prob* pbs, int site, const long* ns, const int* nb) {
  if ((int)blockIdx.x >= nb[blockIdx.y]) return;
  const Prob& pb = pbs[blockIdx.y];
  const void* a = WHICH == DOT_AUX ? pb.aux : pb.r;
  dot_body<T>(pb, a, a, site, ns[blockIdx.y], nb[blockIdx.y], blockIdx.x);
}
template <typename T> __global__ FL_BOUNDS void k_copy_in_aux_b(const Prob* pbs, const long* ns, const int* nb) {
  if ((int)blockIdx.x >= nb[blockIdx.y]) return;
  const Prob& pb = pbs[blockIdx.y];
  const long n = ns[blockIdx.y];
  const T* src = (const T*)pb.in;
  T* dst = (T*)pb.aux;
  const long st = (long)nb[blockIdx.y] * blockDim.x;
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * st < n; i += 4 * st) {  // four loads in flight before the stores
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = src[i + u * st];
#pragma unroll
    for (int u = 0; u < 4; ++u) dst[i + u * st] = v[u];
  }
  for (; i < n; i += st) dst[i] = src[i];
}
template <typename T> __global__ FL_BOUNDS void k_update(Prob pb, Iter it, long n) {
  update_body<T>(pb, it, n, gridDim.x, blockIdx.x);
}
template <typename T> __global__ FL_BOUNDS void k_update_b(const Prob* pbs, Iter it, const long* ns, const int* nb) {
  if ((int)blockIdx.x >= nb[blockIdx.y]) return;
  update_body<T>(pbs[blockIdx.y], it, ns[blockIdx.y], nb[blockIdx.y], blockIdx.x);
}
template <int = 0> __global__ void k_init(Prob pb, double tol, int maxit, int use_rr) {
  init_body(pb, tol, maxit, use_rr);
}
// tols: per-problem tolerances (device), or NULL for tol everywhere
template <int = 0> __global__ void k_init_b(const Prob* pbs, double tol, const double* tols, int maxit, int use_rr) {
  init_body(pbs[blockIdx.y], tols ? tols[blockIdx.y] : tol, maxit, use_rr);
}

}  // namespace fl
