// Exact inverse of the sine-diagonalised preconditioner on an occluded grid
// domain (Sec. 3.1, "Preconditioning"; Sec. 4.4).
//
// On a domain Omega inside the box the paper's preconditioner is the FD
// Laplacian with zero data outside Omega: the principal submatrix A_Omega of
// the box matrix A = p0 I + p1 pcs T (T the (2d+1)-point Laplacian; also the
// shifted and M~ forms).  The paper factors A_Omega with sparse Cholesky.
// Here the box inverse stays the fast sine solve and a capacitance matrix
// corrects it.  Let Gamma be the points outside Omega with a stencil
// neighbour in Omega.  For r on Omega, seek
//     x = A^{-1} (r + E mu),   mu on Gamma,   x = 0 on Gamma,
// with E the injection of Gamma into the grid.  Then x vanishes on the whole
// complement (A x = 0 there, x = 0 on its boundary Gamma) and A x = r on
// Omega, i.e. x = A_Omega^{-1} r.  The condition on Gamma is
//     C mu = -(A^{-1} r)|_Gamma,   C = E^T A^{-1} E   (SPD, k x k, k = |Gamma|).
// One application is: y = A^{-1} r, mu = -C^{-1} y|_Gamma, z = P_Omega A^{-1}
// (r + E mu) -- two box solves, a gather and a dense k x k product.  C is
// built once per (mask, preconditioner) with k box solves in FP64 and
// inverted in place by Gauss-Jordan elimination (SPD: no pivoting).
#include "fl_internal.hpp"

namespace {

// 64-bit mix of a grid index (splitmix64 finaliser).
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Checksum of the set of mask points (sum of mixed indices, mod 2^64).
__global__ __launch_bounds__(256) void k_mask_hash(const uint8_t* __restrict__ m, long N,
                                                   unsigned long long* __restrict__ out) {
  unsigned long long acc = 0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x)
    if (m[i]) acc += mix64((unsigned long long)i);
  __shared__ unsigned long long red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

__global__ void k_set_u64(unsigned long long* p, unsigned long long v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// E[b][idx[b]] = 1 on a zero-filled [B][N] array.
__global__ void k_unit_cols(double* __restrict__ E, const int* __restrict__ idx, int B, long N) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) E[(long)b * N + idx[b]] = 1.0;
}

// Rows j0..j0+B-1 of C: C[(j0+b) k + i] = Z[b][idx[i]] (C is symmetric).
__global__ void k_cap_rows(const double* __restrict__ Z, const int* __restrict__ idx, long k, int B, long N,
                           double* __restrict__ Crows) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)B * k) return;
  const long b = t / k, i = t % k;
  Crows[b * k + i] = Z[b * N + idx[i]];
}

// In-place Gauss-Jordan inversion, pivot p: save row p and column p, then
// a_pp <- 1/a_pp, a_pj <- a_pj / a_pp, a_ip <- -a_ip / a_pp,
// a_ij <- a_ij - a_ip a_pj / a_pp.
__global__ void k_gj_save(const double* __restrict__ A, long k, long p, double* __restrict__ row,
                          double* __restrict__ col) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < k) {
    row[i] = A[p * k + i];
    col[i] = A[i * k + p];
  }
}
__global__ __launch_bounds__(256) void k_gj_update(double* __restrict__ A, long k, long p,
                                                   const double* __restrict__ row, const double* __restrict__ col) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= k * k) return;
  const long i = t / k, j = t % k;
  const double inv = 1.0 / row[p];
  double v;
  if (i == p && j == p) v = inv;
  else if (i == p) v = row[j] * inv;
  else if (j == p) v = -col[i] * inv;
  else v = A[t] - col[i] * row[j] * inv;
  A[t] = v;
}

// g[b][j] = y[b][idx[j]] for every right-hand side b (blockIdx.y).
template <typename T>
__global__ void k_cap_gather(const T* __restrict__ Y, const int* __restrict__ idx, long k, long N,
                             T* __restrict__ G, const Scalars* __restrict__ sc, int chk) {
  if (chk && sc->done) return;
  const long j = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (j < k) G[blockIdx.y * k + j] = Y[blockIdx.y * N + idx[j]];
}

// mu = -Cinv g per right-hand side; S[b][idx[i]] = mu_i.  One wave per row.
template <typename T>
__global__ __launch_bounds__(256) void k_cap_matvec(const T* __restrict__ Cinv, const T* __restrict__ G,
                                                    const int* __restrict__ idx, long k, long N, T* __restrict__ S,
                                                    const Scalars* __restrict__ sc, int chk) {
  if (chk && sc->done) return;
  const int lane = threadIdx.x & 63;
  const long i = blockIdx.x * 4L + (threadIdx.x >> 6);
  if (i >= k) return;  // uniform per wave
  const T* row = Cinv + i * k;
  const T* g = G + blockIdx.y * k;
  double acc = 0.0;
  for (long j = lane; j < k; j += 64) acc += (double)row[j] * (double)g[j];
  acc = wave_sum(acc);
  if (lane == 0) S[blockIdx.y * N + idx[i]] = (T)(-acc);
}

}  // namespace

fl_status cap_hash_launch(fl_op op, const uint8_t* mask, unsigned long long* dst) {
  hipStream_t s = op->stream;
  LAUNCH(k_set_u64, dim3(1), dim3(64), 0, s, dst, 0ull);
  LAUNCH(k_mask_hash, dim3((unsigned)std::min<long>(1024, nblocks_vec(op->N))), dim3(256), 0, s, mask, op->N, dst);
  return FL_OK;
}

static void cap_release(CapCache& c) {
  for (void* p : {(void*)c.idx, c.cinv[0], c.cinv[1], c.Y[0], c.Y[1], c.S[0], c.S[1], c.G[0], c.G[1]})
    if (p) (void)hipFree(p);
  c = CapCache();
}

void cap_destroy(fl_op op) { cap_release(op->cap); }

// Build (or keep) the correction for the box preconditioner described by
// pbox (p0, p1, pcs; sine eigenvalues of T) on the mask with checksum key.
fl_status cap_prepare(fl_op op, const uint8_t* mask, const Prob& pbox, unsigned long long key, bool* active) {
  CapCache& c = op->cap;
  *active = false;
  if (c.valid && c.key == key && c.mask == mask && c.p0 == pbox.p0 && c.p1 == pbox.p1 && c.pcs == pbox.pcs) {
    *active = c.k > 0;
    return FL_OK;
  }
  // iteration graphs captured with the old correction's buffers
  drop_graph(op->ws[0]);
  drop_graph(op->ws[1]);
  cap_release(c);
  hipStream_t s = op->stream;
  const long N = op->N;
  const int d = op->d;
  // Gamma on the host: points outside the mask with an axis neighbour inside
  std::vector<uint8_t> m(N);
  HIPCHK(hipMemcpyAsync(m.data(), mask, N, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  long st[3] = {1, 1, 1};
  for (int a = d - 2; a >= 0; --a) st[a] = st[a + 1] * op->n[a + 1];
  std::vector<int> gam;
  for (long e = 0; e < N; ++e) {
    if (m[e]) continue;
    bool adj = false;
    for (int a = 0; a < d && !adj; ++a) {
      const long ia = (e / st[a]) % op->n[a];
      if (ia > 0 && m[e - st[a]]) adj = true;
      if (ia + 1 < op->n[a] && m[e + st[a]]) adj = true;
    }
    if (adj) gam.push_back((int)e);
  }
  const long k = (long)gam.size();
  c.key = key;
  c.mask = mask;
  c.p0 = pbox.p0;
  c.p1 = pbox.p1;
  c.pcs = pbox.pcs;
  c.k = k;
  c.valid = true;
  if (k == 0) return FL_OK;  // nothing outside the domain touches it: the box inverse is exact
  if (k > kCapMax) {
    cap_release(c);
    return fail(FL_E_UNSUPPORTED, "the occluded domain has " + std::to_string(k) +
                                      " exterior points next to it; the exact preconditioner supports up to " +
                                      std::to_string(kCapMax) + " (FL_PC_FD_BOX applies P_Omega A^-1 P_Omega)");
  }
  STCHK(dalloc((void**)&c.idx, k * sizeof(int)));
  HIPCHK(hipMemcpyAsync(c.idx, gam.data(), k * sizeof(int), hipMemcpyHostToDevice, s));
  STCHK(dalloc(&c.cinv[0], (size_t)k * k * sizeof(double)));
  STCHK(dalloc(&c.cinv[1], (size_t)k * k * sizeof(float)));
  // C = E^T A^{-1} E, B unit right-hand sides per batched box solve
  const long B = std::max<long>(1, std::min<long>(k, (64L << 20) / N));
  Workspace& w = op->ws[0];
  const long cap0 = w.cap_rhs;
  void *E = nullptr, *Z = nullptr;
  STCHK(dalloc(&E, (size_t)B * N * sizeof(double)));
  fl_status stt = dalloc(&Z, (size_t)B * N * sizeof(double));
  if (stt == FL_OK) stt = ensure_ws<double>(op, B, false);
  for (long j0 = 0; j0 < k && stt == FL_OK; j0 += B) {
    const long nb = std::min(B, k - j0);
    if (launch(k_fill<double>, dim3(nblocks_vec(nb * N)), dim3(256), 0, s, (double*)E, 0.0, nb * N) != hipSuccess ||
        launch(k_unit_cols, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, (double*)E,
               (const int*)c.idx + j0, (int)nb, N) != hipSuccess) {
      stt = fail(FL_E_HIP, "capacitance right-hand sides");
      break;
    }
    Prob pb = base_prob<double>(op, nb);
    pb.p0 = pbox.p0;
    pb.p1 = pbox.p1;
    pb.pcs = pbox.pcs;
    pb.in = E;
    pb.out = Z;
    pb.T1 = w.T1;
    pb.sc = w.sc;
    pb.part = w.part;
    pb.pstride = w.npart;
    stt = precond_seq<double, DPRO_PLAIN, DEPI_FINAL>(op, pb, Iter{0, 0}, 0);
    if (stt != FL_OK) break;
    if (launch(k_cap_rows, dim3((unsigned)((nb * k + 255) / 256)), dim3(256), 0, s, (const double*)Z,
               (const int*)c.idx, k, (int)nb, N, (double*)c.cinv[0] + j0 * k) != hipSuccess)
      stt = fail(FL_E_HIP, "capacitance rows");
  }
  if (stt == FL_OK) {
    // invert C in place; the pivot row and column go to E (2k doubles)
    double* row = (double*)E;
    double* col = row + k;
    double* A = (double*)c.cinv[0];
    for (long p = 0; p < k && stt == FL_OK; ++p) {
      if (launch(k_gj_save, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s, (const double*)A, k, p, row, col) !=
              hipSuccess ||
          launch(k_gj_update, dim3((unsigned)((k * k + 255) / 256)), dim3(256), 0, s, A, k, p, (const double*)row,
                 (const double*)col) != hipSuccess)
        stt = fail(FL_E_HIP, "capacitance inverse");
    }
  }
  if (stt == FL_OK &&
      launch(k_cast<float, double>, dim3((unsigned)((k * k + 255) / 256)), dim3(256), 0, s, (const double*)c.cinv[0],
             (float*)c.cinv[1], k * k, 1.0) != hipSuccess)
    stt = fail(FL_E_HIP, "capacitance cast");
  if (hipStreamSynchronize(s) != hipSuccess && stt == FL_OK) stt = fail(FL_E_HIP, "capacitance build");
  (void)hipFree(E);
  if (Z) (void)hipFree(Z);
  if (w.cap_rhs > cap0 && cap0 <= 1) {
    // give back the batched workspace of the build (reallocated at the next call's size)
    drop_graph(w);
    for (void** p : {&w.W1, &w.W2, &w.T1})
      if (*p) { (void)hipFree(*p); *p = nullptr; }
    w.cap_rhs = 0;
  }
  if (stt != FL_OK) {
    cap_release(c);
    return stt;
  }
  *active = true;
  return FL_OK;
}

// Per-precision buffers of the correction for nrhs right-hand sides; S is
// zero everywhere but on Gamma, where each application overwrites mu.
template <typename T> fl_status cap_buffers(fl_op op, long nrhs) {
  CapCache& c = op->cap;
  const int t = tix<T>();
  if (c.cap[t] >= nrhs) return FL_OK;
  for (void** p : {&c.Y[t], &c.S[t], &c.G[t]})
    if (*p) { (void)hipFree(*p); *p = nullptr; }
  // every captured iteration graph of this precision used the old buffers
  drop_graph(op->ws[t]);
  const long N = op->N;
  STCHK(dalloc(&c.Y[t], (size_t)nrhs * N * sizeof(T)));
  STCHK(dalloc(&c.S[t], (size_t)nrhs * N * sizeof(T)));
  STCHK(dalloc(&c.G[t], (size_t)nrhs * c.k * sizeof(T)));
  LAUNCH(k_fill<T>, dim3(nblocks_vec(nrhs * N)), dim3(256), 0, op->stream, (T*)c.S[t], (T)0, nrhs * N);
  c.cap[t] = nrhs;
  return FL_OK;
}

// The preconditioner with the correction: first box solve into Y (the
// fused Krylov update of DPRO_UPD included), mu from the capacitance
// inverse into S on Gamma, second box solve of P_Omega r + S with the
// epilogue DEPI.
template <typename T, int DPRO, int DEPI> fl_status cap_precond_seq(fl_op op, const Prob& pb, Iter it, int chk) {
  CapCache& c = op->cap;
  const int t = tix<T>();
  hipStream_t s = op->stream;
  const long N = op->N;
  Prob p1 = pb;
  p1.out = c.Y[t];
  p1.nomask_out = 1;
  STCHK((precond_seq<T, DPRO, DEPI_FINAL>(op, p1, it, chk)));
  LAUNCH(k_cap_gather<T>, dim3((unsigned)((c.k + 255) / 256), pb.nrhs), dim3(256), 0, s, (const T*)c.Y[t],
         (const int*)c.idx, c.k, N, (T*)c.G[t], (const Scalars*)pb.sc, chk);
  LAUNCH(k_cap_matvec<T>, dim3((unsigned)((c.k + 3) / 4), pb.nrhs), dim3(256), 0, s, (const T*)c.cinv[t],
         (const T*)c.G[t], (const int*)c.idx, c.k, N, (T*)c.S[t], (const Scalars*)pb.sc, chk);
  Prob p2 = pb;
  if (DPRO == DPRO_UPD) p2.in = pb.r;  // the residual the first solve updated
  p2.corr = c.S[t];
  return precond_seq<T, DPRO_PLAIN, DEPI>(op, p2, it, chk);
}

template fl_status cap_buffers<double>(fl_op, long);
template fl_status cap_buffers<float>(fl_op, long);
template fl_status cap_precond_seq<double, DPRO_PLAIN, DEPI_Z>(fl_op, const Prob&, Iter, int);
template fl_status cap_precond_seq<double, DPRO_UPD, DEPI_Z>(fl_op, const Prob&, Iter, int);
template fl_status cap_precond_seq<double, DPRO_PLAIN, DEPI_FINAL>(fl_op, const Prob&, Iter, int);
template fl_status cap_precond_seq<float, DPRO_PLAIN, DEPI_Z>(fl_op, const Prob&, Iter, int);
template fl_status cap_precond_seq<float, DPRO_UPD, DEPI_Z>(fl_op, const Prob&, Iter, int);
template fl_status cap_precond_seq<float, DPRO_PLAIN, DEPI_FINAL>(fl_op, const Prob&, Iter, int);
