// Learned preconditioner: a multilevel convolutional network (BF16 activations,
// FP32 accumulation, FP32 master weights), its training (reverse pass, Adam),
// and flexible CG with z = B (r + s N(r/s, alpha)), B the inverse of the
// operator's sine-basis diagonal, s the RMS of r, and the FD Laplacian
// preconditioner (Sec. 3.1) as the fallback.  Not in the paper.
//
// Network on a 2D grid H x W or a 3D grid D x H x W (every side a multiple of
// 8; ReLU after every convolution but the last; average pooling over 2 x 2
// (x 2) blocks, nearest 2x upsampling, additive skips):
//   a0 = relu(cin([x, alpha-1]))   a1 = relu(d1(pool a0))   a2 = relu(d2(pool a1))
//   a3 = relu(d3(pool a2))         c3 = relu(b3(a3))        c2 = relu(u2(a2 + up c3))
//   c1 = relu(u1(a1 + up c2))      c0 = relu(u0(a0 + up c1)) y = out(c0)
// Zero-padded cross-correlations with K = 9 KD taps (KD = 1: 3 x 3, KD = 3:
// 3 x 3 x 3), tap = 9 kz + 3 ky + kx row-major over the offsets; parameters
// W[tap][ci][co] then b[co] per layer in the order cin, d1, d2, d3, b3, u2,
// u1, u0, out.
//
// Layout: activations channel-last bf16 [B][D][H][W][32] (D = 1 in 2D); input
// and output FP32 [B][D][H][W].  The 32 -> 32 convolutions are implicit GEMMs
// on v_mfma_f32_32x32x16_bf16: D[co][pixel] = sum_k W^T[co][k] X[k][pixel],
// k = (tap, ci), a 64-wide wave computing 2 x 32 pixels of one output row
// against all 32 output channels; in 3D a block accumulates the three input
// slices z-1, z, z+1 of its output slice one after another (one staged slice
// and the nine in-plane taps of that slice at a time).
#include <type_traits>

#include "fl_internal.hpp"

namespace fln {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16;

constexpr int CH = 32;
constexpr int NL32 = 7;  // 32 -> 32 layers d1 d2 d3 b3 u2 u1 u0
enum { LD1 = 0, LD2, LD3, LB3, LU2, LU1, LU0 };

// Parameter layout of a network with K = 9 KD taps per kernel.
template <int KD> struct PL {
  static constexpr int K = 9 * KD;
  static constexpr long L32W = (long)K * CH * CH;        // weights per 32 -> 32 layer
  static constexpr long OFF_CIN_B = (long)K * 2 * CH;    // bias of the input layer
  static constexpr long OFF_L32 = OFF_CIN_B + CH;        // first 32 -> 32 layer
  static constexpr long L32SZ = L32W + CH;               // weights + bias per 32 -> 32 layer
  static constexpr long OFF_OUT = OFF_L32 + NL32 * L32SZ;  // output layer
  static constexpr long NPARAM = OFF_OUT + (long)K * CH + 1;
  static constexpr long PACK = 2L * K * 64 * 8;  // packed bf16 per layer (2K fragments x 64 lanes x 8)
  static constexpr long CIN_PV = (long)K * 2 * CH + CH;  // input-layer gradient values
  static constexpr long OUT_PV = (long)K * CH + 1;       // output-layer gradient values
};
// 2D sizes: 65633 parameters (3 x 3 kernels); 3D: 196385 (3 x 3 x 3)
static_assert(PL<1>::NPARAM == 65633 && PL<3>::NPARAM == 196385, "parameter layout");

// Tile of one conv block: 4 output rows x 64 output columns of one slice.
constexpr int TY = 4, TX = 64, SY = TY + 2, SX = TX + 2;
// Pixel stride (BF16 elements) of tiles staged in LDS: the 32 channels and 8
// of padding.  With 64-byte pixels every fourth pixel starts in the same
// bank, so the 16-byte MFMA fragment reads of 8 or 16 consecutive pixels
// serialise 4 ways; with 80 bytes (5 x 16, 5 odd) consecutive pixels start
// in distinct 16-byte bank groups.
constexpr int CP = 40;

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float bf2f(u16 v) { return __uint_as_float((unsigned)v << 16); }
// FP32 -> BF16 rounded to nearest even by the hardware conversion (NaN stays
// a quiet NaN); the bit-manipulation form costs a dozen instructions and a
// divergent branch per value where this is half an instruction.
__device__ __forceinline__ u16 f2bf(float f) { return __builtin_bit_cast(u16, (__bf16)f); }
// (a, b) -> one 32-bit word of two BF16 (a in the low half), one instruction
__device__ __forceinline__ unsigned pk2(float a, float b) {
  const f32x2_t v = {a, b};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2_t));
}

__device__ __forceinline__ void ld8(const u16* p, float v[8]) {
  const uint4 q = *(const uint4*)p;
  const unsigned w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[2 * i] = __uint_as_float(w[i] << 16);
    v[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
  }
}
__device__ __forceinline__ uint4 pk8(const float v[8]) {
  unsigned w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = pk2(v[2 * i], v[2 * i + 1]);
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// ---------------------------------------------------------------------------
// Staging of a convolution input (8 channels of one in-bounds pixel)
// ---------------------------------------------------------------------------
enum { SM_PLAIN = 0, SM_POOL, SM_UPADD, SM_GPLAIN, SM_GSUMPOOL, SM_GADDUP };
//  PLAIN    s0[p]                                  (this level)
//  POOL     mean of s0 over the 2 x 2 (x 2) block  (s0 at the finer level)
//  UPADD    s0[p] + s1[p/2]                        (s1 at the coarser level)
//  GPLAIN   s0[p] * (y[p] > 0)                     (gradient through a ReLU)
//  GSUMPOOL sum of s0 over the block * (y[p] > 0)
//  GADDUP   (s0[p] + s1[p/2] / 2^d) * (y[p] > 0)
struct Stage {
  const u16* s0;
  const u16* s1;
  const u16* y;
};

// Grid of one level: D = 1 for 2D networks.
struct Dims {
  int B, D, H, W;
  // inference inside flexible CG: the device done flag; a forward kernel
  // returns at once when it is set (an iteration enqueued ahead of the host's
  // convergence test is then nearly free)
  const double* stop = nullptr;
};
__device__ __forceinline__ bool stopped(const Dims& g) { return g.stop && *g.stop != 0.0; }

// Learned-preconditioner input and output on the solver grid m0 x m1 x m2
// (m0 = 1 in 2D) inside the padded network grid P0 x P1 x P2 (one image).
struct PadGrid {
  int m0, m1, m2, P0, P1, P2;
};
// The solver-grid glue of the learned preconditioner, done by the network's
// first and last layers when G = 1 (T = float) or 2 (T = double): the input
// layer takes x = r / s (zero outside the solver grid), the output layer
// writes w = r + s y on the solver grid instead of y, with the RMS
// s = sqrt(rr / N) read from the device (rr = r.r).
struct NetGlue {
  const void* r = nullptr;
  void* w = nullptr;
  const double* rr = nullptr;
  PadGrid q = {};
};
__device__ __forceinline__ long pix(const Dims& g, int b, int z, int y, int x) {
  return ((((long)b * g.D + z) * g.H + y) * g.W + x) * CH;
}
// the finer (pooling source) and coarser (upsampling source) level
template <int KD> __device__ __forceinline__ Dims finer(const Dims& g) {
  return Dims{g.B, KD == 3 ? 2 * g.D : 1, 2 * g.H, 2 * g.W};
}
template <int KD> __device__ __forceinline__ Dims coarser(const Dims& g) {
  return Dims{g.B, KD == 3 ? g.D / 2 : 1, g.H / 2, g.W / 2};
}

template <int SM, int KD>
__device__ __forceinline__ void stage8(const Stage& st, const Dims& g, int b, int z, int y, int x, int c, float v[8]) {
  constexpr int NB = KD == 3 ? 8 : 4;  // pixels per pooling block
  if (SM == SM_PLAIN) {
    ld8(st.s0 + pix(g, b, z, y, x) + c, v);
  } else if (SM == SM_POOL || SM == SM_GSUMPOOL) {
    const Dims f = finer<KD>(g);
    float t[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = 0.f;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int zf = KD == 3 ? 2 * z + (q >> 2) : 0;
      ld8(st.s0 + pix(f, b, zf, 2 * y + ((q >> 1) & 1), 2 * x + (q & 1)) + c, t);
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] += t[i];
    }
    if (SM == SM_POOL)
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] *= 1.f / NB;
  } else {
    ld8(st.s0 + pix(g, b, z, y, x) + c, v);
    if (SM == SM_UPADD || SM == SM_GADDUP) {
      float t[8];
      ld8(st.s1 + pix(coarser<KD>(g), b, KD == 3 ? z >> 1 : 0, y >> 1, x >> 1) + c, t);
      const float f = SM == SM_UPADD ? 1.f : 1.f / NB;
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] += f * t[i];
    }
  }
  if (SM >= SM_GPLAIN && SM <= SM_GADDUP) {
    float a[8];
    ld8(st.y + pix(g, b, z, y, x) + c, a);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = a[i] > 0.f ? v[i] : 0.f;
  }
}

// Stage rows y0-1 .. y0+TY and columns x0-1 .. x0+TX of slice z of image b
// into LDS ([SY][SX] pixels of 32 BF16 channels at stride PS), zero outside
// the grid (a slice z outside 0..D-1 stages zeros).
template <int SM, int KD, int PS = CP>
__device__ __forceinline__ void stage_tile(u16* tile, const Stage& st, const Dims& g, int b, int z, int y0, int x0) {
  const bool zin = z >= 0 && z < g.D;
  for (int e = threadIdx.x; e < SY * SX * 4; e += blockDim.x) {
    const int c = (e & 3) * 8, p = e >> 2;
    const int yy = y0 + p / SX - 1, xx = x0 + p % SX - 1;
    float v[8];
    if (zin && yy >= 0 && yy < g.H && xx >= 0 && xx < g.W) {
      stage8<SM, KD>(st, g, b, z, yy, xx, c, v);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = 0.f;
    }
    *(uint4*)(tile + p * PS + c) = pk8(v);
  }
}

// Forward-mode staging with all global loads of a lane issued before any LDS
// store: the memory latency is paid once per tile instead of once per chunk.
// Plain and skip-add staging, and 2D pooling (3D pooling reads 8 pixels per
// chunk and takes stage_tile).  The 256 threads take one staged row per step
// (64 pixels x 4 chunks of 8 channels: columns x0 .. x0+TX-1), so the row's
// address is uniform across the block and a lane's column offset is fixed;
// a last step takes the two halo columns x0-1 and x0+TX of every row
// (threads 0 .. 8 SY - 1).
template <int SM, int KD, int PS = CP>
__device__ __forceinline__ void stage_tile_batched(u16* tile, const Stage& st, const Dims& g, int b, int z, int y0,
                                                   int x0) {
  constexpr int NQ = SM == SM_POOL ? 4 : SM == SM_UPADD ? 2 : 1;
  static_assert(SM == SM_PLAIN || SM == SM_UPADD || (SM == SM_POOL && KD == 1), "batched staging modes");
  static_assert(TX * 4 == 256 && 8 * SY <= 256, "one staged row per step of 256 threads");
  const int t = threadIdx.x, c = (t & 3) * 8;
  const bool zin = z >= 0 && z < g.D;
  const Dims gf = finer<KD>(g), gc = coarser<KD>(g);
  const int xm = x0 + (t >> 2);                                // column of the row steps
  const int hr = t >> 3, hs = (t >> 2) & 1;                    // halo step: row, side
  const int xh = hs ? x0 + TX : x0 - 1;
  // pixel (y, x) of slice zz of a level d, this lane's 8 channels
  auto at = [&](const u16* base, const Dims& d, int zz, int y, int x) {
    return (const uint4*)(base + (((long)b * d.D + zz) * d.H + y) * (long)d.W * CH + (unsigned)(x * CH + c));
  };
  uint4 q[SY + 1][NQ];
#pragma unroll
  for (int r = 0; r <= SY; ++r) {
    const bool halo = r == SY;
    const int yy = y0 - 1 + (halo ? hr : r), xx = halo ? xh : xm;
    const bool ok = zin && (!halo || t < 8 * SY) && yy >= 0 && yy < g.H && xx >= 0 && xx < g.W;
#pragma unroll
    for (int k = 0; k < NQ; ++k) q[r][k] = make_uint4(0, 0, 0, 0);
    if (ok) {
      if constexpr (SM == SM_PLAIN) {
        q[r][0] = *at(st.s0, g, z, yy, xx);
      } else if constexpr (SM == SM_UPADD) {
        q[r][0] = *at(st.s0, g, z, yy, xx);
        q[r][1] = *at(st.s1, gc, KD == 3 ? z >> 1 : 0, yy >> 1, xx >> 1);
      } else {  // SM_POOL, 2D
#pragma unroll
        for (int k = 0; k < 4; ++k) q[r][k] = *at(st.s0, gf, 0, 2 * yy + (k >> 1), 2 * xx + (k & 1));
      }
    }
  }
#pragma unroll
  for (int r = 0; r <= SY; ++r) {
    const bool halo = r == SY;
    if (halo && t >= 8 * SY) continue;
    const int p = halo ? hr * SX + (hs ? SX - 1 : 0) : r * SX + 1 + (t >> 2);
    if (SM == SM_PLAIN) {
      *(uint4*)(tile + p * PS + c) = q[r][0];
    } else {
      float v[8], u[8];
      const unsigned* w0 = (const unsigned*)&q[r][0];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        v[2 * i] = __uint_as_float(w0[i] << 16);
        v[2 * i + 1] = __uint_as_float(w0[i] & 0xffff0000u);
      }
#pragma unroll
      for (int k = 1; k < NQ; ++k) {
        const unsigned* wk = (const unsigned*)&q[r][k];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          u[2 * i] = __uint_as_float(wk[i] << 16);
          u[2 * i + 1] = __uint_as_float(wk[i] & 0xffff0000u);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] += u[i];
      }
      if (SM == SM_POOL)
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] *= 0.25f;
      *(uint4*)(tile + p * PS + c) = pk8(v);
    }
  }
}

// Tile of the block in a launch over conv_grid (x: tile column, y: tile row,
// z: image * D + slice): no division on the tile index.
template <int KD> __device__ __forceinline__ void tile_here(const Dims& g, int& b, int& z, int& y0, int& x0) {
  x0 = blockIdx.x * TX;
  y0 = blockIdx.y * TY;
  z = KD == 3 ? (int)(blockIdx.z % (unsigned)g.D) : 0;
  b = KD == 3 ? (int)(blockIdx.z / (unsigned)g.D) : (int)blockIdx.z;
}

// Decode a tile index of a level: (b, z, tile row, tile column).
__device__ __forceinline__ void tile_of(long t, const Dims& g, int& b, int& z, int& y0, int& x0) {
  const int tilesX = (g.W + TX - 1) / TX, tilesY = (g.H + TY - 1) / TY;
  x0 = (int)(t % tilesX) * TX;
  t /= tilesX;
  y0 = (int)(t % tilesY) * TY;
  t /= tilesY;
  z = (int)(t % g.D);
  b = (int)(t / g.D);
}

// ---------------------------------------------------------------------------
// 32 -> 32 convolution on MFMA (forward with bias + ReLU, or the transposed
// convolution of the reverse pass with flipped, transposed weights)
// ---------------------------------------------------------------------------
// EPI_RELU: bias + ReLU, BF16 out; EPI_NONE: BF16 out.
enum { EPI_RELU = 0, EPI_NONE = 1 };

// Output tile of a 32-channel layer: lane holds pixel (lane & 31) of each
// 32-pixel half of its wave's row, channels q*8 + (lane>>5)*4 + 0..3 in
// acc[4q .. 4q+3].  The wave's 64 x 32 outputs go through LDS (`tile`, free
// once every wave has passed a barrier after its last read) so that the
// global stores are contiguous 16-byte chunks.
// pout (2D only, else nullptr): also the 2 x 2 average of the tile into the
// coarser level (2 x 32 pooled pixels; tiles start on even rows and columns,
// H and W are even): the mean of four BF16 outputs in FP32, rounded to BF16,
// as pooling staging would compute it from `out`.
template <int EPI>
__device__ __forceinline__ void store_rows(const f32x16& acc0, const f32x16& acc1, u16* tile,
                                           const float* __restrict__ bias, u16* __restrict__ out, const Dims& g, int b,
                                           int z, int y0, int x0, u16* __restrict__ pout = nullptr) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  u16* ot = tile + wave * 64 * CP;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const f32x16& a = m ? acc1 : acc0;
    const int pl = m * 32 + (lane & 31);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int cb = q * 8 + (lane >> 5) * 4;
      float v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        v[i] = a[4 * q + i];
        if (EPI == EPI_RELU) v[i] = fmaxf(v[i] + bias[cb + i], 0.f);
      }
      const unsigned lo = pk2(v[0], v[1]), hi = pk2(v[2], v[3]);
      *(uint2*)(ot + pl * CP + cb) = make_uint2(lo, hi);
    }
  }
  __syncthreads();
  if (pout) {  // one 8-channel chunk of one pooled pixel per thread
    const Dims gc{g.B, 1, g.H / 2, g.W / 2};
    const int q = (threadIdx.x & 3) * 8, pc = (threadIdx.x >> 2) & 31, wr = threadIdx.x >> 7;
    const int px = x0 / 2 + pc, py = y0 / 2 + wr;
    if (px < gc.W && py < gc.H) {
      float v[8], t[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = 0.f;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        ld8(tile + ((2 * wr + (k >> 1)) * 64 + 2 * pc + (k & 1)) * CP + q, t);
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] += t[i];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] *= 0.25f;
      *(uint4*)(pout + pix(gc, b, 0, py, px) + q) = pk8(v);
    }
  }
  const int yo = y0 + wave;
  if (yo >= g.H) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = lane + 64 * k, pl = e >> 2, qq = (e & 3) * 8;
    const int px = x0 + pl;
    if (px < g.W) *(uint4*)(out + pix(g, b, z, yo, px) + qq) = *(const uint4*)(ot + pl * CP + qq);
  }
}

template <int SM, int EPI, int KD>
__global__ __launch_bounds__(256) void k_conv32(Stage st, const u16* __restrict__ wpack, const float* __restrict__ bias,
                                                u16* __restrict__ out, Dims g, u16* __restrict__ pout) {
  __shared__ __align__(16) u16 tile[SY * SX * CP];
  if (stopped(g)) return;
  int b, z, y0, x0;
  tile_here<KD>(g, b, z, y0, x0);
  if (b >= g.B) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  f32x16 acc0 = {}, acc1 = {};
#pragma unroll 1
  for (int kz = 0; kz < KD; ++kz) {
    const int zi = z + kz - (KD == 3 ? 1 : 0);
    if (zi < 0 || zi >= g.D) continue;  // zero slice (uniform over the block)
    if (kz > 0) __syncthreads();         // every wave is done with the previous slice
    if constexpr (SM == SM_PLAIN || SM == SM_UPADD || (SM == SM_POOL && KD == 1))
      stage_tile_batched<SM, KD>(tile, st, g, b, zi, y0, x0);
    else
      stage_tile<SM, KD>(tile, st, g, b, zi, y0, x0);
    bf16x8 wf[18];
#pragma unroll
    for (int f = 0; f < 18; ++f) wf[f] = *(const bf16x8*)(wpack + ((long)(kz * 18 + f) * 64 + lane) * 8);
    __syncthreads();
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int ky = tap / 3, kx = tap % 3;
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const u16* p0 = tile + ((wave + ky) * SX + (lane & 31) + kx) * CP + half * 16 + (lane >> 5) * 8;
        const bf16x8 b0 = *(const bf16x8*)p0;
        const bf16x8 b1 = *(const bf16x8*)(p0 + 32 * CP);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[tap * 2 + half], b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[tap * 2 + half], b1, acc1, 0, 0, 0);
      }
    }
  }
  __syncthreads();  // every wave is done reading the staged tile
  store_rows<EPI>(acc0, acc1, tile, bias, out, g, b, z, y0, x0, pout);
}

// Input layer (2 -> 32) on MFMA with (tap, input channel) packed into K:
// k = 2 tap + ci runs over the 2K values of the stencil, padded to a multiple
// of 16 (2 MFMA steps in 2D, 4 in 3D).  The A fragments (slot NL32 of the
// packed weights) hold W^T[co][k]; each lane gathers its B fragment
// X[k][pixel] from the staged (x, alpha - 1) slices.  Bias + ReLU, BF16 out.
template <int KD, int G = 0>
__global__ __launch_bounds__(256) void k_cin_mfma(const float* __restrict__ x, const float* __restrict__ alpha,
                                                  const u16* __restrict__ wpack, const float* __restrict__ bias,
                                                  u16* __restrict__ out, Dims g, u16* __restrict__ pout, NetGlue gl) {
  constexpr int K = 9 * KD, S = (2 * K + 15) / 16;
  __shared__ __align__(16) u16 tile[TY * TX * CP];  // output staging
  __shared__ unsigned xin[KD][SY * SX];             // bf16 pair (x, alpha - 1) per pixel
  if (stopped(g)) return;
  int b, z, y0, x0;
  tile_here<KD>(g, b, z, y0, x0);
  if (b >= g.B) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const unsigned am1 = (unsigned)f2bf(alpha[b] - 1.f) << 16;
  double inv_s = 0.0;
  if constexpr (G != 0) {
    const double ms = *gl.rr / ((double)gl.q.m0 * gl.q.m1 * gl.q.m2);
    inv_s = ms > 0.0 ? 1.0 / sqrt(ms) : 0.0;
  }
  for (int e = threadIdx.x; e < KD * SY * SX; e += blockDim.x) {
    const int kz = e / (SY * SX), p = e % (SY * SX);
    const int zi = z + kz - (KD == 3 ? 1 : 0), yy = y0 + p / SX - 1, xx = x0 + p % SX - 1;
    const bool in = zi >= 0 && zi < g.D && yy >= 0 && yy < g.H && xx >= 0 && xx < g.W;
    float xv = 0.f;
    if constexpr (G == 0) {
      if (in) xv = x[(((long)b * g.D + zi) * g.H + yy) * g.W + xx];
    } else {  // r / s on the solver grid, zero in the padding (one image)
      const bool inm = in && zi < gl.q.m0 && yy < gl.q.m1 && xx < gl.q.m2;
      const long si = inm ? ((long)zi * gl.q.m1 + yy) * gl.q.m2 + xx : 0;
      const double rv = G == 1 ? (double)((const float*)gl.r)[si] : ((const double*)gl.r)[si];
      if (inm) xv = (float)(rv * inv_s);
    }
    xin[kz][p] = in ? ((unsigned)f2bf(xv) | am1) : 0u;
  }
  bf16x8 wf[S];
#pragma unroll
  for (int st = 0; st < S; ++st) wf[st] = *(const bf16x8*)(wpack + ((long)st * 64 + lane) * 8);
  __syncthreads();
  f32x16 acc0 = {}, acc1 = {};
#pragma unroll
  for (int st = 0; st < S; ++st) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int px = h * 32 + (lane & 31);
      unsigned w[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        unsigned v2[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int k = st * 16 + 8 * (lane >> 5) + 2 * i + j;
          v2[j] = 0;
          if (k < 2 * K) {
            const int tap = k >> 1, kz = tap / 9, ky = (tap % 9) / 3, kx = tap % 3;
            const unsigned pr = xin[kz][(wave + ky) * SX + px + kx];
            v2[j] = (k & 1) ? (pr >> 16) : (pr & 0xffffu);
          }
        }
        w[i] = v2[0] | (v2[1] << 16);
      }
      const bf16x8 bfr = __builtin_bit_cast(bf16x8, make_uint4(w[0], w[1], w[2], w[3]));
      if (h == 0) acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[st], bfr, acc0, 0, 0, 0);
      else acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[st], bfr, acc1, 0, 0, 0);
    }
  }
  store_rows<EPI_RELU>(acc0, acc1, tile, bias, out, g, b, z, y0, x0, pout);
}

// Output layer (32 -> 1): per slice, Z[q][m] = sum_ci c0[q][ci] W[9 kz + m][ci]
// for every pixel q of the staged halo tile and the nine in-plane taps m, on
// MFMA with the taps as rows (slot NL32 + 1 of the packed weights: fragment
// 2 kz + s holds W[9 kz + m][16 s + ...] in row m < 9); then each thread sums
// y[p] += sum_m Z[p + offset(m)][m] for its output pixel.  FP32 out.
template <int KD, int G = 0>
__global__ __launch_bounds__(256) void k_out_mfma(const u16* __restrict__ c0, const u16* __restrict__ wpack,
                                                  const float* __restrict__ bias, Dims g, float* __restrict__ yout,
                                                  NetGlue gl) {
  constexpr int NQ = SY * SX, NCH = (NQ + 31) / 32;
  __shared__ __align__(16) u16 tile[SY * SX * CH];  // unpadded: tile + zt fit four blocks per CU
  __shared__ float zt[NQ][9];
  if (stopped(g)) return;
  int b, z, y0, x0;
  tile_here<KD>(g, b, z, y0, x0);
  if (b >= g.B) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ly = threadIdx.x / TX, lx = threadIdx.x % TX;  // this thread's output pixel
  const Stage st = {c0, nullptr, nullptr};
  float yacc = 0.f;
#pragma unroll 1
  for (int kz = 0; kz < KD; ++kz) {
    const int zi = z + kz - (KD == 3 ? 1 : 0);
    if (zi < 0 || zi >= g.D) continue;  // zero slice (uniform over the block)
    if (kz > 0) __syncthreads();         // every thread is done with the previous slice
    stage_tile_batched<SM_PLAIN, KD, CH>(tile, st, g, b, zi, y0, x0);
    const bf16x8 a0 = *(const bf16x8*)(wpack + ((long)(kz * 2) * 64 + lane) * 8);
    const bf16x8 a1 = *(const bf16x8*)(wpack + ((long)(kz * 2 + 1) * 64 + lane) * 8);
    __syncthreads();
    for (int ch = wave; ch < NCH; ch += 4) {
      const int q = ch * 32 + (lane & 31);
      bf16x8 b0 = {}, b1 = {};
      if (q < NQ) {
        const u16* p0 = tile + q * CH + (lane >> 5) * 8;
        b0 = *(const bf16x8*)p0;
        b1 = *(const bf16x8*)(p0 + 16);
      }
      f32x16 d = {};
      d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, d, 0, 0, 0);
      // rows (taps) of lane l: 8 (r/4) + 4 (l/32) + r%4 -> lanes < 32 hold
      // m = 0..3 (r = 0..3) and 8 (r = 4); lanes >= 32 hold m = 4..7
      if (q < NQ) {
        const int m0 = (lane >> 5) * 4;
#pragma unroll
        for (int r = 0; r < 4; ++r) zt[q][m0 + r] = d[r];
        if (lane < 32) zt[q][8] = d[4];
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 9; ++m) yacc += zt[(ly + m / 3) * SX + lx + m % 3][m];
  }
  const int yo = y0 + ly, xo = x0 + lx;
  if (yo < g.H && xo < g.W) {
    const float yv = yacc + bias[0];
    if constexpr (G == 0) {
      yout[(((long)b * g.D + z) * g.H + yo) * g.W + xo] = yv;
    } else if (z < gl.q.m0 && yo < gl.q.m1 && xo < gl.q.m2) {  // w = r + s y on the solver grid
      const long N = (long)gl.q.m0 * gl.q.m1 * gl.q.m2;
      const double sc = sqrt(fmax(*gl.rr, 0.0) / (double)N);
      const long si = ((long)z * gl.q.m1 + yo) * gl.q.m2 + xo;
      if constexpr (G == 1)
        ((float*)gl.w)[si] = (float)((double)((const float*)gl.r)[si] + sc * (double)yv);
      else
        ((double*)gl.w)[si] = ((const double*)gl.r)[si] + sc * (double)yv;
    }
  }
}

// Pooled activation of a level (3D down path): one 8-channel chunk of one
// coarse pixel per thread, the mean over the 2 x 2 x 2 block exactly as the
// pooling staging forms it.
template <int KD> __global__ __launch_bounds__(256) void k_pool(const u16* __restrict__ src, u16* __restrict__ dst, Dims gc) {
  if (stopped(gc)) return;
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)gc.B * gc.D * gc.H * gc.W * 4) return;
  const int c = (int)(t & 3) * 8;
  const long v = t >> 2;
  const int x = (int)(v % gc.W), y = (int)((v / gc.W) % gc.H);
  const long bz = v / ((long)gc.W * gc.H);
  const int z = (int)(bz % gc.D), b = (int)(bz / gc.D);
  const Stage st = {src, nullptr, nullptr};
  float r[8];
  stage8<SM_POOL, KD>(st, gc, b, z, y, x, c, r);
  *(uint4*)(dst + pix(gc, b, z, y, x) + c) = pk8(r);
}

// Stage the gradient G of the output slice z (TY x TX pixels, no halo).
template <int SMG, int KD>
__device__ __forceinline__ void stage_grad(u16* gt, const Stage& sg, const Dims& g, int b, int z, int y0, int x0) {
  for (int e = threadIdx.x; e < TY * TX * 4; e += blockDim.x) {
    const int c = (e & 3) * 8, p = e >> 2;
    const int yy = y0 + p / TX, xx = x0 + p % TX;
    float v[8];
    if (yy < g.H && xx < g.W) {
      stage8<SMG, KD>(sg, g, b, z, yy, xx, c, v);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = 0.f;
    }
    *(uint4*)(gt + p * CP + c) = pk8(v);
  }
}

// Weight gradient of a 32 -> 32 layer on MFMA: per-block partials of
// dW[tap][ci][co] = sum_p X[p + off(tap)][ci] G[p][co] and db[co] = sum_p G[p][co]
// (X staged by SMI, G by SMG), an implicit GEMM with the pixels as the
// contraction: for each tap C[ci][co] += A[ci][k] B[k][co], A = X and B = G
// over 16 consecutive pixels of one row per v_mfma_f32_32x32x16_bf16, FP32
// accumulation.  Both operands are staged channel-first (one plane of BF16
// pixels per channel) so that a lane's 8 consecutive pixels of one channel
// are one 16-byte read; the tap's column offset kx of X is taken from the
// aligned read and the dword after it (a 2-byte shift for kx = 1).  Wave w
// takes output row w of the 4 x 64 tile for all nine in-plane taps; blocks
// stride over tiles; the waves' sums meet in LDS at the end.  blockIdx.y = kz:
// input slice z + kz - 1 (3D), rows kz*288 .. of the partial (stride L32SZ).
constexpr int WXR = 72;               // X plane row: columns x0-1 .. x0+64, padded
constexpr int WXP = SY * WXR + 8;     // X plane (channel) stride, BF16 elements
constexpr int WGP = TY * TX + 8;      // G plane stride
__device__ __forceinline__ bf16x8 frag_shift(const uint4 a, unsigned nxt, int kx) {
  uint4 r;
  if (kx == 0) {
    r = a;
  } else if (kx == 2) {
    r = make_uint4(a.y, a.z, a.w, nxt);
  } else {  // 2-byte shift: word j = (w[j] >> 16) | (w[j+1] << 16)
    r = make_uint4(__builtin_amdgcn_alignbit(a.y, a.x, 16), __builtin_amdgcn_alignbit(a.z, a.y, 16),
                   __builtin_amdgcn_alignbit(a.w, a.z, 16), __builtin_amdgcn_alignbit(nxt, a.w, 16));
  }
  return __builtin_bit_cast(bf16x8, r);
}

template <int SMI, int SMG, int KD>
__global__ __launch_bounds__(256, 2) void k_conv32_wgrad(Stage si, Stage sg, float* __restrict__ part, Dims g) {
  __shared__ __align__(16) u16 lds[CH * WXP + CH * WGP];
  __shared__ float bsum[8][CH];
  u16* const xs = lds;             // X planes
  u16* const gs = lds + CH * WXP;  // G planes
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kz = blockIdx.y;
  const long ntiles = (long)g.B * g.D * ((g.H + TY - 1) / TY) * ((g.W + TX - 1) / TX);
  f32x16 acc[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[t] = f32x16{};
  float accb = 0.f;
  for (long t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int b, z, y0, x0;
    tile_of(t, g, b, z, y0, x0);
    const int zi = z + kz - (KD == 3 ? 1 : 0);
    const bool zin = zi >= 0 && zi < g.D;  // uniform over the block
    __syncthreads();                        // the previous tile's planes are read
    // X: rows y0-1 .. y0+TY, columns x0-1 .. x0+TX (66), four 8-channel chunks
    if (zin)
      for (int e = threadIdx.x; e < SY * 4 * (TX + 2); e += blockDim.x) {
        const int c = e % (TX + 2), rq = e / (TX + 2), q = rq & 3, r = rq >> 2;
        const int yy = y0 + r - 1, xx = x0 + c - 1;
        float v[8];
        if (yy >= 0 && yy < g.H && xx >= 0 && xx < g.W) {
          stage8<SMI, KD>(si, g, b, zi, yy, xx, q * 8, v);
        } else {
#pragma unroll
          for (int i = 0; i < 8; ++i) v[i] = 0.f;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) xs[(q * 8 + i) * WXP + r * WXR + c] = f2bf(v[i]);
      }
    // G: rows y0 .. y0+TY-1, columns x0 .. x0+TX-1
    for (int e = threadIdx.x; e < TY * 4 * TX; e += blockDim.x) {
      const int c = e % TX, rq = e / TX, q = rq & 3, r = rq >> 2;
      const int yy = y0 + r, xx = x0 + c;
      float v[8];
      if (yy < g.H && xx < g.W) {
        stage8<SMG, KD>(sg, g, b, z, yy, xx, q * 8, v);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = 0.f;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) gs[(q * 8 + i) * WGP + r * TX + c] = f2bf(v[i]);
    }
    __syncthreads();
    if (kz == 0) {  // bias: thread (co, part) sums 32 pixels of plane co
      const u16* gp = gs + (threadIdx.x & 31) * WGP + (threadIdx.x >> 5) * 32;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float v[8];
        ld8(gp + 8 * j, v);
#pragma unroll
        for (int i = 0; i < 8; ++i) accb += v[i];
      }
    }
    if (!zin) continue;
    const int ch = lane & 31, ko = (lane >> 5) * 8;
#pragma unroll
    for (int j = 0; j < TX / 16; ++j) {
      const bf16x8 bg = *(const bf16x8*)(gs + ch * WGP + wave * TX + 16 * j + ko);
#pragma unroll
      for (int ky = 0; ky < 3; ++ky) {
        const u16* xp = xs + ch * WXP + (wave + ky) * WXR + 16 * j + ko;
        const uint4 a = *(const uint4*)xp;
        const unsigned nxt = *(const unsigned*)(xp + 8);
#pragma unroll
        for (int kx = 0; kx < 3; ++kx)
          acc[ky * 3 + kx] =
              __builtin_amdgcn_mfma_f32_32x32x16_bf16(frag_shift(a, nxt, kx), bg, acc[ky * 3 + kx], 0, 0, 0);
      }
    }
  }
  // sum of the four waves in LDS (the planes are free after this barrier)
  __syncthreads();
  float* red = (float*)lds;  // [9 * 32][32] floats
  static_assert(sizeof(float) * 9 * CH * CH <= sizeof(u16) * CH * (WXP + WGP), "wave reduction fits the planes");
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int ci = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3), co = lane & 31;
          float* d = red + (t * CH + ci) * CH + co;
          *d = (w == 0 ? 0.f : *d) + acc[t][v];
        }
    }
    __syncthreads();
  }
  if (kz == 0) bsum[threadIdx.x >> 5][threadIdx.x & 31] = accb;
  __syncthreads();
  float* o = part + (long)blockIdx.x * PL<KD>::L32SZ;
  for (int i = threadIdx.x; i < 9 * CH * CH; i += blockDim.x) o[(long)kz * 9 * CH * CH + i] = red[i];
  if (kz == 0 && threadIdx.x < CH) {
    float sb = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) sb += bsum[k][threadIdx.x];
    o[PL<KD>::L32W + threadIdx.x] = sb;
  }
}

// ---------------------------------------------------------------------------
// Input layer (2 -> 32) and output layer (32 -> 1): VALU, FP32 weights
// ---------------------------------------------------------------------------
// Weight gradient of cin: partials of dW[tap][ci][co] (ci: x and alpha - 1) and
// db, the gradient G staged by SMG; blockIdx.y = kz as in k_conv32_wgrad
// (576 values per kz, then the 32 biases; stride CIN_PV).
template <int SMG, int KD>
__global__ __launch_bounds__(256) void k_cin_wgrad(const float* __restrict__ x, const float* __restrict__ alpha, Stage sg,
                                                   float* __restrict__ part, Dims g) {
  __shared__ __align__(16) u16 gt[TY * TX * CP];
  __shared__ float xs[SY * SX][2];
  const int kz = blockIdx.y;
  const long ntiles = (long)g.B * g.D * ((g.H + TY - 1) / TY) * ((g.W + TX - 1) / TX);
  float acc[3] = {0.f, 0.f, 0.f};
  for (long t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int b, z, y0, x0;
    tile_of(t, g, b, z, y0, x0);
    const int zi = z + kz - (KD == 3 ? 1 : 0);
    for (int p = threadIdx.x; p < SY * SX; p += blockDim.x) {
      const int yy = y0 + p / SX - 1, xx = x0 + p % SX - 1;
      const bool in = zi >= 0 && zi < g.D && yy >= 0 && yy < g.H && xx >= 0 && xx < g.W;
      xs[p][0] = in ? x[(((long)b * g.D + zi) * g.H + yy) * g.W + xx] : 0.f;
      xs[p][1] = in ? alpha[b] - 1.f : 0.f;
    }
    stage_grad<SMG, KD>(gt, sg, g, b, z, y0, x0);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int e = threadIdx.x + r * 256;
      if (e >= 608) break;
      float s = 0.f;
      if (e < 576) {
        const int tap = e / 64, ci = (e / 32) & 1, co = e & 31;
        for (int p = 0; p < TY * TX; ++p)
          s += xs[(p / TX + tap / 3) * SX + p % TX + tap % 3][ci] * bf2f(gt[p * CP + co]);
      } else {
        const int co = e - 576;
        for (int p = 0; p < TY * TX; ++p) s += bf2f(gt[p * CP + co]);
      }
      acc[r] += s;
    }
    __syncthreads();
  }
  float* o = part + (long)blockIdx.x * PL<KD>::CIN_PV;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int e = threadIdx.x + r * 256;
    if (e < 576) o[(long)kz * 576 + e] = acc[r];
    else if (e < 608 && kz == 0) o[PL<KD>::OFF_CIN_B + (e - 576)] = acc[r];
  }
}

// gc0[p][ci] = sum_tap gy[p - off(tap)] W_out[tap][ci] (transposed convolution),
// four lanes per pixel, eight channels each.
template <int KD>
__global__ __launch_bounds__(256) void k_cout_bwd(const float* __restrict__ gy, const float* __restrict__ wout,
                                                  u16* __restrict__ gc0, Dims g) {
  constexpr int K = 9 * KD;
  __shared__ float ws[K * CH];
  for (int i = threadIdx.x; i < K * CH; i += blockDim.x) ws[i] = wout[i];
  __syncthreads();
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long idx = t >> 2;
  if (idx >= (long)g.B * g.D * g.H * g.W) return;
  const int q = (int)(t & 3) * 8;
  const int xx = (int)(idx % g.W), yy = (int)((idx / g.W) % g.H);
  const long bz = idx / ((long)g.W * g.H);  // b * D + z
  const int zz = (int)(bz % g.D);
  float acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = 0.f;
#pragma unroll
  for (int tap = 0; tap < K; ++tap) {
    const int z2 = zz - (KD == 3 ? tap / 9 - 1 : 0);
    const int y2 = yy - ((tap % 9) / 3 - 1), x2 = xx - (tap % 3 - 1);
    if (z2 < 0 || z2 >= g.D || y2 < 0 || y2 >= g.H || x2 < 0 || x2 >= g.W) continue;
    const float gv = gy[((bz + (z2 - zz)) * g.H + y2) * g.W + x2];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] += gv * ws[tap * CH + q + i];
  }
  *(uint4*)(gc0 + idx * CH + q) = pk8(acc);
}

// Weight gradient of out: partials of dW[tap][ci] = sum_p c0[p + tap][ci] gy[p]
// and db = sum gy; blockIdx.y = kz (288 values per kz, then the bias; stride
// OUT_PV).
template <int KD>
__global__ __launch_bounds__(256) void k_cout_wgrad(const u16* __restrict__ c0, const float* __restrict__ gy,
                                                    float* __restrict__ part, Dims g) {
  __shared__ __align__(16) u16 xt[SY * SX * CP];
  __shared__ float gs[TY * TX];
  const int kz = blockIdx.y;
  const long ntiles = (long)g.B * g.D * ((g.H + TY - 1) / TY) * ((g.W + TX - 1) / TX);
  Stage st = {c0, nullptr, nullptr};
  float acc[2] = {0.f, 0.f};
  for (long t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int b, z, y0, x0;
    tile_of(t, g, b, z, y0, x0);
    stage_tile<SM_PLAIN, KD>(xt, st, g, b, z + kz - (KD == 3 ? 1 : 0), y0, x0);
    for (int p = threadIdx.x; p < TY * TX; p += blockDim.x) {
      const int yy = y0 + p / TX, xx = x0 + p % TX;
      gs[p] = (yy < g.H && xx < g.W) ? gy[(((long)b * g.D + z) * g.H + yy) * g.W + xx] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int e = threadIdx.x + r * 256;
      if (e >= 289) break;
      float s = 0.f;
      if (e < 288) {
        const int tap = e / CH, ci = e % CH;
        for (int p = 0; p < TY * TX; ++p)
          s += bf2f(xt[((p / TX + tap / 3) * SX + p % TX + tap % 3) * CP + ci]) * gs[p];
      } else {
        for (int p = 0; p < TY * TX; ++p) s += gs[p];
      }
      acc[r] += s;
    }
    __syncthreads();
  }
  float* o = part + (long)blockIdx.x * PL<KD>::OUT_PV;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int e = threadIdx.x + r * 256;
    if (e < 288) o[(long)kz * 288 + e] = acc[r];
    else if (e == 288 && kz == 0) o[(long)9 * KD * CH] = acc[r];
  }
}

// dst[i] = sum over blocks of part[blk * stride + i] (fixed order)
__global__ void k_reduce_part(const float* __restrict__ part, int nblk, int stride, int nval, float* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nval) return;
  float s = 0.f;
  for (int k = 0; k < nblk; ++k) s += part[(long)k * stride + i];
  dst[i] = s;
}
// First stage of a two-stage sum over many blocks: column y of the grid sums
// blocks y, y + S, y + 2 S, ... (S = gridDim.y, fixed order) into tmp[y][i].
__global__ void k_reduce_part_s1(const float* __restrict__ part, int nblk, int stride, int nval,
                                 float* __restrict__ tmp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nval) return;
  float s = 0.f;
  for (int k = blockIdx.y; k < nblk; k += gridDim.y) s += part[(long)k * stride + i];
  tmp[(long)blockIdx.y * nval + i] = s;
}

// Packed bf16 weights of the 32 -> 32 layers.  Forward (A operand = W^T):
// fw[L][tap][half][lane][e] = W_L[tap][half*16 + 8*(lane/32) + e][lane%32].
// Transposed flipped (reverse pass): bw[L][tap][half][lane][e] =
// W_L[K-1-tap][lane%32][half*16 + 8*(lane/32) + e] (reversing the tap index
// reverses every offset).  Slot L = 7 of fw holds the input layer with
// (tap, ci) packed into K (k_cin_mfma), slot 8 the output layer with the
// in-plane taps as rows (k_out_mfma).
constexpr int NPACK = NL32 + 2;
template <int KD> __global__ void k_pack(const float* __restrict__ th, u16* __restrict__ fw, u16* __restrict__ bw) {
  using P = PL<KD>;
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= NPACK * P::PACK) return;
  const int L = (int)(idx / P::PACK);
  const int r = (int)(idx % P::PACK);
  const int e = r & 7, lane = (r >> 3) & 63, f = r >> 9;
  const int tap = f >> 1, half = f & 1;
  const int kk = half * 16 + 8 * (lane >> 5) + e, j = lane & 31;
  if (L < NL32) {
    const float* W = th + P::OFF_L32 + L * P::L32SZ;
    fw[idx] = f2bf(W[((long)tap * CH + kk) * CH + j]);
    bw[idx] = f2bf(W[((long)(P::K - 1 - tap) * CH + j) * CH + kk]);
  } else if (L == NL32) {  // input layer, K-packed: fragment f = step, k = 16 f + ... = 2 tap + ci
    const int k = f * 16 + 8 * (lane >> 5) + e;
    fw[idx] = k < 2 * P::K ? f2bf(th[(long)k * CH + j]) : (u16)0;
  } else {  // output layer, taps as rows: fragment f = 2 kz + s, row m = lane % 32, k = ci
    const int kz = f >> 1, m = lane & 31, ci = (f & 1) * 16 + 8 * (lane >> 5) + e;
    fw[idx] = (kz < KD && m < 9) ? f2bf(th[P::OFF_OUT + (long)(kz * 9 + m) * CH + ci]) : (u16)0;
  }
}

// Loss (1/count) sum (y - t)^2 per block partials; gy = 2 (y - t) / count.
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ y, const float* __restrict__ t,
                                              float* __restrict__ gy, double* __restrict__ part, long n, double inv) {
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float d = y[i] - t[i];
    gy[i] = (float)(2.0 * inv) * d;
    acc += (double)d * d;
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] * inv;
}

// sum of n partials (one block of 256 threads: strided sums, then a fixed tree)
__global__ __launch_bounds__(256) void k_sum_to(const double* __restrict__ part, int n, float* __restrict__ dst) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *dst = (float)red[0];
}

// Adam (Kingma and Ba 2015): c1 = 1/(1 - b1^k), c2 = 1/(1 - b2^k)
__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       long n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// Minibatch gather: x[k] = R[idx[k]], t[k] = T[idx[k]], a[k] = A[idx[k]]
__global__ void k_gather(const float* __restrict__ R, const float* __restrict__ T, const float* __restrict__ A,
                         const int* __restrict__ idx, float* __restrict__ x, float* __restrict__ t,
                         float* __restrict__ a, int batch, long npix) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)batch * npix) return;
  const int k = (int)(i / npix);
  const long o = (long)idx[k] * npix + i % npix;
  x[i] = R[o];
  t[i] = T[o];
  if (i % npix == 0) a[k] = A[idx[k]];
}


// Flexible CG scalars live on the device: fs[0] = r.z, fs[1] = z.q_old,
// fs[2] = p.q, fs[3] = p.r, fs[4] = r.r, fs[5] = done flag (1 once r.r is
// below the threshold or p.q broke down: later updates are no-ops).
__global__ void k_total_to(Prob pb, int site, double* __restrict__ dst) {
  const double t = get_total(pb, site);
  if (threadIdx.x == 0) *dst = t;
}
// partials of r.z (site S_RZ0) and, after the first iteration, z.q_old (S_RZ1)
template <typename T> __global__ __launch_bounds__(256) void k_fcg_dots(Prob pb, long n, int with_q) {
  const T* z = (const T*)pb.z;
  const T* r = (const T*)pb.r;
  const T* q = (const T*)pb.q;
  double a = 0.0, c = 0.0;
  const long st = (long)gridDim.x * blockDim.x;
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  // four elements' loads in flight before their products (same summation order)
  for (; i + 3 * st < n; i += 4 * st) {
    T zs[4], rs[4], qs[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      zs[u] = z[i + u * st];
      rs[u] = r[i + u * st];
      qs[u] = with_q ? q[i + u * st] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double zi = (double)zs[u];
      a += zi * (double)rs[u];
      if (with_q) c += zi * (double)qs[u];
    }
  }
  for (; i < n; i += st) {
    const double zi = (double)z[i];
    a += zi * (double)r[i];
    if (with_q) c += zi * (double)q[i];
  }
  put_partial(pb, S_RZ0, a, gridDim.x, blockIdx.x);
  put_partial(pb, S_RZ1, c, gridDim.x, blockIdx.x);
}
// p = z + beta p, beta = -z.q_old / p_old.q_old (0 on the first iteration);
// p.r partials (site S_DOT).  Every block sums the r.z and z.q_old partials
// itself (same order in every block); block 0 stores them in fs[0], fs[1].
template <typename T>
__global__ __launch_bounds__(256) void k_fcg_dir(Prob pb, long n, double* __restrict__ fs, int first) {
  const double rz = get_total(pb, S_RZ0);
  const double zq = get_total(pb, S_RZ1);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    fs[0] = rz;
    fs[1] = zq;
  }
  const double beta = (first || !(fs[2] > 0.0)) ? 0.0 : -zq / fs[2];
  const T* z = (const T*)pb.z;
  const T* r = (const T*)pb.r;
  T* p = (T*)pb.p;
  double acc = 0.0;
  const long st = (long)gridDim.x * blockDim.x;
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  // four elements' loads before their stores (same summation order)
  for (; i + 3 * st < n; i += 4 * st) {
    T zs[4], ps[4], rs[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      zs[u] = z[i + u * st];
      ps[u] = beta == 0.0 ? (T)0 : p[i + u * st];
      rs[u] = r[i + u * st];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const T pv = beta == 0.0 ? zs[u] : (T)((double)zs[u] + beta * (double)ps[u]);
      p[i + u * st] = pv;
      acc += (double)pv * (double)rs[u];
    }
  }
  for (; i < n; i += st) {
    const T pv = beta == 0.0 ? z[i] : (T)((double)z[i] + beta * (double)p[i]);
    p[i] = pv;
    acc += (double)pv * (double)r[i];
  }
  put_partial(pb, S_DOT, acc, gridDim.x, blockIdx.x);
}
// alpha = p.r / p.q; x += alpha p; r -= alpha q; r.r partials (site S_RR).
// Every block sums the p.q and p.r partials itself; block 0 stores them in
// fs[2], fs[3].  Nothing happens once the done flag is set (a speculative
// iteration).
template <typename T> __global__ __launch_bounds__(256) void k_fcg_update(Prob pb, long n, double* __restrict__ fs) {
  if (fs[5] != 0.0) return;  // uniform over the grid
  const double pq = get_total(pb, S_PQ);
  const double pr = get_total(pb, S_DOT);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    fs[2] = pq;
    fs[3] = pr;
  }
  const double alpha = (pq > 0.0 && isfinite(pq)) ? pr / pq : 0.0;
  T* x = (T*)pb.x;
  T* r = (T*)pb.r;
  const T* p = (const T*)pb.p;
  const T* q = (const T*)pb.q;
  double acc = 0.0;
  const long st = (long)gridDim.x * blockDim.x;
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  // four elements' loads before their stores (same summation order)
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
    const T rv = r[i] - (T)alpha * q[i];
    r[i] = rv;
    acc += (double)rv * (double)rv;
  }
  put_partial(pb, S_RR, acc, gridDim.x, blockIdx.x);
}
// r.r into fs[4] and the done flag (converged below the threshold fs[6],
// non-finite, or p.q breakdown)
__global__ void k_fcg_check(Prob pb, double* __restrict__ fs) {
  const double rr = get_total(pb, S_RR);
  if (threadIdx.x == 0 && fs[5] == 0.0) {
    const double thr = fs[6];
    fs[4] = rr;
    const double pq = fs[2];
    if (rr <= thr || !isfinite(rr) || !(pq > 0.0) || !isfinite(pq)) {
      fs[5] = 1.0;
      pb.sc->done = 1;  // the sine and FFT passes of later iterations return at once
    }
  }
}

// Training pairs on the operator's grid (FP64 in): R = r / s, T = (D e - r) / s
// with r = M e, s = RMS(r); the pair written into the padded network grid.
__global__ void k_pair_out(const double* __restrict__ r, const double* __restrict__ De, float* __restrict__ R,
                           float* __restrict__ Tt, PadGrid q, const double* __restrict__ rr) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)q.P0 * q.P1 * q.P2) return;
  const int xx = (int)(i % q.P2), yy = (int)((i / q.P2) % q.P1), zz = (int)(i / ((long)q.P1 * q.P2));
  const double ms = *rr / ((double)q.m0 * q.m1 * q.m2);
  const double inv = ms > 0.0 ? 1.0 / sqrt(ms) : 0.0;  // a zero error gives a zero pair
  const bool in = zz < q.m0 && yy < q.m1 && xx < q.m2;
  const long j = ((long)zz * q.m1 + yy) * q.m2 + xx;
  R[i] = in ? (float)(r[j] * inv) : 0.f;
  Tt[i] = in ? (float)((De[j] - r[j]) * inv) : 0.f;
}

}  // namespace fln

using namespace fln;

// ---------------------------------------------------------------------------
// network object
// ---------------------------------------------------------------------------
// Generation counter of network buffers: a graph captured with a network's
// buffers is replayed only while that network's generation is unchanged.
static std::atomic<unsigned long long> g_net_gen{0};

struct fl_net_s {
  hipStream_t stream = nullptr;
  unsigned long long gen = ++g_net_gen;  // renewed by every allocation
  int kd = 1;              // kernel depth: 1 (2D network) or 3 (3D network)
  long nparam = 0, pack = 0;
  float *th = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  u16 *fw = nullptr, *bw = nullptr;
  int step = 0;
  // activations and gradients for capacity B x D x H x W (level 0 pixels)
  long cap = 0;
  u16* act[8] = {};   // a0 a1 a2 a3 c3 c2 c1 c0
  u16* grd[8] = {};   // gc0 gs0 gs1 gs2 ga3 gp3 gp2 gp1
  u16* pool[4] = {};  // pool[l] = pool a[l-1] at level l (1..3)
  float *y = nullptr, *gy = nullptr, *xb = nullptr, *tb = nullptr, *ab = nullptr;
  int ab_cap = 0;
  float* part = nullptr;
  long part_cap = 0;
  double* lpart = nullptr;
  float* losses = nullptr;
  int loss_cap = 0;
  int* idx = nullptr;
  int idx_cap = 0;
  // learned-preconditioner scratch on a solver grid
  long pcap = 0;
  void* pw = nullptr;
  float* palpha = nullptr;
  double* fs = nullptr;   // device scalars of flexible CG
  double* hfs = nullptr;  // pinned host mirror: a seed slot and a ring of two iterations
  hipEvent_t ev[2] = {nullptr, nullptr};
  std::vector<void*> owned;
  ~fl_net_s() {
    for (void* p : owned) (void)hipFree(p);
    if (hfs) (void)hipHostFree(hfs);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  fl_status alloc(void** p, size_t bytes) {
    STCHK(dalloc(p, bytes));
    owned.push_back(*p);
    gen = ++g_net_gen;
    return FL_OK;
  }
};

enum { A0 = 0, A1, A2, A3, C3, C2, C1, C0 };
enum { GC0 = 0, GS0, GS1, GS2, GA3, GP3, GP2, GP1 };

// level-0 pixels shrink by 2^d per level
static int lvl_shift(const fl_net net) { return net->kd == 3 ? 3 : 2; }

static fl_status net_reserve(fl_net net, int B, int D, int H, int W) {
  const long px = (long)B * D * H * W;
  if (px <= net->cap) return FL_OK;
  const int lvl_of_act[8] = {0, 1, 2, 3, 3, 2, 1, 0};
  const int lvl_of_grd[8] = {0, 0, 1, 2, 3, 3, 2, 1};
  const int sh = lvl_shift(net);
  for (int i = 0; i < 8; ++i) {
    STCHK(net->alloc((void**)&net->act[i], (size_t)(px >> (sh * lvl_of_act[i])) * CH * sizeof(u16)));
    STCHK(net->alloc((void**)&net->grd[i], (size_t)(px >> (sh * lvl_of_grd[i])) * CH * sizeof(u16)));
  }
  for (int l = 1; l <= 3; ++l) STCHK(net->alloc((void**)&net->pool[l], (size_t)(px >> (sh * l)) * CH * sizeof(u16)));
  for (float** p : {&net->y, &net->gy, &net->xb, &net->tb}) STCHK(net->alloc((void**)p, px * sizeof(float)));
  net->cap = px;
  return FL_OK;
}

static fl_status net_alphas(fl_net net, int B) {
  if (B <= net->ab_cap) return FL_OK;
  STCHK(net->alloc((void**)&net->ab, (size_t)B * sizeof(float)));
  net->ab_cap = B;
  return FL_OK;
}

static fl_status net_part(fl_net net, long n) {
  if (n <= net->part_cap) return FL_OK;
  STCHK(net->alloc((void**)&net->part, n * sizeof(float)));
  net->part_cap = n;
  return FL_OK;
}

static int conv_blocks(const Dims& g) { return g.B * g.D * ((g.H + TY - 1) / TY) * ((g.W + TX - 1) / TX); }
static dim3 conv_grid(const Dims& g) { return dim3((g.W + TX - 1) / TX, (g.H + TY - 1) / TY, g.B * g.D); }

// 2D networks take D = 1; 3D networks a depth that is a multiple of 8 too
static fl_status check_grid(const fl_net net, int B, int D, int H, int W) {
  if (B < 1 || H < 8 || W < 8) return fail(FL_E_INVALID, "network grid must be at least 8 x 8");
  if (H % 8 || W % 8) return fail(FL_E_INVALID, "network grid sides must be multiples of 8");
  if (net->kd == 1 && D != 1) return fail(FL_E_INVALID, "a 2D network takes D = 1");
  if (net->kd == 3 && (D < 8 || D % 8)) return fail(FL_E_INVALID, "a 3D network needs a depth multiple of 8");
  return FL_OK;
}

// forward pass on x (FP32 [B][D][H][W]) and alphas (device FP32 [B]) into net->y
template <int KD, int G> static fl_status net_forward_t(fl_net net, const float* x, const float* alpha, Dims g0,
                                                        const NetGlue& gl) {
  using P = PL<KD>;
  hipStream_t s = net->stream;
  u16** a = net->act;
  const float* th = net->th;
  auto bias = [&](int L) { return th + P::OFF_L32 + L * P::L32SZ + P::L32W; };
  auto fw = [&](int L) { return (const u16*)(net->fw + L * P::PACK); };
  auto half = [](Dims g) { return Dims{g.B, KD == 3 ? g.D / 2 : 1, g.H / 2, g.W / 2, g.stop}; };
  auto dbl = [](Dims g) { return Dims{g.B, KD == 3 ? g.D * 2 : 1, g.H * 2, g.W * 2, g.stop}; };
  // pooled inputs of the down path, p[l] = pool a[l-1]: in 2D every layer
  // writes the next one's from its output tile, in 3D k_pool forms it
  u16* const* pl = net->pool;
  LAUNCH((k_cin_mfma<KD, G>), conv_grid(g0), dim3(256), 0, s, x, alpha, fw(NL32), th + P::OFF_CIN_B, a[A0], g0,
         KD == 1 ? pl[1] : (u16*)nullptr, gl);
  Dims g = g0;
  // down path
  const int lay[3] = {LD1, LD2, LD3};
  for (int l = 1; l <= 3; ++l) {
    g = half(g);
    u16* po = (KD == 1 && l < 3) ? pl[l + 1] : (u16*)nullptr;
    if constexpr (KD == 3)
      LAUNCH(k_pool<KD>, dim3(nblocks_vec((long)g.B * g.D * g.H * g.W * 4)), dim3(256), 0, s,
             (const u16*)a[A0 + l - 1], pl[l], g);
    Stage st = {pl[l], nullptr, nullptr};
    LAUNCH((k_conv32<SM_PLAIN, EPI_RELU, KD>), conv_grid(g), dim3(256), 0, s, st, fw(lay[l - 1]),
           bias(lay[l - 1]), a[A0 + l], g, po);
  }
  {
    Stage st = {a[A3], nullptr, nullptr};
    LAUNCH((k_conv32<SM_PLAIN, EPI_RELU, KD>), conv_grid(g), dim3(256), 0, s, st, fw(LB3), bias(LB3), a[C3],
           g, (u16*)nullptr);
  }
  // up path: c_l = relu(u_l(a_l + up c_{l+1}))
  const int ulay[3] = {LU2, LU1, LU0};
  const int adst[3] = {C2, C1, C0}, askip[3] = {A2, A1, A0}, acoarse[3] = {C3, C2, C1};
  for (int k = 0; k < 3; ++k) {
    g = dbl(g);
    Stage st = {a[askip[k]], a[acoarse[k]], nullptr};
    LAUNCH((k_conv32<SM_UPADD, EPI_RELU, KD>), conv_grid(g), dim3(256), 0, s, st, fw(ulay[k]), bias(ulay[k]),
           a[adst[k]], g, (u16*)nullptr);
  }
  LAUNCH((k_out_mfma<KD, G>), conv_grid(g0), dim3(256), 0, s, (const u16*)a[C0], fw(NL32 + 1),
         th + P::OFF_OUT + P::K * CH, g0, net->y, gl);
  return FL_OK;
}

// G = 0: input x, output net->y.  G = 1 / 2: the solver-grid glue gl with
// T = float / double (x unused, B = 1).
template <int G = 0>
static fl_status net_forward(fl_net net, const float* x, const float* alpha, int B, int D, int H, int W,
                             const double* stop = nullptr, const NetGlue& gl = NetGlue{}) {
  STCHK(check_grid(net, B, D, H, W));
  STCHK(net_reserve(net, B, D, H, W));
  const Dims g{B, D, H, W, stop};
  return net->kd == 3 ? net_forward_t<3, G>(net, x, alpha, g, gl) : net_forward_t<1, G>(net, x, alpha, g, gl);
}

// reverse pass from net->gy (dL/dy) into net->g (parameter gradient), after net_forward on the same input
template <int KD> static fl_status net_backward_t(fl_net net, const float* x, const float* alpha, Dims g0) {
  using P = PL<KD>;
  hipStream_t s = net->stream;
  const long px = (long)g0.B * g0.D * g0.H * g0.W;
  u16** a = net->act;
  u16** gr = net->grd;
  const float* th = net->th;
  auto bw = [&](int L) { return (const u16*)(net->bw + L * P::PACK); };
  const int maxblk = 1024, nsplit = 32;
  // per-block partials, then the nsplit partial sums of the two-stage reduction
  STCHK(net_part(net, (long)(maxblk + nsplit) * P::L32SZ));
  auto wgrad_blocks = [&](const Dims& g) { return std::min(maxblk, conv_blocks(g)); };
  auto reduce = [&](int nblk, long stride, long nval, long off) -> fl_status {
    const unsigned gx = (unsigned)((nval + 255) / 256);
    if (nblk <= 2 * nsplit) {
      LAUNCH(k_reduce_part, dim3(gx), dim3(256), 0, s, (const float*)net->part, nblk, (int)stride, (int)nval,
             net->g + off);
      return FL_OK;
    }
    float* tmp = net->part + (long)maxblk * P::L32SZ;
    LAUNCH(k_reduce_part_s1, dim3(gx, nsplit), dim3(256), 0, s, (const float*)net->part, nblk, (int)stride,
           (int)nval, tmp);
    LAUNCH(k_reduce_part, dim3(gx), dim3(256), 0, s, (const float*)tmp, nsplit, (int)nval, (int)nval,
           net->g + off);
    return FL_OK;
  };
  // output layer
  LAUNCH(k_cout_bwd<KD>, dim3(nblocks_vec(4 * px)), dim3(256), 0, s, (const float*)net->gy, th + P::OFF_OUT, gr[GC0],
         g0);
  {
    const int nb = wgrad_blocks(g0);
    LAUNCH(k_cout_wgrad<KD>, dim3(nb, KD), dim3(256), 0, s, (const u16*)a[C0], (const float*)net->gy, net->part, g0);
    STCHK(reduce(nb, P::OUT_PV, P::OUT_PV, P::OFF_OUT));
  }
  // one 32 -> 32 layer: reverse convolution into gin (if any) and weight gradient
  auto layer = [&](int L, auto smi, auto smg, Stage si, Stage sg, u16* gin, Dims g) -> fl_status {
    constexpr int SMI = decltype(smi)::value, SMG = decltype(smg)::value;
    if (gin)
      LAUNCH((k_conv32<SMG, EPI_NONE, KD>), conv_grid(g), dim3(256), 0, s, sg, bw(L), (const float*)nullptr,
             gin, g, (u16*)nullptr);
    const int nb = wgrad_blocks(g);
    LAUNCH((k_conv32_wgrad<SMI, SMG, KD>), dim3(nb, KD), dim3(256), 0, s, si, sg, net->part, g);
    return reduce(nb, P::L32SZ, P::L32SZ, P::OFF_L32 + L * P::L32SZ);
  };
  using IP = std::integral_constant<int, SM_PLAIN>;
  using IPO = std::integral_constant<int, SM_POOL>;
  using IU = std::integral_constant<int, SM_UPADD>;
  using GP = std::integral_constant<int, SM_GPLAIN>;
  using GS = std::integral_constant<int, SM_GSUMPOOL>;
  using GA = std::integral_constant<int, SM_GADDUP>;
  auto half = [](Dims g) { return Dims{g.B, KD == 3 ? g.D / 2 : 1, g.H / 2, g.W / 2}; };
  const Dims g1 = half(g0), g2 = half(g1), g3 = half(g2);
  // u0: c0 = relu(u0(a0 + up c1))
  STCHK(layer(LU0, IU{}, GP{}, Stage{a[A0], a[C1], nullptr}, Stage{gr[GC0], nullptr, a[C0]}, gr[GS0], g0));
  STCHK(layer(LU1, IU{}, GS{}, Stage{a[A1], a[C2], nullptr}, Stage{gr[GS0], nullptr, a[C1]}, gr[GS1], g1));
  STCHK(layer(LU2, IU{}, GS{}, Stage{a[A2], a[C3], nullptr}, Stage{gr[GS1], nullptr, a[C2]}, gr[GS2], g2));
  STCHK(layer(LB3, IP{}, GS{}, Stage{a[A3], nullptr, nullptr}, Stage{gr[GS2], nullptr, a[C3]}, gr[GA3], g3));
  STCHK(layer(LD3, IPO{}, GP{}, Stage{a[A2], nullptr, nullptr}, Stage{gr[GA3], nullptr, a[A3]}, gr[GP3], g3));
  STCHK(layer(LD2, IPO{}, GA{}, Stage{a[A1], nullptr, nullptr}, Stage{gr[GS2], gr[GP3], a[A2]}, gr[GP2], g2));
  STCHK(layer(LD1, IPO{}, GA{}, Stage{a[A0], nullptr, nullptr}, Stage{gr[GS1], gr[GP2], a[A1]}, gr[GP1], g1));
  {
    const int nb = wgrad_blocks(g0);
    Stage sg = {gr[GS0], gr[GP1], a[A0]};
    LAUNCH((k_cin_wgrad<SM_GADDUP, KD>), dim3(nb, KD), dim3(256), 0, s, x, alpha, sg, net->part, g0);
    STCHK(reduce(nb, P::CIN_PV, P::CIN_PV, 0));
  }
  return FL_OK;
}

static fl_status net_backward(fl_net net, const float* x, const float* alpha, int B, int D, int H, int W) {
  const Dims g{B, D, H, W};
  return net->kd == 3 ? net_backward_t<3>(net, x, alpha, g) : net_backward_t<1>(net, x, alpha, g);
}

static fl_status net_pack(fl_net net) {
  if (net->kd == 3)
    LAUNCH(k_pack<3>, dim3(nblocks_vec(NPACK * net->pack)), dim3(256), 0, net->stream, (const float*)net->th, net->fw,
           net->bw);
  else
    LAUNCH(k_pack<1>, dim3(nblocks_vec(NPACK * net->pack)), dim3(256), 0, net->stream, (const float*)net->th, net->fw,
           net->bw);
  return FL_OK;
}

static fl_status alphas_to_device(fl_net net, const double* alpha, int B) {
  std::vector<float> h(B);
  for (int i = 0; i < B; ++i) h[i] = (float)alpha[i];
  STCHK(net_alphas(net, B));
  HIPCHK(hipMemcpyAsync(net->ab, h.data(), B * sizeof(float), hipMemcpyHostToDevice, net->stream));
  HIPCHK(hipStreamSynchronize(net->stream));
  return FL_OK;
}

// The op's grid inside the padded network grid (each side rounded up to a
// multiple of 8; D = 1 for 2D).
static PadGrid pad_grid(fl_op op) {
  PadGrid q;
  if (op->d == 3) {
    q = {op->n[0], op->n[1], op->n[2], 0, 0, 0};
  } else {
    q = {1, op->n[0], op->n[1], 0, 0, 0};
  }
  q.P0 = op->d == 3 ? (q.m0 + 7) / 8 * 8 : 1;
  q.P1 = (q.m1 + 7) / 8 * 8;
  q.P2 = (q.m2 + 7) / 8 * 8;
  return q;
}

// ---------------------------------------------------------------------------
// learned flexible CG (host-driven, FP64 reductions)
// ---------------------------------------------------------------------------
// z = B (r + s N(r/s, alpha)), B the inverse of the sine-basis diagonal; s
// from the device value r.r in net->fs[4].
template <typename T> static fl_status learned_prec(fl_op op, fl_net net, const Prob& pb) {
  const PadGrid q = pad_grid(op);
  NetGlue gl;
  gl.r = pb.r;
  gl.w = net->pw;
  gl.rr = net->fs + 4;
  gl.q = q;
  STCHK((net_forward<sizeof(T) == 4 ? 1 : 2>(net, nullptr, net->palpha, 1, q.P0, q.P1, q.P2, net->fs + 5, gl)));
  Prob pz = pb;
  STCHK(set_precond<T>(op, pz, FL_PC_SPECTRAL));
  pz.in = net->pw;
  pz.out = pb.z;
  pz.mask = nullptr;
  return precond_seq<T, DPRO_PLAIN, DEPI_FINAL>(op, pz, Iter{0, 0}, 1);
}

template <typename T> static fl_status fd_prec(fl_op op, const Prob& pb) {
  Prob pz = pb;
  STCHK(set_precond<T>(op, pz, FL_PC_FD));
  pz.pcs = op->cst[0] * std::fabs(op->cst[2]) * std::pow(op->h, -op->alpha);
  pz.in = pb.r;
  pz.out = pb.z;
  return precond_seq<T, DPRO_PLAIN, DEPI_FINAL>(op, pz, Iter{0, 0}, 1);
}

template <typename T> static fl_status dot_to(fl_op op, const Prob& pb, const void* a, const void* b, double* dst) {
  hipStream_t s = op->stream;
  LAUNCH(k_dot<T>, dim3(std::min<long>(1024, nblocks_vec(op->N))), dim3(256), 0, s, pb, a, b, (int)S_DOT, op->N);
  LAUNCH(k_total_to, dim3(1), dim3(256), 0, s, pb, (int)S_DOT, dst);
  return FL_OK;
}

// Flexible CG (truncated to one previous direction): alpha_k = p.r / p.q,
// beta_k = -z_{k+1}.q_k / p_k.q_k, every scalar computed and used on the
// device; the host reads r.z, p.q and r.r of each iteration (a copy into a
// pinned ring, one event per slot).  While the observed contraction of r.r
// predicts that iteration k will not converge, iteration k+1 is enqueued
// before k is read, so the GPU does not wait for the host.  If k converges
// anyway, the device done flag turns the update of k+1 into a no-op and x, r
// stay those of iteration k.  r holds the initial residual, x the initial
// iterate; rr0 = r.r, ff = f.f.  Fallback: the FD preconditioner once
// r.z <= 0 or 5 iterations fail to cut ||r|| by 1% (from the next iteration
// enqueued).  graph != 0: iterations with the learned preconditioner are
// replayed from three captured graphs (the first iteration, and one per ring
// slot after it; kept in the workspace while the Prob and the network's
// buffers stay the same), so that the host enqueues one launch per iteration
// instead of some thirty.
template <typename T>
fl_status learned_fcg(fl_op op, fl_net net, const Prob& pb, double tol, int maxit, double ff, double rr0, int graph,
                      int* iters, double* rr_out, int* status, int* fell_back) {
  hipStream_t s = op->stream;
  const long N = op->N;
  const double thr = tol * tol * ff;
  double* fs = net->fs;
  double rr = rr0;
  int it = 0, stall = 0;
  bool fb = false;
  double best = rr0;
  *status = 0;
  if (!(ff > 0.0) || rr <= thr) {
    *iters = 0;
    *rr_out = rr;
    *status = 1;
    *fell_back = 0;
    return FL_OK;
  }
  double* h = net->hfs;  // [8] seed, then the ring [2][8]
  h[4] = rr0;
  h[5] = 0.0;
  h[6] = thr;
  HIPCHK(hipMemcpyAsync(fs + 4, h + 4, 3 * sizeof(double), hipMemcpyHostToDevice, s));
  // the passes of an iteration check pb.sc->done (set with fs[5] by k_fcg_check)
  HIPCHK(hipMemsetAsync(&pb.sc->done, 0, sizeof(pb.sc->done), s));
  const int nupd = (int)std::min<long>(1024, nblocks_vec(N));
  const int ndot = (int)std::min<long>(512, nblocks_vec(N));
  // the launches of iteration k (its scalars into ring slot k & 1)
  auto body = [&](int k, bool use_fd) -> fl_status {
    if (!use_fd) STCHK(learned_prec<T>(op, net, pb));
    else STCHK(fd_prec<T>(op, pb));
    LAUNCH(k_fcg_dots<T>, dim3(ndot), dim3(256), 0, s, pb, N, k > 0 ? 1 : 0);
    LAUNCH(k_fcg_dir<T>, dim3(ndot), dim3(256), 0, s, pb, N, fs, k == 0 ? 1 : 0);
    Prob pa = pb;
    pa.in = pb.p;
    STCHK((apply_seq<T, PRO_PLAIN, EPI_PQ>(op, pa, Iter{0, 0}, 1)));
    LAUNCH(k_fcg_update<T>, dim3(nupd), dim3(256), 0, s, pb, N, fs);
    LAUNCH(k_fcg_check, dim3(1), dim3(256), 0, s, pb, fs);
    HIPCHK(hipMemcpyAsync(h + 8 + 8 * (k & 1), fs, 6 * sizeof(double), hipMemcpyDeviceToHost, s));
    return FL_OK;
  };
  Workspace& w = op->ws[tix<T>()];
  bool use_graph = graph != 0 && s != nullptr;
  // The sine-basis diagonal is built (once per op) before any capture, so
  // that the captured launches allocate nothing.
  auto capture = [&]() -> fl_status {
    if (w.lexec[0] && w.lexec[1] && w.lexec[2] && w.lgen == net->gen && w.lkey.size() == sizeof(Prob) &&
        std::memcmp(w.lkey.data(), &pb, sizeof(Prob)) == 0)
      return FL_OK;
    for (hipGraphExec_t& g : w.lexec)
      if (g) {
        (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
    w.lkey.clear();
    STCHK(build_tau(op));
    for (int slot = 0; slot < 3; ++slot) {
      hipGraph_t g;
      HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      const fl_status st = body(slot == 0 ? 2 : slot == 1 ? 1 : 0, false);
      const hipError_t e = hipStreamEndCapture(s, &g);
      if (st != FL_OK) return st;
      HIPCHK(e);
      const hipError_t ei = hipGraphInstantiate(&w.lexec[slot], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIPCHK(ei);
    }
    w.lgen = net->gen;
    w.lkey.assign((const unsigned char*)&pb, (const unsigned char*)&pb + sizeof(Prob));
    return FL_OK;
  };
  bool captured = false;
  auto enqueue = [&](int k, bool use_fd) -> fl_status {
    if (!use_fd && use_graph) {
      if (!captured) {
        STCHK(capture());
        captured = true;
      }
      HIPCHK(hipGraphLaunch(w.lexec[k == 0 ? 2 : k & 1], s));
    } else {
      STCHK(body(k, use_fd));
    }
    HIPCHK(hipEventRecord(net->ev[k & 1], s));
    return FL_OK;
  };
  int enq = 0;
  double rr_before = rr0;  // r.r one iteration before the last one read
  for (;;) {
    if (enq == it) {  // the iteration to read next is not in flight yet
      STCHK(enqueue(enq, fb));
      ++enq;
    }
    if (enq == it + 1 && enq < maxit) {  // speculate on the next one?
      // predicted r.r after the iteration in flight: the last contraction again
      const bool ahead = it == 0 || rr * (rr / std::max(rr_before, 1e-300)) > 4.0 * thr;
      if (ahead) {
        STCHK(enqueue(enq, fb));
        ++enq;
      }
    }
    HIPCHK(hipEventSynchronize(net->ev[it & 1]));
    const double* hk = h + 8 + 8 * (it & 1);
    const double rz = hk[0], pq = hk[2];
    rr_before = rr;
    rr = hk[4];
    if (!(pq > 0.0) || !std::isfinite(pq)) {
      *status = 3;
      break;
    }
    ++it;
    if (!std::isfinite(rr)) {
      *status = 3;
      break;
    }
    if (rr <= thr) {
      *status = 1;
      break;
    }
    if (it >= maxit) {
      *status = 2;
      break;
    }
    if (!fb && !(rz > 0.0 && std::isfinite(rz))) fb = true;  // not a descent direction
    if (rr < 0.99 * best) {
      best = rr;
      stall = 0;
    } else if (++stall >= 5 && !fb) {
      fb = true;  // stagnation: judge with the FD preconditioner
    }
  }
  HIPCHK(hipStreamSynchronize(s));  // the speculative iteration has drained
  *iters = it;
  *rr_out = rr;
  *fell_back = fb ? 1 : 0;
  return FL_OK;
}

template fl_status learned_fcg<float>(fl_op, fl_net, const Prob&, double, int, double, double, int, int*, double*, int*,
                                      int*);
template fl_status learned_fcg<double>(fl_op, fl_net, const Prob&, double, int, double, double, int, int*, double*, int*,
                                       int*);

// scratch of the learned preconditioner on op's grid
fl_status learned_prepare(fl_op op, fl_net net, size_t elem) {
  if (!net) return fail(FL_E_INVALID, "the learned preconditioner needs opts->net");
  if (op->d != 2 && op->d != 3) return fail(FL_E_UNSUPPORTED, "the learned preconditioner is built for d = 2, 3");
  if ((op->d == 3) != (net->kd == 3)) return fail(FL_E_INVALID, "the network and the op differ in dimension");
  if (net->stream != op->stream) return fail(FL_E_INVALID, "net and op must share one stream");
  const PadGrid q = pad_grid(op);
  STCHK(check_grid(net, 1, q.P0, q.P1, q.P2));
  if (net->pcap < op->N) {
    STCHK(net->alloc(&net->pw, (size_t)op->N * sizeof(double)));
    net->pcap = op->N;
  }
  if (!net->palpha) STCHK(net->alloc((void**)&net->palpha, sizeof(float)));
  if (!net->fs) STCHK(net->alloc((void**)&net->fs, 8 * sizeof(double)));
  if (!net->hfs && hipHostMalloc((void**)&net->hfs, 24 * sizeof(double)) != hipSuccess)
    return fail(FL_E_NOMEM, "pinned host scalars");
  for (hipEvent_t& e : net->ev)
    if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  // alpha as a kernel argument: no copy from host memory, so no host wait
  LAUNCH(k_fill<float>, dim3(1), dim3(64), 0, op->stream, net->palpha, (float)op->alpha, 1L);
  STCHK(net_reserve(net, 1, q.P0, q.P1, q.P2));
  (void)elem;
  return FL_OK;
}

// one profiled launch (fl_net_profile)
template <int KD> static fl_status profile_one(fl_net net, int which, Dims g) {
  using P = PL<KD>;
  hipStream_t s = net->stream;
  u16** a = net->act;
  if (which == 0) return net_forward(net, net->xb, net->ab, g.B, g.D, g.H, g.W);
  if (which == 1) {
    Stage st = {a[A0], a[C1], nullptr};
    LAUNCH((k_conv32<SM_UPADD, EPI_RELU, KD>), conv_grid(g), dim3(256), 0, s, st,
           (const u16*)(net->fw + LU0 * P::PACK), (const float*)(net->th + P::OFF_L32 + LU0 * P::L32SZ + P::L32W),
           a[C0], g, (u16*)nullptr);
    return FL_OK;
  }
  if (which == 2) {
    LAUNCH(k_cin_mfma<KD>, conv_grid(g), dim3(256), 0, s, (const float*)net->xb, (const float*)net->ab,
           (const u16*)(net->fw + NL32 * P::PACK), (const float*)(net->th + P::OFF_CIN_B), a[A0], g, (u16*)nullptr, NetGlue{});
    return FL_OK;
  }
  LAUNCH(k_out_mfma<KD>, conv_grid(g), dim3(256), 0, s, (const u16*)a[C0],
         (const u16*)(net->fw + (NL32 + 1) * P::PACK), (const float*)(net->th + P::OFF_OUT + P::K * CH), g, net->y, NetGlue{});
  return FL_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

fl_status fl_net_create(int d, void* hip_stream, fl_net* out) {
  if (!out) return fail(FL_E_INVALID, "out is NULL");
  *out = nullptr;
  if (d != 2 && d != 3) return fail(FL_E_INVALID, "d must be 2 or 3");
  fl_net net = new fl_net_s();
  net->stream = (hipStream_t)hip_stream;
  net->kd = d == 3 ? 3 : 1;
  net->nparam = d == 3 ? PL<3>::NPARAM : PL<1>::NPARAM;
  net->pack = d == 3 ? PL<3>::PACK : PL<1>::PACK;
  fl_status st = FL_OK;
  for (float** p : {&net->th, &net->g, &net->m, &net->v})
    if (st == FL_OK) st = net->alloc((void**)p, net->nparam * sizeof(float));
  if (st == FL_OK) st = net->alloc((void**)&net->fw, NPACK * net->pack * sizeof(u16));
  if (st == FL_OK) st = net->alloc((void**)&net->bw, NL32 * net->pack * sizeof(u16));
  if (st != FL_OK) {
    delete net;
    return st;
  }
  for (float* p : {net->th, net->m, net->v})
    if (hipMemsetAsync(p, 0, net->nparam * sizeof(float), net->stream) != hipSuccess) {
      delete net;
      return fail(FL_E_HIP, "clearing the parameters failed");
    }
  if (net_pack(net) != FL_OK || hipStreamSynchronize(net->stream) != hipSuccess) {
    delete net;
    return fail(FL_E_HIP, "packing the weights failed");
  }
  *out = net;
  return FL_OK;
}

int64_t fl_net_nparams(int d) { return d == 3 ? PL<3>::NPARAM : d == 2 ? PL<1>::NPARAM : 0; }

fl_status fl_net_set_params(fl_net net, const float* params) {
  if (!net || !params) return fail(FL_E_INVALID, "NULL argument");
  HIPCHK(hipMemcpyAsync(net->th, params, net->nparam * sizeof(float), hipMemcpyDeviceToDevice, net->stream));
  HIPCHK(hipMemsetAsync(net->m, 0, net->nparam * sizeof(float), net->stream));
  HIPCHK(hipMemsetAsync(net->v, 0, net->nparam * sizeof(float), net->stream));
  net->step = 0;
  STCHK(net_pack(net));
  HIPCHK(hipStreamSynchronize(net->stream));
  return FL_OK;
}

fl_status fl_net_get_params(fl_net net, float* params) {
  if (!net || !params) return fail(FL_E_INVALID, "NULL argument");
  HIPCHK(hipMemcpyAsync(params, net->th, net->nparam * sizeof(float), hipMemcpyDeviceToDevice, net->stream));
  HIPCHK(hipStreamSynchronize(net->stream));
  return FL_OK;
}

fl_status fl_net_forward(fl_net net, const float* x, const double* alpha, float* y, int batch, int D, int H, int W) {
  if (!net || !x || !alpha || !y) return fail(FL_E_INVALID, "NULL argument");
  STCHK(check_grid(net, batch, D, H, W));
  STCHK(alphas_to_device(net, alpha, batch));
  STCHK(net_forward(net, x, net->ab, batch, D, H, W));
  HIPCHK(hipMemcpyAsync(y, net->y, (size_t)batch * D * H * W * sizeof(float), hipMemcpyDeviceToDevice, net->stream));
  HIPCHK(hipStreamSynchronize(net->stream));
  return FL_OK;
}

fl_status fl_net_grad(fl_net net, const float* x, const double* alpha, const float* gy, float* grad, int batch, int D,
                      int H, int W) {
  if (!net || !x || !alpha || !gy || !grad) return fail(FL_E_INVALID, "NULL argument");
  STCHK(check_grid(net, batch, D, H, W));
  STCHK(alphas_to_device(net, alpha, batch));
  STCHK(net_forward(net, x, net->ab, batch, D, H, W));
  HIPCHK(hipMemcpyAsync(net->gy, gy, (size_t)batch * D * H * W * sizeof(float), hipMemcpyDeviceToDevice, net->stream));
  STCHK(net_backward(net, x, net->ab, batch, D, H, W));
  HIPCHK(hipMemcpyAsync(grad, net->g, net->nparam * sizeof(float), hipMemcpyDeviceToDevice, net->stream));
  HIPCHK(hipStreamSynchronize(net->stream));
  return FL_OK;
}

fl_status fl_net_train(fl_net net, const float* R, const float* T, const float* A, int npairs, int D, int H, int W,
                       const int* idx, int steps, int batch, double lr, float* losses) {
  if (!net || !R || !T || !A || !idx || !losses) return fail(FL_E_INVALID, "NULL argument");
  if (npairs < 1 || steps < 0 || !(lr > 0.0)) return fail(FL_E_INVALID, "npairs, steps or lr");
  STCHK(check_grid(net, batch, D, H, W));
  for (long i = 0; i < (long)steps * batch; ++i)
    if (idx[i] < 0 || idx[i] >= npairs) return fail(FL_E_INVALID, "minibatch index out of range");
  hipStream_t s = net->stream;
  STCHK(net_reserve(net, batch, D, H, W));
  STCHK(net_alphas(net, batch));
  const long npix = (long)D * H * W, n = (long)batch * npix;
  if (net->idx_cap < steps * batch) {
    STCHK(net->alloc((void**)&net->idx, (size_t)std::max(1, steps * batch) * sizeof(int)));
    net->idx_cap = steps * batch;
  }
  if (net->loss_cap < steps) {
    STCHK(net->alloc((void**)&net->losses, (size_t)std::max(1, steps) * sizeof(float)));
    net->loss_cap = steps;
  }
  if (!net->lpart) STCHK(net->alloc((void**)&net->lpart, 1024 * sizeof(double)));
  HIPCHK(hipMemcpyAsync(net->idx, idx, (size_t)steps * batch * sizeof(int), hipMemcpyHostToDevice, s));
  const int lblk = (int)std::min<long>(1024, nblocks_vec(n));
  const float b1 = 0.9f, b2 = 0.999f;
  for (int k = 0; k < steps; ++k) {
    LAUNCH(k_gather, dim3(nblocks_vec(n)), dim3(256), 0, s, R, T, A, (const int*)net->idx + (long)k * batch, net->xb,
           net->tb, net->ab, batch, npix);
    STCHK(net_forward(net, net->xb, net->ab, batch, D, H, W));
    LAUNCH(k_loss, dim3(lblk), dim3(256), 0, s, (const float*)net->y, (const float*)net->tb, net->gy, net->lpart, n,
           1.0 / (double)n);
    LAUNCH(k_sum_to, dim3(1), dim3(256), 0, s, (const double*)net->lpart, lblk, net->losses + k);
    STCHK(net_backward(net, net->xb, net->ab, batch, D, H, W));
    ++net->step;
    const double c1 = 1.0 / (1.0 - std::pow((double)b1, net->step));
    const double c2 = 1.0 / (1.0 - std::pow((double)b2, net->step));
    LAUNCH(k_adam, dim3(nblocks_vec(net->nparam)), dim3(256), 0, s, net->th, (const float*)net->g, net->m, net->v,
           net->nparam, (float)lr, b1, b2, 1e-8f, (float)c1, (float)c2);
    STCHK(net_pack(net));
  }
  HIPCHK(hipMemcpyAsync(losses, net->losses, (size_t)steps * sizeof(float), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return FL_OK;
}

fl_status fl_learned_pairs(fl_op op, const double* e, int64_t e_stride, const double* e_sub, int count, float* R,
                           float* T, int Dp, int Hp, int Wp) {
  if (!op || !e || !R || !T) return fail(FL_E_INVALID, "NULL argument");
  if (e_stride != 0 && e_stride != op->N) return fail(FL_E_INVALID, "e_stride must be 0 or the grid size");
  if (op->d != 2 && op->d != 3) return fail(FL_E_UNSUPPORTED, "training pairs are built for d = 2, 3");
  STCHK(need_solver_grid(op));
  PadGrid q = pad_grid(op);
  q.P0 = Dp;
  q.P1 = Hp;
  q.P2 = Wp;
  if (count < 1 || Dp < q.m0 || Hp < q.m1 || Wp < q.m2 || (op->d == 2 && Dp != 1))
    return fail(FL_E_INVALID, "count or padded grid");
  const long np = (long)Dp * Hp * Wp;
  hipStream_t s = op->stream;
  const long N = op->N;
  STCHK(ensure_ws<double>(op, 1, true));
  Workspace& w = op->ws[0];
  for (int k = 0; k < count; ++k) {
    const double* ek = e + (long)k * e_stride;
    if (e_sub) {  // e_k = e - e_sub[k] into the workspace's x
      HIPCHK(hipMemcpyAsync(w.x, ek, N * sizeof(double), hipMemcpyDeviceToDevice, s));
      LAUNCH((k_axpby<double, double>), dim3(nblocks_vec(N)), dim3(256), 0, s, e_sub + (long)k * N, (double*)w.x, -1.0,
             1.0, N);
      ek = (const double*)w.x;
    }
    // r = M e into w.r, D e into w.q (D = inverse of the spectral preconditioner with p0 = 0)
    Prob pb = solver_prob<double>(op, nullptr, 0.0, 1.0, 0.0, 1.0);
    pb.in = ek;
    pb.out = w.r;
    STCHK((apply_seq<double, PRO_PLAIN, EPI_PLAIN>(op, pb, Iter{0, 0}, 0)));
    Prob pd = solver_prob<double>(op, nullptr, 0.0, 1.0, 0.0, 1.0);
    STCHK(set_precond<double>(op, pd, FL_PC_SPECTRAL));
    pd.pmul = 1;
    pd.in = ek;
    pd.out = w.q;
    STCHK((precond_seq<double, DPRO_PLAIN, DEPI_FINAL>(op, pd, Iter{0, 0}, 0)));
    STCHK(dot_to<double>(op, pb, w.r, w.r, &pb.sc->rr));
    LAUNCH(k_pair_out, dim3(nblocks_vec(np)), dim3(256), 0, s, (const double*)w.r, (const double*)w.q, R + (long)k * np,
           T + (long)k * np, q, (const double*)&pb.sc->rr);
  }
  HIPCHK(hipStreamSynchronize(s));
  return FL_OK;
}

fl_status fl_net_profile(fl_net net, int which, int D, int H, int W, int reps, double* avg_ms) {
  if (!net || !avg_ms || reps < 1) return fail(FL_E_INVALID, "NULL argument or reps < 1");
  if (which < 0 || which > 3) return fail(FL_E_INVALID, "which must be 0..3");
  STCHK(check_grid(net, 1, D, H, W));
  STCHK(net_reserve(net, 1, D, H, W));
  STCHK(net_alphas(net, 1));
  hipStream_t s = net->stream;
  const long px = (long)D * H * W;
  LAUNCH(k_fill<float>, dim3(nblocks_vec(px)), dim3(256), 0, s, net->xb, 0.5f, px);
  LAUNCH(k_fill<float>, dim3(1), dim3(256), 0, s, net->ab, 1.0f, 1L);
  STCHK(net_forward(net, net->xb, net->ab, 1, D, H, W));
  const Dims g{1, D, H, W};
  auto one = [&]() { return net->kd == 3 ? profile_one<3>(net, which, g) : profile_one<1>(net, which, g); };
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  for (int i = 0; i < reps; ++i) STCHK(one());
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = (double)ms / reps;
  return FL_OK;
}

fl_status fl_net_destroy(fl_net net) {
  if (!net) return FL_OK;
  if (net->stream) (void)hipStreamSynchronize(net->stream);
  delete net;
  return FL_OK;
}

}  // extern "C"
