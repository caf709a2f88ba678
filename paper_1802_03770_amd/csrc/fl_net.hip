// Learned preconditioner: a multilevel convolutional network (BF16 activations,
// FP32 accumulation, FP32 master weights), its training (reverse pass, Adam),
// and flexible CG with z = B (r + s N(r/s, alpha)), B the inverse of the
// operator's sine-basis diagonal, s the RMS of r, and the FD Laplacian
// preconditioner (Sec. 3.1) as the fallback.  Not in the paper.
//
// Network (H, W multiples of 8; ReLU after every convolution but the last;
// 2x2 average pooling, nearest 2x upsampling, additive skips):
//   a0 = relu(cin([x, alpha-1]))   a1 = relu(d1(pool a0))   a2 = relu(d2(pool a1))
//   a3 = relu(d3(pool a2))         c3 = relu(b3(a3))        c2 = relu(u2(a2 + up c3))
//   c1 = relu(u1(a1 + up c2))      c0 = relu(u0(a0 + up c1)) y = out(c0)
// 3x3 zero-padded cross-correlations; parameters W[tap = 3 ky + kx][ci][co]
// then b[co] per layer in the order cin, d1, d2, d3, b3, u2, u1, u0, out.
//
// Layout: activations NHWC bf16 [B][H][W][32]; input and output FP32 [B][H][W].
// The 32 -> 32 convolutions are implicit GEMMs on v_mfma_f32_32x32x16_bf16:
// D[co][pixel] = sum_k W^T[co][k] X[k][pixel], k = (tap, ci), a 64-wide wave
// computing 2 x 32 pixels of one output row against all 32 output channels.
#include <type_traits>

#include "fl_internal.hpp"

namespace fln {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16;

constexpr int CH = 32;
constexpr int NL32 = 7;                      // 32 -> 32 layers d1 d2 d3 b3 u2 u1 u0
constexpr long L32W = 9 * CH * CH;           // weights per 32 -> 32 layer
constexpr long OFF_CIN_B = 9 * 2 * CH;       // 576
constexpr long OFF_L32 = OFF_CIN_B + CH;     // 608
constexpr long L32SZ = L32W + CH;            // 9248
constexpr long OFF_OUT = OFF_L32 + NL32 * L32SZ;  // 65344
constexpr long NPARAM = OFF_OUT + 9 * CH + 1;     // 65633
constexpr long PACK = 18 * 64 * 8;           // packed bf16 per layer (18 fragments x 64 lanes x 8)
enum { LD1 = 0, LD2, LD3, LB3, LU2, LU1, LU0 };

// Tile of one conv block: 4 output rows x 64 output columns.
constexpr int TY = 4, TX = 64, SY = TY + 2, SX = TX + 2;

__device__ __forceinline__ float bf2f(u16 v) { return __uint_as_float((unsigned)v << 16); }
__device__ __forceinline__ u16 f2bf(float f) {  // round to nearest even
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (u16)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
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
  for (int i = 0; i < 4; ++i) w[i] = (unsigned)f2bf(v[2 * i]) | ((unsigned)f2bf(v[2 * i + 1]) << 16);
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// ---------------------------------------------------------------------------
// Staging of a convolution input (8 channels of one in-bounds pixel)
// ---------------------------------------------------------------------------
enum { SM_PLAIN = 0, SM_POOL, SM_UPADD, SM_GPLAIN, SM_GSUMPOOL, SM_GADDUP, SM_INPUT };
//  PLAIN    s0[p]                          (this level)
//  POOL     mean of s0 over the 2x2 block  (s0 at the finer level)
//  UPADD    s0[p] + s1[p/2]                (s1 at the coarser level)
//  GPLAIN   s0[p] * (y[p] > 0)             (gradient through a ReLU)
//  GSUMPOOL sum of s0 over the 2x2 block * (y[p] > 0)
//  GADDUP   (s0[p] + s1[p/2] / 4) * (y[p] > 0)
//  INPUT    channels (x[p], alpha_b - 1, 0, ..., 0): the input layer as a
//           32 -> 32 convolution whose weights vanish beyond input channel 1
struct Stage {
  const u16* s0;
  const u16* s1;
  const u16* y;
  const float* xf = nullptr;  // SM_INPUT: network input x, FP32 [B][H][W]
  const float* al = nullptr;  // SM_INPUT: alpha per image
};

__device__ __forceinline__ long pix(int b, int y, int x, int H, int W) { return (((long)b * H + y) * W + x) * CH; }

template <int SM>
__device__ __forceinline__ void stage8(const Stage& st, int b, int y, int x, int H, int W, int c, float v[8]) {
  if constexpr (SM == SM_INPUT) {
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = 0.f;
    if (c == 0) {
      v[0] = st.xf[((long)b * H + y) * W + x];
      v[1] = st.al[b] - 1.f;
    }
    return;
  }
  if (SM == SM_PLAIN) {
    ld8(st.s0 + pix(b, y, x, H, W) + c, v);
  } else if (SM == SM_POOL || SM == SM_GSUMPOOL) {
    float t[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ld8(st.s0 + pix(b, 2 * y + (q >> 1), 2 * x + (q & 1), 2 * H, 2 * W) + c, t);
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] += t[i];
    }
    if (SM == SM_POOL)
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] *= 0.25f;
  } else {
    ld8(st.s0 + pix(b, y, x, H, W) + c, v);
    if (SM == SM_UPADD || SM == SM_GADDUP) {
      float t[8];
      ld8(st.s1 + pix(b, y >> 1, x >> 1, H >> 1, W >> 1) + c, t);
      const float f = SM == SM_UPADD ? 1.f : 0.25f;
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] += f * t[i];
    }
  }
  if (SM >= SM_GPLAIN && SM <= SM_GADDUP) {
    float a[8];
    ld8(st.y + pix(b, y, x, H, W) + c, a);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = a[i] > 0.f ? v[i] : 0.f;
  }
}

// Stage rows y0-1 .. y0+TY and columns x0-1 .. x0+TX of image b into LDS
// ([SY][SX][32] bf16), zero outside the image.
template <int SM>
__device__ __forceinline__ void stage_tile(u16* tile, const Stage& st, int b, int y0, int x0, int H, int W) {
  for (int e = threadIdx.x; e < SY * SX * 4; e += blockDim.x) {
    const int c = (e & 3) * 8, p = e >> 2;
    const int yy = y0 + p / SX - 1, xx = x0 + p % SX - 1;
    float v[8];
    if (yy >= 0 && yy < H && xx >= 0 && xx < W) {
      stage8<SM>(st, b, yy, xx, H, W, c, v);
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = 0.f;
    }
    *(uint4*)(tile + p * CH + c) = pk8(v);
  }
}

// Forward-mode staging with all global loads of a lane issued before any LDS
// store (the tile has SY*SX*4 = 1584 16-byte chunks, NIT = 7 per lane): the
// memory latency is paid once per tile instead of once per chunk.
template <int SM>
__device__ __forceinline__ void stage_tile_batched(u16* tile, const Stage& st, int b, int y0, int x0, int H, int W) {
  constexpr int NE = SY * SX * 4, NIT = (NE + 255) / 256;
  constexpr int NQ = SM == SM_POOL ? 4 : SM == SM_UPADD ? 2 : 1;
  if constexpr (SM == SM_INPUT) {
    stage_tile<SM>(tile, st, b, y0, x0, H, W);
    return;
  }
  uint4 q[NIT][NQ];
  bool ok[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int e = threadIdx.x + it * 256;
    const int c = (e & 3) * 8, p = e >> 2;
    const int yy = y0 + p / SX - 1, xx = x0 + p % SX - 1;
    ok[it] = e < NE && yy >= 0 && yy < H && xx >= 0 && xx < W;
#pragma unroll
    for (int k = 0; k < NQ; ++k) q[it][k] = make_uint4(0, 0, 0, 0);
    if (ok[it]) {
      if (SM == SM_PLAIN) {
        q[it][0] = *(const uint4*)(st.s0 + pix(b, yy, xx, H, W) + c);
      } else if (SM == SM_UPADD) {
        q[it][0] = *(const uint4*)(st.s0 + pix(b, yy, xx, H, W) + c);
        q[it][1] = *(const uint4*)(st.s1 + pix(b, yy >> 1, xx >> 1, H >> 1, W >> 1) + c);
      } else {  // SM_POOL
#pragma unroll
        for (int k = 0; k < 4; ++k)
          q[it][k] = *(const uint4*)(st.s0 + pix(b, 2 * yy + (k >> 1), 2 * xx + (k & 1), 2 * H, 2 * W) + c);
      }
    }
  }
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int e = threadIdx.x + it * 256;
    if (e >= NE) continue;
    const int c = (e & 3) * 8, p = e >> 2;
    if (SM == SM_PLAIN) {
      *(uint4*)(tile + p * CH + c) = q[it][0];
    } else {
      float v[8], t[8];
      const unsigned* w0 = (const unsigned*)&q[it][0];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        v[2 * i] = __uint_as_float(w0[i] << 16);
        v[2 * i + 1] = __uint_as_float(w0[i] & 0xffff0000u);
      }
#pragma unroll
      for (int k = 1; k < NQ; ++k) {
        const unsigned* wk = (const unsigned*)&q[it][k];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          t[2 * i] = __uint_as_float(wk[i] << 16);
          t[2 * i + 1] = __uint_as_float(wk[i] & 0xffff0000u);
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] += t[i];
      }
      if (SM == SM_POOL)
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] *= 0.25f;
      *(uint4*)(tile + p * CH + c) = pk8(v);
    }
  }
}

// ---------------------------------------------------------------------------
// 32 -> 32 convolution on MFMA (forward with bias + ReLU, or the transposed
// convolution of the reverse pass with flipped, transposed weights)
// ---------------------------------------------------------------------------
// EPI_RELU: bias + ReLU, BF16 out; EPI_NONE: BF16 out; EPI_OUT: the output
// layer, output channel 0 only, FP32 into yout ([B][H][W]).
enum { EPI_RELU = 0, EPI_NONE = 1, EPI_OUT = 2 };

template <int SM, int EPI>
__global__ __launch_bounds__(256) void k_conv32(Stage st, const u16* __restrict__ wpack, const float* __restrict__ bias,
                                                u16* __restrict__ out, int B, int H, int W, float* __restrict__ yout) {
  __shared__ __align__(16) u16 tile[SY * SX * CH];
  const int tilesX = (W + TX - 1) / TX, tilesY = (H + TY - 1) / TY;
  int t = blockIdx.x;
  const int tx = t % tilesX;
  t /= tilesX;
  const int ty = t % tilesY, b = t / tilesY;
  if (b >= B) return;
  const int x0 = tx * TX, y0 = ty * TY;
  if constexpr (SM == SM_PLAIN || SM == SM_UPADD || SM == SM_POOL)
    stage_tile_batched<SM>(tile, st, b, y0, x0, H, W);
  else
    stage_tile<SM>(tile, st, b, y0, x0, H, W);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  bf16x8 wf[18];
#pragma unroll
  for (int f = 0; f < 18; ++f) wf[f] = *(const bf16x8*)(wpack + ((long)f * 64 + lane) * 8);
  __syncthreads();
  f32x16 acc0 = {}, acc1 = {};
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int ky = tap / 3, kx = tap % 3;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const u16* p0 = tile + ((wave + ky) * SX + (lane & 31) + kx) * CH + half * 16 + (lane >> 5) * 8;
      const bf16x8 b0 = *(const bf16x8*)p0;
      const bf16x8 b1 = *(const bf16x8*)(p0 + 32 * CH);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[tap * 2 + half], b0, acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[tap * 2 + half], b1, acc1, 0, 0, 0);
    }
  }
  // lane holds pixel (lane & 31) of each 32-pixel half, channels
  // g*8 + (lane>>5)*4 + 0..3 in acc[4g .. 4g+3]
  if constexpr (EPI == EPI_OUT) {  // channel 0 sits in acc[0] of lanes 0..31
    const int yo = y0 + wave;
    if (lane < 32 && yo < H) {
      const int px0 = x0 + lane, px1 = x0 + 32 + lane;
      if (px0 < W) yout[((long)b * H + yo) * W + px0] = acc0[0] + bias[0];
      if (px1 < W) yout[((long)b * H + yo) * W + px1] = acc1[0] + bias[0];
    }
    return;
  }
  // the wave's 64 x 32 outputs go through LDS so that the global stores are
  // contiguous 16-byte chunks
  __syncthreads();  // every wave is done reading the staged tile
  u16* ot = tile + wave * 64 * CH;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const f32x16& a = m ? acc1 : acc0;
    const int pl = m * 32 + (lane & 31);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int cb = g * 8 + (lane >> 5) * 4;
      float v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        v[i] = a[4 * g + i];
        if (EPI == EPI_RELU) v[i] = fmaxf(v[i] + bias[cb + i], 0.f);
      }
      const unsigned lo = (unsigned)f2bf(v[0]) | ((unsigned)f2bf(v[1]) << 16);
      const unsigned hi = (unsigned)f2bf(v[2]) | ((unsigned)f2bf(v[3]) << 16);
      *(uint2*)(ot + pl * CH + cb) = make_uint2(lo, hi);
    }
  }
  __syncthreads();
  const int yo = y0 + wave;
  if (yo >= H) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = lane + 64 * k, pl = e >> 2, qq = (e & 3) * 8;
    const int px = x0 + pl;
    if (px < W) *(uint4*)(out + pix(b, yo, px, H, W) + qq) = *(const uint4*)(ot + pl * CH + qq);
  }
}

// Weight gradient of a 32 -> 32 layer: per-block partials of
// dW[tap][ci][co] = sum_p X[p + tap][ci] G[p][co] and db[co] = sum_p G[p][co]
// (X staged by SMI, G by SMG), FP32 accumulation; blocks stride over tiles.
template <int SMI, int SMG>
__global__ __launch_bounds__(256) void k_conv32_wgrad(Stage si, Stage sg, float* __restrict__ part, int B, int H,
                                                      int W) {
  __shared__ __align__(16) u16 xt[SY * SX * CH];
  __shared__ __align__(16) u16 gt[TY * TX * CH];
  const int co = threadIdx.x & 31, grp = threadIdx.x >> 5;  // 8 groups of 36 (tap, ci)
  const int tilesX = (W + TX - 1) / TX, tilesY = (H + TY - 1) / TY;
  const int ntiles = B * tilesY * tilesX;
  float acc[36];
#pragma unroll
  for (int j = 0; j < 36; ++j) acc[j] = 0.f;
  float accb = 0.f;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int u = t;
    const int tx = u % tilesX;
    u /= tilesX;
    const int ty = u % tilesY, b = u / tilesY;
    const int x0 = tx * TX, y0 = ty * TY;
    stage_tile<SMI>(xt, si, b, y0, x0, H, W);
    for (int e = threadIdx.x; e < TY * TX * 4; e += blockDim.x) {
      const int c = (e & 3) * 8, p = e >> 2;
      const int yy = y0 + p / TX, xx = x0 + p % TX;
      float v[8];
      if (yy < H && xx < W) {
        stage8<SMG>(sg, b, yy, xx, H, W, c, v);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = 0.f;
      }
      *(uint4*)(gt + p * CH + c) = pk8(v);
    }
    __syncthreads();
    for (int p = 0; p < TY * TX; ++p) {
      const int ly = p / TX, lx = p % TX;
      const float gv = bf2f(gt[p * CH + co]);
      accb += gv;
#pragma unroll
      for (int j = 0; j < 36; ++j) {
        const int q = grp * 36 + j, tap = q >> 5, ci = q & 31;
        acc[j] += bf2f(xt[((ly + tap / 3) * SX + lx + tap % 3) * CH + ci]) * gv;
      }
    }
    __syncthreads();
  }
  float* o = part + (long)blockIdx.x * L32SZ;
#pragma unroll
  for (int j = 0; j < 36; ++j) {
    const int q = grp * 36 + j;
    o[(long)q * CH + co] = acc[j];
  }
  if (grp == 0) o[L32W + co] = accb;
}

// ---------------------------------------------------------------------------
// Input layer (2 -> 32) and output layer (32 -> 1): VALU, FP32 weights
// ---------------------------------------------------------------------------
// Weight gradient of cin: partials of dW[tap][ci][co] (ci: x and alpha - 1) and
// db, the gradient G staged by SMG; 608 values per block.
template <int SMG>
__global__ __launch_bounds__(256) void k_cin_wgrad(const float* __restrict__ x, const float* __restrict__ alpha, Stage sg,
                                                   float* __restrict__ part, int B, int H, int W) {
  __shared__ __align__(16) u16 gt[TY * TX * CH];
  __shared__ float xs[SY * SX][2];
  const int tilesX = (W + TX - 1) / TX, tilesY = (H + TY - 1) / TY;
  const int ntiles = B * tilesY * tilesX;
  float acc[3] = {0.f, 0.f, 0.f};
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int u = t;
    const int tx = u % tilesX;
    u /= tilesX;
    const int ty = u % tilesY, b = u / tilesY;
    const int x0 = tx * TX, y0 = ty * TY;
    for (int p = threadIdx.x; p < SY * SX; p += blockDim.x) {
      const int yy = y0 + p / SX - 1, xx = x0 + p % SX - 1;
      const bool in = yy >= 0 && yy < H && xx >= 0 && xx < W;
      xs[p][0] = in ? x[((long)b * H + yy) * W + xx] : 0.f;
      xs[p][1] = in ? alpha[b] - 1.f : 0.f;
    }
    for (int e = threadIdx.x; e < TY * TX * 4; e += blockDim.x) {
      const int c = (e & 3) * 8, p = e >> 2;
      const int yy = y0 + p / TX, xx = x0 + p % TX;
      float v[8];
      if (yy < H && xx < W) {
        stage8<SMG>(sg, b, yy, xx, H, W, c, v);
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = 0.f;
      }
      *(uint4*)(gt + p * CH + c) = pk8(v);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int e = threadIdx.x + r * 256;
      if (e >= 608) break;
      float s = 0.f;
      if (e < 576) {
        const int tap = e / 64, ci = (e / 32) & 1, co = e & 31;
        for (int p = 0; p < TY * TX; ++p)
          s += xs[(p / TX + tap / 3) * SX + p % TX + tap % 3][ci] * bf2f(gt[p * CH + co]);
      } else {
        const int co = e - 576;
        for (int p = 0; p < TY * TX; ++p) s += bf2f(gt[p * CH + co]);
      }
      acc[r] += s;
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int e = threadIdx.x + r * 256;
    if (e < 608) part[(long)blockIdx.x * 608 + e] = acc[r];
  }
}

// gc0[p][ci] = sum_tap gy[p - off(tap)] W_out[tap][ci] (transposed convolution),
// four lanes per pixel, eight channels each.
__global__ __launch_bounds__(256) void k_cout_bwd(const float* __restrict__ gy, const float* __restrict__ th,
                                                  u16* __restrict__ gc0, int B, int H, int W) {
  __shared__ float ws[9 * CH];
  for (int i = threadIdx.x; i < 9 * CH; i += blockDim.x) ws[i] = th[OFF_OUT + i];
  __syncthreads();
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long idx = t >> 2;
  if (idx >= (long)B * H * W) return;
  const int q = (int)(t & 3) * 8;
  const int xx = (int)(idx % W), yy = (int)((idx / W) % H), b = (int)(idx / ((long)W * H));
  float acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = 0.f;
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int y2 = yy - (tap / 3 - 1), x2 = xx - (tap % 3 - 1);
    if (y2 < 0 || y2 >= H || x2 < 0 || x2 >= W) continue;
    const float g = gy[((long)b * H + y2) * W + x2];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] += g * ws[tap * CH + q + i];
  }
  *(uint4*)(gc0 + idx * CH + q) = pk8(acc);
}

// Weight gradient of out: partials of dW[tap][ci] = sum_p c0[p + tap][ci] gy[p], db = sum gy (289 per block)
__global__ __launch_bounds__(256) void k_cout_wgrad(const u16* __restrict__ c0, const float* __restrict__ gy,
                                                    float* __restrict__ part, int B, int H, int W) {
  __shared__ __align__(16) u16 xt[SY * SX * CH];
  __shared__ float gs[TY * TX];
  const int tilesX = (W + TX - 1) / TX, tilesY = (H + TY - 1) / TY;
  const int ntiles = B * tilesY * tilesX;
  Stage st = {c0, nullptr, nullptr};
  float acc[2] = {0.f, 0.f};
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    int u = t;
    const int tx = u % tilesX;
    u /= tilesX;
    const int ty = u % tilesY, b = u / tilesY;
    const int x0 = tx * TX, y0 = ty * TY;
    stage_tile<SM_PLAIN>(xt, st, b, y0, x0, H, W);
    for (int p = threadIdx.x; p < TY * TX; p += blockDim.x) {
      const int yy = y0 + p / TX, xx = x0 + p % TX;
      gs[p] = (yy < H && xx < W) ? gy[((long)b * H + yy) * W + xx] : 0.f;
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
          s += bf2f(xt[((p / TX + tap / 3) * SX + p % TX + tap % 3) * CH + ci]) * gs[p];
      } else {
        for (int p = 0; p < TY * TX; ++p) s += gs[p];
      }
      acc[r] += s;
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int e = threadIdx.x + r * 256;
    if (e < 289) part[(long)blockIdx.x * 289 + e] = acc[r];
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

// Packed bf16 weights of the 32 -> 32 layers.  Forward (A operand = W^T):
// fw[L][tap][half][lane][e] = W_L[tap][half*16 + 8*(lane/32) + e][lane%32].
// Transposed flipped (reverse pass): bw[L][tap][half][lane][e] =
// W_L[8 - tap][lane%32][half*16 + 8*(lane/32) + e].  Slots L = 7 and 8 of fw
// hold the input layer (input channels >= 2 zero) and the output layer (output
// channels >= 1 zero) in the same form.
constexpr int NPACK = NL32 + 2;
__global__ void k_pack(const float* __restrict__ th, u16* __restrict__ fw, u16* __restrict__ bw) {
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= NPACK * PACK) return;
  const int L = (int)(idx / PACK);
  const int r = (int)(idx % PACK);
  const int e = r & 7, lane = (r >> 3) & 63, f = r >> 9;
  const int tap = f >> 1, half = f & 1;
  const int kk = half * 16 + 8 * (lane >> 5) + e, j = lane & 31;
  if (L < NL32) {
    const float* W = th + OFF_L32 + L * L32SZ;
    fw[idx] = f2bf(W[((long)tap * CH + kk) * CH + j]);
    bw[idx] = f2bf(W[((long)(8 - tap) * CH + j) * CH + kk]);
  } else if (L == NL32) {
    fw[idx] = kk < 2 ? f2bf(th[(tap * 2 + kk) * CH + j]) : (u16)0;
  } else {
    fw[idx] = j == 0 ? f2bf(th[OFF_OUT + tap * CH + kk]) : (u16)0;
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

__global__ void k_sum_to(const double* __restrict__ part, int n, float* __restrict__ dst) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  *dst = (float)s;
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

// Learned-preconditioner input and output on the solver grid (n0 x n1 inside
// the padded Hp x Wp network grid): xin = r / s, w = r + s y, with the RMS
// s = sqrt(rr / (n0 n1)) read from the device (rr = r.r).
template <typename T>
__global__ void k_net_in(const T* __restrict__ r, float* __restrict__ xin, int n0, int n1, int Hp, int Wp,
                         const double* __restrict__ rr) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)Hp * Wp) return;
  const double ms = *rr / ((double)n0 * n1);
  const double inv_s = ms > 0.0 ? 1.0 / sqrt(ms) : 0.0;
  const int yy = (int)(i / Wp), xx = (int)(i % Wp);
  xin[i] = (yy < n0 && xx < n1) ? (float)((double)r[(long)yy * n1 + xx] * inv_s) : 0.f;
}
template <typename T>
__global__ void k_net_out(const T* __restrict__ r, const float* __restrict__ y, T* __restrict__ w, int n0, int n1, int Wp,
                          const double* __restrict__ rr) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)n0 * n1) return;
  const double sc = sqrt(fmax(*rr, 0.0) / ((double)n0 * n1));
  const int yy = (int)(i / n1), xx = (int)(i % n1);
  w[i] = (T)((double)r[i] + sc * (double)y[(long)yy * Wp + xx]);
}

// Flexible CG scalars live on the device: fs[0] = r.z, fs[1] = z.q_old,
// fs[2] = p.q, fs[3] = p.r, fs[4] = r.r.
__global__ void k_total_to(Prob pb, int site, double* __restrict__ dst) {
  const double t = get_total(pb, site);
  if (threadIdx.x == 0) *dst = t;
}
// p = z + beta p, beta = -z.q_old / p_old.q_old (0 on the first iteration)
template <typename T>
__global__ void k_fcg_dir(const T* __restrict__ z, T* __restrict__ p, long n, const double* __restrict__ fs, int first) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double beta = (first || !(fs[2] > 0.0)) ? 0.0 : -fs[1] / fs[2];
  p[i] = beta == 0.0 ? z[i] : (T)((double)z[i] + beta * (double)p[i]);
}
// alpha = p.r / p.q; x += alpha p; r -= alpha q; r.r partials (site S_RR)
template <typename T> __global__ __launch_bounds__(256) void k_fcg_update(Prob pb, long n, const double* __restrict__ fs) {
  const double pq = fs[2];
  const double alpha = (pq > 0.0 && isfinite(pq)) ? fs[3] / pq : 0.0;
  T* x = (T*)pb.x;
  T* r = (T*)pb.r;
  const T* p = (const T*)pb.p;
  const T* q = (const T*)pb.q;
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    x[i] += (T)alpha * p[i];
    const T rv = r[i] - (T)alpha * q[i];
    r[i] = rv;
    acc += (double)rv * (double)rv;
  }
  put_partial(pb, S_RR, acc, gridDim.x, blockIdx.x);
}

// Training pairs on the operator's grid (FP64 in): R = r / s, T = (D e - r) / s
// with r = M e, s = RMS(r); the pair written into the padded Hp x Wp grid.
__global__ void k_pair_out(const double* __restrict__ r, const double* __restrict__ De, float* __restrict__ R,
                           float* __restrict__ Tt, int n0, int n1, int Hp, int Wp, const double* __restrict__ rr) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)Hp * Wp) return;
  const int yy = (int)(i / Wp), xx = (int)(i % Wp);
  const double ms = *rr / ((double)n0 * n1);
  const double inv = ms > 0.0 ? 1.0 / sqrt(ms) : 0.0;  // a zero error gives a zero pair
  const bool in = yy < n0 && xx < n1;
  const long j = (long)yy * n1 + xx;
  R[i] = in ? (float)(r[j] * inv) : 0.f;
  Tt[i] = in ? (float)((De[j] - r[j]) * inv) : 0.f;
}

}  // namespace fln

using namespace fln;

// ---------------------------------------------------------------------------
// network object
// ---------------------------------------------------------------------------
struct fl_net_s {
  hipStream_t stream = nullptr;
  float *th = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  u16 *fw = nullptr, *bw = nullptr;
  int step = 0;
  // activations and gradients for capacity B x H x W (level 0 pixels)
  long cap = 0;
  u16* act[8] = {};   // a0 a1 a2 a3 c3 c2 c1 c0
  u16* grd[8] = {};   // gc0 gs0 gs1 gs2 ga3 gp3 gp2 gp1
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
  float *pin = nullptr, *pout = nullptr;
  void* pw = nullptr;
  float* palpha = nullptr;
  double* fs = nullptr;   // device scalars of flexible CG
  double* hfs = nullptr;  // pinned host mirror
  std::vector<void*> owned;
  ~fl_net_s() {
    for (void* p : owned) (void)hipFree(p);
    if (hfs) (void)hipHostFree(hfs);
  }
  fl_status alloc(void** p, size_t bytes) {
    STCHK(dalloc(p, bytes));
    owned.push_back(*p);
    return FL_OK;
  }
};

enum { A0 = 0, A1, A2, A3, C3, C2, C1, C0 };
enum { GC0 = 0, GS0, GS1, GS2, GA3, GP3, GP2, GP1 };

static fl_status net_reserve(fl_net net, int B, int H, int W) {
  const long px = (long)B * H * W;
  if (px <= net->cap) return FL_OK;
  const int lvl_of_act[8] = {0, 1, 2, 3, 3, 2, 1, 0};
  const int lvl_of_grd[8] = {0, 0, 1, 2, 3, 3, 2, 1};
  for (int i = 0; i < 8; ++i) {
    STCHK(net->alloc((void**)&net->act[i], (size_t)(px >> (2 * lvl_of_act[i])) * CH * sizeof(u16)));
    STCHK(net->alloc((void**)&net->grd[i], (size_t)(px >> (2 * lvl_of_grd[i])) * CH * sizeof(u16)));
  }
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

static int conv_blocks(int B, int H, int W) { return B * ((H + TY - 1) / TY) * ((W + TX - 1) / TX); }

static fl_status check_grid(int B, int H, int W) {
  if (B < 1 || H < 8 || W < 8) return fail(FL_E_INVALID, "network grid must be at least 8 x 8");
  if (H % 8 || W % 8) return fail(FL_E_INVALID, "network grid sides must be multiples of 8");
  return FL_OK;
}

// forward pass on x (FP32 [B][H][W]) and alphas (device FP32 [B]) into net->y
static fl_status net_forward(fl_net net, const float* x, const float* alpha, int B, int H, int W) {
  STCHK(check_grid(B, H, W));
  STCHK(net_reserve(net, B, H, W));
  hipStream_t s = net->stream;
  u16** a = net->act;
  const float* th = net->th;
  auto bias = [&](int L) { return th + OFF_L32 + L * L32SZ + L32W; };
  auto fw = [&](int L) { return net->fw + L * PACK; };
  {
    Stage st = {nullptr, nullptr, nullptr, x, alpha};
    LAUNCH((k_conv32<SM_INPUT, EPI_RELU>), dim3(conv_blocks(B, H, W)), dim3(256), 0, s, st, (const u16*)fw(NL32),
           th + OFF_CIN_B, a[A0], B, H, W, (float*)nullptr);
  }
  int h = H, w = W;
  // down path
  const int lay[3] = {LD1, LD2, LD3};
  for (int l = 1; l <= 3; ++l) {
    h /= 2;
    w /= 2;
    Stage st = {a[A0 + l - 1], nullptr, nullptr};
    LAUNCH((k_conv32<SM_POOL, EPI_RELU>), dim3(conv_blocks(B, h, w)), dim3(256), 0, s, st, (const u16*)fw(lay[l - 1]),
           bias(lay[l - 1]), a[A0 + l], B, h, w, (float*)nullptr);
  }
  {
    Stage st = {a[A3], nullptr, nullptr};
    LAUNCH((k_conv32<SM_PLAIN, EPI_RELU>), dim3(conv_blocks(B, h, w)), dim3(256), 0, s, st, (const u16*)fw(LB3),
           bias(LB3), a[C3], B, h, w, (float*)nullptr);
  }
  // up path: c_l = relu(u_l(a_l + up c_{l+1}))
  const int ulay[3] = {LU2, LU1, LU0};
  const int adst[3] = {C2, C1, C0}, askip[3] = {A2, A1, A0}, acoarse[3] = {C3, C2, C1};
  for (int k = 0; k < 3; ++k) {
    h *= 2;
    w *= 2;
    Stage st = {a[askip[k]], a[acoarse[k]], nullptr};
    LAUNCH((k_conv32<SM_UPADD, EPI_RELU>), dim3(conv_blocks(B, h, w)), dim3(256), 0, s, st, (const u16*)fw(ulay[k]),
           bias(ulay[k]), a[adst[k]], B, h, w, (float*)nullptr);
  }
  {
    Stage st = {a[C0], nullptr, nullptr};
    LAUNCH((k_conv32<SM_PLAIN, EPI_OUT>), dim3(conv_blocks(B, H, W)), dim3(256), 0, s, st, (const u16*)fw(NL32 + 1),
           th + OFF_OUT + 9 * CH, (u16*)nullptr, B, H, W, net->y);
  }
  return FL_OK;
}

// reverse pass from net->gy (dL/dy) into net->g (parameter gradient), after net_forward on the same input
static fl_status net_backward(fl_net net, const float* x, const float* alpha, int B, int H, int W) {
  hipStream_t s = net->stream;
  const long px = (long)B * H * W;
  u16** a = net->act;
  u16** gr = net->grd;
  const float* th = net->th;
  auto bw = [&](int L) { return (const u16*)(net->bw + L * PACK); };
  const int maxblk = 1024;
  STCHK(net_part(net, (long)maxblk * L32SZ));
  auto wgrad_blocks = [&](int b, int h, int w) { return std::min(maxblk, conv_blocks(b, h, w)); };
  auto reduce = [&](int nblk, int stride, int nval, long off) -> fl_status {
    LAUNCH(k_reduce_part, dim3((nval + 255) / 256), dim3(256), 0, s, (const float*)net->part, nblk, stride, nval,
           net->g + off);
    return FL_OK;
  };
  // output layer
  LAUNCH(k_cout_bwd, dim3(nblocks_vec(4 * px)), dim3(256), 0, s, (const float*)net->gy, th, gr[GC0], B, H, W);
  {
    const int nb = wgrad_blocks(B, H, W);
    LAUNCH(k_cout_wgrad, dim3(nb), dim3(256), 0, s, (const u16*)a[C0], (const float*)net->gy, net->part, B, H, W);
    STCHK(reduce(nb, 289, 289, OFF_OUT));
  }
  // one 32 -> 32 layer: reverse convolution into gin (if any) and weight gradient
  auto layer = [&](int L, auto smi, auto smg, Stage si, Stage sg, u16* gin, int h, int w) -> fl_status {
    constexpr int SMI = decltype(smi)::value, SMG = decltype(smg)::value;
    if (gin)
      LAUNCH((k_conv32<SMG, EPI_NONE>), dim3(conv_blocks(B, h, w)), dim3(256), 0, s, sg, bw(L), (const float*)nullptr,
             gin, B, h, w, (float*)nullptr);
    const int nb = wgrad_blocks(B, h, w);
    LAUNCH((k_conv32_wgrad<SMI, SMG>), dim3(nb), dim3(256), 0, s, si, sg, net->part, B, h, w);
    return reduce(nb, (int)L32SZ, (int)L32SZ, OFF_L32 + L * L32SZ);
  };
  using IP = std::integral_constant<int, SM_PLAIN>;
  using IPO = std::integral_constant<int, SM_POOL>;
  using IU = std::integral_constant<int, SM_UPADD>;
  using GP = std::integral_constant<int, SM_GPLAIN>;
  using GS = std::integral_constant<int, SM_GSUMPOOL>;
  using GA = std::integral_constant<int, SM_GADDUP>;
  const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 8, W3 = W / 8;
  // u0: c0 = relu(u0(a0 + up c1))
  STCHK(layer(LU0, IU{}, GP{}, Stage{a[A0], a[C1], nullptr}, Stage{gr[GC0], nullptr, a[C0]}, gr[GS0], H, W));
  STCHK(layer(LU1, IU{}, GS{}, Stage{a[A1], a[C2], nullptr}, Stage{gr[GS0], nullptr, a[C1]}, gr[GS1], H1, W1));
  STCHK(layer(LU2, IU{}, GS{}, Stage{a[A2], a[C3], nullptr}, Stage{gr[GS1], nullptr, a[C2]}, gr[GS2], H2, W2));
  STCHK(layer(LB3, IP{}, GS{}, Stage{a[A3], nullptr, nullptr}, Stage{gr[GS2], nullptr, a[C3]}, gr[GA3], H3, W3));
  STCHK(layer(LD3, IPO{}, GP{}, Stage{a[A2], nullptr, nullptr}, Stage{gr[GA3], nullptr, a[A3]}, gr[GP3], H3, W3));
  STCHK(layer(LD2, IPO{}, GA{}, Stage{a[A1], nullptr, nullptr}, Stage{gr[GS2], gr[GP3], a[A2]}, gr[GP2], H2, W2));
  STCHK(layer(LD1, IPO{}, GA{}, Stage{a[A0], nullptr, nullptr}, Stage{gr[GS1], gr[GP2], a[A1]}, gr[GP1], H1, W1));
  {
    const int nb = wgrad_blocks(B, H, W);
    Stage sg = {gr[GS0], gr[GP1], a[A0]};
    LAUNCH(k_cin_wgrad<SM_GADDUP>, dim3(nb), dim3(256), 0, s, x, alpha, sg, net->part, B, H, W);
    STCHK(reduce(nb, 608, 608, 0));
  }
  return FL_OK;
}

static fl_status net_pack(fl_net net) {
  LAUNCH(k_pack, dim3(nblocks_vec(NPACK * PACK)), dim3(256), 0, net->stream, (const float*)net->th, net->fw, net->bw);
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

// ---------------------------------------------------------------------------
// learned flexible CG (host-driven, FP64 reductions)
// ---------------------------------------------------------------------------
// z = B (r + s N(r/s, alpha)), B the inverse of the sine-basis diagonal; s
// from the device value r.r in net->fs[4].
template <typename T> static fl_status learned_prec(fl_op op, fl_net net, const Prob& pb) {
  hipStream_t s = op->stream;
  const int n0 = op->n[0], n1 = op->n[1];
  const int Hp = (n0 + 7) / 8 * 8, Wp = (n1 + 7) / 8 * 8;
  LAUNCH(k_net_in<T>, dim3(nblocks_vec((long)Hp * Wp)), dim3(256), 0, s, (const T*)pb.r, net->pin, n0, n1, Hp, Wp,
         (const double*)(net->fs + 4));
  STCHK(net_forward(net, net->pin, net->palpha, 1, Hp, Wp));
  LAUNCH(k_net_out<T>, dim3(nblocks_vec(op->N)), dim3(256), 0, s, (const T*)pb.r, (const float*)net->y, (T*)net->pw,
         n0, n1, Wp, (const double*)(net->fs + 4));
  Prob pz = pb;
  STCHK(set_precond<T>(op, pz, FL_PC_SPECTRAL));
  pz.in = net->pw;
  pz.out = pb.z;
  pz.mask = nullptr;
  return precond_seq<T, DPRO_PLAIN, DEPI_FINAL>(op, pz, Iter{0, 0}, 0);
}

template <typename T> static fl_status fd_prec(fl_op op, const Prob& pb) {
  Prob pz = pb;
  STCHK(set_precond<T>(op, pz, FL_PC_FD));
  pz.pcs = op->cst[0] * std::fabs(op->cst[2]) * std::pow(op->h, -op->alpha);
  pz.in = pb.r;
  pz.out = pb.z;
  return precond_seq<T, DPRO_PLAIN, DEPI_FINAL>(op, pz, Iter{0, 0}, 0);
}

template <typename T> static fl_status dot_to(fl_op op, const Prob& pb, const void* a, const void* b, double* dst) {
  hipStream_t s = op->stream;
  LAUNCH(k_dot<T>, dim3(std::min<long>(1024, nblocks_vec(op->N))), dim3(256), 0, s, pb, a, b, (int)S_DOT, op->N);
  LAUNCH(k_total_to, dim3(1), dim3(256), 0, s, pb, (int)S_DOT, dst);
  return FL_OK;
}

// Flexible CG (truncated to one previous direction): alpha_k = p.r / p.q,
// beta_k = -z_{k+1}.q_k / p_k.q_k, every scalar computed and used on the
// device; the host reads r.z, p.q and r.r once per iteration.  r holds the
// initial residual, x the initial iterate; rr0 = r.r, ff = f.f.  Fallback:
// the FD preconditioner for the rest of the solve once r.z <= 0 or 5
// iterations fail to cut ||r|| by 1%.
template <typename T>
fl_status learned_fcg(fl_op op, fl_net net, const Prob& pb, double tol, int maxit, double ff, double rr0, int* iters,
                      double* rr_out, int* status, int* fell_back) {
  hipStream_t s = op->stream;
  const long N = op->N;
  const double thr = tol * tol * ff;
  double* fs = net->fs;
  double* h = net->hfs;
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
  h[4] = rr0;
  HIPCHK(hipMemcpyAsync(fs + 4, h + 4, sizeof(double), hipMemcpyHostToDevice, s));
  const int nupd = (int)std::min<long>(2048, nblocks_vec(N));
  for (;;) {
    if (!fb) STCHK(learned_prec<T>(op, net, pb));
    else STCHK(fd_prec<T>(op, pb));
    STCHK(dot_to<T>(op, pb, pb.r, pb.z, fs + 0));
    if (it > 0) STCHK(dot_to<T>(op, pb, pb.z, pb.q, fs + 1));
    LAUNCH(k_fcg_dir<T>, dim3(nblocks_vec(N)), dim3(256), 0, s, (const T*)pb.z, (T*)pb.p, N, (const double*)fs,
           it == 0 ? 1 : 0);
    Prob pa = pb;
    pa.in = pb.p;
    STCHK((apply_seq<T, PRO_PLAIN, EPI_PQ>(op, pa, Iter{0, 0}, 0)));
    LAUNCH(k_total_to, dim3(1), dim3(256), 0, s, pb, (int)S_PQ, fs + 2);
    STCHK(dot_to<T>(op, pb, pb.p, pb.r, fs + 3));
    LAUNCH(k_fcg_update<T>, dim3(nupd), dim3(256), 0, s, pb, N, (const double*)fs);
    LAUNCH(k_total_to, dim3(1), dim3(256), 0, s, pb, (int)S_RR, fs + 4);
    HIPCHK(hipMemcpyAsync(h, fs, 5 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double rz = h[0], pq = h[2];
    rr = h[4];
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
  *iters = it;
  *rr_out = rr;
  *fell_back = fb ? 1 : 0;
  return FL_OK;
}

template fl_status learned_fcg<float>(fl_op, fl_net, const Prob&, double, int, double, double, int*, double*, int*,
                                      int*);
template fl_status learned_fcg<double>(fl_op, fl_net, const Prob&, double, int, double, double, int*, double*, int*,
                                       int*);

// scratch of the learned preconditioner on op's grid
fl_status learned_prepare(fl_op op, fl_net net, size_t elem) {
  if (!net) return fail(FL_E_INVALID, "the learned preconditioner needs opts->net");
  if (op->d != 2) return fail(FL_E_UNSUPPORTED, "the learned preconditioner is built for d = 2");
  if (net->stream != op->stream) return fail(FL_E_INVALID, "net and op must share one stream");
  const int Hp = (op->n[0] + 7) / 8 * 8, Wp = (op->n[1] + 7) / 8 * 8;
  STCHK(check_grid(1, Hp, Wp));
  const long need = std::max<long>((long)Hp * Wp, op->N);
  if (net->pcap < need) {
    STCHK(net->alloc((void**)&net->pin, (size_t)Hp * Wp * sizeof(float)));
    STCHK(net->alloc(&net->pw, (size_t)op->N * sizeof(double)));
    net->pcap = need;
  }
  if (!net->palpha) STCHK(net->alloc((void**)&net->palpha, sizeof(float)));
  if (!net->fs) STCHK(net->alloc((void**)&net->fs, 8 * sizeof(double)));
  if (!net->hfs && hipHostMalloc((void**)&net->hfs, 8 * sizeof(double)) != hipSuccess)
    return fail(FL_E_NOMEM, "pinned host scalars");
  const float a = (float)op->alpha;
  HIPCHK(hipMemcpyAsync(net->palpha, &a, sizeof(float), hipMemcpyHostToDevice, op->stream));
  HIPCHK(hipStreamSynchronize(op->stream));
  STCHK(net_reserve(net, 1, Hp, Wp));
  (void)elem;
  return FL_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

fl_status fl_net_create(void* hip_stream, fl_net* out) {
  if (!out) return fail(FL_E_INVALID, "out is NULL");
  *out = nullptr;
  fl_net net = new fl_net_s();
  net->stream = (hipStream_t)hip_stream;
  fl_status st = FL_OK;
  for (float** p : {&net->th, &net->g, &net->m, &net->v})
    if (st == FL_OK) st = net->alloc((void**)p, NPARAM * sizeof(float));
  if (st == FL_OK) st = net->alloc((void**)&net->fw, NPACK * PACK * sizeof(u16));
  if (st == FL_OK) st = net->alloc((void**)&net->bw, NL32 * PACK * sizeof(u16));
  if (st != FL_OK) {
    delete net;
    return st;
  }
  for (float* p : {net->th, net->m, net->v})
    if (hipMemsetAsync(p, 0, NPARAM * sizeof(float), net->stream) != hipSuccess) {
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

int64_t fl_net_nparams(void) { return NPARAM; }

fl_status fl_net_set_params(fl_net net, const float* params) {
  if (!net || !params) return fail(FL_E_INVALID, "NULL argument");
  HIPCHK(hipMemcpyAsync(net->th, params, NPARAM * sizeof(float), hipMemcpyDeviceToDevice, net->stream));
  HIPCHK(hipMemsetAsync(net->m, 0, NPARAM * sizeof(float), net->stream));
  HIPCHK(hipMemsetAsync(net->v, 0, NPARAM * sizeof(float), net->stream));
  net->step = 0;
  STCHK(net_pack(net));
  HIPCHK(hipStreamSynchronize(net->stream));
  return FL_OK;
}

fl_status fl_net_get_params(fl_net net, float* params) {
  if (!net || !params) return fail(FL_E_INVALID, "NULL argument");
  HIPCHK(hipMemcpyAsync(params, net->th, NPARAM * sizeof(float), hipMemcpyDeviceToDevice, net->stream));
  HIPCHK(hipStreamSynchronize(net->stream));
  return FL_OK;
}

fl_status fl_net_forward(fl_net net, const float* x, const double* alpha, float* y, int batch, int H, int W) {
  if (!net || !x || !alpha || !y) return fail(FL_E_INVALID, "NULL argument");
  STCHK(check_grid(batch, H, W));
  STCHK(alphas_to_device(net, alpha, batch));
  STCHK(net_forward(net, x, net->ab, batch, H, W));
  HIPCHK(hipMemcpyAsync(y, net->y, (size_t)batch * H * W * sizeof(float), hipMemcpyDeviceToDevice, net->stream));
  HIPCHK(hipStreamSynchronize(net->stream));
  return FL_OK;
}

fl_status fl_net_grad(fl_net net, const float* x, const double* alpha, const float* gy, float* grad, int batch, int H,
                      int W) {
  if (!net || !x || !alpha || !gy || !grad) return fail(FL_E_INVALID, "NULL argument");
  STCHK(check_grid(batch, H, W));
  STCHK(alphas_to_device(net, alpha, batch));
  STCHK(net_forward(net, x, net->ab, batch, H, W));
  HIPCHK(hipMemcpyAsync(net->gy, gy, (size_t)batch * H * W * sizeof(float), hipMemcpyDeviceToDevice, net->stream));
  STCHK(net_backward(net, x, net->ab, batch, H, W));
  HIPCHK(hipMemcpyAsync(grad, net->g, NPARAM * sizeof(float), hipMemcpyDeviceToDevice, net->stream));
  HIPCHK(hipStreamSynchronize(net->stream));
  return FL_OK;
}

fl_status fl_net_train(fl_net net, const float* R, const float* T, const float* A, int npairs, int H, int W,
                       const int* idx, int steps, int batch, double lr, float* losses) {
  if (!net || !R || !T || !A || !idx || !losses) return fail(FL_E_INVALID, "NULL argument");
  if (npairs < 1 || steps < 0 || !(lr > 0.0)) return fail(FL_E_INVALID, "npairs, steps or lr");
  STCHK(check_grid(batch, H, W));
  for (long i = 0; i < (long)steps * batch; ++i)
    if (idx[i] < 0 || idx[i] >= npairs) return fail(FL_E_INVALID, "minibatch index out of range");
  hipStream_t s = net->stream;
  STCHK(net_reserve(net, batch, H, W));
  STCHK(net_alphas(net, batch));
  const long npix = (long)H * W, n = (long)batch * npix;
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
    STCHK(net_forward(net, net->xb, net->ab, batch, H, W));
    LAUNCH(k_loss, dim3(lblk), dim3(256), 0, s, (const float*)net->y, (const float*)net->tb, net->gy, net->lpart, n,
           1.0 / (double)n);
    LAUNCH(k_sum_to, dim3(1), dim3(1), 0, s, (const double*)net->lpart, lblk, net->losses + k);
    STCHK(net_backward(net, net->xb, net->ab, batch, H, W));
    ++net->step;
    const double c1 = 1.0 / (1.0 - std::pow((double)b1, net->step));
    const double c2 = 1.0 / (1.0 - std::pow((double)b2, net->step));
    LAUNCH(k_adam, dim3(nblocks_vec(NPARAM)), dim3(256), 0, s, net->th, (const float*)net->g, net->m, net->v, NPARAM,
           (float)lr, b1, b2, 1e-8f, (float)c1, (float)c2);
    STCHK(net_pack(net));
  }
  HIPCHK(hipMemcpyAsync(losses, net->losses, (size_t)steps * sizeof(float), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return FL_OK;
}

fl_status fl_learned_pairs(fl_op op, const double* e, int64_t e_stride, const double* e_sub, int count, float* R,
                           float* T, int Hp, int Wp) {
  if (!op || !e || !R || !T) return fail(FL_E_INVALID, "NULL argument");
  if (e_stride != 0 && e_stride != op->N) return fail(FL_E_INVALID, "e_stride must be 0 or the grid size");
  if (op->d != 2) return fail(FL_E_UNSUPPORTED, "training pairs are built for d = 2");
  if (count < 1 || Hp < op->n[0] || Wp < op->n[1]) return fail(FL_E_INVALID, "count or padded grid");
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
    LAUNCH(k_pair_out, dim3(nblocks_vec((long)Hp * Wp)), dim3(256), 0, s, (const double*)w.r, (const double*)w.q,
           R + (long)k * Hp * Wp, T + (long)k * Hp * Wp, op->n[0], op->n[1], Hp, Wp,
           (const double*)&pb.sc->rr);
  }
  HIPCHK(hipStreamSynchronize(s));
  return FL_OK;
}

fl_status fl_net_profile(fl_net net, int which, int H, int W, int reps, double* avg_ms) {
  if (!net || !avg_ms || reps < 1) return fail(FL_E_INVALID, "NULL argument or reps < 1");
  if (which < 0 || which > 3) return fail(FL_E_INVALID, "which must be 0..3");
  STCHK(check_grid(1, H, W));
  STCHK(net_reserve(net, 1, H, W));
  STCHK(net_alphas(net, 1));
  hipStream_t s = net->stream;
  const long px = (long)H * W;
  LAUNCH(k_fill<float>, dim3(nblocks_vec(px)), dim3(256), 0, s, net->xb, 0.5f, px);
  LAUNCH(k_fill<float>, dim3(1), dim3(256), 0, s, net->ab, 1.0f, 1L);
  STCHK(net_forward(net, net->xb, net->ab, 1, H, W));
  auto one = [&]() -> fl_status {
    u16** a = net->act;
    if (which == 0) return net_forward(net, net->xb, net->ab, 1, H, W);
    if (which == 1) {
      Stage st = {a[A0], a[C1], nullptr};
      LAUNCH((k_conv32<SM_UPADD, EPI_RELU>), dim3(conv_blocks(1, H, W)), dim3(256), 0, s, st,
             (const u16*)(net->fw + LU0 * PACK), (const float*)(net->th + OFF_L32 + LU0 * L32SZ + L32W), a[C0], 1, H, W,
             (float*)nullptr);
      return FL_OK;
    }
    if (which == 2) {
      Stage st = {nullptr, nullptr, nullptr, (const float*)net->xb, (const float*)net->ab};
      LAUNCH((k_conv32<SM_INPUT, EPI_RELU>), dim3(conv_blocks(1, H, W)), dim3(256), 0, s, st,
             (const u16*)(net->fw + NL32 * PACK), (const float*)(net->th + OFF_CIN_B), a[A0], 1, H, W, (float*)nullptr);
      return FL_OK;
    }
    Stage st = {a[C0], nullptr, nullptr};
    LAUNCH((k_conv32<SM_PLAIN, EPI_OUT>), dim3(conv_blocks(1, H, W)), dim3(256), 0, s, st,
           (const u16*)(net->fw + (NL32 + 1) * PACK), (const float*)(net->th + OFF_OUT + 9 * CH), (u16*)nullptr, 1, H, W,
           net->y);
    return FL_OK;
  };
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
