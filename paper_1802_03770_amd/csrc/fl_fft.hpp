// Line FFT engine for gfx950: one or more complex lines held in LDS, transformed
// in place by a Stockham autosort FFT whose radix sequence is chosen at run time
// (radices 2, 3, 4, 5, 8; the out-of-place variant adds odd primes 7..43).
// Every thread of a line keeps its butterflies in registers between the LDS read
// and the LDS write of a stage, so one LDS buffer per line suffices.  A workgroup
// holds G lines of equal length; each line is served by `tpl` consecutive lanes
// (a power of two), so G * tpl = blockDim.x.
//
// LDS lines are padded by one element every 128 bytes (Line<T>): the strided
// writes of the first Stockham stages then spread over all banks.
//
// Twiddles come from a table of the L-th roots of unity e^{-2 pi i m / L}
// (computed on the host in extended precision).
#pragma once
#include <hip/hip_runtime.h>

namespace fl {

template <typename T> struct cx { T x, y; };

template <typename T> __device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T> __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T> __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV> __device__ __forceinline__ cx<T> mul_mi(cx<T> a) {
  return INV ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
}

constexpr int kMaxStages = 16;
constexpr int kMaxElems = 16;  // elements of one line held per lane

// A complex line in LDS with one padding element after every 128 bytes.
template <typename T> struct Line {
  static constexpr int S = sizeof(T) == 4 ? 4 : 3;  // log2(elements per 128 bytes)
  cx<T>* p;
  __device__ __forceinline__ cx<T>& operator[](int i) const { return p[i + (i >> S)]; }
  // elements (including padding) one line of length L occupies
  static __host__ __device__ constexpr int stride(int L) { return L + (L >> S) + 2; }
};
template <typename T> __device__ __forceinline__ Line<T> line_at(void* base, long idx, int L) {
  return Line<T>{(cx<T>*)base + idx * (long)Line<T>::stride(L)};
}

// Radix of stage s is kRadix[(radcode >> 4 s) & 15] (no arrays in the plan, so
// it stays in scalar registers when passed by value).
struct FFTPlan {
  int L;                      // transform length
  int nst;                    // number of stages
  int tpl;                    // lanes per line (power of two)
  int fixed;                  // 1: a compile-time specialisation exists for (L, tpl)
  unsigned long long radcode; // 4 bits per stage
  const void* tw;             // cx<T>[L] = e^{-2 pi i m / L}
};
__host__ __device__ constexpr int radix_of_code(int c) {
  return c == 0 ? 2 : c == 1 ? 3 : c == 2 ? 4 : c == 3 ? 5 : c == 4 ? 8 : c == 5 ? 7 : c == 6 ? 11 : c == 7 ? 13
       : c == 8 ? 17 : c == 9 ? 19 : c == 10 ? 23 : c == 11 ? 29 : c == 12 ? 31 : c == 13 ? 37 : c == 14 ? 41 : 43;
}
__host__ __device__ __forceinline__ int stage_radix(const FFTPlan& pl, int s) {
  return radix_of_code((int)((pl.radcode >> (4 * s)) & 15ull));
}

template <typename T, int R, bool INV> struct Bfly;

// run_half: the same butterfly for inputs whose upper half a[R/2..R-1] is
// zero (the first stage of a zero-padded line); those entries are not read.
template <typename T, bool INV> struct Bfly<T, 2, INV> {
  static __device__ __forceinline__ void run(cx<T>* a) {
    cx<T> t = a[1];
    a[1] = csub(a[0], t);
    a[0] = cadd(a[0], t);
  }
  static __device__ __forceinline__ void run_half(cx<T>* a) { a[1] = a[0]; }
};

template <typename T, bool INV> struct Bfly<T, 4, INV> {
  static __device__ __forceinline__ void run(cx<T>* a) {
    cx<T> t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    cx<T> t2 = cadd(a[1], a[3]), t3 = mul_mi<T, INV>(csub(a[1], a[3]));
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
  }
  static __device__ __forceinline__ void run_half(cx<T>* a) {
    const cx<T> x0 = a[0], x1 = a[1], t3 = mul_mi<T, INV>(x1);
    a[0] = cadd(x0, x1);
    a[2] = csub(x0, x1);
    a[1] = cadd(x0, t3);
    a[3] = csub(x0, t3);
  }
};

template <typename T, bool INV> struct Bfly<T, 8, INV> {
  static __device__ __forceinline__ void run(cx<T>* a) {
    // radix-4 on even and odd halves
    cx<T> e[4] = {a[0], a[2], a[4], a[6]};
    cx<T> o[4] = {a[1], a[3], a[5], a[7]};
    Bfly<T, 4, INV>::run(e);
    Bfly<T, 4, INV>::run(o);
    join(e, o, a);
  }
  static __device__ __forceinline__ void run_half(cx<T>* a) {
    cx<T> e[4] = {a[0], a[2], {0, 0}, {0, 0}};
    cx<T> o[4] = {a[1], a[3], {0, 0}, {0, 0}};
    Bfly<T, 4, INV>::run_half(e);
    Bfly<T, 4, INV>::run_half(o);
    join(e, o, a);
  }
  // outputs from the radix-4 transforms of the even and odd entries
  static __device__ __forceinline__ void join(const cx<T>* e, const cx<T>* o, cx<T>* a) {
    const T r2 = (T)0.70710678118654752440084436210484904L;
    // twiddles w8^k, k = 0..3  (w8 = e^{-+2 pi i / 8})
    cx<T> o1 = INV ? cx<T>{r2 * (o[1].x - o[1].y), r2 * (o[1].x + o[1].y)}
                   : cx<T>{r2 * (o[1].x + o[1].y), r2 * (o[1].y - o[1].x)};
    cx<T> o2 = mul_mi<T, INV>(o[2]);
    cx<T> o3 = INV ? cx<T>{-r2 * (o[3].x + o[3].y), r2 * (o[3].x - o[3].y)}
                   : cx<T>{r2 * (o[3].y - o[3].x), -r2 * (o[3].x + o[3].y)};
    a[0] = cadd(e[0], o[0]);
    a[4] = csub(e[0], o[0]);
    a[1] = cadd(e[1], o1);
    a[5] = csub(e[1], o1);
    a[2] = cadd(e[2], o2);
    a[6] = csub(e[2], o2);
    a[3] = cadd(e[3], o3);
    a[7] = csub(e[3], o3);
  }
};

template <typename T, bool INV> struct Bfly<T, 3, INV> {
  static __device__ __forceinline__ void run(cx<T>* a) {
    const T s = (T)0.86602540378443864676372317075293618L;  // sin(2 pi / 3)
    cx<T> sum = cadd(a[1], a[2]);
    cx<T> dif = csub(a[1], a[2]);
    cx<T> m = {a[0].x - (T)0.5 * sum.x, a[0].y - (T)0.5 * sum.y};
    // forward: y1 = m - i s dif, y2 = m + i s dif
    cx<T> isd = {-s * dif.y, s * dif.x};  // i s dif
    a[0] = cadd(a[0], sum);
    if (INV) {
      a[1] = cadd(m, isd);
      a[2] = csub(m, isd);
    } else {
      a[1] = csub(m, isd);
      a[2] = cadd(m, isd);
    }
  }
};

template <typename T, bool INV> struct Bfly<T, 5, INV> {
  static __device__ __forceinline__ void run(cx<T>* a) {
    const T c1 = (T)0.30901699437494742410229341718281906L;   // cos(2pi/5)
    const T c2 = (T)-0.80901699437494742410229341718281906L;  // cos(4pi/5)
    const T s1 = (T)0.95105651629515357211643933337938214L;   // sin(2pi/5)
    const T s2 = (T)0.58778525229247312916870595463907277L;   // sin(4pi/5)
    cx<T> b1 = cadd(a[1], a[4]), d1 = csub(a[1], a[4]);
    cx<T> b2 = cadd(a[2], a[3]), d2 = csub(a[2], a[3]);
    cx<T> m1 = {a[0].x + c1 * b1.x + c2 * b2.x, a[0].y + c1 * b1.y + c2 * b2.y};
    cx<T> m2 = {a[0].x + c2 * b1.x + c1 * b2.x, a[0].y + c2 * b1.y + c1 * b2.y};
    // forward: y1 = m1 - i (s1 d1 + s2 d2), y4 = m1 + i(...)
    //          y2 = m2 - i (s2 d1 - s1 d2), y3 = m2 + i(...)
    cx<T> t1 = {s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y};
    cx<T> t2 = {s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y};
    cx<T> it1 = {-t1.y, t1.x}, it2 = {-t2.y, t2.x};
    a[0] = {a[0].x + b1.x + b2.x, a[0].y + b1.y + b2.y};
    if (INV) {
      a[1] = cadd(m1, it1);
      a[4] = csub(m1, it1);
      a[2] = cadd(m2, it2);
      a[3] = csub(m2, it2);
    } else {
      a[1] = csub(m1, it1);
      a[4] = cadd(m1, it1);
      a[2] = csub(m2, it2);
      a[3] = cadd(m2, it2);
    }
  }
};

// Butterfly j of a stage with stride Ns: k = j mod Ns, g = j / Ns (shift and
// mask while Ns is a power of two, lgNs >= 0).
__device__ __forceinline__ void split_j(int j, int Ns, int lgNs, int& g, int& k) {
  if (lgNs >= 0) {
    k = j & (Ns - 1);
    g = j >> lgNs;
  } else {
    g = (int)((unsigned)j / (unsigned)Ns);
    k = j - g * Ns;
  }
}

// One Stockham stage of radix R on the line `buf` (length L, LDS).  Ns is the
// product of the radices already applied.  Input butterfly j reads
// buf[j + r L/R]; it is twiddled by w_{Ns R}^{r k} with k = j mod Ns and
// written to buf[(j / Ns) Ns R + k + r Ns].
template <typename T, int R, bool INV>
__device__ __forceinline__ void fft_stage(Line<T> buf, int L, int Ns, int lgNs, const cx<T>* __restrict__ tw,
                                          int lane, int tpl) {
  constexpr int MB = kMaxElems / R;
  const int nb = L / R;
  const int tstep = L / (Ns * R);
  cx<T> v[MB][R];
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int j = lane + b * tpl;
    if (j < nb) {
      int g, k;
      split_j(j, Ns, lgNs, g, k);
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = buf[j + r * nb];
      if (Ns > 1) {
        const int st = k * tstep;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tw[r * st];
          v[b][r] = INV ? cmulc(v[b][r], w) : cmul(v[b][r], w);
        }
      }
      Bfly<T, R, INV>::run(v[b]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int j = lane + b * tpl;
    if (j < nb) {
      int g, k;
      split_j(j, Ns, lgNs, g, k);
      const int base = g * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[base + r * Ns] = v[b][r];
    }
  }
  __syncthreads();
}

__device__ __forceinline__ int next_lg(int lgNs, int R) {
  if (lgNs < 0) return -1;
  return R == 2 ? lgNs + 1 : R == 4 ? lgNs + 2 : R == 8 ? lgNs + 3 : -1;
}


// ---------------------------------------------------------------------------
// Compile-time specialised line FFTs for the lengths the workloads use.  The
// radix order matches the run-time plan: 8s, 4, 2, 3s, 5s, then odd primes.
// Lanes per line: the smallest power of two giving <= 8 elements per lane
// (capped at 256) that also fits every stage.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int c_order(int q) {
  return q == 0 ? 8 : q == 1 ? 4 : q == 2 ? 2 : q == 3 ? 3 : q == 4 ? 5 : q == 5 ? 7 : q == 6 ? 11 : q == 7 ? 13
       : q == 8 ? 17 : q == 9 ? 19 : q == 10 ? 23 : q == 11 ? 29 : q == 12 ? 31 : q == 13 ? 37 : q == 14 ? 41 : 43;
}
__host__ __device__ constexpr int c_radix(int L, int s) {
  int m = L, idx = 0;
  for (int q = 0; q < 16; ++q) {
    const int p = c_order(q);
    while (m % p == 0) {
      if (idx == s) return p;
      m /= p;
      ++idx;
    }
  }
  return 1;
}
__host__ __device__ constexpr int c_nst(int L) {
  int m = L, idx = 0;
  for (int q = 0; q < 16; ++q) {
    const int p = c_order(q);
    while (m % p == 0) {
      m /= p;
      ++idx;
    }
  }
  return idx;
}
__host__ __device__ constexpr int c_fixed_tpl(int L) {
  int t = 1;
  while (t * 8 < L && t < 256) t *= 2;
  for (;;) {
    bool ok = true;
    for (int s = 0; s < c_nst(L); ++s) {
      const int R = c_radix(L, s), nb = L / R, per = (nb + t - 1) / t;
      const int cap = 16 / R > 1 ? 16 / R : 1;
      if (per > cap) ok = false;
    }
    if (ok || t >= 256) return t;
    t *= 2;
  }
}
// lengths with a specialisation (apply / chirp-z / cosine lengths, direct sine lengths)
__host__ __device__ constexpr bool c_is_fixed(int L) {
  return L == 128 || L == 256 || L == 512 || L == 768 || L == 1024 || L == 2048 || L == 130 || L == 258 ||
         L == 770 || L == 1026 || L == 2050 || L == 8192;
}

// direct DFT of odd prime radix R on registers a[0..R-1] (conjugate-pair form)
template <typename T, int R, bool INV>
__device__ __forceinline__ void bfly_prime(cx<T>* a, const T* cs, const T* sn) {
  constexpr int H = (R - 1) / 2;
  cx<T> sm[H], df[H];
  cx<T> a0 = a[0], y0 = a[0];
#pragma unroll
  for (int q = 1; q <= H; ++q) {
    sm[q - 1] = cadd(a[q], a[R - q]);
    df[q - 1] = csub(a[q], a[R - q]);
    y0 = cadd(y0, sm[q - 1]);
  }
#pragma unroll
  for (int kk = 1; kk <= H; ++kk) {
    cx<T> re = a0, im = {0, 0};
#pragma unroll
    for (int q = 1; q <= H; ++q) {
      const int m = (q * kk) % R;
      const T c = m <= H ? cs[m] : cs[R - m];
      const T sg = m <= H ? sn[m] : -sn[R - m];
      re.x += sm[q - 1].x * c;
      re.y += sm[q - 1].y * c;
      im.x += df[q - 1].x * sg;
      im.y += df[q - 1].y * sg;
    }
    cx<T> yp = {re.x + im.y, re.y - im.x};
    cx<T> ym = {re.x - im.y, re.y + im.x};
    a[kk] = INV ? ym : yp;
    a[R - kk] = INV ? yp : ym;
  }
  a[0] = y0;
}

// ZI: the line's upper half is zero on entry (a first stage of even radix:
// input r of a butterfly is zero for r >= R/2, and is not read).  ZO: only the
// lower half of the output is used (a last stage of even radix: outputs
// r >= R/2 are not written).
template <typename T, int R, int L, int NS, int TPL, bool INV, bool ZI = false, bool ZO = false>
__device__ __forceinline__ void cstage(Line<T> buf, const cx<T>* __restrict__ tw, int lane) {
  static_assert(!(ZI || ZO) || R % 2 == 0, "pruned stages need an even radix");
  static_assert(!ZI || NS == 1, "input pruning applies to a first stage");
  static_assert(!ZO || NS * R == L, "output pruning applies to a last stage");
  constexpr int NB = L / R;
  constexpr int MB = (NB + TPL - 1) / TPL;
  constexpr bool FULL = (NB % TPL) == 0;
  constexpr int TSTEP = L / (NS * R);
  constexpr bool PRIME = R >= 7 && R != 8;  // odd primes only
  constexpr int H = PRIME ? (R - 1) / 2 : 1;
  T cs[H + 1], sn[H + 1];
  if (PRIME) {
#pragma unroll
    for (int m = 1; m <= H; ++m) {
      cx<T> w = tw[m * (L / R)];
      cs[m] = w.x;
      sn[m] = -w.y;
    }
  }
  cx<T> v[MB][R];
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int j = lane + b * TPL;
    if (FULL || j < NB) {
      const int k = j % NS;
#pragma unroll
      for (int r = 0; r < (ZI ? R / 2 : R); ++r) v[b][r] = buf[j + r * NB];
      if (NS > 1) {
        const int st = k * TSTEP;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tw[r * st];
          v[b][r] = INV ? cmulc(v[b][r], w) : cmul(v[b][r], w);
        }
      }
      if constexpr (PRIME)
        bfly_prime<T, R, INV>(v[b], cs, sn);
      else if constexpr (ZI)
        Bfly<T, R, INV>::run_half(v[b]);
      else
        Bfly<T, R, INV>::run(v[b]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int j = lane + b * TPL;
    if (FULL || j < NB) {
      const int k = j % NS;
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < (ZO ? R / 2 : R); ++r) buf[base + r * NS] = v[b][r];
    }
  }
  __syncthreads();
}

// Output group G of a split prime stage: pairs (y_k, y_{R-k}) for
// k = G*KG+1 .. min(H, G*KG+KG) of butterfly j (group 0 also y_0), from the
// conjugate-pair sums s_q and differences d_q stored in the auxiliary line.
template <typename T, int R, int NS, int KG, bool INV, int G>
__device__ __forceinline__ void split_outputs(Line<T> aux, Line<T> buf, int j, int base, const T* cs, const T* sn) {
  constexpr int H = (R - 1) / 2;
  constexpr int K0 = G * KG + 1, K1 = (G * KG + KG < H) ? G * KG + KG : H, NK = K1 - K0 + 1;
  const cx<T> a0 = aux[j * R];
  cx<T> re[NK], im[NK];
#pragma unroll
  for (int i = 0; i < NK; ++i) {
    re[i] = a0;
    im[i] = {0, 0};
  }
  cx<T> y0 = a0;
#pragma unroll
  for (int q = 1; q <= H; ++q) {
    const cx<T> sq = aux[j * R + q], dq = aux[j * R + H + q];
    if (G == 0) y0 = cadd(y0, sq);
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      const int m = (q * (K0 + i)) % R;
      const T c = m <= H ? cs[m] : cs[R - m];
      const T sg = m <= H ? sn[m] : -sn[R - m];
      re[i].x += sq.x * c;
      re[i].y += sq.y * c;
      im[i].x += dq.x * sg;
      im[i].y += dq.y * sg;
    }
  }
  if (G == 0) buf[base] = y0;
#pragma unroll
  for (int i = 0; i < NK; ++i) {
    const cx<T> yp = {re[i].x + im[i].y, re[i].y - im[i].x};
    const cx<T> ym = {re[i].x - im[i].y, re[i].y + im[i].x};
    buf[base + (K0 + i) * NS] = INV ? ym : yp;
    buf[base + (R - K0 - i) * NS] = INV ? yp : ym;
  }
}

template <typename T, int R, int NS, int KG, bool INV, int G, int NG>
__device__ __forceinline__ void split_dispatch(int gi, Line<T> aux, Line<T> buf, int j, int base, const T* cs,
                                               const T* sn) {
  if constexpr (G < NG) {
    if (gi == G)
      split_outputs<T, R, NS, KG, INV, G>(aux, buf, j, base, cs, sn);
    else
      split_dispatch<T, R, NS, KG, INV, G + 1, NG>(gi, aux, buf, j, base, cs, sn);
  }
}

// Radix-R stage for a large odd prime R (>= 17) split over lanes, so that no
// lane holds a whole butterfly: phase A writes, per butterfly j, the
// twiddled a_0 and the pair sums s_q = a_q + a_{R-q} and differences
// d_q = a_q - a_{R-q} (q = 1..H) into the auxiliary line (NB * R = L entries);
// phase B has each lane form KG output pairs of one butterfly from them, with
// y_k = a_0 + sum_q s_q cos(2 pi q k/R) -+ i sum_q d_q sin(2 pi q k/R).
// Output pairs per item of a split stage: the butterflies of a group are
// padded to whole wavefronts (NBP), so a wavefront runs one group's code per
// round of TPL items; KG is chosen to minimise the rounds of the busiest
// wavefront times the cost of one round (KG * H complex multiply-adds on the
// sums and differences, plus reading the 2H + 1 of them from LDS), with at
// most KGMAX accumulator pairs held per lane.
__host__ __device__ constexpr int split_kg(int H, int NBP, int TPL, int KGMAX) {
  int best = 1, bc = 1 << 30;
  for (int kg = 1; kg <= KGMAX && kg <= H; ++kg) {
    const int ng = (H + kg - 1) / kg, rounds = (ng * NBP + TPL - 1) / TPL;
    const int c = rounds * (4 * kg * H + 2 * (2 * H + 1));
    if (c < bc) {
      bc = c;
      best = kg;
    }
  }
  return best;
}

template <typename T, int R, int L, int NS, int TPL, bool INV>
__device__ __forceinline__ void cstage_split(Line<T> buf, Line<T> aux, const cx<T>* __restrict__ tw, int lane) {
  constexpr int NB = L / R, H = (R - 1) / 2, NBP = (NB + 63) / 64 * 64;
  constexpr int KG = split_kg(H, NBP, TPL, sizeof(T) == 4 ? 10 : 5), NG = (H + KG - 1) / KG;
  constexpr int TSTEP = L / (NS * R);
  for (int t = lane; t < NB * (H + 1); t += TPL) {
    const int j = t / (H + 1), q = t % (H + 1);
    const int k = j % NS;
    if (q == 0) {
      aux[j * R] = buf[j];
    } else {
      cx<T> u = buf[j + q * NB], w = buf[j + (R - q) * NB];
      if (NS > 1) {
        const cx<T> t1 = tw[q * k * TSTEP], t2 = tw[(R - q) * k * TSTEP];
        u = INV ? cmulc(u, t1) : cmul(u, t1);
        w = INV ? cmulc(w, t2) : cmul(w, t2);
      }
      aux[j * R + q] = cadd(u, w);
      aux[j * R + H + q] = csub(u, w);
    }
  }
  T cs[H + 1], sn[H + 1];
#pragma unroll
  for (int m = 1; m <= H; ++m) {
    const cx<T> w = tw[m * NB];  // e^{-2 pi i m / R}
    cs[m] = w.x;
    sn[m] = -w.y;
  }
  __syncthreads();
  // Phase B takes the output groups one after another, each over the
  // butterflies padded to whole wavefronts (NBP), so that the group index --
  // and with it the code path -- is the same for every lane of a wavefront
  // (lanes of one wavefront are consecutive lanes of one line, or whole
  // lines at the same offsets when TPL < 64).
  for (int t = lane; t < NG * NBP; t += TPL) {
    const int gi = t / NBP, j = t % NBP;
    if (j < NB) {
      const int k = j % NS;
      const int base = (j / NS) * NS * R + k;
      split_dispatch<T, R, NS, KG, INV, 0, NG>(gi, aux, buf, j, base, cs, sn);
    }
  }
  __syncthreads();
}

// ZIN: entries L/2 .. L-1 of the input are zero (a zero-padded line; they
// need not be in LDS).  ZOUT: only entries 0 .. L/2-1 of the output are used
// (a cropped line; the others are left unwritten).  Each takes effect where
// the first (last) stage has an even radix.
template <typename T, int L, int TPL, bool INV, int S, int NS, bool ZIN = false, bool ZOUT = false>
__device__ __forceinline__ void cstages(Line<T> buf, Line<T> aux, const cx<T>* __restrict__ tw, int lane) {
  if constexpr (S < c_nst(L)) {
    constexpr int R = c_radix(L, S);
    constexpr bool ZI = ZIN && S == 0 && R % 2 == 0, ZO = ZOUT && S == c_nst(L) - 1 && R % 2 == 0;
    if constexpr (R >= 17)
      cstage_split<T, R, L, NS, TPL, INV>(buf, aux, tw, lane);
    else
      cstage<T, R, L, NS, TPL, INV, ZI, ZO>(buf, tw, lane);
    cstages<T, L, TPL, INV, S + 1, NS * R, ZIN, ZOUT>(buf, aux, tw, lane);
  }
}

// aux: a second line of length L, used as scratch by prime stages >= 17
template <typename T, int L, bool INV, bool ZIN = false, bool ZOUT = false>
__device__ __forceinline__ void fft_fixed(Line<T> buf, Line<T> aux, const cx<T>* __restrict__ tw, int lane) {
  cstages<T, L, c_fixed_tpl(L), INV, 0, 1, ZIN, ZOUT>(buf, aux, tw, lane);
}
// True when the first stage of length L would skip the upper half of the input.
__host__ __device__ constexpr bool c_zin_pruned(int L) { return c_nst(L) > 0 && c_radix(L, 0) % 2 == 0; }

// Prime form of a packed pair, N = n + 1 an odd prime with N - 1 = RL (the FFT
// length; lanes c_fixed_tpl(RL) <= 64).  In: buf[k] = (x_a[k], x_b[k]) for
// k = 1..n.  Out: buf[k] = (S_a[k], S_b[k]), S[k] = sum_j x_j sin(pi j k / N);
// buf2 is scratch.  Three steps:
//  1. y_j = s_j (x_j + x_{N-j}) + (x_j - x_{N-j}) / 2, s_j = sin(pi j / N), for
//     both members at once; the real DFT Y of y then has -Im Y_k = S_{2k} and
//     Re Y_k = S_{2k+1} - S_{2k-1} (with S_{-1} = -S_1).
//  2. The DFT of length N of y_a + i y_b by Rader's identity: with a generator
//     g of the units mod N, Z_{g^q} = sum_p y_{g^-p} b_{q-p}, b_m = e^{-2 pi i
//     g^m / N}, a cyclic convolution of length RL (y_0 = 0), done as an FFT,
//     a product with the table bhat = FFT(b) / RL, and an inverse FFT; Z_0 is
//     the first output of the forward FFT.  The pair (j, N - j) sits at
//     positions (p, p + RL/2) since g^(RL/2) = -1 mod N.
//  3. Y_a, Y_b from Z_k and Z_{N-k}; the odd outputs are a running sum of
//     Re Y over k, taken per lane over a run of consecutive k and then across
//     the lanes of the line with wavefront shuffles.
// Tables: gi = int[RL/2] g^-p mod N, then int[RL/2 + 1] log_g k (entry 0
// unused); sp = T[RL/2] s_{g^-p}; bh = cx<T>[RL]; tw = the FFT's roots of unity.
// A lane's entries of the first three are held in registers (RaderRegs,
// loaded once per kernel by rader_load, before the line data).
template <typename T, int RL> struct RaderRegs {
  static constexpr int TPL = c_fixed_tpl(RL), HALF = RL / 2;
  static constexpr int PM = (HALF + TPL - 1) / TPL, QM = (RL + TPL - 1) / TPL, C = (HALF + 1 + TPL - 1) / TPL;
  int j[PM];     // g^-p for p = lane + m TPL
  T s[PM];       // sin(pi g^-p / N)
  cx<T> b[QM];   // bhat[q] for q = lane + m TPL
  int l[C];      // log_g k for k = lane C + c
};
template <typename T, int RL>
__device__ __forceinline__ void rader_load(RaderRegs<T, RL>& R, const int* __restrict__ gi,
                                           const T* __restrict__ sp, const cx<T>* __restrict__ bh, int lane) {
  using RR = RaderRegs<T, RL>;
#pragma unroll
  for (int m = 0; m < RR::PM; ++m) {
    const int p = lane + m * RR::TPL;
    R.j[m] = p < RR::HALF ? gi[p] : 1;
    R.s[m] = p < RR::HALF ? sp[p] : (T)0;
  }
#pragma unroll
  for (int m = 0; m < RR::QM; ++m) {
    const int q = lane + m * RR::TPL;
    R.b[m] = q < RL ? bh[q] : cx<T>{0, 0};
  }
#pragma unroll
  for (int c = 0; c < RR::C; ++c) {
    const int k = lane * RR::C + c;
    R.l[c] = (k >= 1 && k <= RR::HALF) ? gi[RR::HALF + k] : 0;
  }
}
template <typename T, int RL>
__device__ __forceinline__ void rader_sine(Line<T> buf, Line<T> buf2, int n, const RaderRegs<T, RL>& R,
                                           const cx<T>* __restrict__ tw, int lane) {
  constexpr int N = RL + 1, HALF = RL / 2, TPL = c_fixed_tpl(RL);
  static_assert(TPL <= 64, "the running sum crosses lanes by wavefront shuffles");
#pragma unroll
  for (int m = 0; m < RaderRegs<T, RL>::PM; ++m) {
    const int p = lane + m * TPL;
    if (p >= HALF) break;
    const int j = R.j[m];
    const T sj = R.s[m];
    const cx<T> u = buf[j], w = buf[N - j];
    const cx<T> a = cadd(u, w), h = cscale(csub(u, w), (T)0.5);
    buf2[p] = {sj * a.x + h.x, sj * a.y + h.y};
    buf2[p + HALF] = {sj * a.x - h.x, sj * a.y - h.y};
  }
  __syncthreads();
  fft_fixed<T, RL, false>(buf2, buf2, tw, lane);
#pragma unroll
  for (int m = 0; m < RaderRegs<T, RL>::QM; ++m) {
    const int q = lane + m * TPL;
    if (q >= RL) break;
    const cx<T> v = buf2[q];
    if (q == 0) buf[0] = v;  // Z_0 (slot 0 of the input line is free)
    buf2[q] = cmul(v, R.b[m]);
  }
  __syncthreads();
  fft_fixed<T, RL, true>(buf2, buf2, tw, lane);
  constexpr int C = (HALF + 1 + TPL - 1) / TPL;  // consecutive k per lane
  const cx<T> z0 = buf[0];
  T ra[C], rb[C], sa = 0, sb = 0;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int k = lane * C + c;
    T Ra = 0, Rb = 0;
    if (k <= HALF) {
      cx<T> P = z0, Q = z0;
      if (k > 0) {
        const int q = R.l[c];
        P = buf2[q];
        Q = buf2[(q + HALF) % RL];
      }
      Ra = (T)0.5 * (P.x + Q.x);
      Rb = (T)0.5 * (P.y + Q.y);
      if (k > 0 && 2 * k <= n) buf[2 * k] = {(T)0.5 * (Q.y - P.y), (T)0.5 * (P.x - Q.x)};
    }
    sa += Ra;
    sb += Rb;
    ra[c] = sa;
    rb[c] = sb;
  }
  T ea = sa, eb = sb;  // inclusive scan of the lane totals over the line
#pragma unroll
  for (int o = 1; o < TPL; o <<= 1) {
    const T ta = __shfl_up(ea, o, TPL), tb = __shfl_up(eb, o, TPL);
    if (lane >= o) {
      ea += ta;
      eb += tb;
    }
  }
  ea -= sa + (T)0.5 * z0.x;  // exclusive, less R_0 / 2 (S_1 = R_0 / 2)
  eb -= sb + (T)0.5 * z0.y;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int k = lane * C + c;
    if (2 * k + 1 <= n) buf[2 * k + 1] = {ea + ra[c], eb + rb[c]};
  }
  __syncthreads();
}


// Dispatch to a specialisation; false when the plan has none.
template <typename T, bool INV>
__device__ __forceinline__ bool fft_try_fixed(Line<T> buf, const FFTPlan& pl, int lane) {
  if (!pl.fixed) return false;
  const cx<T>* __restrict__ tw = (const cx<T>*)pl.tw;
  switch (pl.L) {
    case 2048: fft_fixed<T, 2048, INV>(buf, buf, tw, lane); return true;
    case 1024: fft_fixed<T, 1024, INV>(buf, buf, tw, lane); return true;
    case 512: fft_fixed<T, 512, INV>(buf, buf, tw, lane); return true;
    case 256: fft_fixed<T, 256, INV>(buf, buf, tw, lane); return true;
    case 128: fft_fixed<T, 128, INV>(buf, buf, tw, lane); return true;
    case 768: fft_fixed<T, 768, INV>(buf, buf, tw, lane); return true;
    default: return false;
  }
}
template <typename T, bool INV>
__device__ __forceinline__ bool fft_try_fixed_wide(Line<T> buf, Line<T> aux, const FFTPlan& pl, int lane) {
  if (!pl.fixed) return false;
  const cx<T>* __restrict__ tw = (const cx<T>*)pl.tw;
  switch (pl.L) {
    case 2050: fft_fixed<T, 2050, INV>(buf, aux, tw, lane); return true;
    case 1026: fft_fixed<T, 1026, INV>(buf, aux, tw, lane); return true;
    case 770: fft_fixed<T, 770, INV>(buf, aux, tw, lane); return true;
    case 258: fft_fixed<T, 258, INV>(buf, aux, tw, lane); return true;
    case 130: fft_fixed<T, 130, INV>(buf, aux, tw, lane); return true;
    default: return false;
  }
}

// Full in-place FFT of the LDS line `buf` (unnormalised in both directions).
// Every lane of the workgroup must call this (it contains barriers).
template <typename T, bool INV>
__device__ __forceinline__ void fft_line(Line<T> buf, const FFTPlan pl, int lane) {
  if (fft_try_fixed<T, INV>(buf, pl, lane)) return;
  if (pl.L > kMaxElems * pl.tpl) {
    // a line longer than the run-time stages hold (the 8192 plan, which only
    // its specialised kernels take): NaN out rather than a partial transform
    for (int i = lane; i < pl.L; i += pl.tpl) buf[i] = {(T)NAN, (T)NAN};
    __syncthreads();
    return;
  }
  const cx<T>* __restrict__ tw = (const cx<T>*)pl.tw;
  int Ns = 1, lg = 0;
  for (int s = 0; s < pl.nst; ++s) {
    const int R = stage_radix(pl, s);
    switch (R) {
      case 8: fft_stage<T, 8, INV>(buf, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      case 4: fft_stage<T, 4, INV>(buf, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      case 2: fft_stage<T, 2, INV>(buf, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      case 3: fft_stage<T, 3, INV>(buf, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      default: fft_stage<T, 5, INV>(buf, pl.L, Ns, lg, tw, lane, pl.tpl); break;
    }
    lg = next_lg(lg, R);
    Ns *= R;
  }
}


// Out-of-place Stockham stage (src -> dst, one barrier), radices 2..8.
template <typename T, int R, bool INV>
__device__ __forceinline__ void fft_stage_oop(Line<T> src, Line<T> dst, int L, int Ns, int lgNs,
                                              const cx<T>* __restrict__ tw, int lane, int tpl) {
  const int nb = L / R;
  const int tstep = L / (Ns * R);
  for (int j = lane; j < nb; j += tpl) {
    int g, k;
    split_j(j, Ns, lgNs, g, k);
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[j + r * nb];
    if (Ns > 1) {
      const int st = k * tstep;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cx<T> w = tw[r * st];
        v[r] = INV ? cmulc(v[r], w) : cmul(v[r], w);
      }
    }
    Bfly<T, R, INV>::run(v);
    const int base = g * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[base + r * Ns] = v[r];
  }
  __syncthreads();
}

// Out-of-place radix-R stage for an odd prime R >= 7: direct DFT with the
// conjugate-pair reduction.  With s_q = a_q + a_{R-q}, d_q = a_q - a_{R-q},
// q = 1..(R-1)/2:
//   y_k     = a_0 + sum_q s_q cos(2 pi q k / R) -+ i sum_q d_q sin(2 pi q k / R),
//   y_{R-k} = the same with the opposite sign of the sine part
// (upper sign forward).  Only s, d and the R roots live in registers; outputs
// go straight to dst.  The roots are e^{-2 pi i m / R} = tw[m L / R].
template <typename T, int R, bool INV>
__device__ __forceinline__ void fft_stage_prime_oop(Line<T> src, Line<T> dst, int L, int Ns, int lgNs,
                                                    const cx<T>* __restrict__ tw, int lane, int tpl) {
  constexpr int H = (R - 1) / 2;
  const int nb = L / R;
  const int tstep = L / (Ns * R);
  const int cstep = L / R;
  T cs[H + 1], sn[H + 1];
#pragma unroll
  for (int m = 1; m <= H; ++m) {
    cx<T> w = tw[m * cstep];
    cs[m] = w.x;
    sn[m] = -w.y;
  }
  for (int j = lane; j < nb; j += tpl) {
    int g, k;
    split_j(j, Ns, lgNs, g, k);
    const int st = k * tstep;
    cx<T> a0 = src[j];
    cx<T> sm[H], df[H];
    cx<T> y0 = a0;
#pragma unroll
    for (int q = 1; q <= H; ++q) {
      cx<T> u = src[j + q * nb], w = src[j + (R - q) * nb];
      if (Ns > 1) {
        cx<T> t1 = tw[q * st], t2 = tw[(R - q) * st];
        u = INV ? cmulc(u, t1) : cmul(u, t1);
        w = INV ? cmulc(w, t2) : cmul(w, t2);
      }
      sm[q - 1] = cadd(u, w);
      df[q - 1] = csub(u, w);
      y0 = cadd(y0, sm[q - 1]);
    }
    const int base = g * Ns * R + k;
    dst[base] = y0;
#pragma unroll
    for (int kk = 1; kk <= H; ++kk) {
      cx<T> re = a0, im = {0, 0};
#pragma unroll
      for (int q = 1; q <= H; ++q) {
        const int m = (q * kk) % R;
        const T c = m <= H ? cs[m] : cs[R - m];
        const T sg = m <= H ? sn[m] : -sn[R - m];
        re.x += sm[q - 1].x * c;
        re.y += sm[q - 1].y * c;
        im.x += df[q - 1].x * sg;
        im.y += df[q - 1].y * sg;
      }
      cx<T> yp = {re.x + im.y, re.y - im.x};  // re - i im
      cx<T> ym = {re.x - im.y, re.y + im.x};  // re + i im
      dst[base + kk * Ns] = INV ? ym : yp;
      dst[base + (R - kk) * Ns] = INV ? yp : ym;
    }
  }
  __syncthreads();
}

// Out-of-place FFT with the wide radix set (2, 3, 4, 5, 8 and odd primes
// 7..43), ping-ponging between a and b (each of length L).  Returns the buffer
// holding the result.  Used by the sine transforms of length 2(n+1).
template <typename T, bool INV>
__device__ __forceinline__ Line<T> fft_line_wide(Line<T> a, Line<T> b, const FFTPlan pl, int lane) {
  if (fft_try_fixed_wide<T, INV>(a, b, pl, lane)) return a;  // in place (b as scratch)
  const cx<T>* __restrict__ tw = (const cx<T>*)pl.tw;
  int Ns = 1, lg = 0;
  Line<T> src = a, dst = b;
  for (int s = 0; s < pl.nst; ++s) {
    const int R = stage_radix(pl, s);
    switch (R) {
      case 8: fft_stage_oop<T, 8, INV>(src, dst, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      case 4: fft_stage_oop<T, 4, INV>(src, dst, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      case 2: fft_stage_oop<T, 2, INV>(src, dst, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      case 3: fft_stage_oop<T, 3, INV>(src, dst, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      case 5: fft_stage_oop<T, 5, INV>(src, dst, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      case 7: fft_stage_prime_oop<T, 7, INV>(src, dst, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      case 11: fft_stage_prime_oop<T, 11, INV>(src, dst, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      case 13: fft_stage_prime_oop<T, 13, INV>(src, dst, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      case 17: fft_stage_prime_oop<T, 17, INV>(src, dst, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      case 19: fft_stage_prime_oop<T, 19, INV>(src, dst, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      case 23: fft_stage_prime_oop<T, 23, INV>(src, dst, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      case 29: fft_stage_prime_oop<T, 29, INV>(src, dst, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      case 31: fft_stage_prime_oop<T, 31, INV>(src, dst, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      case 37: fft_stage_prime_oop<T, 37, INV>(src, dst, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      case 41: fft_stage_prime_oop<T, 41, INV>(src, dst, pl.L, Ns, lg, tw, lane, pl.tpl); break;
      default: fft_stage_prime_oop<T, 43, INV>(src, dst, pl.L, Ns, lg, tw, lane, pl.tpl); break;
    }
    lg = next_lg(lg, R);
    Ns *= R;
    Line<T> t = src;
    src = dst;
    dst = t;
  }
  return src;
}

}  // namespace fl
