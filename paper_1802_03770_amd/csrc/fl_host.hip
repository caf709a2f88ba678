// Host driver and C ABI of the fractional Laplacian library (gfx950).
//
// Operator construction (Sec. 2.7 constants, Sec. 3.1 operator), FFT
// application (Sec. 3.1), sine-transform preconditioner (Sec. 3.1), PCG with
// the relative-residual test (Sec. 4), FP64 iterative refinement around an
// FP32 inner PCG, implicit theta steps (Sec. 3.2) and batched solves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <complex>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#define FL_MISC_KERNELS
#include "fl_internal.hpp"

using namespace fl;

thread_local std::string g_err;
std::atomic<long long> g_dallocs{0};

// ---------------------------------------------------------------------------
// plans and tables
// ---------------------------------------------------------------------------
static bool smooth235(long m) {
  for (int p : {2, 3, 5})
    while (m % p == 0) m /= p;
  return m == 1;
}
static int padded_length(int n) {
  int P = 2 * n;
  while (!smooth235(P / 2)) P += 2;
  return P;
}
static int smooth_at_least(int m) {
  int L = std::max(m, 2);
  while (!smooth235(L)) ++L;
  return L;
}

// Radix sequence for length L.  wide: also odd primes 7..43 (sine kernels).
static bool make_radices(int L, FFTPlan& pl, bool wide = false) {
  std::vector<int> r;
  int m = L;
  while (m % 8 == 0) { r.push_back(8); m /= 8; }
  while (m % 4 == 0) { r.push_back(4); m /= 4; }
  while (m % 2 == 0) { r.push_back(2); m /= 2; }
  while (m % 3 == 0) { r.push_back(3); m /= 3; }
  while (m % 5 == 0) { r.push_back(5); m /= 5; }
  if (wide)
    for (int p : {7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43})
      while (m % p == 0) { r.push_back(p); m /= p; }
  if (m != 1 || (int)r.size() > kMaxStages) return false;
  pl.L = L;
  pl.nst = (int)r.size();
  pl.fixed = 0;
  pl.radcode = 0;
  for (int i = 0; i < pl.nst; ++i) {
    int c = 0;
    while (radix_of_code(c) != r[i]) ++c;
    pl.radcode |= (unsigned long long)c << (4 * i);
  }
  if (L == 8192 && !wide) {
    // the one line longer than 4096: only its compile-time kernels (256 lanes,
    // four radix-8 butterflies per lane and stage) take it
    pl.tpl = c_fixed_tpl(L);
    pl.fixed = 1;
    return true;
  }
  int tpl = 1;
  while (tpl * kMaxElems < L) tpl *= 2;
  for (;;) {
    bool ok = true;
    for (int R : r) {
      int nb = L / R, per = (nb + tpl - 1) / tpl;
      if (per > std::max(1, kMaxElems / R)) ok = false;
    }
    if (ok) break;
    tpl *= 2;
  }
  if (tpl > 256) return false;  // kernels run 256-lane workgroups
  pl.tpl = tpl;
  pl.fixed = 0;
  if (c_is_fixed(L) && (wide || c_radix(L, c_nst(L) - 1) <= 8)) {
    pl.fixed = 1;  // the device has a compile-time version with these lanes
    pl.tpl = c_fixed_tpl(L);
  }
  return true;
}

static const long double kPiL = 3.141592653589793238462643383279502884197L;

// device table of e^{-2 pi i m / L}, m < L, in T
template <typename T> struct DevTab {
  std::vector<void*> owned;
};

struct fl_op_s;

template <typename T> static std::vector<cx<T>> host_twiddles(int L) {
  std::vector<cx<T>> t(L);
  for (int m = 0; m < L; ++m) {
    long double a = 2.0L * kPiL * (long double)m / (long double)L;
    t[m] = {(T)cosl(a), (T)(-sinl(a))};
  }
  return t;
}

// Tables of the prime-form sine transform, N = n + 1 prime (Rader's identity
// with a generator g of the units mod N; an FFT of length N - 1):
//   rtab  = int[(N-1)/2] g^-p mod N, then int[(N-1)/2 + 1] with entry k = log_g k
//   chirp = T[(N-1)/2] sin(pi g^-p / N)
//   bhat  = cx<T>[N-1] = DFT_{N-1}(b) / (N-1), b_m = e^{-2 pi i g^m / N}
template <typename T> struct RaderHost {
  std::vector<int> tab;
  std::vector<T> sp;
  std::vector<cx<T>> bh;
};
template <typename T> static RaderHost<T> rader_host(int N);

// The host tables depend on N and the precision only: computed once per
// process (the DFT of b is N^2 long-double terms) and uploaded per op.
template <typename T> static fl_status rader_tables(fl_op op, Axis& A, int N) {
  static std::mutex mu;
  static std::map<int, RaderHost<T>> cache;
  const RaderHost<T>* h;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(N);
    if (it == cache.end()) it = cache.emplace(N, rader_host<T>(N)).first;
    h = &it->second;
  }
  STCHK(upload(op, h->tab, &A.rtab));
  STCHK(upload(op, h->sp, &A.chirp));
  STCHK(upload(op, h->bh, &A.bhat));
  return FL_OK;
}

template <typename T> static RaderHost<T> rader_host(int N) {
  const int RL = N - 1, HALF = RL / 2;
  int g = 2;
  for (;; ++g) {  // smallest generator: g^(RL/q) != 1 for every prime q | RL
    bool gen = true;
    for (int q = 2, m = RL; q <= m; ++q) {
      if (m % q) continue;
      while (m % q == 0) m /= q;
      long e = 1, b = g;
      for (int k = RL / q; k; k >>= 1, b = b * b % N)
        if (k & 1) e = e * b % N;
      if (e == 1) gen = false;
    }
    if (gen) break;
  }
  std::vector<long> pw(RL);  // g^m mod N
  pw[0] = 1;
  for (int m = 1; m < RL; ++m) pw[m] = pw[m - 1] * g % N;
  std::vector<int> tab(HALF + HALF + 1, 0);
  std::vector<T> sp(HALF);
  for (int p = 0; p < HALF; ++p) {
    const long j = pw[(RL - p) % RL];  // g^-p
    tab[p] = (int)j;
    sp[p] = (T)sinl(kPiL * (long double)j / (long double)N);
  }
  for (int q = 0; q < RL; ++q)
    if (pw[q] <= HALF) tab[HALF + pw[q]] = q;
  std::vector<cx<T>> bh(RL);
  for (int k = 0; k < RL; ++k) {
    long double re = 0.0L, im = 0.0L;
    for (int m = 0; m < RL; ++m) {
      // b_m e^{-2 pi i m k / RL} = e^{-2 pi i (g^m / N + m k / RL)}
      const long double ph = 2.0L * kPiL * ((long double)pw[m] / N + (long double)((long)m * k % RL) / RL);
      re += cosl(ph);
      im -= sinl(ph);
    }
    bh[k] = {(T)(re / RL), (T)(im / RL)};
  }
  return RaderHost<T>{std::move(tab), std::move(sp), std::move(bh)};
}

template <typename T> static fl_status build_axis(fl_op op, int a, int form) {
  Axis& A = op->ax[tix<T>()][a];
  const int n = op->n[a];
  A.n = n;
  A.P = op->P[a];
  A.H = op->H[a];
  if (!make_radices(A.P, A.fft))
    return fail(FL_E_UNSUPPORTED, "no FFT plan for padded length " + std::to_string(A.P) +
                                      " (lengths above 4096 other than 8192 are not supported)");
  STCHK(upload(op, host_twiddles<T>(A.P), &A.fft.tw));
  if (op->apply_only) return FL_OK;  // no sine transforms on application-only grids
  // sine transform: direct (odd extension of length 2(n+1), two lines per FFT
  // line) when 2(n+1) factors over the wide radix set; the prime form (two lines
  // per FFT line, Rader's identity with an FFT of length 256) when n + 1 = 257;
  // else the chirp-z identity
  A.dst_direct = (form != 2 && make_radices(2 * (n + 1), A.dst, true)) ? 1 : 0;
  A.dst_rader = (form != 2 && !A.dst_direct && n + 1 == kRaderLF) ? 1 : 0;
  if (A.dst_rader) A.dst_direct = 1;
  op->dst_form[tix<T>()][a] = A.dst_rader ? 3 : (A.dst_direct ? 1 : 2);
  const int Lb = A.dst_rader ? kRaderLF - 1 : (A.dst_direct ? 2 * (n + 1) : smooth_at_least(2 * n - 1));
  if ((A.dst_rader || !A.dst_direct) && !make_radices(Lb, A.dst))
    return fail(FL_E_UNSUPPORTED, "sine transform length");
  if (A.dst_rader && !(A.dst.fixed && A.dst.tpl == c_fixed_tpl(Lb)))
    return fail(FL_E_UNSUPPORTED, "prime-form sine transform needs the compile-time FFT of length 256");
  STCHK(upload(op, host_twiddles<T>(Lb), &A.dst.tw));
  const long N1 = n + 1;
  std::vector<T> ev(n);
  for (int k = 0; k < n; ++k) {
    long double sn = sinl(kPiL * (k + 1) / (2.0L * N1));
    ev[k] = (T)(4.0L * sn * sn);
  }
  STCHK(upload(op, ev, &A.eig));
  if (A.dst_rader) return rader_tables<T>(op, A, n + 1);
  if (A.dst_direct) return FL_OK;
  std::vector<cx<T>> ch(n + 1);
  std::vector<std::complex<long double>> chl(n + 1);
  for (long m = 0; m <= n; ++m) {
    long q = (m * m) % (4 * N1);  // e^{i pi m^2 / (2 N1)} has period 4 N1 in m^2
    long double ph = kPiL * (long double)q / (2.0L * (long double)N1);
    chl[m] = {cosl(ph), sinl(ph)};
    ch[m] = {(T)chl[m].real(), (T)chl[m].imag()};
  }
  STCHK(upload(op, ch, &A.chirp));
  // bhat = DFT_Lb(b~) / Lb, b~[m mod Lb] = conj(ch[|m|]) for |m| <= n-1
  std::vector<std::complex<long double>> tw(Lb);
  for (int m = 0; m < Lb; ++m) {
    long double ang = 2.0L * kPiL * m / Lb;
    tw[m] = {cosl(ang), -sinl(ang)};
  }
  std::vector<std::pair<int, std::complex<long double>>> nz;
  for (int m = -(n - 1); m <= n - 1; ++m) nz.push_back({((m % Lb) + Lb) % Lb, std::conj(chl[std::abs(m)])});
  std::vector<cx<T>> bh(Lb);
  for (int k = 0; k < Lb; ++k) {
    std::complex<long double> s = 0;
    for (auto& e : nz) s += e.second * tw[((long)e.first * k) % Lb];
    s /= (long double)Lb;
    bh[k] = {(T)s.real(), (T)s.imag()};
  }
  STCHK(upload(op, bh, &A.bhat));
  return FL_OK;
}

fl_op_s::~fl_op_s() {
  cap_destroy(this);
  for (void* p : tables) hipFree(p);
  for (auto& w : ws) {
    drop_graph(w);
    for (void* p : {w.W1, w.W2, w.T1, w.x, w.r, w.z, w.p, w.q, w.f}) if (p) hipFree(p);
    if (w.sc) hipFree(w.sc);
    if (w.part) hipFree(w.part);
  }
  if (d_cst) hipFree(d_cst);
  if (wf) hipFree(wf);
  for (void* p : lam) if (p) hipFree(p);
  if (hsc) hipHostFree(hsc);
}

// ---------------------------------------------------------------------------
// operator construction
// ---------------------------------------------------------------------------
static fl_status build_symbol(fl_op op) {
  hipStream_t s = op->stream;
  HIPCHK(hipMemcpyAsync(op->lam[0], op->wf, op->NH * sizeof(double), hipMemcpyDeviceToDevice, s));
  for (int a = 0; a < op->d; ++a) {
    long inner = 1, nl = 1;
    for (int b = 0; b < op->d; ++b) {
      if (b > a) inner *= op->H[b];
      if (b != a) nl *= op->H[b];
    }
    const FFTPlan& pl = op->ax[0][a].fft;
    int nt = block_for(pl.tpl), G = nt / pl.tpl;
    long pairs = (nl + 1) / 2;
    const size_t sm = (size_t)G * Line<double>::stride(op->P[a]) * sizeof(cx<double>);
    if (op->P[a] == 8192)
      LAUNCH(k_dct1_axis<8192>, dim3((pairs + G - 1) / G), dim3(nt), sm, s, (double*)op->lam[0], op->H[a], op->P[a],
             inner, nl, pl);
    else
      LAUNCH(k_dct1_axis<>, dim3((pairs + G - 1) / G), dim3(nt), sm, s, (double*)op->lam[0], op->H[a], op->P[a],
             inner, nl, pl);
  }
  LAUNCH(k_cast<float, double>, dim3((op->NH + 255) / 256), dim3(256), 0, s, (const double*)op->lam[0],
         (float*)op->lam[1], op->NH, 1.0);
  return FL_OK;
}

template <typename T> static fl_status profile_t(fl_op op, int pass, int reps, double* avg_ms);

// Autotuner of the sine-transform plan: where some axis admits the direct odd
// extension, time the whole preconditioner with the direct plans and with the
// chirp-z plans (same workspace, HIP events on the op stream) and keep the
// faster for this precision.
// Autotuner of the symbol column pass (lengths 1024 and 2048 along axis 0 of
// a 2D grid): time the pass with the run-time plan and with 64 and 128 lanes
// per column, keep the fastest for this precision.
template <typename T> static fl_status autotune_col(fl_op op) {
  Axis& A = op->ax[tix<T>()][0];
  if (op->d != 2 || !A.fft.fixed || (A.P != 2048 && A.P != 1024)) return FL_OK;
  if (op->col_lanes != 0) {  // forced
    A.col_tplf = op->col_lanes > 0 ? op->col_lanes : 0;
    return FL_OK;
  }
  const int opts[4] = {0, 64, 128, 256};
  double best = 1e30;
  int pick = 0;
  for (int o : opts) {
    if ((o == 128 || o == 256) && (A.P == 1024)) continue;
    if (o == 64 && A.P == 2048 && sizeof(T) == 8) continue;
    A.col_tplf = o;
    double ms = 0.0;
    STCHK(profile_t<T>(op, 1, 5, &ms));
    if (ms < best) {
      best = ms;
      pick = o;
    }
  }
  A.col_tplf = pick;
  return FL_OK;
}

// Autotuner of the sine column pass at direct length 2050 (grids of 1024):
// the plan's lanes per FFT line or 128 (two FFT lines per block), per precision.
template <typename T> static fl_status autotune_dcol(fl_op op) {
  Axis& A = op->ax[tix<T>()][0];
  if (op->d != 2 || !A.dst_direct || !A.dst.fixed || A.dst.L != 2050) return FL_OK;
  if (op->sine_col_lanes != 0) {  // forced
    A.dcol_tplf = op->sine_col_lanes > 0 ? 128 : 0;
    return FL_OK;
  }
  double t0 = 0.0, t1 = 0.0;
  A.dcol_tplf = 0;
  STCHK(profile_t<T>(op, 4, 5, &t0));
  A.dcol_tplf = 128;
  STCHK(profile_t<T>(op, 4, 5, &t1));
  A.dcol_tplf = t1 < t0 ? 128 : 0;
  return FL_OK;
}

template <typename T> static fl_status autotune_dst(fl_op op) {
  bool any = false;
  for (int a = 0; a < op->d; ++a) any = any || op->dst_form[tix<T>()][a] == 1 || op->dst_form[tix<T>()][a] == 3;
  if (!any) return FL_OK;
  double t_direct = 0.0, t_chirp = 0.0;
  STCHK(profile_t<T>(op, 7, 4, &t_direct));
  for (int a = 0; a < op->d; ++a) STCHK(build_axis<T>(op, a, 2));
  STCHK(profile_t<T>(op, 7, 4, &t_chirp));
  if (t_direct <= t_chirp)
    for (int a = 0; a < op->d; ++a) STCHK(build_axis<T>(op, a, 1));
  return FL_OK;
}

// Process-wide record of the autotuners' choices, per device and grid (and
// the forced options the op was created with).
struct TuneKey {
  int dev, d, n[3], dst_mode, col_lanes, sine_col_lanes;
  bool operator<(const TuneKey& o) const {
    return std::tie(dev, d, n[0], n[1], n[2], dst_mode, col_lanes, sine_col_lanes) <
           std::tie(o.dev, o.d, o.n[0], o.n[1], o.n[2], o.dst_mode, o.col_lanes, o.sine_col_lanes);
  }
};
struct TuneVal {
  int dst_form[2][3], col_tplf[2], dcol_tplf[2];
};
static std::mutex g_tune_mu;
static std::map<TuneKey, TuneVal> g_tune;
static bool tune_lookup(const TuneKey& k, TuneVal* v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(k);
  if (it == g_tune.end()) return false;
  *v = it->second;
  return true;
}
static void tune_store(const TuneKey& k, const TuneVal& v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[k] = v;
}

static fl_status make_op(int d, double alpha, double h, const int64_t* n, const fl_weights_opts* o,
                         void* stream, fl_op* out) {
  if (!out) return fail(FL_E_INVALID, "out is NULL");
  *out = nullptr;
  if (d < 1 || d > 3) return fail(FL_E_INVALID, "d must be 1, 2 or 3");
  if (!(alpha > 0.0 && alpha < 2.0)) return fail(FL_E_INVALID, "alpha must lie in (0, 2)");
  if (!(h > 0.0) || !std::isfinite(h)) return fail(FL_E_INVALID, "h must be positive");
  if (!n) return fail(FL_E_INVALID, "n is NULL");
  for (int a = 0; a < d; ++a)
    if (n[a] < 1 || n[a] > (1 << 20)) return fail(FL_E_INVALID, "grid sizes must be >= 1");
  fl_op op = new fl_op_s();
  op->d = d;
  op->alpha = alpha;
  op->h = h;
  op->c = (o && o->delta_over_h > 0) ? o->delta_over_h : 20.0;
  op->stream = (hipStream_t)stream;
  op->N = 1;
  op->NH = 1;
  for (int a = 0; a < d; ++a) {
    op->n[a] = (int)n[a];
    op->P[a] = padded_length(op->n[a]);
    op->H[a] = op->P[a] / 2 + 1;
    op->N *= op->n[a];
    op->NH *= op->H[a];
  }
  auto bail = [&](fl_status s) {
    delete op;
    return s;
  };
  fl_status st;
  if ((st = dalloc((void**)&op->d_cst, 8 * sizeof(double))) != FL_OK) return bail(st);
  if ((st = dalloc((void**)&op->wf, op->NH * sizeof(double))) != FL_OK) return bail(st);
  if ((st = dalloc(&op->lam[0], op->NH * sizeof(double))) != FL_OK) return bail(st);
  if ((st = dalloc(&op->lam[1], op->NH * sizeof(float))) != FL_OK) return bail(st);
  if (hipHostMalloc((void**)&op->hsc, sizeof(Scalars)) != hipSuccess) return bail(fail(FL_E_NOMEM, "pinned"));
  for (int a = 0; a < 3; ++a) {
    memset(&op->ax[0][a], 0, sizeof(Axis));
    memset(&op->ax[1][a], 0, sizeof(Axis));
  }
  op->dst_mode = (o && o->dst_mode >= 0 && o->dst_mode <= 2) ? o->dst_mode : 0;
  op->col_lanes =
      (o && (o->col_lanes == -1 || o->col_lanes == 64 || o->col_lanes == 128 || o->col_lanes == 256)) ? o->col_lanes : 0;
  op->sine_col_lanes = (o && (o->sine_col_lanes == -1 || o->sine_col_lanes == 128)) ? o->sine_col_lanes : 0;
  // Grids padded to 8192 points along an axis (n = 4081 .. 4096) are
  // application-only, in 2D: their FFT lines have compile-time kernels for the
  // application passes and the symbol, but no sine transforms, solves, steps
  // or batches.
  for (int a = 0; a < d; ++a) op->apply_only = op->apply_only || op->P[a] > 4096;
  if (op->apply_only && d != 2) return bail(fail(FL_E_UNSUPPORTED, "padded lengths above 4096 are supported in 2D only"));
  for (int a = 0; a < d; ++a) {
    if ((st = build_axis<double>(op, a, op->dst_mode == 2 ? 2 : 1)) != FL_OK) return bail(st);
    if ((st = build_axis<float>(op, a, op->dst_mode == 2 ? 2 : 1)) != FL_OK) return bail(st);
  }
  hipStream_t s = op->stream;
  if (launch(k_constants, dim3(1), dim3(256), 0, s, d, alpha, h, op->c, op->d_cst) != hipSuccess)
    return bail(fail(FL_E_HIP, "constants kernel"));
  if (launch(k_weights, dim3((op->NH + 255) / 256), dim3(256), 0, s, d, alpha, op->n[0], op->n[1], op->n[2],
             op->H[0], op->H[1], op->H[2], (const double*)op->d_cst, op->wf) != hipSuccess)
    return bail(fail(FL_E_HIP, "weights kernel"));
  if ((st = build_symbol(op)) != FL_OK) return bail(st);
  if (hipMemcpyAsync(op->cst, op->d_cst, 8 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return bail(fail(FL_E_HIP, "constants readback"));
  // the plans depend on the grid and the device only: a shape tuned before
  // on this device takes the recorded choice without timing again
  TuneKey key;
  key.dev = 0;
  (void)hipGetDevice(&key.dev);
  key.d = d;
  for (int a = 0; a < 3; ++a) key.n[a] = op->n[a];
  key.dst_mode = op->dst_mode;
  key.col_lanes = op->col_lanes;
  key.sine_col_lanes = op->sine_col_lanes;
  TuneVal tv;
  if (tune_lookup(key, &tv)) {
    for (int p = 0; p < 2; ++p)
      for (int a = 0; a < d; ++a)
        if (tv.dst_form[p][a] != op->dst_form[p][a]) {
          st = p == 0 ? build_axis<double>(op, a, tv.dst_form[p][a]) : build_axis<float>(op, a, tv.dst_form[p][a]);
          if (st != FL_OK) return bail(st);
        }
    for (int p = 0; p < 2; ++p) {
      op->ax[p][0].col_tplf = tv.col_tplf[p];
      op->ax[p][0].dcol_tplf = tv.dcol_tplf[p];
    }
    *out = op;
    return FL_OK;
  }
  if (op->dst_mode == 0) {
    if ((st = autotune_dst<double>(op)) != FL_OK) return bail(st);
    if ((st = autotune_dst<float>(op)) != FL_OK) return bail(st);
  }
  if ((st = autotune_col<double>(op)) != FL_OK) return bail(st);
  if ((st = autotune_col<float>(op)) != FL_OK) return bail(st);
  if ((st = autotune_dcol<double>(op)) != FL_OK) return bail(st);
  if ((st = autotune_dcol<float>(op)) != FL_OK) return bail(st);
  for (int p = 0; p < 2; ++p) {
    for (int a = 0; a < 3; ++a) tv.dst_form[p][a] = op->dst_form[p][a];
    tv.col_tplf[p] = op->ax[p][0].col_tplf;
    tv.dcol_tplf[p] = op->ax[p][0].dcol_tplf;
  }
  tune_store(key, tv);
  *out = op;
  return FL_OK;
}

// Sine-basis diagonal of M: tau_k = sum_m w_m prod_a G_a(k_a, m_a), one FP64
// mode product per axis (w already carries C h^-alpha), then an FP32 copy.
fl_status build_tau(fl_op op) {
  if (op->tau[0]) return FL_OK;
  hipStream_t s = op->stream;
  const int d = op->d;
  const long N = op->N;
  void *X = nullptr, *Y = nullptr, *G = nullptr, *t32 = nullptr;
  int nmax = 1;
  for (int a = 0; a < d; ++a) nmax = std::max(nmax, op->n[a]);
  STCHK(dalloc(&X, N * sizeof(double)));
  op->tables.push_back(X);
  STCHK(dalloc(&Y, N * sizeof(double)));
  op->tables.push_back(Y);
  STCHK(dalloc(&G, (size_t)nmax * nmax * sizeof(double)));
  op->tables.push_back(G);
  STCHK(dalloc(&t32, N * sizeof(float)));
  op->tables.push_back(t32);
  LAUNCH(k_weight_block, dim3(nblocks_vec(N)), dim3(256), 0, s, (const double*)op->wf, (double*)X, op->n[0],
         op->n[1], op->n[2], op->H[1], op->H[2]);
  for (int a = 0; a < d; ++a) {
    const int na = op->n[a];
    long Aa = 1, Ba = 1;
    for (int b = 0; b < d; ++b) {
      if (b < a) Aa *= op->n[b];
      if (b > a) Ba *= op->n[b];
    }
    LAUNCH(k_sine_corr, dim3(nblocks_vec((long)na * na)), dim3(256), 0, s, (double*)G, na);
    if (Ba > 1) {
      // Y_i(k, j) = sum_m G(k, m) X_i(m, j), one product per leading index i
      if (Aa > 65535) return fail(FL_E_UNSUPPORTED, "grid too large for the diagonal table");
      LAUNCH(k_gemm_f64, dim3((Ba + 63) / 64, (na + 63) / 64, Aa), dim3(256), 0, s, na, (int)Ba, na,
             (const double*)G, (long)na, 1L, 0L, (const double*)X, Ba, 1L, na * Ba, (double*)Y, Ba, 1L, na * Ba);
    } else {
      // last axis: Y(i, k) = sum_m X(i, m) G(k, m)
      LAUNCH(k_gemm_f64, dim3((na + 63) / 64, (Aa + 63) / 64, 1), dim3(256), 0, s, (int)Aa, na, na,
             (const double*)X, (long)na, 1L, 0L, (const double*)G, 1L, (long)na, 0L, (double*)Y, (long)na, 1L, 0L);
    }
    std::swap(X, Y);
  }
  LAUNCH(k_cast<float, double>, dim3(nblocks_vec(N)), dim3(256), 0, s, (const double*)X, (float*)t32, N, 1.0);
  HIPCHK(hipStreamSynchronize(s));
  op->tau[0] = X;
  op->tau[1] = t32;
  return FL_OK;
}

// ---------------------------------------------------------------------------
// Krylov drivers
// ---------------------------------------------------------------------------
// y *= mask (restriction of a grid function to the domain)
template <typename T> __global__ void k_mask_mul(T* __restrict__ y, const uint8_t* __restrict__ m, long n) {
  const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n && !m[i]) y[i] = (T)0;
}

template <typename T> static fl_status one_iteration(fl_op op, const Prob& pb, int pc, int k, bool cap) {
  Iter it = {k & 1, k == 0 ? 1 : 0};
  Prob pz = pb;
  if (!pc) pz.z = pb.r;  // z aliases r without a preconditioner
  STCHK((apply_seq<T, PRO_PUPD, EPI_PQ>(op, pz, it, 1)));
  if (pc && cap) {
    STCHK((cap_precond_seq<T, DPRO_UPD, DEPI_Z>(op, pb, it, 1)));
  } else if (pc) {
    STCHK((precond_seq<T, DPRO_UPD, DEPI_Z>(op, pb, it, 1)));
  } else {
    long nb = std::min<long>(2048, (op->N + 255) / 256);
    LAUNCH(k_update<T>, dim3(nb), dim3(256), 0, op->stream, pb, it, op->N);
  }
  return FL_OK;
}

static fl_status read_scalars(fl_op op, Scalars* dsc) {
  HIPCHK(hipMemcpyAsync(op->hsc, dsc, sizeof(Scalars), hipMemcpyDeviceToHost, op->stream));
  HIPCHK(hipStreamSynchronize(op->stream));
  return FL_OK;
}

// PCG on the workspace of type T: r holds the initial residual, x the initial
// iterate, sc->ff the squared rhs norm (and sc->rr the squared residual norm
// if use_rr).  Returns after convergence / cap / breakdown.
template <typename T> static fl_status krylov(fl_op op, const Prob& pb, int pc, double tol, int maxit,
                                              int use_rr, int graph, int poll, Scalars* out, bool cap) {
  hipStream_t s = op->stream;
  Workspace& w = op->ws[tix<T>()];
  LAUNCH(k_init<>, dim3(1), dim3(64), 0, s, pb, tol, maxit, use_rr);
  if (pc) {
    Prob p0 = pb;
    p0.in = pb.r;
    if (cap) STCHK((cap_precond_seq<T, DPRO_PLAIN, DEPI_Z>(op, p0, Iter{1, 0}, 0)));
    else STCHK((precond_seq<T, DPRO_PLAIN, DEPI_Z>(op, p0, Iter{1, 0}, 0)));
  } else {
    // rz[0] = r.r
    long nb = std::min<long>(1024, (op->N + 255) / 256);
    LAUNCH(k_dot<T>, dim3(nb), dim3(256), 0, s, pb, (const void*)pb.r, (const void*)pb.r, (int)S_RZ0, op->N);
  }
  if (poll <= 0) poll = 8;
  if (poll & 1) ++poll;
  // iteration 0 eagerly, then blocks of `poll` iterations
  STCHK(one_iteration<T>(op, pb, pc, 0, cap));
  int k = 1;
  bool use_graph = graph != 0 && op->stream != nullptr;
  if (use_graph) {
    bool rebuild = !w.gexec || w.gK != poll || w.gpc != pc || w.gs0 != pb.s0 || w.gs1 != pb.s1 ||
                   w.gp0 != pb.p0 || w.gp1 != pb.p1 || w.gmask != pb.mask || w.gcap != (int)cap;
    if (rebuild) {
      if (w.gexec) {
        hipGraphExecDestroy(w.gexec);
        w.gexec = nullptr;
      }
      hipGraph_t g;
      HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      fl_status st = FL_OK;
      for (int j = 0; j < poll && st == FL_OK; ++j) st = one_iteration<T>(op, pb, pc, 1 + j, cap);
      hipError_t e = hipStreamEndCapture(s, &g);
      if (st != FL_OK) return st;
      HIPCHK(e);
      HIPCHK(hipGraphInstantiate(&w.gexec, g, nullptr, nullptr, 0));
      hipGraphDestroy(g);
      w.gK = poll;
      w.gpc = pc;
      w.gs0 = pb.s0;
      w.gs1 = pb.s1;
      w.gp0 = pb.p0;
      w.gp1 = pb.p1;
      w.gmask = pb.mask;
      w.gcap = (int)cap;
    }
  }
  for (;;) {
    STCHK(read_scalars(op, pb.sc));
    if (op->hsc->done) break;
    if (std::max(op->hsc->itc[0], op->hsc->itc[1]) >= maxit + 2 * poll)
      return fail(FL_E_HIP, "iteration bookkeeping lost");
    if (use_graph) {
      HIPCHK(hipGraphLaunch(w.gexec, s));
      k += poll;
    } else {
      for (int j = 0; j < poll; ++j, ++k) STCHK(one_iteration<T>(op, pb, pc, k, cap));
    }
  }
  *out = *op->hsc;
  out->itc[0] = std::max(op->hsc->itc[0], op->hsc->itc[1]);  // iterations done
  return FL_OK;
}



// True FP64 residual r = b - A x into ws64.q; returns ||r||^2 via sc->rr.
static fl_status true_residual(fl_op op, const uint8_t* mask, double s0, double s1, const double* x,
                               const double* b, double* out, double* rr) {
  Workspace& w = op->ws[0];
  Prob pb = solver_prob<double>(op, mask, s0, s1, 0, 1);
  pb.in = x;
  pb.aux = b;
  pb.out = out;
  STCHK((apply_seq<double, PRO_PLAIN, EPI_RESID>(op, pb, Iter{0, 0}, 0)));
  LAUNCH(k_finalize<>, dim3(1), dim3(256), 0, op->stream, pb, (int)S_DOT, (int)FIN_RR);
  STCHK(read_scalars(op, w.sc));
  *rr = op->hsc->rr;
  return FL_OK;
}

// Solve (s0 I + s1 M) x = b where b is ws64.f and x is ws64.x (initial guess
// when use_x0, otherwise zeroed here).  Preconditioner p0 I + p1 pcs T.
static fl_status solve_system(fl_op op, const uint8_t* mask, double s0, double s1, double p0, double p1,
                              double tol, const fl_solve_opts* o, int use_x0, fl_info* info) {
  hipStream_t s = op->stream;
  const long N = op->N;
  int pc = o ? o->pc : FL_PC_FD;
  if (pc == FL_PC_AUTO) pc = op->alpha < 1.0 ? FL_PC_NONE : FL_PC_FD;  // Sec. 4.1-4.2: none below alpha = 1
  if (pc != FL_PC_NONE && !pc_is_sine(pc) && pc != FL_PC_LEARNED) return fail(FL_E_INVALID, "unknown preconditioner");
  fl_net net = o ? o->net : nullptr;
  if (pc == FL_PC_LEARNED) {
    if (mask) return fail(FL_E_UNSUPPORTED, "the learned preconditioner is built for the box (no mask)");
    STCHK(learned_prepare(op, net, 0));
  }
  const int mixed = o ? o->mixed : 0;
  const int graph = o ? o->graph : 1;
  const int poll = (o && o->poll_every > 0) ? o->poll_every : 8;
  int maxit = (o && o->maxit > 0) ? o->maxit : std::max(1000, (int)(10 * std::sqrt((double)N)));
  Workspace& w = op->ws[0];
  fl_info inf;
  memset(&inf, 0, sizeof(inf));
  // the mixed loop ends with the true FP64 residual of the returned x in hand
  bool have_final = false;
  double rr_final = 0.0;
  // on a mask the system lives on Omega: f and the initial iterate restricted to it
  const bool cap_want = mask && pc_exact_on_mask(pc);
  {
    Prob pm = solver_prob<double>(op, mask, s0, s1, p0, p1);
    if (mask) {
      LAUNCH(k_mask_mul<double>, dim3(nblocks_vec(N)), dim3(256), 0, s, (double*)w.f, mask, N);
      if (use_x0) LAUNCH(k_mask_mul<double>, dim3(nblocks_vec(N)), dim3(256), 0, s, (double*)w.x, mask, N);
    }
    if (cap_want) STCHK(cap_hash_launch(op, mask, &w.sc->mhash));
    // ff
    LAUNCH(k_dot<double>, dim3(std::min<long>(1024, nblocks_vec(N))), dim3(256), 0, s, pm, (const void*)w.f,
           (const void*)w.f, (int)S_DOT, N);
    LAUNCH(k_finalize<>, dim3(1), dim3(256), 0, s, pm, (int)S_DOT, (int)FIN_FF);
    if (!use_x0) LAUNCH(k_fill<double>, dim3(nblocks_vec(N)), dim3(256), 0, s, (double*)w.x, 0.0, N);
    STCHK(read_scalars(op, w.sc));
  }
  bool cap = false;
  if (cap_want) {
    // the exact preconditioner on Omega: capacitance correction of the box inverse
    Prob pbox = base_prob<double>(op, 1);
    pbox.p0 = p0;
    pbox.p1 = p1;
    STCHK(set_precond<double>(op, pbox, pc));
    const unsigned long long key = op->hsc->mhash;
    STCHK(cap_prepare(op, mask, pbox, key, &cap));
    STCHK(ensure_ws<double>(op, 1, true));  // the build may have returned its batched workspace
    if (cap) {
      STCHK(cap_buffers<double>(op, 1));
      if (mixed) STCHK(cap_buffers<float>(op, 1));
    }
  }
  Prob pb = solver_prob<double>(op, mask, s0, s1, p0, p1);
  STCHK(set_precond<double>(op, pb, pc));
  const double ff = op->hsc->ff;
  if (!std::isfinite(ff)) {
    info->status = FL_E_INVALID;
    return fail(FL_E_INVALID, "right-hand side is not finite");
  }
  if (!mixed) {
    if (use_x0) {
      double rr;
      STCHK(true_residual(op, mask, s0, s1, (const double*)w.x, (const double*)w.f, (double*)w.r, &rr));
    } else {
      HIPCHK(hipMemcpyAsync(w.r, w.f, N * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    if (pc == FL_PC_LEARNED) {
      double rr0 = ff;
      if (use_x0) {
        STCHK(read_scalars(op, w.sc));
        rr0 = op->hsc->rr;
      }
      int its = 0, stt = 0, fb = 0;
      double rrf = 0.0;
      STCHK(learned_fcg<double>(op, net, pb, tol, maxit, ff, rr0, graph, &its, &rrf, &stt, &fb));
      inf.iters = its;
      inf.fell_back = fb;
      inf.rel_res_recur = ff > 0 ? std::sqrt(rrf / ff) : 0.0;
      inf.status = stt == 1 ? FL_OK : stt == 2 ? FL_E_NOCONV : FL_E_BREAKDOWN;
    } else {
      Scalars res;
      STCHK(krylov<double>(op, pb, pc, tol, maxit, use_x0, graph, poll, &res, cap));
      inf.iters = res.itc[0];
      inf.rel_res_recur = ff > 0 ? std::sqrt(res.rr / ff) : 0.0;
      inf.status = res.done == 1 ? FL_OK : res.done == 2 ? FL_E_NOCONV : FL_E_BREAKDOWN;
    }
  } else {
    have_final = true;
    STCHK(ensure_ws<float>(op, 1, true));
    Workspace& w32 = op->ws[1];
    Prob p32 = solver_prob<float>(op, mask, s0, s1, p0, p1);
    STCHK(set_precond<float>(op, p32, pc));
    const double itol = (o && o->inner_tol > 0) ? o->inner_tol : 1e-4;
    const int max_outer = (o && o->max_outer > 0) ? o->max_outer : 12;
    int inner_cap = (o && o->maxit > 0) ? o->maxit : std::max(1000, (int)(10 * std::sqrt((double)N)));
    inf.status = FL_E_NOCONV;
    for (int outer = 0;; ++outer) {
      double rr;
      const double* r64 = (const double*)w.r;
      if (outer == 0 && !use_x0 && !mask) {
        // x = 0 (filled above): the residual is f itself and rr the ff read
        // above, with no application or host read
        rr = ff;
        r64 = (const double*)w.f;
      } else {
        STCHK(true_residual(op, mask, s0, s1, (const double*)w.x, (const double*)w.f, (double*)w.r, &rr));
      }
      rr_final = rr;  // every exit below leaves x as it was here
      if (ff == 0.0 || std::sqrt(rr / ff) <= tol) {
        inf.status = FL_OK;
        break;
      }
      if (!std::isfinite(rr)) {
        inf.status = FL_E_BREAKDOWN;
        break;
      }
      if (outer >= max_outer) break;
      inf.outer_iters = outer + 1;
      // r32 = r64 / ||r64||, x32 = 0, inner PCG to itol
      const double nr = std::sqrt(rr);
      LAUNCH((k_axpby<double, float>), dim3(nblocks_vec(N)), dim3(256), 0, s, r64, (float*)w32.r, 1.0 / nr, 0.0,
             N);
      LAUNCH(k_fill<float>, dim3(nblocks_vec(N)), dim3(256), 0, s, (float*)w32.x, 0.0f, N);
      Scalars res;
      if (pc == FL_PC_LEARNED) {
        // the scaled residual has unit norm up to FP32 rounding (~1e-7
        // relative), far below the inner tolerance: no device reduction and
        // no host read before the inner solve
        const double ff32 = 1.0;
        int its = 0, stt = 0, fb = 0;
        double rrf = 0.0;
        STCHK(learned_fcg<float>(op, net, p32, itol, inner_cap, ff32, ff32, graph, &its, &rrf, &stt, &fb));
        res.itc[0] = its;
        res.rr = rrf;
        res.ff = ff32;
        res.done = stt;
        inf.fell_back |= fb;
      } else {
        LAUNCH(k_dot<float>, dim3(std::min<long>(1024, nblocks_vec(N))), dim3(256), 0, s, p32,
               (const void*)w32.r, (const void*)w32.r, (int)S_DOT, N);
        LAUNCH(k_finalize<>, dim3(1), dim3(256), 0, s, p32, (int)S_DOT, (int)FIN_FF);
        STCHK(krylov<float>(op, p32, pc, itol, inner_cap, 0, graph, poll, &res, cap));
      }
      inf.iters += res.itc[0];
      inf.rel_res_recur = res.ff > 0 ? std::sqrt(res.rr / res.ff) : 0.0;
      if (res.done == 3) {
        inf.status = FL_E_BREAKDOWN;
        break;
      }
      // x64 += ||r|| x32
      LAUNCH((k_axpby<float, double>), dim3(nblocks_vec(N)), dim3(256), 0, s, (const float*)w32.x,
             (double*)w.x, nr, 1.0, N);
    }
  }
  // true residual in FP64
  double rr = rr_final;
  if (!have_final) STCHK(true_residual(op, mask, s0, s1, (const double*)w.x, (const double*)w.f, (double*)w.q, &rr));
  inf.rel_res_true = ff > 0 ? std::sqrt(rr / ff) : 0.0;
  *info = inf;
  return FL_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
template <typename T>
static fl_status apply_t(fl_op op, const void* u, void* Mu, long batch, const uint8_t* mask, double s0, double s1) {
  STCHK(ensure_ws<T>(op, batch, false));
  Workspace& w = op->ws[tix<T>()];
  Prob pb = base_prob<T>(op, batch);
  pb.s0 = s0;
  pb.s1 = s1;
  pb.in = u;
  pb.out = Mu;
  pb.W1 = w.W1;
  pb.W2 = w.W2;
  pb.mask = mask;
  pb.sc = w.sc;
  pb.part = w.part;
  pb.pstride = w.npart;
  return apply_seq<T, PRO_PLAIN, EPI_PLAIN>(op, pb, Iter{0, 0}, 0);
}

template <typename T>
static fl_status precond_t(fl_op op, const void* r, void* z, long batch, const uint8_t* mask, double p0, double p1,
                           int kind) {
  if (!pc_is_sine(kind)) return fail(FL_E_INVALID, "kind must be FL_PC_FD, SPECTRAL, MTILDE or FD_BOX");
  STCHK(ensure_ws<T>(op, batch, false));
  bool cap = false;
  if (mask && pc_exact_on_mask(kind)) {
    Workspace& w0 = op->ws[tix<T>()];
    STCHK(cap_hash_launch(op, mask, &w0.sc->mhash));
    STCHK(read_scalars(op, w0.sc));
    Prob pbox = base_prob<double>(op, 1);
    pbox.p0 = p0;
    pbox.p1 = p1;
    STCHK(set_precond<double>(op, pbox, kind));
    STCHK(cap_prepare(op, mask, pbox, op->hsc->mhash, &cap));
    STCHK(ensure_ws<T>(op, batch, false));
    if (cap) STCHK(cap_buffers<T>(op, batch));
  }
  Workspace& w = op->ws[tix<T>()];
  Prob pb = base_prob<T>(op, batch);
  pb.p0 = p0;
  pb.p1 = p1;
  STCHK(set_precond<T>(op, pb, kind));
  pb.in = r;
  pb.out = z;
  pb.T1 = w.T1;
  pb.mask = mask;
  pb.sc = w.sc;
  pb.part = w.part;
  pb.pstride = w.npart;
  if (cap) return cap_precond_seq<T, DPRO_PLAIN, DEPI_FINAL>(op, pb, Iter{0, 0}, 0);
  return precond_seq<T, DPRO_PLAIN, DEPI_FINAL>(op, pb, Iter{0, 0}, 0);
}


// Time `reps` back-to-back launches of one pass of the operator application or
// the preconditioner on the op's stream, bracketed by HIP events (inputs are the
// op's own zero-filled workspace).  pass: 0 rows forward, 1 symbol column pass
// (axis 0), 2 rows inverse, 3 first sine pass, 4 scaled sine column pass,
// 5 last sine pass, 6 whole application, 7 whole preconditioner.
template <typename T> static fl_status profile_t(fl_op op, int pass, int reps, double* avg_ms) {
  if (pass < 0 || pass > 7) return fail(FL_E_INVALID, "pass must be 0..7");
  STCHK(ensure_ws<T>(op, 1, true));
  Workspace& w = op->ws[tix<T>()];
  hipStream_t s = op->stream;
  const long N = op->N;
  for (void* v : {w.x, w.q, w.T1}) LAUNCH(k_fill<T>, dim3(nblocks_vec(N)), dim3(256), 0, s, (T*)v, (T)0, N);
  long nW1 = rows_of(op, 1) * op->H[op->d - 1] * 2;
  LAUNCH(k_fill<T>, dim3(nblocks_vec(nW1)), dim3(256), 0, s, (T*)w.W1, (T)0, nW1);
  if (op->d == 3) {
    long nW2 = (long)op->n[0] * op->P[1] * op->H[2] * 2;
    LAUNCH(k_fill<T>, dim3(nblocks_vec(nW2)), dim3(256), 0, s, (T*)w.W2, (T)0, nW2);
  }
  Prob pb = solver_prob<T>(op, nullptr, 0.0, 1.0, 0.0, 1.0);
  pb.in = w.x;
  pb.out = w.q;
  auto one = [&]() -> fl_status {
    if (pass == 6) return apply_seq<T, PRO_PLAIN, EPI_PLAIN>(op, pb, Iter{0, 0}, 0);
    if (pass == 7) return precond_seq<T, DPRO_PLAIN, DEPI_FINAL>(op, pb, Iter{0, 0}, 0);
    if (pass <= 2) return launch_apply_pass<T>(op, pb, pass);
    return launch_precond_pass<T>(op, pb, pass);
  };
  STCHK(one());  // warm-up
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  for (int i = 0; i < reps; ++i) STCHK(one());
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *avg_ms = (double)ms / std::max(reps, 1);
  return FL_OK;
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free application: the complex work arrays of one
// call (W1, then W2 in 3D at the next 256-byte boundary) live in this
// file-scope device array.  Each device holds its own copy until the process
// ends; every call on a device shares it (calls that overlap on one device
// race), and nothing in it needs to start at zero (every element a pass reads
// was written by the pass before it in the same call).
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static void* g_scratch_dev[64] = {};

// Device address of `scratch` on the current device (looked up once per
// device; the host-side name is not a device address).
static fl_status scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(FL_E_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(FL_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return FL_OK;
}

// Bytes of W1 (and W2) one application of `batch` inputs needs.
template <typename T> static size_t apply_scratch_bytes(fl_op op, long batch, size_t* w2_off) {
  if (op->d == 1) {
    *w2_off = 0;
    return 0;
  }
  const size_t w1 = (size_t)rows_of(op, batch) * op->H[op->d - 1] * sizeof(cx<T>);
  *w2_off = (w1 + 255) / 256 * 256;
  if (op->d < 3) return w1;
  return *w2_off + (size_t)batch * op->n[0] * op->P[1] * op->H[2] * sizeof(cx<T>);
}

template <typename T>
static fl_status apply_noalloc_t(fl_op op, const void* u, void* Mu, long batch, const uint8_t* mask, double s0,
                                 double s1) {
  size_t off = 0;
  const size_t need = apply_scratch_bytes<T>(op, batch, &off);
  if (need > kScratchBytes)
    return fail(FL_E_INVALID, "fl_apply_noalloc: this grid and batch need " + std::to_string(need) +
                                  " bytes of scratch; the maximum is " + std::to_string(kScratchBytes));
  void* base = nullptr;
  STCHK(scratch_address(&base));
  Prob pb = base_prob<T>(op, batch);
  pb.s0 = s0;
  pb.s1 = s1;
  pb.in = u;
  pb.out = Mu;
  pb.W1 = base;
  pb.W2 = op->d == 3 ? (void*)((unsigned char*)base + off) : nullptr;
  pb.mask = mask;
  return apply_seq<T, PRO_PLAIN, EPI_PLAIN>(op, pb, Iter{0, 0}, 0);
}

extern "C" {

fl_status fl_make_weights(int d, double alpha, double h, const int64_t* n, const fl_weights_opts* o,
                          void* hip_stream, fl_op* out) {
  g_err.clear();
  return make_op(d, alpha, h, n, o, hip_stream, out);
}

fl_status fl_op_constants(fl_op op, double out[8]) {
  if (!op || !out) return fail(FL_E_INVALID, "NULL argument");
  memcpy(out, op->cst, 8 * sizeof(double));
  return FL_OK;
}

fl_status fl_op_padded(fl_op op, int64_t* out) {
  if (!op || !out) return fail(FL_E_INVALID, "NULL argument");
  for (int a = 0; a < op->d; ++a) out[a] = op->P[a];
  return FL_OK;
}

fl_status fl_op_plan(fl_op op, int64_t* out) {
  if (!op || !out) return fail(FL_E_INVALID, "NULL argument");
  for (int i = 0; i < 16; ++i) out[i] = 0;
  for (int p = 0; p < 2; ++p) {
    for (int a = 0; a < op->d; ++a) {
      out[3 * p + a] = op->dst_form[p][a];
      out[6 + 3 * p + a] = op->ax[p][a].dst.L;
    }
    out[12 + p] = op->ax[p][0].col_tplf;
    out[14 + p] = op->ax[p][0].dcol_tplf;
  }
  return FL_OK;
}

fl_status fl_op_export(fl_op op, int which, void* dst) {
  if (!op || !dst) return fail(FL_E_INVALID, "NULL argument");
  if (which == 3 || which == 4) {
    STCHK(need_solver_grid(op));
    STCHK(build_tau(op));
    HIPCHK(hipMemcpyAsync(dst, op->tau[which - 3], op->N * (which == 4 ? sizeof(float) : sizeof(double)),
                          hipMemcpyDeviceToDevice, op->stream));
    return FL_OK;
  }
  const void* src = which == 0 ? (const void*)op->wf : which == 1 ? op->lam[0] : which == 2 ? op->lam[1] : nullptr;
  if (!src) return fail(FL_E_INVALID, "which must be 0..4");
  size_t b = op->NH * (which == 2 ? sizeof(float) : sizeof(double));
  HIPCHK(hipMemcpyAsync(dst, src, b, hipMemcpyDeviceToDevice, op->stream));
  return FL_OK;
}

fl_status fl_apply(fl_op op, const void* u, void* Mu, int dtype, int64_t batch, const uint8_t* mask, double shift0,
                   double shift1) {
  if (!op || !u || !Mu) return fail(FL_E_INVALID, "NULL argument");
  if (batch < 1) return fail(FL_E_INVALID, "batch must be >= 1");
  if (dtype == FL_F64) return apply_t<double>(op, u, Mu, batch, mask, shift0, shift1);
  if (dtype == FL_F32) return apply_t<float>(op, u, Mu, batch, mask, shift0, shift1);
  return fail(FL_E_INVALID, "dtype must be FL_F64 or FL_F32");
}

fl_status fl_apply_noalloc(fl_op op, const void* u, void* Mu, int dtype, int64_t batch, const uint8_t* mask,
                           double shift0, double shift1) {
  if (!op || !u || !Mu) return fail(FL_E_INVALID, "NULL argument");
  if (batch < 1) return fail(FL_E_INVALID, "batch must be >= 1");
  if (dtype == FL_F64) return apply_noalloc_t<double>(op, u, Mu, batch, mask, shift0, shift1);
  if (dtype == FL_F32) return apply_noalloc_t<float>(op, u, Mu, batch, mask, shift0, shift1);
  return fail(FL_E_INVALID, "dtype must be FL_F64 or FL_F32");
}

fl_status fl_precond(fl_op op, const void* r, void* z, int dtype, int64_t batch, const uint8_t* mask, double p0,
                     double p1) {
  if (!op || !r || !z) return fail(FL_E_INVALID, "NULL argument");
  if (batch < 1) return fail(FL_E_INVALID, "batch must be >= 1");
  STCHK(need_solver_grid(op));
  if (dtype == FL_F64) return precond_t<double>(op, r, z, batch, mask, p0, p1, FL_PC_FD);
  if (dtype == FL_F32) return precond_t<float>(op, r, z, batch, mask, p0, p1, FL_PC_FD);
  return fail(FL_E_INVALID, "dtype must be FL_F64 or FL_F32");
}

fl_status fl_precond_spectral(fl_op op, const void* r, void* z, int dtype, int64_t batch, const uint8_t* mask, double p0,
                     double p1) {
  if (!op || !r || !z) return fail(FL_E_INVALID, "NULL argument");
  if (batch < 1) return fail(FL_E_INVALID, "batch must be >= 1");
  STCHK(need_solver_grid(op));
  if (dtype == FL_F64) return precond_t<double>(op, r, z, batch, mask, p0, p1, FL_PC_SPECTRAL);
  if (dtype == FL_F32) return precond_t<float>(op, r, z, batch, mask, p0, p1, FL_PC_SPECTRAL);
  return fail(FL_E_INVALID, "dtype must be FL_F64 or FL_F32");
}

fl_status fl_precond_any(fl_op op, int kind, const void* r, void* z, int dtype, int64_t batch, const uint8_t* mask,
                          double p0, double p1) {
  if (!op || !r || !z) return fail(FL_E_INVALID, "NULL argument");
  if (batch < 1) return fail(FL_E_INVALID, "batch must be >= 1");
  STCHK(need_solver_grid(op));
  if (dtype == FL_F64) return precond_t<double>(op, r, z, batch, mask, p0, p1, kind);
  if (dtype == FL_F32) return precond_t<float>(op, r, z, batch, mask, p0, p1, kind);
  return fail(FL_E_INVALID, "dtype must be FL_F64 or FL_F32");
}

fl_status fl_solve(fl_op op, const double* f, const uint8_t* mask, double tol, const fl_solve_opts* o, double* u,
                   fl_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  if (!op || !f || !u || !info) return fail(FL_E_INVALID, "NULL argument");
  if (!(tol > 0.0)) return fail(FL_E_INVALID, "tol must be positive");
  STCHK(need_solver_grid(op));
  STCHK(ensure_ws<double>(op, 1, true));
  Workspace& w = op->ws[0];
  const long N = op->N;
  hipStream_t s = op->stream;
  HIPCHK(hipMemcpyAsync(w.f, f, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  int use_x0 = o ? o->use_x0 : 0;
  if (use_x0) HIPCHK(hipMemcpyAsync(w.x, u, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  STCHK(solve_system(op, mask, 0.0, 1.0, 0.0, 1.0, tol, o, use_x0, info));
  HIPCHK(hipMemcpyAsync(u, w.x, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info->status != FL_OK) return fail((fl_status)info->status, "solve did not reach the tolerance");
  return FL_OK;
}

fl_status fl_step(fl_op op, double* u, double dt, double theta, const double* f_k, const double* f_k1,
                  const uint8_t* mask, double tol, const fl_solve_opts* o, fl_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  if (!op || !u || !info) return fail(FL_E_INVALID, "NULL argument");
  if (!(dt > 0.0) || !(theta > 0.0 && theta <= 1.0) || !(tol > 0.0)) return fail(FL_E_INVALID, "dt, theta or tol");
  STCHK(need_solver_grid(op));
  if (o && o->pc == FL_PC_LEARNED) return fail(FL_E_UNSUPPORTED, "the learned preconditioner is trained for M, not steps");
  STCHK(ensure_ws<double>(op, 1, true));
  Workspace& w = op->ws[0];
  const long N = op->N;
  hipStream_t s = op->stream;
  // b = (I - (1-theta) dt M) u + dt (theta f_k1 + (1-theta) f_k)
  if (theta < 1.0) {
    STCHK(apply_t<double>(op, u, w.f, 1, mask, 1.0, -(1.0 - theta) * dt));
  } else {
    HIPCHK(hipMemcpyAsync(w.f, u, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  if (f_k1) LAUNCH((k_axpby<double, double>), dim3(nblocks_vec(N)), dim3(256), 0, s, f_k1, (double*)w.f, dt * theta, 1.0, N);
  if (f_k && theta < 1.0)
    LAUNCH((k_axpby<double, double>), dim3(nblocks_vec(N)), dim3(256), 0, s, f_k, (double*)w.f, dt * (1.0 - theta), 1.0, N);
  HIPCHK(hipMemcpyAsync(w.x, u, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  STCHK(solve_system(op, mask, 1.0, theta * dt, 1.0, theta * dt, tol, o, 1, info));
  HIPCHK(hipMemcpyAsync(u, w.x, N * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  info->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info->status != FL_OK) return fail((fl_status)info->status, "step solve did not reach the tolerance");
  return FL_OK;
}

fl_status fl_op_destroy(fl_op op) {
  if (!op) return FL_OK;
  batch_forget_op(op);
  hipStreamSynchronize(op->stream);
  delete op;
  return FL_OK;
}

fl_status fl_profile_pass(fl_op op, int dtype, int pass, int reps, double* avg_ms) {
  if (!op || !avg_ms || reps < 1) return fail(FL_E_INVALID, "NULL argument or reps < 1");
  if (pass >= 3) STCHK(need_solver_grid(op));
  if (dtype == FL_F64) return profile_t<double>(op, pass, reps, avg_ms);
  if (dtype == FL_F32) return profile_t<float>(op, pass, reps, avg_ms);
  return fail(FL_E_INVALID, "dtype");
}

const char* fl_last_error(void) { return g_err.c_str(); }

int64_t fl_device_allocations(void) { return (int64_t)g_dallocs.load(); }

}  // extern "C"
