// Runs the library's LDS line-FFT engine (fl_fft.hpp, unmodified) on the CPU:
// one std::thread per lane, __syncthreads as a std::barrier, LDS as a host
// vector.  Every specialised and generic path is compared with a direct DFT.
#include <complex>
#include <cstdio>
#include <thread>
#include <vector>

#include "../../paper_1802_03770_amd/csrc/fl_fft.hpp"
thread_local std::barrier<>* g_bar;
thread_local int g_lane;
double* g_shfl;
using namespace fl;

template <typename T, int L> double run(bool fixed_path, bool wide) {
  const int TPL = fixed_path ? c_fixed_tpl(L) : c_fixed_tpl(L);
  std::vector<cx<T>> tw(L);
  for (int m = 0; m < L; ++m) tw[m] = {(T)std::cos(2 * M_PI * m / L), (T)-std::sin(2 * M_PI * m / L)};
  std::vector<cx<T>> lds(Line<T>::stride(L)), lds2(Line<T>::stride(L));
  std::vector<std::complex<double>> x(L);
  for (int i = 0; i < L; ++i) x[i] = {std::sin(1.3 * i + 0.2), std::cos(0.7 * i)};
  Line<T> buf{lds.data()};
  for (int i = 0; i < L; ++i) buf[i] = {(T)x[i].real(), (T)x[i].imag()};
  FFTPlan pl{};
  pl.L = L;
  pl.nst = c_nst(L);
  pl.tpl = TPL;
  pl.fixed = fixed_path ? 1 : 0;
  pl.tw = tw.data();
  for (int s = 0; s < pl.nst; ++s) {
    int c = 0;
    while (radix_of_code(c) != c_radix(L, s)) ++c;
    pl.radcode |= (unsigned long long)c << (4 * s);
  }
  std::barrier<> bar(TPL);
  std::vector<std::thread> th;
  for (int lane = 0; lane < TPL; ++lane)
    th.emplace_back([&, lane] {
      g_bar = &bar;
      if (wide) {
        Line<T> b2{lds2.data()};
        Line<T> r = fft_line_wide<T, false>(buf, b2, pl, lane);
        g_bar->arrive_and_wait();
        if (lane == 0 && r.p != buf.p)
          for (int i = 0; i < L; ++i) buf[i] = r[i];
      } else {
        fft_line<T, false>(buf, pl, lane);
      }
    });
  for (auto& t : th) t.join();
  double err = 0, mx = 0;
  for (int k = 0; k < L; ++k) {
    std::complex<double> s = 0;
    for (int j = 0; j < L; ++j) s += x[j] * std::polar(1.0, -2 * M_PI * double((long)j * k % L) / L);
    cx<T> g = buf[k];
    err = std::max(err, std::abs(std::complex<double>(g.x, g.y) - s));
    mx = std::max(mx, std::abs(s));
  }
  return err / mx;
}

// Pruned specialised transforms: ZIN with the upper half of the line holding
// NaN (a read of it would show in every output), ZOUT compared on the lower
// half of the output only.
template <typename T, int L, bool ZIN, bool ZOUT> double run_pruned() {
  constexpr int TPL = c_fixed_tpl(L);
  std::vector<cx<T>> tw(L);
  for (int m = 0; m < L; ++m) tw[m] = {(T)std::cos(2 * M_PI * m / L), (T)-std::sin(2 * M_PI * m / L)};
  std::vector<cx<T>> lds(Line<T>::stride(L));
  std::vector<std::complex<double>> x(L);
  for (int i = 0; i < L; ++i) x[i] = (ZIN && i >= L / 2) ? 0.0 : std::complex<double>(std::sin(1.1 * i + 0.3), std::cos(0.9 * i));
  Line<T> buf{lds.data()};
  for (int i = 0; i < L; ++i)
    buf[i] = (ZIN && i >= L / 2) ? cx<T>{(T)NAN, (T)NAN} : cx<T>{(T)x[i].real(), (T)x[i].imag()};
  std::barrier<> bar(TPL);
  std::vector<std::thread> th;
  for (int lane = 0; lane < TPL; ++lane)
    th.emplace_back([&, lane] {
      g_bar = &bar;
      fft_fixed<T, L, false, ZIN, ZOUT>(buf, buf, tw.data(), lane);
    });
  for (auto& t : th) t.join();
  double err = 0, mx = 0;
  for (int k = 0; k < (ZOUT ? L / 2 : L); ++k) {
    std::complex<double> s = 0;
    for (int j = 0; j < L; ++j) s += x[j] * std::polar(1.0, -2 * M_PI * double((long)j * k % L) / L);
    cx<T> g = buf[k];
    const double e = std::abs(std::complex<double>(g.x, g.y) - s);
    err = std::isnan(e) ? INFINITY : std::max(err, e);
    mx = std::max(mx, std::abs(s));
  }
  return err / mx;
}

// Prime-form sine transform (n = 256, N = 257) of a packed pair, against the
// sine sums taken directly; the harness builds its own Rader tables.
template <typename T> double run_rader() {
  constexpr int RL = 256, N = RL + 1, HALF = RL / 2, n = N - 1, TPL = c_fixed_tpl(RL);
  const int g = 3;  // a generator of the units mod 257 (3^128 = -1)
  std::vector<int> pw(RL), tab(2 * HALF + 1, 0);
  pw[0] = 1;
  for (int m = 1; m < RL; ++m) pw[m] = pw[m - 1] * g % N;
  for (int p = 0; p < HALF; ++p) tab[p] = pw[(RL - p) % RL];
  for (int q = 0; q < RL; ++q)
    if (pw[q] <= HALF) tab[HALF + pw[q]] = q;
  std::vector<T> sp(HALF);
  for (int p = 0; p < HALF; ++p) sp[p] = (T)std::sin(M_PI * tab[p] / N);
  std::vector<cx<T>> bh(RL), tw(RL);
  for (int m = 0; m < RL; ++m) tw[m] = {(T)std::cos(2 * M_PI * m / RL), (T)-std::sin(2 * M_PI * m / RL)};
  for (int k = 0; k < RL; ++k) {
    std::complex<double> s = 0;
    for (int m = 0; m < RL; ++m)
      s += std::polar(1.0, -2 * M_PI * (double)pw[m] / N) * std::polar(1.0, -2 * M_PI * double((long)m * k % RL) / RL);
    s /= RL;
    bh[k] = {(T)s.real(), (T)s.imag()};
  }
  std::vector<double> xa(n + 1), xb(n + 1);
  for (int j = 1; j <= n; ++j) {
    xa[j] = std::sin(0.37 * j * j + 0.1) + 0.2;
    xb[j] = std::cos(1.7 * j) * (j % 7 - 3);
  }
  std::vector<cx<T>> lds(Line<T>::stride(RL)), lds2(Line<T>::stride(RL));
  Line<T> buf{lds.data()}, buf2{lds2.data()};
  for (int j = 1; j <= n; ++j) buf[j] = {(T)xa[j], (T)xb[j]};
  std::vector<double> shfl(TPL);
  g_shfl = shfl.data();
  std::barrier<> bar(TPL);
  std::vector<std::thread> th;
  for (int lane = 0; lane < TPL; ++lane)
    th.emplace_back([&, lane] {
      g_bar = &bar;
      g_lane = lane;
      RaderRegs<T, RL> rr;
      rader_load(rr, tab.data(), sp.data(), bh.data(), lane);
      rader_sine<T, RL>(buf, buf2, n, rr, tw.data(), lane);
    });
  for (auto& t : th) t.join();
  double err = 0, mx = 0;
  for (int k = 1; k <= n; ++k) {
    double sa = 0, sb = 0;
    for (int j = 1; j <= n; ++j) {
      const double sn = std::sin(M_PI * double((long)j * k % (2 * N)) / N);
      sa += xa[j] * sn;
      sb += xb[j] * sn;
    }
    cx<T> v = buf[k];
    err = std::max(err, std::max(std::abs(v.x - sa), std::abs(v.y - sb)));
    mx = std::max(mx, std::max(std::abs(sa), std::abs(sb)));
  }
  return err / mx;
}

int main() {
  struct R { const char* name; double err, tol; };
  std::vector<R> rs = {
      {"fixed 128", run<double, 128>(true, false), 1e-13},   {"fixed 256", run<double, 256>(true, false), 1e-13},
      {"fixed 512", run<double, 512>(true, false), 1e-13},   {"fixed 768", run<double, 768>(true, false), 1e-13},
      {"fixed 1024", run<double, 1024>(true, false), 1e-13}, {"fixed 2048", run<double, 2048>(true, false), 1e-13},
      {"generic 2048", run<double, 2048>(false, false), 1e-13}, {"generic 80", run<double, 80>(false, false), 1e-13},
      {"generic 96", run<double, 96>(false, false), 1e-13},  {"f32 fixed 2048", run<float, 2048>(true, false), 1e-6},
      {"wide fixed 130", run<double, 130>(true, true), 1e-13}, {"wide fixed 258", run<double, 258>(true, true), 1e-13},
      {"wide fixed 770", run<double, 770>(true, true), 1e-13}, {"wide fixed 1026", run<double, 1026>(true, true), 1e-13},
      {"wide fixed 2050", run<double, 2050>(true, true), 1e-13}, {"wide generic 76", run<double, 76>(false, true), 1e-13},
      {"f32 wide fixed 2050", run<float, 2050>(true, true), 2e-6},
      {"wide generic 82", run<double, 82>(false, true), 1e-13}, {"wide generic 98", run<double, 98>(false, true), 1e-13},
      {"prime sine 257", run_rader<double>(), 1e-13}, {"f32 prime sine 257", run_rader<float>(), 2e-6},
      {"zin 512", run_pruned<double, 512, true, false>(), 1e-13},
      {"zout 512", run_pruned<double, 512, false, true>(), 1e-13},
      {"zin zout 2048", run_pruned<double, 2048, true, true>(), 1e-13},
      {"zin zout 256", run_pruned<double, 256, true, true>(), 1e-13},
      {"zin 768", run_pruned<double, 768, true, true>(), 1e-13},
      {"f32 zin zout 512", run_pruned<float, 512, true, true>(), 1e-6},
      {"zin zout 8", run_pruned<double, 8, true, true>(), 1e-13},
  };
  int bad = 0;
  for (auto& r : rs) {
    printf("%-18s %.2e %s\n", r.name, r.err, r.err <= r.tol ? "ok" : "FAIL");
    bad += r.err > r.tol;
  }
  return bad;
}
