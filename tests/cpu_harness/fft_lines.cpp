// Runs the library's LDS line-FFT engine (fl_fft.hpp, unmodified) on the CPU:
// one std::thread per lane, __syncthreads as a std::barrier, LDS as a host
// vector.  Every specialised and generic path is compared with a direct DFT.
#include <complex>
#include <cstdio>
#include <thread>
#include <vector>

#include "../../paper_1802_03770_amd/csrc/fl_fft.hpp"
thread_local std::barrier<>* g_bar;
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
  };
  int bad = 0;
  for (auto& r : rs) {
    printf("%-18s %.2e %s\n", r.name, r.err, r.err <= r.tol ? "ok" : "FAIL");
    bad += r.err > r.tol;
  }
  return bad;
}
