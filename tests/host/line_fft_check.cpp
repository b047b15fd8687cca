// Host emulation of the cross-lane line FFT of pty_fft.hpp: every lane of a
// line runs stage 1 (in-register DFT, twiddle, exchange write), then every
// lane runs stage 2 (exchange read, second DFT). The result is compared with
// a direct O(N^2) DFT in double precision. Prints the max relative error per
// size and direction; exits non-zero if any exceeds 1e-5.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <vector>

#include "pty_fft.hpp"

using cd = std::complex<double>;

template <int N, bool INV>
double check(unsigned seed) {
  constexpr int L = pty::Cfg<N>::L, E = pty::Cfg<N>::E;
  std::mt19937 rng(seed);
  std::normal_distribution<float> nd;
  std::vector<float2> x(N), tw(N), xch(pty::Xch<N>::SIZE);
  for (int k = 0; k < N; ++k) {
    x[k] = make_float2(nd(rng), nd(rng));
    double a = 2.0 * M_PI * k / N;
    tw[k] = make_float2((float)std::cos(a), (float)-std::sin(a));
  }
  std::vector<std::array<float2, E>> regs(L);
  for (int l = 0; l < L; ++l)
    for (int a = 0; a < E; ++a) regs[l][a] = x[l + L * a];
  for (int l = 0; l < L; ++l) {
    float2(&v)[E] = *reinterpret_cast<float2(*)[E]>(regs[l].data());
    pty::line_fft_stage1<N, INV>(v, l, tw.data(), xch.data());
  }
  for (int l = 0; l < L; ++l) {
    float2(&v)[E] = *reinterpret_cast<float2(*)[E]>(regs[l].data());
    pty::line_fft_stage2<N, INV>(v, l, xch.data());
  }
  double err = 0, ref_max = 0;
  for (int k = 0; k < N; ++k) {
    cd acc = 0;
    for (int n = 0; n < N; ++n)
      acc += cd(x[n].x, x[n].y) * std::polar(1.0, (INV ? 2.0 : -2.0) * M_PI * (double)((long)n * k % N) / N);
    float2 got = regs[k % L][k / L];
    err = std::max(err, std::abs(acc - cd(got.x, got.y)));
    ref_max = std::max(ref_max, std::abs(acc));
  }
  return err / ref_max;
}

int main() {
  double worst = 0;
  auto run = [&](const char* name, double e) {
    std::printf("%s %.3e\n", name, e);
    worst = std::max(worst, e);
  };
  run("N64_fwd", check<64, false>(1));
  run("N64_inv", check<64, true>(2));
  run("N128_fwd", check<128, false>(3));
  run("N128_inv", check<128, true>(4));
  run("N192_fwd", check<192, false>(5));
  run("N192_inv", check<192, true>(6));
  run("N256_fwd", check<256, false>(7));
  run("N256_inv", check<256, true>(8));
  return worst < 1e-5 ? 0 : 1;
}
