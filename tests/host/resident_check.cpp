// Host emulation of the LDS-resident 2D transform used by the resident chain
// kernels: a padded N x P tile, every row transformed in place with the
// padded row exchange (slot pitch L + 1, stride 1), then every column with
// the plain exchange (slot pitch L, stride P), lane by lane. Compared with a
// direct 2D DFT in double; also checks that the padding columns are the only
// storage besides the tile that the row exchange touches.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <vector>

#include "pty_fft.hpp"

using cd = std::complex<double>;

template <int N, bool INV>
double check(unsigned seed) {
  constexpr int L = pty::Cfg<N>::L, E = pty::Cfg<N>::E, P = pty::Res<N>::P;
  std::mt19937 rng(seed);
  std::normal_distribution<float> nd;
  std::vector<float2> x((size_t)N * N), tile((size_t)N * P), tw(N);
  for (auto& z : x) z = make_float2(nd(rng), nd(rng));
  for (int k = 0; k < N; ++k) {
    double a = 2.0 * M_PI * k / N;
    tw[k] = make_float2((float)std::cos(a), (float)-std::sin(a));
  }
  for (int y = 0; y < N; ++y)
    for (int c = 0; c < N; ++c) tile[(size_t)y * P + c] = x[(size_t)y * N + c];
  std::vector<std::array<float2, E>> regs(L);
  // rows
  for (int y = 0; y < N; ++y) {
    float2* base = tile.data() + (size_t)y * P;
    for (int l = 0; l < L; ++l)
      for (int a = 0; a < E; ++a) regs[l][a] = base[l + L * a];
    for (int l = 0; l < L; ++l)
      pty::res_stage1<N, INV, L + 1, 1>(*reinterpret_cast<float2(*)[E]>(regs[l].data()), l, tw.data(), base);
    for (int l = 0; l < L; ++l)
      pty::res_stage2<N, INV, L + 1, 1>(*reinterpret_cast<float2(*)[E]>(regs[l].data()), l, base);
    for (int l = 0; l < L; ++l)
      for (int a = 0; a < E; ++a) base[l + L * a] = regs[l][a];
  }
  // columns
  for (int c = 0; c < N; ++c) {
    float2* base = tile.data() + c;
    for (int l = 0; l < L; ++l)
      for (int a = 0; a < E; ++a) regs[l][a] = base[(size_t)(l + L * a) * P];
    for (int l = 0; l < L; ++l)
      pty::res_stage1<N, INV, L, P>(*reinterpret_cast<float2(*)[E]>(regs[l].data()), l, tw.data(), base);
    for (int l = 0; l < L; ++l)
      pty::res_stage2<N, INV, L, P>(*reinterpret_cast<float2(*)[E]>(regs[l].data()), l, base);
    for (int l = 0; l < L; ++l)
      for (int a = 0; a < E; ++a) base[(size_t)(l + L * a) * P] = regs[l][a];
  }
  // direct 2D DFT (separable, double)
  const double sgn = INV ? 2.0 : -2.0;
  std::vector<cd> rowt((size_t)N * N), ref((size_t)N * N);
  for (int y = 0; y < N; ++y)
    for (int k = 0; k < N; ++k) {
      cd acc = 0;
      for (int n = 0; n < N; ++n)
        acc += cd(x[(size_t)y * N + n].x, x[(size_t)y * N + n].y) * std::polar(1.0, sgn * M_PI * ((long)n * k % N) / N);
      rowt[(size_t)y * N + k] = acc;
    }
  double err = 0, mx = 0;
  for (int k = 0; k < N; ++k)
    for (int c = 0; c < N; ++c) {
      cd acc = 0;
      for (int n = 0; n < N; ++n) acc += rowt[(size_t)n * N + c] * std::polar(1.0, sgn * M_PI * ((long)n * k % N) / N);
      float2 g = tile[(size_t)k * P + c];
      err = std::max(err, std::abs(acc - cd(g.x, g.y)));
      mx = std::max(mx, std::abs(acc));
    }
  return err / mx;
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
  return worst < 1e-5 ? 0 : 1;
}
