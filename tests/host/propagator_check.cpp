// Host check of the propagator construction (pty_prop.hpp), built with g++
// under AddressSanitizer and UndefinedBehaviorSanitizer:
//  * the N x N table equals the Fresnel propagator written out here
//    independently in double: exp(-i pi lambda dz |q|^2) times the tilt ramp
//    exp(2 pi i dz (q_y tan t_y + q_x tan t_x)), over N^2, inside the band
//    limit; the default 2/3-Nyquist limit is the exact integer test
//    9 (k_y^2 + k_x^2) <= N^2;
//  * wherever the factorised form is accepted, [|k_x| <= K_y] Hy Hx
//    reproduces the table to float rounding, zeros included;
//  * masks whose rows are not centred intervals are refused, and the
//    live-column interval is found, or refused, accordingly.
// Exits non-zero on the first failed check.
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "pty_prop.hpp"

using cd = std::complex<double>;
using pty_host::F2;
using pty_host::F4;

static int fails = 0;
#define CHECK(cond, ...)                       \
  do {                                         \
    if (!(cond)) {                             \
      std::printf("FAIL: " __VA_ARGS__);       \
      std::printf("\n");                       \
      ++fails;                                 \
    }                                          \
  } while (0)

static int sbin(int u, int N) { return 2 * u < N ? u : u - N; }

struct Case {
  const char* name;
  int N;
  double dx, lam, dz, frac, ty, tx;
  int mask_kind;   // 0 none, 1 square |k| <= 40, 2 off-centre rows, 3 ring (hole in the middle)
  bool separable;
};

static std::vector<uint8_t> make_mask(int N, int kind) {
  std::vector<uint8_t> m;
  if (kind == 0) return m;
  m.assign((size_t)N * N, 0);
  for (int y = 0; y < N; ++y)
    for (int x = 0; x < N; ++x) {
      const int ky = sbin(y, N), kx = sbin(x, N);
      bool keep = false;
      if (kind == 1) keep = std::abs(ky) <= 40 && std::abs(kx) <= 40;
      if (kind == 2) keep = kx >= -10 && kx <= 20 && std::abs(ky) <= 18;
      if (kind == 3) keep = (ky * ky + kx * kx <= 400) && (ky * ky + kx * kx >= 25);
      m[(size_t)y * N + x] = keep ? 1 : 0;
    }
  return m;
}

int main() {
  const double pi = 3.141592653589793238462643383279502884;
  const Case cases[] = {
      {"N64 circle", 64, 0.2, 0.019688, 2.0, 2.0 / 3.0, 0.0, 0.0, 0, true},
      {"N128 circle tilt", 128, 0.2, 0.019688, 3.5, 2.0 / 3.0, 0.003, -0.005, 0, true},
      {"N192 no limit", 192, 0.2, 0.019688, 2.0, 0.0, 0.0, 0.002, 0, true},
      {"N256 circle", 256, 0.2, 0.019688, 1.0, 2.0 / 3.0, 0.0, 0.0, 0, true},
      {"N128 square mask", 128, 0.2, 0.019688, 2.0, 2.0 / 3.0, 0.001, 0.0, 1, true},
      {"N64 off-centre mask", 64, 0.2, 0.019688, 2.0, 2.0 / 3.0, 0.0, 0.0, 2, false},
      {"N64 ring mask", 64, 0.2, 0.019688, 2.0, 2.0 / 3.0, 0.0, 0.0, 3, false},
  };
  for (const Case& c : cases) {
    const int N = c.N;
    const std::vector<uint8_t> mask = make_mask(N, c.mask_kind);
    const std::vector<F2> H = pty_host::propagator(N, c.dx, c.lam, c.dz, c.frac, c.ty, c.tx, mask);
    CHECK(H.size() == (size_t)N * N, "%s: table size", c.name);
    // the table against the definition
    double worst = 0.0;
    std::vector<uint8_t> live(N, 0);
    for (int y = 0; y < N; ++y)
      for (int x = 0; x < N; ++x) {
        const int ky = sbin(y, N), kx = sbin(x, N);
        bool keep;
        if (c.mask_kind) keep = mask[(size_t)y * N + x] != 0;
        else if (c.frac <= 0.0) keep = true;
        else keep = 9 * (ky * ky + kx * kx) <= N * N;   // 2/3 of Nyquist: radius N / 3
        const double qy = ky / (N * c.dx), qx = kx / (N * c.dx);
        const cd fres = std::exp(cd(0.0, -pi * c.lam * c.dz * (qy * qy + qx * qx)));
        const cd ramp = std::exp(cd(0.0, 2.0 * pi * c.dz * (qy * std::tan(c.ty) + qx * std::tan(c.tx))));
        const cd want = keep ? fres * ramp / double(N * N) : cd(0.0);
        const F2 got = H[(size_t)y * N + x];
        CHECK((got.x != 0.f || got.y != 0.f) == keep, "%s: band limit at (%d, %d)", c.name, ky, kx);
        worst = std::max(worst, std::abs(cd(got.x, got.y) - want) * N * N);
        if (keep) live[x] = 1;
      }
    CHECK(worst < 1e-6, "%s: table differs from the definition by %.3g (x N^2)", c.name, worst);
    // the factorised form
    std::vector<F4> py;
    std::vector<F2> px;
    const bool sep = pty_host::separable_propagator(N, c.dx, c.lam, c.dz, c.frac, c.ty, c.tx, mask, py, px);
    CHECK(sep == c.separable, "%s: separable %d, expected %d", c.name, (int)sep, (int)c.separable);
    double worst_sep = 0.0;
    if (sep) {
      CHECK(py.size() == (size_t)N && px.size() == (size_t)N, "%s: factor sizes", c.name);
      for (int y = 0; y < N; ++y) {
        int K;
        std::memcpy(&K, &py[y].z, sizeof K);
        for (int x = 0; x < N; ++x) {
          const bool keep = std::abs(sbin(x, N)) <= K;
          const cd h = keep ? cd(py[y].x, py[y].y) * cd(px[x].x, px[x].y) : cd(0.0);
          const F2 t = H[(size_t)y * N + x];
          CHECK(keep == (t.x != 0.f || t.y != 0.f), "%s: factor mask at (%d, %d)", c.name, y, x);
          worst_sep = std::max(worst_sep, std::abs(h - cd(t.x, t.y)) * N * N);
        }
      }
      CHECK(worst_sep < 1e-6, "%s: factors differ from the table by %.3g (x N^2)", c.name, worst_sep);
    }
    // the live-column interval
    const int K = pty_host::live_interval(live, N);
    if (c.mask_kind == 0 && c.frac > 0.0) CHECK(K == N / 3, "%s: live interval %d, expected %d", c.name, K, N / 3);
    if (c.mask_kind == 0 && c.frac <= 0.0) CHECK(K == N / 2, "%s: live interval %d, expected %d", c.name, K, N / 2);
    if (c.mask_kind == 1) CHECK(K == 40, "%s: live interval %d, expected 40", c.name, K);
    if (c.mask_kind == 2) CHECK(K == -1, "%s: an off-centre band must be refused (got %d)", c.name, K);
    std::printf("%-22s table err %.2e  factor err %.2e  separable %d  live K %d\n", c.name, worst, worst_sep,
                (int)sep, K);
  }
  if (fails) std::printf("%d check(s) failed\n", fails);
  return fails ? 1 : 0;
}
