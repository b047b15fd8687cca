// pty_prop.hpp -- host-side construction of the Fresnel propagators (Sec. 3:
// the slice-to-slice propagator with its band limit, Sec. 1: beam tilt) and
// of the live-column bookkeeping derived from them. Plain C++ (no HIP types),
// so the host checks can build it with any compiler and sanitizer.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace pty_host {

struct F2 { float x, y; };
struct F4 { float x, y, z, w; };

constexpr double kPi = 3.141592653589793238462643383279502884;

// Signed frequency bin of FFT-order index u (the Nyquist bin of even N is -N/2).
inline int signed_bin(int u, int N) { return u < (N + 1) / 2 ? u : u - N; }

// Band limit B(u): the circle of radius frac * N / 2 on signed integer bins,
// everything (frac <= 0), or the caller's mask [N][N] (nonzero = keep).
inline bool keep_bin(int N, double frac, const std::vector<uint8_t>& mask, int y, int x) {
  if (!mask.empty()) return mask[(size_t)y * N + x] != 0;
  if (frac <= 0.0) return true;
  const double r = frac * N / 2.0;
  const int ky = signed_bin(y, N), kx = signed_bin(x, N);
  return (double)(ky * ky + kx * kx) <= r * r * (1.0 + 1e-9);
}

// Phase of H along one axis: -pi lambda dz q^2 + 2 pi dz q tan(t), q = k / (N dx).
inline double axis_phase(int k, int N, double dx, double lam, double dz, double tan_t) {
  const double q = (double)k / N / dx;
  return -kPi * lam * dz * q * q + 2.0 * kPi * dz * q * tan_t;
}

// Propagator for one gap as an N x N table, divided by N^2 (the normalisation
// of the unnormalised forward and inverse 2D DFTs around it):
// H(u) = B(u) exp(-i pi lambda dz |q|^2 + 2 pi i dz (q_y tan t_y + q_x tan t_x)),
// the phase evaluated in double and rounded once.
inline std::vector<F2> propagator(int N, double dx, double lam, double dz, double frac, double tilt_y,
                                  double tilt_x, const std::vector<uint8_t>& mask) {
  std::vector<F2> H((size_t)N * N);
  const double inv_n2 = 1.0 / ((double)N * (double)N);
  const double ty = std::tan(tilt_y), tx = std::tan(tilt_x);
  for (int y = 0; y < N; ++y) {
    const double phy = axis_phase(signed_bin(y, N), N, dx, lam, dz, ty);
    for (int x = 0; x < N; ++x) {
      const double ph = phy + axis_phase(signed_bin(x, N), N, dx, lam, dz, tx);
      H[(size_t)y * N + x] = keep_bin(N, frac, mask, y, x)
                                 ? F2{(float)(std::cos(ph) * inv_n2), (float)(std::sin(ph) * inv_n2)}
                                 : F2{0.f, 0.f};
    }
  }
  return H;
}

// The phase of H is a sum of a k_y and a k_x term, so H = B(u) Hy(k_y) Hx(k_x).
// When every row y of the band limit keeps exactly the bins |k_x| <= K_y (a
// circle, no limit, or a mask of that shape), the column passes rebuild H
// from the two factors and K_y instead of reading the N x N table:
// py[y] = (Hy / N^2, K_y as int bits, 0) with K_y = -1 for an empty row,
// px[x] = Hx. Returns false when the band limit is not of that form.
inline bool separable_propagator(int N, double dx, double lam, double dz, double frac, double tilt_y,
                                 double tilt_x, const std::vector<uint8_t>& mask, std::vector<F4>& py,
                                 std::vector<F2>& px) {
  py.assign(N, F4{0.f, 0.f, 0.f, 0.f});
  px.assign(N, F2{0.f, 0.f});
  const double inv_n2 = 1.0 / ((double)N * (double)N);
  const double ty = std::tan(tilt_y), tx = std::tan(tilt_x);
  for (int y = 0; y < N; ++y) {
    int K = -1;
    for (int x = 0; x < N; ++x)
      if (keep_bin(N, frac, mask, y, x)) K = std::max(K, std::abs(signed_bin(x, N)));
    for (int x = 0; x < N; ++x)
      if (keep_bin(N, frac, mask, y, x) != (std::abs(signed_bin(x, N)) <= K)) return false;
    const double ph = axis_phase(signed_bin(y, N), N, dx, lam, dz, ty);
    float kb;
    std::memcpy(&kb, &K, sizeof kb);
    py[y] = F4{(float)(std::cos(ph) * inv_n2), (float)(std::sin(ph) * inv_n2), kb, 0.f};
  }
  for (int x = 0; x < N; ++x) {
    const double ph = axis_phase(signed_bin(x, N), N, dx, lam, dz, tx);
    px[x] = F2{(float)std::cos(ph), (float)std::sin(ph)};
  }
  return true;
}

// Live columns (some propagator nonzero) as a symmetric band |k_x| <= K:
// returns K, or -1 when the live set is not of that form.
inline int live_interval(const std::vector<uint8_t>& live, int N) {
  int K = -1;
  for (int x = 0; x < N; ++x)
    if (live[x]) K = std::max(K, std::abs(signed_bin(x, N)));
  for (int x = 0; x < N; ++x)
    if ((live[x] != 0) != (std::abs(signed_bin(x, N)) <= K)) return -1;
  return K;
}

}  // namespace pty_host
