// pty_fft.hpp -- register/LDS building blocks of the batched 2D FFTs (gfx950).
//
// A line (one row or one column of an N x N tile) is held by L lanes with
// E = N / L complex values each, lane l holding x[l + L a] in register a.
// One line transform is the two-level Cooley-Tukey split N = E * L:
//   X[k1 + E k2] = sum_l w_N^{l k1} w_L^{l k2} sum_a x[l + L a] w_E^{a k1},
// i.e. an E-point DFT in each lane's registers, a twiddle by w_N^{l k1}, one
// transpose through LDS, and E / L L-point DFTs in registers. The output
// X[l + L a'] ends up in register a' = c + (E/L) k2 of lane l, which is the
// input layout again, so inverse -> pointwise -> forward chains need no
// extra data movement. Transforms are unnormalised; callers fold the 1/N
// factors of the unitary DFT into their pointwise multipliers.
//
// In-register DFT twiddles are compile-time constants: cos/sin of 2 pi k / n
// evaluated in double by an octant-reduced Taylor series at compile time and
// rounded once to float.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace pty {

// ---------------------------------------------------------------- complex

__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__host__ __device__ __forceinline__ float2 cjmul(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__host__ __device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__host__ __device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }

// ---------------------------------------------------------------- compile-time roots

constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double x) {
  double x2 = x * x, t = x, s = x;
  for (int k = 1; k < 14; ++k) { t *= -x2 / ((2.0 * k) * (2.0 * k + 1.0)); s += t; }
  return s;
}
constexpr double taylor_cos(double x) {
  double x2 = x * x, t = 1.0, s = 1.0;
  for (int k = 1; k < 14; ++k) { t *= -x2 / ((2.0 * k - 1.0) * (2.0 * k)); s += t; }
  return s;
}

struct CosSin { double c, s; };

// cos and sin of 2 pi k / n, reduced exactly to an angle in [0, pi/4].
constexpr CosSin unit_root(long k, long n) {
  k %= n;
  if (k < 0) k += n;
  long a = 2 * k, d = n;            // angle = pi a / d, a in [0, 2d)
  double ss = 1.0, cs = 1.0;
  if (a > d) { a = 2 * d - a; ss = -1.0; }      // 2 pi - angle
  if (2 * a > d) { a = d - a; cs = -1.0; }      // pi - angle
  bool swap = false;
  if (4 * a > d) { a = d - 2 * a; d = 2 * d; swap = true; }  // pi/2 - angle
  double x = kPi * (double)a / (double)d;
  double s = taylor_sin(x), c = taylor_cos(x);
  if (swap) { double t = s; s = c; c = t; }
  return CosSin{cs * c, ss * s};
}

template <int B, int E, typename F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// x * w_n^k with w_n = exp(-2 pi i / n) (forward) or its conjugate (inverse).
template <long k, long n, bool INV>
__host__ __device__ __forceinline__ float2 twiddle_const(float2 x) {
  constexpr long r = ((k % n) + n) % n;
  if constexpr (r == 0) {
    return x;
  } else if constexpr ((4 * r) % n == 0) {
    constexpr long q = (4 * r) / n;     // quarter turns
    if constexpr (q == 2) return make_float2(-x.x, -x.y);
    // forward: w^(n/4) = -i ; inverse: +i
    if constexpr ((q == 1) != INV) return make_float2(x.y, -x.x);   // -i x
    else return make_float2(-x.y, x.x);                              // +i x
  } else {
    constexpr CosSin cs = unit_root(r, n);
    constexpr float c = (float)cs.c;
    constexpr float s = INV ? (float)cs.s : (float)(-cs.s);
    return make_float2(x.x * c - x.y * s, x.x * s + x.y * c);
  }
}

// ---------------------------------------------------------------- register DFTs

template <int n>
constexpr int first_radix() { return n % 4 == 0 ? 4 : (n % 2 == 0 ? 2 : (n % 3 == 0 ? 3 : n)); }

template <int n, bool INV>
struct Dft;

template <bool INV>
struct Dft<1, INV> { __host__ __device__ __forceinline__ static void run(float2*) {} };

template <bool INV>
struct Dft<2, INV> {
  __host__ __device__ __forceinline__ static void run(float2* x) {
    float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<3, INV> {
  __host__ __device__ __forceinline__ static void run(float2* x) {
    constexpr float h = (float)unit_root(1, 3).s;   // sin(2 pi / 3)
    float2 t1 = cadd(x[1], x[2]);
    float2 t2 = make_float2(x[0].x - 0.5f * t1.x, x[0].y - 0.5f * t1.y);
    float2 t3 = csub(x[1], x[2]);
    float2 iht3 = make_float2(-h * t3.y, h * t3.x);   // i h (x1 - x2)
    x[0] = cadd(x[0], t1);
    if constexpr (!INV) { x[1] = csub(t2, iht3); x[2] = cadd(t2, iht3); }
    else                { x[1] = cadd(t2, iht3); x[2] = csub(t2, iht3); }
  }
};

template <bool INV>
struct Dft<4, INV> {
  __host__ __device__ __forceinline__ static void run(float2* x) {
    float2 a0 = cadd(x[0], x[2]), a1 = csub(x[0], x[2]);
    float2 b0 = cadd(x[1], x[3]), b1 = csub(x[1], x[3]);
    float2 ib1 = make_float2(-b1.y, b1.x);   // i b1
    x[0] = cadd(a0, b0);
    x[2] = csub(a0, b0);
    if constexpr (!INV) { x[1] = csub(a1, ib1); x[3] = cadd(a1, ib1); }
    else                { x[1] = cadd(a1, ib1); x[3] = csub(a1, ib1); }
  }
};

// n = A * B:  X[k1 + A k2] = sum_b w_B^{b k2} w_n^{b k1} sum_a x[b + B a] w_A^{a k1}
template <int n, bool INV>
struct Dft {
  static constexpr int A = first_radix<n>();
  static constexpr int B = n / A;
  static_assert(A * B == n && A > 1 && A <= 4, "unsupported DFT size");
  __host__ __device__ __forceinline__ static void run(float2* x) {
    float2 y[n];
    static_for<0, B>([&](auto bI) {
      constexpr int b = decltype(bI)::value;
      float2 t[A];
      static_for<0, A>([&](auto aI) { constexpr int a = decltype(aI)::value; t[a] = x[b + B * a]; });
      Dft<A, INV>::run(t);
      static_for<0, A>([&](auto kI) {
        constexpr int k1 = decltype(kI)::value;
        y[b * A + k1] = twiddle_const<(long)b * k1, n, INV>(t[k1]);
      });
    });
    static_for<0, A>([&](auto kI) {
      constexpr int k1 = decltype(kI)::value;
      float2 t[B];
      static_for<0, B>([&](auto bI) { constexpr int b = decltype(bI)::value; t[b] = y[b * A + k1]; });
      Dft<B, INV>::run(t);
      static_for<0, B>([&](auto k2I) { constexpr int k2 = decltype(k2I)::value; x[k1 + A * k2] = t[k2]; });
    });
  }
};

// ---------------------------------------------------------------- line layout per N

template <int N> struct Cfg;
template <> struct Cfg<64>  { static constexpr int L = 8,  E = 8;  };
template <> struct Cfg<128> { static constexpr int L = 8,  E = 16; };
template <> struct Cfg<192> { static constexpr int L = 8,  E = 24; };
template <> struct Cfg<256> { static constexpr int L = 16, E = 16; };

constexpr int pad_to(int x, int mod, int rem) { return x + ((rem - x % mod) % mod + mod) % mod; }

// Exchange scratch of one line: Z[l][k1] at xch[k1 * XP + l], XP = L + 1.
// Lines of one workgroup are ROW_STRIDE (row passes: the lines of a wave
// are consecutive) or COL_STRIDE (column passes: consecutive lanes belong
// to consecutive columns) float2 apart. Both strides are padded so that the
// 64 lanes of a wave spread over all 64 four-byte LDS banks: a float2
// access then takes the minimum of two bank cycles per wave.
template <int N> struct Xch {
  static constexpr int L = Cfg<N>::L, E = Cfg<N>::E;
  static constexpr int XP = L + 1;
  static constexpr int SIZE = E * XP;
  static constexpr int ROW_STRIDE = (L == 16) ? pad_to(SIZE, 32, 16) : pad_to(SIZE, 32, 8);
  static constexpr int COL_STRIDE = (L == 16) ? pad_to(SIZE, 32, 4) : pad_to(SIZE, 2, 1);
};

// Line FFT of v (layout above), in two stages around the LDS exchange.
// tw: table tw[k] = w_N^k (forward roots), k in [0, N). xch: this line's
// exchange scratch (Xch<N>::SIZE float2). Stage 1: E-point DFT in registers,
// twiddle, write Z[l][k1]. Stage 2: read Z[.][l + L c], L-point DFTs.
template <int N, bool INV>
__host__ __device__ __forceinline__ void line_fft_stage1(float2 (&v)[Cfg<N>::E], int l, const float2* tw,
                                                         float2* xch) {
  constexpr int L = Cfg<N>::L, E = Cfg<N>::E, XP = Xch<N>::XP;
  static_assert(E % L == 0, "line split needs L | E");
  Dft<E, INV>::run(v);
#pragma unroll
  for (int k1 = 1; k1 < E; ++k1) {
    float2 w = tw[l * k1];
    if (INV) w.y = -w.y;
    v[k1] = cmul(v[k1], w);
  }
#pragma unroll
  for (int k1 = 0; k1 < E; ++k1) xch[k1 * XP + l] = v[k1];
}

template <int N, bool INV>
__host__ __device__ __forceinline__ void line_fft_stage2(float2 (&v)[Cfg<N>::E], int l, const float2* xch) {
  constexpr int L = Cfg<N>::L, E = Cfg<N>::E, C = E / L, XP = Xch<N>::XP;
  float2 u[E];
#pragma unroll
  for (int c = 0; c < C; ++c) {
#pragma unroll
    for (int ll = 0; ll < L; ++ll) u[c * L + ll] = xch[(l + L * c) * XP + ll];
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    Dft<L, INV>::run(&u[c * L]);
#pragma unroll
    for (int k2 = 0; k2 < L; ++k2) v[c + C * k2] = u[c * L + k2];
  }
}

// Whole line FFT. SYNC orders the lanes' LDS accesses: it runs before the
// exchange writes (so the scratch may be reused line after line) and
// between the writes and the reads.
template <int N, bool INV, typename SYNC>
__device__ __forceinline__ void line_fft(float2 (&v)[Cfg<N>::E], int l, const float2* tw, float2* xch,
                                         SYNC sync) {
  Dft<Cfg<N>::E, INV>::run(v);
  constexpr int L = Cfg<N>::L, E = Cfg<N>::E, XP = Xch<N>::XP;
#pragma unroll
  for (int k1 = 1; k1 < E; ++k1) {
    float2 w = tw[l * k1];
    if (INV) w.y = -w.y;
    v[k1] = cmul(v[k1], w);
  }
  sync();
#pragma unroll
  for (int k1 = 0; k1 < E; ++k1) xch[k1 * XP + l] = v[k1];
  sync();
  line_fft_stage2<N, INV>(v, l, xch);
  (void)L;
}

// ---------------------------------------------------------------- LDS-resident tiles
// Row pitch (float2) of an LDS-resident N x N tile and the workgroup size of
// the resident chains; the pitch leaves room for the padded row exchange.
template <int N> struct Res;
template <> struct Res<64>  { static constexpr int P = 93,  THREADS = 512; };
template <> struct Res<128> { static constexpr int P = 146, THREADS = 1024; };

// Line transform with the line's slot s stored at base[s * STRIDE] (XP: slot
// pitch of the exchange, L + 1 for rows, L for columns). Stages as in
// line_fft_stage1/2, with the exchange written into the line's own storage.
template <int N, bool INV, int XP, int STRIDE>
__host__ __device__ __forceinline__ void res_stage1(float2 (&v)[Cfg<N>::E], int l, const float2* tw, float2* base) {
  constexpr int L = Cfg<N>::L, E = Cfg<N>::E;
  static_assert((E - 1) * XP + L <= (XP == L ? N : N + E), "exchange exceeds the line storage");
  Dft<E, INV>::run(v);
#pragma unroll
  for (int k1 = 1; k1 < E; ++k1) {
    float2 w = tw[l * k1];
    if (INV) w.y = -w.y;
    v[k1] = cmul(v[k1], w);
  }
#pragma unroll
  for (int k1 = 0; k1 < E; ++k1) base[(k1 * XP + l) * STRIDE] = v[k1];
}

template <int N, bool INV, int XP, int STRIDE>
__host__ __device__ __forceinline__ void res_stage2(float2 (&v)[Cfg<N>::E], int l, const float2* base) {
  constexpr int L = Cfg<N>::L, E = Cfg<N>::E, C = E / L;
  float2 u[E];
#pragma unroll
  for (int c = 0; c < C; ++c) {
#pragma unroll
    for (int ll = 0; ll < L; ++ll) u[c * L + ll] = base[((l + L * c) * XP + ll) * STRIDE];
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    Dft<L, INV>::run(&u[c * L]);
#pragma unroll
    for (int k2 = 0; k2 < L; ++k2) v[c + C * k2] = u[c * L + k2];
  }
}

// Ordering of LDS accesses among the lanes of one wavefront.
struct WaveSync {
  __device__ __forceinline__ void operator()() const {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
};
// Ordering among all waves of the workgroup.
struct BlockSync {
  __device__ __forceinline__ void operator()() const { __syncthreads(); }
};

}  // namespace pty
