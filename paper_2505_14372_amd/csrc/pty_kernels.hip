// pty_kernels.hip -- HIP kernels (gfx950) of the multislice forward model,
// noise-model loss and exact adjoint of arXiv 2505.14372 (Sec. 3 - 3.2).
//
// Data layout (all row-major, complex = float2):
//   workspace tile (item b, mode m):  ws[(tile0(b) + m) * N*N + y*N + x]
//   object slice i:                   obj[(i*H + y)*W + x]
//   propagator for the gap after slice i (already divided by N^2):
//                                     prop[i*N*N + u_y*N + u_x]
//   probe spectrum (unitary):         phat[m*N*N + u_y*N + u_x]
//   entry-wave checkpoints:           ck[(ck0(b) + m + slot * n_items * M) * N*N + ...]
//                                     (slot-major: one slice's waves of the group are contiguous);
//                                     stored in float they hold the row spectrum F_x(psi_i):
//                                     the forward row pass of slice i - 1 leaves its output in
//                                     slot i and the column pass completes it there in place;
//                                     the segment buffers of recomputed slices hold the same
//
// One slice step is two passes over a tile, each a batched launch:
//   row pass    : inverse row DFT -> entry wave psi_i (real space, optionally
//                 checkpointed) -> times the object patch -> forward row DFT
//                 (the adjoint row pass recovers psi_i from a spectral
//                 checkpoint with the same inverse row DFT)
//   column pass : forward column DFT -> times the propagator -> inverse
//                 column DFT
// so that F^-1 H F between slices costs one read and one write of the tile
// per pass. The adjoint runs the same passes backwards with conjugated
// multipliers and accumulates the object gradient in the row pass.
#include <hip/hip_runtime.h>

#include <hip/hip_fp16.h>

#include <cmath>

#include "pty_fft.hpp"
#include "pty_internal.h"

namespace pty {

constexpr int kThreads = 256;

// Rows of a tile per row-pass workgroup, columns per column-pass workgroup.
template <int N> struct Pass {
  static constexpr int L = Cfg<N>::L, E = Cfg<N>::E;
  static constexpr int LINES = kThreads / L;      // lines held by one workgroup at once
  static constexpr int NBLK = N / LINES;          // workgroups per tile
};

__device__ __forceinline__ void raise_flag(int* flags, int bit) {
  if (flags) atomicOr(flags, bit);
}

template <int N>
__device__ __forceinline__ void load_twiddles(float2* tw_lds, const float2* tw_glb) {
  for (int k = threadIdx.x; k < N; k += blockDim.x) tw_lds[k] = tw_glb[k];
}


// Entry-wave checkpoint storage: complex64 (float2) or two IEEE halves
// (__half2, round to nearest).
template <bool HALF> struct Ck;
template <> struct Ck<false> {
  using T = float2;
  __device__ __forceinline__ static void store(T* p, float2 v) { *p = v; }
  __device__ __forceinline__ static float2 load(const T* p) { return *p; }
};
template <> struct Ck<true> {
  using T = __half2;
  __device__ __forceinline__ static void store(T* p, float2 v) { *p = __floats2half2_rn(v.x, v.y); }
  __device__ __forceinline__ static float2 load(const T* p) { return __half22float2(*p); }
};

// Raw buffer view of one tile (base uniform across the workgroup): an offset
// at or past the end (kOff) reads zero and drops a store without touching
// memory, so the lanes of band-limited columns in a column pass need no
// branch. (In the row passes the same form raised register use and was
// slower than plain masked accesses.)
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr unsigned kOff = 0x80000000u;
struct TileBuf {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ TileBuf(const void* base, unsigned bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000)) {}
  __device__ __forceinline__ float2 ld(unsigned off) const {
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
  }
  __device__ __forceinline__ void st(unsigned off, float2 x) const {
    const u32x2 v = {__float_as_uint(x.x), __float_as_uint(x.y)};
    __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, 0);
  }
};
// Is column x of the row spectrum inside the propagators' support?
template <int N>
__device__ __forceinline__ bool col_live(const ReqDev& r, int x) {
  if (!r.live) return true;
  if (r.live_k >= 0) return abs(x < (N + 1) / 2 ? x : x - N) <= r.live_k;
  return r.live[x] != 0;
}

// Does one row-pass slot (L lanes x 8 bytes of a row) cover whole 128-byte
// lines (L = 16, N = 256)? Only then are read-once rows loaded non-temporally:
// with L = 8 an instruction reads half of each line and the next slot the
// other half, which a non-temporal load does not keep, so every line would be
// fetched twice. The store forms that write whole lines at the band edges
// (whole slots in the adjoint row pass, whole column blocks in the
// propagation passes) are used at that size too.
template <int N>
struct WholeLines {
  static constexpr bool on = Cfg<N>::L * sizeof(float2) >= 128;
};
template <int N, bool NT>
struct RowNT {
  static constexpr bool on = NT && WholeLines<N>::on;
};

// Row-pass load of x[l + L a] for the register slots a set in `mask`, zero in
// the others. A masked slot loads the lane's slot-0 element of the same row
// instead (a line the wave reads anyway), so the loads are unconditional: no
// per-slot branch, and the compiler may issue them together.
// (NT: non-temporal loads, for rows read once; see RowNT.)
template <int N, bool NT = false>
__device__ __forceinline__ void load_row_masked(float2 (&v)[Cfg<N>::E], const float2* row, int l, unsigned mask) {
  constexpr int L = Cfg<N>::L, E = Cfg<N>::E;
#pragma unroll
  for (int a = 0; a < E; ++a) {
    const bool on = (mask >> a) & 1u;
    float2 t;
    if constexpr (RowNT<N, NT>::on) {
      const float2* p = row + (on ? l + L * a : l);
      t = make_float2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
    } else {
      t = row[on ? l + L * a : l];
    }
    v[a] = on ? t : make_float2(0.f, 0.f);
  }
}

// The slots set in `mask` of any lane of the wave, as a wave-uniform value:
// the L lanes of a line hold every column residue, and every line of a wave
// has the same residues, so an OR over the L lanes of one line suffices.
template <int N>
__device__ __forceinline__ unsigned wave_slots(unsigned mask) {
#pragma unroll
  for (int off = 1; off < Cfg<N>::L; off <<= 1) mask |= (unsigned)__shfl_xor((int)mask, off);
  return __builtin_amdgcn_readfirstlane(mask);
}

// Row-pass load of x[l + L a] for the register slots a set in `mask`, zero in
// the others. `any` (wave_slots(mask)) is uniform, so a slot no lane of the
// wave needs is skipped by a scalar branch and costs no request; the other
// slots are read by every lane from one base address with immediate offsets
// (no per-slot address registers), and the lanes whose slot is dead take zero.
// A dead column of a tile holds whatever was last written there (stale data,
// or a value a pass stored only to write its line whole), so what a dead lane
// reads is discarded, never used.
// (NT: non-temporal loads, for rows read once; see RowNT.)
template <int N, bool NT = false>
__device__ __forceinline__ void load_row_slots(float2 (&v)[Cfg<N>::E], const float2* row, int l, unsigned mask,
                                               unsigned any) {
  constexpr int L = Cfg<N>::L, E = Cfg<N>::E;
  const float2* p = row + l;
#pragma unroll
  for (int a = 0; a < E; ++a) {
    v[a] = make_float2(0.f, 0.f);
    if ((any >> a) & 1u) {
      if constexpr (RowNT<N, NT>::on)
        v[a] = make_float2(__builtin_nontemporal_load(&p[L * a].x), __builtin_nontemporal_load(&p[L * a].y));
      else v[a] = p[L * a];
    }
  }
  const unsigned part = any & ~mask;
#pragma unroll
  for (int a = 0; a < E; ++a)
    if ((part >> a) & 1u) v[a] = make_float2(0.f, 0.f);
}

// Row-pass store of the slots set in `any` (wave-uniform): every lane of a
// live slot stores, also a lane whose column is dead, since no consumer reads
// dead columns.
template <int N>
__device__ __forceinline__ void store_row_slots(const float2 (&v)[Cfg<N>::E], float2* row, int l, unsigned any) {
  constexpr int L = Cfg<N>::L, E = Cfg<N>::E;
  float2* p = row + l;
#pragma unroll
  for (int a = 0; a < E; ++a)
    if ((any >> a) & 1u) p[L * a] = v[a];
}

// byte offset of element (y, x) of an N x N tile, or kOff when the lane is masked off
template <int N>
__device__ __forceinline__ unsigned tile_off(bool on, int y, int x) {
  return on ? (unsigned)((y * N + x) * 8) : kOff;
}

// ============================================================ items

// One workgroup per batch entry: find its request, integer window offset and
// subpixel remainder (in double, so n = floor(X + 0.5) is exact for float32
// positions), bounds check, workspace offsets, and the two 1D shift ramps
// exp(-2 pi i f(u) d) with f(u) = fftfreq(N).
__global__ void k_items(const ReqTable reqs, int n_reqs, Item* __restrict__ items,
                        float2* __restrict__ ramps, int n_items, int N, int* flags) {
  const int b = blockIdx.x;
  if (b >= n_items) return;
  int q = 0;
  for (int k = 0; k < n_reqs; ++k)
    if (b >= reqs.r[k].item0 && b < reqs.r[k].item0 + reqs.r[k].n_items) q = k;
  const ReqDev& r = reqs.r[q];
  const int local = b - r.item0;
  const int j = r.batch_idx[local];
  const bool ok_idx = (j >= 0 && j < r.J);
  const double X0 = ok_idx ? (double)r.positions[2 * j] : 0.0;
  const double X1 = ok_idx ? (double)r.positions[2 * j + 1] : 0.0;
  const double n0 = floor(X0 + 0.5), n1 = floor(X1 + 0.5);
  const bool ok = ok_idx && (n0 >= 0.0) && (n1 >= 0.0) && (n0 + N <= (double)r.H) &&
                  (n1 + N <= (double)r.W);
  const float d0 = ok ? (float)(X0 - n0) : 0.f, d1 = ok ? (float)(X1 - n1) : 0.f;
  if (threadIdx.x == 0) {
    Item it;
    it.req = q;
    it.j = ok_idx ? j : 0;
    it.ny = ok ? (int)n0 : 0;
    it.nx = ok ? (int)n1 : 0;
    it.dy = d0;
    it.dx = d1;
    it.valid = ok ? 1 : 0;
    it.tile0 = r.tile_base + local * r.M;
    it.ck0 = r.ck_base + (long long)local * r.M;
    items[b] = it;
    if (!ok) raise_flag(flags, kFlagBounds);
  }
  for (int u = threadIdx.x; u < N; u += blockDim.x) {
    const int k = (u < (N + 1) / 2) ? u : u - N;
    const float f = (float)k / (float)N;
    float s0, c0, s1, c1;
    sincospif(2.f * f * d0, &s0, &c0);
    sincospif(2.f * f * d1, &s1, &c1);
    ramps[(size_t)b * 2 * N + u] = make_float2(c0, -s0);
    ramps[(size_t)b * 2 * N + N + u] = make_float2(c1, -s1);
  }
}

// ============================================================ row passes

// Slice step of the forward model, row part (slice i = step):
//   psi = IDFT_x(tile row) ; [checkpoint psi] ; phi = psi * O_i ; tile row = DFT_x(phi)
// With FROM_REAL the entry wave is read from a real-space buffer (the start
// of a segment recomputed from half-precision checkpoints) instead of inverse-transforming the tile. With
// EMAX the maxima over the window of sum_m |psi_i,m|^2 and of |O_i|^2 are
// max-accumulated into r.emax[item][i] (non-negative floats order like their
// bit patterns, so an unsigned atomic max is exact).
template <int N, bool FROM_REAL, bool HALF, bool EMAX = false>
__global__ __launch_bounds__(kThreads) void k_row_fwd(const Item* __restrict__ items,
                                                      const ReqTable reqs,
                                                      float2* __restrict__ ws, void* __restrict__ ck_,
                                                      const float2* __restrict__ twg, int step,
                                                      PsiStore store, int item_off) {
  // items in reverse order (the column passes run them forward; see Launch::col)
  const int by = gridDim.y - 1 - blockIdx.y;
  constexpr int L = Pass<N>::L, E = Pass<N>::E, LINES = Pass<N>::LINES;
  __shared__ float2 tw[N];
  __shared__ float2 xch[LINES * Xch<N>::ROW_STRIDE];
  const Item it = items[item_off + by];
  const ReqDev& r = reqs.r[it.req];
  const int i = step;
  if (!it.valid || i >= r.S) return;
  load_twiddles<N>(tw, twg);
  __syncthreads();
  using CT = typename Ck<HALF>::T;
  CT* ck = static_cast<CT*>(ck_);
  const int l = threadIdx.x % L, line = threadIdx.x / L;
  const int y = blockIdx.x * LINES + line;
  float2* sx = xch + line * Xch<N>::ROW_STRIDE;
  // the row spectrum of slice i >= 1 was written by a propagation column pass,
  // which leaves the columns outside the propagator's support unwritten (zero)
  unsigned live = ~0u;
  if (r.live) {
    live = 0u;
#pragma unroll
    for (int a = 0; a < E; ++a) live |= (col_live<N>(r, l + L * a) ? 1u : 0u) << a;
  }
  const unsigned lmask = i >= 1 ? live : ~0u;
  // the output of slices i < S - 1 feeds only the propagation column pass,
  // which reads the live columns alone
  const unsigned omask = i < r.S - 1 ? live : ~0u;
  const unsigned any_l = wave_slots<N>(lmask), any_o = wave_slots<N>(omask);
  // object patch row, shared by every mode
  float2 o[E];
  const float2* orow = r.obj + ((size_t)i * r.H + it.ny + y) * r.W + it.nx;
#pragma unroll
  for (int a = 0; a < E; ++a) o[a] = orow[l + L * a];
  float pw[EMAX ? E : 1];
  if constexpr (EMAX) {
#pragma unroll
    for (int a = 0; a < E; ++a) pw[a] = 0.f;
  }
  // Each mode's output row is stored as soon as it is transformed: with the
  // masked loads and stores in load_row_slots / store_row_slots the pass
  // holds few enough registers for three waves per SIMD at N = 256, which
  // hides the memory latency better than deferring the stores behind the
  // next mode's requests at two waves.
  for (int m = 0; m < r.M; ++m) {
    float2* trow = ws + ((size_t)(it.tile0 + m) * N + y) * N;
    float2 v[E];
    if constexpr (FROM_REAL) {
      const CT* src = static_cast<const CT*>(store.src) + (ck_tile(it, r, m, store.src_slot) * N + y) * N;
#pragma unroll
      for (int a = 0; a < E; ++a) v[a] = Ck<HALF>::load(src + l + L * a);
    } else {
      // the row spectrum comes from the work tile or, with spectral
      // checkpoints, from where the column pass left it: checkpoint slot
      // i / ck_every for a stored slice, segment slot seg_slot for a slice
      // being recomputed
      const float2* in = trow;
      if (store.mode == 3) {
        if (i % r.ck_every == 0)
          in = static_cast<const float2*>(ck_) + (ck_tile(it, r, m, i / r.ck_every) * N + y) * N;
        else if (store.seg)
          in = static_cast<const float2*>(store.seg) +
               (((size_t)(it.tile0 + m) * store.seg_len + store.seg_slot) * N + y) * N;
      }
      // a checkpoint or segment row spectrum is not read again before the
      // adjoint: loaded non-temporally, so that it does not displace the
      // tiles the next column pass reads from the caches
      if (in != trow) load_row_slots<N, true>(v, in, l, lmask, any_l);
      else load_row_slots<N>(v, in, l, lmask, any_l);
      line_fft<N, true>(v, l, tw, sx, WaveSync{});
    }
    if (store.mode == 1 && (i % r.ck_every) == 0) {
      CT* dst = ck + (ck_tile(it, r, m, i / r.ck_every) * N + y) * N;
#pragma unroll
      for (int a = 0; a < E; ++a) Ck<HALF>::store(dst + l + L * a, v[a]);
    } else if (store.mode == 2) {
      CT* dst = static_cast<CT*>(store.seg) + (((size_t)(it.tile0 + m) * store.seg_len + store.seg_slot) * N + y) * N;
#pragma unroll
      for (int a = 0; a < E; ++a) Ck<HALF>::store(dst + l + L * a, v[a]);
    }
    if constexpr (EMAX) {
#pragma unroll
      for (int a = 0; a < E; ++a) pw[a] += cabs2(v[a]);
    }
    if (store.stop_after_store) continue;
#pragma unroll
    for (int a = 0; a < E; ++a) v[a] = cmul(v[a], o[a]);
    line_fft<N, false>(v, l, tw, sx, WaveSync{});
    // With spectral checkpoints the output of a slice whose successor is
    // stored goes straight into that successor's checkpoint slot, where the
    // column pass completes it in place (a column pass that writes where it
    // read runs faster than one writing lines nothing has touched lately; the
    // row pass pays less for such writes).
    float2* out = trow;
    if (store.mode == 3 && i + 1 < r.S && (i + 1) % r.ck_every == 0)
      out = static_cast<float2*>(ck_) + (ck_tile(it, r, m, (i + 1) / r.ck_every) * N + y) * N;
    store_row_slots<N>(v, out, l, any_o);
  }
  if constexpr (EMAX) {
    float mp = 0.f, mo = 0.f;
#pragma unroll
    for (int a = 0; a < E; ++a) {
      mp = fmaxf(mp, pw[a]);
      mo = fmaxf(mo, cabs2(o[a]));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      mp = fmaxf(mp, __shfl_xor(mp, off));
      mo = fmaxf(mo, __shfl_xor(mo, off));
    }
    if ((threadIdx.x & 63) == 0 && r.emax) {
      unsigned* e = reinterpret_cast<unsigned*>(r.emax + ((size_t)(item_off + by - r.item0) * r.S + i) * 2);
      atomicMax(e, __float_as_uint(mp));
      atomicMax(e + 1, __float_as_uint(mo));
    }
  }
}

// Adjoint slice step, row part (slice i = S - 1 - step for each item):
//   g = IDFT_x(tile row)                (gradient wrt phi_i, real space)
//   grad O_i += sum_m conj(psi_i,m) g   (scatter-added into the object gradient
//                                         with atomics, or, with cscr, stored per
//                                         position for k_obj_gather's ordered sum)
//   h = conj(O_i) g ; tile row = DFT_x(h)
// With WSUM the illumination sum_m |psi_i,m|^2 of the window is also scattered
// into r.wsum (LSQML), or stored in wscr for the ordered sum.
// With SPEC the checkpoint slot holds the row spectrum F_x(psi_i) (float2),
// and psi_i is recovered with the forward pass's own inverse row DFT.
template <int N, bool HALF, bool WSUM = false, bool SPEC = false>
__global__ __launch_bounds__(kThreads) void k_row_adj(const Item* __restrict__ items,
                                                      const ReqTable reqs,
                                                      float2* __restrict__ ws, const void* __restrict__ ck_,
                                                      const float2* __restrict__ twg, int step,
                                                      PsiLoad psi, float scale, int item_off,
                                                      float2* __restrict__ cscr, float* __restrict__ wscr) {
  // items in reverse order (the column passes run them forward; see Launch::col)
  const int by = gridDim.y - 1 - blockIdx.y;
  constexpr int L = Pass<N>::L, E = Pass<N>::E, LINES = Pass<N>::LINES;
  __shared__ float2 tw[N];
  __shared__ float2 xch[LINES * Xch<N>::ROW_STRIDE];
  const Item it = items[item_off + by];
  const ReqDev& r = reqs.r[it.req];
  const int i = r.S - 1 - step;
  if (!it.valid || i < 0) return;
  load_twiddles<N>(tw, twg);
  __syncthreads();
  const int l = threadIdx.x % L, line = threadIdx.x / L;
  const int y = blockIdx.x * LINES + line;
  float2* sx = xch + line * Xch<N>::ROW_STRIDE;
  using CT = typename Ck<HALF>::T;
  const CT* ck = static_cast<const CT*>(ck_);
  // columns outside the propagator's support: zero in g for i < S - 1 (it came
  // through an adjoint propagation column pass) and in a spectral checkpoint
  // for i >= 1 (written by a forward one); in memory they hold zeros or stale
  // data (a dead column is written only when its line holds live ones), so
  // they are masked rather than read
  unsigned live = ~0u;
  if (r.live) {
    live = 0u;
#pragma unroll
    for (int a = 0; a < E; ++a) live |= (col_live<N>(r, l + L * a) ? 1u : 0u) << a;
  }
  const unsigned gmask = (r.live && i < r.S - 1) ? live : ~0u;
  const unsigned cmask = (r.live && i >= 1) ? live : ~0u;
  // the output of slices i >= 1 feeds only the adjoint propagation column
  // pass, which reads the live columns alone (slice 0 feeds the final one).
  // Where a slot is a whole line (N = 256) every lane of a slot with a live
  // column stores, as in the forward row pass: whole-line writes beat partial
  // ones at the band edges (1.070 -> 1.046 ms per launch at 8 modes, 512
  // positions); at 8 lanes per line only the live lanes store.
  const unsigned omask = cmask;
  const unsigned any_o = WholeLines<N>::on ? wave_slots<N>(omask) : omask;
  float2 acc[E];
  const size_t orow = ((size_t)i * r.H + it.ny + y) * r.W + it.nx;
  // ePIE: object step divided by max sum_m |psi_i|^2, wave step by max |O_i|^2
  float sa = 1.f, sb = 1.f;
  if (r.emax) {
    const float* e = r.emax + ((size_t)(item_off + by - r.item0) * r.S + i) * 2;
    sa = e[0] > 0.f ? 1.f / e[0] : 0.f;
    sb = e[1] > 0.f ? 1.f / e[1] : 0.f;
  }
  // the object row is held in registers for all modes, except at 24 values
  // per lane (N = 192), where that would leave one wave per SIMD: there it is
  // read again per mode (from cache)
  constexpr bool OREG = E <= 16;
  float2 o[OREG ? E : 1];
  if constexpr (OREG) {
#pragma unroll
    for (int a = 0; a < E; ++a) o[a] = cscale(r.obj[orow + l + L * a], sb);
  }
#pragma unroll
  for (int a = 0; a < E; ++a) acc[a] = make_float2(0.f, 0.f);
  float pw[WSUM ? E : 1];
  if constexpr (WSUM) {
#pragma unroll
    for (int a = 0; a < E; ++a) pw[a] = 0.f;
  }
  // each mode's output row is stored after the next mode's requests (see k_row_fwd)
  float2 hout[E];
  float2* out_row = nullptr;
  auto flush = [&]() {
    if (!out_row) return;
#pragma unroll
    for (int a = 0; a < E; ++a)
      if ((any_o >> a) & 1u) out_row[l + L * a] = hout[a];
    out_row = nullptr;
  };
  for (int m = 0; m < r.M; ++m) {
    float2* trow = ws + ((size_t)(it.tile0 + m) * N + y) * N;
    const CT* prow;
    if (psi.from_seg) prow = static_cast<const CT*>(psi.seg) + (((size_t)(it.tile0 + m) * psi.seg_len + (i - psi.seg_base)) * N + y) * N;
    else prow = ck + (ck_tile(it, r, m, i / r.ck_every) * N + y) * N;
    // both rows are requested before the first transform (its LDS fences
    // would otherwise hold the second request back by a whole memory latency)
    float2 v[E];
    float2 ps[SPEC ? E : 1];
    load_row_masked<N>(v, trow, l, gmask);
    // the checkpoint row is read once: non-temporal, so that the gradient
    // tiles the adjoint column pass reads next stay in the caches
    if constexpr (SPEC) load_row_masked<N, true>(ps, reinterpret_cast<const float2*>(prow), l, cmask);
    flush();
    line_fft<N, true>(v, l, tw, sx, WaveSync{});
    if constexpr (SPEC) line_fft<N, true>(ps, l, tw, sx, WaveSync{});
#pragma unroll
    for (int a = 0; a < E; ++a) {
      float2 p;
      if constexpr (SPEC) p = ps[a];
      else p = Ck<HALF>::load(prow + l + L * a);
      if constexpr (WSUM) pw[a] += cabs2(p);
      acc[a] = cadd(acc[a], cjmul(p, v[a]));
      if constexpr (OREG) v[a] = cjmul(o[a], v[a]);
      else v[a] = cjmul(cscale(r.obj[orow + l + L * a], sb), v[a]);
    }
    line_fft<N, false>(v, l, tw, sx, WaveSync{});
#pragma unroll
    for (int a = 0; a < E; ++a) hout[a] = v[a];
    out_row = trow;
  }
  flush();
  if (r.gobj) {
    const float sc = adj_scale(r, scale) * sa;
    if (cscr) {
      // ordered reduction: this position's contribution, added in batch order by k_obj_gather
      float2* dst = cscr + ((size_t)(item_off + by) * N + y) * N;
#pragma unroll
      for (int a = 0; a < E; ++a) dst[l + L * a] = cscale(acc[a], sc);
    } else {
      float* g = reinterpret_cast<float*>(r.gobj + orow);
#pragma unroll
      for (int a = 0; a < E; ++a) {
        unsafeAtomicAdd(g + 2 * (l + L * a), sc * acc[a].x);
        unsafeAtomicAdd(g + 2 * (l + L * a) + 1, sc * acc[a].y);
      }
    }
  }
  if constexpr (WSUM) {
    if (r.wsum && wscr) {
      // ordered reduction: stored per position, added in batch order by k_obj_gather
      float* dst = wscr + ((size_t)(item_off + by) * N + y) * N;
#pragma unroll
      for (int a = 0; a < E; ++a) dst[l + L * a] = pw[a];
    } else if (r.wsum) {
#pragma unroll
      for (int a = 0; a < E; ++a) unsafeAtomicAdd(r.wsum + orow + l + L * a, pw[a]);
    }
  }
}

// Plain row DFT of M probe-sized tiles: dst = DFT_x(src) (or inverse).
template <int N, bool INV>
__global__ __launch_bounds__(kThreads) void k_row_plain(const float2* __restrict__ src, float2* __restrict__ dst,
                                                        const float2* __restrict__ twg, float scale,
                                                        int accumulate) {
  constexpr int L = Pass<N>::L, E = Pass<N>::E, LINES = Pass<N>::LINES;
  __shared__ float2 tw[N];
  __shared__ float2 xch[LINES * Xch<N>::ROW_STRIDE];
  load_twiddles<N>(tw, twg);
  __syncthreads();
  const int l = threadIdx.x % L, line = threadIdx.x / L;
  const int y = blockIdx.x * LINES + line;
  const size_t base = ((size_t)blockIdx.y * N + y) * N;
  float2 v[E];
#pragma unroll
  for (int a = 0; a < E; ++a) v[a] = src[base + l + L * a];
  line_fft<N, INV>(v, l, tw, xch + line * Xch<N>::ROW_STRIDE, WaveSync{});
#pragma unroll
  for (int a = 0; a < E; ++a) {
    float2 w = cscale(v[a], scale);
    if (accumulate) w = cadd(w, dst[base + l + L * a]);
    dst[base + l + L * a] = w;
  }
}

// ============================================================ column passes

// Column-pass thread layout: thread t holds column c = t % CB of the block
// and lane l = t / CB of that column's line, so that a load of register a
// reads CB consecutive complex values of row l + L a (coalesced).
#ifndef PTY_COL_CB_L16
#define PTY_COL_CB_L16 32
#endif
#ifndef PTY_COL_CB_L8
#define PTY_COL_CB_L8 32
#endif
template <int N> struct ColPass {
  static constexpr int L = Cfg<N>::L, E = Cfg<N>::E;
  static constexpr int CB = (L == 16) ? PTY_COL_CB_L16 : PTY_COL_CB_L8;   // columns per workgroup
  static constexpr int THREADS = CB * L;
  static constexpr int NBLK = N / CB;
};

// Thread -> (column, lane) mapping of the column passes: column c = t % CB,
// lane l = t / CB, so a load of register a reads CB consecutive values of
// one row per lane group; a column's lanes span several waves and exchange
// through LDS with block barriers. (Keeping each column inside one wave, with
// no block barrier, measured slower: the loads then cover 64 / L values per
// row.)
template <int N> struct ColMap {
  static constexpr int CB = ColPass<N>::CB;
  // per-column exchange stride: with 32 or more columns of 16 lanes an odd
  // stride keeps a wave's accesses at two bank cycles (checked by exhaustive count)
  static constexpr int STRIDE = (CB >= 32 && Cfg<N>::L == 16) ? pad_to(Xch<N>::SIZE, 2, 1) : Xch<N>::COL_STRIDE;
  __device__ __forceinline__ static int col() { return threadIdx.x % CB; }
  __device__ __forceinline__ static int lane() { return threadIdx.x / CB; }
  using Sync = BlockSync;
};

// Column passes over (item, mode) tiles:
//   COL_SHIFT    tile = IDFT_y(phat_m * R_j) / N         (start of the forward model)
//   COL_PROP     tile = IDFT_y(H_i * DFT_y(tile))        (forward, slice i = step < S-1)
//   COL_PROP_ADJ tile = IDFT_y(conj(H_{i-1}) * DFT_y(tile)) (adjoint, i = S-1-step >= 1)
//   COL_FINAL    tile = DFT_y(tile) / N = h_hat          (adjoint, i = 0) and the
//                per-block sums of Im(conj(h_hat) phat R) u_a for the position gradient
template <int N, int OP>
__global__ __launch_bounds__(ColPass<N>::THREADS) void k_col(const Item* __restrict__ items,
                                                  const ReqTable reqs,
                                                  float2* __restrict__ ws, const float2* __restrict__ ramps,
                                                  const float2* __restrict__ twg, int step,
                                                  float* __restrict__ pos_part, int item_off,
                                                  float2* __restrict__ ck_out, unsigned long long colmap,
                                                  SegOut seg_out) {
  constexpr int L = ColPass<N>::L, E = ColPass<N>::E, CB = ColPass<N>::CB, T = ColPass<N>::THREADS;
  constexpr bool PROP = OP == COL_PROP || OP == COL_PROP_ADJ;
  static_assert(T >= N, "the staged tables take one entry per thread");
  static_assert(ColPass<N>::NBLK <= 8, "the column-block map holds 8 entries");
  // column block of this workgroup: entry blockIdx.x of the launch's block list
  const int cb = (int)((colmap >> (8 * blockIdx.x)) & 0xffu);
  __shared__ float2 tw[N];
  __shared__ float4 hy[PROP ? N : 1];
  __shared__ float2 xch[CB * ColMap<N>::STRIDE];
  __shared__ float red[2][T / 64];
  // grid (column blocks, modes, items): dispatched item by item, in item order
  const int b = item_off + blockIdx.z, m = blockIdx.y;
  const Item it = items[b];
  const ReqDev& r = reqs.r[it.req];
  if (!it.valid || m >= r.M) return;
  int i = 0;
  if constexpr (OP == COL_PROP) { i = step; if (i >= r.S - 1) return; }
  if constexpr (OP == COL_PROP_ADJ) { i = r.S - 1 - step; if (i < 1) return; }
  if constexpr (OP == COL_FINAL) { if (r.S - 1 - step != 0 || r.chain_final) return; }
  if constexpr (PROP) {
    // outside the propagator's support the output columns are zero: a
    // workgroup with no live column has nothing to do (its consumers read zeros)
    if (r.live) {
      bool any = false;
      if (r.live_k >= 0) {
        for (int q = 0; q < CB; ++q) {
          const int x = cb * CB + q;
          any |= abs(x < (N + 1) / 2 ? x : x - N) <= r.live_k;
        }
      } else {
        for (int q = 0; q < CB; ++q) any |= r.live[cb * CB + q] != 0;
      }
      if (!any) return;
    }
  }
  const int c = ColMap<N>::col(), l = ColMap<N>::lane(), t = threadIdx.x;
  const int ux = cb * CB + c;
  float2* sx = xch + c * ColMap<N>::STRIDE;
  float2* tile = ws + (size_t)(it.tile0 + m) * N * N;
  // a forward propagation whose output is a stored checkpoint runs in place
  // in that slot, where the forward row pass left its input
  if constexpr (OP == COL_PROP) {
    if (ck_out && (i + 1) % r.ck_every == 0) tile = ck_out + ck_tile(it, r, m, (i + 1) / r.ck_every) * N * N;
  }
  const bool live_col = PROP ? col_live<N>(r, ux) : true;
  // Memory requests in the order they are needed, all before the first wait:
  // the staged tables (twiddles; the y factors and row limits of a separable
  // propagator), this column's x factor, then the tile column.
  const int gap = OP == COL_PROP ? i : i - 1;
  const bool sep = PROP && r.prop_y != nullptr;
  float2 tw_t = make_float2(0.f, 0.f);
  float4 hy_t = make_float4(0.f, 0.f, 0.f, 0.f);
  float2 hx = make_float2(0.f, 0.f);
  if (t < N) {
    tw_t = twg[t];
    if (sep) hy_t = r.prop_y[(size_t)gap * N + t];
  }
  if (sep) hx = r.prop_x[(size_t)gap * N + ux];
  float2 v[E];
  if constexpr (OP != COL_SHIFT) {
    const TileBuf tb(tile, N * N * 8);
#pragma unroll
    for (int a = 0; a < E; ++a) v[a] = tb.ld(tile_off<N>(live_col, l + L * a, ux));
  }
  if (t < N) {
    tw[t] = tw_t;
    if constexpr (PROP) hy[t] = hy_t;
  }
  __syncthreads();
  if constexpr (OP == COL_SHIFT) {
    const float2* ry = ramps + (size_t)b * 2 * N;
    const float2 rx = ramps[(size_t)b * 2 * N + N + ux];
    const float2* ph = r.phat + (size_t)m * N * N;
    const float inv = 1.f / (float)N;
#pragma unroll
    for (int a = 0; a < E; ++a) {
      int uy = l + L * a;
      v[a] = cscale(cmul(cmul(ph[(size_t)uy * N + ux], ry[uy]), rx), inv);
    }
    line_fft<N, true>(v, l, tw, sx, typename ColMap<N>::Sync{});
  } else {
    line_fft<N, false>(v, l, tw, sx, typename ColMap<N>::Sync{});
    if constexpr (PROP) {
      if (sep) {
        // H = [|k_x| <= K_y] Hy(k_y) Hx(k_x), factors staged above
        const int akx = abs(ux < (N + 1) / 2 ? ux : ux - N);
#pragma unroll
        for (int a = 0; a < E; ++a) {
          const float4 q = hy[l + L * a];
          float2 h = cmul(make_float2(q.x, q.y), hx);
          if (akx > __float_as_int(q.z)) h = make_float2(0.f, 0.f);
          v[a] = (OP == COL_PROP) ? cmul(v[a], h) : cjmul(h, v[a]);
        }
      } else {
        const float2* H = r.prop + (size_t)gap * N * N;
#pragma unroll
        for (int a = 0; a < E; ++a) {
          float2 h = H[(size_t)(l + L * a) * N + ux];
          v[a] = (OP == COL_PROP) ? cmul(v[a], h) : cjmul(h, v[a]);
        }
      }
      line_fft<N, true>(v, l, tw, sx, typename ColMap<N>::Sync{});
    } else {  // COL_FINAL
      const float inv = 1.f / (float)N;
      const float2* ry = ramps + (size_t)b * 2 * N;
      const float2 rx = ramps[(size_t)b * 2 * N + N + ux];
      const float2* ph = r.phat + (size_t)m * N * N;
      const float fx = (float)((ux < (N + 1) / 2) ? ux : ux - N) / (float)N;
      float sy = 0.f, sxx = 0.f;
#pragma unroll
      for (int a = 0; a < E; ++a) {
        int uy = l + L * a;
        v[a] = cscale(v[a], inv);
        float2 A = cmul(cmul(ph[(size_t)uy * N + ux], ry[uy]), rx);
        float2 z = cjmul(v[a], A);          // conj(h_hat) * A
        float fy = (float)((uy < (N + 1) / 2) ? uy : uy - N) / (float)N;
        sy += fy * z.y;
        sxx += fx * z.y;
      }
      // block reduction of (sy, sxx)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        sy += __shfl_xor(sy, off);
        sxx += __shfl_xor(sxx, off);
      }
      if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = sy; red[1][threadIdx.x >> 6] = sxx; }
      __syncthreads();
      if (threadIdx.x == 0) {
        float t0 = 0.f, t1 = 0.f;
        for (int w = 0; w < ColPass<N>::THREADS / 64; ++w) { t0 += red[0][w]; t1 += red[1][w]; }
        float* dst = pos_part + ((size_t)(it.tile0 + m) * ColPass<N>::NBLK + cb) * 2;
        dst[0] = t0;
        dst[1] = t1;
      }
    }
  }
  // spectral checkpoints: the row spectrum of the entry wave of slice s1 (0
  // for COL_SHIFT, i + 1 for COL_PROP) goes to checkpoint slot s1 / ck_every
  // when that slice is stored (for COL_PROP the slot it was read from), to its
  // segment slot while a segment is being recomputed, else to the work tile
  float2* dst = tile;
  if constexpr (OP == COL_SHIFT || OP == COL_PROP) {
    if (ck_out) {
      const int s1 = OP == COL_SHIFT ? 0 : i + 1;
      if (s1 % r.ck_every == 0)
        dst = ck_out + ck_tile(it, r, m, s1 / r.ck_every) * N * N;
      else if (seg_out.seg)
        dst = seg_out.seg + ((size_t)(it.tile0 + m) * seg_out.len + (s1 - seg_out.base)) * N * N;
    }
  }
  const TileBuf out(dst, N * N * 8);
  // A dead column of a live block holds zero (it was read as zero and stays
  // zero through the transforms). At N = 256 the whole block is stored, so
  // that the lines at the band edges are written whole (forward and adjoint
  // propagation passes 0.61 -> 0.57 ms per launch at 8 modes and 512
  // positions); at N = 128 and 192 that measured slower (more of each live
  // block is dead there), and only the live columns are stored.
  const bool st_col = (PROP && WholeLines<N>::on) ? true : live_col;
#pragma unroll
  for (int a = 0; a < E; ++a) out.st(tile_off<N>(st_col, l + L * a, ux), v[a]);
}

// Plain column DFT of M probe-sized tiles (in place): tile = scale * DFT_y(tile).
template <int N, bool INV>
__global__ __launch_bounds__(ColPass<N>::THREADS) void k_col_plain(float2* __restrict__ t, const float2* __restrict__ twg,
                                                        float scale) {
  constexpr int L = ColPass<N>::L, E = ColPass<N>::E, CB = ColPass<N>::CB;
  __shared__ float2 tw[N];
  __shared__ float2 xch[CB * ColMap<N>::STRIDE];
  load_twiddles<N>(tw, twg);
  __syncthreads();
  const int c = ColMap<N>::col(), l = ColMap<N>::lane();
  const int ux = blockIdx.x * CB + c;
  float2* tile = t + (size_t)blockIdx.y * N * N;
  float2 v[E];
#pragma unroll
  for (int a = 0; a < E; ++a) v[a] = tile[(size_t)(l + L * a) * N + ux];
  line_fft<N, INV>(v, l, tw, xch + c * ColMap<N>::STRIDE, typename ColMap<N>::Sync{});
#pragma unroll
  for (int a = 0; a < E; ++a) tile[(size_t)(l + L * a) * N + ux] = cscale(v[a], scale);
}

// ============================================================ far field + loss

__device__ __forceinline__ void loss_weight(int kind, float I, float Ie, float eps, float inv_sigma2,
                                            float& ell, float& w) {
  if (kind == PTY_LOSS_POISSON) {
    if (Ie == 0.f) {
      ell = I;
      w = 2.f;
    } else {
      // I - Ie - Ie (ln(I+eps) - ln(Ie+eps)). Near I = Ie the log ratio is
      // log1p of the relative difference (no cancellation); away from it the
      // difference of the two logs, since for I + eps below about 6e-8 of
      // Ie + eps the relative difference rounds to -1 and log1p would return
      // -inf for a finite loss. Invalid counts (negative, NaN) and I + eps = 0
      // give a non-finite loss and raise the flag.
      const float den = Ie + eps;
      const float x = (I - Ie) / den;
      const float lr = fabsf(x) < 0.5f ? log1pf(x) : logf(I + eps) - logf(den);
      ell = (I - Ie) - Ie * lr;
      w = 2.f * (1.f - Ie / (I + eps));
    }
  } else if (kind == PTY_LOSS_GAUSSIAN) {
    float d = I - Ie;
    ell = 0.5f * d * d * inv_sigma2;
    w = 2.f * d * inv_sigma2;
  } else {
    float c = (kind == PTY_LOSS_ANSCOMBE) ? 0.375f : 0.f;
    float a = sqrtf(I + c), ae = sqrtf(Ie + c);
    ell = 0.5f * (a - ae) * (a - ae);
    float den = eps + a;
    w = (den > 0.f) ? 1.f - ae / den : 0.f;
  }
}

// Far field of the last slice, incoherent mode sum and noise model, per
// (item, column block), looping over modes:
//   Psi_m = DFT_y(tile_m) / N ; I = sum_m |Psi_m|^2 ; (l, w) from (I, Ie)
// then, if GRAD, the first adjoint step for every mode:
//   tile_m = IDFT_y(w * Psi_m) / N
// Writes intensities (if requested) and per-block loss partial sums.
// At N = 256 the launch bound asks for four waves per SIMD (128 VGPRs, 40
// bytes per lane spilled), which lets two 512-thread workgroups share a CU
// instead of one: 1.55 -> 1.39 ms per group of 512 positions.
template <int N, bool GRAD>
__global__ __launch_bounds__(ColPass<N>::THREADS, N == 256 ? 4 : 1) void k_far_loss(const Item* __restrict__ items,
                                                       const ReqTable reqs,
                                                       float2* __restrict__ ws, const float2* __restrict__ twg,
                                                       int step, float* __restrict__ loss_part, int* flags,
                                                       int item_off) {
  constexpr int L = ColPass<N>::L, E = ColPass<N>::E, CB = ColPass<N>::CB;
  __shared__ float2 tw[N];
  __shared__ float2 xch[CB * ColMap<N>::STRIDE];
  __shared__ float red[ColPass<N>::THREADS / 64];
  const int b = item_off + blockIdx.y;
  const Item it = items[b];
  const ReqDev& r = reqs.r[it.req];
  if (step != r.S - 1) return;
  const int c = ColMap<N>::col(), l = ColMap<N>::lane();
  const int ux = blockIdx.x * CB + c;
  if (!it.valid) {
    if (r.I_out) {
      float* Io = r.I_out + (size_t)(b - r.item0) * N * N;
#pragma unroll
      for (int a = 0; a < E; ++a) Io[(size_t)(l + L * a) * N + ux] = 0.f;
    }
    if (threadIdx.x == 0) loss_part[(size_t)b * ColPass<N>::NBLK + blockIdx.x] = 0.f;
    return;
  }
  load_twiddles<N>(tw, twg);
  __syncthreads();
  float2* sx = xch + c * ColMap<N>::STRIDE;
  const float inv = 1.f / (float)N;
  float I[E];
#pragma unroll
  for (int a = 0; a < E; ++a) I[a] = 0.f;
  for (int m = 0; m < r.M; ++m) {
    float2* tile = ws + (size_t)(it.tile0 + m) * N * N;
    float2 v[E];
#pragma unroll
    for (int a = 0; a < E; ++a) v[a] = tile[(size_t)(l + L * a) * N + ux];
    line_fft<N, false>(v, l, tw, sx, typename ColMap<N>::Sync{});
#pragma unroll
    for (int a = 0; a < E; ++a) {
      v[a] = cscale(v[a], inv);
      I[a] += cabs2(v[a]);
    }
  }
  float wgt[E];
  float lsum = 0.f;
  bool bad = false;
  const float* pat = r.patterns ? r.patterns + (size_t)it.j * N * N : nullptr;
#pragma unroll
  for (int a = 0; a < E; ++a) {
    size_t p = (size_t)(l + L * a) * N + ux;
    float ell = 0.f, w = 0.f;
    if (pat) {
      loss_weight(r.loss, I[a], pat[p], r.eps, r.inv_sigma2, ell, w);
      // ePIE: (1 - sqrt(Ie + c) / (eps + sqrt(I + c))) Psi is minus the modulus update
      if (r.modulus) {
        float ell_amp;
        loss_weight(r.loss == PTY_LOSS_ANSCOMBE ? PTY_LOSS_ANSCOMBE : PTY_LOSS_AMPLITUDE, I[a], pat[p], r.eps,
                    r.inv_sigma2, ell_amp, w);
      }
    }
    wgt[a] = w;
    lsum += ell;
    bad |= !isfinite(ell) || !isfinite(w);
  }
  if (r.I_out) {
    float* Io = r.I_out + (size_t)(b - r.item0) * N * N;
#pragma unroll
    for (int a = 0; a < E; ++a) Io[(size_t)(l + L * a) * N + ux] = I[a];
  }
  if (bad) raise_flag(flags, kFlagNonFinite);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lsum;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int w = 0; w < ColPass<N>::THREADS / 64; ++w) t += red[w];
    loss_part[(size_t)b * ColPass<N>::NBLK + blockIdx.x] = t;
  }
  if constexpr (GRAD) {
    // the far field of each mode is transformed again rather than stored and
    // re-read: three tile passes (read, read, write) instead of four
    for (int m = 0; m < r.M; ++m) {
      float2* tile = ws + (size_t)(it.tile0 + m) * N * N;
      float2 v[E];
#pragma unroll
      for (int a = 0; a < E; ++a) v[a] = tile[(size_t)(l + L * a) * N + ux];
      line_fft<N, false>(v, l, tw, sx, typename ColMap<N>::Sync{});
#pragma unroll
      for (int a = 0; a < E; ++a) v[a] = cscale(cscale(v[a], inv), wgt[a] * inv);
      line_fft<N, true>(v, l, tw, sx, typename ColMap<N>::Sync{});
#pragma unroll
      for (int a = 0; a < E; ++a) tile[(size_t)(l + L * a) * N + ux] = v[a];
    }
  }
}

// ============================================================ reductions

// Per request: loss = sum over its items and blocks (double).
__global__ void k_loss_reduce(const ReqTable reqs, const float* __restrict__ loss_part, int nblk) {
  const ReqDev& r = reqs.r[blockIdx.x];
  __shared__ double red[kThreads];
  double acc = 0.0;
  const float* part = loss_part + (size_t)r.item0 * nblk;
  const size_t n = (size_t)r.n_items * nblk;
  for (size_t e = threadIdx.x; e < n; e += blockDim.x) acc += (double)part[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && r.loss_out) *r.loss_out = red[0];
}

// Ordered object-gradient reduction for slice i = S - 1 - step of every
// request: one workgroup per TY x 64 tile of the object gradient sums the
// stored contributions of the positions whose windows cover the tile and adds
// the sum to the gradient. Each tile has one owner (no atomics) and the
// summation order is fixed by the batch order and the tile shape alone: the
// covering positions are listed in batch order (a block-wide ordered
// compaction over the request's items, 64 W at a time), wave w sums the w-th
// contiguous part of each list in list order (loads for four positions issued
// ahead of their additions), and the W wave sums are added in wave order at
// the end. With WS the stored illumination sums of LSQML (wscr) are added the
// same way into r.wsum.
// Tile shape per window size (the same for a request alone or in a group, so
// both give the same bits): 8 rows and 4 waves; at N = 128, where a scan's
// object is small for its many positions (a 384 x 384 slice under 1024 windows
// gives 288 tiles of 8 rows for 256 CUs, each summing about 120 positions),
// 2 rows and 8 waves: four times the workgroups and twice the waves per list
// (0.071 -> 0.044 ms per slice, 138.8k -> 142.9k positions/s). Other shapes
// measured no better at 192 and slower at 256.
template <int N> struct Gather { static constexpr int TY = 8, W = 4; };
template <> struct Gather<128> { static constexpr int TY = 2, W = 8; };
template <int N, bool WS>
__global__ __launch_bounds__(64 * Gather<N>::W) void k_obj_gather(const Item* __restrict__ items, const ReqTable reqs,
                                                              const float2* __restrict__ cscr,
                                                              const float* __restrict__ wscr, int step,
                                                              int item_off, int n_items) {
  constexpr int kGatherTY = Gather<N>::TY, kGatherW = Gather<N>::W;
  const ReqDev& r = reqs.r[blockIdx.z];
  const int i = r.S - 1 - step;
  const int x0 = blockIdx.x * 64, y0 = blockIdx.y * kGatherTY;
  if (i < 0 || !r.gobj || x0 >= r.W || y0 >= r.H) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, x = x0 + lane;
  const int lo = max(r.item0, item_off), hi = min(r.item0 + r.n_items, item_off + n_items);
  __shared__ int list[64 * kGatherW];
  __shared__ int wcnt[kGatherW];
  __shared__ float2 part[kGatherW - 1][kGatherTY][64];
  __shared__ float wpart[WS ? kGatherW - 1 : 1][kGatherTY][64];
  float2 acc[kGatherTY];
  float wacc[kGatherTY];
#pragma unroll
  for (int t = 0; t < kGatherTY; ++t) {
    acc[t] = make_float2(0.f, 0.f);
    wacc[t] = 0.f;
  }
  // contribution of position bj to row y0 + t of this thread's column (zero
  // outside its window), and with WS its illumination
  auto fetch = [&](int bj, float2 (&v)[kGatherTY], float (&w)[kGatherTY]) {
    const Item it = items[bj];
    const int wx = x - it.nx;
    const float2* src = cscr + (size_t)bj * N * N;
    const float* wsrc = WS ? wscr + (size_t)bj * N * N : nullptr;
#pragma unroll
    for (int t = 0; t < kGatherTY; ++t) {
      const int wy = y0 + t - it.ny;
      const bool in = wy >= 0 && wy < N && wx >= 0 && wx < N;
      v[t] = in ? src[wy * N + wx] : make_float2(0.f, 0.f);
      if constexpr (WS) w[t] = in ? wsrc[wy * N + wx] : 0.f;
    }
  };
  int total = 0;
  for (int b0 = lo; b0 < hi; b0 += 64 * kGatherW) {
    const int b = b0 + (int)threadIdx.x;
    bool hit = false;
    if (b < hi) {
      const Item it = items[b];
      hit = it.valid && it.ny < y0 + kGatherTY && it.ny + N > y0 && it.nx < x0 + 64 && it.nx + N > x0;
    }
    const unsigned long long m = __ballot(hit);
    if (lane == 0) wcnt[w] = __popcll(m);
    __syncthreads();
    int off = 0, cnt = 0;
#pragma unroll
    for (int q = 0; q < kGatherW; ++q) {
      off += q < w ? wcnt[q] : 0;
      cnt += wcnt[q];
    }
    if (hit) list[off + __popcll(m & ((1ull << lane) - 1ull))] = b;
    __syncthreads();
    total += cnt;
    const int per = (cnt + kGatherW - 1) / kGatherW;
    const int beg = min(w * per, cnt), end = min(beg + per, cnt);
    int k = beg;
    for (; k + 4 <= end; k += 4) {
      float2 v0[kGatherTY], v1[kGatherTY], v2[kGatherTY], v3[kGatherTY];
      float w0[kGatherTY], w1[kGatherTY], w2[kGatherTY], w3[kGatherTY];
      fetch(__builtin_amdgcn_readfirstlane(list[k]), v0, w0);
      fetch(__builtin_amdgcn_readfirstlane(list[k + 1]), v1, w1);
      fetch(__builtin_amdgcn_readfirstlane(list[k + 2]), v2, w2);
      fetch(__builtin_amdgcn_readfirstlane(list[k + 3]), v3, w3);
#pragma unroll
      for (int t = 0; t < kGatherTY; ++t) {
        acc[t] = cadd(cadd(cadd(cadd(acc[t], v0[t]), v1[t]), v2[t]), v3[t]);
        if constexpr (WS) wacc[t] = (((wacc[t] + w0[t]) + w1[t]) + w2[t]) + w3[t];
      }
    }
    for (; k < end; ++k) {
      float2 v0[kGatherTY];
      float w0[kGatherTY];
      fetch(__builtin_amdgcn_readfirstlane(list[k]), v0, w0);
#pragma unroll
      for (int t = 0; t < kGatherTY; ++t) {
        acc[t] = cadd(acc[t], v0[t]);
        if constexpr (WS) wacc[t] += w0[t];
      }
    }
    __syncthreads();   // the list is rebuilt for the next items
  }
  if (total == 0) return;
  if (w > 0) {
#pragma unroll
    for (int t = 0; t < kGatherTY; ++t) {
      part[w - 1][t][lane] = acc[t];
      if constexpr (WS) wpart[w - 1][t][lane] = wacc[t];
    }
  }
  __syncthreads();
  if (w != 0 || x >= r.W) return;
  float2* g = r.gobj + (size_t)i * r.H * r.W;
#pragma unroll
  for (int t = 0; t < kGatherTY; ++t) {
    float2 s = acc[t];
#pragma unroll
    for (int q = 1; q < kGatherW; ++q) s = cadd(s, part[q - 1][t][lane]);
    const int y = y0 + t;
    if (y < r.H) g[(size_t)y * r.W + x] = cadd(g[(size_t)y * r.W + x], s);
  }
  if constexpr (WS) {
    if (!r.wsum) return;
    float* ws = r.wsum + (size_t)i * r.H * r.W;
#pragma unroll
    for (int t = 0; t < kGatherTY; ++t) {
      float s = wacc[t];
#pragma unroll
      for (int q = 1; q < kGatherW; ++q) s += wpart[q - 1][t][lane];
      const int y = y0 + t;
      if (y < r.H) ws[(size_t)y * r.W + x] += s;
    }
  }
}

constexpr int kProbeSplit = 16;
// Probe-spectrum gradient per request: gphat_m(u) = scale * sum_b h_hat_{b,m}(u) conj(R_b(u)).
// A workgroup of PIX x SPLIT threads covers PIX consecutive pixels; thread
// row s sums the items b = item0 + s, s + SPLIT, ... and the rows are added
// in a fixed order (deterministic for a given launch shape).
template <int N, int PIX, int SPLIT>
__global__ __launch_bounds__(PIX * SPLIT) void k_probe_grad(const Item* __restrict__ items, const ReqTable reqs,
                                                            const float2* __restrict__ ws,
                                                            const float2* __restrict__ ramps, float scale) {
  const ReqDev& r = reqs.r[blockIdx.z];
  const int m = blockIdx.y;
  if (m >= r.M || !r.gphat || r.chain_final) return;
  constexpr int split = SPLIT, pix = PIX;
  const int px = threadIdx.x % pix, s = threadIdx.x / pix;
  const int p = blockIdx.x * pix + px;
  const int uy = p / N, ux = p % N;
  auto term = [&](int b) {
    const Item it = items[b];
    if (!it.valid) return make_float2(0.f, 0.f);
    float2 R = cmul(ramps[(size_t)b * 2 * N + uy], ramps[(size_t)b * 2 * N + N + ux]);
    float2 h = ws[(size_t)(it.tile0 + m) * N * N + p];
    return cmul(h, cconj(R));
  };
  if constexpr (SPLIT == 1) {
    // the same summation order as the split form: kProbeSplit interleaved
    // partial sums over the request's items, added in order (so a request's
    // gradient has the same bits whichever form its launch uses)
    float2 part[kProbeSplit];
#pragma unroll
    for (int q = 0; q < kProbeSplit; ++q) part[q] = make_float2(0.f, 0.f);
    for (int b0 = 0; b0 < r.n_items; b0 += kProbeSplit) {
#pragma unroll
      for (int q = 0; q < kProbeSplit; ++q)
        if (b0 + q < r.n_items) part[q] = cadd(part[q], term(r.item0 + b0 + q));
    }
    float2 t = part[0];
#pragma unroll
    for (int q = 1; q < kProbeSplit; ++q) t = cadd(t, part[q]);
    r.gphat[(size_t)m * N * N + p] = cscale(t, adj_scale(r, scale));
  } else {
    static_assert(SPLIT == kProbeSplit, "the split form takes kProbeSplit interleaved partial sums");
    float2 acc = make_float2(0.f, 0.f);
    for (int b = r.item0 + s; b < r.item0 + r.n_items; b += split) acc = cadd(acc, term(b));
    __shared__ float2 red[PIX * SPLIT];
    red[s * pix + px] = acc;
    __syncthreads();
    if (s == 0) {
      float2 t = red[px];
      for (int q = 1; q < split; ++q) t = cadd(t, red[q * pix + px]);
      r.gphat[(size_t)m * N * N + p] = cscale(t, adj_scale(r, scale));
    }
  }
}

// Final column pass and probe-gradient sums in one, for the requests marked
// chain_final. Workgroup (column block, mode, chain), chain = request r and
// residue q < kProbeSplit, walks the request's items q, q + kProbeSplit, ...
// in order: for each it forms h_hat = DFT_y(tile) / N and the block's
// position-gradient partials exactly as COL_FINAL does, and adds
// h_hat conj(R_b) into a sum held in registers. These are k_probe_grad's
// kProbeSplit interleaved sums, added in the same order, so no h_hat tile is
// stored and read back: the chain's sum is stored once, into the column block
// of its first item's tile (that item's work tile is free by then, and no
// other workgroup touches that block), where k_probe_sum adds the chains.
template <int N>
__global__ __launch_bounds__(ColPass<N>::THREADS) void k_col_final_chain(const Item* __restrict__ items,
                                                                 const ReqTable reqs, float2* __restrict__ ws,
                                                                 const float2* __restrict__ ramps,
                                                                 const float2* __restrict__ twg, int step,
                                                                 float* __restrict__ pos_part,
                                                                 unsigned long long colmap) {
  constexpr int L = ColPass<N>::L, E = ColPass<N>::E, CB = ColPass<N>::CB, T = ColPass<N>::THREADS;
  static_assert(T >= N, "the twiddle table takes one entry per thread");
  const int cb = (int)((colmap >> (8 * blockIdx.x)) & 0xffu);
  __shared__ float2 tw[N];
  __shared__ float2 xch[CB * ColMap<N>::STRIDE];
  __shared__ float red[2][T / 64];
  const int rq = blockIdx.z / kProbeSplit, q = blockIdx.z % kProbeSplit, m = blockIdx.y;
  const ReqDev& r = reqs.r[rq];
  if (!r.chain_final || m >= r.M || q >= r.n_items || r.S - 1 - step != 0) return;
  const int t = threadIdx.x;
  if (t < N) tw[t] = twg[t];
  __syncthreads();
  const int c = ColMap<N>::col(), l = ColMap<N>::lane();
  const int ux = cb * CB + c;
  float2* sx = xch + c * ColMap<N>::STRIDE;
  const float2* ph = r.phat + (size_t)m * N * N;
  const float inv = 1.f / (float)N;
  const float fx = (float)((ux < (N + 1) / 2) ? ux : ux - N) / (float)N;
  float2 acc[E];
#pragma unroll
  for (int a = 0; a < E; ++a) acc[a] = make_float2(0.f, 0.f);
  for (int b = r.item0 + q; b < r.item0 + r.n_items; b += kProbeSplit) {
    const Item it = items[b];
    if (!it.valid) {
      // k_probe_grad adds a zero term for a window outside the object
#pragma unroll
      for (int a = 0; a < E; ++a) acc[a] = cadd(acc[a], make_float2(0.f, 0.f));
      continue;
    }
    const float2* tile = ws + (size_t)(it.tile0 + m) * N * N;
    float2 v[E];
#pragma unroll
    for (int a = 0; a < E; ++a) v[a] = tile[(size_t)(l + L * a) * N + ux];
    // (the transform's first barrier also orders the previous item's reads of red)
    line_fft<N, false>(v, l, tw, sx, typename ColMap<N>::Sync{});
    const float2* ry = ramps + (size_t)b * 2 * N;
    const float2 rx = ramps[(size_t)b * 2 * N + N + ux];
    float sy = 0.f, sxx = 0.f;
#pragma unroll
    for (int a = 0; a < E; ++a) {
      const int uy = l + L * a;
      v[a] = cscale(v[a], inv);
      const float2 A = cmul(cmul(ph[(size_t)uy * N + ux], ry[uy]), rx);
      const float2 z = cjmul(v[a], A);          // conj(h_hat) * A
      const float fy = (float)((uy < (N + 1) / 2) ? uy : uy - N) / (float)N;
      sy += fy * z.y;
      sxx += fx * z.y;
      const float2 R = cmul(ry[uy], rx);
      acc[a] = cadd(acc[a], cmul(v[a], cconj(R)));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      sy += __shfl_xor(sy, off);
      sxx += __shfl_xor(sxx, off);
    }
    if ((t & 63) == 0) { red[0][t >> 6] = sy; red[1][t >> 6] = sxx; }
    __syncthreads();
    if (t == 0) {
      float t0 = 0.f, t1 = 0.f;
      for (int w = 0; w < T / 64; ++w) { t0 += red[0][w]; t1 += red[1][w]; }
      float* dst = pos_part + ((size_t)(it.tile0 + m) * ColPass<N>::NBLK + cb) * 2;
      dst[0] = t0;
      dst[1] = t1;
    }
  }
  float2* dst = ws + (size_t)(items[r.item0 + q].tile0 + m) * N * N;
#pragma unroll
  for (int a = 0; a < E; ++a) dst[(size_t)(l + L * a) * N + ux] = acc[a];
}

// Probe-spectrum gradient of the chain_final requests: the kProbeSplit chain
// sums (zero for a residue with no item) added in residue order, as k_probe_grad
// adds its interleaved sums, times the adjoint scale.
template <int N>
__global__ __launch_bounds__(256) void k_probe_sum(const Item* __restrict__ items, const ReqTable reqs,
                                                   const float2* __restrict__ ws, float scale) {
  const ReqDev& r = reqs.r[blockIdx.z];
  const int m = blockIdx.y;
  if (!r.chain_final || m >= r.M || !r.gphat) return;
  const int p = blockIdx.x * 256 + threadIdx.x;
  float2 t = make_float2(0.f, 0.f);
#pragma unroll
  for (int q = 0; q < kProbeSplit; ++q) {
    const float2 part = q < r.n_items ? ws[(size_t)(items[r.item0 + q].tile0 + m) * N * N + p]
                                      : make_float2(0.f, 0.f);
    t = q == 0 ? part : cadd(t, part);
  }
  r.gphat[(size_t)m * N * N + p] = cscale(t, adj_scale(r, scale));
}

// Per item: dL/dX = 2 pi * scale * sum over modes and blocks of the partials;
// written to g_pos[local] (per batch entry) and/or added to a dense [J][2] gradient.
__global__ void k_pos_reduce(const Item* __restrict__ items, const ReqTable reqs,
                             const float* __restrict__ pos_part, int nblk, int n_items, float scale) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_items) return;
  const Item it = items[b];
  const ReqDev& r = reqs.r[it.req];
  float g0 = 0.f, g1 = 0.f;
  if (it.valid) {
    for (int m = 0; m < r.M; ++m)
      for (int k = 0; k < nblk; ++k) {
        const float* p = pos_part + ((size_t)(it.tile0 + m) * nblk + k) * 2;
        g0 += p[0];
        g1 += p[1];
      }
  }
  const float f = 6.283185307179586f * adj_scale(r, scale);
  g0 *= f;
  g1 *= f;
  int local = b - r.item0;
  if (r.gpos) {
    if (r.accumulate) { r.gpos[2 * local] += g0; r.gpos[2 * local + 1] += g1; }
    else { r.gpos[2 * local] = g0; r.gpos[2 * local + 1] = g1; }
  }
  if (r.gpos_dense && it.valid) {
    atomicAdd(r.gpos_dense + 2 * it.j, g0);
    atomicAdd(r.gpos_dense + 2 * it.j + 1, g1);
  }
}

// ============================================================ elementwise

__global__ void k_fill(float* __restrict__ p, size_t n, float v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void k_sgd(float* __restrict__ th, const float* __restrict__ g, size_t n, float lr) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) th[i] -= lr * g[i];
}

// Adam per real component: m = b1 m + (1-b1) g ; v = b2 v + (1-b2) g^2 ;
// th -= step_size * m / (sqrt(v) * inv_sqrt_bc2 + eps), step_size = lr / (1 - b1^t).
// The complements c1 = 1 - b1 and c2 = 1 - b2 come from the host, formed in
// double: 1 - 0.999f in float would be off by 1.3e-5 relative.
__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ mo,
                       float* __restrict__ ve, size_t n, float step_size, float inv_sqrt_bc2, float b1,
                       float c1, float b2, float c2, float eps) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    float gi = g[i];
    float m = b1 * mo[i] + c1 * gi;
    float v = b2 * ve[i] + c2 * gi * gi;
    mo[i] = m;
    ve[i] = v;
    th[i] -= step_size * m / (sqrtf(v) * inv_sqrt_bc2 + eps);
  }
}

// Adam with the step count on the device: one thread per workgroup forms the
// step's factors from t = *step_dev + 1 (the value the whole step reads; the
// step advances it after its last update).
__global__ void k_adam_dev(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ mo,
                           float* __restrict__ ve, size_t n, double lr, const int64_t* __restrict__ step_dev,
                           double b1d, double b2d, float eps) {
  __shared__ float fac[2];
  if (threadIdx.x == 0) {
    const AdamFactors f = adam_factors(lr, b1d, b2d, *step_dev + 1);
    fac[0] = f.step_size;
    fac[1] = f.inv_sqrt_bc2;
  }
  __syncthreads();
  const float step_size = fac[0], inv_sqrt_bc2 = fac[1];
  const float b1 = (float)b1d, c1 = (float)(1.0 - b1d), b2 = (float)b2d, c2 = (float)(1.0 - b2d);
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    float gi = g[i];
    float m = b1 * mo[i] + c1 * gi;
    float v = b2 * ve[i] + c2 * gi * gi;
    mo[i] = m;
    ve[i] = v;
    th[i] -= step_size * m / (sqrtf(v) * inv_sqrt_bc2 + eps);
  }
}

__global__ void k_step_advance(int64_t* step_dev) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step_dev += 1;
}

// ============================================================ launchers

static inline dim3 grid1(size_t n) {
  size_t b = (n + kThreads - 1) / kThreads;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return dim3((unsigned)b);
}

template <int N>
struct Launch {
  template <bool HALF>
  static void rows_fwd_t(const LaunchCtx& L, int step, PsiStore st, bool from_real) {
    dim3 g(Pass<N>::NBLK, L.n_items);
    if (from_real)
      hipLaunchKernelGGL((k_row_fwd<N, true, HALF>), g, dim3(kThreads), 0, L.stream, L.items, L.reqs, L.ws, L.ck, L.tw, step, st, L.item_off);
    else if (L.emax)
      hipLaunchKernelGGL((k_row_fwd<N, false, HALF, true>), g, dim3(kThreads), 0, L.stream, L.items, L.reqs, L.ws, L.ck, L.tw, step, st, L.item_off);
    else
      hipLaunchKernelGGL((k_row_fwd<N, false, HALF>), g, dim3(kThreads), 0, L.stream, L.items, L.reqs, L.ws, L.ck, L.tw, step, st, L.item_off);
  }
  static void rows_fwd(const LaunchCtx& L, int step, PsiStore st, bool from_real) {
    if (L.ck_half) rows_fwd_t<true>(L, step, st, from_real);
    else rows_fwd_t<false>(L, step, st, from_real);
  }
  static void rows_adj(const LaunchCtx& L, int step, PsiLoad psi, float scale) {
    dim3 g(Pass<N>::NBLK, L.n_items);
    if (psi.spec) {
      if (L.wsum)
        hipLaunchKernelGGL((k_row_adj<N, false, true, true>), g, dim3(kThreads), 0, L.stream, L.items, L.reqs, L.ws, L.ck, L.tw, step, psi, scale, L.item_off, L.cscr, L.wscr);
      else
        hipLaunchKernelGGL((k_row_adj<N, false, false, true>), g, dim3(kThreads), 0, L.stream, L.items, L.reqs, L.ws, L.ck, L.tw, step, psi, scale, L.item_off, L.cscr, L.wscr);
      return;
    }
    if (L.wsum) {
      if (L.ck_half)
        hipLaunchKernelGGL((k_row_adj<N, true, true>), g, dim3(kThreads), 0, L.stream, L.items, L.reqs, L.ws, L.ck, L.tw, step, psi, scale, L.item_off, L.cscr, L.wscr);
      else
        hipLaunchKernelGGL((k_row_adj<N, false, true>), g, dim3(kThreads), 0, L.stream, L.items, L.reqs, L.ws, L.ck, L.tw, step, psi, scale, L.item_off, L.cscr, L.wscr);
    } else if (L.ck_half) {
      hipLaunchKernelGGL((k_row_adj<N, true>), g, dim3(kThreads), 0, L.stream, L.items, L.reqs, L.ws, L.ck, L.tw, step, psi, scale, L.item_off, L.cscr, L.wscr);
    } else {
      hipLaunchKernelGGL((k_row_adj<N, false>), g, dim3(kThreads), 0, L.stream, L.items, L.reqs, L.ws, L.ck, L.tw, step, psi, scale, L.item_off, L.cscr, L.wscr);
    }
  }
  static void col(const LaunchCtx& L, int op, int step) {
    // A propagation pass runs only the column blocks holding a live column,
    // listed one after the other in blockIdx.x: consecutive workgroups go to
    // the XCDs in turn, so every XCD gets an equal share of the live blocks
    // (with the whole range, block q would always land on XCD q).
    const unsigned live = (op == COL_PROP || op == COL_PROP_ADJ) ? L.col_live_blocks : 0u;
    unsigned long long map = 0;
    int nb = 0;
    for (int q = 0; q < ColPass<N>::NBLK; ++q)
      if (!live || ((live >> q) & 1u)) map |= (unsigned long long)q << (8 * nb++);
    if (nb == 0) return;
    // item by item (all modes of an item together), in item order, the
    // reverse of the row passes around it: each pass starts on the tiles
    // the previous pass wrote last, which the memory-side cache still holds
    dim3 g(nb, L.max_modes, L.n_items);
    float2* ck_out = L.ck_spec ? static_cast<float2*>(L.ck) : nullptr;
    switch (op) {
      case COL_SHIFT: hipLaunchKernelGGL((k_col<N, COL_SHIFT>), g, dim3(ColPass<N>::THREADS), 0, L.stream, L.items, L.reqs, L.ws, L.ramps, L.tw, step, L.pos_part, L.item_off, ck_out, map, L.seg_out); break;
      case COL_PROP: hipLaunchKernelGGL((k_col<N, COL_PROP>), g, dim3(ColPass<N>::THREADS), 0, L.stream, L.items, L.reqs, L.ws, L.ramps, L.tw, step, L.pos_part, L.item_off, ck_out, map, L.seg_out); break;
      case COL_PROP_ADJ: hipLaunchKernelGGL((k_col<N, COL_PROP_ADJ>), g, dim3(ColPass<N>::THREADS), 0, L.stream, L.items, L.reqs, L.ws, L.ramps, L.tw, step, L.pos_part, L.item_off, nullptr, map, L.seg_out); break;
      default: {
        bool any_chain = false, any_plain = false;
        for (int q = 0; q < L.n_reqs; ++q) (L.reqs.r[q].chain_final ? any_chain : any_plain) = true;
        if (any_plain)
          hipLaunchKernelGGL((k_col<N, COL_FINAL>), g, dim3(ColPass<N>::THREADS), 0, L.stream, L.items, L.reqs, L.ws, L.ramps, L.tw, step, L.pos_part, L.item_off, nullptr, map, L.seg_out);
        if (any_chain)
          hipLaunchKernelGGL((k_col_final_chain<N>), dim3(nb, L.max_modes, L.n_reqs * kProbeSplit), dim3(ColPass<N>::THREADS), 0, L.stream, L.items, L.reqs, L.ws, L.ramps, L.tw, step, L.pos_part, map);
        break;
      }
    }
  }
  static void obj_gather(const LaunchCtx& L, int step, int max_h, int max_w) {
    constexpr int TY = Gather<N>::TY, W = Gather<N>::W;
    dim3 g((max_w + 63) / 64, (max_h + TY - 1) / TY, L.n_reqs);
    if (L.wsum && L.wscr)
      hipLaunchKernelGGL((k_obj_gather<N, true>), g, dim3(64 * W), 0, L.stream, L.items, L.reqs, L.cscr,
                         L.wscr, step, L.item_off, L.n_items);
    else
      hipLaunchKernelGGL((k_obj_gather<N, false>), g, dim3(64 * W), 0, L.stream, L.items, L.reqs, L.cscr,
                         nullptr, step, L.item_off, L.n_items);
  }
  static void far_loss(const LaunchCtx& L, int step, bool grad) {
    dim3 g(ColPass<N>::NBLK, L.n_items);
    if (grad)
      hipLaunchKernelGGL((k_far_loss<N, true>), g, dim3(ColPass<N>::THREADS), 0, L.stream, L.items, L.reqs, L.ws, L.tw, step, L.loss_part, L.flags, L.item_off);
    else
      hipLaunchKernelGGL((k_far_loss<N, false>), g, dim3(ColPass<N>::THREADS), 0, L.stream, L.items, L.reqs, L.ws, L.tw, step, L.loss_part, L.flags, L.item_off);
  }
  static void probe_grad(const LaunchCtx& L, float scale) {
    // many (pixel block, mode) pairs: 256 pixels per workgroup, every thread
    // walks all items; few: 64 pixels per workgroup and the items split 16 ways
    static_assert((N * N) % 256 == 0, "pixel blocks must tile the probe");
    bool any_chain = false, any_plain = false;
    for (int q = 0; q < L.n_reqs; ++q) (L.reqs.r[q].chain_final ? any_chain : any_plain) = true;
    if (any_chain)
      hipLaunchKernelGGL((k_probe_sum<N>), dim3(N * N / 256, L.max_modes, L.n_reqs), dim3(256), 0, L.stream,
                         L.items, L.reqs, L.ws, scale);
    if (!any_plain) return;
    const bool small = (N * N / 256) * L.max_modes * L.n_reqs < 1024;
    if (small)
      hipLaunchKernelGGL((k_probe_grad<N, 64, kProbeSplit>), dim3(N * N / 64, L.max_modes, L.n_reqs), dim3(1024), 0, L.stream,
                         L.items, L.reqs, L.ws, L.ramps, scale);
    else
      hipLaunchKernelGGL((k_probe_grad<N, 256, 1>), dim3(N * N / 256, L.max_modes, L.n_reqs), dim3(256), 0, L.stream,
                         L.items, L.reqs, L.ws, L.ramps, scale);
  }
  static void plain2d(hipStream_t s, const float2* tw, const float2* src, float2* dst, int n_tiles, bool inverse,
                      float scale, bool accumulate) {
    // forward: rows then columns ; inverse: columns then rows (in place on dst)
    dim3 gr(Pass<N>::NBLK, n_tiles), gc(ColPass<N>::NBLK, n_tiles);
    if (!inverse) {
      hipLaunchKernelGGL((k_row_plain<N, false>), gr, dim3(kThreads), 0, s, src, dst, tw, 1.f, 0);
      hipLaunchKernelGGL((k_col_plain<N, false>), gc, dim3(ColPass<N>::THREADS), 0, s, dst, tw, scale);
    } else {
      // columns in place on a copy living in dst is not possible when accumulating:
      // the caller passes src as scratch that may be overwritten.
      hipLaunchKernelGGL((k_col_plain<N, true>), gc, dim3(ColPass<N>::THREADS), 0, s, const_cast<float2*>(src), tw, scale);
      hipLaunchKernelGGL((k_row_plain<N, true>), gr, dim3(kThreads), 0, s, src, dst, tw, 1.f, accumulate ? 1 : 0);
    }
  }
};

void launch_items(const LaunchCtx& L, int N) {
  hipLaunchKernelGGL(k_items, dim3(L.n_items), dim3(64), 0, L.stream, L.reqs, L.n_reqs, L.items, L.ramps,
                     L.n_items, N, L.flags);
}

#define PTY_DISPATCH(N, CALL)                    \
  switch (N) {                                   \
    case 64: Launch<64>::CALL; break;            \
    case 128: Launch<128>::CALL; break;          \
    case 192: Launch<192>::CALL; break;          \
    default: Launch<256>::CALL; break;           \
  }

void launch_rows_fwd(const LaunchCtx& L, int N, int step, PsiStore st, bool from_real) {
  PTY_DISPATCH(N, rows_fwd(L, step, st, from_real));
}
void launch_rows_adj(const LaunchCtx& L, int N, int step, PsiLoad psi, float scale) {
  PTY_DISPATCH(N, rows_adj(L, step, psi, scale));
}
void launch_col(const LaunchCtx& L, int N, int op, int step) { PTY_DISPATCH(N, col(L, op, step)); }
void launch_obj_gather(const LaunchCtx& L, int N, int step, int max_h, int max_w) {
  PTY_DISPATCH(N, obj_gather(L, step, max_h, max_w));
}
void launch_far_loss(const LaunchCtx& L, int N, int step, bool grad) { PTY_DISPATCH(N, far_loss(L, step, grad)); }
void launch_probe_grad(const LaunchCtx& L, int N, float scale) { PTY_DISPATCH(N, probe_grad(L, scale)); }
void set_chain_final(LaunchCtx& L, int N, bool unchunked) {
  // Chains where they measured faster: N = 256 (16 values per lane; at 24 per
  // lane, N = 192, the chain kernel runs one wave per SIMD and loses) with
  // enough (column block, mode, chain) workgroups to cover the CUs (one
  // 512-thread workgroup per CU at its register count). Decided per request,
  // so a request takes the same path alone or in a shared launch.
  for (int q = 0; q < L.n_reqs; ++q)
    L.reqs.r[q].chain_final =
        (unchunked && N == 256 && col_blocks(N) * L.reqs.r[q].M * kProbeSplit >= 512) ? 1 : 0;
}
void launch_plain2d(int N, hipStream_t s, const float2* tw, const float2* src, float2* dst, int n_tiles,
                    bool inverse, float scale, bool accumulate) {
  PTY_DISPATCH(N, plain2d(s, tw, src, dst, n_tiles, inverse, scale, accumulate));
}
void launch_loss_reduce(const LaunchCtx& L, int N) {
  hipLaunchKernelGGL(k_loss_reduce, dim3(L.n_reqs), dim3(kThreads), 0, L.stream, L.reqs, L.loss_part,
                     col_blocks(N));
}
void launch_pos_reduce(const LaunchCtx& L, int N, float scale) {
  hipLaunchKernelGGL(k_pos_reduce, dim3((L.n_items + 127) / 128), dim3(128), 0, L.stream, L.items, L.reqs,
                     L.pos_part, col_blocks(N), L.n_items, scale);
}
void launch_fill(hipStream_t s, float* p, size_t n, float v) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill, grid1(n), dim3(kThreads), 0, s, p, n, v);
}
void launch_sgd(hipStream_t s, float* th, const float* g, size_t n, float lr) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_sgd, grid1(n), dim3(kThreads), 0, s, th, g, n, lr);
}
void launch_adam(hipStream_t s, float* th, const float* g, float* m, float* v, size_t n, float step_size,
                 float inv_sqrt_bc2, double b1, double b2, float eps) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_adam, grid1(n), dim3(kThreads), 0, s, th, g, m, v, n, step_size, inv_sqrt_bc2, (float)b1,
                     (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), eps);
}
void launch_adam_dev(hipStream_t s, float* th, const float* g, float* m, float* v, size_t n, double lr,
                     const int64_t* step_dev, double b1, double b2, float eps) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_adam_dev, grid1(n), dim3(kThreads), 0, s, th, g, m, v, n, lr, step_dev, b1, b2, eps);
}
void launch_step_advance(hipStream_t s, int64_t* step_dev) {
  hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, s, step_dev);
}
int col_blocks(int N) {
  return N == 256 ? ColPass<256>::NBLK : N == 192 ? ColPass<192>::NBLK : N == 128 ? ColPass<128>::NBLK : ColPass<64>::NBLK;
}

}  // namespace pty

namespace pty {

// ============================================================ regularization (Sec. 3.4)
//
// Cost regularizers on the object [S][H][W]: one thread per element adds the
// gradient of every enabled term to g (dR/dRe + i dR/dIm) and accumulates
// the cost of the forward differences it owns (to y+1, x+1, i+1), so that
// each difference is counted once. phi(z) = sqrt(|z|^2 + delta^2).
__device__ __forceinline__ float2 tv_grad(float2 z, float d2) {
  return cscale(z, rsqrtf(cabs2(z) + d2));
}

__global__ void k_reg_object(const float2* __restrict__ O, float2* __restrict__ g, int S, int H, int W,
                             RegDev rg, float* __restrict__ cost_part) {
  __shared__ float red[kThreads / 64];
  const size_t n = (size_t)S * H * W;
  float cost = 0.f;
  const float d2 = rg.tv_delta * rg.tv_delta;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(e % W);
    const int y = (int)((e / W) % H);
    const int i = (int)(e / ((size_t)W * H));
    const float2 o = O[e];
    float2 gr = make_float2(0.f, 0.f);
    if (rg.obj_l2 != 0.f) {
      float2 d = make_float2(o.x - 1.f, o.y);
      gr = cadd(gr, cscale(d, 2.f * rg.obj_l2));
      cost += rg.obj_l2 * cabs2(d);
    }
    if (rg.obj_l1 != 0.f) {
      // the unit vector (O - 1) / |O - 1|, formed without squaring (no underflow)
      float2 d = make_float2(o.x - 1.f, o.y);
      float a = hypotf(d.x, d.y);
      if (a > 0.f) gr = cadd(gr, cscale(make_float2(d.x / a, d.y / a), rg.obj_l1));
      cost += rg.obj_l1 * a;
    }
    if (rg.obj_phase_l1 != 0.f) {
      // |arg O|: d arg O / d(Re, Im), combined as dRe + i dIm, is i O / |O|^2,
      // formed as (i O / |O|) / |O| so that it overflows only where its value
      // exceeds the float range (|O|^2 itself underflows much earlier)
      const float ph = atan2f(o.y, o.x);
      const float a = hypotf(o.x, o.y);
      cost += rg.obj_phase_l1 * fabsf(ph);
      if (ph != 0.f && a > 0.f) {
        const float sc = (ph > 0.f ? rg.obj_phase_l1 : -rg.obj_phase_l1) / a;
        gr = cadd(gr, make_float2(-(o.y / a) * sc, (o.x / a) * sc));
      }
    }
    const bool in_tik = rg.obj_tikhonov != 0.f, in_tv = rg.obj_tv != 0.f;
    const bool z_tik = rg.layers_tikhonov != 0.f, z_tv = rg.layers_tv != 0.f;
    // neighbours along each axis: (stride, has_prev, has_next, weight_tik, weight_tv)
    const size_t strides[3] = {(size_t)W, (size_t)1, (size_t)W * H};
    const bool prev[3] = {y > 0, x > 0, i > 0};
    const bool next[3] = {y + 1 < H, x + 1 < W, i + 1 < S};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const float wt = ax < 2 ? (in_tik ? rg.obj_tikhonov : 0.f) : (z_tik ? rg.layers_tikhonov : 0.f);
      const float wv = ax < 2 ? (in_tv ? rg.obj_tv : 0.f) : (z_tv ? rg.layers_tv : 0.f);
      if (wt == 0.f && wv == 0.f) continue;
      if (prev[ax]) {           // difference D = o - O[prev] enters with +
        float2 D = csub(o, O[e - strides[ax]]);
        if (wt != 0.f) gr = cadd(gr, cscale(D, 2.f * wt));
        if (wv != 0.f) gr = cadd(gr, cscale(tv_grad(D, d2), wv));
      }
      if (next[ax]) {           // difference D = O[next] - o enters with -
        float2 D = csub(O[e + strides[ax]], o);
        if (wt != 0.f) { gr = csub(gr, cscale(D, 2.f * wt)); cost += wt * cabs2(D); }
        if (wv != 0.f) { gr = csub(gr, cscale(tv_grad(D, d2), wv)); cost += wv * sqrtf(cabs2(D) + d2); }
      }
    }
    g[e] = cadd(g[e], gr);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) cost += __shfl_xor(cost, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cost;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int w = 0; w < kThreads / 64; ++w) t += red[w];
    cost_part[blockIdx.x] = t;
  }
}

// Probe L2: g += 2 w P, cost w |P|^2.
__global__ void k_reg_probe(const float2* __restrict__ P, float2* __restrict__ g, size_t n, float w,
                            float* __restrict__ cost_part) {
  __shared__ float red[kThreads / 64];
  float cost = 0.f;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const float2 p = P[e];
    g[e] = cadd(g[e], cscale(p, 2.f * w));
    cost += w * cabs2(p);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) cost += __shfl_xor(cost, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cost;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int w2 = 0; w2 < kThreads / 64; ++w2) t += red[w2];
    cost_part[blockIdx.x] = t;
  }
}

// Probe phase plate (Tikhonov weight wt, TV weight wv) on the unitary spectra
// phat [M][N][N] in FFT order. Centred, frequency index u sits at c = (u + N/2)
// mod N, so the centred neighbours of u are u - 1 and u + 1 (mod N) except
// across the centred array's ends (u = N/2 has no lower neighbour, u = N/2 - 1
// no upper one). A pair (a, b) of neighbours, a the upper one, has
// z = a conj(b) = r e^{it} and cost r^2 t^2 (Tikhonov) or r^2 sqrt(t^2 + d^2)
// (TV): phase steps weighted by the two frequencies' intensities. For a cost
// f(r) h(t) the gradient with respect to z is e^{it} (f' h + i f h' / r), with
// f = r^2 that is G = z (2h + i h'): 2 z (t^2 + it) and z (2q + it/q),
// q = sqrt(t^2 + d^2), which vanishes continuously as z -> 0 (so a dark
// frequency next to a lit one, whose phase is rounding noise, contributes
// nothing); then dC/da = G b and dC/db = conj(G) a. One thread per pixel
// gathers the terms of its (up to four) pairs into gphat and counts the cost
// of the pairs where it is the upper element, so each pair is counted once.
__device__ __forceinline__ float2 phase_pair_grad(float2 z, float wt, float wv, float d2, float& cost) {
  const float r2 = cabs2(z);
  const float t = atan2f(z.y, z.x);
  float2 G = make_float2(0.f, 0.f);
  if (wt != 0.f) {
    cost += wt * r2 * t * t;
    G = cadd(G, cscale(cmul(z, make_float2(2.f * t * t, 2.f * t)), wt));
  }
  if (wv != 0.f) {
    const float q = sqrtf(t * t + d2);
    cost += wv * r2 * q;
    G = cadd(G, cscale(cmul(z, make_float2(2.f * q, t / q)), wv));
  }
  return G;
}

__global__ void k_reg_probe_phase(const float2* __restrict__ phat, float2* __restrict__ gphat, int M, int N,
                                  float wt, float wv, float d2, float* __restrict__ cost_part) {
  __shared__ float red[kThreads / 64];
  const size_t N2 = (size_t)N * N, n = (size_t)M * N2;
  float cost = 0.f;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const size_t base = e - e % N2;
    const int uy = (int)((e % N2) / N), ux = (int)(e % N);
    const float2 a = phat[e];
    float2 g = make_float2(0.f, 0.f);
    float c_own = 0.f, c_other = 0.f;
    const int h = N / 2;
    // neighbours along y then x: lower (this pixel is the upper element), upper
    const int lo_y = (uy + N - 1) % N, hi_y = (uy + 1) % N, lo_x = (ux + N - 1) % N, hi_x = (ux + 1) % N;
    if (uy != h) {
      const float2 b = phat[base + (size_t)lo_y * N + ux];
      g = cadd(g, cmul(phase_pair_grad(cjmul(b, a), wt, wv, d2, c_own), b));
    }
    if (uy != h - 1) {
      const float2 c = phat[base + (size_t)hi_y * N + ux];
      g = cadd(g, cmul(cconj(phase_pair_grad(cjmul(a, c), wt, wv, d2, c_other)), c));
    }
    if (ux != h) {
      const float2 b = phat[base + (size_t)uy * N + lo_x];
      g = cadd(g, cmul(phase_pair_grad(cjmul(b, a), wt, wv, d2, c_own), b));
    }
    if (ux != h - 1) {
      const float2 c = phat[base + (size_t)uy * N + hi_x];
      g = cadd(g, cmul(cconj(phase_pair_grad(cjmul(a, c), wt, wv, d2, c_other)), c));
    }
    gphat[e] = g;
    cost += c_own;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) cost += __shfl_xor(cost, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cost;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int w2 = 0; w2 < kThreads / 64; ++w2) t += red[w2];
    cost_part[blockIdx.x] = t;
  }
}

// Spectral L1 of the object, between the two FFTs of the slices: spec holds
// the unnormalised DFT of every H x W slice; with the unitary spectrum
// F = spec / sqrt(HW), the cost is w |F| summed over every frequency but the
// zero one, and spec is replaced by w F / |F| / sqrt(HW) (0 at the zero
// frequency and where F = 0), whose unnormalised inverse DFT is the
// gradient w F2^H(F / |F|).
__global__ void k_spec_l1(float2* __restrict__ spec, size_t n, size_t HW, float w, float inv_sqrt,
                          float* __restrict__ cost_part) {
  __shared__ float red[kThreads / 64];
  float cost = 0.f;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const float2 F = cscale(spec[e], inv_sqrt);
    const float a = hypotf(F.x, F.y);
    float2 g = make_float2(0.f, 0.f);
    if (e % HW != 0 && a > 0.f) {
      cost += w * a;
      g = cscale(make_float2(F.x / a, F.y / a), w * inv_sqrt);
    }
    spec[e] = g;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) cost += __shfl_xor(cost, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cost;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int w2 = 0; w2 < kThreads / 64; ++w2) t += red[w2];
    cost_part[blockIdx.x] = t;
  }
}

// g += a (complex, n values).
__global__ void k_cadd_inplace(float2* __restrict__ g, const float2* __restrict__ a, size_t n) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    g[e] = cadd(g[e], a[e]);
}

// loss += sum of the cost partials (double), one block.
__global__ void k_add_cost(const float* __restrict__ part, int n, double* __restrict__ loss) {
  __shared__ double red[kThreads];
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) s += (double)part[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss += red[0];
}

// Object amplitude range: O <- O * clip(|O|, lo, hi) / |O| (|O| = 0 -> lo).
__global__ void k_amp_clamp(float2* __restrict__ O, size_t n, float lo, float hi) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    float2 o = O[e];
    float a = hypotf(o.x, o.y);
    float c = fminf(fmaxf(a, lo), hi);
    O[e] = a > 0.f ? cscale(make_float2(o.x / a, o.y / a), c) : make_float2(c, 0.f);
  }
}

// Gaussian depth blur per pixel column, normalised, truncated at radius r.
__global__ void k_layer_blur(float2* __restrict__ O, int S, size_t HW, const float* __restrict__ g, int r) {
  for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < HW; p += (size_t)gridDim.x * blockDim.x) {
    float2 col[kMaxBlurSlices];
    for (int i = 0; i < S; ++i) col[i] = O[(size_t)i * HW + p];
    for (int i = 0; i < S; ++i) {
      float2 acc = make_float2(0.f, 0.f);
      float den = 0.f;
      const int j0 = i - r < 0 ? 0 : i - r, j1 = i + r + 1 > S ? S : i + r + 1;
      for (int j = j0; j < j1; ++j) {
        const float w = g[i - j < 0 ? j - i : i - j];
        acc = cadd(acc, cscale(col[j], w));
        den += w;
      }
      O[(size_t)i * HW + p] = cscale(acc, 1.f / den);
    }
  }
}

// In-plane Gaussian low pass, one axis at a time (AXIS 0: along x, AXIS 1:
// along y) with periodic boundaries: dst[s][y][x] = sum_{t=-r..r} w[|t|] *
// src[s][y][x + t] (or src[s][y + t][x]), indices wrapped. w is normalised
// over the 2r + 1 taps.
template <int AXIS>
__global__ void k_lowpass(const float2* __restrict__ src, float2* __restrict__ dst, int S, int H, int W,
                          const float* __restrict__ w, int r) {
  const size_t n = (size_t)S * H * W;
  const int len = AXIS == 0 ? W : H;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(e % W);
    const size_t row = e / W;                      // s * H + y
    const int y = (int)(row % H);
    const int at = AXIS == 0 ? x : y;
    int q = (at - r) % len;
    if (q < 0) q += len;
    const float2* base = AXIS == 0 ? src + row * W : src + (row - y) * W + x;
    const size_t step = AXIS == 0 ? 1 : (size_t)W;
    float2 acc = make_float2(0.f, 0.f);
    for (int t = -r; t <= r; ++t) {
      acc = cadd(acc, cscale(base[q * step], w[t < 0 ? -t : t]));
      if (++q == len) q = 0;
    }
    dst[e] = acc;
  }
}

// Phase deramp sums of one slice per blockIdx.y, reduced in double.
// PHASE 0: part = (sum O(y,x+1) conj O(y,x), sum O(y+1,x) conj O(y,x)) as
// (re, im, re, im); PHASE 1: part = sum O(y,x) exp(-i(ty y + tx x)) with
// (ty, tx) = theta[s][1..2].
template <int PHASE>
__global__ __launch_bounds__(kThreads) void k_deramp_sums(const float2* __restrict__ O, int H, int W,
                                                           const double* __restrict__ theta,
                                                           double* __restrict__ part) {
  const int s = blockIdx.y;
  const size_t HW = (size_t)H * W;
  const float2* Os = O + s * HW;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  const double ty = PHASE ? theta[s * 3 + 1] : 0.0, tx = PHASE ? theta[s * 3 + 2] : 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < HW; e += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(e % W), y = (int)(e / W);
    const float2 o = Os[e];
    if (PHASE == 0) {
      if (x + 1 < W) {
        const float2 q = Os[e + 1];
        a[0] += (double)q.x * o.x + (double)q.y * o.y;
        a[1] += (double)q.y * o.x - (double)q.x * o.y;
      }
      if (y + 1 < H) {
        const float2 q = Os[e + W];
        a[2] += (double)q.x * o.x + (double)q.y * o.y;
        a[3] += (double)q.y * o.x - (double)q.x * o.y;
      }
    } else {
      double ph = ty * y + tx * x;
      ph -= 6.283185307179586 * rint(ph * 0.15915494309189535);
      float sn, cs;
      sincosf((float)ph, &sn, &cs);
      a[0] += (double)o.x * cs + (double)o.y * sn;     // o * exp(-i ph)
      a[1] += (double)o.y * cs - (double)o.x * sn;
    }
  }
  __shared__ double red[4][kThreads / 64];
  for (int c = 0; c < 4; ++c) {
    double v = a[c];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double t = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) t += red[threadIdx.x][w];
    part[((size_t)s * gridDim.x + blockIdx.x) * 4 + threadIdx.x] = t;
  }
}

// One block per slice: sum the partials of k_deramp_sums and store the
// angles: PHASE 0 theta[s][1] = arg(vertical pair sum), theta[s][2] =
// arg(horizontal pair sum); PHASE 1 theta[s][0] = arg(de-ramped slice sum).
template <int PHASE>
__global__ __launch_bounds__(kThreads) void k_deramp_angles(const double* __restrict__ part, int nblk,
                                                             double* __restrict__ theta) {
  const int s = blockIdx.x;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += kThreads)
    for (int c = 0; c < 4; ++c) a[c] += part[((size_t)s * nblk + b) * 4 + c];
  __shared__ double red[4][kThreads / 64];
  for (int c = 0; c < 4; ++c) {
    double v = a[c];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < 4; ++c)
      for (int w = 0; w < kThreads / 64; ++w) t[c] += red[c][w];
    if (PHASE == 0) {
      theta[s * 3 + 1] = atan2(t[3], t[2]);
      theta[s * 3 + 2] = atan2(t[1], t[0]);
    } else {
      theta[s * 3 + 0] = atan2(t[1], t[0]);
    }
  }
}

// O[s][y][x] *= exp(-i (theta0 + ty y + tx x)).
__global__ void k_deramp_apply(float2* __restrict__ O, int S, int H, int W, const double* __restrict__ theta) {
  const size_t HW = (size_t)H * W, n = HW * S;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int s = (int)(e / HW);
    const size_t p = e % HW;
    const int x = (int)(p % W), y = (int)(p / W);
    double ph = theta[s * 3] + theta[s * 3 + 1] * y + theta[s * 3 + 2] * x;
    ph -= 6.283185307179586 * rint(ph * 0.15915494309189535);
    float sn, cs;
    sincosf((float)ph, &sn, &cs);
    const float2 o = O[e];
    O[e] = make_float2(o.x * cs + o.y * sn, o.y * cs - o.x * sn);
  }
}

// ------------------------------------------------------------ LSQML (Sec. 3.3)

// Transparency of the object stack per object pixel: tau(x) = prod_i |O_i(x)|^2
// (slices multiplied in order).
__global__ void k_lsq_tau(const float2* __restrict__ O, int S, size_t HW, float* __restrict__ tau) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < HW; e += (size_t)gridDim.x * blockDim.x) {
    float t = 1.f;
    for (int i = 0; i < S; ++i) t *= cabs2(O[(size_t)i * HW + e]);
    tau[e] = t;
  }
}

// Transparency in the probe view, partial sums over the items b = split,
// split + kLsqSplit, ...: part[split][r] = sum_b tau(n_b + r).
__global__ __launch_bounds__(kThreads) void k_lsq_transp(const Item* __restrict__ items, int n_items,
                                                          const float* __restrict__ tau, int W, int N,
                                                          float* __restrict__ part) {
  const int r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= N * N) return;
  const int ry = r / N, rx = r % N;
  float acc = 0.f;
  for (int b = blockIdx.y; b < n_items; b += kLsqSplit) {
    const Item it = items[b];
    if (!it.valid) continue;
    acc += tau[(size_t)(it.ny + ry) * W + it.nx + rx];
  }
  part[(size_t)blockIdx.y * N * N + r] = acc;
}

__global__ __launch_bounds__(kThreads) void k_lsq_transp_sum(const float* __restrict__ part, int N2,
                                                              float* __restrict__ wp) {
  const int r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= N2) return;
  float acc = 0.f;
  for (int q = 0; q < kLsqSplit; ++q) acc += part[(size_t)q * N2 + r];
  wp[r] = acc;
}

// Per-slice maximum of the illumination sum in use, A = prev or cur + w:
// partial maxima per block (grid nb x S), then one block per slice.
__global__ __launch_bounds__(kThreads) void k_lsq_obj_pmax(const float* __restrict__ w, const float* __restrict__ cur,
                                                            const float* __restrict__ prev, size_t HW,
                                                            double* __restrict__ pmax) {
  const size_t base = (size_t)blockIdx.y * HW;
  float mx = 0.f;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < HW; e += (size_t)gridDim.x * blockDim.x) {
    const size_t q = base + e;
    mx = fmaxf(mx, prev ? prev[q] : cur[q] + w[q]);
  }
  __shared__ float red[kThreads / 64];
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 1; v < kThreads / 64; ++v) mx = fmaxf(mx, red[v]);
    pmax[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = mx;
  }
}

__global__ __launch_bounds__(kThreads) void k_lsq_obj_amax(const double* __restrict__ pmax, int nblk,
                                                            double* __restrict__ amax) {
  double mx = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kThreads) mx = fmax(mx, pmax[(size_t)blockIdx.x * nblk + b]);
  __shared__ double red[kThreads / 64];
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 1; v < kThreads / 64; ++v) mx = fmax(mx, red[v]);
    amax[blockIdx.x] = mx;
  }
}

// Object step sums per slice (blockIdx.y), with D = -g, A = prev or cur + w
// and A' = A + delta max A: part = (sum |D|^2 / A', sum |D|^2 w / A'^2).
__global__ __launch_bounds__(kThreads) void k_lsq_obj_sums(const float2* __restrict__ g, const float* __restrict__ w,
                                                            const float* __restrict__ cur,
                                                            const float* __restrict__ prev, size_t HW, float delta,
                                                            const double* __restrict__ amax,
                                                            double* __restrict__ part) {
  const size_t base = (size_t)blockIdx.y * HW;
  const double reg = (double)delta * amax[blockIdx.y];
  double num = 0.0, den = 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < HW; e += (size_t)gridDim.x * blockDim.x) {
    const size_t q = base + e;
    const double A = (prev ? (double)prev[q] : (double)cur[q] + (double)w[q]) + reg;
    const double d2 = (double)cabs2(g[q]);
    num += d2 / A;
    den += d2 * (double)w[q] / (A * A);
  }
  __shared__ double red[2][kThreads / 64];
  for (int off = 32; off > 0; off >>= 1) {
    num += __shfl_xor(num, off);
    den += __shfl_xor(den, off);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = num;
    red[1][threadIdx.x >> 6] = den;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
    for (int v = 0; v < kThreads / 64; ++v) t += red[threadIdx.x][v];
    part[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 2 + threadIdx.x] = t;
  }
}

// alpha[s] = num / (den + gamma) from the partials of slice s (0 when the
// denominator is 0). One block per slice.
__global__ __launch_bounds__(kThreads) void k_lsq_alpha(const double* __restrict__ part, int nblk, double gamma,
                                                         double* __restrict__ alpha) {
  double num = 0.0, den = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kThreads) {
    num += part[((size_t)blockIdx.x * nblk + b) * 2];
    den += part[((size_t)blockIdx.x * nblk + b) * 2 + 1];
  }
  __shared__ double red[2][kThreads / 64];
  for (int off = 32; off > 0; off >>= 1) {
    num += __shfl_xor(num, off);
    den += __shfl_xor(den, off);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = num;
    red[1][threadIdx.x >> 6] = den;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double n = 0.0, d = gamma;
    for (int v = 0; v < kThreads / 64; ++v) {
      n += red[0][v];
      d += red[1][v];
    }
    alpha[blockIdx.x] = d > 0.0 ? n / d : 0.0;
  }
}

// O -= beta alpha_s g / (A + delta max A) (that is, O += beta alpha_s dO), then cur += w.
__global__ void k_lsq_obj_update(float2* __restrict__ O, const float2* __restrict__ g, const float* __restrict__ w,
                                 float* __restrict__ cur, const float* __restrict__ prev, int S, size_t HW,
                                 float delta, float beta, const double* __restrict__ alpha,
                                 const double* __restrict__ amax) {
  const size_t n = (size_t)S * HW;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const float ws = w[e];
    const float A = (prev ? prev[e] : cur[e] + ws) + delta * (float)amax[e / HW];
    const float f = beta * (float)alpha[e / HW] / A;
    O[e] = csub(O[e], cscale(g[e], f));
    cur[e] += ws;
  }
}

// Probe step size: one block finds max B (B = prev or cur + wp per pixel),
// stores it in alpha[1], then reduces over M * N2 values (D = -g,
// B' = B + delta max B) and writes alpha[0] = num / (den + gamma).
__global__ __launch_bounds__(1024) void k_lsq_probe_alpha(const float2* __restrict__ g, const float* __restrict__ wp,
                                                           const float* __restrict__ cur,
                                                           const float* __restrict__ prev, int M, int N2,
                                                           float delta, double gamma, double* __restrict__ alpha) {
  __shared__ float rmax[16];
  __shared__ double bmax;
  float mx = 0.f;
  for (int r = threadIdx.x; r < N2; r += blockDim.x) mx = fmaxf(mx, prev ? prev[r] : cur[r] + wp[r]);
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
  if ((threadIdx.x & 63) == 0) rmax[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int v = 1; v < (int)(blockDim.x >> 6); ++v) mx = fmaxf(mx, rmax[v]);
    bmax = mx;
    alpha[1] = mx;
  }
  __syncthreads();
  const double reg = (double)delta * bmax;
  double num = 0.0, den = 0.0;
  for (int e = threadIdx.x; e < M * N2; e += blockDim.x) {
    const int r = e % N2;
    const double A = (prev ? (double)prev[r] : (double)cur[r] + (double)wp[r]) + reg;
    const double d2 = (double)cabs2(g[e]);
    num += d2 / A;
    den += d2 * (double)wp[r] / (A * A);
  }
  __shared__ double red[2][16];
  for (int off = 32; off > 0; off >>= 1) {
    num += __shfl_xor(num, off);
    den += __shfl_xor(den, off);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = num;
    red[1][threadIdx.x >> 6] = den;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double n = 0.0, d = gamma;
    for (int v = 0; v < (int)(blockDim.x >> 6); ++v) {
      n += red[0][v];
      d += red[1][v];
    }
    alpha[0] = d > 0.0 ? n / d : 0.0;
  }
}

__global__ void k_lsq_probe_update(float2* __restrict__ P, const float2* __restrict__ g, const float* __restrict__ wp,
                                   const float* __restrict__ cur, const float* __restrict__ prev, int M, int N2,
                                   float delta, float beta, const double* __restrict__ alpha) {
  const float reg = delta * (float)alpha[1];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < M * N2; e += gridDim.x * blockDim.x) {
    const int r = e % N2;
    const float A = (prev ? prev[r] : cur[r] + wp[r]) + reg;
    P[e] = csub(P[e], cscale(g[e], beta * (float)alpha[0] / A));
  }
}

__global__ void k_add_inplace(float* __restrict__ a, const float* __restrict__ b, int n) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) a[e] += b[e];
}

// t <- t * mask (elementwise over n_tiles tiles of N*N).
__global__ void k_mask_tiles(float2* __restrict__ t, const uint8_t* __restrict__ mask, size_t n, int N2) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    if (!mask[e % N2]) t[e] = make_float2(0.f, 0.f);
}

static inline int reg_blocks(size_t n) {
  size_t b = (n + kThreads - 1) / kThreads;
  return (int)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

int launch_reg_object(hipStream_t s, const float2* O, float2* g, int S, int H, int W, const RegDev& rg,
                      float* cost_part) {
  const int nb = reg_blocks((size_t)S * H * W);
  hipLaunchKernelGGL(k_reg_object, dim3(nb), dim3(kThreads), 0, s, O, g, S, H, W, rg, cost_part);
  return nb;
}
int launch_reg_probe(hipStream_t s, const float2* P, float2* g, size_t n, float w, float* cost_part) {
  const int nb = reg_blocks(n);
  hipLaunchKernelGGL(k_reg_probe, dim3(nb), dim3(kThreads), 0, s, P, g, n, w, cost_part);
  return nb;
}
int launch_reg_probe_phase(hipStream_t s, const float2* phat, float2* gphat, int M, int N, float wt, float wv,
                           float delta, float* cost_part) {
  const int nb = reg_blocks((size_t)M * N * N);
  hipLaunchKernelGGL(k_reg_probe_phase, dim3(nb), dim3(kThreads), 0, s, phat, gphat, M, N, wt, wv, delta * delta,
                     cost_part);
  return nb;
}
int launch_spec_l1(hipStream_t s, float2* spec, size_t n, size_t HW, float w, float* cost_part) {
  const int nb = reg_blocks(n);
  hipLaunchKernelGGL(k_spec_l1, dim3(nb), dim3(kThreads), 0, s, spec, n, HW, w, (float)(1.0 / std::sqrt((double)HW)),
                     cost_part);
  return nb;
}
void launch_cadd_inplace(hipStream_t s, float2* g, const float2* a, size_t n) {
  hipLaunchKernelGGL(k_cadd_inplace, dim3(reg_blocks(n)), dim3(kThreads), 0, s, g, a, n);
}
void launch_add_cost(hipStream_t s, const float* part, int n, double* loss) {
  hipLaunchKernelGGL(k_add_cost, dim3(1), dim3(kThreads), 0, s, part, n, loss);
}
void launch_amp_clamp(hipStream_t s, float2* O, size_t n, float lo, float hi) {
  hipLaunchKernelGGL(k_amp_clamp, dim3(reg_blocks(n)), dim3(kThreads), 0, s, O, n, lo, hi);
}
void launch_layer_blur(hipStream_t s, float2* O, int S, size_t HW, const float* g, int r) {
  hipLaunchKernelGGL(k_layer_blur, dim3(reg_blocks(HW)), dim3(kThreads), 0, s, O, S, HW, g, r);
}
void launch_lowpass(hipStream_t s, float2* O, float2* tmp, int S, int H, int W, const float* w, int r) {
  const size_t n = (size_t)S * H * W;
  hipLaunchKernelGGL(k_lowpass<0>, dim3(reg_blocks(n)), dim3(kThreads), 0, s, O, tmp, S, H, W, w, r);
  hipLaunchKernelGGL(k_lowpass<1>, dim3(reg_blocks(n)), dim3(kThreads), 0, s, tmp, O, S, H, W, w, r);
}
int deramp_blocks(int H, int W) {
  const size_t b = ((size_t)H * W + kThreads - 1) / kThreads;
  return (int)(b > 256 ? 256 : b);
}
void launch_deramp(hipStream_t s, float2* O, int S, int H, int W, double* theta, double* part) {
  const int nb = deramp_blocks(H, W);
  hipLaunchKernelGGL(k_deramp_sums<0>, dim3(nb, S), dim3(kThreads), 0, s, O, H, W, theta, part);
  hipLaunchKernelGGL(k_deramp_angles<0>, dim3(S), dim3(kThreads), 0, s, part, nb, theta);
  hipLaunchKernelGGL(k_deramp_sums<1>, dim3(nb, S), dim3(kThreads), 0, s, O, H, W, theta, part);
  hipLaunchKernelGGL(k_deramp_angles<1>, dim3(S), dim3(kThreads), 0, s, part, nb, theta);
  hipLaunchKernelGGL(k_deramp_apply, dim3(reg_blocks((size_t)S * H * W)), dim3(kThreads), 0, s, O, S, H, W, theta);
}
void launch_lsq_transparency(hipStream_t s, const Item* items, int n_items, const float2* O, int S, int H,
                             int W, int N, float* tau, float* part, float* wp) {
  const int N2 = N * N;
  const size_t HW = (size_t)H * W;
  hipLaunchKernelGGL(k_lsq_tau, dim3(reg_blocks(HW)), dim3(kThreads), 0, s, O, S, HW, tau);
  hipLaunchKernelGGL(k_lsq_transp, dim3((N2 + kThreads - 1) / kThreads, kLsqSplit), dim3(kThreads), 0, s, items,
                     n_items, tau, W, N, part);
  hipLaunchKernelGGL(k_lsq_transp_sum, dim3((N2 + kThreads - 1) / kThreads), dim3(kThreads), 0, s, part, N2, wp);
}
int lsq_blocks(size_t n) {
  const size_t b = (n + kThreads - 1) / kThreads;
  return (int)(b > 256 ? 256 : b);
}
void launch_lsq_object(hipStream_t s, float2* O, const float2* g, const float* w, float* cur, const float* prev,
                       int S, size_t HW, float delta, double gamma, float beta, double* part, double* alpha) {
  const int nb = lsq_blocks(HW);
  double* pmax = part + (size_t)S * nb * 2;      // after the sums: S * nb partial maxima, then S maxima
  double* amax = pmax + (size_t)S * nb;
  hipLaunchKernelGGL(k_lsq_obj_pmax, dim3(nb, S), dim3(kThreads), 0, s, w, cur, prev, HW, pmax);
  hipLaunchKernelGGL(k_lsq_obj_amax, dim3(S), dim3(kThreads), 0, s, pmax, nb, amax);
  hipLaunchKernelGGL(k_lsq_obj_sums, dim3(nb, S), dim3(kThreads), 0, s, g, w, cur, prev, HW, delta, amax, part);
  hipLaunchKernelGGL(k_lsq_alpha, dim3(S), dim3(kThreads), 0, s, part, nb, gamma, alpha);
  hipLaunchKernelGGL(k_lsq_obj_update, dim3(reg_blocks((size_t)S * HW)), dim3(kThreads), 0, s, O, g, w, cur, prev,
                     S, HW, delta, beta, alpha, amax);
}
void launch_lsq_probe(hipStream_t s, float2* P, const float2* g, const float* wp, float* cur, const float* prev,
                      int M, int N2, float delta, double gamma, float beta, double* alpha) {
  hipLaunchKernelGGL(k_lsq_probe_alpha, dim3(1), dim3(1024), 0, s, g, wp, cur, prev, M, N2, delta, gamma, alpha);
  hipLaunchKernelGGL(k_lsq_probe_update, dim3(reg_blocks((size_t)M * N2)), dim3(kThreads), 0, s, P, g, wp, cur,
                     prev, M, N2, delta, beta, alpha);
  hipLaunchKernelGGL(k_add_inplace, dim3(reg_blocks((size_t)N2)), dim3(kThreads), 0, s, cur, wp, N2);
}
void launch_mask_tiles(hipStream_t s, float2* t, const uint8_t* mask, size_t n, int N2) {
  hipLaunchKernelGGL(k_mask_tiles, dim3(reg_blocks(n)), dim3(kThreads), 0, s, t, mask, n, N2);
}

}  // namespace pty

namespace pty {

// ============================================================ LDS-resident chains (N <= 128)
//
// For N = 64 and 128 a whole tile (32 / 128 KiB of complex64) fits in LDS, so
// one workgroup per (position, mode) runs every slice step of the forward (or
// adjoint) model with the tile resident: rows and columns are transformed in
// place, each line using its own storage as its exchange scratch (rows with a
// padded exchange layout inside the padded row pitch, columns with the plain
// one). Only the object rows, the propagator, the checkpoints and the
// gradients are read from or written to memory. The pitch P was chosen so that
// every exchange and line access of a wave hits any LDS bank at most 4 times.
template <int N, bool INV, int XP, int STRIDE>
__device__ __forceinline__ void res_line_fft(float2 (&v)[Cfg<N>::E], int l, const float2* tw, float2* base) {
  WaveSync{}();           // earlier reads of this line's storage are done
  res_stage1<N, INV, XP, STRIDE>(v, l, tw, base);
  WaveSync{}();
  res_stage2<N, INV, XP, STRIDE>(v, l, base);
  WaveSync{}();           // exchange reads are done before the line is rewritten
}

template <int N>
__device__ __forceinline__ void res_load_row(float2 (&v)[Cfg<N>::E], const float2* tile, int y, int l) {
#pragma unroll
  for (int a = 0; a < Cfg<N>::E; ++a) v[a] = tile[y * Res<N>::P + l + Cfg<N>::L * a];
}
template <int N>
__device__ __forceinline__ void res_store_row(const float2 (&v)[Cfg<N>::E], float2* tile, int y, int l) {
#pragma unroll
  for (int a = 0; a < Cfg<N>::E; ++a) tile[y * Res<N>::P + l + Cfg<N>::L * a] = v[a];
}

// Column pass in LDS: tile column x <- IDFT_y(mult * DFT_y(column)), mult from a
// global [N][N] table (conjugated if CONJ).
template <int N, bool CONJ>
__device__ __forceinline__ void res_col_prop(float2* tile, const float2* tw, const float2* __restrict__ Hm) {
  constexpr int L = Cfg<N>::L, E = Cfg<N>::E, P = Res<N>::P, LINES = Res<N>::THREADS / L;
  const int l = threadIdx.x % L;
  for (int x = threadIdx.x / L; x < N; x += LINES) {
    float2 v[E];
#pragma unroll
    for (int a = 0; a < E; ++a) v[a] = tile[(l + L * a) * P + x];
    res_line_fft<N, false, L, P>(v, l, tw, tile + x);
#pragma unroll
    for (int a = 0; a < E; ++a) {
      const float2 h = Hm[(size_t)(l + L * a) * N + x];
      v[a] = CONJ ? cjmul(h, v[a]) : cmul(v[a], h);
    }
    res_line_fft<N, true, L, P>(v, l, tw, tile + x);
#pragma unroll
    for (int a = 0; a < E; ++a) tile[(l + L * a) * P + x] = v[a];
  }
}

// Forward chain of one (item, mode): shift, every slice, ending with the
// forward row DFT of the last exit wave written to the global work tile
// (the far-field kernel takes it from there). Entry waves are checkpointed.
template <int N, bool HALF>
__global__ __launch_bounds__(Res<N>::THREADS) void k_res_fwd(const Item* __restrict__ items, const ReqTable reqs,
                                                             float2* __restrict__ ws, void* __restrict__ ck_,
                                                             const float2* __restrict__ ramps,
                                                             const float2* __restrict__ twg, int save, int item_off) {
  constexpr int L = Cfg<N>::L, E = Cfg<N>::E, LINES = Res<N>::THREADS / L;
  __shared__ float2 tile[N * Res<N>::P];
  __shared__ float2 tw[N];
  const int b = item_off + blockIdx.y, m = blockIdx.z;
  const Item it = items[b];
  const ReqDev& r = reqs.r[it.req];
  if (!it.valid || m >= r.M) return;
  using CT = typename Ck<HALF>::T;
  CT* ck = static_cast<CT*>(ck_);
  for (int k = threadIdx.x; k < N; k += blockDim.x) tw[k] = twg[k];
  __syncthreads();
  const int l = threadIdx.x % L;
  const float inv = 1.f / (float)N;
  // psi_0 = IDFT_2(phat R) / N : columns first (u_x fixed per column)
  {
    const float2* ry = ramps + (size_t)b * 2 * N;
    const float2* ph = r.phat + (size_t)m * N * N;
    for (int x = threadIdx.x / L; x < N; x += LINES) {
      const float2 rx = ramps[(size_t)b * 2 * N + N + x];
      float2 v[E];
#pragma unroll
      for (int a = 0; a < E; ++a) {
        const int uy = l + L * a;
        v[a] = cscale(cmul(cmul(ph[(size_t)uy * N + x], ry[uy]), rx), inv);
      }
      res_line_fft<N, true, L, Res<N>::P>(v, l, tw, tile + x);
#pragma unroll
      for (int a = 0; a < E; ++a) tile[(l + L * a) * Res<N>::P + x] = v[a];
    }
  }
  __syncthreads();
  for (int i = 0; i < r.S; ++i) {
    for (int y = threadIdx.x / L; y < N; y += LINES) {
      float2 v[E];
      res_load_row<N>(v, tile, y, l);
      res_line_fft<N, true, L + 1, 1>(v, l, tw, tile + y * Res<N>::P);       // entry wave psi_i
      if (save && (i % r.ck_every) == 0) {
        CT* dst = ck + (ck_tile(it, r, m, i / r.ck_every) * N + y) * N;
#pragma unroll
        for (int a = 0; a < E; ++a) Ck<HALF>::store(dst + l + L * a, v[a]);
      }
      const float2* orow = r.obj + ((size_t)i * r.H + it.ny + y) * r.W + it.nx;
#pragma unroll
      for (int a = 0; a < E; ++a) v[a] = cmul(v[a], orow[l + L * a]);
      res_line_fft<N, false, L + 1, 1>(v, l, tw, tile + y * Res<N>::P);
      if (i == r.S - 1) {
        float2* trow = ws + ((size_t)(it.tile0 + m) * N + y) * N;
#pragma unroll
        for (int a = 0; a < E; ++a) trow[l + L * a] = v[a];
      } else {
        res_store_row<N>(v, tile, y, l);
      }
    }
    __syncthreads();
    if (i < r.S - 1) {
      res_col_prop<N, false>(tile, tw, r.prop + (size_t)i * N * N);
      __syncthreads();
    }
  }
}

// Adjoint chain of one (item, mode): from the detector seed in the global work
// tile (after its inverse column DFT) back through every slice; the object
// gradient of this mode is scatter-added per slice; the forward row DFT of the
// gradient with respect to psi_0 is written back to the work tile for the
// final column pass.
template <int N, bool HALF>
__global__ __launch_bounds__(Res<N>::THREADS) void k_res_adj(const Item* __restrict__ items, const ReqTable reqs,
                                                             float2* __restrict__ ws, const void* __restrict__ ck_,
                                                             const float2* __restrict__ twg, float scale,
                                                             int item_off) {
  constexpr int L = Cfg<N>::L, E = Cfg<N>::E, LINES = Res<N>::THREADS / L;
  __shared__ float2 tile[N * Res<N>::P];
  __shared__ float2 tw[N];
  const int b = item_off + blockIdx.y, m = blockIdx.z;
  const Item it = items[b];
  const ReqDev& r = reqs.r[it.req];
  if (!it.valid || m >= r.M) return;
  using CT = typename Ck<HALF>::T;
  const CT* ck = static_cast<const CT*>(ck_);
  for (int k = threadIdx.x; k < N; k += blockDim.x) tw[k] = twg[k];
  __syncthreads();
  const int l = threadIdx.x % L;
  float2* wtile = ws + (size_t)(it.tile0 + m) * N * N;
  const float sc = adj_scale(r, scale);
  for (int i = r.S - 1; i >= 0; --i) {
    for (int y = threadIdx.x / L; y < N; y += LINES) {
      float2 v[E];
      if (i == r.S - 1) {
#pragma unroll
        for (int a = 0; a < E; ++a) v[a] = wtile[(size_t)y * N + l + L * a];
      } else {
        res_load_row<N>(v, tile, y, l);
      }
      res_line_fft<N, true, L + 1, 1>(v, l, tw, tile + y * Res<N>::P);       // gradient wrt phi_i
      const CT* prow = ck + (ck_tile(it, r, m, i) * N + y) * N;
      const size_t orow = ((size_t)i * r.H + it.ny + y) * r.W + it.nx;
      float* g = r.gobj ? reinterpret_cast<float*>(r.gobj + orow) : nullptr;
#pragma unroll
      for (int a = 0; a < E; ++a) {
        const float2 p = Ck<HALF>::load(prow + l + L * a);
        const float2 o = r.obj[orow + l + L * a];
        if (g) {
          const float2 d = cjmul(p, v[a]);
          unsafeAtomicAdd(g + 2 * (l + L * a), sc * d.x);
          unsafeAtomicAdd(g + 2 * (l + L * a) + 1, sc * d.y);
        }
        v[a] = cjmul(o, v[a]);
      }
      res_line_fft<N, false, L + 1, 1>(v, l, tw, tile + y * Res<N>::P);
      if (i == 0) {
#pragma unroll
        for (int a = 0; a < E; ++a) wtile[(size_t)y * N + l + L * a] = v[a];
      } else {
        res_store_row<N>(v, tile, y, l);
      }
    }
    __syncthreads();
    if (i > 0) {
      res_col_prop<N, true>(tile, tw, r.prop + (size_t)(i - 1) * N * N);
      __syncthreads();
    }
  }
}

template <int N>
static void res_fwd_n(const LaunchCtx& L, bool save) {
  dim3 g(1, L.n_items, L.max_modes);
  if (L.ck_half)
    hipLaunchKernelGGL((k_res_fwd<N, true>), g, dim3(Res<N>::THREADS), 0, L.stream, L.items, L.reqs, L.ws, L.ck,
                       L.ramps, L.tw, save ? 1 : 0, L.item_off);
  else
    hipLaunchKernelGGL((k_res_fwd<N, false>), g, dim3(Res<N>::THREADS), 0, L.stream, L.items, L.reqs, L.ws, L.ck,
                       L.ramps, L.tw, save ? 1 : 0, L.item_off);
}
template <int N>
static void res_adj_n(const LaunchCtx& L, float scale) {
  dim3 g(1, L.n_items, L.max_modes);
  if (L.ck_half)
    hipLaunchKernelGGL((k_res_adj<N, true>), g, dim3(Res<N>::THREADS), 0, L.stream, L.items, L.reqs, L.ws, L.ck,
                       L.tw, scale, L.item_off);
  else
    hipLaunchKernelGGL((k_res_adj<N, false>), g, dim3(Res<N>::THREADS), 0, L.stream, L.items, L.reqs, L.ws, L.ck,
                       L.tw, scale, L.item_off);
}

bool resident_supported(int N) { return N == 64 || N == 128; }

void launch_res_fwd(const LaunchCtx& L, int N, bool save) {
  if (N == 64) res_fwd_n<64>(L, save);
  else res_fwd_n<128>(L, save);
}
void launch_res_adj(const LaunchCtx& L, int N, float scale) {
  if (N == 64) res_adj_n<64>(L, scale);
  else res_adj_n<128>(L, scale);
}

}  // namespace pty
