// pty_api.cpp -- host side of libpty: contexts, workspace, propagator tables,
// and the launch sequences of forward, loss-and-gradient and one optimiser
// step (arXiv 2505.14372, Sec. 2.2 engine loop, Sec. 3 - 3.2).
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "pty.h"
#include "pty_internal.h"
#include "pty_prop.hpp"

using namespace pty;

// Working memory of pty_forward_static: one array per GPU in this library's
// code object, so that entry point calls no allocation routine. In host code
// the name `scratch` is only a host-side stand-in for the array; kernels are
// given the device address that hipGetSymbolAddress returns for the current
// device (scratch_address below), never the name itself.
static __device__ __align__(256) unsigned char scratch[PTY_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch` per device, set once

// Device address of `scratch` on the current device, looked up once per
// device (at context creation, with the context's device current).
hipError_t scratch_address(void** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

namespace {

constexpr double kPiD = 3.141592653589793238462643383279502884;

bool supported_N(int N) { return N == 64 || N == 128 || N == 192 || N == 256; }

constexpr int kMaxStreams = 8;   // concurrent chunk streams per context

template <typename T>
pty_status dmalloc(T** p, size_t count, std::string& err) {
  *p = nullptr;
  if (count == 0) return PTY_OK;
  if (hipMalloc((void**)p, count * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    err = "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed";
    return PTY_ENOMEM;
  }
  return PTY_OK;
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

// Roots of unity w_N^k = exp(-2 pi i k / N), computed in double.
std::vector<float2> roots(int N) {
  std::vector<float2> t(N);
  for (int k = 0; k < N; ++k) {
    double a = 2.0 * kPiD * (double)k / (double)N;
    t[k] = make_float2((float)std::cos(a), (float)-std::sin(a));
  }
  return t;
}

struct Sizes {
  size_t tiles = 0, ck_tiles = 0, seg_tiles = 0, ws2_tiles = 0;
  size_t bytes = 0;
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Device bytes of one context (fixed part + batch workspace); checkpoints and
// segment buffers hold ck_elem bytes per complex value.
Sizes ctx_sizes(const pty_geometry* g, int max_batch, int k, int ck_elem = 8, bool lsqml = false) {
  Sizes s;
  const size_t N2 = (size_t)g->N * g->N;
  const int S = g->n_slices, M = g->n_modes;
  const int n_ck = (S + k - 1) / k;
  s.tiles = (size_t)max_batch * M;
  s.ck_tiles = (size_t)max_batch * M * n_ck;
  s.seg_tiles = k > 1 ? (size_t)max_batch * M * (k - 1) : 0;
  s.ws2_tiles = k > 1 ? s.tiles : 0;
  size_t b = 0;
  b += align256(g->N * sizeof(float2));                             // roots
  b += align256((size_t)std::max(S - 1, 0) * N2 * sizeof(float2));  // propagators
  b += align256((size_t)std::max(S - 1, 0) * g->N * sizeof(float4));   // separable factors (y)
  b += align256((size_t)std::max(S - 1, 0) * g->N * sizeof(float2));   // separable factors (x)
  b += 3 * align256((size_t)M * N2 * sizeof(float2));               // phat, gphat, gprobe
  b += align256((size_t)S * g->obj_h * g->obj_w * sizeof(float2));  // object gradient
  b += align256((size_t)g->n_positions * 2 * sizeof(float));        // dense position gradient
  b += align256(sizeof(int) * 4);                                   // flags
  if (max_batch > 0) {
    const int nblk = col_blocks(g->N);
    b += align256((s.tiles + s.ws2_tiles) * N2 * sizeof(float2));
    b += align256((s.ck_tiles + s.seg_tiles) * N2 * (size_t)ck_elem);
    b += align256((size_t)max_batch * sizeof(Item));
    b += align256((size_t)max_batch * 2 * g->N * sizeof(float2));
    b += align256((size_t)max_batch * nblk * sizeof(float));
    b += align256((size_t)max_batch * M * nblk * 2 * sizeof(float));
    b += align256((size_t)max_batch * S * 2 * sizeof(float));          // ePIE window maxima
    b += align256((size_t)max_batch * N2 * sizeof(float2));            // ordered reduction scratch
  }
  if (lsqml) {
    const size_t HW = (size_t)g->obj_h * g->obj_w;
    b += align256((size_t)S * HW * sizeof(float));                     // illumination scatter
    b += align256((size_t)(kLsqSplit + 1) * N2 * sizeof(float));       // transparency partials + sum
    b += align256(HW * sizeof(float));                                 // transparency map
    b += align256(((size_t)S * lsq_blocks(HW) * 3 + 2 * S + 2) * sizeof(double));
    b += align256((size_t)max_batch * N2 * sizeof(float));             // ordered illumination scratch
  }
  s.bytes = b;
  return s;
}

pty_status validate_geometry(const pty_geometry* g, std::string& err) {
  if (!g) { err = "geometry is NULL"; return PTY_EINVAL; }
  if (!supported_N(g->N)) { err = "N must be 64, 128, 192 or 256"; return PTY_EUNSUPPORTED; }
  if (g->n_modes < 1 || g->n_slices < 1 || g->n_positions < 1) { err = "n_modes, n_slices, n_positions must be >= 1"; return PTY_EINVAL; }
  if (g->obj_h < g->N || g->obj_w < g->N) { err = "object smaller than the window"; return PTY_EINVAL; }
  if (g->n_slices > 1 && !g->dz) { err = "dz is NULL"; return PTY_EINVAL; }
  if (g->loss < PTY_LOSS_AMPLITUDE || g->loss > PTY_LOSS_GAUSSIAN) { err = "unknown loss kind"; return PTY_EINVAL; }
  if (!(g->dx > 0) || !(g->wavelength > 0)) { err = "dx and wavelength must be positive"; return PTY_EINVAL; }
  if (!(std::fabs(g->tilt_y) < 1.5) || !(std::fabs(g->tilt_x) < 1.5)) { err = "tilt must be finite and below pi/2"; return PTY_EINVAL; }
  if (g->loss == PTY_LOSS_GAUSSIAN && !(g->sigma > 0)) { err = "sigma must be positive"; return PTY_EINVAL; }
  if ((size_t)g->n_slices * g->obj_h * g->obj_w > ((size_t)1 << 40)) { err = "object too large"; return PTY_EUNSUPPORTED; }
  return PTY_OK;
}


// ---------------------------------------------------------------- launch timing
// Optional per-kernel-class timing: when enabled, every launch is bracketed by
// two hipEvents on its own stream; pty_profile_collect() waits for them and
// returns total milliseconds and launch counts per class.
enum ProfClass {
  P_ITEMS, P_COL_SHIFT, P_ROW_FWD, P_COL_PROP, P_FAR_LOSS, P_LOSS_REDUCE, P_ROW_ADJ, P_COL_PROP_ADJ,
  P_COL_FINAL, P_PROBE_GRAD, P_POS_REDUCE, P_PLAIN2D, P_FILL, P_OPTIM, P_RECOMPUTE, P_REG, P_RES_FWD, P_RES_ADJ,
  P_OBJ_GATHER, P_NCLASS
};
const char* kProfNames[P_NCLASS] = {"items", "col_shift", "row_fwd", "col_prop", "far_loss", "loss_reduce",
                                    "row_adj", "col_prop_adj", "col_final", "probe_grad", "pos_reduce",
                                    "plain2d", "fill", "optimizer", "recompute", "regularizers", "res_fwd",
                                    "res_adj", "obj_gather"};

struct ProfRec { int cls; hipEvent_t a, b; };

struct Profiler {
  std::mutex mu;
  bool on = false;
  uint64_t mask = ~0ull;     // classes timed while on (pty_profile_select)
  std::vector<ProfRec> pending;
  std::vector<hipEvent_t> pool;
  double total_ms[P_NCLASS] = {};
  long long count[P_NCLASS] = {};
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
Profiler g_prof;

struct ProfScope {
  int cls;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(int c, hipStream_t st) : cls(c), s(st) {
    if (!g_prof.on || !((g_prof.mask >> c) & 1ull)) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    a = g_prof.get();
    if (a && hipEventRecord(a, s) != hipSuccess) a = nullptr;
  }
  ~ProfScope() {
    if (!a) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    hipEvent_t b = g_prof.get();
    if (b && hipEventRecord(b, s) == hipSuccess) g_prof.pending.push_back({cls, a, b});
  }
};
}  // namespace

struct pty_ctx {
  pty_geometry g{};
  std::vector<double> dz;
  int max_batch = 0, ck_every = 1, n_ck = 1;
  int chunk = 0;              // positions per launch in fused loss-and-gradient calls (0: all)
  // chunks run concurrently on these streams (created by pty_set_streams, default priority)
  int n_streams = 1;
  hipStream_t streams[kMaxStreams] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kMaxStreams] = {};
  int strategy = PTY_STRATEGY_AUTO;
  int reduce = PTY_REDUCE_ATOMIC;
  Sizes sz;
  float2 *tw = nullptr, *prop = nullptr, *phat = nullptr, *gphat = nullptr, *gprobe = nullptr, *gobj = nullptr;
  float* gpos = nullptr;
  int* flags = nullptr;
  float2 *ws = nullptr, *ws2 = nullptr;
  unsigned char *ck = nullptr, *seg = nullptr;   // checkpoint storage (float2 or __half2)
  int ck_half = 0;
  Item* items = nullptr;
  float2* ramps = nullptr;
  float *loss_part = nullptr, *pos_part = nullptr;
  float2* cscr = nullptr;          // ordered object-gradient reduction scratch [max_batch][N][N]
  // regularization
  bool reg_on = false, con_on = false;
  RegDev rg{};
  float probe_l2 = 0.f;
  int amp_clamp = 0;
  float amp_min = 0.f, amp_max = 0.f;
  uint8_t* support = nullptr;      // device [N][N] or null
  uint8_t* support_real = nullptr; // device [N][N] real-space probe support, or null
  float probe_phase_tik = 0.f, probe_phase_tv = 0.f;
  // object spectral L1: weight, batched 2D FFT plan of the slices (in place),
  // spectrum buffer [S][H][W]
  float obj_spec_l1 = 0.f;
  hipfftHandle spec_plan = 0;
  bool spec_plan_ok = false;
  float2* spec = nullptr;
  float* blur = nullptr;           // device Gaussian weights [r + 1]
  int blur_r = 0;
  float* lowpass = nullptr;        // device in-plane Gaussian weights [r + 1], normalised over 2r + 1 taps
  int lowpass_r = 0;
  double* deramp = nullptr;        // device [S][3] angles, then [S][deramp_blocks][4] partial sums
  float* reg_part = nullptr;       // cost partial sums
  float* emax = nullptr;           // ePIE window maxima [max_batch][S][2]
  uint8_t* live = nullptr;         // [N] columns where the propagators are nonzero, or null (all)
  int live_k = -1;                 // live columns are |k_x| <= live_k (-1: look them up in live)
  unsigned live_blocks = 0;        // column-pass blocks holding a live column (bit per block; 0: all)
  float4* prop_y = nullptr;        // [S-1][N] separable propagator factors, or null (table only)
  float2* prop_x = nullptr;        // [S-1][N]
  // LSQML scratch (pty_options.lsqml): illumination scatter [S][H][W],
  // transparency partials [kLsqSplit][N][N] and sum [N][N], step sums
  float* lsq_w = nullptr;
  float* lsq_part = nullptr;
  float* lsq_wp = nullptr;
  float* lsq_tau = nullptr;
  float* lsq_wscr = nullptr;       // ordered reduction of the illumination sums [max_batch][N][N]
  double* lsq_sums = nullptr;
  // tape of pty_forward_save
  bool tape_valid = false;
  LaunchCtx tape{};
  std::string err;
};

struct pty_group {
  int N = 0, max_items = 0, max_tiles = 0;
  long long max_ck = 0;
  float2 *tw = nullptr, *ws = nullptr, *ck = nullptr, *ramps = nullptr;
  Item* items = nullptr;
  float *loss_part = nullptr, *pos_part = nullptr;
  float2* cscr = nullptr;   // ordered object-gradient reduction scratch [max_items][N][N]
  int* flags = nullptr;
  std::string err;
};

namespace {

#define HIPCHECK(ctxp, call)                                               \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess) {                                                \
      (ctxp)->err = std::string(#call) + ": " + hipGetErrorString(e_);     \
      return PTY_EHIP;                                                     \
    }                                                                      \
  } while (0)

// LDS-resident chains: N <= 128 and every slice checkpointed.
bool use_resident(int strategy, int N, int ck_every) {
  if (!resident_supported(N) || ck_every != 1) return false;
  return strategy == PTY_STRATEGY_RESIDENT;
}

ReqDev base_req(pty_ctx* c) {
  ReqDev r{};
  r.prop = c->prop;
  r.phat = c->phat;
  r.gphat = c->gphat;
  r.S = c->g.n_slices;
  r.M = c->g.n_modes;
  r.H = c->g.obj_h;
  r.W = c->g.obj_w;
  r.J = c->g.n_positions;
  r.loss = c->g.loss;
  r.eps = (float)c->g.eps;
  r.inv_sigma2 = c->g.loss == PTY_LOSS_GAUSSIAN ? (float)(1.0 / (c->g.sigma * c->g.sigma)) : 1.f;
  r.ck_every = c->ck_every;
  r.n_ck = c->n_ck;
  r.live = c->live;
  r.live_k = c->live_k;
  r.prop_y = c->prop_y;
  r.prop_x = c->prop_x;
  return r;
}

LaunchCtx ctx_launch(pty_ctx* c, hipStream_t s, const ReqDev& r, int B) {
  LaunchCtx L{};
  L.stream = s;
  L.reqs.r[0] = r;
  L.reqs.r[0].item0 = 0;
  L.reqs.r[0].n_items = B;
  L.n_reqs = 1;
  L.n_items = B;
  L.max_modes = c->g.n_modes;
  L.items = c->items;
  L.ws = c->ws;
  L.ck = c->ck;
  L.ck_half = c->ck_half;
  L.ramps = c->ramps;
  L.tw = c->tw;
  L.loss_part = c->loss_part;
  L.pos_part = c->pos_part;
  L.flags = c->flags;
  L.resident = (use_resident(c->strategy, c->g.N, c->ck_every) && c->reduce != PTY_REDUCE_ORDERED) ? 1 : 0;
  L.cscr = c->reduce == PTY_REDUCE_ORDERED ? c->cscr : nullptr;
  // float checkpoints: the column passes write the stored entry waves' row
  // spectra straight into the checkpoint slots (the resident chains ignore it)
  L.ck_spec = c->ck_half ? 0 : 1;
  L.col_live_blocks = c->live_blocks;
  return L;
}

// Launch sequences. A launch context L covers items [L.item_off,
// L.item_off + L.n_items); prepare/finish steps always cover every item.

std::vector<std::pair<int, int>> split_chunks(int n, int chunk) {
  std::vector<std::pair<int, int>> out;
  if (chunk <= 0 || chunk >= n) { out.push_back({0, n}); return out; }
  for (int a = 0; a < n; a += chunk) out.push_back({a, std::min(chunk, n - a)});
  return out;
}

LaunchCtx sub(const LaunchCtx& L, int off, int n) {
  LaunchCtx R = L;
  R.item_off = off;
  R.n_items = n;
  return R;
}

void run_prepare(const LaunchCtx& L, int N) {
  ProfScope p(P_ITEMS, L.stream);
  launch_items(L, N);
}

// Forward passes of the items of L (steps up to the largest S). save: store
// entry-wave checkpoints and leave the detector-plane gradient seed (after
// its inverse column DFT) in the workspace.
void run_forward_chunk(const LaunchCtx& L, int N, int S_max, const std::vector<int>& far_steps, bool save) {
  if (L.resident) {
    { ProfScope p(P_RES_FWD, L.stream); launch_res_fwd(L, N, save); }
    for (int i : far_steps) {
      ProfScope p(P_FAR_LOSS, L.stream);
      launch_far_loss(L, N, i, save);
    }
    return;
  }
  // F: spectral checkpoints only when the entry waves are kept
  LaunchCtx F = L;
  F.ck_spec = save && L.ck_spec;
  { ProfScope p(P_COL_SHIFT, L.stream); launch_col(F, N, COL_SHIFT, 0); }
  PsiStore st{};
  st.mode = save ? (F.ck_spec ? 3 : 1) : 0;
  for (int i = 0; i < S_max; ++i) {
    { ProfScope p(P_ROW_FWD, L.stream); launch_rows_fwd(F, N, i, st, false); }
    if (i < S_max - 1) { ProfScope p(P_COL_PROP, L.stream); launch_col(F, N, COL_PROP, i); }
    if (std::find(far_steps.begin(), far_steps.end(), i) != far_steps.end()) {
      ProfScope p(P_FAR_LOSS, L.stream);
      launch_far_loss(L, N, i, save);
    }
  }
}

void run_finish_forward(const LaunchCtx& L, int N) {
  ProfScope p(P_LOSS_REDUCE, L.stream);
  launch_loss_reduce(L, N);
}

// Adjoint passes of the items of L (after their forward with save).
// Single-request contexts may use checkpoint intervals k > 1 (entry waves
// recomputed per segment); grouped launches store every slice.
void run_backward_chunk(const LaunchCtx& L, int N, int S_max, const std::vector<int>& final_steps, float scale,
                        int k, float2* ws2, void* seg) {
  if (L.resident) {
    { ProfScope p(P_RES_ADJ, L.stream); launch_res_adj(L, N, scale); }
    for (int t : final_steps) {
      ProfScope p(P_COL_FINAL, L.stream);
      launch_col(L, N, COL_FINAL, t);
    }
    return;
  }
  int seg_lo = -1, seg_hi = -1;   // slices currently held in the segment buffer
  for (int t = 0; t < S_max; ++t) {
    const int i = S_max - 1 - t;   // single-request slice index (k > 1 only)
    PsiLoad psi{};
    psi.spec = L.ck_spec;
    if (k > 1 && i % k != 0) {
      const int i0 = (i / k) * k;
      const int i1 = std::min(i0 + k - 1, S_max - 1);
      if (!(seg_lo == i0 + 1 && seg_hi == i1)) {
        // recompute entry waves i0+1 .. i1 from the checkpoint at i0
        ProfScope p(P_RECOMPUTE, L.stream);
        LaunchCtx R = L;
        R.ws = ws2;
        R.emax = 0;
        if (L.ck_spec) {
          // row spectra: the row pass of slice s reads slot i0 / k (s = i0) or
          // segment slot s - i0 - 1, and the column pass after it leaves the
          // next slice's row spectrum in its segment slot
          R.seg_out = SegOut{static_cast<float2*>(seg), k - 1, i0 + 1};
          PsiStore st{};
          st.mode = 3;
          st.seg = seg;
          st.seg_len = k - 1;
          for (int s = i0; s < i1; ++s) {
            st.seg_slot = s - i0 - 1;
            launch_rows_fwd(R, N, s, st, false);
            launch_col(R, N, COL_PROP, s);
          }
        } else {
          PsiStore st{};
          st.mode = 0;
          st.src = L.ck;
          st.src_slot = i0 / k;
          launch_rows_fwd(R, N, i0, st, true);
          for (int s = i0 + 1; s <= i1; ++s) {
            launch_col(R, N, COL_PROP, s - 1);
            PsiStore ss{};
            ss.mode = 2;
            ss.seg = seg;
            ss.seg_len = k - 1;
            ss.seg_slot = s - i0 - 1;
            ss.stop_after_store = (s == i1) ? 1 : 0;
            launch_rows_fwd(R, N, s, ss, false);
          }
        }
        seg_lo = i0 + 1;
        seg_hi = i1;
      }
      psi.from_seg = 1;
      psi.seg = seg;
      psi.seg_len = k - 1;
      psi.seg_base = i0 + 1;
    }
    { ProfScope p(P_ROW_ADJ, L.stream); launch_rows_adj(L, N, t, psi, scale); }
    if (L.cscr) {
      // ordered reduction: add this slice's stored contributions in batch order
      int mh = 0, mw = 0;
      for (int q = 0; q < L.n_reqs; ++q) {
        mh = std::max(mh, L.reqs.r[q].H);
        mw = std::max(mw, L.reqs.r[q].W);
      }
      ProfScope p(P_OBJ_GATHER, L.stream);
      launch_obj_gather(L, N, t, mh, mw);
    }
    if (t < S_max - 1) { ProfScope p(P_COL_PROP_ADJ, L.stream); launch_col(L, N, COL_PROP_ADJ, t); }
    if (std::find(final_steps.begin(), final_steps.end(), t) != final_steps.end()) {
      ProfScope p(P_COL_FINAL, L.stream);
      launch_col(L, N, COL_FINAL, t);
    }
  }
}

void run_finish_backward(const LaunchCtx& L, int N, float scale) {
  { ProfScope p(P_PROBE_GRAD, L.stream); launch_probe_grad(L, N, scale); }
  { ProfScope p(P_POS_REDUCE, L.stream); launch_pos_reduce(L, N, scale); }
}

pty_status check_call(pty_ctx* c, const void* probe, const void* object, const void* positions,
                      const int32_t* batch_idx, int32_t B) {
  if (!c) return PTY_EINVAL;
  if (!probe || !object || !positions || !batch_idx) { c->err = "NULL input pointer"; return PTY_EINVAL; }
  if (B < 1 || B > c->max_batch) {
    c->err = "batch " + std::to_string(B) + " outside [1, max_batch=" + std::to_string(c->max_batch) + "]";
    return PTY_EINVAL;
  }
  return PTY_OK;
}

// Forward and adjoint of every chunk in turn (so that one chunk's tiles stay
// cached between its passes), then the group reductions.
void run_fused(pty_ctx* c, const LaunchCtx& L0, float scale) {
  const int N = c->g.N, S = c->g.n_slices;
  run_prepare(L0, N);
  const auto chunks = split_chunks(L0.n_items, c->chunk);
  LaunchCtx L = L0;
  set_chain_final(L, N, chunks.size() == 1);
  // Chunks touch disjoint work tiles, checkpoints and partial sums, so they
  // may run concurrently, chunk q on stream q mod n, except where two chunks
  // write the same words without atomics: the ordered object-gradient gather
  // and the recompute buffers (ws2, seg) shared by every chunk.
  int ns = 1;
  if (c->n_streams > 1 && chunks.size() > 1 && !L.cscr && c->ck_every == 1 && !L.resident)
    ns = std::min<int>(c->n_streams, (int)chunks.size());
  if (ns > 1) {
    (void)hipEventRecord(c->ev_fork, L.stream);
    for (int k = 0; k < ns; ++k) (void)hipStreamWaitEvent(c->streams[k], c->ev_fork, 0);
  }
  for (size_t q = 0; q < chunks.size(); ++q) {
    LaunchCtx C = sub(L, chunks[q].first, chunks[q].second);
    if (ns > 1) C.stream = c->streams[q % ns];
    run_forward_chunk(C, N, S, {S - 1}, true);
    run_backward_chunk(C, N, S, {S - 1}, scale, c->ck_every, c->ws2, c->seg);
  }
  if (ns > 1) {
    for (int k = 0; k < ns; ++k) {
      (void)hipEventRecord(c->ev_join[k], c->streams[k]);
      (void)hipStreamWaitEvent(L.stream, c->ev_join[k], 0);
    }
  }
  if (L.reqs.r[0].loss_out) run_finish_forward(L, N);
  run_finish_backward(L, N, scale);
}

}  // namespace

extern "C" {

pty_status pty_workspace_bytes(const pty_geometry* g, int32_t max_batch, int32_t checkpoint_every,
                               size_t* bytes) {
  std::string err;
  pty_status st = validate_geometry(g, err);
  if (st != PTY_OK) return st;
  if (!bytes || max_batch < 0 || checkpoint_every < 1) return PTY_EINVAL;
  *bytes = ctx_sizes(g, max_batch, std::min<int>(checkpoint_every, g->n_slices)).bytes;
  return PTY_OK;
}

int32_t pty_checkpoint_every(const pty_ctx* ctx) { return ctx ? ctx->ck_every : 0; }

pty_status pty_create_ex(const pty_geometry* g, const pty_options* o, pty_ctx** out) {
  if (!out || !o) return PTY_EINVAL;
  *out = nullptr;
  std::string err;
  pty_status st = validate_geometry(g, err);
  if (st != PTY_OK) return st;
  const int max_batch = o->max_batch, checkpoint_every = o->checkpoint_every;
  const size_t hbm_budget = o->hbm_budget;
  if (max_batch < 0 || checkpoint_every < 0 || max_batch > kMaxItems) return PTY_EINVAL;
  const int ck_elem = o->checkpoint_half ? 4 : 8;
  const int S = g->n_slices;
  int k = checkpoint_every;
  if (k == 0) {
    k = 1;
    if (hbm_budget > 0) {
      while (k <= S && ctx_sizes(g, max_batch, k, ck_elem, o->lsqml != 0).bytes > hbm_budget) ++k;
      if (k > S) return PTY_ENOMEM;
    }
  }
  k = std::min(k, S);
  pty_ctx* c = new pty_ctx();
  c->g = *g;
  c->dz.assign(g->dz ? g->dz : nullptr, g->dz ? g->dz + std::max(S - 1, 0) : nullptr);
  c->g.dz = c->dz.data();
  c->max_batch = max_batch;
  c->ck_every = k;
  c->n_ck = (S + k - 1) / k;
  c->ck_half = o->checkpoint_half ? 1 : 0;
  c->sz = ctx_sizes(g, max_batch, k, ck_elem, o->lsqml != 0);
  const int N = g->N, M = g->n_modes;
  const size_t N2 = (size_t)N * N;
  std::string& e = c->err;
  auto fail = [&](pty_status s) { pty_destroy(c); return s; };
  if ((st = dmalloc(&c->tw, N, e)) || (st = dmalloc(&c->prop, (size_t)std::max(S - 1, 0) * N2, e)) ||
      (st = dmalloc(&c->phat, (size_t)M * N2, e)) || (st = dmalloc(&c->gphat, (size_t)M * N2, e)) ||
      (st = dmalloc(&c->gprobe, (size_t)M * N2, e)) ||
      (st = dmalloc(&c->gobj, (size_t)S * g->obj_h * g->obj_w, e)) ||
      (st = dmalloc(&c->gpos, (size_t)g->n_positions * 2, e)) || (st = dmalloc(&c->flags, 4, e)))
    return fail(st);
  if (o->lsqml) {
    const size_t HW = (size_t)g->obj_h * g->obj_w;
    if ((st = dmalloc(&c->lsq_w, (size_t)S * HW, e)) || (st = dmalloc(&c->lsq_part, (size_t)kLsqSplit * N2, e)) ||
        (st = dmalloc(&c->lsq_wp, N2, e)) || (st = dmalloc(&c->lsq_tau, HW, e)) ||
        (st = dmalloc(&c->lsq_sums, (size_t)S * lsq_blocks(HW) * 3 + 2 * S + 2, e)) ||
        (st = dmalloc(&c->lsq_wscr, (size_t)max_batch * N2, e)))
      return fail(st);
  }
  if (max_batch > 0) {
    const int nblk = col_blocks(N);
    if ((st = dmalloc(&c->ws, c->sz.tiles * N2, e)) || (st = dmalloc(&c->ck, c->sz.ck_tiles * N2 * ck_elem, e)) ||
        (st = dmalloc(&c->seg, c->sz.seg_tiles * N2 * ck_elem, e)) || (st = dmalloc(&c->ws2, c->sz.ws2_tiles * N2, e)) ||
        (st = dmalloc(&c->items, (size_t)max_batch, e)) || (st = dmalloc(&c->ramps, (size_t)max_batch * 2 * N, e)) ||
        (st = dmalloc(&c->emax, (size_t)max_batch * S * 2, e)) || (st = dmalloc(&c->cscr, (size_t)max_batch * N2, e)) ||
        (st = dmalloc(&c->loss_part, (size_t)max_batch * nblk, e)) ||
        (st = dmalloc(&c->pos_part, (size_t)max_batch * M * nblk * 2, e)))
      return fail(st);
  }
  std::vector<float2> tw = roots(N);
  if (hipMemcpy(c->tw, tw.data(), N * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess) return fail(PTY_EHIP);
  std::vector<uint8_t> mask;
  if (g->bandlimit_mask) mask.assign(g->bandlimit_mask, g->bandlimit_mask + N2);
  c->g.bandlimit_mask = nullptr;   // copied above; the caller's array is not kept
  static_assert(sizeof(pty_host::F2) == sizeof(float2) && sizeof(pty_host::F4) == sizeof(float4),
                "host propagator tables are copied as float2 / float4");
  std::vector<uint8_t> live(N, 0);
  std::vector<pty_host::F4> py_all;
  std::vector<pty_host::F2> px_all;
  bool sep = S > 1;
  for (int i = 0; i < S - 1; ++i) {
    std::vector<pty_host::F2> H =
        pty_host::propagator(N, g->dx, g->wavelength, c->dz[i], g->bandlimit, g->tilt_y, g->tilt_x, mask);
    if (hipMemcpy(c->prop + (size_t)i * N2, H.data(), N2 * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess)
      return fail(PTY_EHIP);
    for (size_t e = 0; e < N2; ++e)
      if (H[e].x != 0.f || H[e].y != 0.f) live[e % N] = 1;
    std::vector<pty_host::F4> py;
    std::vector<pty_host::F2> px;
    if (sep && pty_host::separable_propagator(N, g->dx, g->wavelength, c->dz[i], g->bandlimit, g->tilt_y,
                                              g->tilt_x, mask, py, px)) {
      py_all.insert(py_all.end(), py.begin(), py.end());
      px_all.insert(px_all.end(), px.begin(), px.end());
    } else {
      sep = false;
    }
  }
  if (sep) {
    if ((st = dmalloc(&c->prop_y, py_all.size(), e)) || (st = dmalloc(&c->prop_x, px_all.size(), e))) return fail(st);
    if (hipMemcpy(c->prop_y, py_all.data(), py_all.size() * sizeof(float4), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->prop_x, px_all.data(), px_all.size() * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess)
      return fail(PTY_EHIP);
  }
  // columns of the row spectrum that every propagator zeroes (band limit):
  // the propagation column passes skip them and their consumers read zeros
  if (S > 1 && std::find(live.begin(), live.end(), 0) != live.end()) {
    if ((st = dmalloc(&c->live, (size_t)N, e))) return fail(st);
    if (hipMemcpy(c->live, live.data(), N, hipMemcpyHostToDevice) != hipSuccess) return fail(PTY_EHIP);
    // a symmetric band |k_x| <= K (any circular limit) is tested without the table
    c->live_k = pty_host::live_interval(live, N);
    const int nb = col_blocks(N), cb = N / nb;
    for (int q = 0; q < nb; ++q)
      for (int x = q * cb; x < (q + 1) * cb; ++x)
        if (live[x]) c->live_blocks |= 1u << q;
  }
  if (hipMemset(c->flags, 0, 4 * sizeof(int)) != hipSuccess) return fail(PTY_EHIP);
  // this device's copy of the static scratch array (pty_forward_static)
  void* sp = nullptr;
  const hipError_t se = scratch_address(&sp);
  if (se != hipSuccess) {
    c->err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(se);
    return fail(PTY_EHIP);
  }
  *out = c;
  return PTY_OK;
}

pty_status pty_create(const pty_geometry* g, int32_t max_batch, int32_t checkpoint_every, size_t hbm_budget,
                      pty_ctx** out) {
  pty_options o{};
  o.max_batch = max_batch;
  o.checkpoint_every = checkpoint_every;
  o.hbm_budget = hbm_budget;
  o.checkpoint_half = 0;
  o.lsqml = 0;
  return pty_create_ex(g, &o, out);
}

pty_status pty_workspace_bytes_ex(const pty_geometry* g, const pty_options* o, size_t* bytes) {
  std::string err;
  pty_status st = validate_geometry(g, err);
  if (st != PTY_OK) return st;
  if (!bytes || !o || o->max_batch < 0 || o->checkpoint_every < 1) return PTY_EINVAL;
  *bytes = ctx_sizes(g, o->max_batch, std::min<int>(o->checkpoint_every, g->n_slices), o->checkpoint_half ? 4 : 8,
                     o->lsqml != 0).bytes;
  return PTY_OK;
}

int32_t pty_checkpoint_half(const pty_ctx* ctx) { return ctx ? ctx->ck_half : 0; }

void pty_destroy(pty_ctx* c) {
  if (!c) return;
  dfree(c->tw); dfree(c->prop); dfree(c->phat); dfree(c->gphat); dfree(c->gprobe); dfree(c->gobj);
  dfree(c->gpos); dfree(c->flags); dfree(c->ws); dfree(c->ws2); dfree(c->ck); dfree(c->seg);
  dfree(c->items); dfree(c->ramps); dfree(c->loss_part); dfree(c->pos_part);
  if (c->spec_plan_ok) (void)hipfftDestroy(c->spec_plan);
  dfree(c->spec);
  dfree(c->support); dfree(c->support_real); dfree(c->blur); dfree(c->lowpass); dfree(c->deramp); dfree(c->reg_part); dfree(c->emax); dfree(c->live);
  dfree(c->prop_y); dfree(c->prop_x); dfree(c->cscr);
  dfree(c->lsq_w); dfree(c->lsq_part); dfree(c->lsq_wp); dfree(c->lsq_sums); dfree(c->lsq_tau); dfree(c->lsq_wscr);
  for (int k = 0; k < kMaxStreams; ++k) {
    if (c->ev_join[k]) (void)hipEventDestroy(c->ev_join[k]);
    if (c->streams[k]) (void)hipStreamDestroy(c->streams[k]);
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  delete c;
}

const char* pty_last_error(const pty_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

pty_status pty_check(pty_ctx* c, void* stream) {
  if (!c) return PTY_EINVAL;
  HIPCHECK(c, hipStreamSynchronize((hipStream_t)stream));
  int f = 0;
  HIPCHECK(c, hipMemcpy(&f, c->flags, sizeof(int), hipMemcpyDeviceToHost));
  if (f) HIPCHECK(c, hipMemset(c->flags, 0, sizeof(int)));
  if (f & kFlagBounds) { c->err = "a probe window left the object"; return PTY_EBOUNDS; }
  if (f & kFlagNonFinite) { c->err = "non-finite loss or detector weight"; return PTY_ENONFINITE; }
  return PTY_OK;
}

pty_status pty_forward(pty_ctx* c, void* stream, const pty_c64* probe, const pty_c64* object,
                       const float* positions, const int32_t* batch_idx, int32_t B, const float* patterns,
                       float* intensities, double* loss) {
  pty_status st = check_call(c, probe, object, positions, batch_idx, B);
  if (st != PTY_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  c->tape_valid = false;
  const int N = c->g.N, S = c->g.n_slices;
  { ProfScope p(P_PLAIN2D, s); launch_plain2d(N, s, c->tw, (const float2*)probe, c->phat, c->g.n_modes, false, 1.f / N, false); }
  ReqDev r = base_req(c);
  r.obj = (const float2*)object;
  r.positions = positions;
  r.batch_idx = batch_idx;
  r.patterns = patterns;
  r.I_out = intensities;
  r.loss_out = (patterns && loss) ? loss : nullptr;
  LaunchCtx L = ctx_launch(c, s, r, B);
  run_prepare(L, N);
  for (auto& ch : split_chunks(B, c->chunk)) run_forward_chunk(sub(L, ch.first, ch.second), N, S, {S - 1}, false);
  if (r.loss_out) run_finish_forward(L, N);
  HIPCHECK(c, hipGetLastError());
  return PTY_OK;
}

static_assert(sizeof(Item) == 40, "pty_forward_static documents 40-byte item descriptors");

pty_status pty_forward_static(pty_ctx* c, void* stream, const pty_c64* probe, const pty_c64* object,
                              const float* positions, const int32_t* batch_idx, int32_t B, const float* patterns,
                              float* intensities, double* loss) {
  if (!c) return PTY_EINVAL;
  if (!probe || !object || !positions || !batch_idx) { c->err = "NULL input pointer"; return PTY_EINVAL; }
  const int N = c->g.N, S = c->g.n_slices, M = c->g.n_modes;
  const size_t N2 = (size_t)N * N;
  if (B < 1 || B > kMaxItems) {
    c->err = "batch " + std::to_string(B) + " outside [1, " + std::to_string(kMaxItems) + "]";
    return PTY_EINVAL;
  }
  // pieces of the static array, each 256-byte aligned
  const size_t o_phat = 0;
  const size_t o_items = o_phat + align256((size_t)M * N2 * sizeof(float2));
  const size_t o_ramps = o_items + align256((size_t)B * sizeof(Item));
  const size_t o_loss = o_ramps + align256((size_t)B * 2 * N * sizeof(float2));
  const size_t o_ws = o_loss + align256((size_t)B * col_blocks(N) * sizeof(float));
  const size_t need = o_ws + align256((size_t)B * M * N2 * sizeof(float2));
  if (need > PTY_STATIC_SCRATCH_BYTES) {
    c->err = "the call needs " + std::to_string(need) + " bytes of static scratch, more than the " +
             std::to_string((size_t)PTY_STATIC_SCRATCH_BYTES) + " it has";
    return PTY_EINVAL;
  }
  void* sp = nullptr;
  HIPCHECK(c, scratch_address(&sp));
  unsigned char* base = static_cast<unsigned char*>(sp);
  float2* phat = reinterpret_cast<float2*>(base + o_phat);
  hipStream_t s = (hipStream_t)stream;
  c->tape_valid = false;
  { ProfScope p(P_PLAIN2D, s); launch_plain2d(N, s, c->tw, (const float2*)probe, phat, M, false, 1.f / N, false); }
  ReqDev r = base_req(c);
  r.phat = phat;
  r.gphat = nullptr;
  r.obj = (const float2*)object;
  r.positions = positions;
  r.batch_idx = batch_idx;
  r.patterns = patterns;
  r.I_out = intensities;
  r.loss_out = (patterns && loss) ? loss : nullptr;
  LaunchCtx L = ctx_launch(c, s, r, B);
  L.items = reinterpret_cast<Item*>(base + o_items);
  L.ramps = reinterpret_cast<float2*>(base + o_ramps);
  L.loss_part = reinterpret_cast<float*>(base + o_loss);
  L.ws = reinterpret_cast<float2*>(base + o_ws);
  L.ck = nullptr;
  L.pos_part = nullptr;
  L.cscr = nullptr;
  run_prepare(L, N);
  for (auto& ch : split_chunks(B, c->chunk)) run_forward_chunk(sub(L, ch.first, ch.second), N, S, {S - 1}, false);
  if (r.loss_out) run_finish_forward(L, N);
  HIPCHECK(c, hipGetLastError());
  return PTY_OK;
}

pty_status pty_forward_save(pty_ctx* c, void* stream, const pty_c64* probe, const pty_c64* object,
                            const float* positions, const float* patterns, const int32_t* batch_idx, int32_t B,
                            float* intensities, double* loss) {
  pty_status st = check_call(c, probe, object, positions, batch_idx, B);
  if (st != PTY_OK) return st;
  if (!patterns) { c->err = "patterns are required for the gradient"; return PTY_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  c->tape_valid = false;
  const int N = c->g.N, S = c->g.n_slices;
  { ProfScope p(P_PLAIN2D, s); launch_plain2d(N, s, c->tw, (const float2*)probe, c->phat, c->g.n_modes, false, 1.f / N, false); }
  ReqDev r = base_req(c);
  r.obj = (const float2*)object;
  r.positions = positions;
  r.batch_idx = batch_idx;
  r.patterns = patterns;
  r.I_out = intensities;
  r.loss_out = loss;
  LaunchCtx L = ctx_launch(c, s, r, B);
  run_prepare(L, N);
  for (auto& ch : split_chunks(B, c->chunk)) run_forward_chunk(sub(L, ch.first, ch.second), N, S, {S - 1}, true);
  if (loss) run_finish_forward(L, N);
  HIPCHECK(c, hipGetLastError());
  c->tape = L;
  c->tape_valid = true;
  return PTY_OK;
}

namespace {
pty_status backward_impl(pty_ctx* c, void* stream, double grad_scale, const double* scale_dev, pty_c64* g_object,
                         pty_c64* g_probe, float* g_pos, uint32_t flags);
}

pty_status pty_backward(pty_ctx* c, void* stream, double grad_scale, pty_c64* g_object, pty_c64* g_probe,
                        float* g_pos, uint32_t flags) {
  return backward_impl(c, stream, grad_scale, nullptr, g_object, g_probe, g_pos, flags);
}

pty_status pty_backward_dev(pty_ctx* c, void* stream, const double* grad_scale, pty_c64* g_object,
                            pty_c64* g_probe, float* g_pos, uint32_t flags) {
  if (c && !grad_scale) { c->err = "grad_scale is NULL"; return PTY_EINVAL; }
  return backward_impl(c, stream, 1.0, grad_scale, g_object, g_probe, g_pos, flags);
}

}  // extern "C"

namespace {
pty_status backward_impl(pty_ctx* c, void* stream, double grad_scale, const double* scale_dev, pty_c64* g_object,
                         pty_c64* g_probe, float* g_pos, uint32_t flags) {
  if (!c) return PTY_EINVAL;
  if (!c->tape_valid) { c->err = "pty_backward needs a preceding pty_forward_save"; return PTY_ESTATE; }
  hipStream_t s = (hipStream_t)stream;
  const int N = c->g.N, S = c->g.n_slices;
  const bool acc = (flags & PTY_ACCUMULATE) != 0;
  LaunchCtx L = c->tape;
  L.stream = s;
  ReqDev& r = L.reqs.r[0];
  const bool dense = (flags & PTY_POS_DENSE) != 0;
  r.gobj = (float2*)g_object;
  r.gpos = dense ? nullptr : g_pos;
  r.gpos_dense = dense ? g_pos : nullptr;
  r.accumulate = acc ? 1 : 0;
  if (dense && g_pos && !acc) {
    ProfScope p(P_FILL, s);
    launch_fill(s, g_pos, (size_t)c->g.n_positions * 2, 0.f);
  }
  r.I_out = nullptr;
  r.loss_out = nullptr;
  r.gphat = g_probe ? c->gphat : nullptr;
  r.scale_dev = scale_dev;
  if (g_object && !acc) {
    ProfScope p(P_FILL, s);
    launch_fill(s, (float*)g_object, (size_t)S * c->g.obj_h * c->g.obj_w * 2, 0.f);
  }
  const auto chunks = split_chunks(L.n_items, c->chunk);
  set_chain_final(L, N, chunks.size() == 1);
  for (auto& ch : chunks)
    run_backward_chunk(sub(L, ch.first, ch.second), N, S, {S - 1}, (float)grad_scale, c->ck_every, c->ws2, c->seg);
  run_finish_backward(L, N, (float)grad_scale);
  if (g_probe)
  { ProfScope p(P_PLAIN2D, s); launch_plain2d(N, s, c->tw, c->gphat, (float2*)g_probe, c->g.n_modes, true, 1.f / N, acc); }
  c->tape_valid = false;
  HIPCHECK(c, hipGetLastError());
  return PTY_OK;
}
}  // namespace

extern "C" {

pty_status pty_loss_and_grad(pty_ctx* c, void* stream, const pty_c64* probe, const pty_c64* object,
                             const float* positions, const float* patterns, const int32_t* batch_idx, int32_t B,
                             double* loss, pty_c64* g_object, pty_c64* g_probe, float* g_pos, uint32_t flags) {
  pty_status st = check_call(c, probe, object, positions, batch_idx, B);
  if (st != PTY_OK) return st;
  if (!patterns) { c->err = "patterns are required for the gradient"; return PTY_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  c->tape_valid = false;
  const int N = c->g.N, S = c->g.n_slices;
  const bool acc = (flags & PTY_ACCUMULATE) != 0;
  { ProfScope p(P_PLAIN2D, s); launch_plain2d(N, s, c->tw, (const float2*)probe, c->phat, c->g.n_modes, false, 1.f / N, false); }
  ReqDev r = base_req(c);
  r.obj = (const float2*)object;
  r.positions = positions;
  r.batch_idx = batch_idx;
  r.patterns = patterns;
  r.loss_out = loss;
  r.gobj = (float2*)g_object;
  const bool dense = (flags & PTY_POS_DENSE) != 0;
  r.gpos = dense ? nullptr : g_pos;
  r.gpos_dense = dense ? g_pos : nullptr;
  r.accumulate = acc ? 1 : 0;
  r.gphat = g_probe ? c->gphat : nullptr;
  if (dense && g_pos && !acc) {
    ProfScope p(P_FILL, s);
    launch_fill(s, g_pos, (size_t)c->g.n_positions * 2, 0.f);
  }
  if (g_object && !acc) {
    ProfScope p(P_FILL, s);
    launch_fill(s, (float*)g_object, (size_t)S * c->g.obj_h * c->g.obj_w * 2, 0.f);
  }
  LaunchCtx L = ctx_launch(c, s, r, B);
  run_fused(c, L, 1.f);
  if (g_probe) { ProfScope p(P_PLAIN2D, s); launch_plain2d(N, s, c->tw, c->gphat, (float2*)g_probe, c->g.n_modes, true, 1.f / N, acc); }
  HIPCHECK(c, hipGetLastError());
  return PTY_OK;
}

}  // extern "C"

namespace {

// Optimiser step of one variable with n real components.
// One variable's update. Adam takes step t from the host, or, with t_dev,
// reads it on the device (t = *t_dev + 1).
void opt_update(hipStream_t s, const pty_optim* o, int64_t t, const int64_t* t_dev, float* th, const float* g,
                float* m, float* v, double lr, size_t n) {
  if (lr == 0.0 || n == 0) return;
  if (o->kind == PTY_OPT_SGD) {
    launch_sgd(s, th, g, n, (float)lr);
  } else if (t_dev) {
    launch_adam_dev(s, th, g, m, v, n, lr, t_dev, o->beta1, o->beta2, (float)o->eps);
  } else {
    const AdamFactors f = adam_factors(lr, o->beta1, o->beta2, t);
    launch_adam(s, th, g, m, v, n, f.step_size, f.inv_sqrt_bc2, o->beta1, o->beta2, (float)o->eps);
  }
}

pty_status check_state(pty_ctx* c, const pty_state* st, const pty_optim* o) {
  if (!st || !o || !st->probe || !st->object || !st->positions) { c->err = "NULL state"; return PTY_EINVAL; }
  if (o->kind != PTY_OPT_SGD && o->kind != PTY_OPT_ADAM && o->kind != PTY_OPT_EPIE) {
    c->err = "unknown optimiser";
    return PTY_EINVAL;
  }
  if (o->kind == PTY_OPT_ADAM) {
    if ((o->lr_object != 0 && (!st->m_object || !st->v_object)) || (o->lr_probe != 0 && (!st->m_probe || !st->v_probe)) ||
        (o->lr_pos != 0 && (!st->m_pos || !st->v_pos))) {
      c->err = "Adam needs moment buffers";
      return PTY_EINVAL;
    }
  }
  return PTY_OK;
}

void apply_optimizer(pty_ctx* c, hipStream_t s, pty_state* st, const pty_optim* o) {
  ProfScope p(P_OPTIM, s);
  const pty_geometry& g = c->g;
  const size_t nO = (size_t)g.n_slices * g.obj_h * g.obj_w * 2;
  const size_t nP = (size_t)g.n_modes * g.N * g.N * 2;
  const size_t nX = (size_t)g.n_positions * 2;
  const int64_t t = st->step + 1;
  const int64_t* t_dev = o->kind == PTY_OPT_ADAM ? st->step_dev : nullptr;
  opt_update(s, o, t, t_dev, (float*)st->object, (const float*)c->gobj, st->m_object, st->v_object, o->lr_object,
             nO);
  opt_update(s, o, t, t_dev, (float*)st->probe, (const float*)c->gprobe, st->m_probe, st->v_probe, o->lr_probe,
             nP);
  opt_update(s, o, t, t_dev, st->positions, c->gpos, st->m_pos, st->v_pos, o->lr_pos, nX);
  if (o->kind == PTY_OPT_ADAM) {
    // the device count advances after the last update that read it
    if (st->step_dev) launch_step_advance(s, st->step_dev);
    else st->step = t;
  }
}

}  // namespace

namespace {

// Cost regularizers: gradients into the dense gradients, cost added to *loss.
// Fails (PTY_EHIP, message in c->err) when the copy or a hipFFT transform of
// the spectral term is refused.
pty_status apply_cost_regularizers(pty_ctx* c, hipStream_t s, const pty_state* st, double* loss) {
  if (!c->reg_on) return PTY_OK;
  const pty_geometry& g = c->g;
  int nb = 0;
  if (c->rg.obj_l2 != 0.f || c->rg.obj_l1 != 0.f || c->rg.obj_tikhonov != 0.f || c->rg.obj_tv != 0.f ||
      c->rg.layers_tikhonov != 0.f || c->rg.layers_tv != 0.f || c->rg.obj_phase_l1 != 0.f)
    nb = launch_reg_object(s, (const float2*)st->object, c->gobj, g.n_slices, g.obj_h, g.obj_w, c->rg, c->reg_part);
  int np = 0;
  if (c->probe_l2 != 0.f)
    np = launch_reg_probe(s, (const float2*)st->probe, c->gprobe, (size_t)g.n_modes * g.N * g.N, c->probe_l2,
                          c->reg_part + 4096);
  int ns = 0;
  if (c->obj_spec_l1 != 0.f && c->spec_plan_ok) {
    // |F2 O|: forward FFT of a copy of the slices, the L1 step, inverse FFT,
    // added into the object gradient (every transform in place, one plan)
    const size_t HW = (size_t)g.obj_h * g.obj_w, n = HW * g.n_slices;
    HIPCHECK(c, hipMemcpyAsync(c->spec, st->object, n * sizeof(float2), hipMemcpyDeviceToDevice, s));
    if (hipfftSetStream(c->spec_plan, s) != HIPFFT_SUCCESS ||
        hipfftExecC2C(c->spec_plan, (hipfftComplex*)c->spec, (hipfftComplex*)c->spec, HIPFFT_FORWARD) !=
            HIPFFT_SUCCESS) {
      c->err = "hipFFT forward transform of the object spectrum failed";
      return PTY_EHIP;
    }
    ns = launch_spec_l1(s, c->spec, n, HW, c->obj_spec_l1, c->reg_part + 3 * 4096);
    if (hipfftExecC2C(c->spec_plan, (hipfftComplex*)c->spec, (hipfftComplex*)c->spec, HIPFFT_BACKWARD) !=
        HIPFFT_SUCCESS) {
      c->err = "hipFFT inverse transform of the object spectrum failed";
      return PTY_EHIP;
    }
    launch_cadd_inplace(s, c->gobj, c->spec, n);
  }
  int nq = 0;
  if (c->probe_phase_tik != 0.f || c->probe_phase_tv != 0.f) {
    // the phase plate acts on the step's probe spectrum (phat, from the state
    // before the update); its gradient, taken with respect to that spectrum in
    // the free gphat buffer, reaches the probe through the adjoint of the
    // unitary DFT
    nq = launch_reg_probe_phase(s, c->phat, c->gphat, g.n_modes, g.N, c->probe_phase_tik, c->probe_phase_tv,
                                c->rg.tv_delta, c->reg_part + 8192);
    launch_plain2d(g.N, s, c->tw, c->gphat, c->gprobe, g.n_modes, true, 1.f / g.N, true);
  }
  if (loss) {
    if (nb) launch_add_cost(s, c->reg_part, nb, loss);
    if (np) launch_add_cost(s, c->reg_part + 4096, np, loss);
    if (nq) launch_add_cost(s, c->reg_part + 8192, nq, loss);
    if (ns) launch_add_cost(s, c->reg_part + 3 * 4096, ns, loss);
  }
  return PTY_OK;
}

// Constraint regularizers on the updated state.
void apply_constraints(pty_ctx* c, hipStream_t s, pty_state* st) {
  if (!c->con_on) return;
  const pty_geometry& g = c->g;
  const size_t HW = (size_t)g.obj_h * g.obj_w;
  if (c->amp_clamp) launch_amp_clamp(s, (float2*)st->object, HW * g.n_slices, c->amp_min, c->amp_max);
  if (c->blur) launch_layer_blur(s, (float2*)st->object, g.n_slices, HW, c->blur, c->blur_r);
  // the object gradient buffer is free once the optimiser has run
  if (c->lowpass) launch_lowpass(s, (float2*)st->object, c->gobj, g.n_slices, g.obj_h, g.obj_w, c->lowpass, c->lowpass_r);
  if (c->deramp)
    launch_deramp(s, (float2*)st->object, g.n_slices, g.obj_h, g.obj_w, c->deramp, c->deramp + 3 * g.n_slices);
  if (c->support) {
    const int N = g.N, M = g.n_modes;
    launch_plain2d(N, s, c->tw, (const float2*)st->probe, c->gphat, M, false, 1.f / N, false);
    launch_mask_tiles(s, c->gphat, c->support, (size_t)M * N * N, N * N);
    launch_plain2d(N, s, c->tw, c->gphat, (float2*)st->probe, M, true, 1.f / N, false);
  }
  if (c->support_real)
    launch_mask_tiles(s, (float2*)st->probe, c->support_real, (size_t)g.n_modes * g.N * g.N, g.N * g.N);
}

}  // namespace

extern "C" pty_status pty_set_regularizers(pty_ctx* c, const pty_regularizers* r) {
  if (!c) return PTY_EINVAL;
  dfree(c->support);
  dfree(c->support_real);
  dfree(c->blur);
  dfree(c->lowpass);
  dfree(c->deramp);
  if (c->spec_plan_ok) (void)hipfftDestroy(c->spec_plan);
  c->spec_plan_ok = false;
  dfree(c->spec);
  c->reg_on = c->con_on = false;
  c->probe_phase_tik = c->probe_phase_tv = c->obj_spec_l1 = 0.f;
  c->amp_clamp = 0;
  c->blur_r = c->lowpass_r = 0;
  if (!r) return PTY_OK;
  const double w[11] = {r->obj_l2, r->probe_l2, r->obj_l1, r->obj_tikhonov, r->obj_tv, r->layers_tikhonov,
                        r->layers_tv, r->obj_phase_l1, r->obj_spectrum_l1, r->probe_phase_tikhonov,
                        r->probe_phase_tv};
  for (double x : w)
    if (!(x >= 0.0) || !std::isfinite(x)) { c->err = "regularizer weights must be finite and >= 0"; return PTY_EINVAL; }
  if ((r->obj_tv > 0 || r->layers_tv > 0 || r->probe_phase_tv > 0) && !(r->tv_delta > 0)) {
    c->err = "tv_delta must be > 0";
    return PTY_EINVAL;
  }
  if (r->amp_clamp && !(r->amp_min >= 0 && r->amp_max >= r->amp_min)) { c->err = "need 0 <= amp_min <= amp_max"; return PTY_EINVAL; }
  if (r->layer_sigma < 0 || (r->layer_sigma > 0 && c->g.n_slices > kMaxBlurSlices)) {
    c->err = "layer blur needs sigma >= 0 and at most 64 slices";
    return PTY_EINVAL;
  }
  if (!(r->obj_lowpass_sigma >= 0 && r->obj_lowpass_sigma <= 64)) {
    c->err = "object low pass needs 0 <= sigma <= 64 pixels";
    return PTY_EINVAL;
  }
  c->rg = RegDev{(float)r->obj_l2, (float)r->obj_l1, (float)r->obj_tikhonov, (float)r->obj_tv,
                 (float)r->layers_tikhonov, (float)r->layers_tv, (float)r->tv_delta, (float)r->obj_phase_l1};
  c->probe_l2 = (float)r->probe_l2;
  c->probe_phase_tik = (float)r->probe_phase_tikhonov;
  c->probe_phase_tv = (float)r->probe_phase_tv;
  for (double x : w) c->reg_on = c->reg_on || x > 0;
  pty_status st;
  // cost partial sums: object terms, probe L2, probe phase plate, object spectrum (4096 each)
  if (!c->reg_part && (st = dmalloc(&c->reg_part, 4 * 4096, c->err))) return st;
  if (r->obj_spectrum_l1 > 0) {
    const int S = c->g.n_slices, H = c->g.obj_h, W = c->g.obj_w;
    if ((st = dmalloc(&c->spec, (size_t)S * H * W, c->err))) return st;
    int dims[2] = {H, W};
    if (hipfftPlanMany(&c->spec_plan, 2, dims, nullptr, 1, H * W, nullptr, 1, H * W, HIPFFT_C2C, S) != HIPFFT_SUCCESS) {
      c->err = "hipfftPlanMany failed for the object spectrum";
      return PTY_EHIP;
    }
    c->spec_plan_ok = true;
    c->obj_spec_l1 = (float)r->obj_spectrum_l1;
  }
  c->amp_clamp = r->amp_clamp ? 1 : 0;
  c->amp_min = (float)r->amp_min;
  c->amp_max = (float)r->amp_max;
  const size_t N2 = (size_t)c->g.N * c->g.N;
  if (r->probe_support) {
    if ((st = dmalloc(&c->support, N2, c->err))) return st;
    std::vector<uint8_t> m(r->probe_support, r->probe_support + N2);
    for (auto& v : m) v = v ? 1 : 0;
    if (hipMemcpy(c->support, m.data(), N2, hipMemcpyHostToDevice) != hipSuccess) return PTY_EHIP;
  }
  if (r->probe_support_real) {
    if ((st = dmalloc(&c->support_real, N2, c->err))) return st;
    std::vector<uint8_t> m(r->probe_support_real, r->probe_support_real + N2);
    for (auto& v : m) v = v ? 1 : 0;
    if (hipMemcpy(c->support_real, m.data(), N2, hipMemcpyHostToDevice) != hipSuccess) return PTY_EHIP;
  }
  if (r->layer_sigma > 0 && c->g.n_slices > 1) {
    c->blur_r = (int)std::ceil(3.0 * r->layer_sigma);
    std::vector<float> gw(c->blur_r + 1);
    for (int k = 0; k <= c->blur_r; ++k) gw[k] = (float)std::exp(-0.5 * (k / r->layer_sigma) * (k / r->layer_sigma));
    if ((st = dmalloc(&c->blur, gw.size(), c->err))) return st;
    if (hipMemcpy(c->blur, gw.data(), gw.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return PTY_EHIP;
  }
  if (r->obj_lowpass_sigma > 0) {
    const double sg = r->obj_lowpass_sigma;
    c->lowpass_r = (int)std::ceil(3.0 * sg);
    std::vector<double> gd(c->lowpass_r + 1);
    double tot = 0.0;
    for (int t = 0; t <= c->lowpass_r; ++t) {
      gd[t] = std::exp(-0.5 * (t / sg) * (t / sg));
      tot += t ? 2 * gd[t] : gd[t];
    }
    std::vector<float> gw(gd.size());
    for (size_t t = 0; t < gd.size(); ++t) gw[t] = (float)(gd[t] / tot);
    if ((st = dmalloc(&c->lowpass, gw.size(), c->err))) return st;
    if (hipMemcpy(c->lowpass, gw.data(), gw.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return PTY_EHIP;
  }
  if (r->phase_deramp) {
    const size_t n = 3 * (size_t)c->g.n_slices + (size_t)c->g.n_slices * deramp_blocks(c->g.obj_h, c->g.obj_w) * 4;
    if ((st = dmalloc(&c->deramp, n, c->err))) return st;
  }
  c->con_on = c->amp_clamp || c->support || c->support_real || c->blur || c->lowpass || c->deramp;
  return PTY_OK;
}

extern "C" pty_status pty_reconstruct_step(pty_ctx* c, void* stream, pty_state* st, const float* patterns,
                                           const int32_t* batch_idx, int32_t B, const pty_optim* o, double* loss) {
  if (!c) return PTY_EINVAL;
  pty_status s0 = check_state(c, st, o);
  if (s0 != PTY_OK) return s0;
  hipStream_t s = (hipStream_t)stream;
  s0 = check_call(c, st->probe, st->object, st->positions, batch_idx, B);
  if (s0 != PTY_OK) return s0;
  if (!patterns) { c->err = "patterns are required for the gradient"; return PTY_EINVAL; }
  c->tape_valid = false;
  const pty_geometry& g = c->g;
  const int N = g.N, S = g.n_slices;
  { ProfScope p(P_PLAIN2D, s); launch_plain2d(N, s, c->tw, (const float2*)st->probe, c->phat, g.n_modes, false, 1.f / N, false); }
  ReqDev r = base_req(c);
  r.obj = (const float2*)st->object;
  r.positions = st->positions;
  r.batch_idx = batch_idx;
  r.patterns = patterns;
  r.loss_out = loss;
  r.gobj = c->gobj;
  r.gpos_dense = c->gpos;
  r.gphat = c->gphat;
  const bool epie = o->kind == PTY_OPT_EPIE;
  if (epie) {
    // ePIE / 3PIE: the same chain with the modulus update at the detector and
    // per-(position, slice) normalisers recorded by the first forward pass
    r.emax = c->emax;
    r.modulus = 1;
  }
  LaunchCtx L = ctx_launch(c, s, r, B);
  if (epie) {
    L.emax = 1;
    L.resident = 0;
  }
  {
    ProfScope p(P_FILL, s);
    launch_fill(s, (float*)c->gobj, (size_t)S * g.obj_h * g.obj_w * 2, 0.f);
    launch_fill(s, c->gpos, (size_t)g.n_positions * 2, 0.f);
    if (epie) launch_fill(s, c->emax, (size_t)B * S * 2, 0.f);
  }
  run_fused(c, L, 1.f);
  { ProfScope p(P_PLAIN2D, s); launch_plain2d(N, s, c->tw, c->gphat, c->gprobe, g.n_modes, true, 1.f / N, false); }
  if (epie) {
    // the chain produced minus the summed updates: O += beta_O dO, P += beta_P dP / B
    ProfScope p(P_OPTIM, s);
    const size_t nO = (size_t)S * g.obj_h * g.obj_w * 2, nP = (size_t)g.n_modes * N * N * 2;
    if (o->lr_object != 0) launch_sgd(s, (float*)st->object, (const float*)c->gobj, nO, (float)o->lr_object);
    if (o->lr_probe != 0) launch_sgd(s, (float*)st->probe, (const float*)c->gprobe, nP, (float)(o->lr_probe / B));
    { ProfScope q(P_REG, s); apply_constraints(c, s, st); }
    HIPCHECK(c, hipGetLastError());
    return PTY_OK;
  }
  {
    ProfScope p(P_REG, s);
    const pty_status rs = apply_cost_regularizers(c, s, st, loss);
    if (rs != PTY_OK) return rs;
  }
  apply_optimizer(c, s, st, o);
  { ProfScope p(P_REG, s); apply_constraints(c, s, st); }
  HIPCHECK(c, hipGetLastError());
  return PTY_OK;
}

extern "C" pty_status pty_lsqml_step(pty_ctx* c, void* stream, pty_state* st, const pty_illum* il,
                                     const float* patterns, const int32_t* batch_idx, int32_t B, const pty_lsqml* o,
                                     double* loss) {
  if (!c) return PTY_EINVAL;
  if (!st || !il || !o || !st->probe || !st->object || !st->positions) { c->err = "NULL argument"; return PTY_EINVAL; }
  if (!c->lsq_w) { c->err = "context created without the LSQML scratch (pty_options.lsqml = 0)"; return PTY_ESTATE; }
  if (!il->obj_cur || !il->probe_cur || (il->obj_prev == nullptr) != (il->probe_prev == nullptr)) {
    c->err = "illumination sums: obj_cur and probe_cur are required, obj_prev and probe_prev both or neither";
    return PTY_EINVAL;
  }
  const float dO = (float)o->delta_object, dP = (float)o->delta_probe;
  if (!std::isfinite(o->beta_object) || !std::isfinite(o->beta_probe) || !(dO > 0.f) || !(dP > 0.f) ||
      !std::isfinite(o->delta_object) || !std::isfinite(o->delta_probe) || !(o->gamma >= 0.0) ||
      !std::isfinite(o->gamma)) {
    c->err = "LSQML needs finite betas, relative deltas > 0 (in float) and gamma >= 0";
    return PTY_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  pty_status s0 = check_call(c, st->probe, st->object, st->positions, batch_idx, B);
  if (s0 != PTY_OK) return s0;
  if (!patterns) { c->err = "patterns are required"; return PTY_EINVAL; }
  c->tape_valid = false;
  const pty_geometry& g = c->g;
  const int N = g.N, S = g.n_slices, M = g.n_modes;
  const size_t HW = (size_t)g.obj_h * g.obj_w;
  { ProfScope p(P_PLAIN2D, s); launch_plain2d(N, s, c->tw, (const float2*)st->probe, c->phat, M, false, 1.f / N, false); }
  ReqDev r = base_req(c);
  r.obj = (const float2*)st->object;
  r.positions = st->positions;
  r.batch_idx = batch_idx;
  r.patterns = patterns;
  r.loss_out = loss;
  r.gobj = c->gobj;
  r.gpos_dense = c->gpos;
  r.gphat = c->gphat;
  r.modulus = 1;
  r.wsum = c->lsq_w;
  LaunchCtx L = ctx_launch(c, s, r, B);
  L.resident = 0;
  L.wsum = 1;
  L.wscr = L.cscr ? c->lsq_wscr : nullptr;   // the illumination sums follow the reduction mode
  {
    ProfScope p(P_FILL, s);
    launch_fill(s, (float*)c->gobj, (size_t)S * HW * 2, 0.f);
    launch_fill(s, c->gpos, (size_t)g.n_positions * 2, 0.f);
    launch_fill(s, c->lsq_w, (size_t)S * HW, 0.f);
  }
  // the chain accumulates minus the summed directions: gobj = -D, gphat -> gprobe = -dP
  run_fused(c, L, 1.f);
  { ProfScope p(P_PLAIN2D, s); launch_plain2d(N, s, c->tw, c->gphat, c->gprobe, M, true, 1.f / N, false); }
  {
    ProfScope p(P_OPTIM, s);
    launch_lsq_transparency(s, c->items, B, (const float2*)st->object, S, g.obj_h, g.obj_w, N, c->lsq_tau,
                            c->lsq_part, c->lsq_wp);
    // lsq_sums: [S*nb*3 + S] sums and maxima of the object step, [S] alpha_i, [2] probe alpha and max
    const size_t nb3 = (size_t)S * lsq_blocks(HW) * 3 + S;
    launch_lsq_object(s, (float2*)st->object, c->gobj, c->lsq_w, il->obj_cur, il->obj_prev, S, HW, dO, o->gamma,
                      (float)o->beta_object, c->lsq_sums, c->lsq_sums + nb3);
    launch_lsq_probe(s, (float2*)st->probe, c->gprobe, c->lsq_wp, il->probe_cur, il->probe_prev, M, N * N, dP,
                     o->gamma, (float)o->beta_probe, c->lsq_sums + nb3 + S);
  }
  { ProfScope p(P_REG, s); apply_constraints(c, s, st); }
  HIPCHECK(c, hipGetLastError());
  return PTY_OK;
}

// ---------------------------------------------------------------- grouped launches

namespace {

Sizes group_sizes(int N, int max_items, int max_tiles, long long max_ck) {
  Sizes s;
  const size_t N2 = (size_t)N * N;
  const int nblk = col_blocks(N);
  s.tiles = max_tiles;
  s.ck_tiles = max_ck;
  size_t b = align256(N * sizeof(float2));
  b += align256(((size_t)max_tiles + (size_t)max_ck) * N2 * sizeof(float2));
  b += align256((size_t)max_items * sizeof(Item));
  b += align256((size_t)max_items * 2 * N * sizeof(float2));
  b += align256((size_t)max_items * nblk * sizeof(float));
  b += align256((size_t)max_tiles * nblk * 2 * sizeof(float));
  b += align256(4 * sizeof(int));
  b += align256((size_t)max_items * N2 * sizeof(float2));   // ordered reduction scratch
  s.bytes = b;
  return s;
}

}  // namespace

extern "C" {

pty_status pty_group_workspace_bytes(int32_t N, int32_t max_items, int32_t max_tiles, int64_t max_ckpt_tiles,
                                     size_t* bytes) {
  if (!supported_N(N)) return PTY_EUNSUPPORTED;
  if (!bytes || max_items < 1 || max_tiles < 1 || max_ckpt_tiles < 1) return PTY_EINVAL;
  *bytes = group_sizes(N, max_items, max_tiles, max_ckpt_tiles).bytes;
  return PTY_OK;
}

pty_status pty_group_create(int32_t N, int32_t max_items, int32_t max_tiles, int64_t max_ckpt_tiles,
                            pty_group** out) {
  if (!out) return PTY_EINVAL;
  *out = nullptr;
  if (!supported_N(N)) return PTY_EUNSUPPORTED;
  if (max_items < 1 || max_items > kMaxItems || max_tiles < 1 || max_ckpt_tiles < 1) return PTY_EINVAL;
  pty_group* G = new pty_group();
  G->N = N;
  G->max_items = max_items;
  G->max_tiles = max_tiles;
  G->max_ck = max_ckpt_tiles;
  const size_t N2 = (size_t)N * N;
  const int nblk = col_blocks(N);
  pty_status st;
  auto fail = [&](pty_status s) { pty_group_destroy(G); return s; };
  if ((st = dmalloc(&G->tw, N, G->err)) || (st = dmalloc(&G->ws, (size_t)max_tiles * N2, G->err)) ||
      (st = dmalloc(&G->ck, (size_t)max_ckpt_tiles * N2, G->err)) || (st = dmalloc(&G->items, (size_t)max_items, G->err)) ||
      (st = dmalloc(&G->ramps, (size_t)max_items * 2 * N, G->err)) ||
      (st = dmalloc(&G->loss_part, (size_t)max_items * nblk, G->err)) ||
      (st = dmalloc(&G->pos_part, (size_t)max_tiles * nblk * 2, G->err)) || (st = dmalloc(&G->flags, 4, G->err)) ||
      (st = dmalloc(&G->cscr, (size_t)max_items * N2, G->err)))
    return fail(st);
  std::vector<float2> tw = roots(N);
  if (hipMemcpy(G->tw, tw.data(), N * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess) return fail(PTY_EHIP);
  if (hipMemset(G->flags, 0, 4 * sizeof(int)) != hipSuccess) return fail(PTY_EHIP);
  *out = G;
  return PTY_OK;
}

void pty_group_destroy(pty_group* G) {
  if (!G) return;
  dfree(G->tw); dfree(G->ws); dfree(G->ck); dfree(G->items); dfree(G->ramps);
  dfree(G->loss_part); dfree(G->pos_part); dfree(G->flags); dfree(G->cscr);
  delete G;
}

const char* pty_group_last_error(const pty_group* G) { return G ? G->err.c_str() : "NULL group"; }

pty_status pty_group_reconstruct_step(pty_group* G, void* stream, const pty_group_item* items, int32_t n) {
  if (!G) return PTY_EINVAL;
  if (!items || n < 1 || n > kMaxReqs) { G->err = "1 to 16 items per grouped step"; return PTY_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  const int N = G->N;
  LaunchCtx L{};
  L.stream = s;
  L.items = G->items;
  L.ws = G->ws;
  L.ck = G->ck;
  L.ck_half = 0;
  L.ck_spec = 1;   // every slice of every request stored in float
  L.resident = use_resident(items[0].ctx ? items[0].ctx->strategy : PTY_STRATEGY_AUTO, N, 1) ? 1 : 0;
  L.ramps = G->ramps;
  L.tw = G->tw;
  L.loss_part = G->loss_part;
  L.pos_part = G->pos_part;
  L.flags = G->flags;
  int item0 = 0, tile0 = 0, S_max = 0, M_max = 0;
  long long ck0 = 0;
  std::vector<int> last_steps;
  for (int q = 0; q < n; ++q) {
    const pty_group_item& it = items[q];
    pty_ctx* c = it.ctx;
    if (!c || c->g.N != N) { G->err = "item context missing or of another N"; return PTY_EINVAL; }
    pty_status st0 = check_state(c, it.state, it.opt);
    if (st0 != PTY_OK) { G->err = c->err; return st0; }
    if (it.opt->kind == PTY_OPT_EPIE) { G->err = "grouped steps take SGD or Adam"; return PTY_EUNSUPPORTED; }
    if (!it.patterns || !it.batch_idx || it.batch < 1) { G->err = "item needs patterns and a batch"; return PTY_EINVAL; }
    const int M = c->g.n_modes, S = c->g.n_slices;
    ReqDev r = base_req(c);
    r.obj = (const float2*)it.state->object;
    r.positions = it.state->positions;
    r.batch_idx = it.batch_idx;
    r.patterns = it.patterns;
    r.loss_out = it.loss;
    r.gobj = c->gobj;
    r.gpos_dense = c->gpos;
    r.item0 = item0;
    r.n_items = it.batch;
    r.tile_base = tile0;
    r.ck_base = ck0;
    r.ck_every = 1;
    r.n_ck = S;
    L.reqs.r[q] = r;
    item0 += it.batch;
    tile0 += it.batch * M;
    ck0 += (long long)it.batch * M * S;
    S_max = std::max(S_max, S);
    M_max = std::max(M_max, M);
    last_steps.push_back(S - 1);
  }
  if (item0 > G->max_items || tile0 > G->max_tiles || ck0 > G->max_ck) {
    G->err = "grouped step exceeds the group's workspace";
    return PTY_EINVAL;
  }
  L.n_reqs = n;
  L.n_items = item0;
  L.max_modes = M_max;
  // the ordered object-gradient reduction when every request asks for it
  bool ordered = true;
  for (int q = 0; q < n; ++q) ordered &= items[q].ctx->reduce == PTY_REDUCE_ORDERED;
  L.cscr = ordered ? G->cscr : nullptr;
  if (ordered) L.resident = 0;
  // a column block runs when any request has a live column in it
  L.col_live_blocks = 0;
  for (int q = 0; q < n; ++q) {
    if (items[q].ctx->live_blocks == 0) { L.col_live_blocks = 0; break; }
    L.col_live_blocks |= items[q].ctx->live_blocks;
  }
  for (int q = 0; q < n; ++q) {
    pty_ctx* c = items[q].ctx;
    launch_plain2d(N, s, G->tw, (const float2*)items[q].state->probe, c->phat, c->g.n_modes, false, 1.f / N, false);
    launch_fill(s, (float*)c->gobj, (size_t)c->g.n_slices * c->g.obj_h * c->g.obj_w * 2, 0.f);
    launch_fill(s, c->gpos, (size_t)c->g.n_positions * 2, 0.f);
  }
  std::sort(last_steps.begin(), last_steps.end());
  last_steps.erase(std::unique(last_steps.begin(), last_steps.end()), last_steps.end());
  // adjoint step t handles slice S_q - 1 - t of request q; slice 0 at t = S_q - 1
  run_prepare(L, N);
  set_chain_final(L, N, true);
  run_forward_chunk(L, N, S_max, last_steps, true);
  run_backward_chunk(L, N, S_max, last_steps, 1.f, 1, nullptr, nullptr);
  run_finish_forward(L, N);
  run_finish_backward(L, N, 1.f);
  for (int q = 0; q < n; ++q) {
    pty_ctx* c = items[q].ctx;
    launch_plain2d(N, s, G->tw, c->gphat, c->gprobe, c->g.n_modes, true, 1.f / N, false);
    if (apply_cost_regularizers(c, s, items[q].state, items[q].loss) != PTY_OK) {
      G->err = c->err;
      return PTY_EHIP;
    }
    apply_optimizer(c, s, items[q].state, items[q].opt);
    apply_constraints(c, s, items[q].state);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { G->err = hipGetErrorString(e); return PTY_EHIP; }
  return PTY_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- recorded steps

struct pty_step_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  pty_ctx* ctx = nullptr;
};

extern "C" pty_status pty_step_graph_create(pty_ctx* c, void* stream, pty_state* st, const float* patterns,
                                            const int32_t* batch_idx, int32_t B, const pty_optim* o,
                                            double* loss, pty_step_graph** out) {
  if (!c) return PTY_EINVAL;
  if (!out) { c->err = "NULL graph output"; return PTY_EINVAL; }
  *out = nullptr;
  pty_status v = check_state(c, st, o);
  if (v != PTY_OK) return v;
  if (o->kind == PTY_OPT_ADAM && !st->step_dev) {
    c->err = "a recorded Adam step needs the device-side step count (pty_state.step_dev)";
    return PTY_EUNSUPPORTED;
  }
  if (c->reg_on && c->obj_spec_l1 != 0.f) {
    c->err = "the object-spectrum L1 regularizer cannot be recorded";
    return PTY_EUNSUPPORTED;
  }
  {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (g_prof.on) { c->err = "launch timing is enabled"; return PTY_EUNSUPPORTED; }
  }
  hipStream_t s = (hipStream_t)stream;
  HIPCHECK(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  // nothing runs while the stream records; an argument error returns before
  // the first launch and the recording is discarded
  const pty_status rs = pty_reconstruct_step(c, stream, st, patterns, batch_idx, B, o, loss);
  hipGraph_t g = nullptr;
  const hipError_t e_end = hipStreamEndCapture(s, &g);
  if (rs != PTY_OK || e_end != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    if (rs != PTY_OK) return rs;
    c->err = std::string("recording the step failed: ") + hipGetErrorString(e_end);
    return PTY_EHIP;
  }
  hipGraphExec_t x = nullptr;
  const hipError_t e_inst = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e_inst != hipSuccess) {
    (void)hipGraphDestroy(g);
    c->err = std::string("hipGraphInstantiate: ") + hipGetErrorString(e_inst);
    return PTY_EHIP;
  }
  pty_step_graph* G = new (std::nothrow) pty_step_graph;
  if (!G) {
    (void)hipGraphExecDestroy(x);
    (void)hipGraphDestroy(g);
    c->err = "out of host memory";
    return PTY_ENOMEM;
  }
  G->graph = g;
  G->exec = x;
  G->ctx = c;
  *out = G;
  return PTY_OK;
}

extern "C" pty_status pty_step_graph_launch(pty_step_graph* G, void* stream) {
  if (!G) return PTY_EINVAL;
  HIPCHECK(G->ctx, hipGraphLaunch(G->exec, (hipStream_t)stream));
  return PTY_OK;
}

extern "C" void pty_step_graph_destroy(pty_step_graph* G) {
  if (!G) return;
  if (G->exec) (void)hipGraphExecDestroy(G->exec);
  if (G->graph) (void)hipGraphDestroy(G->graph);
  delete G;
}

extern "C" void pty_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = on != 0;
}

extern "C" int32_t pty_profile_select(const char* classes) {
  static_assert(P_NCLASS <= 64, "class mask holds 64 classes");
  uint64_t mask = 0;
  int n = 0;
  if (!classes || !*classes) {
    mask = ~0ull;
    n = P_NCLASS;
  } else {
    std::string all(classes);
    size_t b = 0;
    while (b <= all.size()) {
      size_t e = all.find_first_of(",\n", b);
      if (e == std::string::npos) e = all.size();
      const std::string name = all.substr(b, e - b);
      if (!name.empty()) {
        int k = 0;
        while (k < P_NCLASS && name != kProfNames[k]) ++k;
        if (k == P_NCLASS) return -1;
        if (!((mask >> k) & 1ull)) ++n;
        mask |= 1ull << k;
      }
      b = e + 1;
    }
  }
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.mask = mask;
  return n;
}

extern "C" int32_t pty_profile_collect(char* names, size_t names_len, double* total_ms, int64_t* counts,
                                       int32_t max_entries) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  for (const ProfRec& r : g_prof.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      g_prof.total_ms[r.cls] += ms;
      g_prof.count[r.cls] += 1;
    }
    g_prof.pool.push_back(r.a);
    g_prof.pool.push_back(r.b);
  }
  g_prof.pending.clear();
  std::string all;
  int n = 0;
  for (int k = 0; k < P_NCLASS; ++k) {
    if (g_prof.count[k] == 0) continue;
    if (n < max_entries && total_ms && counts) {
      total_ms[n] = g_prof.total_ms[k];
      counts[n] = g_prof.count[k];
    }
    if (n < max_entries) {
      all += kProfNames[k];
      all += '\n';
    }
    ++n;
    g_prof.total_ms[k] = 0.0;
    g_prof.count[k] = 0;
  }
  if (names && names_len > 0) {
    size_t m = std::min(all.size(), names_len - 1);
    std::memcpy(names, all.data(), m);
    names[m] = '\0';
  }
  return std::min(n, max_entries);
}

extern "C" pty_status pty_set_reduction(pty_ctx* c, int32_t mode) {
  if (!c) return PTY_EINVAL;
  if (mode != PTY_REDUCE_ATOMIC && mode != PTY_REDUCE_ORDERED) { c->err = "unknown reduction mode"; return PTY_EINVAL; }
  c->reduce = mode;
  return PTY_OK;
}

extern "C" pty_status pty_set_chunk(pty_ctx* c, int32_t positions) {
  if (!c) return PTY_EINVAL;
  if (positions < 0) { c->err = "chunk must be >= 0 (0: the whole group)"; return PTY_EINVAL; }
  c->chunk = positions;
  return PTY_OK;
}

extern "C" pty_status pty_set_streams(pty_ctx* c, int32_t n) {
  if (!c) return PTY_EINVAL;
  if (n < 1 || n > kMaxStreams) { c->err = "streams must be in [1, 8]"; return PTY_EINVAL; }
  if (!c->ev_fork) HIPCHECK(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  for (int k = 0; k < n; ++k) {
    if (!c->streams[k]) HIPCHECK(c, hipStreamCreateWithFlags(&c->streams[k], hipStreamNonBlocking));
    if (!c->ev_join[k]) HIPCHECK(c, hipEventCreateWithFlags(&c->ev_join[k], hipEventDisableTiming));
  }
  c->n_streams = n;
  return PTY_OK;
}

extern "C" pty_status pty_set_strategy(pty_ctx* c, int32_t strategy) {
  if (!c) return PTY_EINVAL;
  if (strategy < PTY_STRATEGY_AUTO || strategy > PTY_STRATEGY_RESIDENT) { c->err = "unknown strategy"; return PTY_EINVAL; }
  if (strategy == PTY_STRATEGY_RESIDENT && !resident_supported(c->g.N)) {
    c->err = "the LDS-resident chain needs N = 64 or 128";
    return PTY_EUNSUPPORTED;
  }
  c->strategy = strategy;
  return PTY_OK;
}
