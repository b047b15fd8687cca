// pty_internal.h -- device-side descriptors shared by the kernels and the
// host orchestration of libpty (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>

#include "pty.h"

namespace pty {

constexpr int kFlagBounds = 1;
constexpr int kFlagNonFinite = 2;
constexpr int kMaxReqs = 16;   // reconstructions per shared launch
constexpr int kMaxItems = 65535;   // positions per launch (one grid dimension holds them)

// Adam's per-step factors for step t >= 1: lr / (1 - b1^t) and
// 1 / sqrt(1 - b2^t), in double with b^t formed by repeated squaring, so that
// the host (host-side step count) and the device (device-side count) form
// the same values.
struct AdamFactors {
  float step_size, inv_sqrt_bc2;
};
__host__ __device__ inline double pow_int(double b, long long t) {
  double r = 1.0;
  while (t > 0) {
    if (t & 1) r *= b;
    b *= b;
    t >>= 1;
  }
  return r;
}
__host__ __device__ inline AdamFactors adam_factors(double lr, double b1, double b2, long long t) {
  const double bc1 = 1.0 - pow_int(b1, t), bc2 = 1.0 - pow_int(b2, t);
  return AdamFactors{(float)(lr / bc1), (float)(1.0 / sqrt(bc2))};
}

// One batch entry (probe position) of a launch; filled on the device.
struct Item {
  int req;          // index into the launch's request table
  int j;            // position index
  int ny, nx;       // integer window offset (top-left corner)
  float dy, dx;     // subpixel remainder of the position
  int valid;        // window inside the object
  int tile0;        // first workspace tile (modes follow)
  long long ck0;    // first checkpoint tile: slot s of mode m is tile ck0 + m + s * (n_items * M)
};

// One reconstruction taking part in a launch. Passed by value in the kernel
// arguments (a table of kMaxReqs), so no host-to-device staging is needed.
struct ReqDev {
  const float2* obj;        // [S][H][W]
  float2* gobj;             // [S][H][W] or null
  const float2* phat;       // [M][N][N] unitary probe spectrum
  float2* gphat;            // [M][N][N] probe-spectrum gradient (scratch) or null
  const float2* prop;       // [S-1][N][N] propagators divided by N^2
  const float* patterns;    // [J][N][N] or null
  const float* positions;   // [J][2]
  const int32_t* batch_idx; // [n_items]
  float* I_out;             // [n_items][N][N] or null
  double* loss_out;         // device double or null
  float* gpos;              // [n_items][2] or null
  float* gpos_dense;        // [J][2] or null
  int S, M, H, W, J;
  int loss;
  float eps, inv_sigma2;
  int item0, n_items;
  int tile_base;            // first workspace tile of this request
  long long ck_base;        // first checkpoint tile of this request
  int ck_every, n_ck;       // checkpoint interval and stored slices per mode
  int accumulate;           // add into gpos instead of overwriting
  float* emax;              // [n_items][S][2] window maxima of sum_m |psi_i|^2 and |O_i|^2 (ePIE) or null
  int modulus;              // far-field weight: 0 loss gradient, 1 modulus update (ePIE, LSQML)
  float* wsum;              // [S][H][W] scatter of sum_m |psi_i|^2 (LSQML) or null
  const uint8_t* live;      // [N] 1 where the propagators' column u_x has a nonzero value, or null
                            // (no band limit): a propagation column pass leaves the other
                            // columns of its output unwritten, and their consumers read zeros
  int live_k;               // >= 0: the live columns are exactly |k_x| <= live_k (no table lookup)
  const float4* prop_y;     // [S-1][N] (Hy / N^2, K_y bits, 0): H = [|k_x| <= K_y] Hy Hx, or null
  const float2* prop_x;     // [S-1][N] Hx
  const double* scale_dev;  // device double multiplying the adjoint's outputs (gradient of the
                            // caller's objective with respect to the loss), or null (1)
  int chain_final;          // the final column pass walks this request's items in kProbeSplit
                            // chains and keeps the probe-gradient sums in registers
                            // (k_col_final_chain + k_probe_sum) instead of storing h_hat for
                            // k_probe_grad (set per launch by set_chain_final)
};

// Scale of the adjoint outputs: the launch's host factor times the request's
// device factor, read by each workgroup once.
__device__ __forceinline__ float adj_scale(const ReqDev& r, float scale) {
  return r.scale_dev ? scale * (float)(*r.scale_dev) : scale;
}

struct ReqTable {
  ReqDev r[kMaxReqs];
};
// passed by value with a few pointers and ints beside it: keep the kernel
// arguments under 4 KiB
static_assert(sizeof(ReqTable) + 256 <= 4096, "request table too large for the kernel arguments");

// Checkpoint tile of (item, mode m, stored slot s). Slot-major within a
// request, so the entry waves of one slice for the whole group are contiguous.
__device__ __forceinline__ size_t ck_tile(const Item& it, const ReqDev& r, int m, int slot) {
  return (size_t)it.ck0 + (size_t)m + (size_t)slot * ((size_t)r.n_items * (size_t)r.M);
}

// Where the forward row pass stores entry waves.
struct PsiStore {
  int mode;                 // 0: nowhere, 1: checkpoint slots, 2: segment buffer,
                            // 3: none, the input row spectrum is read from checkpoint slot i
                            //    (spectral checkpoints, written by the column passes)
  void* seg;                // segment buffer [tiles][seg_len][N][N] (checkpoint storage type)
  int seg_len, seg_slot;
  const void* src;          // FROM_REAL source (checkpoint buffer)
  int src_slot;
  int stop_after_store;     // skip the transmission and forward DFT
};

// Segment buffer slots a propagation column pass writes its output to while a
// segment of entry waves is recomputed with spectral checkpoints (seg null:
// none). Slice s goes to slot s - base of [tiles][len][N][N].
struct SegOut {
  float2* seg;
  int len, base;
};

// Where the adjoint row pass reads entry waves.
struct PsiLoad {
  int from_seg;             // 0: checkpoint slot i / ck_every, 1: segment buffer
  int spec;                 // the checkpoint slot holds the row spectrum F_x(psi_i) (float2)
  const void* seg;
  int seg_len, seg_base;    // slice i is at slot i - seg_base
};

struct LaunchCtx {
  hipStream_t stream;
  ReqTable reqs;
  int n_reqs, n_items, max_modes;
  int item_off;             // first item of this launch (chunked schedules)
  int resident;             // use the LDS-resident chain kernels
  Item* items;
  float2* ws;               // tile workspace
  void* ck;                 // checkpoint buffer (float2, or __half2 when ck_half)
  int ck_half;
  float2* ramps;            // [n_items][2][N]
  const float2* tw;         // [N] roots of unity
  float* loss_part;         // [n_items][col blocks]
  float* pos_part;          // [tiles][col blocks][2] (tile = item tile0 + mode)
  int* flags;
  int emax;                 // the first forward records the window maxima (ePIE)
  int wsum;                 // the adjoint row pass scatters the illumination (LSQML)
  float* wscr;              // ordered reduction of the LSQML illumination sums: per-item
                            // sum_m |psi_i,m|^2 scratch [items][N][N], or null (atomics)
  float2* cscr;             // ordered object-gradient reduction: per-item contribution scratch
                            // [items][N][N] (the adjoint row pass stores, k_obj_gather adds), or
                            // null (float atomics)
  unsigned col_live_blocks; // column blocks a propagation column pass runs (bit q: columns of
                            // block q; 0: all), the union over the launch's requests
  SegOut seg_out;           // recompute with spectral checkpoints: column-pass output slots
  int ck_spec;              // spectral checkpoints: the forward column passes write the row
                            // spectrum F_x(psi_i) of each stored entry wave into checkpoint
                            // slot i / ck_every (float2 storage, two-pass kernels)
};

void launch_items(const LaunchCtx& L, int N);
void launch_rows_fwd(const LaunchCtx& L, int N, int step, PsiStore st, bool from_real);
void launch_rows_adj(const LaunchCtx& L, int N, int step, PsiLoad psi, float scale);
void launch_col(const LaunchCtx& L, int N, int op, int step);
void launch_far_loss(const LaunchCtx& L, int N, int step, bool grad);
void launch_obj_gather(const LaunchCtx& L, int N, int step, int max_h, int max_w);
void launch_probe_grad(const LaunchCtx& L, int N, float scale);
// Marks the requests of L whose final column pass runs as chains (unchunked
// launches with enough (column block, mode, chain) workgroups to fill the GPU).
void set_chain_final(LaunchCtx& L, int N, bool unchunked);
void launch_loss_reduce(const LaunchCtx& L, int N);
void launch_pos_reduce(const LaunchCtx& L, int N, float scale);
void launch_plain2d(int N, hipStream_t s, const float2* tw, const float2* src, float2* dst, int n_tiles,
                    bool inverse, float scale, bool accumulate);
void launch_fill(hipStream_t s, float* p, size_t n, float v);
void launch_sgd(hipStream_t s, float* th, const float* g, size_t n, float lr);
void launch_adam(hipStream_t s, float* th, const float* g, float* m, float* v, size_t n, float step_size,
                 float inv_sqrt_bc2, double b1, double b2, float eps);
// Adam with the step count read on the device: t = *step_dev + 1
void launch_adam_dev(hipStream_t s, float* th, const float* g, float* m, float* v, size_t n, double lr,
                     const int64_t* step_dev, double b1, double b2, float eps);
void launch_step_advance(hipStream_t s, int64_t* step_dev);
int col_blocks(int N);

enum ColOp { COL_SHIFT = 0, COL_PROP = 1, COL_PROP_ADJ = 2, COL_FINAL = 3 };

// Cost-regularizer weights on the device side (float).
struct RegDev {
  float obj_l2, obj_l1, obj_tikhonov, obj_tv, layers_tikhonov, layers_tv, tv_delta, obj_phase_l1;
};
constexpr int kMaxBlurSlices = 64;

int launch_reg_object(hipStream_t s, const float2* O, float2* g, int S, int H, int W, const RegDev& rg,
                      float* cost_part);
int launch_reg_probe(hipStream_t s, const float2* P, float2* g, size_t n, float w, float* cost_part);
// Probe phase-plate Tikhonov (wt) / TV (wv) on the unitary spectra phat [M][N][N]
// (FFT order): writes the gradient with respect to phat into gphat and cost
// partials; returns the number of partials.
// Spectral L1 step between the forward and inverse FFTs of the object slices
// (see k_spec_l1); returns the number of cost partials.
int launch_spec_l1(hipStream_t s, float2* spec, size_t n, size_t HW, float w, float* cost_part);
void launch_cadd_inplace(hipStream_t s, float2* g, const float2* a, size_t n);
int launch_reg_probe_phase(hipStream_t s, const float2* phat, float2* gphat, int M, int N, float wt, float wv,
                           float delta, float* cost_part);
void launch_add_cost(hipStream_t s, const float* part, int n, double* loss);
void launch_amp_clamp(hipStream_t s, float2* O, size_t n, float lo, float hi);
void launch_layer_blur(hipStream_t s, float2* O, int S, size_t HW, const float* g, int r);
void launch_mask_tiles(hipStream_t s, float2* t, const uint8_t* mask, size_t n, int N2);
// In-plane periodic Gaussian low pass of every slice; tmp holds S*H*W values.
void launch_lowpass(hipStream_t s, float2* O, float2* tmp, int S, int H, int W, const float* w, int r);
// Blocks per slice of the deramp sums (the partials buffer holds S * this * 4 doubles).
int deramp_blocks(int H, int W);
// Affine phase removal per slice; theta: S * 3 doubles, part: see deramp_blocks.
void launch_deramp(hipStream_t s, float2* O, int S, int H, int W, double* theta, double* part);

// LSQML (Sec. 3.3) after the adjoint chain. Transparency sum over the group's
// valid items (first n_items of items): wp[r] = sum_j tau(n_j + r) with
// tau = prod_i |O_i|^2 computed once per object pixel (tau: H * W floats);
// part holds kLsqSplit * N * N floats.
constexpr int kLsqSplit = 32;
void launch_lsq_transparency(hipStream_t s, const Item* items, int n_items, const float2* O, int S, int H,
                             int W, int N, float* tau, float* part, float* wp);
// Object step: D = -g (g the chain's object accumulator), A = prev or cur + w,
// A' = A + delta max A per slice, alpha_i from double sums (part: S *
// lsq_blocks(H * W) * 3 + S doubles of partial sums, partial maxima and
// maxima; alpha: S doubles), O -= beta alpha_i g / A', cur += w.
int lsq_blocks(size_t n);
void launch_lsq_object(hipStream_t s, float2* O, const float2* g, const float* w, float* cur, const float* prev,
                       int S, size_t HW, float delta, double gamma, float beta, double* part, double* alpha);
// Probe step, likewise with the probe accumulator g [M][N][N], the
// transparency sum wp [N][N]; alpha: 2 doubles (step, max B).
void launch_lsq_probe(hipStream_t s, float2* P, const float2* g, const float* wp, float* cur, const float* prev,
                      int M, int N2, float delta, double gamma, float beta, double* alpha);

// LDS-resident forward / adjoint chains (N = 64, 128; every slice checkpointed)
bool resident_supported(int N);
void launch_res_fwd(const LaunchCtx& L, int N, bool save);
void launch_res_adj(const LaunchCtx& L, int N, float scale);

}  // namespace pty
