/*
 * pty.h -- C ABI of the MI355X (gfx950) hot path of gradient-descent
 * mixed-state multislice ptychography (arXiv 2505.14372).
 *
 * What the library computes, per group ("batch") of probe positions:
 *   - the multislice forward model of Sec. 3: each probe mode is shifted to
 *     the position (Fourier subpixel shift, integer window offset), multiplied
 *     by each object slice's transmission function and Fresnel-propagated
 *     between slices (band-limited), then taken to the far field; intensities
 *     of the incoherent modes are summed;
 *   - the loss of one of the noise models of Sec. 3.1 against measured
 *     patterns (sum over pixels and positions);
 *   - the exact vector-Jacobian product of Sec. 3.2 back to the object, the
 *     probe modes and the positions, with overlapping object gradients
 *     scatter-added;
 *   - one optimiser step (SGD or Adam, Sec. 3.2) on all three variables,
 *     with the cost and constraint regularizers of Sec. 3.4;
 *   - the conventional engines of Sec. 3.3 on the same kernels: ePIE / 3PIE
 *     (pty_reconstruct_step, PTY_OPT_EPIE) and LSQML (pty_lsqml_step).
 *
 * Conventions (fixed readings of the paper):
 *   - complex numbers are interleaved float32 pairs (pty_c64);
 *   - the 2D DFT is unitary; detector patterns are in FFT order (DC at [0,0]);
 *   - the propagator for gap dz is H(u) = B(u) exp(-i pi lambda dz |q|^2),
 *     q = fftfreq(N) / dx, B the circular band limit
 *     k_y^2 + k_x^2 <= (bandlimit * N / 2)^2 on signed integer bins
 *     (inclusive; bandlimit <= 0 disables it) or a caller-given mask, times
 *     the tilt phase exp(2 pi i dz q.tan(tilt));
 *   - S slices have S-1 gaps: S-1 propagations, none after the last slice;
 *   - position X_j = (row, col) of the window's top-left corner in object
 *     pixels; the window starts at n_j = floor(X_j + 0.5) and the probe is
 *     shifted by d_j = X_j - n_j in [-0.5, 0.5) with the ramp
 *     exp(-2 pi i (u_y d_y + u_x d_x)), u = fftfreq(N);
 *   - complex gradients are dL/dRe + i dL/dIm;
 *   - Poisson loss l = I - Ie - Ie (ln(I+eps) - ln(Ie+eps)) (l = I if Ie = 0),
 *     amplitude/Anscombe l = (sqrt(I+c) - sqrt(Ie+c))^2 / 2 with the
 *     eps-regularised weight 1 - sqrt(Ie+c)/(eps + sqrt(I+c)),
 *     Gaussian l = (I - Ie)^2 / (2 sigma^2).
 *
 * Memory and ownership:
 *   - every array argument is a DEVICE pointer to C-contiguous memory owned
 *     by the caller, except pty_geometry.dz (host, copied at create);
 *   - the library allocates device memory only in pty_create /
 *     pty_group_create (workspace sized for max_batch) and in
 *     pty_set_regularizers (masks and filter taps), never in a step;
 *   - calls are asynchronous and stream-ordered on the given hipStream_t
 *     (passed as void*; NULL = the null stream); scalar results (loss) are
 *     written to device doubles;
 *   - gradient outputs are overwritten unless PTY_ACCUMULATE is set; a NULL
 *     gradient pointer skips that output.
 *
 * Errors: every entry point returns a pty_status; nothing throws across the
 * ABI. Host-side validation (shapes, sizes, NULL) happens at call time and
 * leaves device state untouched. Conditions only the device can see (a
 * window leaving the object, a non-finite loss or weight) set sticky flags
 * that pty_check() reads (it synchronises the stream) and clears; windows
 * that leave the object are skipped (they contribute nothing).
 * pty_last_error() describes the last failure of a context.
 */
#ifndef PTY_H
#define PTY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } pty_c64;

typedef enum {
  PTY_OK = 0,
  PTY_EINVAL = 1,        /* bad argument (NULL, size, shape) */
  PTY_EBOUNDS = 2,       /* a probe window left the object (device flag) */
  PTY_EUNSUPPORTED = 3,  /* N not in {64, 128, 192, 256}, or a limit exceeded */
  PTY_ENOMEM = 4,        /* device allocation failed at create */
  PTY_EHIP = 5,          /* a HIP runtime call failed */
  PTY_ENONFINITE = 6,    /* non-finite loss or detector weight (device flag) */
  PTY_ESTATE = 7         /* pty_backward without a preceding pty_forward_save; pty_lsqml_step
                            on a context created without its scratch */
} pty_status;

/* Noise models of Sec. 3.1. */
typedef enum {
  PTY_LOSS_AMPLITUDE = 0,   /* c = 0 */
  PTY_LOSS_ANSCOMBE = 1,    /* c = 3/8 */
  PTY_LOSS_POISSON = 2,
  PTY_LOSS_GAUSSIAN = 3
} pty_loss_kind;

#define PTY_ACCUMULATE 1u   /* add into gradient outputs instead of overwriting */
#define PTY_POS_DENSE 2u    /* g_pos is [J][2] indexed by position (batch entries summed) */

/* One reconstruction's geometry (the unknowns of Sec. 3: probe modes, sliced
 * object with gaps dz, positions). */
typedef struct {
  int32_t N;            /* window / probe / pattern side: 64, 128, 192 or 256 */
  int32_t n_modes;      /* M >= 1 incoherent probe modes */
  int32_t n_slices;     /* S >= 1 object slices */
  int32_t obj_h, obj_w; /* object slice size, >= N */
  int32_t n_positions;  /* J, rows of the positions / patterns arrays */
  double dx;            /* pixel size (Angstrom) */
  double wavelength;    /* Angstrom */
  const double* dz;     /* host array [n_slices-1] of gaps (Angstrom); copied */
  double bandlimit;     /* band-limit radius as a fraction of Nyquist; <= 0: none */
  int32_t loss;         /* pty_loss_kind */
  double eps;           /* noise-model epsilon (Sec. 3.1) */
  double sigma;         /* Gaussian noise standard deviation */
  double tilt_y, tilt_x;  /* propagator tilt (Sec. 1), radians: every gap also
                             multiplies by exp(2 pi i dz (q_y tan tilt_y + q_x tan tilt_x)) */
  const uint8_t* bandlimit_mask;  /* optional host [N][N] mask in FFT order (nonzero =
                                     kept) replacing the circular limit; copied */
} pty_geometry;

typedef struct pty_ctx pty_ctx;

/* Create a context for one geometry with workspace for groups of up to
 * max_batch positions (at most 65535: PTY_EINVAL beyond). checkpoint_every = 1 stores every slice's entry wave
 * during the forward pass (in float storage as its row spectrum, which the
 * forward pass produces anyway, so storing costs no extra write; the
 * backward pass recovers the wave with an inverse row DFT); k > 1 stores
 * every k-th and recomputes the others segment by segment in the backward
 * pass (in float storage, as row spectra too, so a recomputed segment costs
 * one row and one column pass per slice); 0 picks 1 if the workspace fits
 * in hbm_budget bytes (0 = no limit), else the smallest k that fits.
 * Builds the propagator tables (and, when the band limit allows, their
 * separable factors) on the device, and holds max_batch x N x N complex64 of
 * scratch for the ordered object-gradient reduction (pty_set_reduction). */
pty_status pty_create(const pty_geometry* g, int32_t max_batch, int32_t checkpoint_every,
                      size_t hbm_budget, pty_ctx** out);

/* Creation options (pty_create_ex). */
typedef struct {
  int32_t max_batch;         /* positions per group (workspace size) */
  int32_t checkpoint_every;  /* as in pty_create */
  size_t hbm_budget;         /* as in pty_create; 0 = no limit */
  int32_t checkpoint_half;   /* 1: store entry-wave checkpoints as pairs of IEEE
                                half floats (round to nearest), halving their HBM
                                traffic; only the object gradient reads them */
  int32_t lsqml;             /* 1: also allocate the scratch of pty_lsqml_step
                                ((S+1)*H*W + 33*N*N floats, a few sums, and
                                max_batch*N*N floats for the ordered reduction) */
} pty_options;

/* pty_create with the options above; pty_create(g, b, k, budget, out) equals
 * pty_create_ex with checkpoint_half = 0 and lsqml = 0. */
pty_status pty_create_ex(const pty_geometry* g, const pty_options* opt, pty_ctx** out);
pty_status pty_workspace_bytes_ex(const pty_geometry* g, const pty_options* opt, size_t* bytes);
/* Checkpoint storage chosen at create (1 = half floats). */
int32_t pty_checkpoint_half(const pty_ctx* ctx);

/* Device bytes pty_create would allocate for these arguments. */
pty_status pty_workspace_bytes(const pty_geometry* g, int32_t max_batch, int32_t checkpoint_every,
                               size_t* bytes);

/* Checkpoint interval chosen at create (1 = store all). */
int32_t pty_checkpoint_every(const pty_ctx* ctx);

/* Kernel strategy. TWO_PASS: every slice step is a row pass and a column pass
 * over tiles in the workspace (all N). RESIDENT: for N = 64 and 128 a tile fits
 * in LDS and one workgroup per (position, mode) runs every slice with its
 * tile resident (used when every slice is checkpointed and the object
 * gradient is accumulated with atomics, else two-pass; the ePIE engine and
 * the ordered reduction always run two-pass). AUTO (default): TWO_PASS, which
 * measured faster than RESIDENT at N = 128 (8 slices, 4 modes) and equal at
 * N = 64. */
#define PTY_STRATEGY_AUTO 0
#define PTY_STRATEGY_TWO_PASS 1
#define PTY_STRATEGY_RESIDENT 2
pty_status pty_set_strategy(pty_ctx* ctx, int32_t strategy);

/* How the object gradient (Sec. 3.2: the sum over the group of every
 * position's windowed contribution, slice by slice) is accumulated.
 * ATOMIC (default): the adjoint row pass adds each contribution with float
 * atomics; the summation order, and so the last bits of the gradient, vary
 * from run to run. ORDERED: the adjoint row pass stores each position's
 * contribution in a scratch area allocated at create (max_batch x N x N
 * complex64) and a second kernel adds them tile by tile in batch order, so
 * loss_and_grad and reconstruct_step give bit-identical results on repeated
 * calls with the same inputs, and a reconstruction gives the same bits alone
 * or in a grouped step (the dense position gradient excepted when a batch
 * lists one position twice). ORDERED also avoids the contention of many
 * overlapping windows (a whole dense scan in one group). It applies to the
 * two-pass kernels; with it set, RESIDENT runs two-pass. The LSQML
 * illumination sums follow the same mode (a context created with lsqml also
 * holds max_batch x N x N floats of scratch for them). Returns PTY_EINVAL for
 * another mode. */
#define PTY_REDUCE_ATOMIC 0
#define PTY_REDUCE_ORDERED 1
pty_status pty_set_reduction(pty_ctx* ctx, int32_t mode);

/* Schedule of pty_loss_and_grad and pty_reconstruct_step: the group is taken
 * through the forward and adjoint passes in consecutive chunks of
 * `positions` batch entries, one chunk after the other, so that a chunk's
 * work tiles can stay in the last-level cache between passes; 0 (the
 * default) processes the whole group in every launch. Results do not depend
 * on the chunk size beyond the order of floating-point additions (under the
 * ordered reduction one chunk size always gives the same bits). */
pty_status pty_set_chunk(pty_ctx* ctx, int32_t positions);

/* Concurrency of a chunked schedule (pty_set_chunk): with n > 1 the chunks of
 * pty_loss_and_grad and pty_reconstruct_step run on n internal streams of
 * the context (chunk q on stream q mod n, forked from and joined back into the
 * caller's stream, so the call stays stream-ordered for the caller), so that
 * the launches of several chunks overlap while each chunk's tiles stay in the
 * last-level cache. Falls back to one stream under the ordered reduction
 * (its gather writes the gradient without atomics) and with checkpoint
 * intervals k > 1 (the recompute buffers are shared). n in [1, 8]; creates
 * the streams on first use (PTY_EHIP if that fails). */
pty_status pty_set_streams(pty_ctx* ctx, int32_t n);

/* Forward model (Sec. 3) for the positions batch_idx[0..batch) (device int32,
 * values in [0, J)). probe [M][N][N], object [S][H][W], positions [J][2]
 * float32 (row, col). Writes intensities [batch][N][N] (FFT order) if not
 * NULL and, if patterns [J][N][N] and loss are both given, the group loss
 * (one device double). */
pty_status pty_forward(pty_ctx* ctx, void* stream, const pty_c64* probe, const pty_c64* object,
                       const float* positions, const int32_t* batch_idx, int32_t batch,
                       const float* patterns, float* intensities, double* loss);

/* Bytes of the static device array that backs pty_forward_static (one copy
 * per GPU the library runs on, held until the process ends). */
#define PTY_STATIC_SCRATCH_BYTES ((size_t)32 << 20)

/* pty_forward for callers that cannot allocate device memory at call time
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, results and errors, but every per-call
 * buffer -- the probe spectrum, the item descriptors and shift ramps, the
 * work tiles and the loss partial sums -- is carved from one static device
 * array of PTY_STATIC_SCRATCH_BYTES per GPU instead of the context's
 * workspace, so the context may be created with max_batch = 0 (tables only).
 * The call takes, each piece rounded up to 256 bytes: the probe spectrum (M
 * N^2 complex64) and, per position, a 40-byte descriptor, two shift ramps of
 * N complex64, N / 32 float loss partials and M work tiles of N^2 complex64
 * (about 8 batch M N^2 bytes in all); PTY_EINVAL (with the bytes needed in
 * pty_last_error) if that exceeds the array, or for batch < 1. Nothing in
 * the array needs to start at zero: every piece is written before it is read
 * in the same call. Every call on a GPU shares that GPU's array and leaves
 * its contents behind: calls that overlap on one GPU (other streams, threads
 * or contexts) race and must be serialised by the caller. Calls no
 * allocation routine (only per-launch timing, when pty_profile_enable turns
 * it on, creates HIP events). */
pty_status pty_forward_static(pty_ctx* ctx, void* stream, const pty_c64* probe, const pty_c64* object,
                              const float* positions, const int32_t* batch_idx, int32_t batch,
                              const float* patterns, float* intensities, double* loss);

/* Loss of the group and its gradients (Sec. 3.1-3.2): g_object [S][H][W],
 * g_probe [M][N][N], g_pos [batch][2] (per batch entry, dL/dX; with
 * PTY_POS_DENSE [J][2] per position). loss may be NULL.
 * flags: PTY_ACCUMULATE | PTY_POS_DENSE. */
pty_status pty_loss_and_grad(pty_ctx* ctx, void* stream, const pty_c64* probe,
                             const pty_c64* object, const float* positions, const float* patterns,
                             const int32_t* batch_idx, int32_t batch, double* loss,
                             pty_c64* g_object, pty_c64* g_probe, float* g_pos, uint32_t flags);

/* Split form of pty_loss_and_grad for automatic differentiation: the forward
 * pass stores the per-slice entry waves (checkpoints) and the detector-plane
 * gradient seed in the context ("tape"); pty_backward runs the adjoint from
 * that tape and scales every gradient by grad_scale. The probe, object,
 * positions and batch_idx buffers must stay unchanged until pty_backward;
 * any other call on the context invalidates the tape (PTY_ESTATE). */
pty_status pty_forward_save(pty_ctx* ctx, void* stream, const pty_c64* probe,
                            const pty_c64* object, const float* positions, const float* patterns,
                            const int32_t* batch_idx, int32_t batch, float* intensities,
                            double* loss);
pty_status pty_backward(pty_ctx* ctx, void* stream, double grad_scale, pty_c64* g_object,
                        pty_c64* g_probe, float* g_pos, uint32_t flags);
/* pty_backward with the scale read on the device: grad_scale points to one
 * device double (the gradient of the caller's objective with respect to the
 * loss, e.g. the incoming gradient of an autograd backward), read by the
 * kernels in stream order, so no value travels to the host and the call never
 * waits for the device. PTY_EINVAL if grad_scale is NULL. */
pty_status pty_backward_dev(pty_ctx* ctx, void* stream, const double* grad_scale, pty_c64* g_object,
                            pty_c64* g_probe, float* g_pos, uint32_t flags);

/* Resident reconstruction state (device pointers). Moments (m_*, v_*) are
 * float32 arrays with the real-component shape of their variable; they are
 * only used by Adam. step counts completed Adam steps (host-side). step_dev,
 * if not NULL, points to one device int64 that holds that count instead: the
 * Adam kernels read it in stream order (bias corrections 1 - beta^t with
 * t = *step_dev + 1, formed on the device) and the step advances it on the
 * device, so no value depends on the host and a recorded step replays
 * correctly (pty_step_graph_*); step is then left unchanged. */
typedef struct {
  pty_c64* probe;      /* [M][N][N] */
  pty_c64* object;     /* [S][H][W] */
  float* positions;    /* [J][2] */
  float* m_probe; float* v_probe;     /* [M][N][N][2] */
  float* m_object; float* v_object;   /* [S][H][W][2] */
  float* m_pos; float* v_pos;         /* [J][2] */
  int64_t step;
  int64_t* step_dev;
} pty_state;

/* PTY_OPT_EPIE is the conventional ePIE / 3PIE engine (Sec. 3.3) rather than
 * an optimiser: every position of the group is evaluated at the current
 * state; at the detector chi = (sqrt(Ie + c) / (eps + sqrt(I + c)) - 1) Psi
 * per mode (c = 3/8 for the Anscombe model, else 0; 0 where eps + sqrt(I + c)
 * is 0); per slice i from the last down, dO_i += a conj(psi_i) chi (summed over
 * modes) and the entry-wave update b conj(O_i) chi is carried back to slice
 * i - 1 through F^-1 conj(H) F, with a = 1 / max over the window of
 * sum_m |psi_i,m|^2 and b = 1 / max over the window of |O_i|^2 (0 when the
 * maximum is 0); the slice-0 entry-wave update, shifted back by -delta_j,
 * is the probe update. Then O += lr_object * sum dO (beta_object) and
 * P += lr_probe * (sum dP) / B (beta_probe). Positions are not refined, the
 * Adam fields and moments are ignored, cost regularizers do not apply, the
 * constraints do. The loss written is the configured noise model's loss at
 * the state before the step. */
typedef enum { PTY_OPT_SGD = 0, PTY_OPT_ADAM = 1, PTY_OPT_EPIE = 2 } pty_opt_kind;

typedef struct {
  int32_t kind;          /* pty_opt_kind */
  double lr_object, lr_probe, lr_pos;   /* 0 freezes a variable */
  double beta1, beta2, eps;             /* Adam */
} pty_optim;

/* Regularization (Sec. 3.4), applied by pty_reconstruct_step and grouped
 * steps of this context. Cost regularizers add lambda * R to the group loss
 * and lambda * dR to the gradients before the optimiser:
 *   obj_l2          sum |O - 1|^2 (distance from vacuum)
 *   probe_l2        sum |P|^2
 *   obj_l1          sum |O - 1|
 *   obj_tikhonov    sum over slices of |D_y O|^2 + |D_x O|^2 (forward differences, no wrap)
 *   obj_tv          sum over slices of phi(D_y O) + phi(D_x O), phi(z) = sqrt(|z|^2 + tv_delta^2)
 *   layers_tikhonov sum |O_{i+1} - O_i|^2
 *   layers_tv       sum phi(O_{i+1} - O_i)
 *   obj_phase_l1    sum |arg O| (arg in (-pi, pi]; gradient 0 where arg O = 0)
 *   obj_spectrum_l1 sum over slices and over every frequency but zero of |F2(O_i)(k)|, F2 the
 *                   unitary 2D DFT of the H x W slice (transformed with hipFFT; the call that
 *                   sets it allocates the plan and an object-sized spectrum buffer)
 *   probe_phase_tikhonov, probe_phase_tv  the phase plate of each mode, the phase of its unitary
 *                   spectrum P^ = F(P) taken centred (zero frequency at N/2): for every pair of
 *                   neighbours (a, b) along either axis, z = a conj(b) = |z| e^{it}, t in (-pi, pi],
 *                   costs |z|^2 t^2 (Tikhonov) or |z|^2 sqrt(t^2 + tv_delta^2) (TV): phase steps
 *                   weighted by the two frequencies' intensities (gradient continuous at z = 0)
 * Constraint regularizers are applied to the state after the optimiser:
 *   amp_clamp       object amplitude limited to [amp_min, amp_max] (phase kept)
 *   probe_support   host [N][N] reciprocal-space mask (FFT order) or NULL: P <- F^-1(mask F(P))
 *   layer_sigma     Gaussian blur along depth (sigma in slices, truncated at 3 sigma, normalised,
 *                   real space; 0 = off; at most 64 slices)
 *   obj_lowpass_sigma  in-plane Gaussian low pass of every slice (sigma in pixels, at most 64; taps
 *                   t = -r..r with r = ceil(3 sigma), weights exp(-t^2 / 2 sigma^2) normalised;
 *                   separable, x then y, periodic boundaries; 0 = off)
 *   phase_deramp    nonzero: per slice, remove the affine phase theta_0 + theta_y y + theta_x x,
 *                   theta_x = arg sum O(y, x+1) conj O(y, x), theta_y likewise along y, theta_0 =
 *                   arg of the sum of the de-ramped slice
 *   probe_support_real  host [N][N] real-space mask or NULL: P <- mask P
 * Order: amplitude range, depth blur, low pass, deramp (object); reciprocal-space
 * support, then real-space support (probe).
 * A NULL argument turns all regularization off. */
typedef struct {
  double obj_l2, probe_l2, obj_l1, obj_tikhonov, obj_tv, layers_tikhonov, layers_tv, tv_delta;
  int32_t amp_clamp;
  double amp_min, amp_max;
  const uint8_t* probe_support;
  double layer_sigma;
  double obj_lowpass_sigma;
  int32_t phase_deramp;
  double obj_phase_l1, obj_spectrum_l1;
  double probe_phase_tikhonov, probe_phase_tv;
  const uint8_t* probe_support_real;
} pty_regularizers;

pty_status pty_set_regularizers(pty_ctx* ctx, const pty_regularizers* reg);

/* One gradient step on one group (Sec. 2.2 engine loop, Sec. 3.2 solver):
 * loss and gradients of the group, then SGD (theta -= lr g) or Adam (per real
 * component, bias-corrected, eps added to sqrt(v)/sqrt(1-beta2^t)) applied
 * densely to object, probe and positions (positions outside the group get a
 * zero gradient). Increments st->step for Adam. loss may be NULL. */
pty_status pty_reconstruct_step(pty_ctx* ctx, void* stream, pty_state* st, const float* patterns,
                                const int32_t* batch_idx, int32_t batch, const pty_optim* opt,
                                double* loss);

/* LSQML engine (Sec. 3.3). Illumination sums over an iteration, caller-owned
 * float device arrays: obj_* [S][H][W] (object view, sum over positions and
 * modes of |psi_i|^2 per slice), probe_* [N][N] (probe view, sum over
 * positions of prod_i |O_i|^2 over the window). A step reads the *_prev sums
 * of the previous iteration, or, when both *_prev are NULL (the first
 * iteration), the *_cur sums with its own group included; it always adds its
 * group's sums to *_cur. At the end of an iteration the caller moves *_cur to
 * *_prev and zeroes *_cur. */
typedef struct {
  const float* obj_prev;
  float* obj_cur;
  const float* probe_prev;
  float* probe_cur;
} pty_illum;

typedef struct {
  double beta_object, beta_probe;   /* step scales (0 freezes) */
  double delta_object, delta_probe; /* relative regularisers (> 0): delta * max of the
                                       illumination sum in use is added to it */
  double gamma;                     /* added to the step-size denominators (>= 0) */
} pty_lsqml;

/* One LSQML step on one group, every position at the current state. At the
 * detector chi = (sqrt(Ie + c) / (eps + sqrt(I + c)) - 1) Psi per mode (as for
 * PTY_OPT_EPIE); per slice i from the last the entry-wave update conj(O_i) chi_i
 * is carried to slice i - 1 by F^-1 conj(H) F (no normalisers). With
 * D_i = sum_j sum_m chi_i conj(psi_i) and W_i = sum_j sum_m |psi_i|^2 scattered
 * into object coordinates, A_i the object-view illumination sum:
 *   dO_i = D_i / (A_i + delta_object max A_i),
 *   alpha_i = Re <dO_i, D_i> / (<|dO_i|^2, W_i> + gamma)   (0 if that is 0),
 *   O_i += beta_object alpha_i dO_i.
 * Probe: dP_m = sum_j (slice-0 entry-wave update shifted back by -delta_j),
 * T = sum_j prod_i |O_i|^2 over window j, Bp the probe-view sum:
 *   dP'_m = dP_m / (Bp + delta_probe max Bp),
 *   alpha_P = Re sum_m <dP'_m, dP_m> / (sum_m <|dP'_m|^2, T> + gamma),
 *   P += beta_probe alpha_P dP'.
 * Positions are kept; the constraints of pty_set_regularizers apply, the cost
 * regularizers do not; the loss written is the noise model's at the state
 * before the step. Needs a context created with pty_options.lsqml = 1
 * (PTY_ESTATE otherwise); always runs the two-pass kernels. */
pty_status pty_lsqml_step(pty_ctx* ctx, void* stream, pty_state* st, const pty_illum* illum,
                          const float* patterns, const int32_t* batch_idx, int32_t batch,
                          const pty_lsqml* opt, double* loss);

/* Synchronise the stream, return PTY_EBOUNDS / PTY_ENONFINITE if a device
 * flag was raised since the last check (then clear it), else PTY_OK. */
pty_status pty_check(pty_ctx* ctx, void* stream);

const char* pty_last_error(const pty_ctx* ctx);
void pty_destroy(pty_ctx* ctx);

/* ---- grouped launches (continuous-batching server) ---------------------
 * A pty_group owns a workspace for one window size N and runs one step over
 * position chunks of several reconstructions (contexts with that N, any M,
 * S, object size, loss) in shared kernel launches. Entry waves are stored for
 * every slice (no recompute) in the group's workspace. A grouped step uses
 * the ordered object-gradient reduction when every context in it is set to
 * PTY_REDUCE_ORDERED (the group holds max_items x N x N complex64 of scratch
 * for it), else atomics. */
typedef struct pty_group pty_group;

typedef struct {
  pty_ctx* ctx;               /* geometry of this reconstruction (same N) */
  pty_state* state;           /* its resident state */
  const float* patterns;      /* [J][N][N] device */
  const int32_t* batch_idx;   /* device [batch] */
  int32_t batch;
  const pty_optim* opt;       /* host */
  double* loss;               /* device double or NULL */
} pty_group_item;

/* max_items bounds sum(batch) over the items of one call (at most 65535),
 * max_tiles bounds sum(batch * M), max_ckpt_tiles bounds sum(batch * M * S). */
pty_status pty_group_create(int32_t N, int32_t max_items, int32_t max_tiles, int64_t max_ckpt_tiles,
                            pty_group** out);
pty_status pty_group_workspace_bytes(int32_t N, int32_t max_items, int32_t max_tiles,
                                     int64_t max_ckpt_tiles, size_t* bytes);
pty_status pty_group_reconstruct_step(pty_group* grp, void* stream, const pty_group_item* items,
                                      int32_t n_items);
const char* pty_group_last_error(const pty_group* grp);
void pty_group_destroy(pty_group* grp);

/* ---- recorded steps -----------------------------------------------------
 * One pty_reconstruct_step recorded as a HIP graph (stream capture) and
 * replayed: for launch-bound problems (small probes, few slices) a replay
 * issues the step's dozen or more kernels without their per-launch host cost.
 * pty_step_graph_create records pty_reconstruct_step(ctx, stream, st,
 * patterns, batch_idx, B, optim, loss) on `stream` (nothing runs while
 * recording) and instantiates it; pty_step_graph_launch replays it on
 * `stream`. Every pointer, size, learning rate and the group size B are fixed
 * at recording; a replay reads the current contents of the same buffers, so
 * a caller changes the minibatch by writing new indices into batch_idx
 * between replays (and the state evolves in place, as with direct calls).
 * The context must outlive the graph and must not be used by another call
 * while a replay runs. Refused (PTY_EUNSUPPORTED, nothing recorded): Adam
 * without st->step_dev (a host-side count would be frozen into the graph),
 * the object-spectrum L1 regularizer (its transforms are library calls that
 * are not recorded), and while launch timing is enabled. PTY_EHIP if the
 * runtime refuses the capture or the instantiation. */
typedef struct pty_step_graph pty_step_graph;
pty_status pty_step_graph_create(pty_ctx* ctx, void* stream, pty_state* st, const float* patterns,
                                 const int32_t* batch_idx, int32_t batch, const pty_optim* optim, double* loss,
                                 pty_step_graph** out);
pty_status pty_step_graph_launch(pty_step_graph* graph, void* stream);
void pty_step_graph_destroy(pty_step_graph* graph);

/* ---- launch timing ------------------------------------------------------
 * When enabled (process-wide), every kernel launch of the library is
 * bracketed by two hipEvents on the stream it is launched on, grouped by
 * kernel class ("row_fwd", "col_prop", "row_adj", ...). pty_profile_collect
 * waits for the recorded events, writes up to max_entries classes (names
 * separated by '\n' into names, total milliseconds and launch counts) and
 * resets the totals; it returns the number of classes written. */
void pty_profile_enable(int32_t on);
/* Restricts the timing to the named classes (comma- or newline-separated,
 * e.g. "row_adj"); NULL or "" selects every class (the default). Returns the
 * number of classes selected, or -1 (selection unchanged) for an unknown name. */
int32_t pty_profile_select(const char* classes);
int32_t pty_profile_collect(char* names, size_t names_len, double* total_ms, int64_t* counts,
                            int32_t max_entries);

#ifdef __cplusplus
}
#endif
#endif /* PTY_H */
