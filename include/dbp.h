/*
 * dbp.h - C ABI of the MI355X (gfx950) digital-backpropagation library.
 *
 * The library backpropagates a dual- (or single-) polarization optical field
 * through a fibre link with the split-step Fourier method (SSFM) or the
 * enhanced SSFM (ESSFM) of Secondini et al., "Coherent 100G Nonlinear
 * Compensation with Single-Step Digital Backpropagation":
 *   - each step is a linear chromatic-dispersion substep, Sec. II Eq. (1),
 *     X_k <- X_k exp(-j 2 pi^2 beta2 f_k^2 dz), done on overlapping blocks with
 *     FFTs (overlap-and-save, Sec. III), followed by
 *   - a nonlinear substep, Sec. II Eqs. (2)-(3): every polarization is rotated
 *     by -gamma dz_eff J_k with J = I (SSFM) or J = the tap-filtered total
 *     intensity I = |x|^2 + |y|^2 (ESSFM, taps c_i of Eq. (3)).
 *
 * Conventions shared by every entry point:
 *   Fields   complex64 (float re, float im interleaved) in device memory,
 *            C-contiguous [batch][n_pol][n_samples].  Caller-owned.
 *   DFT      X_k = sum_n x_n exp(-j 2 pi k n / L); f_k = k fs / L for
 *            k < L/2, (k - L) fs / L otherwise.
 *   Units    ps, km, THz, W.  beta2 in ps^2/km (negative: anomalous), gamma
 *            in 1/(W km), alpha in dB/km, fs in THz (samples per ps).
 *   Link     n_spans identical spans of span_km with ideal amplifiers, the
 *            field power-normalized: attenuation enters only the nonlinear
 *            weight phi = gamma exp(-alpha z_a) (1 - exp(-alpha dz)) / alpha of
 *            a segment starting z_a km into its span (Sec. II effective
 *            length).  Backpropagation negates beta2 dz and phi and takes the
 *            segments from the receiver end, applying each segment's
 *            nonlinear phase at its transmitter-side end.  DBP_FLAG_FORWARD
 *            runs the physical direction instead (channel simulation).
 *   Taps     2Nc+1 real taps w, centre index Nc: J_n = sum_m w[m] I[n-(m-Nc)]
 *            (the paper's symmetric c_i is w[Nc+i] = w[Nc-i] = c_i).
 *   Blocks   overlap-and-save (Sec. III): block b covers samples
 *            (b V - O/2 + m) mod L, m < Nb, V = Nb - O; k steps are applied
 *            circularly inside each block per pass over the signal, and the
 *            centre V samples are kept.  DBP_FLAG_WHOLE uses one block of the
 *            whole signal (Nb = L, O = 0).
 *   Streams  every device call is asynchronous on the given hipStream_t
 *            (passed as void*; NULL = the null stream).  No call synchronizes
 *            unless documented.
 *   Errors   every call returns a dbp_status; nothing aborts or throws across
 *            the ABI.  Validation errors are returned before any device work.
 *   Threads  a plan is immutable after creation; concurrent calls on one plan
 *            are safe when each call has its own workspace.
 *   Tuning   the planner reads four environment variables when a plan is made
 *            (for measurements and tests; results differ between variants by
 *            FP32 rounding only, and the streaming kernel reproduces the
 *            per-block kernel bit for bit):
 *            DBP_FORCE_E=4|8|16 values per thread of the pass kernel;
 *            DBP_FORCE_SPLIT=0|1 polarization-split blocks off / on;
 *            DBP_STREAM=0|1 the streaming (resident-grid) pass kernel off / on
 *            where one is built, DBP_STREAM_GRID=n its grid (a multiple of 8).
 *   Faults   DBP_FAULT_INJECT="<tag>:<n>" (tests of the cleanup paths): the
 *            library's n-th device allocation counted since the tag last
 *            changed fails as out of memory; the call then returns
 *            DBP_ERR_OOM (or DBP_ERR_HIP) having released what it allocated.
 *   Tracing  DBP_LOG=1: every plan made (dbp_plan, dbp_plan_batch) writes its
 *            decisions to stderr: the descriptor's shape, the geometry (Nb,
 *            O, steps per pass, passes, values per thread), the kernel and
 *            the workspace sizes; a batch, its kernel groups.
 */
#ifndef DBP_H
#define DBP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dbp_status {
    DBP_OK = 0,
    DBP_ERR_INVALID_ARG = 1,   /* a descriptor field, pointer or size is invalid */
    DBP_ERR_UNSUPPORTED = 2,   /* valid but not built (e.g. a block size without a kernel) */
    DBP_ERR_WORKSPACE = 3,     /* workspace missing or smaller than dbp_workspace_size */
    DBP_ERR_OOM = 4,           /* host or device allocation failed */
    DBP_ERR_HIP = 5            /* a HIP runtime call failed (no device, launch error, ...) */
} dbp_status;

typedef enum dbp_method { DBP_SSFM = 0, DBP_ESSFM = 1 } dbp_method;

/* Linear substep: FFT filter of Eq. (1) on overlap-and-save blocks, or a
 * complex FIR (learnable dispersion taps).  FIR plans on signals of at least
 * 1024 samples apply the FIR's frequency response on overlap-and-save FFT
 * blocks of 1024 with overlap 256 (exact up to rounding: the FIR has finite
 * support), as many steps per pass as the halo covers ((n_fir - 1) / 2 + N_c
 * samples per step and side), the responses made from the taps of each call in
 * the workspace; shorter signals take one time-domain launch per step. */
typedef enum dbp_linear { DBP_LINEAR_FFT = 0, DBP_LINEAR_FIR = 1 } dbp_linear;

/* DBP_FP32: dispersion tables and nonlinear phase argument in FP32.
 * DBP_FP32_FP64PHASE: dispersion tables generated in FP64, nonlinear phase
 *   argument formed and reduced to [-pi, pi] in FP64, all else FP32.
 * DBP_BF16X3: as DBP_FP32_FP64PHASE, with the block DFTs as split-precision
 *   bfloat16 matrix products (hi*hi + hi*lo + lo*hi, FP32 accumulation). */
typedef enum dbp_precision {
    DBP_FP32 = 0, DBP_FP32_FP64PHASE = 1, DBP_BF16X3 = 2
} dbp_precision;

#define DBP_FLAG_FORWARD 0x1u   /* physical direction (forward propagation) */
#define DBP_FLAG_WHOLE   0x2u   /* one circular block of the whole signal */
#define DBP_FLAG_GRAD_SPARSE 0x4u  /* gradient: FIR, checkpoint every 8th step only;
                                      FFT steps, keep pass inputs only */
#define DBP_FLAG_TUNE    0x8u   /* measured geometry: time candidates at plan creation */
#define DBP_FLAG_PERSISTENT 0x10u  /* all passes in one resident launch, halos exchanged */

typedef struct dbp_desc {
    int32_t n_pol;            /* 1 or 2 */
    int32_t batch;            /* >= 1 signals of equal length, back to back */
    int64_t n_samples;        /* L, samples per polarization (>= block) */
    double fs_thz;            /* sampling rate, > 0 */
    int32_t n_spans;          /* >= 1 */
    int32_t steps_per_span;   /* >= 1; N_s = n_spans * steps_per_span */
    double span_km;           /* > 0 */
    double beta2_ps2_km;
    double gamma_w_km;        /* >= 0 */
    double alpha_db_km;       /* >= 0 */
    int32_t method;           /* dbp_method */
    int32_t n_taps;           /* ESSFM: odd, 1..DBP_MAX_TAPS; SSFM: ignored (1) */
    const float* taps;        /* host; ESSFM: [n_taps] (every step) or [N_s][n_taps] */
    int32_t taps_per_step;    /* 0: taps holds one vector, 1: one per step */
    int32_t linear;           /* dbp_linear */
    int32_t n_fir;            /* FIR: odd, 1..DBP_MAX_FIR */
    const float* fir;         /* host complex64 [n_fir] or [N_s][n_fir]; NULL: taps designed
                                 from the all-pass response of Eq. (1), see fir_band_thz */
    int32_t fir_per_step;     /* 0: fir holds one vector, 1: one per step */
    double fir_band_thz;      /* designed taps (fir == NULL): 0 -> the centre n_fir samples of
                                 the impulse response; > 0 -> least squares on the 4096-point
                                 DFT grid, target Eq. (1) for |f| <= fir_band_thz, target 0
                                 with weight 1e-3 outside */
    int32_t block;            /* Nb, power of two; 0: chosen by the planner */
    int32_t overlap;          /* O, even, < Nb (ignored when block == 0) */
    int32_t steps_per_pass;   /* k >= 1; 0: chosen by the planner */
    int32_t precision;        /* dbp_precision */
    uint32_t flags;           /* DBP_FLAG_* */
    int32_t spans_per_step;   /* 1 (or 0): steps_per_span steps in every span.  m > 1: each
                                 step covers m whole spans (steps_per_span must be 1 and m
                                 must divide n_spans; N_s = n_spans / m), as in the
                                 experiment of Sec. IV; such a step applies the dispersion of
                                 its m spans and one nonlinear phase weighted by the sum of
                                 their effective lengths, m (1 - e^{-alpha L}) / alpha */
} dbp_desc;

#define DBP_MAX_TAPS 129
#define DBP_MAX_FIR 129

typedef struct dbp_plan_s* dbp_plan_t;

/* Fill *d with defaults: one dual-polarization signal, SSFM, FFT linear step,
 * planner-chosen geometry, FP32_FP64PHASE.  Caller sets the link and size. */
void dbp_desc_init(dbp_desc* d);

/* Create a plan: validate, build the step schedule in FP64, choose the
 * geometry, build the dispersion and twiddle tables and copy them to the
 * current HIP device.  The plan owns its device tables.  With block = 0 the
 * geometry comes from an analytic cost per sample (overlap inflation times
 * FFT depth and per-pass cost; O the smallest overlap covering k steps, Sec. III);
 * with DBP_FLAG_TUNE (FFT steps, block = 0, not DBP_FLAG_WHOLE or BF16X3) the
 * planner instead times candidate geometries on a zero signal of the plan's
 * own size and batch -- for every block size the model's best step count per
 * pass and the largest one that fits (fewest passes; at large blocks the
 * whole link in one pass, the paper's arrangement) -- each as a full
 * backpropagation (one warm-up and three timed runs on a private stream,
 * synchronously, with temporary buffers of three states), and keeps the
 * fastest; DBP_AUTOTUNE_LOG names a file that receives one JSON line per
 * candidate.  dbp_plan_geometry reports the choice.  Returns
 * DBP_ERR_INVALID_ARG for an invalid descriptor (no device work done),
 * DBP_ERR_UNSUPPORTED for a geometry without a kernel, DBP_ERR_HIP or
 * DBP_ERR_OOM if the device upload fails.  *out is NULL on error. */
dbp_status dbp_plan(const dbp_desc* desc, dbp_plan_t* out);

/* DBP_FLAG_PERSISTENT (FFT steps, at least two passes): dbp_backprop runs every pass in
 * one cooperative launch of one workgroup per block.  A block keeps its samples in
 * registers from pass to pass and only the samples other windows read cross memory
 * between passes (as 64-bit value-and-flag words in a plan-owned buffer of
 * 3 x batch x n_pol x n_blocks x V x 16 bytes, zeroed at creation), instead of the whole
 * state being written and re-read by one launch per pass.  Results equal the per-pass
 * launches bit for bit.  Calls on one such plan share that buffer and must not overlap
 * in time; in-place calls (in == out) use the per-pass launches.  The plan falls back to
 * per-pass launches where no persistent variant is built (1024-point blocks with four
 * values per thread are), the blocks cannot all be resident, the device has no
 * cooperative launch, or a window reads a block more than two dependency hops from it
 * (tiny signals); dbp_plan_kernel names the kernel used. */

/* Release a plan and its device tables (NULL is a no-op).  The caller must
 * ensure no call using the plan is still running on any stream. */
void dbp_destroy(dbp_plan_t plan);

/* Name of the kernel variant the plan launches for its steps, in the form the
 * profiler reports template kernels (e.g. "dbp_pass_kernel<1024, 4, 2, true, 9>");
 * owned by the plan, valid until dbp_destroy; "" for NULL. */
const char* dbp_plan_kernel(dbp_plan_t plan);

/* Geometry the plan uses: block Nb, overlap O, steps per pass k, total steps
 * N_s, number of passes.  Any pointer may be NULL. */
dbp_status dbp_plan_geometry(dbp_plan_t plan, int32_t* block, int32_t* overlap,
                             int32_t* steps_per_pass, int32_t* n_steps, int32_t* n_passes);

/* Host-only: the geometry dbp_plan would choose for desc, without touching
 * the device (same validation as dbp_plan). */
dbp_status dbp_choose_geometry(const dbp_desc* desc, int32_t* block, int32_t* overlap,
                               int32_t* steps_per_pass);

/* Host-only: the FP64 step schedule for desc: b[s] = +-beta2 dz and
 * phi[s] = +-gamma exp(-alpha z_a) dz_eff for s < N_s (steps covering m whole
 * spans: +-beta2 m L and +-gamma m L_eff(L)); arrays of n entries, returns
 * DBP_ERR_INVALID_ARG if n < N_s. */
dbp_status dbp_schedule(const dbp_desc* desc, double* b, double* phi, int32_t n);

/* Host-only: the designed FIR taps (desc->fir == NULL, linear == DBP_LINEAR_FIR)
 * of step `step`: n_fir complex values (re, im interleaved) into out[2 n_fir].
 * Same validation as dbp_plan. */
dbp_status dbp_fir_taps(const dbp_desc* desc, int32_t step, float* out);

/* Bytes of device workspace dbp_backprop (grad = 0) or dbp_backprop_grad
 * (grad = 1) needs with this plan.  0 for an invalid plan (and, grad = 1, for
 * a plan whose gradient is not supported). */
size_t dbp_workspace_size(dbp_plan_t plan, int32_t grad);

/* Backpropagate (or, with DBP_FLAG_FORWARD, propagate) in -> out.
 *   in, out   device complex64 [batch][n_pol][n_samples]; in == out is
 *             allowed, any other overlap is DBP_ERR_INVALID_ARG.
 *   taps      device float32 [N_s][n_taps] overriding the plan's taps, or
 *             NULL for the plan's own (ESSFM only).
 *   fir       device complex64 [N_s][n_fir] overriding the plan's FIR taps, or
 *             NULL (FIR linear step only).
 *   ws        device workspace of ws_bytes >= dbp_workspace_size(plan, 0)
 *             (may be NULL when that size is 0).
 *   stream    hipStream_t. */
dbp_status dbp_backprop(dbp_plan_t plan, const void* in, void* out, const float* taps,
                        const void* fir, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dbp_backprop
 * with its workspace taken from a fixed device array of
 * DBP_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs on
 * until the process ends.  Arguments as dbp_backprop (the caller still owns in,
 * out, taps and fir); the call allocates and frees nothing.
 *   DBP_ERR_WORKSPACE     dbp_workspace_size(plan, 0) > DBP_NOALLOC_SCRATCH_BYTES
 *                         (two states of at most 16 MiB, e.g. 2 x 1048576
 *                         samples, or one state of 32 MiB for single-pass plans)
 *   DBP_ERR_INVALID_ARG   as dbp_backprop (batch plans, overlap, wrong device)
 *   DBP_ERR_HIP           the array's device address could not be found
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (nothing in it has to start at zero: each pass writes its
 * whole output state before the next reads it).  Calls that overlap in time on
 * one device (other streams, other host threads) race on it and must be
 * serialized by the caller. */
#define DBP_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
dbp_status dbp_backprop_noalloc(dbp_plan_t plan, const void* in, void* out, const float* taps,
                                const void* fir, void* stream);

/* Gradient of a real loss through dbp_backprop (reverse mode).  Given
 * grad_out = dL/dRe(out) + j dL/dIm(out) (device complex64, same shape as
 * in), writes grad_in (same convention; may be NULL; must not overlap
 * grad_out), grad_taps (device float32 [N_s][n_taps], ESSFM; may be NULL)
 * and grad_fir (device complex64 [N_s][n_fir], FIR plans; may be NULL; must
 * be NULL for FFT-step plans, which have no FIR taps).  taps and fir
 * override the plan's parameters as in dbp_backprop.
 *   FIR plans: the forward pass runs once storing the input of every step
 *     (FFT-block passes that keep each step's state; one time-domain launch
 *     per step on signals under 1024 samples), then the adjoint steps run in
 *     reverse, each from its step's input and output (the output gives the
 *     nonlinear substep's intensity and the FIR output without evaluating the
 *     FIR again).  With DBP_FLAG_GRAD_SPARSE, or when those N_s states would
 *     take more than 4 GiB, it stores every 8th step's input instead (each
 *     8-step segment run as FFT-block passes on signals of at least 1024
 *     samples) and recomputes each segment from its checkpoint before the
 *     segment's adjoint steps (less workspace, about one more forward pass of
 *     time).
 *   FFT-step plans (overlap-and-save, Sec. III): the derivative of exactly the
 *     blocked cascade dbp_backprop computes (same Nb, O, k).  The passes run
 *     forward once, keeping every block's field after the linear substep of
 *     every step; then each pass, in reverse, runs its blocks' step adjoints
 *     from those fields, and the window gradients of overlapping blocks are
 *     summed per sample in block order.  With DBP_FLAG_GRAD_SPARSE, or when
 *     the kept fields would take more than 4 GiB, or the plan's forward kernel
 *     is not the plain per-block one (polarization-split or streaming blocks,
 *     other values per thread, DBP_FP32), the forward keeps the pass inputs
 *     only and each reverse pass first re-runs its blocks' steps from them
 *     (less workspace, about one more forward pass of time; the same
 *     gradients, bit for bit, where both modes apply).  Block sizes
 *     256..4096; not the BF16X3 precision (UNSUPPORTED).  The phase argument
 *     of the reverse steps is formed in FP64.
 * Parameter gradients are summed over blocks, tiles and the batch in a fixed
 * order (bitwise reproducible).  ws_bytes >= dbp_workspace_size(plan, 1).
 * Gradients are overwritten, not accumulated. */
dbp_status dbp_backprop_grad(dbp_plan_t plan, const void* in, const float* taps,
                             const void* fir, const void* grad_out, void* grad_in,
                             float* grad_taps, void* grad_fir, void* ws, size_t ws_bytes,
                             void* stream);

/* The two halves of dbp_backprop_grad, for callers that run the forward pass
 * anyway (an autograd forward) and differentiate later: no forward step runs
 * twice.  dbp_backprop_save computes out = dbp_backprop(in) (out must not
 * overlap in) and leaves in ws (ws_bytes >= dbp_workspace_size(plan, 1)) what
 * the reverse pass reads: for FIR plans the checkpointed step inputs, for
 * FFT-step plans the kept block fields (or the pass inputs).  dbp_backprop_grad_saved then writes the
 * gradients of dbp_backprop_grad for upstream grad_out, given the same plan,
 * in, out, taps and fir, and ws as dbp_backprop_save left it (the reverse pass
 * overwrites only the parts of ws it recomputes, so it may run again for
 * another grad_out).  Errors as dbp_backprop_grad (DBP_ERR_INVALID_ARG also for
 * a field that overlaps ws); a ws, in or out changed in between gives wrong
 * gradients, which the library cannot detect. */
dbp_status dbp_backprop_save(dbp_plan_t plan, const void* in, void* out, const float* taps,
                             const void* fir, void* ws, size_t ws_bytes, void* stream);
dbp_status dbp_backprop_grad_saved(dbp_plan_t plan, const void* in, const void* out,
                                   const float* taps, const void* fir, const void* grad_out,
                                   void* grad_in, float* grad_taps, void* grad_fir, void* ws,
                                   size_t ws_bytes, void* stream);

/* Ragged batch: n descriptors (each batch == 1; any mix of lengths, links,
 * methods and taps, same n_pol) planned together.  Signal i occupies
 * [n_pol][L_i] at element offset offsets[i] of one packed buffer. */
dbp_status dbp_plan_batch(const dbp_desc* descs, int32_t n, dbp_plan_t* out);

/* Element (complex64) offsets of every signal of a batch plan in the packed
 * buffer, host array of n + 1 entries (the last is the total). */
dbp_status dbp_batch_offsets(dbp_plan_t plan, int64_t* offsets, int32_t n_plus_1);

/* Geometry chosen for signal i of a batch plan (the autotuner measures the
 * cost of each block size once per process and kernel variant, timing the batch
 * kernel on a synthetic signal at 1 and 4 steps per pass, then picks
 * for every signal the block, overlap and steps per pass of least modelled
 * time; explicit block/overlap/steps_per_pass in a descriptor are kept).
 * DBP_TUNE_CACHE=<file> keeps the measured costs across processes: JSON
 * lines keyed by GPU architecture, CU count and kernel variant, read before
 * timing and appended after it (unparsable lines and non-positive or
 * non-finite costs are ignored; the last matching line wins). */
dbp_status dbp_batch_geometry(dbp_plan_t plan, int32_t i, int32_t* block, int32_t* overlap,
                              int32_t* steps_per_pass);

/* Backpropagate every signal of a batch plan: in_packed -> out_packed (device
 * complex64, layout of dbp_batch_offsets; in == out allowed).  ws_bytes >=
 * dbp_workspace_size(plan, 0) (twice the packed size).  All passes of all
 * signals run in one persistent launch per kernel variant, pass n+1 of a
 * block waiting only on its neighbours' pass n, the launches captured once
 * into a HIP graph (per in/out/ws triple) and replayed on `stream`. */
dbp_status dbp_backprop_batch(dbp_plan_t plan, const void* in_packed, void* out_packed,
                              void* ws, size_t ws_bytes, void* stream);

/* Synchronous: error flags of the last completed batch run, or of the last
 * persistent run of a DBP_FLAG_PERSISTENT plan (0: none; bit 0:
 * a dependency wait exceeded its bound and the block was skipped). */
dbp_status dbp_batch_status(dbp_plan_t plan, int32_t* flags);

/* Receiver mode (the latency discussion of Sec. III): the received field as an
 * unbounded stream x[n], n >= 0, preceded by silence, pushed in chunks and
 * backpropagated through the same passes and overlap-and-save blocks as
 * dbp_backprop, without the wrap at the signal ends: block b of every pass has
 * the window [bV - O/2, bV - O/2 + Nb) and keeps [bV, bV + V), and a pass
 * computes a block once its window lies inside the samples it has.  Each pass
 * trails the previous one by c = ceil((O/2) / V) blocks, so the output trails the
 * input by D = n_passes * c * V samples: push i (counted from creation or the
 * last reset) returns the output samples [i C - D, (i + 1) C - D), zeros before
 * n = 0.  The output equals that of dbp_backprop on the whole stream preceded by
 * enough silence, up to the end effects of the latter's wrap. */
typedef struct dbp_rx_s* dbp_rx_t;

/* Create a receiver for desc's link, method and geometry (batch 1, FFT linear
 * step, not BF16X3, not DBP_FLAG_WHOLE; desc->n_samples is ignored: the planner
 * sees the chunk length).  chunk: samples per polarization per push, >= Nb and a
 * multiple of V = Nb - O (DBP_ERR_INVALID_ARG otherwise), at most 2^29
 * (DBP_ERR_UNSUPPORTED above, checked before any device work: the rings hold at
 * most 2^31 samples).  Block sizes
 * 256..4096 (DBP_ERR_UNSUPPORTED otherwise).  The receiver owns its device
 * state (one ring per pass, allocated and cleared here, synchronously, on the
 * current device); *out is NULL on error. */
dbp_status dbp_rx_create(const dbp_desc* desc, int64_t chunk, dbp_rx_t* out);

/* Latency D in samples and the geometry in use.  Any pointer may be NULL. */
dbp_status dbp_rx_info(dbp_rx_t rx, int64_t* latency, int32_t* block, int32_t* overlap,
                       int32_t* steps_per_pass, int32_t* n_passes);

/* Push the next chunk: in and out are device complex64 [n_pol][chunk] (not
 * overlapping).  Asynchronous on stream; pushes on one receiver must be issued in
 * order on one stream (the receiver's state advances on the host at each call). */
dbp_status dbp_rx_push(dbp_rx_t rx, const void* in, void* out, void* stream);

/* Restart at n = 0 with silence before it (asynchronous on stream). */
dbp_status dbp_rx_reset(dbp_rx_t rx, void* stream);

/* Release the receiver (NULL is a no-op); no push may still be running. */
void dbp_rx_destroy(dbp_rx_t rx);

/* Receiver DSP after backpropagation (Sec. IV): the captured blocks are
 * backpropagated at the scope's sampling rate (about 1.8 samples per symbol),
 * resampled to two samples per symbol, passed through a butterfly equalizer
 * that adapts to polarization effects and residual dispersion, and detected at
 * the symbol rate with phase-noise tracking.  The paper names these stages but
 * not their algorithms; this library implements:
 *   resampling   y[m] = sum_k x[(i_m + k) mod n] h(t_m - i_m - k), t_m = m down / up,
 *                i_m = floor(t_m), k = -K/2+1 .. K/2, h(tau) = sinc(tau) I0(beta
 *                sqrt(1 - (tau / (K/2))^2)) / I0(beta) (Kaiser-windowed sinc), up >= down
 *   equalizer    y_p[k] = sum_q sum_j W[p][q][j] x_q[(2k + j - N/2) mod n2], the taps the
 *                data-aided least-squares (Wiener) solution on the first n_train symbols
 *   phase        theta_k = arg(-sum_{|j|<=W} y[(k+j) mod n]^4) / 4 per polarization,
 *                phi_k = theta_0 + sum_{0<j<=k} wrap_{pi/2}(theta_j - theta_{j-1}),
 *                z = y exp(-j phi) (quarter turns resolved on known symbols);
 *                QPSK decisions by the signs of Re z and Im z.
 * All fields are complex64 [2][n] (two polarizations) on the current device. */
typedef struct dbp_dsp_s* dbp_dsp_t;

typedef struct {
    int32_t up, down;          /* output/input rate ratio, 1 <= down <= up <= 4096 (e.g. 28/25) */
    int32_t resample_taps;     /* K: even, 2..64 */
    double  kaiser_beta;       /* beta >= 0 */
    int32_t eq_taps;           /* N: odd, 1..31, taps per butterfly branch (T/2-spaced) */
    int32_t cpr_half_window;   /* W: 0..256 */
} dbp_dsp_desc;

/* Create the receiver DSP for input blocks of n_in samples per polarization at
 * the input rate; n_out = n_in up / down must be an integer and even (n_sym =
 * n_out / 2 symbols).  Allocates its tables and all scratch of the later calls
 * on the current device (synchronously; no later call allocates); *out is NULL
 * on error (DBP_ERR_INVALID_ARG for a bad desc or size).  Calls on one dsp share
 * its scratch: issue them in order on one stream, with the device current that
 * was current at create (else DBP_ERR_INVALID_ARG, no device work). */
dbp_status dbp_dsp_create(const dbp_dsp_desc* desc, int64_t n_in, dbp_dsp_t* out);

/* Sizes: n_out samples per polarization after resampling, n_sym symbols.  Either
 * pointer may be NULL. */
dbp_status dbp_dsp_info(dbp_dsp_t dsp, int64_t* n_out, int64_t* n_sym);

/* in [2][n_in] -> out [2][n_out] (device, not overlapping).  Asynchronous on stream. */
dbp_status dbp_dsp_resample(dbp_dsp_t dsp, const void* in, void* out, void* stream);

/* Least-squares butterfly taps from the resampled field x2 [2][n_out] and the
 * transmitted symbols sym [2][n_sym] (device): the normal equations are summed
 * on the GPU (per-chunk FP32 sums added in FP64 in a fixed order) and solved
 * there in FP64 (Gaussian elimination with partial pivoting in one workgroup);
 * taps [2][2][N] complex64 are written to device memory.  1 <= n_train <= n_sym.
 * Asynchronous on stream; a singular system leaves NaN taps and sets bit 0 of
 * dbp_dsp_status. */
dbp_status dbp_dsp_train(dbp_dsp_t dsp, const void* x2, const void* sym, int64_t n_train, void* taps,
                         void* stream);

/* Synchronous: flags of the last completed training (0: none; bit 0: its system
 * was singular). */
dbp_status dbp_dsp_status(dbp_dsp_t dsp, int32_t* flags);

/* y [2][n_sym] = the butterfly with device taps [2][2][N] applied to x2 [2][n_out].
 * Asynchronous on stream. */
dbp_status dbp_dsp_equalize(dbp_dsp_t dsp, const void* x2, const void* taps, void* y, void* stream);

/* Carrier-phase recovery and decisions: z [2][n_sym] from y [2][n_sym].  The
 * fourth-power estimate is blind to quarter turns; with the transmitted symbols
 * sym (device [2][n_sym]) and 0 < n_ref <= n_sym, the rotation by q pi/2 that best
 * aligns the first n_ref derotated symbols with them (q the nearest integer to
 * arg(sum z_k conj(s_k)) / (pi/2), per polarization) is applied as well (n_ref = 0:
 * none).  With sym and bit_errors (host) the number of wrong decision bits is
 * counted on the GPU and returned (then the call synchronizes stream); otherwise
 * asynchronous.  sym may be NULL when n_ref = 0; z may not overlap y. */
dbp_status dbp_dsp_cpr(dbp_dsp_t dsp, const void* y, const void* sym, int64_t n_ref, void* z, int64_t* bit_errors,
                       void* stream);

/* Release (NULL is a no-op); no call on it may still be running. */
void dbp_dsp_destroy(dbp_dsp_t dsp);

/* Loss head of the differentiation workload (Sec. IV footnote: the ESSFM
 * coefficients can be optimized for the mean squared error between the detected
 * symbols and the transmitted ones), and its reverse mode, so that a training
 * step runs entirely in this library:
 *   loss = (1 / (batch n_pol L/2)) sum |y[2m] / amp - s[m]|^2,
 *   y = IDFT_L(DFT_L(z) mf) per signal and polarization (circular over L),
 * i.e. the receive filter mf (real, on the length-L DFT grid, hence
 * self-adjoint) followed by one sample per symbol at two samples per symbol;
 * amp is the symbol amplitude of the field.  The reverse mode is
 *   grad_z = g IDFT_L(DFT_L(up) mf),  up[2m] = 2 (y[2m] / amp - s[m]) / (amp N),
 *   up[2m + 1] = 0,  N = batch n_pol L/2,  g = dL/dloss,
 * with complex gradients dL/dRe + j dL/dIm.  No length-L transform is run: the
 * even and odd bins are two L/2-point transforms and the decimated output two
 * L/4-point ones.  L = n_samples, a power of two from 2048 to 32768; z and
 * grad_z device complex64 [batch][n_pol][L], symbols device complex64
 * [batch][n_pol][L/2].  Allocates its tables and every scratch of the later
 * calls on the current device at create (mf: host float64 [L], copied). */
typedef struct dbp_mse_s* dbp_mse_t;

/* DBP_ERR_INVALID_ARG for a bad size, count, amplitude or non-finite mf;
 * DBP_ERR_UNSUPPORTED for L outside 2048..32768.  *out is NULL on error. */
dbp_status dbp_mse_create(int64_t n_samples, int32_t n_pol, int32_t batch, const double* mf,
                          double amplitude, dbp_mse_t* out);

/* loss (device float32, one value) of the field z against the symbols.  Keeps
 * the residual y[2m] / amp - s[m] in the handle for dbp_mse_backward.
 * Asynchronous on stream; the per-signal sums are added in FP64 in a fixed
 * order (bitwise reproducible). */
dbp_status dbp_mse_forward(dbp_mse_t mse, const void* z, const void* symbols, float* loss,
                           void* stream);

/* grad_z for the residual of the last dbp_mse_forward on this handle, scaled by
 * the device float32 *grad_loss (NULL: 1).  Asynchronous on stream; calls on one
 * handle share its scratch and must be issued in order on one stream, with
 * the device current that was current at create (else DBP_ERR_INVALID_ARG). */
dbp_status dbp_mse_backward(dbp_mse_t mse, const float* grad_loss, void* grad_z, void* stream);

/* Release (NULL is a no-op); no call on it may still be running. */
void dbp_mse_destroy(dbp_mse_t mse);

/* Short static description of a status code; any value is accepted ("unknown
 * status" for values that are not a dbp_status). */
const char* dbp_status_string(int32_t s);

/* Library version, e.g. 0x000100 for 0.1.0. */
int32_t dbp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DBP_H */
