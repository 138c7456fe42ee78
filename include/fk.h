/*
 * fk.h -- C ABI of the MI355X fused preprocessing-chain library (libfkmi.so).
 *
 * The library executes a chain made of ONE read operation, a list of
 * elementwise compute operations and ONE write operation as a single
 * vertically fused kernel (every intermediate stays in registers), over a
 * batch of independent items in a single horizontally fused launch.  This
 * follows the paper's problem statement: compute ops (unary and binary, the
 * operation-types table of Section IV-A), memory ops that read from and
 * write to device memory using the thread's coordinates (Section IV-B),
 * batch memory ops that select per-item parameters (Section IV-B,
 * BatchRead), a transform data-parallel pattern that connects them
 * (Section IV-C), and lazy execution through an executor that receives the
 * whole chain (Section IV-D).
 *
 * Conventions for every call:
 *  - All integers are fixed width.  Pointers named d_* or marked "device"
 *    point to device memory of the current HIP device; everything else is
 *    host memory.
 *  - The caller owns every device buffer (frames, outputs, scratch) and every
 *    stream.  The library never frees them.  The library owns fk_plan and
 *    frees it in fk_plan_destroy.
 *  - Every call returns an fk_status.  All argument checks happen before any
 *    device work is queued; on a negative status nothing was launched.  HIP
 *    errors map to FK_ERR_HIP.  The message of the last failure on the
 *    calling thread is available from fk_last_error().
 *  - No C++ exception crosses this interface.
 *  - A plan is not thread-safe: use one plan per host thread / stream.
 */
#ifndef FK_H
#define FK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fk_status;
#define FK_OK 0
#define FK_ERR_INVALID_ARG (-1)  /* null pointer, bad size, ROI outside its frame, ... */
#define FK_ERR_UNSUPPORTED (-2)  /* valid request the library does not implement */
#define FK_ERR_OUT_OF_MEMORY (-3)
#define FK_ERR_HIP (-4)          /* a HIP runtime call failed; see fk_last_error() */
#define FK_ERR_BAD_STATE (-5)    /* call not allowed in the object's current state */
#define FK_ERR_BUDGET (-6)       /* request exceeds a memory budget */

/* Element types.  FK_F64 is the output type of the stats write, and the
 * input and output type of double-precision chains (below). */
#define FK_U8 0
#define FK_F16 1
#define FK_F32 2
#define FK_F64 3

/* Image layouts: packed HWC (out[(y*W + x)*C + c]) or planar CHW
 * (out[(c*H + y)*W + x]); Split is the packed-to-planar write op
 * (Section IV-B, the memory-ops figure). */
#define FK_PACKED 0
#define FK_PLANAR 1

/* Stats write: the reduction pattern of Section IV-C, several reductions of
 * one matrix from a single read.  Instead of an image, an item's output is,
 * for each channel c, four doubles at dst[4c .. 4c+3]: the minimum, the
 * maximum, the sum and the mean of the chain's fp32 values over the item's
 * output pixels.  Min and max are IEEE minNum/maxNum (a NaN value is
 * skipped; all NaN gives +inf / -inf); the sum accumulates the values in
 * fp64 (in an order that depends on the launch configuration, within
 * 2 (n - 1) 2^-53 sum|x| of any other order); mean = sum / n in fp64.
 * Requires out_dtype = FK_F64; dst must be 8-byte aligned.  A run is two
 * launches on the caller's stream (block partials, then one combine block
 * per item); the partials live in the plan, so runs of one plan must not
 * overlap on different streams. */
#define FK_STATS 2

/* Read operations (Section IV-B).
 * FK_READ_PLAIN: the item's region of interest read 1:1 (a crop when the
 *   ROI is smaller than the frame); output size = ROI size.
 * FK_READ_CROP_RESIZE: the ROI is bilinearly resized to the item's output
 *   size: half-pixel centres, no antialiasing, taps clamped to the ROI,
 *   source coordinate s = max(fma(o + 0.5, in/out, -0.5), 0) in fp32, lerps
 *   written as fma(a, p1 - p0, p0); the resized value stays fp32. */
#define FK_READ_PLAIN 0
#define FK_READ_CROP_RESIZE 1
/* FK_READ_CROP_NEAREST: the ROI is resized to the output size by nearest
 *   neighbour: output index o takes ROI index floor((2o + 1) * in / (2 out))
 *   in exact integer arithmetic (the pixel holding the output pixel's
 *   centre; a centre on a boundary takes the higher index).
 * FK_READ_NV12 / FK_READ_NV12_RESIZE: the frame is NV12 (in_dtype FK_U8,
 *   channels 3): a width x height luma plane at src.ptr, then height/2 rows
 *   of width/2 interleaved (U, V) byte pairs at src.ptr + height *
 *   pitch_bytes, same pitch; width and height even; 3 * height / 2 rows
 *   readable.  Pixel (x, y) takes Y[y][x] and the pair of (x/2, y/2) and
 *   becomes B, G, R in fp32 by the ITU-R BT.601 limited-range matrix: with
 *   y' = Y - 16, u = U - 128, v = V - 128, c = 1.164 y', B = c + 2.018 u,
 *   G = (c - 0.813 v) - 0.391 u, R = c + 1.596 v, one fp32 operation each
 *   in that order.  The ROI is in luma pixels; FK_READ_NV12 reads it 1:1,
 *   FK_READ_NV12_RESIZE resizes the converted ROI bilinearly as above. */
#define FK_READ_CROP_NEAREST 2
#define FK_READ_NV12 3
#define FK_READ_NV12_RESIZE 4

/* Compute operations (Section IV-A; the hot chain of Sections VI-F/VI-J).
 * SWAP_RB: exchange channels 0 and 2 (BGR<->RGB), channel 3 kept, no-op for
 *   1 channel.  CVT_F32: convert to fp32 (exact from u8/f16; identity on
 *   fp32).  Arithmetic on a u8/f16 value promotes it to fp32 first.
 * MUL/ADD/SUB/DIV: one fp32 operation with a scalar (n_consts = 1) or
 *   per-channel (n_consts = channels) constant; per-channel constants index
 *   the channel position after earlier swaps.  DIV is an IEEE division.
 * LOOP: the repeat op of Section VI-B (one op instance applied many times
 *   without spending kernel parameters on each copy): the loop_span ops just
 *   before it run loop_count times in all, in order (the first of those runs
 *   is the one the chain reaches before the LOOP).  The body may hold
 *   MUL/ADD/SUB/DIV only (no swap, no cvt, no other loop); n_consts = 0.
 *   A loop is one entry of the op list whatever its count. */
#define FK_OP_SWAP_RB 0
#define FK_OP_CVT_F32 1
#define FK_OP_MUL 2
#define FK_OP_ADD 3
#define FK_OP_SUB 4
#define FK_OP_DIV 5
#define FK_OP_LOOP 6

#define FK_MAX_OPS 4096

typedef struct {
    int32_t kind;      /* FK_READ_* */
    int32_t in_dtype;  /* FK_U8, FK_F16, FK_F32; FK_F64 for a plain read whose
                          write is FK_F64 */
    int32_t channels;  /* 1, 3 or 4, packed in the source frame */
} fk_read_desc;

typedef struct {
    int32_t kind;      /* FK_OP_* */
    int32_t n_consts;  /* 0 for SWAP_RB/CVT_F32/LOOP; 1 or `channels` otherwise */
    float consts[4];
    int32_t loop_span;  /* LOOP: 1 .. (index of this op); ignored otherwise */
    int32_t loop_count; /* LOOP: >= 1; ignored otherwise */
} fk_op_desc;

typedef struct {
    int32_t out_dtype; /* FK_F32 or FK_F16 (round to nearest even); FK_F64 with FK_STATS,
                          or a double-precision chain */
    int32_t layout;    /* FK_PACKED, FK_PLANAR or FK_STATS */
} fk_write_desc;

/* Double-precision chains (the data-type experiment of Section VI-I, whose
 * float->double and double->double kernels compute in double): a plain read
 * with an FK_F64 packed or planar write computes in fp64 from the read on.
 * The read takes FK_U8/FK_F16/FK_F32 elements exactly and FK_F64 elements
 * as they are; CVT_F32 is then the identity; each MUL/ADD/SUB/DIV is one
 * IEEE fp64 operation with the op's fp32 constant taken exactly; strict_fp
 * = 0 fuses a MUL followed by ADD/SUB into one fp64 FMA.  Other read kinds
 * with an FK_F64 image write, and an FK_F64 frame with any other write,
 * are refused with FK_ERR_UNSUPPORTED.  The cost model does not cover these
 * chains (fk_model_features returns FK_ERR_UNSUPPORTED). */

/* A chain: read -> ops[0..n_ops) -> write.  `ops` is copied at plan
 * creation. */
typedef struct {
    fk_read_desc read;
    const fk_op_desc *ops;
    int32_t n_ops;     /* 0 .. FK_MAX_OPS */
    fk_write_desc write;
} fk_chain_desc;

/* A frame in device memory, packed HWC with `channels` channels of
 * `in_dtype` (the RawPtr/Ptr data descriptor of Section IV-B).
 * pitch_bytes >= width * channels * sizeof(element) and a multiple of the
 * element size; every row must be readable.  Width and height are at most
 * 65535 (larger frames are refused with FK_ERR_UNSUPPORTED: row and column
 * indices feed 24-bit multiplies in the kernels). */
typedef struct {
    const void *ptr;   /* device */
    int32_t width, height;
    int64_t pitch_bytes;
} fk_image;

/* One batch slot (one element of the BatchRead parameter array).  The ROI
 * (x, y, w, h) must lie inside `src`.  `dst` (device) receives out_w x
 * out_h x channels elements of the write dtype in the write layout,
 * densely (row pitch = out_w elements; planes of out_w*out_h).  For
 * FK_READ_PLAIN, out_w/out_h must be 0 or equal to w/h.  A resizing read's
 * out_w and out_h are at most 65535 each and out_w * out_h at most 2^28
 * (else FK_ERR_UNSUPPORTED); a plain read's ROI at most 2^28 pixels. */
typedef struct {
    fk_image src;
    int32_t x, y, w, h;
    void *dst;         /* device */
    int32_t out_w, out_h;
} fk_item;

/* Launch configuration: threads per block (64, 128, 256, 512 or 1024) and
 * thread coarsening (1, 2, 4 or 8 units of four output pixels per thread;
 * Section IV-C's transform pattern with thread coarsening). */
typedef struct {
    int32_t block_threads;
    int32_t coarsen;
} fk_launch_config;

#define FK_CONFIG_DEFAULT 0  /* 256 threads; coarsening 1, except: 4 for the
                                256-op compile-time chain and other compile-time
                                chains of more than 32 normalised ops; 2 for a
                                run-time op list of more than 32 records after
                                a plain read; 8 for a stats write */
#define FK_CONFIG_MANUAL 1   /* opts.manual */
#define FK_CONFIG_AUTOTUNE 2 /* set by fk_autotune (default until then) */
#define FK_CONFIG_MODEL 3    /* predicted by a cost model (fk_plan_use_model) */

#define FK_TIER_AUTO 0       /* compile-time chain when one matches, else run-time op list */
#define FK_TIER_RUNTIME 1    /* always the run-time op list */

typedef struct {
    int32_t config_source;   /* FK_CONFIG_* */
    fk_launch_config manual; /* used when config_source == FK_CONFIG_MANUAL */
    int32_t use_graph;       /* 1: fk_run replays a captured hipGraph */
    int32_t strict_fp;       /* 1: no mul+add contraction: bit-exact with the
                                per-op definition; 0: a multiply followed by an
                                add/sub is one fused multiply-add */
    int32_t tier;            /* FK_TIER_* */
    int32_t unfused_loop_kernel; /* fk_run_unfused only: 1 = a loop over a single
                                    op is one kernel applying it loop_count times
                                    (an op of that many instructions, Section
                                    VI-E); 0 = one kernel per run of the op */
    int32_t gather;          /* FK_GATHER_*: how the compile-time normalise
                                chain (crop + bilinear resize of a u8 BGR frame
                                -> planar fp32) reads its taps; other chains
                                ignore it */
} fk_plan_opts;

#define FK_GATHER_DIRECT 0   /* each lane loads its taps' byte windows from the frame */
#define FK_GATHER_LDS 1      /* a block stages the tap rows of a band of output rows in
                                LDS with 16-byte loads over the ROI's width, then reads
                                the taps from LDS (same results); items whose frame base
                                or pitch is not a multiple of 16 bytes, or whose staged
                                rows do not fit, read directly */

typedef struct fk_plan fk_plan;

/* Status text of a code, and the last error message on this thread. */
const char *fk_status_string(fk_status s);
const char *fk_last_error(void);

/* Library version and the device architecture the library is compiled for. */
const char *fk_version(void);

/* Check a chain without touching the device.  FK_OK or FK_ERR_INVALID_ARG /
 * FK_ERR_UNSUPPORTED. */
fk_status fk_chain_validate(const fk_chain_desc *chain);

/* Check items against a chain without touching the device (host fields
 * only; device pointers are checked for null).  `n_items` may be 0. */
fk_status fk_items_validate(const fk_chain_desc *chain, const fk_item *items, int32_t n_items);

/* Create a plan for `chain` and up to `max_batch` items per run (the batch
 * capacity; each run passes its own count, Section IV-B).  `opts` may be
 * NULL (defaults).  Allocates the plan's op list on the device; the ring
 * of four run tables for batches too large for the kernel arguments (and
 * for graph replays) is allocated whole by the first run that needs a
 * table, so that later runs allocate no memory.
 * Selects the kernel: a compile-time composed chain when the chain matches
 * one built into the library, else the run-time op-list kernel. */
fk_status fk_plan_create(const fk_chain_desc *chain, int32_t max_batch, const fk_plan_opts *opts,
                         fk_plan **out);

/* Destroy a plan (waits for its pending work).  NULL is allowed. */
fk_status fk_plan_destroy(fk_plan *plan);

fk_status fk_plan_get_config(const fk_plan *plan, fk_launch_config *out);
fk_status fk_plan_set_config(fk_plan *plan, const fk_launch_config *cfg);

/* Which kernel the plan uses: 1 = compile-time chain, 0 = run-time list. */
fk_status fk_plan_get_tier(const fk_plan *plan, int32_t *is_static);

/* Fused execution (asynchronous on `stream`, a hipStream_t; NULL = the
 * default stream): one horizontally and vertically fused launch covering
 * all `n_items` items (1 <= n_items <= max_batch).  The items' parameters
 * travel in the kernel arguments (up to 32 items; up to 312 items that
 * share one frame and one output size and whose outputs lie at a constant
 * stride), else in a device run table that a small upload kernel fills
 * on the same stream just before the launch.  A constant-stride batch of
 * more than 312 items (not a stats write) goes out as consecutive launches
 * of up to 312 items.  `items` is copied before the call returns; a
 * table run first waits for the run that used the same table slot four
 * table runs earlier.
 *
 * Under the caller's stream capture (hipStreamBeginCapture on `stream`,
 * e.g. to replay several runs as one graph: a graph launch costs about as
 * much host time as several direct launches, so one graph per run does not
 * pay), a run whose items travel in the kernel arguments is captured as
 * its kernel launches, parameters included; any other run returns
 * FK_ERR_UNSUPPORTED before touching the stream (its table is staged in
 * host memory that later runs rewrite), and so does a plan with use_graph
 * or a timed run. */
fk_status fk_run(fk_plan *plan, const fk_item *items, int32_t n_items, void *stream);

/* fk_run with the launch's device time: `start_event` and `stop_event`
 * (hipEvent_t, created with timing enabled by the caller, who owns them)
 * are recorded by the fused launch itself as its kernel starts and ends
 * (hipExtLaunchKernel), so hipEventElapsedTime gives the kernel's
 * duration without the latency of separate event markers.  A stats write
 * brackets both of its kernels, a batch split into several launches the
 * first and the last; the table upload kernel stays outside.  A plan that
 * replays a graph records the events around the graph launch.  Either
 * event may be NULL. */
fk_status fk_run_timed(fk_plan *plan, const fk_item *items, int32_t n_items, void *stream,
                       void *start_event, void *stop_event);

/* Bytes of device scratch fk_run_unfused needs for these items. */
fk_status fk_unfused_scratch_bytes(const fk_plan *plan, const fk_item *items, int32_t n_items,
                                   int64_t *bytes);

/* Unfused baseline (the separate-kernel pipeline of the kernel-call
 * algorithm, Section II): one kernel per operation and per item, every
 * intermediate materialised in `d_scratch` (device, caller-owned, at least
 * fk_unfused_scratch_bytes).  Same results as fk_run with strict_fp = 1. */
fk_status fk_run_unfused(fk_plan *plan, const fk_item *items, int32_t n_items, void *d_scratch,
                         int64_t scratch_bytes, void *stream);

/* Workspace the library holds for fk_run_unfused_noalloc: 32 MiB per
 * device, reserved when the library's code is loaded on that device and
 * held until the process ends. */
#define FK_NOALLOC_SCRATCH_BYTES (32ll << 20)

/* fk_run_unfused for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, with the workspace taken from the
 * library's own FK_NOALLOC_SCRATCH_BYTES device array instead of a caller
 * buffer.  No hipMalloc, hipFree or other allocating call is made.  The
 * caller still owns the frames and outputs.  Items whose workspace
 * (fk_unfused_scratch_bytes) exceeds FK_NOALLOC_SCRATCH_BYTES are rejected
 * with FK_ERR_UNSUPPORTED before any launch.  The first call on a device
 * looks up the array's address there (hipGetSymbolAddress, current
 * device).  All calls on one device share the one array and it keeps the
 * last call's contents: calls on the same stream are ordered, calls that
 * overlap on one device (other streams, other threads) race. */
fk_status fk_run_unfused_noalloc(fk_plan *plan, const fk_item *items, int32_t n_items,
                                 void *stream);

/* Number of launch configurations the autotuner tries (20); fills space[i]
 * with the i-th for i < max_configs (space may be NULL). */
int32_t fk_autotune_space(fk_launch_config *space, int32_t max_configs);

/* Time every launch configuration on these items (one warm-up launch, then
 * the median of 3 samples of `reps` back-to-back launches timed by HIP
 * events on an internal stream, divided by `reps`), write the 20
 * median times in milliseconds to `times_ms` (may be NULL), select the
 * fastest (ties: fewer threads, then less coarsening) into the plan and
 * `best` (may be NULL).  Synchronous; outputs are overwritten.  The
 * internal stream does not wait for the caller's streams: the frames must
 * be ready (e.g. the stream that wrote them synchronized) before the call.
 * Every launch reads the same items, so frames that fit the 256 MB
 * Infinity Cache are timed from it; the times are those of an n_items
 * launch, and a batched launch ranks configurations differently from a
 * single-item one. */
fk_status fk_autotune(fk_plan *plan, const fk_item *items, int32_t n_items, int32_t reps,
                      float *times_ms, fk_launch_config *best);

/* ------------------------------------------------------------------------
 * Launch-configuration cost model (not in the paper: the paper fixes its
 * launch shapes, e.g. 32x8x1 blocks).  A fully connected ReLU network,
 * FK_MODEL_FEATURES -> hidden -> hidden -> hidden -> FK_MODEL_OUTPUTS,
 * fp32, that predicts the log-time ratio t(config) / t(best) of each of the
 * autotuner's 20 configurations; the prediction's argmin is the chosen
 * configuration.  Trained and run on the GPU by the library's own kernels
 * (tiled fp32 GEMM with bias/ReLU epilogues, column sums, MSE, Adam). */
#define FK_MODEL_FEATURES 32
#define FK_MODEL_OUTPUTS 20

typedef struct fk_model fk_model;

/* New model with `hidden` units per hidden layer (1..1024), weights drawn
 * He-uniform from `seed`, biases zero, feature normalisation identity.
 * Allocates device memory. */
fk_status fk_model_create(int32_t hidden, uint64_t seed, fk_model **out);
fk_status fk_model_destroy(fk_model *model);

/* Number of fp32 parameters; layout: for each layer l, W_l (out x in,
 * row-major) then b_l (out). */
int64_t fk_model_param_count(const fk_model *model);
fk_status fk_model_get_params(const fk_model *model, float *out, int64_t n);
fk_status fk_model_set_params(fk_model *model, const float *in, int64_t n);
/* Per-feature normalisation x' = (x - mean) / std applied before the
 * network (host arrays of FK_MODEL_FEATURES). */
fk_status fk_model_get_normalization(const fk_model *model, float *mean, float *std);
fk_status fk_model_set_normalization(fk_model *model, const float *mean, const float *std);

/* Features of a (plan, items) pair: chain shape (read kind, dtypes,
 * channels, layout, normalised op counts, tier) and item geometry (sizes,
 * scales, bytes, alignment), FK_MODEL_FEATURES floats into `out` (host).
 * Host only. */
fk_status fk_model_features(const fk_plan *plan, const fk_item *items, int32_t n_items, float *out);

/* Train on n samples (host arrays: features n x FK_MODEL_FEATURES, targets
 * n x FK_MODEL_OUTPUTS) for `epochs` passes of shuffled mini-batches of
 * `batch` rows, Adam (beta1 0.9, beta2 0.999, eps 1e-8) at learning rate lr,
 * MSE loss.  The first training call fixes the feature normalisation from
 * these features (per-feature mean and standard deviation, fp64 sums; 1 for
 * a constant feature).  loss_curve (host, may be NULL) receives each
 * epoch's mean mini-batch loss.  Synchronous: copies the arrays to the
 * device and runs fk_model_train_device on the model's stream, so both
 * calls give the same parameters from the same inputs and seed. */
fk_status fk_model_train(fk_model *model, const float *features, const float *targets, int32_t n,
                         int32_t epochs, int32_t batch, float lr, uint64_t seed, float *loss_curve);

/* fk_model_train on device arrays, queued on `stream` (a hipStream_t; NULL
 * = the default stream): d_features (n x FK_MODEL_FEATURES, raw features),
 * d_targets (n x FK_MODEL_OUTPUTS) and d_loss_curve (`epochs` floats, may
 * be NULL) are device memory that must stay valid until the stream has
 * run the work.  The mini-batch permutations (SplitMix64-driven
 * Fisher-Yates, one per epoch) are drawn on the host into a pinned buffer
 * the model owns.  Returns once the work is queued, except that the first
 * training call of a model waits for its normalisation statistics.  Any
 * later call on the model first waits for this training to finish. */
fk_status fk_model_train_device(fk_model *model, const float *d_features, const float *d_targets,
                                int32_t n, int32_t epochs, int32_t batch, float lr, uint64_t seed,
                                float *d_loss_curve, void *stream);

/* The network's kernels one by one, on device arrays, asynchronous on
 * `stream` (used by the gradient checks and by callers that train their
 * own way).  None of them normalises features: d_x holds the network's
 * inputs.  Each first waits for a training run queued by
 * fk_model_train_device.
 *
 * Workspace of n rows, in floats: the three hidden layers' outputs
 * (n x hidden each, left by fk_mlp_forward for fk_mlp_backward), then two
 * propagated-gradient buffers of n x max(hidden, FK_MODEL_OUTPUTS).  -1 on
 * a bad argument. */
int64_t fk_mlp_workspace_floats(const fk_model *model, int32_t n);

/* Forward pass: d_x (n x FK_MODEL_FEATURES) -> d_y (n x FK_MODEL_OUTPUTS),
 * hidden outputs kept in d_ws. */
fk_status fk_mlp_forward(const fk_model *model, const float *d_x, int32_t n, float *d_ws,
                         float *d_y, void *stream);

/* Backward pass: the gradient of a loss with respect to every parameter
 * (d_grad: fk_model_param_count floats, the parameter layout) from the
 * loss's gradient d_dy (n x FK_MODEL_OUTPUTS) with respect to the outputs
 * of the fk_mlp_forward call that filled d_ws from the same d_x.  d_dy must
 * not lie inside d_ws. */
fk_status fk_mlp_backward(const fk_model *model, const float *d_x, int32_t n, float *d_ws,
                          const float *d_dy, float *d_grad, void *stream);

/* Mean-squared-error loss of n x FK_MODEL_OUTPUTS outputs against targets:
 * d_loss[0] = mean (y - t)^2 and d_dy = 2 (y - t) / (n FK_MODEL_OUTPUTS). */
fk_status fk_mlp_mse(const float *d_y, const float *d_t, int32_t n, float *d_dy, float *d_loss,
                     void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) of the
 * model's parameters along d_grad (device, the parameter layout), with the
 * model's moment estimates; advances the model's step count t (bias
 * corrections 1 - beta^t). */
fk_status fk_mlp_step(fk_model *model, const float *d_grad, float lr, void *stream);

/* Network outputs for n feature rows (host in, host out n x
 * FK_MODEL_OUTPUTS).  Synchronous. */
fk_status fk_model_predict_batch(fk_model *model, const float *features, int32_t n, float *out);

/* One forward + backward pass without an update: mean-squared-error loss of
 * n rows against `targets` and its gradient w.r.t. every parameter (host,
 * fk_model_param_count floats, same layout as the parameters). */
fk_status fk_model_loss_grad(fk_model *model, const float *features, const float *targets,
                             int32_t n, float *loss, float *grad);

/* Predicted best launch configuration for running `plan` on these items,
 * and the same applied to the plan (config source FK_CONFIG_MODEL). */
fk_status fk_model_predict(fk_model *model, const fk_plan *plan, const fk_item *items, int32_t n,
                           fk_launch_config *out);
fk_status fk_plan_use_model(fk_plan *plan, fk_model *model, const fk_item *items, int32_t n);

/* Save / load: one JSON header line, then feature mean, feature std and
 * parameters as little-endian fp32. */
fk_status fk_model_save(const fk_model *model, const char *path);
fk_status fk_model_load(const char *path, fk_model **out);

/* ------------------------------------------------------------------------
 * Serving loop (not in the paper; its production use is the motivation of
 * Sections I and VII).  Requests -- one host frame with crops -- are admitted
 * first-in first-out against a device-memory budget; each admitted frame is
 * copied to the device on a copy stream and stays there until released; a
 * scheduler thread continuously batches the crops of every request whose
 * frame has arrived into horizontally fused launches (several in flight on
 * a compute stream), so requests arriving while others run join the next
 * launch.  Each crop's result depends only on its own pixels, so it is the
 * same alone and in any mix. */
typedef struct {
    int32_t x, y, w, h;  /* ROI in the request's frame */
    int32_t out_w, out_h;
} fk_crop;

typedef struct {
    const void *frame;   /* packed HWC of the chain's read dtype/channels, valid
                            until the request completes: host memory (pinned
                            memory gives an asynchronous copy), or device memory
                            when frame_on_device is 1 */
    int32_t width, height;
    int64_t pitch_bytes;
    const fk_crop *crops; /* copied by fk_server_submit */
    int32_t n_crops;      /* 1..max_batch_items */
    double t_arrival;     /* fk_server_clock() seconds; latency starts here */
    int32_t frame_on_device; /* 1: `frame` is already on the device (e.g. a
                                decoder's output): no copy, and the request's
                                budget block holds only its outputs (and the
                                unfused baseline's scratch) */
} fk_request;

#define FK_SERVER_BATCHED 0      /* continuous batching across requests */
#define FK_SERVER_PER_REQUEST 1  /* one fused launch per request, FIFO */
#define FK_SERVER_UNFUSED 2      /* one kernel per op per crop, FIFO */

typedef struct {
    const fk_chain_desc *chain;  /* read kind FK_READ_CROP_RESIZE; copied */
    void *arena;                 /* device memory for frames, outputs, scratch; caller-owned */
    int64_t arena_bytes;
    int64_t budget_bytes;        /* admission budget, 0 = arena_bytes */
    int32_t max_batch_items;     /* crops per launch (1..65536) */
    int32_t max_inflight;        /* launches in flight (1..4) */
    int32_t mode;                /* FK_SERVER_* */
    int32_t strict_fp;
    fk_launch_config config;     /* {0, 0}: the plan's default */
} fk_server_opts;

typedef struct {
    uint64_t ticket;
    int32_t status;              /* FK_OK, or the failure */
    int32_t n_crops;
    void *outputs;               /* device: crop i starts at the 256-byte aligned
                                    offset after crop i-1's output (dense, in the
                                    chain's write layout and dtype) */
    int64_t output_bytes;
    double t_arrival, t_admit, t_launch, t_done;  /* fk_server_clock() seconds */
} fk_completion;

typedef struct {
    int64_t submitted, admitted, completed, launches, crops_launched;
    int64_t bytes_in_use, peak_bytes;
    int64_t pending;             /* submitted, not yet admitted */
} fk_server_stats;

typedef struct fk_server fk_server;

/* Seconds on the monotonic clock used for every server timestamp. */
double fk_server_clock(void);

/* Start a server (creates its streams, plan and scheduler thread). */
fk_status fk_server_create(const fk_server_opts *opts, fk_server **out);

/* Queue a request; returns at once with its ticket.  FK_ERR_BUDGET if the
 * request alone exceeds the budget; FK_ERR_BAD_STATE after a device error or
 * while shutting down. */
fk_status fk_server_submit(fk_server *srv, const fk_request *req, uint64_t *ticket);

/* Up to `max` completions (oldest first) into `out`; their count in *n. */
fk_status fk_server_poll(fk_server *srv, fk_completion *out, int32_t max, int32_t *n);

/* Return a completed request's device memory to the budget.  Only a
 * ticket whose completion fk_server_poll has returned (and that was not
 * released before) is accepted; any other ticket -- unknown, released
 * before, or not yet returned by a poll (still queued, copying or
 * running) -- gives FK_ERR_BAD_STATE and changes nothing. */
fk_status fk_server_release(fk_server *srv, uint64_t ticket);

fk_status fk_server_stats_get(fk_server *srv, fk_server_stats *out);

/* Stop the scheduler after the work in flight, free everything the server
 * owns (not the arena).  NULL is allowed. */
fk_status fk_server_destroy(fk_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* FK_H */
