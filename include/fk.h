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
#define FK_ERR_UNSUPPORTED (-2)  /* valid request this build does not implement */
#define FK_ERR_OUT_OF_MEMORY (-3)
#define FK_ERR_HIP (-4)          /* a HIP runtime call failed; see fk_last_error() */
#define FK_ERR_BAD_STATE (-5)    /* call not allowed in the object's current state */
#define FK_ERR_BUDGET (-6)       /* request exceeds a memory budget */

/* Element types. */
#define FK_U8 0
#define FK_F16 1
#define FK_F32 2

/* Image layouts: packed HWC (out[(y*W + x)*C + c]) or planar CHW
 * (out[(c*H + y)*W + x]); Split is the packed-to-planar write op
 * (Section IV-B, the memory-ops figure). */
#define FK_PACKED 0
#define FK_PLANAR 1

/* Read operations (Section IV-B).
 * FK_READ_PLAIN: the item's region of interest read 1:1 (a crop when the
 *   ROI is smaller than the frame); output size = ROI size.
 * FK_READ_CROP_RESIZE: the ROI is bilinearly resized to the item's output
 *   size: half-pixel centres, no antialiasing, taps clamped to the ROI,
 *   source coordinate s = max(fma(o + 0.5, in/out, -0.5), 0) in fp32, lerps
 *   written as fma(a, p1 - p0, p0); the resized value stays fp32. */
#define FK_READ_PLAIN 0
#define FK_READ_CROP_RESIZE 1

/* Compute operations (Section IV-A; the hot chain of Sections VI-F/VI-J).
 * SWAP_RB: exchange channels 0 and 2 (BGR<->RGB), channel 3 kept, no-op for
 *   1 channel.  CVT_F32: convert to fp32 (exact from u8/f16; identity on
 *   fp32).  Arithmetic on a u8/f16 value promotes it to fp32 first.
 * MUL/ADD/SUB/DIV: one fp32 operation with a scalar (n_consts = 1) or
 *   per-channel (n_consts = channels) constant; per-channel constants index
 *   the channel position after earlier swaps.  DIV is an IEEE division. */
#define FK_OP_SWAP_RB 0
#define FK_OP_CVT_F32 1
#define FK_OP_MUL 2
#define FK_OP_ADD 3
#define FK_OP_SUB 4
#define FK_OP_DIV 5

#define FK_MAX_OPS 4096

typedef struct {
    int32_t kind;      /* FK_READ_* */
    int32_t in_dtype;  /* FK_U8, FK_F16, FK_F32 */
    int32_t channels;  /* 1, 3 or 4, packed in the source frame */
} fk_read_desc;

typedef struct {
    int32_t kind;      /* FK_OP_* */
    int32_t n_consts;  /* 0 for SWAP_RB/CVT_F32; 1 or `channels` otherwise */
    float consts[4];
} fk_op_desc;

typedef struct {
    int32_t out_dtype; /* FK_F32 or FK_F16 (round to nearest even) */
    int32_t layout;    /* FK_PACKED or FK_PLANAR */
} fk_write_desc;

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
 * element size; every row must be readable. */
typedef struct {
    const void *ptr;   /* device */
    int32_t width, height;
    int64_t pitch_bytes;
} fk_image;

/* One batch slot (one element of the BatchRead parameter array).  The ROI
 * (x, y, w, h) must lie inside `src`.  `dst` (device) receives out_w x
 * out_h x channels elements of the write dtype in the write layout,
 * densely (row pitch = out_w elements; planes of out_w*out_h).  For
 * FK_READ_PLAIN, out_w/out_h must be 0 or equal to w/h. */
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

#define FK_CONFIG_DEFAULT 0  /* 256 threads; coarsening 1, or 4 for chains of
                                more than 32 normalised ops */
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
} fk_plan_opts;

typedef struct fk_plan fk_plan;

/* Status text of a code, and the last error message on this thread. */
const char *fk_status_string(fk_status s);
const char *fk_last_error(void);

/* Library version and the device architecture this build targets. */
const char *fk_version(void);

/* Check a chain without touching the device.  FK_OK or FK_ERR_INVALID_ARG /
 * FK_ERR_UNSUPPORTED. */
fk_status fk_chain_validate(const fk_chain_desc *chain);

/* Check items against a chain without touching the device (host fields
 * only; device pointers are checked for null).  `n_items` may be 0. */
fk_status fk_items_validate(const fk_chain_desc *chain, const fk_item *items, int32_t n_items);

/* Create a plan for `chain` and up to `max_batch` items per run (the batch
 * capacity; each run passes its own count, Section IV-B).  `opts` may be
 * NULL (defaults).  Allocates the plan's device item tables (a small ring).
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
 * all `n_items` items (1 <= n_items <= max_batch).  `items` is copied
 * before the call returns. */
fk_status fk_run(fk_plan *plan, const fk_item *items, int32_t n_items, void *stream);

/* Bytes of device scratch fk_run_unfused needs for these items. */
fk_status fk_unfused_scratch_bytes(const fk_plan *plan, const fk_item *items, int32_t n_items,
                                   int64_t *bytes);

/* Unfused baseline (the separate-kernel pipeline of the kernel-call
 * algorithm, Section II): one kernel per operation and per item, every
 * intermediate materialised in `d_scratch` (device, caller-owned, at least
 * fk_unfused_scratch_bytes).  Same results as fk_run with strict_fp = 1. */
fk_status fk_run_unfused(fk_plan *plan, const fk_item *items, int32_t n_items, void *d_scratch,
                         int64_t scratch_bytes, void *stream);

/* Number of launch configurations the autotuner tries (20) and the i-th. */
int32_t fk_autotune_space(fk_launch_config *configs, int32_t max_configs);

/* Time every launch configuration on these items (median of `reps` timed
 * launches after warm-up, HIP events on an internal stream), write the 20
 * median times in milliseconds to `times_ms` (may be NULL), select the
 * fastest (ties: fewer threads, then less coarsening) into the plan and
 * `best` (may be NULL).  Synchronous; outputs are overwritten. */
fk_status fk_autotune(fk_plan *plan, const fk_item *items, int32_t n_items, int32_t reps,
                      float *times_ms, fk_launch_config *best);

#ifdef __cplusplus
}
#endif

#endif /* FK_H */
