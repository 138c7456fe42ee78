// fk_internal.hpp -- records shared by the host runtime and the kernels.
//
// The host turns a chain descriptor into these plain records once per plan
// (compute ops) and once per run (batch items); the kernels read them with
// uniform (scalar) loads.
#pragma once
#include <stdint.h>

namespace fk {

enum : int32_t {
    RD_PLAIN = 0,
    RD_CROP_RESIZE = 1,
    RD_CROP_NEAREST = 2,
    RD_NV12 = 3,
    RD_NV12_RESIZE = 4,
};
// read kinds with an output size of their own (not the ROI's)
constexpr bool rd_resizes(int rk) { return rk == RD_CROP_RESIZE || rk == RD_CROP_NEAREST || rk == RD_NV12_RESIZE; }
// read kinds whose kernels use the fp32 scales w/ow and h/oh
constexpr bool rd_bilinear(int rk) { return rk == RD_CROP_RESIZE || rk == RD_NV12_RESIZE; }
enum : int32_t { DT_U8 = 0, DT_F16 = 1, DT_F32 = 2, DT_F64 = 3 };
enum : int32_t { LY_PACKED = 0, LY_PLANAR = 1, LY_STATS = 2 };
// Kernel selection only: a planar write from pixel-strided lanes (bilinear
// reads on launches of at least kStridedMinPixels output pixels).
enum : int32_t { LY_PLANAR_PX = 3 };

// Normalised compute op codes.  SUB becomes ADD of the negated constant
// (IEEE x - y is x + (-y)), CVT disappears (fp32 from the read on), swaps
// move to the read, and in the contracted mode a MUL followed by ADD/SUB
// becomes FMA.  LOOP sends execution back over the `span` records before
// it until they have run `count` times.
enum : int32_t { OPC_MUL = 0, OPC_ADD = 1, OPC_DIV = 2, OPC_FMA = 3, OPC_LOOP = 4 };

constexpr int kUnitPx = 4;       // output pixels per unit: one 16-byte planar fp32 store
constexpr int kMaxBlock = 1024;  // largest block the kernels accept
constexpr int kWave = 64;        // CDNA wavefront

struct OpRec {          // 48 bytes
    int32_t code;
    int32_t span;       // LOOP: body records just before this one
    int32_t count;      // LOOP: runs of the body in all (>= 1)
    int32_t pad;
    float a[4];         // MUL/ADD/DIV constant per channel, or FMA multiplier
    float b[4];         // FMA addend per channel
};

// Item flags.
enum : int32_t {
    IF_SRC_VEC = 1,     // source rows 4-byte aligned: unit loads as dwords
    IF_DST_VEC = 2,     // output rows hold whole units and are 16/8-byte aligned
    IF_CONTIG = 4,      // plain read of whole frame rows stored back to back, whole
                        // units per row, under 2^31 pixels: unit u starts u * 4
                        // pixels after row y
    IF_SMALL_FRAME = 8, // frame below 4 GiB, rows below 16 MiB: 32-bit row offsets
};

struct ItemRec {        // 64 bytes: one batch slot's parameters
    uint64_t src;       // frame base address (device)
    uint64_t dst;       // output base address (device)
    int64_t pitch;      // frame row pitch in bytes
    int32_t x, y, w, h; // region of interest in the frame
    int32_t ow, oh;     // output size
    float sx, sy;       // crop+resize scales w/ow and h/oh (fp32)
    uint16_t fw, fh;    // frame size in pixels (bounds of window reads)
    int32_t flags;      // IF_*
};
static_assert(sizeof(ItemRec) == 64, "ItemRec layout");

struct RunHeader {      // per-run header read by the kernel (graph-friendly)
    int32_t n_items;
    uint32_t total_tiles;
    int32_t pad[2];
};

// Small batches ride in the kernel arguments instead of a device table:
//  - full:    ItemRec[inl_n] at inl[0..], uint32 tile_begin[inl_n + 1] at
//             inl[kInlineTileBegin..] (inl_n <= kInlineItems);
//  - compact: items sharing one frame, one output size and a constant
//             output stride: an ItemRec template at inl[0..64) (item 0) and
//             one Roi16 (x, y, w, h) per item at inl[64 + 8 b]
//             (inl_n <= kCompactItems); item b owns tiles
//             [b * inl_tiles_per_item, (b + 1) * inl_tiles_per_item).
#ifndef FK_INLINE_BYTES
#define FK_INLINE_BYTES 2560
#endif
constexpr int kInlineBytes = FK_INLINE_BYTES;
constexpr int kInlineItems = (kInlineBytes - 4) / 68 < 32 ? (kInlineBytes - 4) / 68 : 32;
constexpr int kInlineTileBegin = kInlineItems * 64;
constexpr int kCompactItems = (kInlineBytes - 64) / 8;  // 312

struct Roi16 {
    uint16_t x, y, w, h;
};

// Stats write: a block's partial result for one channel.
struct StatPartial {    // 16 bytes
    float mn, mx;
    double sum;
};

// Stats write: a batch slot's output is covered by at most kStatSlots
// blocks (each striding over the item's tiles); each leaves one partial per
// channel, and a second kernel combines each item's partials.
constexpr int kStatSlots = 512;
// Partials a stats plan holds (slots over a whole batch); a batch of n
// items gives each at most kStatCapacity / n slots, and at most the
// resident grid's blocks / n, so that each block walks several tiles.
constexpr int kStatCapacity = 65536;

// Kernel arguments (by value, the only kernel argument, so it starts the
// kernarg segment).  Device table layout of one run:
//   RunHeader | ItemRec[max_batch] | uint32 tile_begin[max_batch + 1]
struct KArgs {
    const RunHeader *hdr;
    const ItemRec *items;
    const uint32_t *tile_begin;
    const OpRec *ops;      // run-time tier op list (device), n_ops entries
    const float *consts;   // compile-time tier constants (device)
    int32_t n_ops;
    int32_t swap;          // net BGR<->RGB swap applied at the read
    int32_t strict;        // compile-time tier: 1 = no contraction
    int32_t loop_count;    // compile-time loop chain: pairs to run
    int32_t inl_n;         // > 0: the run's items are in `inl`
    int32_t inl_compact;   // 1: compact form
    uint32_t inl_total_tiles;
    uint32_t inl_tiles_per_item;  // compact form
    int64_t inl_dst_stride;       // compact form: bytes between item outputs
    StatPartial *st_part;  // stats write: one partial per (slot, channel)
    alignas(16) uint8_t inl[kInlineBytes];
};

// Kernel families.
enum : int32_t {
    FAM_RUNTIME = 0,       // any chain: run-time op list
    FAM_NORMALIZE = 1,     // crop+resize u8x3 -> swap,cvt,mul,sub,div -> planar f32
    FAM_MULADD = 2,        // plain u8x3 -> cvt, N x (mul, add) -> packed f32
    FAM_MULADD_LOOP = 3,   // plain u8/f32 x1/x3 -> [cvt,] mul, add, loop(2, P) -> packed f32
    FAM_F64 = 4,           // plain read -> run-time op list in fp64 -> fp64 packed/planar
};

// Kernel lookup (defined by the kernel translation units).  Returns the
// host-side kernel handle to pass to hipLaunchKernel, or nullptr if the
// combination is not built.
const void *kernel_runtime(int read_kind, int in_dt, int channels, int out_dt, int layout,
                           int coarsen);
// strided: pixel-strided lanes (launches of at least kStridedMinPixels
// output pixels), else 4-pixel units
const void *kernel_normalize(int coarsen, int strict, int strided);
constexpr uint64_t kStridedMinPixels = 1u << 20;
// crop+resize of a u8 frame with the tapped rows staged in LDS
const void *kernel_normalize_lds(int coarsen, int strict);
// LDS of a staged-row gather block of T threads (dynamic shared memory)
constexpr uint32_t lds_gather_bytes(uint32_t T) { return T * 128u < 65536u ? T * 128u : 65536u; }
const void *kernel_muladd(int n_ops, int coarsen, int strict);
// plain read of in_dt elements -> run-time op list in fp64 -> fp64 write
const void *kernel_f64(int in_dt, int channels, int layout, int coarsen);
const void *kernel_muladd_loop(int in_dt, int channels, int coarsen, int strict);
const void *kernel_loop_px(int in_dt, int channels, int coarsen, int strict);
// The compile-time loop chain runs per pixel (k_loop_px, a tile = T*K
// pixels) from this many pairs on; shorter loops keep the 4-pixel unit.
constexpr int kLoopPxMinPairs = 32;
const void *kernel_stats(int read_kind, int in_dt, int channels, int coarsen);
// stats write of a plain u8 read with no arithmetic after the cast
const void *kernel_stats_u8(int channels, int coarsen);
const void *kernel_stats_final(int channels);

}  // namespace fk
