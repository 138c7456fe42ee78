// fk_device.hpp -- device operations and the fused transform kernel.
//
// Structure (Section IV of the paper, re-designed for CDNA4):
//  - Read ops produce a register tile of fp32 pixels from device memory
//    using the thread's coordinates (Section IV-B, read operations).
//  - Compute ops transform the tile in registers (Section IV-A).  Two tiers:
//      * compile-time ops composed by C++17 templates (StaticChain below),
//        with a compile-time contraction rule fusing Mul+Add/Sub into one
//        FMA;
//      * a run-time op list (uniform, read with scalar loads) for chains
//        only known when a plan is created.
//  - Write ops store the tile (Section IV-B, write operations; Split is the
//    planar write).
//  - k_transform is the transform data-parallel pattern (Section IV-C): it
//    owns the thread behaviour -- batch-slot lookup (BatchRead), work
//    decomposition, thread coarsening -- and connects read -> compute ->
//    write without touching memory in between.
//
// Work decomposition: an item's output is cut into units of kUnitPx = 4
// consecutive pixels of one row.  A tile is blockDim.x * K units of one
// item; thread t handles units tile_base + j * blockDim.x + t (j < K), so
// every load/store instruction of a wave touches consecutive units, and
// takes them through its registers in groups small enough that the tile is
// never spilled (unit_group).  The grid strides over the tiles of all items
// (persistent horizontal fusion).
//
// Also here: k_resize_px, the same pattern with pixel-strided lanes for the
// bilinear gathers of large launches; k_loop_px, one pixel per lane for long
// compile-time loop chains; and the reduction pattern (k_stats, k_stats_u8,
// k_stats_final).
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>
#include <utility>

#include "fk_internal.hpp"

namespace fk {

// Read-only tables live in the constant address space so that uniform
// accesses become scalar loads through the scalar cache.
#define FK_CONST __attribute__((address_space(4)))

template <typename T>
__device__ __forceinline__ const FK_CONST T *cptr(const T *p)
{
    return (const FK_CONST T *)p;
}

// Frames and outputs are global memory: explicit global pointers give
// global_load/global_store instead of flat accesses.
#define FK_GLOBAL __attribute__((address_space(1)))
typedef const FK_GLOBAL uint8_t *gsrc_t;
typedef FK_GLOBAL uint8_t *gdst_t;

// Native vector types (usable through address-space qualified pointers).
typedef float fx4 __attribute__((ext_vector_type(4)));
typedef uint32_t ux4 __attribute__((ext_vector_type(4)));
typedef uint32_t ux2 __attribute__((ext_vector_type(2)));

template <int DT>
struct DSize;
template <>
struct DSize<DT_U8> { static constexpr int v = 1; };
template <>
struct DSize<DT_F16> { static constexpr int v = 2; };
template <>
struct DSize<DT_F32> { static constexpr int v = 4; };
template <>
struct DSize<DT_F64> { static constexpr int v = 8; };

// ------------------------------------------------------------ elements --

template <int DT>
__device__ __forceinline__ float load_elem(gsrc_t p);
template <>
__device__ __forceinline__ float load_elem<DT_U8>(gsrc_t p)
{
    return (float)(*p);
}
template <>
__device__ __forceinline__ float load_elem<DT_F16>(gsrc_t p)
{
    return (float)(*(const FK_GLOBAL _Float16 *)p);
}
template <>
__device__ __forceinline__ float load_elem<DT_F32>(gsrc_t p)
{
    return *(const FK_GLOBAL float *)p;
}

// Element i of a dword array holding packed elements of type DT.
template <int DT, int NW>
__device__ __forceinline__ float unpack_elem(const uint32_t (&w)[NW], int i)
{
    if constexpr (DT == DT_U8) {
        return (float)((w[i >> 2] >> (8 * (i & 3))) & 0xffu);
    } else if constexpr (DT == DT_F16) {
        uint16_t h = (uint16_t)(w[i >> 1] >> (16 * (i & 1)));
        return (float)__builtin_bit_cast(_Float16, h);
    } else {
        return __builtin_bit_cast(float, w[i]);
    }
}

// Outputs are written once and never read back by the kernel: nontemporal
// stores keep them from displacing the streamed input in the caches (a
// measured ~1.3x on the 1:4 read:write expansion of u8 -> fp32).
template <typename V>
__device__ __forceinline__ void store_nt(gdst_t p, V v)
{
    __builtin_nontemporal_store(v, (FK_GLOBAL V *)p);
}

// Dwords of a streamed input that only a reduction reads: nontemporal
// loads (measured on the u8 statistics of 16 4K frames: 67.5-69.0 us
// against 75.9-76.7 us with ordinary loads).  The transform's plain read
// keeps ordinary loads: on frames already in the Infinity Cache they hit
// there (18.9 us against 22.2 us per 4K launch), from HBM the two are even.
__device__ __forceinline__ uint32_t load_stream(const FK_GLOBAL uint32_t *p)
{
    return __builtin_nontemporal_load(p);
}

template <int DT>
__device__ __forceinline__ void store_elem(gdst_t p, float v);
template <>
__device__ __forceinline__ void store_elem<DT_F32>(gdst_t p, float v)
{
    store_nt(p, v);
}
template <>
__device__ __forceinline__ void store_elem<DT_F16>(gdst_t p, float v)
{
    store_nt(p, (_Float16)v);  // round to nearest even
}

// ---------------------------------------------------------- read ops --

// Plain read: the ROI 1:1.  Loads one unit (4 pixels) of output row oy
// starting at column ox0; returns the number of valid pixels.
template <int DT, int C>
struct ReadPlain {
    static constexpr int kind = RD_PLAIN;
    static constexpr int dtype = DT;
    static constexpr int elem_size = DSize<DT>::v;
    __device__ __forceinline__ static void load(const ItemRec &it, int oy, int ox0, int n,
                                                float (&r)[kUnitPx][C])
    {
        constexpr int ES = DSize<DT>::v;
        gsrc_t row = (gsrc_t)it.src + (int64_t)(it.y + oy) * it.pitch +
                     (int64_t)(it.x + ox0) * (C * ES);
        if (n == kUnitPx && (it.flags & IF_SRC_VEC)) {
            constexpr int NW = kUnitPx * C * ES / 4;
            uint32_t w[NW];
            const FK_GLOBAL uint32_t *p = (const FK_GLOBAL uint32_t *)row;
#pragma unroll
            for (int i = 0; i < NW; ++i)
                w[i] = p[i];
#pragma unroll
            for (int i = 0; i < kUnitPx; ++i)
#pragma unroll
                for (int c = 0; c < C; ++c)
                    r[i][c] = unpack_elem<DT, NW>(w, i * C + c);
        } else {
#pragma unroll
            for (int i = 0; i < kUnitPx; ++i)
#pragma unroll
                for (int c = 0; c < C; ++c)
                    r[i][c] = i < n ? load_elem<DT>(row + (i * C + c) * ES) : 0.0f;
        }
    }
};

// Half-pixel source coordinate of output index o, clamped below at 0, with
// its two taps (clamped to the ROI) and the fractional weight.
__device__ __forceinline__ void bilinear_coord(int o, float scale, int in_size, int &i0, int &i1,
                                               float &a)
{
    float s = fmaf((float)o + 0.5f, scale, -0.5f);
    s = s < 0.0f ? 0.0f : s;
    int lo = (int)floorf(s);
    lo = lo > in_size - 1 ? in_size - 1 : lo;
    i0 = lo;
    i1 = lo + 1 < in_size ? lo + 1 : in_size - 1;
    a = s - (float)lo;
}

// Crop + bilinear resize: the ROI resized to (ow, oh).
//
// u8 frames: each tap row of a pixel (its two neighbouring source pixels,
// 2C bytes) is fetched as one dword-aligned window of WB bytes and the bytes
// are picked out with v_alignbyte -- one load instead of 2C byte loads.  A
// window may extend up to WB - 1 bytes past the last tapped pixel and 3
// bytes before the first, so it is used only when the frame base is dword
// aligned, a frame row holds at least WB bytes, and either the ROI stops
// above the frame's last row or its last window still ends inside that
// row.  Other items, and fp16/fp32 frames, load element by element.
template <int DT, int C>
struct ReadCropResize {
    static constexpr int kind = RD_CROP_RESIZE;
    static constexpr int elem_size = DSize<DT>::v;
    static constexpr int WB = (C == 1) ? 8 : 12;  // window bytes

    __device__ __forceinline__ static bool window_ok(const ItemRec &it)
    {
        if constexpr (DT != DT_U8) {
            return false;
        } else {
            // the overrun past a row's last pixel stays inside the row, or
            // inside the next row (which holds at least WB bytes)
            return (it.src % 4 == 0) && C * (int)it.fw >= WB &&
                   (it.y + it.h < (int)it.fh || C * (it.x + it.w - 1) + WB <= C * (int)it.fw);
        }
    }

    // bytes [0, 2C) of the tap pair starting at absolute address `addr`
    __device__ __forceinline__ static void window(uint64_t addr, uint32_t (&d)[2])
    {
        const FK_GLOBAL uint32_t *p = (const FK_GLOBAL uint32_t *)(addr & ~(uint64_t)3);
        const uint32_t sh = (uint32_t)(addr & 3);
        if constexpr (WB == 8) {
            const uint32_t w0 = p[0], w1 = p[1];
            d[0] = __builtin_amdgcn_alignbyte(w1, w0, sh);
            d[1] = 0;
        } else {
            const uint32_t w0 = p[0], w1 = p[1], w2 = p[2];
            d[0] = __builtin_amdgcn_alignbyte(w1, w0, sh);
            d[1] = __builtin_amdgcn_alignbyte(w2, w1, sh);
        }
    }

    __device__ __forceinline__ static float byte_at(const uint32_t (&d)[2], int k)
    {
        return (float)((d[k >> 2] >> (8 * (k & 3))) & 0xffu);
    }

    // one output pixel from its source rows r0, r1 (ROI-relative column 0)
    // and its output column ox
    __device__ __forceinline__ static void pixel(const ItemRec &it, gsrc_t r0, gsrc_t r1, float ay,
                                                 int ox, bool win, float (&r)[C])
    {
        constexpr int ES = DSize<DT>::v;
        int x0, x1;
        float ax;
        bilinear_coord(ox, it.sx, it.w, x0, x1, ax);
        if (DT == DT_U8 && win) {
            uint32_t t[2], b[2];
            window((uint64_t)(uintptr_t)(r0 + x0 * C), t);
            window((uint64_t)(uintptr_t)(r1 + x0 * C), b);
            lerp_windows(t, b, x1 == x0, ax, ay, r);
            return;
        }
        float p00[C], p01[C], p10[C], p11[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            p00[c] = load_elem<DT>(r0 + (x0 * C + c) * ES);
            p01[c] = load_elem<DT>(r0 + (x1 * C + c) * ES);
            p10[c] = load_elem<DT>(r1 + (x0 * C + c) * ES);
            p11[c] = load_elem<DT>(r1 + (x1 * C + c) * ES);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float top = fmaf(ax, p01[c] - p00[c], p00[c]);
            const float bot = fmaf(ax, p11[c] - p10[c], p10[c]);
            r[c] = fmaf(ay, bot - top, top);
        }
    }

    // the pixel from the byte windows of its top and bottom tap rows (tap
    // pair at bytes [0, 2C), or one pixel at [0, C) when the right tap is
    // clamped onto the left one)
    __device__ __forceinline__ static void lerp_windows(const uint32_t (&t)[2], const uint32_t (&b)[2],
                                                        bool clamped, float ax, float ay, float (&r)[C])
    {
        const int o1 = clamped ? 0 : C;
        float p00[C], p01[C], p10[C], p11[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
            p00[c] = byte_at(t, c);
            p01[c] = byte_at(t, o1 + c);
            p10[c] = byte_at(b, c);
            p11[c] = byte_at(b, o1 + c);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float top = fmaf(ax, p01[c] - p00[c], p00[c]);
            const float bot = fmaf(ax, p11[c] - p10[c], p10[c]);
            r[c] = fmaf(ay, bot - top, top);
        }
    }

    // source rows of output row oy, and the vertical weight.  A frame
    // below 4 GiB with rows under 16 MiB (IF_SMALL_FRAME) takes 32-bit
    // offsets from full-rate 24-bit multiplies.
    __device__ __forceinline__ static void rows(const ItemRec &it, int oy, gsrc_t &r0, gsrc_t &r1,
                                                float &ay)
    {
        constexpr int ES = DSize<DT>::v;
        int y0, y1;
        bilinear_coord(oy, it.sy, it.h, y0, y1, ay);
        gsrc_t base = (gsrc_t)it.src + (int64_t)it.x * (C * ES);
        if (it.flags & IF_SMALL_FRAME) {
            r0 = base + __umul24((uint32_t)(it.y + y0), (uint32_t)it.pitch);
            r1 = base + __umul24((uint32_t)(it.y + y1), (uint32_t)it.pitch);
        } else {
            r0 = base + (int64_t)(it.y + y0) * it.pitch;
            r1 = base + (int64_t)(it.y + y1) * it.pitch;
        }
    }

    // one output pixel on its own (pixel-strided lanes); prep = window_ok
    __device__ __forceinline__ static bool px_prep(const ItemRec &it) { return window_ok(it); }
    __device__ __forceinline__ static void load_px(const ItemRec &it, bool win, int oy, int ox,
                                                   float (&r)[C])
    {
        gsrc_t r0, r1;
        float ay;
        rows(it, oy, r0, r1, ay);
        pixel(it, r0, r1, ay, ox, win, r);
    }

    __device__ __forceinline__ static void load(const ItemRec &it, int oy, int ox0, int n,
                                                float (&r)[kUnitPx][C])
    {
        gsrc_t r0, r1;
        float ay;
        rows(it, oy, r0, r1, ay);
        const bool win = window_ok(it);
#pragma unroll
        for (int i = 0; i < kUnitPx; ++i) {
            if (i < n) {
                pixel(it, r0, r1, ay, ox0 + i, win, r[i]);
            } else {
#pragma unroll
                for (int c = 0; c < C; ++c)
                    r[i][c] = 0.0f;
            }
        }
    }
};

// Nearest-neighbour crop+resize: output index o takes ROI index
// floor((2o + 1) * in / (2 out)).  The quotient comes from an fp32
// estimate (off by at most one: the quotient is below 2^16 and the estimate
// carries three roundings of 2^-24) corrected by exact integer products.
__device__ __forceinline__ int nearest_index(int o, int in, int out)
{
    const uint64_t num = (uint64_t)(2 * o + 1) * (uint64_t)in;
    const uint64_t den = 2ull * (uint64_t)out;
    int q = (int)((float)num * (1.0f / (float)den));
    if ((uint64_t)q * den > num)
        --q;
    else if ((uint64_t)(q + 1) * den <= num)
        ++q;
    return q;
}

template <int DT, int C>
struct ReadCropNearest {
    static constexpr int kind = RD_CROP_NEAREST;
    static constexpr int elem_size = DSize<DT>::v;

    // the ROI row holding output row oy's source pixels
    __device__ __forceinline__ static gsrc_t row_of(const ItemRec &it, int oy)
    {
        constexpr int ES = DSize<DT>::v;
        const int sy = nearest_index(oy, it.h, it.oh);
        return (gsrc_t)it.src + (int64_t)(it.y + sy) * it.pitch + (int64_t)it.x * (C * ES);
    }
    // u8 pixels of 3 or 4 channels come out of one dword-aligned 8-byte
    // window (two dword loads, the bytes picked with v_alignbyte) in place
    // of C byte loads, where the crop+resize read's rule keeps its (wider)
    // windows inside the frame's allocation
    __device__ __forceinline__ static bool window_ok(const ItemRec &it)
    {
        if constexpr (DT == DT_U8 && C >= 3)
            return ReadCropResize<DT_U8, C>::window_ok(it);
        else
            return false;
    }
    __device__ __forceinline__ static void pixel(const ItemRec &it, gsrc_t row, int ox, bool win,
                                                 float (&r)[C])
    {
        constexpr int ES = DSize<DT>::v;
        const int sx = nearest_index(ox, it.w, it.ow);
        if constexpr (DT == DT_U8 && C >= 3) {
            if (win) {
                const uint64_t a = (uint64_t)(uintptr_t)(row + sx * C);
                const FK_GLOBAL uint32_t *p = (const FK_GLOBAL uint32_t *)(a & ~(uint64_t)3);
                const uint32_t d = __builtin_amdgcn_alignbyte(p[1], p[0], (uint32_t)(a & 3));
#pragma unroll
                for (int c = 0; c < C; ++c)
                    r[c] = (float)((d >> (8 * c)) & 0xffu);
                return;
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c)
            r[c] = load_elem<DT>(row + (sx * C + c) * ES);
    }
    __device__ __forceinline__ static bool px_prep(const ItemRec &it) { return window_ok(it); }
    __device__ __forceinline__ static void load_px(const ItemRec &it, bool win, int oy, int ox, float (&r)[C])
    {
        pixel(it, row_of(it, oy), ox, win, r);
    }

    __device__ __forceinline__ static void load(const ItemRec &it, int oy, int ox0, int n,
                                                float (&r)[kUnitPx][C])
    {
        gsrc_t row = row_of(it, oy);
        const bool win = window_ok(it);
#pragma unroll
        for (int i = 0; i < kUnitPx; ++i) {
            if (i < n) {
                pixel(it, row, ox0 + i, win, r[i]);
            } else {
#pragma unroll
                for (int c = 0; c < C; ++c)
                    r[i][c] = 0.0f;
            }
        }
    }
};

// NV12 (BT.601 limited range) -> B, G, R in fp32, one IEEE operation per
// product and sum in a fixed order (compiled without contraction).
__device__ __forceinline__ void nv12_to_bgr(float Y, float U, float V, float (&o)[3])
{
    const float u = U - 128.0f;
    const float v = V - 128.0f;
    const float c = 1.164f * (Y - 16.0f);
    o[0] = c + 2.018f * u;
    o[1] = (c - 0.813f * v) - 0.391f * u;
    o[2] = c + 1.596f * v;
}

// Pixel (x, y) of an NV12 frame (absolute luma coordinates): the luma byte
// and the chroma pair serving its 2x2 block; the chroma plane starts
// `fh` rows (the luma height) below the frame base, at the same pitch.
__device__ __forceinline__ void nv12_pixel(const ItemRec &it, int x, int y, float (&o)[3])
{
    gsrc_t base = (gsrc_t)it.src;
    const float Y = load_elem<DT_U8>(base + (int64_t)y * it.pitch + x);
    gsrc_t uv = base + ((int64_t)it.fh + (y >> 1)) * it.pitch + (x & ~1);
    nv12_to_bgr(Y, load_elem<DT_U8>(uv), load_elem<DT_U8>(uv + 1), o);
}

// NV12 crop read 1:1 (three output channels).
template <int C>
struct ReadNV12 {
    static_assert(C == 3, "NV12 reads give three channels");
    static constexpr int kind = RD_NV12;
    static constexpr int elem_size = 1;

    __device__ __forceinline__ static bool px_prep(const ItemRec &) { return false; }
    __device__ __forceinline__ static void load_px(const ItemRec &it, bool, int oy, int ox, float (&r)[C])
    {
        nv12_pixel(it, it.x + ox, it.y + oy, r);
    }

    // A whole unit of a frame whose base, pitch and ROI column are
    // multiples of 4 (IF_SRC_VEC) reads its 4 luma bytes and the 2 chroma
    // pairs serving them as one dword each; otherwise byte by byte.
    __device__ __forceinline__ static void load(const ItemRec &it, int oy, int ox0, int n,
                                                float (&r)[kUnitPx][C])
    {
        if (n == kUnitPx && (it.flags & IF_SRC_VEC)) {
            gsrc_t base = (gsrc_t)it.src;
            const int x = it.x + ox0;
            const int y = it.y + oy;
            const uint32_t yw = *(const FK_GLOBAL uint32_t *)(base + (int64_t)y * it.pitch + x);
            const uint32_t cw =
                *(const FK_GLOBAL uint32_t *)(base + ((int64_t)it.fh + (y >> 1)) * it.pitch + x);
#pragma unroll
            for (int i = 0; i < kUnitPx; ++i) {
                const int k = i & ~1;  // the chroma pair of pixel i
                nv12_to_bgr((float)((yw >> (8 * i)) & 0xffu), (float)((cw >> (8 * k)) & 0xffu),
                            (float)((cw >> (8 * k + 8)) & 0xffu), r[i]);
            }
            return;
        }
#pragma unroll
        for (int i = 0; i < kUnitPx; ++i) {
            if (i < n) {
                nv12_pixel(it, it.x + ox0 + i, it.y + oy, r[i]);
            } else {
#pragma unroll
                for (int c = 0; c < C; ++c)
                    r[i][c] = 0.0f;
            }
        }
    }
};

// NV12 crop + bilinear resize of the converted values (taps converted,
// then the same lerps as the u8/f16/f32 resize).
template <int C>
struct ReadNV12Resize {
    static_assert(C == 3, "NV12 reads give three channels");
    static constexpr int kind = RD_NV12_RESIZE;
    static constexpr int elem_size = 1;

    // Windows: in a frame whose base is a multiple of 4 and whose rows hold
    // at least 8 bytes, a tap row's two luma bytes come from one
    // dword-aligned 8-byte window and the chroma pairs serving them from
    // another (two dword loads each, bytes picked with v_alignbyte) in place
    // of six byte loads.  A window reads up to 3 bytes before and 7 after
    // its first byte: a luma window past its row runs into the next luma
    // row or the chroma plane, so only a chroma window on the last chroma
    // row must be kept inside the row's pixels.
    __device__ __forceinline__ static bool window_ok(const ItemRec &it)
    {
        if ((it.src & 3u) || (int)it.fw < 8)
            return false;
        const int last_y = it.y + it.h - 1;
        const bool last_chroma_row = (last_y >> 1) == ((int)it.fh >> 1) - 1;
        return !last_chroma_row || ((it.x + it.w - 1) & ~1) + 8 <= (int)it.fw;
    }

    // the taps at absolute columns X0 and X1 = X0 or X0 + 1 of absolute
    // source row Y, from a luma and a chroma window
    __device__ __forceinline__ static void row_taps(const ItemRec &it, int Y, int X0, int X1, float (&a)[3],
                                                    float (&b)[3])
    {
        gsrc_t base = (gsrc_t)it.src;
        const uint64_t la = (uint64_t)(uintptr_t)(base + (int64_t)Y * it.pitch + X0);
        const FK_GLOBAL uint32_t *lp = (const FK_GLOBAL uint32_t *)(la & ~(uint64_t)3);
        const uint32_t lw = __builtin_amdgcn_alignbyte(lp[1], lp[0], (uint32_t)(la & 3));
        const int c0 = X0 & ~1;
        const uint64_t ca = (uint64_t)(uintptr_t)(base + ((int64_t)it.fh + (Y >> 1)) * it.pitch + c0);
        const FK_GLOBAL uint32_t *cp = (const FK_GLOBAL uint32_t *)(ca & ~(uint64_t)3);
        const uint32_t cw = __builtin_amdgcn_alignbyte(cp[1], cp[0], (uint32_t)(ca & 3));
        const int dl = X1 - X0;          // 0 or 1
        const int dc = (X1 & ~1) - c0;   // 0 or 2
        nv12_to_bgr((float)(lw & 0xffu), (float)(cw & 0xffu), (float)((cw >> 8) & 0xffu), a);
        nv12_to_bgr((float)((lw >> (8 * dl)) & 0xffu), (float)((cw >> (8 * dc)) & 0xffu),
                    (float)((cw >> (8 * dc + 8)) & 0xffu), b);
    }

    // output column ox of the output row whose source rows are y0, y1
    __device__ __forceinline__ static void pixel(const ItemRec &it, int y0, int y1, float ay, int ox, bool win,
                                                 float (&r)[C])
    {
        int x0, x1;
        float ax;
        bilinear_coord(ox, it.sx, it.w, x0, x1, ax);
        float p00[3], p01[3], p10[3], p11[3];
        if (win) {
            row_taps(it, it.y + y0, it.x + x0, it.x + x1, p00, p01);
            row_taps(it, it.y + y1, it.x + x0, it.x + x1, p10, p11);
        } else {
            nv12_pixel(it, it.x + x0, it.y + y0, p00);
            nv12_pixel(it, it.x + x1, it.y + y0, p01);
            nv12_pixel(it, it.x + x0, it.y + y1, p10);
            nv12_pixel(it, it.x + x1, it.y + y1, p11);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float top = fmaf(ax, p01[c] - p00[c], p00[c]);
            const float bot = fmaf(ax, p11[c] - p10[c], p10[c]);
            r[c] = fmaf(ay, bot - top, top);
        }
    }
    __device__ __forceinline__ static bool px_prep(const ItemRec &it) { return window_ok(it); }
    __device__ __forceinline__ static void load_px(const ItemRec &it, bool win, int oy, int ox, float (&r)[C])
    {
        int y0, y1;
        float ay;
        bilinear_coord(oy, it.sy, it.h, y0, y1, ay);
        pixel(it, y0, y1, ay, ox, win, r);
    }

    __device__ __forceinline__ static void load(const ItemRec &it, int oy, int ox0, int n,
                                                float (&r)[kUnitPx][C])
    {
        int y0, y1;
        float ay;
        bilinear_coord(oy, it.sy, it.h, y0, y1, ay);
        const bool win = window_ok(it);
#pragma unroll
        for (int i = 0; i < kUnitPx; ++i) {
            if (i < n) {
                pixel(it, y0, y1, ay, ox0 + i, win, r[i]);
            } else {
#pragma unroll
                for (int c = 0; c < C; ++c)
                    r[i][c] = 0.0f;
            }
        }
    }
};

// ------------------------------------------------- compile-time ops --
// Storage-less op types with a static exec on one pixel (a C-vector in
// registers); binary ops take their constants from the plan's constant
// table at a compile-time slot (Section IV-A: unary and binary operation
// types; instantiable ops carry the parameters).

struct OpSwapRB {
    template <int C>
    __device__ __forceinline__ static void exec(float (&px)[C], const FK_CONST float *)
    {
        if constexpr (C >= 3) {
            float t = px[0];
            px[0] = px[2];
            px[2] = t;
        }
    }
};

struct OpCvtF32 {  // values are fp32 from the read on: nothing to do
    template <int C>
    __device__ __forceinline__ static void exec(float (&)[C], const FK_CONST float *) {}
};

// Per-channel constants at slot S (S .. S+C-1); PerCh = false: one scalar.
template <int S, bool PerCh>
struct OpMul {
    template <int C>
    __device__ __forceinline__ static void exec(float (&px)[C], const FK_CONST float *k)
    {
#pragma unroll
        for (int c = 0; c < C; ++c)
            px[c] = px[c] * k[PerCh ? S + c : S];
    }
};
template <int S, bool PerCh>
struct OpAdd {
    template <int C>
    __device__ __forceinline__ static void exec(float (&px)[C], const FK_CONST float *k)
    {
#pragma unroll
        for (int c = 0; c < C; ++c)
            px[c] = px[c] + k[PerCh ? S + c : S];
    }
};
template <int S, bool PerCh>
struct OpSub {
    template <int C>
    __device__ __forceinline__ static void exec(float (&px)[C], const FK_CONST float *k)
    {
#pragma unroll
        for (int c = 0; c < C; ++c)
            px[c] = px[c] - k[PerCh ? S + c : S];
    }
};
template <int S, bool PerCh>
struct OpDiv {
    template <int C>
    __device__ __forceinline__ static void exec(float (&px)[C], const FK_CONST float *k)
    {
#pragma unroll
        for (int c = 0; c < C; ++c)
            px[c] = px[c] / k[PerCh ? S + c : S];
    }
};
// Contracted Mul followed by Add (Neg = false) or Sub (Neg = true).
template <int S1, bool P1, int S2, bool P2, bool Neg>
struct OpMulAddFused {
    template <int C>
    __device__ __forceinline__ static void exec(float (&px)[C], const FK_CONST float *k)
    {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const float m = k[P1 ? S1 + c : S1];
            const float a = k[P2 ? S2 + c : S2];
            px[c] = fmaf(px[c], m, Neg ? -a : a);
        }
    }
};

// Ops apply to a thread's whole register tile, op by op.  A plain op is
// defined on one pixel and applied to every pixel of the tile; a tile op
// (tile_op = true) owns the loop itself.
template <class Op, class = void>
struct IsTileOp : std::false_type {};
template <class Op>
struct IsTileOp<Op, std::void_t<decltype(Op::tile_op)>> : std::true_type {};

template <class Op, int K, int C>
__device__ __forceinline__ void run_on_tile(float (&v)[K][kUnitPx][C], const FK_CONST float *k)
{
    if constexpr (IsTileOp<Op>::value) {
        Op::template exec_tile<K, C>(v, k);
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int i = 0; i < kUnitPx; ++i)
                Op::exec(v[j][i], k);
    }
}

template <class... Ops>
struct StaticChain {
    template <int K, int C>
    __device__ __forceinline__ static void exec_tile(float (&v)[K][kUnitPx][C],
                                                     const FK_CONST float *k)
    {
        (run_on_tile<Ops, K, C>(v, k), ...);
    }
};

// StaticLoop: one Mul+Add op pair repeated NPAIRS times inside the kernel,
// pair p taking its constants from slots S + 2p and S + 2p + 1 -- the
// paper's StaticLoop op (Section VI-B), which repeats an op without
// spending kernel-parameter space or instruction space per repetition.  A
// loop (partly unrolled) keeps the scalar registers bounded for long
// chains, where full unrolling would hoist every constant at once.
template <int S, int NPAIRS, bool Strict>
struct OpMulAddLoop {
    static constexpr bool tile_op = true;
    template <int K, int C>
    __device__ __forceinline__ static void exec_tile(float (&v)[K][kUnitPx][C],
                                                     const FK_CONST float *k)
    {
#pragma unroll 4
        for (int p = 0; p < NPAIRS; ++p) {
            const float m = k[S + 2 * p];
            const float a = k[S + 2 * p + 1];
#pragma unroll
            for (int j = 0; j < K; ++j)
#pragma unroll
                for (int i = 0; i < kUnitPx; ++i)
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        if constexpr (Strict) {
                            const float t = v[j][i][c] * m;
                            v[j][i][c] = t + a;
                        } else {
                            v[j][i][c] = fmaf(v[j][i][c], m, a);
                        }
                    }
        }
    }
};

// Compile-time contraction: rewrite the op list so that every Mul directly
// followed by an Add or Sub becomes one fused multiply-add.
template <class... T>
struct TypeList {};

template <class Done, class Rest>
struct Contract;
template <class... D>
struct Contract<TypeList<D...>, TypeList<>> {
    using type = StaticChain<D...>;
};
template <class... D, class H, class... R>
struct Contract<TypeList<D...>, TypeList<H, R...>> {
    using type = typename Contract<TypeList<D..., H>, TypeList<R...>>::type;
};
template <class... D, int S1, bool P1, int S2, bool P2, class... R>
struct Contract<TypeList<D...>, TypeList<OpMul<S1, P1>, OpAdd<S2, P2>, R...>> {
    using type = typename Contract<TypeList<D..., OpMulAddFused<S1, P1, S2, P2, false>>,
                                   TypeList<R...>>::type;
};
template <class... D, int S1, bool P1, int S2, bool P2, class... R>
struct Contract<TypeList<D...>, TypeList<OpMul<S1, P1>, OpSub<S2, P2>, R...>> {
    using type = typename Contract<TypeList<D..., OpMulAddFused<S1, P1, S2, P2, true>>,
                                   TypeList<R...>>::type;
};

template <bool Strict, class... Ops>
struct Compose {
    using type = typename std::conditional<
        Strict, StaticChain<Ops...>,
        typename Contract<TypeList<>, TypeList<Ops...>>::type>::type;
};

// The hot normalise chain: swap, cvt, *k, -mean, /std.  Constant table:
// [k, mean0..2, std0..2].
template <bool Strict>
using NormalizeChain = typename Compose<Strict, OpSwapRB, OpCvtF32, OpMul<0, false>,
                                        OpSub<1, true>, OpDiv<4, true>>::type;

// cvt then N alternating Mul (even op) / Add (odd op), scalar constants in
// op order at slots 0..N-1.
template <size_t I>
using MulOrAdd = typename std::conditional<(I % 2 == 0), OpMul<(int)I, false>,
                                           OpAdd<(int)I, false>>::type;
template <bool Strict, class Seq>
struct MulAddSeq;
template <bool Strict, size_t... I>
struct MulAddSeq<Strict, std::index_sequence<I...>> {
    using type = typename Compose<Strict, OpCvtF32, MulOrAdd<I>...>::type;
};
template <int N, bool Strict>
using MulAddChain = typename std::conditional<
    (N <= 16), typename MulAddSeq<Strict, std::make_index_sequence<N>>::type,
    StaticChain<OpCvtF32, OpMulAddLoop<0, N / 2, Strict>>>::type;
static_assert(IsTileOp<OpMulAddLoop<0, 2, true>>::value && !IsTileOp<OpCvtF32>::value, "");

// Compute stage over a thread's whole register tile.
template <class Chain>
struct StaticCompute {
    template <int K, int C>
    __device__ __forceinline__ static void apply(const KArgs &a, float (&v)[K][kUnitPx][C])
    {
        Chain::template exec_tile<K, C>(v, cptr(a.consts));
    }
};

// A uniform value held in a VGPR.  A VOP3 instruction reads at most one
// SGPR on this architecture, so an FMA with two uniform operands needs one
// of them in a VGPR; left to itself the compiler re-copies it inside hot
// loops.
__device__ __forceinline__ float in_vgpr(float x)
{
    float r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
    return r;
}

// Compile-time loop chain: one Mul and one Add (scalar constants, loaded
// once) applied loop_count times; the body is compiled, the trip count is
// a kernel argument, so code size does not grow with the count.
template <bool Strict>
struct LoopMulAddCompute {
    template <int K, int C>
    __device__ __forceinline__ static void apply(const KArgs &a, float (&v)[K][kUnitPx][C])
    {
        const FK_CONST float *k = cptr(a.consts);
        const float m = k[0];
        const float ad = in_vgpr(k[1]);
        const int n = a.loop_count;
#pragma unroll 32
        for (int p = 0; p < n; ++p) {
#pragma unroll
            for (int j = 0; j < K; ++j)
#pragma unroll
                for (int i = 0; i < kUnitPx; ++i)
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        if constexpr (Strict) {
                            const float t = v[j][i][c] * m;
                            v[j][i][c] = t + ad;
                        } else {
                            v[j][i][c] = fmaf(v[j][i][c], m, ad);
                        }
                    }
        }
    }
};

// ------------------------------------------------------ run-time ops --
// The op list is uniform across the grid: each op is one scalar branch and
// its constants come through the scalar cache, then applied to all values
// the thread holds (a register group of its units).  A LOOP record over one record
// makes that record run `count` times in a register loop; a longer LOOP
// jumps back over its body until the body has run `count` times (bodies
// hold no loops, so one counter serves every loop of the list).
// fused multiply-add in the running value's precision
__device__ __forceinline__ float fma_v(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_v(double a, double b, double c) { return fma(a, b, c); }

// The run-time op list on fp32 values, or on fp64 values for a chain with
// an fp64 write (the op's fp32 constants taken exactly).
struct RuntimeCompute {
    template <int K, int C, typename V, int P>
    __device__ __forceinline__ static void apply(const KArgs &a, V (&v)[K][P][C])
    {
        const FK_CONST OpRec *ops = cptr(a.ops);
        int runs = 1;  // runs of the current loop body so far
        for (int o = 0; o < a.n_ops; ++o) {
            const int code = ops[o].code;
            if (code == OPC_LOOP) {
                if (ops[o].span == 1)
                    continue;  // already run by its one-record body, below
                if (runs < ops[o].count) {
                    ++runs;
                    o -= ops[o].span + 1;  // the loop's ++o lands on the body's first record
                } else {
                    runs = 1;
                }
                continue;
            }
            // a record followed by a one-record LOOP runs `count` times here,
            // in a register loop with its constants loaded once
            int reps = 1;
            if (o + 1 < a.n_ops && ops[o + 1].code == OPC_LOOP && ops[o + 1].span == 1)
                reps = ops[o + 1].count;
            V ka[C], kb[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                ka[c] = (V)ops[o].a[c];
                kb[c] = (V)ops[o].b[c];
            }
            if (code == OPC_FMA) {
                for (int r = 0; r < reps; ++r)
#pragma unroll
                    for (int j = 0; j < K; ++j)
#pragma unroll
                        for (int i = 0; i < P; ++i)
#pragma unroll
                            for (int c = 0; c < C; ++c)
                                v[j][i][c] = fma_v(v[j][i][c], ka[c], kb[c]);
            } else if (code == OPC_MUL) {
                for (int r = 0; r < reps; ++r)
#pragma unroll
                    for (int j = 0; j < K; ++j)
#pragma unroll
                        for (int i = 0; i < P; ++i)
#pragma unroll
                            for (int c = 0; c < C; ++c)
                                v[j][i][c] = v[j][i][c] * ka[c];
            } else if (code == OPC_ADD) {
                for (int r = 0; r < reps; ++r)
#pragma unroll
                    for (int j = 0; j < K; ++j)
#pragma unroll
                        for (int i = 0; i < P; ++i)
#pragma unroll
                            for (int c = 0; c < C; ++c)
                                v[j][i][c] = v[j][i][c] + ka[c];
            } else {
                for (int r = 0; r < reps; ++r)
#pragma unroll
                    for (int j = 0; j < K; ++j)
#pragma unroll
                        for (int i = 0; i < P; ++i)
#pragma unroll
                            for (int c = 0; c < C; ++c)
                                v[j][i][c] = v[j][i][c] / ka[c];
            }
        }
    }
};

// --------------------------------------------------------- write ops --

// Planar write (Split): channel c of pixel p goes to plane c.
template <int DT, int C>
struct WritePlanar {
    static constexpr int layout = LY_PLANAR;
    static constexpr int dtype = DT;
    static constexpr int lds_bytes_per_thread = 0;
    __device__ __forceinline__ static void store(const ItemRec &it, int oy, int ox0, int n,
                                                 const float (&r)[kUnitPx][C], uint8_t *, bool)
    {
        constexpr int ES = DSize<DT>::v;
        const int64_t plane = (int64_t)it.ow * it.oh;
        const int64_t p0 = (int64_t)oy * it.ow + ox0;
        gdst_t dst = (gdst_t)it.dst;
        if (n == kUnitPx && (it.flags & IF_DST_VEC)) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                gdst_t q = dst + (c * plane + p0) * ES;
                if constexpr (DT == DT_F32) {
                    store_nt(q, fx4{r[0][c], r[1][c], r[2][c], r[3][c]});
                } else {
                    uint32_t lo = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)r[0][c]) |
                                  ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)r[1][c]) << 16);
                    uint32_t hi = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)r[2][c]) |
                                  ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)r[3][c]) << 16);
                    store_nt(q, ux2{lo, hi});
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < kUnitPx; ++i)
                if (i < n)
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        store_elem<DT>(dst + (c * plane + p0 + i) * ES, r[i][c]);
        }
    }
};

// Packed write.  A wave whose 64 units are all whole and contiguous stages
// its output through LDS so that each global store instruction writes one
// contiguous run (16 bytes per lane); otherwise per-element stores.
template <int DT, int C>
struct WritePacked {
    static constexpr int layout = LY_PACKED;
    static constexpr int dtype = DT;
    static constexpr int ES = DSize<DT>::v;
    static constexpr int UB = kUnitPx * C * ES;                 // bytes per unit
    static constexpr bool kStage = (UB != 16 && UB != 8);       // else already lane-contiguous
    static constexpr int lds_bytes_per_thread = kStage ? UB : 0;
    static constexpr int CH = (UB % 16 == 0) ? 16 : 8;          // chunk per store

    __device__ __forceinline__ static void pack(const float (&r)[kUnitPx][C],
                                                uint32_t (&w)[UB / 4])
    {
        if constexpr (DT == DT_F32) {
#pragma unroll
            for (int i = 0; i < kUnitPx; ++i)
#pragma unroll
                for (int c = 0; c < C; ++c)
                    w[i * C + c] = __builtin_bit_cast(uint32_t, r[i][c]);
        } else {
#pragma unroll
            for (int e = 0; e < kUnitPx * C; e += 2) {
                const float a = r[e / C][e % C];
                const float b = r[(e + 1) / C][(e + 1) % C];
                w[e / 2] = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)a) |
                           ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)b) << 16);
            }
        }
    }

    // wave_lds: this wave's LDS region (64 * UB bytes); all_whole: the
    // whole wave holds whole, contiguous units (wave-uniform).
    __device__ __forceinline__ static void store(const ItemRec &it, int oy, int ox0, int n,
                                                 const float (&r)[kUnitPx][C], uint8_t *wave_lds,
                                                 bool all_whole)
    {
        const int64_t p0 = (int64_t)oy * it.ow + ox0;
        gdst_t dst = (gdst_t)it.dst + p0 * (C * ES);
        if (all_whole) {
            uint32_t w[UB / 4];
            pack(r, w);
            if constexpr (!kStage) {
                if constexpr (UB == 16)
                    store_nt(dst, ux4{w[0], w[1], w[2], w[3]});
                else
                    store_nt(dst, ux2{w[0], w[1]});
            } else {
                const int lane = threadIdx.x & (kWave - 1);
                // lane's unit -> LDS, then 64 * UB bytes out in contiguous chunks
                uint32_t *mine = (uint32_t *)(wave_lds + lane * UB);
#pragma unroll
                for (int i = 0; i < UB / 4; ++i)
                    mine[i] = w[i];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                gdst_t wdst = dst - (int64_t)lane * UB;  // the wave's first unit
                constexpr int NCH = kWave * UB / CH;
#pragma unroll
                for (int k = 0; k < (NCH + kWave - 1) / kWave; ++k) {
                    const int ch = k * kWave + lane;
                    if (NCH % kWave == 0 || ch < NCH) {
                        if constexpr (CH == 16)
                            store_nt(wdst + ch * 16, *(const ux4 *)(wave_lds + ch * 16));
                        else
                            store_nt(wdst + ch * 8, *(const ux2 *)(wave_lds + ch * 8));
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
        } else {
#pragma unroll
            for (int i = 0; i < kUnitPx; ++i)
                if (i < n)
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        store_elem<DT>(dst + (i * C + c) * ES, r[i][c]);
        }
    }
};

// ------------------------------------------------ transform pattern --

// Copy one item record out of the constant table (scalar loads).
__device__ __forceinline__ ItemRec load_item(const FK_CONST ItemRec *p)
{
    const FK_CONST uint32_t *q = (const FK_CONST uint32_t *)p;
    uint32_t w[sizeof(ItemRec) / 4];
#pragma unroll
    for (int i = 0; i < (int)(sizeof(ItemRec) / 4); ++i)
        w[i] = q[i];
    ItemRec it;
    __builtin_memcpy(&it, w, sizeof(ItemRec));
    return it;
}

// Row of index u (a unit or a pixel) for d indices per row: a
// double-precision reciprocal estimate, within one of the quotient (u <
// 2^28, a 53-bit product), corrected by exact 32-bit products ((q + 1) * d
// <= u + 2d < 2^29 for d < 2^16).  Cheaper than a 32-bit integer
// division; the reciprocal is taken once per tile.
// The quotients here are row indices (below 2^16), so the corrections use
// the full-rate 24-bit multiply.
struct RowDiv {
    uint32_t upr;
    double rcp;
    __device__ __forceinline__ explicit RowDiv(uint32_t d) : upr(d), rcp(1.0 / (double)d) {}
    __device__ __forceinline__ uint32_t operator()(uint32_t u) const
    {
        uint32_t q = (uint32_t)((double)u * rcp);
        if (__umul24(q + 1, upr) <= u)
            ++q;
        else if (__umul24(q, upr) > u)
            --q;
        return q;
    }
};

// Batch slot owning a tile: the last item whose first tile is <= tile.
__device__ __forceinline__ int find_item(const FK_CONST uint32_t *tb, int n_items, uint32_t tile)
{
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tb[mid] <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// The same search for a transform tile (tile < total = tb[n_items]).  The
// first probe is where the tile would fall if every item had the same
// number of tiles, which is exact for a batch of equal items: one pair of
// adjacent offsets instead of a search.  A miss leaves the search on one
// side of the probe.  tb holds n_items + 1 offsets.  Up to 4 items the
// plain search takes at most two loads and no division (one item: none).
__device__ __forceinline__ int find_item_guess(const FK_CONST uint32_t *tb, int n_items,
                                               uint32_t tile, uint32_t total)
{
    if (n_items <= 4)
        return find_item(tb, n_items, tile);
    int lo = 0, hi = n_items - 1;
    const int g = (int)(((uint64_t)tile * (uint64_t)n_items) / total);  // 0 <= g < n_items
    if (tb[g] <= tile) {
        if (tb[g + 1] > tile)
            return g;
        lo = g + 1;
    } else {
        hi = g - 1;
    }
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tb[mid] <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// The item owning `tile` (with the compact form's per-item fields filled
// in), and the tile's first unit within it.
template <class Read, int C>
__device__ __forceinline__ void tile_item(const KArgs &a, const FK_CONST KArgs *ka, bool compact,
                                          const FK_CONST uint32_t *tb, const FK_CONST ItemRec *items,
                                          int n_items, uint32_t tile, uint32_t total,
                                          uint32_t tile_units, ItemRec &it, uint32_t &ubase)
{
    uint32_t first_tile;
    if (compact) {
        const int b = (int)(tile / a.inl_tiles_per_item);
        first_tile = (uint32_t)b * a.inl_tiles_per_item;
        it = load_item(items);  // the template (item 0)
        const FK_CONST Roi16 *roi = (const FK_CONST Roi16 *)(ka->inl + 64) + b;
        it.x = roi->x;
        it.y = roi->y;
        it.w = roi->w;
        it.h = roi->h;
        it.dst += (uint64_t)b * (uint64_t)a.inl_dst_stride;
        if constexpr (rd_bilinear(Read::kind)) {
            // the same IEEE fp32 divisions the host performs for the table forms
            it.sx = (float)it.w / (float)it.ow;
            it.sy = (float)it.h / (float)it.oh;
        }
        // template bit: frame base and pitch dword-aligned; the ROI's
        // column offset decides the rest
        if ((it.x * C * Read::elem_size) % 4 != 0)
            it.flags &= ~IF_SRC_VEC;
    } else {
        const int b = find_item_guess(tb, n_items, tile, total);
        it = load_item(items + b);
        first_tile = tb[b];
    }
    ubase = (tile - first_tile) * tile_units;
}

// Units of a thread's K that k_transform holds in registers at once.  A
// block of up to 1024 threads leaves each lane 128 VGPRs; past that the
// compiler spills the register tile to scratch, and such launches ran 4-5x
// slower than unspilled ones (a plain u8 read into packed fp32: 103 us at
// K = 8 against 24 us at K <= 4).  So the K units go through in groups of
// G, each loaded, computed and stored before the next: G = K where the
// whole tile fits, else the largest group that compiles without scratch
// (from the kernels' scratch sizes): 4 units of 3 channels, 2 of 4, and
// half that for the run-time op list into planar fp32, whose per-channel
// 16-byte stores gather each value anew (once more halved for fp32 plain
// reads); 2 for the NV12 resize read.
template <class Read, class Compute, class Write, int C, int K>
constexpr int unit_group()
{
    constexpr bool rt = std::is_same<Compute, RuntimeCompute>::value;
    constexpr bool planar32 = Write::layout == LY_PLANAR && Write::dtype == DT_F32;
    int g = C == 1 ? 8 : C == 3 ? 4 : 2;
    if (rt && planar32 && C == 3)
        g = 2;
    if (rt && planar32 && Read::kind == RD_PLAIN && Read::elem_size == 4)
        g /= 2;
    if (Read::kind == RD_NV12_RESIZE && g > 2)
        g = 2;  // four converted taps per pixel
    return K < g ? K : g;
}

template <class Read, class Compute, class Write, int C, int K>
__global__ __launch_bounds__(kMaxBlock) void k_transform(const KArgs a)
{
    extern __shared__ __align__(16) uint8_t lds[];
    // Small batches travel inside the kernel arguments (no table copy);
    // larger ones, and graph replays, read the device table.
    const FK_CONST KArgs *ka = (const FK_CONST KArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    const bool inl = a.inl_n > 0;
    const bool compact = inl && a.inl_compact;
    const FK_CONST uint32_t *tb =
        inl ? (const FK_CONST uint32_t *)(ka->inl + kInlineTileBegin) : cptr(a.tile_begin);
    const FK_CONST ItemRec *items = inl ? (const FK_CONST ItemRec *)ka->inl : cptr(a.items);
    const int n_items = inl ? a.inl_n : cptr(a.hdr)->n_items;
    const uint32_t total = inl ? a.inl_total_tiles : cptr(a.hdr)->total_tiles;
    const int T = blockDim.x;
    const int tid = threadIdx.x;
    const uint32_t tile_units = (uint32_t)T * K;
    uint8_t *wave_lds = lds + (tid / kWave) * (kWave * Write::lds_bytes_per_thread);
    const bool swap = a.swap != 0;

    for (uint32_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
        ItemRec it;
        uint32_t ubase;
        tile_item<Read, C>(a, ka, compact, tb, items, n_items, tile, total, tile_units, it, ubase);
        const uint32_t upr = (uint32_t)(it.ow + kUnitPx - 1) / kUnitPx;
        const uint32_t units = upr * (uint32_t)it.oh;
        const RowDiv rowdiv(upr);

        // a plain read of whole frame rows stored back to back (and its
        // output) is one row of ow * oh pixels: no row division
        bool contig = false;
        if constexpr (Read::kind == RD_PLAIN)
            contig = it.flags & IF_CONTIG;
        constexpr int G = unit_group<Read, Compute, Write, C, K>();
#pragma unroll 1
        for (int g0 = 0; g0 < K; g0 += G) {
            float v[G][kUnitPx][C];
            int oy[G], ox0[G], nv[G];
#pragma unroll
            for (int j = 0; j < G; ++j) {
                const uint32_t u = ubase + (uint32_t)((g0 + j) * T + tid);
                if (u < units) {
                    if (contig) {
                        oy[j] = 0;
                        ox0[j] = (int)(u * kUnitPx);
                        nv[j] = kUnitPx;
                    } else {
                        const uint32_t row = rowdiv(u);
                        oy[j] = (int)row;
                        ox0[j] = (int)(u - row * upr) * kUnitPx;
                        const int left = it.ow - ox0[j];
                        nv[j] = left < kUnitPx ? left : kUnitPx;
                    }
                    Read::load(it, oy[j], ox0[j], nv[j], v[j]);
                } else {
                    oy[j] = 0;
                    ox0[j] = 0;
                    nv[j] = 0;
#pragma unroll
                    for (int i = 0; i < kUnitPx; ++i)
#pragma unroll
                        for (int c = 0; c < C; ++c)
                            v[j][i][c] = 0.0f;
                }
            }
            if constexpr (C >= 3) {
                // run-time tier: the chain's net channel swap, applied at the read
                if (swap) {
#pragma unroll
                    for (int j = 0; j < G; ++j)
#pragma unroll
                        for (int i = 0; i < kUnitPx; ++i) {
                            const float t = v[j][i][0];
                            v[j][i][0] = v[j][i][2];
                            v[j][i][2] = t;
                        }
                }
            }

            Compute::template apply<G, C>(a, v);

#pragma unroll
            for (int j = 0; j < G; ++j) {
                const bool whole = nv[j] == kUnitPx && (it.flags & IF_DST_VEC);
                const bool wave_whole = __all(whole ? 1 : 0);
                if (nv[j] > 0)
                    Write::store(it, oy[j], ox0[j], nv[j], v[j], wave_lds, wave_whole);
            }
        }
    }
}

// ----------------------------------------- gathers, pixel-strided lanes --
// The transform pattern for a gathering read (bilinear or nearest crop+
// resize, NV12) with a planar write, laid out for the gather: lane t of a
// tile takes output pixels
// pbase + q * T + t (q < 4K) instead of K units of 4 adjacent pixels.  Each
// gather instruction of a wave then reads the taps of 64 consecutive output
// pixels, a segment of one or two source rows, instead of 64 units spread
// over several output rows, so the L1 sees far fewer distinct lines per
// instruction.  Tiles are those of k_transform (T * K units = 4 T K
// pixels); the per-pixel planar stores of consecutive lanes are
// consecutive.
// Store pixel i's C channels of v to its planar output position.
template <int DO, int C>
__device__ __forceinline__ void store_planar_px(gdst_t dst, int64_t plane, const ItemRec &it, int oy,
                                                int ox, const float (&v)[C])
{
    constexpr int ES = DSize<DO>::v;
    // below ow * oh < 2^32
    const uint32_t p = __umul24((uint32_t)oy, (uint32_t)it.ow) + (uint32_t)ox;
#pragma unroll
    for (int c = 0; c < C; ++c)
        store_elem<DO>(dst + (c * plane + (int64_t)p) * ES, v[c]);
}

// The chain on 4 gathered pixels per lane (v), then their planar stores;
// oy[i] < 0 marks a lane's pixel outside the tile.
template <class Compute, int DO, int C>
__device__ __forceinline__ void chain_store_px(const KArgs &a, const ItemRec &it, float (&v)[1][kUnitPx][C],
                                               const int (&oy)[kUnitPx], const int (&ox)[kUnitPx])
{
    if constexpr (C >= 3) {
        // run-time tier: the chain's net channel swap, applied at the read
        if (a.swap) {
#pragma unroll
            for (int i = 0; i < kUnitPx; ++i) {
                const float t = v[0][i][0];
                v[0][i][0] = v[0][i][2];
                v[0][i][2] = t;
            }
        }
    }

    Compute::template apply<1, C>(a, v);

    const int64_t plane = (int64_t)it.ow * it.oh;
#pragma unroll
    for (int i = 0; i < kUnitPx; ++i)
        if (oy[i] >= 0)
            store_planar_px<DO, C>((gdst_t)it.dst, plane, it, oy[i], ox[i], v[0][i]);
}

// One tile of pixel-strided lanes: output pixels [pbase, pbase + 4 T K)
// of the item, pixel pbase + q T + t on lane t.
template <class Read, class Compute, int DO, int C, int K>
__device__ __forceinline__ void px_tile(const KArgs &a, const ItemRec &it, uint32_t ubase, int T, int tid)
{
    const uint32_t npx = (uint32_t)it.ow * (uint32_t)it.oh;  // < 2^32
    const uint32_t pbase = ubase * kUnitPx;
    const RowDiv rowdiv((uint32_t)it.ow);  // exact below 2^28 pixels
    const bool big = npx >= (1u << 28);
    const bool prep = Read::px_prep(it);

    // groups of 4 pixels per lane, one after another: registers do not
    // grow with K (K only sizes the tile)
    for (int j = 0; j < K; ++j) {
        float v[1][kUnitPx][C];
        int oy[kUnitPx], ox[kUnitPx];
#pragma unroll
        for (int i = 0; i < kUnitPx; ++i) {
            const uint32_t q = (uint32_t)(j * kUnitPx + i);
            const uint32_t p = pbase + q * (uint32_t)T + (uint32_t)tid;
            if (p < npx && p >= pbase) {
                const uint32_t row = big ? p / (uint32_t)it.ow : rowdiv(p);
                oy[i] = (int)row;
                ox[i] = (int)(p - __umul24(row, (uint32_t)it.ow));
                Read::load_px(it, prep, oy[i], ox[i], v[0][i]);
            } else {
                oy[i] = -1;
                ox[i] = 0;
#pragma unroll
                for (int c = 0; c < C; ++c)
                    v[0][i][c] = 0.0f;
            }
        }
        chain_store_px<Compute, DO, C>(a, it, v, oy, ox);
    }
}

template <class Read, class Compute, int DO, int C, int K>
__global__ __launch_bounds__(kMaxBlock) void k_resize_px(const KArgs a)
{
    const FK_CONST KArgs *ka = (const FK_CONST KArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    const bool inl = a.inl_n > 0;
    const bool compact = inl && a.inl_compact;
    const FK_CONST uint32_t *tb =
        inl ? (const FK_CONST uint32_t *)(ka->inl + kInlineTileBegin) : cptr(a.tile_begin);
    const FK_CONST ItemRec *items = inl ? (const FK_CONST ItemRec *)ka->inl : cptr(a.items);
    const int n_items = inl ? a.inl_n : cptr(a.hdr)->n_items;
    const uint32_t total = inl ? a.inl_total_tiles : cptr(a.hdr)->total_tiles;
    const int T = blockDim.x;
    const int tid = threadIdx.x;
    const uint32_t tile_units = (uint32_t)T * K;

    for (uint32_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
        ItemRec it;
        uint32_t ubase;
        tile_item<Read, C>(a, ka, compact, tb, items, n_items, tile, total, tile_units, it, ubase);
        px_tile<Read, Compute, DO, C, K>(a, it, ubase, T, tid);
    }
}

// ------------------------------- bilinear gather from LDS-staged rows --
// The pixel-strided pattern with the tapped source rows staged in LDS
// (u8 frames).  A tile's output rows are taken a band at a time: the two
// tap rows of every output row of the band are copied from the frame into
// LDS over the ROI's whole width, in 16-byte chunks (each load instruction
// of a wave reads up to 1 KiB of consecutive bytes), and after a barrier
// the lanes read their taps from LDS as two aligned 8-byte reads per tap
// row, from which the same byte window as the global read is cut out (the
// interpolation is ReadCropResize's, so the results are the same bits).
// Items whose frame base or pitch is not a multiple of 16, whose staged row
// does not fit twice in the block's LDS, or whose last 16-byte chunk would
// pass the end of the frame's last row take the direct per-pixel gathers.
struct LdsGather {
    uint32_t start;   // first staged byte of a row, from the row's base (16-aligned)
    uint32_t n16;     // 16-byte chunks per staged row
    uint32_t stride;  // LDS bytes per staged row: the chunks + 16 bytes of slack
                      // for the 8-byte reads past the last tap
    uint32_t band;    // output rows per band (two staged rows each)
};

template <int C>
__device__ __forceinline__ bool lds_gather_plan(const ItemRec &it, uint32_t lds, LdsGather &g)
{
    if ((it.src & 15u) || (it.pitch & 15))
        return false;
    const uint32_t b0 = (uint32_t)it.x * C, b1 = (uint32_t)(it.x + it.w) * C;
    g.start = b0 & ~15u;
    const uint32_t end = (b1 + 15u) & ~15u;
    // the chunk holding a row's last ROI byte ends inside the row's pitch;
    // on the frame's last row it must also end inside the row's pixels
    if (it.y + it.h >= (int)it.fh && end > (uint32_t)it.fw * C)
        return false;
    g.n16 = (end - g.start) >> 4;
    g.stride = end - g.start + 16u;
    g.band = lds / (2u * g.stride);
    return g.band >= 1;
}

// bytes [0, 8) from LDS byte address a (any alignment), as two dwords
__device__ __forceinline__ void lds_window(const uint8_t *lds, uint32_t a, uint32_t (&d)[2])
{
    const uint32_t a8 = a & ~7u;
    const ux2 lo = *(const ux2 *)(lds + a8);
    const ux2 hi = *(const ux2 *)(lds + a8 + 8);
    const bool k = (a & 4u) != 0;
    const uint32_t sh = a & 3u;
    const uint32_t w0 = k ? lo.y : lo.x;
    const uint32_t w1 = k ? hi.x : lo.y;
    const uint32_t w2 = k ? hi.y : hi.x;
    d[0] = __builtin_amdgcn_alignbyte(w1, w0, sh);
    d[1] = __builtin_amdgcn_alignbyte(w2, w1, sh);
}

template <class Compute, int DO, int C, int K>
__global__ __launch_bounds__(kMaxBlock) void k_resize_lds(const KArgs a)
{
    using Read = ReadCropResize<DT_U8, C>;
    extern __shared__ __align__(16) uint8_t lds[];
    const FK_CONST KArgs *ka = (const FK_CONST KArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    const bool inl = a.inl_n > 0;
    const bool compact = inl && a.inl_compact;
    const FK_CONST uint32_t *tb =
        inl ? (const FK_CONST uint32_t *)(ka->inl + kInlineTileBegin) : cptr(a.tile_begin);
    const FK_CONST ItemRec *items = inl ? (const FK_CONST ItemRec *)ka->inl : cptr(a.items);
    const int n_items = inl ? a.inl_n : cptr(a.hdr)->n_items;
    const uint32_t total = inl ? a.inl_total_tiles : cptr(a.hdr)->total_tiles;
    const int T = blockDim.x;
    const int tid = threadIdx.x;
    const uint32_t tile_units = (uint32_t)T * K;
    const uint32_t lds_bytes = lds_gather_bytes((uint32_t)T);

    for (uint32_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
        ItemRec it;
        uint32_t ubase;
        tile_item<Read, C>(a, ka, compact, tb, items, n_items, tile, total, tile_units, it, ubase);
        LdsGather g;
        const uint32_t npx = (uint32_t)it.ow * (uint32_t)it.oh;
        // uniform over the block: every lane takes the same branch
        if (npx >= (1u << 28) || !lds_gather_plan<C>(it, lds_bytes, g)) {
            px_tile<Read, Compute, DO, C, K>(a, it, ubase, T, tid);
            continue;
        }
        const uint32_t ow = (uint32_t)it.ow;
        const uint32_t pbase = ubase * kUnitPx;
        const uint32_t pend = min(pbase + (uint32_t)kUnitPx * tile_units, npx);
        const RowDiv rowdiv(ow);
        const RowDiv chunkdiv(g.n16);
        const uint32_t r_last = rowdiv(pend - 1);
        gsrc_t rowbase = (gsrc_t)it.src + g.start;
        for (uint32_t r0 = rowdiv(pbase); r0 <= r_last; r0 += g.band) {
            const uint32_t nr = min(g.band, r_last + 1 - r0);
            __syncthreads();  // every lane is done with the previous band (or tile)
            for (uint32_t i = tid; i < 2u * nr * g.n16; i += (uint32_t)T) {
                const uint32_t slot = chunkdiv(i);
                const uint32_t c = i - slot * g.n16;
                int y0, y1;
                float ay;
                bilinear_coord((int)(r0 + (slot >> 1)), it.sy, it.h, y0, y1, ay);
                const int sy = it.y + ((slot & 1u) ? y1 : y0);
                const ux4 v = *(const FK_GLOBAL ux4 *)(rowbase + (int64_t)sy * it.pitch + c * 16u);
                *(ux4 *)(lds + slot * g.stride + c * 16u) = v;
            }
            __syncthreads();
            const uint32_t p0 = max(pbase, r0 * ow);
            const uint32_t p1 = min(pend, (r0 + nr) * ow);
            for (uint32_t pb = p0; pb < p1; pb += (uint32_t)kUnitPx * (uint32_t)T) {
                float v[1][kUnitPx][C];
                int oy[kUnitPx], ox[kUnitPx];
#pragma unroll
                for (int i = 0; i < kUnitPx; ++i) {
                    const uint32_t p = pb + (uint32_t)(i * T + tid);
                    if (p < p1) {
                        const uint32_t row = rowdiv(p);
                        oy[i] = (int)row;
                        ox[i] = (int)(p - __umul24(row, ow));
                        int x0, x1, y0, y1;
                        float ax, ay;
                        bilinear_coord(ox[i], it.sx, it.w, x0, x1, ax);
                        bilinear_coord(oy[i], it.sy, it.h, y0, y1, ay);
                        const uint32_t off = (uint32_t)(it.x + x0) * C - g.start;
                        const uint32_t top = 2u * (row - r0) * g.stride + off;
                        uint32_t tw[2], bw[2];
                        lds_window(lds, top, tw);
                        lds_window(lds, top + g.stride, bw);
                        Read::lerp_windows(tw, bw, x1 == x0, ax, ay, v[0][i]);
                    } else {
                        oy[i] = -1;
                        ox[i] = 0;
#pragma unroll
                        for (int c = 0; c < C; ++c)
                            v[0][i][c] = 0.0f;
                    }
                }
                chain_store_px<Compute, DO, C>(a, it, v, oy, ox);
            }
        }
    }
}

// ------------------------------------------------- compile-time loop chain, per pixel --
// For the compile-time loop chain (plain read, [cvt,] mul, add, loop(2, P),
// packed fp32) with a long loop the arithmetic dwarfs the memory traffic,
// and the 4-pixel unit leaves too few waves on small batches: 50 images of
// 60x120 give 1,406 waves of 4-pixel lanes for 1,024 SIMDs, so the last
// round runs 37% full.  This kernel gives each lane one pixel per round:
// a tile is T*K pixels of one item in row-major order, lane t of round j
// taking pixel j*T + t of the tile (5,625 waves for the same batch).
// Loads are C elements per lane; stores are C nontemporal floats per lane,
// consecutive across the wave.
template <int DI, int C, bool Strict, int K>
__global__ __launch_bounds__(kMaxBlock) void k_loop_px(const KArgs a)
{
    constexpr int ES = DSize<DI>::v;
    const FK_CONST KArgs *ka = (const FK_CONST KArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    const bool inl = a.inl_n > 0;
    const bool compact = inl && a.inl_compact;
    const FK_CONST uint32_t *tb =
        inl ? (const FK_CONST uint32_t *)(ka->inl + kInlineTileBegin) : cptr(a.tile_begin);
    const FK_CONST ItemRec *items = inl ? (const FK_CONST ItemRec *)ka->inl : cptr(a.items);
    const int n_items = inl ? a.inl_n : cptr(a.hdr)->n_items;
    const uint32_t total = inl ? a.inl_total_tiles : cptr(a.hdr)->total_tiles;
    const int T = blockDim.x;
    const int tid = threadIdx.x;
    const uint32_t tile_px = (uint32_t)T * K;
    const FK_CONST float *k = cptr(a.consts);
    const float m = k[0];
    const float ad = in_vgpr(k[1]);
    const int n = a.loop_count;

    for (uint32_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
        int b;
        ItemRec it;
        uint32_t first_tile;
        if (compact) {
            b = (int)(tile / a.inl_tiles_per_item);
            first_tile = (uint32_t)b * a.inl_tiles_per_item;
            it = load_item(items);
            const FK_CONST Roi16 *roi = (const FK_CONST Roi16 *)(ka->inl + 64) + b;
            it.x = roi->x;
            it.y = roi->y;
            it.w = roi->w;
            it.h = roi->h;
            it.dst += (uint64_t)b * (uint64_t)a.inl_dst_stride;
        } else {
            b = find_item_guess(tb, n_items, tile, total);
            it = load_item(items + b);
            first_tile = tb[b];
        }
        const uint32_t ow = (uint32_t)it.ow;
        const uint32_t npx = ow * (uint32_t)it.oh;
        const uint32_t pbase = (tile - first_tile) * tile_px;
        const RowDiv rowdiv(ow);  // pixel p < 2^28 in a row of ow <= 65535 pixels
        gsrc_t src = (gsrc_t)it.src + (int64_t)it.x * (C * ES);
        FK_GLOBAL float *dst = (FK_GLOBAL float *)(uintptr_t)it.dst;

        float v[K][C];
        uint32_t p[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            p[j] = pbase + (uint32_t)(j * T + tid);
            if (p[j] < npx) {
                const uint32_t row = rowdiv(p[j]);
                const uint32_t col = p[j] - row * ow;
                gsrc_t e = src + (int64_t)(it.y + (int)row) * it.pitch + (int64_t)col * (C * ES);
#pragma unroll
                for (int c = 0; c < C; ++c)
                    v[j][c] = load_elem<DI>(e + c * ES);
            } else {
#pragma unroll
                for (int c = 0; c < C; ++c)
                    v[j][c] = 0.0f;
            }
        }
#pragma unroll 32
        for (int q = 0; q < n; ++q) {
#pragma unroll
            for (int j = 0; j < K; ++j)
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    if constexpr (Strict) {
                        const float t = v[j][c] * m;
                        v[j][c] = t + ad;
                    } else {
                        v[j][c] = fmaf(v[j][c], m, ad);
                    }
                }
        }
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (p[j] < npx) {
#pragma unroll
                for (int c = 0; c < C; ++c)
                    __builtin_nontemporal_store(v[j][c], dst + (size_t)p[j] * C + c);
            }
    }
}

// ------------------------------------------------------------- stats --
// The reduction pattern (Section IV-C's second data-parallel pattern): the
// same read and compute ops as the transform, then per channel min, max and
// an fp64 sum of the item's values, from one read of the source.
//
// Two kernels.  k_stats: a batch slot (item) is covered by `nslots` blocks;
// block slot s strides over the item's tiles s, s + nslots, ...; each block
// reduces its values in a fixed order (lane order within a wave by
// xor-shuffles, then waves in order) and stores one StatPartial per
// channel.  k_stats_final: one block per item combines the item's partials
// in slot order and writes {min, max, sum, mean}.  The kernel boundary
// orders the partials' stores before their loads, so no block needs a
// device-scope fence (on a multi-XCD part each such fence writes back the
// XCD's L2).

template <int C>
struct StatAcc {
    float mn[C], mx[C];
    double sum[C];
    __device__ __forceinline__ void init()
    {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            mn[c] = __builtin_inff();
            mx[c] = -__builtin_inff();
            sum[c] = 0.0;
        }
    }
    __device__ __forceinline__ void add(const StatAcc &o)
    {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            mn[c] = fminf(mn[c], o.mn[c]);
            mx[c] = fmaxf(mx[c], o.mx[c]);
            sum[c] += o.sum[c];
        }
    }
    // lane 0 of the wave ends up with the wave's reduction (fixed xor tree)
    __device__ __forceinline__ void wave_reduce()
    {
#pragma unroll
        for (int m = kWave / 2; m >= 1; m >>= 1) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                mn[c] = fminf(mn[c], __shfl_xor(mn[c], m, kWave));
                mx[c] = fmaxf(mx[c], __shfl_xor(mx[c], m, kWave));
                sum[c] += __shfl_xor(sum[c], m, kWave);
            }
        }
    }
};

// Block-wide reduction into thread 0 (waves combined in wave order).
template <int C>
__device__ __forceinline__ void block_reduce(StatAcc<C> &acc, StatPartial (*lds)[C], int tid,
                                             int T)
{
    acc.wave_reduce();
    const int wave = tid / kWave;
    if ((tid % kWave) == 0) {
#pragma unroll
        for (int c = 0; c < C; ++c)
            lds[wave][c] = StatPartial{acc.mn[c], acc.mx[c], acc.sum[c]};
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < T / kWave; ++w) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                acc.mn[c] = fminf(acc.mn[c], lds[w][c].mn);
                acc.mx[c] = fmaxf(acc.mx[c], lds[w][c].mx);
                acc.sum[c] += lds[w][c].sum;
            }
        }
    }
    __syncthreads();
}

// One tile of a plain read whose units are all whole and dword-aligned:
// a group of the K units' raw dwords is fetched first (GW loads in flight
// per lane), then each unit is unpacked, run through the ops and
// accumulated.  All K units form one group while their words fit in 48
// dwords for up to 3 channels (28 for 4, whose accumulators take more
// registers); past that, groups of at most 24 (16) dwords.  With all K
// units' words live, fp32 frames of 3 channels at K = 8 and of 4 channels
// at K >= 4 spilled to scratch and took 2-3x longer.
template <int NW, int C, int K>
constexpr int stats_group()
{
    if (NW * K <= (C <= 3 ? 48 : 28))
        return K;
    const int budget = C <= 3 ? 24 : 16;
    int g = 1;
    while (g * 2 * NW <= budget)
        g *= 2;
    return g;
}

template <class Read, class Compute, int C, int K>
__device__ __forceinline__ void stats_tile_vec(const KArgs &a, const ItemRec &it, uint32_t ubase,
                                               uint32_t units, const RowDiv &rowdiv, int T, int tid,
                                               bool swap, StatAcc<C> &acc)
{
    constexpr int DT = Read::dtype;
    constexpr int NW = kUnitPx * C * DSize<DT>::v / 4;
    constexpr int GW = stats_group<NW, C, K>();
#pragma unroll 1
    for (int g0 = 0; g0 < K; g0 += GW) {
        uint32_t w[GW][NW];
        bool ok[GW];
#pragma unroll
        for (int j = 0; j < GW; ++j) {
            const uint32_t u = ubase + (uint32_t)((g0 + j) * T + tid);
            ok[j] = u < units;
            if (ok[j]) {
                const uint32_t row = rowdiv(u);
                const int ox0 = (int)(u - row * rowdiv.upr) * kUnitPx;
                const FK_GLOBAL uint32_t *p =
                    (const FK_GLOBAL uint32_t *)((gsrc_t)it.src + (int64_t)(it.y + (int)row) * it.pitch +
                                                 (int64_t)(it.x + ox0) * (C * DSize<DT>::v));
#pragma unroll
                for (int i = 0; i < NW; ++i)
                    w[j][i] = p[i];
            }
        }
#pragma unroll
        for (int j = 0; j < GW; ++j) {
            if (!ok[j])
                continue;
            float v[1][kUnitPx][C];
#pragma unroll
            for (int i = 0; i < kUnitPx; ++i)
#pragma unroll
                for (int c = 0; c < C; ++c)
                    v[0][i][c] = unpack_elem<DT, NW>(w[j], i * C + c);
            if constexpr (C >= 3) {
                if (swap) {
#pragma unroll
                    for (int i = 0; i < kUnitPx; ++i) {
                        const float s = v[0][i][0];
                        v[0][i][0] = v[0][i][2];
                        v[0][i][2] = s;
                    }
                }
            }
            Compute::template apply<1, C>(a, v);
#pragma unroll
            for (int i = 0; i < kUnitPx; ++i)
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    acc.mn[c] = fminf(acc.mn[c], v[0][i][c]);
                    acc.mx[c] = fmaxf(acc.mx[c], v[0][i][c]);
                    acc.sum[c] += (double)v[0][i][c];
                }
        }
    }
}

// Statistics of u8 values with no arithmetic after the cast, in integer
// registers.  A unit's C dwords hold its 4C bytes; byte k of dword i is
// channel (4i + k) % C.  Sums: a dot product of each dword with a 0/1 byte
// mask per channel (one v_dot4_u32_u8 adds up to four bytes).  Min/max: a
// dword's even and odd bytes, spread over two 16-bit halves, go through
// packed 16-bit min/max, so one instruction covers two bytes.  The results
// equal the fp32/fp64 path's exactly: the values are integers in [0, 255]
// and every partial sum is an integer below 2^53.
typedef unsigned short us2 __attribute__((ext_vector_type(2)));

template <int C>
struct U8Acc {
    uint32_t s[C];       // per channel; moved into the fp64 sums after each tile
    us2 mx[C][2], mn[C][2];  // [dword][parity]: halves hold bytes p and p + 2

    static constexpr uint32_t mask(int i, int c)
    {
        uint32_t m = 0;
        for (int k = 0; k < 4; ++k)
            if ((4 * i + k) % C == c)
                m |= 1u << (8 * k);
        return m;
    }
    __device__ __forceinline__ void init()
    {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            s[c] = 0;
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                // neutral here because every value lies in [0, 255]
                mx[c][p] = us2{0, 0};
                mn[c][p] = us2{255, 255};
            }
        }
    }
    __device__ __forceinline__ void add(const uint32_t (&w)[C])
    {
#pragma unroll
        for (int i = 0; i < C; ++i) {
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (mask(i, c) != 0)  // constant once unrolled
                    s[c] = __builtin_amdgcn_udot4(w[i], mask(i, c), s[c], false);
            const us2 even = __builtin_bit_cast(us2, w[i] & 0x00ff00ffu);
            const us2 odd = __builtin_bit_cast(us2, (w[i] >> 8) & 0x00ff00ffu);
            mx[i][0] = __builtin_elementwise_max(mx[i][0], even);
            mn[i][0] = __builtin_elementwise_min(mn[i][0], even);
            mx[i][1] = __builtin_elementwise_max(mx[i][1], odd);
            mn[i][1] = __builtin_elementwise_min(mn[i][1], odd);
        }
    }
    template <int K>
    __device__ __forceinline__ void add_tile(const uint32_t (&w)[K][C], const bool (&ok)[K])
    {
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (ok[j])
                add(w[j]);
    }
    // into the float accumulators, by source channel
    __device__ __forceinline__ void flush_sums(StatAcc<C> &acc)
    {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            acc.sum[c] += (double)s[c];
            s[c] = 0;
        }
    }
    __device__ __forceinline__ void merge_minmax(StatAcc<C> &acc) const
    {
#pragma unroll
        for (int i = 0; i < C; ++i)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int c = (4 * i + p + 2 * h) % C;
                    acc.mx[c] = fmaxf(acc.mx[c], (float)mx[i][p][h]);
                    acc.mn[c] = fminf(acc.mn[c], (float)mn[i][p][h]);
                }
    }
};

template <class Read>
constexpr bool plain_u8()
{
    if constexpr (Read::kind == RD_PLAIN)
        return Read::dtype == DT_U8;
    else
        return false;
}

// Fetch one tile of u8 units (whole and dword-aligned) for the integer
// statistics.  Lanes past the item's last unit load its last unit instead
// and are masked out (ok = false): every lane issues the same loads, so the
// wait for this tile counts exactly the loads issued after it.
template <int C, int K>
__device__ __forceinline__ void fetch_tile_u8(const ItemRec &it, uint32_t ubase, uint32_t units,
                                              const RowDiv &rowdiv, int T, int tid,
                                              uint32_t (&w)[K][C], bool (&ok)[K])
{
    const bool contig = it.flags & IF_CONTIG;  // uniform
    gsrc_t base = (gsrc_t)it.src + (int64_t)it.y * it.pitch;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        uint32_t u = ubase + (uint32_t)(j * T + tid);
        ok[j] = u < units;
        u = ok[j] ? u : units - 1;
        gsrc_t q;
        if (contig) {
            q = base + (uint64_t)u * (kUnitPx * C);
        } else {
            const uint32_t row = rowdiv(u);
            const int ox0 = (int)(u - row * rowdiv.upr) * kUnitPx;
            q = base + (int64_t)row * it.pitch + (int64_t)(it.x + ox0) * C;
        }
        const FK_GLOBAL uint32_t *p = (const FK_GLOBAL uint32_t *)q;
#pragma unroll
        for (int i = 0; i < C; ++i)
            w[j][i] = load_stream(p + i);
    }
}

// The batch slot owning stats block `slot`: its item (with the compact
// form's per-item fields filled in), the item's first block and its number
// of blocks.
template <class Read, int C>
__device__ __forceinline__ void stats_slot_item(const KArgs &a, const FK_CONST KArgs *ka, bool compact,
                                                const FK_CONST uint32_t *tb,
                                                const FK_CONST ItemRec *items, int n_items,
                                                uint32_t slot, ItemRec &it, uint32_t &first,
                                                uint32_t &nslots)
{
    if (compact) {
        const int b = (int)(slot / a.inl_tiles_per_item);
        first = (uint32_t)b * a.inl_tiles_per_item;
        nslots = a.inl_tiles_per_item;
        it = load_item(items);
        const FK_CONST Roi16 *roi = (const FK_CONST Roi16 *)(ka->inl + 64) + b;
        it.x = roi->x;
        it.y = roi->y;
        it.w = roi->w;
        it.h = roi->h;
        it.dst += (uint64_t)b * (uint64_t)a.inl_dst_stride;
        if constexpr (rd_bilinear(Read::kind)) {
            it.sx = (float)it.w / (float)it.ow;
            it.sy = (float)it.h / (float)it.oh;
        }
        if ((it.x * C * Read::elem_size) % 4 != 0)
            it.flags &= ~IF_SRC_VEC;
    } else {
        const int b = find_item(tb, n_items, slot);
        it = load_item(items + b);
        first = tb[b];
        nslots = tb[b + 1] - first;
    }
}

// The block's statistics into thread 0, then one StatPartial per channel.
template <int C>
__device__ __forceinline__ void stats_store_partial(const KArgs &a, StatAcc<C> &acc,
                                                    StatPartial (*red)[C], uint32_t slot, int tid,
                                                    int T)
{
    block_reduce<C>(acc, red, tid, T);
    if (tid == 0) {
#pragma unroll
        for (int c = 0; c < C; ++c)
            a.st_part[(size_t)slot * C + c] = StatPartial{acc.mn[c], acc.mx[c], acc.sum[c]};
    }
    __syncthreads();  // `red` is reused by the next slot
}

template <class Read, class Compute, int C, int K>
__global__ __launch_bounds__(kMaxBlock) void k_stats(const KArgs a)
{
    __shared__ StatPartial red[kMaxBlock / kWave][C];
    const FK_CONST KArgs *ka = (const FK_CONST KArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    const bool inl = a.inl_n > 0;
    const bool compact = inl && a.inl_compact;
    const FK_CONST uint32_t *tb =
        inl ? (const FK_CONST uint32_t *)(ka->inl + kInlineTileBegin) : cptr(a.tile_begin);
    const FK_CONST ItemRec *items = inl ? (const FK_CONST ItemRec *)ka->inl : cptr(a.items);
    const int n_items = inl ? a.inl_n : cptr(a.hdr)->n_items;
    const uint32_t total = inl ? a.inl_total_tiles : cptr(a.hdr)->total_tiles;
    const int T = blockDim.x;
    const int tid = threadIdx.x;
    const uint32_t tile_units = (uint32_t)T * K;
    const bool swap = a.swap != 0;

    for (uint32_t slot = blockIdx.x; slot < total; slot += gridDim.x) {
        ItemRec it;
        uint32_t first, nslots;
        stats_slot_item<Read, C>(a, ka, compact, tb, items, n_items, slot, it, first, nslots);
        const uint32_t upr = (uint32_t)(it.ow + kUnitPx - 1) / kUnitPx;
        const uint32_t units = upr * (uint32_t)it.oh;
        const uint32_t item_tiles = (units + tile_units - 1) / tile_units;
        const RowDiv rowdiv(upr);

        StatAcc<C> acc;
        acc.init();
        // the K units of a thread run one at a time (read, ops, accumulate):
        // only one unit's values are live, whatever K
        for (uint32_t t = slot - first; t < item_tiles; t += nslots) {
            const uint32_t ubase = t * tile_units;
            if constexpr (Read::kind == RD_PLAIN) {
                // whole dword-aligned units everywhere in the item: a flag of
                // the item, so the branch is uniform
                if ((it.flags & IF_SRC_VEC) && it.ow % kUnitPx == 0) {
                    stats_tile_vec<Read, Compute, C, K>(a, it, ubase, units, rowdiv, T, tid, swap, acc);
                    continue;
                }
            }
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const uint32_t u = ubase + (uint32_t)(j * T + tid);
                if (u >= units)
                    continue;
                const uint32_t row = rowdiv(u);
                const int ox0 = (int)(u - row * upr) * kUnitPx;
                const int left = it.ow - ox0;
                const int nv = left < kUnitPx ? left : kUnitPx;
                float v[1][kUnitPx][C];
                Read::load(it, (int)row, ox0, nv, v[0]);
                if constexpr (C >= 3) {
                    if (swap) {
#pragma unroll
                        for (int i = 0; i < kUnitPx; ++i) {
                            const float s = v[0][i][0];
                            v[0][i][0] = v[0][i][2];
                            v[0][i][2] = s;
                        }
                    }
                }
                Compute::template apply<1, C>(a, v);
#pragma unroll
                for (int i = 0; i < kUnitPx; ++i)
                    if (i < nv) {
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            acc.mn[c] = fminf(acc.mn[c], v[0][i][c]);
                            acc.mx[c] = fmaxf(acc.mx[c], v[0][i][c]);
                            acc.sum[c] += (double)v[0][i][c];
                        }
                    }
            }
        }
        stats_store_partial<C>(a, acc, red, slot, tid, T);
    }
}

// The stats write of a u8 plain read with no arithmetic after the cast:
// the same slots, tiles and partials as k_stats, with integer accumulation
// (U8Acc).  A kernel of its own, so that it keeps fewer registers live than
// the float path and more waves stay resident.  Items whose units are not
// all whole and dword-aligned take a byte-by-byte loop.
template <int C, int K>
__global__ __launch_bounds__(kMaxBlock) void k_stats_u8(const KArgs a)
{
    using Read = ReadPlain<DT_U8, C>;
    __shared__ StatPartial red[kMaxBlock / kWave][C];
    const FK_CONST KArgs *ka = (const FK_CONST KArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    const bool inl = a.inl_n > 0;
    const bool compact = inl && a.inl_compact;
    const FK_CONST uint32_t *tb =
        inl ? (const FK_CONST uint32_t *)(ka->inl + kInlineTileBegin) : cptr(a.tile_begin);
    const FK_CONST ItemRec *items = inl ? (const FK_CONST ItemRec *)ka->inl : cptr(a.items);
    const int n_items = inl ? a.inl_n : cptr(a.hdr)->n_items;
    const uint32_t total = inl ? a.inl_total_tiles : cptr(a.hdr)->total_tiles;
    const int T = blockDim.x;
    const int tid = threadIdx.x;
    const uint32_t tile_units = (uint32_t)T * K;
    const bool swap = a.swap != 0;

    for (uint32_t slot = blockIdx.x; slot < total; slot += gridDim.x) {
        ItemRec it;
        uint32_t first, nslots;
        stats_slot_item<Read, C>(a, ka, compact, tb, items, n_items, slot, it, first, nslots);
        const uint32_t upr = (uint32_t)(it.ow + kUnitPx - 1) / kUnitPx;
        const uint32_t units = upr * (uint32_t)it.oh;
        const uint32_t item_tiles = (units + tile_units - 1) / tile_units;
        const RowDiv rowdiv(upr);

        StatAcc<C> acc;
        acc.init();
        if ((it.flags & IF_SRC_VEC) && it.ow % kUnitPx == 0) {
            // software pipeline over two register buffers: tile t + nslots
            // is in flight while tile t is accumulated
            U8Acc<C> iacc;
            iacc.init();
            uint32_t wa[K][C], wb[K][C];
            bool oka[K], okb[K];
            uint32_t t = slot - first;
            fetch_tile_u8<C, K>(it, t * tile_units, units, rowdiv, T, tid, wa, oka);
            for (;;) {
                const uint32_t t1 = t + nslots;
                if (t1 >= item_tiles) {
                    iacc.add_tile(wa, oka);
                    break;
                }
                fetch_tile_u8<C, K>(it, t1 * tile_units, units, rowdiv, T, tid, wb, okb);
                iacc.add_tile(wa, oka);
                iacc.flush_sums(acc);
                const uint32_t t2 = t1 + nslots;
                if (t2 >= item_tiles) {
                    iacc.add_tile(wb, okb);
                    break;
                }
                fetch_tile_u8<C, K>(it, t2 * tile_units, units, rowdiv, T, tid, wa, oka);
                iacc.add_tile(wb, okb);
                iacc.flush_sums(acc);
                t = t2;
            }
            iacc.flush_sums(acc);  // at most 2 * K * 4 * 255 per channel between flushes
            iacc.merge_minmax(acc);
        } else {
            for (uint32_t t = slot - first; t < item_tiles; t += nslots) {
                for (int j = 0; j < K; ++j) {
                    const uint32_t u = t * tile_units + (uint32_t)(j * T + tid);
                    if (u >= units)
                        break;
                    const uint32_t row = rowdiv(u);
                    const int ox0 = (int)(u - row * upr) * kUnitPx;
                    const int left = it.ow - ox0;
                    const int nv = left < kUnitPx ? left : kUnitPx;
                    gsrc_t p = (gsrc_t)it.src + (int64_t)(it.y + (int)row) * it.pitch +
                               (int64_t)(it.x + ox0) * C;
                    for (int i = 0; i < nv; ++i)
#pragma unroll
                        for (int c = 0; c < C; ++c) {
                            const float x = (float)p[i * C + c];
                            acc.mn[c] = fminf(acc.mn[c], x);
                            acc.mx[c] = fmaxf(acc.mx[c], x);
                            acc.sum[c] += (double)x;
                        }
                }
            }
        }
        if constexpr (C >= 3) {
            // the chain's net swap: statistics of source channel 2 are
            // those of output channel 0, and the other way round
            if (swap) {
                const float mn0 = acc.mn[0], mx0 = acc.mx[0];
                const double s0 = acc.sum[0];
                acc.mn[0] = acc.mn[2];
                acc.mx[0] = acc.mx[2];
                acc.sum[0] = acc.sum[2];
                acc.mn[2] = mn0;
                acc.mx[2] = mx0;
                acc.sum[2] = s0;
            }
        }
        stats_store_partial<C>(a, acc, red, slot, tid, T);
    }
}

// One block per item: the item's partials, combined in slot order.
template <int C>
__global__ __launch_bounds__(kMaxBlock) void k_stats_final(const KArgs a)
{
    __shared__ StatPartial red[kMaxBlock / kWave][C];
    const FK_CONST KArgs *ka = (const FK_CONST KArgs *)__builtin_amdgcn_kernarg_segment_ptr();
    const bool inl = a.inl_n > 0;
    const bool compact = inl && a.inl_compact;
    const FK_CONST uint32_t *tb =
        inl ? (const FK_CONST uint32_t *)(ka->inl + kInlineTileBegin) : cptr(a.tile_begin);
    const FK_CONST ItemRec *items = inl ? (const FK_CONST ItemRec *)ka->inl : cptr(a.items);
    const int n_items = inl ? a.inl_n : cptr(a.hdr)->n_items;
    const int T = blockDim.x;
    const int tid = threadIdx.x;
    for (int b = blockIdx.x; b < n_items; b += gridDim.x) {
        uint32_t first, nslots;
        uint64_t dst;
        int ow, oh;
        if (compact) {
            const ItemRec t = load_item(items);
            first = (uint32_t)b * a.inl_tiles_per_item;
            nslots = a.inl_tiles_per_item;
            dst = t.dst + (uint64_t)b * (uint64_t)a.inl_dst_stride;
            ow = t.ow;  // one output size for the whole compact batch
            oh = t.oh;
        } else {
            const ItemRec t = load_item(items + b);
            first = tb[b];
            nslots = tb[b + 1] - first;
            dst = t.dst;
            ow = t.ow;
            oh = t.oh;
        }
        StatAcc<C> fin;
        fin.init();
        for (uint32_t s = (uint32_t)tid; s < nslots; s += (uint32_t)T) {
            const StatPartial *q = a.st_part + (size_t)(first + s) * C;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                fin.mn[c] = fminf(fin.mn[c], q[c].mn);
                fin.mx[c] = fmaxf(fin.mx[c], q[c].mx);
                fin.sum[c] += q[c].sum;
            }
        }
        block_reduce<C>(fin, red, tid, T);
        if (tid == 0) {
            FK_GLOBAL double *out = (FK_GLOBAL double *)(uintptr_t)dst;
            const double n = (double)ow * (double)oh;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                out[4 * c + 0] = (double)fin.mn[c];
                out[4 * c + 1] = (double)fin.mx[c];
                out[4 * c + 2] = fin.sum[c];
                out[4 * c + 3] = fin.sum[c] / n;
            }
        }
        __syncthreads();
    }
}

}  // namespace fk
