// fk_f64.hip -- chains computed in double precision: a plain read of u8,
// fp16, fp32 or fp64 elements, the run-time op list in fp64, and an fp64
// write, packed or planar (the double-precision pairs of the data-type
// experiment, Section VI-I: the cast takes the value to double and every
// later op rounds to double).  Pixel-strided lanes over the tiles of
// k_transform (T * K units of 4 pixels): lane t holds pixels
// pbase + q T + t, q < 4K, so each load and store instruction of a wave
// touches consecutive pixels; the op list runs over up to 12 of the lane's
// values at a time.
#include "fk_device.hpp"

namespace fk {

template <int DI>
__device__ __forceinline__ double load_f64(gsrc_t p)
{
    if constexpr (DI == DT_F64)
        return *(const FK_GLOBAL double *)p;
    else
        return (double)load_elem<DI>(p);  // u8, fp16, fp32: exact in fp32, then in fp64
}

// tile_item's view of the read: a plain read of DI elements
template <int DI>
struct ReadPlainF64 {
    static constexpr int kind = RD_PLAIN;
    static constexpr int elem_size = DSize<DI>::v;
};

template <int DI, int C, bool Planar, int K>
__global__ __launch_bounds__(kMaxBlock) void k_f64(const KArgs a)
{
    using Read = ReadPlainF64<DI>;
    constexpr int ES = Read::elem_size;
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
        const uint32_t npx = (uint32_t)it.ow * (uint32_t)it.oh;  // <= 2^28
        const uint32_t pbase = ubase * kUnitPx;
        const RowDiv rowdiv((uint32_t)it.ow);
        gsrc_t roi = (gsrc_t)it.src + (int64_t)it.y * it.pitch + (int64_t)it.x * (C * ES);
        FK_GLOBAL double *dst = (FK_GLOBAL double *)it.dst;
        // the lane's 4K pixels in chunks of P: one pass of the op list
        // serves P * C values (its constants are scalar loads); P keeps at
        // most 12 doubles live (8 for one channel), so the fp64 divisions'
        // temporaries fit the 128 VGPRs of a 1024-thread block
        constexpr int P0 = C == 1 ? 8 : C == 3 ? 4 : 2;
        constexpr int P = P0 < 4 * K ? P0 : 4 * K;
        for (int q0 = 0; q0 < 4 * K; q0 += P) {
            double v[1][P][C];
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const uint32_t p = pbase + (uint32_t)((q0 + i) * T + tid);
                if (p < npx) {
                    const uint32_t row = rowdiv(p);
                    const uint32_t col = p - row * (uint32_t)it.ow;
                    gsrc_t s = roi + (int64_t)row * it.pitch + (int64_t)col * (C * ES);
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        v[0][i][c] = load_f64<DI>(s + c * ES);
                } else {
#pragma unroll
                    for (int c = 0; c < C; ++c)
                        v[0][i][c] = 0.0;
                }
            }
            if constexpr (C >= 3) {
                if (a.swap) {  // the chain's net channel swap, at the read
#pragma unroll
                    for (int i = 0; i < P; ++i) {
                        const double t = v[0][i][0];
                        v[0][i][0] = v[0][i][2];
                        v[0][i][2] = t;
                    }
                }
            }
            RuntimeCompute::template apply<1, C>(a, v);
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const uint32_t p = pbase + (uint32_t)((q0 + i) * T + tid);
                if (p < npx) {
#pragma unroll
                    for (int c = 0; c < C; ++c) {
                        // planar: plane c; packed: channel c of the pixel
                        const int64_t o = Planar ? (int64_t)c * npx + p : (int64_t)p * C + c;
                        __builtin_nontemporal_store(v[0][i][c], dst + o);
                    }
                }
            }
        }
    }
}

template <int DI, int C>
static const void *f64_ptr(int layout, int coarsen)
{
    const bool planar = layout == LY_PLANAR;
    switch (coarsen) {
    case 1: return planar ? (const void *)&k_f64<DI, C, true, 1> : (const void *)&k_f64<DI, C, false, 1>;
    case 2: return planar ? (const void *)&k_f64<DI, C, true, 2> : (const void *)&k_f64<DI, C, false, 2>;
    case 4: return planar ? (const void *)&k_f64<DI, C, true, 4> : (const void *)&k_f64<DI, C, false, 4>;
    case 8: return planar ? (const void *)&k_f64<DI, C, true, 8> : (const void *)&k_f64<DI, C, false, 8>;
    }
    return nullptr;
}

template <int DI>
static const void *f64_by_channels(int channels, int layout, int coarsen)
{
    switch (channels) {
    case 1: return f64_ptr<DI, 1>(layout, coarsen);
    case 3: return f64_ptr<DI, 3>(layout, coarsen);
    case 4: return f64_ptr<DI, 4>(layout, coarsen);
    }
    return nullptr;
}

const void *kernel_f64(int in_dt, int channels, int layout, int coarsen)
{
    switch (in_dt) {
    case DT_U8: return f64_by_channels<DT_U8>(channels, layout, coarsen);
    case DT_F16: return f64_by_channels<DT_F16>(channels, layout, coarsen);
    case DT_F32: return f64_by_channels<DT_F32>(channels, layout, coarsen);
    case DT_F64: return f64_by_channels<DT_F64>(channels, layout, coarsen);
    }
    return nullptr;
}

}  // namespace fk
