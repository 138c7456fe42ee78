// fk_static.hip -- compile-time composed chains (the paper's method: the
// op types are fixed when the library is compiled, only their parameters
// arrive at run time) and the lookup of every fused kernel.
#include "fk_device.hpp"

namespace fk {

const void *kernel_runtime_plain_u8(int, int, int, int);
const void *kernel_runtime_plain_f16(int, int, int, int);
const void *kernel_runtime_plain_f32(int, int, int, int);
const void *kernel_runtime_resize_u8(int, int, int, int);
const void *kernel_runtime_resize_f16(int, int, int, int);
const void *kernel_runtime_resize_f32(int, int, int, int);

const void *kernel_stats_plain(int, int, int);
const void *kernel_stats_resize(int, int, int);
const void *kernel_stats_other(int, int, int, int);
const void *kernel_runtime_nearest_u8(int, int, int, int);
const void *kernel_runtime_nearest_f16(int, int, int, int);
const void *kernel_runtime_nearest_f32(int, int, int, int);
const void *kernel_runtime_nv12(int, int, int, int, int);

const void *kernel_stats_final(int channels)
{
    switch (channels) {
    case 1: return (const void *)&k_stats_final<1>;
    case 3: return (const void *)&k_stats_final<3>;
    case 4: return (const void *)&k_stats_final<4>;
    }
    return nullptr;
}

const void *kernel_stats(int read_kind, int in_dt, int channels, int coarsen)
{
    if (read_kind == RD_PLAIN)
        return kernel_stats_plain(in_dt, channels, coarsen);
    if (read_kind == RD_CROP_RESIZE)
        return kernel_stats_resize(in_dt, channels, coarsen);
    return kernel_stats_other(read_kind, in_dt, channels, coarsen);
}

const void *kernel_runtime(int read_kind, int in_dt, int channels, int out_dt, int layout,
                           int coarsen)
{
    if (read_kind == RD_PLAIN) {
        switch (in_dt) {
        case DT_U8: return kernel_runtime_plain_u8(channels, out_dt, layout, coarsen);
        case DT_F16: return kernel_runtime_plain_f16(channels, out_dt, layout, coarsen);
        case DT_F32: return kernel_runtime_plain_f32(channels, out_dt, layout, coarsen);
        }
    } else if (read_kind == RD_CROP_RESIZE) {
        switch (in_dt) {
        case DT_U8: return kernel_runtime_resize_u8(channels, out_dt, layout, coarsen);
        case DT_F16: return kernel_runtime_resize_f16(channels, out_dt, layout, coarsen);
        case DT_F32: return kernel_runtime_resize_f32(channels, out_dt, layout, coarsen);
        }
    } else if (read_kind == RD_CROP_NEAREST) {
        switch (in_dt) {
        case DT_U8: return kernel_runtime_nearest_u8(channels, out_dt, layout, coarsen);
        case DT_F16: return kernel_runtime_nearest_f16(channels, out_dt, layout, coarsen);
        case DT_F32: return kernel_runtime_nearest_f32(channels, out_dt, layout, coarsen);
        }
    } else if ((read_kind == RD_NV12 || read_kind == RD_NV12_RESIZE) && in_dt == DT_U8) {
        return kernel_runtime_nv12(read_kind, channels, out_dt, layout, coarsen);
    }
    return nullptr;
}

// Crop+resize u8x3 -> swap, cvt, *k, -mean, /std -> planar fp32: 4-pixel
// units, or pixel-strided lanes for the gather of large launches.
template <bool Strict, int K>
static const void *norm_ptr(bool strided)
{
    if (strided)
        return (const void *)&k_resize_px<ReadCropResize<DT_U8, 3>, StaticCompute<NormalizeChain<Strict>>,
                                          DT_F32, 3, K>;
    return (const void *)&k_transform<ReadCropResize<DT_U8, 3>, StaticCompute<NormalizeChain<Strict>>,
                                      WritePlanar<DT_F32, 3>, 3, K>;
}

template <bool Strict, int K>
static const void *norm_lds_ptr()
{
    return (const void *)&k_resize_lds<StaticCompute<NormalizeChain<Strict>>, DT_F32, 3, K>;
}

const void *kernel_normalize_lds(int coarsen, int strict)
{
    switch (coarsen) {
    case 1: return strict ? norm_lds_ptr<true, 1>() : norm_lds_ptr<false, 1>();
    case 2: return strict ? norm_lds_ptr<true, 2>() : norm_lds_ptr<false, 2>();
    case 4: return strict ? norm_lds_ptr<true, 4>() : norm_lds_ptr<false, 4>();
    case 8: return strict ? norm_lds_ptr<true, 8>() : norm_lds_ptr<false, 8>();
    }
    return nullptr;
}

const void *kernel_normalize(int coarsen, int strict, int strided)
{
    switch (coarsen) {
    case 1: return strict ? norm_ptr<true, 1>(strided) : norm_ptr<false, 1>(strided);
    case 2: return strict ? norm_ptr<true, 2>(strided) : norm_ptr<false, 2>(strided);
    case 4: return strict ? norm_ptr<true, 4>(strided) : norm_ptr<false, 4>(strided);
    case 8: return strict ? norm_ptr<true, 8>(strided) : norm_ptr<false, 8>(strided);
    }
    return nullptr;
}

// Plain u8x3 -> cvt, N alternating mul/add -> packed fp32.
template <int N, bool Strict, int K>
static const void *muladd_ptr()
{
    return (const void *)&k_transform<ReadPlain<DT_U8, 3>, StaticCompute<MulAddChain<N, Strict>>,
                                      WritePacked<DT_F32, 3>, 3, K>;
}

template <int N>
static const void *muladd_k(int coarsen, int strict)
{
    switch (coarsen) {
    case 1: return strict ? muladd_ptr<N, true, 1>() : muladd_ptr<N, false, 1>();
    case 2: return strict ? muladd_ptr<N, true, 2>() : muladd_ptr<N, false, 2>();
    case 4: return strict ? muladd_ptr<N, true, 4>() : muladd_ptr<N, false, 4>();
    case 8: return strict ? muladd_ptr<N, true, 8>() : muladd_ptr<N, false, 8>();
    }
    return nullptr;
}

const void *kernel_muladd(int n_ops, int coarsen, int strict)
{
    switch (n_ops) {
    case 1: return muladd_k<1>(coarsen, strict);
    case 4: return muladd_k<4>(coarsen, strict);
    case 16: return muladd_k<16>(coarsen, strict);
    case 64: return muladd_k<64>(coarsen, strict);
    case 256: return muladd_k<256>(coarsen, strict);
    }
    return nullptr;
}

// Plain u8 or fp32 (1 or 3 channels) -> (mul, add) looped -> packed fp32.
template <int DI, int C, bool Strict, int K>
static const void *loop_ptr()
{
    return (const void *)&k_transform<ReadPlain<DI, C>, LoopMulAddCompute<Strict>,
                                      WritePacked<DT_F32, C>, C, K>;
}

template <int DI, int C>
static const void *loop_k(int coarsen, int strict)
{
    switch (coarsen) {
    case 1: return strict ? loop_ptr<DI, C, true, 1>() : loop_ptr<DI, C, false, 1>();
    case 2: return strict ? loop_ptr<DI, C, true, 2>() : loop_ptr<DI, C, false, 2>();
    case 4: return strict ? loop_ptr<DI, C, true, 4>() : loop_ptr<DI, C, false, 4>();
    case 8: return strict ? loop_ptr<DI, C, true, 8>() : loop_ptr<DI, C, false, 8>();
    }
    return nullptr;
}

template <int DI, int C, bool Strict>
static const void *loop_px_k(int coarsen)
{
    switch (coarsen) {
    case 1: return (const void *)&k_loop_px<DI, C, Strict, 1>;
    case 2: return (const void *)&k_loop_px<DI, C, Strict, 2>;
    case 4: return (const void *)&k_loop_px<DI, C, Strict, 4>;
    case 8: return (const void *)&k_loop_px<DI, C, Strict, 8>;
    }
    return nullptr;
}

template <int DI, int C>
static const void *loop_px_s(int coarsen, int strict)
{
    return strict ? loop_px_k<DI, C, true>(coarsen) : loop_px_k<DI, C, false>(coarsen);
}

const void *kernel_loop_px(int in_dt, int channels, int coarsen, int strict)
{
    if (in_dt == DT_U8)
        return channels == 1 ? loop_px_s<DT_U8, 1>(coarsen, strict)
               : channels == 3 ? loop_px_s<DT_U8, 3>(coarsen, strict) : nullptr;
    if (in_dt == DT_F32)
        return channels == 1 ? loop_px_s<DT_F32, 1>(coarsen, strict)
               : channels == 3 ? loop_px_s<DT_F32, 3>(coarsen, strict) : nullptr;
    return nullptr;
}

const void *kernel_muladd_loop(int in_dt, int channels, int coarsen, int strict)
{
    if (in_dt == DT_U8)
        return channels == 1 ? loop_k<DT_U8, 1>(coarsen, strict)
               : channels == 3 ? loop_k<DT_U8, 3>(coarsen, strict) : nullptr;
    if (in_dt == DT_F32)
        return channels == 1 ? loop_k<DT_F32, 1>(coarsen, strict)
               : channels == 3 ? loop_k<DT_F32, 3>(coarsen, strict) : nullptr;
    return nullptr;
}

}  // namespace fk
