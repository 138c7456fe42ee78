// fk_rt_nv12.hip -- instantiations of the fused transform kernel: run-time op list, NV12 reads (1:1 and bilinear resize), three channels.
#include "fk_device.hpp"

namespace fk {

template <int RK>
using NV12Read = typename std::conditional<RK == RD_NV12, ReadNV12<3>, ReadNV12Resize<3>>::type;
template <int DO, int LY>
using NV12Write = typename std::conditional<LY == LY_PLANAR, WritePlanar<DO, 3>, WritePacked<DO, 3>>::type;

template <int RK, int DO, int LY>
static const void *pick_k(int k)
{
    switch (k) {
    case 1: return (const void *)&k_transform<NV12Read<RK>, RuntimeCompute, NV12Write<DO, LY>, 3, 1>;
    case 2: return (const void *)&k_transform<NV12Read<RK>, RuntimeCompute, NV12Write<DO, LY>, 3, 2>;
    case 4: return (const void *)&k_transform<NV12Read<RK>, RuntimeCompute, NV12Write<DO, LY>, 3, 4>;
    case 8: return (const void *)&k_transform<NV12Read<RK>, RuntimeCompute, NV12Write<DO, LY>, 3, 8>;
    }
    return nullptr;
}
template <int RK, int DO>
static const void *pick_px(int k)
{
    switch (k) {
    case 1: return (const void *)&k_resize_px<NV12Read<RK>, RuntimeCompute, DO, 3, 1>;
    case 2: return (const void *)&k_resize_px<NV12Read<RK>, RuntimeCompute, DO, 3, 2>;
    case 4: return (const void *)&k_resize_px<NV12Read<RK>, RuntimeCompute, DO, 3, 4>;
    case 8: return (const void *)&k_resize_px<NV12Read<RK>, RuntimeCompute, DO, 3, 8>;
    }
    return nullptr;
}
template <int RK, int DO>
static const void *pick_ly(int ly, int k)
{
    if constexpr (RK == RD_NV12_RESIZE) {
        if (ly == LY_PLANAR_PX)
            return pick_px<RK, DO>(k);
    }
    return ly == LY_PLANAR ? pick_k<RK, DO, LY_PLANAR>(k) : pick_k<RK, DO, LY_PACKED>(k);
}
template <int RK>
static const void *pick_do(int dout, int ly, int k)
{
    return dout == DT_F16 ? pick_ly<RK, DT_F16>(ly, k) : pick_ly<RK, DT_F32>(ly, k);
}

const void *kernel_runtime_nv12(int read_kind, int channels, int out_dt, int layout, int coarsen)
{
    if (channels != 3)
        return nullptr;
    if (read_kind == RD_NV12)
        return pick_do<RD_NV12>(out_dt, layout, coarsen);
    if (read_kind == RD_NV12_RESIZE)
        return pick_do<RD_NV12_RESIZE>(out_dt, layout, coarsen);
    return nullptr;
}

}  // namespace fk
