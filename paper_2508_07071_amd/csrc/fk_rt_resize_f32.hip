// fk_rt_resize_f32.hip -- instantiations of the fused transform kernel: run-time op list, resize read of f32 frames
// (4-pixel units, and pixel-strided lanes for planar writes).
#include "fk_device.hpp"

namespace fk {

template <int RK, int DI, int C>
using ReadOf = typename std::conditional<RK == RD_PLAIN, ReadPlain<DI, C>, ReadCropResize<DI, C>>::type;
template <int DO, int C, int LY>
using WriteOf = typename std::conditional<LY == LY_PLANAR, WritePlanar<DO, C>, WritePacked<DO, C>>::type;

template <int RK, int DI, int C, int DO, int LY>
static const void *pick_k(int k)
{
    switch (k) {
    case 1: return (const void *)&k_transform<ReadOf<RK, DI, C>, RuntimeCompute, WriteOf<DO, C, LY>, C, 1>;
    case 2: return (const void *)&k_transform<ReadOf<RK, DI, C>, RuntimeCompute, WriteOf<DO, C, LY>, C, 2>;
    case 4: return (const void *)&k_transform<ReadOf<RK, DI, C>, RuntimeCompute, WriteOf<DO, C, LY>, C, 4>;
    case 8: return (const void *)&k_transform<ReadOf<RK, DI, C>, RuntimeCompute, WriteOf<DO, C, LY>, C, 8>;
    }
    return nullptr;
}
template <int RK, int DI, int C, int DO>
static const void *pick_px(int k)
{
    switch (k) {
    case 1: return (const void *)&k_resize_px<ReadCropResize<DI, C>, RuntimeCompute, DO, C, 1>;
    case 2: return (const void *)&k_resize_px<ReadCropResize<DI, C>, RuntimeCompute, DO, C, 2>;
    case 4: return (const void *)&k_resize_px<ReadCropResize<DI, C>, RuntimeCompute, DO, C, 4>;
    case 8: return (const void *)&k_resize_px<ReadCropResize<DI, C>, RuntimeCompute, DO, C, 8>;
    }
    return nullptr;
}
template <int RK, int DI, int C, int DO>
static const void *pick_ly(int ly, int k)
{
    if (ly == LY_PLANAR_PX)
        return pick_px<RK, DI, C, DO>(k);
    return ly == LY_PLANAR ? pick_k<RK, DI, C, DO, LY_PLANAR>(k) : pick_k<RK, DI, C, DO, LY_PACKED>(k);
}
template <int RK, int DI, int C>
static const void *pick_do(int dout, int ly, int k)
{
    return dout == DT_F16 ? pick_ly<RK, DI, C, DT_F16>(ly, k) : pick_ly<RK, DI, C, DT_F32>(ly, k);
}
template <int RK, int DI>
static const void *pick_c(int c, int dout, int ly, int k)
{
    switch (c) {
    case 1: return pick_do<RK, DI, 1>(dout, ly, k);
    case 3: return pick_do<RK, DI, 3>(dout, ly, k);
    case 4: return pick_do<RK, DI, 4>(dout, ly, k);
    }
    return nullptr;
}

const void *kernel_runtime_resize_f32(int channels, int out_dt, int layout, int coarsen)
{
    return pick_c<RD_CROP_RESIZE, DT_F32>(channels, out_dt, layout, coarsen);
}

}  // namespace fk
