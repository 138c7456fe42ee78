// fk_rt_nearest_f32.hip -- instantiations of the fused transform kernel: run-time op list, nearest-neighbour crop+resize of f32 frames.
#include "fk_device.hpp"

namespace fk {

template <int DO, int C, int LY>
using NearestWrite = typename std::conditional<LY == LY_PLANAR, WritePlanar<DO, C>, WritePacked<DO, C>>::type;

template <int C, int DO, int LY>
static const void *pick_k(int k)
{
    switch (k) {
    case 1: return (const void *)&k_transform<ReadCropNearest<DT_F32, C>, RuntimeCompute, NearestWrite<DO, C, LY>, C, 1>;
    case 2: return (const void *)&k_transform<ReadCropNearest<DT_F32, C>, RuntimeCompute, NearestWrite<DO, C, LY>, C, 2>;
    case 4: return (const void *)&k_transform<ReadCropNearest<DT_F32, C>, RuntimeCompute, NearestWrite<DO, C, LY>, C, 4>;
    case 8: return (const void *)&k_transform<ReadCropNearest<DT_F32, C>, RuntimeCompute, NearestWrite<DO, C, LY>, C, 8>;
    }
    return nullptr;
}
template <int C, int DO>
static const void *pick_ly(int ly, int k)
{
    return ly == LY_PLANAR ? pick_k<C, DO, LY_PLANAR>(k) : pick_k<C, DO, LY_PACKED>(k);
}
template <int C>
static const void *pick_do(int dout, int ly, int k)
{
    return dout == DT_F16 ? pick_ly<C, DT_F16>(ly, k) : pick_ly<C, DT_F32>(ly, k);
}

const void *kernel_runtime_nearest_f32(int channels, int out_dt, int layout, int coarsen)
{
    switch (channels) {
    case 1: return pick_do<1>(out_dt, layout, coarsen);
    case 3: return pick_do<3>(out_dt, layout, coarsen);
    case 4: return pick_do<4>(out_dt, layout, coarsen);
    }
    return nullptr;
}

}  // namespace fk
