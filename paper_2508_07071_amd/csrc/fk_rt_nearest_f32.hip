// fk_rt_nearest_f32.hip -- run-time tier kernels: nearest-neighbour crop+resize read of f32 frames.
#include "fk_rt_dispatch.hpp"

namespace fk {

template <int C>
using ReadCropNearestF32 = ReadCropNearest<DT_F32, C>;

const void *kernel_runtime_nearest_f32(int channels, int out_dt, int layout, int coarsen)
{
    return RuntimeTable<ReadCropNearestF32, false, kChannels134>::get(channels, out_dt, layout, coarsen);
}

}  // namespace fk
