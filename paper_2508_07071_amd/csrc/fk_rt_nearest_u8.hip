// fk_rt_nearest_u8.hip -- run-time tier kernels: nearest-neighbour crop+resize read of u8 frames.
#include "fk_rt_dispatch.hpp"

namespace fk {

template <int C>
using ReadCropNearestU8 = ReadCropNearest<DT_U8, C>;

const void *kernel_runtime_nearest_u8(int channels, int out_dt, int layout, int coarsen)
{
    return RuntimeTable<ReadCropNearestU8, false, kChannels134>::get(channels, out_dt, layout, coarsen);
}

}  // namespace fk
