// fk_rt_nearest_f16.hip -- run-time tier kernels: nearest-neighbour crop+resize read of f16 frames.
#include "fk_rt_dispatch.hpp"

namespace fk {

template <int C>
using ReadCropNearestF16 = ReadCropNearest<DT_F16, C>;

const void *kernel_runtime_nearest_f16(int channels, int out_dt, int layout, int coarsen)
{
    return RuntimeTable<ReadCropNearestF16, false, kChannels134>::get(channels, out_dt, layout, coarsen);
}

}  // namespace fk
