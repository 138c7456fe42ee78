// fk_rt_resize_f16.hip -- run-time tier kernels: bilinear crop+resize read of f16 frames
// (4-pixel units, and pixel-strided lanes for planar writes).
#include "fk_rt_dispatch.hpp"

namespace fk {

template <int C>
using ReadCropResizeF16 = ReadCropResize<DT_F16, C>;

const void *kernel_runtime_resize_f16(int channels, int out_dt, int layout, int coarsen)
{
    return RuntimeTable<ReadCropResizeF16, true, kChannels134>::get(channels, out_dt, layout, coarsen);
}

}  // namespace fk
