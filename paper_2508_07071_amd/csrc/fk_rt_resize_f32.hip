// fk_rt_resize_f32.hip -- run-time tier kernels: bilinear crop+resize read of f32 frames
// (4-pixel units, and pixel-strided lanes for planar writes).
#include "fk_rt_dispatch.hpp"

namespace fk {

template <int C>
using ReadCropResizeF32 = ReadCropResize<DT_F32, C>;

const void *kernel_runtime_resize_f32(int channels, int out_dt, int layout, int coarsen)
{
    return RuntimeTable<ReadCropResizeF32, true, kChannels134>::get(channels, out_dt, layout, coarsen);
}

}  // namespace fk
