// fk_rt_resize_u8.hip -- run-time tier kernels: bilinear crop+resize read of u8 frames
// (4-pixel units, and pixel-strided lanes for planar writes).
#include "fk_rt_dispatch.hpp"

namespace fk {

template <int C>
using ReadCropResizeU8 = ReadCropResize<DT_U8, C>;

const void *kernel_runtime_resize_u8(int channels, int out_dt, int layout, int coarsen)
{
    return RuntimeTable<ReadCropResizeU8, true, kChannels134>::get(channels, out_dt, layout, coarsen);
}

}  // namespace fk
