// fk_rt_nv12.hip -- run-time tier kernels: NV12 reads (1:1, and bilinear
// crop+resize with pixel-strided lanes for planar writes), three channels.
#include "fk_rt_dispatch.hpp"

namespace fk {

const void *kernel_runtime_nv12(int read_kind, int channels, int out_dt, int layout, int coarsen)
{
    if (read_kind == RD_NV12)
        return RuntimeTable<ReadNV12, false, kChannels3>::get(channels, out_dt, layout, coarsen);
    if (read_kind == RD_NV12_RESIZE)
        return RuntimeTable<ReadNV12Resize, true, kChannels3>::get(channels, out_dt, layout, coarsen);
    return nullptr;
}

}  // namespace fk
