// fk_rt_plain_f32.hip -- run-time tier kernels: plain read of f32 frames.
#include "fk_rt_dispatch.hpp"

namespace fk {

template <int C>
using ReadPlainF32 = ReadPlain<DT_F32, C>;

const void *kernel_runtime_plain_f32(int channels, int out_dt, int layout, int coarsen)
{
    return RuntimeTable<ReadPlainF32, false, kChannels134>::get(channels, out_dt, layout, coarsen);
}

}  // namespace fk
