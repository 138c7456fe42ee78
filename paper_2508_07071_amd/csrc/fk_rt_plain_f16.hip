// fk_rt_plain_f16.hip -- run-time tier kernels: plain read of f16 frames.
#include "fk_rt_dispatch.hpp"

namespace fk {

template <int C>
using ReadPlainF16 = ReadPlain<DT_F16, C>;

const void *kernel_runtime_plain_f16(int channels, int out_dt, int layout, int coarsen)
{
    return RuntimeTable<ReadPlainF16, false, kChannels134>::get(channels, out_dt, layout, coarsen);
}

}  // namespace fk
