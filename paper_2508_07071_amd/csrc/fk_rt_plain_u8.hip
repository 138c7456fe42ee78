// fk_rt_plain_u8.hip -- run-time tier kernels: plain read of u8 frames.
#include "fk_rt_dispatch.hpp"

namespace fk {

template <int C>
using ReadPlainU8 = ReadPlain<DT_U8, C>;

const void *kernel_runtime_plain_u8(int channels, int out_dt, int layout, int coarsen)
{
    return RuntimeTable<ReadPlainU8, false, kChannels134>::get(channels, out_dt, layout, coarsen);
}

}  // namespace fk
