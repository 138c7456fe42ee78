// fk_stats_plain.hip -- instantiations of the stats (reduction) kernel:
// run-time op list, plain read of u8, fp16 and fp32 frames; and the
// integer kernel for u8 frames with no arithmetic after the cast.
#include "fk_device.hpp"

namespace fk {

template <int DI, int C>
static const void *stats_k(int k)
{
    switch (k) {
    case 1: return (const void *)&k_stats<ReadPlain<DI, C>, RuntimeCompute, C, 1>;
    case 2: return (const void *)&k_stats<ReadPlain<DI, C>, RuntimeCompute, C, 2>;
    case 4: return (const void *)&k_stats<ReadPlain<DI, C>, RuntimeCompute, C, 4>;
    case 8: return (const void *)&k_stats<ReadPlain<DI, C>, RuntimeCompute, C, 8>;
    }
    return nullptr;
}

template <int DI>
static const void *stats_c(int c, int k)
{
    switch (c) {
    case 1: return stats_k<DI, 1>(k);
    case 3: return stats_k<DI, 3>(k);
    case 4: return stats_k<DI, 4>(k);
    }
    return nullptr;
}

const void *kernel_stats_plain(int in_dt, int channels, int coarsen)
{
    switch (in_dt) {
    case DT_U8: return stats_c<DT_U8>(channels, coarsen);
    case DT_F16: return stats_c<DT_F16>(channels, coarsen);
    case DT_F32: return stats_c<DT_F32>(channels, coarsen);
    }
    return nullptr;
}

template <int C>
static const void *stats_u8_k(int k)
{
    switch (k) {
    case 1: return (const void *)&k_stats_u8<C, 1>;
    case 2: return (const void *)&k_stats_u8<C, 2>;
    case 4: return (const void *)&k_stats_u8<C, 4>;
    case 8: return (const void *)&k_stats_u8<C, 8>;
    }
    return nullptr;
}

const void *kernel_stats_u8(int channels, int coarsen)
{
    switch (channels) {
    case 1: return stats_u8_k<1>(coarsen);
    case 3: return stats_u8_k<3>(coarsen);
    case 4: return stats_u8_k<4>(coarsen);
    }
    return nullptr;
}

}  // namespace fk
