// fk_stats_other.hip -- instantiations of the stats (reduction) kernel for
// the nearest-neighbour crop+resize read (u8, fp16, fp32 frames) and the
// NV12 reads (three channels).
#include "fk_device.hpp"

namespace fk {

template <class R, int C>
static const void *stats_k(int k)
{
    switch (k) {
    case 1: return (const void *)&k_stats<R, RuntimeCompute, C, 1>;
    case 2: return (const void *)&k_stats<R, RuntimeCompute, C, 2>;
    case 4: return (const void *)&k_stats<R, RuntimeCompute, C, 4>;
    case 8: return (const void *)&k_stats<R, RuntimeCompute, C, 8>;
    }
    return nullptr;
}

template <int DI>
static const void *nearest_c(int c, int k)
{
    switch (c) {
    case 1: return stats_k<ReadCropNearest<DI, 1>, 1>(k);
    case 3: return stats_k<ReadCropNearest<DI, 3>, 3>(k);
    case 4: return stats_k<ReadCropNearest<DI, 4>, 4>(k);
    }
    return nullptr;
}

const void *kernel_stats_other(int read_kind, int in_dt, int channels, int coarsen)
{
    if (read_kind == RD_CROP_NEAREST) {
        switch (in_dt) {
        case DT_U8: return nearest_c<DT_U8>(channels, coarsen);
        case DT_F16: return nearest_c<DT_F16>(channels, coarsen);
        case DT_F32: return nearest_c<DT_F32>(channels, coarsen);
        }
        return nullptr;
    }
    if (in_dt != DT_U8 || channels != 3)
        return nullptr;
    if (read_kind == RD_NV12)
        return stats_k<ReadNV12<3>, 3>(coarsen);
    if (read_kind == RD_NV12_RESIZE)
        return stats_k<ReadNV12Resize<3>, 3>(coarsen);
    return nullptr;
}

}  // namespace fk
