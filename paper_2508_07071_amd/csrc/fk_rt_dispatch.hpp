// fk_rt_dispatch.hpp -- the run-time tier's kernel table for one read op:
// the fused transform kernel with the run-time op list, for every channel
// count, output type, layout and coarsening.  Each read op and input type
// instantiates it in a translation unit of its own (fk_rt_*.hip), so that
// the kernels compile in parallel.
#pragma once
#include "fk_device.hpp"

namespace fk {

// Read: the read op as a template of the channel count.  Strided: the read
// also has the pixel-strided planar kernel (bilinear gathers, selected with
// LY_PLANAR_PX).  Channels: a bit mask of the channel counts built (bit c
// for c channels).
template <template <int> class Read, bool Strided, int Channels>
struct RuntimeTable {
    template <int C, int DO, int LY, int K>
    static const void *kernel()
    {
        if constexpr (LY == LY_PLANAR_PX)
            return (const void *)&k_resize_px<Read<C>, RuntimeCompute, DO, C, K>;
        else if constexpr (LY == LY_PLANAR)
            return (const void *)&k_transform<Read<C>, RuntimeCompute, WritePlanar<DO, C>, C, K>;
        else
            return (const void *)&k_transform<Read<C>, RuntimeCompute, WritePacked<DO, C>, C, K>;
    }

    template <int C, int DO, int LY>
    static const void *by_coarsening(int k)
    {
        switch (k) {
        case 1: return kernel<C, DO, LY, 1>();
        case 2: return kernel<C, DO, LY, 2>();
        case 4: return kernel<C, DO, LY, 4>();
        case 8: return kernel<C, DO, LY, 8>();
        }
        return nullptr;
    }

    template <int C, int DO>
    static const void *by_layout(int ly, int k)
    {
        if constexpr (Strided) {
            if (ly == LY_PLANAR_PX)
                return by_coarsening<C, DO, LY_PLANAR_PX>(k);
        }
        // a read without the strided kernel takes the 4-pixel-unit planar one
        if (ly == LY_PLANAR || ly == LY_PLANAR_PX)
            return by_coarsening<C, DO, LY_PLANAR>(k);
        return ly == LY_PACKED ? by_coarsening<C, DO, LY_PACKED>(k) : nullptr;
    }

    template <int C>
    static const void *by_output(int dout, int ly, int k)
    {
        if constexpr ((Channels >> C) & 1) {
            if (dout == DT_F16)
                return by_layout<C, DT_F16>(ly, k);
            if (dout == DT_F32)
                return by_layout<C, DT_F32>(ly, k);
        }
        return nullptr;
    }

    static const void *get(int channels, int dout, int ly, int k)
    {
        switch (channels) {
        case 1: return by_output<1>(dout, ly, k);
        case 3: return by_output<3>(dout, ly, k);
        case 4: return by_output<4>(dout, ly, k);
        }
        return nullptr;
    }
};

constexpr int kChannels134 = (1 << 1) | (1 << 3) | (1 << 4);
constexpr int kChannels3 = 1 << 3;

}  // namespace fk
