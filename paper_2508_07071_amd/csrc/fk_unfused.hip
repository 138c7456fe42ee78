// fk_unfused.hip -- the unfused baseline: one kernel per operation and per
// item, every intermediate written to and read back from device memory
// (the separate-kernel pipeline of Section II's kernel-call algorithm and
// of the vertical-fusion figure, part A).  The ops run in chain order with
// per-op fp32 rounding, so the results equal the fused path's strict mode.
//
// Per item: [crop: 2-D copy of the ROI] -> [resize: bilinear to fp32] ->
// one elementwise kernel per compute op (swap, cvt, mul, add, sub, div) ->
// [write: packed or planar, fp32/fp16].  The last compute op writes the
// output directly when the write is packed fp32 (no extra copy).  A stats
// write instead runs one reduction per statistic over the fp32 image (min,
// max, sum, and mean as its own pass), as separate library calls would:
// each pass reads the whole image again.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "fk_device.hpp"
#include "fk_host.hpp"

namespace fk {

constexpr int kUnfusedBlock = 256;

template <int DT>
__device__ __forceinline__ float uload(const FK_GLOBAL uint8_t *p, int64_t e)
{
    return load_elem<DT>(p + e * DSize<DT>::v);
}

// Packed TIn image (contiguous w*h*C) -> packed fp32 resized image.
template <int DT>
__global__ __launch_bounds__(kUnfusedBlock) void k_resize(const uint8_t *src, int w, int h, int C,
                                                         float *dst, int ow, int oh, float sx,
                                                         float sy)
{
    const int64_t npix = (int64_t)ow * oh;
    gsrc_t s = (gsrc_t)src;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npix;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int oy = (int)(p / ow), ox = (int)(p - (int64_t)oy * ow);
        int y0, y1, x0, x1;
        float ay, ax;
        bilinear_coord(oy, sy, h, y0, y1, ay);
        bilinear_coord(ox, sx, w, x0, x1, ax);
        for (int c = 0; c < C; ++c) {
            const float p00 = uload<DT>(s, ((int64_t)y0 * w + x0) * C + c);
            const float p01 = uload<DT>(s, ((int64_t)y0 * w + x1) * C + c);
            const float p10 = uload<DT>(s, ((int64_t)y1 * w + x0) * C + c);
            const float p11 = uload<DT>(s, ((int64_t)y1 * w + x1) * C + c);
            const float top = fmaf(ax, p01 - p00, p00);
            const float bot = fmaf(ax, p11 - p10, p10);
            ((FK_GLOBAL float *)dst)[p * C + c] = fmaf(ay, bot - top, top);
        }
    }
}

// Packed TIn image (contiguous w*h*C) -> packed fp32 nearest-resized image:
// output o takes source floor((2o + 1) * in / (2 out)), exact in 64 bits.
template <int DT>
__global__ __launch_bounds__(kUnfusedBlock) void k_nearest(const uint8_t *src, int w, int h, int C,
                                                          float *dst, int ow, int oh)
{
    const int64_t npix = (int64_t)ow * oh;
    gsrc_t s = (gsrc_t)src;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npix;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int oy = (int)(p / ow), ox = (int)(p - (int64_t)oy * ow);
        const int64_t sy = (2 * (int64_t)oy + 1) * h / (2 * (int64_t)oh);
        const int64_t sx = (2 * (int64_t)ox + 1) * w / (2 * (int64_t)ow);
        for (int c = 0; c < C; ++c)
            ((FK_GLOBAL float *)dst)[p * C + c] = uload<DT>(s, (sy * w + sx) * C + c);
    }
}

// NV12 ROI -> packed fp32 B, G, R (the colour-conversion op of the
// unfused pipeline; the ROI's rows are read in place).
__global__ __launch_bounds__(kUnfusedBlock) void k_nv12(const uint8_t *frame, int64_t pitch,
                                                       int fh, int x, int y, int w, int h,
                                                       float *dst)
{
    const int64_t npix = (int64_t)w * h;
    gsrc_t base = (gsrc_t)frame;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npix;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(p / w), i = (int)(p - (int64_t)j * w);
        const int ax = x + i, ay = y + j;
        const float Y = load_elem<DT_U8>(base + (int64_t)ay * pitch + ax);
        gsrc_t uv = base + ((int64_t)fh + (ay >> 1)) * pitch + (ax & ~1);
        float o[3];
        nv12_to_bgr(Y, load_elem<DT_U8>(uv), load_elem<DT_U8>(uv + 1), o);
        for (int c = 0; c < 3; ++c)
            ((FK_GLOBAL float *)dst)[p * 3 + c] = o[c];
    }
}

// One elementwise op over a packed image of n elements: TIn -> fp32.
// code: -1 cvt (copy), OPC_MUL, OPC_ADD (SUB arrives as ADD of -k), OPC_DIV.
// (`reps` > 1: the op applied that many times in one kernel -- an op of
// `reps` instructions.)
template <int DT>
__global__ __launch_bounds__(kUnfusedBlock) void k_elem(const uint8_t *src, float *dst, int64_t n,
                                                       int C, int code, float k0, float k1, float k2,
                                                       float k3, int reps)
{
    gsrc_t s = (gsrc_t)src;
    FK_GLOBAL float *d = (FK_GLOBAL float *)dst;
    const float kk[4] = {k0, k1, k2, k3};
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        float r = uload<DT>(s, e);
        const float k = kk[(int)(e % C)];
        if (code == OPC_MUL) {
            for (int q = 0; q < reps; ++q)
                r = r * k;
        } else if (code == OPC_ADD) {
            for (int q = 0; q < reps; ++q)
                r = r + k;
        } else if (code == OPC_DIV) {
            for (int q = 0; q < reps; ++q)
                r = r / k;
        }
        d[e] = r;
    }
}

// The same op, four consecutive elements per thread: one 4/8/16-byte load,
// one 16-byte nontemporal store (n divisible by 4, buffers aligned).
template <int DT>
__global__ __launch_bounds__(kUnfusedBlock) void k_elem4(const uint8_t *src, float *dst, int64_t n4,
                                                        int C, int code, float k0, float k1,
                                                        float k2, float k3, int reps)
{
    const float kk[4] = {k0, k1, k2, k3};
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n4;
         q += (int64_t)gridDim.x * blockDim.x) {
        float v[4];
        if constexpr (DT == DT_U8) {
            const uint32_t w = ((const FK_GLOBAL uint32_t *)src)[q];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                v[t] = (float)((w >> (8 * t)) & 0xffu);
        } else if constexpr (DT == DT_F16) {
            const ux2 w = ((const FK_GLOBAL ux2 *)src)[q];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                v[t] = (float)__builtin_bit_cast(_Float16, (uint16_t)(w[t >> 1] >> (16 * (t & 1))));
        } else {
            const fx4 w = ((const FK_GLOBAL fx4 *)src)[q];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                v[t] = w[t];
        }
        int c = (int)((uint64_t)(4 * q) % (uint64_t)C);
        float kt[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            kt[t] = kk[c];
            c = c + 1 == C ? 0 : c + 1;
        }
        // the op's branch outside its repetitions (uniform across the grid)
        if (code == OPC_MUL) {
            for (int r = 0; r < reps; ++r)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    v[t] = v[t] * kt[t];
        } else if (code == OPC_ADD) {
            for (int r = 0; r < reps; ++r)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    v[t] = v[t] + kt[t];
        } else if (code == OPC_DIV) {
            for (int r = 0; r < reps; ++r)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    v[t] = v[t] / kt[t];
        }
        store_nt((gdst_t)(dst + 4 * q), fx4{v[0], v[1], v[2], v[3]});
    }
}

// ---- double-precision chains: the same ops on fp64 images ----

template <int DT>
__device__ __forceinline__ double uload_d(gsrc_t s, int64_t e)
{
    if constexpr (DT == DT_F64)
        return ((const FK_GLOBAL double *)s)[e];
    else
        return (double)uload<DT>(s, e);  // u8, fp16, fp32: exact
}

// One elementwise op in fp64 over a packed image of n elements: TIn -> fp64
// (code and reps as in k_elem; the constants are the ops' fp32 values).
template <int DT>
__global__ __launch_bounds__(kUnfusedBlock) void k_elem_d(const uint8_t *src, double *dst, int64_t n,
                                                         int C, int code, double k0, double k1,
                                                         double k2, double k3, int reps)
{
    gsrc_t s = (gsrc_t)src;
    FK_GLOBAL double *d = (FK_GLOBAL double *)dst;
    const double kk[4] = {k0, k1, k2, k3};
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        double r = uload_d<DT>(s, e);
        const double k = kk[(int)(e % C)];
        if (code == OPC_MUL) {
            for (int q = 0; q < reps; ++q)
                r = r * k;
        } else if (code == OPC_ADD) {
            for (int q = 0; q < reps; ++q)
                r = r + k;
        } else if (code == OPC_DIV) {
            for (int q = 0; q < reps; ++q)
                r = r / k;
        }
        d[e] = r;
    }
}

// BGR <-> RGB in fp64: TIn -> fp64.
template <int DT>
__global__ __launch_bounds__(kUnfusedBlock) void k_swap_d(const uint8_t *src, double *dst,
                                                         int64_t npix, int C)
{
    gsrc_t s = (gsrc_t)src;
    FK_GLOBAL double *d = (FK_GLOBAL double *)dst;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npix;
         p += (int64_t)gridDim.x * blockDim.x) {
        for (int c = 0; c < C; ++c) {
            const int sc = (C >= 3 && c != 1 && c != 3) ? 2 - c : c;
            d[p * C + c] = uload_d<DT>(s, p * C + sc);
        }
    }
}

// Final fp64 write: packed TIn image -> fp64, packed or planar.
template <int DT>
__global__ __launch_bounds__(kUnfusedBlock) void k_write_d(const uint8_t *src, double *dst,
                                                          int64_t npix, int C, int planar)
{
    gsrc_t s = (gsrc_t)src;
    FK_GLOBAL double *d = (FK_GLOBAL double *)dst;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npix;
         p += (int64_t)gridDim.x * blockDim.x) {
        for (int c = 0; c < C; ++c) {
            const int64_t o = planar ? (int64_t)c * npix + p : p * C + c;
            d[o] = uload_d<DT>(s, p * C + c);
        }
    }
}

// BGR <-> RGB over a packed image of npix pixels: TIn -> fp32.
template <int DT>
__global__ __launch_bounds__(kUnfusedBlock) void k_swap(const uint8_t *src, float *dst,
                                                       int64_t npix, int C)
{
    gsrc_t s = (gsrc_t)src;
    FK_GLOBAL float *d = (FK_GLOBAL float *)dst;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npix;
         p += (int64_t)gridDim.x * blockDim.x) {
        for (int c = 0; c < C; ++c) {
            const int sc = (C >= 3 && c != 1 && c != 3) ? 2 - c : c;
            d[p * C + c] = uload<DT>(s, p * C + sc);
        }
    }
}

// Final write: packed TIn image -> output dtype, packed or planar (Split).
template <int DT, int DTO>
__global__ __launch_bounds__(kUnfusedBlock) void k_write(const uint8_t *src, uint8_t *dst,
                                                        int64_t npix, int C, int planar)
{
    gsrc_t s = (gsrc_t)src;
    gdst_t d = (gdst_t)dst;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npix;
         p += (int64_t)gridDim.x * blockDim.x) {
        for (int c = 0; c < C; ++c) {
            const float v = uload<DT>(s, p * C + c);
            const int64_t o = planar ? (int64_t)c * npix + p : p * C + c;
            store_elem<DTO>(d + o * DSize<DTO>::v, v);
        }
    }
}

// One statistic over a packed fp32 image, stage 1: block g reduces the
// pixels g*T + t, g*T + t + G*T, ... (fixed order) into part[g][c].
enum : int { RED_MIN = 0, RED_MAX = 1, RED_SUM = 2, RED_MEAN = 3 };
constexpr int kRedBlocks = 256;

template <int OP>
__device__ __forceinline__ double red_op(double a, double b)
{
    if constexpr (OP == RED_MIN)
        return fmin(a, b);
    else if constexpr (OP == RED_MAX)
        return fmax(a, b);
    else
        return a + b;
}

template <int OP>
__device__ __forceinline__ double red_init()
{
    if constexpr (OP == RED_MIN)
        return __builtin_inf();
    else if constexpr (OP == RED_MAX)
        return -__builtin_inf();
    else
        return 0.0;
}

// Block-wide reduction of one value per channel in a fixed tree; thread 0
// gets the result.
template <int OP>
__device__ __forceinline__ void red_block(double (&acc)[4], int C, double (*lds)[4])
{
    const int tid = threadIdx.x;
    for (int c = 0; c < C; ++c)
        lds[tid][c] = acc[c];
    __syncthreads();
    for (int s = kUnfusedBlock / 2; s >= 1; s >>= 1) {
        if (tid < s)
            for (int c = 0; c < C; ++c)
                lds[tid][c] = red_op<OP>(lds[tid][c], lds[tid + s][c]);
        __syncthreads();
    }
    for (int c = 0; c < C; ++c)
        acc[c] = lds[0][c];
}

template <int OP>
__global__ __launch_bounds__(kUnfusedBlock) void k_red_partial(const float *src, int64_t npix,
                                                              int C, double *part)
{
    __shared__ double lds[kUnfusedBlock][4];
    double acc[4];
    for (int c = 0; c < 4; ++c)
        acc[c] = red_init<OP>();
    const FK_GLOBAL float *s = (const FK_GLOBAL float *)src;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npix;
         p += (int64_t)gridDim.x * blockDim.x)
        for (int c = 0; c < C; ++c) {
            const float v = s[p * C + c];
            if constexpr (OP == RED_MIN)
                acc[c] = (double)fminf((float)acc[c], v);
            else if constexpr (OP == RED_MAX)
                acc[c] = (double)fmaxf((float)acc[c], v);
            else
                acc[c] += (double)v;
        }
    red_block<OP>(acc, C, lds);
    if (threadIdx.x == 0)
        for (int c = 0; c < C; ++c)
            part[(int64_t)blockIdx.x * 4 + c] = acc[c];
}

// Stage 2: one block combines the G partials; dst[4c + OP] = the statistic.
template <int OP>
__global__ __launch_bounds__(kUnfusedBlock) void k_red_final(const double *part, int G, int C,
                                                            double *dst, double npix)
{
    __shared__ double lds[kUnfusedBlock][4];
    double acc[4];
    for (int c = 0; c < 4; ++c)
        acc[c] = red_init<OP>();
    for (int g = threadIdx.x; g < G; g += blockDim.x)
        for (int c = 0; c < C; ++c)
            acc[c] = red_op<OP>(acc[c], part[(int64_t)g * 4 + c]);
    red_block<OP>(acc, C, lds);
    if (threadIdx.x == 0)
        for (int c = 0; c < C; ++c)
            dst[4 * c + OP] = OP == RED_MEAN ? acc[c] / npix : acc[c];
}

template <int OP>
static void stat_pass(const float *img, int64_t npix, int C, double *part, double *dst,
                      hipStream_t st)
{
    constexpr int K = OP == RED_MEAN ? RED_SUM : OP;
    const int G = (int)std::max<int64_t>(
        1, std::min<int64_t>(kRedBlocks, (npix + kUnfusedBlock - 1) / kUnfusedBlock));
    k_red_partial<K><<<G, kUnfusedBlock, 0, st>>>(img, npix, C, part);
    k_red_final<OP><<<1, kUnfusedBlock, 0, st>>>(part, G, C, dst, (double)npix);
}

static unsigned grid_for(int64_t n)
{
    const int64_t g = (n + kUnfusedBlock - 1) / kUnfusedBlock;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 1 << 16));
}

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

struct ScratchPlan {
    size_t crop = 0, buf = 0, part = 0;
    size_t total() const { return align_up(crop) + 2 * align_up(buf) + align_up(part); }
};

static ScratchPlan scratch_for(const fk_plan *p, const fk_item &it)
{
    const int C = p->chain.read.channels;
    const int es = dtype_size(p->chain.read.in_dtype);
    ScratchPlan s;
    s.crop = (size_t)it.w * it.h * C * es;
    size_t npix = (size_t)it.w * it.h;
    if (rd_resizes(p->chain.read.kind))
        npix = std::max(npix, (size_t)it.out_w * it.out_h);
    // intermediates hold the running value: fp64 for a double-precision chain
    s.buf = npix * C * (p->family == FAM_F64 ? sizeof(double) : sizeof(float));
    if (p->chain.write.layout == FK_STATS)
        s.part = (size_t)kRedBlocks * 4 * sizeof(double);
    return s;
}

template <int DT>
static void launch_elem(const void *src, float *dst, int64_t n, int C, int code, const float *k,
                        int reps, hipStream_t st)
{
    const uintptr_t need = DT == DT_U8 ? 4 : DT == DT_F16 ? 8 : 16;
    if (n % 4 == 0 && (uintptr_t)src % need == 0 && (uintptr_t)dst % 16 == 0) {
        k_elem4<DT><<<grid_for(n / 4), kUnfusedBlock, 0, st>>>((const uint8_t *)src, dst, n / 4, C,
                                                              code, k[0], k[1], k[2], k[3], reps);
        return;
    }
    k_elem<DT><<<grid_for(n), kUnfusedBlock, 0, st>>>((const uint8_t *)src, dst, n, C, code, k[0],
                                                      k[1], k[2], k[3], reps);
}

static void elem_any(int dt, const void *src, float *dst, int64_t n, int C, int code,
                     const float *k, int reps, hipStream_t st)
{
    if (dt == DT_U8)
        launch_elem<DT_U8>(src, dst, n, C, code, k, reps, st);
    else if (dt == DT_F16)
        launch_elem<DT_F16>(src, dst, n, C, code, k, reps, st);
    else
        launch_elem<DT_F32>(src, dst, n, C, code, k, reps, st);
}

static void swap_any(int dt, const void *src, float *dst, int64_t npix, int C, hipStream_t st)
{
    const unsigned g = grid_for(npix);
    if (dt == DT_U8)
        k_swap<DT_U8><<<g, kUnfusedBlock, 0, st>>>((const uint8_t *)src, dst, npix, C);
    else if (dt == DT_F16)
        k_swap<DT_F16><<<g, kUnfusedBlock, 0, st>>>((const uint8_t *)src, dst, npix, C);
    else
        k_swap<DT_F32><<<g, kUnfusedBlock, 0, st>>>((const uint8_t *)src, dst, npix, C);
}

template <int DTO>
static void write_out(int dt, const void *src, void *dst, int64_t npix, int C, int planar,
                      hipStream_t st)
{
    const unsigned g = grid_for(npix);
    if (dt == DT_U8)
        k_write<DT_U8, DTO><<<g, kUnfusedBlock, 0, st>>>((const uint8_t *)src, (uint8_t *)dst, npix, C, planar);
    else if (dt == DT_F16)
        k_write<DT_F16, DTO><<<g, kUnfusedBlock, 0, st>>>((const uint8_t *)src, (uint8_t *)dst, npix, C, planar);
    else
        k_write<DT_F32, DTO><<<g, kUnfusedBlock, 0, st>>>((const uint8_t *)src, (uint8_t *)dst, npix, C, planar);
}

// One kernel per op as the chain executes: a loop's body once per run; with
// unfused_loop_kernel, a loop over one op is that op's kernel applying it
// loop_count times.  seq[s] = op index, reps[s] = applications in its kernel.
static void op_sequence(const fk_plan *p, std::vector<int> &seq, std::vector<int> &reps)
{
    const int C = p->chain.read.channels;
    for (int i = 0; i < p->chain.n_ops; ++i) {
        const fk_op_desc &d = p->chain.ops[i];
        if (d.kind == FK_OP_LOOP) {
            if (p->opts.unfused_loop_kernel && d.loop_span == 1) {
                reps.back() = d.loop_count;  // the body: the entry just pushed
                continue;
            }
            for (int r = 1; r < d.loop_count; ++r)
                for (int j = i - d.loop_span; j < i; ++j) {
                    seq.push_back(j);
                    reps.push_back(1);
                }
        } else if (d.kind != FK_OP_SWAP_RB || C >= 3) {  // a 1-channel swap is no kernel
            seq.push_back(i);
            reps.push_back(1);
        }
    }
}

// Kernel code and per-channel constants of an arithmetic op (SUB as ADD of
// the negated constant: exact).
static int op_code(const fk_op_desc &d, int C, float (&k)[4])
{
    for (int c = 0; c < 4; ++c)
        k[c] = d.n_consts == 1 ? d.consts[0] : (c < C ? d.consts[c] : 0.0f);
    if (d.kind == FK_OP_MUL)
        return OPC_MUL;
    if (d.kind == FK_OP_ADD)
        return OPC_ADD;
    if (d.kind == FK_OP_SUB) {
        for (int c = 0; c < 4; ++c)
            k[c] = -k[c];
        return OPC_ADD;
    }
    if (d.kind == FK_OP_DIV)
        return OPC_DIV;
    return -1;
}

static void elem_d(int dt, const void *src, double *dst, int64_t n, int C, int code,
                   const float (&k)[4], int reps, hipStream_t st)
{
    const unsigned g = grid_for(n);
    const uint8_t *s = (const uint8_t *)src;
    const double k0 = k[0], k1 = k[1], k2 = k[2], k3 = k[3];
    switch (dt) {
    case DT_U8: k_elem_d<DT_U8><<<g, kUnfusedBlock, 0, st>>>(s, dst, n, C, code, k0, k1, k2, k3, reps); break;
    case DT_F16: k_elem_d<DT_F16><<<g, kUnfusedBlock, 0, st>>>(s, dst, n, C, code, k0, k1, k2, k3, reps); break;
    case DT_F32: k_elem_d<DT_F32><<<g, kUnfusedBlock, 0, st>>>(s, dst, n, C, code, k0, k1, k2, k3, reps); break;
    default: k_elem_d<DT_F64><<<g, kUnfusedBlock, 0, st>>>(s, dst, n, C, code, k0, k1, k2, k3, reps); break;
    }
}

static void swap_d(int dt, const void *src, double *dst, int64_t npix, int C, hipStream_t st)
{
    const unsigned g = grid_for(npix);
    const uint8_t *s = (const uint8_t *)src;
    switch (dt) {
    case DT_U8: k_swap_d<DT_U8><<<g, kUnfusedBlock, 0, st>>>(s, dst, npix, C); break;
    case DT_F16: k_swap_d<DT_F16><<<g, kUnfusedBlock, 0, st>>>(s, dst, npix, C); break;
    case DT_F32: k_swap_d<DT_F32><<<g, kUnfusedBlock, 0, st>>>(s, dst, npix, C); break;
    default: k_swap_d<DT_F64><<<g, kUnfusedBlock, 0, st>>>(s, dst, npix, C); break;
    }
}

static void write_d(int dt, const void *src, double *dst, int64_t npix, int C, int planar,
                    hipStream_t st)
{
    const unsigned g = grid_for(npix);
    const uint8_t *s = (const uint8_t *)src;
    switch (dt) {
    case DT_U8: k_write_d<DT_U8><<<g, kUnfusedBlock, 0, st>>>(s, dst, npix, C, planar); break;
    case DT_F16: k_write_d<DT_F16><<<g, kUnfusedBlock, 0, st>>>(s, dst, npix, C, planar); break;
    case DT_F32: k_write_d<DT_F32><<<g, kUnfusedBlock, 0, st>>>(s, dst, npix, C, planar); break;
    default: k_write_d<DT_F64><<<g, kUnfusedBlock, 0, st>>>(s, dst, npix, C, planar); break;
    }
}

// A double-precision chain (plain read, fp64 write): the ROI in place when
// its rows are contiguous (else one 2-D copy), one kernel per op writing an
// fp64 image, and the fp64 write (the last op writes a packed output
// directly).
static fk_status run_item_unfused_f64(const fk_plan *p, const fk_item &it, uint8_t *ws,
                                      hipStream_t st)
{
    const int C = p->chain.read.channels;
    const int din = p->chain.read.in_dtype;
    const int es = dtype_size(din);
    const ScratchPlan sp = scratch_for(p, it);
    double *buf[2] = {(double *)(ws + align_up(sp.crop)),
                      (double *)(ws + align_up(sp.crop) + align_up(sp.buf))};
    const uint8_t *roi = (const uint8_t *)it.src.ptr + (int64_t)it.y * it.src.pitch_bytes +
                         (int64_t)it.x * C * es;
    const size_t row_bytes = (size_t)it.w * C * es;
    const void *cur = roi;
    if ((size_t)it.src.pitch_bytes != row_bytes && it.h > 1) {
        hipError_t e = hipMemcpy2DAsync(ws, row_bytes, roi, it.src.pitch_bytes, row_bytes, it.h,
                                        hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess)
            return hip_error(e, "crop copy");
        cur = ws;
    }
    int cur_dt = din;
    int nb = 0;
    const int64_t npix = (int64_t)it.w * it.h;
    const bool direct = p->chain.write.layout == FK_PACKED;
    std::vector<int> seq, reps;
    op_sequence(p, seq, reps);
    for (size_t s = 0; s < seq.size(); ++s) {
        const fk_op_desc &d = p->chain.ops[seq[s]];
        double *o = (direct && s + 1 == seq.size()) ? (double *)it.dst : buf[nb];
        if (o != (double *)it.dst)
            nb ^= 1;
        if (d.kind == FK_OP_SWAP_RB) {
            swap_d(cur_dt, cur, o, npix, C, st);
        } else {
            float k[4];
            const int code = op_code(d, C, k);
            elem_d(cur_dt, cur, o, npix * C, C, code, k, reps[s], st);
        }
        cur = o;
        cur_dt = DT_F64;
    }
    if (!(direct && !seq.empty()))
        write_d(cur_dt, cur, (double *)it.dst, npix, C, p->chain.write.layout == FK_PLANAR, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_error(e, "unfused launch");
    return FK_OK;
}

static fk_status run_item_unfused(const fk_plan *p, const fk_item &it, uint8_t *ws,
                                  hipStream_t st)
{
    if (p->family == FAM_F64)
        return run_item_unfused_f64(p, it, ws, st);
    const int C = p->chain.read.channels;
    const int din = p->chain.read.in_dtype;
    const int es = dtype_size(din);
    const ScratchPlan sp = scratch_for(p, it);
    uint8_t *crop = ws;
    float *buf[2] = {(float *)(ws + align_up(sp.crop)),
                     (float *)(ws + align_up(sp.crop) + align_up(sp.buf))};
    const uint8_t *roi = (const uint8_t *)it.src.ptr + (int64_t)it.y * it.src.pitch_bytes +
                         (int64_t)it.x * C * es;
    const size_t row_bytes = (size_t)it.w * C * es;
    const void *cur = nullptr;
    int cur_dt = din;
    int nb = 0;  // next ping-pong buffer
    int64_t npix = (int64_t)it.w * it.h;
    hipError_t e = hipSuccess;

    const bool contiguous = (size_t)it.src.pitch_bytes == row_bytes ||
                            (it.h == 1);
    const int rk = p->chain.read.kind;
    if (rk == FK_READ_NV12 || rk == FK_READ_NV12_RESIZE) {
        // crop + colour conversion to fp32 BGR in one pass
        float *o = buf[nb];
        nb ^= 1;
        k_nv12<<<grid_for(npix), kUnfusedBlock, 0, st>>>((const uint8_t *)it.src.ptr,
                                                         it.src.pitch_bytes, it.src.height, it.x,
                                                         it.y, it.w, it.h, o);
        cur = o;
        cur_dt = DT_F32;
    } else if (rk == FK_READ_PLAIN && contiguous) {
        cur = roi;  // the ROI already is a dense image: no crop kernel
    } else {
        e = hipMemcpy2DAsync(crop, row_bytes, roi, it.src.pitch_bytes, row_bytes, it.h,
                             hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess)
            return hip_error(e, "crop copy");
        cur = crop;
    }
    if (rk == FK_READ_CROP_NEAREST) {
        npix = (int64_t)it.out_w * it.out_h;
        float *o = buf[nb];
        nb ^= 1;
        const unsigned g = grid_for(npix);
        if (din == DT_U8)
            k_nearest<DT_U8><<<g, kUnfusedBlock, 0, st>>>((const uint8_t *)cur, it.w, it.h, C, o, it.out_w, it.out_h);
        else if (din == DT_F16)
            k_nearest<DT_F16><<<g, kUnfusedBlock, 0, st>>>((const uint8_t *)cur, it.w, it.h, C, o, it.out_w, it.out_h);
        else
            k_nearest<DT_F32><<<g, kUnfusedBlock, 0, st>>>((const uint8_t *)cur, it.w, it.h, C, o, it.out_w, it.out_h);
        cur = o;
        cur_dt = DT_F32;
    }
    if (rk == FK_READ_CROP_RESIZE || rk == FK_READ_NV12_RESIZE) {
        const float sx = (float)it.w / (float)it.out_w, sy = (float)it.h / (float)it.out_h;
        npix = (int64_t)it.out_w * it.out_h;
        float *o = buf[nb];
        nb ^= 1;
        const unsigned g = grid_for(npix);
        if (cur_dt == DT_U8)
            k_resize<DT_U8><<<g, kUnfusedBlock, 0, st>>>((const uint8_t *)cur, it.w, it.h, C, o, it.out_w, it.out_h, sx, sy);
        else if (cur_dt == DT_F16)
            k_resize<DT_F16><<<g, kUnfusedBlock, 0, st>>>((const uint8_t *)cur, it.w, it.h, C, o, it.out_w, it.out_h, sx, sy);
        else
            k_resize<DT_F32><<<g, kUnfusedBlock, 0, st>>>((const uint8_t *)cur, it.w, it.h, C, o, it.out_w, it.out_h, sx, sy);
        cur = o;
        cur_dt = DT_F32;
    }
    const bool direct = p->chain.write.layout == FK_PACKED && p->chain.write.out_dtype == FK_F32;
    std::vector<int> seq, reps;
    op_sequence(p, seq, reps);
    for (size_t s = 0; s < seq.size(); ++s) {
        const fk_op_desc &d = p->chain.ops[seq[s]];
        const bool last = s + 1 == seq.size();
        float *o = (direct && last) ? (float *)it.dst : buf[nb];
        if (o != (float *)it.dst)
            nb ^= 1;
        if (d.kind == FK_OP_SWAP_RB) {
            swap_any(cur_dt, cur, o, npix, C, st);
        } else {
            float k[4];
            const int code = op_code(d, C, k);
            elem_any(cur_dt, cur, o, npix * C, C, code, k, reps[s], st);
        }
        cur = o;
        cur_dt = DT_F32;
    }
    if (p->chain.write.layout == FK_STATS) {
        if (cur_dt != DT_F32) {  // no arithmetic op ran: make the fp32 image
            float *o = buf[nb];
            write_out<DT_F32>(cur_dt, cur, o, npix, C, 0, st);
            cur = o;
        }
        const float *img = (const float *)cur;
        double *part = (double *)(ws + align_up(sp.crop) + 2 * align_up(sp.buf));
        double *out = (double *)it.dst;
        stat_pass<RED_MIN>(img, npix, C, part, out, st);
        stat_pass<RED_MAX>(img, npix, C, part, out, st);
        stat_pass<RED_SUM>(img, npix, C, part, out, st);
        stat_pass<RED_MEAN>(img, npix, C, part, out, st);
    } else if (!(direct && !seq.empty())) {
        const int planar = p->chain.write.layout == FK_PLANAR;
        if (p->chain.write.out_dtype == FK_F16)
            write_out<DT_F16>(cur_dt, cur, it.dst, npix, C, planar, st);
        else
            write_out<DT_F32>(cur_dt, cur, it.dst, npix, C, planar, st);
    }
    e = hipGetLastError();
    if (e != hipSuccess)
        return hip_error(e, "unfused launch");
    return FK_OK;
}

}  // namespace fk

using namespace fk;

extern "C" fk_status fk_unfused_scratch_bytes(const fk_plan *plan, const fk_item *items,
                                              int32_t n_items, int64_t *bytes)
{
    try {
        if (!plan || !bytes)
            return set_error(FK_ERR_INVALID_ARG, "null argument");
        fk_status s = validate_items(&plan->chain, items, n_items);
        if (s)
            return s;
        size_t need = 0;
        for (int32_t b = 0; b < n_items; ++b)
            need = std::max(need, scratch_for(plan, items[b]).total());
        *bytes = (int64_t)need;
        return FK_OK;
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

// Checks shared by both unfused entries; the workspace bytes the items
// need go to `need`.
static fk_status check_unfused(const fk_plan *plan, const fk_item *items, int32_t n_items,
                               int64_t *need)
{
    if (!plan)
        return set_error(FK_ERR_INVALID_ARG, "plan is null");
    if (n_items < 1 || n_items > plan->max_batch)
        return set_error(FK_ERR_INVALID_ARG, "n_items outside 1..max_batch");
    fk_status s = validate_items(&plan->chain, items, n_items);
    if (s)
        return s;
    *need = 0;
    for (int32_t b = 0; b < n_items; ++b)
        *need = std::max<int64_t>(*need, (int64_t)scratch_for(plan, items[b]).total());
    return FK_OK;
}

// The items one after another, each in the whole workspace (stream order
// keeps an item's kernels after the previous item's).
static fk_status run_unfused_items(const fk_plan *plan, const fk_item *items, int32_t n_items,
                                   uint8_t *ws, hipStream_t stream)
{
    for (int32_t b = 0; b < n_items; ++b) {
        fk_status s = run_item_unfused(plan, items[b], ws, stream);
        if (s)
            return s;
    }
    return FK_OK;
}

extern "C" fk_status fk_run_unfused(fk_plan *plan, const fk_item *items, int32_t n_items,
                                    void *d_scratch, int64_t scratch_bytes, void *stream)
{
    try {
        int64_t need = 0;
        fk_status s = check_unfused(plan, items, n_items, &need);
        if (s)
            return s;
        if (!d_scratch || scratch_bytes < need)
            return set_error(FK_ERR_INVALID_ARG, "scratch too small: %lld < %lld bytes",
                             (long long)scratch_bytes, (long long)need);
        return run_unfused_items(plan, items, n_items, (uint8_t *)d_scratch, (hipStream_t)stream);
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

// ------------------------------------------------ no-allocation variant --

// Workspace of fk_run_unfused_noalloc: one copy per device, loaded with the
// code object and held until the process ends.  Host code never passes the
// array's name to a kernel or a copy (on the host it only names the
// symbol); it uses the device address that hipGetSymbolAddress gives for
// the current device.  Nothing in it has to start at zero: every
// intermediate is written whole before it is read.
static __device__ __align__(256) uint8_t scratch[FK_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices];  // device address of `scratch`, per device
}  // namespace

// The array's address on the current device, looked up on the first call
// on that device.
static fk_status scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(FK_ERR_UNSUPPORTED, "device %d beyond the %d the workspace table holds",
                         dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!ptr)
            return set_error(FK_ERR_HIP, "hipGetSymbolAddress(scratch) gave a null address");
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return FK_OK;
}

extern "C" fk_status fk_run_unfused_noalloc(fk_plan *plan, const fk_item *items, int32_t n_items,
                                            void *stream)
{
    try {
        int64_t need = 0;
        fk_status s = check_unfused(plan, items, n_items, &need);
        if (s)
            return s;
        if (need > (int64_t)FK_NOALLOC_SCRATCH_BYTES)
            return set_error(FK_ERR_UNSUPPORTED,
                             "the items need %lld bytes of workspace; the no-allocation entry "
                             "holds %lld",
                             (long long)need, (long long)FK_NOALLOC_SCRATCH_BYTES);
        void *ws = nullptr;
        s = scratch_address(&ws);
        if (s)
            return s;
        return run_unfused_items(plan, items, n_items, (uint8_t *)ws, (hipStream_t)stream);
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}
