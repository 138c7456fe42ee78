// fk_model.cpp -- the launch-configuration cost model: features of a
// (plan, items) pair, a ReLU network trained and evaluated on the GPU with
// the kernels of fk_mlp.hip, and its use to pick a plan's launch config.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fk.h"
#include "fk_host.hpp"
#include "fk_internal.hpp"
#include "fk_mlp.hpp"

using namespace fk;

namespace {

constexpr int F = FK_MODEL_FEATURES;
constexpr int O = FK_MODEL_OUTPUTS;
constexpr int kLayers = 4;  // F -> H -> H -> H -> O

// SplitMix64 (Steele, Lea and Flood, 2014): seeded host-side random numbers
// for weight initialisation and mini-batch shuffling.
uint64_t splitmix(uint64_t &s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
double uniform01(uint64_t &s) { return (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0); }

}  // namespace

struct fk_model {
    int H = 128;
    int dims[kLayers + 1] = {F, 128, 128, 128, O};
    int64_t w_off[kLayers] = {}, b_off[kLayers] = {};
    int64_t n_params = 0;
    float *d_params = nullptr, *d_grads = nullptr, *d_m = nullptr, *d_v = nullptr;
    float mean[F], stdv[F];
    bool norm_set = false;
    int adam_step = 0;
    hipStream_t stream = nullptr;
    // workspace for up to ws_rows rows
    int ws_rows = 0;
    float *d_act[kLayers + 1] = {};
    float *d_delta[2] = {};
    float *d_target = nullptr;
    float *d_loss = nullptr;  // one slot per mini-batch of an epoch
    int loss_slots = 0;
};

namespace {

void free_ws(fk_model *m)
{
    for (auto &p : m->d_act)
        if (p) {
            (void)hipFree(p);
            p = nullptr;
        }
    for (auto &p : m->d_delta)
        if (p) {
            (void)hipFree(p);
            p = nullptr;
        }
    if (m->d_target)
        (void)hipFree(m->d_target);
    m->d_target = nullptr;
    m->ws_rows = 0;
}

void free_model(fk_model *m)
{
    if (!m)
        return;
    free_ws(m);
    for (float *p : {m->d_params, m->d_grads, m->d_m, m->d_v, m->d_loss})
        if (p)
            (void)hipFree(p);
    if (m->stream)
        (void)hipStreamDestroy(m->stream);
    delete m;
}

fk_status ensure_ws(fk_model *m, int rows)
{
    if (rows <= m->ws_rows)
        return FK_OK;
    free_ws(m);
    const int widest = std::max(m->H, std::max(F, O));
    hipError_t e = hipSuccess;
    for (int l = 0; l <= kLayers && e == hipSuccess; ++l)
        e = hipMalloc(&m->d_act[l], sizeof(float) * (size_t)rows * m->dims[l]);
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
        e = hipMalloc(&m->d_delta[i], sizeof(float) * (size_t)rows * widest);
    if (e == hipSuccess)
        e = hipMalloc(&m->d_target, sizeof(float) * (size_t)rows * O);
    if (e != hipSuccess) {
        free_ws(m);
        return hip_error(e, "model workspace");
    }
    m->ws_rows = rows;
    return FK_OK;
}

fk_status ensure_loss_slots(fk_model *m, int n)
{
    if (n <= m->loss_slots)
        return FK_OK;
    if (m->d_loss)
        (void)hipFree(m->d_loss);
    m->d_loss = nullptr;
    m->loss_slots = 0;
    hipError_t e = hipMalloc(&m->d_loss, sizeof(float) * (size_t)n);
    if (e != hipSuccess)
        return hip_error(e, "loss buffer");
    m->loss_slots = n;
    return FK_OK;
}

void standardize(const fk_model *m, const float *in, int n, std::vector<float> &out)
{
    out.resize((size_t)n * F);
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < F; ++c)
            out[(size_t)r * F + c] = (in[(size_t)r * F + c] - m->mean[c]) / m->stdv[c];
}

// act[0] (rows x F) -> act[kLayers] (rows x O)
hipError_t forward(fk_model *m, int rows)
{
    hipError_t e = hipSuccess;
    for (int l = 0; l < kLayers && e == hipSuccess; ++l) {
        const bool last = l == kLayers - 1;
        e = mlp_gemm(false, true, m->d_act[l], m->d_params + m->w_off[l], m->d_act[l + 1], rows,
                     m->dims[l + 1], m->dims[l], m->d_params + m->b_off[l], nullptr,
                     last ? EPI_BIAS : EPI_BIAS_RELU, m->stream);
    }
    return e;
}

// gradients of the loss whose output delta is in d_delta[0] (rows x O)
hipError_t backward(fk_model *m, int rows)
{
    hipError_t e = hipSuccess;
    int cur = 0;
    for (int l = kLayers - 1; l >= 0 && e == hipSuccess; --l) {
        const int out = m->dims[l + 1], in = m->dims[l];
        // dW = dY^T act[l]   (out x in),  db = column sums of dY
        e = mlp_gemm(true, false, m->d_delta[cur], m->d_act[l], m->d_grads + m->w_off[l], out, in,
                     rows, nullptr, nullptr, EPI_NONE, m->stream);
        if (e == hipSuccess)
            e = mlp_colsum(m->d_delta[cur], rows, out, m->d_grads + m->b_off[l], m->stream);
        if (e == hipSuccess && l > 0) {
            // dX = dY W, masked by the ReLU of layer l-1's output (act[l])
            e = mlp_gemm(false, false, m->d_delta[cur], m->d_params + m->w_off[l],
                         m->d_delta[cur ^ 1], rows, in, out, nullptr, m->d_act[l], EPI_RELU_MASK,
                         m->stream);
            cur ^= 1;
        }
    }
    return e;
}

fk_status check_model(const fk_model *m)
{
    return m ? FK_OK : set_error(FK_ERR_INVALID_ARG, "model is null");
}

}  // namespace

extern "C" fk_status fk_model_create(int32_t hidden, uint64_t seed, fk_model **out)
{
    try {
        if (!out)
            return set_error(FK_ERR_INVALID_ARG, "out is null");
        *out = nullptr;
        if (hidden < 1 || hidden > 1024)
            return set_error(FK_ERR_INVALID_ARG, "hidden must be 1..1024");
        fk_model *m = new (std::nothrow) fk_model();
        if (!m)
            return set_error(FK_ERR_OUT_OF_MEMORY, "model allocation");
        m->H = hidden;
        m->dims[1] = m->dims[2] = m->dims[3] = hidden;
        int64_t off = 0;
        for (int l = 0; l < kLayers; ++l) {
            m->w_off[l] = off;
            off += (int64_t)m->dims[l + 1] * m->dims[l];
            m->b_off[l] = off;
            off += m->dims[l + 1];
        }
        m->n_params = off;
        for (int c = 0; c < F; ++c) {
            m->mean[c] = 0.0f;
            m->stdv[c] = 1.0f;
        }
        std::vector<float> init((size_t)off, 0.0f);
        uint64_t s = seed;
        for (int l = 0; l < kLayers; ++l) {
            const double a = std::sqrt(6.0 / m->dims[l]);
            for (int64_t i = 0; i < (int64_t)m->dims[l + 1] * m->dims[l]; ++i)
                init[(size_t)(m->w_off[l] + i)] = (float)((2.0 * uniform01(s) - 1.0) * a);
        }
        hipError_t e = hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking);
        for (float **p : {&m->d_params, &m->d_grads, &m->d_m, &m->d_v})
            if (e == hipSuccess)
                e = hipMalloc(p, sizeof(float) * (size_t)off);
        if (e == hipSuccess)
            e = hipMemcpy(m->d_params, init.data(), sizeof(float) * (size_t)off,
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemset(m->d_m, 0, sizeof(float) * (size_t)off);
        if (e == hipSuccess)
            e = hipMemset(m->d_v, 0, sizeof(float) * (size_t)off);
        if (e == hipSuccess)
            e = hipMemset(m->d_grads, 0, sizeof(float) * (size_t)off);
        if (e != hipSuccess) {
            free_model(m);
            return hip_error(e, "model allocation");
        }
        *out = m;
        return FK_OK;
    } catch (...) {
        return set_error(FK_ERR_OUT_OF_MEMORY, "exception");
    }
}

extern "C" fk_status fk_model_destroy(fk_model *model)
{
    if (model) {
        (void)hipStreamSynchronize(model->stream);
        free_model(model);
    }
    return FK_OK;
}

extern "C" int64_t fk_model_param_count(const fk_model *model)
{
    return model ? model->n_params : -1;
}

extern "C" fk_status fk_model_get_params(const fk_model *m, float *out, int64_t n)
{
    if (check_model(m) || !out || n != m->n_params)
        return set_error(FK_ERR_INVALID_ARG, "bad model, buffer or count");
    hipError_t e = hipMemcpy(out, m->d_params, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost);
    return e == hipSuccess ? FK_OK : hip_error(e, "hipMemcpy");
}

extern "C" fk_status fk_model_set_params(fk_model *m, const float *in, int64_t n)
{
    if (check_model(m) || !in || n != m->n_params)
        return set_error(FK_ERR_INVALID_ARG, "bad model, buffer or count");
    hipError_t e = hipMemcpy(m->d_params, in, sizeof(float) * (size_t)n, hipMemcpyHostToDevice);
    return e == hipSuccess ? FK_OK : hip_error(e, "hipMemcpy");
}

extern "C" fk_status fk_model_get_normalization(const fk_model *m, float *mean, float *stdv)
{
    if (check_model(m) || !mean || !stdv)
        return set_error(FK_ERR_INVALID_ARG, "null argument");
    std::memcpy(mean, m->mean, sizeof m->mean);
    std::memcpy(stdv, m->stdv, sizeof m->stdv);
    return FK_OK;
}

extern "C" fk_status fk_model_set_normalization(fk_model *m, const float *mean, const float *stdv)
{
    if (check_model(m) || !mean || !stdv)
        return set_error(FK_ERR_INVALID_ARG, "null argument");
    for (int c = 0; c < F; ++c)
        if (!(stdv[c] > 0.0f) || !std::isfinite(mean[c]))
            return set_error(FK_ERR_INVALID_ARG, "std must be positive and mean finite");
    std::memcpy(m->mean, mean, sizeof m->mean);
    std::memcpy(m->stdv, stdv, sizeof m->stdv);
    m->norm_set = true;
    return FK_OK;
}

// ------------------------------------------------------------- features --

static float lg2(double x) { return (float)std::log2(std::max(x, 1.0)); }

extern "C" fk_status fk_model_features(const fk_plan *p, const fk_item *items, int32_t n,
                                       float *out)
{
    try {
        if (!p || !out)
            return set_error(FK_ERR_INVALID_ARG, "null argument");
        if (n < 1)
            return set_error(FK_ERR_INVALID_ARG, "n_items must be >= 1");
        fk_status s = validate_items(&p->chain, items, n);
        if (s)
            return s;
        const fk_chain_desc &ch = p->chain;
        const int C = ch.read.channels;
        const int es_in = dtype_size(ch.read.in_dtype), es_out = dtype_size(ch.write.out_dtype);
        float f[F];
        std::fill(f, f + F, 0.0f);
        f[0] = rd_resizes(ch.read.kind) ? 1.0f : 0.0f;
        f[1 + ch.read.in_dtype] = 1.0f;
        f[4 + (C == 1 ? 0 : C == 3 ? 1 : 2)] = 1.0f;
        f[7] = ch.write.out_dtype == FK_F16 ? 1.0f : 0.0f;
        f[8] = ch.write.layout == FK_PLANAR ? 1.0f : 0.0f;
        f[9] = lg2(n);
        double out_px = 0, out_b = 0, in_b = 0, sw = 0, sh = 0, sow = 0, soh = 0, ssx = 0, ssy = 0,
               max_px = 0, vsrc = 0, vdst = 0, ragged = 0;
        for (int32_t b = 0; b < n; ++b) {
            const fk_item &it = items[b];
            const bool rs = rd_resizes(ch.read.kind);
            const double ow = rs ? it.out_w : it.w, oh = rs ? it.out_h : it.h;
            const double px = ow * oh;
            out_px += px;
            max_px = std::max(max_px, px);
            out_b += px * C * es_out;
            const double rows = rs ? std::min<double>(it.h, 2.0 * oh) : it.h;
            in_b += rows * it.w * C * es_in;
            sw += it.w;
            sh += it.h;
            sow += ow;
            soh += oh;
            ssx += it.w / ow;
            ssy += it.h / oh;
            if ((uintptr_t)it.src.ptr % 4 == 0 && it.src.pitch_bytes % 4 == 0 &&
                ((int64_t)it.x * C * es_in) % 4 == 0)
                vsrc += 1;
            if ((int64_t)ow % kUnitPx == 0 && (uintptr_t)it.dst % 16 == 0)
                vdst += 1;
            if ((int64_t)ow % kUnitPx != 0)
                ragged += 1;
        }
        f[10] = lg2(out_px);
        f[11] = lg2(out_px / n);
        f[12] = lg2(out_b);
        f[13] = lg2(in_b);
        f[14] = lg2(sw / n);
        f[15] = lg2(sh / n);
        f[16] = lg2(sow / n);
        f[17] = lg2(soh / n);
        f[18] = (float)std::log2(ssx / n);
        f[19] = (float)std::log2(ssy / n);
        double cnt[4];
        executed_counts(p->ops, cnt);
        f[20] = (float)((cnt[0] + cnt[1] + cnt[2] + cnt[3]) / 64.0);
        f[21] = (float)(cnt[OPC_FMA] / 64.0);
        f[22] = (float)(cnt[OPC_MUL] / 64.0);
        f[23] = (float)(cnt[OPC_ADD] / 64.0);
        f[24] = (float)(cnt[OPC_DIV] / 64.0);
        f[25] = (float)p->swap;
        f[26] = p->family != FAM_RUNTIME ? 1.0f : 0.0f;
        f[27] = (float)(vsrc / n);
        f[28] = (float)(vdst / n);
        f[29] = (float)(ragged / n);
        f[30] = lg2(max_px);
        f[31] = p->opts.strict_fp ? 1.0f : 0.0f;
        std::memcpy(out, f, sizeof f);
        return FK_OK;
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

// ------------------------------------------------------------- training --

extern "C" fk_status fk_model_loss_grad(fk_model *m, const float *features, const float *targets,
                                        int32_t n, float *loss, float *grad)
{
    try {
        if (check_model(m) || !features || !targets || !loss || !grad || n < 1)
            return set_error(FK_ERR_INVALID_ARG, "bad argument");
        fk_status s = ensure_ws(m, n);
        if (!s)
            s = ensure_loss_slots(m, 1);
        if (s)
            return s;
        std::vector<float> x;
        standardize(m, features, n, x);
        hipError_t e = hipMemcpyAsync(m->d_act[0], x.data(), sizeof(float) * x.size(),
                                      hipMemcpyHostToDevice, m->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(m->d_target, targets, sizeof(float) * (size_t)n * O,
                               hipMemcpyHostToDevice, m->stream);
        if (e == hipSuccess)
            e = forward(m, n);
        if (e == hipSuccess)
            e = mlp_mse(m->d_act[kLayers], m->d_target, (int64_t)n * O, m->d_delta[0], m->d_loss,
                        m->stream);
        if (e == hipSuccess)
            e = backward(m, n);
        if (e == hipSuccess)
            e = hipMemcpyAsync(grad, m->d_grads, sizeof(float) * (size_t)m->n_params,
                               hipMemcpyDeviceToHost, m->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(loss, m->d_loss, sizeof(float), hipMemcpyDeviceToHost, m->stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(m->stream);
        return e == hipSuccess ? FK_OK : hip_error(e, "loss/grad pass");
    } catch (...) {
        return set_error(FK_ERR_OUT_OF_MEMORY, "exception");
    }
}

extern "C" fk_status fk_model_train(fk_model *m, const float *features, const float *targets,
                                    int32_t n, int32_t epochs, int32_t batch, float lr, uint64_t seed,
                                    float *loss_curve)
{
    try {
        if (check_model(m) || !features || !targets || n < 1 || epochs < 0 || batch < 1 ||
            !(lr > 0.0f))
            return set_error(FK_ERR_INVALID_ARG, "bad argument");
        batch = std::min(batch, n);
        if (!m->norm_set) {
            for (int c = 0; c < F; ++c) {
                double s1 = 0, s2 = 0;
                for (int r = 0; r < n; ++r) {
                    const double v = features[(size_t)r * F + c];
                    s1 += v;
                    s2 += v * v;
                }
                const double mu = s1 / n, var = std::max(0.0, s2 / n - mu * mu);
                m->mean[c] = (float)mu;
                m->stdv[c] = var > 1e-12 ? (float)std::sqrt(var) : 1.0f;
            }
            m->norm_set = true;
        }
        const int nb = (n + batch - 1) / batch;
        fk_status s = ensure_ws(m, batch);
        if (!s)
            s = ensure_loss_slots(m, nb);
        if (s)
            return s;
        std::vector<float> x;
        standardize(m, features, n, x);
        float *d_x = nullptr, *d_t = nullptr;
        int32_t *d_idx = nullptr;
        hipError_t e = hipMalloc(&d_x, sizeof(float) * x.size());
        if (e == hipSuccess)
            e = hipMalloc(&d_t, sizeof(float) * (size_t)n * O);
        if (e == hipSuccess)
            e = hipMalloc(&d_idx, sizeof(int32_t) * (size_t)n);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_x, x.data(), sizeof(float) * x.size(), hipMemcpyHostToDevice,
                               m->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_t, targets, sizeof(float) * (size_t)n * O, hipMemcpyHostToDevice,
                               m->stream);
        std::vector<int32_t> perm(n);
        std::vector<float> losses(nb);
        uint64_t rs = seed;
        for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) {
            for (int i = 0; i < n; ++i)
                perm[i] = i;
            for (int i = n - 1; i > 0; --i) {  // Fisher-Yates
                const int j = (int)(splitmix(rs) % (uint64_t)(i + 1));
                std::swap(perm[i], perm[j]);
            }
            e = hipMemcpyAsync(d_idx, perm.data(), sizeof(int32_t) * (size_t)n,
                               hipMemcpyHostToDevice, m->stream);
            for (int b = 0; b < nb && e == hipSuccess; ++b) {
                const int r0 = b * batch, rows = std::min(batch, n - r0);
                e = mlp_gather(d_x, F, d_idx + r0, rows, m->d_act[0], m->stream);
                if (e == hipSuccess)
                    e = mlp_gather(d_t, O, d_idx + r0, rows, m->d_target, m->stream);
                if (e == hipSuccess)
                    e = forward(m, rows);
                if (e == hipSuccess)
                    e = mlp_mse(m->d_act[kLayers], m->d_target, (int64_t)rows * O, m->d_delta[0],
                                m->d_loss + b, m->stream);
                if (e == hipSuccess)
                    e = backward(m, rows);
                if (e == hipSuccess)
                    e = mlp_adam(m->d_params, m->d_grads, m->d_m, m->d_v, m->n_params, lr, 0.9f,
                                 0.999f, 1e-8f, ++m->adam_step, m->stream);
            }
            if (e == hipSuccess && loss_curve) {
                e = hipMemcpyAsync(losses.data(), m->d_loss, sizeof(float) * nb,
                                   hipMemcpyDeviceToHost, m->stream);
                if (e == hipSuccess)
                    e = hipStreamSynchronize(m->stream);
                double acc = 0;
                for (float l : losses)
                    acc += l;
                loss_curve[ep] = (float)(acc / nb);
            }
        }
        if (e == hipSuccess)
            e = hipStreamSynchronize(m->stream);
        (void)hipFree(d_x);
        (void)hipFree(d_t);
        (void)hipFree(d_idx);
        return e == hipSuccess ? FK_OK : hip_error(e, "training");
    } catch (...) {
        return set_error(FK_ERR_OUT_OF_MEMORY, "exception");
    }
}

extern "C" fk_status fk_model_predict_batch(fk_model *m, const float *features, int32_t n,
                                            float *out)
{
    try {
        if (check_model(m) || !features || !out || n < 1)
            return set_error(FK_ERR_INVALID_ARG, "bad argument");
        const int chunk = std::min(n, 4096);
        fk_status s = ensure_ws(m, chunk);
        if (s)
            return s;
        std::vector<float> x;
        hipError_t e = hipSuccess;
        for (int r0 = 0; r0 < n && e == hipSuccess; r0 += chunk) {
            const int rows = std::min(chunk, n - r0);
            standardize(m, features + (size_t)r0 * F, rows, x);
            e = hipMemcpyAsync(m->d_act[0], x.data(), sizeof(float) * x.size(),
                               hipMemcpyHostToDevice, m->stream);
            if (e == hipSuccess)
                e = forward(m, rows);
            if (e == hipSuccess)
                e = hipMemcpyAsync(out + (size_t)r0 * O, m->d_act[kLayers],
                                   sizeof(float) * (size_t)rows * O, hipMemcpyDeviceToHost,
                                   m->stream);
            if (e == hipSuccess)
                e = hipStreamSynchronize(m->stream);
        }
        return e == hipSuccess ? FK_OK : hip_error(e, "prediction");
    } catch (...) {
        return set_error(FK_ERR_OUT_OF_MEMORY, "exception");
    }
}

extern "C" fk_status fk_model_predict(fk_model *m, const fk_plan *plan, const fk_item *items,
                                      int32_t n, fk_launch_config *out)
{
    if (check_model(m) || !plan || !out)
        return set_error(FK_ERR_INVALID_ARG, "null argument");
    float f[F], y[O];
    fk_status s = fk_model_features(plan, items, n, f);
    if (!s)
        s = fk_model_predict_batch(m, f, 1, y);
    if (s)
        return s;
    fk_launch_config space[O];
    fk_autotune_space(space, O);
    int best = 0;
    for (int i = 1; i < O; ++i)
        if (y[i] < y[best])
            best = i;
    *out = space[best];
    return FK_OK;
}

extern "C" fk_status fk_plan_use_model(fk_plan *plan, fk_model *m, const fk_item *items, int32_t n)
{
    fk_launch_config c;
    fk_status s = fk_model_predict(m, plan, items, n, &c);
    if (s)
        return s;
    plan->cfg = c;
    plan->opts.config_source = FK_CONFIG_MODEL;
    return FK_OK;
}

// ---------------------------------------------------------- persistence --

extern "C" fk_status fk_model_save(const fk_model *m, const char *path)
{
    if (check_model(m) || !path)
        return set_error(FK_ERR_INVALID_ARG, "null argument");
    std::vector<float> params((size_t)m->n_params);
    hipError_t e = hipMemcpy(params.data(), m->d_params, sizeof(float) * params.size(),
                             hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_error(e, "hipMemcpy");
    FILE *fp = std::fopen(path, "wb");
    if (!fp)
        return set_error(FK_ERR_INVALID_ARG, "cannot open %s", path);
    std::fprintf(fp,
                 "{\"format\": \"fk-mlp\", \"version\": 1, \"features\": %d, \"hidden\": %d, "
                 "\"outputs\": %d, \"layers\": %d, \"params\": %lld}\n",
                 F, m->H, O, kLayers, (long long)m->n_params);
    bool ok = std::fwrite(m->mean, sizeof(float), F, fp) == (size_t)F &&
              std::fwrite(m->stdv, sizeof(float), F, fp) == (size_t)F &&
              std::fwrite(params.data(), sizeof(float), params.size(), fp) == params.size();
    ok = (std::fclose(fp) == 0) && ok;
    return ok ? FK_OK : set_error(FK_ERR_INVALID_ARG, "write failed: %s", path);
}

extern "C" fk_status fk_model_load(const char *path, fk_model **out)
{
    if (!path || !out)
        return set_error(FK_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    FILE *fp = std::fopen(path, "rb");
    if (!fp)
        return set_error(FK_ERR_INVALID_ARG, "cannot open %s", path);
    char line[512];
    if (!std::fgets(line, sizeof line, fp)) {
        std::fclose(fp);
        return set_error(FK_ERR_INVALID_ARG, "empty model file");
    }
    int f = 0, h = 0, o = 0, layers = 0, ver = 0;
    long long np = 0;
    if (std::sscanf(line,
                    "{\"format\": \"fk-mlp\", \"version\": %d, \"features\": %d, \"hidden\": %d, "
                    "\"outputs\": %d, \"layers\": %d, \"params\": %lld}",
                    &ver, &f, &h, &o, &layers, &np) != 6 ||
        ver != 1 || f != F || o != O || layers != kLayers) {
        std::fclose(fp);
        return set_error(FK_ERR_INVALID_ARG, "not an fk-mlp v1 file of this shape");
    }
    fk_model *m = nullptr;
    fk_status s = fk_model_create(h, 0, &m);
    if (s) {
        std::fclose(fp);
        return s;
    }
    std::vector<float> params((size_t)m->n_params);
    const bool ok = np == m->n_params && std::fread(m->mean, sizeof(float), F, fp) == (size_t)F &&
                    std::fread(m->stdv, sizeof(float), F, fp) == (size_t)F &&
                    std::fread(params.data(), sizeof(float), params.size(), fp) == params.size();
    std::fclose(fp);
    if (!ok) {
        fk_model_destroy(m);
        return set_error(FK_ERR_INVALID_ARG, "truncated model file");
    }
    m->norm_set = true;
    s = fk_model_set_params(m, params.data(), m->n_params);
    if (s) {
        fk_model_destroy(m);
        return s;
    }
    *out = m;
    return FK_OK;
}
