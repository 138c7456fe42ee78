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
    float *d_norm = nullptr;  // feature mean (F) then std (F), mirrors mean/stdv
    // training inputs: standardised features and mini-batch index lists
    float *d_xs = nullptr;
    int32_t *d_idx = nullptr;
    int train_rows = 0;
    // every epoch's permutation, pinned so that its copies are asynchronous
    int32_t *h_perm = nullptr;
    int64_t perm_cap = 0;
    hipEvent_t train_done = nullptr;  // recorded after the last queued training pass
    bool train_pending = false;
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
    for (float *p : {m->d_params, m->d_grads, m->d_m, m->d_v, m->d_loss, m->d_norm, m->d_xs})
        if (p)
            (void)hipFree(p);
    if (m->d_idx)
        (void)hipFree(m->d_idx);
    if (m->h_perm)
        (void)hipHostFree(m->h_perm);
    if (m->train_done)
        (void)hipEventDestroy(m->train_done);
    if (m->stream)
        (void)hipStreamDestroy(m->stream);
    delete m;
}

// Wait for training queued on a caller's stream before the model's
// buffers are read or changed by another call.
fk_status sync_pending(fk_model *m)
{
    if (!m->train_pending)
        return FK_OK;
    hipError_t e = hipEventSynchronize(m->train_done);
    if (e != hipSuccess)
        return hip_error(e, "pending training");
    m->train_pending = false;
    return FK_OK;
}

// Copy the host feature normalisation to its device mirror.
fk_status upload_norm(fk_model *m)
{
    hipError_t e = hipMemcpy(m->d_norm, m->mean, sizeof m->mean, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(m->d_norm + F, m->stdv, sizeof m->stdv, hipMemcpyHostToDevice);
    return e == hipSuccess ? FK_OK : hip_error(e, "normalisation upload");
}

fk_status ensure_train_bufs(fk_model *m, int rows)
{
    if (rows <= m->train_rows)
        return FK_OK;
    if (m->d_xs)
        (void)hipFree(m->d_xs);
    if (m->d_idx)
        (void)hipFree(m->d_idx);
    m->d_xs = nullptr;
    m->d_idx = nullptr;
    m->train_rows = 0;
    hipError_t e = hipMalloc(&m->d_xs, sizeof(float) * (size_t)rows * F);
    if (e == hipSuccess)
        e = hipMalloc(&m->d_idx, sizeof(int32_t) * (size_t)rows);
    if (e != hipSuccess)
        return hip_error(e, "training buffers");
    m->train_rows = rows;
    return FK_OK;
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

// x (rows x F) -> hidden layers hid[0..2] (rows x H each) -> y (rows x O)
hipError_t forward_p(const fk_model *m, const float *x, float *const hid[kLayers - 1], float *y,
                     int rows, hipStream_t st)
{
    hipError_t e = hipSuccess;
    const float *in = x;
    for (int l = 0; l < kLayers && e == hipSuccess; ++l) {
        const bool last = l == kLayers - 1;
        float *out = last ? y : hid[l];
        e = mlp_gemm(false, true, in, m->d_params + m->w_off[l], out, rows, m->dims[l + 1],
                     m->dims[l], m->d_params + m->b_off[l], nullptr, last ? EPI_BIAS : EPI_BIAS_RELU,
                     st);
        in = out;
    }
    return e;
}

// Gradient of every parameter into `grad` (the parameter layout) from the
// loss gradient dy (rows x O) of the forward pass that left x and hid;
// tmp[0], tmp[1] (rows x max(H, O) each) hold the propagated gradients and
// must not overlap dy.
hipError_t backward_p(const fk_model *m, const float *x, float *const hid[kLayers - 1],
                      const float *dy, float *const tmp[2], float *grad, int rows, hipStream_t st)
{
    hipError_t e = hipSuccess;
    const float *cur = dy;
    int nb = 0;
    for (int l = kLayers - 1; l >= 0 && e == hipSuccess; --l) {
        const int out = m->dims[l + 1], in = m->dims[l];
        const float *act = l == 0 ? x : hid[l - 1];  // the layer's input
        // dW = dY^T act   (out x in),  db = column sums of dY
        e = mlp_gemm(true, false, cur, act, grad + m->w_off[l], out, in, rows, nullptr, nullptr,
                     EPI_NONE, st);
        if (e == hipSuccess)
            e = mlp_colsum(cur, rows, out, grad + m->b_off[l], st);
        if (e == hipSuccess && l > 0) {
            // dX = dY W, masked by the ReLU of the previous layer's output
            e = mlp_gemm(false, false, cur, m->d_params + m->w_off[l], tmp[nb], rows, in, out,
                         nullptr, act, EPI_RELU_MASK, st);
            cur = tmp[nb];
            nb ^= 1;
        }
    }
    return e;
}

// the model's own workspace: act[0] (rows x F) -> act[kLayers] (rows x O)
hipError_t forward(fk_model *m, int rows, hipStream_t st)
{
    float *hid[kLayers - 1] = {m->d_act[1], m->d_act[2], m->d_act[3]};
    return forward_p(m, m->d_act[0], hid, m->d_act[kLayers], rows, st);
}

// gradients of the loss whose output delta is in d_delta[0] (rows x O)
hipError_t backward(fk_model *m, int rows, hipStream_t st)
{
    float *hid[kLayers - 1] = {m->d_act[1], m->d_act[2], m->d_act[3]};
    float *tmp[2] = {m->d_delta[1], m->d_delta[0]};
    return backward_p(m, m->d_act[0], hid, m->d_delta[0], tmp, m->d_grads, rows, st);
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
        if (e == hipSuccess)
            e = hipMalloc(&m->d_norm, sizeof(float) * 2 * F);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&m->train_done, hipEventDisableTiming);
        if (e != hipSuccess) {
            free_model(m);
            return hip_error(e, "model allocation");
        }
        fk_status st = upload_norm(m);
        if (st) {
            free_model(m);
            return st;
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
        (void)sync_pending(model);
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
    fk_status st = sync_pending(const_cast<fk_model *>(m));
    if (st)
        return st;
    hipError_t e = hipMemcpy(out, m->d_params, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost);
    return e == hipSuccess ? FK_OK : hip_error(e, "hipMemcpy");
}

extern "C" fk_status fk_model_set_params(fk_model *m, const float *in, int64_t n)
{
    if (check_model(m) || !in || n != m->n_params)
        return set_error(FK_ERR_INVALID_ARG, "bad model, buffer or count");
    fk_status st = sync_pending(m);
    if (st)
        return st;
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
    fk_status st = sync_pending(m);
    if (st)
        return st;
    std::memcpy(m->mean, mean, sizeof m->mean);
    std::memcpy(m->stdv, stdv, sizeof m->stdv);
    m->norm_set = true;
    return upload_norm(m);
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
        if (p->family == FAM_F64)
            return set_error(FK_ERR_UNSUPPORTED, "the cost model covers fp32 and fp16 writes only");
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
        fk_status s = sync_pending(m);
        if (!s)
            s = ensure_ws(m, n);
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
            e = forward(m, n, m->stream);
        if (e == hipSuccess)
            e = mlp_mse(m->d_act[kLayers], m->d_target, (int64_t)n * O, m->d_delta[0], m->d_loss,
                        m->stream);
        if (e == hipSuccess)
            e = backward(m, n, m->stream);
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

namespace {

// One training run, queued on `st`: mini-batches of shuffled rows (host
// Fisher-Yates permutations from SplitMix64, one per epoch), forward, MSE,
// backward, Adam.  d_feat are raw features; the first training call fixes
// the normalisation from them.
fk_status train_queued(fk_model *m, const float *d_feat, const float *d_targets, int32_t n,
                       int32_t epochs, int32_t batch, float lr, uint64_t seed, float *d_loss_curve,
                       hipStream_t st)
{
    batch = std::min(batch, n);
    const int nb = (n + batch - 1) / batch;
    fk_status s = sync_pending(m);
    if (!s)
        s = ensure_ws(m, batch);
    if (!s)
        s = ensure_loss_slots(m, nb);
    if (!s)
        s = ensure_train_bufs(m, n);
    if (s)
        return s;
    hipError_t e = hipSuccess;
    if (!m->norm_set) {
        // per-feature mean and std of these features, also kept on the host
        // (the features of a single prediction are standardised there)
        e = mlp_colstats(d_feat, n, F, m->d_norm, m->d_norm + F, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(m->mean, m->d_norm, sizeof m->mean, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(m->stdv, m->d_norm + F, sizeof m->stdv, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            return hip_error(e, "feature normalisation");
        m->norm_set = true;
    }
    e = mlp_standardize(d_feat, n, F, m->d_norm, m->d_norm + F, m->d_xs, st);
    // every epoch's permutation into the pinned buffer (free again: the
    // previous run was waited for above)
    const int64_t need = (int64_t)epochs * n;
    if (e == hipSuccess && need > m->perm_cap) {
        if (m->h_perm)
            (void)hipHostFree(m->h_perm);
        m->h_perm = nullptr;
        m->perm_cap = 0;
        e = hipHostMalloc(&m->h_perm, sizeof(int32_t) * (size_t)need, hipHostMallocDefault);
        if (e == hipSuccess)
            m->perm_cap = need;
    }
    if (e != hipSuccess)
        return hip_error(e, "training set-up");
    uint64_t rs = seed;
    for (int ep = 0; ep < epochs; ++ep) {
        int32_t *perm = m->h_perm + (int64_t)ep * n;
        for (int i = 0; i < n; ++i)
            perm[i] = i;
        for (int i = n - 1; i > 0; --i) {  // Fisher-Yates
            const int j = (int)(splitmix(rs) % (uint64_t)(i + 1));
            std::swap(perm[i], perm[j]);
        }
    }
    for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) {
        e = hipMemcpyAsync(m->d_idx, m->h_perm + (int64_t)ep * n, sizeof(int32_t) * (size_t)n,
                           hipMemcpyHostToDevice, st);
        for (int b = 0; b < nb && e == hipSuccess; ++b) {
            const int r0 = b * batch, rows = std::min(batch, n - r0);
            e = mlp_gather(m->d_xs, F, m->d_idx + r0, rows, m->d_act[0], st);
            if (e == hipSuccess)
                e = mlp_gather(d_targets, O, m->d_idx + r0, rows, m->d_target, st);
            if (e == hipSuccess)
                e = forward(m, rows, st);
            if (e == hipSuccess)
                e = mlp_mse(m->d_act[kLayers], m->d_target, (int64_t)rows * O, m->d_delta[0],
                            m->d_loss + b, st);
            if (e == hipSuccess)
                e = backward(m, rows, st);
            if (e == hipSuccess)
                e = mlp_adam(m->d_params, m->d_grads, m->d_m, m->d_v, m->n_params, lr, 0.9f,
                             0.999f, 1e-8f, ++m->adam_step, st);
        }
        if (e == hipSuccess && d_loss_curve)
            e = mlp_mean(m->d_loss, nb, d_loss_curve + ep, st);
    }
    if (e == hipSuccess)
        e = hipEventRecord(m->train_done, st);
    if (e != hipSuccess)
        return hip_error(e, "training");
    m->train_pending = true;
    return FK_OK;
}

}  // namespace

extern "C" fk_status fk_model_train_device(fk_model *m, const float *d_features,
                                           const float *d_targets, int32_t n, int32_t epochs,
                                           int32_t batch, float lr, uint64_t seed,
                                           float *d_loss_curve, void *stream)
{
    try {
        if (check_model(m) || !d_features || !d_targets || n < 1 || epochs < 0 || batch < 1 ||
            !(lr > 0.0f))
            return set_error(FK_ERR_INVALID_ARG, "bad argument");
        return train_queued(m, d_features, d_targets, n, epochs, batch, lr, seed, d_loss_curve,
                            (hipStream_t)stream);
    } catch (const std::bad_alloc &) {
        return set_error(FK_ERR_OUT_OF_MEMORY, "host allocation");
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
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
        fk_status s = sync_pending(m);
        if (s)
            return s;
        // the host arrays go to the device once; the run is the device-pointer one
        float *d_x = nullptr, *d_t = nullptr, *d_curve = nullptr;
        hipError_t e = hipMalloc(&d_x, sizeof(float) * (size_t)n * F);
        if (e == hipSuccess)
            e = hipMalloc(&d_t, sizeof(float) * (size_t)n * O);
        if (e == hipSuccess)
            e = hipMalloc(&d_curve, sizeof(float) * (size_t)std::max(epochs, 1));
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_x, features, sizeof(float) * (size_t)n * F, hipMemcpyHostToDevice,
                               m->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_t, targets, sizeof(float) * (size_t)n * O, hipMemcpyHostToDevice,
                               m->stream);
        if (e == hipSuccess)
            s = train_queued(m, d_x, d_t, n, epochs, batch, lr, seed, d_curve, m->stream);
        if (e == hipSuccess && !s)
            e = hipStreamSynchronize(m->stream);
        if (e == hipSuccess && !s) {
            m->train_pending = false;
            if (loss_curve && epochs > 0)
                e = hipMemcpy(loss_curve, d_curve, sizeof(float) * (size_t)epochs,
                              hipMemcpyDeviceToHost);
        }
        (void)hipStreamSynchronize(m->stream);
        (void)hipFree(d_x);
        (void)hipFree(d_t);
        (void)hipFree(d_curve);
        if (s)
            return s;
        return e == hipSuccess ? FK_OK : hip_error(e, "training");
    } catch (const std::bad_alloc &) {
        return set_error(FK_ERR_OUT_OF_MEMORY, "host allocation");
    } catch (...) {
        return set_error(FK_ERR_OUT_OF_MEMORY, "exception");
    }
}

// ------------------------------------------------- network kernels, raw --

extern "C" int64_t fk_mlp_workspace_floats(const fk_model *m, int32_t n)
{
    if (!m || n < 1)
        return -1;
    return (int64_t)n * ((kLayers - 1) * (int64_t)m->H + 2 * (int64_t)std::max(m->H, O));
}

static void ws_parts(const fk_model *m, float *ws, int32_t n, float *hid[kLayers - 1],
                     float *tmp[2])
{
    for (int l = 0; l < kLayers - 1; ++l)
        hid[l] = ws + (int64_t)l * n * m->H;
    float *t = ws + (int64_t)(kLayers - 1) * n * m->H;
    const int64_t w = (int64_t)n * std::max(m->H, O);
    tmp[0] = t;
    tmp[1] = t + w;
}

extern "C" fk_status fk_mlp_forward(const fk_model *m, const float *d_x, int32_t n, float *d_ws,
                                    float *d_y, void *stream)
{
    try {
        if (check_model(m) || !d_x || !d_ws || !d_y || n < 1)
            return set_error(FK_ERR_INVALID_ARG, "bad argument");
        fk_status s = sync_pending(const_cast<fk_model *>(m));
        if (s)
            return s;
        float *hid[kLayers - 1], *tmp[2];
        ws_parts(m, d_ws, n, hid, tmp);
        hipError_t e = forward_p(m, d_x, hid, d_y, n, (hipStream_t)stream);
        return e == hipSuccess ? FK_OK : hip_error(e, "forward");
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

extern "C" fk_status fk_mlp_backward(const fk_model *m, const float *d_x, int32_t n, float *d_ws,
                                     const float *d_dy, float *d_grad, void *stream)
{
    try {
        if (check_model(m) || !d_x || !d_ws || !d_dy || !d_grad || n < 1)
            return set_error(FK_ERR_INVALID_ARG, "bad argument");
        fk_status s = sync_pending(const_cast<fk_model *>(m));
        if (s)
            return s;
        float *hid[kLayers - 1], *tmp[2];
        ws_parts(m, d_ws, n, hid, tmp);
        hipError_t e = backward_p(m, d_x, hid, d_dy, tmp, d_grad, n, (hipStream_t)stream);
        return e == hipSuccess ? FK_OK : hip_error(e, "backward");
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

extern "C" fk_status fk_mlp_mse(const float *d_y, const float *d_t, int32_t n, float *d_dy,
                                float *d_loss, void *stream)
{
    try {
        if (!d_y || !d_t || !d_dy || !d_loss || n < 1)
            return set_error(FK_ERR_INVALID_ARG, "bad argument");
        hipError_t e = mlp_mse(d_y, d_t, (int64_t)n * O, d_dy, d_loss, (hipStream_t)stream);
        return e == hipSuccess ? FK_OK : hip_error(e, "mse");
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

extern "C" fk_status fk_mlp_step(fk_model *m, const float *d_grad, float lr, void *stream)
{
    try {
        if (check_model(m) || !d_grad || !(lr > 0.0f))
            return set_error(FK_ERR_INVALID_ARG, "bad argument");
        fk_status s = sync_pending(m);
        if (s)
            return s;
        hipError_t e = mlp_adam(m->d_params, d_grad, m->d_m, m->d_v, m->n_params, lr, 0.9f, 0.999f,
                                1e-8f, ++m->adam_step, (hipStream_t)stream);
        return e == hipSuccess ? FK_OK : hip_error(e, "adam step");
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

extern "C" fk_status fk_model_predict_batch(fk_model *m, const float *features, int32_t n,
                                            float *out)
{
    try {
        if (check_model(m) || !features || !out || n < 1)
            return set_error(FK_ERR_INVALID_ARG, "bad argument");
        const int chunk = std::min(n, 4096);
        fk_status s = sync_pending(m);
        if (!s)
            s = ensure_ws(m, chunk);
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
                e = forward(m, rows, m->stream);
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
    try {
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
    } catch (const std::bad_alloc &) {
        return set_error(FK_ERR_OUT_OF_MEMORY, "host allocation");
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

extern "C" fk_status fk_plan_use_model(fk_plan *plan, fk_model *m, const fk_item *items, int32_t n)
{
    try {
        fk_launch_config c;
        fk_status s = fk_model_predict(m, plan, items, n, &c);
        if (s)
            return s;
        plan->cfg = c;
        plan->opts.config_source = FK_CONFIG_MODEL;
        return FK_OK;
    } catch (const std::bad_alloc &) {
        return set_error(FK_ERR_OUT_OF_MEMORY, "host allocation");
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

// ---------------------------------------------------------- persistence --

extern "C" fk_status fk_model_save(const fk_model *m, const char *path)
{
    try {
        if (check_model(m) || !path)
            return set_error(FK_ERR_INVALID_ARG, "null argument");
        fk_status st = sync_pending(const_cast<fk_model *>(m));
        if (st)
            return st;
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
    } catch (const std::bad_alloc &) {
        return set_error(FK_ERR_OUT_OF_MEMORY, "host allocation");
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

extern "C" fk_status fk_model_load(const char *path, fk_model **out)
{
    try {
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
        std::vector<float> params;
        bool ok = false;
        try {
            params.resize((size_t)m->n_params);
            ok = np == m->n_params && std::fread(m->mean, sizeof(float), F, fp) == (size_t)F &&
                 std::fread(m->stdv, sizeof(float), F, fp) == (size_t)F &&
                 std::fread(params.data(), sizeof(float), params.size(), fp) == params.size();
        } catch (...) {
            ok = false;
        }
        std::fclose(fp);
        if (!ok) {
            fk_model_destroy(m);
            return set_error(FK_ERR_INVALID_ARG, "truncated model file");
        }
        m->norm_set = true;
        s = upload_norm(m);
        if (!s)
            s = fk_model_set_params(m, params.data(), m->n_params);
        if (s) {
            fk_model_destroy(m);
            return s;
        }
        *out = m;
        return FK_OK;
    } catch (const std::bad_alloc &) {
        return set_error(FK_ERR_OUT_OF_MEMORY, "host allocation");
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}
