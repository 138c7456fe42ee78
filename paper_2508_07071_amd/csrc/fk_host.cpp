// fk_host.cpp -- host runtime of the fused chain library: validation, chain
// normalisation, plans (the executor of Section IV-D: parameters are
// computed on the host once per plan and per run, then the fused kernel is
// launched), batch tables (BatchRead parameter arrays, Section IV-B), the
// hipGraph replay path and the launch-configuration autotuner.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fk.h"
#include "fk_host.hpp"
#include "fk_internal.hpp"

using namespace fk;

// ---------------------------------------------------------------- errors --

static thread_local std::string g_last_error;

fk_status fk::set_error(fk_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

fk_status fk::hip_error(hipError_t e, const char *what)
{
    return set_error(FK_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char *fk_status_string(fk_status s)
{
    switch (s) {
    case FK_OK: return "ok";
    case FK_ERR_INVALID_ARG: return "invalid argument";
    case FK_ERR_UNSUPPORTED: return "unsupported";
    case FK_ERR_OUT_OF_MEMORY: return "out of memory";
    case FK_ERR_HIP: return "HIP error";
    case FK_ERR_BAD_STATE: return "bad state";
    case FK_ERR_BUDGET: return "over budget";
    }
    return "unknown status";
}

extern "C" const char *fk_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *fk_version(void) { return "fk-mi355x 0.1 (gfx950)"; }

// ------------------------------------------------------------ validation --

int fk::dtype_size(int32_t dt) { return dt == FK_U8 ? 1 : dt == FK_F16 ? 2 : dt == FK_F64 ? 8 : 4; }

fk_status fk::validate_chain(const fk_chain_desc *ch)
{
    if (!ch)
        return set_error(FK_ERR_INVALID_ARG, "chain is null");
    const fk_read_desc &r = ch->read;
    if (r.kind < FK_READ_PLAIN || r.kind > FK_READ_NV12_RESIZE)
        return set_error(FK_ERR_INVALID_ARG, "unknown read kind %d", r.kind);
    if ((r.kind == FK_READ_NV12 || r.kind == FK_READ_NV12_RESIZE) &&
        (r.in_dtype != FK_U8 || r.channels != 3))
        return set_error(FK_ERR_INVALID_ARG, "NV12 reads take FK_U8 frames and give 3 channels");
    if (r.in_dtype != FK_U8 && r.in_dtype != FK_F16 && r.in_dtype != FK_F32 && r.in_dtype != FK_F64)
        return set_error(FK_ERR_INVALID_ARG, "unknown input dtype %d", r.in_dtype);
    if (r.channels != 1 && r.channels != 3 && r.channels != 4)
        return set_error(FK_ERR_UNSUPPORTED, "channels must be 1, 3 or 4 (got %d)", r.channels);
    if (ch->write.layout == FK_STATS) {
        if (ch->write.out_dtype != FK_F64)
            return set_error(FK_ERR_UNSUPPORTED, "the stats write produces FK_F64 only");
    } else {
        if (ch->write.out_dtype != FK_F32 && ch->write.out_dtype != FK_F16 &&
            ch->write.out_dtype != FK_F64)
            return set_error(FK_ERR_UNSUPPORTED, "output dtype must be FK_F32, FK_F16 or FK_F64");
        if (ch->write.layout != FK_PACKED && ch->write.layout != FK_PLANAR)
            return set_error(FK_ERR_INVALID_ARG, "unknown layout %d", ch->write.layout);
        if (ch->write.out_dtype == FK_F64 && r.kind != FK_READ_PLAIN)
            return set_error(FK_ERR_UNSUPPORTED, "fp64 chains take the plain read only");
    }
    if (r.in_dtype == FK_F64 && (ch->write.layout == FK_STATS || ch->write.out_dtype != FK_F64))
        return set_error(FK_ERR_UNSUPPORTED, "an FK_F64 frame needs an FK_F64 packed or planar write");
    if (ch->n_ops < 0 || ch->n_ops > FK_MAX_OPS)
        return set_error(FK_ERR_INVALID_ARG, "n_ops %d outside 0..%d", ch->n_ops, FK_MAX_OPS);
    if (ch->n_ops > 0 && !ch->ops)
        return set_error(FK_ERR_INVALID_ARG, "ops is null");
    for (int32_t i = 0; i < ch->n_ops; ++i) {
        const fk_op_desc &op = ch->ops[i];
        if (op.kind < FK_OP_SWAP_RB || op.kind > FK_OP_LOOP)
            return set_error(FK_ERR_INVALID_ARG, "op %d: unknown kind %d", i, op.kind);
        if (op.kind == FK_OP_LOOP) {
            if (op.n_consts != 0)
                return set_error(FK_ERR_INVALID_ARG, "op %d: a loop takes no constants", i);
            if (op.loop_span < 1 || op.loop_span > i)
                return set_error(FK_ERR_INVALID_ARG, "op %d: loop span %d outside 1..%d", i,
                                 op.loop_span, i);
            if (op.loop_count < 1)
                return set_error(FK_ERR_INVALID_ARG, "op %d: loop count %d < 1", i, op.loop_count);
            for (int32_t j = i - op.loop_span; j < i; ++j)
                if (ch->ops[j].kind < FK_OP_MUL || ch->ops[j].kind > FK_OP_DIV)
                    return set_error(FK_ERR_INVALID_ARG,
                                     "op %d: a loop body holds MUL/ADD/SUB/DIV only (op %d)", i, j);
        } else if (op.kind == FK_OP_SWAP_RB || op.kind == FK_OP_CVT_F32) {
            if (op.n_consts != 0)
                return set_error(FK_ERR_INVALID_ARG, "op %d: takes no constants", i);
        } else if (op.n_consts != 1 && op.n_consts != r.channels) {
            return set_error(FK_ERR_INVALID_ARG, "op %d: n_consts must be 1 or %d", i, r.channels);
        }
    }
    return FK_OK;
}

fk_status fk::validate_items(const fk_chain_desc *ch, const fk_item *items, int32_t n)
{
    if (n < 0)
        return set_error(FK_ERR_INVALID_ARG, "n_items < 0");
    if (n > 0 && !items)
        return set_error(FK_ERR_INVALID_ARG, "items is null");
    const int64_t es = dtype_size(ch->read.in_dtype);
    const int64_t C = ch->read.channels;
    const bool nv12 = ch->read.kind == FK_READ_NV12 || ch->read.kind == FK_READ_NV12_RESIZE;
    for (int32_t b = 0; b < n; ++b) {
        const fk_item &it = items[b];
        if (!it.src.ptr || !it.dst)
            return set_error(FK_ERR_INVALID_ARG, "item %d: null src or dst", b);
        if (it.src.width < 1 || it.src.height < 1)
            return set_error(FK_ERR_INVALID_ARG, "item %d: empty frame", b);
        if (it.src.width > 65535 || it.src.height > 65535)
            return set_error(FK_ERR_UNSUPPORTED, "item %d: frame sides above 65535", b);
        if (nv12) {
            if (it.src.width % 2 || it.src.height % 2 || it.src.pitch_bytes < it.src.width)
                return set_error(FK_ERR_INVALID_ARG,
                                 "item %d: NV12 frames need even sides and pitch >= width", b);
        } else if (it.src.pitch_bytes < it.src.width * C * es || it.src.pitch_bytes % es != 0) {
            return set_error(FK_ERR_INVALID_ARG, "item %d: bad pitch %lld", b,
                             (long long)it.src.pitch_bytes);
        }
        if ((uintptr_t)it.src.ptr % es != 0)
            return set_error(FK_ERR_INVALID_ARG, "item %d: src not element aligned", b);
        if ((uintptr_t)it.dst % dtype_size(ch->write.out_dtype) != 0)
            return set_error(FK_ERR_INVALID_ARG, "item %d: dst not element aligned", b);
        if (it.w < 1 || it.h < 1 || it.x < 0 || it.y < 0 ||
            (int64_t)it.x + it.w > it.src.width || (int64_t)it.y + it.h > it.src.height)
            return set_error(FK_ERR_INVALID_ARG,
                             "item %d: ROI (%d,%d,%d,%d) not inside the %dx%d frame", b, it.x,
                             it.y, it.w, it.h, it.src.width, it.src.height);
        if (rd_resizes(ch->read.kind)) {
            if (it.out_w < 1 || it.out_h < 1)
                return set_error(FK_ERR_INVALID_ARG, "item %d: output size must be positive", b);
            // output rows and columns feed 24-bit multiplies in the kernels
            if (it.out_w > 65535 || it.out_h > 65535)
                return set_error(FK_ERR_UNSUPPORTED, "item %d: output sides above 65535", b);
            if ((int64_t)it.out_w * it.out_h > (1LL << 28))
                return set_error(FK_ERR_UNSUPPORTED, "item %d: output too large", b);
        } else {
            if (!((it.out_w == 0 && it.out_h == 0) || (it.out_w == it.w && it.out_h == it.h)))
                return set_error(FK_ERR_INVALID_ARG,
                                 "item %d: plain read output must be 0x0 or the ROI size", b);
            if ((int64_t)it.w * it.h > (1LL << 28))
                return set_error(FK_ERR_UNSUPPORTED, "item %d: ROI too large", b);
        }
    }
    return FK_OK;
}

extern "C" fk_status fk_chain_validate(const fk_chain_desc *chain)
{
    try {
        return validate_chain(chain);
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

extern "C" fk_status fk_items_validate(const fk_chain_desc *chain, const fk_item *items,
                                       int32_t n_items)
{
    try {
        fk_status s = validate_chain(chain);
        if (s)
            return s;
        return validate_items(chain, items, n_items);
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

// ------------------------------------------------------------------ plan --

static const fk_launch_config kDefaultConfig = {256, 1};

// Default launch configuration: 256 threads.  A compile-time chain of more
// than 32 records (or 64 mul/add ops) takes coarsening 4, so that each
// scalar constant load serves more values (measured on 4K frames from HBM:
// 94.0 us at 256 x 4 for 256 ops against 97.5 us at 256 x 1).  A run-time
// op list of more than 32 records takes coarsening 2 after a plain read
// and stays at 1 after the other reads: over the 22,000 labelled random
// chains, those lists reach 0.85 (plain) and 0.92 (crop+resize) of their
// autotuned best that way, against 0.78 and 0.63 at coarsening 4.  The
// compile-time loop chain loads its two constants once, so it keeps
// coarsening 1 and with it the most waves for its arithmetic.  The stats
// write takes coarsening 8: its plain-read tiles issue all K loads first
// (measured: 16 4K frames in 96 us at 256 x 8, 117 us at 256 x 1).
static fk_launch_config default_config(const fk_plan *p)
{
    fk_launch_config c = kDefaultConfig;
    if (p->family == FAM_MULADD && p->static_n > 64)
        c.coarsen = 4;
    else if (p->ops.size() > 32)
        c.coarsen = !runs_op_list(p) ? 4 : p->chain.read.kind == FK_READ_PLAIN ? 2 : 1;
    if (p->chain.write.layout == FK_STATS)
        c.coarsen = 8;  // whole tiles fetch K units before reducing them
    return c;
}

bool fk::config_valid(const fk_launch_config &c)
{
    const bool t = c.block_threads == 64 || c.block_threads == 128 || c.block_threads == 256 ||
                   c.block_threads == 512 || c.block_threads == 1024;
    const bool k = c.coarsen == 1 || c.coarsen == 2 || c.coarsen == 4 || c.coarsen == 8;
    return t && k;
}

const void *fk::plan_kernel(const fk_plan *p, const fk_launch_config &cfg, bool large)
{
    if (p->chain.write.layout == FK_STATS) {
        if (p->chain.read.kind == FK_READ_PLAIN && p->chain.read.in_dtype == FK_U8 && p->ops.empty())
            return kernel_stats_u8(p->chain.read.channels, cfg.coarsen);
        return kernel_stats(p->chain.read.kind, p->chain.read.in_dtype, p->chain.read.channels,
                            cfg.coarsen);
    }
    switch (p->family) {
    case FAM_F64:
        return kernel_f64(p->chain.read.in_dtype, p->chain.read.channels, p->chain.write.layout,
                          cfg.coarsen);
    case FAM_NORMALIZE:
        if (p->opts.gather == FK_GATHER_LDS)
            return kernel_normalize_lds(cfg.coarsen, p->opts.strict_fp);
        // measured: 4-pixel units win on small, latency-bound launches
        // (B <= 50 crops of 64x128); pixel-strided lanes from about 1M
        // output pixels on (B = 256: 16.0 vs 20.1 us)
        return kernel_normalize(cfg.coarsen, p->opts.strict_fp, large);
    case FAM_MULADD: return kernel_muladd(p->static_n, cfg.coarsen, p->opts.strict_fp);
    case FAM_MULADD_LOOP:
        if (per_pixel(p))
            return kernel_loop_px(p->chain.read.in_dtype, p->chain.read.channels, cfg.coarsen,
                                  p->opts.strict_fp);
        return kernel_muladd_loop(p->chain.read.in_dtype, p->chain.read.channels, cfg.coarsen,
                                  p->opts.strict_fp);
    default: {
        // bilinear reads with a planar write take pixel-strided lanes on
        // large launches, as the normalise kernel does (256 NV12 crops:
        // 33.0 vs 35.5 us; nearest and 1:1 NV12 reads gained nothing)
        int layout = p->chain.write.layout;
        if (large && layout == FK_PLANAR && rd_bilinear(p->chain.read.kind))
            layout = LY_PLANAR_PX;
        return kernel_runtime(p->chain.read.kind, p->chain.read.in_dtype, p->chain.read.channels,
                              p->chain.write.out_dtype, layout, cfg.coarsen);
    }
    }
}

bool fk::runs_op_list(const fk_plan *p)
{
    return p->family == FAM_RUNTIME || p->family == FAM_F64;
}

bool fk::per_pixel(const fk_plan *p)
{
    return p->family == FAM_MULADD_LOOP && p->static_n >= kLoopPxMinPairs;
}

size_t fk::lds_bytes(const fk_plan *p, const fk_launch_config &cfg)
{
    if (p->family == FAM_F64)
        return 0;
    if (p->family == FAM_NORMALIZE && p->opts.gather == FK_GATHER_LDS)
        return lds_gather_bytes((uint32_t)cfg.block_threads);
    if (p->chain.write.layout != FK_PACKED || per_pixel(p))
        return 0;
    const int ub = kUnitPx * p->chain.read.channels * dtype_size(p->chain.write.out_dtype);
    if (ub == 16 || ub == 8)
        return 0;
    return (size_t)cfg.block_threads * ub;
}

static void free_slot(fk_plan::Slot &s)
{
    if (s.gexec)
        (void)hipGraphExecDestroy(s.gexec);
    if (s.done)
        (void)hipEventDestroy(s.done);
    if (s.d_table)
        (void)hipFree(s.d_table);
    if (s.h_stage)
        (void)hipHostFree(s.h_stage);
    s = fk_plan::Slot();
}

static void plan_free(fk_plan *p)
{
    if (!p)
        return;
    for (auto &s : p->slots)
        free_slot(s);
    if (p->d_ops)
        (void)hipFree(p->d_ops);
    if (p->d_consts)
        (void)hipFree(p->d_consts);
    if (p->d_st_part)
        (void)hipFree(p->d_st_part);
    if (p->capture_stream)
        (void)hipStreamDestroy(p->capture_stream);
    if (p->tune_stream)
        (void)hipStreamDestroy(p->tune_stream);
    delete p;
}

extern "C" fk_status fk_plan_create(const fk_chain_desc *chain, int32_t max_batch,
                                    const fk_plan_opts *opts, fk_plan **out)
{
    try {
        if (!out)
            return set_error(FK_ERR_INVALID_ARG, "out is null");
        *out = nullptr;
        fk_status s = validate_chain(chain);
        if (s)
            return s;
        if (max_batch < 1 || max_batch > (1 << 20))
            return set_error(FK_ERR_INVALID_ARG, "max_batch %d outside 1..2^20", max_batch);
        const bool stats = chain->write.layout == FK_STATS;
        if (stats && max_batch > kStatCapacity)
            return set_error(FK_ERR_UNSUPPORTED, "stats write: max_batch above %d", kStatCapacity);
        fk_plan_opts o = {FK_CONFIG_DEFAULT, kDefaultConfig, 0, 0, FK_TIER_AUTO, 0, FK_GATHER_DIRECT};
        if (opts)
            o = *opts;
        if (o.config_source == FK_CONFIG_MANUAL && !config_valid(o.manual))
            return set_error(FK_ERR_INVALID_ARG, "manual config (%d threads, coarsen %d) invalid",
                             o.manual.block_threads, o.manual.coarsen);
        if (o.config_source < FK_CONFIG_DEFAULT || o.config_source > FK_CONFIG_MODEL)
            return set_error(FK_ERR_INVALID_ARG, "unknown config source");
        if (o.tier != FK_TIER_AUTO && o.tier != FK_TIER_RUNTIME)
            return set_error(FK_ERR_INVALID_ARG, "unknown tier");
        if (o.gather != FK_GATHER_DIRECT && o.gather != FK_GATHER_LDS)
            return set_error(FK_ERR_INVALID_ARG, "unknown gather mode %d", o.gather);

        fk_plan *p = new (std::nothrow) fk_plan();
        if (!p)
            return set_error(FK_ERR_OUT_OF_MEMORY, "plan allocation");
        p->chain = *chain;
        p->op_descs.assign(chain->ops, chain->ops + chain->n_ops);
        p->chain.ops = p->op_descs.data();
        p->max_batch = max_batch;
        p->opts = o;
        p->cfg = kDefaultConfig;
        hipError_t e = hipGetDevice(&p->device);
        if (e != hipSuccess) {
            plan_free(p);
            return hip_error(e, "hipGetDevice");
        }
        int cus = 0;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
        p->num_cus = cus > 0 ? cus : 256;

        std::vector<float> consts;
        int sn = 0;
        const bool f64 = chain->write.out_dtype == FK_F64 && !stats;
        p->family = f64 ? FAM_F64
                        : o.tier == FK_TIER_AUTO && !stats ? match_static(&p->chain, consts, sn)
                                                           : FAM_RUNTIME;
        p->static_n = sn;
        normalise_chain(&p->chain, o.strict_fp != 0, p->ops, p->swap);
        p->cfg = o.config_source == FK_CONFIG_MANUAL ? o.manual : default_config(p);
        if (!runs_op_list(p)) {
            e = hipMalloc(&p->d_consts, std::max<size_t>(consts.size(), 1) * sizeof(float));
            if (e == hipSuccess)
                e = hipMemcpy(p->d_consts, consts.data(), consts.size() * sizeof(float),
                              hipMemcpyHostToDevice);
        }
        if (e == hipSuccess) {
            e = hipMalloc(&p->d_ops, std::max<size_t>(p->ops.size(), 1) * sizeof(OpRec));
            if (e == hipSuccess && !p->ops.empty())
                e = hipMemcpy(p->d_ops, p->ops.data(), p->ops.size() * sizeof(OpRec),
                              hipMemcpyHostToDevice);
        }
        if (e == hipSuccess && stats) {
            // partials for every slot of a full batch
            p->st_capacity = (uint32_t)std::min<int64_t>((int64_t)max_batch * kStatSlots, kStatCapacity);
            e = hipMalloc(&p->d_st_part, (size_t)p->st_capacity * chain->read.channels *
                                             sizeof(StatPartial));
        }
        p->table_bytes = sizeof(RunHeader) + sizeof(ItemRec) * (size_t)max_batch +
                         sizeof(uint32_t) * ((size_t)max_batch + 1);
        p->table_bytes = (p->table_bytes + 255) & ~(size_t)255;
        if (e != hipSuccess) {
            plan_free(p);
            return e == hipErrorOutOfMemory ? set_error(FK_ERR_OUT_OF_MEMORY, "plan buffers")
                                            : hip_error(e, "plan buffers");
        }
        for (int k : {1, 2, 4, 8}) {
            fk_launch_config c = {256, k};
            if (!plan_kernel(p, c, false) || !plan_kernel(p, c, true)) {
                plan_free(p);
                return set_error(FK_ERR_UNSUPPORTED, "no kernel built for this chain");
            }
        }
        *out = p;
        return FK_OK;
    } catch (const std::bad_alloc &) {
        return set_error(FK_ERR_OUT_OF_MEMORY, "host allocation");
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

extern "C" fk_status fk_plan_destroy(fk_plan *plan)
{
    try {
        if (!plan)
            return FK_OK;
        for (auto &s : plan->slots)
            if (s.used)
                (void)hipEventSynchronize(s.done);
        plan_free(plan);
        return FK_OK;
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

extern "C" fk_status fk_plan_get_config(const fk_plan *plan, fk_launch_config *out)
{
    if (!plan || !out)
        return set_error(FK_ERR_INVALID_ARG, "null argument");
    *out = plan->cfg;
    return FK_OK;
}

extern "C" fk_status fk_plan_set_config(fk_plan *plan, const fk_launch_config *cfg)
{
    if (!plan || !cfg)
        return set_error(FK_ERR_INVALID_ARG, "null argument");
    if (!config_valid(*cfg))
        return set_error(FK_ERR_INVALID_ARG, "config (%d threads, coarsen %d) invalid",
                         cfg->block_threads, cfg->coarsen);
    plan->cfg = *cfg;
    return FK_OK;
}

extern "C" fk_status fk_plan_get_tier(const fk_plan *plan, int32_t *is_static)
{
    if (!plan || !is_static)
        return set_error(FK_ERR_INVALID_ARG, "null argument");
    *is_static = runs_op_list(plan) ? 0 : 1;
    return FK_OK;
}

// -------------------------------------------------------------- run path --

// Fill the item records and tile prefix sums of a run; returns the number
// of tiles.
// Row offsets of the frame fit 32 bits and its pitch 24 bits (full-rate
// 24-bit multiplies in the kernels).
static bool small_frame(const fk_image &f)
{
    return f.pitch_bytes < ((int64_t)1 << 24) && f.pitch_bytes * (int64_t)f.height < ((int64_t)1 << 32);
}

uint32_t fk::build_items(const fk_plan *p, const fk_item *items, int32_t n,
                         const fk_launch_config &cfg, ItemRec *recs, uint32_t *tb,
                         int32_t batch_n)
{
    const int C = p->chain.read.channels;
    const int es_in = dtype_size(p->chain.read.in_dtype);
    // a per-pixel kernel's tile is T*K pixels: T*K/4 units of 4 pixels
    const uint64_t tile_units = per_pixel(p) ? (uint64_t)cfg.block_threads * cfg.coarsen / kUnitPx
                                             : (uint64_t)cfg.block_threads * cfg.coarsen;
    // stats write: an item's "tiles" are its blocks, at most slot_cap each;
    // a batch shares about one resident grid, so each block walks several
    // tiles
    const bool stats = p->chain.write.layout == FK_STATS;
    const uint64_t batch = (uint64_t)(batch_n > 0 ? batch_n : n);
    const uint64_t slot_cap =
        stats ? std::max<uint64_t>(1, std::min<uint64_t>({(uint64_t)kStatSlots, p->st_capacity / batch,
                                                          persistent_grid(p, cfg) / batch}))
              : ~0ull;
    uint64_t tiles = 0;
    for (int32_t b = 0; b < n; ++b) {
        const fk_item &it = items[b];
        ItemRec &r = recs[b];
        std::memset(&r, 0, sizeof r);
        r.src = (uint64_t)(uintptr_t)it.src.ptr;
        r.dst = (uint64_t)(uintptr_t)it.dst;
        r.pitch = it.src.pitch_bytes;
        r.x = it.x;
        r.y = it.y;
        r.w = it.w;
        r.h = it.h;
        if (rd_resizes(p->chain.read.kind)) {
            r.ow = it.out_w;
            r.oh = it.out_h;
            r.sx = (float)it.w / (float)it.out_w;
            r.sy = (float)it.h / (float)it.out_h;
        } else {
            r.ow = it.w;
            r.oh = it.h;
            r.sx = 1.0f;
            r.sy = 1.0f;
        }
        r.fw = (uint16_t)it.src.width;
        r.fh = (uint16_t)it.src.height;
        const int64_t upr = (r.ow + kUnitPx - 1) / kUnitPx;
        int flags = 0;
        if ((uintptr_t)it.src.ptr % 4 == 0 && it.src.pitch_bytes % 4 == 0 &&
            ((int64_t)it.x * C * es_in) % 4 == 0)
            flags |= IF_SRC_VEC;
        if (r.ow % kUnitPx == 0 && (uintptr_t)it.dst % 16 == 0)
            flags |= IF_DST_VEC;
        if (small_frame(it.src))
            flags |= IF_SMALL_FRAME;
        if (p->chain.read.kind == FK_READ_PLAIN && it.x == 0 && it.w == it.src.width &&
            it.src.pitch_bytes == (int64_t)it.src.width * C * es_in && r.ow % kUnitPx == 0 &&
            (int64_t)r.ow * r.oh < ((int64_t)1 << 31))
            flags |= IF_CONTIG;
        r.flags = flags;
        tb[b] = (uint32_t)tiles;
        const uint64_t units = (uint64_t)upr * (uint64_t)r.oh;
        tiles += std::min<uint64_t>((units + tile_units - 1) / tile_units, slot_cap);
    }
    tb[n] = (uint32_t)tiles;
    return (uint32_t)tiles;
}

// Fill the host staging table of a run (header, items, prefix sums).
uint32_t fk::build_table(const fk_plan *p, const fk_item *items, int32_t n,
                         const fk_launch_config &cfg, void *stage)
{
    RunHeader *hdr = (RunHeader *)stage;
    ItemRec *recs = (ItemRec *)(hdr + 1);
    uint32_t *tb = (uint32_t *)(recs + p->max_batch);
    const uint32_t tiles = build_items(p, items, n, cfg, recs, tb);
    hdr->n_items = n;
    hdr->total_tiles = tiles;
    hdr->pad[0] = hdr->pad[1] = 0;
    return tiles;
}

KArgs fk::make_args(const fk_plan *p, void *d_table)
{
    KArgs a;
    std::memset(&a, 0, sizeof a);
    a.hdr = (const RunHeader *)d_table;
    a.items = (const ItemRec *)((const RunHeader *)d_table + 1);
    a.tile_begin = (const uint32_t *)(a.items + p->max_batch);
    a.ops = (const OpRec *)p->d_ops;
    a.consts = (const float *)p->d_consts;
    a.n_ops = (int32_t)p->ops.size();
    a.swap = runs_op_list(p) ? p->swap : 0;
    a.strict = p->opts.strict_fp;
    a.loop_count = p->family == FAM_MULADD_LOOP ? p->static_n : 0;
    a.st_part = p->d_st_part;
    return a;
}

// Blocks resident at once (persistent grid for graph replays).
uint32_t fk::persistent_grid(const fk_plan *p, const fk_launch_config &cfg)
{
    const uint32_t per_cu = std::max(1, 2048 / cfg.block_threads);
    return (uint32_t)p->num_cus * per_cu;
}

// The plan's kernel over `grid` blocks; a stats write then launches its
// combine kernel (one block per item, same arguments) on the same stream.
// Given events, the launches record them as the first kernel starts and
// the last one ends.
static hipError_t launch_one(const void *fn, dim3 grid, dim3 block, void **args, size_t lds,
                             hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1)
{
    if (!ev0 && !ev1)
        return hipLaunchKernel(fn, grid, block, args, lds, stream);
    return hipExtLaunchKernel(fn, grid, block, args, lds, stream, ev0, ev1, 0);
}

fk_status fk::launch_args(const fk_plan *p, const fk_launch_config &cfg, KArgs &a, uint32_t grid,
                          int32_t n_items, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1)
{
    // output pixels the launch covers: grid blocks of T * K units of 4 pixels
    const bool large = (uint64_t)grid * (uint64_t)cfg.block_threads * (uint64_t)cfg.coarsen * kUnitPx >=
                       kStridedMinPixels;
    const void *fn = plan_kernel(p, cfg, large);
    if (!fn)
        return set_error(FK_ERR_UNSUPPORTED, "no kernel for coarsening %d", cfg.coarsen);
    const bool stats = p->chain.write.layout == FK_STATS;
    void *args[] = {&a};
    hipError_t e = launch_one(fn, dim3(grid), dim3(cfg.block_threads), args, lds_bytes(p, cfg),
                              stream, ev0, stats ? nullptr : ev1);
    if (e == hipSuccess && stats) {
        const void *fin = kernel_stats_final(p->chain.read.channels);
        if (!fin)
            return set_error(FK_ERR_UNSUPPORTED, "no stats combine kernel");
        e = launch_one(fin, dim3((unsigned)n_items), dim3(256), args, 0, stream, nullptr, ev1);
    }
    if (e != hipSuccess)
        return hip_error(e, "hipLaunchKernel");
    return FK_OK;
}

fk_status fk::launch(const fk_plan *p, const fk_launch_config &cfg, void *d_table, uint32_t grid,
                     int32_t n_items, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1)
{
    KArgs a = make_args(p, d_table);
    return launch_args(p, cfg, a, grid, n_items, stream, ev0, ev1);
}

// A batch that can travel in the compact kernel-argument form: one frame,
// one output size, outputs at a constant non-negative stride, coordinates
// that fit 16 bits.
bool fk::compact_batch(const fk_plan *p, const fk_item *items, int32_t n)
{
    if (n < 2)
        return false;
    const fk_item &f = items[0];
    const bool rs = rd_resizes(p->chain.read.kind);
    const intptr_t stride = (intptr_t)items[1].dst - (intptr_t)items[0].dst;
    if (stride < 0 || f.src.width > 65535 || f.src.height > 65535)
        return false;
    for (int32_t b = 0; b < n; ++b) {
        const fk_item &it = items[b];
        if (it.src.ptr != f.src.ptr || it.src.width != f.src.width ||
            it.src.height != f.src.height || it.src.pitch_bytes != f.src.pitch_bytes)
            return false;
        if ((intptr_t)it.dst != (intptr_t)f.dst + (intptr_t)b * stride)
            return false;
        if (rs ? (it.out_w != f.out_w || it.out_h != f.out_h) : (it.w != f.w || it.h != f.h))
            return false;
    }
    return true;
}

// One compact kernel-argument launch of n items (1 <= n <= kCompactItems)
// that share the template of items[0]; item b's output is items[0].dst +
// b * stride.  batch_n is the batch size the per-item tiling assumes.
static fk_status launch_compact(const fk_plan *p, const fk_item *items, int32_t n, intptr_t stride,
                                int32_t batch_n, const fk_launch_config &cfg, hipStream_t stream,
                                hipEvent_t ev0, hipEvent_t ev1)
{
    KArgs a = make_args(p, nullptr);
    a.hdr = nullptr;
    a.items = nullptr;
    a.tile_begin = nullptr;
    a.inl_n = n;
    a.inl_compact = 1;
    uint32_t tb[2];
    ItemRec &t = *(ItemRec *)a.inl;
    a.inl_tiles_per_item = build_items(p, items, 1, cfg, &t, tb, batch_n);
    a.inl_total_tiles = a.inl_tiles_per_item * (uint32_t)n;
    a.inl_dst_stride = (int64_t)stride;
    // template flags: frame base and pitch dword-aligned; outputs aligned
    // for every item (base and stride multiples of 16)
    t.flags = 0;
    if ((uintptr_t)items[0].src.ptr % 4 == 0 && items[0].src.pitch_bytes % 4 == 0)
        t.flags |= IF_SRC_VEC;
    if (t.ow % kUnitPx == 0 && (uintptr_t)items[0].dst % 16 == 0 && a.inl_dst_stride % 16 == 0)
        t.flags |= IF_DST_VEC;
    if (small_frame(items[0].src))
        t.flags |= IF_SMALL_FRAME;
    Roi16 *roi = (Roi16 *)(a.inl + 64);
    for (int32_t b = 0; b < n; ++b)
        roi[b] = Roi16{(uint16_t)items[b].x, (uint16_t)items[b].y, (uint16_t)items[b].w,
                       (uint16_t)items[b].h};
    const uint32_t grid = std::min<uint32_t>(a.inl_total_tiles, 1u << 20);
    return launch_args(p, cfg, a, grid, n, stream, ev0, ev1);
}

static_assert(sizeof(RunHeader) % 16 == 0 && sizeof(ItemRec) % 16 == 0,
              "the run table uploads in 16-byte units");

// Queue the copy of a slot's table to the device: the header, items
// [0, n) and tile_begin[0 .. n], in 16-byte units (the prefix sums rounded
// up; the table's size is a multiple of 256 bytes, so the rounding stays
// inside it).
static hipError_t upload_table(const fk_plan *p, const fk_plan::Slot &sl, int32_t n,
                               hipStream_t stream)
{
    uint32_t n0 = (uint32_t)((sizeof(RunHeader) + sizeof(ItemRec) * (size_t)n) / 16);
    uint32_t off1 = (uint32_t)((sizeof(RunHeader) + sizeof(ItemRec) * (size_t)p->max_batch) / 16);
    uint32_t n1 = (uint32_t)((sizeof(uint32_t) * ((size_t)n + 1) + 15) / 16);
    const void *src = sl.h_dev;
    void *dst = sl.d_table;
    void *args[] = {&src, &dst, &n0, &off1, &n1};
    return hipLaunchKernel(kernel_table_upload(), dim3((n0 + n1 + 255) / 256), dim3(256), args, 0,
                           stream);
}

// The batch travels in kernel arguments only (no run table): up to
// kInlineItems items, or items of one frame, one output size and a constant
// output stride (consecutive launches of kCompactItems beyond that, except
// for a stats write).
static bool argument_form(const fk_plan *p, const fk_item *items, int32_t n)
{
    if (n <= kInlineItems)
        return true;
    return compact_batch(p, items, n) && (n <= kCompactItems || p->chain.write.layout != FK_STATS);
}

// Under the caller's stream capture only argument-form batches may run: a
// table batch's parameters are staged in host memory that later runs
// rewrite, and a plan's own graph replay is a graph launch.
static fk_status check_capture(const fk_plan *p, const fk_item *items, int32_t n, bool graph,
                               bool timed, hipStream_t stream)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &cs);
    if (e != hipSuccess)
        return hip_error(e, "hipStreamIsCapturing");
    if (cs == hipStreamCaptureStatusNone)
        return FK_OK;
    if (graph || timed)
        return set_error(FK_ERR_UNSUPPORTED,
                         "under stream capture: no plan graph replay and no timed run");
    if (!argument_form(p, items, n))
        return set_error(FK_ERR_UNSUPPORTED,
                         "under stream capture only batches carried in kernel arguments can run "
                         "(up to %d items, or items of one frame, one output size and a constant "
                         "output stride)",
                         kInlineItems);
    return FK_OK;
}

fk_status fk::run_fused(fk_plan *p, const fk_item *items, int32_t n, const fk_launch_config &cfg,
                        bool graph, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1)
{
    fk_status cs = check_capture(p, items, n, graph, ev0 || ev1, stream);
    if (cs)
        return cs;
    if (!graph && n <= kInlineItems) {
        // small batch: the parameters travel in the kernel arguments
        KArgs a = make_args(p, nullptr);
        a.hdr = nullptr;
        a.items = nullptr;
        a.tile_begin = nullptr;
        a.inl_n = n;
        a.inl_total_tiles = build_items(p, items, n, cfg, (ItemRec *)a.inl,
                                        (uint32_t *)(a.inl + kInlineTileBegin));
        const uint32_t grid = std::min<uint32_t>(a.inl_total_tiles, 1u << 20);
        return launch_args(p, cfg, a, grid, n, stream, ev0, ev1);
    }
    if (!graph && compact_batch(p, items, n)) {
        const intptr_t stride = (intptr_t)items[1].dst - (intptr_t)items[0].dst;
        if (n <= kCompactItems)
            return launch_compact(p, items, n, stride, n, cfg, stream, ev0, ev1);
        if (p->chain.write.layout != FK_STATS) {
            // beyond one launch's argument capacity: consecutive compact
            // launches of up to kCompactItems items, still no table copy
            for (int32_t b0 = 0; b0 < n; b0 += kCompactItems) {
                const int32_t m = std::min(n - b0, kCompactItems);
                fk_status s = launch_compact(p, items + b0, m, stride, m, cfg, stream,
                                             b0 == 0 ? ev0 : nullptr, b0 + m == n ? ev1 : nullptr);
                if (s)
                    return s;
            }
            return FK_OK;
        }
    }
    fk_plan::Slot &sl = p->slots[p->next_slot];
    hipError_t e = hipSuccess;
    if (!sl.h_stage) {
        // the whole table ring is allocated on the first table run, so
        // later runs allocate nothing
        for (fk_plan::Slot &r : p->slots) {
            // coherent: the upload kernel reads each byte once, straight
            // from host memory, after the host has rewritten the slot
            e = hipHostMalloc(&r.h_stage, p->table_bytes, hipHostMallocMapped | hipHostMallocCoherent);
            if (e == hipSuccess)
                e = hipHostGetDevicePointer(&r.h_dev, r.h_stage, 0);
            if (e == hipSuccess)
                e = hipMalloc(&r.d_table, p->table_bytes);
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(&r.done, hipEventDisableTiming);
            if (e != hipSuccess) {
                for (fk_plan::Slot &q : p->slots)
                    free_slot(q);
                return e == hipErrorOutOfMemory ? set_error(FK_ERR_OUT_OF_MEMORY, "run table")
                                                : hip_error(e, "run table");
            }
        }
    }
    p->next_slot = (p->next_slot + 1) % fk_plan::kRing;
    if (graph && !p->capture_stream) {
        e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess)
            return hip_error(e, "hipStreamCreate");
    }
    if (sl.used) {
        e = hipEventSynchronize(sl.done);
        if (e != hipSuccess)
            return hip_error(e, "hipEventSynchronize");
    }
    const uint32_t tiles = build_table(p, items, n, cfg, sl.h_stage);
    if (tiles == 0)
        return FK_OK;
    if (graph) {
        const bool stale = !sl.gexec || sl.gcfg.block_threads != cfg.block_threads ||
                           sl.gcfg.coarsen != cfg.coarsen;
        if (stale) {
            if (sl.gexec) {
                (void)hipGraphExecDestroy(sl.gexec);
                sl.gexec = nullptr;
            }
            hipGraph_t g = nullptr;
            e = hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess)
                return hip_error(e, "hipStreamBeginCapture");
            e = upload_table(p, sl, p->max_batch, p->capture_stream);
            fk_status s = FK_OK;
            if (e == hipSuccess)
                s = launch(p, cfg, sl.d_table, persistent_grid(p, cfg), std::min(p->max_batch, 4096),
                           p->capture_stream);
            hipError_t e2 = hipStreamEndCapture(p->capture_stream, &g);
            if (e != hipSuccess)
                return hip_error(e, "table upload (capture)");
            if (s)
                return s;
            if (e2 != hipSuccess)
                return hip_error(e2, "hipStreamEndCapture");
            e = hipGraphInstantiate(&sl.gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess)
                return hip_error(e, "hipGraphInstantiate");
            sl.gcfg = cfg;
        }
        if (ev0)
            e = hipEventRecord(ev0, stream);
        if (e == hipSuccess)
            e = hipGraphLaunch(sl.gexec, stream);
        if (e == hipSuccess && ev1)
            e = hipEventRecord(ev1, stream);
        if (e != hipSuccess)
            return hip_error(e, "hipGraphLaunch");
    } else {
        e = upload_table(p, sl, n, stream);
        if (e != hipSuccess)
            return hip_error(e, "table upload");
        const uint32_t grid = std::min<uint32_t>(tiles, 1u << 20);
        fk_status s = launch(p, cfg, sl.d_table, grid, n, stream, ev0, ev1);
        if (s)
            return s;
    }
    e = hipEventRecord(sl.done, stream);
    if (e != hipSuccess)
        return hip_error(e, "hipEventRecord");
    sl.used = true;
    return FK_OK;
}

extern "C" fk_status fk_run(fk_plan *plan, const fk_item *items, int32_t n_items, void *stream)
{
    try {
        if (!plan)
            return set_error(FK_ERR_INVALID_ARG, "plan is null");
        if (n_items < 1 || n_items > plan->max_batch)
            return set_error(FK_ERR_INVALID_ARG, "n_items %d outside 1..max_batch (%d)", n_items,
                             plan->max_batch);
        fk_status s = validate_items(&plan->chain, items, n_items);
        if (s)
            return s;
        return run_fused(plan, items, n_items, plan->cfg, plan->opts.use_graph != 0,
                         (hipStream_t)stream);
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

extern "C" fk_status fk_run_timed(fk_plan *plan, const fk_item *items, int32_t n_items,
                                  void *stream, void *start_event, void *stop_event)
{
    try {
        if (!plan)
            return set_error(FK_ERR_INVALID_ARG, "plan is null");
        if (n_items < 1 || n_items > plan->max_batch)
            return set_error(FK_ERR_INVALID_ARG, "n_items %d outside 1..max_batch (%d)", n_items,
                             plan->max_batch);
        fk_status s = validate_items(&plan->chain, items, n_items);
        if (s)
            return s;
        return run_fused(plan, items, n_items, plan->cfg, plan->opts.use_graph != 0,
                         (hipStream_t)stream, (hipEvent_t)start_event, (hipEvent_t)stop_event);
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

// ------------------------------------------------------------- autotune --

extern "C" int32_t fk_autotune_space(fk_launch_config *space, int32_t max_configs)
{
    int32_t n = 0;
    for (int t : {64, 128, 256, 512, 1024})
        for (int k : {1, 2, 4, 8}) {
            if (space && n < max_configs)
                space[n] = fk_launch_config{t, k};
            ++n;
        }
    return n;
}

extern "C" fk_status fk_autotune(fk_plan *plan, const fk_item *items, int32_t n_items, int32_t reps,
                                 float *times_ms, fk_launch_config *best)
{
    try {
        if (!plan)
            return set_error(FK_ERR_INVALID_ARG, "plan is null");
        if (n_items < 1 || n_items > plan->max_batch)
            return set_error(FK_ERR_INVALID_ARG, "n_items outside 1..max_batch");
        if (reps < 1 || reps > 10000)
            return set_error(FK_ERR_INVALID_ARG, "reps outside 1..10000");
        fk_status s = validate_items(&plan->chain, items, n_items);
        if (s)
            return s;
        hipError_t e;
        if (!plan->tune_stream) {
            e = hipStreamCreateWithFlags(&plan->tune_stream, hipStreamNonBlocking);
            if (e != hipSuccess)
                return hip_error(e, "hipStreamCreate");
        }
        fk_launch_config space[32];
        const int n = fk_autotune_space(space, 32);
        std::vector<float> med(n);
        hipEvent_t t0, t1;
        e = hipEventCreate(&t0);
        if (e == hipSuccess)
            e = hipEventCreate(&t1);
        if (e != hipSuccess)
            return hip_error(e, "hipEventCreate");
        s = FK_OK;
        // per config: one warm-up launch, then 3 samples of `reps`
        // back-to-back launches between two events; the per-launch time is
        // the median of the 3 sample averages
        for (int i = 0; i < n && !s; ++i) {
            std::vector<float> ts;
            s = run_fused(plan, items, n_items, space[i], false, plan->tune_stream);
            for (int r = 0; r < 3 && !s; ++r) {
                e = hipEventRecord(t0, plan->tune_stream);
                for (int k = 0; k < reps && e == hipSuccess && !s; ++k)
                    s = run_fused(plan, items, n_items, space[i], false, plan->tune_stream);
                if (e == hipSuccess && !s)
                    e = hipEventRecord(t1, plan->tune_stream);
                if (e == hipSuccess && !s)
                    e = hipEventSynchronize(t1);
                float ms = 0.0f;
                if (e == hipSuccess && !s)
                    e = hipEventElapsedTime(&ms, t0, t1);
                if (e != hipSuccess && !s)
                    s = hip_error(e, "autotune timing");
                ts.push_back(ms / (float)reps);
            }
            if (!s) {
                std::sort(ts.begin(), ts.end());
                med[i] = ts[1];
            }
        }
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
        if (s)
            return s;
        int bi = 0;
        for (int i = 1; i < n; ++i)  // strict < keeps the earlier (smaller T, then k) on ties
            if (med[i] < med[bi])
                bi = i;
        plan->cfg = space[bi];
        plan->opts.config_source = FK_CONFIG_AUTOTUNE;
        if (times_ms)
            for (int i = 0; i < n; ++i)
                times_ms[i] = med[i];
        if (best)
            *best = space[bi];
        return FK_OK;
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}
