// fk_server.cpp -- serving loop: FIFO admission against a device-memory
// budget, frames copied to the device on a copy stream and kept there,
// continuous batching of ready crops into fused launches on a compute
// stream, latency timestamps per request.
//
// Threads: callers only enqueue (submit), dequeue (poll) and mark releases
// under one mutex; a single scheduler thread owns every HIP call, the arena
// allocator and the launch bookkeeping.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <vector>

#include "../../include/fk.h"
#include "fk_arena.hpp"
#include "fk_host.hpp"
#include "fk_internal.hpp"

using namespace fk;

namespace {

int64_t align256(int64_t v) { return (v + 255) & ~(int64_t)255; }

struct Req {
    uint64_t ticket = 0;
    fk_request desc{};
    std::vector<fk_crop> crops;
    std::vector<int64_t> out_off;  // relative to the block
    int64_t frame_bytes = 0, out_bytes = 0, scratch_bytes = 0, block_bytes = 0;
    int64_t dev_pitch = 0;         // row pitch of the frame on the device
    int64_t off = -1;              // block offset in the arena
    const uint8_t *dev_frame = nullptr;  // the frame on the device (arena copy or caller's)
    hipEvent_t ready = nullptr;    // frame copy done (none for a frame already on the device)
    int launched = 0, done = 0;
    double t_admit = 0, t_launch = 0;
};

struct Launch {
    hipEvent_t done = nullptr;
    std::vector<std::pair<Req *, int>> parts;  // request, crops it carries
};

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace

struct fk_server {
    fk_server_opts opts{};
    fk_chain_desc chain{};
    std::vector<fk_op_desc> op_descs;
    fk_plan *plan = nullptr;
    hipStream_t copy_stream = nullptr, compute_stream = nullptr;
    int device = 0;
    int es_in = 1, es_out = 4, C = 3;
    std::unique_ptr<Arena> arena;
    int64_t budget = 0, in_use = 0;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::unique_ptr<Req>> incoming;  // submitted, not seen by the scheduler
    std::deque<fk_completion> completions;
    std::set<uint64_t> releasable;  // completions handed out by poll, not yet released
    std::vector<uint64_t> releases;
    fk_server_stats stats{};
    bool stop = false;
    std::atomic<bool> failed{false};
    std::string fail_msg;
    uint64_t next_ticket = 1;

    // scheduler-owned
    std::deque<std::unique_ptr<Req>> pending;   // waiting for memory
    std::deque<Req *> admitted;                 // on the device, crops not all done
    std::map<uint64_t, std::unique_ptr<Req>> live;
    std::deque<Launch> inflight;
    std::vector<hipEvent_t> event_pool;
    std::thread thread;
};

namespace {

hipEvent_t get_event(fk_server *s)
{
    if (!s->event_pool.empty()) {
        hipEvent_t e = s->event_pool.back();
        s->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
        return nullptr;
    return e;
}

void put_event(fk_server *s, hipEvent_t e)
{
    if (e)
        s->event_pool.push_back(e);
}

void fail(fk_server *s, const char *what, hipError_t e)
{
    std::lock_guard<std::mutex> g(s->mu);
    if (!s->failed.exchange(true))
        s->fail_msg = std::string(what) + ": " + hipGetErrorString(e);
}

void complete(fk_server *s, Req *r, int32_t status)
{
    fk_completion c{};
    c.ticket = r->ticket;
    c.status = status;
    c.n_crops = (int32_t)r->crops.size();
    c.outputs = (uint8_t *)s->opts.arena + r->off;
    c.output_bytes = r->out_bytes;
    c.t_arrival = r->desc.t_arrival;
    c.t_admit = r->t_admit;
    c.t_launch = r->t_launch;
    c.t_done = now_s();
    std::lock_guard<std::mutex> g(s->mu);
    s->completions.push_back(c);
    s->stats.completed += 1;
}

fk_item crop_item(fk_server *s, Req *r, int i)
{
    const fk_crop &c = r->crops[(size_t)i];
    fk_item it{};
    uint8_t *base = (uint8_t *)s->opts.arena + r->off;
    it.src.ptr = r->dev_frame;
    it.src.width = r->desc.width;
    it.src.height = r->desc.height;
    it.src.pitch_bytes = r->dev_pitch;
    it.x = c.x;
    it.y = c.y;
    it.w = c.w;
    it.h = c.h;
    it.dst = base + r->out_off[(size_t)i];
    it.out_w = c.out_w;
    it.out_h = c.out_h;
    return it;
}

// Queue the copy of a host frame into its block (after the outputs) on the
// copy stream, then the request's ready event.
hipError_t copy_frame(fk_server *s, Req *r)
{
    uint8_t *dframe = (uint8_t *)s->opts.arena + r->off + r->out_bytes;
    r->dev_frame = dframe;
    const int64_t row = (int64_t)r->desc.width * s->C * s->es_in;
    hipError_t e;
    if (r->dev_pitch == r->desc.pitch_bytes)  // one contiguous copy, rows keep their pitch
        e = hipMemcpyAsync(dframe, r->desc.frame, (size_t)((r->desc.height - 1) * r->dev_pitch + row),
                           hipMemcpyHostToDevice, s->copy_stream);
    else
        e = hipMemcpy2DAsync(dframe, (size_t)row, r->desc.frame, (size_t)r->desc.pitch_bytes,
                             (size_t)row, (size_t)r->desc.height, hipMemcpyHostToDevice,
                             s->copy_stream);
    if (e == hipSuccess && r->ready)
        e = hipEventRecord(r->ready, s->copy_stream);
    return e;
}

// Admit pending requests in order while memory allows; queue their copies.
bool admit(fk_server *s)
{
    bool progress = false;
    while (!s->pending.empty()) {
        Req *r = s->pending.front().get();
        if (s->in_use + r->block_bytes > s->budget)
            break;
        const int64_t off = s->arena->alloc(r->block_bytes);
        if (off < 0)
            break;
        r->off = off;
        r->t_admit = now_s();
        hipError_t e = hipSuccess;
        if (r->desc.frame_on_device) {
            r->dev_frame = (const uint8_t *)r->desc.frame;  // read in place
        } else {
            r->ready = get_event(s);
            e = copy_frame(s, r);
        }
        if (e != hipSuccess || (!r->desc.frame_on_device && !r->ready)) {
            fail(s, "frame copy", e);
            return progress;
        }
        s->in_use += r->block_bytes;
        s->admitted.push_back(r);
        s->live[r->ticket] = std::move(s->pending.front());
        s->pending.pop_front();
        progress = true;
        std::lock_guard<std::mutex> g(s->mu);
        s->stats.admitted += 1;
        s->stats.bytes_in_use = s->in_use;
        s->stats.peak_bytes = std::max(s->stats.peak_bytes, s->in_use);
        s->stats.pending = (int64_t)s->pending.size();
    }
    return progress;
}

// Build and issue one launch from the ready crops (mode dependent).
bool launch_one(fk_server *s)
{
    if ((int)s->inflight.size() >= s->opts.max_inflight)
        return false;
    std::vector<fk_item> items;
    Launch L;
    const int cap = s->opts.max_batch_items;
    for (Req *r : s->admitted) {
        if (r->launched == (int)r->crops.size())
            continue;
        if (r->ready) {
            const hipError_t q = hipEventQuery(r->ready);
            if (q == hipErrorNotReady)
                break;  // first in, first out: later requests wait for this frame
            if (q != hipSuccess) {
                fail(s, "frame copy", q);  // the scheduler completes everything with the error
                return false;
            }
        }
        if (s->opts.mode != FK_SERVER_BATCHED && !items.empty())
            break;  // one request per launch
        const int take = std::min((int)r->crops.size() - r->launched, cap - (int)items.size());
        for (int i = 0; i < take; ++i)
            items.push_back(crop_item(s, r, r->launched + i));
        if (r->launched == 0)
            r->t_launch = now_s();
        r->launched += take;
        L.parts.emplace_back(r, take);
        if ((int)items.size() >= cap || s->opts.mode != FK_SERVER_BATCHED)
            break;
    }
    if (items.empty())
        return false;
    fk_status st;
    if (s->opts.mode == FK_SERVER_UNFUSED) {
        Req *r = L.parts.front().first;
        uint8_t *scratch = (uint8_t *)s->opts.arena + r->off + r->out_bytes + r->frame_bytes;
        st = fk_run_unfused(s->plan, items.data(), (int32_t)items.size(), scratch, r->scratch_bytes,
                            s->compute_stream);
    } else {
        st = fk_run(s->plan, items.data(), (int32_t)items.size(), s->compute_stream);
    }
    L.done = get_event(s);
    hipError_t e = L.done ? hipEventRecord(L.done, s->compute_stream) : hipErrorOutOfMemory;
    if (st != FK_OK || e != hipSuccess) {
        fail(s, "launch", e == hipSuccess ? hipErrorLaunchFailure : e);
        put_event(s, L.done);
        return false;
    }
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stats.launches += 1;
        s->stats.crops_launched += (int64_t)items.size();
    }
    s->inflight.push_back(std::move(L));
    return true;
}

bool retire(fk_server *s)
{
    bool progress = false;
    while (!s->inflight.empty()) {
        Launch &L = s->inflight.front();
        const hipError_t q = hipEventQuery(L.done);
        if (q == hipErrorNotReady)
            break;
        if (q != hipSuccess) {
            fail(s, "kernel", q);
            break;
        }
        for (auto &pr : L.parts) {
            Req *r = pr.first;
            r->done += pr.second;
            if (r->done == (int)r->crops.size()) {
                complete(s, r, FK_OK);
                s->admitted.erase(std::find(s->admitted.begin(), s->admitted.end(), r));
                put_event(s, r->ready);
                r->ready = nullptr;
            }
        }
        put_event(s, L.done);
        s->inflight.pop_front();
        progress = true;
    }
    return progress;
}

void apply_releases(fk_server *s, std::vector<uint64_t> &rel)
{
    for (uint64_t t : rel) {
        auto it = s->live.find(t);
        if (it == s->live.end())
            continue;
        Req *r = it->second.get();
        s->arena->release(r->off, r->block_bytes);
        s->in_use -= r->block_bytes;
        s->live.erase(it);
    }
    rel.clear();
}

void scheduler(fk_server *s)
{
    (void)hipSetDevice(s->device);
    std::vector<uint64_t> rel;
    for (;;) {
        bool stopping;
        {
            std::unique_lock<std::mutex> g(s->mu);
            const bool idle = s->pending.empty() && s->admitted.empty() && s->inflight.empty() &&
                              s->incoming.empty() && s->releases.empty();
            if (idle && !s->stop)
                s->cv.wait_for(g, std::chrono::milliseconds(2));
            while (!s->incoming.empty()) {
                s->pending.push_back(std::move(s->incoming.front()));
                s->incoming.pop_front();
            }
            rel.swap(s->releases);
            stopping = s->stop;
            s->stats.bytes_in_use = s->in_use;
        }
        apply_releases(s, rel);
        if (s->failed.load()) {
            // complete everything outstanding with the failure status
            while (!s->inflight.empty()) {
                (void)hipEventSynchronize(s->inflight.front().done);
                s->inflight.pop_front();
            }
            for (Req *r : s->admitted)
                complete(s, r, FK_ERR_HIP);
            s->admitted.clear();
            while (!s->pending.empty()) {
                Req *r = s->pending.front().get();
                r->off = 0;
                complete(s, r, FK_ERR_HIP);
                s->pending.pop_front();
            }
            if (stopping)
                break;
            std::this_thread::sleep_for(std::chrono::microseconds(200));
            continue;
        }
        if (stopping && s->pending.empty() && s->admitted.empty() && s->inflight.empty())
            break;
        bool progress = retire(s);
        progress |= admit(s);
        while (launch_one(s))
            progress = true;
        // with launches in flight or frames copying, poll again at once
        // (a short sleep lasts the kernel's timer slack, ~50 us, which would
        // add that much to a request's latency); the thread gives up its
        // core to other threads between polls
        if (!progress && (!s->inflight.empty() || !s->admitted.empty()))
            std::this_thread::yield();
    }
}

}  // namespace

extern "C" double fk_server_clock(void) { return now_s(); }

extern "C" fk_status fk_server_create(const fk_server_opts *opts, fk_server **out)
{
    try {
        if (!opts || !out)
            return set_error(FK_ERR_INVALID_ARG, "null argument");
        *out = nullptr;
        fk_status st = validate_chain(opts->chain);
        if (st)
            return st;
        if (opts->chain->read.kind != FK_READ_CROP_RESIZE || opts->chain->write.layout == FK_STATS)
            return set_error(FK_ERR_UNSUPPORTED, "the server runs crop+resize chains with an image write");
        if (!opts->arena || opts->arena_bytes < 4096)
            return set_error(FK_ERR_INVALID_ARG, "arena missing or too small");
        if (opts->budget_bytes < 0 || opts->budget_bytes > opts->arena_bytes)
            return set_error(FK_ERR_INVALID_ARG, "budget outside 0..arena_bytes");
        if (opts->max_batch_items < 1 || opts->max_batch_items > 65536 || opts->max_inflight < 1 ||
            opts->max_inflight > fk_plan::kRing)
            return set_error(FK_ERR_INVALID_ARG, "max_batch_items 1..65536, max_inflight 1..%d",
                             fk_plan::kRing);
        if (opts->mode < FK_SERVER_BATCHED || opts->mode > FK_SERVER_UNFUSED)
            return set_error(FK_ERR_INVALID_ARG, "unknown mode");
        if ((uintptr_t)opts->arena % 256 != 0)
            return set_error(FK_ERR_INVALID_ARG, "arena must be 256-byte aligned");
        std::unique_ptr<fk_server> s(new fk_server());
        s->opts = *opts;
        s->op_descs.assign(opts->chain->ops, opts->chain->ops + opts->chain->n_ops);
        s->chain = *opts->chain;
        s->chain.ops = s->op_descs.data();
        s->opts.chain = &s->chain;
        s->C = s->chain.read.channels;
        s->es_in = dtype_size(s->chain.read.in_dtype);
        s->es_out = dtype_size(s->chain.write.out_dtype);
        s->budget = opts->budget_bytes ? opts->budget_bytes : opts->arena_bytes;
        s->arena.reset(new Arena(opts->arena_bytes));
        hipError_t e = hipGetDevice(&s->device);
        if (e == hipSuccess)
            e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipStreamCreateWithFlags(&s->compute_stream, hipStreamNonBlocking);
        if (e != hipSuccess)
            return hip_error(e, "server streams");
        fk_plan_opts po = {FK_CONFIG_DEFAULT, {256, 1}, 0, opts->strict_fp, FK_TIER_AUTO, 0,
                           FK_GATHER_DIRECT};
        if (opts->config.block_threads != 0) {
            po.config_source = FK_CONFIG_MANUAL;
            po.manual = opts->config;
        }
        const int cap = opts->mode == FK_SERVER_UNFUSED ? 1 : opts->max_batch_items;
        st = fk_plan_create(&s->chain, std::max(cap, opts->max_batch_items), &po, &s->plan);
        if (st) {
            (void)hipStreamDestroy(s->copy_stream);
            (void)hipStreamDestroy(s->compute_stream);
            return st;
        }
        fk_server *raw = s.release();
        raw->thread = std::thread(scheduler, raw);
        *out = raw;
        return FK_OK;
    } catch (const std::bad_alloc &) {
        return set_error(FK_ERR_OUT_OF_MEMORY, "host allocation");
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

extern "C" fk_status fk_server_submit(fk_server *s, const fk_request *req, uint64_t *ticket)
{
    try {
        if (!s || !req || !ticket)
            return set_error(FK_ERR_INVALID_ARG, "null argument");
        if (s->failed.load()) {
            // fail() writes the message under the mutex after raising the flag
            std::lock_guard<std::mutex> g(s->mu);
            return set_error(FK_ERR_BAD_STATE, "server failed: %s", s->fail_msg.c_str());
        }
        if (!req->frame || req->width < 1 || req->height < 1 ||
            req->pitch_bytes < (int64_t)req->width * s->C * s->es_in)
            return set_error(FK_ERR_INVALID_ARG, "bad frame");
        if (req->n_crops < 1 || req->n_crops > s->opts.max_batch_items || !req->crops)
            return set_error(FK_ERR_INVALID_ARG, "n_crops outside 1..max_batch_items");
        std::unique_ptr<Req> r(new Req());
        r->desc = *req;
        r->crops.assign(req->crops, req->crops + req->n_crops);
        r->desc.crops = nullptr;
        int64_t off = 0;
        for (const fk_crop &c : r->crops) {
            if (c.w < 1 || c.h < 1 || c.x < 0 || c.y < 0 || (int64_t)c.x + c.w > req->width ||
                (int64_t)c.y + c.h > req->height || c.out_w < 1 || c.out_h < 1)
                return set_error(FK_ERR_INVALID_ARG, "crop outside the frame or empty output");
            r->out_off.push_back(off);
            off = align256(off + (int64_t)c.out_w * c.out_h * s->C * s->es_out);
        }
        r->out_bytes = off;
        if (req->frame_on_device != 0 && req->frame_on_device != 1)
            return set_error(FK_ERR_INVALID_ARG, "frame_on_device must be 0 or 1");
        if (req->frame_on_device) {
            // the kernels read the frame in place: it must be device memory
            hipPointerAttribute_t attr;
            std::memset(&attr, 0, sizeof attr);
            const hipError_t e = hipPointerGetAttributes(&attr, req->frame);
            if (e != hipSuccess ||
                (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)) {
                (void)hipGetLastError();  // clear the failed query's error
                return set_error(FK_ERR_INVALID_ARG, "frame_on_device: the frame is not device memory");
            }
        }
        const int64_t row = (int64_t)req->width * s->C * s->es_in;
        if (req->frame_on_device) {
            // read in place: no copy, no frame bytes in the block
            r->dev_pitch = req->pitch_bytes;
            r->frame_bytes = 0;
        } else {
            // a pitched frame is copied in one piece (rows keep the host
            // pitch) unless its padding would more than double the bytes moved
            r->dev_pitch = req->pitch_bytes <= 2 * row ? req->pitch_bytes : row;
            r->frame_bytes = align256((int64_t)(req->height - 1) * r->dev_pitch + row);
        }
        if (s->opts.mode == FK_SERVER_UNFUSED) {
            int64_t need = 0;
            for (int i = 0; i < req->n_crops; ++i) {
                fk_item it{};
                it.src.ptr = (void *)(uintptr_t)256;
                it.src.width = req->width;
                it.src.height = req->height;
                it.src.pitch_bytes = r->dev_pitch;
                const fk_crop &c = r->crops[(size_t)i];
                it.x = c.x;
                it.y = c.y;
                it.w = c.w;
                it.h = c.h;
                it.dst = (void *)(uintptr_t)256;
                it.out_w = c.out_w;
                it.out_h = c.out_h;
                int64_t b = 0;
                fk_status st = fk_unfused_scratch_bytes(s->plan, &it, 1, &b);
                if (st)
                    return st;
                need = std::max(need, b);
            }
            r->scratch_bytes = align256(need);
        }
        r->block_bytes = r->out_bytes + r->frame_bytes + r->scratch_bytes;
        if (r->block_bytes > s->budget)
            return set_error(FK_ERR_BUDGET, "request needs %lld bytes, budget %lld",
                             (long long)r->block_bytes, (long long)s->budget);
        {
            std::lock_guard<std::mutex> g(s->mu);
            if (s->stop)
                return set_error(FK_ERR_BAD_STATE, "server is stopping");
            r->ticket = s->next_ticket++;
            *ticket = r->ticket;
            s->incoming.push_back(std::move(r));
            s->stats.submitted += 1;
            s->stats.pending += 1;
        }
        s->cv.notify_one();
        return FK_OK;
    } catch (const std::bad_alloc &) {
        return set_error(FK_ERR_OUT_OF_MEMORY, "host allocation");
    } catch (...) {
        return set_error(FK_ERR_INVALID_ARG, "exception");
    }
}

extern "C" fk_status fk_server_poll(fk_server *s, fk_completion *out, int32_t max, int32_t *n)
{
    try {
        if (!s || !n || (max > 0 && !out) || max < 0)
            return set_error(FK_ERR_INVALID_ARG, "bad argument");
        std::lock_guard<std::mutex> g(s->mu);
        int32_t k = 0;
        while (k < max && !s->completions.empty()) {
            out[k] = s->completions.front();
            s->releasable.insert(out[k].ticket);
            s->completions.pop_front();
            ++k;
        }
        *n = k;
        return FK_OK;
    } catch (...) {
        return set_error(FK_ERR_BAD_STATE, "exception");
    }
}

extern "C" fk_status fk_server_release(fk_server *s, uint64_t ticket)
{
    try {
        if (!s)
            return set_error(FK_ERR_INVALID_ARG, "server is null");
        {
            // only a request whose completion the caller has polled may
            // return its block to the arena: one still queued, copying or
            // running keeps its memory
            std::lock_guard<std::mutex> g(s->mu);
            auto it = s->releasable.find(ticket);
            if (it == s->releasable.end())
                return set_error(FK_ERR_BAD_STATE,
                                 "ticket %llu is not completed, unknown or already released",
                                 (unsigned long long)ticket);
            s->releasable.erase(it);
            s->releases.push_back(ticket);
        }
        s->cv.notify_one();
        return FK_OK;
    } catch (...) {
        return set_error(FK_ERR_OUT_OF_MEMORY, "exception");
    }
}

extern "C" fk_status fk_server_stats_get(fk_server *s, fk_server_stats *out)
{
    try {
        if (!s || !out)
            return set_error(FK_ERR_INVALID_ARG, "null argument");
        std::lock_guard<std::mutex> g(s->mu);
        *out = s->stats;
        return FK_OK;
    } catch (...) {
        return set_error(FK_ERR_BAD_STATE, "exception");
    }
}

extern "C" fk_status fk_server_destroy(fk_server *s)
{
    if (!s)
        return FK_OK;
    try {
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->stop = true;
        }
        s->cv.notify_one();
        if (s->thread.joinable())
            s->thread.join();
    } catch (...) {
        // the scheduler could not be joined: its thread may still use the
        // server, so nothing is freed
        return set_error(FK_ERR_BAD_STATE, "scheduler thread could not be joined");
    }
    (void)hipStreamSynchronize(s->copy_stream);
    (void)hipStreamSynchronize(s->compute_stream);
    for (auto &kv : s->live)
        if (kv.second->ready)
            (void)hipEventDestroy(kv.second->ready);
    for (hipEvent_t e : s->event_pool)
        (void)hipEventDestroy(e);
    fk_plan_destroy(s->plan);
    (void)hipStreamDestroy(s->copy_stream);
    (void)hipStreamDestroy(s->compute_stream);
    delete s;
    return FK_OK;
}
