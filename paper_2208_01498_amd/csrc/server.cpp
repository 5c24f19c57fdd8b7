// Serving loop: continuous batching of amplitude requests.
//
// A scheduler thread takes queued requests in arrival order, merges queued
// requests on the same plan and precision into one device batch (up to
// max_batch bitstrings), admits the batch when an execution slot is idle and
// the arena can hold the plan's workspace for it (the workspace of a chunk
// of one bitstring at least; larger chunks when memory allows), and hands it
// to the slot.  A batch whose algorithmic work reaches the heavy threshold
// counts against a limit of concurrently running heavy batches, so light
// requests keep finding a slot beside long contractions; a batch that
// cannot start does not block the ones queued behind it.  Each slot owns a HIP stream and a worker thread, so admitted
// batches run concurrently on the device while new requests keep arriving.
// A result does not depend on what it was batched or overlapped with: the
// per-bitstring arithmetic is the same for any chunk size.
#include <algorithm>

#include "tn_internal.h"

namespace tn {

bool arena_alloc(tn_ctx* ctx, size_t bytes, size_t* off) {
    for (auto it = ctx->free_list.begin(); it != ctx->free_list.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            size_t rest = it->second - bytes;
            size_t noff = it->first + bytes;
            ctx->free_list.erase(it);
            if (rest) ctx->free_list[noff] = rest;
            return true;
        }
    }
    return false;
}

void arena_free(tn_ctx* ctx, size_t off, size_t bytes) {
    auto it = ctx->free_list.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != ctx->free_list.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        ctx->free_list.erase(nx);
    }
    if (it != ctx->free_list.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            ctx->free_list.erase(it);
        }
    }
}

size_t largest_free(tn_ctx* ctx) {
    size_t m = 0;
    for (auto& kv : ctx->free_list) m = std::max(m, kv.second);
    return m;
}

static void worker(tn_ctx* ctx, Slot* sl) {
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> lk(ctx->smu);
    for (;;) {
        sl->cv.wait(lk, [&] { return sl->has_job || ctx->stop; });
        if (ctx->stop && !sl->has_job) return;
        auto job = sl->job;
        const tn_plan* plan = sl->plan;
        int prec = sl->precision;
        size_t off = sl->off, bytes = sl->bytes;
        const int sr = sl->shape_r, sc = sl->shape_chunk;
        lk.unlock();
        std::vector<uint64_t> bits;
        for (auto& r : job) bits.insert(bits.end(), r->bits.begin(), r->bits.end());
        std::vector<double> res(2 * bits.size());
        int64_t t0 = now_ns();
        for (auto& r : job) r->st.t_start_ns = t0;
        int rc = execute(ctx, plan, bits.data(), (int)bits.size(), prec, sl->stream,
                         ctx->arena + off, bytes, res.data(), nullptr, sr, sc);
        int64_t t1 = now_ns();
        lk.lock();
        size_t pos = 0;
        for (auto& r : job) {
            r->st.t_end_ns = t1;
            r->st.batch = (int)bits.size();
            if (r->cancelled) r->status = TN_ECANCELLED;
            else if (rc != TN_OK) r->status = rc;
            else {
                r->result.assign(res.begin() + 2 * pos, res.begin() + 2 * (pos + r->bits.size()));
                r->status = TN_OK;
            }
            pos += r->bits.size();
            const_cast<tn_plan*>(r->plan)->pending--;
        }
        arena_free(ctx, off, bytes);
        sl->job.clear();
        sl->has_job = false;
        sl->busy = false;
        ctx->scv.notify_all();
    }
}

static void scheduler(tn_ctx* ctx) {
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> lk(ctx->smu);
    for (;;) {
        ctx->scv.wait(lk, [&] {
            if (ctx->stop) return true;
            if (ctx->queue.empty()) return false;
            for (auto& s : ctx->slots)
                if (!s->busy) return true;
            return false;
        });
        if (ctx->stop) return;
        Slot* slot = nullptr;
        bool any_busy = false;
        int heavy_busy = 0;
        for (auto& s : ctx->slots) {
            if (!s->busy && !slot) slot = s.get();
            any_busy |= s->busy;
            heavy_busy += s->busy && s->heavy;
        }
        if (!slot) continue;
        // first admissible batch in arrival order: a queued request plus the
        // later ones on the same plan and precision (up to max_batch); a
        // batch that cannot start now (memory, or the heavy-batch limit)
        // does not hold back the requests behind it
        bool admitted = false;
        for (auto hit = ctx->queue.begin(); hit != ctx->queue.end(); ++hit) {
            auto head = *hit;
            tn_plan* plan = const_cast<tn_plan*>(head->plan);
            int total = 0;
            for (auto it = hit; it != ctx->queue.end(); ++it) {
                auto& r = *it;
                if (r->plan == head->plan && r->precision == head->precision && !r->cancelled &&
                    (total == 0 || total + (int)r->bits.size() <= ctx->max_batch))
                    total += (int)r->bits.size();
            }
            const bool heavy = plan->host.flops_total_per_b * total >= ctx->heavy_flops;
            if (heavy && heavy_busy >= ctx->max_heavy) continue;
            const size_t avail = largest_free(ctx);
            const bool scales = head->precision == TN_SPLIT_FP16;
            const size_t need1 = plan->mem(1, 0, scales).bytes;
            if (need1 > avail) {
                if (!any_busy) {
                    // the whole arena is free and still too small
                    ctx->queue.erase(hit);
                    head->status = TN_ENOMEM;
                    plan->pending--;
                    admitted = true;     // the queue changed: scan again
                    break;
                }
                continue;
            }
            std::vector<std::shared_ptr<Request>> job;
            int taken = 0;
            for (auto it = hit; it != ctx->queue.end();) {
                auto& r = *it;
                if (r->plan == head->plan && r->precision == head->precision && !r->cancelled &&
                    (job.empty() || taken + (int)r->bits.size() <= ctx->max_batch)) {
                    taken += (int)r->bits.size();
                    job.push_back(r);
                    it = ctx->queue.erase(it);
                } else {
                    ++it;
                }
            }
            // execution shape for the free region, one batch taking at most
            // half of the arena when it can run in less; reserve exactly
            // that shape's workspace
            int r = 0, ch = 0;
            const size_t cap = std::max(need1, std::min(avail, ctx->arena_bytes / 2));
            choose_shape(plan, taken, cap, ctx->force_slice_block, r, ch, scales);
            const size_t bytes = plan->mem(ch, r, scales).bytes;
            size_t off = 0;
            arena_alloc(ctx, bytes, &off);
            const int64_t t = now_ns();
            for (auto& q : job) q->st.t_admit_ns = t;
            slot->busy = true;
            slot->heavy = heavy;
            slot->job = job;
            slot->plan = plan;
            slot->precision = head->precision;
            slot->off = off;
            slot->bytes = bytes;
            slot->shape_r = r;
            slot->shape_chunk = ch;
            slot->has_job = true;
            slot->cv.notify_all();
            admitted = true;
            break;
        }
        if (!admitted) ctx->scv.wait(lk);
    }
}

static int ensure_server(tn_ctx* ctx) {
    if (ctx->sched_started) return TN_OK;
    (void)hipSetDevice(ctx->device);
    for (int i = 0; i < ctx->n_slots; ++i) {
        std::unique_ptr<Slot> s(new Slot());
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            set_error("stream creation failed");
            return TN_EDEVICE;
        }
        ctx->slots.push_back(std::move(s));
    }
    for (auto& s : ctx->slots) s->th = std::thread(worker, ctx, s.get());
    ctx->sched = std::thread(scheduler, ctx);
    ctx->sched_started = true;
    return TN_OK;
}

}  // namespace tn

using namespace tn;

extern "C" {

int tn_server_config(tn_ctx* ctx, int32_t n_slots, int32_t max_batch) {
    if (!ctx || n_slots < 1 || n_slots > 16 || max_batch < 1) { set_error("bad server config"); return TN_EINVAL; }
    std::lock_guard<std::mutex> g(ctx->smu);
    if (ctx->sched_started) { set_error("server already running"); return TN_EBUSY; }
    ctx->n_slots = n_slots;
    ctx->max_batch = max_batch;
    return TN_OK;
}

int tn_server_set_heavy(tn_ctx* ctx, double heavy_flops, int32_t max_heavy) {
    if (!ctx || !(heavy_flops >= 0) || max_heavy < 1) { set_error("bad heavy-batch limit"); return TN_EINVAL; }
    std::lock_guard<std::mutex> g(ctx->smu);
    ctx->heavy_flops = heavy_flops;
    ctx->max_heavy = max_heavy;
    ctx->scv.notify_all();
    return TN_OK;
}

int tn_server_stop(tn_ctx* ctx) {
    {
        std::lock_guard<std::mutex> g(ctx->smu);
        if (!ctx->sched_started) return TN_OK;
        ctx->stop = true;
        ctx->scv.notify_all();
        for (auto& s : ctx->slots) s->cv.notify_all();
    }
    if (ctx->sched.joinable()) ctx->sched.join();
    for (auto& s : ctx->slots) {
        if (s->th.joinable()) s->th.join();
        (void)hipStreamDestroy(s->stream);
    }
    ctx->slots.clear();
    ctx->sched_started = false;
    return TN_OK;
}

int tn_submit(tn_ctx* ctx, const tn_plan* plan, const uint64_t* bits, int32_t nb, int32_t precision,
              uint64_t* ticket) {
    if (!ctx || !plan || !bits || !ticket) { set_error("null argument"); return TN_EINVAL; }
    if (nb <= 0) { set_error("nb must be positive"); return TN_EINVAL; }
    if (!precision_ok(precision)) { set_error("precision mode not available"); return TN_EINVAL; }
    if (ctx->poisoned) { set_error("context poisoned"); return TN_EDEVICE; }
    for (int i = 0; i < nb; ++i)
        if (bits[i] & ~plan->host.out_mask) { set_error("bitstring has a bit at a position >= n_qubits"); return TN_EINVAL; }
    if (const_cast<tn_plan*>(plan)->mem(1, 0, precision == TN_SPLIT_FP16).bytes > ctx->arena_bytes) {
        set_error("one bitstring of this plan needs more workspace than the arena holds");
        return TN_ENOMEM;
    }
    auto r = std::make_shared<Request>();
    r->plan = plan;
    r->bits.assign(bits, bits + nb);
    r->precision = precision;
    r->st.t_arrive_ns = now_ns();
    r->st.plan_id = plan->id;
    std::lock_guard<std::mutex> g(ctx->smu);
    int rc = ensure_server(ctx);
    if (rc) return rc;
    r->ticket = ctx->next_ticket++;
    const_cast<tn_plan*>(plan)->pending++;
    ctx->reqs[r->ticket] = r;
    ctx->queue.push_back(r);
    *ticket = r->ticket;
    ctx->scv.notify_all();
    return TN_OK;
}

int tn_poll(tn_ctx* ctx, uint64_t ticket, double* out_re_im, tn_req_stats* st) {
    if (!ctx) return TN_EINVAL;
    std::lock_guard<std::mutex> g(ctx->smu);
    auto it = ctx->reqs.find(ticket);
    if (it == ctx->reqs.end()) { set_error("unknown ticket"); return TN_ENOTFOUND; }
    auto r = it->second;
    if (r->status == TN_PENDING) return TN_PENDING;
    if (st) *st = r->st;
    if (r->status == TN_OK && out_re_im) std::copy(r->result.begin(), r->result.end(), out_re_im);
    int s = r->status;
    ctx->reqs.erase(it);
    if (s == TN_ECANCELLED) set_error("request cancelled");
    return s;
}

int tn_cancel(tn_ctx* ctx, uint64_t ticket) {
    if (!ctx) return TN_EINVAL;
    std::lock_guard<std::mutex> g(ctx->smu);
    auto it = ctx->reqs.find(ticket);
    if (it == ctx->reqs.end()) { set_error("unknown ticket"); return TN_ENOTFOUND; }
    it->second->cancelled = true;
    for (auto q = ctx->queue.begin(); q != ctx->queue.end(); ++q)
        if ((*q)->ticket == ticket) {
            (*q)->status = TN_ECANCELLED;
            const_cast<tn_plan*>((*q)->plan)->pending--;
            ctx->queue.erase(q);
            break;
        }
    return TN_OK;
}

}  // extern "C"
