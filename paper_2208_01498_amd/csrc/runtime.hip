// Context, plan residency and the executor of the amplitude engine.
//
// The executor walks the plan's pairwise steps for every slice of a chunk of
// bitstrings: leaves are gathered (bitstring bits replace output labels,
// slice bits replace sliced labels), operands that do not fit the step's
// batched-GEMM form are permuted, the step's complex GEMM writes the result,
// and after the last step the chunk's scalars are added in float64 to the
// per-bitstring accumulators (slices in ascending order).  A step whose
// subtree depends only on slice bits that did not change since the previous
// slice keeps its previous result.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <limits>
#include <mutex>

#include "kernels.h"
#include "tn_internal.h"

namespace tn {

static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

#define HIPCHK(ctx, expr)                                                        \
    do {                                                                         \
        hipError_t e_ = (expr);                                                  \
        if (e_ != hipSuccess) {                                                  \
            set_error(std::string("HIP error: ") + hipGetErrorString(e_) +       \
                      " at " #expr);                                             \
            if (ctx) (ctx)->poisoned = true;                                     \
            return TN_EDEVICE;                                                   \
        }                                                                        \
    } while (0)

static void fill_perm(PermArgs& pa, const int* map, int r) {
    int inv[kMaxRank];
    for (int p = 0; p < r; ++p) inv[map[p]] = p;
    const int target = std::min(r, 12);
    std::vector<char> inT(r, 0);
    int a = 0, c = 0, t = 0;
    auto add = [&](int q) { if (!inT[q]) { inT[q] = 1; ++t; } };
    while (t < target) {
        if (a <= c && a < r) add(a++);
        else if (c < r) add(map[c++]);
        else if (a < r) add(a++);
        else break;
    }
    pa.rank = r;
    pa.nt = t;
    int m = 0;
    for (int q = 0; q < r; ++q)
        if (inT[q]) pa.t_in[m++] = q;
    m = 0;
    for (int p = 0; p < r; ++p)
        if (inT[map[p]]) {
            pa.t_out[m] = p;
            int rk = 0;
            while (pa.t_in[rk] != map[p]) ++rk;
            pa.t_rank[m] = rk;
            ++m;
        }
    m = 0;
    for (int q = 0; q < r; ++q)
        if (!inT[q]) {
            pa.n_in[m] = q;
            pa.n_out[m] = inv[q];
            ++m;
        }
    pa.nn = m;
}

// Execution shape for a workspace: r low slice bits are computed together
// as a slice block (2^r slices per pass), `chunk` bitstrings per pass.  The
// largest block that fits with at least one bitstring is taken (a forced r
// from the context option wins when it fits), then the largest chunk.
bool choose_shape(const tn_plan* plan, int nb, size_t ws_bytes, int force_r, int& r_out,
                  int& chunk_out, bool scales) {
    tn_plan* pl = const_cast<tn_plan*>(plan);
    const int S = (int)plan->host.sliced.size();
    int r = -1;
    if (force_r >= 0 && force_r <= S && pl->mem(1, force_r, scales).bytes <= ws_bytes) r = force_r;
    for (int rr = S; r < 0 && rr >= 0; --rr)
        if (pl->mem(1, rr, scales).bytes <= ws_bytes) r = rr;
    if (r < 0) return false;
    int lo = 1, hi = nb;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (pl->mem(mid, r, scales).bytes <= ws_bytes) lo = mid;
        else hi = mid - 1;
    }
    r_out = r;
    chunk_out = lo;
    return true;
}

static void add_stats(tn_exec_stats& a, const tn_exec_stats& d, int sign) {
    a.kernels_gemm += sign * d.kernels_gemm;
    a.kernels_permute += sign * d.kernels_permute;
    a.kernels_gather += sign * d.kernels_gather;
    a.steps_executed += sign * d.steps_executed;
    a.steps_reused += sign * d.steps_reused;
    a.algorithmic_flops += sign * d.algorithmic_flops;
    a.permute_bytes += sign * d.permute_bytes;
    for (int i = 0; i < kKernelClasses; ++i) {
        a.launches[i] += sign * d.launches[i];
        a.flops[i] += sign * d.flops[i];
        a.bytes[i] += sign * d.bytes[i];
    }
}

// Run the kernels of one chunk: directly the first time a (plan, workspace,
// chunk size, bitstrings in this chunk, slice block, precision) shape is
// seen, captured into a HIP graph the second time, replayed with one launch
// after that.  The chunk size is part of the key because the workspace
// layout (tensor offsets, the bitstring and accumulator slots) is planned
// for it: a last chunk of 10 bitstrings under a chunk size of 20 does not
// issue the launches of a call whose chunk size is 10.  Graphs are off
// while per-launch events are recorded, and once a context holds
// kMaxGraphs of them.
static constexpr size_t kMaxGraphs = 256;

template <class F>
static int run_chunk(tn_ctx* ctx, const tn_plan* plan, const char* ws, int chunk, int cb, int r,
                     int precision, hipStream_t stream, bool graphable, tn_exec_stats& es,
                     F&& launches) {
    graphable = graphable && ctx && ctx->use_graphs;
    hipGraphExec_t replay = nullptr;
    tn_exec_stats delta{};
    bool capture = false;
    const auto key = std::make_tuple(plan, ws, chunk, cb, r, precision);
    if (graphable) {
        std::lock_guard<std::mutex> g(ctx->gmu);
        auto it = ctx->graphs.find(key);
        if (it == ctx->graphs.end()) {
            if (ctx->graphs.size() < kMaxGraphs) ctx->graphs[key].stamp = ++ctx->graph_clock;
        } else if (it->second.exec) {
            replay = it->second.exec;
            delta = it->second.delta;
        } else {
            capture = true;
        }
    }
    if (replay) {
        HIPCHK(ctx, hipGraphLaunch(replay, stream));
        add_stats(es, delta, 1);
        es.graph_replays++;
        return TN_OK;
    }
    if (!capture) return launches();
    const tn_exec_stats before = es;
    HIPCHK(ctx, hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    const int rc = launches();
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(stream, &graph);
    if (rc || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (rc) return rc;
        set_error(std::string("HIP error: ") + hipGetErrorString(e) + " at hipStreamEndCapture");
        ctx->poisoned = true;
        return TN_EDEVICE;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        set_error(std::string("HIP error: ") + hipGetErrorString(ei) + " at hipGraphInstantiate");
        ctx->poisoned = true;
        return TN_EDEVICE;
    }
    delta = es;
    add_stats(delta, before, -1);
    {
        std::lock_guard<std::mutex> g(ctx->gmu);
        auto& ent = ctx->graphs[key];
        if (ent.exec) {
            // captured meanwhile by another call of the same shape: keep that one
            (void)hipGraphExecDestroy(exec);
            exec = ent.exec;
        } else {
            ent.exec = exec;
            ent.delta = delta;
        }
    }
    HIPCHK(ctx, hipGraphLaunch(exec, stream));
    return TN_OK;
}

// drop the graphs of one plan (all plans when plan is null)
void drop_graphs(tn_ctx* ctx, const tn_plan* plan) {
    std::lock_guard<std::mutex> g(ctx->gmu);
    for (auto it = ctx->graphs.begin(); it != ctx->graphs.end();) {
        if (!plan || std::get<0>(it->first) == plan) {
            if (it->second.exec) (void)hipGraphExecDestroy(it->second.exec);
            it = ctx->graphs.erase(it);
        } else {
            ++it;
        }
    }
}

int execute(tn_ctx* ctx, const tn_plan* plan, const uint64_t* bits, int nb, int precision,
            hipStream_t stream, char* ws, size_t ws_bytes, double* out, tn_exec_stats* stats,
            int shape_r, int shape_chunk) {
    const PlanHost& p = plan->host;
    tn_plan* pl = const_cast<tn_plan*>(plan);
    tn_exec_stats es{};
    int r = shape_r, chunk = shape_chunk;
    const bool scales = precision == TN_SPLIT_FP16;
    if (shape_chunk > 0 && pl->mem(shape_chunk, shape_r, scales).bytes <= ws_bytes) {
        // shape fixed by the caller (the serving loop reserved its memory)
    } else if (!choose_shape(plan, nb, ws_bytes, ctx ? ctx->force_slice_block : -1, r, chunk, scales)) {
        set_error("one bitstring of this plan needs more workspace than available");
        return TN_ENOMEM;
    }
    const MemPlan& mp = pl->mem(chunk, r, scales);
    const int S = (int)p.sliced.size();
    const int R = 1 << r;
    const uint32_t low = (uint32_t)R - 1;
    const uint64_t ngroups = 1ull << (S - r);
    const int nL = (int)p.leaves.size();
    es.chunk = chunk;
    es.slice_block = R;
    // event timing: pairs (start, end) per launch, harvested at every chunk
    // end and whenever the pool is used up
    const bool prof = ctx && ctx->profile && stats;
    struct Rec { int kind; };
    std::vector<Rec> recs;
    size_t ev_used = 0;
    auto harvest = [&]() -> int {
        if (!prof || recs.empty()) return TN_OK;
        HIPCHK(ctx, hipStreamSynchronize(stream));
        for (size_t i = 0; i < recs.size(); ++i) {
            float ms = 0.f;
            HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->events[2 * i], ctx->events[2 * i + 1]));
            es.time_ms[recs[i].kind] += ms;
        }
        recs.clear();
        ev_used = 0;
        return TN_OK;
    };
    auto ev_begin = [&]() -> int {
        if (!prof) return TN_OK;
        if (ev_used + 2 > 8192) { int rc = harvest(); if (rc) return rc; }
        while (ctx->events.size() < ev_used + 2) {
            hipEvent_t e;
            HIPCHK(ctx, hipEventCreate(&e));
            ctx->events.push_back(e);
        }
        HIPCHK(ctx, hipEventRecord(ctx->events[ev_used], stream));
        return TN_OK;
    };
    auto ev_end = [&](int kind, double flops, double bytes) -> int {
        es.launches[kind]++;
        es.flops[kind] += flops;
        es.bytes[kind] += bytes;
        if (!prof) return TN_OK;
        HIPCHK(ctx, hipEventRecord(ctx->events[ev_used + 1], stream));
        recs.push_back({kind});
        ev_used += 2;
        return TN_OK;
    };
    for (int c0 = 0; c0 < nb; c0 += chunk) {
        const int cb = std::min(chunk, nb - c0);
        es.n_chunks++;
        uint64_t* d_bits = reinterpret_cast<uint64_t*>(ws + mp.bits_off);
        double2* d_acc = reinterpret_cast<double2*>(ws + mp.acc_off);
        HIPCHK(ctx, hipMemcpyAsync(d_bits, bits + c0, sizeof(uint64_t) * cb, hipMemcpyHostToDevice, stream));
        // every kernel of the chunk: the same launches, with the same
        // arguments, for any call with this plan, workspace and shape
        auto launches = [&]() -> int {
        HIPCHK(ctx, launch_zero_acc(d_acc, cb, stream));
        // tensor layout in the workspace: [copy][bitstring][labels], one copy
        // per value of the low slice bits the tensor depends on
        auto dlow = [&](int t) -> uint32_t { return p.dep[t] & low; };
        auto ncopy = [&](int t) -> int { return 1 << __builtin_popcount(dlow(t)); };
        auto nbt = [&](int t) { return p.has_b[t] ? cb : 1; };
        auto per_r = [&](int t) -> long long { return (1ll << p.rank[t]) * nbt(t); };
        // positions of the bits of `sub` within the bits of `sup` (pext)
        auto pext_mask = [](uint32_t sub, uint32_t sup) -> unsigned {
            unsigned r = 0;
            int k = 0;
            for (uint32_t m = sup; m; m &= m - 1, ++k)
                if (sub & (m & (~m + 1))) r |= 1u << k;
            return r;
        };
        auto tensor_ptr = [&](int t) -> float2* {
            if (t < nL && p.leaves[t].identity)
                return reinterpret_cast<float2*>(plan->d_leaves) + p.leaves[t].dev_off;
            return reinterpret_cast<float2*>(ws + mp.tensor_off[t]);
        };
        for (uint64_t G = 0; G < ngroups; ++G) {
            const uint32_t changed = G == 0 ? 0xffffffffu : (uint32_t)(G ^ (G - 1));
            auto redo = [&](uint32_t dep) { return G == 0 || ((dep >> r) & changed); };
            const uint32_t slice0 = (uint32_t)(G << r);
            auto gather = [&](int t) -> int {
                if (t >= nL) return TN_OK;
                const Leaf& lf = p.leaves[t];
                if (lf.identity || !redo(lf.slice_mask)) return TN_OK;
                GatherArgs g{};
                g.src = reinterpret_cast<const float2*>(plan->d_leaves) + lf.dev_off;
                g.dst = tensor_ptr(t);
                g.bits = d_bits;
                g.slice = slice0;
                g.dmask = dlow(t);
                g.nb = lf.has_b ? cb : 1;
                g.nr = ncopy(t);
                g.n_mat = lf.n_mat;
                g.n_out = lf.n_out;
                g.n_sl = lf.n_sl;
                for (int i = 0; i < lf.n_mat; ++i) g.mat_src[i] = lf.mat_src[i];
                for (int i = 0; i < lf.n_out; ++i) { g.out_src[i] = lf.out_src[i]; g.out_qubit[i] = lf.out_qubit[i]; }
                for (int i = 0; i < lf.n_sl; ++i) { g.sl_src[i] = lf.sl_src[i]; g.sl_bit[i] = lf.sl_bit[i]; }
                int rc0 = ev_begin();
                if (rc0) return rc0;
                HIPCHK(ctx, launch_gather(g, stream));
                es.kernels_gather++;
                return ev_end(5, 0.0, 8.0 * std::ldexp(1.0, g.n_mat) * g.nb * g.nr);
            };
            if (p.steps.empty()) {
                int rc = gather(0);
                if (rc) return rc;
            }
            for (size_t si = 0; si < p.steps.size(); ++si) {
                const Step& st = p.steps[si];
                if (!redo(st.dep_mask)) {
                    es.steps_reused++;
                    continue;
                }
                int rc = gather(st.a);
                if (rc) return rc;
                rc = gather(st.b);
                if (rc) return rc;
                const float2* pa = tensor_ptr(st.a);
                const float2* pb = tensor_ptr(st.b);
                const bool redoA = redo(p.dep[st.a]);
                const bool redoB = redo(p.dep[st.b]);
                for (int w = 0; w < 2; ++w) {
                    const bool perm = w ? st.permB : st.permA;
                    if (!perm) continue;
                    const int t = w ? st.b : st.a;
                    float2* dst = reinterpret_cast<float2*>(ws + (w ? mp.permB_off[si] : mp.permA_off[si]));
                    if (w ? redoB : redoA) {
                        PermArgs a{};
                        fill_perm(a, w ? st.permB_map : st.permA_map, (int)(w ? st.orderB : st.orderA).size());
                        a.src = w ? pb : pa;
                        a.dst = dst;
                        a.nb = nbt(t) * ncopy(t);
                        rc = ev_begin();
                        if (rc) return rc;
                        HIPCHK(ctx, launch_permute(a, stream));
                        es.kernels_permute++;
                        es.permute_bytes += 16.0 * std::ldexp(1.0, a.rank) * a.nb;
                        rc = ev_end(4, 0.0, 16.0 * std::ldexp(1.0, a.rank) * a.nb);
                        if (rc) return rc;
                    }
                    if (w) pb = dst; else pa = dst;
                }
                const long long nbat = 1ll << st.batch_bits;
                const long long M = 1ll << st.m_bits, N = 1ll << st.n_bits, K = 1ll << st.k_bits;
                const uint32_t DA = dlow(st.a), DB = dlow(st.b), DC = dlow(st.c);
                GemmArgs g{};
                const int nbC = st.hbC ? cb : 1;
                float2* pc = tensor_ptr(st.c);
                // operands in kernel roles (C stored [N][M] -> C^T = B^T A^T)
                const float2 *ka = pa, *kb = pb;
                int tA = st.transA, tB = st.transB;
                bool hA = st.hbA, hB = st.hbB;
                unsigned mA = pext_mask(DA, DC), mB = pext_mask(DB, DC);
                long long km = M, kn = N, lenA = M * K, lenB = K * N;
                long long pA = per_r(st.a), pB = per_r(st.b);
                if (st.swapC) {
                    std::swap(ka, kb);
                    tA = !st.transB; tB = !st.transA;
                    std::swap(hA, hB); std::swap(mA, mB);
                    std::swap(km, kn); std::swap(lenA, lenB); std::swap(pA, pB);
                }
                g.A = ka; g.B = kb; g.C = pc;
                g.M = (int)km; g.N = (int)kn; g.K = (int)K;
                g.transA = tA; g.transB = tB;
                g.sAb = hA ? nbat * lenA : 0; g.sAi = lenA;
                g.sBb = hB ? nbat * lenB : 0; g.sBi = lenB;
                g.sCb = nbat * M * N; g.sCi = M * N;
                g.scatter = st.scatterC;
                g.cPM = st.cPM;
                g.cPN = st.cPN;
                g.nbatch = (int)nbat;
                g.nb = nbC;
                g.nr = ncopy(st.c);
                const unsigned all = (unsigned)g.nr - 1;
                g.mA = mA;
                g.mB = mB;
                g.sAr = mA ? pA : 0;
                g.sBr = mB ? pB : 0;
                g.sCr = g.nr > 1 ? per_r(st.c) : 0;
                // copies fold into the free index of the operand that has them:
                // all of them into N (1) or M (2), or, when the two operands
                // carry disjoint copy bits, A's into M and B's into N (3);
                // copy bits both operands carry stay an outer batch (0)
                g.fold = 0;
                if (g.nr > 1) {
                    if (mA == 0 && mB == all) g.fold = 1;
                    else if (mB == 0 && mA == all) g.fold = 2;
                    else if (mA && mB && (mA & mB) == 0 && (mA | mB) == all) g.fold = 3;
                }
                if (mp.scratch_off[si] != std::numeric_limits<size_t>::max())
                    g.P = reinterpret_cast<float2*>(ws + mp.scratch_off[si]);
                if (scales && mp.scale_off[si] != std::numeric_limits<size_t>::max())
                    g.X = reinterpret_cast<unsigned*>(ws + mp.scale_off[si]);
                rc = ev_begin();
                if (rc) return rc;
                HIPCHK(ctx, launch_gemm(g, precision, stream));
                es.kernels_gemm++;
                es.steps_executed++;
                const double mult = (double)nbC * g.nr;
                es.algorithmic_flops += st.flops_per_b * mult;
                rc = ev_end(gemm_kind(g, precision), st.flops_per_b * mult,
                            8.0 * ((double)nbat * (M * K * (st.hbA ? nbC : 1) * ncopy(st.a) +
                                                   K * N * (st.hbB ? nbC : 1) * ncopy(st.b) +
                                                   M * N * nbC * g.nr)));
                if (rc) return rc;
            }
            const int root = p.root;
            HIPCHK(ctx, launch_accumulate(d_acc, tensor_ptr(root), cb, p.has_b[root],
                                          ncopy(root), per_r(root), stream));
        }
        HIPCHK(ctx, launch_finalize(d_acc, cb, p.scale.real(), p.scale.imag(), stream));
        return TN_OK;
        };
        int rcc = run_chunk(ctx, plan, ws, chunk, cb, r, precision, stream, !prof, es, launches);
        if (rcc) return rcc;
        HIPCHK(ctx, hipMemcpyAsync(out + 2 * (size_t)c0, d_acc, sizeof(double2) * cb, hipMemcpyDeviceToHost, stream));
        HIPCHK(ctx, hipStreamSynchronize(stream));
        int rch = harvest();
        if (rch) return rch;
    }
    if (stats) *stats = es;
    return TN_OK;
}

}  // namespace tn

using namespace tn;

extern "C" {

const char* tn_last_error(void) { return g_err.c_str(); }

int tn_ctx_create(int device, void* arena, size_t arena_bytes, tn_ctx** out) {
    if (!out) { set_error("null out"); return TN_EINVAL; }
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        set_error("no such HIP device");
        return TN_EINVAL;
    }
    if (arena_bytes < (1u << 20)) { set_error("arena too small (< 1 MiB)"); return TN_EINVAL; }
    std::unique_ptr<tn_ctx> c(new tn_ctx());
    c->device = device;
    HIPCHK((tn_ctx*)nullptr, hipSetDevice(device));
    HIPCHK((tn_ctx*)nullptr, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    if (arena) {
        c->arena = static_cast<char*>(arena);
        c->own_arena = false;
    } else {
        void* ptr = nullptr;
        hipError_t e = hipMalloc(&ptr, arena_bytes);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(c->stream);
            set_error(std::string("arena allocation failed: ") + hipGetErrorString(e));
            return TN_EDEVICE;
        }
        c->arena = static_cast<char*>(ptr);
        c->own_arena = true;
    }
    c->arena_bytes = arena_bytes;
    c->free_list[0] = arena_bytes;
    *out = c.release();
    return TN_OK;
}

int tn_server_stop(tn_ctx* ctx);

int tn_ctx_destroy(tn_ctx* ctx) {
    if (!ctx) return TN_EINVAL;
    tn_server_stop(ctx);
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    drop_graphs(ctx, nullptr);
    (void)hipStreamDestroy(ctx->stream);
    for (auto e : ctx->events) (void)hipEventDestroy(e);
    for (tn_plan* p : ctx->plans) {      // plans still loaded
        (void)hipFree(p->d_leaves);
        delete p;
    }
    ctx->plans.clear();
    if (ctx->own_arena) (void)hipFree(ctx->arena);
    delete ctx;
    return TN_OK;
}

int tn_plan_validate(const void* blob, size_t nbytes, tn_plan_info_t* info) {
    PlanHost p;
    int rc = parse_plan(blob, nbytes, p);
    if (rc) return rc;
    if (info) {
        tn_plan tmp;
        tmp.host = std::move(p);
        return tn_plan_info(&tmp, info);
    }
    return TN_OK;
}

int tn_plan_info(const tn_plan* plan, tn_plan_info_t* out) {
    if (!plan || !out) { set_error("null argument"); return TN_EINVAL; }
    const PlanHost& p = plan->host;
    tn_plan* pl = const_cast<tn_plan*>(plan);
    out->n_qubits = p.n_qubits;
    out->n_leaves = (int)p.leaves.size();
    out->n_steps = (int)p.steps.size();
    out->n_sliced = (int)p.sliced.size();
    out->max_rank = p.max_rank;
    out->reserved = 0;
    out->flops_per_slice_per_b = p.flops_per_slice_per_b;
    out->flops_total_per_b = p.flops_total_per_b;
    size_t m1 = pl->mem(1, 0).bytes, m2 = pl->mem(2, 0).bytes;
    out->peak_bytes_per_b = m2 > m1 ? m2 - m1 : 0;
    out->peak_bytes_fixed = m1 > out->peak_bytes_per_b ? m1 - out->peak_bytes_per_b : 0;
    return TN_OK;
}

int tn_plan_load(tn_ctx* ctx, const void* blob, size_t nbytes, tn_plan** out) {
    if (!ctx || !out) { set_error("null argument"); return TN_EINVAL; }
    if (ctx->poisoned) { set_error("context poisoned by an earlier device error"); return TN_EDEVICE; }
    *out = nullptr;
    std::unique_ptr<tn_plan> pl(new tn_plan());
    int rc = parse_plan(blob, nbytes, pl->host);
    if (rc) return rc;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const size_t elems = pl->host.leaf_pool_elems;
    HIPCHK(ctx, hipMalloc(&pl->d_leaves, std::max<size_t>(elems, 1) * 8));
    std::vector<float> staging(2 * elems);
    for (auto& lf : pl->host.leaves) {
        std::copy(lf.data.begin(), lf.data.end(), staging.begin() + 2 * lf.dev_off);
    }
    HIPCHK(ctx, hipMemcpy(pl->d_leaves, staging.data(), staging.size() * sizeof(float), hipMemcpyHostToDevice));
    pl->id = ctx->next_plan_id++;
    {
        std::lock_guard<std::mutex> g(ctx->smu);
        ctx->plans.insert(pl.get());
    }
    *out = pl.release();
    return TN_OK;
}

int tn_plan_unload(tn_ctx* ctx, tn_plan* plan) {
    if (!ctx || !plan) { set_error("null argument"); return TN_EINVAL; }
    {
        std::lock_guard<std::mutex> g(ctx->smu);
        if (!ctx->plans.count(plan)) { set_error("plan is not loaded in this context"); return TN_EINVAL; }
        if (plan->pending.load() > 0) { set_error("plan has pending requests"); return TN_EBUSY; }
        ctx->plans.erase(plan);
    }
    (void)hipSetDevice(ctx->device);
    drop_graphs(ctx, plan);
    (void)hipFree(plan->d_leaves);
    delete plan;
    return TN_OK;
}

int tn_contract_amplitudes(tn_ctx* ctx, const tn_plan* plan, const uint64_t* bits, int32_t nb,
                           int32_t precision, void* hip_stream, double* out_re_im) {
    if (!ctx || !plan || !bits || !out_re_im) { set_error("null argument"); return TN_EINVAL; }
    if (nb <= 0) { set_error("nb must be positive"); return TN_EINVAL; }
    if (!precision_ok(precision)) {
        set_error("precision mode not available");
        return TN_EINVAL;
    }
    if (ctx->poisoned) { set_error("context poisoned by an earlier device error"); return TN_EDEVICE; }
    const uint64_t allowed = plan->host.out_mask;
    for (int i = 0; i < nb; ++i)
        if (bits[i] & ~allowed) { set_error("bitstring has a bit at a position >= n_qubits"); return TN_EINVAL; }
    std::lock_guard<std::mutex> g(ctx->mu);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t s = hip_stream ? static_cast<hipStream_t>(hip_stream) : ctx->stream;
    // workspace: the largest free region of the arena (all of it when the
    // serving loop is idle); wait for served batches to release memory when
    // not even one bitstring fits
    const size_t need1 = const_cast<tn_plan*>(plan)->mem(1, 0, precision == TN_SPLIT_FP16).bytes;
    if (need1 > ctx->arena_bytes) {
        set_error("one bitstring of this plan needs more workspace than the arena holds");
        return TN_ENOMEM;
    }
    size_t off = 0, bytes = 0;
    {
        std::unique_lock<std::mutex> lk(ctx->smu);
        ctx->scv.wait(lk, [&] { return largest_free(ctx) >= need1; });
        bytes = largest_free(ctx);
        arena_alloc(ctx, bytes, &off);
    }
    tn_exec_stats st{};
    int rc = execute(ctx, plan, bits, nb, precision, s, ctx->arena + off, bytes, out_re_im, &st);
    {
        std::lock_guard<std::mutex> lk(ctx->smu);
        arena_free(ctx, off, bytes);
        ctx->scv.notify_all();
    }
    ctx->last = st;
    return rc;
}

static bool pow2(long long x) { return x > 0 && (x & (x - 1)) == 0; }

// split-K partials (rounded up to 256 bytes), then the row and column
// maxima of the split fp16 products
static size_t cgemm_partial_bytes(int M, int N, int K, int nbatch, int nb) {
    return (gemm_scratch_elems(M, N, K, nbatch, nb) * 8 + 255) / 256 * 256;
}

size_t tn_kernel_cgemm_scratch_bytes(int32_t M, int32_t N, int32_t K, int32_t nbatch, int32_t nb) {
    if (!pow2(M) || !pow2(N) || !pow2(K) || nbatch <= 0 || nb <= 0) return 0;
    return cgemm_partial_bytes(M, N, K, nbatch, nb) + gemm_scale_words(M, N, K, nbatch, nb) * 4;
}

int tn_kernel_cgemm_shape(int32_t M, int32_t N, int32_t K, int32_t nbatch, int32_t* kind,
                          int32_t* splits) {
    if (!kind || !splits || !pow2(M) || !pow2(N) || !pow2(K) || nbatch <= 0) {
        set_error("bad gemm shape (M, N, K must be powers of two)");
        return TN_EINVAL;
    }
    const GemmChoice c = choose_gemm(M, N, K, nbatch);
    *kind = c.kind;
    *splits = c.splits;
    return TN_OK;
}

int tn_kernel_cgemm(const void* A, const void* B, void* C, int32_t M, int32_t N, int32_t K,
                    int32_t transA, int32_t transB, int32_t nbatch, int32_t nb,
                    int64_t sAb, int64_t sBb, int64_t sCb, int64_t sAi, int64_t sBi,
                    int64_t sCi, int32_t precision, void* scratch, size_t scratch_bytes,
                    void* hip_stream) {
    if (!A || !B || !C || !pow2(M) || !pow2(N) || !pow2(K) || nbatch <= 0 || nb <= 0) {
        set_error("bad gemm arguments (M, N, K must be powers of two)");
        return TN_EINVAL;
    }
    if (!precision_ok(precision)) { set_error("precision mode not available"); return TN_EINVAL; }
    const size_t part = gemm_scratch_elems(M, N, K, nbatch, nb) ? cgemm_partial_bytes(M, N, K, nbatch, nb) : 0;
    const size_t words = precision == TN_SPLIT_FP16 ? gemm_scale_words(M, N, K, nbatch, nb) : 0;
    const size_t need = part + words * 4;
    if (need > scratch_bytes || (need && !scratch)) {
        set_error("gemm needs " + std::to_string(need) + " bytes of scratch");
        return TN_EINVAL;
    }
    GemmArgs g{};
    g.A = static_cast<const float2*>(A);
    g.B = static_cast<const float2*>(B);
    g.C = static_cast<float2*>(C);
    g.M = M; g.N = N; g.K = K;
    g.transA = transA ? 1 : 0; g.transB = transB ? 1 : 0;
    g.nbatch = nbatch; g.nb = nb;
    g.sAb = sAb; g.sBb = sBb; g.sCb = sCb; g.sAi = sAi; g.sBi = sBi; g.sCi = sCi;
    g.P = static_cast<float2*>(scratch);
    if (words) g.X = reinterpret_cast<unsigned*>(static_cast<char*>(scratch) + part);
    tn_ctx* none = nullptr;
    HIPCHK(none, launch_gemm(g, precision, static_cast<hipStream_t>(hip_stream)));
    return TN_OK;
}

// Scratch of tn_kernel_cgemm_noalloc: one array per GPU, reserved when the
// library's code object is loaded on that GPU and held until the process
// ends.  Host code never uses the symbol itself (its host-side name is not a
// device address): the address comes from hipGetSymbolAddress, looked up once
// per device with that device current.
static constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char noalloc_scratch[kNoAllocScratchBytes];
static constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_noalloc_mu;
static void* g_noalloc_ptr[kNoAllocMaxDevices] = {};

static int noalloc_scratch_ptr(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        set_error(std::string("HIP error: ") + hipGetErrorString(e) + " at hipGetDevice");
        return TN_EDEVICE;
    }
    if (dev < 0 || dev >= kNoAllocMaxDevices) { set_error("device index out of range"); return TN_EINVAL; }
    std::lock_guard<std::mutex> g(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("HIP error: ") + hipGetErrorString(e) + " at hipGetSymbolAddress");
            return TN_EDEVICE;
        }
        g_noalloc_ptr[dev] = p;
    }
    *out = g_noalloc_ptr[dev];
    return TN_OK;
}

size_t tn_kernel_cgemm_noalloc_max_scratch(void) { return kNoAllocScratchBytes; }

int tn_kernel_cgemm_noalloc(const void* A, const void* B, void* C, int32_t M, int32_t N, int32_t K,
                            int32_t transA, int32_t transB, int32_t nbatch, int32_t nb,
                            int64_t sAb, int64_t sBb, int64_t sCb, int64_t sAi, int64_t sBi,
                            int64_t sCi, int32_t precision, void* hip_stream) {
    if (!A || !B || !C || !pow2(M) || !pow2(N) || !pow2(K) || nbatch <= 0 || nb <= 0) {
        set_error("bad gemm arguments (M, N, K must be powers of two)");
        return TN_EINVAL;
    }
    if (!precision_ok(precision)) { set_error("precision mode not available"); return TN_EINVAL; }
    const size_t part = gemm_scratch_elems(M, N, K, nbatch, nb) ? cgemm_partial_bytes(M, N, K, nbatch, nb) : 0;
    const size_t words = precision == TN_SPLIT_FP16 ? gemm_scale_words(M, N, K, nbatch, nb) : 0;
    const size_t need = part + words * 4;
    if (need > kNoAllocScratchBytes) {
        set_error("gemm needs " + std::to_string(need) + " bytes of scratch, more than the " +
                  std::to_string(kNoAllocScratchBytes) + " of the library's array");
        return TN_EINVAL;
    }
    void* ptr = nullptr;
    const int rc = noalloc_scratch_ptr(&ptr);
    if (rc) return rc;
    return tn_kernel_cgemm(A, B, C, M, N, K, transA, transB, nbatch, nb, sAb, sBb, sCb, sAi, sBi,
                           sCi, precision, ptr, kNoAllocScratchBytes, hip_stream);
}

int tn_kernel_permute(const void* src, void* dst, int32_t rank, const int32_t* perm, int32_t nb,
                      void* hip_stream) {
    if (!src || !dst || !perm || rank < 0 || rank > 40 || nb <= 0) { set_error("bad permute arguments"); return TN_EINVAL; }
    int map[kMaxRank];
    std::vector<char> seen(rank, 0);
    for (int p = 0; p < rank; ++p) {
        if (perm[p] < 0 || perm[p] >= rank || seen[perm[p]]) { set_error("perm is not a permutation"); return TN_EINVAL; }
        seen[perm[p]] = 1;
        map[p] = perm[p];
    }
    PermArgs a{};
    fill_perm(a, map, rank);
    a.src = static_cast<const float2*>(src);
    a.dst = static_cast<float2*>(dst);
    a.nb = nb;
    tn_ctx* none = nullptr;
    HIPCHK(none, launch_permute(a, static_cast<hipStream_t>(hip_stream)));
    return TN_OK;
}

int tn_ctx_set_profiling(tn_ctx* ctx, int32_t on) {
    if (!ctx) return TN_EINVAL;
    ctx->profile = on != 0;
    return TN_OK;
}

int tn_ctx_set_graphs(tn_ctx* ctx, int32_t on) {
    if (!ctx) { set_error("null argument"); return TN_EINVAL; }
    ctx->use_graphs = on != 0;
    return TN_OK;
}

int tn_ctx_set_slice_block(tn_ctx* ctx, int32_t log2_block) {
    if (!ctx || log2_block < -1 || log2_block > 30) { set_error("bad slice block"); return TN_EINVAL; }
    ctx->force_slice_block = log2_block;
    return TN_OK;
}

int tn_last_exec_stats(tn_ctx* ctx, tn_exec_stats* out) {
    if (!ctx || !out) return TN_EINVAL;
    *out = ctx->last;
    return TN_OK;
}

}  // extern "C"
