// Internal structures of the amplitude engine (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <complex>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/tnamp.h"

namespace tn {

constexpr int kMaxRank = 48;        // labels per tensor (dims are 2)
constexpr int kMaxLeafRank = 24;    // labels per stored leaf
constexpr int kMaxQubits = 64;

void set_error(const std::string& msg);

struct LabelInfo {
    uint8_t dim = 2;
    uint8_t kind = 0;   // 0 wire, 1 output
    int32_t qubit = -1;
};

// A leaf as stored in the plan and the gather that turns it into the
// operand of its step: out[b][j] = src[addr(j, x^(b), slice bits)].
struct Leaf {
    int rank = 0;
    std::vector<int> labels;        // storage order (C order)
    std::vector<int> mat;           // gathered order
    std::vector<int> gates;
    std::vector<float> data;        // complex64, interleaved, storage order
    bool has_b = false;
    uint32_t slice_mask = 0;
    bool identity = false;          // gathered == stored, no b, no slice
    // gather descriptor (bit positions counted from the least significant)
    int n_mat = 0;
    int mat_src[kMaxLeafRank];      // for gathered bit p (LSB = 0): source bit
    int n_out = 0;
    int out_src[kMaxLeafRank];
    int out_qubit[kMaxLeafRank];
    int n_sl = 0;
    int sl_src[kMaxLeafRank];
    int sl_bit[kMaxLeafRank];
    size_t dev_off = 0;             // element offset of the stored data in the leaf pool
};

struct Step {
    int a = -1, b = -1, c = -1;     // tensor ids
    bool permA = false, permB = false;
    std::vector<int> orderA, orderB, orderC;   // after permutation
    std::vector<int> srcA, srcB;               // stored orders (when permuted)
    bool hbA = false, hbB = false, hbC = false;
    int batch_bits = 0, m_bits = 0, n_bits = 0, k_bits = 0;
    bool transA = false, transB = false, swapC = false;
    // C written with its row bits deposited at cPM and column bits at cPN
    // (element index within one batch entry)
    bool scatterC = false;
    uint64_t cPM = 0, cPN = 0;
    uint32_t dep_mask = 0;
    double flops_per_b = 0;         // 8 * 2^(union bits) (times 1 per bitstring)
    // bit permutation maps: dst bit p takes src bit perm[p]
    int permA_map[kMaxRank];
    int permB_map[kMaxRank];
};

struct PlanHost {
    int n_qubits = 0;
    std::complex<double> scale{1.0, 0.0};
    std::vector<LabelInfo> labels;
    std::vector<Leaf> leaves;
    std::vector<Step> steps;
    std::vector<int> sliced;        // label ids, bit j = sliced[j]
    std::vector<double> meta;
    // per tensor (leaves then step results)
    std::vector<int> rank;          // gathered rank for leaves
    std::vector<char> has_b;
    std::vector<uint32_t> dep;      // slice-bit dependency mask
    std::vector<int> consumer;      // step index consuming the tensor (-1 for root)
    int root = -1;
    int max_rank = 0;
    uint64_t out_mask = 0;          // qubits with an output label
    double flops_per_slice_per_b = 0;
    double flops_total_per_b = 0;
    size_t leaf_pool_elems = 0;
};

int parse_plan(const void* blob, size_t n, PlanHost& p);   // TN_OK / TN_EINVAL

// Buffer assignment for one chunk size.
struct MemPlan {
    int chunk = 0;
    int r = 0;                                  // log2 slices per pass
    size_t bytes = 0;                           // total workspace bytes
    std::vector<size_t> tensor_off;             // per tensor id (bytes), SIZE_MAX if none
    std::vector<size_t> permA_off, permB_off;   // per step, SIZE_MAX if none
    std::vector<size_t> scratch_off;            // per step split-K partials, SIZE_MAX if none
    std::vector<size_t> scale_off;              // per step row/column maxima (split fp16 only)
    bool scales = false;                        // laid out for the split fp16 products
    size_t acc_off = 0;                         // FP64 accumulators
    size_t bits_off = 0;                        // bitstrings
    size_t maps_off = 0;                        // per-step tables (none yet)
};
MemPlan plan_memory(const PlanHost& p, int chunk, int r, bool scales = false);

struct DevicePlan;

}  // namespace tn

struct tn_plan {
    tn::PlanHost host;
    float* d_leaves = nullptr;          // complex64 pool (stored order)
    std::atomic<int> pending{0};
    int id = 0;
    std::mutex mcache;
    std::map<long long, tn::MemPlan> memcache;
    // workspace layout for `chunk` bitstrings and 2^r slices per pass
    // (`scales`: with the per-step words of the split fp16 products)
    const tn::MemPlan& mem(int chunk, int r, bool scales = false);
};

namespace tn {

struct Request {
    uint64_t ticket = 0;
    const tn_plan* plan = nullptr;
    std::vector<uint64_t> bits;
    int precision = 0;
    std::vector<double> result;
    int status = TN_PENDING;
    bool cancelled = false;
    tn_req_stats st{};
};

// An execution slot of the serving loop: a stream, a worker thread and the
// arena region of the batch it runs.
struct Slot {
    hipStream_t stream = nullptr;
    std::thread th;
    bool busy = false;
    bool has_job = false;
    std::vector<std::shared_ptr<Request>> job;
    const tn_plan* plan = nullptr;
    int precision = 0;
    size_t off = 0, bytes = 0;
    int shape_r = 0, shape_chunk = 0;
    bool heavy = false;
    std::condition_variable cv;
};

}  // namespace tn

struct tn_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    bool own_arena = false;
    std::atomic<bool> poisoned{false};
    std::mutex mu;                      // serialises blocking calls on the ctx stream
    tn_exec_stats last{};
    int next_plan_id = 1;
    // serving
    std::mutex smu;
    std::condition_variable scv;
    std::deque<std::shared_ptr<tn::Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<tn::Request>> reqs;
    uint64_t next_ticket = 1;
    std::thread sched;
    bool sched_started = false;
    bool stop = false;
    int n_slots = 4;
    int max_batch = 64;
    double heavy_flops = 1e14;           // algorithmic flops of a heavy batch
    int max_heavy = 1;                   // heavy batches running at once
    std::vector<std::unique_ptr<tn::Slot>> slots;
    // arena sub-allocation for served batches: (offset, size) free list
    std::map<size_t, size_t> free_list;
    // per-launch event timing (blocking calls only)
    bool profile = false;
    std::vector<hipEvent_t> events;
    std::set<tn_plan*> plans;            // loaded and not yet unloaded (guarded by smu)
    int force_slice_block = -1;          // log2 slices per pass, -1 = automatic
    // captured chunks: (plan, workspace, chunk, slice-block bits, precision)
    // -> graph and the launch statistics it stands for (guarded by gmu)
    bool use_graphs = true;
    std::mutex gmu;
    struct GraphEntry {
        hipGraphExec_t exec = nullptr;   // null: seen once, not captured yet
        tn_exec_stats delta{};
        uint64_t stamp = 0;
    };
    std::map<std::tuple<const tn_plan*, const char*, int, int, int, int>, GraphEntry> graphs;
    uint64_t graph_clock = 0;
};

namespace tn {
// executor: run a batch of bitstrings through the plan on a stream, using
// workspace [ws, ws + ws_bytes).  Blocking iff sync.
int execute(tn_ctx* ctx, const tn_plan* plan, const uint64_t* bits, int nb,
            int precision, hipStream_t stream, char* ws, size_t ws_bytes,
            double* out, tn_exec_stats* stats, int shape_r = 0, int shape_chunk = 0);
// destroy the captured graphs of a plan (of every plan when plan is null)
void drop_graphs(tn_ctx* ctx, const tn_plan* plan);
// execution shape (log2 slices per pass, bitstrings per pass) for a workspace
bool choose_shape(const tn_plan* plan, int nb, size_t ws_bytes, int force_r, int& r, int& chunk,
                  bool scales = false);
// precision modes the executor runs
inline bool precision_ok(int p) {
    return p == TN_FP32_4M || p == TN_FP32_3M || p == TN_SPLIT_BF16 || p == TN_SPLIT_FP16 ||
           p == TN_BF16_1TERM;
}
int64_t now_ns();
// arena sub-allocation (callers hold ctx->smu)
bool arena_alloc(tn_ctx* ctx, size_t bytes, size_t* off);
void arena_free(tn_ctx* ctx, size_t off, size_t bytes);
size_t largest_free(tn_ctx* ctx);
}  // namespace tn
