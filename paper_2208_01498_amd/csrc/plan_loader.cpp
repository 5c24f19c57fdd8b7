// TNP1 parser, validator and descriptor derivation (host only).
//
// A plan is a list of leaves (dense complex128 tensors over binary labels)
// and pairwise steps.  For each step the labels of A, B and C fall into
// batch (A, B, C), K (A, B: summed), MA (A, C) and NB (B, C); the step's cost
// is the product of the dimensions of the union of A's and B's labels, the
// quantity of Eq. (3).  The loader checks that every step's stored orders
// form a strided-batched complex GEMM and derives its shapes.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>
#include <set>

#include "kernels.h"
#include "tn_internal.h"

namespace tn {

namespace {

struct Reader {
    const uint8_t* p;
    size_t n, off = 0;
    bool ok = true;
    Reader(const void* b, size_t nn) : p(static_cast<const uint8_t*>(b)), n(nn) {}
    bool need(size_t k) {
        if (!ok || off + k > n || off + k < off) { ok = false; return false; }
        return true;
    }
    uint32_t u32() {
        if (!need(4)) return 0;
        uint32_t v;
        std::memcpy(&v, p + off, 4);
        off += 4;
        return v;
    }
    int32_t i32() { return static_cast<int32_t>(u32()); }
    double f64() {
        if (!need(8)) return 0;
        double v;
        std::memcpy(&v, p + off, 8);
        off += 8;
        return v;
    }
    uint8_t u8() {
        if (!need(1)) return 0;
        return p[off++];
    }
};

int fail(const std::string& m) {
    set_error("invalid plan: " + m);
    return TN_EINVAL;
}

// bit position (from the least significant) of each label in an order
void positions(const std::vector<int>& order, std::map<int, int>& pos) {
    pos.clear();
    int r = static_cast<int>(order.size());
    for (int i = 0; i < r; ++i) pos[order[i]] = r - 1 - i;
}

std::vector<int> sub(const std::vector<int>& order, const std::set<int>& s) {
    std::vector<int> o;
    for (int l : order)
        if (s.count(l)) o.push_back(l);
    return o;
}

bool slice_eq(const std::vector<int>& v, size_t at, const std::vector<int>& w) {
    if (at + w.size() > v.size()) return false;
    for (size_t i = 0; i < w.size(); ++i)
        if (v[at + i] != w[i]) return false;
    return true;
}

}  // namespace

int parse_plan(const void* blob, size_t nbytes, PlanHost& p) {
    if (!blob) return fail("null blob");
    Reader r(blob, nbytes);
    if (!r.need(4) || std::memcmp(r.p, "TNP1", 4) != 0) return fail("bad magic");
    r.off = 4;
    uint32_t version = r.u32();
    if (version != 1) return fail("unsupported version");
    uint32_t n_qubits = r.u32(), n_labels = r.u32(), n_leaves = r.u32(), n_steps = r.u32(),
             n_sliced = r.u32();
    const uint32_t flags = r.u32();  // bit 0: U and its conjugate (projector mode)
    if (flags & ~1u) return fail("unknown flags");
    const bool doubled = (flags & 1u) != 0;
    double sre = r.f64(), sim = r.f64();
    if (!r.ok) return fail("truncated header");
    if (n_qubits == 0 || n_qubits > (uint32_t)kMaxQubits) return fail("qubit count out of range");
    if (n_labels > (1u << 20) || n_leaves == 0 || n_leaves > (1u << 22) ||
        n_steps != n_leaves - 1 || n_sliced > 30)
        return fail("bad counts");
    p = PlanHost();
    p.n_qubits = (int)n_qubits;
    p.scale = {sre, sim};
    p.labels.resize(n_labels);
    std::vector<int> outs_of_qubit(n_qubits, 0);
    for (uint32_t i = 0; i < n_labels; ++i) {
        LabelInfo& L = p.labels[i];
        L.dim = r.u8();
        L.kind = r.u8();
        r.u8();
        r.u8();
        L.qubit = r.i32();
        if (!r.ok) return fail("truncated labels");
        if (L.dim != 2) return fail("only binary labels are supported");
        if (L.kind > 1) return fail("bad label kind");
        if (L.kind == 1) {
            if (L.qubit < 0 || L.qubit >= (int)n_qubits) return fail("output label qubit out of range");
            // one output label per qubit; two (U and its conjugate) in
            // projector mode
            if (++outs_of_qubit[L.qubit] > (doubled ? 2 : 1))
                return fail(doubled ? "more than two output labels on one qubit"
                                    : "two output labels on one qubit");
            p.out_mask |= (1ull << L.qubit);
        }
    }
    // leaves
    p.leaves.resize(n_leaves);
    size_t pool = 0;
    for (uint32_t i = 0; i < n_leaves; ++i) {
        Leaf& lf = p.leaves[i];
        uint32_t rk = r.u32();
        if (!r.ok || rk > (uint32_t)kMaxLeafRank) return fail("leaf rank");
        lf.rank = (int)rk;
        lf.labels.resize(rk);
        for (auto& l : lf.labels) {
            l = (int)r.u32();
            if (l < 0 || l >= (int)n_labels) return fail("leaf label out of range");
        }
        uint32_t nm = r.u32();
        if (!r.ok || nm > rk) return fail("leaf gathered rank");
        lf.mat.resize(nm);
        for (auto& l : lf.mat) l = (int)r.u32();
        uint32_t ng = r.u32();
        if (!r.ok || ng > (1u << 20)) return fail("leaf gate count");
        lf.gates.resize(ng);
        for (auto& g : lf.gates) g = (int)r.u32();
        size_t ne = size_t(1) << rk;
        if (!r.need(ne * 16)) return fail("truncated leaf data");
        lf.data.resize(2 * ne);
        for (size_t e = 0; e < 2 * ne; ++e) {
            double v;
            std::memcpy(&v, r.p + r.off + 8 * e, 8);
            lf.data[e] = static_cast<float>(v);   // round to nearest even
        }
        r.off += ne * 16;
        std::set<int> ls(lf.labels.begin(), lf.labels.end());
        if (ls.size() != lf.labels.size()) return fail("repeated label on a leaf");
        lf.dev_off = pool;
        pool += ne;
    }
    p.leaf_pool_elems = pool;
    p.sliced.resize(n_sliced);
    std::set<int> sliced_set;
    for (uint32_t j = 0; j < n_sliced; ++j) {
        int l = (int)r.u32();
        if (!r.ok || l < 0 || l >= (int)n_labels) return fail("sliced label out of range");
        if (p.labels[l].kind != 0) return fail("output label cannot be sliced");
        if (!sliced_set.insert(l).second) return fail("label sliced twice");
        p.sliced[j] = l;
    }
    std::map<int, int> slice_bit;
    for (uint32_t j = 0; j < n_sliced; ++j) slice_bit[p.sliced[j]] = (int)j;

    const int T = (int)(n_leaves + n_steps);
    p.rank.assign(T, 0);
    p.has_b.assign(T, 0);
    p.dep.assign(T, 0);
    p.consumer.assign(T, -1);
    std::vector<std::vector<int>> order(T);
    std::vector<int> label_uses(n_labels, 0);

    // gather descriptors
    for (uint32_t i = 0; i < n_leaves; ++i) {
        Leaf& lf = p.leaves[i];
        std::map<int, int> spos;
        positions(lf.labels, spos);
        std::set<int> expect;
        for (int l : lf.labels) {
            if (p.labels[l].kind == 1) {
                lf.has_b = true;
                lf.out_src[lf.n_out] = spos[l];
                lf.out_qubit[lf.n_out] = p.labels[l].qubit;
                lf.n_out++;
            } else if (sliced_set.count(l)) {
                lf.slice_mask |= 1u << slice_bit[l];
                lf.sl_src[lf.n_sl] = spos[l];
                lf.sl_bit[lf.n_sl] = slice_bit[l];
                lf.n_sl++;
            } else {
                expect.insert(l);
            }
        }
        std::set<int> got(lf.mat.begin(), lf.mat.end());
        if (got != expect || got.size() != lf.mat.size())
            return fail("leaf gathered order must list exactly its non-output, non-sliced labels");
        lf.n_mat = (int)lf.mat.size();
        for (int j = 0; j < lf.n_mat; ++j) lf.mat_src[lf.n_mat - 1 - j] = spos[lf.mat[j]];
        lf.identity = !lf.has_b && lf.slice_mask == 0 && lf.mat == lf.labels;
        order[i] = lf.mat;
        p.rank[i] = lf.n_mat;
        p.has_b[i] = lf.has_b;
        p.dep[i] = lf.slice_mask;
        for (int l : lf.mat) label_uses[l]++;
    }

    // steps
    p.steps.resize(n_steps);
    std::vector<char> used(T, 0);
    double fps = 0.0, ftot = 0.0;
    for (uint32_t s = 0; s < n_steps; ++s) {
        Step& st = p.steps[s];
        st.a = (int)r.u32();
        st.b = (int)r.u32();
        st.c = (int)(n_leaves + s);
        if (!r.ok) return fail("truncated steps");
        if (st.a < 0 || st.b < 0 || st.a >= st.c || st.b >= st.c || st.a == st.b)
            return fail("step operand out of range");
        if (used[st.a] || used[st.b]) return fail("tensor consumed twice");
        used[st.a] = used[st.b] = 1;
        p.consumer[st.a] = p.consumer[st.b] = (int)s;
        std::vector<int> pa, pb, oc;
        for (int which = 0; which < 2; ++which) {
            uint32_t k = r.u32();
            if (!r.ok || k > (uint32_t)kMaxRank) return fail("permutation rank");
            std::vector<int>& v = which ? pb : pa;
            v.resize(k);
            for (auto& l : v) l = (int)r.u32();
        }
        uint32_t kc = r.u32();
        if (!r.ok || kc > (uint32_t)kMaxRank) return fail("output rank");
        oc.resize(kc);
        for (auto& l : oc) l = (int)r.u32();
        if (!r.ok) return fail("truncated step");
        const std::vector<int>& sa = order[st.a];
        const std::vector<int>& sb = order[st.b];
        std::set<int> SA(sa.begin(), sa.end()), SB(sb.begin(), sb.end()), SC(oc.begin(), oc.end());
        if (SC.size() != oc.size()) return fail("repeated label in output order");
        st.permA = !pa.empty();
        st.permB = !pb.empty();
        if (st.permA && std::set<int>(pa.begin(), pa.end()) != SA) return fail("permA is not a permutation of A");
        if (st.permB && std::set<int>(pb.begin(), pb.end()) != SB) return fail("permB is not a permutation of B");
        if (st.permA && pa.size() != sa.size()) return fail("permA size");
        if (st.permB && pb.size() != sb.size()) return fail("permB size");
        st.srcA = sa;
        st.srcB = sb;
        st.orderA = st.permA ? pa : sa;
        st.orderB = st.permB ? pb : sb;
        st.orderC = oc;
        std::set<int> batch, K, MA, NB, U;
        for (int l : SA) {
            U.insert(l);
            if (SB.count(l)) (SC.count(l) ? batch : K).insert(l);
            else MA.insert(l);
        }
        for (int l : SB) {
            U.insert(l);
            if (!SA.count(l)) NB.insert(l);
        }
        for (int l : MA)
            if (!SC.count(l)) return fail("label of one operand only must survive (no single-operand sums)");
        for (int l : NB)
            if (!SC.count(l)) return fail("label of one operand only must survive (no single-operand sums)");
        for (int l : SC)
            if (!U.count(l)) return fail("output label not in operands");
        const size_t nb = batch.size();
        std::vector<int> bo(oc.begin(), oc.begin() + std::min(nb, oc.size()));
        if (std::set<int>(bo.begin(), bo.end()) != batch) return fail("C must start with the batch labels");
        std::vector<int> kA = sub(st.orderA, K);
        std::vector<int> maA = sub(st.orderA, MA);
        std::vector<int> nbB = sub(st.orderB, NB);
        // A
        if (!slice_eq(st.orderA, 0, bo)) return fail("A batch order differs from C");
        if (slice_eq(st.orderA, nb, maA) && slice_eq(st.orderA, nb + maA.size(), kA)) st.transA = false;
        else if (slice_eq(st.orderA, nb, kA) && slice_eq(st.orderA, nb + kA.size(), maA)) st.transA = true;
        else return fail("A is not [batch][M][K] or [batch][K][M]");
        // B
        if (!slice_eq(st.orderB, 0, bo)) return fail("B batch order differs from C");
        if (sub(st.orderB, K) != kA) return fail("K order differs between A and B");
        if (slice_eq(st.orderB, nb, kA) && slice_eq(st.orderB, nb + kA.size(), nbB)) st.transB = false;
        else if (slice_eq(st.orderB, nb, nbB) && slice_eq(st.orderB, nb + nbB.size(), kA)) st.transB = true;
        else return fail("B is not [batch][K][N] or [batch][N][K]");
        // C: [batch][M][N], [batch][N][M], or after the batch labels any
        // interleaving of the M labels (in A's order) with the N labels (in
        // B's order), written through bit-deposit masks
        st.scatterC = false;
        st.cPM = st.cPN = 0;
        if (slice_eq(oc, nb, maA) && slice_eq(oc, nb + maA.size(), nbB)) st.swapC = false;
        else if (slice_eq(oc, nb, nbB) && slice_eq(oc, nb + nbB.size(), maA)) st.swapC = true;
        else {
            std::vector<int> rest(oc.begin() + nb, oc.end());
            if (sub(rest, MA) != maA || sub(rest, NB) != nbB)
                return fail("C is not [batch] followed by M labels in A's order interleaved "
                            "with N labels in B's order");
            st.swapC = false;
            st.scatterC = true;
            const int rc = (int)rest.size();
            for (int i = 0; i < rc; ++i) {
                const uint64_t bit = uint64_t(1) << (rc - 1 - i);
                if (MA.count(rest[i])) st.cPM |= bit;
                else st.cPN |= bit;
            }
        }
        st.batch_bits = (int)nb;
        st.m_bits = (int)MA.size();
        st.n_bits = (int)NB.size();
        st.k_bits = (int)K.size();
        if ((int)oc.size() > kMaxRank) return fail("output rank too large");
        // permutation maps
        auto mkmap = [](const std::vector<int>& src, const std::vector<int>& dst, int* map) {
            std::map<int, int> ps, pd;
            positions(src, ps);
            positions(dst, pd);
            for (auto& kv : pd) map[kv.second] = ps[kv.first];
        };
        if (st.permA) mkmap(sa, pa, st.permA_map);
        if (st.permB) mkmap(sb, pb, st.permB_map);
        st.hbA = p.has_b[st.a];
        st.hbB = p.has_b[st.b];
        st.hbC = st.hbA || st.hbB;
        st.dep_mask = p.dep[st.a] | p.dep[st.b];
        st.flops_per_b = 8.0 * std::ldexp(1.0, (int)U.size());
        order[st.c] = oc;
        p.rank[st.c] = (int)oc.size();
        p.has_b[st.c] = st.hbC;
        p.dep[st.c] = st.dep_mask;
        p.max_rank = std::max(p.max_rank, (int)oc.size());
        fps += st.flops_per_b;
        // every slice value a step depends on, once (all slices in one pass)
        ftot += st.flops_per_b * std::ldexp(1.0, __builtin_popcount(st.dep_mask));
    }
    uint32_t nmeta = r.u32();
    if (!r.ok || nmeta > 64) return fail("meta");
    p.meta.resize(nmeta);
    for (auto& v : p.meta) v = r.f64();
    if (!r.ok) return fail("truncated meta");
    if (r.off != nbytes) return fail("trailing bytes");
    p.root = T - 1;
    if (n_steps == 0) p.root = 0;
    if (p.rank[p.root] != 0) return fail("the last step must leave no labels");
    for (int t = 0; t < T - 1; ++t)
        if (!used[t]) return fail("tensor never consumed");
    // amplitudes project every qubit; in projector mode a traced qubit has
    // no output label (its bitstring bit must be 0)
    if (!doubled && p.out_mask != ((n_qubits == 64) ? ~0ull : ((1ull << n_qubits) - 1)))
        return fail("every qubit needs an output label");
    p.flops_per_slice_per_b = fps;
    p.flops_total_per_b = ftot;
    for (int l : p.sliced) {
        bool found = false;
        for (auto& lf : p.leaves)
            for (int x : lf.labels)
                if (x == l) found = true;
        if (!found) return fail("sliced label on no leaf");
    }
    return TN_OK;
}

// ---------------------------------------------------------------------------
// Workspace assignment for a chunk of `chunk` bitstrings.
//
// Slice s recomputes a tensor whose subtree holds sliced bits D only when a
// bit of D changed since slice s-1 (the lowest changed bit of s is ctz(s));
// a tensor read by a step that recomputes more often than the tensor itself
// (or one that no slice changes) therefore persists over the whole slice
// loop; all others live from their producing step to their consuming step.
// Buffers are placed first-fit by decreasing size, never overlapping a
// buffer whose lifetime overlaps.
MemPlan plan_memory(const PlanHost& p, int chunk, int r, bool scales) {
    MemPlan mp;
    mp.chunk = chunk;
    mp.r = r;
    mp.scales = scales;
    const uint32_t low = (1u << r) - 1;
    const int nL = (int)p.leaves.size();
    const int T = (int)p.rank.size();
    const int S = (int)p.sliced.size();
    const size_t kNone = std::numeric_limits<size_t>::max();
    mp.tensor_off.assign(T, kNone);
    mp.permA_off.assign(p.steps.size(), kNone);
    mp.permB_off.assign(p.steps.size(), kNone);
    mp.scratch_off.assign(p.steps.size(), kNone);
    mp.scale_off.assign(p.steps.size(), kNone);
    struct Buf { size_t bytes; int start, end; size_t* off; };
    std::vector<Buf> bufs;
    // a tensor whose subtree holds low slice bits exists once per slice of the
    // block; recomputation follows the high bits, pass by pass
    auto elems = [&](int rk, bool hb, uint32_t dep) {
        return (size_t(1) << rk) * (hb ? (size_t)chunk : 1) * (size_t(1) << __builtin_popcount(dep & low));
    };
    auto period = [&](uint32_t m) { m >>= r; return m ? __builtin_ctz(m) : S + 1; };
    const int INF = std::numeric_limits<int>::max();
    // accumulators + bitstrings + root
    size_t fixed = 0;
    mp.acc_off = fixed;
    fixed += ((size_t)chunk * 16 + 255) / 256 * 256;
    mp.bits_off = fixed;
    fixed += ((size_t)chunk * 8 + 255) / 256 * 256;
    for (int t = 0; t < T; ++t) {
        int start, end;
        if (t < nL) {
            if (p.leaves[t].identity) continue;   // read from the resident pool
            start = -1;
            end = INF;                             // gathered leaves persist
        } else {
            int s = t - nL;
            int q = p.consumer[t];
            start = s;
            if (q < 0) end = INF;
            else if (period(p.steps[q].dep_mask) < period(p.dep[t])) start = -1, end = INF;
            else end = q;
        }
        bufs.push_back({elems(p.rank[t], p.has_b[t], p.dep[t]) * 8, start, end, &mp.tensor_off[t]});
    }
    // a permuted operand is re-permuted only when the operand itself changed,
    // so its copy lives like the operand
    auto operand_life = [&](int t, int s, int& start, int& end) {
        const int q = s;
        if (t < nL || period(p.steps[q].dep_mask) < period(p.dep[t])) { start = -1; end = INF; }
        else { start = s; end = s; }
    };
    for (size_t s = 0; s < p.steps.size(); ++s) {
        const Step& st = p.steps[s];
        int a0, a1;
        if (st.permA) {
            operand_life(st.a, (int)s, a0, a1);
            bufs.push_back({elems((int)st.orderA.size(), st.hbA, p.dep[st.a]) * 8, a0, a1, &mp.permA_off[s]});
        }
        if (st.permB) {
            operand_life(st.b, (int)s, a0, a1);
            bufs.push_back({elems((int)st.orderB.size(), st.hbB, p.dep[st.b]) * 8, a0, a1, &mp.permB_off[s]});
        }
        const int M = 1 << st.m_bits, N = 1 << st.n_bits, K = 1 << st.k_bits;
        const int Mk = st.swapC ? N : M, Nk = st.swapC ? M : N;
        const int nouter = (st.hbC ? chunk : 1) * (1 << __builtin_popcount(st.dep_mask & low));
        size_t se = gemm_scratch_elems(Mk, Nk, K, 1 << st.batch_bits, nouter);
        if (se) bufs.push_back({se * 8, (int)s, (int)s, &mp.scratch_off[s]});
        if (scales) {
            size_t sw = gemm_scale_words(Mk, Nk, K, 1 << st.batch_bits, nouter);
            if (sw) bufs.push_back({sw * 4, (int)s, (int)s, &mp.scale_off[s]});
        }
    }
    for (auto& b : bufs) b.bytes = (b.bytes + 255) / 256 * 256;
    std::vector<int> idx(bufs.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return bufs[x].bytes > bufs[y].bytes; });
    struct Placed { size_t off, bytes; int start, end; };
    std::vector<Placed> placed;
    size_t top = fixed;
    for (int i : idx) {
        Buf& b = bufs[i];
        std::vector<std::pair<size_t, size_t>> busy;
        for (auto& q : placed)
            if (!(q.end < b.start || b.end < q.start)) busy.push_back({q.off, q.off + q.bytes});
        std::sort(busy.begin(), busy.end());
        size_t cand = fixed;
        for (auto& iv : busy) {
            if (cand + b.bytes <= iv.first) break;
            cand = std::max(cand, iv.second);
        }
        *b.off = cand;
        placed.push_back({cand, b.bytes, b.start, b.end});
        top = std::max(top, cand + b.bytes);
    }
    mp.bytes = top;
    return mp;
}

}  // namespace tn

const tn::MemPlan& tn_plan::mem(int chunk, int r, bool scales) {
    std::lock_guard<std::mutex> g(mcache);
    const long long key = ((long long)chunk * 64 + r) * 2 + (scales ? 1 : 0);
    auto it = memcache.find(key);
    if (it != memcache.end()) return it->second;
    auto& v = memcache[key] = tn::plan_memory(host, chunk, r, scales);
    return v;
}
