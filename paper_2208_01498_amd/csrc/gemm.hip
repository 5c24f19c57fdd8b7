// Complex GEMM kernels of the pairwise steps (gfx950).
//
// C[m][n] = sum_k A(m,k) B(k,n) for every (bitstring b, batch-label value),
// complex64 in HBM, FP32 accumulation.  Four families, chosen from the shape
// only (never from the batch size, so a result is bitwise the same in any
// chunk):
//   k_cgemm<0,...>  FP32 4M on v_mfma_f32_32x32x2_f32: interleaved complex A
//                   gives the real operand rows (Ar, Ai) directly and B is
//                   expanded on the fly to [[Br Bi] [-Bi Br]], so one MFMA is
//                   a 32 (m) x 16 (complex n) x 1 (complex k) product
//   k_cgemm<2,...>  split bf16 on v_mfma_f32_32x32x16_bf16: operands are
//                   split x = hi + lo when staged into LDS, and
//                   hi*hi + hi*lo + lo*hi are accumulated in FP32; one MFMA is
//                   32 x 16 x 8 (complex)
//   k_cgemm<3,...>  split fp16 on v_mfma_f32_32x32x16_f16: every row of A
//                   and column of B is first scaled by a power of two that
//                   puts its largest |re|, |im| in [2^14, 2^15) (k_opmax
//                   finds the maxima), then split into fp16 hi + lo as
//                   above; the epilogue undoes both scales exactly
//   k_cgemm<4,...>  the same with hi*hi only (plain bf16 rounding of the
//                   operands), kept as the lower-accuracy reference point
//   k_cgemm3m       FP32 3M on the same MFMA used as a real 32 x 32 x 2
//                   product: three real products per complex product
//                   (6 MNK executed flops instead of 8 MNK)
//   k_cgemm_wave    small products (at most 64 x 64 outputs per batch
//                   entry, K <= 256, FP32 modes): one wave per 32 x 32
//                   block, operands straight from global memory
//   k_cgemm_dot     tiny M*N with long K: a K-parallel dot product (every
//                   precision mode)
//   split-K         when a shape has too few output tiles to fill the chip,
//                   K is cut into a fixed number of ranges whose partial
//                   products are summed in range order by k_reduce_splitk
// Tiles: WGM x WGN waves per workgroup (4 or 8); a wave owns WMF x WNF
// blocks of 32 x 16 (4M, split) or 32 x 32 (3M) complex outputs; 8 complex k
// per stage (16 for 3M); the global loads of the next stage are issued back
// to back before the MFMAs of the current one and land in the other half of
// a double-buffered LDS, one barrier per stage.  Workgroups are renumbered
// so that each XCD takes one contiguous range of tiles, walked in groups of
// TILE_GROUP tile rows (xcd_logical, tile_rc).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>
#include <mutex>

#include "kernels.h"

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int KT_SPLIT = 8;    // complex k per LDS stage, split modes (one MFMA k-step; keeps
                               // two workgroups per CU)
constexpr int KT_FP32 = 8;     // complex k per LDS stage, FP32 (keeps two workgroups per CU)
constexpr int KT_3M = 16;      // complex k per LDS stage, FP32 3M (two real planes per operand)
constexpr int KT = 16;         // K granularity of the split-K ranges

constexpr int TILE_GROUP = 4;  // tile rows per group in the tile order (tile_rc)

// Logical index of workgroup b of n: workgroups go to the eight XCDs in
// turn (b mod 8), each XCD with an L2 of its own; renumbered so that each
// XCD takes one contiguous range of logical indices
__device__ __forceinline__ size_t xcd_logical(size_t b, size_t n) {
    const size_t x = b & 7, i = b >> 3, q = n >> 3, r = n & 7;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Tile (tm, tn) of logical tile t: groups of TILE_GROUP tile rows, walked
// column by column, so that the workgroups resident on one XCD at a time
// cover a block of rows and columns and share their A and B panels in L2
__device__ __forceinline__ void tile_rc(size_t t, int tiles_m, int tiles_n, int& tm, int& tn) {
    const size_t per = (size_t)TILE_GROUP * tiles_n;
    const int first = (int)(t / per) * TILE_GROUP;
    const int gs = min(TILE_GROUP, tiles_m - first);
    const int w = (int)(t % per);
    tm = first + w % gs;
    tn = w / gs;
}

// bits of x at the set positions of m, compacted (parallel bit extract)
__device__ __forceinline__ size_t pext_u(size_t x, unsigned m) {
    size_t r = 0;
    int k = 0;
    for (; m; m &= m - 1, ++k)
        if (x & (m & (~m + 1))) r |= size_t(1) << k;
    return r;
}

// Operand copy read by the GEMM block of outer bitstring bb, inner batch ib
// and slice-block copy rr, numbered over the copies that exist: bitstrings
// only when the operand has them (stride != 0), slice-block copies only when
// they form an outer batch (fold 0).  Indexes the row (column) maxima of the
// split fp16 products, so each copy's maxima are found once.
__device__ __forceinline__ size_t operand_copy(const GemmArgs& g, int op, size_t bb, size_t ib, size_t rr) {
    const long long sb = op ? g.sBb : g.sAb;
    const unsigned m = op ? g.mB : g.mA;
    const size_t nc = g.fold == 0 ? (size_t(1) << __builtin_popcount(m)) : 1;
    const size_t c = g.fold == 0 ? pext_u(rr, m) : 0;
    return ((sb ? bb : 0) * g.nbatch + ib) * nc + c;
}

// Row deposits for a 32-row MFMA output block under a scattered C: row
// 8*(r/4) + 4*half + r%4 of the block sets row bits 0,1 from r, bit 2 from
// half and bits 3,4 from r/4; with M >= 32 the block's base row has those
// five bits clear, so the deposit of the whole row is the base's deposit OR
// the deposit of the low five bits (the five lowest set bits of cPM).
struct RowDep {
    unsigned long long d[5];
    __device__ void init(unsigned long long pm) {
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            d[i] = pm & (~pm + 1);
            pm &= pm - 1;
        }
    }
    __device__ unsigned long long low(int r, int half) const {
        return ((r & 1) ? d[0] : 0ull) | ((r & 2) ? d[1] : 0ull) | (half ? d[2] : 0ull) |
               ((r & 4) ? d[3] : 0ull) | ((r & 8) ? d[4] : 0ull);
    }
};

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
    hi = __float2bfloat16(x);
    lo = __float2bfloat16(x - __bfloat162float(hi));
}

// fp16 halves of a value already scaled into the fp16 range: x - hi is
// exact in FP32, and both conversions round to nearest even
__device__ __forceinline__ void split_f16(float x, _Float16& hi, _Float16& lo) {
    hi = (_Float16)x;
    lo = (_Float16)(x - (float)hi);
}

// Power-of-two scale 2^t for a row whose largest |re|, |im| has the float
// bit pattern `mx` (2^e <= max < 2^(e+1)): t = 14 - e puts the scaled
// maximum in [2^14, 2^15), below the fp16 limit of 65504; t is clamped so
// that 2^t and 2^-t are normal floats; an all-zero row keeps scale 1
__device__ __forceinline__ int scale_exp(unsigned mx) {
    if (mx == 0) return 0;
    const int e = (int)((mx >> 23) & 255u) - 127;
    return min(126, max(-126, 14 - e));
}
__device__ __forceinline__ float exp2i(int t) { return __uint_as_float((unsigned)(127 + t) << 23); }

template <int PREC, int WGM, int WGN, int WMF, int WNF>
struct Smem {
    static constexpr int KT = PREC == 0 ? KT_FP32 : KT_SPLIT;
    static constexpr int BM = WGM * 32 * WMF;
    static constexpr int BN = WGN * 16 * WNF;
    // FP32: A as [k][m] complex; B as [k][n] with each complex stored as the
    // four reals (Br, Bi, -Bi, Br) of its 2 x 2 real block, so every lane
    // reads its MFMA operand with one 4-byte load and no select
    static constexpr int PA = BM + 2;
    static constexpr int PB = BN + 1;            // in 16-byte units
    // 16-bit halves: rows of KT words (one 4-byte word per complex k, its
    // two 16-bit reals) at a stride of RW = KT + 4 words, so that a lane
    // reads its 8 reals of an MFMA step as one 16-byte word.  A row m sits
    // at row (m mod 2) GA + m / 2 and real column r of B at (r mod 4) GB +
    // r / 4, so the rows one store instruction writes (every second A row
    // when m is the contiguous index, every fourth B column) are
    // consecutive.  Row x starts at bank 12 x mod 64, distinct for x mod 16;
    // with GA = 8 and GB = 4 (mod 16) the 16 rows that 16 consecutive lanes
    // read (8 in each of two A groups, 4 in each of four B groups) cover
    // the 64 banks once, so a 16-byte read has no bank conflict
    static constexpr int RW = KT + 4;
    static constexpr int GA = (BM / 2 + 15) / 16 * 16 + 8;
    static constexpr int GB = (BN / 2 + 15) / 16 * 16 + 4;
    static constexpr int RAh = GA + BM / 2;            // rows per A plane
    static constexpr int RBh = 3 * GB + BN / 2;        // rows per B plane
    static constexpr size_t bytes_fp32 = 2 * (size_t)KT * (PA * 8 + PB * 16);
    static constexpr size_t bytes_bf16 = 2 * (size_t)(RAh + RBh) * RW * 4 * 2;
    static constexpr size_t bytes = PREC == 0 ? bytes_fp32 : bytes_bf16;
};

}  // namespace

template <int PREC, int WGM, int WGN, int WMF, int WNF, bool TA, bool TB>
__global__ void __launch_bounds__(64 * WGM * WGN) __attribute__((amdgpu_waves_per_eu(4)))
k_cgemm(GemmArgs g) {
    using S = Smem<PREC, WGM, WGN, WMF, WNF>;
    constexpr int KT = S::KT;
    constexpr int NT = 64 * WGM * WGN;
    constexpr int BM = S::BM, BN = S::BN, PA = S::PA, PB = S::PB, RW = S::RW;
    constexpr int GA = S::GA, GB = S::GB, RAh = S::RAh, RBh = S::RBh;
    constexpr int FA = BM * KT / 2;      // float4 (2 complex) loads per A tile
    constexpr int FB = KT * BN / 2;
    constexpr int LA = (FA + NT - 1) / NT;
    constexpr int LB = (FB + NT - 1) / NT;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

    // slice-block folding: the folded index m' = a * M + m selects operand
    // and output copy a (likewise n')
    const int Mt = gemm_rows(g);
    const int Nt = gemm_cols(g);
    const int lgM = __builtin_ctz((unsigned)g.M), lgN = __builtin_ctz((unsigned)g.N);
    const int tiles_m = (Mt + BM - 1) / BM;
    const int tiles_n = (Nt + BN - 1) / BN;
    const size_t tiles = (size_t)tiles_m * tiles_n;
    size_t blk = xcd_logical(blockIdx.x, gridDim.x);
    const size_t tile = blk % tiles;
    blk /= tiles;
    const int split = (int)(blk % g.splits);
    blk /= g.splits;
    const size_t ib = blk % g.nbatch;
    blk /= g.nbatch;
    const size_t bb = blk % g.nb;
    const size_t rr = g.fold == 0 ? blk / g.nb : 0;
    const size_t outer = g.fold == 0 ? rr * g.nb + bb : bb;
    const size_t n_outer = g.fold == 0 ? (size_t)g.nr * g.nb : (size_t)g.nb;
    int tm, tn;
    tile_rc(tile, tiles_m, tiles_n, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int kper = g.K / g.splits;
    const int kb = split * kper, ke = kb + kper;
    const float2* A = g.A + bb * g.sAb + ib * g.sAi + pext_u(rr, g.mA) * g.sAr;
    const float2* B = g.B + bb * g.sBb + ib * g.sBi + pext_u(rr, g.mB) * g.sBr;
    const long long sAf = (g.fold == 2 || g.fold == 3) ? g.sAr : 0;    // per folded block
    const long long sBf = (g.fold == 1 || g.fold == 3) ? g.sBr : 0;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = (wave % WGM) * (32 * WMF);
    const int wn = (wave / WGM) * (16 * WNF);
    const int half = lane >> 5;
    const int l32 = lane & 31;

    floatx16 acc[WMF][WNF];
#pragma unroll
    for (int i = 0; i < WMF; ++i)
#pragma unroll
        for (int j = 0; j < WNF; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    float4 ra[LA], rb[LB];
    // split fp16: scales of the rows (A) and columns (B) this thread stages;
    // element 0 of a staged pair at index 0, element 1 at index 1
    float sca[LA][2], scb[LB][2];
    if constexpr (PREC == 3) {
        const unsigned* xa = g.xA + operand_copy(g, 0, bb, ib, rr) * Mt;
        const unsigned* xb = g.xB + operand_copy(g, 1, bb, ib, rr) * Nt;
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            const int f = tid + i * NT;
            const int m = !TA ? f / (KT / 2) : 2 * (f % (BM / 2));
            const int m2 = !TA ? m : m + 1;
            sca[i][0] = (f < FA && m0 + m < Mt) ? exp2i(scale_exp(xa[m0 + m])) : 1.f;
            sca[i][1] = (f < FA && m0 + m2 < Mt) ? exp2i(scale_exp(xa[m0 + m2])) : 1.f;
        }
#pragma unroll
        for (int i = 0; i < LB; ++i) {
            const int f = tid + i * NT;
            const int n = !TB ? 2 * (f % (BN / 2)) : f / (KT / 2);
            const int n2 = !TB ? n + 1 : n;
            scb[i][0] = (f < FB && n0 + n < Nt) ? exp2i(scale_exp(xb[n0 + n])) : 1.f;
            scb[i][1] = (f < FB && n0 + n2 < Nt) ? exp2i(scale_exp(xb[n0 + n2])) : 1.f;
        }
    }
    // address of A(m', k) / B(k, n') for folded indices
    auto adA = [&](int mp, int k) -> size_t {
        const int m = mp & (g.M - 1);
        return (size_t)(mp >> lgM) * sAf + (TA ? (size_t)k * g.M + m : (size_t)m * g.K + k);
    };
    auto adB = [&](int k, int np) -> size_t {
        const int n = np & (g.N - 1);
        return (size_t)(np >> lgN) * sBf + (TB ? (size_t)n * g.K + k : (size_t)k * g.N + n);
    };
    auto ldA = [&](int m, int k) -> float2 {
        if (m0 + m >= Mt || k >= ke) return make_float2(0.f, 0.f);
        return A[adA(m0 + m, k)];
    };
    auto ldB = [&](int k, int n) -> float2 {
        if (n0 + n >= Nt || k >= ke) return make_float2(0.f, 0.f);
        return B[adB(k, n0 + n)];
    };
    // full: a stage known to be whole and inside the matrix (no bounds test
    // is compiled in); otherwise decided here
    auto load = [&](auto full, int k0) {
        constexpr bool FULL = decltype(full)::value;
        // vector loads need the element pair inside one folded block
        const bool fullA = FULL || ((m0 + BM <= Mt) && (k0 + KT <= ke) && (!TA || g.M >= 2));
        const bool fullB = FULL || ((n0 + BN <= Nt) && (k0 + KT <= ke) && (TB || g.N >= 2));
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            const int f = tid + i * NT;
            if (FA % NT != 0 && f >= FA) break;
            if (!TA) {
                const int m = f / (KT / 2), k = 2 * (f % (KT / 2));
                if (fullA) ra[i] = *reinterpret_cast<const float4*>(A + adA(m0 + m, k0 + k));
                else {
                    float2 x = ldA(m, k0 + k), y = ldA(m, k0 + k + 1);
                    ra[i] = make_float4(x.x, x.y, y.x, y.y);
                }
            } else {
                const int k = f / (BM / 2), m = 2 * (f % (BM / 2));
                if (fullA) ra[i] = *reinterpret_cast<const float4*>(A + adA(m0 + m, k0 + k));
                else {
                    float2 x = ldA(m, k0 + k), y = ldA(m + 1, k0 + k);
                    ra[i] = make_float4(x.x, x.y, y.x, y.y);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < LB; ++i) {
            const int f = tid + i * NT;
            if (FB % NT != 0 && f >= FB) break;
            if (!TB) {
                const int k = f / (BN / 2), n = 2 * (f % (BN / 2));
                if (fullB) rb[i] = *reinterpret_cast<const float4*>(B + adB(k0 + k, n0 + n));
                else {
                    float2 x = ldB(k0 + k, n), y = ldB(k0 + k, n + 1);
                    rb[i] = make_float4(x.x, x.y, y.x, y.y);
                }
            } else {
                const int n = f / (KT / 2), k = 2 * (f % (KT / 2));
                if (fullB) rb[i] = *reinterpret_cast<const float4*>(B + adB(k0 + k, n0 + n));
                else {
                    float2 x = ldB(k0 + k, n), y = ldB(k0 + k + 1, n);
                    rb[i] = make_float4(x.x, x.y, y.x, y.y);
                }
            }
        }
    };

    // ---------------------------------------------------------------- FP32
    float2* As = reinterpret_cast<float2*>(smem);              // [2][KT][PA]
    float4* Bs = reinterpret_cast<float4*>(As + 2 * KT * PA);  // [2][KT][PB]
    // ---------------------------------------------------------------- bf16
    uint32_t* Ah = reinterpret_cast<uint32_t*>(smem);           // [2][RAh][RW] words
    uint32_t* Al = Ah + 2 * RAh * RW;
    uint32_t* Bh = Al + 2 * RAh * RW;                            // [2][RBh][RW]
    uint32_t* Bl = Bh + 2 * RBh * RW;
    // word w (complex k) of A row m / B real column r
    auto wa = [](int m, int w) { return ((m & 1) * GA + (m >> 1)) * RW + w; };
    auto wb = [](int r, int w) { return ((r & 3) * GB + (r >> 2)) * RW + w; };

    // two floats (one complex, both times the scale sc of its row or
    // column in fp16 mode) -> packed 16-bit pairs (hi, lo), x = hi + lo; the
    // 16-bit planes hold bf16 or fp16 bit patterns
    auto split2 = [](float a, float b, float sc, uint32_t& hi, uint32_t& lo) {
        uint16_t h0, l0, h1, l1;
        if constexpr (PREC == 3) {
            _Float16 ha, la, hb, lb;
            split_f16(a * sc, ha, la);
            split_f16(b * sc, hb, lb);
            h0 = __builtin_bit_cast(uint16_t, ha); l0 = __builtin_bit_cast(uint16_t, la);
            h1 = __builtin_bit_cast(uint16_t, hb); l1 = __builtin_bit_cast(uint16_t, lb);
        } else {
            (void)sc;
            __bf16 ha, la, hb, lb;
            split_bf16(a, ha, la);
            split_bf16(b, hb, lb);
            h0 = __builtin_bit_cast(uint16_t, ha); l0 = __builtin_bit_cast(uint16_t, la);
            h1 = __builtin_bit_cast(uint16_t, hb); l1 = __builtin_bit_cast(uint16_t, lb);
        }
        hi = (uint32_t)h0 | ((uint32_t)h1 << 16);
        lo = (uint32_t)l0 | ((uint32_t)l1 << 16);
    };

    auto store = [&](int buf) {
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            const int f = tid + i * NT;
            if (FA % NT != 0 && f >= FA) break;
            int m, k, m2, k2;   // element 0 at (m,k), element 1 at (m2,k2)
            if (!TA) { m = f / (KT / 2); k = 2 * (f % (KT / 2)); m2 = m; k2 = k + 1; }
            else { k = f / (BM / 2); m = 2 * (f % (BM / 2)); m2 = m + 1; k2 = k; }
            if constexpr (PREC == 0) {
                float2* a = As + buf * KT * PA;
                if (TA) *reinterpret_cast<float4*>(a + k * PA + m) = ra[i];
                else {
                    a[k * PA + m] = make_float2(ra[i].x, ra[i].y);
                    a[k2 * PA + m2] = make_float2(ra[i].z, ra[i].w);
                }
            } else {
                uint32_t* ah = Ah + buf * RAh * RW;
                uint32_t* al = Al + buf * RAh * RW;
                uint32_t h0, l0, h1, l1;
                split2(ra[i].x, ra[i].y, sca[i][0], h0, l0);
                split2(ra[i].z, ra[i].w, sca[i][1], h1, l1);
                // real index 2k + (re, im) of row m: one 4-byte word per complex
                ah[wa(m, k)] = h0; al[wa(m, k)] = l0;
                ah[wa(m2, k2)] = h1; al[wa(m2, k2)] = l1;
            }
        }
#pragma unroll
        for (int i = 0; i < LB; ++i) {
            const int f = tid + i * NT;
            if (FB % NT != 0 && f >= FB) break;
            int k, n, k2, n2;
            if (!TB) { k = f / (BN / 2); n = 2 * (f % (BN / 2)); k2 = k; n2 = n + 1; }
            else { n = f / (KT / 2); k = 2 * (f % (KT / 2)); n2 = n; k2 = k + 1; }
            if constexpr (PREC == 0) {
                float4* b = Bs + buf * KT * PB;
                b[k * PB + n] = make_float4(rb[i].x, rb[i].y, -rb[i].y, rb[i].x);
                b[k2 * PB + n2] = make_float4(rb[i].z, rb[i].w, -rb[i].w, rb[i].z);
            } else {
                uint32_t* bh = Bh + buf * RBh * RW;
                uint32_t* bl = Bl + buf * RBh * RW;
                // real column 2n: rows (2k, 2k+1) = (Br, -Bi); column 2n+1:
                // (Bi, Br).  Each real is split once; the negated halves of
                // -Bi are the halves of Bi with the sign bit flipped (exact)
                uint32_t h0, l0, h1, l1;
                split2(rb[i].x, rb[i].y, scb[i][0], h0, l0);   // (Br, Bi) of element 0
                split2(rb[i].z, rb[i].w, scb[i][1], h1, l1);   // element 1
                auto neg_hi = [](uint32_t v) {           // (r, i) -> (r, -i)
                    return v ^ 0x80000000u;
                };
                auto swap = [](uint32_t v) {             // (r, i) -> (i, r)
                    return (v >> 16) | (v << 16);
                };
                bh[wb(2 * n, k)] = neg_hi(h0); bl[wb(2 * n, k)] = neg_hi(l0);
                bh[wb(2 * n + 1, k)] = swap(h0); bl[wb(2 * n + 1, k)] = swap(l0);
                bh[wb(2 * n2, k2)] = neg_hi(h1); bl[wb(2 * n2, k2)] = neg_hi(l1);
                bh[wb(2 * n2 + 1, k2)] = swap(h1); bl[wb(2 * n2 + 1, k2)] = swap(l1);
            }
        }
    };

    auto compute = [&](int buf) {
        if constexpr (PREC == 0) {
            // lane (half, l32): A real row l32 col half = (re, im)[half] of
            // A[m][k]; B real row half, col l32 = entry 2*half + (l32 & 1) of
            // the expanded 2 x 2 block of B[k][n = l32/2]
            const float* a = reinterpret_cast<const float*>(As + buf * KT * PA);
            const float* b = reinterpret_cast<const float*>(Bs + buf * KT * PB);
            const int boff = 4 * (l32 >> 1) + 2 * half + (l32 & 1);
            // operands of step kk + 1 are read into the other register set
            // while the MFMAs of step kk issue
            float av[2][WMF], bv[2][WNF];
            auto rd = [&](int kk, int q) {
#pragma unroll
                for (int i = 0; i < WMF; ++i) av[q][i] = a[2 * (kk * PA + wm + i * 32 + l32) + half];
#pragma unroll
                for (int j = 0; j < WNF; ++j) bv[q][j] = b[4 * (kk * PB + wn + j * 16) + boff];
            };
            rd(0, 0);
#pragma unroll
            for (int kk = 0; kk < KT; ++kk) {
                if (kk + 1 < KT) rd(kk + 1, (kk + 1) & 1);
                __builtin_amdgcn_sched_barrier(0);    // keep the reads ahead of the MFMAs
#pragma unroll
                for (int i = 0; i < WMF; ++i)
#pragma unroll
                    for (int j = 0; j < WNF; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[kk & 1][i], bv[kk & 1][j], acc[i][j], 0, 0, 0);
            }
        } else {
            const uint32_t* ah = Ah + buf * RAh * RW;
            const uint32_t* al = Al + buf * RAh * RW;
            const uint32_t* bh = Bh + buf * RBh * RW;
            const uint32_t* bl = Bl + buf * RBh * RW;
            // the 8 reals k = 8 half .. 8 half + 7 of a 16-k MFMA step are the
            // four words 4 half .. 4 half + 3 of the row: one 16-byte read
            auto rd8 = [&](const uint32_t* row) {
                return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(row));
            };
#pragma unroll
            for (int kc = 0; kc < KT / 8; ++kc) {
                // A halves of the step first, then B column block by block:
                // block j + 1 is read while the MFMAs of block j issue (two
                // B blocks live instead of WNF keeps the kernel within 128
                // VGPRs)
                bf16x8 xh[WMF], xl[WMF], yh[2], yl[2];
#pragma unroll
                for (int i = 0; i < WMF; ++i) {
                    const int o = wa(wm + i * 32 + l32, 8 * kc + 4 * half);
                    xh[i] = rd8(ah + o);
                    xl[i] = rd8(al + o);
                }
                auto rdb = [&](int j, int q) {
                    const int o = wb(2 * (wn + j * 16) + l32, 8 * kc + 4 * half);
                    yh[q] = rd8(bh + o);
                    yl[q] = rd8(bl + o);
                };
                rdb(0, 0);
#pragma unroll
                for (int j = 0; j < WNF; ++j) {
                    if (j + 1 < WNF) rdb(j + 1, (j + 1) & 1);
                    __builtin_amdgcn_sched_barrier(0);
                    const int q = j & 1;
#pragma unroll
                    for (int i = 0; i < WMF; ++i) {
                        if constexpr (PREC == 3) {
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                                __builtin_bit_cast(halfx8, xl[i]), __builtin_bit_cast(halfx8, yh[q]), acc[i][j], 0, 0, 0);
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                                __builtin_bit_cast(halfx8, xh[i]), __builtin_bit_cast(halfx8, yl[q]), acc[i][j], 0, 0, 0);
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                                __builtin_bit_cast(halfx8, xh[i]), __builtin_bit_cast(halfx8, yh[q]), acc[i][j], 0, 0, 0);
                        } else {
                            if constexpr (PREC == 2) {
                                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl[i], yh[q], acc[i][j], 0, 0, 0);
                                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[i], yl[q], acc[i][j], 0, 0, 0);
                            }
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[i], yh[q], acc[i][j], 0, 0, 0);
                        }
                    }
                }
            }
        }
    };

    // Stages 0 .. nfull-1 of a tile inside the matrix are whole: their loads
    // are compiled with no bounds test.  Every pass ends with the store of
    // the stage it loaded.  Both keep the three or four global loads of a
    // stage issuing back to back: where a bounds-tested load and its
    // unchecked form write the same registers on merging paths, or a load
    // may still be outstanding where the loop begins again, the compiler
    // waits for each load before issuing the next.
    const bool inner = (m0 + BM <= Mt) && (n0 + BN <= Nt) && (!TA || g.M >= 2) && (TB || g.N >= 2);
    const int nk = (kper + KT - 1) / KT;
    const int nfull = inner ? kper / KT : 0;
    load(std::false_type{}, kb);
    store(0);
    __syncthreads();
    int t = 0;
    for (; t + 1 < nfull; ++t) {
        load(std::true_type{}, kb + (t + 1) * KT);
        __builtin_amdgcn_sched_barrier(0);     // the stage's loads issue before its MFMAs
        compute(t & 1);
        store((t & 1) ^ 1);
        __syncthreads();
    }
    for (; t + 1 < nk; ++t) {
        load(std::false_type{}, kb + (t + 1) * KT);
        compute(t & 1);
        store((t & 1) ^ 1);
        __syncthreads();
    }
    if (nk > 0) compute((nk - 1) & 1);

    // epilogue: acc[i][j][r] is real row 8*(r/4) + 4*half + r%4, column l32
    const bool part = g.splits > 1;
    float2* Cb = part ? g.P + (((size_t)split * n_outer + outer) * g.nbatch + ib) * (size_t)Mt * Nt
                      : g.C + bb * g.sCb + ib * g.sCi + rr * g.sCr;
    const bool fastdep = g.scatter && !part && g.M >= 32;
    RowDep rd;
    if (fastdep) rd.init(g.cPM);
#pragma unroll
    for (int i = 0; i < WMF; ++i) {
        // split fp16: the inverse scales of this lane's 16 rows, shared by
        // all column blocks
        float urow[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            urow[r] = 1.f;
            if constexpr (PREC == 3) {
                const int mp = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                if (mp < Mt) urow[r] = exp2i(-scale_exp(g.xA[operand_copy(g, 0, bb, ib, rr) * Mt + mp]));
            }
        }
#pragma unroll
        for (int j = 0; j < WNF; ++j) {
            const int np = n0 + wn + j * 16 + (l32 >> 1);
            if (np >= Nt) continue;
            const int n = np & (g.N - 1);
            unsigned long long dbase = 0;
            if (fastdep)
                dbase = pdep64((unsigned)((m0 + wm + i * 32) & (g.M - 1)), g.cPM) | pdep64((unsigned)n, g.cPN);
            // split fp16: undo the column scale, then the row scale (exact
            // multiplications by powers of two)
            float ucol = 1.f;
            if constexpr (PREC == 3)
                ucol = exp2i(-scale_exp(g.xB[operand_copy(g, 1, bb, ib, rr) * Nt + np]));
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int mp = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                if (mp >= Mt) continue;
                size_t e;
                if (part) e = (size_t)mp * Nt + np;
                else {
                    const int m = mp & (g.M - 1);
                    e = (size_t)gemm_c_copy(g, (unsigned)(mp >> lgM), (unsigned)(np >> lgN)) +
                        (fastdep ? (size_t)(dbase | rd.low(r, half)) : gemm_c_elem(g, m, n));
                }
                float v = acc[i][j][r];
                if constexpr (PREC == 3) v = (v * ucol) * urow[r];
                reinterpret_cast<float*>(Cb + e)[l32 & 1] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// FP32 3M: three real products per complex product,
//   P1 = Ar Br,  P2 = Ai Bi,  P3 = (Ar + Ai)(Br + Bi),
//   Re C = P1 - P2,  Im C = P3 - P1 - P2,
// each a real 32 x 32 x 2 MFMA (6 MNK executed flops against 8 MNK for 4M).
// Operands are staged in LDS as complex rows ([k][m] and [k][n], real and
// imaginary parts interleaved, as they are in memory), the sum operand formed
// at read time; a wave owns WMF x WNF blocks of 32 x 32 (complex) outputs
// with three accumulators each.  Same
// decomposition (slice-block fold, outer copies, split-K ranges) and the
// same K order as k_cgemm, so a result does not depend on the tile chosen.
template <int WGM, int WGN, int WMF, int WNF>
struct Smem3 {
    // 16 complex k per stage, double buffered
    static constexpr int KT = KT_3M;
    static constexpr int BM = WGM * 32 * WMF;
    static constexpr int BN = WGN * 32 * WNF;
    // row pitch in floats, 2 BM + 4: the eight even rows that one 64-bit
    // store instruction writes when k is the contiguous global index start
    // in eight different groups of 8 banks, so its 32-lane halves hit 64
    // distinct banks; a row is 16-byte aligned for the 128-bit stores
    static constexpr int PA = 2 * BM + 4;
    static constexpr int PB = 2 * BN + 4;
    static constexpr size_t bytes = 2 * (size_t)KT * (PA + PB) * 4;
};

template <int WGM, int WGN, int WMF, int WNF, bool TA, bool TB>
__global__ void __launch_bounds__(64 * WGM * WGN) __attribute__((amdgpu_waves_per_eu(2)))
k_cgemm3m(GemmArgs g) {
    using S = Smem3<WGM, WGN, WMF, WNF>;
    constexpr int KT = S::KT;
    constexpr int NT = 64 * WGM * WGN;
    constexpr int BM = S::BM, BN = S::BN, PA = S::PA, PB = S::PB;
    constexpr int FA = BM * KT / 2;
    constexpr int FB = KT * BN / 2;
    constexpr int LA = (FA + NT - 1) / NT;
    constexpr int LB = (FB + NT - 1) / NT;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];

    const int Mt = gemm_rows(g);
    const int Nt = gemm_cols(g);
    const int lgM = __builtin_ctz((unsigned)g.M), lgN = __builtin_ctz((unsigned)g.N);
    const int tiles_m = (Mt + BM - 1) / BM;
    const int tiles_n = (Nt + BN - 1) / BN;
    const size_t tiles = (size_t)tiles_m * tiles_n;
    size_t blk = xcd_logical(blockIdx.x, gridDim.x);
    const size_t tile = blk % tiles;
    blk /= tiles;
    const int split = (int)(blk % g.splits);
    blk /= g.splits;
    const size_t ib = blk % g.nbatch;
    blk /= g.nbatch;
    const size_t bb = blk % g.nb;
    const size_t rr = g.fold == 0 ? blk / g.nb : 0;
    const size_t outer = g.fold == 0 ? rr * g.nb + bb : bb;
    const size_t n_outer = g.fold == 0 ? (size_t)g.nr * g.nb : (size_t)g.nb;
    int tm, tn;
    tile_rc(tile, tiles_m, tiles_n, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int kper = g.K / g.splits;
    const int kb = split * kper, ke = kb + kper;
    const float2* A = g.A + bb * g.sAb + ib * g.sAi + pext_u(rr, g.mA) * g.sAr;
    const float2* B = g.B + bb * g.sBb + ib * g.sBi + pext_u(rr, g.mB) * g.sBr;
    const long long sAf = (g.fold == 2 || g.fold == 3) ? g.sAr : 0;
    const long long sBf = (g.fold == 1 || g.fold == 3) ? g.sBr : 0;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = (wave % WGM) * (32 * WMF);
    const int wn = (wave / WGM) * (32 * WNF);
    const int half = lane >> 5;
    const int l32 = lane & 31;

    floatx16 acc[WMF][WNF][3];
#pragma unroll
    for (int i = 0; i < WMF; ++i)
#pragma unroll
        for (int j = 0; j < WNF; ++j)
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[i][j][p][r] = 0.f;

    float4 ra[LA], rb[LB];
    auto adA = [&](int mp, int k) -> size_t {
        const int m = mp & (g.M - 1);
        return (size_t)(mp >> lgM) * sAf + (TA ? (size_t)k * g.M + m : (size_t)m * g.K + k);
    };
    auto adB = [&](int k, int np) -> size_t {
        const int n = np & (g.N - 1);
        return (size_t)(np >> lgN) * sBf + (TB ? (size_t)n * g.K + k : (size_t)k * g.N + n);
    };
    auto ldA = [&](int m, int k) -> float2 {
        if (m0 + m >= Mt || k >= ke) return make_float2(0.f, 0.f);
        return A[adA(m0 + m, k)];
    };
    auto ldB = [&](int k, int n) -> float2 {
        if (n0 + n >= Nt || k >= ke) return make_float2(0.f, 0.f);
        return B[adB(k, n0 + n)];
    };
    auto load = [&](auto full, int k0) {
        constexpr bool FULL = decltype(full)::value;
        const bool fullA = FULL || ((m0 + BM <= Mt) && (k0 + KT <= ke) && (!TA || g.M >= 2));
        const bool fullB = FULL || ((n0 + BN <= Nt) && (k0 + KT <= ke) && (TB || g.N >= 2));
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            const int f = tid + i * NT;
            if (FA % NT != 0 && f >= FA) break;
            if (!TA) {
                const int m = f / (KT / 2), k = 2 * (f % (KT / 2));
                if (fullA) ra[i] = *reinterpret_cast<const float4*>(A + adA(m0 + m, k0 + k));
                else {
                    float2 x = ldA(m, k0 + k), y = ldA(m, k0 + k + 1);
                    ra[i] = make_float4(x.x, x.y, y.x, y.y);
                }
            } else {
                const int k = f / (BM / 2), m = 2 * (f % (BM / 2));
                if (fullA) ra[i] = *reinterpret_cast<const float4*>(A + adA(m0 + m, k0 + k));
                else {
                    float2 x = ldA(m, k0 + k), y = ldA(m + 1, k0 + k);
                    ra[i] = make_float4(x.x, x.y, y.x, y.y);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < LB; ++i) {
            const int f = tid + i * NT;
            if (FB % NT != 0 && f >= FB) break;
            if (!TB) {
                const int k = f / (BN / 2), n = 2 * (f % (BN / 2));
                if (fullB) rb[i] = *reinterpret_cast<const float4*>(B + adB(k0 + k, n0 + n));
                else {
                    float2 x = ldB(k0 + k, n), y = ldB(k0 + k, n + 1);
                    rb[i] = make_float4(x.x, x.y, y.x, y.y);
                }
            } else {
                const int n = f / (KT / 2), k = 2 * (f % (KT / 2));
                if (fullB) rb[i] = *reinterpret_cast<const float4*>(B + adB(k0 + k, n0 + n));
                else {
                    float2 x = ldB(k0 + k, n), y = ldB(k0 + k + 1, n);
                    rb[i] = make_float4(x.x, x.y, y.x, y.y);
                }
            }
        }
    };

    float* As = reinterpret_cast<float*>(smem);     // [2][KT][PA]: complex rows of A
    float* Bs = As + 2 * KT * PA;                   // [2][KT][PB]: complex rows of B

    // the staged registers go to LDS as they were loaded: one 128-bit store
    // when the pair is adjacent in a row, two 64-bit stores (rows k, k + 1)
    // when it runs along k
    auto store = [&](int buf) {
        float* a = As + buf * KT * PA;
        float* b = Bs + buf * KT * PB;
#pragma unroll
        for (int i = 0; i < LA; ++i) {
            const int f = tid + i * NT;
            if (FA % NT != 0 && f >= FA) break;
            const float4 v = ra[i];
            if (TA) {
                const int k = f / (BM / 2), m = 2 * (f % (BM / 2));
                *reinterpret_cast<float4*>(a + k * PA + 2 * m) = v;
            } else {
                const int m = f / (KT / 2), k = 2 * (f % (KT / 2));
                *reinterpret_cast<float2*>(a + k * PA + 2 * m) = make_float2(v.x, v.y);
                *reinterpret_cast<float2*>(a + (k + 1) * PA + 2 * m) = make_float2(v.z, v.w);
            }
        }
#pragma unroll
        for (int i = 0; i < LB; ++i) {
            const int f = tid + i * NT;
            if (FB % NT != 0 && f >= FB) break;
            const float4 v = rb[i];
            if (!TB) {
                const int k = f / (BN / 2), n = 2 * (f % (BN / 2));
                *reinterpret_cast<float4*>(b + k * PB + 2 * n) = v;
            } else {
                const int n = f / (KT / 2), k = 2 * (f % (KT / 2));
                *reinterpret_cast<float2*>(b + k * PB + 2 * n) = make_float2(v.x, v.y);
                *reinterpret_cast<float2*>(b + (k + 1) * PB + 2 * n) = make_float2(v.z, v.w);
            }
        }
    };

    auto compute = [&](int buf) {
        const float* a = As + buf * KT * PA;
        const float* b = Bs + buf * KT * PB;
        // lane (half, l32): A[m = l32][k = half], B[k = half][n = l32], one
        // 64-bit read each; operands of step ks + 1 are read while the MFMAs
        // of step ks issue; the third operand of 3M is re + im, formed here
        // in FP32
        float av[2][WMF][3], bv[2][WNF][3];
        auto rd = [&](int ks, int q) {
            const int kr = 2 * ks + half;
#pragma unroll
            for (int i = 0; i < WMF; ++i) {
                const float2 x = *reinterpret_cast<const float2*>(a + kr * PA + 2 * (wm + i * 32 + l32));
                av[q][i][0] = x.x;
                av[q][i][1] = x.y;
                av[q][i][2] = x.x + x.y;
            }
#pragma unroll
            for (int j = 0; j < WNF; ++j) {
                const float2 x = *reinterpret_cast<const float2*>(b + kr * PB + 2 * (wn + j * 32 + l32));
                bv[q][j][0] = x.x;
                bv[q][j][1] = x.y;
                bv[q][j][2] = x.x + x.y;
            }
        };
        rd(0, 0);
#pragma unroll
        for (int ks = 0; ks < KT / 2; ++ks) {
            if (ks + 1 < KT / 2) rd(ks + 1, (ks + 1) & 1);
            __builtin_amdgcn_sched_barrier(0);        // keep the reads ahead of the MFMAs
#pragma unroll
            for (int i = 0; i < WMF; ++i)
#pragma unroll
                for (int j = 0; j < WNF; ++j)
#pragma unroll
                    for (int p = 0; p < 3; ++p)
                        acc[i][j][p] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[ks & 1][i][p], bv[ks & 1][j][p],
                                                                            acc[i][j][p], 0, 0, 0);
        }
    };

    // Stages 0 .. nfull-1 of a tile inside the matrix are whole: their loads
    // are compiled with no bounds test.  Every pass ends with the store of
    // the stage it loaded.  Both keep the three or four global loads of a
    // stage issuing back to back: where a bounds-tested load and its
    // unchecked form write the same registers on merging paths, or a load
    // may still be outstanding where the loop begins again, the compiler
    // waits for each load before issuing the next.
    const bool inner = (m0 + BM <= Mt) && (n0 + BN <= Nt) && (!TA || g.M >= 2) && (TB || g.N >= 2);
    const int nk = (kper + KT - 1) / KT;
    const int nfull = inner ? kper / KT : 0;
    load(std::false_type{}, kb);
    store(0);
    __syncthreads();
    int t = 0;
    for (; t + 1 < nfull; ++t) {
        load(std::true_type{}, kb + (t + 1) * KT);
        compute(t & 1);
        store((t & 1) ^ 1);
        __syncthreads();
    }
    for (; t + 1 < nk; ++t) {
        load(std::false_type{}, kb + (t + 1) * KT);
        compute(t & 1);
        store((t & 1) ^ 1);
        __syncthreads();
    }
    if (nk > 0) compute((nk - 1) & 1);

    // epilogue: acc[i][j][p][r] is row 8*(r/4) + 4*half + r%4, column l32
    const bool part = g.splits > 1;
    float2* Cb = part ? g.P + (((size_t)split * n_outer + outer) * g.nbatch + ib) * (size_t)Mt * Nt
                      : g.C + bb * g.sCb + ib * g.sCi + rr * g.sCr;
    const bool fastdep = g.scatter && !part && g.M >= 32;
    RowDep rd;
    if (fastdep) rd.init(g.cPM);
#pragma unroll
    for (int i = 0; i < WMF; ++i)
#pragma unroll
        for (int j = 0; j < WNF; ++j) {
            const int np = n0 + wn + j * 32 + l32;
            if (np >= Nt) continue;
            const int n = np & (g.N - 1);
            unsigned long long dbase = 0;
            if (fastdep)
                dbase = pdep64((unsigned)((m0 + wm + i * 32) & (g.M - 1)), g.cPM) | pdep64((unsigned)n, g.cPN);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int mp = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                if (mp >= Mt) continue;
                size_t e;
                if (part) e = (size_t)mp * Nt + np;
                else {
                    const int m = mp & (g.M - 1);
                    e = (size_t)gemm_c_copy(g, (unsigned)(mp >> lgM), (unsigned)(np >> lgN)) +
                        (fastdep ? (size_t)(dbase | rd.low(r, half)) : gemm_c_elem(g, m, n));
                }
                const float p1 = acc[i][j][0][r], p2 = acc[i][j][1][r], p3 = acc[i][j][2][r];
                Cb[e] = make_float2(p1 - p2, p3 - p1 - p2);
            }
            // one block at a time: keeps the accumulators from being copied
            // out all at once (register pressure sets the occupancy)
            __builtin_amdgcn_sched_barrier(0);
        }
}

// ---------------------------------------------------------------------------
// Small products (at most 64 x 64 outputs per batch entry, K <= 256, one K
// range), FP32 4M and 3M:
// one wave per 32 x 32 complex output block of one batch entry, four waves
// per workgroup, operands read straight from global memory (a batch entry's
// operands are a few KiB) with no LDS and no barrier.  Each output element
// sees the same MFMA sequence over k as in k_cgemm / k_cgemm3m (two k per
// step for 3M, one complex k per step for 4M, from k = 0 up), so the
// results are bitwise those of the tile kernels; the kernel only packs the
// many tiny batch entries that leave a 128 x 32 tile mostly empty.
template <int PREC, bool TA, bool TB>
__global__ void __launch_bounds__(256) k_cgemm_wave(GemmArgs g) {
    const int Mt = gemm_rows(g);
    const int Nt = gemm_cols(g);
    const int lgM = __builtin_ctz((unsigned)g.M), lgN = __builtin_ctz((unsigned)g.N);
    const int bm = (Mt + 31) / 32, bnb = (Nt + 31) / 32;
    const size_t nblk = (size_t)bm * bnb;
    const size_t n_outer = g.fold == 0 ? (size_t)g.nr * g.nb : (size_t)g.nb;
    const size_t wid = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wid >= nblk * g.nbatch * n_outer) return;          // whole wave exits
    size_t blk = wid;
    const size_t tile = blk % nblk;
    blk /= nblk;
    const size_t ib = blk % g.nbatch;
    blk /= g.nbatch;
    const size_t bb = blk % g.nb;
    const size_t rr = g.fold == 0 ? blk / g.nb : 0;
    const int m0 = (int)(tile % bm) * 32, n0 = (int)(tile / bm) * 32;
    const float2* A = g.A + bb * g.sAb + ib * g.sAi + pext_u(rr, g.mA) * g.sAr;
    const float2* B = g.B + bb * g.sBb + ib * g.sBi + pext_u(rr, g.mB) * g.sBr;
    const long long sAf = (g.fold == 2 || g.fold == 3) ? g.sAr : 0;
    const long long sBf = (g.fold == 1 || g.fold == 3) ? g.sBr : 0;
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5;
    const int l32 = lane & 31;
    const int K = g.K;
    auto ldA = [&](int mp, int k) -> float2 {
        if (mp >= Mt || k >= K) return make_float2(0.f, 0.f);
        const int m = mp & (g.M - 1);
        return A[(size_t)(mp >> lgM) * sAf + (TA ? (size_t)k * g.M + m : (size_t)m * K + k)];
    };
    auto ldB = [&](int k, int np) -> float2 {
        if (np >= Nt || k >= K) return make_float2(0.f, 0.f);
        const int n = np & (g.N - 1);
        return B[(size_t)(np >> lgN) * sBf + (TB ? (size_t)n * K + k : (size_t)k * g.N + n)];
    };
    float2* Cb = g.C + bb * g.sCb + ib * g.sCi + rr * g.sCr;
    if constexpr (PREC == 1) {
        // 3M: lane (half, l32) holds A[m0 + l32][k] and B[k][n0 + l32] for
        // k = 2 ks + half; P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi)
        floatx16 acc[3];
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[p][r] = 0.f;
        const int nks = (K + 1) / 2;
        float2 a = ldA(m0 + l32, half), b = ldB(half, n0 + l32);
        for (int ks = 0; ks < nks; ++ks) {
            const float2 an = ldA(m0 + l32, 2 * ks + 2 + half), bn = ldB(2 * ks + 2 + half, n0 + l32);
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, acc[1], 0, 0, 0);
            acc[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x + a.y, b.x + b.y, acc[2], 0, 0, 0);
            a = an;
            b = bn;
        }
        // acc[p][r]: row 8 (r/4) + 4 half + r % 4, column l32
        const int np = n0 + l32;
        if (np >= Nt) return;
        const int n = np & (g.N - 1);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int mp = m0 + 8 * (r >> 2) + 4 * half + (r & 3);
            if (mp >= Mt) continue;
            const int m = mp & (g.M - 1);
            const size_t e = (size_t)gemm_c_copy(g, (unsigned)(mp >> lgM), (unsigned)(np >> lgN)) +
                             gemm_c_elem(g, m, n);
            const float p1 = acc[0][r], p2 = acc[1][r], p3 = acc[2][r];
            Cb[e] = make_float2(p1 - p2, p3 - p1 - p2);
        }
    } else {
        // 4M: one complex k per step; lane (half, l32) holds component half
        // of A[m0 + l32][k] and entry 2 half + (l32 & 1) of the expanded
        // 2 x 2 block [[Br, Bi], [-Bi, Br]] of B[k][n0 + 16 j + l32 / 2]
        floatx16 acc[2];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[j][r] = 0.f;
        auto bop = [&](float2 v) {
            return half == 0 ? ((l32 & 1) ? v.y : v.x) : ((l32 & 1) ? v.x : -v.y);
        };
        float2 a = ldA(m0 + l32, 0);
        float2 b0 = ldB(0, n0 + (l32 >> 1)), b1 = ldB(0, n0 + 16 + (l32 >> 1));
        for (int k = 0; k < K; ++k) {
            const float2 an = ldA(m0 + l32, k + 1);
            const float2 bn0 = ldB(k + 1, n0 + (l32 >> 1)), bn1 = ldB(k + 1, n0 + 16 + (l32 >> 1));
            const float av = half ? a.y : a.x;
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bop(b0), acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bop(b1), acc[1], 0, 0, 0);
            a = an;
            b0 = bn0;
            b1 = bn1;
        }
        // acc[j][r]: real row 8 (r/4) + 4 half + r % 4, real column l32 =
        // component l32 & 1 of complex column 16 j + l32 / 2
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int np = n0 + 16 * j + (l32 >> 1);
            if (np >= Nt) continue;
            const int n = np & (g.N - 1);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int mp = m0 + 8 * (r >> 2) + 4 * half + (r & 3);
                if (mp >= Mt) continue;
                const int m = mp & (g.M - 1);
                const size_t e = (size_t)gemm_c_copy(g, (unsigned)(mp >> lgM), (unsigned)(np >> lgN)) +
                                 gemm_c_elem(g, m, n);
                reinterpret_cast<float*>(Cb + e)[l32 & 1] = acc[j][r];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Tiny outputs (M*N <= 16), any K: each wave sums one K range of one batch
// entry (four waves per workgroup, no LDS); its 64 lanes are split into
// M*N groups of L = 64/(M*N) consecutive lanes, one output per group, lanes
// striding along k, then a butterfly over the group's lanes (fixed order).
// The products of the FP32 operands are exact in float64, and the lane sums
// and the butterfly run in float64: the only FP32 rounding is the final
// store (and the float64 partials of a split K are summed by
// k_reduce_splitk before it).
template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_cgemm_dot(GemmArgs g) {
    const size_t n_outer = (size_t)g.nr * g.nb;
    size_t blk = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (blk >= (size_t)g.splits * g.nbatch * n_outer) return;   // whole wave exits
    const int split = (int)(blk % g.splits);
    blk /= g.splits;
    const size_t ib = blk % g.nbatch;
    blk /= g.nbatch;
    const size_t bb = blk % g.nb;
    const size_t rr = blk / g.nb;                    // slice block as an outer batch
    const size_t outer = rr * g.nb + bb;
    const int kper = g.K / g.splits;
    const int kb = split * kper, ke = kb + kper;
    const float2* A = g.A + bb * g.sAb + ib * g.sAi + pext_u(rr, g.mA) * g.sAr;
    const float2* B = g.B + bb * g.sBb + ib * g.sBi + pext_u(rr, g.mB) * g.sBr;
    const int M = g.M, N = g.N, MN = M * N;
    const int L = 64 / MN;
    const int lane = threadIdx.x & 63;
    const int o = lane / L, kl = lane % L;
    const int m = o / N, n = o % N;
    double cr = 0.0, ci = 0.0;
    for (int k = kb + kl; k < ke; k += L) {
        const float2 a = TA ? A[(size_t)k * M + m] : A[(size_t)m * g.K + k];
        const float2 b = TB ? B[(size_t)n * g.K + k] : B[(size_t)k * N + n];
        cr = fma((double)a.x, (double)b.x, cr);
        cr = fma(-(double)a.y, (double)b.y, cr);
        ci = fma((double)a.x, (double)b.y, ci);
        ci = fma((double)a.y, (double)b.x, ci);
    }
    for (int w = L / 2; w > 0; w >>= 1) {
        cr += __shfl_xor(cr, w);
        ci += __shfl_xor(ci, w);
    }
    if (kl == 0) {
        if (g.splits > 1) {
            g.Pd[(((size_t)split * n_outer + outer) * g.nbatch + ib) * (size_t)MN + o] = make_double2(cr, ci);
        } else {
            float2* C = g.C + bb * g.sCb + ib * g.sCi + rr * g.sCr;
            C[gemm_c_elem(g, m, n)] = make_float2((float)cr, (float)ci);
        }
    }
}

// Sum of split-K partials in range order, in float64 and rounded to FP32
// once, written in C's layout.  Partial layout: [split][outer][inner
// batch][m'][n'] over the folded sizes; FP32 partials from the MFMA
// kernels, float64 partials (Pd, same layout) from the dot kernel.
template <bool DP>
__global__ void k_reduce_splitk(GemmArgs g) {
    const int Mt = gemm_rows(g);
    const int Nt = gemm_cols(g);
    const int lgM = __builtin_ctz((unsigned)g.M), lgN = __builtin_ctz((unsigned)g.N);
    const size_t n_outer = g.fold == 0 ? (size_t)g.nr * g.nb : (size_t)g.nb;
    const size_t MN = (size_t)Mt * Nt;
    const size_t per = MN * g.nbatch * n_outer;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < per;
         e += (size_t)gridDim.x * blockDim.x) {
        double sx = 0.0, sy = 0.0;
        for (int sp = 0; sp < g.splits; ++sp) {
            if (DP) {
                const double2 v = g.Pd[(size_t)sp * per + e];
                sx += v.x;
                sy += v.y;
            } else {
                const float2 v = g.P[(size_t)sp * per + e];
                sx += (double)v.x;
                sy += (double)v.y;
            }
        }
        const size_t mn = e % MN;
        const size_t bi = e / MN;
        const size_t ib = bi % g.nbatch, outer = bi / g.nbatch;
        const size_t bb = outer % g.nb, rr = g.fold == 0 ? outer / g.nb : 0;
        const int mp = (int)(mn / Nt), np = (int)(mn % Nt);
        const int m = mp & (g.M - 1), n = np & (g.N - 1);
        const size_t c = bb * g.sCb + ib * g.sCi + rr * g.sCr +
                         (size_t)gemm_c_copy(g, (unsigned)(mp >> lgM), (unsigned)(np >> lgN)) +
                         gemm_c_elem(g, m, n);
        g.C[c] = make_float2((float)sx, (float)sy);
    }
}

// ---------------------------------------------------------------------------
// Largest |re|, |im| over k of every row of A (OP = 0) or column of B
// (OP = 1), for every operand copy the GEMM reads, as the float's bit
// pattern (non-negative floats order like their bits): out[copy * R + row],
// copy as numbered by operand_copy, R = folded rows (columns).  CONTIG:
// k is the contiguous index, so L = min(K, 64) consecutive lanes read
// consecutive k of one row and combine by shuffles; otherwise consecutive
// lanes take consecutive rows at the same k.  Each thread covers OPMAX_KS
// values of k; the partial maxima meet by atomicMax (the words start at 0).
constexpr int OPMAX_KS = 32;

__global__ void k_zero_words(unsigned* p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

template <int OP, bool CONTIG>
__global__ void __launch_bounds__(256) k_opmax(GemmArgs g, unsigned* out, size_t total) {
    const int R = OP == 0 ? gemm_rows(g) : gemm_cols(g);
    const int lgX = __builtin_ctz((unsigned)(OP == 0 ? g.M : g.N));
    const int X = OP == 0 ? g.M : g.N;
    const int K = g.K;
    const int L = K < 64 ? K : 64;                  // CONTIG lanes per row
    const size_t per = (size_t)(CONTIG ? L : 1) * OPMAX_KS;
    const size_t kchunks = (K + per - 1) / per;
    const size_t items = total * kchunks * (CONTIG ? L : 1);
    // grid-stride over work items; the bound is rounded up to whole
    // workgroups so that every lane of a wave runs the same number of
    // rounds (the shuffles below need the whole wave)
    const size_t bound = (items + 255) / 256 * 256;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < bound; t += stride) {
        size_t row_all, kc;
        int lane_k;
        if (CONTIG) {
            lane_k = (int)(t % L);
            const size_t grp = t / L;
            kc = grp % kchunks;
            row_all = grp / kchunks;
        } else {
            lane_k = 0;
            row_all = t % total;
            kc = t / total;
        }
        float mx = 0.f;
        const bool live = t < items;
        if (live) {
            // operand copy (numbered as operand_copy does) and row within it
            const size_t inst = row_all / R;
            const int row = (int)(row_all % R);
            const unsigned m = OP ? g.mB : g.mA;
            const size_t nc = g.fold == 0 ? (size_t(1) << __builtin_popcount(m)) : 1;
            const size_t c = inst % nc;
            const size_t ib = (inst / nc) % g.nbatch, bx = inst / nc / g.nbatch;
            const float2* base;
            long long sF;
            bool trans;
            if (OP == 0) {
                base = g.A + bx * g.sAb + ib * g.sAi + c * g.sAr;
                sF = (g.fold == 2 || g.fold == 3) ? g.sAr : 0;
                trans = g.transA;
            } else {
                base = g.B + bx * g.sBb + ib * g.sBi + c * g.sBr;
                sF = (g.fold == 1 || g.fold == 3) ? g.sBr : 0;
                trans = !g.transB;       // B stored [k][n]: k is not contiguous
            }
            const int x = row & (X - 1);
            const float2* p = base + (size_t)(row >> lgX) * sF;
            const int kb = (int)(kc * per);
            for (int s = 0; s < OPMAX_KS; ++s) {
                const int k = CONTIG ? kb + s * L + lane_k : kb + s;
                if (k >= K) break;
                const float2 v = trans ? p[(size_t)k * X + x] : p[(size_t)x * K + k];
                mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
            }
        }
        if (CONTIG) {
            for (int o = 1; o < L; o <<= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
            if (live && lane_k == 0) atomicMax(out + row_all, __float_as_uint(mx));
        } else if (live) {
            atomicMax(out + row_all, __float_as_uint(mx));
        }
    }
}

// ---------------------------------------------------------------------------
// host-side dispatch

GemmChoice choose_gemm(int M, int N, int K, int nbatch, int Mt, int Nt) {
    GemmChoice c{};
    c.swap = 0;
    c.splits = 1;
    if (Mt <= 0) Mt = M;
    if (Nt <= 0) Nt = N;
    if ((long long)M * N <= 16) {
        c.kind = GEMM_DOT;
        long long want = K / 2048;
        c.splits = (int)std::max(1ll, std::min(1024ll, want));
        return c;
    }
    // K split from the unfolded shape only
    {
        int m = M, n = N;
        if (n > m && !(m >= 64 && n >= 64)) std::swap(m, n);
        long long tiles;
        if (m >= 128 && n >= 128) tiles = (long long)(m / 128) * (n / 128);
        else if (m >= 64 && n >= 64) tiles = (long long)(m / 64) * (n / 64);
        else tiles = (long long)((m + 127) / 128) * ((n + 15) / 16);
        long long wgs = tiles * nbatch;
        // an output of at most 32 x 32 per batch entry runs on one-wave
        // tiles (FP32 3M), which need more K ranges to fill the chip
        const int cap = (long long)M * N <= 1024 ? 256 : 64;
        int s = 1;
        while (wgs * s < 512 && (long long)K / (2 * s) >= 4 * KT && s < cap) s *= 2;
        c.splits = s;
    }
    // operand roles from the unfolded shape too: computing C^T = B^T A^T sums
    // the two real products of an imaginary part in the other order, so the
    // choice must not depend on the slice block
    c.swap = (N > M && !(M >= 64 && N >= 64)) ? 1 : 0;
    // tile shape from the folded sizes (does not change any summation)
    int m = c.swap ? Nt : Mt, n = c.swap ? Mt : Nt;
    if (m >= 128 && n >= 128) c.kind = GEMM_MFMA_128x128;
    else if (m >= 64 && n >= 64) c.kind = GEMM_MFMA_64x64;
    else c.kind = GEMM_MFMA_128x16;
    // small products of one K range (at most 64 x 64 outputs per batch
    // entry, K <= 256): one wave per 32 x 32 block (FP32 modes; the same
    // MFMA sequence per element as the tile kernels).  Decided from the
    // unfolded shape, like everything else here.
    if (c.splits == 1 && (long long)M * N <= 4096 && K <= 256) c.kind = GEMM_WAVE;
    return c;
}

// split-K partials in complex64 units: the dot kernel's partials are
// complex128 and take two units each
size_t gemm_scratch_elems(int M, int N, int K, int nbatch, int nouter) {
    GemmChoice c = choose_gemm(M, N, K, nbatch);
    if (c.splits <= 1) return 0;
    const size_t per = c.kind == GEMM_DOT ? 2 : 1;
    return per * c.splits * nouter * nbatch * (size_t)M * N;
}

size_t gemm_scale_words(int M, int N, int K, int nbatch, int nouter) {
    GemmChoice c = choose_gemm(M, N, K, nbatch);
    if (c.kind == GEMM_DOT) return 0;
    return (size_t)nouter * nbatch * ((size_t)M + N);
}

template <int PREC, int WGM, int WGN, int WMF, int WNF, bool TA, bool TB>
static void launch_one(const GemmArgs& g, size_t grid, hipStream_t s) {
    using SM = Smem<PREC, WGM, WGN, WMF, WNF>;
    const size_t lds = SM::bytes;
    auto* fn = &k_cgemm<PREC, WGM, WGN, WMF, WNF, TA, TB>;
    static std::once_flag attr;     // one per instantiation, safe from concurrent slots
    std::call_once(attr, [&] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    });
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(64 * WGM * WGN), lds, s, g);
}

template <int PREC, int WGM, int WGN, int WMF, int WNF>
static void launch_cfg(const GemmArgs& g, size_t grid, hipStream_t s) {
    if (g.transA) {
        if (g.transB) launch_one<PREC, WGM, WGN, WMF, WNF, true, true>(g, grid, s);
        else launch_one<PREC, WGM, WGN, WMF, WNF, true, false>(g, grid, s);
    } else {
        if (g.transB) launch_one<PREC, WGM, WGN, WMF, WNF, false, true>(g, grid, s);
        else launch_one<PREC, WGM, WGN, WMF, WNF, false, false>(g, grid, s);
    }
}

template <int WGM, int WGN, int WMF, int WNF, bool TA, bool TB>
static void launch_one3(const GemmArgs& g, size_t grid, hipStream_t s) {
    const size_t lds = Smem3<WGM, WGN, WMF, WNF>::bytes;
    auto* fn = &k_cgemm3m<WGM, WGN, WMF, WNF, TA, TB>;
    static std::once_flag attr;
    std::call_once(attr, [&] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    });
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(64 * WGM * WGN), lds, s, g);
}

template <int WGM, int WGN, int WMF, int WNF>
static void launch_cfg3(const GemmArgs& g, size_t grid, hipStream_t s) {
    if (g.transA) {
        if (g.transB) launch_one3<WGM, WGN, WMF, WNF, true, true>(g, grid, s);
        else launch_one3<WGM, WGN, WMF, WNF, true, false>(g, grid, s);
    } else {
        if (g.transB) launch_one3<WGM, WGN, WMF, WNF, false, true>(g, grid, s);
        else launch_one3<WGM, WGN, WMF, WNF, false, false>(g, grid, s);
    }
}

template <int WGM, int WGN, int WMF, int WNF>
static void launch_prec(const GemmArgs& g, int precision, size_t grid, hipStream_t s) {
    if (precision == 2) launch_cfg<2, WGM, WGN, WMF, WNF>(g, grid, s);
    else if (precision == 3) launch_cfg<3, WGM, WGN, WMF, WNF>(g, grid, s);
    else if (precision == 4) launch_cfg<4, WGM, WGN, WMF, WNF>(g, grid, s);
    else launch_cfg<0, WGM, WGN, WMF, WNF>(g, grid, s);
}

hipError_t launch_gemm(const GemmArgs& g0, int precision, hipStream_t s) {
    GemmArgs g = g0;
    if (g.nr < 1) g.nr = 1;
    if (g.nr == 1) g.fold = 0;
    const int Mt0 = gemm_rows(g);
    const int Nt0 = gemm_cols(g);
    GemmChoice c = choose_gemm(g.M, g.N, g.K, g.nbatch, Mt0, Nt0);
    if (c.kind == GEMM_DOT && g.fold != 0) {
        // copies as an outer batch: with fold 1 or 2 the folded operand takes
        // every copy; fold 3 keeps its masks
        const unsigned all = (unsigned)g.nr - 1;
        if (g.fold == 1) { g.mA = 0; g.mB = all; }
        else if (g.fold == 2) { g.mA = all; g.mB = 0; }
        g.fold = 0;
    }
    // FP32 3M forms each complex product from three real products, each the
    // same value whichever operand takes the row role, summed over k in the
    // same order, so operand roles change no 3M result.  A thin 3M product
    // (at most 32 folded rows, at least 128 columns) therefore keeps its
    // roles and takes a 32 x 128 tile: lanes then run along C's contiguous
    // columns, where the swapped form would write C one 8-byte element per
    // lane at a stride of the whole row count.
    const bool wide3 = precision == 1 && c.kind == GEMM_MFMA_128x16 && c.swap && Mt0 <= 32 && Nt0 >= 128;
    if (c.swap && !wide3) {
        // C^T = B^T A^T, written transposed
        g.A = g0.B; g.B = g0.A;
        g.M = g0.N; g.N = g0.M;
        g.transA = !g0.transB; g.transB = !g0.transA;
        g.sAb = g0.sBb; g.sAi = g0.sBi; g.sAr = g0.sBr; g.mA = g0.mB;
        g.sBb = g0.sAb; g.sBi = g0.sAi; g.sBr = g0.sAr; g.mB = g0.mA;
        g.transC = !g0.transC;
        g.cPM = g0.cPN; g.cPN = g0.cPM;
        g.fold = g.fold == 1 ? 2 : g.fold == 2 ? 1 : g.fold;
    }
    g.splits = c.splits;
    if (c.splits > 1 && !g.P) return hipErrorInvalidValue;
    g.Pd = reinterpret_cast<double2*>(g.P);
    const int Mt = gemm_rows(g);
    const int Nt = gemm_cols(g);
    const size_t n_outer = g.fold == 0 ? (size_t)g.nr * g.nb : (size_t)g.nb;
    const size_t batches = (size_t)g.nbatch * n_outer * c.splits;
    if (c.kind == GEMM_DOT) {
        const unsigned grid = (unsigned)((batches + 3) / 4);     // one wave per batch entry and K range
        if (g.transA) {
            if (g.transB) hipLaunchKernelGGL((k_cgemm_dot<true, true>), dim3(grid), dim3(256), 0, s, g);
            else hipLaunchKernelGGL((k_cgemm_dot<true, false>), dim3(grid), dim3(256), 0, s, g);
        } else {
            if (g.transB) hipLaunchKernelGGL((k_cgemm_dot<false, true>), dim3(grid), dim3(256), 0, s, g);
            else hipLaunchKernelGGL((k_cgemm_dot<false, false>), dim3(grid), dim3(256), 0, s, g);
        }
    } else {
        if (precision == 3) {
            // row maxima of A, column maxima of B over every operand copy
            if (!g.X) return hipErrorInvalidValue;
            // one set of maxima per operand copy (see operand_copy)
            auto copies = [&](long long sb, unsigned m) -> size_t {
                return (sb ? (size_t)g.nb : 1) * g.nbatch * (g.fold == 0 ? (size_t(1) << __builtin_popcount(m)) : 1);
            };
            const size_t ra = (size_t)Mt * copies(g.sAb, g.mA), rb = (size_t)Nt * copies(g.sBb, g.mB);
            unsigned* xa = g.X;
            unsigned* xb = g.X + ra;
            g.xA = xa;
            g.xB = xb;
            const unsigned zb = (unsigned)std::min<size_t>((ra + rb + 255) / 256, 1u << 16);
            hipLaunchKernelGGL(k_zero_words, dim3(zb), dim3(256), 0, s, xa, ra + rb);
            const int L = std::min(g.K, 64);
            for (int op = 0; op < 2; ++op) {
                const size_t rows = op ? rb : ra;
                const bool contig = op ? g.transB : !g.transA;
                const size_t per = contig ? (size_t)L * OPMAX_KS : (size_t)OPMAX_KS;
                const size_t items = rows * ((g.K + per - 1) / per) * (contig ? L : 1);
                const size_t blocks = std::min<size_t>((items + 255) / 256, 1u << 16);
                unsigned* out = op ? xb : xa;
                if (op == 0) {
                    if (contig) hipLaunchKernelGGL((k_opmax<0, true>), dim3((unsigned)blocks), dim3(256), 0, s, g, out, rows);
                    else hipLaunchKernelGGL((k_opmax<0, false>), dim3((unsigned)blocks), dim3(256), 0, s, g, out, rows);
                } else {
                    if (contig) hipLaunchKernelGGL((k_opmax<1, true>), dim3((unsigned)blocks), dim3(256), 0, s, g, out, rows);
                    else hipLaunchKernelGGL((k_opmax<1, false>), dim3((unsigned)blocks), dim3(256), 0, s, g, out, rows);
                }
            }
        }
        if (c.kind == GEMM_WAVE && (precision == 0 || precision == 1)) {
            const size_t waves = (size_t)((Mt + 31) / 32) * ((Nt + 31) / 32) * g.nbatch * n_outer;
            const unsigned grid = (unsigned)((waves + 3) / 4);
            if (precision == 1) {
                if (g.transA) {
                    if (g.transB) hipLaunchKernelGGL((k_cgemm_wave<1, true, true>), dim3(grid), dim3(256), 0, s, g);
                    else hipLaunchKernelGGL((k_cgemm_wave<1, true, false>), dim3(grid), dim3(256), 0, s, g);
                } else {
                    if (g.transB) hipLaunchKernelGGL((k_cgemm_wave<1, false, true>), dim3(grid), dim3(256), 0, s, g);
                    else hipLaunchKernelGGL((k_cgemm_wave<1, false, false>), dim3(grid), dim3(256), 0, s, g);
                }
            } else {
                if (g.transA) {
                    if (g.transB) hipLaunchKernelGGL((k_cgemm_wave<0, true, true>), dim3(grid), dim3(256), 0, s, g);
                    else hipLaunchKernelGGL((k_cgemm_wave<0, true, false>), dim3(grid), dim3(256), 0, s, g);
                } else {
                    if (g.transB) hipLaunchKernelGGL((k_cgemm_wave<0, false, true>), dim3(grid), dim3(256), 0, s, g);
                    else hipLaunchKernelGGL((k_cgemm_wave<0, false, false>), dim3(grid), dim3(256), 0, s, g);
                }
            }
            return hipGetLastError();
        }
        if (c.kind == GEMM_WAVE) c.kind = GEMM_MFMA_128x16;     // split modes: the tile kernel
        int bm = 128, bn = 128;
        if (c.kind == GEMM_MFMA_128x128 && precision == 1) bn = 64;
        if (c.kind == GEMM_MFMA_64x64) { bm = 64; bn = 64; }
        if (c.kind == GEMM_MFMA_128x16) { bm = 128; bn = precision == 1 ? 32 : 16; }
        // 3M skinny products with at most 64 (32) folded rows and 32 columns:
        // a 64 x 32 (32 x 32) tile on two waves (one) instead of a 128 x 32
        // tile that is half (three quarters) zero rows; same MFMA sequence
        // per output element, so the choice from the folded sizes changes
        // no result
        const bool thin3 = precision == 1 && c.kind == GEMM_MFMA_128x16 && Nt <= 32 && Mt <= 64;
        if (thin3) bm = Mt <= 32 ? 32 : 64;
        if (wide3) { bm = 32; bn = 128; }
        const size_t grid = (size_t)((Mt + bm - 1) / bm) * ((Nt + bn - 1) / bn) * batches;
        if (precision == 1) {
            // 3M tiles: 128 x 128, 64 x 64, and 128 x 32 (64 x 32, 32 x 32)
            // for the skinny shapes
            if (c.kind == GEMM_MFMA_128x128) launch_cfg3<4, 2, 1, 1>(g, grid, s);
            else if (c.kind == GEMM_MFMA_64x64) launch_cfg3<2, 2, 1, 1>(g, grid, s);
            else if (wide3) launch_cfg3<1, 4, 1, 1>(g, grid, s);
            else if (thin3 && bm == 32) launch_cfg3<1, 1, 1, 1>(g, grid, s);
            else if (thin3) launch_cfg3<2, 1, 1, 1>(g, grid, s);
            else launch_cfg3<4, 1, 1, 1>(g, grid, s);
        } else if (c.kind == GEMM_MFMA_128x128) launch_prec<4, 2, 1, 4>(g, precision, grid, s);
        else if (c.kind == GEMM_MFMA_64x64) launch_prec<2, 2, 1, 2>(g, precision, grid, s);
        else launch_prec<4, 1, 1, 1>(g, precision, grid, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || c.splits <= 1) return e;
    const size_t per = (size_t)Mt * Nt * g.nbatch * n_outer;
    unsigned blocks = (unsigned)std::min<size_t>((per + 255) / 256, 1u << 16);
    if (c.kind == GEMM_DOT) hipLaunchKernelGGL(k_reduce_splitk<true>, dim3(blocks), dim3(256), 0, s, g);
    else hipLaunchKernelGGL(k_reduce_splitk<false>, dim3(blocks), dim3(256), 0, s, g);
    return hipGetLastError();
}

int gemm_kind(const GemmArgs& g, int precision) {
    GemmArgs f = g;
    if (f.nr <= 1) { f.nr = 1; f.fold = 0; }
    const int Mt = gemm_rows(f);
    const int Nt = gemm_cols(f);
    const int k = choose_gemm(g.M, g.N, g.K, g.nbatch, Mt, Nt).kind;
    return k == GEMM_WAVE && precision != 0 && precision != 1 ? GEMM_MFMA_128x16 : k;
}
