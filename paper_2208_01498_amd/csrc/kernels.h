// Kernel argument blocks and launchers (device code in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define TN_MAX_GATHER 24
#define TN_MAX_TILE 16
#define TN_MAX_BITS 48

struct GatherArgs {
    const float2* src;
    float2* dst;
    const uint64_t* bits;     // bitstrings of the chunk (one per b)
    uint32_t slice;           // high bits of the slice index (the pass)
    uint32_t dmask;           // low slice bits the leaf depends on
    int nb;                   // batch count (chunk if the leaf has outputs, else 1)
    int nr;                   // copies: 2^popcount(dmask); copy c has low bits pdep(c, dmask)
    int n_mat, n_out, n_sl;
    int mat_src[TN_MAX_GATHER];
    int out_src[TN_MAX_GATHER];
    int out_qubit[TN_MAX_GATHER];
    int sl_src[TN_MAX_GATHER];
    int sl_bit[TN_MAX_GATHER];
};

struct PermArgs {
    const float2* src;
    float2* dst;
    int rank;                 // bits per b
    int nb;                   // batch count
    int nt;                   // tile bits
    int nn;                   // non-tile bits
    int t_in[TN_MAX_TILE];    // tile bit m (input order) -> input bit position
    int t_out[TN_MAX_TILE];   // tile bit m (output order) -> output bit position
    int t_rank[TN_MAX_TILE];  // tile bit m (output order) -> its index in input order
    int n_in[TN_MAX_BITS];    // non-tile bit m -> input bit position
    int n_out[TN_MAX_BITS];   // non-tile bit m -> output bit position
};

struct GemmArgs {
    const float2* A;
    const float2* B;
    float2* C;
    float2* P;                // split-K partials (splits x nb x nbatch x M x N)
    double2* Pd;              // set by the dispatcher: P as float64 partials (dot kernel)
    int splits;               // set by the dispatcher
    int transC;               // C stored [N][M]
    int M, N, K;
    int transA, transB;       // A stored [K][M] / B stored [N][K]
    int nbatch;               // inner batch count (batch labels)
    int nb;                   // outer batch count (bitstrings)
    int nr;                   // copies of C over the slice block, 1 if none
    int fold;                 // 0: copies as an outer batch; 1: folded into N
                              // (only B and C vary with it); 2: folded into M;
                              // 3: A's copies into M and B's into N (disjoint
                              // copy bits covering C's)
    unsigned mA, mB;          // A's copy = pext(c, mA), B's copy = pext(c, mB)
                              // for C's copy c
    long long sAb, sBb, sCb;  // outer strides (elements); 0 = broadcast
    long long sAi, sBi, sCi;  // inner strides
    long long sAr, sBr, sCr;  // slice-block strides; 0 = broadcast
    int scatter;              // C element (m, n) at pdep(m, cPM) | pdep(n, cPN)
    unsigned long long cPM, cPN;
    unsigned* X;              // split fp16 only: workspace for the largest |re|, |im|
                              // of every row of A and column of B (float bits),
                              // gemm_scale_words() words
    const unsigned* xA;       // set by the dispatcher: [outer][inner batch][m']
    const unsigned* xB;       // [outer][inner batch][n']
};

// Folded GEMM sizes: the row index m' = a * M + m and column index
// n' = b * N + n carry operand copies a, b when they are folded.
__host__ __device__ inline int gemm_rows(const GemmArgs& g) {
    return g.fold == 2 ? g.M * g.nr : g.fold == 3 ? g.M << __builtin_popcount(g.mA) : g.M;
}
__host__ __device__ inline int gemm_cols(const GemmArgs& g) {
    return g.fold == 1 ? g.N * g.nr : g.fold == 3 ? g.N << __builtin_popcount(g.mB) : g.N;
}
// scatter the low bits of x to the set positions of m (parallel bit deposit)
__host__ __device__ inline unsigned pdep_bits(unsigned x, unsigned m) {
    unsigned r = 0;
    for (; m; m &= m - 1, x >>= 1)
        if (x & 1) r |= m & (~m + 1);
    return r;
}
__host__ __device__ inline unsigned long long pdep64(unsigned long long x, unsigned long long m) {
    unsigned long long r = 0;
    for (; m; m &= m - 1, x >>= 1)
        if (x & 1) r |= m & (~m + 1);
    return r;
}
// offset of C element (m, n) within one batch entry
__host__ __device__ inline size_t gemm_c_elem(const GemmArgs& g, int m, int n) {
    if (g.scatter) return (size_t)(pdep64((unsigned)m, g.cPM) | pdep64((unsigned)n, g.cPN));
    return g.transC ? (size_t)n * g.M + m : (size_t)m * g.N + n;
}
// element offset of C's copy for folded row block a and column block b
__host__ __device__ inline long long gemm_c_copy(const GemmArgs& g, unsigned a, unsigned b) {
    if (g.fold == 3) return (long long)(pdep_bits(a, g.mA) | pdep_bits(b, g.mB)) * g.sCr;
    return (long long)a * (g.fold == 2 ? g.sCr : 0) + (long long)b * (g.fold == 1 ? g.sCr : 0);
}

hipError_t launch_gather(const GatherArgs& g, hipStream_t s);
hipError_t launch_permute(const PermArgs& a, hipStream_t s);
// kernel classes of the GEMMs (the values index the per-class statistics,
// where 4 and 5 are the permute and gather kernels)
enum { GEMM_DOT = 0, GEMM_MFMA_64x64 = 1, GEMM_MFMA_128x128 = 2, GEMM_MFMA_128x16 = 3,
       GEMM_WAVE = 6 };
constexpr int kKernelClasses = 7;
struct GemmChoice {
    int kind;                 // GEMM_*
    int splits;               // K ranges (1 = no split-K)
    int swap;                 // compute C^T = B^T A^T
};
// Kernel choice.  The arithmetic (dot-product kernel or MFMA kernel, and the
// number of K ranges) depends on the per-matrix shape M, N, K and the inner
// batch only; the tile shape may also depend on the folded sizes, which does
// not change any element's summation order.
GemmChoice choose_gemm(int M, int N, int K, int nbatch, int Mt = 0, int Nt = 0);
size_t gemm_scratch_elems(int M, int N, int K, int nbatch, int nouter);
// 32-bit words of row and column maxima the split fp16 products need (0 for
// shapes that take the dot-product kernel); nouter counts bitstrings times
// slice-block copies of C
size_t gemm_scale_words(int M, int N, int K, int nbatch, int nouter);
hipError_t launch_gemm(const GemmArgs& g, int precision, hipStream_t s);
int gemm_kind(const GemmArgs& g, int precision);
hipError_t launch_zero_acc(double2* acc, int nb, hipStream_t s);
// acc[b] += sum over r < nr (ascending) of v[r * vr + (v_has_b ? b : 0)]
hipError_t launch_accumulate(double2* acc, const float2* v, int nb, int v_has_b, int nr,
                             long long vr, hipStream_t s);
hipError_t launch_finalize(double2* acc, int nb, double sre, double sim, hipStream_t s);
