// HIP kernels of the amplitude engine for gfx950 (MI355X).
//
//  k_gather_leaf    leaf -> operand: output labels replaced by the
//                   bitstring's bits (gives the batch index b), sliced labels
//                   by the slice's bits, remaining labels in gathered order
//  k_permute_tiled  bit permutation of a tensor's address, staged through LDS
//                   so that reads run along the lowest input bits and writes
//                   along the lowest output bits
//  k_cgemm_small    complex GEMM on the vector ALU for small M, N, K
//  k_cgemm_mfma     complex GEMM on v_mfma_f32_32x32x2_f32: with interleaved
//                   complex operands one instruction multiplies a 32 x 1
//                   complex column of A by a 1 x 16 complex row of B (the
//                   real 4M form [Ar Ai] [[Br Bi] [-Bi Br]] = [Cr Ci])
//  k_cgemm_split    the same on v_mfma_f32_32x32x16_bf16 with x = hi + lo
//                   bf16 halves and hi*hi + hi*lo + lo*hi, FP32 accumulation
//  k_accumulate     FP64 slice sums;  k_finalize  scale and write out
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include "kernels.h"

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef short shortx8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
__global__ void k_gather_leaf(GatherArgs g) {
    const size_t per = size_t(1) << g.n_mat;
    const size_t total = per * (size_t)g.nb;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t b = idx >> g.n_mat;
        const size_t j = idx & (per - 1);
        size_t src = 0;
        for (int p = 0; p < g.n_mat; ++p)
            if ((j >> p) & 1) src |= size_t(1) << g.mat_src[p];
        if (g.n_out) {
            const uint64_t x = g.bits[b];
            for (int i = 0; i < g.n_out; ++i)
                if ((x >> g.out_qubit[i]) & 1) src |= size_t(1) << g.out_src[i];
        }
        for (int i = 0; i < g.n_sl; ++i)
            if ((g.slice >> g.sl_bit[i]) & 1) src |= size_t(1) << g.sl_src[i];
        g.dst[idx] = g.src[src];
    }
}

// ---------------------------------------------------------------------------
// One workgroup per tile: the tile holds every combination of the tile bits
// T (the lowest input bits plus the input bits that become the lowest
// output bits) for fixed values of all other bits and of b.
__global__ void __launch_bounds__(256) k_permute_tiled(PermArgs a) {
    extern __shared__ float2 lds[];
    const int t = a.nt;
    const size_t tile_elems = size_t(1) << t;
    const size_t r_elems = size_t(1) << a.rank;
    const size_t tid = blockIdx.x;
    const size_t b = blockIdx.y;
    size_t base_in = 0, base_out = 0;
    for (int m = 0; m < a.nn; ++m)
        if ((tid >> m) & 1) {
            base_in |= size_t(1) << a.n_in[m];
            base_out |= size_t(1) << a.n_out[m];
        }
    const float2* src = a.src + b * r_elems + base_in;
    float2* dst = a.dst + b * r_elems + base_out;
    for (size_t e = threadIdx.x; e < tile_elems; e += blockDim.x) {
        size_t off = 0;
        for (int m = 0; m < t; ++m)
            if ((e >> m) & 1) off |= size_t(1) << a.t_in[m];
        lds[e + (e >> 5)] = src[off];
    }
    __syncthreads();
    for (size_t f = threadIdx.x; f < tile_elems; f += blockDim.x) {
        size_t off = 0, e = 0;
        for (int m = 0; m < t; ++m)
            if ((f >> m) & 1) {
                off |= size_t(1) << a.t_out[m];
                e |= size_t(1) << a.t_rank[m];
            }
        dst[off] = lds[e + (e >> 5)];
    }
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ float2 ld_a(const GemmArgs& g, const float2* A, int m, int k) {
    return g.transA ? A[(size_t)k * g.M + m] : A[(size_t)m * g.K + k];
}
__device__ __forceinline__ float2 ld_b(const GemmArgs& g, const float2* B, int k, int n) {
    return g.transB ? B[(size_t)n * g.K + k] : B[(size_t)k * g.N + n];
}

__global__ void k_cgemm_small(GemmArgs g) {
    const size_t MN = (size_t)g.M * g.N;
    const size_t total = MN * (size_t)g.nbatch * (size_t)g.nb;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t mn = idx % MN;
        const size_t bi = idx / MN;
        const size_t ib = bi % g.nbatch;
        const size_t bb = bi / g.nbatch;
        const int m = (int)(mn / g.N);
        const int n = (int)(mn % g.N);
        const float2* A = g.A + bb * g.sAb + ib * g.sAi;
        const float2* B = g.B + bb * g.sBb + ib * g.sBi;
        float cr = 0.f, ci = 0.f;
        for (int k = 0; k < g.K; ++k) {
            const float2 x = ld_a(g, A, m, k);
            const float2 y = ld_b(g, B, k, n);
            cr = fmaf(x.x, y.x, cr);
            cr = fmaf(-x.y, y.y, cr);
            ci = fmaf(x.x, y.y, ci);
            ci = fmaf(x.y, y.x, ci);
        }
        g.C[bb * g.sCb + ib * g.sCi + mn] = make_float2(cr, ci);
    }
}

// ---------------------------------------------------------------------------
// MFMA complex GEMM, FP32 4M.  Workgroup = 4 waves (2 x 2); a wave owns
// WMF x WNF blocks of 32 (m) x 16 (complex n); a stage stages KT complex k of
// A (BM x KT) and B (KT x BN) in LDS, A as [k][m] and B as [k][n].
template <int WMF, int WNF>
__global__ void __launch_bounds__(256) k_cgemm_mfma(GemmArgs g) {
    constexpr int BM = 64 * WMF;
    constexpr int BN = 32 * WNF;
    constexpr int KT = 8;
    constexpr int PA = BM + 4;   // padded row lengths (complex)
    constexpr int PB = BN + 4;
    __shared__ float2 As[KT * PA];
    __shared__ float2 Bs[KT * PB];

    const int tiles_m = (g.M + BM - 1) / BM;
    const int tiles_n = (g.N + BN - 1) / BN;
    const size_t tiles = (size_t)tiles_m * tiles_n;
    const size_t blk = blockIdx.x;
    const size_t tile = blk % tiles;
    const size_t bi = blk / tiles;
    const size_t ib = bi % g.nbatch;
    const size_t bb = bi / g.nbatch;
    const int tm = (int)(tile % tiles_m);
    const int tn = (int)(tile / tiles_m);
    const int m0 = tm * BM, n0 = tn * BN;
    const float2* A = g.A + bb * g.sAb + ib * g.sAi;
    const float2* B = g.B + bb * g.sBb + ib * g.sBi;
    float* C = reinterpret_cast<float*>(g.C + bb * g.sCb + ib * g.sCi);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = (wave & 1) * (32 * WMF);
    const int wn = (wave >> 1) * (16 * WNF);
    const int half = lane >> 5;       // k-row of the MFMA operands
    const int l32 = lane & 31;

    floatx16 acc[WMF][WNF];
#pragma unroll
    for (int i = 0; i < WMF; ++i)
#pragma unroll
        for (int j = 0; j < WNF; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    for (int k0 = 0; k0 < g.K; k0 += KT) {
        // ---- global -> LDS
        for (int e = tid; e < BM * KT; e += 256) {
            int m, k;
            if (g.transA) { m = e % BM; k = e / BM; }
            else { k = e % KT; m = e / KT; }
            float2 v = make_float2(0.f, 0.f);
            if (m0 + m < g.M && k0 + k < g.K) v = ld_a(g, A, m0 + m, k0 + k);
            As[k * PA + m] = v;
        }
        for (int e = tid; e < KT * BN; e += 256) {
            int n, k;
            if (g.transB) { k = e % KT; n = e / KT; }
            else { n = e % BN; k = e / BN; }
            float2 v = make_float2(0.f, 0.f);
            if (n0 + n < g.N && k0 + k < g.K) v = ld_b(g, B, k0 + k, n0 + n);
            Bs[k * PB + n] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KT; ++kk) {
            float av[WMF];
            float bv[WNF];
#pragma unroll
            for (int i = 0; i < WMF; ++i) {
                const float2 x = As[kk * PA + wm + i * 32 + l32];
                av[i] = half ? x.y : x.x;
            }
#pragma unroll
            for (int j = 0; j < WNF; ++j) {
                const float2 y = Bs[kk * PB + wn + j * 16 + (l32 >> 1)];
                const int c = l32 & 1;
                // real row kr = half, column 2n + c of [[Br Bi] [-Bi Br]]
                bv[j] = half ? (c ? y.x : -y.y) : (c ? y.y : y.x);
            }
#pragma unroll
            for (int i = 0; i < WMF; ++i)
#pragma unroll
                for (int j = 0; j < WNF; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // ---- epilogue: acc[i][j][r] is real row 8*(r/4) + 4*half + r%4, column l32
#pragma unroll
    for (int i = 0; i < WMF; ++i)
#pragma unroll
        for (int j = 0; j < WNF; ++j) {
            const int n = n0 + wn + j * 16 + (l32 >> 1);
            if (n >= g.N) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                if (m < g.M) C[(size_t)m * (2 * (size_t)g.N) + 2 * (size_t)n + (l32 & 1)] = acc[i][j][r];
            }
        }
}

// ---------------------------------------------------------------------------
// Split bf16 complex GEMM.  One v_mfma_f32_32x32x16_bf16 takes 8 complex k:
// lane (half h, row/col l32) holds real k = 8h..8h+7, i.e. complex k =
// 4h..4h+3 as (re, im) pairs for A, and the matching rows of the 2 x 2 real
// expansion of B.  Operands are split x = hi + lo (bf16, round to nearest
// even) when staged; three products hi*hi + hi*lo + lo*hi are accumulated.
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
    hi = __float2bfloat16(x);
    lo = __float2bfloat16(x - __bfloat162float(hi));
}

template <int WMF, int WNF>
__global__ void __launch_bounds__(256) k_cgemm_split(GemmArgs g) {
    constexpr int BM = 64 * WMF;
    constexpr int BN = 32 * WNF;
    constexpr int KT = 8;                 // complex k per stage = one MFMA
    // A staged as [m][2*KT real] hi and lo; B as [n-col (real, 2*BN)][2*KT real]
    constexpr int RA = 2 * KT + 8;        // padded row (bf16 elements)
    __shared__ __attribute__((aligned(16))) __bf16 Ah[BM * RA];
    __shared__ __attribute__((aligned(16))) __bf16 Al[BM * RA];
    __shared__ __attribute__((aligned(16))) __bf16 Bh[2 * BN * RA];
    __shared__ __attribute__((aligned(16))) __bf16 Bl[2 * BN * RA];

    const int tiles_m = (g.M + BM - 1) / BM;
    const int tiles_n = (g.N + BN - 1) / BN;
    const size_t tiles = (size_t)tiles_m * tiles_n;
    const size_t blk = blockIdx.x;
    const size_t tile = blk % tiles;
    const size_t bi = blk / tiles;
    const size_t ib = bi % g.nbatch;
    const size_t bb = bi / g.nbatch;
    const int tm = (int)(tile % tiles_m);
    const int tn = (int)(tile / tiles_m);
    const int m0 = tm * BM, n0 = tn * BN;
    const float2* A = g.A + bb * g.sAb + ib * g.sAi;
    const float2* B = g.B + bb * g.sBb + ib * g.sBi;
    float* C = reinterpret_cast<float*>(g.C + bb * g.sCb + ib * g.sCi);

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = (wave & 1) * (32 * WMF);
    const int wn = (wave >> 1) * (16 * WNF);
    const int half = lane >> 5;
    const int l32 = lane & 31;

    floatx16 acc[WMF][WNF];
#pragma unroll
    for (int i = 0; i < WMF; ++i)
#pragma unroll
        for (int j = 0; j < WNF; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    for (int k0 = 0; k0 < g.K; k0 += KT) {
        for (int e = tid; e < BM * KT; e += 256) {
            int m, k;
            if (g.transA) { m = e % BM; k = e / BM; }
            else { k = e % KT; m = e / KT; }
            float2 v = make_float2(0.f, 0.f);
            if (m0 + m < g.M && k0 + k < g.K) v = ld_a(g, A, m0 + m, k0 + k);
            __bf16 h, l;
            split_bf16(v.x, h, l);
            Ah[m * RA + 2 * k] = h;
            Al[m * RA + 2 * k] = l;
            split_bf16(v.y, h, l);
            Ah[m * RA + 2 * k + 1] = h;
            Al[m * RA + 2 * k + 1] = l;
        }
        for (int e = tid; e < KT * BN; e += 256) {
            int n, k;
            if (g.transB) { k = e % KT; n = e / KT; }
            else { n = e % BN; k = e / BN; }
            float2 v = make_float2(0.f, 0.f);
            if (n0 + n < g.N && k0 + k < g.K) v = ld_b(g, B, k0 + k, n0 + n);
            // real column 2n:   rows (2k, 2k+1) = ( Br, -Bi)
            // real column 2n+1: rows (2k, 2k+1) = ( Bi,  Br)
            __bf16 h, l;
            split_bf16(v.x, h, l);
            Bh[(2 * n) * RA + 2 * k] = h;      Bl[(2 * n) * RA + 2 * k] = l;
            Bh[(2 * n + 1) * RA + 2 * k + 1] = h; Bl[(2 * n + 1) * RA + 2 * k + 1] = l;
            split_bf16(-v.y, h, l);
            Bh[(2 * n) * RA + 2 * k + 1] = h;  Bl[(2 * n) * RA + 2 * k + 1] = l;
            split_bf16(v.y, h, l);
            Bh[(2 * n + 1) * RA + 2 * k] = h;  Bl[(2 * n + 1) * RA + 2 * k] = l;
        }
        __syncthreads();
        bf16x8 ah[WMF], al[WMF], bh[WNF], bl[WNF];
#pragma unroll
        for (int i = 0; i < WMF; ++i) {
            const int m = wm + i * 32 + l32;
            ah[i] = *reinterpret_cast<const bf16x8*>(&Ah[m * RA + 8 * half]);
            al[i] = *reinterpret_cast<const bf16x8*>(&Al[m * RA + 8 * half]);
        }
#pragma unroll
        for (int j = 0; j < WNF; ++j) {
            const int col = 2 * (wn + j * 16) + l32;
            bh[j] = *reinterpret_cast<const bf16x8*>(&Bh[col * RA + 8 * half]);
            bl[j] = *reinterpret_cast<const bf16x8*>(&Bl[col * RA + 8 * half]);
        }
#pragma unroll
        for (int i = 0; i < WMF; ++i)
#pragma unroll
            for (int j = 0; j < WNF; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < WMF; ++i)
#pragma unroll
        for (int j = 0; j < WNF; ++j) {
            const int n = n0 + wn + j * 16 + (l32 >> 1);
            if (n >= g.N) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = m0 + wm + i * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                if (m < g.M) C[(size_t)m * (2 * (size_t)g.N) + 2 * (size_t)n + (l32 & 1)] = acc[i][j][r];
            }
        }
}

// ---------------------------------------------------------------------------
__global__ void k_zero_acc(double2* acc, int nb) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) acc[b] = make_double2(0.0, 0.0);
}

__global__ void k_accumulate(double2* acc, const float2* v, int nb, int v_has_b) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) {
        const float2 x = v[v_has_b ? b : 0];
        double2 a = acc[b];
        a.x += (double)x.x;
        a.y += (double)x.y;
        acc[b] = a;
    }
}

__global__ void k_finalize(double2* acc, int nb, double sre, double sim) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) {
        double2 a = acc[b];
        acc[b] = make_double2(a.x * sre - a.y * sim, a.x * sim + a.y * sre);
    }
}

// ---------------------------------------------------------------------------
// launchers
hipError_t launch_gather(const GatherArgs& g, hipStream_t s) {
    size_t total = (size_t(1) << g.n_mat) * (size_t)g.nb;
    unsigned blocks = (unsigned)((total + 255) / 256);
    if (blocks > 65536u) blocks = 65536u;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_gather_leaf, dim3(blocks), dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_permute(const PermArgs& a, hipStream_t s) {
    size_t tiles = size_t(1) << a.nn;
    size_t tile_elems = size_t(1) << a.nt;
    size_t lds = (tile_elems + (tile_elems >> 5)) * sizeof(float2);
    int threads = tile_elems >= 256 ? 256 : (int)((tile_elems + 63) / 64 * 64);
    hipLaunchKernelGGL(k_permute_tiled, dim3((unsigned)tiles, (unsigned)a.nb), dim3(threads), lds, s, a);
    return hipGetLastError();
}

int gemm_kind(const GemmArgs& g, int precision) {
    if (g.M >= 128 && g.N >= 128 && g.K >= 8) return 2;   // 128 x 128 tile
    if (g.M >= 64 && g.N >= 64 && g.K >= 8) return 1;     // 64 x 64 tile
    return 0;
}

hipError_t launch_gemm(const GemmArgs& g, int precision, hipStream_t s) {
    const int kind = gemm_kind(g, precision);
    const bool split = (precision == 2);
    const size_t batches = (size_t)g.nbatch * (size_t)g.nb;
    if (kind == 0) {
        size_t total = (size_t)g.M * g.N * batches;
        unsigned blocks = (unsigned)((total + 255) / 256);
        if (blocks > (1u << 20)) blocks = 1u << 20;
        if (blocks == 0) blocks = 1;
        hipLaunchKernelGGL(k_cgemm_small, dim3(blocks), dim3(256), 0, s, g);
    } else if (kind == 2) {
        size_t tiles = (size_t)((g.M + 127) / 128) * ((g.N + 127) / 128) * batches;
        if (split) hipLaunchKernelGGL((k_cgemm_split<2, 4>), dim3((unsigned)tiles), dim3(256), 0, s, g);
        else hipLaunchKernelGGL((k_cgemm_mfma<2, 4>), dim3((unsigned)tiles), dim3(256), 0, s, g);
    } else {
        size_t tiles = (size_t)((g.M + 63) / 64) * ((g.N + 63) / 64) * batches;
        if (split) hipLaunchKernelGGL((k_cgemm_split<1, 2>), dim3((unsigned)tiles), dim3(256), 0, s, g);
        else hipLaunchKernelGGL((k_cgemm_mfma<1, 2>), dim3((unsigned)tiles), dim3(256), 0, s, g);
    }
    return hipGetLastError();
}

hipError_t launch_zero_acc(double2* acc, int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_acc, dim3((nb + 255) / 256), dim3(256), 0, s, acc, nb);
    return hipGetLastError();
}

hipError_t launch_accumulate(double2* acc, const float2* v, int nb, int v_has_b, hipStream_t s) {
    hipLaunchKernelGGL(k_accumulate, dim3((nb + 255) / 256), dim3(256), 0, s, acc, v, nb, v_has_b);
    return hipGetLastError();
}

hipError_t launch_finalize(double2* acc, int nb, double sre, double sim, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3((nb + 255) / 256), dim3(256), 0, s, acc, nb, sre, sim);
    return hipGetLastError();
}
