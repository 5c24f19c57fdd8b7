// HIP kernels of the amplitude engine for gfx950 (MI355X).
//
//  k_gather_leaf    leaf -> operand: output labels replaced by the
//                   bitstring's bits (gives the batch index b), sliced labels
//                   by the slice's bits, remaining labels in gathered order
//  k_permute_tiled  bit permutation of a tensor's address, staged through LDS
//                   so that reads run along the lowest input bits and writes
//                   along the lowest output bits
//  k_accumulate     FP64 slice sums;  k_finalize  scale and write out
// (the complex GEMMs are in gemm.hip)
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include "kernels.h"


// ---------------------------------------------------------------------------
__global__ void k_gather_leaf(GatherArgs g) {
    const size_t per = size_t(1) << g.n_mat;
    const size_t total = per * (size_t)g.nb * (size_t)g.nr;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t outer = idx >> g.n_mat;
        const size_t b = outer % g.nb;
        // low slice bits of this copy: deposit the copy index into dmask
        uint32_t c = (uint32_t)(outer / g.nb), slice = g.slice;
        for (uint32_t m = g.dmask; m; m &= m - 1) {
            if (c & 1) slice |= m & (~m + 1);
            c >>= 1;
        }
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
            if ((slice >> g.sl_bit[i]) & 1) src |= size_t(1) << g.sl_src[i];
        g.dst[idx] = g.src[src];
    }
}

// ---------------------------------------------------------------------------
// One workgroup per tile: the tile holds every combination of the tile bits
// T (the lowest input bits plus the input bits that become the lowest output
// bits) for fixed values of all other bits and of b.  Tile bit 0 is input bit
// 0 and, in output order, output bit 0, so elements move in adjacent pairs:
// 16-byte reads along the lowest input bits, 16-byte writes along the lowest
// output bits.  Tile bits 1..8 (input order for the reads, output order for
// the writes) are the thread id, deposited once per thread.  The LDS index
// keeps bit 0 and XORs bits 5..8 into bits 1..4, so the strided reads of the
// write phase spread over the banks.
__device__ __forceinline__ unsigned swz(unsigned e) { return e ^ (((e >> 5) & 15u) << 1); }

__global__ void __launch_bounds__(256) k_permute_tiled(PermArgs a) {
    extern __shared__ float2 lds[];
    const int t = a.nt;
    const size_t r_elems = size_t(1) << a.rank;
    const size_t tid_blk = blockIdx.x;
    const size_t b = blockIdx.y;
    size_t base_in = 0, base_out = 0;
    for (int m = 0; m < a.nn; ++m)
        if ((tid_blk >> m) & 1) {
            base_in |= size_t(1) << a.n_in[m];
            base_out |= size_t(1) << a.n_out[m];
        }
    const float2* src = a.src + b * r_elems + base_in;
    float2* dst = a.dst + b * r_elems + base_out;
    const unsigned th = threadIdx.x;
    if (t == 0) {
        if (th == 0) dst[0] = src[0];
        return;
    }
    const int tp = t - 1;                         // pair-index bits
    const int tl = tp < 8 ? tp : 8;               // carried by the thread id
    const unsigned iters = 1u << (tp - tl);
    if (th >= (1u << tl)) {
        __syncthreads();
        return;
    }
    size_t in_lo = 0, out_lo = 0;
    unsigned e_lo = 0;
    for (int m = 0; m < tl; ++m)
        if ((th >> m) & 1) {
            in_lo |= size_t(1) << a.t_in[m + 1];
            out_lo |= size_t(1) << a.t_out[m + 1];
            e_lo |= 1u << a.t_rank[m + 1];
        }
    const unsigned e_bit0 = 1u << a.t_rank[0];    // input tile index of output bit 0
    if (tp - tl <= 3) {
        // tiles of at most 2^12 elements (the size the host picks): a
        // thread's at most 8 pairs have their high index bits in three
        // masks, all 8 reads are issued before the first LDS write, and the
        // reads and writes beyond the tile (pair index >= iters) repeat pair
        // 0 into LDS rows past the tile (the LDS holds 2^12 elements)
        size_t hin[3] = {0, 0, 0}, hout[3] = {0, 0, 0};
        unsigned he[3] = {0, 0, 0};
        for (int j = 0; j < tp - tl; ++j) {
            hin[j] = size_t(1) << a.t_in[tl + 1 + j];
            hout[j] = size_t(1) << a.t_out[tl + 1 + j];
            he[j] = 1u << a.t_rank[tl + 1 + j];
        }
        float4 v[8];
#pragma unroll
        for (unsigned k = 0; k < 8; ++k) {
            const unsigned kk = k < iters ? k : 0u;
            const size_t off = in_lo | ((kk & 1) ? hin[0] : 0) | ((kk & 2) ? hin[1] : 0) |
                               ((kk & 4) ? hin[2] : 0);
            v[k] = *reinterpret_cast<const float4*>(src + off);
        }
#pragma unroll
        for (unsigned k = 0; k < 8; ++k)
            *reinterpret_cast<float4*>(&lds[swz((((k << tl) | th) << 1))]) = v[k];
        __syncthreads();
#pragma unroll
        for (unsigned k = 0; k < 8; ++k) {
            if (k >= iters) break;
            const size_t off = out_lo | ((k & 1) ? hout[0] : 0) | ((k & 2) ? hout[1] : 0) |
                               ((k & 4) ? hout[2] : 0);
            const unsigned e = e_lo | ((k & 1) ? he[0] : 0) | ((k & 2) ? he[1] : 0) | ((k & 4) ? he[2] : 0);
            const float2 x = lds[swz(e)], y = lds[swz(e | e_bit0)];
            *reinterpret_cast<float4*>(dst + off) = make_float4(x.x, x.y, y.x, y.y);
        }
        return;
    }
    for (unsigned k = 0; k < iters; ++k) {
        size_t off = in_lo;
        for (int m = tl; m < tp; ++m)
            if ((k >> (m - tl)) & 1) off |= size_t(1) << a.t_in[m + 1];
        const float4 v = *reinterpret_cast<const float4*>(src + off);
        *reinterpret_cast<float4*>(&lds[swz((((k << tl) | th) << 1))]) = v;
    }
    __syncthreads();
    for (unsigned k = 0; k < iters; ++k) {
        size_t off = out_lo;
        unsigned e = e_lo;
        for (int m = tl; m < tp; ++m)
            if ((k >> (m - tl)) & 1) {
                off |= size_t(1) << a.t_out[m + 1];
                e |= 1u << a.t_rank[m + 1];
            }
        const float2 x = lds[swz(e)], y = lds[swz(e | e_bit0)];
        *reinterpret_cast<float4*>(dst + off) = make_float4(x.x, x.y, y.x, y.y);
    }
}

// ---------------------------------------------------------------------------
__global__ void k_zero_acc(double2* acc, int nb) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) acc[b] = make_double2(0.0, 0.0);
}

__global__ void k_accumulate(double2* acc, const float2* v, int nb, int v_has_b, int nr,
                             long long vr) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) {
        double2 a = acc[b];
        for (int r = 0; r < nr; ++r) {          // ascending slice order
            const float2 x = v[(size_t)r * vr + (v_has_b ? b : 0)];
            a.x += (double)x.x;
            a.y += (double)x.y;
        }
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
    size_t total = (size_t(1) << g.n_mat) * (size_t)g.nb * (size_t)g.nr;
    unsigned blocks = (unsigned)((total + 255) / 256);
    if (blocks > 65536u) blocks = 65536u;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_gather_leaf, dim3(blocks), dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_permute(const PermArgs& a, hipStream_t s) {
    size_t tiles = size_t(1) << a.nn;
    size_t tile_elems = size_t(1) << a.nt;
    // the swizzle moves an index within its 1024-element block; tiles up to
    // 2^12 elements get the whole 2^12 (their eight-pair path writes past a
    // smaller tile)
    size_t lds = (tile_elems < 4096 ? 4096 : tile_elems) * sizeof(float2);
    int threads = tile_elems >= 512 ? 256 : (int)((tile_elems / 2 + 63) / 64 * 64);
    if (threads < 64) threads = 64;
    hipLaunchKernelGGL(k_permute_tiled, dim3((unsigned)tiles, (unsigned)a.nb), dim3(threads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_zero_acc(double2* acc, int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_acc, dim3((nb + 255) / 256), dim3(256), 0, s, acc, nb);
    return hipGetLastError();
}

hipError_t launch_accumulate(double2* acc, const float2* v, int nb, int v_has_b, int nr,
                             long long vr, hipStream_t s) {
    hipLaunchKernelGGL(k_accumulate, dim3((nb + 255) / 256), dim3(256), 0, s, acc, v, nb, v_has_b,
                       nr, vr);
    return hipGetLastError();
}

hipError_t launch_finalize(double2* acc, int nb, double sre, double sim, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3((nb + 255) / 256), dim3(256), 0, s, acc, nb, sre, sim);
    return hipGetLastError();
}
