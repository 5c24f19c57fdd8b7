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
    size_t lds = (tile_elems + (tile_elems >> 5)) * sizeof(float2);
    int threads = tile_elems >= 256 ? 256 : (int)((tile_elems + 63) / 64 * 64);
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
