// Device-side reduction helpers shared by the kernels: wavefront (64-lane)
// shuffles and a 256-thread block sum.  Cross-block results are finished by a
// separate one-block kernel in a fixed summation order (deterministic from run
// to run); finishing inside the producing launch would need an agent-scope
// release fence per block, which on gfx950 writes back the XCD's whole L2.
#pragma once

#include "jfnk_internal.hpp"

namespace jfnk {

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Sums a[0..NV) over the 64 lanes of a wavefront by recursive halving: each
// exchange step hands half of the values held to the partner lane, so NV
// values cost NV - 1 + log2(64 / NV) shuffles instead of 6 NV.  On return the
// lane holds the wavefront total of value lane / (64 / NV).
template <int NV>
__device__ __forceinline__ double wave_sum_scatter(double (&a)[NV], int lane) {
    static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "NV must be a power of two up to 64");
    int d = 32;
#pragma unroll
    for (int K = NV; K > 1; K >>= 1, d >>= 1) {
        const int half = K >> 1;
        const bool up = (lane & d) != 0;
#pragma unroll
        for (int k = 0; k < half; ++k) {
            const double lo = a[k], hi = a[k + half];
            const double recv = __shfl_xor(up ? lo : hi, d, 64);
            a[k] = (up ? hi : lo) + recv;
        }
    }
    double s = a[0];
    for (; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
    return s;
}

// Sum of one value per thread of a 256-thread block; valid in thread 0.
__device__ __forceinline__ double block_sum256(double v, double* red4) {
    v = wave_sum64(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red4[wid] = v;
    __syncthreads();
    return threadIdx.x == 0 ? (red4[0] + red4[1]) + (red4[2] + red4[3]) : 0.0;
}

__device__ __forceinline__ int block_linear_id() { return blockIdx.y * gridDim.x + blockIdx.x; }
__device__ __forceinline__ int grid_blocks() { return gridDim.x * gridDim.y; }

// Fixed-order sum of partials[b * stride + k] over b < nblk by one block.  Each
// thread adds its partials b = tid, tid + 256, ... in ascending order; the
// loads are issued eight at a time before the adds (one at a time, each
// waits a full memory round trip, which is most of a finishing launch).
__device__ __forceinline__ double sum_partials(const double* partials, int nblk, int stride, int k, double* red4) {
    double acc = 0.0;
    for (int b0 = threadIdx.x; b0 < nblk; b0 += 8 * 256) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int b = b0 + u * 256;
            x[u] = b < nblk ? partials[(long long)b * stride + k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += x[u];
    }
    return block_sum256(acc, red4);
}

__device__ __forceinline__ void finish_eps(const EpsArgs& a, double vn2) {
    const double nv = sqrt(vn2);
    const double nu = sqrt(*a.unorm2);
    *a.vnorm2 = vn2;
    *a.eps = nv > 0.0 ? a.sqrt_eps * (nu > a.sqrt_n ? nu : a.sqrt_n) / nv : 0.0;
}

// Block contribution acc to ||v||^2 (finished by k_eps_finish).
__device__ __forceinline__ void partial_eps(const EpsArgs& a, double acc, double* red4) {
    const double s = block_sum256(acc, red4);
    if (threadIdx.x == 0) a.partials[block_linear_id()] = s;
}

}  // namespace jfnk
