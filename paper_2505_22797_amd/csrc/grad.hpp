// Kernels of the unrolled-iteration gradient: accumulator fills and the last
// step that scales the accumulated per-sample gradients by -tau and puts them
// back in time order.
#pragma once
#include "common.hpp"

namespace mpik {

template <typename T>
__global__ void k_fill(T* __restrict__ x, int64_t n, T v) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) x[i] = v;
}

// g_h[b] = -tau_b acc_h[b]; g_r[k(p)] = -tau_b acc_r[p], g_v likewise (the
// accumulators are in cell order, the outputs in time order).
template <typename T>
__global__ void k_vjp_finish(const Prob* __restrict__ P, const char* __restrict__ plan,
                             const T* __restrict__ acc_r, const T* __restrict__ acc_v, T* __restrict__ g_r,
                             T* __restrict__ g_v, const double* __restrict__ acc_h, double* __restrict__ g_h,
                             const double* __restrict__ taus) {
    const Prob& p = P[blockIdx.y];
    const double tau = taus[blockIdx.y];
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i == 0) g_h[blockIdx.y] = -tau * acc_h[blockIdx.y];
    if (i >= p.t) return;
    const int64_t k = at<int2>(plan, p.o_sidx)[i].y;
    const T t = T(-tau);
    const int64_t a = p.o_s + 2 * i, o = p.o_s + 2 * k;
    g_r[o] = t * acc_r[a];
    g_r[o + 1] = t * acc_r[a + 1];
    g_v[o] = t * acc_v[a];
    g_v[o + 1] = t * acc_v[a + 1];
}

}  // namespace mpik
