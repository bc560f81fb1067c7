// Kernels of the unrolled-iteration gradient: accumulator fills and the last
// step that scales the accumulated per-sample gradients by -tau and puts them
// back in time order; the trajectory of given unit shapes scaled by its
// amplitudes, and the reduction of per-sample gradients to the amplitudes'.
#pragma once
#include "common.hpp"
#include "direct.hpp"

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
    if (!chk_of(p, plan).time(k)) return;
    const T t = T(-tau);
    const int64_t a = p.o_s + 2 * i, o = p.o_s + 2 * k;
    g_r[o] = t * acc_r[a];
    g_r[o + 1] = t * acc_r[a + 1];
    g_v[o] = t * acc_v[a];
    g_v[o + 1] = t * acc_v[a + 1];
}

// Trajectory of amplitudes (ax, ay) over unit-amplitude shapes: r_k =
// (ax rho_k,x, ay rho_k,y), v_k = (ax nu_k,x, ay nu_k,y) -- the Lissajous
// figure of eq. (lissajous) with its amplitudes as the parameters.  Each
// product is formed in float64 and rounded once.  [n][2] arrays.
template <typename T>
__global__ void k_scale_traj(const T* __restrict__ rho, const T* __restrict__ nu, int64_t n, double ax, double ay,
                             T* __restrict__ r, T* __restrict__ v) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    r[2 * k] = T(ax * double(rho[2 * k]));
    r[2 * k + 1] = T(ay * double(rho[2 * k + 1]));
    v[2 * k] = T(ax * double(nu[2 * k]));
    v[2 * k + 1] = T(ay * double(nu[2 * k + 1]));
}

// Chain rule to the amplitudes: with g_r = dL/dr_k and g_v = dL/dv_k per
// sample (time order, [T][2]),
//   dL/dax = sum_k g_r,k,x rho_k,x + g_v,k,x nu_k,x,  dL/day likewise with y,
// in float64 by a fixed order: part q of problem b sums a fixed contiguous
// slice of its samples (thread-strided inside the slice, then a fixed tree)
// into part[(b kDotParts + q) 2 + comp]; k_amp_final adds each problem's
// parts by a fixed tree.
template <typename T>
__global__ void __launch_bounds__(256) k_amp_part(const Prob* __restrict__ P, const T* __restrict__ g_r,
                                                  const T* __restrict__ g_v, const T* __restrict__ rho,
                                                  const T* __restrict__ nu, double* __restrict__ part) {
    __shared__ double red[2][256];
    const Prob& p = P[blockIdx.y];
    const int tid = threadIdx.x;
    const int64_t m = p.t;
    const int64_t per = (m + kDotParts - 1) / kDotParts;
    const int64_t lo = min(m, per * blockIdx.x), hi = min(m, lo + per);
    double ax = 0.0, ay = 0.0;
    for (int64_t k = lo + tid; k < hi; k += 256) {
        const int64_t i = p.o_s + 2 * k;
        ax += double(g_r[i]) * double(rho[i]) + double(g_v[i]) * double(nu[i]);
        ay += double(g_r[i + 1]) * double(rho[i + 1]) + double(g_v[i + 1]) * double(nu[i + 1]);
    }
    red[0][tid] = ax;
    red[1][tid] = ay;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            red[0][tid] += red[0][tid + w];
            red[1][tid] += red[1][tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const int64_t o = (int64_t(blockIdx.y) * kDotParts + blockIdx.x) * 2;
        part[o] = red[0][0];
        part[o + 1] = red[1][0];
    }
}

__global__ void __launch_bounds__(kDotParts) k_amp_final(const double* __restrict__ part, double* __restrict__ g_ax,
                                                        double* __restrict__ g_ay) {
    __shared__ double red[2][kDotParts];
    const int tid = threadIdx.x;
    const int64_t o = (int64_t(blockIdx.x) * kDotParts + tid) * 2;
    red[0][tid] = part[o];
    red[1][tid] = part[o + 1];
    __syncthreads();
    for (int w = kDotParts / 2; w > 0; w >>= 1) {
        if (tid < w) {
            red[0][tid] += red[0][tid + w];
            red[1][tid] += red[1][tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        g_ax[blockIdx.x] = red[0][0];
        g_ay[blockIdx.x] = red[1][0];
    }
}

}  // namespace mpik
