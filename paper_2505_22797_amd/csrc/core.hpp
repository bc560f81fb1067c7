// Kernels of the Core Stage (Section "MPI Core Stage", eq. first:step): the
// variational reconstruction of the symmetric core-operator field
// a = [A_xx, A_xy, A_yy] from (s_k, r_k, v_k) by conjugate gradients on the
// Euler-Lagrange equations
//     (1/L) I^T I a + gamma delta^2 W Delta Delta a = (1/L) I^T s,
// I the plan's sampling (the interpolation weights of the plan: bilinear or
// cosine) contracted with the velocity, W = diag(1, 2, 1) the Frobenius
// weights of the channels, Delta the 5-point graph Laplacian (in-grid
// neighbours, spacing delta = 2/N), L the number of samples.
//
// Fields are [3][N][N] per problem at element offset 3 o_c of the caller's
// concatenated buffer; signals in cell order at element offset o_s.  One step
// is five launches: the gather I p (per base-cell row), the Laplacian of p,
// the transpose sampling with the epilogue q = (1/L) I^T I p + gamma delta^2 W
// Delta (Delta p) and per-row partial sums of <p, q>, then the CG updates of
// the Deconvolution Stage with three components per cell.
//
// Precision: the sampling runs in the plan's dtype T on p rounded to T; the
// regulariser, q and the CG vectors are float64.  The biharmonic stencil
// cancels on smooth fields (its coefficients sum to 0 and reach 20 gamma /
// delta^2 per cell), so in float32 its rounding error would be a perturbation
// of the operator near eps_32 times its largest eigenvalue, which is
// comparable to the smallest eigenvalues that decide the step count.
#pragma once
#include "common.hpp"
#include "deconv.hpp"
#include "sampling.hpp"

namespace mpik {

constexpr int kCoreParts = 1024;       // partial sums of <p, q> per problem: one per grid row

// y = I a in cell order.  grid (base-cell rows, problems), 256 threads;
// dynamic LDS 6 N values (rows b and b+1 of the three channels).
template <typename T>
__global__ void __launch_bounds__(256) k_core_gather(const Prob* __restrict__ P, const T* __restrict__ a,
                                                     T* __restrict__ y, const char* __restrict__ plan,
                                                     const int* __restrict__ skip) {
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.y];
    if (skip && skip[blockIdx.y]) return;
    const int N = p.n, nb = p.nb, b = blockIdx.x;
    if (b >= nb) return;
    const int* binstart = at<int>(plan, p.o_binstart);
    const int p0 = binstart[b * nb], p1 = binstart[(b + 1) * nb];
    if (p0 == p1) return;
    const T* A = a + 3 * p.o_c;
    T* g0 = reinterpret_cast<T*>(smem);
    T* g1 = g0 + 3 * N;
    for (int i = threadIdx.x; i < 6 * N; i += blockDim.x) {
        const int half = i / (3 * N), rem = i % (3 * N), ch = rem / N, x = rem % N;
        g0[i] = A[int64_t(ch) * N * N + int64_t(b + half) * N + x];
    }
    __syncthreads();
    gather_band<T, 4>(g0, g1, N, p0, p1, at<vec4<T>>(plan, p.o_samp), at<int2>(plan, p.o_sidx), nullptr, nullptr,
                      y + p.o_s, nullptr, nullptr, nullptr, nullptr, p.t, nullptr, p.chan == 1, threadIdx.x,
                      blockDim.x);
}

// Graph Laplacian of one value of a [N][N] channel (in-grid neighbours only,
// without the 1/delta^2 factor).
template <typename T>
__device__ __forceinline__ T lap5(const T* __restrict__ c, int N, int j, int i) {
    const T v = c[int64_t(j) * N + i];
    T s = T(0);
    if (j > 0) s += c[int64_t(j - 1) * N + i] - v;
    if (j + 1 < N) s += c[int64_t(j + 1) * N + i] - v;
    if (i > 0) s += c[int64_t(j) * N + i - 1] - v;
    if (i + 1 < N) s += c[int64_t(j) * N + i + 1] - v;
    return s;
}

// l = Delta a without the 1/delta^2 factor, every channel, float64.  grid
// (ceil(3 N^2 / 256), problems), 256 threads.
__global__ void __launch_bounds__(256) k_core_lap(const Prob* __restrict__ P, const double* __restrict__ a,
                                                  double* __restrict__ l, const int* __restrict__ skip) {
    const Prob& p = P[blockIdx.y];
    if (skip && skip[blockIdx.y]) return;
    const int N = p.n;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x, nn = int64_t(N) * N;
    if (e >= 3 * nn) return;
    const int64_t ch = e / nn, rem = e % nn;
    const int j = int(rem / N), i = int(rem % N);
    const int64_t base = 3 * p.o_c + ch * nn;
    l[base + rem] = lap5(a + base, N, j, i);
}

// Grid row j of the three channels of (1/L) I^T y (cell-order y, sums in
// T), then, in float64,
//   EPI 0: out = that (the right-hand side);
//   EPI 1: out = that + gamma delta^2 W Delta l with l = Delta p (as
//          k_core_lap left it, unscaled: the two 1/delta^2 factors and
//          delta^2 make gamma / delta^2), and part[b][j] = the row's sum of
//          p * out.
// grid (max N, problems), 256 threads; dynamic LDS as the operator's
// row-wise transpose sampling.
template <typename T, int EPI>
__global__ void __launch_bounds__(256) k_core_scatter(const Prob* __restrict__ P, const T* __restrict__ y,
                                                      double* __restrict__ out, const double* __restrict__ pv,
                                                      const double* __restrict__ l, double gamma,
                                                      double* __restrict__ part, const char* __restrict__ plan,
                                                      const int* __restrict__ skip) {
    extern __shared__ __align__(16) char smem[];
    __shared__ double red[256];
    const Prob& p = P[blockIdx.y];
    if (skip && skip[blockIdx.y]) return;
    const int N = p.n, j = blockIdx.x;
    if (j >= N) return;
    T* g = reinterpret_cast<T*>(smem);
    char* sc = smem + lds_align(size_t(3) * N * sizeof(T));
    scatter_row<T, true, 256>(g, scatter_lds<T>(sc, N, 256), N, j, at<int>(plan, p.o_binstart),
                              at<vec4<T>>(plan, p.o_samp), at<int2>(plan, p.o_sidx),
                              reinterpret_cast<const vec2<T>*>(y + p.o_s), nullptr, threadIdx.x, p.chan == 1);
    const double inv_l = 1.0 / double(p.t);
    const int64_t nn = int64_t(N) * N;
    double* o = out + 3 * p.o_c;
    if (EPI == 0) {
        for (int i = threadIdx.x; i < 3 * N; i += blockDim.x) {
            const int ch = i / N, x = i % N;
            o[ch * nn + int64_t(j) * N + x] = inv_l * double(g[i]);
        }
        return;
    }
    const double d2 = 4.0 / (double(N) * N);                   // delta^2
    const double reg = gamma / d2;                               // gamma delta^2 / delta^4
    const double* pp = pv + 3 * p.o_c;
    const double* ll = l + 3 * p.o_c;
    double acc = 0.0;
    for (int i = threadIdx.x; i < 3 * N; i += blockDim.x) {
        const int ch = i / N, x = i % N;
        const double w = ch == 1 ? 2.0 : 1.0;
        const int64_t off = ch * nn + int64_t(j) * N + x;
        const double q = inv_l * double(g[i]) + reg * w * lap5(ll + ch * nn, N, j, x);
        o[off] = q;
        acc += pp[off] * q;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[int64_t(blockIdx.y) * kCoreParts + j] = red[0];
}

// y[o_s + 2i..] = s[o_s + 2k(i)..]: the caller's time-ordered signal in cell
// order.  grid (ceil(max T / 256), problems).
template <typename T>
__global__ void k_core_permute(const Prob* __restrict__ P, const T* __restrict__ s, T* __restrict__ y,
                               const char* __restrict__ plan) {
    const Prob& p = P[blockIdx.y];
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= p.t) return;
    const int64_t k = at<int2>(plan, p.o_sidx)[i].y;
    y[p.o_s + 2 * i] = s[p.o_s + 2 * k];
    y[p.o_s + 2 * i + 1] = s[p.o_s + 2 * k + 1];
}

// v_k = (r_{k+1} - r_k) / dt, the last sample repeating the previous
// difference (velocities by forward differences, Section "Experiment 2").
template <typename T>
__global__ void k_forward_difference(const T* __restrict__ r, T* __restrict__ v, int64_t n, double dt) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t a = (k + 1 < n) ? k : k - 1;     // n >= 2
    v[2 * k] = T((double(r[2 * a + 2]) - double(r[2 * a])) / dt);
    v[2 * k + 1] = T((double(r[2 * a + 3]) - double(r[2 * a + 1])) / dt);
}

// u = A_xx + A_yy for every problem (the trace image the Deconvolution Stage
// takes, eq. convolution:trace).  grid (ceil(N^2 / 256), problems).
template <typename T>
__global__ void k_field_trace(const Prob* __restrict__ P, const T* __restrict__ a, T* __restrict__ u) {
    const Prob& p = P[blockIdx.y];
    const int64_t nn = int64_t(p.n) * p.n, e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nn) return;
    const T* A = a + 3 * p.o_c;
    u[p.o_c + e] = A[e] + A[2 * nn + e];
}

}  // namespace mpik
