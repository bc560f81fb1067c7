// Plan-build kernels: the float64 kernel table K_h(delta d) (eq. kernel:matrix
// with K_h(y) = K(y/h)/h), its spectra for the FFT path, the FFT twiddles and
// the sample-to-cell binning (base cell, bilinear fractions, stable sort by
// base cell).
#pragma once
#include "common.hpp"

namespace mpik {

// Taylor coefficients of L(z) = coth z - 1/z = sum_{n>=1} b_n z^(2n-1).
// f(z) = z coth z = 1 + sum b_n z^(2n) solves z f' = f - f^2 + z^2, which gives
// (2n+1) b_n = [n == 1] - sum_{k=1}^{n-1} b_k b_{n-k}.  Filled once per build.
constexpr int kSeriesTerms = 24;
constexpr double kSeriesCut = 1.0;   // |z| below: series (radius of convergence pi)

__device__ __forceinline__ void langevin_all(double z, const double* __restrict__ b,
                                             double& L, double& L1, double& L2) {
    // z >= 0 in every use here (a distance over h)
    if (z < kSeriesCut) {
        const double z2 = z * z;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        // Horner in z^2 from the highest term
        for (int n = kSeriesTerms; n >= 1; --n) {
            const double p = 2.0 * n - 1.0;
            s0 = s0 * z2 + b[n - 1];
            s1 = s1 * z2 + b[n - 1] * p;
            if (n >= 2) s2 = s2 * z2 + b[n - 1] * p * (p - 1.0);
        }
        L = s0 * z;         // sum_{n>=1} b_n z^(2n-1)
        L1 = s1;            // sum_{n>=1} b_n (2n-1) z^(2n-2)
        L2 = s2 * z;        // sum_{n>=2} b_n (2n-1)(2n-2) z^(2n-3)
    } else {
        const double u = exp(-2.0 * z);           // e^{-2z}
        const double om = -expm1(-2.0 * z);       // 1 - e^{-2z}
        const double iz = 1.0 / z;
        L = (1.0 + u) / om - iz;                  // coth z - 1/z
        L1 = iz * iz - 4.0 * u / (om * om);       // 1/z^2 - 1/sinh^2 z
        L2 = 8.0 * u * (1.0 + u) / (om * om * om) - 2.0 * iz * iz * iz;   // 2 cosh/sinh^3 - 2/z^3
    }
}

// One thread, the coefficients held in registers (the recurrence reads every
// earlier one) and stored at the end.  The leading 1 comes from the thread
// index, so that the recurrence runs on the device, with its fused
// multiply-adds, rather than being folded at compile time with other
// roundings.
__global__ void k_series(double* __restrict__ b) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double one = double(1 - int(threadIdx.x));
        double c[kSeriesTerms];
#pragma unroll
        for (int n = 1; n <= kSeriesTerms; ++n) {
            double acc = (n == 1) ? one : 0.0;
#pragma unroll
            for (int k = 1; k < n; ++k) acc -= c[k - 1] * c[n - k - 1];
            c[n - 1] = acc / (2.0 * n + 1.0);
        }
#pragma unroll
        for (int n = 0; n < kSeriesTerms; ++n) b[n] = c[n];
    }
}

// Kernel table in float64, [3][2R+1][2R+1] indexed [ch][dy+R][dx+R], and the
// delta^2-scaled copy for the direct path in the compute type, reversed in x
// (taps[ch][dy+R][t] = delta^2 K_ch(R - t, dy)) with rows zero-padded to taps_w.
// With q = dx^2 + dy^2 and r = delta sqrt(q) / h:
//   K_xx = (L'(r) dx^2 + L(r)/r dy^2) / (q h),  K_xy = (L'(r) - L(r)/r) dx dy / (q h),
//   K_yy = (L'(r) dy^2 + L(r)/r dx^2) / (q h),  K(0) = I / (3h).
// With `deriv` the table holds dK_h/dh instead:
//   -h^-2 [(L' + r L'') P + L' (I - P)],  -I/(3h^2) at 0.
template <typename T>
__global__ void k_table(const Prob* __restrict__ P, char* __restrict__ plan, const double* __restrict__ series,
                        double* __restrict__ tab64, T* __restrict__ taps, int deriv) {
    const Prob& p = *P;
    const int R = p.radius, W = 2 * R + 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= W * W) return;
    const int dy = idx / W - R, dx = idx % W - R;
    const double h = p.h, delta = 2.0 / p.n;
    // the kernel at G y (selection-field gradient G = diag(gx, gy); exact for G = I)
    const double ex = p.gx * dx, ey = p.gy * dy;
    const double q = ex * ex + ey * ey;
    double kxx, kxy, kyy;
    if (q == 0.0) {
        kxx = kyy = deriv ? -1.0 / (3.0 * h * h) : 1.0 / (3.0 * h);
        kxy = 0.0;
    } else {
        const double r = delta * sqrt(q) / h;
        double L, L1, L2;
        langevin_all(r, series, L, L1, L2);
        double a, b, s;
        if (!deriv) { a = L1; b = L / r; s = 1.0 / (q * h); }
        else { a = L1 + r * L2; b = L1; s = -1.0 / (q * h * h); }
        kxx = (a * ex * ex + b * ey * ey) * s;
        kxy = (a - b) * ex * ey * s;
        kyy = (a * ey * ey + b * ex * ex) * s;
    }
    const int plane = W * W;
    if (tab64) {
        tab64[idx] = kxx;
        tab64[plane + idx] = kxy;
        tab64[2 * plane + idx] = kyy;
    }
    if (taps) {
        const double d2 = delta * delta;
        const int tw = p.taps_w;
        const int o = (dy + R) * tw + (R - dx);
        taps[o] = T(d2 * kxx);
        taps[W * tw + o] = T(d2 * kxy);
        taps[2 * W * tw + o] = T(d2 * kyy);
    }
}

// Zero the padding columns of the direct-path tap rows.
template <typename T>
__global__ void k_taps_pad(const Prob* __restrict__ P, T* __restrict__ taps) {
    const Prob& p = *P;
    const int W = 2 * p.radius + 1, tw = p.taps_w;
    const int pad = tw - W;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 3 * W * pad) return;
    const int row = idx / pad, col = W + idx % pad;
    taps[row * tw + col] = T(0);
}

// cos / sin of 2 pi m / M in float64 and the twiddles e^{-2 pi i m/M}.
template <typename T>
__global__ void k_trig(const Prob* __restrict__ P, double* __restrict__ cs, cx<T>* __restrict__ tw) {
    const int M = P->m;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    double s, c;
    sincospi(2.0 * m / M, &s, &c);
    cs[2 * m] = c;
    cs[2 * m + 1] = s;
    tw[m] = cx<T>{T(c), T(-s)};
}

// Spectra of the circularly embedded table on the M x M grid.  Every channel
// has a real spectrum: K_xx, K_yy are even in each axis, K_xy odd in each:
//   xx, yy:  S(kx, ky) =  sum_{dx,dy} K cos(2 pi kx dx/M) cos(2 pi ky dy/M)
//   xy:      S(kx, ky) = -sum_{dx,dy} K sin(2 pi kx dx/M) sin(2 pi ky dy/M)
// computed separably in float64 over the half ranges; stored for
// kx, ky in [0, M/2] as [ch][kx][ky], scaled by delta^2 / M^2 (the Riemann
// weight and the inverse-FFT normalisation).
// Pass 1: U[ch][dy][kx] for dy in [0, R].
__global__ void k_spec_rows(const Prob* __restrict__ P, const double* __restrict__ tab64,
                            const double* __restrict__ cs, double* __restrict__ U) {
    const Prob& p = *P;
    const int R = p.radius, W = 2 * R + 1, M = p.m, H = M / 2 + 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 3 * (R + 1) * H) return;
    const int ch = idx / ((R + 1) * H);
    const int rem = idx % ((R + 1) * H);
    const int dy = rem / H, kx = rem % H;
    const double* row = tab64 + ch * W * W + (dy + R) * W + R;   // row[dx], dx in [-R, R]
    double acc;
    if (ch != 1) {
        acc = row[0];
        for (int dx = 1; dx <= R; ++dx) acc += 2.0 * row[dx] * cs[2 * ((kx * dx) & (M - 1))];
    } else {
        acc = 0.0;
        for (int dx = 1; dx <= R; ++dx) acc += 2.0 * row[dx] * cs[2 * ((kx * dx) & (M - 1)) + 1];
    }
    U[idx] = acc;
}

template <typename T>
__global__ void k_spec_cols(const Prob* __restrict__ P, const double* __restrict__ U,
                            const double* __restrict__ cs, T* __restrict__ spec) {
    const Prob& p = *P;
    const int R = p.radius, M = p.m, H = M / 2 + 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 3 * H * H) return;
    const int ch = idx / (H * H);
    const int rem = idx % (H * H);
    const int kx = rem / H, ky = rem % H;
    const double* u = U + ch * (R + 1) * H + kx;   // u[dy * H]
    double acc;
    if (ch != 1) {
        acc = u[0];
        for (int dy = 1; dy <= R; ++dy) acc += 2.0 * u[dy * H] * cs[2 * ((ky * dy) & (M - 1))];
    } else {
        acc = 0.0;
        for (int dy = 1; dy <= R; ++dy) acc -= 2.0 * u[dy * H] * cs[2 * ((ky * dy) & (M - 1)) + 1];
    }
    const double delta = 2.0 / p.n;
    spec[idx] = T(acc * delta * delta / (double(M) * double(M)));
}

// ---------------------------------------------------------------------------
// Binning.  g = (x + 1)/delta - 1/2 in float64; a sample needs 0 <= g <= N-1
// on both axes (else the error flag is raised); i0 = min(floor g, N-2),
// fraction g - i0 in [0, 1].
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_bin_prep(const Prob* __restrict__ P, const T* __restrict__ r, int* __restrict__ cell,
                           double* __restrict__ frac, int* __restrict__ bincount, int* __restrict__ err) {
    const Prob& p = *P;
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= p.t) return;
    const int n = p.n;
    const double delta = 2.0 / n;
    const double gx = (double(r[2 * k]) + 1.0) / delta - 0.5;
    const double gy = (double(r[2 * k + 1]) + 1.0) / delta - 0.5;
    const bool ok = (gx >= 0.0) && (gx <= double(n - 1)) && (gy >= 0.0) && (gy <= double(n - 1));
    if (!ok) {
        err[0] = 1;
        cell[k] = -1;
        return;
    }
    const int i0 = min(int(floor(gx)), n - 2);
    const int j0 = min(int(floor(gy)), n - 2);
    cell[k] = j0 * (n - 1) + i0;
    frac[2 * k] = gx - i0;
    frac[2 * k + 1] = gy - j0;
    atomicAdd(&bincount[j0 * (n - 1) + i0], 1);
}

// Exclusive scan of `count` ints by one work-group of 1024 threads, in tiles
// of 4096 entries (four consecutive entries per thread, wave scans through
// lane shuffles, a running carry between tiles); out has count + 1 entries,
// out[count] being the total.
constexpr int kScanThreads = 1024;
// In place (in == out) is allowed: a tile is read completely before it is written.
__global__ void __launch_bounds__(kScanThreads) k_scan(const int* in, int* out, int64_t count) {
    __shared__ int wsum[kScanThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    constexpr int kWaves = kScanThreads / 64;
    int carry = 0;
    for (int64_t base = 0; base < count; base += 4 * kScanThreads) {
        int v[4];
        int sum = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t idx = base + 4 * tid + j;
            v[j] = idx < count ? in[idx] : 0;
            sum += v[j];
        }
        int x = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[w] = x;
        __syncthreads();
        if (w == 0) {
            int t = lane < kWaves ? wsum[lane] : 0;
#pragma unroll
            for (int off = 1; off < kWaves; off <<= 1) {
                const int y = __shfl_up(t, off, 64);
                if (lane >= off) t += y;
            }
            if (lane < kWaves) wsum[lane] = t;
        }
        __syncthreads();
        int run = carry + (w > 0 ? wsum[w - 1] : 0) + x - sum;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t idx = base + 4 * tid + j;
            if (idx < count) out[idx] = run;
            run += v[j];
        }
        carry += wsum[kWaves - 1];
        __syncthreads();    // wsum is rewritten by the next tile
    }
    if (tid == 0) out[count] = carry;
}

// Stable sort of the samples by base cell: a least-significant-digit radix
// sort over 8-bit digits of the cell index.  Per pass: digit histograms of
// tiles of 2048 consecutive entries (k_sort_hist) into a digit-major table,
// an exclusive scan of that table (k_scan), and a stable scatter (k_sort_pass)
// that ranks every entry among the entries of its tile with the same digit
// (earlier rounds, earlier waves, earlier lanes), the wave-local rank from
// eight ballots.  Every position is an integer function of the input, so the
// order is the same on every run: by cell, and by time inside a cell.
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortThreads * kSortRounds;

__global__ void __launch_bounds__(kSortThreads) k_sort_hist(const int* __restrict__ keys, int64_t t, int shift,
                                                            int* __restrict__ table, int tiles) {
    __shared__ int hist[256];
    const int tid = threadIdx.x;
    hist[tid] = 0;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t idx = base + r * kSortThreads + tid;
        if (idx < t) atomicAdd(&hist[(unsigned(keys[idx]) >> shift) & 255u], 1);
    }
    __syncthreads();
    table[int64_t(tid) * tiles + blockIdx.x] = hist[tid];
}

// vals_in == nullptr: the values are the input positions (the time index);
// keys_out == nullptr: only the values are written (the last pass).
__global__ void __launch_bounds__(kSortThreads) k_sort_pass(const int* __restrict__ keys_in,
                                                            const int* __restrict__ vals_in,
                                                            int* __restrict__ keys_out, int* __restrict__ vals_out,
                                                            int64_t t, int shift, const int* __restrict__ offs,
                                                            int tiles) {
    __shared__ int run[256];
    __shared__ int wcnt[kSortThreads / 64][256];
    constexpr int kWaves = kSortThreads / 64;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    run[tid] = offs[int64_t(tid) * tiles + blockIdx.x];
    const uint64_t lt = (uint64_t(1) << lane) - 1;
    const int64_t base = int64_t(blockIdx.x) * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t idx = base + r * kSortThreads + tid;
        const bool valid = idx < t;
        const int key = valid ? keys_in[idx] : 0;
        const int val = valid ? (vals_in ? vals_in[idx] : int(idx)) : 0;
        const unsigned d = (unsigned(key) >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
#pragma unroll
        for (int q = 0; q < kWaves; ++q) wcnt[q][tid] = 0;
        __syncthreads();
        const int rank = __popcll(peers & lt);
        if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int pos = run[d] + rank;
            for (int q = 0; q < w; ++q) pos += wcnt[q][d];
            if (keys_out) keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        int add = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) add += wcnt[q][tid];
        run[tid] += add;
        __syncthreads();
    }
}

// Writes the sorted sample records: position i holds sample k = order[i].
// The records carry the per-axis weight of the upper neighbour: the fraction
// f itself (bilinear) or (1 - cos pi f)/2 (cosine), evaluated in float64; the
// derivative tables get d w/d f = (pi/2) sin pi f.
template <typename T>
__global__ void k_place(const Prob* __restrict__ P, const int* __restrict__ order, const int* __restrict__ cell,
                        const double* __restrict__ frac, const T* __restrict__ v, char* __restrict__ plan) {
    const Prob& p = *P;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= p.t) return;
    const int k = order[i];
    const Chk ck = chk_of(p, plan);
    if (!ck.time(k)) return;
    const int q = cell[k];
    if (q < 0) return;        // outside the hull: the build reports the error
    const int nb = p.nb;
    if (!ck.ok(q < nb * nb, kChkCell)) return;
    at<int2>(plan, p.o_sidx)[i] = make_int2((q % nb) | ((q / nb) << 16), k);
    const double fx = frac[2 * k], fy = frac[2 * k + 1];
    vec4<T> e;
    vec2<T> d;
    if (p.interp == 1) {
        constexpr double kPi = 3.14159265358979323846;
        e.x = T(0.5 * (1.0 - cos(kPi * fx)));
        e.y = T(0.5 * (1.0 - cos(kPi * fy)));
        d.x = T(0.5 * kPi * sin(kPi * fx));
        d.y = T(0.5 * kPi * sin(kPi * fy));
    } else {
        e.x = T(fx);
        e.y = T(fy);
        d.x = T(1);
        d.y = T(1);
    }
    if (p.o_dw) at<vec2<T>>(plan, p.o_dw)[i] = d;
    e.z = v[2 * k];
    e.w = v[2 * k + 1];
    at<vec4<T>>(plan, p.o_samp)[i] = e;
}

// Copies one problem's sorted (base cell, time index) pairs out of the plan.
__global__ void k_sample_order(const Prob* __restrict__ P, const char* __restrict__ plan, int* __restrict__ order,
                               int* __restrict__ cell) {
    const Prob& p = *P;
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= p.t) return;
    const int2 e = at<int2>(plan, p.o_sidx)[i];
    order[i] = e.y;
    cell[i] = e.x;
}

}  // namespace mpik
