// Kernels of the Deconvolution Stage (Section "Deconvolution Stage"): the
// batched conjugate-gradient solver of the Tikhonov sub-step (eq. dec:sub:tik)
// on its normal equations (C^T C + nu I) x = b, the percentile trimming
// (Section "Denoiser Artifact Reduction") and the noise estimate
// sigma = sqrt(Var) that drives the ZeroShot-PnP schedule.
//
// Mixed precision: the Krylov vectors x, r, p are float64 whatever the
// operator's dtype T; the operator is applied to pt, p rounded to T (written
// next to p), and returns q in T.  In float32 this keeps the recursively
// updated residual close to the true one over thousands of steps (with
// float32 vectors it drifts above the tolerance in long solves).
//
// Every problem of a batch runs its own CG; the scalars live in device memory
// and every kernel of a step skips problems whose flag done[b] is set, so the
// host only polls the flags from time to time.  The residual norm and the flag
// are double-buffered by the parity of the step: step i reads slot i & 1 and
// its last kernel writes slot (i + 1) & 1, so no kernel writes what another
// work-group of the same launch still reads.  All sums are float64 in a fixed
// order: per problem, fixed partial sums (kDotParts contiguous slices, or one
// per row pair where the FFT row stage forms them) added one after another by
// every work-group that needs the total, so all of them see the same value.
#pragma once
#include <type_traits>

#include "common.hpp"
#include "direct.hpp"
#include "fft_conv.hpp"

namespace mpik {

// per-problem solver state, arrays of `count` entries each (rr and done: two
// slots of `count`, by step parity)
struct CgState {
    double* rr;     // |r|^2 of the current residual
    double* bb;     // |b|^2
    double* nu;     // Tikhonov weight of the problem
    int* iters;     // steps taken
    int* done;      // 1 once |r| <= tol |b| or iters == max_iter
};

__device__ __forceinline__ double sum_parts(const double* __restrict__ part, int n = kDotParts) {
    double s = 0.0;
    for (int q = 0; q < n; ++q) s += part[q];
    return s;
}

// Partial sums of <p, q> per problem (`stride` slots): the FFT row stage
// fills one per row pair, the direct path's k_cg_pq the first kDotParts.
__device__ __forceinline__ int pq_parts(const Prob& p) { return p.mode == 1 ? (p.n + 1) / 2 : kDotParts; }

// The work-group's slice [lo, hi) of a problem with m elements.
__device__ __forceinline__ void slice_of(int64_t m, int64_t& lo, int64_t& hi) {
    const int64_t per = (m + kDotParts - 1) / kDotParts;
    lo = min(m, per * int64_t(blockIdx.x));
    hi = min(m, lo + per);
}

// Fixed tree over the 256 threads' values; thread 0 writes part[b][slice]
// (`stride` slots per problem).
__device__ __forceinline__ void reduce_to_part(double v, double* red, double* __restrict__ part,
                                               int stride = kDotParts) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) part[int64_t(blockIdx.y) * stride + blockIdx.x] = red[0];
}

// Shares one float64 value computed by thread 0 with the work-group.
__device__ __forceinline__ double broadcast0(double v, double* slot) {
    if (threadIdx.x == 0) *slot = v;
    __syncthreads();
    return *slot;
}

// ------------------------------------------------------------------ CG ---
// The CG vectors hold `comps` values per grid cell (1: concentrations, 3:
// the Core Stage's field), at element offset comps * o_c.
//
// grid (kDotParts, problems), 256 threads.  b = cu + nu rho2 in float64
// (rho2 may be null: b = cu); x = 0, r = p = b, pt = b rounded to T;
// part = slices of |b|^2.
template <typename T>
__global__ void __launch_bounds__(256) k_cg_init(const Prob* __restrict__ P, int comps, const T* __restrict__ cu,
                                                 const T* __restrict__ rho2, CgState s, double* __restrict__ x,
                                                 double* __restrict__ r, double* __restrict__ pv, T* __restrict__ pt,
                                                 double* __restrict__ part) {
    __shared__ double red[256];
    const Prob& p = P[blockIdx.y];
    const int64_t m = int64_t(comps) * p.n * p.n, o = int64_t(comps) * p.o_c;
    int64_t lo, hi;
    slice_of(m, lo, hi);
    const double nu = rho2 ? s.nu[blockIdx.y] : 0.0;
    double acc = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += 256) {
        const double b = rho2 ? double(cu[o + e]) + nu * double(rho2[o + e]) : double(cu[o + e]);
        x[o + e] = 0.0;
        r[o + e] = b;
        pv[o + e] = b;
        pt[o + e] = T(b);
        acc += b * b;
    }
    reduce_to_part(acc, red, part);
}

// out = x rounded to T (the solver's result in the caller's dtype).
template <typename T>
__global__ void __launch_bounds__(256) k_cg_store(const Prob* __restrict__ P, int comps,
                                                  const double* __restrict__ x, T* __restrict__ out) {
    const Prob& p = P[blockIdx.y];
    const int64_t m = int64_t(comps) * p.n * p.n, o = int64_t(comps) * p.o_c;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < m; e += int64_t(gridDim.x) * blockDim.x)
        out[o + e] = T(x[o + e]);
}

// one thread per problem: rr = bb = |b|^2, no step taken yet (slot 0).
__global__ void k_cg_begin(int count, CgState s, const double* __restrict__ part, double tol, int max_iter) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    const double rr = sum_parts(part + int64_t(b) * kDotParts);
    s.rr[b] = rr;
    s.bb[b] = rr;
    s.iters[b] = 0;
    s.done[b] = (0 < max_iter && rr > tol * tol * rr) ? 0 : 1;
}

// Direct-path problems: q <- q + nu pt (q holds C^T C pt); part = slices of
// <pt, q>.  (The FFT row stage does this for the FFT problems.)
template <typename T>
__global__ void __launch_bounds__(256) k_cg_pq(const Prob* __restrict__ P, CgState s, int par,
                                               const T* __restrict__ pv, T* __restrict__ q,
                                               double* __restrict__ part) {
    __shared__ double red[256];
    const int cnt = gridDim.y;
    if (s.done[par * cnt + blockIdx.y] || P[blockIdx.y].mode == 1) return;
    const Prob& p = P[blockIdx.y];
    const int64_t m = int64_t(p.n) * p.n, o = p.o_c;
    int64_t lo, hi;
    slice_of(m, lo, hi);
    const T nu = T(s.nu[blockIdx.y]);
    double acc = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += 256) {
        const T pe = pv[o + e];
        const T qe = q[o + e] + nu * pe;
        q[o + e] = qe;
        acc += double(pe) * double(qe);
    }
    reduce_to_part(acc, red, part, kCgRowParts);
}

// alpha = rr / <p, q>; x += alpha p; r -= alpha q (float64); part_rr =
// slices of |r|^2.
template <typename T>
__global__ void __launch_bounds__(256) k_cg_update(const Prob* __restrict__ P, CgState s, int par, int comps,
                                                   int pq_stride, const double* __restrict__ pv,
                                                   const T* __restrict__ q, double* __restrict__ x,
                                                   double* __restrict__ r, const double* __restrict__ part_pq,
                                                   double* __restrict__ part_rr) {
    __shared__ double red[256];
    __shared__ double slot;
    const int b = blockIdx.y, cnt = gridDim.y;
    if (s.done[par * cnt + b]) return;
    const Prob& p = P[b];
    const int64_t m = int64_t(comps) * p.n * p.n, o = int64_t(comps) * p.o_c;
    int64_t lo, hi;
    slice_of(m, lo, hi);
    const double alpha = broadcast0(
        threadIdx.x == 0
            ? s.rr[par * cnt + b] / sum_parts(part_pq + int64_t(b) * pq_stride, pq_parts(p))
            : 0.0,
        &slot);
    double acc = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += 256) {
        x[o + e] += alpha * pv[o + e];
        const double re = r[o + e] - alpha * double(q[o + e]);
        r[o + e] = re;
        acc += re * re;
    }
    reduce_to_part(acc, red, part_rr);
}

// beta = |r_new|^2 / rr; p = r + beta p.  The first work-group of a problem
// also writes the next slot of the state: rr = |r_new|^2, one more step
// counted, and the stop rule (|r| <= tol |b| or max_iter steps); a stopped
// problem's state is carried over unchanged.
template <typename T>
__global__ void __launch_bounds__(256) k_cg_dir(const Prob* __restrict__ P, CgState s, int par, int comps,
                                                const double* __restrict__ r, double* __restrict__ pv,
                                                T* __restrict__ pt, const double* __restrict__ part_rr, double tol,
                                                int max_iter) {
    __shared__ double slot;
    const int b = blockIdx.y, cnt = gridDim.y;
    const int cur = par * cnt + b, nxt = (1 - par) * cnt + b;
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (s.done[cur]) {
        if (lead) {
            s.done[nxt] = 1;
            s.rr[nxt] = s.rr[cur];
        }
        return;
    }
    const Prob& p = P[b];
    const int64_t m = int64_t(comps) * p.n * p.n, o = int64_t(comps) * p.o_c;
    int64_t lo, hi;
    slice_of(m, lo, hi);
    const double rr_new = broadcast0(threadIdx.x == 0 ? sum_parts(part_rr + int64_t(b) * kDotParts) : 0.0, &slot);
    const double bt = rr_new / s.rr[cur];
    for (int64_t e = lo + threadIdx.x; e < hi; e += 256) {
        const double pn = r[o + e] + bt * pv[o + e];
        pv[o + e] = pn;
        pt[o + e] = T(pn);
    }
    if (lead) {
        const int it = s.iters[b] + 1;
        s.iters[b] = it;
        s.rr[nxt] = rr_new;
        s.done[nxt] = (it < max_iter && rr_new > tol * tol * s.bb[b]) ? 0 : 1;
    }
}

// ------------------------------------------------------ percentile trim ---
// Order-preserving unsigned keys of IEEE values: flip the sign bit of
// non-negative values, every bit of negative ones.
__device__ __forceinline__ uint32_t order_key(float v) {
    const uint32_t b = __float_as_uint(v);
    return b ^ ((b >> 31) ? 0xffffffffu : 0x80000000u);
}
__device__ __forceinline__ uint64_t order_key(double v) {
    const uint64_t b = uint64_t(__double_as_longlong(v));
    return b ^ ((b >> 63) ? ~uint64_t(0) : (uint64_t(1) << 63));
}
__device__ __forceinline__ float key_value(uint32_t k) {
    return __uint_as_float(k ^ ((k >> 31) ? 0x80000000u : 0xffffffffu));
}
__device__ __forceinline__ double key_value(uint64_t k) {
    return __longlong_as_double(int64_t(k ^ ((k >> 63) ? (uint64_t(1) << 63) : ~uint64_t(0))));
}

// One work-group of 1024 threads per problem: the pct-th percentile of the
// problem's n^2 values with the linear rule -- the order statistics of rank
// i = floor(pos) and i + 1, pos = pct/100 (n^2 - 1), found together by an
// 8-bit radix select over the keys (most significant digit first, one read of
// the data per digit, integer histograms in LDS), then
// q = v_i + (pos - i)(v_{i+1} - v_i) in float64 (v_i itself when i is the last
// rank).
template <typename T>
__global__ void __launch_bounds__(1024) k_percentile(const Prob* __restrict__ P, const T* __restrict__ x,
                                                     double pct, double* __restrict__ q_out) {
    using K = typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type;
    constexpr int kBits = 8 * int(sizeof(T));
    __shared__ int hist[2][256];
    __shared__ K prefix[2];
    __shared__ int64_t rank[2], rank_next[2];
    __shared__ int digit[2];
    __shared__ int wtot[8];
    const Prob& p = P[blockIdx.x];
    const int64_t m = int64_t(p.n) * p.n;
    const T* xp = x + p.o_c;
    const double pos = pct / 100.0 * double(m - 1);
    const int64_t i0 = int64_t(floor(pos));
    const double f = pos - double(i0);
    const bool last = i0 + 1 >= m;
    const int tid = threadIdx.x;
    if (tid < 2) {
        prefix[tid] = K(0);
        rank[tid] = tid == 0 ? i0 : (last ? i0 : i0 + 1);
    }
    for (int shift = kBits - 8; shift >= 0; shift -= 8) {
        for (int i = tid; i < 512; i += 1024) hist[i >> 8][i & 255] = 0;
        __syncthreads();
        const K hi_mask = shift + 8 >= kBits ? K(0) : ~K(0) << (shift + 8);
        const K pa = prefix[0] & hi_mask, pb = prefix[1] & hi_mask;
        const bool shared_prefix = pa == pb;     // then one histogram serves both ranks
        // kLoads values per thread in flight before their histogram updates
        constexpr int kLoads = 16;
        for (int64_t e0 = tid; e0 < m; e0 += int64_t(1024) * kLoads) {
            K kk[kLoads];
#pragma unroll
            for (int u = 0; u < kLoads; ++u) {
                const int64_t e = e0 + int64_t(u) * 1024;
                kk[u] = e < m ? order_key(xp[e]) : K(0);
            }
#pragma unroll
            for (int u = 0; u < kLoads; ++u) {
                if (e0 + int64_t(u) * 1024 >= m) break;
                const K k = kk[u];
                const int d = int((k >> shift) & K(255));
                if ((k & hi_mask) == pa) atomicAdd(&hist[0][d], 1);
                if (!shared_prefix && (k & hi_mask) == pb) atomicAdd(&hist[1][d], 1);
            }
        }
        __syncthreads();
        // the digit of each rank: threads s 256 + d scan histogram s; the bin
        // whose range [cum, cum + hist) holds the rank takes it (the last bin
        // also takes a rank past the total), as a walk from digit 0 would
        int sc = 0, h = 0;
        if (tid < 512) {
            h = hist[shared_prefix ? 0 : tid >> 8][tid & 255];
            sc = h;                                 // inclusive scan within the wave
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int y = __shfl_up(sc, off, 64);
                if ((tid & 63) >= off) sc += y;
            }
            if ((tid & 63) == 63) wtot[tid >> 6] = sc;
        }
        __syncthreads();
        if (tid < 512) {
            const int s = tid >> 8, d = tid & 255, wv = tid >> 6;
            int64_t cum = sc - h;
            for (int q = s * 4; q < wv; ++q) cum += wtot[q];
            const int64_t r = rank[s];
            if (cum <= r && (r < cum + h || d == 255)) {
                rank_next[s] = r - cum;
                digit[s] = d;
            }
        }
        __syncthreads();
        if (tid < 2) {
            rank[tid] = rank_next[tid];
            prefix[tid] |= K(digit[tid]) << shift;
        }
        __syncthreads();
    }
    if (tid == 0) {
#pragma clang fp contract(off)
        // rounded step by step (no fused multiply-add), as the linear rule reads
        const double v0 = double(key_value(prefix[0])), v1 = double(key_value(prefix[1]));
        const double d = v1 - v0;
        const double fd = f * d;
        q_out[blockIdx.x] = last ? v0 : v0 + fd;
    }
}

// -------------------------------------------------- trim and moments ---
// grid (kDotParts, problems), 256 threads: x <- max(x, q_b) when q is given
// (values below the percentile raised to it), part = slices of sum x.
template <typename T>
__global__ void __launch_bounds__(256) k_clamp_sum(const Prob* __restrict__ P, T* __restrict__ x,
                                                   const double* __restrict__ q, double* __restrict__ part) {
    __shared__ double red[256];
    const Prob& p = P[blockIdx.y];
    const int64_t m = int64_t(p.n) * p.n, o = p.o_c;
    int64_t lo, hi;
    slice_of(m, lo, hi);
    const T qb = q ? T(q[blockIdx.y]) : T(0);
    double acc = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += 256) {
        T v = x[o + e];
        if (q && v < qb) {
            v = qb;
            x[o + e] = v;
        }
        acc += double(v);
    }
    reduce_to_part(acc, red, part);
}

// part = slices of sum (x - mean_b)^2.
template <typename T>
__global__ void __launch_bounds__(256) k_sq_dev(const Prob* __restrict__ P, const T* __restrict__ x,
                                                const double* __restrict__ mean, double* __restrict__ part) {
    __shared__ double red[256];
    const Prob& p = P[blockIdx.y];
    const int64_t m = int64_t(p.n) * p.n, o = p.o_c;
    int64_t lo, hi;
    slice_of(m, lo, hi);
    const double mu = mean[blockIdx.y];
    double acc = 0.0;
    for (int64_t e = lo + threadIdx.x; e < hi; e += 256) {
        const double d = double(x[o + e]) - mu;
        acc += d * d;
    }
    reduce_to_part(acc, red, part);
}

// one thread per problem: out[b] = (sum of the problem's slices) / n^2.
__global__ void k_part_mean(const Prob* __restrict__ P, int count, const double* __restrict__ part,
                            double* __restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= count) return;
    out[b] = sum_parts(part + int64_t(b) * kDotParts) / double(int64_t(P[b].n) * P[b].n);
}

// y = x over the problems' grids (concatenated layout), n elements.
template <typename T>
__global__ void k_copy(const T* __restrict__ x, T* __restrict__ y, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i];
}

}  // namespace mpik
