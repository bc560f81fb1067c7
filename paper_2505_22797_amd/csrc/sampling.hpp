// Sampling along the trajectory (bilinear interpolation of the three field
// channels, contraction with the velocity: s_k = A[c](r_k) v_k, eq.
// core:formula) and its exact transpose.  Both work on a band of grid rows
// held in LDS by one work-group.
//
// The transpose is deterministic: contributions (sample, corner) are grouped
// by target cell at plan time; the work-group splits its contiguous range of
// contributions evenly over its threads, each thread sums runs of equal cells
// in order, and partial sums of cells that straddle thread boundaries are
// combined by the lowest thread in a fixed order.  No floating-point atomics.
#pragma once
#include "common.hpp"

namespace mpik {

// Gather for the samples of base-cell row b (cell order [p0, p1)).  g0/g1 hold
// the three channels of grid rows b and b+1: g0[ch * N + i], g1[ch * N + i].
// RESID: write s - y (cell order) to out_sorted[p]; else s to s_time[perm[p]].
template <typename T, bool RESID>
__device__ __forceinline__ void gather_band(const T* g0, const T* g1, int N, int p0, int p1,
                                            const vec4<T>* __restrict__ samp, const int* __restrict__ bcell,
                                            const int* __restrict__ perm, const vec2<T>* __restrict__ ysort,
                                            vec2<T>* __restrict__ out_sorted, T* __restrict__ s_time,
                                            int tid, int nthreads) {
    for (int p = p0 + tid; p < p1; p += nthreads) {
        const vec4<T> e = samp[p];
        const int i0 = bcell[p] & 0xffff;
        const T fx = e.x, fy = e.y, gx = T(1) - fx, gy = T(1) - fy;
        T g[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const T lo = gx * g0[ch * N + i0] + fx * g0[ch * N + i0 + 1];
            const T hi = gx * g1[ch * N + i0] + fx * g1[ch * N + i0 + 1];
            g[ch] = gy * lo + fy * hi;
        }
        const T sx = g[0] * e.z + g[1] * e.w;
        const T sy = g[1] * e.z + g[2] * e.w;
        if (RESID) {
            const vec2<T> y = ysort[p];
            vec2<T> o;
            o.x = sx - y.x;
            o.y = sy - y.y;
            out_sorted[p] = o;
        } else {
            const int k = perm[p];
            s_time[2 * k] = sx;
            s_time[2 * k + 1] = sy;
        }
    }
}

// Shared-memory layout of scatter_band for a band of `rows` grid rows.
template <typename T> struct ScatterSmem {
    static constexpr int kThreads = 192;
    int cs[2 * 1024 + 1];            // cell starts of the band (<= 2 rows of N <= 1024)
    int first_cell[kThreads], last_cell[kThreads];
    T first_val[kThreads][3], last_val[kThreads][3];
};

// Transpose of the sampling for the cells of `rows` consecutive grid rows
// starting at row0.  Writes g[ch * rows * N + local_cell] in LDS (zeroed here).
// SORTED: signal/residual read in cell order from ys[p]; else in time order
// from s_time[perm[p]].
template <typename T, bool SORTED>
__device__ __forceinline__ void scatter_band(T* g, ScatterSmem<T>& sm, int N, int row0, int rows,
                                             const int* __restrict__ cellstart, const int* __restrict__ items,
                                             const vec4<T>* __restrict__ samp, const int* __restrict__ perm,
                                             const vec2<T>* __restrict__ ys, const T* __restrict__ s_time,
                                             int tid) {
    constexpr int NT = ScatterSmem<T>::kThreads;
    const int nc = rows * N;
    const int cbase = row0 * N;
    for (int i = tid; i <= nc; i += NT) sm.cs[i] = cellstart[cbase + i];
    for (int i = tid; i < 3 * nc; i += NT) g[i] = T(0);
    __syncthreads();
    const int I0 = sm.cs[0], I1 = sm.cs[nc];
    const int E = (I1 - I0 + NT - 1) / NT;
    const int a = min(I0 + tid * E, I1), b = min(a + E, I1);
    int fc = -1, lc = -1;
    T acc0 = T(0), acc1 = T(0), acc2 = T(0);
    T f0 = T(0), f1 = T(0), f2 = T(0);
    if (a < b) {
        // largest cell with cs[cell] <= a (it holds item a)
        int lo = 0, hi = nc;          // invariant: cs[lo] <= a < cs[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (sm.cs[mid] <= a) lo = mid; else hi = mid;
        }
        lc = lo;
        fc = lo;
        for (int it = a; it < b; ++it) {
            while (it >= sm.cs[lc + 1]) {       // leaving cell lc
                if (lc == fc) { f0 = acc0; f1 = acc1; f2 = acc2; }
                else { g[lc] = acc0; g[nc + lc] = acc1; g[2 * nc + lc] = acc2; }
                acc0 = acc1 = acc2 = T(0);
                ++lc;
            }
            const unsigned item = unsigned(items[it]);
            const int p = int(item & 0x3fffffffu);
            const unsigned corner = item >> 30;
            const vec4<T> e = samp[p];
            vec2<T> y;
            if (SORTED) {
                y = ys[p];
            } else {
                const int k = perm[p];
                y.x = s_time[2 * k];
                y.y = s_time[2 * k + 1];
            }
            const T wx = (corner & 1u) ? e.x : T(1) - e.x;
            const T wy = (corner & 2u) ? e.y : T(1) - e.y;
            const T w = wx * wy;
            acc0 += w * (y.x * e.z);
            acc1 += w * (y.x * e.w + y.y * e.z);
            acc2 += w * (y.y * e.w);
        }
        if (lc == fc) { f0 = acc0; f1 = acc1; f2 = acc2; }
    }
    sm.first_cell[tid] = fc;
    sm.last_cell[tid] = lc;
    sm.first_val[tid][0] = f0; sm.first_val[tid][1] = f1; sm.first_val[tid][2] = f2;
    sm.last_val[tid][0] = acc0; sm.last_val[tid][1] = acc1; sm.last_val[tid][2] = acc2;
    __syncthreads();
    if (a < b) {
        const bool shared_head = tid > 0 && sm.last_cell[tid - 1] == fc;
        if (fc != lc && !shared_head) {          // first cell lies wholly in this thread
            g[fc] = f0; g[nc + fc] = f1; g[2 * nc + fc] = f2;
        }
        if (!(fc == lc && shared_head)) {         // this thread owns its last cell
            T s0 = acc0, s1 = acc1, s2 = acc2;
            for (int u = tid + 1; u < NT && sm.first_cell[u] == lc; ++u) {
                s0 += sm.first_val[u][0];
                s1 += sm.first_val[u][1];
                s2 += sm.first_val[u][2];
                if (sm.last_cell[u] != lc) break;
            }
            g[lc] = s0; g[nc + lc] = s1; g[2 * nc + lc] = s2;
        }
    }
    __syncthreads();
}

}  // namespace mpik
