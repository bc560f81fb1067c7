// Sampling along the trajectory (interpolation of the three field channels
// from the four surrounding cell centres with the per-axis weights stored in
// the sample records, bilinear or cosine; contraction with the velocity:
// s_k = A[c](r_k) v_k, eq. core:formula) and its exact transpose.  Both work on a band of grid rows
// held in LDS by one work-group.
//
// The transpose is deterministic: samples are sorted by base cell at plan
// time; a work-group splits its contiguous range of samples evenly over its
// threads, each thread sums runs of equal base cells in order, partial sums of
// base cells that straddle thread boundaries are combined by the lowest thread
// in a fixed order, and every grid cell adds its four base cells in a fixed
// order.  No floating-point atomics.  Loads are issued in batches so that a
// thread keeps several in flight.
#pragma once
#include "common.hpp"

namespace mpik {

// Gather for the samples of base-cell row b (cell order [p0, p1)).  g0/g1 hold
// the three channels of grid rows b and b+1: g0[ch * N + i], g1[ch * N + i].
// MODE 0: s = G(r_k) v_k to out0[k] (time order).
// MODE 1: s - y (y = ysort, cell order) to out_sorted[p].
// MODE 3: s - y (y = in0, time order) to out0[k].
// MODE 2: the gradients of <y, s> (y = in0, time order) with respect to the
//         sample position and velocity, inside the interpolation patch:
//         out0[k] = (y^T M(dG/dx) v, y^T M(dG/dy) v), out1[k] = M(G) y,
//         with M(g) = [[g_xx, g_xy], [g_xy, g_yy]] and
//         d/dx = (N/2) (dwx/dfx) d/dwx with the slopes dw (plans built for
//         derivatives; the derivative modes read them unconditionally).
// MODE 4: s to out0[p] (cell order).
// MODE 5: s - y (y = ysort) to out0[p], and the sampled field with its
//         position gradient, nine planes f[q * fstride + p]:
//         (G_xx, G_xy, G_yy, dG/dx (3), dG/dy (3)), all in cell order.
// MODE 6: with y = in0[p] and the field F' of planes f (as MODE 5 wrote them):
//         q = G v to out0[p]; out1[p] += (y^T M(dG/dx) v + q^T M(dF'/dx) v,
//         y^T M(dG/dy) v + q^T M(dF'/dy) v); out2[p] += M(G) y + M(F') q;
//         all in cell order.
// The sample records of one pass of gather_band: thread tid handles cell-order
// positions base + u * nthreads, u < U.
template <typename T, int U> struct GatherRecs {
    vec4<T> e[U];
    int2 id[U];
    vec2<T> y[U];
#ifdef MPIK_CHECK
    bool valid[U];       // the record's base cell and time index passed the checks
#endif
    __device__ __forceinline__ bool usable(int u) const {
#ifdef MPIK_CHECK
        return valid[u];
#else
        (void)u;
        return true;
#endif
    }
};

// chx (x receive channel alone): the y components of the signals read are
// taken as 0, and the y components written are 0.
template <typename T, int MODE, int U>
__device__ __forceinline__ void gather_fetch(GatherRecs<T, U>& r, int base, int p1, int nthreads,
                                             const vec4<T>* __restrict__ samp, const int2* __restrict__ sidx,
                                             const vec2<T>* __restrict__ ysort, const T* __restrict__ in0,
                                             bool chx, const Chk& ck) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int p = base + u * nthreads;
        if (p < p1) {
            r.e[u] = samp[p];
            r.id[u] = sidx[p];
#ifdef MPIK_CHECK
            r.valid[u] = ck.cell(r.id[u].x) && ck.time(r.id[u].y);
#endif
            if (MODE == 1 || MODE == 5) r.y[u] = ysort[p];
            if (MODE == 6) {
                r.y[u].x = in0[2 * p];
                r.y[u].y = in0[2 * p + 1];
            }
        }
    }
    if (MODE == 2 || MODE == 3) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = base + u * nthreads;
            if (p < p1 && r.usable(u)) {
                r.y[u].x = in0[2 * r.id[u].y];
                r.y[u].y = in0[2 * r.id[u].y + 1];
            }
        }
    }
    if (MODE != 0 && MODE != 4 && chx) {
#pragma unroll
        for (int u = 0; u < U; ++u) r.y[u].y = T(0);
    }
}

// sq (MODE 4 only, may be null): the thread's running sum of |s_k|^2 in
// float64, of the values as stored.
template <typename T, int MODE, int U>
__device__ __forceinline__ void gather_apply(const GatherRecs<T, U>& r, int base, int p1, int nthreads,
                                             const T* g0, const T* g1, int N, vec2<T>* __restrict__ out_sorted,
                                             T* __restrict__ out0, T* __restrict__ out1, T* __restrict__ out2,
                                             T* __restrict__ f, int64_t fstride, const vec2<T>* __restrict__ dw,
                                             bool chx, double* sq = nullptr) {
    constexpr bool GRAD = MODE == 2 || MODE == 5 || MODE == 6;
    const T inv_d = T(0.5) * T(N);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int p = base + u * nthreads;
        if (p >= p1) break;
        if (!r.usable(u)) continue;
        const int i0 = r.id[u].x & 0xffff;
        const T fx = r.e[u].x, fy = r.e[u].y, gx = T(1) - fx, gy = T(1) - fy;
        vec2<T> sl;                       // weight slopes (read here: kept out of the prefetched records)
        if (GRAD) sl = dw[p];
        T g[3], dx[3], dy[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const T a00 = g0[ch * N + i0], a10 = g0[ch * N + i0 + 1];
            const T a01 = g1[ch * N + i0], a11 = g1[ch * N + i0 + 1];
            const T lo = gx * a00 + fx * a10;
            const T hi = gx * a01 + fx * a11;
            g[ch] = gy * lo + fy * hi;
            if (GRAD) {
                dx[ch] = (inv_d * sl.x) * (gy * (a10 - a00) + fy * (a11 - a01));
                dy[ch] = (inv_d * sl.y) * (gx * (a01 - a00) + fx * (a11 - a10));
            }
        }
        const T vx = r.e[u].z, vy = r.e[u].w;
        const int k = r.id[u].y;
        const vec2<T> y = r.y[u];
        if (MODE == 2) {
            const T yx = y.x, yy = y.y;
            out0[2 * k] = yx * (dx[0] * vx + dx[1] * vy) + yy * (dx[1] * vx + dx[2] * vy);
            out0[2 * k + 1] = yx * (dy[0] * vx + dy[1] * vy) + yy * (dy[1] * vx + dy[2] * vy);
            out1[2 * k] = g[0] * yx + g[1] * yy;
            out1[2 * k + 1] = g[1] * yx + g[2] * yy;
        } else if (MODE == 6) {
            const T yx = y.x, yy = y.y;
            const T qx = g[0] * vx + g[1] * vy;
            const T qy = chx ? T(0) : g[1] * vx + g[2] * vy;
            T h[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) h[q] = f[q * fstride + p];
            const T gr_x = (yx * (dx[0] * vx + dx[1] * vy) + yy * (dx[1] * vx + dx[2] * vy)) +
                           (qx * (h[3] * vx + h[4] * vy) + qy * (h[4] * vx + h[5] * vy));
            const T gr_y = (yx * (dy[0] * vx + dy[1] * vy) + yy * (dy[1] * vx + dy[2] * vy)) +
                           (qx * (h[6] * vx + h[7] * vy) + qy * (h[7] * vx + h[8] * vy));
            const T gv_x = (g[0] * yx + g[1] * yy) + (h[0] * qx + h[1] * qy);
            const T gv_y = (g[1] * yx + g[2] * yy) + (h[1] * qx + h[2] * qy);
            out0[2 * p] = qx;
            out0[2 * p + 1] = qy;
            out1[2 * p] += gr_x;
            out1[2 * p + 1] += gr_y;
            out2[2 * p] += gv_x;
            out2[2 * p + 1] += gv_y;
        } else {
            const T sx = g[0] * vx + g[1] * vy;
            const T sy = chx ? T(0) : g[1] * vx + g[2] * vy;
            if (MODE == 1) {
                vec2<T> o;
                o.x = sx - y.x;
                o.y = sy - y.y;
                out_sorted[p] = o;
            } else if (MODE == 5) {
                out0[2 * p] = sx - y.x;
                out0[2 * p + 1] = sy - y.y;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    f[ch * fstride + p] = g[ch];
                    f[(3 + ch) * fstride + p] = dx[ch];
                    f[(6 + ch) * fstride + p] = dy[ch];
                }
            } else if (MODE == 4) {
                out0[2 * p] = sx;
                out0[2 * p + 1] = sy;
                if (sq) *sq += double(sx) * double(sx) + double(sy) * double(sy);
            } else if (MODE == 3) {
                vec2<T> o;
                o.x = sx - y.x;
                o.y = sy - y.y;
                reinterpret_cast<vec2<T>*>(out0)[k] = o;
            } else {
                vec2<T> o;
                o.x = sx;
                o.y = sy;
                reinterpret_cast<vec2<T>*>(out0)[k] = o;
            }
        }
    }
}

// `first`, when given, holds the records of the first pass (fetched by the
// caller ahead of time so that their loads overlap its other work).
template <typename T, int MODE, int U = 4>
__device__ __forceinline__ void gather_band(const T* g0, const T* g1, int N, int p0, int p1,
                                            const vec4<T>* __restrict__ samp, const int2* __restrict__ sidx,
                                            const vec2<T>* __restrict__ ysort, vec2<T>* __restrict__ out_sorted,
                                            T* __restrict__ out0, const T* __restrict__ in0, T* __restrict__ out1,
                                            T* __restrict__ out2, T* __restrict__ f, int64_t fstride,
                                            const vec2<T>* __restrict__ dw, bool chx, int tid, int nthreads,
                                            const Chk& ck, const GatherRecs<T, U>* first = nullptr,
                                            double* sq = nullptr) {
    int base = p0 + tid;
    if (first) {
        if (base < p1) gather_apply<T, MODE, U>(*first, base, p1, nthreads, g0, g1, N, out_sorted, out0, out1, out2, f,
                                                fstride, dw, chx, sq);
        base += U * nthreads;
    }
    for (; base < p1; base += U * nthreads) {
        GatherRecs<T, U> r;
        gather_fetch<T, MODE, U>(r, base, p1, nthreads, samp, sidx, ysort, in0, chx, ck);
        gather_apply<T, MODE, U>(r, base, p1, nthreads, g0, g1, N, out_sorted, out0, out1, out2, f, fstride, dw, chx,
                                 sq);
    }
}

// Shared-memory part of scatter_row, carved from a dynamic LDS region: per
// base cell of the two base-cell rows (left, right) x 3 channel sums, and the
// first/last base cell of every thread with the partial sum of the first.
template <typename T> struct ScatterLds {
    T* K;
    short* first_key;      // keys are below 2 (N - 1) <= 2046, or -1
    short* last_key;
    T* first_val;
};

__host__ __device__ constexpr size_t lds_align(size_t b) { return (b + 15) / 16 * 16; }

// byte offset of first_val in the region (the sums K and the keys come first)
template <typename T>
__host__ __device__ constexpr size_t scatter_lds_first_val(int N, int NT) {
    return lds_align(size_t(2) * (N - 1) * 6 * sizeof(T)) + lds_align(size_t(2) * NT * sizeof(short));
}

template <typename T>
__host__ __device__ constexpr size_t scatter_lds_bytes(int N, int NT) {
    return scatter_lds_first_val<T>(N, NT) + lds_align(size_t(NT) * 6 * sizeof(T));
}

template <typename T>
__device__ __forceinline__ ScatterLds<T> scatter_lds(char* base, int N, int NT) {
    ScatterLds<T> v;
    v.K = reinterpret_cast<T*>(base);
    v.first_key = reinterpret_cast<short*>(base + lds_align(size_t(2) * (N - 1) * 6 * sizeof(T)));
    v.last_key = v.first_key + NT;
    v.first_val = reinterpret_cast<T*>(base + scatter_lds_first_val<T>(N, NT));
    return v;
}

// Transpose of the sampling for the cells of grid row j.  Those cells receive
// from the samples of base-cell rows j-1 (weight fy) and j (weight 1 - fy),
// which are one contiguous range in cell order.  Pass 1 splits that range
// evenly over the threads; every thread walks its samples in order and sums,
// per base cell, the contributions to the cell on its left (weight 1 - fx)
// and on its right (fx); base cells that straddle thread boundaries are
// combined by their first thread in thread order.  Pass 2 assembles every
// cell from its (at most) four base cells in a fixed order.  The result goes
// to g[ch * N + i] in LDS.  SORTED: the signal/residual is read in cell order
// from ys[p]; else in time order from s_time[k].  chx: the y components
// are taken as 0 (x receive channel alone).
template <typename T, bool SORTED, int NT, int U = 4>
__device__ __forceinline__ void scatter_row(T* g, ScatterLds<T> sm, int N, int j,
                                            const int* __restrict__ binstart, const vec4<T>* __restrict__ samp,
                                            const int2* __restrict__ sidx, const vec2<T>* __restrict__ ys,
                                            const T* __restrict__ s_time, int tid, bool chx, const Chk& ck) {
    const int nb = N - 1;
    const int rlo = max(j - 1, 0), rhi = min(j, nb - 1);       // base-cell rows that reach row j
    const int nkeys = 2 * nb;
    for (int i = tid; i < nkeys * 6; i += NT) sm.K[i] = T(0);
#ifdef MPIK_CHECK
    int P0 = binstart[rlo * nb], P1 = binstart[(rhi + 1) * nb];
    ck.range(P0, P1);
#else
    (void)ck;
    const int P0 = binstart[rlo * nb], P1 = binstart[(rhi + 1) * nb];
#endif
    const int E = (P1 - P0 + NT - 1) / NT;
    const int a = min(P0 + tid * E, P1), b = min(a + E, P1);
    int fk = -1, lk = -1;
    T acc[6], fv[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) acc[q] = fv[q] = T(0);
    __syncthreads();
    for (int base = a; base < b; base += U) {
        vec4<T> e[U];
        int2 id[U];
        vec2<T> y[U];
#ifdef MPIK_CHECK
        bool use[U];
#endif
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (base + u < b) {
                e[u] = samp[base + u];
                id[u] = sidx[base + u];
                if (SORTED) y[u] = ys[base + u];
#ifdef MPIK_CHECK
                use[u] = ck.cell_near(id[u].x, j) && (SORTED || ck.time(id[u].y));
#endif
            }
        }
        if (!SORTED) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
#ifdef MPIK_CHECK
                if (base + u < b && use[u]) {
#else
                if (base + u < b) {
#endif
                    const int k = id[u].y;
                    y[u].x = s_time[2 * k];
                    y[u].y = s_time[2 * k + 1];
                }
            }
        }
        if (chx) {
#pragma unroll
            for (int u = 0; u < U; ++u) y[u].y = T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (base + u >= b) break;
#ifdef MPIK_CHECK
            if (!use[u]) continue;
#endif
            const int i0 = id[u].x & 0xffff, j0 = id[u].x >> 16;
            const int key = (j0 - (j - 1)) * nb + i0;      // 0 .. nb-1: row j-1, nb .. 2nb-1: row j
            if (key != lk) {
                if (lk >= 0) {
                    if (lk == fk) {
#pragma unroll
                        for (int q = 0; q < 6; ++q) fv[q] = acc[q];
                    } else {
#pragma unroll
                        for (int q = 0; q < 6; ++q) sm.K[lk * 6 + q] = acc[q];
                    }
                } else {
                    fk = key;
                }
#pragma unroll
                for (int q = 0; q < 6; ++q) acc[q] = T(0);
                lk = key;
            }
            const T wy = (j0 == j) ? T(1) - e[u].y : e[u].y;
            const T wl = (T(1) - e[u].x) * wy, wr = e[u].x * wy;
            const T p0 = y[u].x * e[u].z;
            const T p1 = y[u].x * e[u].w + y[u].y * e[u].z;
            const T p2 = y[u].y * e[u].w;
            acc[0] += wl * p0; acc[1] += wl * p1; acc[2] += wl * p2;
            acc[3] += wr * p0; acc[4] += wr * p1; acc[5] += wr * p2;
        }
    }
    if (lk >= 0 && lk == fk) {
#pragma unroll
        for (int q = 0; q < 6; ++q) fv[q] = acc[q];
    }
    sm.first_key[tid] = short(fk);
    sm.last_key[tid] = short(lk);
#pragma unroll
    for (int q = 0; q < 6; ++q) sm.first_val[tid * 6 + q] = fv[q];
    __syncthreads();
    if (lk >= 0) {
        const bool shared_head = tid > 0 && sm.last_key[tid - 1] == fk;
        if (fk != lk && !shared_head) {          // first key lies wholly in this thread
#pragma unroll
            for (int q = 0; q < 6; ++q) sm.K[fk * 6 + q] = fv[q];
        }
        if (!(fk == lk && shared_head)) {         // this thread owns its last key
            T tot[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) tot[q] = acc[q];
            for (int u = tid + 1; u < NT && sm.first_key[u] == lk; ++u) {
#pragma unroll
                for (int q = 0; q < 6; ++q) tot[q] += sm.first_val[u * 6 + q];
                if (sm.last_key[u] != lk) break;
            }
#pragma unroll
            for (int q = 0; q < 6; ++q) sm.K[lk * 6 + q] = tot[q];
        }
    }
    __syncthreads();
    // cell (j, i) <- row j base cells i (left) and i-1 (right), then row j-1 likewise
    for (int i = tid; i < N; i += NT) {
        T v0 = T(0), v1 = T(0), v2 = T(0);
        if (j <= nb - 1) {
            if (i <= nb - 1) { const T* k = sm.K + (nb + i) * 6; v0 += k[0]; v1 += k[1]; v2 += k[2]; }
            if (i >= 1) { const T* k = sm.K + (nb + i - 1) * 6; v0 += k[3]; v1 += k[4]; v2 += k[5]; }
        }
        if (j >= 1) {
            if (i <= nb - 1) { const T* k = sm.K + i * 6; v0 += k[0]; v1 += k[1]; v2 += k[2]; }
            if (i >= 1) { const T* k = sm.K + (i - 1) * 6; v0 += k[3]; v1 += k[4]; v2 += k[5]; }
        }
        g[i] = v0;
        g[N + i] = v1;
        g[2 * N + i] = v2;
    }
    __syncthreads();
}

}  // namespace mpik
