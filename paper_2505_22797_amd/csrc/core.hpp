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
// concatenated buffer; signals in cell order at element offset o_s.
//
// One CG step is two launches over the grid rows of every problem:
//   A (k_core_dir_gather): the stop rule on |r|^2, then the new search
//     direction p = r + beta p_prev for grid rows j-1 .. j+1 (row j stored),
//     l = Delta p for row j (unscaled), the sampling y = I p of the samples in
//     base-cell row j, and per-row partial sums of sum_ch w_ch |l|^2 and |y|^2;
//   B (k_core_update): alpha = |r|^2 / <p, A p> with
//     <p, A p> = (1/L) |I p|^2 + gamma delta^2 sum_ch w_ch |Delta p|^2
//     (A = (1/L) I^T I + gamma delta^2 W Delta^2 with Delta symmetric), the
//     transpose sampling of y for grid row j, q = (1/L) I^T y + gamma delta^2
//     W Delta l for that row, x += alpha p, r -= alpha q, and the row's |r|^2.
// So q never goes to memory, and the direction update needs no pass of its
// own.  The search direction is double-buffered (a step reads the previous
// one while writing the next).
//
// Precision: the sampling runs in T on p rounded to T; the Laplacians, q, the
// CG vectors and all sums are float64.  The biharmonic stencil cancels on
// smooth fields, so in float32 its rounding would perturb the operator by
// about eps_32 times its largest eigenvalue, comparable to the smallest
// eigenvalues that decide the step count.
//
// Control: every problem runs its own CG.  Steps run in captured blocks; the
// state (|r|^2 of the step's residual, steps taken, stop flag) is double-
// buffered by step parity: launch A of step i reads slot i & 1 and its first
// work-group writes slot (i + 1) & 1, which launch B of the same step reads.
// Totals of partial sums are taken by every work-group that needs them in the
// same fixed order (tree_sum), so all of them see the same value.
#pragma once
#include "common.hpp"
#include "deconv.hpp"
#include "sampling.hpp"

namespace mpik {

constexpr int kCoreParts = 1024;       // partial sums per problem: one per grid row

struct CoreCg {
    double* rr;      // [2][count] |r|^2 of the residual a step starts from
    double* bb;      // [count] |b|^2
    int* steps;      // [2][count] steps taken before the slot's step
    int* done;       // [2][count] 1: stopped
    double* part_r;  // [count][kCoreParts] per grid row: |r|^2
    double* part_l;  // per grid row: sum_ch w_ch |lap5 p|^2
    double* part_y;  // per base-cell row: |I p|^2 (0 for the last grid row)
};

// Total of one value per thread over a work-group of 256 threads by a fixed
// tree (red: 256 entries); every thread gets it.
__device__ __forceinline__ double block_total(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double t = red[0];
    __syncthreads();
    return t;
}

// Fixed-order total of n partial sums, the same value in every work-group of
// 256 threads: thread t adds parts t, t + 256, ... in turn, then block_total.
__device__ __forceinline__ double tree_sum(const double* __restrict__ part, int n, double* red) {
    double v = 0.0;
    for (int q = threadIdx.x; q < n; q += 256) v += part[q];
    return block_total(v, red);
}

// The fixed tree of tree_sum over two values per thread at once (red holds
// 512 entries); every thread gets both totals.
__device__ __forceinline__ void tree_sum2(double& a, double& b, double* red) {
    const int t = threadIdx.x;
    red[t] = a;
    red[256 + t] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            red[t] += red[t + w];
            red[256 + t] += red[256 + t + w];
        }
        __syncthreads();
    }
    a = red[0];
    b = red[256];
    __syncthreads();
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

// Grid row j of the three channels of (1/L) I^T y, y in cell order (sums in
// T, the result in float64): the right-hand side.  grid (max N, problems),
// 256 threads; dynamic LDS as the operator's row-wise transpose sampling.
template <typename T>
__global__ void __launch_bounds__(256) k_core_rhs(const Prob* __restrict__ P, const T* __restrict__ y,
                                                  double* __restrict__ out, const char* __restrict__ plan) {
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.y];
    const int N = p.n, j = blockIdx.x;
    if (j >= N) return;
    T* g = reinterpret_cast<T*>(smem);
    char* sc = smem + lds_align(size_t(3) * N * sizeof(T));
    scatter_row<T, true, 256>(g, scatter_lds<T>(sc, N, 256), N, j, at<int>(plan, p.o_binstart),
                              at<vec4<T>>(plan, p.o_samp), at<int2>(plan, p.o_sidx),
                              reinterpret_cast<const vec2<T>*>(y + p.o_s), nullptr, threadIdx.x, p.chan == 1,
                              chk_of(p, plan));
    const double inv_l = 1.0 / double(p.t);
    const int64_t nn = int64_t(N) * N;
    double* o = out + 3 * p.o_c;
    for (int i = threadIdx.x; i < 3 * N; i += blockDim.x) {
        const int ch = i / N, x = i % N;
        o[ch * nn + int64_t(j) * N + x] = inv_l * double(g[i]);
    }
}

// x = 0, r = b, p_prev = 0 and part_r = the rows' |b|^2.  grid (max N,
// problems), 256 threads.
__global__ void __launch_bounds__(256) k_core_init(const Prob* __restrict__ P, const double* __restrict__ rhs,
                                                   double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ p_prev, CoreCg s) {
    __shared__ double red[256];
    const Prob& p = P[blockIdx.y];
    const int N = p.n, j = blockIdx.x;
    if (j >= N) return;
    const int64_t nn = int64_t(N) * N, o = 3 * p.o_c;
    double acc = 0.0;
    for (int i = threadIdx.x; i < 3 * N; i += 256) {
        const int ch = i / N, xx = i - ch * N;
        const int64_t off = o + ch * nn + int64_t(j) * N + xx;
        const double b = rhs[off];
        x[off] = 0.0;
        r[off] = b;
        p_prev[off] = 0.0;
        acc += b * b;
    }
    reduce_to_part(acc, red, s.part_r, kCoreParts);
}

// One work-group per problem: bb = rr = |b|^2 (slot 0), no step taken, and
// stopped at once when b = 0 or max_iter = 0.
__global__ void __launch_bounds__(256) k_core_begin(const Prob* __restrict__ P, CoreCg s, int max_iter) {
    __shared__ double red[256];
    const int b = blockIdx.x;
    const double bb = tree_sum(s.part_r + int64_t(b) * kCoreParts, P[b].n, red);
    if (threadIdx.x == 0) {
        s.bb[b] = bb;
        s.rr[b] = bb;
        s.steps[b] = 0;
        s.done[b] = (max_iter > 0 && bb > 0.0) ? 0 : 1;
    }
}

// Launch A's dynamic LDS: rows j-1 .. j+1 of p in float64 (at least 512
// doubles: the region also holds the reductions' scratch while the rows are
// not live), then rows j, j+1 rounded to T.
__host__ __device__ constexpr size_t core_dir_rows_bytes(int N) {
    return size_t(9) * N * 8 > 4096 ? size_t(9) * N * 8 : 4096;
}
__host__ __device__ constexpr size_t core_dir_lds_bytes(int N, int elem) {
    return core_dir_rows_bytes(N) + lds_align(size_t(6) * N * elem);
}

// Launch A of step par (see the file comment).  Stops the problem (state
// slot 1 - par) once |r| <= tol |b| or max_iter steps were taken; otherwise
// beta = |r|^2 / |r_prev|^2 (1 on the first step, where p_prev = 0).  grid
// (xcd_grid(max N), problems), 256 threads, grid rows dealt to the XCDs in
// contiguous bands (the neighbouring rows a work-group reads then share an
// L2); dynamic LDS core_dir_lds_bytes: rows j-1 .. j+1 of p in float64, then
// rows j, j+1 rounded to T for the sampling.
template <typename T>
__global__ void __launch_bounds__(256) k_core_dir_gather(const Prob* __restrict__ P, CoreCg s, int par,
                                                         const double* __restrict__ r,
                                                         const double* __restrict__ p_prev,
                                                         double* __restrict__ p_new, double* __restrict__ l,
                                                         T* __restrict__ y, double tol, int max_iter,
                                                         const char* __restrict__ plan) {
    extern __shared__ __align__(16) char smem[];
    double* red = reinterpret_cast<double*>(smem);                 // reductions, while pd is not live
    const int b = blockIdx.y, cnt = gridDim.y, cur = par * cnt + b, nxt = (1 - par) * cnt + b;
    const Prob& p = P[b];
    const int N = p.n, j = xcd_unit(blockIdx.x, N, b), tid = threadIdx.x;
    if (j < 0) return;
    const bool lead = j == 0 && tid == 0;
    if (s.done[cur]) {
        if (lead) {
            s.done[nxt] = 1;
            s.rr[nxt] = s.rr[cur];
            s.steps[nxt] = s.steps[cur];
        }
        return;
    }
    const int64_t nn = int64_t(N) * N, o = 3 * p.o_c;
    const int W = 3 * N;
    double* pd = reinterpret_cast<double*>(smem);                  // [3 rows][3 ch][N]
    T* pr = reinterpret_cast<T*>(smem + core_dir_rows_bytes(N));   // [2 rows][3 ch][N]
    // The thread's first column of r and p_prev on rows j-1 .. j+1 (all nine
    // row-channel pairs) is loaded before the |r|^2 total, so the loads
    // overlap its reduction; later columns (N > 256) follow in the loop below.
    double rv[9], pv9[9];
    const int x0 = tid;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int rw = q / 3, ch = q % 3, row = j - 1 + rw;
        if (x0 < N && row >= 0 && row < N) {
            const int64_t off = o + ch * nn + int64_t(row) * N + x0;
            rv[q] = r[off];
            pv9[q] = p_prev[off];
        }
    }
    const double rr = tree_sum(s.part_r + int64_t(b) * kCoreParts, N, red);
    const int taken = s.steps[cur];
    const bool stop = taken >= max_iter || !(rr > tol * tol * s.bb[b]);
    if (lead) {
        s.done[nxt] = stop ? 1 : 0;
        s.rr[nxt] = rr;
        s.steps[nxt] = stop ? taken : taken + 1;
    }
    if (stop) return;
    const double beta = rr / s.rr[cur];
    for (int x = x0; x < N; x += 256) {
        if (x != x0) {
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int rw = q / 3, ch = q % 3, row = j - 1 + rw;
                if (row >= 0 && row < N) {
                    const int64_t off = o + ch * nn + int64_t(row) * N + x;
                    rv[q] = r[off];
                    pv9[q] = p_prev[off];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const int rw = q / 3, ch = q % 3, row = j - 1 + rw;
            if (row >= 0 && row < N) {
                const double v = rv[q] + beta * pv9[q];
                pd[rw * W + ch * N + x] = v;
                if (rw == 1) p_new[o + ch * nn + int64_t(row) * N + x] = v;
                if (rw >= 1) pr[(rw - 1) * W + ch * N + x] = T(v);
            }
        }
    }
    __syncthreads();
    double accl = 0.0, accy = 0.0;
    for (int i = tid; i < W; i += 256) {
        const int ch = i / N, xx = i - ch * N;
        const double* m = pd + W + ch * N;                          // row j of channel ch
        const double v = m[xx];
        double sl = 0.0;                                             // lap5's order
        if (j > 0) sl += m[xx - W] - v;
        if (j + 1 < N) sl += m[xx + W] - v;
        if (xx > 0) sl += m[xx - 1] - v;
        if (xx + 1 < N) sl += m[xx + 1] - v;
        l[o + ch * nn + int64_t(j) * N + xx] = sl;
        accl += (ch == 1 ? 2.0 : 1.0) * sl * sl;
    }
    if (j < p.nb) {
        const int nb = p.nb;
        const int* binstart = at<int>(plan, p.o_binstart);
        int p0 = binstart[j * nb], p1 = binstart[(j + 1) * nb];
        const Chk ck = chk_of(p, plan).in_row(j);
        ck.range(p0, p1);
        gather_band<T, 4, 4>(pr, pr + W, N, p0, p1, at<vec4<T>>(plan, p.o_samp), at<int2>(plan, p.o_sidx), nullptr,
                          nullptr, y + p.o_s, nullptr, nullptr, nullptr, nullptr, p.t, nullptr, p.chan == 1, tid, 256,
                          ck, nullptr, &accy);
    }
    __syncthreads();                                                 // pd is read no more
    tree_sum2(accl, accy, red);
    if (tid == 0) {
        s.part_l[int64_t(b) * kCoreParts + j] = accl;
        s.part_y[int64_t(b) * kCoreParts + j] = accy;
    }
}

// Launch B of step par (see the file comment).  grid (xcd_grid(max N),
// problems), 256 threads, rows in contiguous bands per XCD as in launch A;
// dynamic LDS as the operator's row-wise transpose sampling.
template <typename T>
__global__ void __launch_bounds__(256) k_core_update(const Prob* __restrict__ P, CoreCg s, int par,
                                                     const T* __restrict__ y, const double* __restrict__ l,
                                                     const double* __restrict__ p_new, double* __restrict__ x,
                                                     double* __restrict__ r, double gamma,
                                                     const char* __restrict__ plan) {
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.y, cnt = gridDim.y, nxt = (1 - par) * cnt + b;
    const Prob& p = P[b];
    const int N = p.n, j = xcd_unit(blockIdx.x, N, b), tid = threadIdx.x;
    if (j < 0 || s.done[nxt]) return;
    const double d2 = 4.0 / (double(N) * N);                   // delta^2
    const double reg = gamma / d2;                               // gamma delta^2 / delta^4
    const double inv_l = 1.0 / double(p.t);
    // this thread's shares of the |I p|^2 and |Delta p|^2 partials, loaded
    // before the transpose sampling and reduced after it (tree_sum's order)
    double yy = 0.0, ll = 0.0;
    for (int q = tid; q < N; q += 256) {
        yy += s.part_y[int64_t(b) * kCoreParts + q];
        ll += s.part_l[int64_t(b) * kCoreParts + q];
    }
    const int64_t nn = int64_t(N) * N, o = 3 * p.o_c;
    // K elements per thread at a time; the first K elements' loads (Laplacian
    // neighbours, direction, field, residual) are issued before the transpose
    // sampling, which they do not depend on, so their latency overlaps it
    constexpr int K = 3;
    double lv[K][5], pv_[K], xv[K], rv[K];
    auto load_k = [&](int i0) {
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int i = i0 + u * 256;
            if (i < 3 * N) {
                const int ch = i / N, xx = i - ch * N;
                const double* lc = l + o + ch * nn + int64_t(j) * N + xx;
                const int64_t off = o + ch * nn + int64_t(j) * N + xx;
                lv[u][0] = lc[0];
                lv[u][1] = j > 0 ? lc[-N] : 0.0;
                lv[u][2] = j + 1 < N ? lc[N] : 0.0;
                lv[u][3] = xx > 0 ? lc[-1] : 0.0;
                lv[u][4] = xx + 1 < N ? lc[1] : 0.0;
                pv_[u] = p_new[off];
                xv[u] = x[off];
                rv[u] = r[off];
            }
        }
    };
    load_k(tid);
    T* g = reinterpret_cast<T*>(smem);
    char* sc = smem + lds_align(size_t(3) * N * sizeof(T));
    scatter_row<T, true, 256>(g, scatter_lds<T>(sc, N, 256), N, j, at<int>(plan, p.o_binstart),
                              at<vec4<T>>(plan, p.o_samp), at<int2>(plan, p.o_sidx),
                              reinterpret_cast<const vec2<T>*>(y + p.o_s), nullptr, tid, p.chan == 1,
                              chk_of(p, plan));
    // the sampling's scratch (at least 6 * 256 values of T after g) now holds the reductions
    double* red = reinterpret_cast<double*>(sc);
    tree_sum2(yy, ll, red);
    const double alpha = s.rr[nxt] / (inv_l * yy + reg * ll);
    double acc = 0.0;
    for (int i0 = tid; i0 < 3 * N; i0 += K * 256) {
        if (i0 != tid) load_k(i0);
#pragma unroll
        for (int u = 0; u < K; ++u) {
            const int i = i0 + u * 256;
            if (i < 3 * N) {
                const int ch = i / N, xx = i - ch * N;
                const int64_t off = o + ch * nn + int64_t(j) * N + xx;
                const double v = lv[u][0];
                double sl = 0.0;                                     // lap5's order
                if (j > 0) sl += lv[u][1] - v;
                if (j + 1 < N) sl += lv[u][2] - v;
                if (xx > 0) sl += lv[u][3] - v;
                if (xx + 1 < N) sl += lv[u][4] - v;
                const double q = inv_l * double(g[i]) + reg * (ch == 1 ? 2.0 : 1.0) * sl;
                x[off] = xv[u] + alpha * pv_[u];
                const double re = rv[u] - alpha * q;
                r[off] = re;
                acc += re * re;
            }
        }
    }
    acc = block_total(acc, red);
    if (tid == 0) s.part_r[int64_t(b) * kCoreParts + j] = acc;
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
    if (!chk_of(p, plan).time(k)) return;
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
