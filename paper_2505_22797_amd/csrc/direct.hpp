// Direct path of the operator for truncated kernels, plus the element-wise
// kernels shared by both paths (sampling bands from global memory, the
// denoiser step, permutations).
//
// conv_direct: out_ch[j][i] = sum_{|dx|,|dy|<=R} delta^2 K_ch(dx,dy) in[j-dy][i-dx]
// (eq. coreoperator as a Riemann sum, zero outside the grid).  A work-group
// computes a 16 x 16 output tile; its input tile with an R-halo sits in LDS.
// Lane l of every wave owns a 1 x 4 strip of outputs (row l/4, columns
// 4(l%4)..+3); the waves split the dy range (wave w takes dy = -R + w,
// -R + w + S, ...), so the tap address is uniform per wave and the taps come
// through scalar loads.  Along dx a sliding window of input values in
// registers gives 4 x COUT multiply-adds per LDS read.  The S wave partials
// are summed in wave order in LDS (deterministic).
//   CIN = 1, COUT = 3: the forward field (one input, three kernel channels)
//   CIN = 3, COUT = 1: the transpose (sum over channels; each K_ch is even)
//   CIN = 1, COUT = 1: the scalar convolution with the trace kernel
//                      kappa_h = K_xx + K_yy (eq. kernel:trace)
#pragma once
#include "common.hpp"
#include "sampling.hpp"

namespace mpik {

constexpr int kTile = 16;
constexpr int kStrip = 4;

__host__ __device__ constexpr int direct_row_len(int R) {
    // columns read: up to 12 + taps_w + 7 with taps_w <= 2R + 4
    return ((kTile + 2 * R + 12) + 3) / 4 * 4;
}

// One channel's input tile with its R-halo (zero outside the grid).
template <typename T>
__device__ __forceinline__ void load_tile(T* tile, const T* __restrict__ in, int N, int R, int y0, int x0,
                                          int row_len, int tid, int nt) {
    const int rows = kTile + 2 * R;
    const int total = rows * row_len;
    for (int idx = tid; idx < total; idx += nt) {
        const int ly = idx / row_len, lx = idx % row_len;
        const int gy = y0 - R + ly, gx = x0 - R + lx;
        T v = T(0);
        if (lx < kTile + 2 * R && gy >= 0 && gy < N && gx >= 0 && gx < N) v = in[int64_t(gy) * N + gx];
        tile[idx] = v;
    }
}

// EPI 0: out = conv;  1: out = c_in - tau * conv;  2: as 1 into the problem's
// work buffer u (COUT == 1 only for 1 and 2).  skip (optional): problems with a
// nonzero flag leave at once.
template <typename T, int CIN, int COUT, int S, int EPI>
__global__ void __launch_bounds__(64 * S) k_conv_direct(const Prob* __restrict__ P, const T* in, T* out,
                                                        const T* c_in, const double* __restrict__ taus,
                                                        const char* __restrict__ plan, int in_is_caller,
                                                        int out_is_caller, int dh, const int* __restrict__ skip) {
    static_assert(!(CIN == 1 && COUT == 1 && EPI != 0), "the trace convolution has no epilogue");
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.z];
    if (p.mode != 0 || p.slices != S || (skip && skip[blockIdx.z])) return;
    const T tau = EPI ? T(taus[blockIdx.z]) : T(0);
    const int N = p.n, R = p.radius, tw = p.taps_w;
    const int tiles = (N + kTile - 1) / kTile;
    const int ty0 = blockIdx.y * kTile, tx0 = blockIdx.x * kTile;
    if (blockIdx.x >= tiles || blockIdx.y >= tiles) return;
    // caller buffers are offset by the problem's element offset, work buffers
    // (passed as the work base) by the problem's field offset
    in = in_is_caller ? in + p.o_c : reinterpret_cast<const T*>(reinterpret_cast<const char*>(in) + p.w_g);
    if (EPI == 2) out = reinterpret_cast<T*>(reinterpret_cast<char*>(out) + p.w_u);
    else out = out_is_caller ? out + p.o_c : reinterpret_cast<T*>(reinterpret_cast<char*>(out) + p.w_g);
    if (c_in) c_in += p.o_c;
    const int row_len = direct_row_len(R);
    T* tile = reinterpret_cast<T*>(smem);
    const int tid = threadIdx.x;
    const int wave = uniform(tid / kWave), lane = tid % kWave;
    const int ly = lane / 4, sx = (lane % 4) * kStrip;
    const T* taps = at<T>(plan, dh ? p.o_taps_dh : p.o_taps);   // dK/dh for the h-derivative
    const int W = 2 * R + 1;
    T acc[COUT][kStrip];
#pragma unroll
    for (int o = 0; o < COUT; ++o)
#pragma unroll
        for (int w = 0; w < kStrip; ++w) acc[o][w] = T(0);
    // the input channels one after another through one LDS tile (a third of
    // the LDS of all three at once: four work-groups per CU instead of one)
    for (int ci = 0; ci < CIN; ++ci) {
        if (ci > 0) __syncthreads();              // every wave is done with the previous channel
        load_tile<T>(tile, in + int64_t(ci) * N * N, N, R, ty0, tx0, row_len, tid, 64 * S);
        __syncthreads();
        for (int dy = -R + wave; dy <= R; dy += S) {
            const int trow = (dy + R) * tw;
            const T* row = tile + (ly - dy + R) * row_len + sx;
            T x[8];
#pragma unroll
            for (int u = 0; u < 4; ++u) x[u] = row[u];
            for (int t0 = 0; t0 < tw; t0 += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) x[4 + u] = row[t0 + 4 + u];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (COUT == 3) {
                        const T k0 = taps[trow + t0 + u];
                        const T k1 = taps[W * tw + trow + t0 + u];
                        const T k2 = taps[2 * W * tw + trow + t0 + u];
#pragma unroll
                        for (int w = 0; w < kStrip; ++w) {
                            acc[0][w] += k0 * x[u + w];
                            acc[COUT > 1 ? 1 : 0][w] += k1 * x[u + w];
                            acc[COUT > 2 ? 2 : 0][w] += k2 * x[u + w];
                        }
                    } else if (CIN == 1) {   // trace kernel (the two diagonal channels), or K_xx for x-channel problems
                        const T k = p.chan == 1 ? taps[trow + t0 + u]
                                                : taps[trow + t0 + u] + taps[2 * W * tw + trow + t0 + u];
#pragma unroll
                        for (int w = 0; w < kStrip; ++w) acc[0][w] += k * x[u + w];
                    } else {
                        const T k = taps[ci * W * tw + trow + t0 + u];
#pragma unroll
                        for (int w = 0; w < kStrip; ++w) acc[0][w] += k * x[u + w];
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) x[u] = x[4 + u];
            }
        }
    }
    // fixed-order reduction over the S waves
    __syncthreads();
    T* red = tile;   // [S][64][COUT * 4]
#pragma unroll
    for (int o = 0; o < COUT; ++o)
#pragma unroll
        for (int w = 0; w < kStrip; ++w) red[(wave * kWave + lane) * COUT * kStrip + o * kStrip + w] = acc[o][w];
    __syncthreads();
    if (wave == 0) {
        const int gy = ty0 + ly;
#pragma unroll
        for (int o = 0; o < COUT; ++o) {
#pragma unroll
            for (int w = 0; w < kStrip; ++w) {
                T s = red[lane * COUT * kStrip + o * kStrip + w];
                for (int q = 1; q < S; ++q) s += red[(q * kWave + lane) * COUT * kStrip + o * kStrip + w];
                const int gx = tx0 + sx + w;
                if (gy < N && gx < N) {
                    const int64_t off = int64_t(o) * N * N + int64_t(gy) * N + gx;
                    if (EPI == 0) out[off] = s;
                    else out[off] = c_in[off] - tau * s;
                }
            }
        }
    }
}

// Bilinear gather + contraction for base-cell row b from a field in global
// memory ([3][N][N]): rows b and b+1 are staged in LDS first.
template <typename T, int MODE>
__global__ void __launch_bounds__(256) k_gather_rows(const Prob* __restrict__ P, GatherIO<T> io,
                                                     const char* __restrict__ plan, char* __restrict__ work) {
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.y];
    if (p.mode != 0) return;
    const T* G = at<T>(work, p.w_g);
    const int N = p.n, nb = p.nb, b = blockIdx.x;
    if (b >= nb) return;
    const int* binstart = at<int>(plan, p.o_binstart);
    int p0 = binstart[b * nb], p1 = binstart[(b + 1) * nb];
    const Chk ck = chk_of(p, plan).in_row(b);
    ck.range(p0, p1);
    if (p0 == p1) return;
    T* g0 = reinterpret_cast<T*>(smem);
    T* g1 = g0 + 3 * N;
    for (int i = threadIdx.x; i < 6 * N; i += blockDim.x) {
        const int half = i / (3 * N), rem = i % (3 * N), ch = rem / N, x = rem % N;
        g0[i] = G[int64_t(ch) * N * N + int64_t(b + half) * N + x];
    }
    __syncthreads();
    gather_band<T, MODE>(g0, g1, N, p0, p1, at<vec4<T>>(plan, p.o_samp), at<int2>(plan, p.o_sidx),
                         at<vec2<T>>(work, p.w_ysort), at<vec2<T>>(work, p.w_res),
                         io.out0 ? io.out0 + p.o_s : nullptr, io.in0 ? io.in0 + p.o_s : nullptr,
                         io.out1 ? io.out1 + p.o_s : nullptr, io.out2 ? io.out2 + p.o_s : nullptr,
                         io.f ? io.f + 9 * (p.o_s / 2) : nullptr, p.t,
                         p.o_dw ? at<vec2<T>>(plan, p.o_dw) : nullptr, p.chan == 1, threadIdx.x, blockDim.x, ck);
}

// Deterministic transpose sampling for one grid row into a field in global
// memory ([3][N][N]).
template <typename T, bool SORTED>
__global__ void __launch_bounds__(256) k_scatter_rows(const Prob* __restrict__ P, const T* __restrict__ s,
                                                      const char* __restrict__ plan, char* __restrict__ work) {
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.y];
    if (p.mode != 0) return;
    T* G = at<T>(work, p.w_g);
    const int N = p.n, j = blockIdx.x;
    if (j >= N) return;
    T* g = reinterpret_cast<T*>(smem);
    char* sc = smem + lds_align(size_t(3) * N * sizeof(T));
    const T* sp = s ? s + p.o_s : nullptr;
    // SORTED: the signal in cell order, from s when given, else the problem's residual in work
    const vec2<T>* ys = (SORTED && sp) ? reinterpret_cast<const vec2<T>*>(sp) : at<vec2<T>>(work, p.w_res);
    scatter_row<T, SORTED, 256>(g, scatter_lds<T>(sc, N, 256), N, j, at<int>(plan, p.o_binstart),
                                at<vec4<T>>(plan, p.o_samp), at<int2>(plan, p.o_sidx), ys, sp, threadIdx.x,
                                p.chan == 1, chk_of(p, plan));
    for (int i = threadIdx.x; i < 3 * N; i += blockDim.x) {
        const int ch = i / N, x = i % N;
        G[int64_t(ch) * N * N + int64_t(j) * N + x] = g[i];
    }
}

// ysort[p] = s[k(p)]: the measured signal in cell order.
template <typename T>
__global__ void k_permute_signal(const Prob* __restrict__ P, const T* __restrict__ s, const char* __restrict__ plan,
                                 char* __restrict__ work) {
    const Prob& p = P[blockIdx.y];
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= p.t) return;
    const int k = at<int2>(plan, p.o_sidx)[i].y;
    if (!chk_of(p, plan).time(k)) return;
    const T* sp = s + p.o_s;
    vec2<T> y;
    y.x = sp[2 * k];
    y.y = sp[2 * k + 1];
    at<vec2<T>>(work, p.w_ysort)[i] = y;
}

// c = D(u): separable Gaussian (weights w[0..2r], zero padding), rows then
// columns, on a 32 x 32 output tile with an r-halo in LDS.
constexpr int kDnTile = 32;
constexpr int kDnMaxR = 8;

// u is read from the problem's work buffer, or from the caller's buffer u_in
// (concentration-shaped) when that is given.  RAD: the half-width r, fixed
// per instance so that every loop has a fixed trip count.  256 threads as 32
// columns x 8 rows: every load, pass and store walks whole tile rows, so
// consecutive threads touch consecutive addresses and no index needs a
// division; all of a thread's loads are in flight before its first store to
// LDS; the weights wait in LDS.  Each output sums its taps in the order
// k = 0..2r in both passes.
template <typename T, int RAD>
__global__ void __launch_bounds__(256) k_denoise(const Prob* __restrict__ P, const char* __restrict__ work,
                                                 const T* __restrict__ u_in, T* __restrict__ c,
                                                 const double* __restrict__ wts) {
    constexpr int L = kDnTile + 2 * RAD;           // the halo tile's side
    constexpr int RY = 256 / kDnTile;              // tile rows per pass of the work-group
    constexpr int RI = (L + RY - 1) / RY, CJ = (L + kDnTile - 1) / kDnTile;
    static_assert(256 % kDnTile == 0 && RAD >= 0 && RAD <= kDnMaxR, "the launch is 256 threads, r <= 8");
    __shared__ T a[L * L];
    __shared__ T b[kDnTile * L];
    __shared__ T w[2 * RAD + 1];
    const Prob& p = P[blockIdx.z];
    const int N = p.n;
    const int y0 = blockIdx.y * kDnTile, x0 = blockIdx.x * kDnTile;
    if (y0 >= N || x0 >= N) return;
    const T* up = u_in ? u_in + p.o_c : at<T>(work, p.w_u);
    T* cp = c + p.o_c;
    const int tx = threadIdx.x % kDnTile, ty = threadIdx.x / kDnTile;
    if (int(threadIdx.x) <= 2 * RAD) w[threadIdx.x] = T(wts[threadIdx.x]);
    T v[RI][CJ];
#pragma unroll
    for (int i = 0; i < RI; ++i) {
        const int ly = ty + i * RY, gy = y0 - RAD + ly;
#pragma unroll
        for (int j = 0; j < CJ; ++j) {
            const int lx = tx + j * kDnTile, gx = x0 - RAD + lx;
            v[i][j] = (ly < L && lx < L && gy >= 0 && gy < N && gx >= 0 && gx < N) ? up[int64_t(gy) * N + gx] : T(0);
        }
    }
#pragma unroll
    for (int i = 0; i < RI; ++i)
#pragma unroll
        for (int j = 0; j < CJ; ++j) {
            const int ly = ty + i * RY, lx = tx + j * kDnTile;
            if (ly < L && lx < L) a[ly * L + lx] = v[i][j];
        }
    __syncthreads();
    // vertical pass (over y) first: b[ly][x] for ly in [0, 32), then horizontal
#pragma unroll
    for (int i = 0; i < kDnTile / RY; ++i)
#pragma unroll
        for (int j = 0; j < CJ; ++j) {
            const int ly = ty + i * RY, lx = tx + j * kDnTile;
            if (lx < L) {
                T s = T(0);
#pragma unroll
                for (int k = 0; k <= 2 * RAD; ++k) s += w[k] * a[(ly + k) * L + lx];
                b[ly * L + lx] = s;
            }
        }
    __syncthreads();
    const int gx = x0 + tx;
#pragma unroll
    for (int i = 0; i < kDnTile / RY; ++i) {
        const int ly = ty + i * RY, gy = y0 + ly;
        T s = T(0);
#pragma unroll
        for (int k = 0; k <= 2 * RAD; ++k) s += w[k] * b[ly * L + tx + k];
        if (gy < N && gx < N) cp[int64_t(gy) * N + gx] = s;
    }
}

// Launches k_denoise with the instance of half-width rad (0..kDnMaxR; the
// callers check the range).
template <typename T>
void launch_denoise(dim3 grid, hipStream_t st, const Prob* P, const char* work, const T* u_in, T* c,
                    const double* wts, int rad) {
    switch (rad) {
#define MPIK_DN_CASE(R) \
    case R: k_denoise<T, R><<<grid, 256, 0, st>>>(P, work, u_in, c, wts); break;
        MPIK_DN_CASE(0) MPIK_DN_CASE(1) MPIK_DN_CASE(2) MPIK_DN_CASE(3) MPIK_DN_CASE(4)
        MPIK_DN_CASE(5) MPIK_DN_CASE(6) MPIK_DN_CASE(7) MPIK_DN_CASE(8)
#undef MPIK_DN_CASE
        default: break;
    }
}

// Deterministic per-problem dot products: out[b] = sum_i a_b[i] b_b[i] in
// float64, in two launches.  k_dot_part: grid (kDotParts, problems) of 256
// threads; part q sums a fixed contiguous slice of the problem's elements
// (thread-strided inside the slice, then a fixed tree) into part[b][q].
// k_dot_final: one work-group per problem adds its kDotParts partials by a
// fixed tree (and to out[b] when accumulating).  space 0: signal arrays
// ([T][2]; comp 0 = x components only, 1 = y only, 2 = both); space 1:
// concentration arrays ([N][N]).
constexpr int kDotParts = 64;

template <typename T>
__global__ void __launch_bounds__(256) k_dot_part(const Prob* __restrict__ P, const T* __restrict__ a,
                                                  const T* __restrict__ bb, int space, int comp,
                                                  double* __restrict__ part) {
    __shared__ double red[256];
    const Prob& p = P[blockIdx.y];
    const int tid = threadIdx.x;
    int64_t n, off, stride = 1, first = 0;
    if (space == 0) {
        off = p.o_s;
        n = 2 * p.t;
        if (comp != 2) { stride = 2; first = comp; }
    } else {
        off = p.o_c;
        n = int64_t(p.n) * p.n;
    }
    const int64_t m = (n - first + stride - 1) / stride;          // elements taken
    const int64_t per = (m + kDotParts - 1) / kDotParts;
    const int64_t lo = min(m, per * blockIdx.x), hi = min(m, lo + per);
    double acc = 0.0;
    for (int64_t e = lo + tid; e < hi; e += 256) {
        const int64_t i = off + first + e * stride;
        acc += double(a[i]) * double(bb[i]);
    }
    red[tid] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) part[int64_t(blockIdx.y) * kDotParts + blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kDotParts) k_dot_final(const double* __restrict__ part, double* __restrict__ out,
                                                        int accumulate) {
    __shared__ double red[kDotParts];
    const int tid = threadIdx.x;
    red[tid] = part[int64_t(blockIdx.x) * kDotParts + tid];
    __syncthreads();
    for (int w = kDotParts / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) out[blockIdx.x] = (accumulate ? out[blockIdx.x] : 0.0) + red[0];
}

}  // namespace mpik
