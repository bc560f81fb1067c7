// FFT path of the operator for wide kernels.  The linear convolution with the
// square-windowed kernel is a circular one on an M x M grid (M a power of two
// >= N + R), with the input zero-padded and the output cropped to N x N.
// The kernel spectra are real (K_xx, K_yy even, K_xy odd in each axis), so
// every channel is a real multiplier on the spectrum of c.
//
// Forward (c -> s), three launches:
//   fwd_rows : pairs of real rows of c as one complex row FFT -> half spectra,
//              stored column-major T1[kx][row]
//   fwd_cols : per column kx: forward column FFT, times the three channel
//              spectra, three inverse column FFTs cropped to N rows -> T2[ch][row][kx]
//   fwd_rows_gather : per base-cell row b: inverse row FFTs of rows b, b+1 for
//              the three channels (two real rows per complex FFT), then the
//              bilinear gather and velocity contraction of the row's samples.
// Transpose (s -> c), three launches:
//   adj_scatter_row : per grid row: deterministic transpose sampling into LDS,
//              then the row FFTs of the three channels -> T1[ch][kx][row]
//   adj_cols : per column: three forward column FFTs, multiply-accumulate the
//              channel spectra, one inverse column FFT cropped to N rows
//   adj_rows : per pair of rows: inverse row FFT -> c, with an optional fused
//              gradient-step epilogue.
// Work-groups are one to three 64-lane waves; each wave owns one FFT line.
#pragma once
#include "common.hpp"
#include "sampling.hpp"

namespace mpik {

template <typename T, int M> struct RowSmem {      // fwd_rows, adj_rows: one wave
    cx<T> tw[M];
    cx<T> buf[2][M];
};
template <typename T, int M> struct ColSmem {      // fwd_cols, adj_cols: three waves
    cx<T> tw[M];
    cx<T> buf[8][M];
};
template <typename T, int M> struct GatherSmem {   // fwd_rows_gather: three waves
    cx<T> tw[M];
    cx<T> buf[6][M];
    T g[6 * M];
};
template <typename T, int M> struct ScatterRowSmem {   // adj_scatter_row: four waves
    cx<T> tw[M];
    T g[3 * M];
    union {                     // the sampling transpose and the row FFTs run one after the other
        ScatterSmem<T, 256, M> sc;
        cx<T> buf[4][M];
    };
};

template <typename T, int M>
__device__ __forceinline__ void load_twiddles(cx<T>* tw_s, const char* plan, const Prob& p, int tid, int nt) {
    const cx<T>* tw = at<cx<T>>(plan, p.o_tw);
    for (int i = tid; i < M; i += nt) tw_s[i] = tw[i];
}

// spectrum value of channel ch at (kx, ky), kx in [0, M/2], ky in [0, M)
template <typename T, int M>
__device__ __forceinline__ T spec_at(const T* __restrict__ spec, int ch, int kx, int ky) {
    constexpr int H = M / 2 + 1;
    const bool up = ky > M / 2;
    const int kq = up ? M - ky : ky;
    const T v = spec[(ch * H + kx) * H + kq];
    return (ch == 1 && up) ? -v : v;
}

// Full-length spectrum Z = A + iB of the complex row a + ib from the half
// spectra A, B of two real rows.
template <typename T, int M>
__device__ __forceinline__ cx<T> pair_spectrum(const cx<T>* __restrict__ ra, const cx<T>* __restrict__ rb,
                                               int kx, bool two) {
    cx<T> A, B{T(0), T(0)};
    if (kx <= M / 2) {
        A = ra[kx];
        if (two) B = rb[kx];
        if (kx == 0 || kx == M / 2) { A.y = T(0); B.y = T(0); }   // real at DC and Nyquist
    } else {
        A = cconj(ra[M - kx]);
        if (two) B = cconj(rb[M - kx]);
    }
    return cx<T>{A.x - B.y, A.y + B.x};
}

// Half spectra of two real rows a, b from the spectrum Z of a + ib:
// A = (Z_k + conj Z_-k)/2, B = (Z_k - conj Z_-k)/(2i), k in [0, M/2].
template <typename T, int M>
__device__ __forceinline__ void split_pair(const cx<T>* Z, int k, cx<T>& A, cx<T>& B) {
    const cx<T> z = Z[k], zc = cconj(Z[(M - k) & (M - 1)]);
    const cx<T> s = cadd(z, zc), d = csub(z, zc);
    A = cx<T>{s.x * T(0.5), s.y * T(0.5)};
    B = cx<T>{d.y * T(0.5), -d.x * T(0.5)};
}

// ---------------------------------------------------------------- forward ---
template <typename T, int M>
__device__ void fwd_rows_body(const Prob& p, const T* __restrict__ c, const char* __restrict__ plan,
                              char* __restrict__ work, char* smem) {
    auto& sm = *reinterpret_cast<RowSmem<T, M>*>(smem);
    constexpr int H = M / 2 + 1;
    const int N = p.n, q = blockIdx.x, lane = threadIdx.x;
    const int r0 = 2 * q, r1 = 2 * q + 1;
    if (r0 >= N) return;
    const bool two = r1 < N;
    load_twiddles<T, M>(sm.tw, plan, p, lane, kWave);
    const T* c0 = c + int64_t(r0) * N;
    const T* c1 = c + int64_t(r1) * N;
    for (int i = lane; i < M; i += kWave) {
        cx<T> z{T(0), T(0)};
        if (i < N) {
            z.x = c0[i];
            if (two) z.y = c1[i];
        }
        sm.buf[0][i] = z;
    }
    __syncthreads();
    const cx<T>* Z = fft_line<T, false, M>(sm.buf[0], sm.buf[1], sm.tw, lane, true);
    cx<T>* t1 = at<cx<T>>(work, p.w_t1);
    for (int k = lane; k < H; k += kWave) {
        cx<T> A, B;
        split_pair<T, M>(Z, k, A, B);
        t1[int64_t(k) * N + r0] = A;
        if (two) t1[int64_t(k) * N + r1] = B;
    }
}

template <typename T, int M>
__device__ void fwd_cols_body(const Prob& p, const char* __restrict__ plan, char* __restrict__ work, char* smem) {
    auto& sm = *reinterpret_cast<ColSmem<T, M>*>(smem);
    constexpr int H = M / 2 + 1;
    const int N = p.n, kx = blockIdx.x;
    if (kx >= H) return;
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    load_twiddles<T, M>(sm.tw, plan, p, tid, 3 * kWave);
    const cx<T>* t1 = at<cx<T>>(work, p.w_t1) + int64_t(kx) * N;
    for (int i = tid; i < M; i += 3 * kWave) sm.buf[0][i] = (i < N) ? t1[i] : cx<T>{T(0), T(0)};
    __syncthreads();
    const cx<T>* C = fft_line<T, false, M>(sm.buf[0], sm.buf[1], sm.tw, lane, wave == 0);
    const T* spec = at<T>(plan, p.o_spec);
    cx<T>* a = sm.buf[2 + 2 * wave];
    for (int ky = lane; ky < M; ky += kWave) a[ky] = cscale(C[ky], spec_at<T, M>(spec, wave, kx, ky));
    __syncthreads();
    const cx<T>* G = fft_line<T, true, M>(a, sm.buf[3 + 2 * wave], sm.tw, lane, true);
    cx<T>* t2 = at<cx<T>>(work, p.w_t2) + int64_t(wave) * N * H;
    for (int j = lane; j < N; j += kWave) t2[int64_t(j) * H + kx] = G[j];
}

template <typename T, int M, bool RESID>
__device__ void fwd_rows_gather_body(const Prob& p, T* __restrict__ s, const char* __restrict__ plan,
                                     char* __restrict__ work, char* smem) {
    auto& sm = *reinterpret_cast<GatherSmem<T, M>*>(smem);
    constexpr int H = M / 2 + 1;
    const int N = p.n, nb = p.nb, b = blockIdx.x;
    if (b >= nb) return;
    const int* binstart = at<int>(plan, p.o_binstart);
    const int p0 = binstart[b * nb], p1 = binstart[(b + 1) * nb];
    if (p0 == p1) return;
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    load_twiddles<T, M>(sm.tw, plan, p, tid, 3 * kWave);
    const cx<T>* t2 = at<cx<T>>(work, p.w_t2) + int64_t(wave) * N * H;
    const cx<T>* ra = t2 + int64_t(b) * H;
    const cx<T>* rb = t2 + int64_t(b + 1) * H;
    cx<T>* a = sm.buf[2 * wave];
    for (int kx = lane; kx < M; kx += kWave) a[kx] = pair_spectrum<T, M>(ra, rb, kx, true);
    __syncthreads();
    const cx<T>* Gz = fft_line<T, true, M>(a, sm.buf[2 * wave + 1], sm.tw, lane, true);
    T* g0 = sm.g;            // row b:   [ch][N]
    T* g1 = sm.g + 3 * N;    // row b+1: [ch][N]
    for (int i = lane; i < N; i += kWave) {
        g0[wave * N + i] = Gz[i].x;
        g1[wave * N + i] = Gz[i].y;
    }
    __syncthreads();
    gather_band<T, RESID>(g0, g1, N, p0, p1, at<vec4<T>>(plan, p.o_samp), at<int2>(plan, p.o_sidx),
                          at<vec2<T>>(work, p.w_ysort), at<vec2<T>>(work, p.w_res), s, tid, 3 * kWave);
}

// ----------------------------------------------------------------- adjoint ---
// One grid row j per work-group of four waves: the deterministic transpose
// sampling of the row's cells into LDS, then the row FFTs of its three
// channels: wave 0 transforms xx + i xy (split into the two half spectra),
// wave 1 transforms yy alone.
template <typename T, int M, bool SORTED>
__device__ void adj_scatter_row_body(const Prob& p, const T* __restrict__ s, const char* __restrict__ plan,
                                     char* __restrict__ work, char* smem) {
    auto& sm = *reinterpret_cast<ScatterRowSmem<T, M>*>(smem);
    constexpr int H = M / 2 + 1;
    const int N = p.n, j = blockIdx.x;
    if (j >= N) return;
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    load_twiddles<T, M>(sm.tw, plan, p, tid, 4 * kWave);
    scatter_row<T, SORTED, 256, M>(sm.g, sm.sc, N, j, at<int>(plan, p.o_binstart), at<vec4<T>>(plan, p.o_samp),
                                   at<int2>(plan, p.o_sidx), at<vec2<T>>(work, p.w_res), s, tid);
    const bool active = wave < 2;
    cx<T>* a = sm.buf[2 * (wave & 1)];
    if (active) {
        const T* re = sm.g + (wave == 0 ? 0 : 2 * N);
        const T* im = sm.g + N;
        for (int i = lane; i < M; i += kWave) {
            cx<T> z{T(0), T(0)};
            if (i < N) {
                z.x = re[i];
                if (wave == 0) z.y = im[i];
            }
            a[i] = z;
        }
    }
    __syncthreads();
    const cx<T>* Z = fft_line<T, false, M>(a, sm.buf[2 * (wave & 1) + 1], sm.tw, lane, active);
    if (!active) return;
    cx<T>* t1 = at<cx<T>>(work, p.w_t1);
    for (int k = lane; k < H; k += kWave) {
        if (wave == 0) {
            cx<T> A, B;
            split_pair<T, M>(Z, k, A, B);
            t1[int64_t(k) * N + j] = A;
            t1[(int64_t(H) + k) * N + j] = B;
        } else {
            t1[(int64_t(2) * H + k) * N + j] = Z[k];
        }
    }
}

template <typename T, int M>
__device__ void adj_cols_body(const Prob& p, const char* __restrict__ plan, char* __restrict__ work, char* smem) {
    auto& sm = *reinterpret_cast<ColSmem<T, M>*>(smem);
    constexpr int H = M / 2 + 1;
    constexpr int par = FftPasses<M>::count & 1;    // result of a line lands in buf[2w + par]
    const int N = p.n, kx = blockIdx.x;
    if (kx >= H) return;
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    load_twiddles<T, M>(sm.tw, plan, p, tid, 3 * kWave);
    const cx<T>* t1 = at<cx<T>>(work, p.w_t1) + (int64_t(wave) * H + kx) * N;
    cx<T>* a = sm.buf[2 * wave];
    for (int i = lane; i < M; i += kWave) a[i] = (i < N) ? t1[i] : cx<T>{T(0), T(0)};
    __syncthreads();
    cx<T>* C = fft_line<T, false, M>(a, sm.buf[2 * wave + 1], sm.tw, lane, true);
    const T* spec = at<T>(plan, p.o_spec);
    for (int ky = lane; ky < M; ky += kWave) C[ky] = cscale(C[ky], spec_at<T, M>(spec, wave, kx, ky));
    __syncthreads();
    // fixed-order channel sum (xx + xy) + yy into wave 0's free line
    const cx<T>* C0 = sm.buf[par];
    const cx<T>* C1 = sm.buf[2 + par];
    const cx<T>* C2 = sm.buf[4 + par];
    cx<T>* X = sm.buf[1 - par];
    cx<T>* Y = sm.buf[6];
    for (int ky = tid; ky < M; ky += 3 * kWave) X[ky] = cadd(cadd(C0[ky], C1[ky]), C2[ky]);
    __syncthreads();
    const cx<T>* Cc = fft_line<T, true, M>(X, Y, sm.tw, lane, wave == 0);
    cx<T>* t2 = at<cx<T>>(work, p.w_t2);
    for (int j = tid; j < N; j += 3 * kWave) t2[int64_t(j) * H + kx] = Cc[j];
}

// EPI 0: c_out = A^T s;  1, 2: c_out = c_in - tau * A^T r (c_in may alias c_out)
template <typename T, int M, int EPI>
__device__ void adj_rows_body(const Prob& p, T* c_out, const T* c_in, T tau,
                              const char* __restrict__ plan, char* __restrict__ work, char* smem) {
    auto& sm = *reinterpret_cast<RowSmem<T, M>*>(smem);
    constexpr int H = M / 2 + 1;
    const int N = p.n, q = blockIdx.x, lane = threadIdx.x;
    const int r0 = 2 * q, r1 = 2 * q + 1;
    if (r0 >= N) return;
    const bool two = r1 < N;
    load_twiddles<T, M>(sm.tw, plan, p, lane, kWave);
    const cx<T>* t2 = at<cx<T>>(work, p.w_t2);
    const cx<T>* ra = t2 + int64_t(r0) * H;
    const cx<T>* rb = t2 + int64_t(two ? r1 : r0) * H;
    for (int kx = lane; kx < M; kx += kWave) sm.buf[0][kx] = pair_spectrum<T, M>(ra, rb, kx, two);
    __syncthreads();
    const cx<T>* z = fft_line<T, true, M>(sm.buf[0], sm.buf[1], sm.tw, lane, true);
    for (int i = lane; i < N; i += kWave) {
        const T v0 = z[i].x, v1 = z[i].y;
        const int64_t o0 = int64_t(r0) * N + i, o1 = int64_t(r1) * N + i;
        if (EPI == 0) {
            c_out[o0] = v0;
            if (two) c_out[o1] = v1;
        } else {
            c_out[o0] = c_in[o0] - tau * v0;
            if (two) c_out[o1] = c_in[o1] - tau * v1;
        }
    }
}

// ------------------------------------------------------------- launchers ---
#define MPIK_DISPATCH_M(M_, BODY)                         \
    switch (M_) {                                         \
        case 64: { constexpr int MM = 64; BODY; } break;  \
        case 128: { constexpr int MM = 128; BODY; } break; \
        case 256: { constexpr int MM = 256; BODY; } break; \
        case 512: { constexpr int MM = 512; BODY; } break; \
        case 1024: { constexpr int MM = 1024; BODY; } break; \
        default: break;                                   \
    }

template <typename T>
__global__ void __launch_bounds__(64) k_fwd_rows(const Prob* __restrict__ P, const T* __restrict__ c,
                                                 const char* __restrict__ plan, char* __restrict__ work) {
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.y];
    if (p.mode != 1) return;
    MPIK_DISPATCH_M(p.m, (fwd_rows_body<T, MM>(p, c + p.o_c, plan, work, smem)));
}

template <typename T>
__global__ void __launch_bounds__(192) k_fwd_cols(const Prob* __restrict__ P, const char* __restrict__ plan,
                                                  char* __restrict__ work) {
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.y];
    if (p.mode != 1) return;
    MPIK_DISPATCH_M(p.m, (fwd_cols_body<T, MM>(p, plan, work, smem)));
}

template <typename T, bool RESID>
__global__ void __launch_bounds__(192) k_fwd_rows_gather(const Prob* __restrict__ P, T* __restrict__ s,
                                                         const char* __restrict__ plan, char* __restrict__ work) {
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.y];
    if (p.mode != 1) return;
    MPIK_DISPATCH_M(p.m, (fwd_rows_gather_body<T, MM, RESID>(p, s + p.o_s, plan, work, smem)));
}

template <typename T, bool SORTED>
__global__ void __launch_bounds__(256) k_adj_scatter_row(const Prob* __restrict__ P, const T* __restrict__ s,
                                                         const char* __restrict__ plan, char* __restrict__ work) {
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.y];
    if (p.mode != 1) return;
    MPIK_DISPATCH_M(p.m, (adj_scatter_row_body<T, MM, SORTED>(p, s + p.o_s, plan, work, smem)));
}

template <typename T>
__global__ void __launch_bounds__(192) k_adj_cols(const Prob* __restrict__ P, const char* __restrict__ plan,
                                                  char* __restrict__ work) {
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.y];
    if (p.mode != 1) return;
    MPIK_DISPATCH_M(p.m, (adj_cols_body<T, MM>(p, plan, work, smem)));
}

template <typename T, int EPI>
__global__ void __launch_bounds__(64) k_adj_rows(const Prob* __restrict__ P, T* c_out, const T* c_in,
                                                 const double* __restrict__ taus, const char* __restrict__ plan,
                                                 char* __restrict__ work) {
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.y];
    if (p.mode != 1) return;
    const T tau = EPI ? T(taus[blockIdx.y]) : T(0);
    // EPI 2 writes the step into the problem's work buffer u (before the denoiser)
    T* out = EPI == 2 ? at<T>(work, p.w_u) : c_out + p.o_c;
    MPIK_DISPATCH_M(p.m, (adj_rows_body<T, MM, EPI>(p, out, c_in + p.o_c, tau, plan, work, smem)));
}

}  // namespace mpik
