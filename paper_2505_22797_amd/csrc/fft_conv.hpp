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
//              then the row FFTs of the three channels -> T1[ch][row][kx]
//   adj_cols : per column: three forward column FFTs, multiply-accumulate the
//              channel spectra, one inverse column FFT cropped to N rows
//   adj_rows : per pair of rows: inverse row FFT -> c, with an optional fused
//              gradient-step epilogue.
// Rows of T1[ch][row][.] and T2[ch][row][.] are spec_pitch(M) elements apart
// (M/2 + 1 rounded up to four), so that the column stages' four-column runs
// are 32-byte aligned.
// Every FFT line belongs to one 64-lane wave (in place in LDS, no work-group
// barrier inside the transform).  The column stages come in two shapes: SPLIT
// spreads one column over three waves (shortest latency for few problems);
// otherwise each wave owns a whole column (four columns per work-group, most
// columns in flight for large batches).
#pragma once
#include "common.hpp"
#include "sampling.hpp"

namespace mpik {

template <typename T, int M> struct RowSmem {      // fwd_rows, adj_rows: four waves, a row pair each
    cx<T> tw[M];
    cx<T> line[4][M];
};
template <typename T, int M> struct ColSmem {      // column stages: four lines + a shared one
    cx<T> tw[M];
    cx<T> c[M];
    cx<T> line[4][M];
};
// The transpose column stage at M = 512 in the four-column shape: four
// exchange buffers, the twiddle table and one channel's four columns, each
// padded to SN elements (four more than N, so that the staging stores of four
// columns fall on different banks).
__host__ __device__ constexpr int adj_cols_stage_stride(int N) { return N + 4; }
template <typename T>
__host__ __device__ constexpr size_t adj_cols_smem_bytes(int N) {
    return sizeof(cx<T>) * (size_t(4) * kXbStride<T> + 512 + size_t(4) * adj_cols_stage_stride(N));
}
// fwd_rows_gather: twiddles, three FFT lines, then rows b, b+1 of the three
// channels (6N values).
template <typename T, int M> struct GatherSmem {
    cx<T> tw[M];
    cx<T> line[3][M];
    T g[1];
};
template <typename T, int M>
__host__ __device__ constexpr size_t gather_smem_bytes(int N) {
    return sizeof(GatherSmem<T, M>) + size_t(6) * N * sizeof(T);
}
// adj_scatter_row: a region used first by the sampling transpose and then by
// the twiddles and the two row-FFT lines (the twiddles wait in registers
// meanwhile), or by the two waves' exchange buffers at M = 512 in float32.
// The row's three channels (3N values) are assembled once the transpose's
// per-thread partial sums (first_val) are consumed, so they take that part of
// the region when the transforms stay clear of it, and otherwise a part of
// their own in front of the region.
template <typename T, int M>
__host__ __device__ constexpr size_t scatter_fft_bytes() {
    return (M == 512 && sizeof(T) == 4) ? 2 * kXbStride<T> * sizeof(cx<T>) : 3 * sizeof(cx<T>) * M;
}
template <typename T, int M>
__host__ __device__ constexpr bool scatter_g_in_region(int N) {
    return scatter_fft_bytes<T, M>() <= scatter_lds_first_val<T>(N, 256) && 3 * N <= 6 * 256;
}
template <typename T, int M>
__host__ __device__ constexpr size_t scatter_row_smem_bytes(int N) {
    const size_t fft = scatter_fft_bytes<T, M>(), sc = scatter_lds_bytes<T>(N, 256);
    const size_t region = fft > sc ? fft : sc;
    return scatter_g_in_region<T, M>(N) ? region : lds_align(size_t(3) * N * sizeof(T)) + region;
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
// spectra A, B of two real rows (B = 0 when `two` is false).
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

// Loads issued ahead of the work-group barrier that publishes the twiddles: a
// kernel first puts its share of the twiddles and its input line in
// registers, so that every load of the work-group is in flight at once, and
// only then waits and moves them to LDS.
template <typename T, int M, int NT> struct TwiddleRegs {
    static constexpr int PER = (M + NT - 1) / NT;
    cx<T> v[PER];
    __device__ __forceinline__ void load(const char* plan, const Prob& p, int tid) {
        const cx<T>* tw = at<cx<T>>(plan, p.o_tw);
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if (M % NT == 0 || tid + q * NT < M) v[q] = tw[tid + q * NT];
    }
    __device__ __forceinline__ void store(cx<T>* tw_s, int tid) const {
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if (M % NT == 0 || tid + q * NT < M) tw_s[tid + q * NT] = v[q];
    }
};

// The half-spectrum values pair_spectrum reads for kx = lane + 64 m, loaded
// ahead; spectrum(m) then gives the same value as pair_spectrum(ra, rb, kx).
template <typename T, int M> struct PairRegs {
    static constexpr int PL = M / kWave;
    cx<T> a[PL], b[PL];
    __device__ __forceinline__ void load(const cx<T>* __restrict__ ra, const cx<T>* __restrict__ rb, bool two,
                                         int lane) {
#pragma unroll
        for (int m = 0; m < PL; ++m) {
            const int kx = lane + m * kWave, k = kx <= M / 2 ? kx : M - kx;
            a[m] = ra[k];
            b[m] = two ? rb[k] : cx<T>{T(0), T(0)};
        }
    }
    __device__ __forceinline__ cx<T> spectrum(int m, int lane) const {
        const int kx = lane + m * kWave;
        cx<T> A = a[m], B = b[m];
        if (kx <= M / 2) {
            if (kx == 0 || kx == M / 2) { A.y = T(0); B.y = T(0); }   // real at DC and Nyquist
        } else {
            A = cconj(A);
            B = cconj(B);
        }
        return cx<T>{A.x - B.y, A.y + B.x};
    }
};

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
    const int N = p.n, tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const int unit = xcd_unit(blockIdx.x, (N + 7) / 8);   // four row pairs per work-group
    if (unit < 0) return;
    TwiddleRegs<T, M, 4 * kWave> twr;
    twr.load(plan, p, tid);
    const int q = 4 * unit + wave;
    const int r0 = 2 * q, r1 = 2 * q + 1;
    const bool active = r0 < N, two = r1 < N;
    constexpr int PL = M / kWave;
    cx<T> x[PL];
    if (active) {
        const T* c0 = c + int64_t(r0) * N;
        const T* c1 = c + int64_t(r1) * N;
#pragma unroll
        for (int m = 0; m < PL; ++m) {
            const int i = lane + m * kWave;
            cx<T> z{T(0), T(0)};
            if (i < N) {
                z.x = c0[i];
                if (two) z.y = c1[i];
            }
            x[m] = z;
        }
    }
    twr.store(sm.tw, tid);
    __syncthreads();
    cx<T>* line = sm.line[wave];
    if (active) {
        if constexpr (M == 512 && sizeof(T) == 4) {
            // register-resident transform with the twiddles read from the LDS
            // table (registers for them would cost occupancy); the wave's
            // line holds the exchange, then the spectrum in natural order
            static_assert(XbLayout<T>::kSlots <= M, "exchange exceeds the line");
            Fft512TwLds<T> tl;
            tl.init(sm.tw, lane);
            fft512_regs<T, false>(x, line, tl, lane);
#pragma unroll
            for (int m = 0; m < PL; ++m) line[lane + m * kWave] = x[m];
        } else {
#pragma unroll
            for (int m = 0; m < PL; ++m) line[lane + m * kWave] = x[m];
            wave_sync();
            fft_wave<T, false, M>(line, sm.tw, lane);
        }
    }
    __syncthreads();
    // the work-group's eight rows go out together: T1[k][row0 .. row0+7], so
    // eight consecutive threads write one contiguous 64-byte run
    cx<T>* t1 = at<cx<T>>(work, p.w_t1);
    const int row0 = 8 * unit;
    for (int i = tid; i < 8 * H; i += 4 * kWave) {
        const int k = i >> 3, r = i & 7;
        if (row0 + r >= N) continue;
        cx<T> A, B;
        split_pair<T, M>(sm.line[r >> 1], k, A, B);
        const bool odd = r & 1;
        t1[int64_t(k) * N + row0 + r] = cx<T>{odd ? B.x : A.x, odd ? B.y : A.y};
    }
}

// Column kx: forward column FFT of T1[kx][.] (zero-padded), then for each
// channel the product with its spectrum, the inverse FFT and rows 0..N-1 of
// the result to T2[ch][row][kx].  TRACE (four-column shape): one channel, the
// trace kernel kappa_h = K_xx + K_yy (eq. kernel:trace), whose spectrum is the
// sum of the two diagonal channels' spectra.
template <typename T, int M, bool SPLIT, bool TRACE = false>
__device__ void fwd_cols_body(const Prob& p, const char* __restrict__ plan, char* __restrict__ work, char* smem,
                              int dh) {
    static_assert(!(SPLIT && TRACE), "the trace convolution runs in the four-column shape");
    auto& sm = *reinterpret_cast<ColSmem<T, M>*>(smem);
    constexpr int H = M / 2 + 1;
    constexpr int HP = spec_pitch(M);   // row pitch of T1[ch][row] and T2[ch][row]
    const int N = p.n, tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const T* spec = at<T>(plan, dh ? p.o_spec_dh : p.o_spec);   // dK/dh for the h-derivative
    cx<T>* t2 = at<cx<T>>(work, p.w_t2);
    if (SPLIT) {                                    // one column, waves 0..2
        const int kx = xcd_unit(blockIdx.x, H);
        if (kx < 0) return;
        TwiddleRegs<T, M, 3 * kWave> twr;
        twr.load(plan, p, tid);
        const cx<T>* t1 = at<cx<T>>(work, p.w_t1) + int64_t(kx) * N;
        if constexpr (M == 512 && sizeof(T) == 4) {
            // register-resident transforms, twiddles from the LDS table, each
            // wave's line its exchange buffer
            static_assert(XbLayout<T>::kSlots <= M, "exchange exceeds the line");
            cx<T> x[8];
            if (wave == 0) {
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int i = lane + m * kWave;
                    x[m] = (i < N) ? t1[i] : cx<T>{T(0), T(0)};
                }
            }
            twr.store(sm.tw, tid);
            __syncthreads();
            Fft512TwLds<T> tl;
            tl.init(sm.tw, lane);
            if (wave == 0) {
                fft512_regs<T, false>(x, sm.line[0], tl, lane);
#pragma unroll
                for (int m = 0; m < 8; ++m) sm.c[lane + m * kWave] = x[m];
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int ky = lane + m * kWave;
                x[m] = cscale(sm.c[ky], spec_at<T, M>(spec, wave, kx, ky));
            }
            fft512_regs<T, true>(x, sm.line[wave], tl, lane);
            cx<T>* out = t2 + int64_t(wave) * N * HP;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int j = lane + m * kWave;
                if (j < N) out[int64_t(j) * HP + kx] = x[m];
            }
            return;
        }
        constexpr int PC = (M + 3 * kWave - 1) / (3 * kWave);
        cx<T> x[PC];
#pragma unroll
        for (int q = 0; q < PC; ++q) {
            const int i = tid + q * 3 * kWave;
            x[q] = (i < N) ? t1[i] : cx<T>{T(0), T(0)};
        }
        twr.store(sm.tw, tid);
#pragma unroll
        for (int q = 0; q < PC; ++q)
            if (tid + q * 3 * kWave < M) sm.c[tid + q * 3 * kWave] = x[q];
        __syncthreads();
        if (wave == 0) fft_wave<T, false, M>(sm.c, sm.tw, lane);
        __syncthreads();
        cx<T>* line = sm.line[wave];
        for (int ky = lane; ky < M; ky += kWave) line[ky] = cscale(sm.c[ky], spec_at<T, M>(spec, wave, kx, ky));
        wave_sync();
        fft_wave<T, true, M>(line, sm.tw, lane);
        cx<T>* out = t2 + int64_t(wave) * N * HP;
        for (int j = lane; j < N; j += kWave) out[int64_t(j) * HP + kx] = line[j];
    } else if constexpr (M == 512) {                // four columns, register-resident transforms
        static_assert(4 * kXbStride<T> * sizeof(cx<T>) <= sizeof(ColSmem<T, M>), "exchange buffers exceed the LDS");
        const int unit = xcd_unit(blockIdx.x, (H + 3) / 4);
        if (unit < 0) return;
        const int kx0 = 4 * unit, kx = kx0 + wave;
        const bool active = kx < H;     // inactive waves stay for the work-group barriers
        // each wave's exchange buffer, also the staging of its rows for the stores
        cx<T>(*xb)[kXbStride<T>] = reinterpret_cast<cx<T>(*)[kXbStride<T>]>(smem);
        Fft512Tw<T> tw;
        cx<T> cr[8], v[8];
        if (active) {
            const cx<T>* t1 = at<cx<T>>(work, p.w_t1) + int64_t(kx) * N;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int i = lane + m * kWave;
                cr[m] = (i < N) ? t1[i] : cx<T>{T(0), T(0)};
            }
            tw.load(at<cx<T>>(plan, p.o_tw), lane);
            fft512_regs<T, false>(cr, xb[wave], tw, lane);
        }
        for (int ch = 0; ch < (TRACE ? 1 : 3); ++ch) {
            if (active) {
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int ky = lane + m * kWave;
                    const T k = TRACE ? (p.chan == 1 ? spec_at<T, M>(spec, 0, kx, ky)
                                                     : spec_at<T, M>(spec, 0, kx, ky) + spec_at<T, M>(spec, 2, kx, ky))
                                      : spec_at<T, M>(spec, ch, kx, ky);
                    v[m] = cscale(cr[m], k);
                }
                fft512_regs<T, true>(v, xb[wave], tw, lane);
                wave_sync();
#pragma unroll
                for (int m = 0; m < 8; ++m)
                    if (lane + m * kWave < N) xb[wave][lane + m * kWave] = v[m];
            }
            __syncthreads();
            cx<T>* out = t2 + int64_t(ch) * N * HP;
            for (int i = tid; i < 4 * N; i += 4 * kWave) {
                const int j = i >> 2, cc = i & 3;
                if (kx0 + cc < H) out[int64_t(j) * HP + kx0 + cc] = xb[cc][j];
            }
            __syncthreads();
        }
    } else {                                        // four columns, one per wave
        const int unit = xcd_unit(blockIdx.x, (H + 3) / 4);
        if (unit < 0) return;
        TwiddleRegs<T, M, 4 * kWave> twr;
        twr.load(plan, p, tid);
        const int kx0 = 4 * unit, kx = kx0 + wave;
        const bool active = kx < H;     // inactive waves stay for the work-group barriers
        cx<T>* line = sm.line[wave];
        constexpr int PL = M / kWave;
        cx<T> cr[PL];
        if (active) {
            const cx<T>* t1 = at<cx<T>>(work, p.w_t1) + int64_t(kx) * N;
#pragma unroll
            for (int m = 0; m < PL; ++m) {
                const int i = lane + m * kWave;
                cr[m] = (i < N) ? t1[i] : cx<T>{T(0), T(0)};
            }
        }
        twr.store(sm.tw, tid);
        __syncthreads();
        if (active) {
#pragma unroll
            for (int m = 0; m < PL; ++m) line[lane + m * kWave] = cr[m];
            wave_sync();
            fft_wave<T, false, M>(line, sm.tw, lane);
#pragma unroll
            for (int i = 0; i < PL; ++i) cr[i] = line[lane + i * kWave];
        }
        for (int ch = 0; ch < (TRACE ? 1 : 3); ++ch) {
            if (active) {
                wave_sync();
#pragma unroll
                for (int i = 0; i < PL; ++i) {
                    const int ky = lane + i * kWave;
                    // the trace kernel, or K_xx alone for x-channel problems
                    const T k = TRACE ? (p.chan == 1 ? spec_at<T, M>(spec, 0, kx, ky)
                                                     : spec_at<T, M>(spec, 0, kx, ky) + spec_at<T, M>(spec, 2, kx, ky))
                                      : spec_at<T, M>(spec, ch, kx, ky);
                    line[ky] = cscale(cr[i], k);
                }
                wave_sync();
                fft_wave<T, true, M>(line, sm.tw, lane);
            }
            __syncthreads();
            // the four columns go out together: four consecutive threads write
            // T2[ch][j][kx0 .. kx0+3], one contiguous 32-byte run
            cx<T>* out = t2 + int64_t(ch) * N * HP;
            for (int i = tid; i < 4 * N; i += 4 * kWave) {
                const int j = i >> 2, cc = i & 3;
                if (kx0 + cc < H) out[int64_t(j) * HP + kx0 + cc] = sm.line[cc][j];
            }
            __syncthreads();
        }
    }
}

template <typename T, int M, int MODE>
__device__ void fwd_rows_gather_body(const Prob& p, T* __restrict__ out0, const T* __restrict__ in0,
                                     T* __restrict__ out1, T* __restrict__ out2, T* __restrict__ f,
                                     const char* __restrict__ plan, char* __restrict__ work, char* smem) {
    auto& sm = *reinterpret_cast<GatherSmem<T, M>*>(smem);
    constexpr int H = M / 2 + 1;
    constexpr int HP = spec_pitch(M);   // row pitch of T1[ch][row] and T2[ch][row]
    const int N = p.n, nb = p.nb, b = xcd_unit(blockIdx.x, nb, blockIdx.y);
    if (b < 0) return;
    const int* binstart = at<int>(plan, p.o_binstart);
    int p0 = binstart[b * nb], p1 = binstart[(b + 1) * nb];
    const Chk ck = chk_of(p, plan).in_row(b);
    ck.range(p0, p1);
    if (p0 == p1) return;
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    // every load of the work-group in flight together: twiddles, the two
    // spectrum rows of this wave's channel, and the first samples' records
    TwiddleRegs<T, M, 4 * kWave> twr;
    twr.load(plan, p, tid);
    PairRegs<T, M> pr;
    if (wave < 3) {
        const cx<T>* t2 = at<cx<T>>(work, p.w_t2) + int64_t(wave) * N * HP;
        pr.load(t2 + int64_t(b) * HP, t2 + int64_t(b + 1) * HP, true, lane);
    }
    const vec4<T>* samp = at<vec4<T>>(plan, p.o_samp);
    const int2* sidx = at<int2>(plan, p.o_sidx);
    const vec2<T>* ysort = at<vec2<T>>(work, p.w_ysort);
    const vec2<T>* dw = p.o_dw ? at<vec2<T>>(plan, p.o_dw) : nullptr;
    // records per thread and pass: 4, or 2 for the modes that also read a
    // signal by time index (trajectory gradients, residual), which would spill
    constexpr int U = (MODE == 2 || MODE == 3) ? 2 : 4;
    GatherRecs<T, U> first;
    gather_fetch<T, MODE, U>(first, p0 + tid, p1, 4 * kWave, samp, sidx, ysort, in0, p.chan == 1, ck);
    twr.store(sm.tw, tid);
    __syncthreads();
    T* g0 = sm.g;            // row b:   [ch][N]
    T* g1 = sm.g + 3 * N;    // row b+1: [ch][N]
    if (wave < 3) {
        if constexpr (M == 512 && sizeof(T) == 4) {
            // register-resident transform with the twiddles read from the LDS
            // table (registers for them would cost occupancy here); the
            // wave's line holds the exchange
            static_assert(XbLayout<T>::kSlots <= M, "exchange exceeds the line");
            Fft512TwLds<T> tl;
            tl.init(sm.tw, lane);
            cx<T> x[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) x[m] = pr.spectrum(m, lane);
            fft512_regs<T, true>(x, sm.line[wave], tl, lane);
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int i = lane + m * kWave;
                if (i < N) {
                    g0[wave * N + i] = x[m].x;
                    g1[wave * N + i] = x[m].y;
                }
            }
        } else {
            cx<T>* line = sm.line[wave];
#pragma unroll
            for (int m = 0; m < M / kWave; ++m) line[lane + m * kWave] = pr.spectrum(m, lane);
            wave_sync();
            fft_wave<T, true, M>(line, sm.tw, lane);
            for (int i = lane; i < N; i += kWave) {
                g0[wave * N + i] = line[i].x;
                g1[wave * N + i] = line[i].y;
            }
        }
    }
    __syncthreads();
    gather_band<T, MODE, U>(g0, g1, N, p0, p1, samp, sidx, ysort, at<vec2<T>>(work, p.w_res), out0, in0, out1, out2,
                            f, p.t, dw, p.chan == 1, tid, 4 * kWave, ck, &first);
}

// ----------------------------------------------------------------- adjoint ---
// One grid row j per work-group of four waves: the deterministic transpose
// sampling of the row's cells into LDS, then the row FFTs of its three
// channels: wave 0 transforms xx + i xy (split into the two half spectra),
// wave 1 transforms yy alone.
template <typename T, int M, bool SORTED>
__device__ void adj_scatter_row_body(const Prob& p, const T* __restrict__ s, const char* __restrict__ plan,
                                     char* __restrict__ work, char* smem) {
    constexpr int H = M / 2 + 1;
    constexpr int HP = spec_pitch(M);   // row pitch of T1[ch][row] and T2[ch][row]
    const int N = p.n, j = xcd_unit(blockIdx.x, N, blockIdx.y);
    if (j < 0) return;
    const bool g_in = scatter_g_in_region<T, M>(N);
    char* shared_area = smem + (g_in ? 0 : lds_align(size_t(3) * N * sizeof(T)));
    const ScatterLds<T> sl = scatter_lds<T>(shared_area, N, 256);
    T* g = g_in ? sl.first_val : reinterpret_cast<T*>(smem);
    cx<T>* tw = reinterpret_cast<cx<T>*>(shared_area);     // after the sampling
    cx<T>* lines = tw + M;
    const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    TwiddleRegs<T, M, 4 * kWave> twr;       // in flight during the transpose sampling
    if constexpr (M != 512 || sizeof(T) != 4) twr.load(plan, p, tid);
    // SORTED: the signal in cell order, from s when given, else the problem's residual in work
    const vec2<T>* ys = (SORTED && s) ? reinterpret_cast<const vec2<T>*>(s) : at<vec2<T>>(work, p.w_res);
    scatter_row<T, SORTED, 256>(g, sl, N, j, at<int>(plan, p.o_binstart),
                                at<vec4<T>>(plan, p.o_samp), at<int2>(plan, p.o_sidx), ys,
                                s, tid, p.chan == 1, chk_of(p, plan));
    if constexpr (M == 512 && sizeof(T) == 4) {   // register-resident transforms (float32)
        static_assert(2 * kXbStride<T> <= 3 * M, "exchange buffers exceed the transform region");
        __syncthreads();
        if (wave >= 2) return;
        Fft512Tw<T> tw5;
        tw5.load(at<cx<T>>(plan, p.o_tw), lane);
        const T* re = g + (wave == 0 ? 0 : 2 * N);
        const T* im = g + N;
        cx<T> x[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int i = lane + m * kWave;
            x[m] = cx<T>{T(0), T(0)};
            if (i < N) {
                x[m].x = re[i];
                if (wave == 0) x[m].y = im[i];
            }
        }
        cx<T>* xb = reinterpret_cast<cx<T>*>(shared_area) + wave * kXbStride<T>;
        fft512_regs<T, false>(x, xb, tw5, lane);
        cx<T>* t1 = at<cx<T>>(work, p.w_t1);
        if (wave == 1) {
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                const int k = lane + m * kWave;
                if (k < H) t1[(int64_t(2) * N + j) * HP + k] = x[m];
            }
            return;
        }
#pragma unroll
        for (int m = 0; m < 8; ++m) xb[lane + m * kWave] = x[m];
        wave_sync();
        for (int k = lane; k < H; k += kWave) {
            cx<T> A, B;
            split_pair<T, M>(xb, k, A, B);
            t1[int64_t(j) * HP + k] = A;
            t1[(int64_t(N) + j) * HP + k] = B;
        }
        return;
    }
    twr.store(tw, tid);
    __syncthreads();
    if (wave >= 2) return;
    cx<T>* line = lines + wave * M;
    const T* re = g + (wave == 0 ? 0 : 2 * N);
    const T* im = g + N;
    for (int i = lane; i < M; i += kWave) {
        cx<T> z{T(0), T(0)};
        if (i < N) {
            z.x = re[i];
            if (wave == 0) z.y = im[i];
        }
        line[i] = z;
    }
    wave_sync();
    fft_wave<T, false, M>(line, tw, lane);
    cx<T>* t1 = at<cx<T>>(work, p.w_t1);
    for (int k = lane; k < H; k += kWave) {
        if (wave == 0) {
            cx<T> A, B;
            split_pair<T, M>(line, k, A, B);
            t1[int64_t(j) * HP + k] = A;
            t1[(int64_t(N) + j) * HP + k] = B;
        } else {
            t1[(int64_t(2) * N + j) * HP + k] = line[k];
        }
    }
}

// Column kx: forward FFTs of the three channels' columns, sum of the
// products with the channel spectra in the fixed order xx, xy, yy, one
// inverse FFT, rows 0..N-1 to T2[row][kx].  DUAL (four-column shape only):
// the same with the dK/dh spectra as well, to the second T2 slot.
template <typename T, int M, bool SPLIT, bool DUAL = false>
__device__ void adj_cols_body(const Prob& p, const char* __restrict__ plan, char* __restrict__ work, char* smem) {
    auto& sm = *reinterpret_cast<ColSmem<T, M>*>(smem);
    constexpr int H = M / 2 + 1;
    constexpr int HP = spec_pitch(M);   // row pitch of T1[ch][row] and T2[ch][row]
    const int N = p.n, tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const T* spec = at<T>(plan, p.o_spec);
    cx<T>* t2 = at<cx<T>>(work, p.w_t2);
    if (SPLIT) {                                    // one column, waves 0..2
        const int kx = xcd_unit(blockIdx.x, H);
        if (kx < 0) return;
        TwiddleRegs<T, M, 3 * kWave> twr;
        twr.load(plan, p, tid);
        constexpr int PL = M / kWave;
        cx<T> x[PL];
        const cx<T>* t1 = at<cx<T>>(work, p.w_t1) + int64_t(wave) * N * HP + kx;    // column kx of T1[ch]
#pragma unroll
        for (int m = 0; m < PL; ++m) {
            const int i = lane + m * kWave;
            x[m] = (i < N) ? t1[int64_t(i) * HP] : cx<T>{T(0), T(0)};
        }
        twr.store(sm.tw, tid);
        __syncthreads();
        if constexpr (M == 512 && sizeof(T) == 4) {
            // register-resident transforms, twiddles from the LDS table, each
            // wave's line its exchange buffer
            static_assert(XbLayout<T>::kSlots <= M, "exchange exceeds the line");
            Fft512TwLds<T> tl;
            tl.init(sm.tw, lane);
            fft512_regs<T, false>(x, sm.line[wave], tl, lane);
            wave_sync();
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int ky = lane + m * kWave;
                sm.line[wave][ky] = cscale(x[m], spec_at<T, M>(spec, wave, kx, ky));
            }
            __syncthreads();
            if (wave != 0) return;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int ky = lane + m * kWave;
                x[m] = cadd(cadd(sm.line[0][ky], sm.line[1][ky]), sm.line[2][ky]);
            }
            fft512_regs<T, true>(x, sm.line[0], tl, lane);
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int j = lane + m * kWave;
                if (j < N) t2[int64_t(j) * HP + kx] = x[m];
            }
            return;
        }
        cx<T>* line = sm.line[wave];
#pragma unroll
        for (int m = 0; m < PL; ++m) line[lane + m * kWave] = x[m];
        wave_sync();
        fft_wave<T, false, M>(line, sm.tw, lane);
        for (int ky = lane; ky < M; ky += kWave) line[ky] = cscale(line[ky], spec_at<T, M>(spec, wave, kx, ky));
        __syncthreads();
        for (int ky = tid; ky < M; ky += 3 * kWave)
            sm.c[ky] = cadd(cadd(sm.line[0][ky], sm.line[1][ky]), sm.line[2][ky]);
        __syncthreads();
        if (wave != 0) return;
        fft_wave<T, true, M>(sm.c, sm.tw, lane);
        for (int j = lane; j < N; j += kWave) t2[int64_t(j) * HP + kx] = sm.c[j];
    } else if constexpr (M == 512) {                // four columns, register-resident transforms
        const int unit = xcd_unit(blockIdx.x, (H + 3) / 4);
        if (unit < 0) return;
        const int kx0 = 4 * unit, kx = kx0 + wave;
        const bool active = kx < H;     // inactive waves stay for the work-group barriers
        // each wave's exchange buffer, also the staging of its rows for the stores
        cx<T>(*xb)[kXbStride<T>] = reinterpret_cast<cx<T>(*)[kXbStride<T>]>(smem);
        // twiddles from a table staged after the exchange buffers (registers
        // for them measured slower here), then one channel's four columns
        cx<T>* tws = reinterpret_cast<cx<T>*>(smem) + 4 * kXbStride<T>;
        cx<T>* stg = tws + M;                       // [4][SN]: column c of the channel at stg[c * SN]
        const int SN = adj_cols_stage_stride(N);
        // The work-group reads a channel's four columns row by row (element
        // e = row * 4 + column, four consecutive threads one row's 32 contiguous
        // bytes, as T1 is stored row-major) and stages them in LDS, where each
        // wave takes its own column: four times fewer cache lines per load
        // than a wave reading its column alone.  The next channel's loads are
        // issued before the current channel's transform.
        constexpr int PT = (4 * 512 + 4 * kWave - 1) / (4 * kWave);   // elements per thread (N < 512)
        cx<T> rg[PT];
        auto load_channel = [&](int ch) {
            const cx<T>* t1 = at<cx<T>>(work, p.w_t1) + int64_t(ch) * N * HP + kx0;
#pragma unroll
            for (int q = 0; q < PT; ++q) {
                const int e = tid + q * 4 * kWave, row = e >> 2, col = e & 3;
                rg[q] = (row < N && kx0 + col < H) ? t1[int64_t(row) * HP + col] : cx<T>{T(0), T(0)};
            }
        };
        load_channel(0);
        {
            TwiddleRegs<T, M, 4 * kWave> twr;
            twr.load(plan, p, tid);
            twr.store(tws, tid);
        }
        Fft512TwLds<T> tw;
        tw.init(tws, lane);
        const T* spec_dh = DUAL ? at<T>(plan, p.o_spec_dh) : nullptr;
        cx<T> acc[8], acc2[DUAL ? 8 : 1], v[8];
        for (int ch = 0; ch < 3; ++ch) {
#pragma unroll
            for (int q = 0; q < PT; ++q) {
                const int e = tid + q * 4 * kWave, row = e >> 2, col = e & 3;
                if (row < N) stg[col * SN + row] = rg[q];
            }
            __syncthreads();
            if (ch < 2) load_channel(ch + 1);
            if (active) {
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int i = lane + m * kWave;
                    v[m] = (i < N) ? stg[wave * SN + i] : cx<T>{T(0), T(0)};
                }
                fft512_regs<T, false>(v, xb[wave], tw, lane);
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int ky = lane + m * kWave;
                    const cx<T> z = cscale(v[m], spec_at<T, M>(spec, ch, kx, ky));
                    acc[m] = ch == 0 ? z : cadd(acc[m], z);
                    if constexpr (DUAL) {
                        const cx<T> w = cscale(v[m], spec_at<T, M>(spec_dh, ch, kx, ky));
                        acc2[m] = ch == 0 ? w : cadd(acc2[m], w);
                    }
                }
            }
            __syncthreads();                        // the staging area is read before the next channel's stores
        }
        auto emit = [&](cx<T> (&src)[8], int slot) {
            if (active) {
                fft512_regs<T, true>(src, xb[wave], tw, lane);
#pragma unroll
                for (int m = 0; m < 8; ++m)
                    if (lane + m * kWave < N) xb[wave][lane + m * kWave] = src[m];
            }
            __syncthreads();
            cx<T>* out = t2 + int64_t(slot) * N * HP;
            for (int i = tid; i < 4 * N; i += 4 * kWave) {
                const int j = i >> 2, cc = i & 3;
                if (kx0 + cc < H) out[int64_t(j) * HP + kx0 + cc] = xb[cc][j];
            }
            __syncthreads();
        };
        emit(acc, 0);
        if constexpr (DUAL) emit(acc2, 1);
    } else {                                        // four columns, one per wave
        const int unit = xcd_unit(blockIdx.x, (H + 3) / 4);
        if (unit < 0) return;
        TwiddleRegs<T, M, 4 * kWave> twr;
        twr.load(plan, p, tid);
        const int kx0 = 4 * unit, kx = kx0 + wave;
        const bool active = kx < H;     // inactive waves stay for the work-group barriers
        cx<T>* line = sm.line[wave];
        constexpr int PL = M / kWave;
        const T* spec_dh = DUAL ? at<T>(plan, p.o_spec_dh) : nullptr;
        cx<T> acc[PL];
        cx<T> acc2[DUAL ? PL : 1];
        cx<T> x[PL];                    // channel 0's column, loaded with the twiddles
        if (active) {
            const cx<T>* t1 = at<cx<T>>(work, p.w_t1) + kx;
#pragma unroll
            for (int m = 0; m < PL; ++m) {
                const int i = lane + m * kWave;
                x[m] = (i < N) ? t1[int64_t(i) * HP] : cx<T>{T(0), T(0)};
            }
        }
        twr.store(sm.tw, tid);
        __syncthreads();
        for (int ch = 0; ch < 3 && active; ++ch) {
            if (ch == 0) {
#pragma unroll
                for (int m = 0; m < PL; ++m) line[lane + m * kWave] = x[m];
            } else {
                const cx<T>* t1 = at<cx<T>>(work, p.w_t1) + int64_t(ch) * N * HP + kx;
                for (int i = lane; i < M; i += kWave) line[i] = (i < N) ? t1[int64_t(i) * HP] : cx<T>{T(0), T(0)};
            }
            wave_sync();
            fft_wave<T, false, M>(line, sm.tw, lane);
#pragma unroll
            for (int i = 0; i < PL; ++i) {
                const int ky = lane + i * kWave;
                const cx<T> z = line[ky];
                const cx<T> v = cscale(z, spec_at<T, M>(spec, ch, kx, ky));
                acc[i] = ch == 0 ? v : cadd(acc[i], v);
                if constexpr (DUAL) {
                    const cx<T> w = cscale(z, spec_at<T, M>(spec_dh, ch, kx, ky));
                    acc2[i] = ch == 0 ? w : cadd(acc2[i], w);
                }
            }
            wave_sync();
        }
        // one or two outputs; the four columns go out together (four
        // consecutive threads write one contiguous 32-byte run of T2[slot][j])
        auto emit = [&](const cx<T>* src, int slot) {
            if (active) {
                wave_sync();
#pragma unroll
                for (int i = 0; i < PL; ++i) line[lane + i * kWave] = src[i];
                wave_sync();
                fft_wave<T, true, M>(line, sm.tw, lane);
            }
            __syncthreads();
            cx<T>* out = t2 + int64_t(slot) * N * HP;
            for (int i = tid; i < 4 * N; i += 4 * kWave) {
                const int j = i >> 2, cc = i & 3;
                if (kx0 + cc < H) out[int64_t(j) * HP + kx0 + cc] = sm.line[cc][j];
            }
            __syncthreads();
        };
        emit(acc, 0);
        if constexpr (DUAL) emit(acc2, 1);
    }
}

// Sum over the 64 lanes of a wave in a fixed butterfly order; every lane gets it.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = kWave / 2; m > 0; m >>= 1) v += __shfl_xor(v, m, kWave);
    return v;
}

// Partial sums of the conjugate-gradient epilogue: one per row pair.
constexpr int kCgRowParts = 512;

// EPI 0: c_out = A^T s;  1, 2: c_out = c_in - tau * A^T r (c_in may alias c_out);
// 3 (conjugate gradients): c_out = conv + tau * c_in with tau = nu and c_in = p,
// and part[row pair] = the row pair's sum of c_in * c_out in float64.
template <typename T, int M, int EPI>
__device__ void adj_rows_body(const Prob& p, T* c_out, const T* c_in, T tau, int slot,
                              const char* __restrict__ plan, char* __restrict__ work, char* smem,
                              double* __restrict__ part) {
    auto& sm = *reinterpret_cast<RowSmem<T, M>*>(smem);
    constexpr int H = M / 2 + 1;
    constexpr int HP = spec_pitch(M);   // row pitch of T1[ch][row] and T2[ch][row]
    const int N = p.n, tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const int unit = xcd_unit(blockIdx.x, (N + 7) / 8);   // four row pairs per work-group
    if (unit < 0) return;
    const int q = 4 * unit + wave;
    const int r0 = 2 * q, r1 = 2 * q + 1;
    const bool active = r0 < N, two = r1 < N;
    double acc = 0.0;
    auto put = [&](int i, T v0, T v1) {
        const int64_t o0 = int64_t(r0) * N + i, o1 = int64_t(r1) * N + i;
        if (EPI == 0) {
            c_out[o0] = v0;
            if (two) c_out[o1] = v1;
        } else if (EPI == 3) {
            const T p0 = c_in[o0], a0 = v0 + tau * p0;
            c_out[o0] = a0;
            acc += double(p0) * double(a0);
            if (two) {
                const T p1 = c_in[o1], a1 = v1 + tau * p1;
                c_out[o1] = a1;
                acc += double(p1) * double(a1);
            }
        } else {
            c_out[o0] = c_in[o0] - tau * v0;
            if (two) c_out[o1] = c_in[o1] - tau * v1;
        }
    };
    auto finish = [&]() {
        if (EPI == 3) {
            const double tot = wave_sum(acc);
            if (lane == 0) part[q] = tot;
        }
    };
    if constexpr (M == 512) {                       // register-resident transform, no barrier
        static_assert(4 * kXbStride<T> * sizeof(cx<T>) <= sizeof(RowSmem<T, M>), "exchange buffers exceed the LDS");
        if (!active) return;
        Fft512Tw<T> tw;
        tw.load(at<cx<T>>(plan, p.o_tw), lane);
        PairRegs<T, M> pr;
        const cx<T>* t2 = at<cx<T>>(work, p.w_t2) + int64_t(slot) * N * HP;
        pr.load(t2 + int64_t(r0) * HP, t2 + int64_t(two ? r1 : r0) * HP, two, lane);
        cx<T> x[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m] = pr.spectrum(m, lane);
        cx<T>(*xb)[kXbStride<T>] = reinterpret_cast<cx<T>(*)[kXbStride<T>]>(smem);
        fft512_regs<T, true>(x, xb[wave], tw, lane);
#pragma unroll
        for (int m = 0; m < 8; ++m)
            if (lane + m * kWave < N) put(lane + m * kWave, x[m].x, x[m].y);
        finish();
    } else {
        TwiddleRegs<T, M, 4 * kWave> twr;
        twr.load(plan, p, tid);
        PairRegs<T, M> pr;
        if (active) {
            const cx<T>* t2 = at<cx<T>>(work, p.w_t2) + int64_t(slot) * N * HP;
            pr.load(t2 + int64_t(r0) * HP, t2 + int64_t(two ? r1 : r0) * HP, two, lane);
        }
        twr.store(sm.tw, tid);
        __syncthreads();
        if (!active) return;
        cx<T>* line = sm.line[wave];
#pragma unroll
        for (int m = 0; m < M / kWave; ++m) line[lane + m * kWave] = pr.spectrum(m, lane);
        wave_sync();
        fft_wave<T, true, M>(line, sm.tw, lane);
        for (int i = lane; i < N; i += kWave) put(i, line[i].x, line[i].y);
        finish();
    }
}

// The composition of an inverse row stage and the next forward row stage on
// the same rows (the middle of C^T C p = C (C p) without writing C p): per row
// pair, the inverse FFT of T2 rows r0, r1 gives the pair as one complex line;
// the entries beyond the N grid columns are cut (the convolution's output is
// the N x N window), and the forward FFT of the cut line gives the half
// spectra of the two rows, stored to T1[kx][row] as the forward row stage
// does.
template <typename T, int M>
__device__ void rows_inv_fwd_body(const Prob& p, const char* __restrict__ plan, char* __restrict__ work, char* smem) {
    constexpr int H = M / 2 + 1;
    constexpr int HP = spec_pitch(M);   // row pitch of T1[ch][row] and T2[ch][row]
    const int N = p.n, tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
    const int unit = xcd_unit(blockIdx.x, (N + 7) / 8);   // four row pairs per work-group
    if (unit < 0) return;
    const int q = 4 * unit + wave;
    const int r0 = 2 * q, r1 = 2 * q + 1;
    const bool active = r0 < N, two = r1 < N;
    const cx<T>* t2 = at<cx<T>>(work, p.w_t2);
    const cx<T>* lines;                          // the four waves' forward spectra, natural order
    int stride;
    if constexpr (M == 512) {                    // register-resident transforms
        static_assert(4 * kXbStride<T> * sizeof(cx<T>) <= sizeof(RowSmem<T, M>), "exchange buffers exceed the LDS");
        cx<T>(*xb)[kXbStride<T>] = reinterpret_cast<cx<T>(*)[kXbStride<T>]>(smem);
        if (active) {
            Fft512Tw<T> tw;
            tw.load(at<cx<T>>(plan, p.o_tw), lane);
            PairRegs<T, M> pr;
            pr.load(t2 + int64_t(r0) * HP, t2 + int64_t(two ? r1 : r0) * HP, two, lane);
            cx<T> x[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) x[m] = pr.spectrum(m, lane);
            fft512_regs<T, true>(x, xb[wave], tw, lane);
#pragma unroll
            for (int m = 0; m < 8; ++m)
                if (lane + m * kWave >= N) x[m] = cx<T>{T(0), T(0)};
            fft512_regs<T, false>(x, xb[wave], tw, lane);
            wave_sync();
#pragma unroll
            for (int m = 0; m < 8; ++m) xb[wave][lane + m * kWave] = x[m];
        }
        lines = &xb[0][0];
        stride = kXbStride<T>;
    } else {
        auto& sm = *reinterpret_cast<RowSmem<T, M>*>(smem);
        TwiddleRegs<T, M, 4 * kWave> twr;
        twr.load(plan, p, tid);
        PairRegs<T, M> pr;
        if (active) pr.load(t2 + int64_t(r0) * HP, t2 + int64_t(two ? r1 : r0) * HP, two, lane);
        twr.store(sm.tw, tid);
        __syncthreads();
        if (active) {
            cx<T>* line = sm.line[wave];
#pragma unroll
            for (int m = 0; m < M / kWave; ++m) line[lane + m * kWave] = pr.spectrum(m, lane);
            wave_sync();
            fft_wave<T, true, M>(line, sm.tw, lane);
            for (int i = N + lane; i < M; i += kWave) line[i] = cx<T>{T(0), T(0)};
            wave_sync();
            fft_wave<T, false, M>(line, sm.tw, lane);
        }
        lines = &sm.line[0][0];
        stride = M;
    }
    __syncthreads();
    cx<T>* t1 = at<cx<T>>(work, p.w_t1);
    const int row0 = 8 * unit;
    for (int i = tid; i < 8 * H; i += 4 * kWave) {
        const int k = i >> 3, r = i & 7;
        if (row0 + r >= N) continue;
        cx<T> A, B;
        split_pair<T, M>(lines + (r >> 1) * stride, k, A, B);
        const bool odd = r & 1;
        t1[int64_t(k) * N + row0 + r] = cx<T>{odd ? B.x : A.x, odd ? B.y : A.y};
    }
}

// ------------------------------------------------------------- launchers ---
// One instance per FFT size M, so that registers are allocated for that size
// alone; a launch covers every problem of the batch (grid.y) and problems of
// another size, or on the direct path, leave at once.  skip (optional, one
// flag per problem): problems with a nonzero flag leave at once as well (the
// batched solvers use it for problems that have converged).

// grid.x: xcd_grid(ceil(row pairs / 4)), grid.y: problem; 256 threads
template <typename T, int M>
__global__ void __launch_bounds__(256) k_fwd_rows(const Prob* __restrict__ P, const T* __restrict__ c,
                                                  const char* __restrict__ plan, char* __restrict__ work,
                                                  const int* __restrict__ skip) {
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.y];
    if (p.mode != 1 || p.m != M || (skip && skip[blockIdx.y])) return;
    fwd_rows_body<T, M>(p, c + p.o_c, plan, work, smem);
}

// SPLIT: grid.x = xcd_grid(M/2 + 1), 192 threads; else xcd_grid(ceil((M/2 + 1)/4)), 256 threads
template <typename T, int M, bool SPLIT, bool TRACE = false>
__global__ void __launch_bounds__(256) k_fwd_cols(const Prob* __restrict__ P, const char* __restrict__ plan,
                                                  char* __restrict__ work, int dh, const int* __restrict__ skip) {
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.y];
    if (p.mode != 1 || p.m != M || (skip && skip[blockIdx.y])) return;
    fwd_cols_body<T, M, SPLIT, TRACE>(p, plan, work, smem, dh);
}

// grid.x: xcd_grid(base-cell rows), 256 threads.  MODE as gather_band; the
// caller buffers are offset to the problem here.
template <typename T, int M, int MODE>
__global__ void __launch_bounds__(256) k_fwd_rows_gather(const Prob* __restrict__ P, GatherIO<T> io,
                                                         const char* __restrict__ plan, char* __restrict__ work) {
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.y];
    if (p.mode != 1 || p.m != M) return;
    fwd_rows_gather_body<T, M, MODE>(p, io.out0 ? io.out0 + p.o_s : nullptr, io.in0 ? io.in0 + p.o_s : nullptr,
                                     io.out1 ? io.out1 + p.o_s : nullptr, io.out2 ? io.out2 + p.o_s : nullptr,
                                     io.f ? io.f + 9 * (p.o_s / 2) : nullptr, plan, work, smem);
}

// grid.x: xcd_grid(grid rows), 256 threads
template <typename T, int M, bool SORTED>
__global__ void __launch_bounds__(256) k_adj_scatter_row(const Prob* __restrict__ P, const T* __restrict__ s,
                                                         const char* __restrict__ plan, char* __restrict__ work) {
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.y];
    if (p.mode != 1 || p.m != M) return;
    adj_scatter_row_body<T, M, SORTED>(p, s ? s + p.o_s : nullptr, plan, work, smem);
}

// SPLIT: grid.x = xcd_grid(M/2 + 1), 192 threads; else xcd_grid(ceil((M/2 + 1)/4)), 256 threads.
// DUAL needs the four-column shape.
template <typename T, int M, bool SPLIT, bool DUAL = false>
__global__ void __launch_bounds__(256) k_adj_cols(const Prob* __restrict__ P, const char* __restrict__ plan,
                                                  char* __restrict__ work) {
    static_assert(!(SPLIT && DUAL), "the dual transpose runs in the four-column shape");
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.y];
    if (p.mode != 1 || p.m != M) return;
    adj_cols_body<T, M, SPLIT, DUAL>(p, plan, work, smem);
}

// grid.x: xcd_grid(ceil(row pairs / 4)), 256 threads; slot: which T2 field.
// EPI 3: taus holds nu per problem, part kCgRowParts partial sums per problem.
template <typename T, int M, int EPI>
__global__ void __launch_bounds__(256) k_adj_rows(const Prob* __restrict__ P, T* c_out, const T* c_in,
                                                  const double* __restrict__ taus, const char* __restrict__ plan,
                                                  char* __restrict__ work, int slot, const int* __restrict__ skip,
                                                  double* __restrict__ part) {
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.y];
    if (p.mode != 1 || p.m != M || (skip && skip[blockIdx.y])) return;
    const T tau = EPI ? T(taus[blockIdx.y]) : T(0);
    // EPI 2 writes the step into the problem's work buffer u (before the denoiser)
    T* out = EPI == 2 ? at<T>(work, p.w_u) : c_out + p.o_c;
    adj_rows_body<T, M, EPI>(p, out, EPI ? c_in + p.o_c : nullptr, tau, slot, plan, work, smem,
                             EPI == 3 ? part + int64_t(blockIdx.y) * kCgRowParts : nullptr);
}

// grid.x: xcd_grid(ceil(row pairs / 4)), 256 threads
template <typename T, int M>
__global__ void __launch_bounds__(256) k_rows_inv_fwd(const Prob* __restrict__ P, const char* __restrict__ plan,
                                                      char* __restrict__ work, const int* __restrict__ skip) {
    extern __shared__ __align__(16) char smem[];
    const Prob& p = P[blockIdx.y];
    if (p.mode != 1 || p.m != M || (skip && skip[blockIdx.y])) return;
    rows_inv_fwd_body<T, M>(p, plan, work, smem);
}

}  // namespace mpik
