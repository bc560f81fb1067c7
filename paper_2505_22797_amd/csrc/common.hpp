// Device-side types shared by every kernel of the library: complex numbers,
// the per-problem descriptor, the in-LDS Stockham FFT and small helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpik {

constexpr int kWave = 64;

template <typename T> struct cx { T x, y; };

template <typename T> __device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.x, -a.y}; }
template <typename T> __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV> __device__ __forceinline__ cx<T> mul_mi(cx<T> a) {
    return INV ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
}

template <typename T> struct v4;
template <> struct v4<float> { using type = float4; };
template <> struct v4<double> { using type = double4; };
template <typename T> struct v2;
template <> struct v2<float> { using type = float2; };
template <> struct v2<double> { using type = double2; };
template <typename T> using vec4 = typename v4<T>::type;
template <typename T> using vec2 = typename v2<T>::type;

// Row pitch, in complex elements, of the half-spectrum intermediates laid out
// by grid row ([ch][row][kx], kx < M/2 + 1): M/2 + 1 rounded up to four, so
// that every row starts on a 32-byte boundary in float32 and a column
// stage's four-column run of a row never straddles two 32-byte sectors.
__host__ __device__ constexpr int spec_pitch(int M) { return (M / 2 + 4) / 4 * 4; }

// ---------------------------------------------------------------------------
// Problem descriptor, resident in plan memory.  Offsets are in bytes from the
// plan base (o_*) or from the work base (w_*); every buffer is 256-byte aligned.
// ---------------------------------------------------------------------------
struct Prob {
    int32_t n;         // grid side N
    int32_t nb;        // bins per side, N - 1
    int32_t radius;    // effective window half-width R <= N - 1
    int32_t m;         // FFT size M (0 on the direct path)
    int32_t log2m;
    int32_t mode;      // 0 direct, 1 FFT
    int32_t taps_w;    // padded row length of the direct-path tap table
    int32_t slices;    // direct path: waves splitting the dy range of a tile
    int32_t interp;    // 0 bilinear, 1 cosine (the weights in o_samp already applied)
    int32_t chan;      // 0 both receive channels, 1 the x channel alone
    double gx, gy;     // selection-field gradient G = diag(gx, gy): the kernel is K_h(G y)
    int64_t t;         // samples
    double h;
    int64_t o_c;       // element offset of this problem's concentration in the caller's buffer
    int64_t o_s;       // element offset of this problem's signal in the caller's buffer
    // plan memory
    int64_t o_taps;      // T [3][2R+1][taps_w]   delta^2 K_h (direct path)
    int64_t o_spec;      // T [3][M/2+1][M/2+1]   delta^2/M^2 * DFT of K_h, [ch][kx][ky]
    int64_t o_taps_dh;   // as o_taps for dK_h/dh (plans built for derivatives), else 0
    int64_t o_spec_dh;   // as o_spec for dK_h/dh, else 0
    int64_t o_tw;        // cx<T> [M]             e^{-2 pi i k / M}
    int64_t o_samp;      // vec4<T> [T]           (wx, wy, vx, vy) in cell order, w the upper-neighbour weight
    int64_t o_dw;        // vec2<T> [T]           (dwx/dfx, dwy/dfy) in cell order (plans built for
                         //                       derivatives, else 0; all ones when bilinear)
    int64_t o_sidx;      // int2 [T]              (base cell i0 | j0 << 16, time index), cell order
    int64_t o_binstart;  // int32 [nb*nb + 1]     first sample of every base cell
    int64_t o_err;       // int32 [4]             build error flags
    int64_t o_scratch;   // build-time scratch
    // work memory
    int64_t w_g;       // T [3][N][N]       sampled field G or its transpose image
    int64_t w_t1;      // cx<T> [M/2+1][N] (forward), [3][N][spec_pitch(M)] (transpose)
    int64_t w_t2;      // cx<T> [3][N][spec_pitch(M)]
    int64_t w_ysort;   // vec2<T> [T]       measured signal in cell order
    int64_t w_res;     // vec2<T> [T]       residual in cell order
    int64_t w_u;       // T [N][N]          pre-denoise iterate
    int64_t w_grad;    // T [N][N]
};

template <typename P> __device__ __forceinline__ P* at(char* base, int64_t off) {
    return reinterpret_cast<P*>(base + off);
}
template <typename P> __device__ __forceinline__ const P* at(const char* base, int64_t off) {
    return reinterpret_cast<const P*>(base + off);
}

// ---------------------------------------------------------------------------
// Bounds checks of the debug build (-DMPIK_CHECK).  The indices that kernels
// read from the plan's sample tables -- a sample's base cell and time index,
// the sample range of a base-cell row -- are checked before they address
// memory.  A failed check ORs its bit into the problem's check word (the
// second int32 at o_err in plan memory) and the access it guards is skipped,
// so every kernel still runs to its normal end; the host reads the word with
// mpi_plan_check.  Without MPIK_CHECK every check is `true` and compiles away.
// ---------------------------------------------------------------------------
enum : int { kChkCell = 1, kChkTime = 2, kChkRange = 4 };

struct Chk {
#ifdef MPIK_CHECK
    int* word;
    int nb;          // base cells per side
    int row;         // base-cell row the samples must lie in, or -1: any
    int64_t t;       // samples
#endif
    __device__ __forceinline__ bool ok(bool cond, int bit) const {
#ifdef MPIK_CHECK
        if (!cond) atomicOr(word, bit);
        return cond;
#else
        (void)cond;
        (void)bit;
        return true;
#endif
    }
    // base cell (i0, j0) of a sample: inside the grid, and in `row` if set
    __device__ __forceinline__ bool cell(int packed) const {
#ifdef MPIK_CHECK
        const int i0 = packed & 0xffff, j0 = packed >> 16;
        return ok(i0 < nb && j0 >= 0 && j0 < nb && (row < 0 || j0 == row), kChkCell);
#else
        (void)packed;
        return true;
#endif
    }
    // base cell of a sample that reaches grid row j: base-cell row j-1 or j
    __device__ __forceinline__ bool cell_near(int packed, int j) const {
#ifdef MPIK_CHECK
        const int i0 = packed & 0xffff, j0 = packed >> 16;
        return ok(i0 < nb && j0 >= 0 && j0 < nb && (j0 == j || j0 == j - 1), kChkCell);
#else
        (void)packed;
        (void)j;
        return true;
#endif
    }
    __device__ __forceinline__ bool time(int64_t k) const {
#ifdef MPIK_CHECK
        return ok(k >= 0 && k < t, kChkTime);
#else
        (void)k;
        return true;
#endif
    }
    // a cell-order sample range [p0, p1); an invalid one becomes empty
    __device__ __forceinline__ void range(int& p0, int& p1) const {
#ifdef MPIK_CHECK
        if (!ok(p0 >= 0 && p0 <= p1 && p1 <= t, kChkRange)) p0 = p1 = 0;
#else
        (void)p0;
        (void)p1;
#endif
    }
    __device__ __forceinline__ Chk in_row(int r) const {
        Chk c = *this;
#ifdef MPIK_CHECK
        c.row = r;
#else
        (void)r;
#endif
        return c;
    }
};

__device__ __forceinline__ Chk chk_of(const Prob& p, const char* plan) {
    Chk c;
#ifdef MPIK_CHECK
    c.word = reinterpret_cast<int*>(const_cast<char*>(plan) + p.o_err) + 1;
    c.nb = p.nb;
    c.row = -1;
    c.t = p.t;
#else
    (void)p;
    (void)plan;
#endif
    return c;
}

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Work-groups are dealt to the 8 XCDs (each with its own L2) round-robin by
// their linear index.  With grid.x a multiple of 8, block x runs on XCD x % 8;
// mapping it to unit ((x + rot) % 8) * ceil(n/8) + x / 8 gives every XCD one
// contiguous band of units, so the transposing stores of neighbouring rows or
// columns fill whole cache lines in one L2, and the stages that read the
// samples of two neighbouring rows find the shared row in the same L2.  rot
// (the problem's index in the launch, for the sampling stages) turns the
// bands over the XCDs from problem to problem: a trajectory's dense rows (a
// Lissajous figure's turning lines hold up to nine times the mean samples)
// then load every XCD alike over a batch instead of always the same two.
// The map is one-to-one from blocks [0, 8 * ceil(n/8)) onto units; it returns
// -1 for padding blocks and for blocks beyond that range (a batched launch is
// sized for its largest problem).
constexpr int kXcds = 8;
__host__ __device__ constexpr int xcd_grid(int n) { return (n + kXcds - 1) / kXcds * kXcds; }
__device__ __forceinline__ int xcd_unit(int x, int n, int rot = 0) {
    const int per = (n + kXcds - 1) / kXcds;
    if (x / kXcds >= per) return -1;
    const int u = ((x + rot) % kXcds) * per + x / kXcds;
    return u < n ? u : -1;
}

// ---------------------------------------------------------------------------
// Stockham autosort FFT of one line of M points held in LDS, done in place by
// one 64-lane wavefront with no work-group barrier.  Mixed radix 8 (then 4 or
// 2 for the remaining factor): a pass of radix R with span Ns takes butterfly
// j (j < M/R) from line[j + r M/R], applies the twiddle w^(r (j mod Ns)
// M/(Ns R)), does a length-R DFT and writes line[(j / Ns) Ns R + (j mod Ns)
// + r Ns]; the result comes out in natural order.  Every lane reads all of its
// butterfly inputs before any lane writes (a wave executes its LDS operations
// in order), so one buffer suffices.  Forward uses w = e^{-2 pi i/M}, inverse
// the conjugate; no scaling.
// ---------------------------------------------------------------------------
// Caller buffers of a gather launch, all flat over the batch: signal-shaped
// out0/in0/out1/out2 (problem b at element o_s), and f, nine planes of the
// sampled field per problem (problem b at element 9 o_s / 2, plane stride T_b).
template <typename T> struct GatherIO {
    T* out0 = nullptr;
    const T* in0 = nullptr;
    T* out1 = nullptr;
    T* out2 = nullptr;
    T* f = nullptr;
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, bool INV>
__device__ __forceinline__ void dft2(cx<T>* v) {
    cx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cx<T>* v) {
    cx<T> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    cx<T> s13 = cadd(v[1], v[3]), d13 = mul_mi<T, INV>(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cx<T>* v) {
    const T h = T(0.70710678118654752440084436210484903928);
    // even half: DFT4 of v0, v2, v4, v6
    cx<T> a0 = cadd(v[0], v[4]), a1 = csub(v[0], v[4]);
    cx<T> a2 = cadd(v[2], v[6]), a3 = mul_mi<T, INV>(csub(v[2], v[6]));
    cx<T> e0 = cadd(a0, a2), e2 = csub(a0, a2), e1 = cadd(a1, a3), e3 = csub(a1, a3);
    // odd half: DFT4 of v1, v3, v5, v7
    cx<T> b0 = cadd(v[1], v[5]), b1 = csub(v[1], v[5]);
    cx<T> b2 = cadd(v[3], v[7]), b3 = mul_mi<T, INV>(csub(v[3], v[7]));
    cx<T> o0 = cadd(b0, b2), o2 = csub(b0, b2), o1 = cadd(b1, b3), o3 = csub(b1, b3);
    // twiddles w^1 = (1 -+ i)/sqrt2, w^2 = -+i, w^3 = (-1 -+ i)/sqrt2
    cx<T> t1 = INV ? cx<T>{h * (o1.x - o1.y), h * (o1.x + o1.y)} : cx<T>{h * (o1.x + o1.y), h * (o1.y - o1.x)};
    cx<T> t2 = mul_mi<T, INV>(o2);
    cx<T> t3 = INV ? cx<T>{-h * (o3.x + o3.y), h * (o3.x - o3.y)} : cx<T>{h * (o3.y - o3.x), -h * (o3.x + o3.y)};
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, t1); v[5] = csub(e1, t1);
    v[2] = cadd(e2, t2); v[6] = csub(e2, t2);
    v[3] = cadd(e3, t3); v[7] = csub(e3, t3);
}

template <typename T, bool INV, int R, int M, int NS>
__device__ __forceinline__ void fft_pass(cx<T>* line, const cx<T>* __restrict__ tw, int lane) {
    constexpr int NB = M / R;                       // butterflies in the pass
    constexpr int PER = (NB + kWave - 1) / kWave;   // butterflies per lane
    constexpr int STEP = M / (NS * R);
    cx<T> v[PER][R];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = lane + q * kWave;
        if (NB % kWave == 0 || j < NB) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = line[j + r * NB];
        }
    }
    wave_sync();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int j = lane + q * kWave;
        if (NB % kWave == 0 || j < NB) {
            const int k = j & (NS - 1);
            if (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cx<T> w = tw[r * k * STEP];
                    if (INV) w.y = -w.y;
                    v[q][r] = cmul(v[q][r], w);
                }
            }
            if (R == 8) dft8<T, INV>(v[q]);
            else if (R == 4) dft4<T, INV>(v[q]);
            else dft2<T, INV>(v[q]);
            const int base = (j / NS) * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) line[base + r * NS] = v[q][r];
        }
    }
    wave_sync();
}

template <typename T, bool INV, int M, int NS = 1>
__device__ __forceinline__ void fft_wave(cx<T>* line, const cx<T>* __restrict__ tw, int lane) {
    static_assert(M >= 64 && (M & (M - 1)) == 0, "M must be a power of two >= 64");
    if constexpr (NS < M) {
        constexpr int REM = M / NS;
        constexpr int R = (REM % 8 == 0) ? 8 : REM;
        fft_pass<T, INV, R, M, NS>(line, tw, lane);
        fft_wave<T, INV, M, NS * R>(line, tw, lane);
    }
}

// 512-point FFT of one wave with the data in registers: lane l holds x[l + 64 m]
// in v[m] on entry and X[l + 64 m] on exit (natural order both ways;
// unnormalised, conjugate twiddles when INV).  With n = n2 + 64 n1 and
// k = k1 + 8 k2:  X = sum_n2 W64^(n2 k2) W512^(n2 k1) sum_n1 x W8^(n1 k1), so each
// lane first takes an 8-point DFT over its registers and applies W512^(l k1);
// the 64-point DFT over the lanes n2 = a + 8b, k2 = c + 8d is then
// sum_a W8^(a d) W64^(a c) sum_b W8^(b c), two 8-point DFTs with an exchange
// through LDS before each.  Each exchange is one write-then-read round trip; a
// 512-point transform makes two, against four for the in-LDS passes.
//
// Exchange layout.  Element i = 64x + 8y + z (x, y, z in [0, 8)) goes to slot
// XbLayout<T>::slot(i) of the wave's buffer.  The three access shapes are: lane a + 8b
// writes (x, y, z) = (k, a, b) for k = 0..7; lane lo + 8hi reads (lo, hi, k);
// lane lo + 8hi writes (lo, k, hi).
//  * float32 (8-byte elements): slot = XOR of a fixed 9-bit image of each set
//    bit of i (a bijection of [0, 512), linear over GF(2)).  The images are
//    chosen so that every 16-lane group of every access touches 16 distinct
//    bank pairs (32 four-byte banks) and every 32-lane group 32 distinct
//    ones (64 banks); a plain padding of one slot in nine leaves 4-way
//    conflicts in the read and the second write.  Linearity splits every
//    slot into a per-lane part (computed once per kernel with the twiddles)
//    XOR a constant per register.
//  * float64 (16-byte elements): slot = i + i/8 (one pad slot in nine), which
//    keeps every 8-lane group on 8 distinct four-bank groups.
// kXbStride<T> is the distance between the waves' buffers, chosen so that the
// column stages' four-wave staging reads (thread t reads element t/4 of wave
// t%4) spread over the banks as well.
template <typename T> struct XbLayout;
template <> struct XbLayout<float> {
    static constexpr int kImage[9] = {140, 16, 256, 8, 49, 66, 1, 2, 4};
    static constexpr int kSlots = 512;
    static constexpr int kStride = 516;
    __host__ __device__ static constexpr int slot(int i) {
        int s = 0;
        for (int b = 0; b < 9; ++b) s ^= ((i >> b) & 1) ? kImage[b] : 0;
        return s;
    }
};
template <> struct XbLayout<double> {
    static constexpr int kSlots = 576;
    static constexpr int kStride = 578;
    __host__ __device__ static constexpr int slot(int i) { return i + (i >> 3); }
};
template <typename T> inline constexpr int kXbStride = XbLayout<T>::kStride;

namespace detail {
template <typename T> __host__ __device__ constexpr bool xb_layout_ok() {
    int seen[XbLayout<T>::kSlots] = {};
    for (int i = 0; i < 512; ++i) {
        const int s = XbLayout<T>::slot(i);
        if (s < 0 || s >= XbLayout<T>::kSlots || seen[s]) return false;
        seen[s] = 1;
    }
    return XbLayout<T>::kSlots <= XbLayout<T>::kStride;
}
static_assert(xb_layout_ok<float>() && xb_layout_ok<double>(), "exchange layout must be a bijection into the buffer");
}  // namespace detail

// Per-lane constants of fft512_regs, read or computed once per kernel:
// twiddles from the plan's table (tw[j] = W512^j), w1(k) = W512^(lane k) and
// w2(k) = W64^((lane >> 3) k), k = 1..7, kept in registers; and the lane's
// exchange slots (float32 only): s1 for the first write, s2 for both reads,
// s3 for the second write.
template <typename T> struct Fft512Tw {
    cx<T> w1_[7];
    cx<T> w2_[7];
    int s1, s2, s3;
    __device__ __forceinline__ void load(const cx<T>* __restrict__ tw, int lane) {
#pragma unroll
        for (int k = 1; k < 8; ++k) {
            w1_[k - 1] = tw[(lane * k) & 511];
            w2_[k - 1] = tw[(8 * (lane >> 3) * k) & 511];
        }
        const int lo = lane & 7, hi = lane >> 3;
        s1 = XbLayout<T>::slot(8 * lo + hi);
        s2 = XbLayout<T>::slot(64 * lo + 8 * hi);
        s3 = XbLayout<T>::slot(64 * lo + hi);
    }
    __device__ __forceinline__ cx<T> w1(int k) const { return w1_[k - 1]; }
    __device__ __forceinline__ cx<T> w2(int k) const { return w2_[k - 1]; }
};

// The same constants with the twiddles read from a table already in LDS at
// each use: fewer registers, for kernels whose occupancy they would limit.
template <typename T> struct Fft512TwLds {
    const cx<T>* tw;
    int lane, s1, s2, s3;
    __device__ __forceinline__ void init(const cx<T>* tw_lds, int ln) {
        tw = tw_lds;
        lane = ln;
        const int lo = lane & 7, hi = lane >> 3;
        s1 = XbLayout<T>::slot(8 * lo + hi);
        s2 = XbLayout<T>::slot(64 * lo + 8 * hi);
        s3 = XbLayout<T>::slot(64 * lo + hi);
    }
    __device__ __forceinline__ cx<T> w1(int k) const { return tw[(lane * k) & 511]; }
    __device__ __forceinline__ cx<T> w2(int k) const { return tw[(8 * (lane >> 3) * k) & 511]; }
};

template <typename T, bool INV, class TW>
__device__ __forceinline__ void fft512_regs(cx<T> (&v)[8], cx<T>* xb, const TW& tw, int lane) {
    using L = XbLayout<T>;
    constexpr bool kSwz = sizeof(T) == 4;
    const int lo = lane & 7, hi = lane >> 3;
    dft8<T, INV>(v);
#pragma unroll
    for (int k = 1; k < 8; ++k) {
        cx<T> w = tw.w1(k);
        if (INV) w.y = -w.y;
        v[k] = cmul(v[k], w);
    }
    // exchange 1: lane a + 8b holds index k1 in register k1; lane k1 + 8a gathers b = 0..7
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) xb[kSwz ? (tw.s1 ^ L::slot(64 * k1)) : L::slot(k1 * 64 + lo * 8 + hi)] = v[k1];
    wave_sync();
#pragma unroll
    for (int b = 0; b < 8; ++b) v[b] = xb[kSwz ? (tw.s2 ^ L::slot(b)) : L::slot(lo * 64 + hi * 8 + b)];
    wave_sync();
    dft8<T, INV>(v);                          // over b: index c
#pragma unroll
    for (int c = 1; c < 8; ++c) {
        cx<T> w = tw.w2(c);
        if (INV) w.y = -w.y;
        v[c] = cmul(v[c], w);
    }
    // exchange 2: lane k1 + 8a holds c in register c; lane k1 + 8c gathers a = 0..7
#pragma unroll
    for (int c = 0; c < 8; ++c) xb[kSwz ? (tw.s3 ^ L::slot(8 * c)) : L::slot(lo * 64 + c * 8 + hi)] = v[c];
    wave_sync();
#pragma unroll
    for (int a = 0; a < 8; ++a) v[a] = xb[kSwz ? (tw.s2 ^ L::slot(a)) : L::slot(lo * 64 + hi * 8 + a)];
    wave_sync();
    dft8<T, INV>(v);                          // over a: index d, X[lane + 64 d]
}

}  // namespace mpik
