// Host side of the C ABI declared in include/mpik.h: descriptor validation,
// plan/work layout, the plan build, and the launch sequences of the forward
// operator, its transpose and the iteration (optionally replayed as a HIP
// graph).  The library never allocates device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "../../include/mpik.h"
#include "build.hpp"
#include "direct.hpp"
#include "fft_conv.hpp"

using namespace mpik;

namespace {

constexpr size_t kAlign = 256;
constexpr int kDirectSlices = 8;
constexpr int64_t kMaxSamples = int64_t(1) << 26;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    Prob p;
    size_t plan_bytes = 0, work_bytes = 0;
    // build scratch (bytes from plan base)
    int64_t o_series = 0, o_tab64 = 0, o_cs = 0, o_U = 0, o_cell = 0, o_frac = 0, o_bincount = 0,
            o_cellcount = 0, o_cursor = 0;
    int64_t w_wts = 0;
    int elem = 4;
};

int pow2_at_least(int x) {
    int m = 1;
    while (m < x) m *= 2;
    return m;
}

size_t direct_smem(int R, int cin, int cout, int elem) {
    const size_t tile = size_t(cin) * (kTile + 2 * R) * direct_row_len(R);
    const size_t red = size_t(kDirectSlices) * kWave * cout * kStrip;
    return std::max(tile, red) * elem;
}

// Picks the convolution path and fills the layout.  Returns MPI_OK or an error.
int make_layout(const mpi_problem* d, Layout& L) {
    if (!d) return MPI_ERR_ARG;
    if (d->dtype != MPI_F32 && d->dtype != MPI_F64) return MPI_ERR_DTYPE;
    if (d->n < 2 || d->n > 1024) return MPI_ERR_ARG;
    if (!(d->h > 0.0) || !std::isfinite(d->h)) return MPI_ERR_ARG;
    if (d->radius < 0) return MPI_ERR_ARG;
    if (d->n_samples < 1 || d->n_samples >= kMaxSamples) return MPI_ERR_ARG;
    if (d->conv_mode < MPI_CONV_AUTO || d->conv_mode > MPI_CONV_FFT) return MPI_ERR_ARG;
    if (d->interp != MPI_INTERP_BILINEAR || d->channels != MPI_CH_XY) return MPI_ERR_UNSUPPORTED;
    const int elem = d->dtype == MPI_F64 ? 8 : 4;
    L.elem = elem;
    const int N = d->n, R = std::min(d->radius, N - 1), nb = N - 1;
    const int64_t T = d->n_samples;
    const int maxM = elem == 8 ? 512 : 1024;
    const int M = std::max(64, pow2_at_least(N + R));
    const bool fft_ok = M <= maxM && N <= 512;
    const bool direct_ok = direct_smem(R, 3, 1, elem) <= 160 * 1024 && direct_smem(R, 1, 3, elem) <= 160 * 1024;
    int mode;
    if (d->conv_mode == MPI_CONV_FFT) {
        if (!fft_ok) return MPI_ERR_UNSUPPORTED;
        mode = 1;
    } else if (d->conv_mode == MPI_CONV_DIRECT) {
        if (!direct_ok) return MPI_ERR_UNSUPPORTED;
        mode = 0;
    } else {
        // direct while the window is small, FFT otherwise
        mode = (R <= 7 && direct_ok) ? 0 : (fft_ok ? 1 : (direct_ok ? 0 : -1));
        if (mode < 0) return MPI_ERR_UNSUPPORTED;
    }
    Prob& p = L.p;
    std::memset(&p, 0, sizeof(p));
    p.n = N;
    p.nb = nb;
    p.radius = R;
    p.mode = mode;
    p.m = mode ? M : 0;
    p.log2m = mode ? __builtin_ctz(M) : 0;
    p.taps_w = (2 * R + 1 + 3) / 4 * 4;
    p.t = T;
    p.h = d->h;
    const int W = 2 * R + 1, H = M / 2 + 1;
    size_t off = align_up(sizeof(Prob));
    auto take = [&off](size_t bytes) { int64_t o = int64_t(off); off = align_up(off + std::max<size_t>(bytes, 1)); return o; };
    if (mode == 0) p.o_taps = take(size_t(3) * W * p.taps_w * elem);
    if (mode == 1) {
        p.o_spec = take(size_t(3) * H * H * elem);
        p.o_tw = take(size_t(M) * 2 * elem);
    }
    p.o_samp = take(size_t(T) * 4 * elem);
    p.o_perm = take(size_t(T) * 4);
    p.o_bcell = take(size_t(T) * 4);
    p.o_binstart = take((size_t(nb) * nb + 1) * 4);
    p.o_items = take(size_t(4 * T) * 4);
    p.o_cellstart = take((size_t(N) * N + 1) * 4);
    p.o_err = take(16);
    p.o_scratch = int64_t(off);
    L.o_series = take(kSeriesTerms * 8);
    L.o_tab64 = take(size_t(3) * W * W * 8);
    if (mode == 1) {
        L.o_cs = take(size_t(2) * M * 8);
        L.o_U = take(size_t(3) * (R + 1) * H * 8);
    }
    L.o_cell = take(size_t(T) * 4);
    L.o_frac = take(size_t(T) * 16);
    L.o_bincount = take(size_t(nb) * nb * 4);
    L.o_cellcount = take(size_t(N) * N * 4);
    L.o_cursor = take(size_t(nb) * nb * 4);
    L.plan_bytes = off;
    // work memory
    off = 0;
    p.w_g = take(size_t(3) * N * N * elem);
    if (mode == 1) {
        p.w_t1 = take(size_t(3) * H * N * 2 * elem);
        p.w_t2 = take(size_t(3) * N * H * 2 * elem);
    }
    p.w_ysort = take(size_t(T) * 2 * elem);
    p.w_res = take(size_t(T) * 2 * elem);
    p.w_u = take(size_t(N) * N * elem);
    p.w_grad = take(size_t(N) * N * elem);
    L.w_wts = take(32 * 8);
    L.work_bytes = off;
    return MPI_OK;
}

bool misaligned(const void* ptr, size_t a) { return (reinterpret_cast<uintptr_t>(ptr) % a) != 0; }

template <typename K>
hipError_t allow_smem(K kernel, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               int(bytes));
}

template <typename T, template <typename, int> class S>
size_t smem_for(int M) {
    switch (M) {
        case 64: return sizeof(S<T, 64>);
        case 128: return sizeof(S<T, 128>);
        case 256: return sizeof(S<T, 256>);
        case 512: return sizeof(S<T, 512>);
        default: return sizeof(S<T, 1024>);
    }
}

}  // namespace

struct mpi_plan {
    Layout L;
    int dtype = MPI_F32;
    char* plan = nullptr;
    const Prob* dprob = nullptr;
    double wts[32] = {0};
    // cached iteration graph
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    const void *g_s = nullptr, *g_c = nullptr, *g_work = nullptr;
    double g_tau = 0, g_sigma = 0;
    int g_rad = -1;
};

namespace {

#define HIP_TRY(expr)                               \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return MPI_ERR_HIP;   \
    } while (0)

int blocks(int64_t n, int b) { return int((n + b - 1) / b); }

template <typename T>
int build_impl(const mpi_problem* d, Layout& L, char* plan, hipStream_t st) {
    const Prob& p = L.p;
    const Prob* P = reinterpret_cast<const Prob*>(plan);
    const int N = p.n, R = p.radius, W = 2 * R + 1, nb = p.nb;
    HIP_TRY(hipMemcpyAsync(plan, &p, sizeof(Prob), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemsetAsync(plan + p.o_err, 0, 16, st));
    HIP_TRY(hipMemsetAsync(plan + L.o_bincount, 0, size_t(nb) * nb * 4, st));
    double* series = reinterpret_cast<double*>(plan + L.o_series);
    double* tab64 = reinterpret_cast<double*>(plan + L.o_tab64);
    k_series<<<1, 1, 0, st>>>(series);
    T* taps = p.mode == 0 ? reinterpret_cast<T*>(plan + p.o_taps) : nullptr;
    k_table<T><<<blocks(int64_t(W) * W, 256), 256, 0, st>>>(P, plan, series, tab64, taps, 0);
    if (p.mode == 0 && p.taps_w > W)
        k_taps_pad<T><<<blocks(int64_t(3) * W * (p.taps_w - W), 256), 256, 0, st>>>(P, taps);
    if (p.mode == 1) {
        const int M = p.m, H = M / 2 + 1;
        double* cs = reinterpret_cast<double*>(plan + L.o_cs);
        double* U = reinterpret_cast<double*>(plan + L.o_U);
        k_trig<T><<<blocks(M, 256), 256, 0, st>>>(P, cs, reinterpret_cast<cx<T>*>(plan + p.o_tw));
        k_spec_rows<<<blocks(int64_t(3) * (R + 1) * H, 256), 256, 0, st>>>(P, tab64, cs, U);
        k_spec_cols<T><<<blocks(int64_t(3) * H * H, 256), 256, 0, st>>>(P, U, cs, reinterpret_cast<T*>(plan + p.o_spec));
    }
    int* cell = reinterpret_cast<int*>(plan + L.o_cell);
    double* frac = reinterpret_cast<double*>(plan + L.o_frac);
    int* bincount = reinterpret_cast<int*>(plan + L.o_bincount);
    int* cursor = reinterpret_cast<int*>(plan + L.o_cursor);
    int* err = reinterpret_cast<int*>(plan + p.o_err);
    k_bin_prep<T><<<blocks(p.t, 256), 256, 0, st>>>(P, static_cast<const T*>(d->r), cell, frac, bincount, err);
    k_scan<<<1, 1024, 0, st>>>(bincount, reinterpret_cast<int*>(plan + p.o_binstart), nb * nb, cursor);
    k_place<T><<<1, 1024, 1024 * sizeof(int), st>>>(P, cell, frac, static_cast<const T*>(d->v), cursor, plan);
    int* cellcount = reinterpret_cast<int*>(plan + L.o_cellcount);
    k_cell_count<<<blocks(int64_t(N) * N, 256), 256, 0, st>>>(P, plan, cellcount);
    k_scan<<<1, 1024, 0, st>>>(cellcount, reinterpret_cast<int*>(plan + p.o_cellstart), N * N, nullptr);
    k_cell_items<<<blocks(int64_t(N) * N, 256), 256, 0, st>>>(P, plan);
    HIP_TRY(hipGetLastError());
    // smem opt-in for the kernels this plan launches
    if (p.mode == 1) {
        HIP_TRY(allow_smem(k_fwd_cols<T>, smem_for<T, ColSmem>(p.m)));
        HIP_TRY(allow_smem(k_adj_cols<T>, smem_for<T, ColSmem>(p.m)));
        HIP_TRY(allow_smem(k_fwd_rows_gather<T, false>, smem_for<T, GatherSmem>(p.m)));
        HIP_TRY(allow_smem(k_fwd_rows_gather<T, true>, smem_for<T, GatherSmem>(p.m)));
        HIP_TRY(allow_smem(k_adj_scatter_rows<T, false>, smem_for<T, ScatterRowSmem>(p.m)));
        HIP_TRY(allow_smem(k_adj_scatter_rows<T, true>, smem_for<T, ScatterRowSmem>(p.m)));
    } else {
        HIP_TRY(allow_smem(k_conv_direct<T, 1, 3, kDirectSlices, 0>, direct_smem(R, 1, 3, sizeof(T))));
        HIP_TRY(allow_smem(k_conv_direct<T, 3, 1, kDirectSlices, 0>, direct_smem(R, 3, 1, sizeof(T))));
        HIP_TRY(allow_smem(k_conv_direct<T, 3, 1, kDirectSlices, 1>, direct_smem(R, 3, 1, sizeof(T))));
    }
    int herr[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(herr, err, 16, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (herr[0]) return MPI_ERR_DOMAIN;
    return MPI_OK;
}

size_t scatter_rows_smem(int N, int elem) {
    return ((sizeof(ScatterSmem<double>) + 15) / 16) * 16 + size_t(6) * N * elem;
}

// Stages of the forward operator: FFT path {rows, columns, rows + gather},
// direct path {convolution, gather}.  RESID: write A c - y in cell order to the
// work buffer instead of A c in time order to s.
template <typename T, bool RESID>
void fwd_stage(const mpi_plan* pl, int k, const T* c, T* s, char* work, hipStream_t st) {
    const Prob& p = pl->L.p;
    const char* plan = pl->plan;
    const Prob* P = pl->dprob;
    const int N = p.n;
    if (p.mode == 1) {
        const int M = p.m, H = M / 2 + 1;
        if (k == 0) k_fwd_rows<T><<<dim3((N + 1) / 2, 1), 64, smem_for<T, RowSmem>(M), st>>>(P, c, plan, work);
        if (k == 1) k_fwd_cols<T><<<dim3(H, 1), 192, smem_for<T, ColSmem>(M), st>>>(P, plan, work);
        if (k == 2)
            k_fwd_rows_gather<T, RESID><<<dim3(p.nb, 1), 192, smem_for<T, GatherSmem>(M), st>>>(P, s, plan, work);
    } else {
        const int tiles = (N + kTile - 1) / kTile;
        T* G = reinterpret_cast<T*>(work + p.w_g);
        if (k == 0)
            k_conv_direct<T, 1, 3, kDirectSlices, 0><<<dim3(tiles, tiles, 1), 64 * kDirectSlices,
                                                        direct_smem(p.radius, 1, 3, sizeof(T)), st>>>(
                P, c, G, nullptr, 0.0, plan, 1, 0);
        if (k == 1)
            k_gather_rows<T, RESID><<<dim3(p.nb, 1), 256, size_t(6) * N * sizeof(T), st>>>(P, G, s, plan, work);
    }
}

// Stages of the transpose: FFT path {scatter + rows, columns, rows}, direct
// path {scatter, convolution}.  SORTED: the signal is the residual already in
// cell order in the work buffer.  EPI 0: c_out = A^T s; EPI 1: c_out = c_in - tau A^T r.
template <typename T, bool SORTED, int EPI>
void adj_stage(const mpi_plan* pl, int k, const T* s, T* c_out, const T* c_in, double tau, char* work,
               hipStream_t st) {
    const Prob& p = pl->L.p;
    const char* plan = pl->plan;
    const Prob* P = pl->dprob;
    const int N = p.n;
    if (p.mode == 1) {
        const int M = p.m, H = M / 2 + 1;
        if (k == 0)
            k_adj_scatter_rows<T, SORTED><<<dim3((N + 1) / 2, 1), 192, smem_for<T, ScatterRowSmem>(M), st>>>(
                P, s, plan, work);
        if (k == 1) k_adj_cols<T><<<dim3(H, 1), 192, smem_for<T, ColSmem>(M), st>>>(P, plan, work);
        if (k == 2)
            k_adj_rows<T, EPI><<<dim3((N + 1) / 2, 1), 64, smem_for<T, RowSmem>(M), st>>>(P, c_out, c_in, tau, plan,
                                                                                         work);
    } else {
        const int tiles = (N + kTile - 1) / kTile;
        T* G = reinterpret_cast<T*>(work + p.w_g);
        if (k == 0)
            k_scatter_rows<T, SORTED><<<dim3((N + 1) / 2, 1), 192, scatter_rows_smem(N, sizeof(T)), st>>>(
                P, s, G, plan, work);
        if (k == 1)
            k_conv_direct<T, 3, 1, kDirectSlices, EPI><<<dim3(tiles, tiles, 1), 64 * kDirectSlices,
                                                          direct_smem(p.radius, 3, 1, sizeof(T)), st>>>(
                P, G, c_out, c_in, tau, plan, 0, 1);
    }
}

int stage_count(const Prob& p) { return p.mode == 1 ? 3 : 2; }

template <typename T>
int forward_impl(const mpi_plan* pl, const T* c, T* s, char* work, hipStream_t st) {
    for (int k = 0; k < stage_count(pl->L.p); ++k) fwd_stage<T, false>(pl, k, c, s, work, st);
    return hipGetLastError() == hipSuccess ? MPI_OK : MPI_ERR_HIP;
}

template <typename T, bool SORTED, int EPI>
int adjoint_impl(const mpi_plan* pl, const T* s, T* c_out, const T* c_in, double tau, char* work, hipStream_t st) {
    for (int k = 0; k < stage_count(pl->L.p); ++k) adj_stage<T, SORTED, EPI>(pl, k, s, c_out, c_in, tau, work, st);
    return hipGetLastError() == hipSuccess ? MPI_OK : MPI_ERR_HIP;
}

// One iteration c <- D(c - tau A^T (A c - s)); the measured signal is already
// in cell order (work.ysort).
template <typename T>
int iteration_impl(const mpi_plan* pl, T* c, double tau, bool denoise, int rad, char* work, hipStream_t st) {
    const Prob& p = pl->L.p;
    const int N = p.n;
    for (int k = 0; k < stage_count(p); ++k) fwd_stage<T, true>(pl, k, c, nullptr, work, st);
    T* u = reinterpret_cast<T*>(work + p.w_u);
    int rc = adjoint_impl<T, true, 1>(pl, nullptr, denoise ? u : c, c, tau, work, st);
    if (rc != MPI_OK) return rc;
    if (denoise) {
        const int tiles = (N + kDnTile - 1) / kDnTile;
        k_denoise<T><<<dim3(tiles, tiles, 1), 256, 0, st>>>(pl->dprob, u, c,
                                                            reinterpret_cast<const double*>(work + pl->L.w_wts), rad);
    }
    return hipGetLastError() == hipSuccess ? MPI_OK : MPI_ERR_HIP;
}

int check_call(const mpi_plan* pl, const void* a, const void* b, const void* work, size_t work_bytes) {
    if (!pl || !a || !b || !work) return MPI_ERR_ARG;
    if (work_bytes < pl->L.work_bytes) return MPI_ERR_WORKSPACE;
    if (misaligned(work, kAlign)) return MPI_ERR_ARG;
    const size_t el = pl->L.elem;
    if (misaligned(a, el) || misaligned(b, el)) return MPI_ERR_ARG;
    return MPI_OK;
}

}  // namespace

extern "C" {

int mpi_abi_version(void) { return MPIK_ABI_VERSION; }

const char* mpi_status_str(int status) {
    switch (status) {
        case MPI_OK: return "ok";
        case MPI_ERR_ARG: return "invalid argument";
        case MPI_ERR_DOMAIN: return "trajectory sample outside the grid";
        case MPI_ERR_WORKSPACE: return "plan or work buffer too small";
        case MPI_ERR_DTYPE: return "unknown dtype";
        case MPI_ERR_HIP: return "HIP runtime error";
        case MPI_ERR_UNSUPPORTED: return "unsupported option";
        default: return "unknown status";
    }
}

int mpi_plan_bytes(const mpi_problem* prob, size_t* plan_bytes, size_t* work_bytes) {
    if (!plan_bytes || !work_bytes) return MPI_ERR_ARG;
    Layout L;
    const int rc = make_layout(prob, L);
    if (rc != MPI_OK) return rc;
    *plan_bytes = L.plan_bytes;
    *work_bytes = L.work_bytes;
    return MPI_OK;
}

int mpi_kernel_build(const mpi_problem* prob, void* plan_mem, size_t plan_bytes, hipStream_t stream, mpi_plan** out) {
    if (!out) return MPI_ERR_ARG;
    *out = nullptr;
    Layout L;
    int rc = make_layout(prob, L);
    if (rc != MPI_OK) return rc;
    if (!plan_mem || !prob->r || !prob->v) return MPI_ERR_ARG;
    if (misaligned(plan_mem, kAlign)) return MPI_ERR_ARG;
    if (misaligned(prob->r, L.elem) || misaligned(prob->v, L.elem)) return MPI_ERR_ARG;
    if (plan_bytes < L.plan_bytes) return MPI_ERR_WORKSPACE;
    mpi_plan* pl = new (std::nothrow) mpi_plan;
    if (!pl) return MPI_ERR_ARG;
    pl->L = L;
    pl->dtype = prob->dtype;
    pl->plan = static_cast<char*>(plan_mem);
    pl->dprob = static_cast<const Prob*>(plan_mem);
    rc = prob->dtype == MPI_F64 ? build_impl<double>(prob, pl->L, pl->plan, stream)
                                : build_impl<float>(prob, pl->L, pl->plan, stream);
    if (rc != MPI_OK) {
        delete pl;
        return rc;
    }
    *out = pl;
    return MPI_OK;
}

int mpi_plan_info(const mpi_plan* plan, int32_t* radius, int32_t* fft_size, int32_t* conv_mode) {
    if (!plan) return MPI_ERR_ARG;
    if (radius) *radius = plan->L.p.radius;
    if (fft_size) *fft_size = plan->L.p.m;
    if (conv_mode) *conv_mode = plan->L.p.mode ? MPI_CONV_FFT : MPI_CONV_DIRECT;
    return MPI_OK;
}

int mpi_forward(const mpi_plan* plan, const void* c, void* s, void* work, size_t work_bytes, hipStream_t stream) {
    int rc = check_call(plan, c, s, work, work_bytes);
    if (rc != MPI_OK) return rc;
    if (hipPeekAtLastError() != hipSuccess) return MPI_ERR_HIP;
    char* w = static_cast<char*>(work);
    return plan->dtype == MPI_F64
               ? forward_impl<double>(plan, static_cast<const double*>(c), static_cast<double*>(s), w, stream)
               : forward_impl<float>(plan, static_cast<const float*>(c), static_cast<float*>(s), w, stream);
}

int mpi_adjoint(const mpi_plan* plan, const void* s, void* c, void* work, size_t work_bytes, hipStream_t stream) {
    int rc = check_call(plan, s, c, work, work_bytes);
    if (rc != MPI_OK) return rc;
    if (hipPeekAtLastError() != hipSuccess) return MPI_ERR_HIP;
    char* w = static_cast<char*>(work);
    return plan->dtype == MPI_F64
               ? adjoint_impl<double, false, 0>(plan, static_cast<const double*>(s), static_cast<double*>(c), nullptr,
                                                0.0, w, stream)
               : adjoint_impl<float, false, 0>(plan, static_cast<const float*>(s), static_cast<float*>(c), nullptr,
                                               0.0, w, stream);
}

}  // extern "C"

namespace {

template <typename T>
int iterate_impl(mpi_plan* pl, const T* s, T* c, const mpi_iter_params* ip, char* work, hipStream_t st) {
    const Prob& p = pl->L.p;
    const bool denoise = ip->denoise_sigma_px > 0.0;
    const int rad = denoise ? ip->denoise_radius : 0;
    if (denoise) {
        double sum = 0.0;
        for (int k = -rad; k <= rad; ++k) {
            pl->wts[k + rad] = std::exp(-0.5 * k * k / (ip->denoise_sigma_px * ip->denoise_sigma_px));
            sum += pl->wts[k + rad];
        }
        for (int k = 0; k <= 2 * rad; ++k) pl->wts[k] /= sum;
        HIP_TRY(hipMemcpyAsync(work + pl->L.w_wts, pl->wts, sizeof(double) * (2 * rad + 1), hipMemcpyHostToDevice, st));
    }
    k_permute_signal<T><<<dim3(blocks(p.t, 256), 1), 256, 0, st>>>(pl->dprob, s, pl->plan, work);
    HIP_TRY(hipGetLastError());
    if (ip->n_iter == 0) return MPI_OK;
    if (!ip->use_graph) {
        for (int it = 0; it < ip->n_iter; ++it) {
            const int rc = iteration_impl<T>(pl, c, ip->tau, denoise, rad, work, st);
            if (rc != MPI_OK) return rc;
        }
        return MPI_OK;
    }
    const bool same = pl->gexec && pl->g_s == s && pl->g_c == c && pl->g_work == work && pl->g_tau == ip->tau &&
                      pl->g_sigma == (denoise ? ip->denoise_sigma_px : 0.0) && pl->g_rad == rad;
    if (!same) {
        if (pl->gexec) {
            HIP_TRY(hipStreamSynchronize(st));
            (void)hipGraphExecDestroy(pl->gexec);
            (void)hipGraphDestroy(pl->graph);
            pl->gexec = nullptr;
            pl->graph = nullptr;
        }
        hipStream_t cap;
        HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        int rc = MPI_ERR_HIP;
        if (e == hipSuccess) {
            rc = iteration_impl<T>(pl, c, ip->tau, denoise, rad, work, cap);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(cap, &g);
            if (e == hipSuccess && rc == MPI_OK) {
                e = hipGraphInstantiate(&pl->gexec, g, nullptr, nullptr, 0);
                if (e == hipSuccess) pl->graph = g;
                else (void)hipGraphDestroy(g);
            } else if (g) {
                (void)hipGraphDestroy(g);
            }
        }
        (void)hipStreamDestroy(cap);
        if (e != hipSuccess || rc != MPI_OK || !pl->gexec) {
            pl->gexec = nullptr;
            return MPI_ERR_HIP;
        }
        pl->g_s = s;
        pl->g_c = c;
        pl->g_work = work;
        pl->g_tau = ip->tau;
        pl->g_sigma = denoise ? ip->denoise_sigma_px : 0.0;
        pl->g_rad = rad;
    }
    for (int it = 0; it < ip->n_iter; ++it) HIP_TRY(hipGraphLaunch(pl->gexec, st));
    return MPI_OK;
}

}  // namespace

extern "C" {

int mpi_iterate(const mpi_plan* plan, const void* s, void* c, const mpi_iter_params* params, void* work,
                size_t work_bytes, hipStream_t stream) {
    int rc = check_call(plan, s, c, work, work_bytes);
    if (rc != MPI_OK) return rc;
    if (!params || params->n_iter < 0 || !std::isfinite(params->tau)) return MPI_ERR_ARG;
    if (params->denoise_sigma_px > 0.0 && (params->denoise_radius < 0 || params->denoise_radius > kDnMaxR))
        return MPI_ERR_ARG;
    if (hipPeekAtLastError() != hipSuccess) return MPI_ERR_HIP;
    mpi_plan* pl = const_cast<mpi_plan*>(plan);
    char* w = static_cast<char*>(work);
    return plan->dtype == MPI_F64
               ? iterate_impl<double>(pl, static_cast<const double*>(s), static_cast<double*>(c), params, w, stream)
               : iterate_impl<float>(pl, static_cast<const float*>(s), static_cast<float*>(c), params, w, stream);
}

int mpi_stage_count(const mpi_plan* plan) {
    if (!plan) return MPI_ERR_ARG;
    return 2 * stage_count(plan->L.p);
}

const char* mpi_stage_name(const mpi_plan* plan, int stage) {
    static const char* fft_names[] = {"fwd_rows", "fwd_cols", "fwd_rows_gather",
                                      "adj_scatter_rows", "adj_cols", "adj_rows"};
    static const char* direct_names[] = {"conv_direct_fwd", "gather_rows", "scatter_rows", "conv_direct_adj"};
    if (!plan || stage < 0 || stage >= 2 * stage_count(plan->L.p)) return nullptr;
    return plan->L.p.mode == 1 ? fft_names[stage] : direct_names[stage];
}

int mpi_stage_launch(const mpi_plan* plan, int stage, int reps, void* c, void* s, void* work,
                     size_t work_bytes, hipStream_t stream) {
    int rc = check_call(plan, c, s, work, work_bytes);
    if (rc != MPI_OK) return rc;
    const int ns = stage_count(plan->L.p);
    if (stage < 0 || stage >= 2 * ns || reps < 0) return MPI_ERR_ARG;
    char* w = static_cast<char*>(work);
    for (int r = 0; r < reps; ++r) {
        if (plan->dtype == MPI_F64) {
            if (stage < ns) fwd_stage<double, false>(plan, stage, static_cast<const double*>(c), static_cast<double*>(s), w, stream);
            else adj_stage<double, false, 0>(plan, stage - ns, static_cast<const double*>(s), static_cast<double*>(c),
                                            nullptr, 0.0, w, stream);
        } else {
            if (stage < ns) fwd_stage<float, false>(plan, stage, static_cast<const float*>(c), static_cast<float*>(s), w, stream);
            else adj_stage<float, false, 0>(plan, stage - ns, static_cast<const float*>(s), static_cast<float*>(c),
                                           nullptr, 0.0, w, stream);
        }
    }
    return hipGetLastError() == hipSuccess ? MPI_OK : MPI_ERR_HIP;
}

int mpi_plan_destroy(mpi_plan* plan) {
    if (!plan) return MPI_ERR_ARG;
    if (plan->gexec) {
        (void)hipDeviceSynchronize();
        (void)hipGraphExecDestroy(plan->gexec);
        (void)hipGraphDestroy(plan->graph);
    }
    delete plan;
    return MPI_OK;
}

}  // extern "C"
