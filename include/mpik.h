/*
 * mpik.h -- C ABI of the MI355X (gfx950) library for the model operator of
 * trajectory-independent, model-based Magnetic Particle Imaging.
 *
 * Operator (Gapyak, Maerz, Weinmann, arXiv 2505.22797, Section "Methods"):
 *   the MPI kernel K (eq. kernel:matrix), rescaled K_h(y) = K(y/h)/h, is
 *   convolved with the particle concentration (eq. coreoperator), the
 *   matrix-valued result is sampled along the field-free-point trajectory
 *   r(t) and contracted with its velocity v(t) (eq. core:formula):
 *       s_k = A_h[c](r_k) v_k.
 *   A maps the concentration c to the signal s; A^T is its exact transpose.
 *
 * Discretisation (the readings the library and its tests share):
 *   - N x N cell-centred grid over the field of view [-1, 1]^2, pitch
 *     delta = 2/N, centre x_i = -1 + (i + 1/2) delta; c is row-major
 *     c[j][i] with j the y index;
 *   - the convolution is the Riemann sum delta^2 * sum_d K_h(delta d) c[. - d]
 *     over integer offsets |d_x|, |d_y| <= R (square window, zero outside the
 *     grid); R >= N-1 is the untruncated kernel;
 *   - the field is interpolated between the four surrounding cell centres
 *     (bilinear or cosine weights, see MPI_INTERP_*); a sample needs
 *     g = (r + 1)/delta - 1/2 in [0, N-1] on both axes;
 *   - s is [T][2] interleaved (x, y), matching a contiguous (T, 2) tensor;
 *     signal buffers the library writes must be aligned to two elements
 *     (else MPI_ERR_ARG).
 *
 * Memory ownership: the caller owns every device buffer -- inputs, outputs,
 * the plan memory and the work memory.  The library never allocates device
 * memory.  An mpi_plan is a small host object owned by the library
 * (mpi_plan_destroy frees it); it refers into the caller's plan memory, which
 * must outlive it.  A plan's results are fixed at the build; only its launch
 * schedule may change later (mpi_batch_schedule), which never changes them.
 * The buffers an apply call writes (its outputs and the work memory) must not
 * share a byte with any other buffer of the call, except where a call says
 * it works in place (mpi_iterate's c; mpi_batch_adjoint_step with c_out ==
 * c_in); buffers it only reads may share memory.  Every call except the
 * per-stage diagnostics (mpi_stage_launch) compares the byte ranges that the
 * plan or its size arguments give each buffer and returns MPI_ERR_ARG on an
 * overlap, before anything is enqueued.  Calls on different
 * streams may run concurrently if each passes its own work buffer.  A batch
 * whose problems use several FFT sizes (or both paths) runs each group on a
 * side stream of the plan, forked from and joined back to the caller's
 * stream; the plan creates them at build and destroys them with the plan.
 *
 * Errors: every call returns an mpi_status; nothing throws or aborts across
 * the ABI.  Argument errors are found on the host before anything is
 * enqueued.  Every apply call only enqueues work on the given stream and
 * never synchronises (except where its description says so); a fault of an
 * earlier kernel surfaces as MPI_ERR_HIP on a later call.  mpi_kernel_build synchronises its stream once, to report
 * samples outside the grid (MPI_ERR_DOMAIN).
 */
#ifndef MPIK_H
#define MPIK_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPIK_ABI_VERSION 2

typedef enum {
    MPI_OK = 0,
    MPI_ERR_ARG = -1,          /* NULL pointer, bad size, misaligned pointer  */
    MPI_ERR_DOMAIN = -2,       /* a trajectory sample lies outside the grid   */
    MPI_ERR_WORKSPACE = -3,    /* plan or work buffer smaller than required   */
    MPI_ERR_DTYPE = -4,        /* unknown dtype                               */
    MPI_ERR_HIP = -5,          /* HIP runtime error (incl. earlier faults)    */
    MPI_ERR_UNSUPPORTED = -6,  /* valid but not implemented option            */
    MPI_ERR_ALLOC = -7         /* host memory allocation failed               */
} mpi_status;

enum { MPI_F32 = 0, MPI_F64 = 1 };
enum { MPI_CONV_AUTO = 0, MPI_CONV_DIRECT = 1, MPI_CONV_FFT = 2 };
/* Interpolation of the field between the four surrounding cell centres, per
 * axis with weight w(f) on the upper neighbour and 1 - w(f) on the lower one,
 * f the fraction of the way between them: f (bilinear), or (1 - cos pi f)/2,
 * the cosine interpolation the paper names for the core stage (section on
 * the core stage; the formula is the textbook scheme, C^1 across cells). */
enum { MPI_INTERP_BILINEAR = 0, MPI_INTERP_COSINE = 1 };
/* Receive channels: both, or the x channel alone (Section "Experiment 2":
 * s_x = (A_xx, A_xy) v; the library writes s_y = 0 and ignores the y
 * components of the signals it reads; the Deconvolution Stage then inverts
 * the convolution with K_xx in place of the trace kernel). */
enum { MPI_CH_XY = 0, MPI_CH_X = 1 };

/* One reconstruction problem.  r and v are device pointers to [T][2] arrays
 * of the given dtype, read only during mpi_kernel_build. */
typedef struct {
    int32_t n;             /* grid side N, 2 <= N <= 1024                      */
    int32_t dtype;         /* MPI_F32 or MPI_F64: every array of the problem   */
    double h;              /* kernel resolution in field-of-view units, > 0    */
    int32_t radius;        /* window half-width R >= 0 in pixels; capped N-1   */
    int32_t conv_mode;     /* MPI_CONV_*: selects speed only, never the result */
    int32_t interp;        /* MPI_INTERP_BILINEAR or MPI_INTERP_COSINE         */
    int32_t channels;      /* MPI_CH_XY or MPI_CH_X                            */
    int64_t n_samples;     /* T >= 1, T < 2^26                                 */
    const void* r;         /* device [T][2] sample positions r_k               */
    const void* v;         /* device [T][2] velocities: -G dr/dt(t_k) (= dr/dt  */
                           /* for the isotropic G = -I)                        */
    double grad_x, grad_y; /* selection-field gradient G = diag(grad_x, grad_y) */
                           /* in units of the isotropic one: the kernel is     */
                           /* evaluated at G y (Section "Experiment 2"); both  */
                           /* 0 means (1, 1), else both finite and nonzero     */
} mpi_problem;

/* Parameters of mpi_iterate: c <- D(c - tau A^T (A c - s)), n_iter times.
 * D is the identity when denoise_sigma_px <= 0, else a separable Gaussian of
 * standard deviation denoise_sigma_px pixels and half-width denoise_radius
 * (weights normalised to sum 1, zero padding) -- a stand-in for the learned
 * denoiser of the half-quadratic-splitting loop (eqs. dec:sub:tik and
 * dec:sub:den). */
typedef struct {
    int32_t n_iter;            /* >= 0                                         */
    double tau;                /* step size (the caller's 1/lambda_max(A^T A)) */
    double denoise_sigma_px;   /* <= 0: no denoiser                            */
    int32_t denoise_radius;    /* 0..8                                         */
    int32_t use_graph;         /* 1: capture one iteration as a HIP graph and  */
                               /*    replay it (needs a non-null stream)       */
} mpi_iter_params;
/* With use_graph the captured graphs stay in the plan, keyed by the buffers
 * (s, c, work) and the denoiser.  A call with other buffers or another
 * denoiser records them again after synchronising its own stream, so such a
 * call must be on the stream of the plan's previous graph-replayed call, or
 * come after that call's work has finished; and graph-replayed calls on one
 * plan come from one host thread at a time (the same holds for the
 * Deconvolution and Core Stage solvers, which replay cached graphs too). */

typedef struct mpi_plan mpi_plan;

/* Bytes of plan memory (kept for the plan's lifetime) and of work memory
 * (scratch for each apply call) the problem needs.  Host-only; validates the
 * descriptor (except the sample positions, checked by the build). */
int mpi_plan_bytes(const mpi_problem* prob, size_t* plan_bytes, size_t* work_bytes);

/* Build the plan in caller-owned device memory plan_mem (256-byte aligned,
 * >= plan_bytes): the kernel table K_h(delta d) for |d_x|,|d_y| <= R
 * (eq. kernel:matrix, computed in float64 on the device), its spectra for
 * the FFT path, and the sample-to-cell binning (base cell, bilinear fractions
 * in float64, a stable sort by cell).  Enqueued on `stream`, then the stream
 * is synchronised once; returns MPI_ERR_DOMAIN if a sample is outside the
 * grid.  On success *out receives a new host plan object. */
int mpi_kernel_build(const mpi_problem* prob, void* plan_mem, size_t plan_bytes,
                     hipStream_t stream, mpi_plan** out);

/* s = A c (eq. core:formula).  c: device [N][N], s: device [T][2], both of
 * the plan's dtype; s is overwritten.  work: >= work_bytes, 256-byte aligned. */
int mpi_forward(const mpi_plan* plan, const void* c, void* s,
                void* work, size_t work_bytes, hipStream_t stream);

/* c = A^T s, the exact transpose of mpi_forward.  The sampling transpose is
 * deterministic: contributions are summed per cell in a fixed order, without
 * floating-point atomics, so repeated calls give bitwise identical results. */
int mpi_adjoint(const mpi_plan* plan, const void* s, void* c,
                void* work, size_t work_bytes, hipStream_t stream);

/* c <- D(c - tau A^T(A c - s)) repeated params->n_iter times, in place on c
 * (device [N][N], holding c_0 on entry).  s: device [T][2]. */
int mpi_iterate(const mpi_plan* plan, const void* s, void* c, const mpi_iter_params* params,
                void* work, size_t work_bytes, hipStream_t stream);

/* Query a built plan (its first problem): effective radius, FFT size (0 on
 * the direct path) and the convolution path taken (MPI_CONV_DIRECT or
 * MPI_CONV_FFT). */
int mpi_plan_info(const mpi_plan* plan, int32_t* radius, int32_t* fft_size, int32_t* conv_mode);

/* ---------------------------------------------------------------- batches --
 * Many independent problems (different N, T, h, R, trajectories) in one plan:
 * every stage of the forward operator, its transpose and the iteration is one
 * launch over the whole batch.  The concentrations of all problems are
 * concatenated in one buffer (problem b at element offset c_off[b], N_b^2
 * elements each) and so are the signals (s_off[b], 2 T_b elements each);
 * mpi_batch_offsets reports both (count + 1 entries each, the last one the
 * total).  All problems share one dtype.
 *
 * With MPI_BUILD_TUNE and a work buffer of at least work_bytes, problems whose
 * conv_mode is MPI_CONV_AUTO (and that fit both paths) are built for both
 * convolution paths and the faster one -- FFT, or the direct path with 4, 8 or
 * 16 waves splitting a tile's window rows -- is kept, timed with HIP events on
 * `stream`.  Choices are cached per (dtype, N, R, log2 T) in the process and
 * appended to the file named by the environment variable MPIK_TUNE_CACHE. */
enum { MPI_BUILD_TUNE = 1 };
/* Shape of the column-FFT kernels: by default three waves share a column
 * when the plan holds one or two problems (shortest latency) and one wave
 * owns a column otherwise (most columns in flight).  These flags force one
 * shape.  Both compute the same values; they may differ in the last bit
 * because the channel sum is contracted into multiply-adds differently. */
enum { MPI_BUILD_COL_SPLIT = 2, MPI_BUILD_COL_WAVE = 4 };
/* Also build the tables of dK_h/dh (plan memory grows by one table or one set
 * of spectra per problem) and every sample's interpolation-weight slopes
 * d w/d f (two values per sample); needed by mpi_batch_forward_dh,
 * mpi_batch_traj_vjp and mpi_batch_unrolled_vjp. */
enum { MPI_BUILD_DERIV = 8 };
/* Direct-path problems use this many waves splitting a tile's window rows
 * (one flag at most, else MPI_ERR_ARG), instead of 8 or the tuner's choice;
 * the path choice of MPI_BUILD_TUNE is then left to the batch-size rule.
 * Every count computes the same operator; the waves' partial sums are added
 * in a fixed order, so results may differ in the last bits between counts.
 * For tests and tuning studies. */
enum { MPI_BUILD_SLICES_4 = 16, MPI_BUILD_SLICES_8 = 32, MPI_BUILD_SLICES_16 = 64 };

/* Plan and work bytes of a batch built with `flags` (MPI_BUILD_*).  Problems
 * that have the same kernel -- equal n, effective radius, h, grad_x, grad_y
 * and requested conv_mode -- share one copy of the kernel tables (spectra,
 * twiddles, direct-path taps and their dK_h/dh versions), built once for the
 * first of them; the plan holds that copy only, and the apply stages of a
 * batch of such problems read it from cache.  Results are those of separate
 * copies, bitwise. */
int mpi_batch_bytes(const mpi_problem* probs, int count, int flags, size_t* plan_bytes, size_t* work_bytes);
int mpi_batch_build(const mpi_problem* probs, int count, void* plan_mem, size_t plan_bytes,
                    void* work, size_t work_bytes, int flags, hipStream_t stream, mpi_plan** out);
int mpi_batch_count(const mpi_plan* plan);
int mpi_batch_offsets(const mpi_plan* plan, int64_t* c_offsets, int64_t* s_offsets);
/* per problem: effective radius, FFT size (0: direct), path, direct-path wave slices */
int mpi_batch_info(const mpi_plan* plan, int index, int32_t* radius, int32_t* fft_size,
                   int32_t* conv_mode, int32_t* slices);
/* s_all = A_b c_b for every problem b, one launch per stage */
int mpi_batch_forward(const mpi_plan* plan, const void* c_all, void* s_all,
                      void* work, size_t work_bytes, hipStream_t stream);
/* c_all = A_b^T s_b for every problem b */
int mpi_batch_adjoint(const mpi_plan* plan, const void* s_all, void* c_all,
                      void* work, size_t work_bytes, hipStream_t stream);
/* s_all = A_b c_b and then g_all = A_b^T s_b for every problem b in one call
 * (the operator of eq. model and its exact transpose, the pair applied in
 * Landweber, power and normal-equation iterations).  Same buffers and layout
 * as mpi_batch_forward (c_all, s_all) and mpi_batch_adjoint (s_all -> g_all);
 * g_all must not alias c_all or s_all.  Results are those of the two separate
 * calls, bitwise.  Unlike the two calls, each problem range of a batch (the
 * plan splits batches of 16 or more problems into ranges on its own side
 * streams) starts its transpose as soon as its own forward is done.
 * Enqueued on `stream`. */
int mpi_batch_pair(const mpi_plan* plan, const void* c_all, void* s_all, void* g_all,
                   void* work, size_t work_bytes, hipStream_t stream);
/* Launch schedule of a batch: each FFT-size group of the batch is split into
 * `ranges` contiguous problem ranges, each range on its own side stream, so
 * that the stages of different ranges overlap (the direct-path problems stay
 * on the caller's stream).  The build picks the count from the batch size
 * (one size group: 4 ranges below 48 problems, 2 from 48 on; two groups: 2
 * each; fewer than 16 problems: 1).  Results never depend on it: every problem
 * runs the same kernels in any split.
 *   ranges < 0: only report the count in use; c, s, g and work may be NULL.
 *   ranges > 0: use that count (1 .. min(count, 8 / size groups), else
 *               MPI_ERR_ARG); c, s, g and work may be NULL.
 *   ranges = 0: reserved for choosing the count by timing the pair;
 *               switched off (MPI_ERR_UNSUPPORTED): its graph-captured timing
 *               runs once ended in a host-side fault whose cause is not
 *               established.
 * The count in use is written to *chosen (may be NULL).  Changing it
 * re-creates the plan's side streams and synchronises `stream`; no other call
 * may use the plan meanwhile.  Only a plan that has not yet recorded a graph
 * (a graph-replayed iteration, CG or Core Stage call) may change it: after
 * that, a different count returns MPI_ERR_UNSUPPORTED and the plan keeps its
 * schedule (a capture after the side streams were re-created ended a process
 * with a host-side fault whose cause is not established).  Set the schedule
 * right after the build. */
int mpi_batch_schedule(mpi_plan* plan, int32_t ranges, const void* c_all, void* s_all, void* g_all,
                       void* work, size_t work_bytes, hipStream_t stream, int32_t* chosen);

/* Allocation-free pair, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): mpi_batch_pair with the work memory taken from a fixed array
 * that the library's code object holds on every GPU it is loaded on (one
 * array per GPU, MPI_NOALLOC_SCRATCH_BYTES bytes, kept until the process
 * ends; the plan records its GPU's copy at the build).  The caller still
 * passes the inputs and outputs, with mpi_batch_pair's layouts and rules.
 * Plans whose work memory (mpi_batch_bytes) exceeds the array return
 * MPI_ERR_WORKSPACE before anything is enqueued.  Nothing is allocated:
 * no hipMalloc, hipFree or allocating library call.  Every call on one GPU
 * shares that GPU's array, so calls that overlap in time on one GPU (other
 * streams, other host threads) race and must be serialised by the caller;
 * nothing in the array needs to start at zero.  Enqueued on `stream`. */
#define MPI_NOALLOC_SCRATCH_BYTES (64u << 20)
int mpi_batch_pair_noalloc(const mpi_plan* plan, const void* c_all, void* s_all, void* g_all,
                           hipStream_t stream);
/* c_b <- D(c_b - taus[b] A_b^T (A_b c_b - s_b)), params->n_iter times for all
 * problems at once (params->tau is ignored; taus is a host array of count). */
int mpi_batch_iterate(const mpi_plan* plan, const void* s_all, void* c_all,
                      const mpi_iter_params* params, const double* taus,
                      void* work, size_t work_bytes, hipStream_t stream);

/* ------------------------------------------------------------ derivatives --
 * Building blocks of hand-written vector-Jacobian products, all batched like
 * mpi_batch_forward (concatenated buffers, one launch per stage):
 *
 * mpi_batch_forward_dh: s = (dA/dh) x -- the sampling and contraction of the
 *   convolution of x with delta^2 dK_h/dh, where dK_h/dh =
 *   -h^-2 [(L'(r) + r L''(r)) P + L'(r)(I - P)] (r = |y|/h, P = y y^T/|y|^2;
 *   -I/(3h^2) at the origin), the h-derivative of K_h(y) = K(y/h)/h of
 *   eq. kernel:matrix.  Needs a plan built with MPI_BUILD_DERIV.
 *
 * mpi_batch_residual: out = A c - y (y and out signal-shaped, time order).
 *
 * mpi_batch_traj_vjp: for the field G = K_h * x and signal-shaped y, the
 *   gradients of <y, A x> with respect to every sample's position and
 *   velocity: g_r[k] = (y_k^T M(dG/dx) v_k, y_k^T M(dG/dy) v_k),
 *   g_v[k] = M(G(r_k)) y_k, with M(g) the symmetric 2x2 field and the spatial
 *   derivatives taken inside the sample's interpolation patch (its base cell
 *   held fixed: the bilinear interpolant is only piecewise smooth; the cosine
 *   one is C^1, so there the result is the derivative itself).  Time order, [T][2].
 *   Needs a plan built with MPI_BUILD_DERIV.
 *
 * mpi_batch_adjoint_step: c_out = c_in - taus[b] A^T s (s in time order;
 *   c_in may equal c_out).  taus is a host array of count values.
 *
 * mpi_batch_denoise: c = D(u), the separable Gaussian of mpi_iter_params
 *   (sigma_px > 0, radius 0..8, weights summing to 1, zero padding); u and c
 *   must not overlap.
 *   D is symmetric, so it is also its own transpose.
 *
 * mpi_batch_dot: out[b] = sum a_b . b_b in float64 for every problem, with a
 *   fixed summation order (deterministic).  space 0: signal-shaped arrays
 *   (comp 0: x components only, 1: y only, 2: both); space 1: concentration-
 *   shaped.  out: device array of count doubles. */
int mpi_batch_forward_dh(const mpi_plan* plan, const void* x_all, void* s_all,
                         void* work, size_t work_bytes, hipStream_t stream);
int mpi_batch_residual(const mpi_plan* plan, const void* c_all, const void* y_all, void* out_all,
                       void* work, size_t work_bytes, hipStream_t stream);
int mpi_batch_traj_vjp(const mpi_plan* plan, const void* x_all, const void* y_all,
                       void* g_r_all, void* g_v_all, void* work, size_t work_bytes, hipStream_t stream);
int mpi_batch_adjoint_step(const mpi_plan* plan, const void* s_all, const void* c_in_all,
                           void* c_out_all, const double* taus, void* work, size_t work_bytes,
                           hipStream_t stream);
int mpi_batch_denoise(const mpi_plan* plan, const void* u_all, void* c_all, double sigma_px,
                      int radius, void* work, size_t work_bytes, hipStream_t stream);
int mpi_batch_dot(const mpi_plan* plan, const void* a_all, const void* b_all, int space, int comp,
                  double* out, void* work, size_t work_bytes, hipStream_t stream);

/* Composite vector-Jacobian products of the operator in its parameters
 * theta = (c or y, h, r_k, v_k), the compositions of the building blocks above
 * that reverse-mode differentiation of s = A c and c' = A^T y needs; plans built
 * with MPI_BUILD_DERIV (else MPI_ERR_UNSUPPORTED).  All arrays batched as in
 * mpi_batch_forward; g_h is a device array of count doubles; g_r and g_v are
 * signal-shaped, time order.  Every output buffer is distinct from every
 * input and from each other.
 *
 * mpi_vjp_forward: for s = A c and an upstream gradient gs (signal-shaped):
 *   gc = A^T gs, g_h[b] = <(dA/dh) c, gs>_b, and g_r, g_v the gradients of
 *   <gs, A c> in every sample's position and velocity (as mpi_batch_traj_vjp
 *   with x = c, y = gs).
 * mpi_vjp_adjoint: for c' = A^T y and an upstream gradient gc (concentration-
 *   shaped), using <gc, A^T y> = <A gc, y>: gy = A gc, g_h[b] =
 *   <(dA/dh) gc, y>_b, and g_r, g_v as mpi_batch_traj_vjp with x = gc.
 * Each equals its building-block sequence (mpi_batch_adjoint or _forward,
 * mpi_batch_forward_dh, mpi_batch_dot, mpi_batch_traj_vjp) bit for bit.  The
 * amplitude gradients then follow from mpi_reduce_lissajous.  Enqueued on
 * `stream`. */
int mpi_vjp_forward(const mpi_plan* plan, const void* c_all, const void* gs_all, void* gc_all, double* g_h,
                    void* g_r_all, void* g_v_all, void* work, size_t work_bytes, hipStream_t stream);
int mpi_vjp_adjoint(const mpi_plan* plan, const void* y_all, const void* gc_all, void* gy_all, double* g_h,
                    void* g_r_all, void* g_v_all, void* work, size_t work_bytes, hipStream_t stream);

/* The amplitudes of a trajectory as parameters (the Lissajous figure of eq.
 * lissajous, r = (a_x rho_x, a_y rho_y) over unit-amplitude shapes rho, and
 * v = (a_x nu_x, a_y nu_y)).
 *
 * mpi_scale_trajectory: r_k = (ax rho_k,x, ay rho_k,y), v_k = (ax nu_k,x,
 *   ay nu_k,y) for k < n_samples, each product in float64 rounded once to
 *   `dtype`; device [T][2] arrays, r and v distinct from each other and from
 *   rho and nu.  The result feeds the problem descriptor of a plan build.
 *
 * mpi_reduce_lissajous: the chain rule from per-sample gradients to the
 *   amplitudes' for every problem b of the plan:
 *     g_ax[b] = sum_k g_r,k,x rho_k,x + g_v,k,x nu_k,x,
 *     g_ay[b] = sum_k g_r,k,y rho_k,y + g_v,k,y nu_k,y,
 *   with g_r = dL/dr_k and g_v = dL/dv_k (as mpi_batch_traj_vjp or
 *   mpi_batch_unrolled_vjp give them) and the unit shapes rho, nu, all
 *   signal-shaped over the batch (time order).  One pass in float64 with a
 *   fixed order (fixed slices, then fixed trees): bitwise repeatable.  g_ax,
 *   g_ay: device arrays of count doubles.  Uses the plan's work memory. */
int mpi_scale_trajectory(const void* rho, const void* nu, int64_t n_samples, double ax, double ay,
                         int32_t dtype, void* r, void* v, hipStream_t stream);
int mpi_reduce_lissajous(const mpi_plan* plan, const void* g_r_all, const void* g_v_all, const void* rho_all,
                         const void* nu_all, double* g_ax, double* g_ay, void* work, size_t work_bytes,
                         hipStream_t stream);

/* Reverse sweep (vector-Jacobian product) of K = n_iter steps of the
 * denoised Landweber iteration of the deconvolution stage,
 *   r_k = A c_k - s,  c_{k+1} = D(c_k - tau_b A^T r_k),
 * with tau_b fixed and D the Gaussian of mpi_batch_denoise (identity when
 * denoise_sigma_px <= 0).  The loss gradient gbar = dL/dc_K comes in and
 * dL/dc_0 goes out in the same buffer; also, per problem,
 *   g_h[b] = dL/dh (device, count doubles), and per sample, in time order,
 *   g_r = dL/dr_k, g_v = dL/dv_k (signal-shaped, base cells held fixed).
 * The reverse recursion is, from k = K-1 down to 0:
 *   g_u = D gbar,  gbar <- g_u - tau A^T A g_u,
 *   dL/dtheta += -tau [<(dA/dtheta) g_u, r_k> + <A g_u, (dA/dtheta) c_k>].
 * checkpoints: ceil(K / every) concentration vectors of the batch, back to
 * back, c_0, c_every, c_2every, ... (as the forward iteration passed them);
 * each segment is recomputed from its checkpoint.  The plan must be built with
 * MPI_BUILD_DERIV.  vjp_work: caller-owned device memory of at least
 * mpi_batch_unrolled_vjp_bytes(plan, every) bytes, 256-byte aligned; its size
 * grows with `every` (per step of a segment: two concentration vectors, a
 * residual and nine planes of the sampled field).  Deterministic: every sum
 * has a fixed order.  Enqueued on `stream`; nothing is synchronised. */
int mpi_batch_unrolled_vjp_bytes(const mpi_plan* plan, int32_t every, size_t* vjp_bytes);
int mpi_batch_unrolled_vjp(const mpi_plan* plan, const void* s_all, const void* checkpoints, int32_t n_iter,
                           int32_t every, double denoise_sigma_px, int32_t denoise_radius, const double* taus,
                           void* gbar_all, double* g_h, void* g_r_all, void* g_v_all, void* work,
                           size_t work_bytes, void* vjp_work, size_t vjp_bytes, hipStream_t stream);

/* ------------------------------------------------------ deconvolution --
 * The Deconvolution Stage (Section "Deconvolution Stage", Algorithm
 * "ZeroShot-PnP", Section "Denoiser Artifact Reduction") on the grids of a
 * built plan; the plan's samples are not used.  Buffers are concentration-
 * shaped and concatenated like c_all; dwork is caller-owned device memory of
 * at least mpi_batch_deconv_bytes(plan) bytes, 256-byte aligned, shared by
 * the calls below (none of them keeps anything in it between calls).
 *
 * mpi_batch_trace_conv: y_b = C_b x_b, the convolution with delta^2 kappa_h,
 *   kappa_h = tr K_h the trace kernel (eq. kernel:trace), on the problem's
 *   window and path: the trace of the operator's field (eq.
 *   convolution:trace); for MPI_CH_X problems delta^2 K_xx instead (the
 *   trace is not measured; Section "Experiment 2").  Both include the
 *   problem's gradient G.  C_b is symmetric.  x != y.  Enqueued on `stream`.
 *
 * mpi_batch_cg: for every problem, conjugate gradients on
 *   (C_b^T C_b + nus[b] I) x_b = rhs_b started from x_b = 0 (the normal
 *   equations of the Tikhonov sub-step, eq. dec:sub:tik); a problem stops
 *   once its recursively updated residual meets |r| <= tol |rhs_b| (tested
 *   before every step) or after max_iter steps.  nus: host array of count
 *   values >= 0; iters: host array of count entries for the steps taken (may
 *   be NULL).  rhs != x.  Synchronises `stream`: the host polls the stop flags
 *   between batches of steps.
 *
 * mpi_batch_trim_sigma: for every problem, when pct >= 0 the values of x_b
 *   below their pct-th percentile (linear interpolation between the two
 *   neighbouring order statistics) are raised to it (in place; q[b] receives
 *   the percentile when q is not NULL), then sigma[b] = sqrt of the
 *   population variance of x_b over its pixels (the noise estimate).  q and
 *   sigma are host arrays of count doubles (either may be NULL).  pct > 100
 *   is an error.  Synchronises `stream`.
 *
 * mpi_batch_pnp: the ZeroShot-PnP deconvolution of the trace images u_b into
 *   rho_b: passes k = 0 .. n_it of
 *     rho_1 = the CG of mpi_batch_cg on (C^T C + nu_k I) rho_1 = C u + nu_k rho_2,
 *     trimming of rho_1 below its clip_percentile-th percentile,
 *     sigma_{k+1} = sqrt(Var rho_1), lambda = nu0 sigma_1^2 (first pass),
 *     rho_2 = D(rho_1), nu_{k+1} = lambda / sigma_{k+1}^2 (kept if sigma = 0),
 *   from rho_2 = 0 and nu_0 = nu0; rho receives the last rho_2.  D is the
 *   Gaussian of mpi_batch_denoise standing in for the learned denoiser
 *   (identity when denoise_sigma_px <= 0).  cg_iters, sigmas and nus are host
 *   arrays of (n_it + 1) * count entries, pass-major, for the steps, noise
 *   estimates and Tikhonov weights of every pass (each may be NULL).  u != rho.
 *   Synchronises `stream`. */
typedef struct {
    int32_t n_it;              /* passes k = 0 .. n_it, n_it >= 0                  */
    int32_t cg_max_iter;       /* CG steps per pass at most, >= 0                  */
    double nu0;                /* starting Tikhonov weight, > 0                     */
    double cg_tol;             /* relative residual of the CG stop rule, >= 0       */
    double clip_percentile;    /* trimming percentile in [0, 100]; < 0: no trimming */
    double denoise_sigma_px;   /* Gaussian stand-in, pixels; <= 0: identity         */
    int32_t denoise_radius;    /* 0 .. 8 when the Gaussian is on                    */
    int32_t reserved;
} mpi_pnp_params;

int mpi_batch_deconv_bytes(const mpi_plan* plan, size_t* bytes);
int mpi_batch_trace_conv(const mpi_plan* plan, const void* x_all, void* y_all, void* work, size_t work_bytes,
                         hipStream_t stream);
int mpi_batch_cg(const mpi_plan* plan, const void* rhs_all, void* x_all, const double* nus, double tol,
                 int32_t max_iter, int32_t* iters, void* work, size_t work_bytes, void* dwork, size_t dbytes,
                 hipStream_t stream);
int mpi_batch_trim_sigma(const mpi_plan* plan, void* x_all, double pct, double* q, double* sigma, void* work,
                         size_t work_bytes, void* dwork, size_t dbytes, hipStream_t stream);
int mpi_batch_pnp(const mpi_plan* plan, const void* u_all, void* rho_all, const mpi_pnp_params* params,
                  int32_t* cg_iters, double* sigmas, double* nus, void* work, size_t work_bytes, void* dwork,
                  size_t dbytes, hipStream_t stream);

/* ---------------------------------------------------------- core stage --
 * The Core Stage (Section "MPI Core Stage", eq. first:step): for every
 * problem, the symmetric core-operator field a = [A_xx, A_xy, A_yy] on the
 * N x N grid that minimises
 *   (1/L) sum_k |s_k - M(a(r_k)) v_k|^2 + gamma * delta^2 * sum |Delta a|_F^2,
 * with the plan's samples, velocities and interpolation weights (the paper
 * uses MPI_INTERP_COSINE), L = T, delta = 2/N, Delta the 5-point graph
 * Laplacian over in-grid neighbours (over delta^2) and the Frobenius norm of
 * the symmetric 2x2 field (the off-diagonal channel counted twice).  Solved
 * by conjugate gradients on the Euler-Lagrange equations
 *   (1/L) I^T I a + gamma delta^2 W Delta Delta a = (1/L) I^T s,  W = diag(1, 2, 1),
 * from a = 0, stopping per problem once the recursively updated residual
 * meets |r| <= tol |rhs| or after max_iter steps (the paper: tol 1e-3,
 * 10,000 steps).  s_all: signals in time order as for mpi_batch_forward;
 * field_all: 3 * c_elems values, problem b's [3][N][N] field (channels xx,
 * xy, yy) at element offset 3 * c_offsets[b].  Precision: the sampling
 * (I and I^T) runs in the plan's dtype on the search direction rounded to
 * it; the regulariser, the CG vectors and the dot products are float64, and
 * the solution is rounded to the dtype once at the end.  iters: host array of
 * count step counts (may be NULL).  cwork: caller-owned device memory of at least
 * mpi_batch_core_bytes(plan) bytes, 256-byte aligned.  MPI_ERR_UNSUPPORTED
 * when the row-wise sampling of the largest grid does not fit in LDS.
 * Synchronises `stream` (the stop flags are polled between blocks of steps).
 *
 * mpi_batch_field_trace: u_b = A_xx + A_yy of every problem's field (the
 * trace image that the Deconvolution Stage inverts, eq. convolution:trace);
 * u_all concentration-shaped.  For MPI_CH_X problems the Core Stage leaves
 * A_yy = 0 (no data reaches it), so u_b = A_xx, the image the Deconvolution
 * Stage then inverts with K_xx.  Enqueued on `stream`. */
int mpi_batch_core_bytes(const mpi_plan* plan, size_t* bytes);
int mpi_batch_core_stage(const mpi_plan* plan, const void* s_all, void* field_all, double gamma, double tol,
                         int32_t max_iter, int32_t* iters, void* work, size_t work_bytes, void* cwork, size_t cbytes,
                         hipStream_t stream);
int mpi_batch_field_trace(const mpi_plan* plan, const void* field_all, void* u_all, hipStream_t stream);

/* Velocities by forward differences of sampled positions (Section
 * "Experiment 2"): v_k = (r_{k+1} - r_k) / dt for k < T-1, and v_{T-1} =
 * v_{T-2}; evaluated in float64 and rounded to the dtype.  r, v: device
 * [T][2] arrays of `dtype`, r != v, T >= 2, dt > 0.  For a gradient G the
 * operator's velocity is -G times this (the caller's scaling).  Enqueued on
 * `stream`. */
int mpi_velocity_forward_difference(const void* r, void* v, int64_t n_samples, double dt, int32_t dtype,
                                    hipStream_t stream);

/* Diagnostics for timing one kernel at a time.  The forward operator and its
 * transpose each run as a short sequence of kernels (stages); stages
 * 0 .. count/2-1 are those of mpi_forward, the rest those of mpi_adjoint;
 * stages of the path a plan does not use launch nothing.
 * mpi_stage_launch enqueues `reps` launches of one stage exactly as the full
 * call would launch it (same grid, same buffers: c is read by the forward
 * stages and written by the last transpose stage, s the other way round,
 * intermediates live in `work`).  A stage reads what the previous stage of its
 * sequence left in `work`, so run the full call once first for meaningful
 * data.  Names are static strings. */
int mpi_stage_count(const mpi_plan* plan);
const char* mpi_stage_name(const mpi_plan* plan, int stage);
int mpi_stage_launch(const mpi_plan* plan, int stage, int reps, void* c, void* s,
                     void* work, size_t work_bytes, hipStream_t stream);

/* The order in which a plan holds problem `index`'s samples: order[i] is the
 * time index of the i-th sample and cell[i] its base cell (i0 | j0 << 16),
 * sorted by base cell (j0 major) and by time inside a cell.  Both are device
 * arrays of T_index int32 entries owned by the caller; enqueued on `stream`. */
int mpi_batch_sample_order(const mpi_plan* plan, int index, int32_t* order, int32_t* cell, hipStream_t stream);

/* ---------------------------------------------------------- diagnostics --
 * Not part of the operator: debugging and test hooks.
 *
 * mpi_checks_enabled: 1 if this library is the bounds-checked debug build
 * (compiled with -DMPIK_CHECK, libmpik_check.so), else 0.  In that build the
 * kernels check every index they read from the plan's sample tables (a
 * sample's base cell and time index, the sample range of a base-cell row)
 * before it addresses memory; a failed check skips the access it guards and
 * sets a bit in the problem's check word (1: base cell, 2: time index,
 * 4: sample range), and every kernel runs to its normal end.  The release
 * build compiles the checks away and its words stay 0.
 *
 * mpi_plan_check: OR of the check words of every problem of the plan into
 * *word (0: no check failed since the build).  Synchronises `stream` after
 * enqueueing the copies.
 *
 * mpi_debug_fail_alloc: arms a process-wide test hook: the k-th resource
 * acquisition made by the library after this call fails once -- a host
 * allocation of the plan sizing, build or graph caches (the call returns
 * MPI_ERR_ALLOC), or a side stream, event or captured graph (MPI_ERR_HIP) --
 * so that tests can drive every error path; k = 0 disarms it, k < 0 is
 * MPI_ERR_ARG.  A failed call leaves no plan, stream or graph behind and
 * later calls behave normally. */
int mpi_checks_enabled(void);
int mpi_plan_check(const mpi_plan* plan, int32_t* word, hipStream_t stream);
int mpi_debug_fail_alloc(int32_t k);

int mpi_plan_destroy(mpi_plan* plan);
const char* mpi_status_str(int status);
int mpi_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MPIK_H */
