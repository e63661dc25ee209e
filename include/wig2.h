/*
 * wig2.h -- C ABI of the MI355X (gfx950) two-body Wigner step library.
 *
 * The library advances the two-particle Wigner function f(x1, x2, p1, p2) of
 * Liang & Xiong, arXiv:2511.11354 (the two-body truncated Wigner equation of
 * Sec. 2.4, eq. two_body_truncated_Wigner) on a 4-D grid:
 *
 *   df/dt + (p1/m) df/dx1 + (p2/m) df/dx2
 *        = Theta_{V_eff[n1]} f + Theta_{V_eff[n2]} f + Theta_{V12} f,
 *
 * V_eff = V_ext + lambda * V_H[n] + V_xc[n] - V_xc[n0] (Sec. 2.2-2.3).  The
 * step splits the characteristic advection (cubic B-spline interpolation,
 * Sec. 4.1) from the pseudo-differential operator Theta (Sec. 3):
 *   - torus [x_min, x_max): pseudo-difference operators (Sec. 3.1,
 *     eqs. Hartree_FSM and two_body_FSM), dp = hbar*pi/L;
 *   - box [x_min, x_max] (non-periodic): natural-boundary spline and the
 *     Chebyshev spectral-element single-body operator (Sec. 3.2.1,
 *     eq. Chebyshev_PDO).
 *
 * Conventions for every entry point:
 *   - Return 0 on success, a negative WIG2_E* code otherwise.  No C++
 *     exception crosses the ABI.  wig2_last_error() holds a message for the
 *     last failing call on a context until the next call on it.
 *   - State layout: f[((i1*nx + i2)*nk + n1)*nk + n2] (n2 fastest), i.e. each
 *     x-pair owns one contiguous nk x nk momentum plane.
 *   - Host arrays are read or written only during the call.  Device pointers
 *     ("_dev") are caller-owned hipMalloc (or torch) memory of the state's
 *     element type and size; the library only reads/writes them on the
 *     context's stream during the call.
 *   - Calls on one context are ordered on its stream.  Use one context per
 *     host thread.  wig2_get_state, wig2_observables and the *_host variants
 *     synchronise the stream; the others are asynchronous.
 */
#ifndef WIG2_H
#define WIG2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WIG2_OK 0
#define WIG2_EINVAL (-1)   /* invalid argument or grid/parameter combination   */
#define WIG2_ENOMEM (-2)   /* device or host allocation failed                 */
#define WIG2_EDEVICE (-3)  /* HIP runtime error (message has the HIP string)   */
#define WIG2_ESTATE (-4)   /* call out of order (step before state/potentials)  */
#define WIG2_ENOTSUP (-5)  /* combination not supported by this library        */
#define WIG2_ENUMERIC (-6) /* NaN or Inf met in the observables                */

enum { WIG2_STRANG = 0, WIG2_LAWSON_PC = 1 };
enum { WIG2_FP64 = 0, WIG2_FP32 = 1, WIG2_BF16X2 = 2 };

typedef struct wig2_ctx wig2_ctx;

/* Host callback: potential value at x (V_ext) or at separation r (V12).
 * Called synchronously inside wig2_set_potentials only, never retained. */
typedef double (*wig2_fn1)(double x, void* user);

/* Grid (Sec. 3.1 torus / Sec. 3.2 box).
 *  nx        points per x-dimension.  Torus: distinct points, dx = L/nx.
 *            Box: nodes including both ends, dx = L/(nx-1).  nx >= 4.
 *  nk        points per p-dimension.  Supported: 16, 32, 48, 64, 96, 128;
 *            on a box also 256 (dense SEM operator on LDS-staged panels).
 *            Other sizes: WIG2_ENOTSUP.
 *  periodic  1: torus, p_n = (n - nk/2) hbar pi / L.
 *            0: box; nk = sem_cells * N Chebyshev-Gauss nodes on
 *               [-hbar k_max, hbar k_max].
 *  sem_cells spectral-element cells per p-dimension (box only; nk % sem_cells == 0).
 *  x_min, x_max  spatial extent, x_max > x_min.
 *  k_max     box only: half-width of the p-box in wave-number units. */
typedef struct {
    int32_t nx, nk, periodic, sem_cells;
    double x_min, x_max, k_max;
} wig2_grid;

/* Physical and numerical parameters.
 *  hbar, mass, dt   > 0.
 *  scheme           WIG2_STRANG: A(dt/2), Heun on Theta (potential frozen at
 *                   the sub-step start), A(dt/2).
 *                   WIG2_LAWSON_PC: the Lawson predictor-corrector of Sec. 4.1.
 *  precision        WIG2_FP64; WIG2_FP32 (state, advection and Theta in FP32);
 *                   WIG2_BF16X2 (FP32 state and advection, Theta on bf16
 *                   matrix cores with hi+lo split operands, FP32 accumulate).
 *                   Symbol tables and all reductions stay FP64.
 *  meanfield_lambda weight of the Hartree term lambda * (V12 * n_j) on
 *                   particle j (the (N-k)/(N-1) prefactor of Sec. 2.1; 0 for N=2).
 *  xc               1: add the Hedin-Lundqvist potential (Sec. 2.2) in atomic
 *                   units, evaluated at n_scale * n_j(x), minus its value at xc_n0.
 *  Mean field (lambda != 0 or xc): on the torus V_eff,j enters particle j's
 *  symbol; on a box (Sec. 3.2.1) particle j's SEM matrices become those of
 *  V_ext + V_eff,j, rebuilt on the device before every Theta evaluation
 *  (the Hartree term is the direct convolution dx sum_l V12(x_i - x_l) n_l,
 *  equal to the zero-padded transform on 3 nx points, no wrap-around). */
typedef struct {
    double hbar, mass, dt;
    int32_t scheme, precision;
    double meanfield_lambda;
    int32_t xc;
    double xc_n0, n_scale;
} wig2_params;

/* Scalar observables (Sec. 2.2, Appendix B).
 *  mass = int f, energy = int f (p1^2/2m + p2^2/2m + V_ext(x1) + V_ext(x2)
 *  + V12(x1-x2)), l2 = int f^2, entropy_vn = -sum lam ln lam of the trace-one
 *  1-RDM occupations.  fallbacks counts surrogate blocks redone exactly. */
typedef struct {
    int64_t step;
    double t, mass, energy, l2, entropy_vn;
    int32_t fallbacks;
} wig2_obs;

/* Create a context on the current HIP device.  hip_stream: a hipStream_t to
 * run on, or NULL for a stream owned by the context.  Allocates the state and
 * work buffers (3 state-sized arrays) on the device.  *out owns them. */
int wig2_create(const wig2_grid* grid, const wig2_params* params, void* hip_stream,
                wig2_ctx** out);

/* Sample the potentials and build the symbol tables (FP64, host) then upload.
 * Torus: V_ext at y_j = x_min + j L/(2nk) for its symbol (Sec. 3.1.1),
 * V12 at r_j = -L/2 + j L/(2nk) for its Fourier modes (Sec. 3.1.2, even V12
 * assumed), both at the grid nodes / minimum-image separations for the
 * energy and the Hartree term.  Box: V_ext at the nodes for the SEM operator
 * (Sec. 3.2.1); V12 at l dx + d dy (|l| < nx, |d| < nk, dy = pi / (2 k_max))
 * for the two-body SEM operator (Sec. 3.2.2: y-lattice of nk midpoints,
 * D_V, the two-body tensor), which then joins every Theta application
 * (24 nk flops per point on the matrix cores; tables of 12 nk^2 values and
 * workspaces of two chunks of at most 512 MiB plus one state-sized array,
 * allocated here on the first call with a pair potential).  A box with a
 * pair potential needs nk a multiple of 32, at most 256 (WIG2_ENOTSUP
 * otherwise).  v_ext or v12 NULL means zero. */
int wig2_set_potentials(wig2_ctx* ctx, wig2_fn1 v_ext, wig2_fn1 v12, void* user);

/* Upload / download the state as FP64 host arrays of nx*nx*nk*nk values
 * (converted to the state's element type). */
int wig2_set_state(wig2_ctx* ctx, const double* f_host);
int wig2_get_state(wig2_ctx* ctx, double* f_host);

/* Device-side state access for zero-copy interop: *f_dev receives the
 * context-owned state buffer, *elem_bytes its element size (8 = FP64,
 * 4 = FP32).  Valid until wig2_destroy. */
int wig2_state_buffer(wig2_ctx* ctx, void** f_dev, int32_t* elem_bytes);
/* Mark the state buffer as initialised after the caller wrote it. */
int wig2_state_written(wig2_ctx* ctx);

/* Bind a caller-owned device buffer as the state (the problem of Sec. 2.4 is
 * posed on the caller's f(x1, x2, p1, p2)): from then on wig2_step,
 * wig2_observables, wig2_get_state / wig2_set_state and the surrogate read
 * and write f_dev in place, in the layout above; the context's own state
 * buffer is left unused.  f_dev: nx*nx*nk*nk elements on the context's
 * device, 16-byte aligned, holding the initial state (the step count and
 * time restart at 0).  dtype: WIG2_FP64 for an FP64 context, WIG2_FP32 for
 * FP32 and BF16X2 contexts (else WIG2_EINVAL, as for host or other-device
 * memory).  The buffer stays caller-owned: it must outlive its binding and
 * must not be written by others while a call on the context may use it
 * (calls are ordered on the context stream).  f_dev == NULL unbinds: the
 * context returns to its own buffer, which then needs wig2_set_state.
 * Synchronises the context stream first. */
int wig2_bind_state(wig2_ctx* ctx, void* f_dev, int32_t dtype);

/* Advance nsteps steps of the configured scheme (asynchronous).
 * Strang (Sec. 4.1 splitting of the advection from the Theta term): each
 * step is A(dt/2), Heun on Theta with V_eff frozen, A(dt/2), where the
 * entering A sweeps x1 then x2 and the leaving A sweeps x2 then x1 (the
 * sweeps act on different axes and commute).  Within one call the x1
 * half-sweep that ends a step and the one that begins the next run as one
 * launch, bitwise equal to nsteps calls of one step each.  Lawson
 * predictor-corrector (Sec. 4.1): a = A_dt f, b = A_dt Theta[f],
 * f+ = a + (dt/2) Theta[a + dt b] + (dt/2) b. */
int wig2_step(wig2_ctx* ctx, int64_t nsteps);

/* Hartree term of the mean field (meanfield_lambda != 0): V_eff gains
 * lambda V_H[n_j] with
 *   WIG2_HARTREE_PAIR     V_H(x_i) = dx sum_j V12(x_i - x_j) n_j(x_j), the
 *                         pair potential of wig2_set_potentials (Sec. 2.3;
 *                         the default);
 *   WIG2_HARTREE_POISSON  the neutralised 1-D Coulomb potential of a uniform
 *                         background (Sec. 3.1.1 example, the Wigner-Poisson
 *                         system): -V_H'' = n_j - mean(n_j) on the torus,
 *                         V_H = sum_{0<|m|<nx/2} (L/(2 pi m))^2 a_m e_m(x)
 *                         from the density's Fourier modes a_m.
 * Torus only for POISSON (WIG2_ENOTSUP on a box); WIG2_EINVAL for another
 * form.  May be called before or after wig2_set_potentials; synchronises. */
enum { WIG2_HARTREE_PAIR = 0, WIG2_HARTREE_POISSON = 1 };
int wig2_set_hartree(wig2_ctx* ctx, int32_t form);

/* Strang only: enable (default) or disable the joint launch of consecutive
 * x1 half-sweeps within a wig2_step call (results are bitwise the same; for
 * verification and timing).  0 on success. */
int wig2_set_sweep_fusion(wig2_ctx* ctx, int32_t enable);

/* Observables of the current state (synchronises).  n1[nx], n12[nx*nx] (x1
 * major), f1[nx*nk] (reduced Wigner function W_red(x1,p1)) may be NULL.
 * Entropy from the 1-RDM of f1 on the even sub-lattice (Appendix B). */
int wig2_observables(wig2_ctx* ctx, wig2_obs* obs, double* n1, double* n12, double* f1);

/* Operator-level entry points (for verification and composition).
 *  wig2_theta: out = Theta[in] with the current potentials (mean field, if
 *    on, from the density of `in`).  in == out is allowed except on a box
 *    with nk = 256 in FP64 or BF16X2 (several workgroups share a plane
 *    there): WIG2_EINVAL.
 *  wig2_advect: one spline sweep along x_dim (dim 1 or 2) by time s:
 *    out(x, p) = in(x_dim - s p_dim / m, p).  in != out.
 * Both run asynchronously on the context's stream (the one passed to
 * wig2_create, else the context's own): work that other streams do on
 * in_dev or out_dev must be complete (or ordered before the call by the
 * caller) when the call is made. */
int wig2_theta(wig2_ctx* ctx, const void* in_dev, void* out_dev);
int wig2_advect(wig2_ctx* ctx, int32_t dim, double s, const void* in_dev, void* out_dev);

/* Allocation-free variant of wig2_advect, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments, result and stream as wig2_advect.
 * Where wig2_advect lazily allocates a state-sized coefficient buffer (the
 * general sweep: displacements of more than one cell, or an nx without a
 * register-resident sweep), this call uses a static device array of 64 MiB
 * instead, one per device, held until the process ends; it calls no
 * hipMalloc / hipFree.  Sweeps that need the buffer are rejected with
 * WIG2_EINVAL when nx*nx*nk*nk*elem_bytes exceeds 64 MiB; register-resident
 * sweeps need no buffer and have no size limit.  All calls on one device
 * share that array: calls that overlap in time on one device (other streams,
 * other contexts, other host threads) race and must be serialised by the
 * caller.  The array's contents are not meaningful between calls. */
int wig2_advect_noalloc(wig2_ctx* ctx, int32_t dim, double s, const void* in_dev, void* out_dev);

/* Per-kernel-class timing of wig2_step with HIP events on the context stream
 * (a tracing aid; adds two event records per launch while enabled).
 * wig2_profile_read synchronises, then fills ms[WIG2_PROF_N] (total
 * milliseconds) and counts[WIG2_PROF_N] (launches) accumulated since the
 * last reset; reset != 0 clears them.  Either array may be NULL. */
enum {
    WIG2_PROF_ADVECT_X1 = 0,
    WIG2_PROF_ADVECT_X2 = 1,
    WIG2_PROF_THETA_STAGE1 = 2, /* general: Theta[f];  stream: f + tau Theta[f]   */
    WIG2_PROF_THETA_STAGE2 = 3, /* second Heun stage (both kernels)               */
    WIG2_PROF_MEANFIELD = 4,    /* density moments + mean-field symbols     */
    WIG2_PROF_THETA_HEUN = 5,   /* stream, Strang: both Heun stages in one pass */
    WIG2_PROF_ADVECT_X1X1 = 6,  /* Strang: two x1 half-sweeps in one launch     */
    WIG2_PROF_PAIR_SEM = 7,     /* box two-body SEM operator (inside the Theta
                                   stages, which include its time as well)       */
    WIG2_PROF_N = 8
};
int wig2_profile(wig2_ctx* ctx, int32_t enable);
int wig2_profile_read(wig2_ctx* ctx, double* ms, int64_t* counts, int32_t reset);

/* Largest single-body mode the Theta kernels visit: the symbol's support
 * (modes below 1e-13 of the largest are dropped), nk-1 when dense or when the
 * mean field is on.  >= 0 on success. */
int wig2_band(const wig2_ctx* ctx);

/* Theta kernel selection.  WIG2_THETA_GENERAL: one plane per workgroup,
 * single-body products on the matrix cores over the symbol's band (any band,
 * box SEM matrices, bf16x2); on the torus at nk = 32 .. 128 its Strang Heun
 * step runs in one pass per plane as well (FP64 / FP32; the potentials
 * frozen over the step).  WIG2_THETA_STREAM: persistent workgroups that
 * prefetch the next plane while the matrix cores contract the pair term of
 * the current one; single-body differences on the vector ALUs; needs a
 * torus, FP64 or FP32, nk in {32, 48, 64, 96, 128} and a single-body band of
 * at most 4 modes (e.g. V_ext = V0 cos(2 pi x / L)).  Its Heun step is
 * g = f + dt Theta f, f' = (f + g)/2 + (dt/2) Theta g, equal to the general
 * kernels' f + (dt/2)(Theta f + Theta g) up to rounding; with the Strang
 * scheme both Heun stages run in one pass per plane (f read and f' written
 * once; the plane stays in LDS between the two applications of Theta).
 * WIG2_THETA_AUTO (default): the streaming kernel wherever it applies (it
 * is the faster one on MI355X at every plane size it supports).
 * wig2_set_theta_path returns WIG2_ENOTSUP for STREAM when the current
 * potentials rule it out (the choice then stays unchanged); with AUTO or
 * STREAM, potentials set later that rule it out select GENERAL.
 * wig2_theta_path returns the kernel the next step uses (>= 0), or
 * WIG2_ESTATE before wig2_set_potentials.  WIG2_THETA_PANEL (reported only):
 * box contexts with nk = 256 always use the panel kernel, which stages the
 * dense SEM products through LDS in k panels.  WIG2_THETA_FFT (chosen only
 * when asked for): the FFT-accelerated route of the two-body cost statement
 * (Sec. 3.1.2).  On each momentum plane the row, column and anti-diagonal
 * pseudo-differences form one 2-D linear convolution with an odd kernel.  It
 * is evaluated as IFFT2(W . FFT2(f)) on the plane zero-padded to
 * N >= 2 nk points per direction (2 nk rounded up to a multiple of 64),
 * W(k1, k2) = -2i [S1(k1) + S2(k2) +
 * K(k1 - k2)], S(k) = sum_m s_m sin(2 pi k m / N).  The result equals the
 * direct sums up to rounding, for any single-body band (mean field
 * included).  Needs a torus, nk in {16, 32, 48, 64, 96, 128} and FP64 or FP32 (else
 * WIG2_ENOTSUP).  Heun runs as its two stages.  On MI355X it is slower than
 * the direct products at every one of these sizes. */
enum { WIG2_THETA_AUTO = 0, WIG2_THETA_GENERAL = 1, WIG2_THETA_STREAM = 2, WIG2_THETA_PANEL = 3, WIG2_THETA_FFT = 4 };
int wig2_set_theta_path(wig2_ctx* ctx, int32_t path);
int wig2_theta_path(const wig2_ctx* ctx);

/* Grid nodes: x[nx], p[nk] and p-quadrature weights w[nk] (any may be NULL). */
int wig2_nodes(const wig2_ctx* ctx, double* x, double* p, double* w);

/* ------------------------------------------------------------------------
 * Batched ensembles of uneven periodic instances.
 * Every instance has its own grid, parameters, potentials and state; one
 * Strang step of the whole ensemble is six launches (two half-step sweeps,
 * the two Theta stages, two half-step sweeps); in each phase every size
 * class (nx for sweeps, nk for Theta) is one persistent launch over a work
 * list spanning its instances, the class launches run as parallel branches
 * of a HIP graph captured once and replayed per step.  Restrictions (WIG2_ENOTSUP otherwise):
 * torus, Strang, no mean field, one precision (FP64 or FP32) for all
 * instances, nx in {16,32,48,64,96,128}, nk in {16,32,48,64,96,128},
 * half-step displacement at most one cell.
 * ------------------------------------------------------------------------ */
typedef struct wig2_batch wig2_batch;

/* grids[n], params[n]: per-instance grid and parameters.  hip_stream as in
 * wig2_create.  Allocates 3 pooled state arrays (sum of instance sizes). */
int wig2_batch_create(int32_t n, const wig2_grid* grids, const wig2_params* params,
                      void* hip_stream, wig2_batch** out);
/* Per instance i in [0, n): potentials (as wig2_set_potentials), FP64 host
 * state upload / download (as wig2_set_state / wig2_get_state). */
int wig2_batch_set_potentials(wig2_batch* b, int32_t i, wig2_fn1 v_ext, wig2_fn1 v12, void* user);
int wig2_batch_set_state(wig2_batch* b, int32_t i, const double* f_host);
int wig2_batch_get_state(wig2_batch* b, int32_t i, double* f_host);
/* Advance every instance by nsteps steps.  The first call after a change of
 * potentials or tiling runs one step directly and captures the graph. */
int wig2_batch_step(wig2_batch* b, int64_t nsteps);
int wig2_batch_observables(wig2_batch* b, int32_t i, wig2_obs* obs, double* n1, double* n12,
                           double* f1);
/* Autotuner: times the candidate tilings (sweep grid, planes per Theta
 * workgroup for each plane size, Theta grid) on this ensemble's data and
 * keeps the fastest.  cache_path (may be NULL): JSON file of earlier results
 * keyed by architecture, precision and plane size; read unless force != 0,
 * rewritten after tuning.  The state is left unchanged. */
int wig2_batch_tune(wig2_batch* b, const char* cache_path, int32_t force);
/* Total points and the current tiling per size class 16, 32, 48, 64, 96, 128:
 * theta_grid[6] (by nk), advect_grid[6] (by nx), planes_per_group[6] (by nk).
 * Any array may be NULL. */
int wig2_batch_info(const wig2_batch* b, int64_t* total_points, int32_t* theta_grid,
                    int32_t* advect_grid, int32_t* planes_per_group);
void wig2_batch_destroy(wig2_batch* b);
const char* wig2_batch_last_error(const wig2_batch* b);

/* ------------------------------------------------------------------------
 * Learned surrogate for the pair increment over blocks of fine steps.
 * Not part of the paper's method: an accelerator with an exact fallback.
 * For a block of B fine steps from f_t, the exact block gives f_full and the
 * same B steps without Theta[V12] (Sec. 3.1.2) give f_nov; the model learns
 * Delta = f_full - f_nov as a function of f_t.
 * Model: a 4-D separable convolutional network with 16 channels.  Input
 * features per grid point, in the form of the pair term (kernel
 * V12_m sin(m a), a = 2 pi (i1 - i2)/nx, on antisymmetric differences along
 * the anti-diagonal through the point): c_0 = s_in f_t(n1, n2) and
 * c_m = s_in U sin(m a) [f_t(n1 - m, n2 + m) - f_t(n1 + m, n2 - m)],
 * m = 1..15 (U = V12(0)).  Then `blocks` blocks of four layers, one
 * convolution along each axis p1, p2 (k_p taps, zero off the p-box), x1, x2
 * (k_x taps, periodic), 16 -> 16 channels, each h <- h + tanh(b + W * h);
 * output y = b_o + w_o . h + a . c, Delta = s_out y.  Parameters:
 * blocks (2 (256 k_p + 16) + 2 (256 k_x + 16)) + 33; with blocks = 9,
 * k_p = 35, k_x = 7: 194,145.  Weights and activations in BF16 on the bf16
 * matrix cores, FP32 accumulation and FP32 master weights (Adam), forward
 * and backward in the library's own kernels; each training step is a
 * full-grid gradient of the mean squared error.  Torus contexts with a pair
 * potential, FP64 or FP32 state, nk a multiple of 16, no mean field.
 * ------------------------------------------------------------------------ */
typedef struct wig2_surrogate wig2_surrogate;
typedef struct {
    int32_t channels;     /* must be 16                                          */
    int32_t blocks;       /* blocks of four axis convolutions, 1..16             */
    int32_t k_p;          /* taps of the p1 / p2 convolutions, odd, 1..63        */
    int32_t k_x;          /* taps of the x1 / x2 convolutions, odd, 1..15        */
    int32_t block;        /* fine steps per block (B), >= 1                      */
    int32_t epochs;       /* Adam steps per collected block                      */
    double lr;            /* Adam step size                                      */
    uint64_t seed;        /* weight initialisation                               */
    int32_t train_blocks; /* wig2_surrogate_train: blocks collected per instance */
    int32_t max_points;   /* wig2_surrogate_train: larger instances skipped (0: none) */
} wig2_train_cfg;

/* Create an untrained model on the current device (small uniform weights
 * from `seed`, zero biases and linear path).  The input / output scales are
 * fixed by the first collected block (1 / max|f_t| and max|Delta|).
 * WIG2_ENOTSUP for channels != 16, WIG2_EINVAL for other bad fields. */
int wig2_surrogate_create(const wig2_train_cfg* cfg, wig2_surrogate** out);
void wig2_surrogate_destroy(wig2_surrogate* s);
const char* wig2_surrogate_last_error(const wig2_surrogate* s);
/* Parameter count and number of convolution layers. */
int wig2_surrogate_size(const wig2_surrogate* s, int64_t* nparams, int32_t* nlayers);
/* Train a new model on trajectories of a batched ensemble: for every
 * instance with state, potentials and a pair term (and at most max_points
 * points), train_blocks blocks of its exact dynamics from its current state
 * are run in a context of its own on the batch's stream (the batch's states
 * are not changed), and the model takes `epochs` full-grid Adam steps per
 * block.  WIG2_EINVAL if no instance qualifies.  *out owns the model. */
int wig2_surrogate_train(wig2_batch* data_source, const wig2_train_cfg* cfg, wig2_surrogate** out);
/* Run `blocks` blocks of the context's exact dynamics from its current state.
 * For each block the pair (f_t, Delta) is formed on the device; with train
 * != 0 the model takes `epochs` full-grid Adam steps on it, otherwise it is
 * only evaluated.  The context ends on the exact trajectory (its step
 * count advances by blocks x B).  Allocates two state-sized buffers in the
 * context on first use.  The model remembers the context's dt; contexts with
 * another dt are rejected (WIG2_EINVAL). */
int wig2_surrogate_collect(wig2_surrogate* s, wig2_ctx* ctx, int32_t blocks, int32_t train);
/* Mean squared error (in units of the output scale) of the last training
 * epoch and of the last evaluation, Adam steps taken, samples seen. */
int wig2_surrogate_stats(const wig2_surrogate* s, double* train_loss, double* eval_loss,
                         int64_t* updates, int64_t* samples);
/* Parameters (FP32 master copy, nparams values: per layer W[16][K][16]
 * (c_out, tap, c_in) then its bias[16]; then w_o[16], b_o, a[16]) and
 * scales[3] = {in_scale, out_scale, U}.  set resets Adam. */
int wig2_surrogate_get_params(const wig2_surrogate* s, float* params, float* scales);
int wig2_surrogate_set_params(wig2_surrogate* s, const float* params, const float* scales);
/* Gradient of the mean squared error over all points of caller-owned device
 * fields ft and delta (the context's element type and grid) with the
 * current weights; grad[nparams] and the loss are written to host memory. */
int wig2_surrogate_grad(wig2_surrogate* s, wig2_ctx* ctx, const void* ft_dev, const void* delta_dev,
                        float* grad, double* loss);
/* Attach to a context: from then on wig2_step advances whole blocks of B
 * steps as B steps without Theta[V12] plus the model's increment.  After
 * each block the mass and energy are compared with those at the end of the
 * last exactly computed block (at attach: the current state); if either
 * moved by more than drift_tol (relative) the block is redone exactly (a
 * fallback).  Every exact_check_every blocks (0: never) the block is also
 * computed exactly, the surrogate error eps_inf is recorded and the exact
 * result kept.  Steps left over (nsteps mod B) run exactly.  The model must
 * outlive the attachment; detach with wig2_surrogate_detach. */
int wig2_surrogate_attach(wig2_ctx* ctx, const wig2_surrogate* s, double drift_tol,
                          int32_t exact_check_every);
int wig2_surrogate_detach(wig2_ctx* ctx);
/* Blocks advanced with the model, fallbacks, exact checks and the eps_inf
 * of the last check (-1 if none). */
int wig2_surrogate_report(const wig2_ctx* ctx, int64_t* blocks, int64_t* fallbacks, int64_t* checks,
                          double* last_check_eps);

void wig2_destroy(wig2_ctx* ctx);
const char* wig2_strerror(int code);
const char* wig2_last_error(const wig2_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
