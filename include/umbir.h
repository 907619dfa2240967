/*
 * umbir.h -- C ABI of the MI355X (gfx950) library for multi-layer,
 * collimated-beam ultrasound model-based reconstruction (Alanazi,
 * Venkatakrishnan, Santos-Villalobos, Buzzard, Bouman, "Model-Based
 * Reconstruction for Collimated Beam Ultrasound Systems", ICASSP 2022,
 * arXiv:2202.09703).
 *
 * The library applies the system matrix A of the measurement model
 * y = A x + D g + w (Sec. 2, Eq. (1)) without storing it, applies its exact
 * transpose, and runs MAP reconstruction of Eq. (18) with a QGGMRF prior
 * (Eqs. (14)-(17)).
 *
 * Conventions for every entry point:
 *  - Return value: UMBIR_OK (0) or a negative status below.  No C++
 *    exception crosses this boundary.  umbir_last_error() gives detail text
 *    for the calling thread's last failure.
 *  - Device pointers ("_dev") are HIP device memory on the device that was
 *    current when the geometry was built; the caller owns them.  All device
 *    arrays are dense and row-major.  Images and g are float32; trace buffers
 *    (void*) hold the problem's storage type (umbir_acq.storage).
 *  - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *    Every call except umbir_build_geometry is asynchronous in stream order.
 *  - Argument checks (null pointers, sizes, parameter ranges) run before any
 *    HIP call, so they also work on a machine without a GPU.
 *  - Layouts: image x is [nz][nx] (row = depth, column = lateral position,
 *    index v = row * nx + col); traces y, r are [P][K][M] (scan position i,
 *    receiver j, time sample m; sample m is at t = m / fs after firing);
 *    direct-arrival weights g are [P][K].
 *  - Workspace: compute calls take a caller-owned device buffer `work` of at
 *    least umbir_workspace_bytes() bytes.  If `work` is NULL the library
 *    allocates one on `stream` (hipMallocAsync) and releases it in stream
 *    order after the call.  One workspace must not be used by two calls that
 *    may overlap.
 */
#ifndef UMBIR_H
#define UMBIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    UMBIR_OK = 0,
    UMBIR_EINVAL = -1,    /* invalid argument, problem or prior */
    UMBIR_ENOMEM = -2,    /* device allocation failed */
    UMBIR_EDEVICE = -3,   /* HIP runtime or kernel launch error, or no device */
    UMBIR_ENOTSUP = -4,   /* valid input outside what the library implements */
    UMBIR_EDIVERGED = -5  /* the MAP cost became non-finite */
};

#define UMBIR_MAX_LAYERS 8

/* Planar layers below the array face (Sec. 2, "Multi-layered structures",
 * Fig. 1).  Layer 0 starts at z = 0; the last layer is unbounded.
 * speed c_l [m/s] > 0, thickness [m] > 0 of layers 0..n_layers-2,
 * atten alpha_l [s/m] (Eq. (3)) >= 0, density [kg/m^3] > 0.
 * With some alpha_l > 0 the pulse of each (trace, voxel) pair is attenuated
 * by its path (Eqs. (7), (9)): see umbir_acq.n_gamma. */
typedef struct {
    int n_layers;              /* 1..UMBIR_MAX_LAYERS */
    const double* speed;       /* [n_layers] */
    const double* thickness;   /* [n_layers - 1] (may be NULL if n_layers == 1) */
    const double* atten;       /* [n_layers] (may be NULL: all zero) */
    const double* density;     /* [n_layers] */
} umbir_medium;

/* Voxel grid: centre of (row, col) is (x0 + (col + 1/2) dx, z0 + (row + 1/2) dz). */
typedef struct {
    int nx, nz;
    double dx, dz;             /* > 0 [m] */
    double x0, z0;             /* left edge of column 0, top edge of row 0 [m]; z0 >= 0 */
} umbir_grid;

/* Transducers on the face z = 0.  Scan position i fires from tx_x[i];
 * receiver j of that scan sits at tx_x[i] + rx_offset[j].  beta is the
 * integer apodization power of Eq. (12).  Every transducer must lie on the
 * half-voxel lattice of the grid, i.e. 2 (x0 - x) / dx must be an integer
 * (ENOTSUP otherwise): then the lateral distance of any voxel from any
 * transducer is a multiple of dx / 2 and travel-time legs are shared. */
typedef struct {
    int n_scans;               /* P >= 1 */
    const double* tx_x;        /* [P] [m] */
    int n_rx;                  /* K >= 1 */
    const double* rx_offset;   /* [K] [m] */
    int beta;                  /* 0..64 */
} umbir_array;

/* Sampling and pulse.  The transmitted pulse is a Gaussian-windowed sine of
 * centre f_c and width sigma_t centred at t_win / 2; Eq. (10) keeps it on the
 * open window (0, t_win).  L_h = t_win * fs must be an integer >= 2.  The
 * windowed response is tabulated once on a grid `oversample` (Q) times finer
 * than the sampling grid and interpolated linearly between grid points;
 * Q must be a power of two in 1..64.
 * `storage` is the element type of every trace buffer (y, r, residuals), of
 * the tabulated pulse as the sweeps use it and of the fine-grid workspace:
 * UMBIR_STORAGE_F32, _F16 (IEEE half) or _BF16 (bfloat16, passed as 16-bit
 * words).  Images, direct-arrival weights and all accumulation stay FP32 and
 * the leg search FP64 in every mode.  16-bit storage needs Q = 32 or 64. */
enum { UMBIR_STORAGE_F32 = 0, UMBIR_STORAGE_F16 = 1, UMBIR_STORAGE_BF16 = 2 };
typedef struct {
    int n_samples;             /* M >= 1 */
    double fs;                 /* sampling rate [Hz] */
    double f_c;                /* pulse centre frequency [Hz] */
    double sigma_t;            /* Gaussian width [s] */
    double t_win;              /* window t_0 of Eq. (10) [s] */
    int oversample;            /* Q */
    int storage;               /* UMBIR_STORAGE_* */
    /* Attenuation templates (used only when some alpha_l > 0; 0 means 16,
     * else 2..64; needs FP32 storage).  Eq. (9) gives every pair its own
     * h(gamma(v), t); the templates are tabulated once at gamma_g = g dgamma,
     * g = 0 .. n_gamma - 1, dgamma = 2 Gamma_max / (n_gamma - 1), Gamma_max the
     * largest one-way path attenuation sum_l alpha_l eta_l / cos(theta_l) of
     * the problem's legs, and each pair uses the template nearest its gamma,
     * floor((Gamma_tx + Gamma_rx) / dgamma + 1/2) in float64 (at most
     * n_gamma - 1).  The forward runs one
     * splat + convolution per template; the adjoint one correlation per
     * template, each into its own resident fine grid (its workspace grows
     * n_gamma-fold), then one gather over all of them. */
    int n_gamma;
} umbir_acq;

typedef struct {
    umbir_medium medium;
    umbir_grid grid;
    umbir_array array;
    umbir_acq acq;
} umbir_problem;

/* MAP prior and noise (Eqs. (2), (15)-(18)).  sigma: noise standard deviation
 * (> 0); p, q: QGGMRF shapes with 1 < p <= q and q == 2 (Sec. 2 requires
 * 1 < p < q = 2; p == q == 2 is accepted as the quadratic limit); T: threshold
 * (> 0); sigma0 (> 0), m (> 0), a (>= 0): scale and depth modulation of
 * Eqs. (16)-(17).  estimate_direct != 0 also estimates g of Eq. (1). */
typedef struct {
    double sigma, p, q, T, sigma0, m, a;
    int estimate_direct;
} umbir_prior;

typedef struct umbir_geometry umbir_geometry;

/* Builds the geometry of a problem on the current HIP device: for every
 * distinct one-way leg (voxel row, lateral distance on the half-voxel
 * lattice) the Snell ray parameter by an FP64 binary search (Sec. 2,
 * Eqs. (4)-(6) and the binary search that follows them), its travel time as
 * Q32.32 fixed-point samples and cos^beta of its angle sum (Eq. (12)); the
 * per-row transmittance product (Eqs. (3), (7)); the tabulated windowed pulse
 * (Eqs. (9)-(10)); and the direct-arrival columns of D (Eq. (1)).
 * The tables stay resident in device memory owned by *out until
 * umbir_geometry_free.  Blocks until the tables are built.  The handle is
 * immutable afterwards and may be shared by streams and threads.
 * With attenuation it also builds each leg's path attenuation (Eq. (3)) in
 * template units and the n_gamma attenuated templates (Eq. (9), by float64
 * quadrature of the pulse spectrum times e^{-gamma |f|}).
 * Errors: EINVAL (bad problem, n_gamma out of range), ENOTSUP (attenuation
 * with 16-bit storage, off-lattice transducers, unsupported Q, 16-bit
 * storage with Q other than 32 or 64, nx * n_layers > 4096,
 * window * Q > 16384), ENOMEM, EDEVICE. */
int umbir_build_geometry(const umbir_problem* problem, void* stream, umbir_geometry** out);

/* Frees a geometry and its device tables.  NULL is a no-op.  The caller must
 * make sure no queued call still uses it. */
void umbir_geometry_free(umbir_geometry* geom);

/* Device bytes held by a geometry, and an estimate for a problem before it is
 * built (0 if the problem is invalid).  Workspace is not included. */
size_t umbir_geometry_bytes(const umbir_geometry* geom);
size_t umbir_estimate_bytes(const umbir_problem* problem);

/* Workspace bytes needed by a compute call of the given kind. */
enum { UMBIR_WORK_FORWARD = 0, UMBIR_WORK_ADJOINT = 1, UMBIR_WORK_RECONSTRUCT = 2 };
size_t umbir_workspace_bytes(const umbir_geometry* geom, int kind);

/* y = A x (accumulate == 0) or y += A x (accumulate != 0), Eq. (13):
 * y[i][j][m] = sum_v W_ij(v) x(v) h~(m / fs - T_ij(v)) with the tabulated,
 * linearly interpolated h~, W = tau(v) phi^(beta)(v).  Scan positions are
 * separate firings stacked as rows of y.  x_dev: [nz][nx]; y_dev: [P][K][M].
 * Deterministic: the same inputs give bitwise the same output. */
int umbir_forward(const umbir_geometry* geom, const float* x_dev, void* y_dev,
                  int accumulate, void* work, size_t work_bytes, void* stream);

/* x = A^T r, the exact transpose of umbir_forward (same W, delays and
 * interpolation).  r_dev: [P][K][M]; x_dev: [nz][nx].  Deterministic: the
 * same inputs give bitwise the same output. */
int umbir_adjoint(const umbir_geometry* geom, const void* r_dev, float* x_dev,
                  void* work, size_t work_bytes, void* stream);

/* y = D g (accumulate == 0) or y += D g: column (i, j) of D is the tabulated
 * pulse delayed by the direct path |x_rx - x_tx| / c_1 in layer 0 (Eq. (1)).
 * g_dev: [P][K]; y_dev: [P][K][M]. */
int umbir_direct(const umbir_geometry* geom, const float* g_dev, void* y_dev,
                 int accumulate, void* stream);

/* d = |A|^T |A| 1 / sigma^2, the separable-surrogate curvature of the data
 * term of Eq. (18), with |A| built from |W| and the absolute tabulated pulse
 * (an entrywise upper bound of |A|).  d_dev: [nz][nx]. */
int umbir_sqs_denominator(const umbir_geometry* geom, double sigma, float* d_dev,
                          void* work, size_t work_bytes, void* stream);

/* MAP reconstruction of Eq. (18) by n_iter separable-surrogate iterations,
 * each one A x and one A^T e: residual e = y - A x - D g, exact per-trace g
 * update (if estimate_direct), then the simultaneous surrogate step for x
 * with the QGGMRF prior on the 8-neighbourhood.  x_io_dev ([nz][nx]) and
 * g_io_dev ([P][K]) hold the warm start on entry and the result on exit.
 * cost_dev (float64, n_iter + 1 entries, may be NULL) receives the MAP cost
 * before every iteration and after the last one.  y_dev: [P][K][M].
 * Errors: EINVAL (prior), ENOMEM, EDEVICE.  Cost divergence is not checked
 * on the device (the call stays asynchronous); callers compare cost_dev. */
int umbir_reconstruct(const umbir_geometry* geom, const umbir_prior* prior,
                      const void* y_dev, int n_iter, float* x_io_dev, float* g_io_dev,
                      double* cost_dev, void* work, size_t work_bytes, void* stream);

/* umbir_reconstruct for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same iteration, arguments and results (bitwise), with the
 * workspace taken from a static device array of UMBIR_NOALLOC_SCRATCH_MIB MiB
 * that the library holds on each GPU it runs on until the process ends, in
 * place of a caller buffer.  The call allocates and frees nothing.  Every call
 * on one GPU shares that GPU's array (no clearing is needed: each call writes
 * every part of it before reading it), so calls whose work may overlap on one
 * GPU (other streams, other threads) race and must not be made.  The
 * geometry's device must be current.
 * Errors: EINVAL (arguments, prior, wrong device), ENOTSUP (the problem needs
 * more than the scratch holds: umbir_workspace_bytes(geom,
 * UMBIR_WORK_RECONSTRUCT) > UMBIR_NOALLOC_SCRATCH_MIB MiB; the plain
 * 256 x 256 workload needs 137 MiB), EDEVICE. */
#define UMBIR_NOALLOC_SCRATCH_MIB 160
int umbir_reconstruct_noalloc(const umbir_geometry* geom, const umbir_prior* prior, const void* y_dev,
                              int n_iter, float* x_io_dev, float* g_io_dev, double* cost_dev, void* stream);

/* MAP reconstruction of Eq. (18) by ICD (Sec. 2, "Optimization") run over a
 * lattice of voxel groups.  Group (a, b), a < group_rows, b < group_cols,
 * holds the voxels with row % group_rows == a and col % group_cols == b
 * (both >= 2, so no two members are 8-neighbours); groups are visited in the
 * order a, then b.  A group moves at once: member v takes its one-voxel ICD
 * step with the prior's neighbours held fixed and the data curvature
 * (Abar^T Abar 1_G)_v / sigma^2 (Abar: the operator of |W| and |b|; 1_G the
 * group's indicator), which bounds the group's block of A^T A, so every group
 * step lowers the cost; the residual is then updated by the group's columns.
 * A sweep records the cost, takes the exact per-trace g step (if
 * estimate_direct), then visits every group.  The curvatures cost one
 * |A| + |A|^T pair per group at the start of the call.  x_io_dev, g_io_dev:
 * warm start in, result out (updated in place as the sweeps run); cost_dev
 * (float64, n_sweeps + 1 entries, may be NULL): the cost before every sweep
 * and after the last.  Deterministic (bitwise reproducible).
 * work: at least umbir_icd_workspace_bytes() bytes, or NULL (allocated in
 * stream order).  Errors: EINVAL (prior, group sizes), ENOTSUP (16-bit
 * storage, attenuation, 8 n_samples + 4 (window * Q + 2) > 64512), ENOMEM,
 * EDEVICE. */
int umbir_reconstruct_icd(const umbir_geometry* geom, const umbir_prior* prior, const void* y_dev,
                          int n_sweeps, int group_rows, int group_cols, float* x_io_dev,
                          float* g_io_dev, double* cost_dev, void* work, size_t work_bytes,
                          void* stream);
size_t umbir_icd_workspace_bytes(const umbir_geometry* geom, int group_rows, int group_cols);

/* Resident MAP solver for one problem (the serving building block): owns a
 * copy of y, the iterate state (x, g), the data-term curvature, a cost history
 * of max_iter + 1 entries and its workspace, all allocated at creation, and
 * one captured HIP graph per iteration so that stepping launches no kernels
 * individually and allocates nothing.  The iteration is the one of
 * umbir_reconstruct (Eq. (18), QGGMRF prior of Eqs. (14)-(17)); a session
 * stepped n times holds bitwise the result of umbir_reconstruct with n
 * iterations.  The geometry must outlive the session.
 *
 * umbir_solver_create: x0_dev ([nz][nx]) and g0_dev ([P][K]) may be NULL
 *   (zeros); y_dev ([P][K][M]) is copied.  Blocks until the state is ready.
 * umbir_solver_step: queues n_iter iterations on `stream` (asynchronous);
 *   EINVAL if the total would exceed max_iter.
 * umbir_solver_read: queues copies of the current x and g (either may be
 *   NULL) and, if cost_dev is not NULL, evaluates the cost of the current
 *   state and copies iterations() + 1 history entries (float64) to cost_dev.
 * umbir_solver_bytes: device bytes a session would hold (for admission).
 * One session must not be stepped from two streams at once. */
typedef struct umbir_solver umbir_solver;
size_t umbir_solver_bytes(const umbir_geometry* geom, int max_iter);
int umbir_solver_create(const umbir_geometry* geom, const umbir_prior* prior, const void* y_dev,
                        const float* x0_dev, const float* g0_dev, int max_iter, void* stream,
                        umbir_solver** out);
int umbir_solver_step(umbir_solver* solver, int n_iter, void* stream);
int umbir_solver_iterations(const umbir_solver* solver);
int umbir_solver_read(umbir_solver* solver, float* x_dev, float* g_dev, double* cost_dev, void* stream);
size_t umbir_solver_state_bytes(const umbir_solver* solver);
void umbir_solver_free(umbir_solver* solver);

/* Batched sessions, for many problems at once (of any mix of shapes): one
 * call advances every session of the batch.
 *  UMBIR_BATCH_STREAMS     the problems run side by side on four internal
 *                          streams (session i on stream i mod 4), forked from
 *                          and joined back to the caller's stream, each
 *                          session's own captured iteration graph on its stream;
 *  UMBIR_BATCH_GRAPH       one graph per iteration, captured once across the
 *                          four streams (one chain of sessions per stream),
 *                          holding every session's iteration;
 *  UMBIR_BATCH_WORKLIST    the problems split into four lanes of about equal
 *                          work, one per internal stream; per lane one launch
 *                          per stage of the iteration (image prescale, splat,
 *                          convolution with the residual, g step, correlation,
 *                          gather (one launch per batch of traces), prior
 *                          update, cost) over all its problems together: the
 *                          blocks of a launch walk a device work list of
 *                          (problem, tile) items of the uneven problems, and
 *                          the lanes' launches of one iteration are one
 *                          captured graph.  Needs FP32 storage, no attenuation,
 *                          the factored operator form and one oversampling
 *                          factor (32 or 64) across the batch (ENOTSUP
 *                          otherwise).
 *                          A session that reaches its max_iter leaves the
 *                          batch (its items are skipped from the next
 *                          iteration on), so one batch can be stepped to the
 *                          largest max_iter of its sessions.
 * Each session's results are bitwise those of stepping it alone.  The
 * sessions must outlive the batch, must all live on the current device, and
 * may appear once each.  While in a batch a session may be read
 * (umbir_solver_read) but must not be stepped alone: umbir_batch_step returns
 * EINVAL if any session's iteration count no longer matches the batch, or
 * (streams and graph modes) if a step would pass a session's max_iter.  umbir_batch_free (like
 * umbir_solver_free) first waits for the last launch it queued to end.
 * Errors: EINVAL, ENOMEM, ENOTSUP, EDEVICE. */
typedef struct umbir_batch umbir_batch;
enum { UMBIR_BATCH_STREAMS = 0, UMBIR_BATCH_GRAPH = 1, UMBIR_BATCH_WORKLIST = 2 };
int umbir_batch_create(umbir_solver* const* sessions, int n, int mode, umbir_batch** out);
int umbir_batch_step(umbir_batch* batch, int n_iter, void* stream);
void umbir_batch_free(umbir_batch* batch);

/* Dimensions of a built geometry, for callers that size buffers. */
typedef struct {
    int nx, nz, n_scans, n_rx, n_samples;
    int n_off;        /* lateral lattice positions per leg-table row */
    int window;       /* L_h */
    int oversample;   /* Q */
    int n_layers;
    int trace_groups; /* traces are summed in this many groups by the adjoint's gather */
    int storage;      /* UMBIR_STORAGE_* of trace buffers */
    int n_gamma;      /* attenuation templates in use (1 without attenuation) */
    double gamma_step;/* dgamma [s] between templates (0 with one template) */
} umbir_dims;
int umbir_get_dims(const umbir_geometry* geom, umbir_dims* out);

/* Launch and tile shapes of the sweeps, tunable per problem shape.  None
 * changes a result beyond rounding order, nor any memory size:
 *  splat_blocks     target workgroup count of the splat: the fine grid of each
 *                   trace is cut into ceil(splat_blocks / traces) chunks of at
 *                   least 1024 positions.  Results are bitwise identical for
 *                   every value (the splat sums in fixed point).
 *  gather_batch_kb  fine-grid KiB of each trace group per gather launch (at
 *                   least one trace per launch).  Default at build: 4096,
 *                   or with the windowed gather (gather_form 2 by default)
 *                   16 traces for every tile one of its workgroups takes
 *                   when that is more.
 *                   Changes only the order of the adjoint's sums across
 *                   launches.
 *  conv_grid        tile order of the matrix-core convolution (32 traces per
 *                   workgroup): 1 trace tiles fastest, 2 sample tiles
 *                   fastest.  Bitwise identical results.
 *  conv_tile_rows   output samples per matrix-core convolution workgroup:
 *                   32, 64 or 128; the workgroup's waves (eight with
 *                   bf16-piece products when the grid leaves fewer than two
 *                   workgroups per CU, else four) share each fetched chunk of
 *                   fine-grid rows among its 32-sample tiles.  Default at build: with bf16-piece products, 128
 *                   when that leaves at least 256 workgroups, else 64
 *                   likewise; otherwise 64 when that leaves at least 512
 *                   workgroups, else 32.  Changes only the order of the
 *                   sums.
 *  corr_tile_rows   rows (output samples) of one wave's tile in the
 *                   matrix-core correlation with FP32 products: 32, 64 or
 *                   128 (default; a workgroup of four waves covers four
 *                   tiles).  Bitwise identical results.  (With bf16-piece
 *                   products a workgroup's row block is 256 rows, two
 *                   8-strided tiles per wave, whatever this field says.)
 *  corr_blocks      target workgroup count of the correlation: each workgroup
 *                   walks ceil(traces x row blocks / corr_blocks) row blocks of
 *                   one trace with the taps staged once (default 512 with
 *                   bf16-piece products, 1024 with FP32 products).  Bitwise
 *                   identical.
 *  operator_form    1: the factored form (default): A = splat then polyphase
 *                   convolution, A^T = polyphase correlation then gather;
 *                   2: the direct form of Eq. (13): every (trace, voxel) pair
 *                   sums its window of L_h taps (A: one workgroup per trace
 *                   accumulating its samples in LDS; A^T: per voxel over the
 *                   traces).  The same operator summed in another order
 *                   (results agree to rounding).  Direct needs FP32 storage,
 *                   no attenuation and 8 M + 4 (Q L_h + 2) <= 65536 (ENOTSUP
 *                   from umbir_set_tuning otherwise); it suits small problems.
 *  products         how the matrix-core convolution and correlation (FP32
 *                   storage) form their FP32 products: 1 as FP32 products
 *                   (v_mfma_f32_32x32x2f32); 2 (default) on the bf16 matrix
 *                   cores, each factor split exactly into three bf16 pieces
 *                   and the product taken as the six piece products whose
 *                   orders sum to at most 4 (v_mfma_f32_32x32x16_bf16, FP32
 *                   accumulation; the three left out are below 2^-23 of the
 *                   product).  Results agree to rounding.  Where the
 *                   pieces' tables would not fit a workgroup's LDS (long
 *                   templates) the library uses the FP32 products.
 *  gather_form      the factored adjoint's gather (one template): 1
 *                   row-wise, each voxel's two taps loaded from the fine
 *                   grid in global memory; 2 windowed, each 32 x 64 voxel
 *                   tile's window of a trace's fine grid staged in LDS first
 *                   (windows over 64 KiB loaded as in 1).  2 needs the
 *                   geometry's window table, built where attenuation or a
 *                   record of fine positions not a multiple of 16 bytes
 *                   does not rule it out (ENOTSUP from umbir_set_tuning
 *                   otherwise).
 *                   Default at build: 2 when its workgroups fill at least
 *                   three quarters of one generation (two per CU), else 1.
 *                   Bitwise identical results.
 * A field of 0 (or less) in umbir_set_tuning keeps the current value (EINVAL
 * for a conv_grid, conv_tile_rows, corr_tile_rows, products or gather_form
 * outside the values above).  The tuning of
 * a geometry must not change while another call uses it.
 * umbir_autotune times candidates of each field on `stream` (an A + A^T pair
 * for the form, the forward for the splat and the convolution, the adjoint
 * for the correlation and the gather, a dense all-ones image), applies the
 * fastest and writes the chosen values to *chosen (may be NULL); it allocates
 * its own workspace and synchronizes the stream.  Errors: EINVAL, ENOMEM,
 * EDEVICE. */
typedef struct {
    int splat_blocks;
    int gather_batch_kb;
    int conv_grid;
    int conv_tile_rows;
    int corr_tile_rows;
    int corr_blocks;
    int operator_form;
    int products;
    int gather_form;
} umbir_tuning;
int umbir_get_tuning(const umbir_geometry* geom, umbir_tuning* out);
int umbir_set_tuning(umbir_geometry* geom, const umbir_tuning* tuning);
int umbir_autotune(umbir_geometry* geom, void* stream, umbir_tuning* chosen);

/* Copies a resident table to host memory (synchronous), for inspection:
 *  UMBIR_TABLE_DELAY  int64 [nz][n_off]  one-way leg delay, Q32.32 samples
 *  UMBIR_TABLE_APOD   float [nz][n_off]  cos^beta of the leg's angle sum
 *  UMBIR_TABLE_TAU    float [nz]         transmittance product of the row
 *  UMBIR_TABLE_BANK   float [n_gamma][Q*L_h + 2]  tabulated windowed responses
 *                                        (+ zero pad), one per attenuation template
 *  UMBIR_TABLE_DBASIS float [P][K][M]    direct-arrival columns of D
 *  UMBIR_TABLE_OFFSET int32 [P + P*K]    lattice index base of each transducer
 *  UMBIR_TABLE_ATTEN  double [nz][n_off] leg path attenuation Gamma_leg /
 *                                        gamma_step in template bins (0 without
 *                                        attenuation)
 * `bytes` must equal the table's size.  Errors: EINVAL, EDEVICE. */
enum { UMBIR_TABLE_DELAY = 0, UMBIR_TABLE_APOD = 1, UMBIR_TABLE_TAU = 2,
       UMBIR_TABLE_BANK = 3, UMBIR_TABLE_DBASIS = 4, UMBIR_TABLE_OFFSET = 5,
       UMBIR_TABLE_ATTEN = 6 };
int umbir_copy_table(const umbir_geometry* geom, int which, void* host_dst, size_t bytes);

/* Opt-in per-kernel timing for callers that measure the library (benchmarks,
 * profilers).  While enabled, every kernel launch is bracketed by two HIP
 * events on its stream (this adds event records between launches).
 * umbir_profile_collect waits for the recorded events, writes one entry per
 * kernel name (launch count and summed duration since the last collect) into
 * out[0 .. max_entries), sets *n_out to the number of names, and resets the
 * totals.  Process-wide; thread-safe.  Errors: EINVAL, EDEVICE. */
typedef struct {
    char name[48];
    long long launches;
    double total_ms;
} umbir_kernel_time;
void umbir_profile_enable(int on);
/* Restricts the timing to the kernels named in `names` (comma-separated, the
 * names umbir_profile_collect reports); NULL or "" times every kernel.  The
 * fewer launches are bracketed, the less the events perturb the work timed. */
void umbir_profile_select(const char* names);
/* While a selection is set, times only every `every`-th launch of each
 * selected kernel, counted from this call or from the last
 * umbir_profile_select (every <= 1: every launch).  Launches of identical
 * work are then measured on a sample, with fewer event records between the
 * launches of the work being timed. */
void umbir_profile_stride(int every);
int umbir_profile_collect(umbir_kernel_time* out, int max_entries, int* n_out);

const char* umbir_strerror(int status);
const char* umbir_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* UMBIR_H */
