/*
 * hipoisson -- spectral Poisson solver for AMD Instinct MI355X (gfx950).
 *
 * Solves lap(psi) = f on 1D/2D/3D rectangular grids by the four steps of the
 * SailFFish method (Section 2.2): forward transform, pointwise multiply by a
 * spectral multiplier, optional spectral derivative, backward transform.
 *
 *   periodic    DFT, PS or FD2 eigenvalues             (Table 1, last row)
 *   Dirichlet   DST-I / DST-II+III, PS or FD2          (Table 1)
 *   Neumann     DCT-I / DCT-II+III, PS or FD2          (Table 1; the printed
 *               "DST-III" backward transform for the staggered grid is read
 *               as DCT-III, the inverse of DCT-II)
 *   unbounded   Hockney-Eastwood domain doubling with a precomputed spectral
 *               Green's function (Section 2.5), R2C / C2R for real data
 *
 * Grids (Section 2.3.2, eq. gridpos): REGULAR solves on cell boundaries,
 * STAGGERED on cell centres.  Unknown counts per axis for N_c cells:
 *   Dirichlet REGULAR N_c - 1 (output N_c + 1 nodes incl. boundary nodes),
 *   Neumann REGULAR N_c + 1, unbounded REGULAR N_c + 1, all others N_c.
 *
 * Memory layout: every field is a C-contiguous array [n_0][n_1][n_2] (last
 * axis contiguous) of float (HP_F32) or double (HP_F64); a 3-component field
 * is three separate arrays, one per component.
 *
 * Ownership: the plan owns its workspaces and tables.  The caller owns every
 * input, boundary and output buffer.  Device pointers passed with
 * on_device = 1 are bound, not copied: they are read or written by the solve
 * when it runs on the plan's stream and must stay valid until it completes.
 * Host pointers (on_device = 0) are copied with stream-ordered copies.
 *
 * Errors: every call returns hp_status; no C++ exception crosses this
 * interface.  hp_last_error() gives a message for the last failure of a plan.
 * A plan is not re-entrant: use one plan per stream.  Descriptor validation
 * happens before any GPU call, so invalid descriptors are reported on
 * machines without a GPU.
 */
#ifndef HIPOISSON_H
#define HIPOISSON_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define HP_API __attribute__((visibility("default")))
#else
#define HP_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hp_plan_s* hp_plan; /* opaque, library-owned */
typedef void* hp_stream;           /* a hipStream_t; NULL = the null stream */

typedef enum {
  HP_OK = 0,
  HP_E_ARG = -1,         /* invalid argument or descriptor */
  HP_E_UNSUPPORTED = -2, /* valid, but not provided by this library */
  HP_E_NOMEM = -3,       /* device or host allocation failed */
  HP_E_DEVICE = -4,      /* a HIP runtime call failed */
  HP_E_STATE = -5        /* call out of order (e.g. output before a solve) */
} hp_status;

/* HP_MIXED: a different condition per axis, each periodic, Dirichlet or
 * Neumann (bc_axis of the descriptor; both faces of an axis alike).  The
 * paper builds its solves from 1D transforms per axis (Section 2.6 names
 * mixed conditions through combinations of DST, DCT and DFT); here a periodic
 * axis runs the discrete Hartley transform (real to real, its own inverse up
 * to n, diagonal for the periodic Laplacian) beside the Table 1 sine and
 * cosine transforms, with the eigenvalue sum of eq. (pois_spec) over the
 * axes.  PS or FD2; boundary values (FD2) on the Dirichlet / Neumann faces.
 * Derivative outputs (GRAD, CURL, DIV, NABLA) take each axis's own rule: the
 * sine / cosine series of Table 1's eigenfunctions, the Hartley spectral
 * derivative along periodic axes; with boundary values second-order
 * differences of psi instead (NABLA then HP_E_UNSUPPORTED).
 * Semi-unbounded: one axis (of 2 or 3) may be HP_UNBOUNDED.  Each bounded
 * mode, eigenvalue sum Lambda, then solves psi'' - kappa^2 psi = f along the
 * free axis (kappa^2 = -Lambda, Section 2.6's Helmholtz split), convolved by
 * the Hockney-Eastwood doubling (M = 2 n, Section 2.5) with the exact 1D
 * Green's function -exp(-kappa |x|) / (2 kappa) (|x| / 2 for kappa = 0) times
 * the cell length.  The free axis has no faces.  GRAD, CURL and DIV of
 * homogeneous problems: the free axis's derivative is the convolution with
 * the kernel's derivative sign(x) exp(-kappa |x|) / 2; NABLA, or derivatives
 * with boundary values, return HP_E_UNSUPPORTED. */
typedef enum { HP_PERIODIC = 0, HP_DIRICHLET = 1, HP_NEUMANN = 2, HP_UNBOUNDED = 3,
               HP_MIXED = 4 } hp_bc;
typedef enum { HP_REGULAR = 0, HP_STAGGERED = 1 } hp_grid;
/* Spectral multiplier: PS / FD2 eigenvalues (Table 1) for bounded BCs; for
 * unbounded ones a 3D free-space kernel of Section 2.5.2, which names Gaussian
 * kernels of orders 2 to 10 and a spectral kernel without printing them.  Each
 * is read here through its spectrum G^(k) = -zeta^(k) / k^2:
 *   HP_G_GAUSS<2m>: zeta^ = exp(-s) sum_{j<m} s^j / j!, s = (k sigma)^2 / 2
 *     (error O(sigma^(2m)); sigma = reg_sigma_cells * max_a H_a); in space
 *     G(r) = -(1/(4 pi r)) [erf(rho/sqrt2) + sqrt(2/pi) exp(-rho^2/2)
 *            sum_{j=1}^{m-1} (-1)^(j-1) He_{2j-1}(rho) / (2^j j!)], rho = r / sigma;
 *   HP_G_SPECTRAL: zeta^ = 1 for |k| <= pi / max_a H_a, else 0; in space
 *     G(r) = -Si(k_c r) / (2 pi^2 r).
 * 2D and 1D plans use the same spectra, whose kernels grow as ln(r) / (2 pi)
 * and |x| / 2; every kernel is available in every dimension.  1D order 2m:
 * G(x) = (x/2) erf(rho/sqrt2) + (sigma / sqrt(2 pi)) exp(-rho^2/2)
 *        [1 + sum_{j=1}^{m-1} (-1)^j He_{2j-2}(rho) / (2^j j!)]. */
typedef enum {
  HP_OP_PS = 0, HP_OP_FD2 = 1,
  HP_G_GAUSS2 = 2, HP_G_GAUSS4 = 3, HP_G_GAUSS6 = 4, HP_G_GAUSS8 = 5, HP_G_GAUSS10 = 6,
  HP_G_SPECTRAL = 7
} hp_kernel;
/* Spectral operator applied to psi after the convolution (Section 2.3.3's
 * list): GRAD of a scalar (ndim extra outputs), CURL of a 3D vector (3
 * outputs) or of a 2D scalar ((d_y psi, -d_x psi), 2 outputs, the form
 * Section 4.3 treats as the gradient's 2D counterpart), DIV of a 3D vector
 * (1 output), NABLA, the Laplacian of every
 * component (ncomp outputs).  Derivatives multiply by i k_a with the Nyquist
 * mode set to zero; NABLA is that first derivative applied twice per axis and
 * summed.  Periodic and free-space
 * plans take every operator; Dirichlet / Neumann plans take every operator
 * with homogeneous boundary values (HP_E_UNSUPPORTED otherwise), as
 * derivatives of the Table 1 sine (cosine) series through psi evaluated at the
 * output points: a first derivative along an axis turns that axis's series
 * into a cosine (sine) series (REGULAR Dirichlet: every node, the normal
 * derivative on the boundary nodes); NABLA keeps each series, every
 * eigenfunction times -(pi kappa / L)^2 per axis.  Batched plans take
 * HP_D_NONE only. */
typedef enum { HP_D_NONE = 0, HP_D_GRAD = 1, HP_D_CURL = 2, HP_D_DIV = 3, HP_D_NABLA = 4 } hp_diff;
typedef enum { HP_F32 = 0, HP_F64 = 1 } hp_prec;

typedef struct {
  int ndim;             /* 1, 2 or 3 */
  int ncomp;            /* 1 (scalar) or 3 (3D vector, component-wise) */
  int64_t nc[3];        /* cells per axis N_c (entries >= ndim ignored) */
  double lo[3], hi[3];  /* domain bounds X_l < X_u per axis */
  int bc;               /* hp_bc, the same on every face (HP_MIXED: per axis) */
  int grid;             /* hp_grid */
  int kernel;           /* hp_kernel */
  int diff;             /* hp_diff */
  int prec;             /* hp_prec: data and FFT precision; tables are FP64-built */
  int inhomogeneous;    /* 1: boundary values from hp_set_boundary (FD2 only) */
  double reg_sigma_cells; /* G2 width sigma in units of max_a H_a; 0 -> 2.0 */
  int bc_axis[3];       /* bc == HP_MIXED: hp_bc of each axis (HP_PERIODIC,
                           HP_DIRICHLET, HP_NEUMANN, or HP_UNBOUNDED on at
                           most one axis); ignored otherwise */
} hp_desc;

/* Query keys for hp_query. */
enum {
  HP_Q_MODEL_BYTES = 1,     /* algorithmic HBM bytes of one hp_solve */
  HP_Q_WORKSPACE_BYTES = 2, /* device workspace held by the plan */
  HP_Q_NUM_PASSES = 3,      /* kernel launches of one hp_solve */
  HP_Q_NUM_OUTPUTS = 4,     /* psi components + derivative components */
  HP_Q_NUM_DERIVS = 5,      /* derivative components (gradient or curl) */
  HP_Q_BATCH_ERROR = 6,     /* batched plans: 1 if the last solve hit a dependency-wait
                               limit (results invalid), else 0; synchronises */
  HP_Q_TUNED_PASSES = 7,    /* pass signatures whose configuration hp_autotune changed */
  HP_Q_TUNE_DEFAULT_MS = 8, /* milliseconds of one solve with the planner's defaults,
                               measured by the last hp_autotune */
  HP_Q_TUNE_BEST_MS = 9,    /* the same with the configuration it kept */
  HP_Q_BATCH_TILES = 10,    /* batched plans: tiles per work item of the persistent kernel */
  HP_Q_ZERO_MODE = 11,      /* periodic / Neumann plans: the part of the bound source (with its
                               FD2 boundary terms) that the k = 0 projection removes, i.e. the
                               k = 0 coefficient of its forward transform over that of a field
                               of ones (the weighted mean, DCT-I ends weighted 1/2); 0 for a
                               compatible source and for other BCs; 3-component plans give
                               the component of largest magnitude; synchronises */
  HP_Q_BATCH_KERNEL = 12    /* batched plans: 0 = one persistent launch of the general passes,
                               1 = one persistent launch of the wavefront-FFT tile bodies (FP32,
                               every transform length 64, 96, 128, 192 or 256), 2 = the same
                               tile bodies as one launch per pass level (chosen by hp_autotune
                               only) */
};

/* Create a plan for one problem (the initialisation of Section 3.2.1): grid
 * geometry, eigenvalue tables or the Green's spectrum (computed in FP64 on
 * the GPU for unbounded problems), twiddle tables, workspaces.  Any cell count
 * is accepted (Section 2.3.2): transform lengths with prime factors above 5
 * run a direct stage per such prime (R multiply-adds per output), so they are
 * slower than 2^a 3^b 5^c lengths; a length above 8192 (FP32) or 4096 (FP64),
 * or a doubled free-space length above 4096 (the Green's function is
 * transformed in FP64), returns HP_E_UNSUPPORTED.  Returns HP_E_ARG / HP_E_UNSUPPORTED for
 * descriptors it cannot serve.  Blocking. */
HP_API hp_status hp_plan_create(const hp_desc* desc, hp_stream stream, hp_plan* out);

/* A plan over `count` independent problems (descs[0..count-1]); they must
 * share bc, grid, kernel, diff, prec and ndim and may differ in size.  One
 * hp_solve launches a single persistent kernel that runs every pass of every
 * problem.  Supported for bounded, non-periodic, homogeneous problems.  When
 * every transform length of every problem is 64, 96, 128, 192 or 256 (FP32)
 * the launch runs one FFT per wavefront, otherwise the general LDS-staged
 * passes (HP_Q_BATCH_KERNEL; hp_autotune may choose either). */
HP_API hp_status hp_plan_create_batched(const hp_desc* descs, int count, hp_stream stream, hp_plan* out);

/* Unknown (input) and output point counts per axis of problem `problem`;
 * shape[a] = 1 for a >= ndim. */
HP_API hp_status hp_input_shape(hp_plan plan, int problem, int64_t shape[3]);
HP_API hp_status hp_output_shape(hp_plan plan, int problem, int64_t shape[3]);

/* Source f of component `comp` (Section 3.2.2, Set_Input): an array with the
 * input shape.  on_device = 1 binds a device pointer; 0 copies from host. */
HP_API hp_status hp_set_input(hp_plan plan, int problem, int comp, const void* f, int on_device);

/* Boundary values of face (axis, side) (side 0 = lower, 1 = upper) for
 * inhomogeneous FD2 Dirichlet / Neumann plans (Section 2.4.2): an array with
 * the output shape of the other axes (ascending axis order).  Dirichlet: psi
 * on the face; Neumann: d(psi)/dx_axis on the face.  NULL = homogeneous.  A
 * periodic or free axis of an HP_MIXED plan has no faces (HP_E_ARG unless g
 * is NULL). */
HP_API hp_status hp_set_boundary(hp_plan plan, int problem, int axis, int side, int comp,
                          const void* g, int on_device);

/* Bind caller-owned device buffers that the solve writes directly: psi of
 * component `comp` (output shape), and derivative component `comp`
 * (gradient d/dx_comp or curl component comp, output shape).  Without a
 * binding the plan writes into buffers it owns. */
HP_API hp_status hp_bind_output(hp_plan plan, int problem, int comp, void* psi);
HP_API hp_status hp_bind_gradient(hp_plan plan, int problem, int comp, void* out);

/* Run the solve (Section 3.2.2 steps 2-4) on the plan's stream, without host
 * synchronisation.  Returns HP_E_STATE if an input is missing. */
HP_API hp_status hp_solve(hp_plan plan);

/* Transpose of the solve map f -> (psi, derivatives), for back-propagation.
 * Reads the upstream gradients from the buffers bound with hp_bind_output /
 * hp_bind_gradient (a NULL binding is a zero gradient) and writes the
 * gradient with respect to f into the buffers bound with hp_set_input
 * (on_device = 1 required).  Unbounded plans: the Green's operator is
 * symmetric, the curl symmetric and the gradient's transpose is minus the
 * divergence.  Other plans: HP_E_UNSUPPORTED. */
HP_API hp_status hp_solve_adjoint(hp_plan plan);

/* Copy psi / a derivative component to `dst` (Get_Output).  Stream-ordered;
 * a device-to-host copy synchronises the stream.  HP_E_STATE before the
 * first solve. */
HP_API hp_status hp_get_output(hp_plan plan, int problem, int comp, void* dst, int on_device);
HP_API hp_status hp_get_gradient(hp_plan plan, int problem, int comp, void* dst, int on_device);

/* Per-pass instrumentation for benchmarks.  enable: 0 off; 1: hp_solve
 * records a HIP event pair around every kernel it launches on the plan's
 * stream; 2 + k: around pass k only (one pair per solve, so the solve's own
 * time is barely perturbed); negative: HP_E_ARG.  hp_pass_stats synchronises
 * the stream and returns, for each of the `*npass` passes of a solve (at most
 * `max`), the mean elapsed milliseconds over the solves recorded since the
 * last call (ms; 0 for a pass that was not timed), the algorithmic HBM bytes
 * of the pass (bytes: stored input read once plus stored output written once,
 * plus the Green's octant) and a static name (names); any output may be NULL. */
HP_API hp_status hp_set_timing(hp_plan plan, int enable);
HP_API hp_status hp_pass_stats(hp_plan plan, int max, int* npass, double* ms, double* bytes,
                               const char** names);

/* Autotuning of the plan's kernel configurations (not a step of the paper's
 * method: the paper leaves the FFT plan to its FFT library).  For every
 * distinct pass geometry of the plan it times, on the plan's stream, `reps`
 * runs (< 1: 5; at most 100) of each configuration the kernels are built for:
 * general kernels, every radix order of the length over radices 2, 3, 4, 5, 8
 * with tile widths of 1/2, 1 and 2 times the planner's choice and both
 * register budgets; wavefront passes, 8- and 16-pencil tiles and both
 * output-tile schemes; batched plans, 1, 2, 4 or 8 tiles per work item.  A
 * configuration replaces the default when it is at least 3% faster, and the
 * choices are kept only if the whole solve (batched plans: the whole batch,
 * which also decides the work-item size) is faster with them; later solves of
 * this plan use them.  Batched plans keep every pass within the register
 * budget and LDS of the default persistent kernel.  The tuned plan is then run against the default
 * on the same pseudo-random input and every output must agree to rounding
 * (relative L2 difference <= 1e-5 FP32, <= 1e-12 FP64); otherwise the tuning
 * is dropped and HP_E_DEVICE returned.  Works on scratch arrays it allocates
 * and frees: bound inputs, outputs and workspaces keep their bindings (plan
 * workspaces are overwritten).  Blocking; HP_E_STATE under stream capture.
 * A batched plan must run one hp_solve after tuning before it is captured. */
HP_API hp_status hp_autotune(hp_plan plan, int reps);

/* Numeric plan properties (HP_Q_* keys). */
HP_API hp_status hp_query(hp_plan plan, int what, double* value);

/* Measurement utility (not a step of the method): copy `bytes` of device
 * memory from src to dst on `stream` with a plain streaming kernel (16-byte
 * loads and stores), the reference rate of a kernel that only moves data,
 * for stating the solve's bandwidth against what the device reaches.  Both
 * pointers 16-byte aligned and not overlapping; HP_E_ARG otherwise. */
HP_API hp_status hp_device_copy(const void* src, void* dst, size_t bytes, hp_stream stream);

/* The zero mode of HP_Q_ZERO_MODE without allocation or host
 * synchronisation, for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Writes out[c], c < ncomp, for every component of the bound source (device
 * memory owned by the caller, ncomp doubles): the k = 0 coefficient of its
 * forward transform over that of a field of ones, 0 for BCs without a zero
 * eigenvalue; out[] holds the same values as the per-component results of
 * HP_Q_ZERO_MODE, which returns the one of largest magnitude.  Runs
 * asynchronously on the plan's stream (two small kernels per component, no
 * memset, so it can be captured).  Its partial sums (256 FP64 values per
 * component, 3 components at most: 6 KiB) live in a static device array of
 * the library, one per GPU, held until the process ends; this call allocates
 * nothing.  Calls that overlap on one GPU (other streams, other threads) share
 * that array and race.  HP_E_ARG for a NULL plan or out or a batched plan,
 * HP_E_STATE if an input is not set, HP_E_UNSUPPORTED above 3 components,
 * HP_E_DEVICE if a launch fails. */
HP_API hp_status hp_zero_mode_noalloc(hp_plan plan, double* out);

/* Release the plan and everything it owns (synchronises its stream). */
HP_API hp_status hp_plan_destroy(hp_plan plan);

/* Static text for a status code; message of the last failure on `plan`
 * (or of the last failed plan creation when plan is NULL). */
HP_API const char* hp_status_string(hp_status status);
HP_API const char* hp_last_error(hp_plan plan);

#ifdef __cplusplus
}
#endif

#endif /* HIPOISSON_H */
