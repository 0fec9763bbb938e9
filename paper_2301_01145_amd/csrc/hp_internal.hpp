// Internal types shared by the host planner and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hp {

// Transform applied along the pencil axis of a pass.  Real-to-real and
// real/complex conversions are computed with one complex FFT of length L on a
// pair of real pencils (a + i b) and an extension or twiddle around it.
enum Xform : int {
  X_C2C_F = 0,  // complex DFT, exponent sign -1 (eq. dft, forward)
  X_C2C_B = 1,  // complex DFT, exponent sign +1, unscaled
  X_R2C = 2,    // real -> half spectrum (L/2 + 1), L = FFT length
  X_C2R = 3,    // half spectrum -> real, unscaled
  X_PAIR_F = 4, // two real pencils as one complex pencil, forward DFT
  X_PAIR_B = 5, // inverse of X_PAIR_F (real part -> first, imag -> second)
  X_DST1 = 6,   // L = 2 (n + 1), odd extension
  X_DST2 = 7,   // via DCT-II of (-1)^j x_j, reversed output
  X_DST3 = 8,   // via DCT-III of the reversed input, (-1)^k output
  X_DCT1 = 9,   // L = 2 (n - 1), even extension
  X_DCT2 = 10,  // L = 2 n, symmetric extension and e^{-i pi k / 2n}
  X_DCT3 = 11,  // L = 2 n, e^{+i pi j / 2n} Hermitian input, inverse DFT
  X_DHT = 12    // discrete Hartley transform, L = n: H_k = Re X_k - Im X_k of the
                // DFT X; real to real and its own inverse up to n (periodic axes
                // of mixed-boundary plans)
};

enum PassKind : int { PK_ONEWAY = 0, PK_SANDWICH = 1 };
enum MultKind : int { M_NONE = 0, M_EIGEN = 1, M_GREEN = 2,
                      // semi-unbounded free axis: one real-even row of the
                      // Helmholtz Green's spectrum per bounded mode of the
                      // pencil (green[m g_s[ax_j] + p g_s[ax_p] + o g_s[ax_o]],
                      // m <= L / 2), paired real pencils
                      M_GREEN_ROWS = 3,
                      // the same for the free-axis derivative: rows b of the
                      // odd kernel's spectrum i b(m) (b real, odd in m)
                      M_GREEN_ROWS_ODD = 4 };
// Derivative coupling inside the sandwich pass (D_ADJ_*: the transposes used
// by the adjoint solve).
enum DiffKind : int { D_NONE = 0, D_GRAD = 1, D_CURL = 2, D_ADJ_GRAD = 3, D_ADJ_CURL = 4,
                      D_DIV = 5, D_NABLA = 6, D_ADJ_DIV = 7, D_ADJ_NABLA = 8 };
__host__ __device__ inline bool diff_is_adjoint(int d) {
  return d == D_ADJ_GRAD || d == D_ADJ_CURL || d == D_ADJ_DIV || d == D_ADJ_NABLA;
}

// Threads per workgroup of the general pencil kernels (and the persistent
// batched kernel); the wavefront-FFT kernels size their own workgroups.
#ifndef HP_GEN_THREADS
#define HP_GEN_THREADS 256
#endif
constexpr int kThreads = HP_GEN_THREADS;
// Longest transform of the general path: 32 (FP32) or 16 (FP64) elements per
// thread of a 256-thread workgroup.
constexpr int kMaxLenThreads = 256;
constexpr int kMaxStages = 8;
constexpr int kMaxFields = 6;

struct PassArgs {
  int kind;          // PassKind
  int xf, xb;        // forward transform (and backward for the sandwich)
  int L;             // FFT length
  int n;             // transform length n of the real-to-real family
  int nin, nout;     // stored elements along the pencil on input / output
  int P;             // pencils per tile
  int Np, No;        // pencils along the tile axis / outer axis
  int in_jfast, out_jfast;  // 1: pencil axis has unit stride on that side
  int nstage;
  int radix[kMaxStages];
  long long in_sj, in_sp, in_so;    // strides (elements) of the input side
  long long out_sj, out_sp, out_so; // strides (elements) of the output side
  int n_in, n_out;   // field counts (sandwich: coupled; one-way: per blockIdx.y)
  const void* in[kMaxFields];
  void* out[kMaxFields];
  const void* tw;    // complex T, W_L^m = exp(-2 pi i m / L), m < L
  const void* qtw;   // complex T, exp(-i pi j / (2 n)), j < n (DCT-II/III family)
  int ax_j, ax_p, ax_o;  // logical axis of the pencil / tile / outer index (-1: none)
  // multiplier of the sandwich
  int mult;
  const double* lam[3];  // per-axis eigenvalues (FP64)
  double norm;           // product of the backward normalisations
  const void* green;     // Ghat octant (T), norm folded in, layout [k2][i1][i0]
  long long g_s[3];      // octant strides of i0, i1, k2
  int gM[3];             // doubled sizes M_a
  int diff;
  const void* kvec[3];   // T, angular wavenumber per index (Nyquist 0)
  // boundary terms added while loading the first pass (FD2 inhomogeneous)
  const void* face[3][2];
  long long face_s[3][2];  // strides of the two remaining axes (ascending)
  int face_off;            // bit b: face arrays include the boundary nodes of axis b
                           // (REGULAR Dirichlet axes)
  double face_w[3][2];     // weight applied to g
  int nunk[3];             // unknown counts per logical axis
  int lds_bytes;
  int big;                 // general kernels: 1 = the larger per-thread register budget
  // wavefront-FFT kernels of the free-space path (0: general pass)
  int fast;                // FAST_* below
  int un[3];               // physical (undoubled) sizes n_a
  double kc[3];            // 2 pi / (M_a H_a): angular wavenumber per index
  int iy_mode;             // InvYMode of the backward y pass
  int kz_base, kz_count;   // kz slab of the y and x passes (B2 / C2 hold kz_count planes)
  int emit_dbl;            // x / backward-y passes: double-buffered output tiles
  int c1_ld;               // row length (kz) of C1: K2 rounded up to 16
  long long c1_sx, c1_sy;  // C1 strides (elements) of x and y
  int ngrp;                // x pass: output groups per tile (set at launch)
  int pad;                 // 1: doubled free-space pencils (physical half), 0: periodic
  // signature of the pass geometry (host planner): passes with equal keys
  // share the configuration chosen by the autotuner
  unsigned long long tune_key;
  // FAST_GRAD_PREP (series derivative along ax_j): output element i (logical
  // axes, extents gp_ext, strides gp_os) is active where s = i - gp_off lies
  // in [0, gp_len) on every axis.  gp_basis[b] names axis b's series: 0 sine
  // (index k carries wavenumber k + 1), 1 cosine (k), 2 Hartley (signed k,
  // Nyquist 0).  Along ax_j a sine / cosine source is read at src = s +
  // gp_shift and scaled by gp_scale times src's wavenumber; a Hartley source
  // at -s (mod nunk), scaled by -gp_scale times s's signed wavenumber.  Other
  // axes read src = s (strides gp_is, extents nunk).  With gp_eigen the value
  // is divided by sum_b lam[b][src_b] / norm (0 where that sum is 0).
  // ax_j < 0 without D_NABLA: a copy, src = s on every axis, times gp_scale.
  // Elements that are not active, or whose source lies outside, are 0.
  int gp_ext[3], gp_off[3], gp_len[3];
  int gp_shift, gp_basis[3], gp_eigen;
  double gp_scale;
  long long gp_is[3], gp_os[3];
};

enum FastKind : int { FAST_NONE = 0, FAST_R2C = 1, FAST_FWD_Y = 2, FAST_SANDWICH = 3,
                      FAST_INV_Y = 4, FAST_C2R = 5,
                      // bounded real-to-real passes (hp_bounded.hip)
                      FAST_R2R_C = 6, FAST_R2R_S = 7, FAST_R2R_SW = 8,
                      // elementwise: spectral derivative coefficients (hp_bounded.hip)
                      FAST_GRAD_PREP = 9,
                      // elementwise: out[0] += in[0] (+ in[1]) over gp_ext[0] elements
                      FAST_ADD = 10,
                      // the whole 2D periodic solve in one workgroup (hp_small.hip):
                      // lengths gM[0] x gM[1], twiddles of the x FFT in tw and of
                      // the y FFT in qtw, n_in inputs, n_out outputs
                      FAST_SMALL2D = 11 };
// Derivative completion in the backward y pass of the free-space path.
enum InvYMode : int { IY_PLAIN = 0, IY_CURL5 = 1, IY_GRAD2 = 2 };

// Elements per lane of the wavefront FFT of length L (0: no such FFT):
// powers of two 64 .. 1024 (8, 16 from 1024) and 48, 96, 192 (12).
__host__ __device__ constexpr int wf_r0(int L) {
  return (L == 48 || L == 96 || L == 192) ? 12
         : (L >= 64 && L <= 1024 && (L & (L - 1)) == 0) ? (L >= 1024 ? 16 : 8)
                                                         : 0;
}

// Launch one wavefront-FFT pass (power-of-two L in [64, 1024]).
hipError_t launch_fast(const PassArgs& a, int prec, int grid_y, hipStream_t s);
hipError_t launch_bounded(const PassArgs& a, int prec, hipStream_t s);
// Derivatives of a Dirichlet / Neumann (or mixed) FD2 solve with boundary
// values (hp_bounded.hip): out = sum of up to three terms sign * d psi_c /
// d x_axis, centred second-order differences at every output point, closed by
// the Neumann ghost rules and one-sided second-order differences at Dirichlet
// faces, wrapped along periodic axes.  Arrays are C-contiguous over the output
// points N[0..nd).
enum FdBc : int { FD_PERIODIC = 0, FD_DIRICHLET = 1, FD_NEUMANN = 2 };
struct FdTerm {
  const void* psi;                // component on the output points
  const void* g_lo;               // face values of `axis` (lower, upper side;
  const void* g_hi;               //  null = 0), over the other axes' output points
  int axis;
  double sign;
};
struct FdArgs {
  void* out;
  int nd;
  int N[3];
  double h[3];
  int bc[3];  // FdBc of each axis
  int regular;
  int nterm;
  FdTerm t[3];
};
hipError_t launch_fd_deriv(const FdArgs& a, int prec, hipStream_t s);

// single-launch 2D periodic solve (hp_small.hip): LDS bytes with nbuf
// spectral buffers (-1: no kernel for these lengths) and the launch
int small2d_lds_bytes(int L0, int L1, int prec, int nbuf);
hipError_t launch_small2d(const PassArgs& a, int prec, hipStream_t s);
int r2r_tile(int prec);
int r2r_lds_bytes(int fast, int L, int n, int prec);
// Dynamic LDS bytes of a wavefront-FFT pass; 0 if the pass is not available.
int fast_lds_bytes(int fast, int L, int P, int K2, int prec, int dbl, int pad);
int fast_emit_dbl(int fast, int prec);
// Pencils per workgroup of the wavefront-FFT passes.
int fast_tile(int fast, int L, int prec);
// Tile widths a wavefront-FFT pass is built for.
bool fast_tile_ok(int fast, int L, int P, int prec);

// Launch one pass over `grid_y` independent field groups.
hipError_t launch_pass(const PassArgs& a, int prec, int grid_y, hipStream_t s);
// Free-space kernel of the plan (Section 2.5.2 readings) in `dim` = 1, 2 or
// 3 dimensions: Gaussian order `kind` = 2, 4, ..., 10 of width sigma, or
// `kind` = 0, the spectral cutoff at kc with its integral (Si in 1D / 3D,
// F(x) = int_0^x (1 - J0(t)) / t dt in 2D) tabulated at j si_step, j < si_n,
// and an 8-point Gauss-Legendre rule (nodes gl_x, weights gl_w on [-1, 1])
// for the rest.
struct GreenEval {
  int kind;
  int dim;
  double sigma;
  double kc;
  const double* si;
  double si_step;
  int si_n;
  double gl_x[8], gl_w[8];
};
// Evaluate scale * G on the doubled grid (FP64, real, [M0][M1][M2]) at the
// mirrored distances.
hipError_t launch_green_eval(double* g, const int M[3], const double h[3], const GreenEval& ge,
                             double scale, hipStream_t s);
// Keep the real part of an FP64 half spectrum [M0][M1][M2/2+1] (complex) on the
// octant, scaled, as T, stored [M2/2+1][M1/2+1][M0/2+1] (axis 0 contiguous).
// Rows of the free-axis Green's spectrum of a semi-unbounded plan: out[m + K
// (i1 + n1 i2)], K = M / 2 + 1, is scale times the DFT bin m of the 1D
// Helmholtz kernel sampled on the doubled axis (spacing h, M points, mirrored)
// for kappa^2 = -(lam1[i1] + lam2[i2]) (lam2 may be null, n2 = 1).  odd: the
// kernel's derivative instead (odd samples, 0 at distances 0 and n h), whose
// bin m is i times the stored value.
hipError_t launch_semi_green(void* out, const double* lam1, int n1, const double* lam2, int n2,
                             int M, double h, double scale, int odd, int prec, hipStream_t s);
hipError_t launch_octant(const double* spec, const int M[3], double scale, void* out,
                         int prec, hipStream_t s);
// Write the boundary nodes of the REGULAR Dirichlet axes (bit a of `axes`)
// of an output [N0][N1][N2] from face arrays (node with several faces:
// highest axis wins).
hipError_t launch_dirichlet_fill(void* out, const int N[3], int ndim, int axes, const void* face[3][2],
                                 int prec, hipStream_t s);
// Consecutive tiles of one pass of the batched persistent solve.  `dep` is the global
// index of the pass that must be complete first (-1: none) and `need` its tile
// count; items are ordered so that every dependency has lower item indices.
struct BatchItem {
  int pass;
  int tile;   // first tile of the item
  int ntile;  // consecutive tiles of the pass in the item
  int dep;    // pass whose tiles must all be done first (-1: none)
  int need;   // tile count of that pass
};

// Zero mode of a periodic / Neumann source: per-block partial sums (nb blocks,
// FP64) of prod_a w_a(i_a) (f(i) + boundary terms of `a`) over the unknowns
// n[0] x n[1] x n[2] (row-major), w_a = 1/2 at the two ends of an axis with
// trap[a] set (DCT-I), else 1.
hipError_t launch_zero_mode(const PassArgs& a, const void* f, const int n[3], const int trap[3],
                            double* partial, int nb, int prec, hipStream_t s);
// Plain streaming copy of `bytes` (16-byte accesses; src and dst 16-byte aligned).
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
// Allocation-free form of the same query: the partial sums of component c
// (kZeroModeBlocks of them) go to a static per-device scratch array, and a
// second kernel writes out[c] = (their sum in block order) / W[c] (0 where
// W[c] = 0) to caller-owned device memory.  Stream-ordered, no host
// synchronisation, no allocation; concurrent calls on one device share the
// scratch array and race.
constexpr int kZeroModeBlocks = 256;
constexpr int kZeroModeMaxComp = 3;
hipError_t launch_zero_mode_noalloc(const PassArgs* a, const void* const* f, int ncomp,
                                    const int n[3], const int trap[3], const double* W,
                                    double* out, int prec, hipStream_t s);
// Persistent batched solve: counters[0] is the work-queue head, counters[1 + i]
// the completed tiles of pass i (zeroed by the launch itself); err[0] is set
// to 1 if a dependency wait exceeds its spin limit (the item is then skipped).
hipError_t launch_batched(const PassArgs* passes, const BatchItem* items, int nitems,
                          unsigned* counters, int ncounters, int* err, int grid, int lds,
                          int prec, int big, hipStream_t s);
// Batched persistent solve on the wavefront kernels (FP32, transform lengths
// 64, 96, 128, 192, 256; hp_bounded.hip).  Passes carry fast = FAST_R2R_C /
// FAST_R2R_S / FAST_R2R_SW, the wavefront twiddles and P = 32; xf is the
// forward type of the batch (DCT-II, DST-II or DCT-I; the backward type is
// its Table 1 partner).  Tiles: batched_wf_tiles per pass; a strided item
// should hold a multiple of batched_wf_group tiles (one per group of
// wavefronts of the workgroup).  LDS: the largest batched_wf_lds of its passes.
bool batched_wf_length(int L);
int batched_wf_lds(int fast, int L);
int batched_wf_tiles(const PassArgs& a);
int batched_wf_group(const PassArgs& a);
int batched_wf_blocks_per_cu(int xf, int lds);
hipError_t launch_batched_wf(int xf, const PassArgs* passes, const BatchItem* items, int nitems,
                             unsigned* counters, int ncounters, int* err, int grid, int lds,
                             hipStream_t s);
// The same tile bodies as one launch per pass level, transform length and
// pass kind (no queue, no waits): group k runs items [first, first + count),
// all of one level, one length L and one kind (0 / 1 contiguous pass of the
// forward / backward type, 2 / 3 strided pass of the forward / backward type,
// 4 sandwich), one workgroup each with lds bytes of LDS, in group order;
// err[0] is cleared (there is no wait to fail).
// One launch of the level form: items [first, first + count) of one pass
// level (`level`), all of transform length L and pass kind `kind`.
struct BatchGroup {
  int first, count, L, kind, lds, level;
};
// The launch of one group (its items' err flag: err, may be null).
hipError_t launch_batched_group(int xf, const PassArgs* passes, const BatchItem* items,
                                const BatchGroup& g, int* err, hipStream_t s);
// Resident workgroups per CU of the persistent kernel with `lds` bytes of LDS.
int batched_blocks_per_cu(int lds, int prec, int big);
}  // namespace hp
