// C-ABI of the spectral Poisson solver: descriptor validation, plans, passes.
//
// A plan follows the initialisation steps of Section 3.2.1 (grid setup, data
// setup, Green's function / eigenvalues, derivative operators) and a solve the
// execution steps of Section 3.2.2 (set input, forward transform, convolution
// with spectral derivative, backward transform, get output).  Every transform
// is a sequence of pencil passes (hp_kernels.hip); the multiply and derivative
// are fused into the pass of the last forward axis.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "hp_plan.hpp"

using namespace hp;

namespace {

thread_local std::string g_create_error;

}  // namespace

namespace {

const char* kStatusText[] = {"ok", "invalid argument", "unsupported", "out of memory",
                             "device error", "bad call order"};

hp_status fail(hp_plan p, hp_status s, const std::string& msg) {
  if (p) p->err = msg;
  else g_create_error = msg;
  return s;
}

hp_status dev_alloc(hp_plan p, size_t bytes, void** out) {
  *out = nullptr;
  if (bytes == 0) bytes = 16;
  if (p->fail_alloc_at >= 0 && p->alloc_count++ == p->fail_alloc_at)
    return fail(p, HP_E_NOMEM, "injected allocation failure");
  if (hipMalloc(out, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *out = nullptr;
    return fail(p, HP_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  p->allocs.push_back(*out);
  p->ws_bytes += bytes;
  return HP_OK;
}

#define HP_TRY(expr)                      \
  do {                                    \
    hp_status _s = (expr);                \
    if (_s != HP_OK) return _s;           \
  } while (0)
#define HP_HIP(p, expr)                                                          \
  do {                                                                           \
    hipError_t _e = (expr);                                                      \
    if (_e != hipSuccess)                                                        \
      return fail((p), HP_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// ------------------------------------------------------------ geometry
int unknowns(int bc, int grid, int nc) {
  switch (bc) {
    case HP_DIRICHLET: return grid == HP_REGULAR ? nc - 1 : nc;
    case HP_NEUMANN: return grid == HP_REGULAR ? nc + 1 : nc;
    case HP_UNBOUNDED: return grid == HP_REGULAR ? nc + 1 : nc;
    default: return nc;
  }
}

int outputs(int bc, int grid, int nc) {
  if (bc == HP_DIRICHLET && grid == HP_REGULAR) return nc + 1;
  return unknowns(bc, grid, nc);
}

// Condition of axis a (the descriptor's, or its per-axis entry for HP_MIXED).
int axis_bc(const hp_desc& d, int a) { return d.bc == HP_MIXED ? d.bc_axis[a] : d.bc; }
// Plans solved by the real-to-real passes: Dirichlet, Neumann and mixed.
bool r2r_plan(const hp_desc& d) {
  return d.bc == HP_DIRICHLET || d.bc == HP_NEUMANN || d.bc == HP_MIXED;
}
// A k = 0 eigenvalue sum of zero (periodic and Neumann on every axis).
bool has_zero_mode(const hp_desc& d) {
  for (int a = 0; a < d.ndim; ++a)
    if (axis_bc(d, a) != HP_PERIODIC && axis_bc(d, a) != HP_NEUMANN) return false;
  return true;
}
// Bit a set: axis a is a REGULAR Dirichlet axis (output carries its boundary nodes).
int dreg_axes(const hp_desc& d) {
  int m = 0;
  for (int a = 0; a < d.ndim; ++a)
    if (axis_bc(d, a) == HP_DIRICHLET && d.grid == HP_REGULAR) m |= 1 << a;
  return m;
}

// Forward / backward transform of Table 1 and the FFT length they need (a
// periodic axis of a mixed plan: the Hartley transform, its own inverse up to n).
void r2r_ops(int bc, int grid, int n, int* xf, int* xb, int* L, double* c) {
  if (bc == HP_PERIODIC) { *xf = X_DHT; *xb = X_DHT; *L = n; *c = (double)n; }
  else if (bc == HP_DIRICHLET && grid == HP_REGULAR) { *xf = X_DST1; *xb = X_DST1; *L = 2 * (n + 1); *c = 2.0 * (n + 1); }
  else if (bc == HP_DIRICHLET) { *xf = X_DST2; *xb = X_DST3; *L = 2 * n; *c = 2.0 * n; }
  else if (grid == HP_REGULAR) { *xf = X_DCT1; *xb = X_DCT1; *L = 2 * (n - 1); *c = 2.0 * (n - 1); }
  else { *xf = X_DCT2; *xb = X_DCT3; *L = 2 * n; *c = 2.0 * n; }
}

bool factorize(int L, int* radix, int* nstage) {
  if (L < 1) return false;
  int s = 0, r = L;
  while (r > 1) {
    int f = 0;
    if (r % 8 == 0) f = 8;
    else if (r % 4 == 0) f = 4;
    else if (r % 2 == 0) f = 2;
    else if (r % 3 == 0) f = 3;
    else if (r % 5 == 0) f = 5;
    else {
      // the smallest prime factor (> 5): a direct prime-radix stage
      f = 7;
      while (r % f != 0 && (long long)f * f <= r) f += 2;
      if (r % f != 0) f = r;
    }
    if (s >= kMaxStages) return false;
    radix[s++] = f;
    r /= f;
  }
  *nstage = s;
  return true;
}

// Complex elements per thread of a general-kernel FFT stage (PassArgs.big).
int maxe(int prec, int big) { return (big ? 32 : 16) / (prec == 0 ? 1 : 2); }

// Pick the tile width P (power of two) for a pass; returns 0 if nothing fits.
// lds(P) gives the LDS bytes, nfft(P) the transforms per FFT call.
template <class F1, class F2>
int choose_P(int want, int minP, int Np, int L, int prec, int big, F1 lds, F2 nfft, int* lds_out) {
  int cap = 1;
  while (cap < Np) cap <<= 1;
  int P = want;
  if (P > cap) P = cap < minP ? minP : cap;
  const int budgets[2] = {64 * 1024, 160 * 1024};
  for (int b = 0; b < 2; ++b) {
    for (int q = P; q >= minP; q >>= 1) {
      if ((long long)nfft(q) * L <= (long long)maxe(prec, big) * kThreads && lds(q) <= budgets[b]) {
        *lds_out = (int)lds(q);
        return q;
      }
    }
  }
  return 0;
}

// ---------------------------------------------------------- validation
hp_status validate(const hp_desc* d) {
  if (!d) return fail(nullptr, HP_E_ARG, "null descriptor");
  if (d->ndim < 1 || d->ndim > 3) return fail(nullptr, HP_E_ARG, "ndim must be 1, 2 or 3");
  if (d->ncomp != 1 && d->ncomp != 3) return fail(nullptr, HP_E_ARG, "ncomp must be 1 or 3");
  if (d->ncomp == 3 && d->ndim != 3) return fail(nullptr, HP_E_ARG, "vector fields need ndim 3");
  if (d->bc < 0 || d->bc > 4) return fail(nullptr, HP_E_ARG, "bad bc");
  if (d->bc == HP_MIXED) {
    int nfree = 0;
    for (int a = 0; a < d->ndim; ++a) {
      if (d->bc_axis[a] == HP_UNBOUNDED) { ++nfree; continue; }
      if (d->bc_axis[a] != HP_PERIODIC && d->bc_axis[a] != HP_DIRICHLET && d->bc_axis[a] != HP_NEUMANN)
        return fail(nullptr, HP_E_ARG, "mixed plans take a periodic, Dirichlet, Neumann or free axis each");
    }
    if (nfree == d->ndim) return fail(nullptr, HP_E_ARG, "a plan that is free on every axis is HP_UNBOUNDED");
    if (nfree > 1) return fail(nullptr, HP_E_UNSUPPORTED, "semi-unbounded plans take one free axis");
    // derivatives of a semi-unbounded solve: first derivatives of homogeneous
    // problems (the free axis's closure for boundary-value differences and
    // a second-derivative series are not defined here)
    if (nfree && d->diff == HP_D_NABLA)
      return fail(nullptr, HP_E_UNSUPPORTED, "semi-unbounded plans take no NABLA output");
    if (nfree && d->diff != HP_D_NONE && d->inhomogeneous)
      return fail(nullptr, HP_E_UNSUPPORTED, "semi-unbounded derivatives need homogeneous boundary values");
  }
  if (d->grid < 0 || d->grid > 1) return fail(nullptr, HP_E_ARG, "bad grid");
  if (d->kernel < 0 || d->kernel > HP_G_SPECTRAL) return fail(nullptr, HP_E_ARG, "bad kernel");
  if (d->diff < 0 || d->diff > HP_D_NABLA) return fail(nullptr, HP_E_ARG, "bad diff");
  if (d->prec < 0 || d->prec > 1) return fail(nullptr, HP_E_ARG, "bad prec");
  if (d->reg_sigma_cells < 0.0 || !std::isfinite(d->reg_sigma_cells))
    return fail(nullptr, HP_E_ARG, "bad reg_sigma_cells");
  for (int a = 0; a < d->ndim; ++a) {
    if (d->nc[a] < 1 || d->nc[a] > (1 << 20)) return fail(nullptr, HP_E_ARG, "nc out of range");
    if (!(d->hi[a] > d->lo[a]) || !std::isfinite(d->lo[a]) || !std::isfinite(d->hi[a]))
      return fail(nullptr, HP_E_ARG, "need lo < hi on every axis");
    const int n = unknowns(axis_bc(*d, a), d->grid, (int)d->nc[a]);
    if (n < 1) return fail(nullptr, HP_E_ARG, "too few cells for this BC and grid");
    if (axis_bc(*d, a) == HP_NEUMANN && d->grid == HP_REGULAR && n < 2)
      return fail(nullptr, HP_E_ARG, "too few cells for this BC and grid");
  }
  const bool unb = d->bc == HP_UNBOUNDED;
  if (unb && d->kernel < HP_G_GAUSS2)
    return fail(nullptr, HP_E_ARG, "unbounded plans take a Green's kernel (HP_G_GAUSS2 .. HP_G_SPECTRAL)");
  if (!unb && d->kernel >= HP_G_GAUSS2)
    return fail(nullptr, HP_E_ARG, "bounded plans take PS or FD2 eigenvalues");
  if (d->inhomogeneous) {
    bool faces = false;
    for (int a = 0; a < d->ndim; ++a)
      faces = faces || axis_bc(*d, a) == HP_DIRICHLET || axis_bc(*d, a) == HP_NEUMANN;
    if (!r2r_plan(*d) || !faces)
      return fail(nullptr, HP_E_ARG, "boundary values need a Dirichlet or Neumann BC");
    if (d->kernel != HP_OP_FD2)
      return fail(nullptr, HP_E_UNSUPPORTED, "inhomogeneous BCs need FD2 eigenvalues");
  }
  if (d->diff == HP_D_CURL && !((d->ncomp == 3 && d->ndim == 3) || (d->ncomp == 1 && d->ndim == 2)))
    return fail(nullptr, HP_E_ARG, "curl needs a 3-component 3D field or a 2D scalar");
  if (d->diff == HP_D_DIV && (d->ncomp != 3 || d->ndim != 3))
    return fail(nullptr, HP_E_ARG, "div needs a 3-component 3D field");
  if (d->diff == HP_D_GRAD && d->ncomp != 1)
    return fail(nullptr, HP_E_ARG, "grad is for scalar fields");
  if (d->diff != HP_D_NONE && r2r_plan(*d)) {
    // with boundary values the first derivatives are FD2 differences (the
    // series of the unknowns does not carry g); no second derivatives
    if (d->inhomogeneous && d->diff == HP_D_NABLA)
      return fail(nullptr, HP_E_UNSUPPORTED,
                  "Dirichlet/Neumann NABLA needs homogeneous boundary values");
    for (int a = 0; a < d->ndim; ++a)
      if (axis_bc(*d, a) == HP_NEUMANN && d->grid == HP_REGULAR && d->nc[a] < 2)
        return fail(nullptr, HP_E_ARG, "Neumann regular derivatives need 2 cells per axis");
  }
  // any transform length whose radix stages (2, 3, 4, 5, 8 and primes) number at
  // most kMaxStages, up to the largest tile of one pencil
  for (int a = 0; a < d->ndim; ++a) {
    const int n = unknowns(axis_bc(*d, a), d->grid, (int)d->nc[a]);
    int L = n, xf, xb, rad[kMaxStages], ns;
    double c;
    if (r2r_plan(*d)) r2r_ops(axis_bc(*d, a), d->grid, n, &xf, &xb, &L, &c);
    if (unb || axis_bc(*d, a) == HP_UNBOUNDED) L = 2 * n;
    if (!factorize(L, rad, &ns))
      return fail(nullptr, HP_E_UNSUPPORTED,
                  "transform length " + std::to_string(L) + " needs too many radix stages");
    if ((long long)L > (long long)(d->prec == 0 ? 32 : 16) * kMaxLenThreads)
      return fail(nullptr, HP_E_UNSUPPORTED, "transform length too large");
    // the Green's function of free space is transformed in FP64 at plan time
    if (unb && (long long)L > 16LL * kMaxLenThreads)
      return fail(nullptr, HP_E_UNSUPPORTED, "doubled free-space length above 4096");
  }
  return HP_OK;
}

// ----------------------------------------------------------- tables
hp_status twiddles(hp_plan p, int L, const void** out) {
  auto it = p->tw.find(L);
  if (it != p->tw.end()) { *out = it->second; return HP_OK; }
  std::vector<double> w(2 * (size_t)L);
  for (int m = 0; m < L; ++m) {
    const double ang = 2.0 * M_PI * (double)m / (double)L;
    w[2 * m] = std::cos(ang);
    w[2 * m + 1] = -std::sin(ang);
  }
  void* d;
  HP_TRY(dev_alloc(p, (size_t)L * 2 * p->es, &d));
  if (p->prec == 0) {
    std::vector<float> f(w.begin(), w.end());
    HP_HIP(p, hipMemcpy(d, f.data(), f.size() * 4, hipMemcpyHostToDevice));
  } else {
    HP_HIP(p, hipMemcpy(d, w.data(), w.size() * 8, hipMemcpyHostToDevice));
  }
  p->tw[L] = d;
  *out = d;
  return HP_OK;
}

// Twiddles of the wavefront FFT of length L (wf_r0), per stage after the
// first: stage 1 (radix G <= 8 after R0, the last one; after R0 = 12 radix
// 4; else radix 8) then stage 2 (radix G/4 after 4 R0, or G/8 after 8 R0),
// each stored [t - 1][k] = W_{NS R}^{t k}, so that the lanes of a wavefront
// read consecutive entries.  L entries are allocated (the
// kernels copy L entries to LDS); unused ones are zero.
hp_status fast_twiddles(hp_plan p, int L, const void** out) {
  auto it = p->ftw.find(L);
  if (it != p->ftw.end()) { *out = it->second; return HP_OK; }
  const int R0 = wf_r0(L);
  if (R0 <= 0) return fail(p, HP_E_UNSUPPORTED, "no wavefront FFT of length " + std::to_string(L));
  const int G = L / R0;
  std::vector<double> w(2 * (size_t)L, 0.0);
  size_t off = 0;
  auto stage = [&](int NS, int R) {
    const long long N = (long long)NS * R;
    for (int t = 1; t < R; ++t)
      for (int k = 0; k < NS; ++k) {
        const double ang = 2.0 * M_PI * (double)(((long long)t * k) % N) / (double)N;
        w[2 * (off + (size_t)(t - 1) * NS + k)] = std::cos(ang);
        w[2 * (off + (size_t)(t - 1) * NS + k) + 1] = -std::sin(ang);
      }
    off += (size_t)(R - 1) * NS;
  };
  if (G <= 8 && R0 % G == 0) {
    stage(R0, G);
  } else if (R0 % 3 == 0) {
    stage(R0, 4);
    stage(4 * R0, G / 4);
  } else {
    stage(R0, 8);
    stage(8 * R0, G / 8);
  }
  if (off > (size_t)L) return fail(p, HP_E_UNSUPPORTED, "wavefront FFT twiddle table overflow");
  void* d;
  HP_TRY(dev_alloc(p, (size_t)L * 2 * p->es, &d));
  if (p->prec == 0) {
    std::vector<float> f(w.begin(), w.end());
    HP_HIP(p, hipMemcpy(d, f.data(), f.size() * 4, hipMemcpyHostToDevice));
  } else {
    HP_HIP(p, hipMemcpy(d, w.data(), w.size() * 8, hipMemcpyHostToDevice));
  }
  p->ftw[L] = d;
  *out = d;
  return HP_OK;
}

hp_status quarter(hp_plan p, int n, const void** out) {
  auto it = p->qtw.find(n);
  if (it != p->qtw.end()) { *out = it->second; return HP_OK; }
  std::vector<double> w(2 * (size_t)n);
  for (int j = 0; j < n; ++j) {
    const double ang = M_PI * (double)j / (2.0 * n);
    w[2 * j] = std::cos(ang);
    w[2 * j + 1] = -std::sin(ang);
  }
  void* d;
  HP_TRY(dev_alloc(p, (size_t)n * 2 * p->es, &d));
  if (p->prec == 0) {
    std::vector<float> f(w.begin(), w.end());
    HP_HIP(p, hipMemcpy(d, f.data(), f.size() * 4, hipMemcpyHostToDevice));
  } else {
    HP_HIP(p, hipMemcpy(d, w.data(), w.size() * 8, hipMemcpyHostToDevice));
  }
  p->qtw[n] = d;
  *out = d;
  return HP_OK;
}

hp_status upload(hp_plan p, const std::vector<double>& v, bool as_T, void** out) {
  const size_t es = as_T ? p->es : 8;
  HP_TRY(dev_alloc(p, v.size() * es, out));
  if (!as_T || p->prec == 1) {
    HP_HIP(p, hipMemcpy(*out, v.data(), v.size() * 8, hipMemcpyHostToDevice));
  } else {
    std::vector<float> f(v.begin(), v.end());
    HP_HIP(p, hipMemcpy(*out, f.data(), f.size() * 4, hipMemcpyHostToDevice));
  }
  return HP_OK;
}

// Table 1 eigenvalues, k = 0 .. n-1 (N of the table is n).
std::vector<double> eigen(int bc, int grid, int op, int n, double L, double h) {
  std::vector<double> v(n);
  for (int k = 0; k < n; ++k) {
    double e = 0.0;
    if (op == HP_OP_PS) {
      if (bc == HP_DIRICHLET) e = -std::pow(M_PI * (k + 1.0) / L, 2);
      else if (bc == HP_NEUMANN) e = -std::pow(M_PI * k / L, 2);
      else {
        const double kk = (k < n / 2.0) ? k : n - k;
        e = -std::pow(2.0 * M_PI * kk / L, 2);
      }
    } else {
      double s;
      if (bc == HP_DIRICHLET && grid == HP_REGULAR) s = std::sin(M_PI * (k + 1.0) / (2.0 * (n + 1)));
      else if (bc == HP_DIRICHLET) s = std::sin(M_PI * (k + 1.0) / (2.0 * n));
      else if (bc == HP_NEUMANN && grid == HP_REGULAR) s = std::sin(M_PI * k / (2.0 * (n - 1)));
      else if (bc == HP_NEUMANN) s = std::sin(M_PI * k / (2.0 * n));
      else s = std::sin(M_PI * k / n);
      e = -4.0 / (h * h) * s * s;
    }
    v[k] = e;
  }
  return v;
}

// Angular wavenumbers 2 pi m~ / (N h) over N points (m~ in (-N/2, N/2)),
// zero at the Nyquist index N/2.
std::vector<double> wavenumbers(int N, double h, int count) {
  std::vector<double> k(count);
  for (int m = 0; m < count; ++m) {
    double mm = (2 * m < N) ? m : m - N;
    if (2 * m == N) mm = 0.0;
    k[m] = 2.0 * M_PI * mm / (N * h);
  }
  return k;
}

// ----------------------------------------------------------- Green's spectrum
// Nodes and weights of 8-point Gauss-Legendre quadrature on [-1, 1]: the roots
// of the Legendre polynomial P_8 by Newton's method from the Chebyshev-like
// first guesses cos(pi (i + 3/4) / (8 + 1/2)), weights 2 / ((1 - x^2) P_8'(x)^2).
void gauss_legendre8(double* x, double* w) {
  const int n = 8;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;  // P_0, P_1; recurrence (k+1) P_{k+1} = (2k+1) z P_k - k P_{k-1}
      for (int k = 1; k < n; ++k) {
        const double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1);
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 1; k < n; ++k) {
      const double p2 = ((2 * k + 1) * z * p1 - k * p0) / (k + 1);
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// int_0^(j step) g(t) dt, j < n, for a smooth g: accumulated interval by
// interval (four 8-point Gauss-Legendre panels per interval, compensated sum).
// g(t) = sin(t) / t gives Si; g(t) = (1 - J0(t)) / t the 2D spectral kernel's F.
template <class G>
std::vector<double> integral_table(int n, double step, const double* gx, const double* gw, G g) {
  std::vector<double> tab(n, 0.0);
  double sum = 0.0, comp = 0.0;
  for (int j = 1; j < n; ++j) {
    for (int q = 0; q < 4; ++q) {
      const double a = (j - 1) * step + q * step / 4, b = a + step / 4;
      const double mid = 0.5 * (a + b), half = 0.5 * (b - a);
      double acc = 0.0;
      for (int i = 0; i < 8; ++i) {
        acc += gw[i] * g(mid + half * gx[i]);
      }
      const double y = half * acc - comp;
      const double t2 = sum + y;
      comp = (t2 - sum) - y;
      sum = t2;
    }
    tab[j] = sum;
  }
  return tab;
}

hp_status green_spectrum(hp_plan p, Problem& P) {
  const int M[3] = {P.M[0], P.M[1], P.M[2]};
  const int K2 = M[2] / 2 + 1;
  // (axes beyond the problem's dimension are unit placeholders)
  double hmax = 0.0;
  for (int a = 0; a < P.nd; ++a) hmax = std::max(hmax, P.h[a]);
  const double sigma = (P.d.reg_sigma_cells > 0 ? P.d.reg_sigma_cells : 2.0) * hmax;
  const size_t nreal = (size_t)M[0] * M[1] * M[2];
  const size_t ncplx = (size_t)M[0] * M[1] * K2;
  void *g = nullptr, *spec = nullptr;
  if (hipMalloc(&g, nreal * 8) != hipSuccess) { (void)hipGetLastError(); return fail(p, HP_E_NOMEM, "Green's grid allocation failed"); }
  if (hipMalloc(&spec, ncplx * 16) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(g);
    return fail(p, HP_E_NOMEM, "Green's spectrum allocation failed");
  }
  hp_status st = HP_OK;
  GreenEval ge{};
  ge.kind = P.d.kernel == HP_G_SPECTRAL ? 0 : 2 * (P.d.kernel - HP_G_GAUSS2 + 1);
  ge.dim = P.nd;
  ge.sigma = sigma;
  ge.kc = M_PI / hmax;
  gauss_legendre8(ge.gl_x, ge.gl_w);
  void* si_dev = nullptr;
  if (ge.kind == 0) {
    // Si (1D, 3D) or F (2D) on a table of step 1/2 up to past k_c times the
    // largest distance
    double rmax2 = 0.0;
    for (int a = 0; a < 3; ++a) rmax2 += std::pow(0.5 * M[a] * P.h[a], 2);
    ge.si_step = 0.5;
    ge.si_n = (int)std::ceil(ge.kc * std::sqrt(rmax2) / ge.si_step) + 2;
    const std::vector<double> tab =
        ge.dim == 2 ? integral_table(ge.si_n, ge.si_step, ge.gl_x, ge.gl_w,
                                     [](double t) { return (1.0 - ::j0(t)) / t; })
                    : integral_table(ge.si_n, ge.si_step, ge.gl_x, ge.gl_w,
                                     [](double t) { return std::sin(t) / t; });
    if (hipMalloc(&si_dev, tab.size() * 8) != hipSuccess ||
        hipMemcpy(si_dev, tab.data(), tab.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      if (si_dev) (void)hipFree(si_dev);
      (void)hipFree(g);
      (void)hipFree(spec);
      return fail(p, HP_E_NOMEM, "sine-integral table allocation failed");
    }
    ge.si = (const double*)si_dev;
  }
  auto run = [&]() -> hp_status {
    HP_HIP(p, launch_green_eval((double*)g, M, P.h, ge, P.h[0] * P.h[1] * P.h[2], p->stream));
    // FP64 forward transform with the general passes (a temporary FP64 view)
    const int saved_prec = p->prec;
    const size_t saved_es = p->es;
    std::map<int, void*> saved_tw;
    saved_tw.swap(p->tw);
    p->prec = 1;
    p->es = 8;
    auto restore = [&]() {
      p->prec = saved_prec;
      p->es = saved_es;
      p->tw.swap(saved_tw);
      for (auto& kv : saved_tw) (void)kv;  // FP64 tables stay owned by the plan
    };
    for (int axis = 2; axis >= 0; --axis) {
      PassArgs a{};
      a.kind = PK_ONEWAY;
      a.xf = axis == 2 ? X_R2C : X_C2C_F;
      a.L = M[axis];
      a.n = M[axis];
      a.nin = M[axis];
      a.nout = axis == 2 ? K2 : M[axis];
      if (!factorize(a.L, a.radix, &a.nstage)) { restore(); return fail(p, HP_E_UNSUPPORTED, "Green's length"); }
      const void* tw;
      hp_status s = twiddles(p, a.L, &tw);
      if (s != HP_OK) { restore(); return s; }
      a.tw = tw;
      a.ax_j = a.ax_p = a.ax_o = -1;
      a.n_in = a.n_out = 1;
      if (axis == 2) {
        a.in[0] = g;
        a.out[0] = spec;
        a.in_sj = 1; a.in_sp = M[2]; a.in_so = (long long)M[1] * M[2];
        a.out_sj = 1; a.out_sp = K2; a.out_so = (long long)M[1] * K2;
        a.Np = M[1]; a.No = M[0];
        a.in_jfast = a.out_jfast = 1;
        int lds;
        a.big = 1;
        a.P = choose_P(16, 2, a.Np, a.L, 1, 1,
                       [&](int q) { return (long long)(q / 2) * a.L * 16 + (long long)q * a.nin * 8; },
                       [&](int q) { return q / 2; }, &lds);
        a.lds_bytes = lds;
      } else {
        a.in[0] = spec;
        a.out[0] = spec;
        a.in_sj = a.out_sj = axis == 1 ? K2 : (long long)M[1] * K2;
        a.in_sp = a.out_sp = 1;
        a.in_so = a.out_so = axis == 1 ? (long long)M[1] * K2 : K2;
        a.Np = K2; a.No = axis == 1 ? M[0] : M[1];
        a.in_jfast = a.out_jfast = 0;
        int lds;
        a.big = 1;
        a.P = choose_P(8, 1, a.Np, a.L, 1, 1, [&](int q) { return (long long)q * a.L * 16; },
                       [&](int q) { return q; }, &lds);
        a.lds_bytes = lds;
      }
      if (a.P == 0) { restore(); return fail(p, HP_E_UNSUPPORTED, "Green's transform does not fit"); }
      hipError_t e = launch_pass(a, 1, 1, p->stream);
      if (e != hipSuccess) { restore(); return fail(p, HP_E_DEVICE, std::string("Green's pass: ") + hipGetErrorString(e)); }
    }
    restore();
    const size_t oct = (size_t)(M[0] / 2 + 1) * (M[1] / 2 + 1) * K2;
    HP_TRY(dev_alloc(p, oct * p->es, &P.green));
    HP_HIP(p, launch_octant((const double*)spec, M, 1.0 / ((double)M[0] * M[1] * M[2]), P.green,
                            p->prec, p->stream));
    P.g_s[0] = 1;
    P.g_s[1] = M[0] / 2 + 1;
    P.g_s[2] = (long long)(M[0] / 2 + 1) * (M[1] / 2 + 1);
    HP_HIP(p, hipStreamSynchronize(p->stream));
    return HP_OK;
  };
  st = run();
  (void)hipStreamSynchronize(p->stream);
  (void)hipFree(g);
  (void)hipFree(spec);
  if (si_dev) (void)hipFree(si_dev);
  return st;
}

// ----------------------------------------------------------- plan setup
bool fast_unbounded_ok(hp_plan p, const Problem& P);
size_t count_elems(const int* dims, int nd);

hp_status setup_problem(hp_plan p, Problem& P) {
  const hp_desc& d = P.d;
  P.nd = d.ndim;
  P.ncomp = d.ncomp;
  P.nder = d.diff == HP_D_GRAD    ? d.ndim
           : d.diff == HP_D_CURL  ? (d.ndim == 2 ? 2 : 3)
           : d.diff == HP_D_DIV   ? 1
           : d.diff == HP_D_NABLA ? d.ncomp
                                  : 0;
  for (int a = 0; a < 3; ++a) {
    P.n[a] = P.nout[a] = P.M[a] = 1;
    P.h[a] = P.len[a] = 1.0;
  }
  for (int a = 0; a < P.nd; ++a) {
    P.len[a] = d.hi[a] - d.lo[a];
    P.h[a] = P.len[a] / (double)d.nc[a];
    P.n[a] = unknowns(axis_bc(d, a), d.grid, (int)d.nc[a]);
    P.nout[a] = outputs(axis_bc(d, a), d.grid, (int)d.nc[a]);
    P.M[a] = 2 * P.n[a];
  }
  const size_t es = p->es;
  if (r2r_plan(d)) {
    P.norm = 1.0;
    for (int a = 0; a < P.nd; ++a) {
      if (axis_bc(d, a) == HP_UNBOUNDED) {
        P.free_axis = a;
        P.M[a] = 2 * P.n[a];
        continue;
      }
      int xf, xb, L;
      double c;
      r2r_ops(axis_bc(d, a), d.grid, P.n[a], &xf, &xb, &L, &c);
      P.norm /= c;
      HP_TRY(upload(p, eigen(axis_bc(d, a), d.grid, d.kernel, P.n[a], P.len[a], P.h[a]), false,
                    (void**)&P.lam[a]));
    }
    if (P.free_axis >= 0) {
      // rows of the free axis's Helmholtz Green's spectrum per bounded mode,
      // scaled by the bounded inverse normalisation, 1 / M of the free axis's
      // inverse FFT and its cell length; logical-axis strides g_s
      const int u = P.free_axis, M = P.M[u], K = M / 2 + 1;
      int b[2] = {-1, -1}, nb = 0;
      for (int a = 0; a < P.nd; ++a)
        if (a != u) b[nb++] = a;
      const int n1 = P.n[b[0]], n2 = nb > 1 ? P.n[b[1]] : 1;
      for (int a = 0; a < 3; ++a) P.g_s[a] = 0;
      P.g_s[u] = 1;
      P.g_s[b[0]] = K;
      if (nb > 1) P.g_s[b[1]] = (long long)K * n1;
      HP_TRY(dev_alloc(p, (size_t)K * n1 * n2 * es, &P.green));
      HP_HIP(p, launch_semi_green(P.green, P.lam[b[0]], n1, nb > 1 ? P.lam[b[1]] : nullptr, n2, M,
                                  P.h[u], P.norm * P.h[u] / (double)M, 0, p->prec, p->stream));
      if (P.nder) {  // rows of the kernel's derivative, same layout and scale
        HP_TRY(dev_alloc(p, (size_t)K * n1 * n2 * es, &P.green_odd));
        HP_HIP(p, launch_semi_green(P.green_odd, P.lam[b[0]], n1, nb > 1 ? P.lam[b[1]] : nullptr, n2,
                                    M, P.h[u], P.norm * P.h[u] / (double)M, 1, p->prec, p->stream));
      }
    }
    if (P.nder && P.free_axis < 0) HP_TRY(dev_alloc(p, count_elems(P.nout, P.nd) * es, &P.grad_s));
    // second terms of DIV (d_y psi_y, d_z psi_z) and of the 3D curl, added
    // into the outputs at the end of the solve
    const int ntmp = d.diff == HP_D_DIV ? 2 : (d.diff == HP_D_CURL && P.nd == 3 ? 3 : 0);
    for (int t = 0; t < ntmp; ++t) HP_TRY(dev_alloc(p, count_elems(P.nout, P.nd) * es, &P.dtmp[t]));
  } else if (d.bc == HP_PERIODIC) {
    P.norm = 1.0;
    for (int a = 0; a < P.nd; ++a) {
      P.norm /= P.n[a];
      HP_TRY(upload(p, eigen(d.bc, d.grid, d.kernel, P.n[a], P.len[a], P.h[a]), false, (void**)&P.lam[a]));
      if (P.nder) HP_TRY(upload(p, wavenumbers(P.n[a], P.h[a], P.n[a]), true, &P.kvec[a]));
    }
    const int nf = P.ncomp + P.nder;
    // 3D power-of-two plans: the wavefront passes of the free-space path on
    // undoubled pencils (transform lengths M = n)
    if (!p->batched) {
      for (int a = 0; a < 3; ++a) P.M[a] = P.n[a];
      P.fast_periodic = fast_unbounded_ok(p, P);
      if (!P.fast_periodic)
        for (int a = 0; a < 3; ++a) P.M[a] = 2 * P.n[a];
    }
    if (P.fast_periodic) {
      const size_t K2 = (size_t)P.n[2] / 2 + 1, K2c = (K2 + 15) / 16 * 16;
      P.slabs.assign(1, {0, (int)K2});
      for (int f = 0; f < nf; ++f) {
        void* b;
        HP_TRY(dev_alloc(p, (size_t)P.n[0] * K2c * P.n[1] * 2 * es, &b));
        P.a1.push_back(b);
        HP_TRY(dev_alloc(p, K2 * P.n[1] * (size_t)P.n[0] * 2 * es, &b));
        P.b2.push_back(b);
        HP_TRY(dev_alloc(p, K2 * P.n[1] * (size_t)P.n[0] * 2 * es, &b));
        P.c2.push_back(b);
      }
    } else if (P.nd >= 2) {
      const size_t K = (size_t)P.n[P.nd - 1] / 2 + 1;
      size_t sz = K;
      for (int a = 0; a < P.nd - 1; ++a) sz *= P.n[a];
      for (int f = 0; f < nf; ++f) {
        void* b;
        HP_TRY(dev_alloc(p, sz * 2 * es, &b));
        P.b2.push_back(b);
      }
    }
  } else {
    for (int a = 0; a < 3; ++a) {
      const int cnt = a == 2 ? P.M[2] / 2 + 1 : P.M[a];
      HP_TRY(upload(p, wavenumbers(P.M[a], P.h[a], cnt), true, &P.kvec[a]));
    }
    HP_TRY(green_spectrum(p, P));
    const int nf = P.ncomp + P.nder;
    const size_t K2 = (size_t)P.M[2] / 2 + 1;
    const bool fast = fast_unbounded_ok(p, P);
    // kz slabs of the y / x passes (fast path): B2 and C2 then hold one slab
    P.slabs.clear();
    int sl = 0;
    if (fast) {
      if (const char* e = std::getenv("HP_SLAB")) sl = std::atoi(e);
    }
    if (sl > 0 && sl < (int)K2) {
      for (int k = 0; k < (int)K2; k += sl) P.slabs.push_back({k, std::min(sl, (int)K2 - k)});
      if (P.slabs.size() > 1 && P.slabs.back().second < sl / 2) {
        P.slabs[P.slabs.size() - 2].second += P.slabs.back().second;
        P.slabs.pop_back();
      }
    } else {
      P.slabs.push_back({0, (int)K2});
    }
    size_t kzmax = 0;
    for (auto& s : P.slabs) kzmax = std::max(kzmax, (size_t)s.second);
    // C1 [x][y][kz] rows (fast path) are padded to a multiple of 16 elements,
    // so that the backward y pass writes whole 128-byte lines
    const size_t K2c = fast ? (K2 + 15) / 16 * 16 : K2;
    for (int f = 0; f < nf; ++f) {
      void* b;
      HP_TRY(dev_alloc(p, (size_t)P.n[0] * K2c * P.n[1] * 2 * es, &b));
      P.a1.push_back(b);
      HP_TRY(dev_alloc(p, (fast ? kzmax : K2) * P.M[1] * (size_t)P.n[0] * 2 * es, &b));
      P.b2.push_back(b);
      if (fast) {
        HP_TRY(dev_alloc(p, kzmax * P.M[1] * (size_t)P.n[0] * 2 * es, &b));
        P.c2.push_back(b);
        // with several kz slabs the backward y pass must not write over A1,
        // which later slabs still read: C1 gets its own buffers
        if (P.slabs.size() > 1) {
          HP_TRY(dev_alloc(p, (size_t)P.n[0] * K2c * P.n[1] * 2 * es, &b));
          P.c1.push_back(b);
        }
      }
    }
  }
  return HP_OK;
}

size_t count_elems(const int* dims, int nd) {
  size_t s = 1;
  for (int a = 0; a < nd; ++a) s *= (size_t)dims[a];
  return s;
}

// Output buffers: bound pointers or plan-owned ones.
hp_status ensure_outputs(hp_plan p, Problem& P) {
  const size_t cnt = count_elems(P.nout, P.nd);
  for (int c = 0; c < P.ncomp; ++c)
    if (!P.out[c]) {
      if (!P.own_out[c]) HP_TRY(dev_alloc(p, cnt * p->es, &P.own_out[c]));
      P.out[c] = P.own_out[c];
    }
  for (int c = 0; c < P.nder; ++c)
    if (!P.der[c]) {
      if (!P.own_der[c]) HP_TRY(dev_alloc(p, cnt * p->es, &P.own_der[c]));
      P.der[c] = P.own_der[c];
    }
  return HP_OK;
}

void strides_of(const int* dims, long long* s) {
  s[2] = 1;
  s[1] = dims[2];
  s[0] = (long long)dims[1] * dims[2];
}

// Boundary terms of component `comp` of an inhomogeneous FD2 problem
// (Section 2.4.2 reading): face arrays, their strides over the remaining axes
// (output layout) and the weights added to the unknowns next to each face.
void fill_face_terms(const Problem& P, int comp, PassArgs& a) {
  const hp_desc& d = P.d;
  if (!d.inhomogeneous) return;
  const int nd = P.nd;
  a.face_off = dreg_axes(d);
  for (int ax = 0; ax < nd; ++ax) {
    int rem[2], nr = 0;
    for (int b = 0; b < nd; ++b)
      if (b != ax) rem[nr++] = b;
    a.face_s[ax][0] = a.face_s[ax][1] = 0;
    if (nr == 2) { a.face_s[ax][1] = 1; a.face_s[ax][0] = P.nout[rem[1]]; }
    else if (nr == 1) { a.face_s[ax][0] = 1; }
    const double h = P.h[ax];
    const int bc = axis_bc(d, ax);
    for (int side = 0; side < 2; ++side) {
      a.face[ax][side] = (bc == HP_PERIODIC || bc == HP_UNBOUNDED) ? nullptr : P.face[ax][side][comp];
      double w;
      if (bc == HP_DIRICHLET) w = (d.grid == HP_REGULAR ? -1.0 : -2.0) / (h * h);
      else if (d.grid == HP_REGULAR) w = (side == 0 ? 2.0 : -2.0) / h;
      else w = (side == 0 ? 1.0 : -1.0) / h;
      a.face_w[ax][side] = w;
    }
  }
}

// Sandwich coupling of the descriptor's operator (forward or transposed).
int diff_kind(int dk, bool adjoint) {
  switch (dk) {
    case HP_D_GRAD: return adjoint ? D_ADJ_GRAD : D_GRAD;
    case HP_D_CURL: return adjoint ? D_ADJ_CURL : D_CURL;
    case HP_D_DIV: return adjoint ? D_ADJ_DIV : D_DIV;
    case HP_D_NABLA: return adjoint ? D_ADJ_NABLA : D_NABLA;
    default: return D_NONE;
  }
}

// FNV-1a over the integers that fix a pass's geometry.
unsigned long long tune_hash(const long long* v, int n) {
  unsigned long long h = 1469598103934665603ull;
  for (int i = 0; i < n; ++i) {
    unsigned long long x = (unsigned long long)v[i];
    for (int b = 0; b < 8; ++b) {
      h ^= (x >> (8 * b)) & 0xffu;
      h *= 1099511628211ull;
    }
  }
  return h;
}

// Signature of a general pass from the fields its builder sets before the
// tile is chosen.
unsigned long long general_key(const PassArgs& a, int prec, int want, int minP, int lds_kind) {
  const long long v[] = {0,        prec,      a.kind,    a.xf,      a.xb,      a.L,
                         a.n,      a.nin,     a.nout,    a.Np,      a.No,      a.in_jfast,
                         a.out_jfast, a.in_sj, a.in_sp,  a.in_so,   a.out_sj,  a.out_sp,
                         a.out_so, a.n_in,    a.n_out,   a.diff,    a.mult,    want,
                         minP,     lds_kind};
  return tune_hash(v, (int)(sizeof(v) / sizeof(v[0])));
}

// Fill the FFT fields of a pass for length L; P from the LDS model.  A tuned
// configuration (radix order, tile width, register budget) replaces the
// default when it fits this pass; otherwise the default stands.
hp_status finish_pass_with(hp_plan p, PassArgs& a, int want, int minP, int lds_kind,
                           const Tune* tn) {
  if (tn) {
    a.nstage = tn->nstage;
    for (int s = 0; s < tn->nstage; ++s) a.radix[s] = tn->radix[s];
    want = tn->P;
  } else if (!factorize(a.L, a.radix, &a.nstage)) {
    return fail(p, HP_E_UNSUPPORTED, "length");
  }
  const void* tw;
  HP_TRY(twiddles(p, a.L, &tw));
  a.tw = tw;
  const long long cs = 2 * (long long)p->es, es = p->es;
  int lds = 0;
  auto nfft_pair = [](int q) { return q / 2; };
  auto nfft_one = [](int q) { return q; };
  // the smaller register budget first (more resident waves), the larger one
  // when a tile of this length does not fit it
  for (int big = tn ? tn->big : 0; big < (tn ? tn->big + 1 : 2); ++big) {
    a.big = big;
    switch (lds_kind) {
      case 0:  // one-way complex
        a.P = choose_P(want, minP, a.Np, a.L, p->prec, big, [&](int q) { return (long long)q * a.L * cs; }, nfft_one, &lds);
        break;
      case 1:  // one-way real input (pairs)
        a.P = choose_P(want, 2, a.Np, a.L, p->prec, big,
                       [&](int q) { return (long long)(q / 2) * a.L * cs + (long long)q * a.nin * es; }, nfft_pair, &lds);
        break;
      case 2:  // one-way C2R (pairs, complex staging)
        a.P = choose_P(want, 2, a.Np, a.L, p->prec, big,
                       [&](int q) { return (long long)(q / 2) * a.L * cs + (long long)q * a.nin * cs; }, nfft_pair, &lds);
        break;
      case 3:  // r2r sandwich
        a.P = choose_P(want, 2, a.Np, a.L, p->prec, big,
                       [&](int q) { return (long long)(q / 2) * a.L * cs + (long long)q * a.nin * es; }, nfft_pair, &lds);
        break;
      case 4: {  // c2c sandwich: (nS + 1) complex tiles
        const int nS = diff_is_adjoint(a.diff) ? a.n_out : a.n_in;
        a.P = choose_P(want, minP, a.Np, a.L, p->prec, big,
                       [&](int q) { return (long long)(nS + 1) * q * a.L * cs; }, nfft_one, &lds);
      } break;
      case 5: {  // paired c2c sandwich (1D periodic)
        const int nS = a.n_in;
        a.P = choose_P(want, 2, a.Np, a.L, p->prec, big,
                       [&](int q) {
                         return (long long)nS * (q / 2) * a.L * cs +
                                std::max((long long)(q / 2) * a.L * cs, (long long)q * a.nin * es);
                       },
                       nfft_pair, &lds);
      } break;
    }
    if (a.P > 0) break;
  }
  if (tn && a.P != tn->P) return HP_E_UNSUPPORTED;  // does not fit: caller takes the default
  if (a.P == 0) return fail(p, HP_E_UNSUPPORTED, "pass of length " + std::to_string(a.L) + " does not fit in LDS");
  a.lds_bytes = lds;
  return HP_OK;
}

hp_status finish_pass(hp_plan p, PassArgs& a, int want, int minP, long long lds_per_P_fixed,
                      int lds_kind) {
  (void)lds_per_P_fixed;
  const unsigned long long key = general_key(a, p->prec, want, minP, lds_kind);
  auto it = p->tuned.find(key);
  if (it != p->tuned.end() && it->second.fast == FAST_NONE &&
      radix_ok(a.L, it->second.radix, it->second.nstage)) {
    PassArgs t = a;
    if (finish_pass_with(p, t, want, minP, lds_kind, &it->second) == HP_OK) {
      a = t;
      a.tune_key = key;
      return HP_OK;
    }
  }
  HP_TRY(finish_pass_with(p, a, want, minP, lds_kind, nullptr));
  a.tune_key = key;
  return HP_OK;
}

// --------------------------------------------------------- pass lists
// Wavefront-FFT kernels for the bounded passes (hp_bounded.hip): 2D / 3D
// single plans whose every Dirichlet / Neumann transform length is a power of
// two in [64, 512], or 96 or 192 (the Hartley passes of periodic axes stay on
// the general kernels).
bool bounded_fast_ok(hp_plan p, const Problem& P, const int* L) {
  if (std::getenv("HP_GENERIC") || p->batched || P.nd < 2) return false;
  int bounded = 0;
  for (int a = 0; a < P.nd; ++a) {
    // Hartley (periodic) axes and the free axis of a mixed plan keep the
    // general kernels; the passes along the other axes switch one by one
    // (to_fast_r2r)
    if (axis_bc(P.d, a) == HP_PERIODIC || axis_bc(P.d, a) == HP_UNBOUNDED) continue;
    ++bounded;
    if (L[a] < 64 || L[a] > 512 || wf_r0(L[a]) <= 0) return false;
    for (int k = FAST_R2R_C; k <= FAST_R2R_SW; ++k) {
      const int lds = r2r_lds_bytes(k, L[a], P.n[a], p->prec);
      if (lds <= 0 || lds > 160 * 1024) return false;
    }
  }
  return bounded > 0;
}

// Switch a general bounded pass (same descriptor) to its wavefront kernel.
hp_status to_fast_r2r(hp_plan p, PassArgs& a) {
  if (a.fast == FAST_GRAD_PREP || a.fast == FAST_ADD) return HP_OK;
  // Hartley passes and the free axis's Green's-row sandwich: general kernels
  if (a.xf == X_DHT || (a.kind == PK_SANDWICH && a.xb == X_DHT)) return HP_OK;
  if (a.mult == M_GREEN_ROWS || a.mult == M_GREEN_ROWS_ODD || a.xf == X_PAIR_F) return HP_OK;
  const bool contig = a.kind == PK_ONEWAY && a.in_jfast && a.out_jfast;
  bool faces = false;
  for (int ax = 0; ax < 3; ++ax) faces |= a.face[ax][0] != nullptr || a.face[ax][1] != nullptr;
  if (faces && !contig) return HP_OK;  // boundary terms: contiguous passes only
  const int kind = a.kind == PK_SANDWICH ? FAST_R2R_SW : (contig ? FAST_R2R_C : FAST_R2R_S);
  const int lds = r2r_lds_bytes(kind, a.L, a.n, p->prec);
  if (lds <= 0 || lds > 160 * 1024) return HP_OK;  // stays on the general kernel
  a.fast = kind;
  const void* tw;
  HP_TRY(fast_twiddles(p, a.L, &tw));
  a.tw = tw;
  a.P = r2r_tile(p->prec);
  a.lds_bytes = r2r_lds_bytes(a.fast, a.L, a.n, p->prec);
  return HP_OK;
}

// The derivative terms of every operator on the real-to-real paths: component
// `comp` contributes d psi_comp / d x_axis (axis -1: NABLA) times `sign` to
// slot `dst` (an output, or a temporary added into an output at the end).
// With boundary values the derivatives are differences of psi taken after the
// solve (hp_solve, launch_fd_deriv), not series terms: no terms.
struct DerivTerm {
  int comp, axis;
  void* dst;
  double sign;
};

std::vector<DerivTerm> derivative_terms(const Problem& P) {
  const hp_desc& d = P.d;
  const int nd = P.nd;
  std::vector<DerivTerm> terms;
  switch (d.inhomogeneous ? HP_D_NONE : d.diff) {
    case HP_D_GRAD:
      for (int g = 0; g < nd; ++g) terms.push_back({0, g, P.der[g], 1.0});
      break;
    case HP_D_NABLA:
      for (int c = 0; c < P.ncomp; ++c) terms.push_back({c, -1, P.der[c], 1.0});
      break;
    case HP_D_DIV:  // d_x psi_x into the output, d_y psi_y and d_z psi_z added
      terms.push_back({0, 0, P.der[0], 1.0});
      terms.push_back({1, 1, P.dtmp[0], 1.0});
      terms.push_back({2, 2, P.dtmp[1], 1.0});
      break;
    case HP_D_CURL:
      if (nd == 2) {  // (d_y psi, -d_x psi)
        terms.push_back({0, 1, P.der[0], 1.0});
        terms.push_back({0, 0, P.der[1], -1.0});
      } else {  // u_x = d_y psi_z - d_z psi_y, u_y = d_z psi_x - d_x psi_z, u_z = d_x psi_y - d_y psi_x
        terms.push_back({0, 1, P.dtmp[2], -1.0});
        terms.push_back({0, 2, P.der[1], 1.0});
        terms.push_back({1, 0, P.der[2], 1.0});
        terms.push_back({1, 2, P.dtmp[0], -1.0});
        terms.push_back({2, 0, P.dtmp[1], -1.0});
        terms.push_back({2, 1, P.der[0], 1.0});
      }
      break;
    default:
      break;
  }
  return terms;
}

// DIV / 3D CURL: the second terms added into the outputs (elementwise)
void add_second_terms(const Problem& P, size_t es, std::vector<PassRec>& out) {
  if (P.d.inhomogeneous) return;
  auto add_into = [&](void* dst, const void* t0, const void* t1) {
    PassArgs a{};
    a.ax_j = a.ax_p = a.ax_o = -1;
    a.No = a.Np = 1;
    a.n_in = a.n_out = 1;
    a.fast = FAST_ADD;
    a.out[0] = dst;
    a.in[0] = t0;
    a.in[1] = t1;
    long long cnt = 1;
    for (int b = 0; b < P.nd; ++b) cnt *= P.nout[b];
    a.gp_ext[0] = (int)cnt;
    a.gp_ext[1] = a.gp_ext[2] = 1;
    PassRec r{a, 1};
    r.bytes = (double)cnt * (double)es * (t1 ? 4.0 : 3.0);
    out.push_back(r);
  };
  if (P.d.diff == HP_D_DIV) add_into(P.der[0], P.dtmp[0], P.dtmp[1]);
  if (P.d.diff == HP_D_CURL && P.nd == 3)
    for (int c = 0; c < 3; ++c) add_into(P.der[c], P.dtmp[c], nullptr);
}

hp_status passes_bounded(hp_plan p, Problem& P, std::vector<PassRec>& out) {
  const hp_desc& d = P.d;
  const int nd = P.nd;
  int xf[3], xb[3], L[3];
  double c[3];
  for (int a = 0; a < nd; ++a) r2r_ops(axis_bc(d, a), d.grid, P.n[a], &xf[a], &xb[a], &L[a], &c[a]);
  const size_t first_pass = out.size();
  // work view = the output array (interior for REGULAR Dirichlet)
  int od[3] = {1, 1, 1}, idims[3] = {1, 1, 1};
  for (int a = 0; a < nd; ++a) { od[a] = P.nout[a]; idims[a] = P.n[a]; }
  // logical axis a of an nd-D array maps to storage dim (3 - nd + a)
  int sod[3] = {1, 1, 1}, sid[3] = {1, 1, 1};
  for (int a = 0; a < nd; ++a) { sod[3 - nd + a] = od[a]; sid[3 - nd + a] = idims[a]; }
  long long os3[3], is3[3];
  strides_of(sod, os3);
  strides_of(sid, is3);
  long long ws[3], fs[3];
  for (int a = 0; a < 3; ++a) ws[a] = fs[a] = 0;
  for (int a = 0; a < nd; ++a) { ws[a] = os3[3 - nd + a]; fs[a] = is3[3 - nd + a]; }
  const bool dreg = d.bc == HP_DIRICHLET && d.grid == HP_REGULAR;
  const int dmask = dreg_axes(d);
  long long woff = 0;
  for (int a = 0; a < nd; ++a)
    if ((dmask >> a) & 1) woff += ws[a];
  const size_t es = p->es;
  auto work = [&](int comp) { return (void*)((char*)P.out[comp] + woff * es); };

  auto base = [&]() {
    PassArgs a{};
    a.ax_j = a.ax_p = a.ax_o = -1;
    a.No = 1;
    a.Np = 1;
    a.n_in = a.n_out = 1;
    for (int b = 0; b < 3; ++b) a.nunk[b] = b < nd ? P.n[b] : 0;
    return a;
  };
  auto set_faces = [&](PassArgs& a, int comp) { fill_face_terms(P, comp, a); };
  (void)dreg;
  const int last = nd - 1;
  // Gradient (homogeneous Dirichlet / Neumann).  The passes of psi are
  // unchanged.  d/dx_0: the forward pass along axis 0 is done once more, out
  // of place, so that grad_s holds the source transformed along every axis;
  // a prep pass writes the coefficients of the derivative series (divided by
  // the eigenvalue sum) into the output of d/dx_0, and backward passes along
  // every axis evaluate it, with the transform of the other parity along
  // axis 0.  d/dx_g, g > 0: psi's own array after the sandwich already holds
  // the divided coefficients along axes 1.. (axis 0 physical), so the prep
  // reads it and only the axes 1.. are transformed back.
  auto grad_forward_x = [&](int comp) -> hp_status {
    PassArgs a = base();
    a.kind = PK_ONEWAY;
    a.xf = xf[0];
    a.L = L[0]; a.n = P.n[0]; a.nin = a.nout = P.n[0];
    a.in[0] = nd == 1 ? P.in[comp] : work(comp);
    a.out[0] = (void*)((char*)P.grad_s + woff * es);
    a.ax_j = 0;
    if (nd == 1) {
      a.in_sj = a.out_sj = 1;
      a.in_jfast = a.out_jfast = 1;
    } else {
      a.in_sj = a.out_sj = ws[0];
      a.in_sp = a.out_sp = ws[last];
      a.Np = P.n[last]; a.ax_p = last;
      if (nd == 3) { a.in_so = a.out_so = ws[1]; a.No = P.n[1]; a.ax_o = 1; }
    }
    HP_TRY(finish_pass(p, a, nd == 1 ? 2 : 32, 2, 0, 1));
    const void* q;
    HP_TRY(quarter(p, a.n, &q));
    a.qtw = q;
    out.push_back({a, 1});
    return HP_OK;
  };
  // derivative g from coefficients `src` (the work-view layout) into `dst`,
  // times `sign`; `eigen`: the eigenvalue sum still has to be divided out
  // (source transformed along every axis), else src is psi's array after the
  // sandwich.  `lap`: NABLA instead, the sum over the axes of the second
  // derivatives, which keeps every axis's basis (-w_b^2 per eigenfunction),
  // from the transformed source.
  auto grad_deriv = [&](int g, const void* src, bool eigen, void* dst, double sign,
                        bool lap) -> hp_status {
    const int bcg = axis_bc(d, g);
    const bool dir = bcg == HP_DIRICHLET, reg = d.grid == HP_REGULAR, per = bcg == HP_PERIODIC;
    // active view of the derivative output: extent len[b] from off[b]
    int off[3] = {0, 0, 0}, len[3] = {1, 1, 1};
    for (int b = 0; b < nd; ++b) { off[b] = (dmask >> b) & 1; len[b] = P.n[b]; }
    int xd = 0;
    if (lap) xd = xb[0];
    else if (per) xd = X_DHT;  // a Hartley series stays one (index mirrored)
    else if (dir && reg) { xd = X_DCT1; len[g] = P.n[g] + 2; off[g] = 0; }  // n + 2 nodes
    else if (dir) xd = X_DCT3;
    else if (reg) { xd = X_DST1; len[g] = P.n[g] - 2; off[g] = 1; }   // interior nodes
    else xd = X_DST3;
    {
      PassArgs a = base();
      a.fast = FAST_GRAD_PREP;
      a.ax_j = lap ? -1 : g;
      a.in[0] = src;
      a.out[0] = dst;
      double cnt_in = 1.0, cnt_out = 1.0;
      for (int b = 0; b < 3; ++b) {
        a.gp_ext[b] = b < nd ? P.nout[b] : 1;
        a.gp_off[b] = off[b];
        a.gp_len[b] = len[b];
        a.gp_is[b] = a.gp_os[b] = b < nd ? ws[b] : 0;
        a.nunk[b] = b < nd ? P.n[b] : 1;
        a.lam[b] = eigen && b < nd ? P.lam[b] : nullptr;
        const int bb = b < nd ? axis_bc(d, b) : HP_NEUMANN;
        a.gp_basis[b] = bb == HP_PERIODIC ? 2 : (bb == HP_DIRICHLET ? 0 : 1);
        a.kc[b] = lap && b < nd ? (bb == HP_PERIODIC ? 2.0 : 1.0) * M_PI / P.len[b] : 0.0;
        if (b < nd) { cnt_in *= P.n[b]; cnt_out *= P.nout[b]; }
      }
      a.gp_eigen = eigen ? 1 : 0;
      if (lap) {
        a.diff = D_NABLA;
        a.gp_shift = 0;
        a.gp_scale = sign;
      } else if (per) {
        a.gp_shift = 0;
        a.gp_scale = sign * 2.0 * M_PI / P.len[g];
      } else {
        a.gp_shift = dir ? -1 : 1;
        a.gp_scale = sign * (dir ? 1.0 : -1.0) * M_PI / P.len[g];
      }
      a.norm = P.norm;
      PassRec r{a, 1};
      r.bytes = (cnt_in + cnt_out) * (double)es;
      out.push_back(r);
    }
    long long vo = 0;
    for (int b = 0; b < nd; ++b) vo += (long long)off[b] * ws[b];
    void* view = (void*)((char*)dst + vo * (long long)es);
    // axis 0 is already physical when the coefficients come from psi's array
    for (int c = last; c >= (eigen ? 0 : 1); --c) {
      PassArgs a = base();
      a.kind = PK_ONEWAY;
      a.xf = (!lap && c == g) ? xd : xb[c];
      a.L = L[c]; a.n = len[c]; a.nin = a.nout = len[c];
      a.in[0] = view; a.out[0] = view;
      a.in_sj = a.out_sj = ws[c];
      a.ax_j = c;
      if (nd == 1) {
        a.in_jfast = a.out_jfast = 1;
      } else if (c == last) {
        a.in_sp = a.out_sp = ws[last - 1]; a.Np = len[last - 1]; a.ax_p = last - 1;
        if (nd == 3) { a.in_so = a.out_so = ws[0]; a.No = len[0]; a.ax_o = 0; }
        a.in_jfast = a.out_jfast = 1;
      } else {
        a.in_sp = a.out_sp = ws[last]; a.Np = len[last]; a.ax_p = last;
        if (nd == 3) {
          const int o = c == 0 ? 1 : 0;
          a.in_so = a.out_so = ws[o]; a.No = len[o]; a.ax_o = o;
        }
      }
      for (int b = 0; b < 3; ++b) a.nunk[b] = b < nd ? len[b] : 0;
      HP_TRY(finish_pass(p, a, nd == 1 ? 2 : (c == last ? 16 : 32), 2, 0, 1));
      const void* q;
      HP_TRY(quarter(p, a.n, &q));
      a.qtw = q;
      out.push_back({a, 1});
    }
    return HP_OK;
  };
  const std::vector<DerivTerm> terms = derivative_terms(P);
  // before the sandwich: the terms along axis 0 and NABLA, from the source
  // transformed along every axis (one more forward pass along axis 0, out of place)
  auto pre_terms = [&](int comp) -> hp_status {
    bool any = false;
    for (auto& t : terms) any |= t.comp == comp && t.axis <= 0;
    if (!any) return HP_OK;
    HP_TRY(grad_forward_x(comp));
    const void* src = (const void*)((char*)P.grad_s + woff * es);
    for (auto& t : terms)
      if (t.comp == comp && t.axis <= 0) HP_TRY(grad_deriv(0, src, true, t.dst, t.sign, t.axis < 0));
    return HP_OK;
  };
  // after the sandwich: the terms along axes 1.., from psi's array (before
  // the backward passes change it)
  auto post_terms = [&](int comp) -> hp_status {
    for (auto& t : terms)
      if (t.comp == comp && t.axis > 0) HP_TRY(grad_deriv(t.axis, work(comp), false, t.dst, t.sign, false));
    return HP_OK;
  };
  // one pass per component (faces differ per component)
  for (int comp = 0; comp < P.ncomp; ++comp) {
    if (nd == 1) {
      HP_TRY(pre_terms(comp));
      PassArgs a = base();
      a.kind = PK_SANDWICH;
      a.xf = xf[0]; a.xb = xb[0];
      a.L = L[0]; a.n = P.n[0]; a.nin = a.nout = P.n[0];
      a.in[0] = P.in[comp]; a.out[0] = work(comp);
      a.in_sj = 1; a.out_sj = 1; a.in_jfast = a.out_jfast = 1;
      a.ax_j = 0;
      a.mult = M_EIGEN; a.lam[0] = P.lam[0]; a.norm = P.norm;
      set_faces(a, comp);
      HP_TRY(finish_pass(p, a, 2, 2, 0, 3));
      const void* q;
      HP_TRY(quarter(p, a.n, &q));
      a.qtw = q;
      out.push_back({a, 1});
      continue;
    }
    // P1: forward along the last (contiguous) axis, source + boundary terms
    {
      PassArgs a = base();
      a.kind = PK_ONEWAY;
      a.xf = xf[last];
      a.L = L[last]; a.n = P.n[last]; a.nin = a.nout = P.n[last];
      a.in[0] = P.in[comp]; a.out[0] = work(comp);
      a.in_sj = fs[last]; a.out_sj = ws[last];
      a.in_sp = fs[last - 1]; a.out_sp = ws[last - 1];
      a.Np = P.n[last - 1];
      a.ax_j = last; a.ax_p = last - 1;
      if (nd == 3) { a.in_so = fs[0]; a.out_so = ws[0]; a.No = P.n[0]; a.ax_o = 0; }
      a.in_jfast = a.out_jfast = 1;
      set_faces(a, comp);
      HP_TRY(finish_pass(p, a, 16, 2, 0, 1));
      const void* q;
      HP_TRY(quarter(p, a.n, &q));
      a.qtw = q;
      out.push_back({a, 1});
    }
    // P2 (3D): forward along axis 1, in place, tile across the last axis
    PassArgs p2{};
    if (nd == 3) {
      PassArgs a = base();
      a.kind = PK_ONEWAY;
      a.xf = xf[1];
      a.L = L[1]; a.n = P.n[1]; a.nin = a.nout = P.n[1];
      a.in[0] = work(comp); a.out[0] = work(comp);
      a.in_sj = a.out_sj = ws[1];
      a.in_sp = a.out_sp = ws[2];
      a.in_so = a.out_so = ws[0];
      a.Np = P.n[2]; a.No = P.n[0];
      a.ax_j = 1; a.ax_p = 2; a.ax_o = 0;
      HP_TRY(finish_pass(p, a, 32, 2, 0, 1));
      const void* q;
      HP_TRY(quarter(p, a.n, &q));
      a.qtw = q;
      out.push_back({a, 1});
      p2 = a;
    }
    HP_TRY(pre_terms(comp));
    // P3: sandwich along axis 0
    {
      PassArgs a = base();
      a.kind = PK_SANDWICH;
      a.xf = xf[0]; a.xb = xb[0];
      a.L = L[0]; a.n = P.n[0]; a.nin = a.nout = P.n[0];
      a.in[0] = work(comp); a.out[0] = work(comp);
      a.in_sj = a.out_sj = ws[0];
      a.in_sp = a.out_sp = ws[last];
      a.Np = P.n[last];
      a.ax_j = 0; a.ax_p = last;
      if (nd == 3) { a.in_so = a.out_so = ws[1]; a.No = P.n[1]; a.ax_o = 1; }
      a.mult = M_EIGEN;
      for (int b = 0; b < nd; ++b) a.lam[b] = P.lam[b];
      a.norm = P.norm;
      HP_TRY(finish_pass(p, a, 32, 2, 0, 3));
      const void* q;
      HP_TRY(quarter(p, a.n, &q));
      a.qtw = q;
      out.push_back({a, 1});
    }
    // after the sandwich: d/dx_g, g > 0, from psi's array (before P4 changes it)
    HP_TRY(post_terms(comp));
    // P4 (3D): backward along axis 1
    if (nd == 3) {
      PassArgs a = p2;  // same geometry as P2
      a.xf = xb[1];
      out.push_back({a, 1});
    }
    // P5: backward along the last axis, in place
    {
      PassArgs a = base();
      a.kind = PK_ONEWAY;
      a.xf = xb[last];
      a.L = L[last]; a.n = P.n[last]; a.nin = a.nout = P.n[last];
      a.in[0] = work(comp); a.out[0] = work(comp);
      a.in_sj = a.out_sj = ws[last];
      a.in_sp = a.out_sp = ws[last - 1];
      a.Np = P.n[last - 1];
      a.ax_j = last; a.ax_p = last - 1;
      if (nd == 3) { a.in_so = a.out_so = ws[0]; a.No = P.n[0]; a.ax_o = 0; }
      a.in_jfast = a.out_jfast = 1;
      HP_TRY(finish_pass(p, a, 16, 2, 0, 1));
      const void* q;
      HP_TRY(quarter(p, a.n, &q));
      a.qtw = q;
      out.push_back({a, 1});
    }
  }
  add_second_terms(P, es, out);
  if (bounded_fast_ok(p, P, L))
    for (size_t i = first_pass; i < out.size(); ++i) HP_TRY(to_fast_r2r(p, out[i].a));
  return HP_OK;
}

hp_status passes_periodic(hp_plan p, Problem& P, std::vector<PassRec>& out) {
  const int nd = P.nd;
  const bool coupled = P.nder > 0;
  const int nin = P.ncomp, nfo = P.ncomp + P.nder;
  auto base = [&]() {
    PassArgs a{};
    a.ax_j = a.ax_p = a.ax_o = -1;
    a.No = 1;
    a.Np = 1;
    a.n_in = a.n_out = 1;
    return a;
  };
  auto outptr = [&](int f) -> void* { return f < P.ncomp ? P.out[f] : P.der[f - P.ncomp]; };
  auto sandwich_common = [&](PassArgs& a) {
    a.kind = PK_SANDWICH;
    a.mult = M_EIGEN;
    for (int b = 0; b < nd; ++b) { a.lam[b] = P.lam[b]; a.kvec[b] = P.kvec[b]; }
    a.norm = P.norm;
    a.diff = diff_kind(P.d.diff, false);
    a.n_in = coupled ? nin : 1;
    a.n_out = coupled ? nfo : 1;
  };
  if (nd == 1) {
    PassArgs a = base();
    sandwich_common(a);
    a.xf = X_PAIR_F; a.xb = X_PAIR_B;
    a.L = P.n[0]; a.n = P.n[0]; a.nin = a.nout = P.n[0];
    for (int f = 0; f < nin; ++f) a.in[f] = P.in[f];
    for (int f = 0; f < nfo; ++f) a.out[f] = outptr(f);
    a.in_sj = a.out_sj = 1;
    a.in_jfast = a.out_jfast = 1;
    a.ax_j = 0;
    HP_TRY(finish_pass(p, a, 2, 2, 0, 5));
    out.push_back({a, coupled ? 1 : nin});
    return HP_OK;
  }
  // 2D grids whose half spectrum fits one workgroup's LDS: the whole solve
  // in one launch (HP_SMALL2D=0 keeps the three general passes)
  if (nd == 2) {
    const int dk = diff_kind(P.d.diff, false);
    const char* e = std::getenv("HP_SMALL2D");
    const bool ok_diff = dk == D_NONE || dk == D_GRAD || dk == D_NABLA || (dk == D_CURL && nin == 1);
    const int nbuf = dk == D_NONE ? nin : nin + 1;
    const int lds = small2d_lds_bytes(P.n[0], P.n[1], p->prec, nbuf);
    bool bound = true;
    for (int f = 0; f < nin; ++f) bound = bound && P.in[f];
    if (ok_diff && bound && lds > 0 && lds <= 160 * 1024 && !(e && std::atoi(e) == 0)) {
      PassArgs a = base();
      sandwich_common(a);
      a.fast = FAST_SMALL2D;
      a.gM[0] = P.n[0];
      a.gM[1] = P.n[1];
      HP_TRY(fast_twiddles(p, P.n[0], &a.tw));
      HP_TRY(fast_twiddles(p, P.n[1], &a.qtw));
      a.n_in = nin;
      a.n_out = nfo;
      for (int f = 0; f < nin; ++f) a.in[f] = P.in[f];
      for (int f = 0; f < nfo; ++f) a.out[f] = outptr(f);
      a.lds_bytes = lds;
      PassRec r{a, 1};
      r.bytes = (double)(nin + nfo) * P.n[0] * P.n[1] * p->es;
      out.push_back(r);
      return HP_OK;
    }
  }
  const int last = nd - 1;
  const int n_last = P.n[last];
  const int K = n_last / 2 + 1;
  // spectral buffer dims (storage): [n0][n1][K] (3D) or [n0][K] (2D)
  long long ss[3] = {0, 0, 0};  // strides per logical axis
  if (nd == 3) { ss[2] = 1; ss[1] = K; ss[0] = (long long)P.n[1] * K; }
  else { ss[1] = 1; ss[0] = K; }
  long long fs[3] = {0, 0, 0};
  if (nd == 3) { fs[2] = 1; fs[1] = P.n[2]; fs[0] = (long long)P.n[1] * P.n[2]; }
  else { fs[1] = 1; fs[0] = P.n[1]; }
  // P1: R2C along the last axis, per input component
  {
    PassArgs a = base();
    a.kind = PK_ONEWAY;
    a.xf = X_R2C;
    a.L = n_last; a.n = n_last; a.nin = n_last; a.nout = K;
    for (int f = 0; f < nin; ++f) { a.in[f] = P.in[f]; a.out[f] = P.b2[f]; }
    a.in_sj = fs[last]; a.in_sp = fs[last - 1];
    a.out_sj = ss[last]; a.out_sp = ss[last - 1];
    a.Np = P.n[last - 1];
    if (nd == 3) { a.in_so = fs[0]; a.out_so = ss[0]; a.No = P.n[0]; }
    a.in_jfast = a.out_jfast = 1;
    HP_TRY(finish_pass(p, a, 16, 2, 0, 1));
    out.push_back({a, nin});
  }
  // P2 (3D): forward C2C along axis 1, in place
  PassArgs p2{};
  if (nd == 3) {
    PassArgs a = base();
    a.kind = PK_ONEWAY;
    a.xf = X_C2C_F;
    a.L = P.n[1]; a.n = P.n[1]; a.nin = a.nout = P.n[1];
    for (int f = 0; f < nin; ++f) { a.in[f] = P.b2[f]; a.out[f] = P.b2[f]; }
    a.in_sj = a.out_sj = ss[1];
    a.in_sp = a.out_sp = ss[2];
    a.in_so = a.out_so = ss[0];
    a.Np = K; a.No = P.n[0];
    HP_TRY(finish_pass(p, a, 16, 1, 0, 0));
    p2 = a;
    out.push_back({a, nin});
  }
  // P3: sandwich along axis 0
  {
    PassArgs a = base();
    sandwich_common(a);
    a.xf = X_C2C_F; a.xb = X_C2C_B;
    a.L = P.n[0]; a.n = P.n[0]; a.nin = a.nout = P.n[0];
    for (int f = 0; f < nin; ++f) a.in[f] = P.b2[f];
    for (int f = 0; f < nfo; ++f) a.out[f] = P.b2[f];
    a.in_sj = a.out_sj = ss[0];
    a.in_sp = a.out_sp = ss[last];
    a.Np = K;
    a.ax_j = 0; a.ax_p = last;
    if (nd == 3) { a.in_so = a.out_so = ss[1]; a.No = P.n[1]; a.ax_o = 1; }
    HP_TRY(finish_pass(p, a, 16, 1, 0, 4));
    out.push_back({a, coupled ? 1 : nin});
  }
  // P4 (3D): backward C2C along axis 1 on every output field
  if (nd == 3) {
    PassArgs a = p2;
    a.xf = X_C2C_B;
    for (int f = 0; f < nfo; ++f) { a.in[f] = P.b2[f]; a.out[f] = P.b2[f]; }
    out.push_back({a, nfo});
  }
  // P5: C2R along the last axis into the outputs
  {
    PassArgs a = base();
    a.kind = PK_ONEWAY;
    a.xf = X_C2R;
    a.L = n_last; a.n = n_last; a.nin = K; a.nout = n_last;
    for (int f = 0; f < nfo; ++f) { a.in[f] = P.b2[f]; a.out[f] = outptr(f); }
    a.in_sj = ss[last]; a.in_sp = ss[last - 1];
    a.out_sj = fs[last]; a.out_sp = fs[last - 1];
    a.Np = P.n[last - 1];
    if (nd == 3) { a.in_so = ss[0]; a.out_so = fs[0]; a.No = P.n[0]; }
    a.in_jfast = a.out_jfast = 1;
    HP_TRY(finish_pass(p, a, 16, 2, 0, 2));
    out.push_back({a, nfo});
  }
  return HP_OK;
}

// Unbounded (3D): pruned doubled-domain transform with transposing layouts
//   f [x][y][z] -R2C z-> A1 [x][kz][y] -C2C y-> B2 [kz][ky][x]
//   -sandwich x (Ghat, derivative)-> B2 -C2C^-1 y-> [kz][y][x] -C2R z-> out [x][y][z]
// Only the physical half of every doubled axis is ever loaded or stored.
hp_status passes_unbounded(hp_plan p, Problem& P, bool adjoint, std::vector<PassRec>& out) {
  const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
  const int M0 = P.M[0], M1 = P.M[1], M2 = P.M[2];
  const int K2 = M2 / 2 + 1;
  const int nc = P.ncomp, nder = P.nder;
  const int nslot = nc + nder;
  // input / output fields of this direction
  const void* src[kMaxFields] = {};
  void* dst[kMaxFields] = {};
  int n_src, n_dst;
  if (!adjoint) {
    n_src = nc;
    n_dst = nslot;
    for (int c = 0; c < nc; ++c) src[c] = P.in[c];
    for (int f = 0; f < nslot; ++f) dst[f] = f < nc ? P.out[f] : P.der[f - nc];
  } else {
    n_src = nslot;
    n_dst = nc;
    for (int f = 0; f < nslot; ++f) src[f] = f < nc ? P.out[f] : P.der[f - nc];
    for (int c = 0; c < nc; ++c) dst[c] = (void*)P.in[c];
  }
  auto base = [&]() {
    PassArgs a{};
    a.ax_j = a.ax_p = a.ax_o = -1;
    a.n_in = a.n_out = 1;
    return a;
  };
  // P1: R2C along z (pruned input: z < n2 of M2)
  {
    PassArgs a = base();
    a.kind = PK_ONEWAY;
    a.xf = X_R2C;
    a.L = M2; a.n = M2; a.nin = n2; a.nout = K2;
    for (int f = 0; f < n_src; ++f) { a.in[f] = src[f]; a.out[f] = P.a1[f]; }
    a.in_sj = 1; a.in_sp = n2; a.in_so = (long long)n1 * n2;
    a.out_sj = n1; a.out_sp = 1; a.out_so = (long long)K2 * n1;
    a.Np = n1; a.No = n0;
    a.in_jfast = 1; a.out_jfast = 0;
    HP_TRY(finish_pass(p, a, p->prec == 0 ? 32 : 16, 2, 0, 1));
    out.push_back({a, n_src});
  }
  // P2: C2C along y (pruned input y < n1 of M1), transposing to [kz][ky][x]
  {
    PassArgs a = base();
    a.kind = PK_ONEWAY;
    a.xf = X_C2C_F;
    a.L = M1; a.n = M1; a.nin = n1; a.nout = M1;
    for (int f = 0; f < n_src; ++f) { a.in[f] = src[f] ? P.a1[f] : nullptr; a.out[f] = P.b2[f]; }
    a.in_sj = 1; a.in_sp = (long long)K2 * n1; a.in_so = n1;
    a.out_sj = n0; a.out_sp = 1; a.out_so = (long long)M1 * n0;
    a.Np = n0; a.No = K2;
    a.in_jfast = 1; a.out_jfast = 0;
    HP_TRY(finish_pass(p, a, p->prec == 0 ? 32 : 16, 1, 0, 0));
    out.push_back({a, n_src});
  }
  // P3: sandwich along x: forward (x < n0 of M0), Ghat, derivative, backward (x < n0)
  {
    PassArgs a = base();
    a.kind = PK_SANDWICH;
    a.xf = X_C2C_F; a.xb = X_C2C_B;
    a.L = M0; a.n = M0; a.nin = n0; a.nout = n0;
    for (int f = 0; f < n_src; ++f) a.in[f] = src[f] ? P.b2[f] : nullptr;
    for (int f = 0; f < n_dst; ++f) a.out[f] = P.b2[f];
    a.in_sj = a.out_sj = 1;
    a.in_sp = a.out_sp = n0;
    a.in_so = a.out_so = (long long)M1 * n0;
    a.Np = M1; a.No = K2;
    a.in_jfast = a.out_jfast = 1;
    a.ax_j = 0; a.ax_p = 1; a.ax_o = 2;
    a.mult = M_GREEN;
    a.green = P.green;
    for (int b = 0; b < 3; ++b) a.g_s[b] = P.g_s[b];
    a.gM[0] = M0; a.gM[1] = M1; a.gM[2] = M2;
    for (int b = 0; b < 3; ++b) a.kvec[b] = P.kvec[b];
    a.diff = diff_kind(P.d.diff, adjoint);
    const bool coupled = a.diff != D_NONE;
    a.n_in = coupled ? n_src : 1;
    a.n_out = coupled ? n_dst : 1;
    HP_TRY(finish_pass(p, a, 16, 1, 0, 4));
    out.push_back({a, coupled ? 1 : nc});
  }
  // P4: backward C2C along y, keep y < n1, in place in B2
  {
    PassArgs a = base();
    a.kind = PK_ONEWAY;
    a.xf = X_C2C_B;
    a.L = M1; a.n = M1; a.nin = M1; a.nout = n1;
    for (int f = 0; f < n_dst; ++f) { a.in[f] = P.b2[f]; a.out[f] = P.b2[f]; }
    a.in_sj = a.out_sj = n0;
    a.in_sp = a.out_sp = 1;
    a.in_so = a.out_so = (long long)M1 * n0;
    a.Np = n0; a.No = K2;
    a.in_jfast = a.out_jfast = 0;
    HP_TRY(finish_pass(p, a, p->prec == 0 ? 32 : 16, 1, 0, 0));
    out.push_back({a, n_dst});
  }
  // P5: C2R along z, keep z < n2, into the destination arrays [x][y][z]
  {
    PassArgs a = base();
    a.kind = PK_ONEWAY;
    a.xf = X_C2R;
    a.L = M2; a.n = M2; a.nin = K2; a.nout = n2;
    for (int f = 0; f < n_dst; ++f) { a.in[f] = P.b2[f]; a.out[f] = dst[f]; }
    a.in_sj = (long long)M1 * n0; a.in_sp = 1; a.in_so = n0;
    a.out_sj = 1; a.out_sp = (long long)n1 * n2; a.out_so = n2;
    a.Np = n0; a.No = n1;
    a.in_jfast = 0; a.out_jfast = 1;
    HP_TRY(finish_pass(p, a, p->prec == 0 ? 32 : 16, 2, 0, 2));
    out.push_back({a, n_dst});
  }
  return HP_OK;
}

// Wavefront-FFT free-space passes (every doubled length a power of two in
// [64, 1024]).  Layouts (complex): A1 [x][kz][y], B2 [kz][ky][x],
// C2 [kz][x][ky], C1 [x][y][kz] (C1 reuses the A1 buffers).  Every pass reads
// contiguous pencils; strided sides are written through LDS tiles.
// Also used for 3D periodic plans, whose transform lengths M are then n.
bool fast_unbounded_ok(hp_plan p, const Problem& P) {
  if (std::getenv("HP_GENERIC") || P.nd != 3) return false;
  const bool pad = P.d.bc == HP_UNBOUNDED;
  auto pow2 = [](int v) { return v >= 64 && v <= 1024 && (v & (v - 1)) == 0; };
  for (int a = 0; a < 3; ++a)
    if (!pow2(P.M[a])) return false;
  const int kinds[5] = {FAST_R2C, FAST_FWD_Y, FAST_SANDWICH, FAST_INV_Y, FAST_C2R};
  const int axisL[5] = {P.M[2], P.M[1], P.M[0], P.M[1], P.M[2]};
  const int K2 = P.M[2] / 2 + 1;
  for (int i = 0; i < 5; ++i) {
    const int Pt = fast_tile(kinds[i], axisL[i], p->prec);
    if (fast_lds_bytes(kinds[i], axisL[i], Pt, K2, p->prec, 0, pad) > 160 * 1024) return false;
  }
  return true;
}

// Free-space passes, or (periodic) the same five passes on undoubled
// pencils with the Table 1 eigenvalue multiplier in place of the Green's
// function.
hp_status passes_unbounded_fast(hp_plan p, Problem& P, bool adjoint, std::vector<PassRec>& out) {
  const bool periodic = P.d.bc == HP_PERIODIC;
  const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
  const int M0 = P.M[0], M1 = P.M[1], M2 = P.M[2];
  const int K2 = M2 / 2 + 1;
  const int nc = P.ncomp, nder = P.nder;
  const double es = (double)p->es, cs = 2.0 * p->es;
  const void* src[kMaxFields] = {};
  void* dst[kMaxFields] = {};
  int n_src, n_dst, n_mid, iy_mode;
  const int dk = P.d.diff;
  if (!adjoint) {
    n_src = nc;
    n_dst = nc + nder;
    for (int c = 0; c < nc; ++c) src[c] = P.in[c];
    for (int f = 0; f < n_dst; ++f) dst[f] = f < nc ? P.out[f] : P.der[f - nc];
    // spectra between the x and the backward y pass: the curl completes its
    // y / z derivatives there (5), the gradient its y / z (2); psi, the
    // divergence and the Laplacian leave the x pass complete
    n_mid = dk == HP_D_CURL ? 5 : (dk == HP_D_GRAD ? 2 : n_dst);
    iy_mode = dk == HP_D_CURL ? IY_CURL5 : (dk == HP_D_GRAD ? IY_GRAD2 : IY_PLAIN);
  } else {
    n_src = nc + nder;
    n_dst = nc;
    for (int f = 0; f < n_src; ++f) src[f] = f < nc ? P.out[f] : P.der[f - nc];
    for (int c = 0; c < nc; ++c) dst[c] = (void*)P.in[c];
    n_mid = nc;
    iy_mode = IY_PLAIN;
  }
  int n_live = 0;
  for (int f = 0; f < n_src; ++f) n_live += src[f] ? 1 : 0;
  auto base = [&](int kind, int L) -> hp_status {
    PassArgs a{};
    a.ax_j = a.ax_p = a.ax_o = -1;
    a.n_in = a.n_out = 1;
    a.fast = kind;
    a.L = a.n = L;
    a.P = fast_tile(kind, L, p->prec);
    for (int b = 0; b < 3; ++b) {
      a.un[b] = P.n[b];
      a.gM[b] = P.M[b];
      a.kc[b] = 2.0 * M_PI / (P.M[b] * P.h[b]);
    }
    const void* tw;
    HP_TRY(fast_twiddles(p, L, &tw));
    a.tw = tw;
    a.c1_ld = (K2 + 15) / 16 * 16;
    // C1 [x][y][kz]: the backward y pass writes rows y of one x close together
    a.c1_sx = (long long)P.n[1] * a.c1_ld;
    a.c1_sy = a.c1_ld;
    a.pad = periodic ? 0 : 1;
    a.emit_dbl = fast_emit_dbl(kind, p->prec);
    if (fast_lds_bytes(kind, L, a.P, K2, p->prec, a.emit_dbl, a.pad) > 160 * 1024) a.emit_dbl = 0;
    {
      const long long v[] = {1,      p->prec, kind,   L,      a.pad,  P.n[0],  P.n[1], P.n[2],
                             P.M[0], P.M[1],  P.M[2], dk,     adjoint ? 1 : 0, n_src, n_live};
      a.tune_key = tune_hash(v, (int)(sizeof(v) / sizeof(v[0])));
      auto it = p->tuned.find(a.tune_key);
      if (it != p->tuned.end() && it->second.fast == kind &&
          fast_tile_ok(kind, L, it->second.P, p->prec) &&
          fast_lds_bytes(kind, L, it->second.P, K2, p->prec, it->second.emit_dbl, a.pad) <= 160 * 1024) {
        a.P = it->second.P;
        a.emit_dbl = it->second.emit_dbl;
      }
    }
    a.lds_bytes = fast_lds_bytes(kind, L, a.P, K2, p->prec, a.emit_dbl, a.pad);
    out.push_back({a, 1});
    return HP_OK;
  };
  // P1: R2C along z into A1
  HP_TRY(base(FAST_R2C, M2));
  {
    PassRec& r = out.back();
    for (int f = 0; f < n_src; ++f) { r.a.in[f] = src[f]; r.a.out[f] = P.a1[f]; }
    r.grid_y = n_src;
    r.bytes = n_live * ((double)n0 * n1 * n2 * es + (double)n0 * K2 * n1 * cs);
  }
  // P2 - P4 per kz slab (one slab covering all K2 planes unless HP_SLAB set)
  for (const auto& slab : P.slabs) {
    const int kb = slab.first, kc = slab.second;
    // P2: forward C2C along y into B2
    HP_TRY(base(FAST_FWD_Y, M1));
    {
      PassRec& r = out.back();
      r.a.kz_base = kb;
      r.a.kz_count = kc;
      for (int f = 0; f < n_src; ++f) { r.a.in[f] = src[f] ? P.a1[f] : nullptr; r.a.out[f] = P.b2[f]; }
      r.grid_y = n_src;
      r.bytes = n_live * ((double)n0 * kc * n1 * cs + (double)kc * M1 * n0 * cs);
    }
    // P3: sandwich along x into C2
    HP_TRY(base(FAST_SANDWICH, M0));
    {
      PassRec& r = out.back();
      PassArgs& a = r.a;
      a.kz_base = kb;
      a.kz_count = kc;
      if (periodic) {
        a.mult = M_EIGEN;
        for (int b = 0; b < 3; ++b) a.lam[b] = P.lam[b];
        a.norm = P.norm;
      } else {
        a.mult = M_GREEN;
        a.green = P.green;
        for (int b = 0; b < 3; ++b) a.g_s[b] = P.g_s[b];
      }
      a.diff = diff_kind(dk, adjoint);
      for (int f = 0; f < n_src; ++f) a.in[f] = src[f] ? P.b2[f] : nullptr;
      for (int f = 0; f < n_mid; ++f) a.out[f] = P.c2[f];
      // one output group per component, or one coupled group
      r.grid_y = (a.diff == D_NONE || a.diff == D_CURL || a.diff == D_NABLA || a.diff == D_ADJ_NABLA)
                     ? nc : 1;
      const double oct = periodic ? 0.0 : (double)(M0 / 2 + 1) * (M1 / 2 + 1) * kc * es;
      r.bytes = (n_live + n_mid) * (double)kc * M1 * n0 * cs + oct;
    }
    // P4: backward C2C along y (with derivative completion) into C1 (= A1 buffers)
    HP_TRY(base(FAST_INV_Y, M1));
    {
      PassRec& r = out.back();
      r.a.kz_base = kb;
      r.a.kz_count = kc;
      r.a.iy_mode = iy_mode;
      for (int f = 0; f < n_mid; ++f) r.a.in[f] = P.c2[f];
      for (int f = 0; f < n_dst; ++f) r.a.out[f] = P.c1.empty() ? P.a1[f] : P.c1[f];
      r.grid_y = iy_mode == IY_PLAIN ? n_mid : (iy_mode == IY_CURL5 ? 2 : 1);
      r.bytes = n_mid * (double)kc * n0 * M1 * cs + n_dst * (double)n1 * n0 * kc * cs;
    }
  }
  // P5: C2R along z into the destination arrays
  HP_TRY(base(FAST_C2R, M2));
  {
    PassRec& r = out.back();
    for (int f = 0; f < n_dst; ++f) { r.a.in[f] = P.c1.empty() ? P.a1[f] : P.c1[f]; r.a.out[f] = dst[f]; }
    r.grid_y = n_dst;
    r.bytes = n_dst * ((double)n1 * n0 * K2 * cs + (double)n0 * n1 * n2 * es);
  }
  return HP_OK;
}

// 1D / 2D free space (the problem lifted to 3D with unit trailing axes, whose
// Green's table is the 1D / 2D kernel): the real transform runs along the
// last physical axis, so the x pass works on the half spectrum only.
//   2D: f [x][y] -R2C y (y < n1 of M1)-> B2 [ky][x] -sandwich x (Ghat,
//       derivative)-> B2 -C2R y (keep y < n1)-> out [x][y]
//   1D: one paired real sandwich along x (x < n0 of M0 in and out)
hp_status passes_unbounded_low(hp_plan p, Problem& P, bool adjoint, std::vector<PassRec>& out) {
  const int n0 = P.n[0], n1 = P.n[1];
  const int M0 = P.M[0], M1 = P.M[1];
  const int nc = P.ncomp, nder = P.nder, nslot = nc + nder;
  const void* src[kMaxFields] = {};
  void* dst[kMaxFields] = {};
  int n_src, n_dst;
  if (!adjoint) {
    n_src = nc;
    n_dst = nslot;
    for (int c = 0; c < nc; ++c) src[c] = P.in[c];
    for (int f = 0; f < nslot; ++f) dst[f] = f < nc ? P.out[f] : P.der[f - nc];
  } else {
    n_src = nslot;
    n_dst = nc;
    for (int f = 0; f < nslot; ++f) src[f] = f < nc ? P.out[f] : P.der[f - nc];
    for (int c = 0; c < nc; ++c) dst[c] = (void*)P.in[c];
  }
  auto sandwich_common = [&](PassArgs& a) {
    a.kind = PK_SANDWICH;
    a.mult = M_GREEN;
    a.green = P.green;
    for (int b = 0; b < 3; ++b) {
      a.g_s[b] = P.g_s[b];
      a.gM[b] = P.M[b];
      a.kvec[b] = P.kvec[b];
    }
    a.diff = diff_kind(P.d.diff, adjoint);
    const bool coupled = a.diff != D_NONE;
    a.n_in = coupled ? n_src : 1;
    a.n_out = coupled ? n_dst : 1;
    return coupled;
  };
  if (P.nd == 1) {
    PassArgs a{};
    a.ax_j = 0; a.ax_p = a.ax_o = -1;
    a.Np = a.No = 1;
    const bool coupled = sandwich_common(a);
    a.xf = X_PAIR_F; a.xb = X_PAIR_B;
    a.L = M0; a.n = M0; a.nin = n0; a.nout = n0;
    for (int f = 0; f < n_src; ++f) a.in[f] = src[f];
    for (int f = 0; f < n_dst; ++f) a.out[f] = dst[f];
    a.in_sj = a.out_sj = 1;
    a.in_jfast = a.out_jfast = 1;
    HP_TRY(finish_pass(p, a, 2, 2, 0, 5));
    out.push_back({a, coupled ? 1 : nc});
    return HP_OK;
  }
  const int K1 = M1 / 2 + 1;
  // P1: R2C along y (pruned input y < n1), transposing to [ky][x]
  {
    PassArgs a{};
    a.ax_j = a.ax_p = a.ax_o = -1;
    a.n_in = a.n_out = 1;
    a.No = 1;
    a.kind = PK_ONEWAY;
    a.xf = X_R2C;
    a.L = M1; a.n = M1; a.nin = n1; a.nout = K1;
    for (int f = 0; f < n_src; ++f) { a.in[f] = src[f]; a.out[f] = P.b2[f]; }
    a.in_sj = 1; a.in_sp = n1;
    a.out_sj = n0; a.out_sp = 1;
    a.Np = n0;
    a.in_jfast = 1; a.out_jfast = 0;
    HP_TRY(finish_pass(p, a, p->prec == 0 ? 32 : 16, 2, 0, 1));
    out.push_back({a, n_src});
  }
  // P2: sandwich along x on the half spectrum ky < K1
  {
    PassArgs a{};
    a.ax_j = 0; a.ax_p = 1; a.ax_o = 2;
    a.No = 1;
    const bool coupled = sandwich_common(a);
    a.xf = X_C2C_F; a.xb = X_C2C_B;
    a.L = M0; a.n = M0; a.nin = n0; a.nout = n0;
    for (int f = 0; f < n_src; ++f) a.in[f] = src[f] ? P.b2[f] : nullptr;
    for (int f = 0; f < n_dst; ++f) a.out[f] = P.b2[f];
    a.in_sj = a.out_sj = 1;
    a.in_sp = a.out_sp = n0;
    a.Np = K1;
    a.in_jfast = a.out_jfast = 1;
    HP_TRY(finish_pass(p, a, 16, 1, 0, 4));
    out.push_back({a, coupled ? 1 : nc});
  }
  // P3: C2R along y, keep y < n1, into the destination arrays [x][y]
  {
    PassArgs a{};
    a.ax_j = a.ax_p = a.ax_o = -1;
    a.n_in = a.n_out = 1;
    a.No = 1;
    a.kind = PK_ONEWAY;
    a.xf = X_C2R;
    a.L = M1; a.n = M1; a.nin = K1; a.nout = n1;
    for (int f = 0; f < n_dst; ++f) { a.in[f] = P.b2[f]; a.out[f] = dst[f]; }
    a.in_sj = n0; a.in_sp = 1;
    a.out_sj = 1; a.out_sp = n1;
    a.Np = n0;
    a.in_jfast = 0; a.out_jfast = 1;
    HP_TRY(finish_pass(p, a, p->prec == 0 ? 32 : 16, 2, 0, 2));
    out.push_back({a, n_dst});
  }
  return HP_OK;
}

// Semi-unbounded plans (Section 2.6): one free axis u beside periodic,
// Dirichlet and Neumann axes.  Forward transforms along the bounded axes (the
// contiguous one first, boundary terms added on the first load), then the free
// axis as a doubled paired-real sandwich whose multiplier is the row of the
// Helmholtz Green's spectrum of each pencil's bounded mode (M_GREEN_ROWS),
// then the backward transforms.  In place in the output array, as on the
// Dirichlet / Neumann path; one pass list per component.
hp_status passes_semi(hp_plan p, Problem& P, std::vector<PassRec>& out) {
  const hp_desc& d = P.d;
  const int nd = P.nd, u = P.free_axis;
  const size_t first_pass = out.size();
  int xf[3] = {0, 0, 0}, xb[3] = {0, 0, 0}, L[3] = {1, 1, 1};
  double c[3] = {1, 1, 1};
  for (int a = 0; a < nd; ++a) {
    if (a == u) L[a] = P.M[u];
    else r2r_ops(axis_bc(d, a), d.grid, P.n[a], &xf[a], &xb[a], &L[a], &c[a]);
  }
  // strides of the input array and of the work view (the output array, its
  // interior along REGULAR Dirichlet axes), logical axis a -> storage dim 3 - nd + a
  int sod[3] = {1, 1, 1}, sid[3] = {1, 1, 1};
  for (int a = 0; a < nd; ++a) { sod[3 - nd + a] = P.nout[a]; sid[3 - nd + a] = P.n[a]; }
  long long os3[3], is3[3];
  strides_of(sod, os3);
  strides_of(sid, is3);
  long long ws[3] = {0, 0, 0}, fs[3] = {0, 0, 0};
  for (int a = 0; a < nd; ++a) { ws[a] = os3[3 - nd + a]; fs[a] = is3[3 - nd + a]; }
  const int dmask = dreg_axes(d);
  long long woff = 0;
  for (int a = 0; a < nd; ++a)
    if ((dmask >> a) & 1) woff += ws[a];
  const size_t es = p->es;
  auto work = [&](int comp) { return (void*)((char*)P.out[comp] + woff * es); };
  auto base = [&]() {
    PassArgs a{};
    a.ax_j = a.ax_p = a.ax_o = -1;
    a.No = 1;
    a.Np = 1;
    a.n_in = a.n_out = 1;
    for (int b = 0; b < 3; ++b) a.nunk[b] = b < nd ? P.n[b] : 0;
    return a;
  };
  // pencils along axis j: the tile runs along the last of the other axes
  // (contiguous unless j is the last axis, whose pencils are contiguous);
  // extents ext (default: the unknowns)
  auto geom = [&](PassArgs& a, int j, bool from_input, const int* ext = nullptr) {
    if (!ext) ext = P.n;
    const long long* is = from_input ? fs : ws;
    int others[2], no = 0;
    for (int b = 0; b < nd; ++b)
      if (b != j) others[no++] = b;
    a.ax_j = j;
    a.in_sj = is[j];
    a.out_sj = ws[j];
    const int pa = others[no - 1];
    a.ax_p = pa;
    a.Np = ext[pa];
    a.in_sp = is[pa];
    a.out_sp = ws[pa];
    if (no == 2) {
      const int oa = others[0];
      a.ax_o = oa;
      a.No = ext[oa];
      a.in_so = is[oa];
      a.out_so = ws[oa];
    }
    a.in_jfast = a.out_jfast = j == nd - 1 ? 1 : 0;
  };
  auto oneway = [&](int comp, int j, int x, bool first) -> hp_status {
    PassArgs a = base();
    a.kind = PK_ONEWAY;
    a.xf = x;
    a.L = L[j]; a.n = P.n[j]; a.nin = a.nout = P.n[j];
    a.in[0] = first ? P.in[comp] : work(comp);
    a.out[0] = work(comp);
    geom(a, j, first);
    if (first) fill_face_terms(P, comp, a);
    HP_TRY(finish_pass(p, a, j == nd - 1 ? 16 : 32, 2, 0, 1));
    const void* q;
    HP_TRY(quarter(p, a.n, &q));
    a.qtw = q;
    out.push_back({a, 1});
    return HP_OK;
  };
  // one real-to-real pass along j, in place on the view at `view` (extents ext)
  auto oneway_view = [&](void* view, int j, int x, const int* ext) -> hp_status {
    PassArgs a = base();
    a.kind = PK_ONEWAY;
    a.xf = x;
    a.L = L[j]; a.n = ext[j]; a.nin = a.nout = ext[j];
    a.in[0] = view;
    a.out[0] = view;
    geom(a, j, false, ext);
    for (int b = 0; b < 3; ++b) a.nunk[b] = b < nd ? ext[b] : 0;
    HP_TRY(finish_pass(p, a, j == nd - 1 ? 16 : 32, 2, 0, 1));
    const void* q;
    HP_TRY(quarter(p, a.n, &q));
    a.qtw = q;
    out.push_back({a, 1});
    return HP_OK;
  };
  // the free-axis sandwich on the view at `v`: Green's rows, or the rows of
  // the kernel's derivative
  auto sandwich = [&](void* v, bool odd) -> hp_status {
    PassArgs a = base();
    a.kind = PK_SANDWICH;
    a.xf = X_PAIR_F;
    a.xb = X_PAIR_B;
    a.L = L[u]; a.n = P.n[u]; a.nin = a.nout = P.n[u];
    a.in[0] = v;
    a.out[0] = v;
    geom(a, u, false);
    a.mult = odd ? M_GREEN_ROWS_ODD : M_GREEN_ROWS;
    a.green = odd ? P.green_odd : P.green;
    for (int b = 0; b < 3; ++b) a.g_s[b] = P.g_s[b];
    a.diff = D_NONE;
    HP_TRY(finish_pass(p, a, 16, 2, 0, 5));
    out.push_back({a, 1});
    return HP_OK;
  };
  // elementwise prep into the whole output array `dst` (zero outside the
  // active view off / len): along a bounded axis g the series derivative of
  // psi's coefficients src (the derivative's basis and index shift, times
  // sign), or with g < 0 a copy of src times sign
  auto prep = [&](const void* src, const long long* is, void* dst, int g, const int* off, const int* len,
                  double sign) {
    PassArgs a = base();
    a.fast = FAST_GRAD_PREP;
    a.ax_j = g;
    a.diff = D_NONE;
    a.in[0] = src;
    a.out[0] = dst;
    double cnt_in = 1.0, cnt_out = 1.0;
    for (int b = 0; b < 3; ++b) {
      a.gp_ext[b] = b < nd ? P.nout[b] : 1;
      a.gp_off[b] = off[b];
      a.gp_len[b] = len[b];
      a.gp_is[b] = b < nd ? is[b] : 0;
      a.gp_os[b] = b < nd ? ws[b] : 0;
      a.nunk[b] = b < nd ? P.n[b] : 1;
      a.lam[b] = nullptr;
      const int bb = b < nd ? axis_bc(d, b) : HP_NEUMANN;
      a.gp_basis[b] = bb == HP_PERIODIC ? 2 : (bb == HP_DIRICHLET ? 0 : 1);
      a.kc[b] = 0.0;
      if (b < nd) { cnt_in *= P.n[b]; cnt_out *= P.nout[b]; }
    }
    a.gp_eigen = 0;
    a.gp_shift = 0;
    a.gp_scale = sign;
    if (g >= 0) {
      const int bcg = axis_bc(d, g);
      if (bcg == HP_PERIODIC) {
        a.gp_scale = sign * 2.0 * M_PI / P.len[g];
      } else {
        const bool dir = bcg == HP_DIRICHLET;
        a.gp_shift = dir ? -1 : 1;
        a.gp_scale = sign * (dir ? 1.0 : -1.0) * M_PI / P.len[g];
      }
    }
    a.norm = P.norm;
    PassRec r{a, 1};
    r.bytes = (cnt_in + cnt_out) * (double)es;
    out.push_back(r);
  };
  // Derivatives of homogeneous solves.  Along a bounded axis g: after the
  // sandwich psi's array holds the bounded coefficients (the free axis
  // physical); the prep writes the derivative series along g and backward
  // transforms along the bounded axes (the other parity's along g) evaluate
  // it.  Along the free axis: the source copied into the output (times the
  // term's sign), forward bounded transforms, the sandwich with the odd
  // kernel's rows and the backward transforms.
  const std::vector<DerivTerm> terms = derivative_terms(P);
  auto bounded_term = [&](int comp, int g, void* dst, double sign) -> hp_status {
    const int bcg = axis_bc(d, g);
    const bool dir = bcg == HP_DIRICHLET, reg = d.grid == HP_REGULAR;
    int off[3] = {0, 0, 0}, len[3] = {1, 1, 1};
    for (int b = 0; b < nd; ++b) { off[b] = (dmask >> b) & 1; len[b] = P.n[b]; }
    int xd;
    if (bcg == HP_PERIODIC) xd = X_DHT;
    else if (dir && reg) { xd = X_DCT1; len[g] = P.n[g] + 2; off[g] = 0; }  // n + 2 nodes
    else if (dir) xd = X_DCT3;
    else if (reg) { xd = X_DST1; len[g] = P.n[g] - 2; off[g] = 1; }   // interior nodes
    else xd = X_DST3;
    prep(work(comp), ws, dst, g, off, len, sign);
    long long vo = 0;
    for (int b = 0; b < nd; ++b) vo += (long long)off[b] * ws[b];
    void* view = (void*)((char*)dst + vo * (long long)es);
    for (int c = nd - 1; c >= 0; --c)
      if (c != u) HP_TRY(oneway_view(view, c, c == g ? xd : xb[c], len));
    return HP_OK;
  };
  auto free_term = [&](int comp, void* dst, double sign) -> hp_status {
    int off[3] = {0, 0, 0}, len[3] = {1, 1, 1};
    for (int b = 0; b < nd; ++b) { off[b] = (dmask >> b) & 1; len[b] = P.n[b]; }
    prep(P.in[comp], fs, dst, -1, off, len, sign);
    void* view = (void*)((char*)dst + woff * es);
    for (int j = nd - 1; j >= 0; --j)
      if (j != u) HP_TRY(oneway_view(view, j, xf[j], P.n));
    HP_TRY(sandwich(view, true));
    for (int j = 0; j < nd; ++j)
      if (j != u) HP_TRY(oneway_view(view, j, xb[j], P.n));
    return HP_OK;
  };
  for (int comp = 0; comp < P.ncomp; ++comp) {
    bool first = true;
    for (int j = nd - 1; j >= 0; --j) {
      if (j == u) continue;
      HP_TRY(oneway(comp, j, xf[j], first));
      first = false;
    }
    HP_TRY(sandwich(work(comp), false));
    // bounded-axis terms from psi's array before the backward passes change it
    for (const DerivTerm& t : terms)
      if (t.comp == comp && t.axis != u) HP_TRY(bounded_term(comp, t.axis, t.dst, t.sign));
    for (int j = 0; j < nd; ++j) {
      if (j == u) continue;
      HP_TRY(oneway(comp, j, xb[j], false));
    }
    for (const DerivTerm& t : terms)
      if (t.comp == comp && t.axis == u) HP_TRY(free_term(comp, t.dst, t.sign));
  }
  add_second_terms(P, es, out);
  // the passes along Dirichlet / Neumann axes on the wavefront kernels where
  // their lengths allow (the free axis and Hartley axes stay general)
  if (bounded_fast_ok(p, P, L))
    for (size_t i = first_pass; i < out.size(); ++i) HP_TRY(to_fast_r2r(p, out[i].a));
  return HP_OK;
}

hp_status build_passes(hp_plan p, Problem& P, bool adjoint, std::vector<PassRec>& out) {
  if (P.d.bc == HP_UNBOUNDED) {
    if (P.nd < 3) return passes_unbounded_low(p, P, adjoint, out);
    if (fast_unbounded_ok(p, P)) return passes_unbounded_fast(p, P, adjoint, out);
    return passes_unbounded(p, P, adjoint, out);
  }
  if (adjoint) return fail(p, HP_E_UNSUPPORTED, "adjoint solve is provided for unbounded plans");
  if (P.d.bc == HP_PERIODIC && P.fast_periodic) return passes_unbounded_fast(p, P, false, out);
  if (P.d.bc == HP_PERIODIC) return passes_periodic(p, P, out);
  if (P.free_axis >= 0) return passes_semi(p, P, out);
  return passes_bounded(p, P, out);
}

// Algorithmic bytes: every pass reads its stored input and writes its stored
// output once; the Green's octant is read once.
double model_bytes(hp_plan p, const std::vector<PassRec>& ps) {
  double b = 0.0;
  const double es = (double)p->es;
  for (auto& r : ps) {
    if (r.bytes >= 0.0) {
      b += r.bytes;
      continue;
    }
    const PassArgs& a = r.a;
    const double pencils = (double)a.Np * a.No;
    auto elem_in = [&](int x) {
      return (x == X_C2C_F || x == X_C2C_B || x == X_C2R) ? 2 * es : es;
    };
    auto elem_out = [&](int x) {
      return (x == X_C2C_F || x == X_C2C_B || x == X_R2C) ? 2 * es : es;
    };
    int nin_f, nout_f;
    if (a.kind == PK_SANDWICH && a.diff != D_NONE) {
      nin_f = 0;
      for (int f = 0; f < a.n_in; ++f) nin_f += a.in[f] ? 1 : 0;
      nout_f = a.n_out;
    } else {
      nin_f = 0;
      for (int f = 0; f < r.grid_y; ++f) nin_f += a.in[f] ? 1 : 0;
      nout_f = nin_f;
    }
    const int xb = a.kind == PK_SANDWICH ? a.xb : a.xf;
    b += pencils * a.nin * elem_in(a.xf) * nin_f + pencils * a.nout * elem_out(xb) * nout_f;
    if (a.mult == M_GREEN)
      b += (double)(a.gM[0] / 2 + 1) * (a.gM[1] / 2 + 1) * (a.gM[2] / 2 + 1) * es;
  }
  return b;
}

const char* pass_name(const PassArgs& a) {
  static const char* fast_names[] = {"",       "r2c_z",      "fwd_y",       "sandwich_x", "inv_y",
                                     "c2r_z",  "r2r_contig", "r2r_strided", "r2r_sandwich",
                                     "grad_prep", "add", "small2d"};
  constexpr int nfast = (int)(sizeof(fast_names) / sizeof(fast_names[0]));
  if (a.fast > 0 && a.fast < nfast) return fast_names[a.fast];
  if (a.fast) return "wavefront";
  if (a.kind == PK_SANDWICH) return "sandwich";
  switch (a.xf) {
    case X_C2C_F: return "c2c_fwd";
    case X_C2C_B: return "c2c_inv";
    case X_R2C: return "r2c";
    case X_C2R: return "c2r";
    default: return "r2r";
  }
}

hp_status next_event(hp_plan p, hipEvent_t* e) {
  if (p->ev_used == p->ev_pool.size()) {
    hipEvent_t n;
    HP_HIP(p, hipEventCreate(&n));
    p->ev_pool.push_back(n);
  }
  *e = p->ev_pool[p->ev_used++];
  return HP_OK;
}

hp_status run_passes(hp_plan p, const std::vector<PassRec>& ps) {
  std::vector<PassEvents> evs;
  if (p->timing) {
    p->pass_bytes.clear();
    p->pass_names.clear();
  }
  for (size_t i = 0; i < ps.size(); ++i) {
    const PassRec& r = ps[i];
    // every pass, or only pass timing_pass (one event pair per solve)
    const bool rec = p->timing && (p->timing_pass < 0 || p->timing_pass == (int)i);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rec) {
      HP_TRY(next_event(p, &e0));
      HP_TRY(next_event(p, &e1));
      HP_HIP(p, hipEventRecord(e0, p->stream));
    }
    hipError_t e = r.a.fast >= FAST_R2R_C ? launch_bounded(r.a, p->prec, p->stream)
                   : r.a.fast               ? launch_fast(r.a, p->prec, r.grid_y, p->stream)
                                            : launch_pass(r.a, p->prec, r.grid_y, p->stream);
    if (e != hipSuccess) return fail(p, HP_E_DEVICE, std::string("pass launch: ") + hipGetErrorString(e));
    if (rec) {
      HP_HIP(p, hipEventRecord(e1, p->stream));
      evs.push_back({(int)i, e0, e1});
    }
    if (p->timing) {
      p->pass_bytes.push_back(model_bytes(p, std::vector<PassRec>{r}));
      p->pass_names.push_back(pass_name(r.a));
    }
  }
  if (p->timing) p->ev_solves.push_back(evs);
  return HP_OK;
}

// Arguments of the zero-mode reduction of component c: the boundary terms of
// the first pass, DCT-I end weights (trap) and the total weight W, the k = 0
// coefficient of the forward transform of a field of ones.
void zero_mode_setup(const Problem& P, int c, PassArgs& a, int trap[3], double* W) {
  a = PassArgs{};
  a.ax_j = 0; a.ax_p = 1; a.ax_o = 2;
  for (int b = 0; b < 3; ++b) a.nunk[b] = b < P.nd ? P.n[b] : 0;
  fill_face_terms(P, c, a);
  trap[0] = trap[1] = trap[2] = 0;
  *W = 1.0;
  for (int b = 0; b < P.nd; ++b) {
    trap[b] = (axis_bc(P.d, b) == HP_NEUMANN && P.d.grid == HP_REGULAR) ? 1 : 0;
    *W *= trap[b] ? (double)(P.n[b] - 1) : (double)P.n[b];
  }
}

// GRAD / CURL / DIV of a Dirichlet / Neumann solve with boundary values: FD2
// differences of psi on the output points (after the boundary-node fill),
// closed at the faces by the boundary rules (launch_fd_deriv).
hp_status fd_derivatives(hp_plan p, const Problem& P) {
  const int nd = P.nd;
  FdArgs base{};
  base.nd = nd;
  for (int a = 0; a < 3; ++a) {
    base.N[a] = a < nd ? P.nout[a] : 1;
    base.h[a] = P.h[a];
  }
  for (int a = 0; a < 3; ++a) {
    const int b = a < nd ? axis_bc(P.d, a) : HP_NEUMANN;
    base.bc[a] = b == HP_PERIODIC ? FD_PERIODIC : (b == HP_DIRICHLET ? FD_DIRICHLET : FD_NEUMANN);
  }
  base.regular = P.d.grid == HP_REGULAR;
  auto term = [&](int comp, int axis, double sign) {
    FdTerm t{};
    t.psi = P.out[comp];
    const bool faces = axis_bc(P.d, axis) != HP_PERIODIC;
    t.g_lo = faces ? P.face[axis][0][comp] : nullptr;
    t.g_hi = faces ? P.face[axis][1][comp] : nullptr;
    t.axis = axis;
    t.sign = sign;
    return t;
  };
  auto launch = [&](int slot, std::initializer_list<FdTerm> ts) -> hp_status {
    FdArgs a = base;
    a.out = P.der[slot];
    for (const FdTerm& t : ts) a.t[a.nterm++] = t;
    HP_HIP(p, launch_fd_deriv(a, p->prec, p->stream));
    return HP_OK;
  };
  switch (P.d.diff) {
    case HP_D_GRAD:
      for (int g = 0; g < nd; ++g) HP_TRY(launch(g, {term(0, g, 1.0)}));
      break;
    case HP_D_CURL:
      if (nd == 2) {  // (d_y psi, -d_x psi)
        HP_TRY(launch(0, {term(0, 1, 1.0)}));
        HP_TRY(launch(1, {term(0, 0, -1.0)}));
      } else {
        HP_TRY(launch(0, {term(2, 1, 1.0), term(1, 2, -1.0)}));
        HP_TRY(launch(1, {term(0, 2, 1.0), term(2, 0, -1.0)}));
        HP_TRY(launch(2, {term(1, 0, 1.0), term(0, 1, -1.0)}));
      }
      break;
    case HP_D_DIV:
      HP_TRY(launch(0, {term(0, 0, 1.0), term(1, 1, 1.0), term(2, 2, 1.0)}));
      break;
    default:
      return fail(p, HP_E_UNSUPPORTED, "derivative with boundary values");
  }
  return HP_OK;
}

Problem* get_problem(hp_plan p, int problem) {
  if (!p || problem < 0 || problem >= (int)p->probs.size()) return nullptr;
  return &p->probs[problem];
}

hp_status copy_in(hp_plan p, const void* src, size_t bytes, int on_device, void** own,
                  const void** slot) {
  if (on_device) {
    *slot = src;
    return HP_OK;
  }
  if (!*own) HP_TRY(dev_alloc(p, bytes, own));
  HP_HIP(p, hipMemcpyAsync(*own, src, bytes, hipMemcpyHostToDevice, p->stream));
  HP_HIP(p, hipStreamSynchronize(p->stream));
  *slot = *own;
  return HP_OK;
}

hp_status create(const hp_desc* descs, int count, hp_stream stream, hp_plan* out, bool batched) {
  if (!out) return fail(nullptr, HP_E_ARG, "null plan pointer");
  *out = nullptr;
  if (count < 1) return fail(nullptr, HP_E_ARG, "count must be >= 1");
  if (!descs) return fail(nullptr, HP_E_ARG, "null descriptor");
  for (int i = 0; i < count; ++i) HP_TRY(validate(&descs[i]));
  if (batched) {
    const hp_desc& d0 = descs[0];
    for (int i = 1; i < count; ++i) {
      const hp_desc& d = descs[i];
      if (d.bc != d0.bc || d.grid != d0.grid || d.kernel != d0.kernel || d.diff != d0.diff ||
          d.prec != d0.prec || d.ndim != d0.ndim || d.ncomp != d0.ncomp)
        return fail(nullptr, HP_E_ARG, "batched problems must share bc/grid/kernel/diff/prec/ndim/ncomp");
    }
    if (d0.bc != HP_DIRICHLET && d0.bc != HP_NEUMANN)
      return fail(nullptr, HP_E_UNSUPPORTED, "batched plans take Dirichlet or Neumann problems");
    if (d0.inhomogeneous)
      return fail(nullptr, HP_E_UNSUPPORTED, "batched plans take homogeneous problems");
    if (d0.ndim != 3)
      return fail(nullptr, HP_E_UNSUPPORTED, "batched plans take 3D problems");
    if (d0.diff != HP_D_NONE)
      return fail(nullptr, HP_E_UNSUPPORTED, "batched plans take no derivatives");
  }
  hp_plan p = new (std::nothrow) hp_plan_s();
  if (!p) return fail(nullptr, HP_E_NOMEM, "host allocation failed");
  p->stream = (hipStream_t)stream;
  p->prec = descs[0].prec;
  p->es = p->prec == 0 ? 4 : 8;
  p->batched = batched;
  if (const char* f = std::getenv("HP_FAULT_ALLOC")) p->fail_alloc_at = std::atoi(f);
  p->probs.resize(count);
  hp_status st = HP_OK;
  for (int i = 0; i < count && st == HP_OK; ++i) {
    p->probs[i].d = descs[i];
    st = setup_problem(p, p->probs[i]);
  }
  if (st == HP_OK && !batched) {
    // dry build: every pass must fit (strides / LDS), with placeholder bindings
    std::vector<PassRec> dry;
    st = build_passes(p, p->probs[0], false, dry);
  }
  if (st != HP_OK) {
    g_create_error = p->err;
    for (void* a : p->allocs) (void)hipFree(a);
    delete p;
    return st;
  }
  *out = p;
  return HP_OK;
}

}  // namespace

namespace hp {
hp_status plan_fail(hp_plan p, hp_status s, const std::string& msg) { return fail(p, s, msg); }
hp_status plan_alloc(hp_plan p, size_t bytes, void** out) { return dev_alloc(p, bytes, out); }
void plan_free(hp_plan p, void* ptr) {
  if (!ptr) return;
  auto it = std::find(p->allocs.begin(), p->allocs.end(), ptr);
  if (it == p->allocs.end()) return;
  p->allocs.erase(it);
  (void)hipFree(ptr);
}
hp_status plan_outputs(hp_plan p, Problem& P) { return ensure_outputs(p, P); }
hp_status plan_fast_twiddles(hp_plan p, int L, const void** out) { return fast_twiddles(p, L, out); }
hp_status launch_rec(hp_plan p, const PassRec& r) {
  hipError_t e = r.a.fast >= FAST_R2R_C ? launch_bounded(r.a, p->prec, p->stream)
                 : r.a.fast               ? launch_fast(r.a, p->prec, r.grid_y, p->stream)
                                          : launch_pass(r.a, p->prec, r.grid_y, p->stream);
  if (e != hipSuccess) return fail(p, HP_E_DEVICE, std::string("pass launch: ") + hipGetErrorString(e));
  return HP_OK;
}
// A radix order the general kernels run: radices 2, 3, 4, 5, 8 whose product is L.
bool radix_ok(int L, const int* radix, int nstage) {
  if (nstage < 1 || nstage > kMaxStages) return false;
  long long prod = 1;
  for (int s = 0; s < nstage; ++s) {
    const int r = radix[s];
    if (r != 2 && r != 3 && r != 4 && r != 5 && r != 8) return false;
    prod *= r;
  }
  return prod == L;
}
hp_status passes_for(hp_plan p, Problem& P, bool adjoint, std::vector<PassRec>& out) {
  return build_passes(p, P, adjoint, out);
}
double passes_model_bytes(hp_plan p, const std::vector<PassRec>& ps) { return model_bytes(p, ps); }
}  // namespace hp

extern "C" {

const char* hp_status_string(hp_status s) {
  const int i = -(int)s;
  if (i < 0 || i > 5) return "unknown status";
  return kStatusText[i];
}

const char* hp_last_error(hp_plan plan) {
  if (!plan) return g_create_error.c_str();
  return plan->err.c_str();
}

hp_status hp_plan_create(const hp_desc* desc, hp_stream stream, hp_plan* out) {
  return create(desc, 1, stream, out, false);
}

hp_status hp_input_shape(hp_plan plan, int problem, int64_t shape[3]) {
  Problem* P = get_problem(plan, problem);
  if (!P || !shape) return fail(plan, HP_E_ARG, "bad problem index or shape pointer");
  for (int a = 0; a < 3; ++a) shape[a] = P->n[a];
  return HP_OK;
}

hp_status hp_output_shape(hp_plan plan, int problem, int64_t shape[3]) {
  Problem* P = get_problem(plan, problem);
  if (!P || !shape) return fail(plan, HP_E_ARG, "bad problem index or shape pointer");
  for (int a = 0; a < 3; ++a) shape[a] = P->nout[a];
  return HP_OK;
}

hp_status hp_set_input(hp_plan plan, int problem, int comp, const void* f, int on_device) {
  Problem* P = get_problem(plan, problem);
  if (!P) return fail(plan, HP_E_ARG, "bad plan or problem index");
  if (comp < 0 || comp >= P->ncomp) return fail(plan, HP_E_ARG, "bad component");
  if (!f) {
    P->in[comp] = nullptr;
    return HP_OK;
  }
  const size_t bytes = count_elems(P->n, P->nd) * plan->es;
  return copy_in(plan, f, bytes, on_device, &P->own_in[comp], &P->in[comp]);
}

hp_status hp_set_boundary(hp_plan plan, int problem, int axis, int side, int comp, const void* g,
                          int on_device) {
  Problem* P = get_problem(plan, problem);
  if (!P) return fail(plan, HP_E_ARG, "bad plan or problem index");
  if (!P->d.inhomogeneous) return fail(plan, HP_E_STATE, "plan was created homogeneous");
  if (axis < 0 || axis >= P->nd || side < 0 || side > 1 || comp < 0 || comp >= P->ncomp)
    return fail(plan, HP_E_ARG, "bad axis, side or component");
  if (!g) {
    P->face[axis][side][comp] = nullptr;
    return HP_OK;
  }
  if (axis_bc(P->d, axis) == HP_PERIODIC || axis_bc(P->d, axis) == HP_UNBOUNDED)
    return fail(plan, HP_E_ARG, "a periodic or free axis has no faces");
  size_t cnt = 1;
  for (int b = 0; b < P->nd; ++b)
    if (b != axis) cnt *= (size_t)P->nout[b];
  return copy_in(plan, g, cnt * plan->es, on_device, &P->own_face[axis][side][comp],
                 &P->face[axis][side][comp]);
}

hp_status hp_bind_output(hp_plan plan, int problem, int comp, void* psi) {
  Problem* P = get_problem(plan, problem);
  if (!P) return fail(plan, HP_E_ARG, "bad plan or problem index");
  if (comp < 0 || comp >= P->ncomp) return fail(plan, HP_E_ARG, "bad component");
  P->out[comp] = psi ? psi : P->own_out[comp];
  return HP_OK;
}

hp_status hp_bind_gradient(hp_plan plan, int problem, int comp, void* out) {
  Problem* P = get_problem(plan, problem);
  if (!P) return fail(plan, HP_E_ARG, "bad plan or problem index");
  if (comp < 0 || comp >= P->nder) return fail(plan, HP_E_ARG, "bad derivative component");
  P->der[comp] = out ? out : P->own_der[comp];
  return HP_OK;
}

hp_status hp_solve(hp_plan plan) {
  if (!plan) return HP_E_ARG;
  if (plan->batched) return hp::batched_solve(plan);
  Problem& P = plan->probs[0];
  for (int c = 0; c < P.ncomp; ++c)
    if (!P.in[c]) return fail(plan, HP_E_STATE, "input component " + std::to_string(c) + " not set");
  HP_TRY(ensure_outputs(plan, P));
  std::vector<PassRec> ps;
  HP_TRY(build_passes(plan, P, false, ps));
  HP_TRY(run_passes(plan, ps));
  if (dreg_axes(P.d)) {
    for (int c = 0; c < P.ncomp; ++c) {
      const void* faces[3][2] = {};
      for (int a = 0; a < P.nd; ++a)
        for (int s = 0; s < 2; ++s) faces[a][s] = P.d.inhomogeneous ? P.face[a][s][c] : nullptr;
      int N[3] = {1, 1, 1};
      for (int a = 0; a < P.nd; ++a) N[3 - P.nd + a] = P.nout[a];
      // the fill kernel indexes logical axes; pass dims in logical order
      int Nl[3] = {P.nout[0], P.nd > 1 ? P.nout[1] : 1, P.nd > 2 ? P.nout[2] : 1};
      (void)N;
      HP_HIP(plan, launch_dirichlet_fill(P.out[c], Nl, P.nd, dreg_axes(P.d), faces, plan->prec,
                                         plan->stream));
    }
  }
  if (P.d.inhomogeneous && P.nder > 0) HP_TRY(fd_derivatives(plan, P));
  plan->solved = true;
  return HP_OK;
}

hp_status hp_solve_adjoint(hp_plan plan) {
  if (!plan) return HP_E_ARG;
  if (plan->batched) return fail(plan, HP_E_UNSUPPORTED, "adjoint of a batched plan");
  Problem& P = plan->probs[0];
  if (P.d.bc != HP_UNBOUNDED) return fail(plan, HP_E_UNSUPPORTED, "adjoint solve is provided for unbounded plans");
  for (int c = 0; c < P.ncomp; ++c) {
    if (!P.in[c] || P.in[c] == P.own_in[c])
      return fail(plan, HP_E_STATE, "adjoint needs device buffers bound with hp_set_input");
  }
  // unbound upstream gradients are zero: use null sources
  Problem Q = P;
  for (int c = 0; c < P.ncomp; ++c)
    if (Q.out[c] == P.own_out[c]) Q.out[c] = nullptr;
  for (int c = 0; c < P.nder; ++c)
    if (Q.der[c] == P.own_der[c]) Q.der[c] = nullptr;
  bool any = false;
  for (int c = 0; c < P.ncomp; ++c) any |= Q.out[c] != nullptr;
  for (int c = 0; c < P.nder; ++c) any |= Q.der[c] != nullptr;
  if (!any) return fail(plan, HP_E_STATE, "adjoint needs at least one bound upstream gradient");
  std::vector<PassRec> ps;
  HP_TRY(build_passes(plan, Q, true, ps));
  HP_TRY(run_passes(plan, ps));
  return HP_OK;
}

static hp_status get_field(hp_plan plan, int problem, int comp, void* dst, int on_device, bool der) {
  Problem* P = get_problem(plan, problem);
  if (!P) return fail(plan, HP_E_ARG, "bad plan or problem index");
  if (!plan->solved) return fail(plan, HP_E_STATE, "no solve has run");
  if (!dst) return fail(plan, HP_E_ARG, "null destination");
  void* srcp;
  if (der) {
    if (comp < 0 || comp >= P->nder) return fail(plan, HP_E_ARG, "bad derivative component");
    srcp = P->der[comp];
  } else {
    if (comp < 0 || comp >= P->ncomp) return fail(plan, HP_E_ARG, "bad component");
    srcp = P->out[comp];
  }
  if (!srcp) return fail(plan, HP_E_STATE, "output not available");
  const size_t bytes = count_elems(P->nout, P->nd) * plan->es;
  if (on_device) {
    if (dst == srcp) return HP_OK;
    HP_HIP(plan, hipMemcpyAsync(dst, srcp, bytes, hipMemcpyDeviceToDevice, plan->stream));
  } else {
    HP_HIP(plan, hipMemcpyAsync(dst, srcp, bytes, hipMemcpyDeviceToHost, plan->stream));
    HP_HIP(plan, hipStreamSynchronize(plan->stream));
  }
  return HP_OK;
}

hp_status hp_get_output(hp_plan plan, int problem, int comp, void* dst, int on_device) {
  return get_field(plan, problem, comp, dst, on_device, false);
}

hp_status hp_get_gradient(hp_plan plan, int problem, int comp, void* dst, int on_device) {
  return get_field(plan, problem, comp, dst, on_device, true);
}

hp_status hp_set_timing(hp_plan plan, int enable) {
  if (!plan || enable < 0) return HP_E_ARG;
  plan->timing = enable != 0;
  if (enable) plan->timing_pass = enable == 1 ? -1 : enable - 2;
  return HP_OK;
}

hp_status hp_pass_stats(hp_plan plan, int max, int* npass, double* ms, double* bytes,
                        const char** names) {
  if (!plan || max < 0) return HP_E_ARG;
  HP_HIP(plan, hipStreamSynchronize(plan->stream));
  const size_t np = plan->pass_names.size();
  if (npass) *npass = (int)np;
  std::vector<double> acc(np, 0.0);
  std::vector<size_t> cnt(np, 0);
  for (auto& evs : plan->ev_solves)
    for (const PassEvents& pe : evs) {
      if (pe.pass < 0 || (size_t)pe.pass >= np) continue;
      float t = 0.f;
      HP_HIP(plan, hipEventElapsedTime(&t, pe.e0, pe.e1));
      acc[pe.pass] += t;
      ++cnt[pe.pass];
    }
  for (size_t i = 0; i < np && (int)i < max; ++i) {
    if (ms) ms[i] = cnt[i] ? acc[i] / cnt[i] : 0.0;
    if (bytes) bytes[i] = plan->pass_bytes[i];
    if (names) names[i] = plan->pass_names[i];
  }
  plan->ev_solves.clear();
  plan->ev_used = 0;
  return HP_OK;
}

hp_status hp_query(hp_plan plan, int what, double* value) {
  if (!plan || !value) return HP_E_ARG;
  Problem& P = plan->probs[0];
  switch (what) {
    case HP_Q_WORKSPACE_BYTES:
      *value = (double)plan->ws_bytes;
      return HP_OK;
    case HP_Q_NUM_OUTPUTS:
      *value = P.ncomp + P.nder;
      return HP_OK;
    case HP_Q_NUM_DERIVS:
      *value = P.nder;
      return HP_OK;
    case HP_Q_BATCH_ERROR: {
      if (!plan->batched) return fail(plan, HP_E_ARG, "not a batched plan");
      int err = 0;
      HP_HIP(plan, hipStreamSynchronize(plan->stream));
      HP_HIP(plan, hipMemcpy(&err, plan->batch_counters + plan->batch_ncounters, sizeof(int),
                             hipMemcpyDeviceToHost));
      *value = err;
      return HP_OK;
    }
    case HP_Q_TUNED_PASSES:
      *value = plan->tuned_passes;
      return HP_OK;
    case HP_Q_TUNE_DEFAULT_MS:
      *value = plan->tune_default_ms;
      return HP_OK;
    case HP_Q_TUNE_BEST_MS:
      *value = plan->tune_best_ms;
      return HP_OK;
    case HP_Q_ZERO_MODE: {
      if (plan->batched) return fail(plan, HP_E_ARG, "zero mode: single-problem plans");
      *value = 0.0;
      if (!has_zero_mode(P.d)) return HP_OK;
      const int nb = kZeroModeBlocks;
      if (!plan->zm_partial) HP_TRY(dev_alloc(plan, nb * sizeof(double), (void**)&plan->zm_partial));
      double best = 0.0;
      for (int c = 0; c < P.ncomp; ++c) {
        if (!P.in[c]) return fail(plan, HP_E_STATE, "input component " + std::to_string(c) + " not set");
        PassArgs a;
        int trap[3];
        double W;
        zero_mode_setup(P, c, a, trap, &W);
        HP_HIP(plan, launch_zero_mode(a, P.in[c], P.n, trap, plan->zm_partial, nb, plan->prec, plan->stream));
        double part[nb];
        HP_HIP(plan, hipMemcpyAsync(part, plan->zm_partial, sizeof part, hipMemcpyDeviceToHost, plan->stream));
        HP_HIP(plan, hipStreamSynchronize(plan->stream));
        double sum = 0.0;
        for (int i = 0; i < nb; ++i) sum += part[i];
        const double m = sum / W;
        if (c == 0 || std::fabs(m) > std::fabs(best)) best = m;
      }
      *value = best;
      return HP_OK;
    }
    case HP_Q_BATCH_TILES:
      if (!plan->batched) return fail(plan, HP_E_ARG, "not a batched plan");
      *value = batch_tiles_of(plan);
      return HP_OK;
    case HP_Q_BATCH_KERNEL:
      if (!plan->batched) return fail(plan, HP_E_ARG, "not a batched plan");
      *value = (double)plan->batch_wf;
      return HP_OK;
    case HP_Q_MODEL_BYTES:
    case HP_Q_NUM_PASSES: {
      if (plan->batched) {
        *value = what == HP_Q_MODEL_BYTES ? model_bytes(plan, plan->batch_passes)
                                          : (double)plan->batch_passes.size();
        return HP_OK;
      }
      // model with placeholder (non-null) bindings
      Problem Q = P;
      static char dummy;
      for (int c = 0; c < Q.ncomp; ++c) if (!Q.in[c]) Q.in[c] = &dummy;
      for (int c = 0; c < Q.ncomp; ++c) if (!Q.out[c]) Q.out[c] = &dummy;
      for (int c = 0; c < Q.nder; ++c) if (!Q.der[c]) Q.der[c] = &dummy;
      std::vector<PassRec> ps;
      HP_TRY(build_passes(plan, Q, false, ps));
      *value = what == HP_Q_MODEL_BYTES ? model_bytes(plan, ps) : (double)ps.size();
      return HP_OK;
    }
    default:
      return fail(plan, HP_E_ARG, "unknown query");
  }
}

hp_status hp_device_copy(const void* src, void* dst, size_t bytes, hp_stream stream) {
  if (bytes == 0) return HP_OK;
  if (!src || !dst || ((uintptr_t)src % 16) || ((uintptr_t)dst % 16)) return HP_E_ARG;
  if (launch_copy(src, dst, bytes, (hipStream_t)stream) != hipSuccess) return HP_E_DEVICE;
  return HP_OK;
}

hp_status hp_zero_mode_noalloc(hp_plan plan, double* out) {
  if (!plan || !out) return HP_E_ARG;
  if (plan->batched) return fail(plan, HP_E_ARG, "zero mode: single-problem plans");
  Problem& P = plan->probs[0];
  if (P.ncomp > kZeroModeMaxComp)
    return fail(plan, HP_E_UNSUPPORTED, "zero mode without allocation: at most " +
                                            std::to_string(kZeroModeMaxComp) + " components");
  PassArgs a[kZeroModeMaxComp];
  const void* f[kZeroModeMaxComp] = {};
  double W[kZeroModeMaxComp] = {0.0, 0.0, 0.0};
  int trap[3] = {0, 0, 0};
  const bool has_zero = has_zero_mode(P.d);
  for (int c = 0; c < P.ncomp; ++c) {
    if (!P.in[c]) return fail(plan, HP_E_STATE, "input component " + std::to_string(c) + " not set");
    f[c] = P.in[c];
    if (has_zero) zero_mode_setup(P, c, a[c], trap, &W[c]);
    else a[c] = PassArgs{};  // W = 0: only zeros are written
  }
  HP_HIP(plan, launch_zero_mode_noalloc(a, f, P.ncomp, P.n, trap, W, out, plan->prec, plan->stream));
  return HP_OK;
}

hp_status hp_plan_destroy(hp_plan plan) {
  if (!plan) return HP_E_ARG;
  (void)hipStreamSynchronize(plan->stream);
  for (hipEvent_t e : plan->ev_pool) (void)hipEventDestroy(e);
  for (hipStream_t st : plan->batch_aux) (void)hipStreamSynchronize(st);
  for (hipEvent_t e : plan->batch_ev) (void)hipEventDestroy(e);
  for (hipStream_t st : plan->batch_aux) (void)hipStreamDestroy(st);
  for (void* a : plan->allocs) (void)hipFree(a);
  delete plan;
  return HP_OK;
}

}  // extern "C"

extern "C" hp_status hp_plan_create_batched(const hp_desc* descs, int count, hp_stream stream,
                                            hp_plan* out) {
  hp_status s = create(descs, count, stream, out, true);
  if (s != HP_OK) return s;
  s = hp::batched_setup(*out);
  if (s != HP_OK) {
    g_create_error = (*out)->err;
    hp_plan_destroy(*out);
    *out = nullptr;
  }
  return s;
}
