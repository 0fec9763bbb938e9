// Bounded (Dirichlet / Neumann) passes with one FFT per wavefront, for
// power-of-two transform lengths L = 64 .. 1024 (hp_wavefft.hpp).
//
// The real-to-real transforms of Table 1 (DST-I/II/III, DCT-I/II/III) run as
// one complex FFT of length L on a pair of real pencils packed as a + ib,
// after extending each pencil to the symmetry of its transform:
//   DST-I   L = 2(n+1): [0, x_0..x_{n-1}, 0, -x_{n-1}..-x_0]
//   DCT-I   L = 2(n-1): [x_0..x_{n-1}, x_{n-2}..x_1]
//   DCT-II  L = 2n:     [x_0..x_{n-1}, x_{n-1}..x_0] (DST-II: (-1)^j x_j)
//   DCT-III L = 2n:     e^{+i pi j / 2n} (a_j + i b_j) below n, 0 at n, the
//                       conjugate twist above (inverse FFT; DST-III reversed)
// Every output of these transforms is read from a single FFT bin (with the
// quarter-wave twist e^{-i pi k / 2n} for DCT-II / DST-II), and lane g holds
// bins g + G i, so the outputs stay in the lanes that computed them.
//
// Passes (the pencil descriptors are those of the general path, in place in
// the output array): contiguous one-way passes load the pencil pair straight
// into the wavefront's LDS slot; strided passes stage a tile of P pencils
// (runs of P elements along the contiguous axis) through LDS; the sandwich
// pass transforms forward, multiplies by norm / sum_a lambda_a (Table 1,
// eq. pois_spec; 0 where the sum is 0) and transforms back before the tile is
// stored.  Inhomogeneous FD2 boundary terms are added while loading.
#include "hp_device.hpp"
#include "hp_faces.hpp"
#include "hp_internal.hpp"
#include "hp_wavefft.hpp"

namespace hp {

namespace {

__device__ __forceinline__ bool r2r_inverse_fft(int x) { return x == X_DCT3 || x == X_DST3; }

// FFT input z[m] of the pair (a, b) for transform x of n points (length L);
// get(s, w) is element s of pencil a (w = 0) or b (w = 1).
template <typename T, class Get>
__device__ __forceinline__ C2<T> r2r_build(int x, int m, int n, int L, const C2<T>* q, Get get) {
  switch (x) {
    case X_DST1:
      if (m >= 1 && m <= n) return {get(m - 1, 0), get(m - 1, 1)};
      if (m > n + 1) return {-get(L - m - 1, 0), -get(L - m - 1, 1)};
      return {(T)0, (T)0};
    case X_DCT1: {
      const int s = m < n ? m : L - m;
      return {get(s, 0), get(s, 1)};
    }
    case X_DCT2:
    case X_DST2: {
      const int s = m < n ? m : L - 1 - m;
      C2<T> z = {get(s, 0), get(s, 1)};
      if (x == X_DST2 && (s & 1)) z = {-z.re, -z.im};
      return z;
    }
    case X_DCT3:
    case X_DST3: {
      if (m == n) return {(T)0, (T)0};
      const int s = m < n ? m : L - m;
      const int src = x == X_DST3 ? n - 1 - s : s;
      const C2<T> v = {get(src, 0), get(src, 1)};
      C2<T> w = q[s];  // e^{-i pi s / 2n}
      if (m < n) w.im = -w.im;
      return cmul(v, w);
    }
    default:
      return {(T)0, (T)0};
  }
}

// Output index carried by FFT bin m of transform x (-1: none) and the two
// real outputs (pencils a and b).
template <typename T>
__device__ __forceinline__ int r2r_extract(int x, int m, int n, C2<T> z, const C2<T>* q, T& oa,
                                           T& ob) {
  switch (x) {
    case X_DST1:
      if (m < 1 || m > n) return -1;
      oa = -z.im;
      ob = z.re;
      return m - 1;
    case X_DCT1:
    case X_DCT3:
      if (m >= n) return -1;
      oa = z.re;
      ob = z.im;
      return m;
    case X_DST3:
      if (m >= n) return -1;
      oa = (m & 1) ? -z.re : z.re;
      ob = (m & 1) ? -z.im : z.im;
      return m;
    case X_DCT2:
    case X_DST2: {
      if (m >= n) return -1;
      const C2<T> v = cmul(z, q[m]);
      oa = v.re;
      ob = v.im;
      return x == X_DST2 ? n - 1 - m : m;
    }
    default:
      return -1;
  }
}

__device__ __forceinline__ bool has_faces(const PassArgs& a) {
  bool f = false;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) f |= a.face[ax][0] != nullptr || a.face[ax][1] != nullptr;
  return f;
}

// Transform the pair held as reals by get() with transform x; on return
// v[i] holds bin g + G i.
template <typename T, int L, class Get>
__device__ __forceinline__ void r2r_fft(C2<T> (&v)[WF<L>::R0], int x, int n, C2<T>* slot, int g,
                                        const C2<T>* tw, const C2<T>* q, Get get) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G;
#pragma unroll
  for (int i = 0; i < R0; ++i) v[i] = r2r_build<T>(x, g + G * i, n, L, q, get);
  wave_sync();  // the FFT overwrites the slot the inputs may have come from
  if (r2r_inverse_fft(x)) wave_fft<T, L, true>(v, slot, 1, g, tw);
  else wave_fft<T, L, false>(v, slot, 1, g, tw);
}

// Runs f with the transform type as a compile-time constant: one branch per
// FFT (uniform per wavefront) instead of a switch per element.
template <class F>
__device__ __forceinline__ void with_xform(int x, F&& f) {
  switch (x) {
    case X_DST1: f(std::integral_constant<int, X_DST1>{}); break;
    case X_DST2: f(std::integral_constant<int, X_DST2>{}); break;
    case X_DST3: f(std::integral_constant<int, X_DST3>{}); break;
    case X_DCT1: f(std::integral_constant<int, X_DCT1>{}); break;
    case X_DCT2: f(std::integral_constant<int, X_DCT2>{}); break;
    default: f(std::integral_constant<int, X_DCT3>{}); break;
  }
}

// Backward transform of the Table 1 pair that starts with forward type x.
__host__ __device__ constexpr int r2r_partner(int x) {
  return x == X_DST2 ? X_DST3 : (x == X_DCT2 ? X_DCT3 : x);
}

// Multiplier norm / (sum of the eigenvalues) at spectral index k along the
// pencil axis, given the eigenvalue sum `rest` of the other axes.
// (the eigenvalue sum is formed in FP64; an FP32 plan divides in FP32)
template <typename T>
__device__ __forceinline__ T eigen_mult(const PassArgs& a, int k, double rest) {
  const double lam = a.lam[a.ax_j][k] + rest;
  if (lam == 0.0) return (T)0;
  return (T)a.norm / (T)lam;
}

__device__ __forceinline__ double eigen_rest(const PassArgs& a, int p, int o) {
  double r = 0.0;
  if (a.ax_p >= 0) r += a.lam[a.ax_p][p];
  if (a.ax_o >= 0) r += a.lam[a.ax_o][o];
  return r;
}

}  // namespace

constexpr int kR2RContigWaves = 4;

// ----------------------------------------------- contiguous one-way pass
// Pairs (p, p+1) of pencils at one o; the pencil axis is unit stride.
template <typename T, int L>
__global__ void __launch_bounds__(64 * kR2RContigWaves) kb_contig(const PassArgs a) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G, PPW = WF<L>::PPW;
  constexpr int NT = 64 * kR2RContigWaves;
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = a.n;
  C2<T>* tw = (C2<T>*)smem;
  C2<T>* q = tw + L;
  C2<T>* slots = q + n;
  for (int m = threadIdx.x; m < L; m += NT) tw[m] = ((const C2<T>*)a.tw)[m];
  if (a.qtw)
    for (int m = threadIdx.x; m < n; m += NT) q[m] = ((const C2<T>*)a.qtw)[m];
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int qq = lane / G, g = lane % G;
  C2<T>* slot = slots + (wave * PPW + qq) * slot_len(L);
  T* R = (T*)slot;  // the pair's reals: a at R[0..n), b at R[n..2n)
  const int pairs_p = (a.Np + 1) / 2;
  const long long total = (long long)pairs_p * a.No;
  const long long pr = ((long long)blockIdx.x * kR2RContigWaves + wave) * PPW + qq;
  const bool valid = pr < total;
  const int o = valid ? (int)(pr / pairs_p) : 0;
  const int pa = valid ? 2 * (int)(pr % pairs_p) : 0;
  const bool vb = valid && pa + 1 < a.Np;
  const bool faces = has_faces(a);
  const T* in = (const T*)a.in[0];
  const long long ib = (long long)o * a.in_so + (long long)pa * a.in_sp;
  for (int j = g; j < n; j += G) {
    T va = (T)0, vb_ = (T)0;
    if (valid) {
      va = in[ib + (long long)j * a.in_sj];
      if (faces) va = (T)((double)va + face_terms<T>(a, j, pa, o));
    }
    if (vb) {
      vb_ = in[ib + a.in_sp + (long long)j * a.in_sj];
      if (faces) vb_ = (T)((double)vb_ + face_terms<T>(a, j, pa + 1, o));
    }
    R[j] = va;
    R[n + j] = vb_;
  }
  wave_sync();
  T* out = (T*)a.out[0];
  const long long ob = (long long)o * a.out_so + (long long)pa * a.out_sp;
  with_xform(a.xf, [&](auto XF) {
    constexpr int X = decltype(XF)::value;
    C2<T> v[R0];
    r2r_fft<T, L>(v, X, n, slot, g, tw, q, [&](int s, int w) { return R[w * n + s]; });
#pragma unroll
    for (int i = 0; i < R0; ++i) {
      T oa, obv;
      const int k = r2r_extract<T>(X, g + G * i, n, v[i], q, oa, obv);
      if (k < 0) continue;
      if (valid) out[ob + (long long)k * a.out_sj] = oa;
      if (vb) out[ob + a.out_sp + (long long)k * a.out_sj] = obv;
    }
  });
}

// ------------------------------------------- strided one-way and sandwich
// A tile is P pencils (p0 .. p0+P-1, o) whose pencil axis is strided; the
// contiguous axis is p.  The tile [n][P] (reals) is loaded as runs of P,
// wavefront pairs transform columns (2f, 2f+1) in place in it, and it is
// stored as runs of P.  SW: sandwich (forward, multiplier, backward).
//
// PERS (persistent): a workgroup walks tiles blockIdx-strided; every thread
// loads its share of the next tile into registers before the current tile's
// FFTs and writes it to LDS after the current tile has been stored.  Chosen
// when there are many more tiles than resident workgroups.
// (Boundary terms enter in the contiguous first pass only.)
template <typename T, int L, int P, int W, bool SW, bool PERS>
__global__ void __launch_bounds__(64 * W) kb_strided(const PassArgs a) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G, PPW = WF<L>::PPW;
  constexpr int NT = 64 * W, TS = P + 1;
  constexpr int MAXN = L / 2 + 1;             // rows of a tile (n <= L/2 + 1)
  constexpr int PER = (MAXN * P + NT - 1) / NT;  // tile elements per thread
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = a.n;
  C2<T>* tw = (C2<T>*)smem;
  C2<T>* q = tw + L;
  C2<T>* slots = q + n;
  T* tile = (T*)(slots + W * PPW * slot_len(L));
  const int tiles_p = (a.Np + P - 1) / P;
  const int ntiles = tiles_p * a.No;
  int t = blockIdx.x;
  if (t >= ntiles) return;  // whole workgroup
  for (int m = threadIdx.x; m < L; m += NT) tw[m] = ((const C2<T>*)a.tw)[m];
  if (a.qtw)
    for (int m = threadIdx.x; m < n; m += NT) q[m] = ((const C2<T>*)a.qtw)[m];
  const T* in = (const T*)a.in[0];
  T* out = (T*)a.out[0];
  T pre[PER];
  auto fetch = [&](int tt) {
    const int o = tt / tiles_p, p0 = (tt % tiles_p) * P;
    const int np = min(P, a.Np - p0);
    const long long ib = (long long)o * a.in_so + (long long)p0 * a.in_sp;
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = threadIdx.x + r * NT;
      const int j = e / P, c = e - (e / P) * P;
      pre[r] = (j < n && c < np) ? in[ib + (long long)j * a.in_sj + (long long)c * a.in_sp] : (T)0;
    }
  };
  auto put = [&]() {
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = threadIdx.x + r * NT;
      const int j = e / P, c = e - (e / P) * P;
      if (j < n) tile[j * TS + c] = pre[r];
    }
  };
  if constexpr (PERS) {
    fetch(t);
    put();
  } else {
    const int o = t / tiles_p, p0 = (t % tiles_p) * P;
    const int np = min(P, a.Np - p0);
    const long long ib = (long long)o * a.in_so + (long long)p0 * a.in_sp;
    for (int e = threadIdx.x; e < n * P; e += NT) {
      const int j = e / P, c = e - (e / P) * P;
      tile[j * TS + c] = c < np ? in[ib + (long long)j * a.in_sj + (long long)c * a.in_sp] : (T)0;
    }
  }
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int qq = lane / G, g_lane = lane % G;
  C2<T>* slot = slots + (wave * PPW + qq) * slot_len(L);
  for (;;) {
    const int o = t / tiles_p, p0 = (t % tiles_p) * P;
    const int np = min(P, a.Np - p0);
    const int nxt = PERS ? t + (int)gridDim.x : ntiles;
    if (PERS && nxt < ntiles) fetch(nxt);
    // the FFT's LDS addresses depend only on the lane: keep the compiler from
    // holding them in registers across the tile loop
    int g = g_lane;
    if constexpr (PERS) asm volatile("" : "+v"(g));
    static_assert(P / 2 == W * PPW, "one pair per wavefront lane group");
    {
      const int f = wave * PPW + qq;  // pair: columns 2f, 2f + 1
      T* ca = tile + 2 * f;
      auto get = [&](int s, int w) { return ca[s * TS + w]; };
      // the sandwich's backward type is the Table 1 partner of its forward
      // type (checked at launch)
      with_xform(a.xf, [&](auto XF) {
        constexpr int XFc = decltype(XF)::value;
        constexpr int XO = SW ? r2r_partner(XFc) : XFc;
        C2<T> v[R0];
        r2r_fft<T, L>(v, XFc, n, slot, g, tw, q, get);
        if constexpr (SW) {
          // spectra times the multiplier, back into the pair's columns
          const int pa = min(p0 + 2 * f, a.Np - 1), pb = min(p0 + 2 * f + 1, a.Np - 1);
          const double ra = eigen_rest(a, pa, o), rb = eigen_rest(a, pb, o);
#pragma unroll
          for (int i = 0; i < R0; ++i) {
            T sa, sb;
            const int k = r2r_extract<T>(XFc, g + G * i, n, v[i], q, sa, sb);
            if (k < 0) continue;
            ca[k * TS] = sa * eigen_mult<T>(a, k, ra);
            ca[k * TS + 1] = sb * eigen_mult<T>(a, k, rb);
          }
          wave_sync();
          r2r_fft<T, L>(v, XO, n, slot, g, tw, q, get);
        }
        // outputs into the pair's columns (the inputs were consumed above)
#pragma unroll
        for (int i = 0; i < R0; ++i) {
          T oa, obv;
          const int k = r2r_extract<T>(XO, g + G * i, n, v[i], q, oa, obv);
          if (k < 0) continue;
          ca[k * TS] = oa;
          ca[k * TS + 1] = obv;
        }
      });
      wave_sync();  // the slot is reused by the next pair
    }
    __syncthreads();
    const long long ob = (long long)o * a.out_so + (long long)p0 * a.out_sp;
    for (int e = threadIdx.x; e < n * P; e += NT) {
      const int j = e / P, c = e - (e / P) * P;
      if (c < np) out[ob + (long long)j * a.out_sj + (long long)c * a.out_sp] = tile[j * TS + c];
    }
    t = nxt;
    if (!PERS || t >= ntiles) break;
    __syncthreads();  // the tile has been read out
    put();
    __syncthreads();
  }
}

// ---------------------------------------------------------------- launch
// Pencils per tile of the strided passes: runs of 128 bytes.
int r2r_tile(int prec) { return prec == 0 ? 32 : 16; }

// Wavefronts per strided workgroup: one per pair (PPW pairs per wavefront
// for short transforms).
constexpr int r2r_waves(int P, int ppw) { return (P / 2) / ppw; }

int r2r_lds_bytes(int fast, int L, int n, int prec) {
  const int cs = prec == 0 ? 8 : 16, es = cs / 2;
  const int R0 = L >= 1024 ? 16 : 8, ppw = 64 / (L / R0);
  const int SL = slot_len(L);
  if (fast == FAST_R2R_C) return (L + n + kR2RContigWaves * ppw * SL) * cs;
  const int P = r2r_tile(prec);
  return (L + n + r2r_waves(P, ppw) * ppw * SL) * cs + n * (P + 1) * es;
}

namespace {

template <typename T, int L>
hipError_t launch_bounded_L(const PassArgs& a, hipStream_t s) {
  constexpr int PPW = WF<L>::PPW;
  const int lds = a.lds_bytes;
  if (a.fast == FAST_R2R_C) {
    const long long pairs = (long long)((a.Np + 1) / 2) * a.No;
    const long long per_block = (long long)kR2RContigWaves * PPW;
    allow_lds<kb_contig<T, L>>();
    hipLaunchKernelGGL((kb_contig<T, L>), dim3((unsigned)((pairs + per_block - 1) / per_block)),
                       dim3(64 * kR2RContigWaves), lds, s, a);
    return hipGetLastError();
  }
  constexpr int P = sizeof(T) == 4 ? 32 : 16;
  constexpr int W = r2r_waves(P, PPW);
  if (a.P != P) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(((a.Np + P - 1) / P) * a.No));
  const int ntiles = (int)grid.x;
  if (a.fast == FAST_R2R_SW) {
    if (a.xb != r2r_partner(a.xf)) return hipErrorInvalidValue;
    allow_lds<kb_strided<T, L, P, W, true, true>>();
    const int nb = persistent_grid<kb_strided<T, L, P, W, true, true>>(64 * W, lds, ntiles);
    if (ntiles > 4 * nb && !std::getenv("HP_R2R_NOPERS")) {
      hipLaunchKernelGGL((kb_strided<T, L, P, W, true, true>), dim3(nb), dim3(64 * W), lds, s, a);
    } else {
      allow_lds<kb_strided<T, L, P, W, true, false>>();
      hipLaunchKernelGGL((kb_strided<T, L, P, W, true, false>), grid, dim3(64 * W), lds, s, a);
    }
  } else {
    allow_lds<kb_strided<T, L, P, W, false, true>>();
    const int nb = persistent_grid<kb_strided<T, L, P, W, false, true>>(64 * W, lds, ntiles);
    if (ntiles > 4 * nb) {
      hipLaunchKernelGGL((kb_strided<T, L, P, W, false, true>), dim3(nb), dim3(64 * W), lds, s, a);
    } else {
      allow_lds<kb_strided<T, L, P, W, false, false>>();
      hipLaunchKernelGGL((kb_strided<T, L, P, W, false, false>), grid, dim3(64 * W), lds, s, a);
    }
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bounded_T(const PassArgs& a, hipStream_t s) {
  switch (a.L) {
    case 64: return launch_bounded_L<T, 64>(a, s);
    case 128: return launch_bounded_L<T, 128>(a, s);
    case 256: return launch_bounded_L<T, 256>(a, s);
    case 512: return launch_bounded_L<T, 512>(a, s);
    case 1024: return launch_bounded_L<T, 1024>(a, s);
    default: return hipErrorInvalidValue;
  }
}

// Coefficients of the derivative along ax_j of a Dirichlet / Neumann solve.
// The source holds the forward-transformed right-hand side (every axis; with
// gp_eigen, dividing by the eigenvalue sum gives the coefficients u of psi)
// or already the coefficients u (axis 0 physical); d/dx of
// the sine (cosine) series is the cosine (sine) series with coefficients
// +-(pi kappa / L) u, one index over.  Written so that the backward transform
// along ax_j of the other type (DST-I -> DCT-I on the n + 2 nodes, DST-III ->
// DCT-III, DCT-III -> DST-III, DCT-I -> DST-I on the n - 2 interior nodes)
// and the usual backward transforms along the other axes evaluate it.
// One thread per output element; consecutive threads take consecutive
// elements of the last logical axis.
template <typename T>
__global__ void __launch_bounds__(256) k_grad_prep(PassArgs a) {
  const long long total = (long long)a.gp_ext[0] * a.gp_ext[1] * a.gp_ext[2];
  const T* src = (const T*)a.in[0];
  T* dst = (T*)a.out[0];
  const long long step = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += step) {
    long long r = e;
    int i[3];
    i[2] = (int)(r % a.gp_ext[2]);
    r /= a.gp_ext[2];
    i[1] = (int)(r % a.gp_ext[1]);
    i[0] = (int)(r / a.gp_ext[1]);
    bool ok = true;
    long long so = 0, dof = 0;
    double lam = 0.0;
    int kap = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      dof += (long long)i[b] * a.gp_os[b];
      const int sb = i[b] - a.gp_off[b];
      const int k = b == a.ax_j ? sb + a.gp_shift : sb;
      ok = ok && sb >= 0 && sb < a.gp_len[b] && k >= 0 && k < a.nunk[b];
      if (ok) {
        so += (long long)k * a.gp_is[b];
        if (a.lam[b]) lam += a.lam[b][k];
        if (b == a.ax_j) kap = k + a.gp_kadd;
      }
    }
    T v = (T)0;
    if (ok) {
      double m = a.gp_scale * (double)kap;
      if (a.gp_eigen) m = lam == 0.0 ? 0.0 : m * a.norm / lam;
      v = (T)m * src[so];
    }
    dst[dof] = v;
  }
}

template <typename T>
hipError_t launch_grad_prep(const PassArgs& a, hipStream_t s) {
  const long long total = (long long)a.gp_ext[0] * a.gp_ext[1] * a.gp_ext[2];
  if (total <= 0) return hipSuccess;
  const long long blocks = (total + 255) / 256;
  const int grid = (int)(blocks < 8192 ? blocks : 8192);
  hipLaunchKernelGGL(k_grad_prep<T>, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_bounded(const PassArgs& a, int prec, hipStream_t s) {
  if (a.fast == FAST_GRAD_PREP)
    return prec == 0 ? launch_grad_prep<float>(a, s) : launch_grad_prep<double>(a, s);
  if (prec == 0) return launch_bounded_T<float>(a, s);
  return launch_bounded_T<double>(a, s);
}

}  // namespace hp
