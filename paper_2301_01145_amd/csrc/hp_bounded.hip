// Bounded (Dirichlet / Neumann) passes with one FFT per wavefront, for
// transform lengths L = 64 .. 1024 (powers of two), 96 and 192
// (hp_wavefft.hpp).
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
  // every load of the pair is issued before the first is used (n <= L/2 + 1,
  // checked at launch): one memory latency per pass, not one per row
  constexpr int NJ = (L / 2 + 1 + G - 1) / G;
  T va[NJ], vbv[NJ];
  // (unconditional loads from clamped addresses: pencil pa + 1 only where it
  // exists, rows below n; the conditions apply where the values are kept)
  const long long ibb = ib + (vb ? a.in_sp : 0);
#pragma unroll
  for (int r = 0; r < NJ; ++r) {
    const long long jo = (long long)min(g + G * r, n - 1) * a.in_sj;
    va[r] = in[ib + jo];
    vbv[r] = in[ibb + jo];
  }
  if (faces) {
#pragma unroll
    for (int r = 0; r < NJ; ++r) {
      const int j = g + G * r;
      if (j < n && valid) va[r] = (T)((double)va[r] + face_terms<T>(a, j, pa, o));
      if (j < n && vb) vbv[r] = (T)((double)vbv[r] + face_terms<T>(a, j, pa + 1, o));
    }
  }
#pragma unroll
  for (int r = 0; r < NJ; ++r) {
    const int j = g + G * r;
    if (j < n) {
      R[j] = valid ? va[r] : (T)0;
      R[n + j] = vb ? vbv[r] : (T)0;
    }
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
      if (valid) st_stream(&out[ob + (long long)k * a.out_sj], oa);
      if (vb) st_stream(&out[ob + a.out_sp + (long long)k * a.out_sj], obv);
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
    // unconditional loads from clamped (in-tile) addresses: no branches
    // between the loads, so all of them are in flight at once; put() drops
    // the rows beyond n and zeroes the pencils beyond np
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = threadIdx.x + r * NT;
      const int j = e / P, c = e - (e / P) * P;
      pre[r] = in[ib + (long long)min(j, n - 1) * a.in_sj + (long long)min(c, np - 1) * a.in_sp];
    }
  };
  auto put = [&](int tt) {
    const int np = min(P, a.Np - (tt % tiles_p) * P);
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int e = threadIdx.x + r * NT;
      const int j = e / P, c = e - (e / P) * P;
      if (j < n) tile[j * TS + c] = c < np ? pre[r] : (T)0;
    }
  };
  // the whole tile's loads in flight at once (registers, then LDS)
  fetch(t);
  put(t);
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
      if (c < np) st_stream(&out[ob + (long long)j * a.out_sj + (long long)c * a.out_sp], tile[j * TS + c]);
    }
    t = nxt;
    if (!PERS || t >= ntiles) break;
    __syncthreads();  // the tile has been read out
    put(t);
    __syncthreads();
  }
}

// ------------------------------------------ batched persistent solve
// Every pass of every problem of a batched plan, one persistent launch: a
// workgroup of kBatchWaves wavefronts takes work items (consecutive tiles of
// one pass of one problem) from a queue ordered pass level by pass level and
// waits for the pass it depends on (per-pass completion counters, agent-scope
// acquire / release), as the general batched kernel does.  The tile bodies
// are those of kb_contig / kb_strided with the transform length and type as
// compile-time constants:
//   contiguous pass: a tile is kBatchWaves * PPW pencil pairs (one per lane
//     group) taken in (o, pair) order;
//   strided pass / sandwich: a tile is P = 32 pencils adjacent along the
//     contiguous axis (16 pairs), transformed by W = min(P / (2 PPW),
//     kBatchWaves) wavefronts, each lane group taking P / (2 W PPW) pairs in
//     turn; the workgroup holds S = kBatchWaves / W tiles at once (one per
//     group of W wavefronts).
// LDS: twiddles [L] | quarter twists [L/2 + 1] | exchange slots | S tiles.
// Four wavefronts per workgroup keep the exchange slots small enough for
// three or four workgroups per CU at every length.
constexpr int kBatchWaves = 4;

namespace {

template <int L>
struct BW {
  static constexpr int PPW = WF<L>::PPW;
  static constexpr int P = 32;  // FP32 pencils per strided tile (128-byte runs)
  static constexpr int W = (P / 2) / PPW < kBatchWaves ? (P / 2) / PPW : kBatchWaves;
  static constexpr int PPL = (P / 2) / (W * PPW);  // pairs per lane group
  static constexpr int S = kBatchWaves / W;
  static constexpr int MAXN = L / 2 + 1;
  static constexpr int TS = P + 1;
  static_assert(W >= 1 && kBatchWaves % W == 0 && PPL * W * PPW == P / 2, "batched strided tile");
};

// The fields of a pass that the tile bodies read, as wavefront-uniform
// values.  The pass table is read with vector loads (the kernel also writes
// global memory, so the compiler cannot use scalar loads for it); passing
// each field through readfirstlane lets it live in scalar registers instead
// of vector registers for the whole item.
struct BwArgs {
  int L, fast, xf, n, Np, No;
  long long in_sj, in_sp, in_so, out_sj, out_sp, out_so;
  const float* in;
  float* out;
  const C2<float>* tw;
  const C2<float>* qtw;
  const double* lam_j;  // eigenvalues along the pencil axis (sandwich)
  const double* lam_p;  // along the tile axis (null: none)
  const double* lam_o;  // along the outer axis (null: none)
  double norm;
};

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uni(long long v) {
  const unsigned lo = (unsigned)uni((int)(v & 0xffffffffLL)), hi = (unsigned)uni((int)(v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
template <typename P>
__device__ __forceinline__ P* uni(P* p) { return (P*)uni((long long)p); }
__device__ __forceinline__ double uni(double d) { return __longlong_as_double(uni(__double_as_longlong(d))); }

__device__ __forceinline__ BwArgs bw_args(const PassArgs& a) {
  BwArgs b;
  b.L = uni(a.L);
  b.fast = uni(a.fast);
  b.xf = uni(a.xf);
  b.n = uni(a.n);
  b.Np = uni(a.Np);
  b.No = uni(a.No);
  b.in_sj = uni(a.in_sj);
  b.in_sp = uni(a.in_sp);
  b.in_so = uni(a.in_so);
  b.out_sj = uni(a.out_sj);
  b.out_sp = uni(a.out_sp);
  b.out_so = uni(a.out_so);
  b.in = uni((const float*)a.in[0]);
  b.out = uni((float*)a.out[0]);
  b.tw = uni((const C2<float>*)a.tw);
  b.qtw = uni((const C2<float>*)a.qtw);
  const int aj = uni(a.ax_j), ap = uni(a.ax_p), ao = uni(a.ax_o);
  b.lam_j = aj >= 0 ? uni(a.lam[aj]) : nullptr;
  b.lam_p = ap >= 0 ? uni(a.lam[ap]) : nullptr;
  b.lam_o = ao >= 0 ? uni(a.lam[ao]) : nullptr;
  b.norm = uni(a.norm);
  return b;
}

__device__ __forceinline__ BwArgs bw_uniform(const BwArgs& a) {
  BwArgs b;
  b.L = uni(a.L);
  b.fast = uni(a.fast);
  b.xf = uni(a.xf);
  b.n = uni(a.n);
  b.Np = uni(a.Np);
  b.No = uni(a.No);
  b.in_sj = uni(a.in_sj);
  b.in_sp = uni(a.in_sp);
  b.in_so = uni(a.in_so);
  b.out_sj = uni(a.out_sj);
  b.out_sp = uni(a.out_sp);
  b.out_so = uni(a.out_so);
  b.in = uni(a.in);
  b.out = uni(a.out);
  b.tw = uni(a.tw);
  b.qtw = uni(a.qtw);
  b.lam_j = uni(a.lam_j);
  b.lam_p = uni(a.lam_p);
  b.lam_o = uni(a.lam_o);
  b.norm = uni(a.norm);
  return b;
}

// The thread index, opaque to the optimiser: everything a tile body derives
// from it (lane splits, LDS slot addresses) is then computed inside the body
// instead of being hoisted out of the persistent loop, where the values of
// every (length, kind) body would stay live together and spill.
__device__ __forceinline__ int bw_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Load the twiddles of the pass (and the quarter-wave twists) into LDS.
template <int L>
__device__ __forceinline__ void bw_tables(const BwArgs& a, C2<float>* tw, C2<float>* q, int tid) {
  constexpr int NT = 64 * kBatchWaves;
  for (int m = tid; m < L; m += NT) tw[m] = a.tw[m];
  if (a.qtw)
    for (int m = tid; m < a.n; m += NT) q[m] = a.qtw[m];
}

template <int L, int X>
__device__ __forceinline__ void bw_contig(const BwArgs& a, unsigned char* smem, int tile, int ntile) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G, PPW = WF<L>::PPW;
  using T = float;
  const int n = a.n;
  C2<T>* tw = (C2<T>*)smem;
  C2<T>* q = tw + L;
  C2<T>* slots = q + BW<L>::MAXN;
  const int tid = bw_tid();
  bw_tables<L>(a, tw, q, tid);
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int qq = lane / G, g = lane % G;
  C2<T>* slot = slots + (wave * PPW + qq) * slot_len(L);
  T* R = (T*)slot;
  const int pairs_p = (a.Np + 1) / 2;
  const long long total = (long long)pairs_p * a.No;
  for (int k = 0; k < ntile; ++k) {
    const long long pr = ((long long)(tile + k) * kBatchWaves + wave) * PPW + qq;
    const bool valid = pr < total;
    const int o = valid ? (int)(pr / pairs_p) : 0;
    const int pa = valid ? 2 * (int)(pr % pairs_p) : 0;
    const bool vb = valid && pa + 1 < a.Np;
    const long long ib = (long long)o * a.in_so + (long long)pa * a.in_sp;
    // every load of the pair in flight at once (compile-time trip count)
    constexpr int NJ = (BW<L>::MAXN + G - 1) / G;
    T va[NJ], vbv[NJ];
#pragma unroll
    for (int r = 0; r < NJ; ++r) {
      const int j = g + r * G;
      va[r] = (valid && j < n) ? a.in[ib + (long long)j * a.in_sj] : (T)0;
      vbv[r] = (vb && j < n) ? a.in[ib + a.in_sp + (long long)j * a.in_sj] : (T)0;
    }
#pragma unroll
    for (int r = 0; r < NJ; ++r) {
      const int j = g + r * G;
      if (j < n) {
        R[j] = va[r];
        R[n + j] = vbv[r];
      }
    }
    wave_sync();
    const long long ob = (long long)o * a.out_so + (long long)pa * a.out_sp;
    C2<T> v[R0];
    r2r_fft<T, L>(v, X, n, slot, g, tw, q, [&](int s, int w) { return R[w * n + s]; });
#pragma unroll
    for (int i = 0; i < R0; ++i) {
      T oa, obv;
      const int kk = r2r_extract<T>(X, g + G * i, n, v[i], q, oa, obv);
      if (kk < 0) continue;
      if (valid) st_stream(&a.out[ob + (long long)kk * a.out_sj], oa);
      if (vb) st_stream(&a.out[ob + a.out_sp + (long long)kk * a.out_sj], obv);
    }
    wave_sync();  // the slot is reused by the next pair
  }
}

template <int L, int XF, int XO, bool SW>
__device__ __forceinline__ void bw_strided(const BwArgs& a, unsigned char* smem, int tile, int ntile) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G, PPW = WF<L>::PPW;
  constexpr int P = BW<L>::P, W = BW<L>::W, S = BW<L>::S, TS = BW<L>::TS, PPL = BW<L>::PPL;
  constexpr int MAXN = BW<L>::MAXN, NTS = 64 * W;
  using T = float;
  const int n = a.n;
  C2<T>* tw = (C2<T>*)smem;
  C2<T>* q = tw + L;
  C2<T>* slots = q + MAXN;
  T* tiles = (T*)(slots + kBatchWaves * PPW * slot_len(L));
  const int tid = bw_tid();
  bw_tables<L>(a, tw, q, tid);
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int sub = wave / W, wv = wave - sub * W;  // tile group and wavefront in it
  const int ts = tid - sub * NTS;                  // thread in the group
  const int qq = lane / G, g = lane % G;
  C2<T>* slot = slots + (wave * PPW + qq) * slot_len(L);
  T* tile_s = tiles + sub * MAXN * TS;
  const int tiles_p = (a.Np + P - 1) / P;
  for (int base = 0; base < ntile; base += S) {
    const bool active = base + sub < ntile;
    const int t = tile + base + sub;
    const int o = active ? t / tiles_p : 0, p0 = active ? (t % tiles_p) * P : 0;
    const int np = active ? min(P, a.Np - p0) : 0;
    const long long ib = (long long)o * a.in_so + (long long)p0 * a.in_sp;
    // eight loads in flight per thread before their LDS stores: one load at a
    // time waits out the memory latency once per element (a register copy of
    // the whole tile spilled)
    constexpr int U = 8;
    for (int e0 = ts; e0 < n * P; e0 += U * NTS) {
      T v8[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * NTS;
        const int j = e / P, c = e % P;
        v8[u] = (j < n && c < np) ? a.in[ib + (long long)j * a.in_sj + (long long)c * a.in_sp] : (T)0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = e0 + u * NTS;
        if (e < n * P) tile_s[(e / P) * TS + e % P] = v8[u];
      }
    }
    __syncthreads();
    for (int r = 0; r < PPL && active; ++r) {
      const int f = (r * W + wv) * PPW + qq;  // pair: columns 2f, 2f + 1
      T* ca = tile_s + 2 * f;
      auto get = [&](int s, int w) { return ca[s * TS + w]; };
      C2<T> v[R0];
      r2r_fft<T, L>(v, XF, n, slot, g, tw, q, get);
      if constexpr (SW) {
        // multiplier norm / (sum of the eigenvalues), FP64 sum (Table 1)
        const int pa = min(p0 + 2 * f, a.Np - 1), pb = min(p0 + 2 * f + 1, a.Np - 1);
        const double ro = a.lam_o ? a.lam_o[o] : 0.0;
        const double ra = ro + (a.lam_p ? a.lam_p[pa] : 0.0), rb = ro + (a.lam_p ? a.lam_p[pb] : 0.0);
#pragma unroll
        for (int i = 0; i < R0; ++i) {
          T sa, sb;
          const int k = r2r_extract<T>(XF, g + G * i, n, v[i], q, sa, sb);
          if (k < 0) continue;
          const double la = a.lam_j[k] + ra, lb = a.lam_j[k] + rb;
          ca[k * TS] = la == 0.0 ? (T)0 : sa * ((T)a.norm / (T)la);
          ca[k * TS + 1] = lb == 0.0 ? (T)0 : sb * ((T)a.norm / (T)lb);
        }
        wave_sync();
        r2r_fft<T, L>(v, XO, n, slot, g, tw, q, get);
      }
#pragma unroll
      for (int i = 0; i < R0; ++i) {
        T oa, obv;
        const int k = r2r_extract<T>(XO, g + G * i, n, v[i], q, oa, obv);
        if (k < 0) continue;
        ca[k * TS] = oa;
        ca[k * TS + 1] = obv;
      }
      wave_sync();  // the slot is reused by the next pair
    }
    __syncthreads();
    const long long ob = (long long)o * a.out_so + (long long)p0 * a.out_sp;
    for (int e = ts; e < n * P; e += NTS) {
      const int j = e / P, c = e - (e / P) * P;
      if (c < np) st_stream(&a.out[ob + (long long)j * a.out_sj + (long long)c * a.out_sp], tile_s[j * TS + c]);
    }
    __syncthreads();  // the tiles are reloaded by the next step
  }
}

// The persistent kernel calls every tile body as a function of its own (not
// inlined), so that each is register-allocated on its own: inlined into the
// loop over items their values stayed live together and spilled.  The
// arguments are copied into scalar registers on entry (bw_uniform).  The
// level launches have no loop over items and inline the bodies.
template <int L, int X>
__device__ __attribute__((noinline)) void bw_contig_call(const BwArgs* ap, unsigned char* smem,
                                                         int tile, int ntile) {
  bw_contig<L, X>(bw_uniform(*ap), smem, tile, ntile);
}
template <int L, int XF, int XO, bool SW>
__device__ __attribute__((noinline)) void bw_strided_call(const BwArgs* ap, unsigned char* smem,
                                                          int tile, int ntile) {
  bw_strided<L, XF, XO, SW>(bw_uniform(*ap), smem, tile, ntile);
}

// One item: ntile tiles of pass a, for the transform pair (XF, XB) of the batch.
template <int L, int XF, int XB, bool CALL>
__device__ __forceinline__ void bw_item_L(const BwArgs& a, unsigned char* smem, int tile, int ntile) {
  if (a.fast == FAST_R2R_C) {
    if constexpr (CALL) {
      if (a.xf == XF) bw_contig_call<L, XF>(&a, smem, tile, ntile);
      else bw_contig_call<L, XB>(&a, smem, tile, ntile);
    } else {
      if (a.xf == XF) bw_contig<L, XF>(a, smem, tile, ntile);
      else bw_contig<L, XB>(a, smem, tile, ntile);
    }
  } else if (a.fast == FAST_R2R_S) {
    if constexpr (CALL) {
      if (a.xf == XF) bw_strided_call<L, XF, XF, false>(&a, smem, tile, ntile);
      else bw_strided_call<L, XB, XB, false>(&a, smem, tile, ntile);
    } else {
      if (a.xf == XF) bw_strided<L, XF, XF, false>(a, smem, tile, ntile);
      else bw_strided<L, XB, XB, false>(a, smem, tile, ntile);
    }
  } else {
    if constexpr (CALL) bw_strided_call<L, XF, XB, true>(&a, smem, tile, ntile);
    else bw_strided<L, XF, XB, true>(a, smem, tile, ntile);
  }
}

template <int XF, int XB, bool CALL>
__device__ __forceinline__ void bw_item(const BwArgs& a, unsigned char* smem, int tile, int ntile) {
  switch (a.L) {
    case 64: bw_item_L<64, XF, XB, CALL>(a, smem, tile, ntile); break;
    case 96: bw_item_L<96, XF, XB, CALL>(a, smem, tile, ntile); break;
    case 128: bw_item_L<128, XF, XB, CALL>(a, smem, tile, ntile); break;
    case 192: bw_item_L<192, XF, XB, CALL>(a, smem, tile, ntile); break;
    default: bw_item_L<256, XF, XB, CALL>(a, smem, tile, ntile); break;
  }
}

__global__ void k_bw_zero(unsigned* c, int n, int* err) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) c[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) err[0] = 0;
}

// Four wavefronts per SIMD: at most 128 VGPRs.
template <int XF, int XB>
__global__ void __launch_bounds__(64 * kBatchWaves, 4)
    k_batched_wf(const PassArgs* passes, const BatchItem* items, int nitems, unsigned* counters,
                 int* err) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_item, s_ok;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(&counters[0], 1u);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= nitems) break;
    BatchItem bi = items[it];
    bi.pass = uni(bi.pass);
    bi.tile = uni(bi.tile);
    bi.ntile = uni(bi.ntile);
    bi.dep = uni(bi.dep);
    bi.need = uni(bi.need);
    if (threadIdx.x == 0) {
      int ok = 1;
      if (bi.dep >= 0) {
        unsigned spins = 0;
        while (__hip_atomic_load(&counters[1 + bi.dep], __ATOMIC_ACQUIRE,
                                 __HIP_MEMORY_SCOPE_AGENT) < (unsigned)bi.need) {
          __builtin_amdgcn_s_sleep(2);
          // bounded wait: report and skip (also stop at once if another wait failed)
          if (++spins > (1u << 22) ||
              __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            ok = 0;
            atomicExch(err, 1);
            break;
          }
        }
      }
      s_ok = ok;
    }
    __syncthreads();
    const int ok = __builtin_amdgcn_readfirstlane(s_ok);
    // acquire: the tiles written by the workgroups that completed the pass
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (ok) {
      const BwArgs args = bw_args(passes[bi.pass]);
      bw_item<XF, XB, true>(args, smem, bi.tile, bi.ntile);
    }
    // release: this item's stores before its tiles are counted
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(&counters[1 + bi.pass], (unsigned)bi.ntile, __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
  }
}

// One pass level of the batch for one transform length L and one pass kind
// (the passes of every problem that have no dependency left, transform along
// L and are of that kind): one workgroup per item, no queue, no waiting; the
// launch boundaries order the levels.  One instance per (L, kind) holds a
// single tile body, register-allocated like the single-plan kernels (all
// lengths and kinds in one kernel did not fit in 128 VGPRs).
// KIND: 0 / 1 contiguous pass of type XF / XB, 2 / 3 strided pass of type
// XF / XB, 4 sandwich (XF, multiplier, XB).
template <int XF, int XB, int L, int KIND>
__global__ void __launch_bounds__(64 * kBatchWaves, 4)
    k_batched_level(const PassArgs* passes, const BatchItem* items, int* err) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (blockIdx.x == 0 && threadIdx.x == 0 && err) err[0] = 0;  // no waits: never set
  BatchItem bi = items[blockIdx.x];
  bi.pass = uni(bi.pass);
  bi.tile = uni(bi.tile);
  bi.ntile = uni(bi.ntile);
  const BwArgs a = bw_args(passes[bi.pass]);
  if constexpr (KIND == 0) bw_contig<L, XF>(a, smem, bi.tile, bi.ntile);
  else if constexpr (KIND == 1) bw_contig<L, XB>(a, smem, bi.tile, bi.ntile);
  else if constexpr (KIND == 2) bw_strided<L, XF, XF, false>(a, smem, bi.tile, bi.ntile);
  else if constexpr (KIND == 3) bw_strided<L, XB, XB, false>(a, smem, bi.tile, bi.ntile);
  else bw_strided<L, XF, XB, true>(a, smem, bi.tile, bi.ntile);
}

template <int XF, int XB, int L, int KIND>
hipError_t bw_launch_group(const PassArgs* passes, const BatchItem* items, int n, int* err, int lds,
                           hipStream_t s) {
  allow_lds<k_batched_level<XF, XB, L, KIND>>();
  hipLaunchKernelGGL((k_batched_level<XF, XB, L, KIND>), dim3(n), dim3(64 * kBatchWaves), lds, s,
                     passes, items, err);
  return hipGetLastError();
}

template <int XF, int XB, int L>
hipError_t bw_launch_kind(const BatchGroup& g, const PassArgs* passes, const BatchItem* it, int* e,
                          hipStream_t s) {
  switch (g.kind) {
    case 0: return bw_launch_group<XF, XB, L, 0>(passes, it, g.count, e, g.lds, s);
    case 1: return bw_launch_group<XF, XB, L, 1>(passes, it, g.count, e, g.lds, s);
    case 2: return bw_launch_group<XF, XB, L, 2>(passes, it, g.count, e, g.lds, s);
    case 3: return bw_launch_group<XF, XB, L, 3>(passes, it, g.count, e, g.lds, s);
    case 4: return bw_launch_group<XF, XB, L, 4>(passes, it, g.count, e, g.lds, s);
    default: return hipErrorInvalidValue;
  }
}

template <int XF, int XB>
hipError_t bw_launch_one(const BatchGroup& g, const PassArgs* passes, const BatchItem* items, int* err,
                         hipStream_t s) {
  if (g.count <= 0) return hipSuccess;
  const BatchItem* it = items + g.first;
  switch (g.L) {
    case 64: return bw_launch_kind<XF, XB, 64>(g, passes, it, err, s);
    case 96: return bw_launch_kind<XF, XB, 96>(g, passes, it, err, s);
    case 128: return bw_launch_kind<XF, XB, 128>(g, passes, it, err, s);
    case 192: return bw_launch_kind<XF, XB, 192>(g, passes, it, err, s);
    case 256: return bw_launch_kind<XF, XB, 256>(g, passes, it, err, s);
    default: return hipErrorInvalidValue;
  }
}

template <int XF, int XB>
int bw_blocks_per_cu(int lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batched_wf<XF, XB>, 64 * kBatchWaves, lds) !=
      hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n > 0 ? n : 1;
}

template <int XF, int XB>
hipError_t bw_launch(const PassArgs* passes, const BatchItem* items, int nitems, unsigned* counters,
                     int ncounters, int* err, int grid, int lds, hipStream_t s) {
  allow_lds<k_batched_wf<XF, XB>>();
  hipLaunchKernelGGL(k_bw_zero, dim3(1 + ncounters / 256), dim3(256), 0, s, counters, ncounters, err);
  hipLaunchKernelGGL((k_batched_wf<XF, XB>), dim3(grid), dim3(64 * kBatchWaves), lds, s, passes, items,
                     nitems, counters, err);
  return hipGetLastError();
}

template <int L>
int bw_lds_L(int fast) {
  using B = BW<L>;
  const int base = (L + B::MAXN + kBatchWaves * B::PPW * slot_len(L)) * 8;
  return fast == FAST_R2R_C ? base : base + B::S * B::MAXN * B::TS * 4;
}

}  // namespace

bool batched_wf_length(int L) { return L == 64 || L == 96 || L == 128 || L == 192 || L == 256; }

int batched_wf_lds(int fast, int L) {
  switch (L) {
    case 64: return bw_lds_L<64>(fast);
    case 96: return bw_lds_L<96>(fast);
    case 128: return bw_lds_L<128>(fast);
    case 192: return bw_lds_L<192>(fast);
    case 256: return bw_lds_L<256>(fast);
    default: return -1;
  }
}

int batched_wf_tiles(const PassArgs& a) {
  int ppw = 0, P = 32;
  switch (a.L) {
    case 64: ppw = WF<64>::PPW; break;
    case 96: ppw = WF<96>::PPW; break;
    case 128: ppw = WF<128>::PPW; break;
    case 192: ppw = WF<192>::PPW; break;
    case 256: ppw = WF<256>::PPW; break;
    default: return 0;
  }
  if (a.fast == FAST_R2R_C) {
    const long long pairs = (long long)((a.Np + 1) / 2) * a.No;
    const long long per = (long long)kBatchWaves * ppw;
    return (int)((pairs + per - 1) / per);
  }
  return ((a.Np + P - 1) / P) * a.No;
}

int batched_wf_group(const PassArgs& a) {
  if (a.fast == FAST_R2R_C) return 1;
  switch (a.L) {
    case 64: return BW<64>::S;
    case 96: return BW<96>::S;
    case 128: return BW<128>::S;
    case 192: return BW<192>::S;
    default: return BW<256>::S;
  }
}

int batched_wf_blocks_per_cu(int xf, int lds) {
  if (xf == X_DCT2) return bw_blocks_per_cu<X_DCT2, X_DCT3>(lds);
  if (xf == X_DST2) return bw_blocks_per_cu<X_DST2, X_DST3>(lds);
  return bw_blocks_per_cu<X_DCT1, X_DCT1>(lds);
}

hipError_t launch_batched_group(int xf, const PassArgs* passes, const BatchItem* items,
                                const BatchGroup& g, int* err, hipStream_t s) {
  if (xf == X_DCT2) return bw_launch_one<X_DCT2, X_DCT3>(g, passes, items, err, s);
  if (xf == X_DST2) return bw_launch_one<X_DST2, X_DST3>(g, passes, items, err, s);
  if (xf == X_DCT1) return bw_launch_one<X_DCT1, X_DCT1>(g, passes, items, err, s);
  return hipErrorInvalidValue;
}

hipError_t launch_batched_wf(int xf, const PassArgs* passes, const BatchItem* items, int nitems,
                             unsigned* counters, int ncounters, int* err, int grid, int lds,
                             hipStream_t s) {
  if (xf == X_DCT2)
    return bw_launch<X_DCT2, X_DCT3>(passes, items, nitems, counters, ncounters, err, grid, lds, s);
  if (xf == X_DST2)
    return bw_launch<X_DST2, X_DST3>(passes, items, nitems, counters, ncounters, err, grid, lds, s);
  if (xf == X_DCT1)
    return bw_launch<X_DCT1, X_DCT1>(passes, items, nitems, counters, ncounters, err, grid, lds, s);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- launch
// Pencils per tile of the strided passes: runs of 128 bytes.
int r2r_tile(int prec) { return prec == 0 ? 32 : 16; }

// Wavefronts per strided workgroup: one per pair (PPW pairs per wavefront
// for short transforms).
constexpr int r2r_waves(int P, int ppw) { return (P / 2) / ppw; }

int r2r_lds_bytes(int fast, int L, int n, int prec) {
  const int cs = prec == 0 ? 8 : 16, es = cs / 2;
  const int R0 = wf_r0(L);
  if (R0 <= 0 || (R0 % 3 == 0 && prec != 0)) return -1;  // 3 x 2^k: FP32 only
  const int ppw = 64 / (L / R0);
  const int SL = slot_len(L);
  if (fast == FAST_R2R_C) return (L + n + kR2RContigWaves * ppw * SL) * cs;
  const int P = r2r_tile(prec);
  // one pencil pair per lane group: the tile's pairs must fill whole wavefronts
  if ((P / 2) % ppw != 0) return -1;
  return (L + n + r2r_waves(P, ppw) * ppw * SL) * cs + n * (P + 1) * es;
}

namespace {

template <typename T, int L>
hipError_t launch_bounded_L(const PassArgs& a, hipStream_t s) {
  constexpr int PPW = WF<L>::PPW;
  const int lds = a.lds_bytes;
  if (a.n < 1 || a.n > L / 2 + 1) return hipErrorInvalidValue;  // rows per pencil of every Table 1 type
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
  if constexpr (W < 1 || (P / 2) % PPW != 0) {
    return hipErrorInvalidValue;  // the planner keeps such passes on the general kernels
  } else {
    const dim3 grid((unsigned)(((a.Np + P - 1) / P) * a.No));
    const int ntiles = (int)grid.x;
    // radix-12 lengths: the register prefetch of the persistent form would
    // cost occupancy, so their tiles are one workgroup each
    constexpr bool kPers = WF<L>::R0 % 3 != 0;
    if (a.fast == FAST_R2R_SW) {
      if (a.xb != r2r_partner(a.xf)) return hipErrorInvalidValue;
      if constexpr (kPers) {
        allow_lds<kb_strided<T, L, P, W, true, true>>();
        const int nb = persistent_grid<kb_strided<T, L, P, W, true, true>>(64 * W, lds, ntiles);
        if (ntiles > 4 * nb && !std::getenv("HP_R2R_NOPERS")) {
          hipLaunchKernelGGL((kb_strided<T, L, P, W, true, true>), dim3(nb), dim3(64 * W), lds, s, a);
          return hipGetLastError();
        }
      }
      allow_lds<kb_strided<T, L, P, W, true, false>>();
      hipLaunchKernelGGL((kb_strided<T, L, P, W, true, false>), grid, dim3(64 * W), lds, s, a);
    } else {
      if constexpr (kPers) {
        allow_lds<kb_strided<T, L, P, W, false, true>>();
        const int nb = persistent_grid<kb_strided<T, L, P, W, false, true>>(64 * W, lds, ntiles);
        if (ntiles > 4 * nb) {
          hipLaunchKernelGGL((kb_strided<T, L, P, W, false, true>), dim3(nb), dim3(64 * W), lds, s, a);
          return hipGetLastError();
        }
      }
      allow_lds<kb_strided<T, L, P, W, false, false>>();
      hipLaunchKernelGGL((kb_strided<T, L, P, W, false, false>), grid, dim3(64 * W), lds, s, a);
    }
    return hipGetLastError();
  }
}

template <typename T>
hipError_t launch_bounded_T(const PassArgs& a, hipStream_t s) {
  switch (a.L) {
    case 64: return launch_bounded_L<T, 64>(a, s);
    // 3 x 2^k lengths: FP32 only (radix-12 first stage; FP64 stays on the
    // general kernels, see r2r_lds_bytes)
    case 96:
      if constexpr (sizeof(T) == 4) return launch_bounded_L<T, 96>(a, s);
      else return hipErrorInvalidValue;
    case 192:
      if constexpr (sizeof(T) == 4) return launch_bounded_L<T, 192>(a, s);
      else return hipErrorInvalidValue;
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
    double lam = 0.0, w2 = 0.0, kap = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      dof += (long long)i[b] * a.gp_os[b];
      const int sb = i[b] - a.gp_off[b];
      const int basis = a.gp_basis[b];
      int k = sb;
      if (b == a.ax_j) k = basis == 2 ? (sb == 0 ? 0 : a.nunk[b] - sb) : sb + a.gp_shift;
      ok = ok && sb >= 0 && sb < a.gp_len[b] && k >= 0 && k < a.nunk[b];
      if (ok) {
        so += (long long)k * a.gp_is[b];
        if (a.lam[b]) lam += a.lam[b][k];
        // wavenumber index of coefficient k: k + 1 (sine), k (cosine), signed k (Hartley)
        const double kk = basis == 2 ? (double)signed_index(k, a.nunk[b]) : (double)(k + (basis == 0 ? 1 : 0));
        if (b == a.ax_j) kap = basis == 2 ? -(double)signed_index(sb, a.nunk[b]) : kk;
        const double w = a.kc[b] * kk;  // NABLA: the wavenumber of axis b
        w2 += w * w;
      }
    }
    T v = (T)0;
    if (ok) {
      // gradient: +-(pi kappa / L) one index over (Hartley: -(2 pi k~ / L)
      // from the mirrored index); NABLA (diff = D_NABLA): -sum_b w_b^2 on the
      // same index
      // (ax_j < 0 otherwise: a plain copy times gp_scale)
      double m = a.diff == D_NABLA ? -a.gp_scale * w2 : (a.ax_j < 0 ? a.gp_scale : a.gp_scale * kap);
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

// out[0][i] += in[0][i] (+ in[1][i]), i < gp_ext[0]: the second terms of the
// Dirichlet / Neumann divergence and curl.
template <typename T>
__global__ void __launch_bounds__(256) k_add(PassArgs a) {
  const long long total = a.gp_ext[0];
  T* dst = (T*)a.out[0];
  const T* x = (const T*)a.in[0];
  const T* y = (const T*)a.in[1];
  const long long step = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += step) {
    T v = dst[e] + x[e];
    if (y) v += y[e];
    dst[e] = v;
  }
}

template <typename T>
hipError_t launch_add(const PassArgs& a, hipStream_t s) {
  const long long total = a.gp_ext[0];
  if (total <= 0) return hipSuccess;
  const long long blocks = (total + 255) / 256;
  const int grid = (int)(blocks < 8192 ? blocks : 8192);
  hipLaunchKernelGGL(k_add<T>, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

// One thread per output point; every term reads the three points around it
// along its axis (the faces' values or the one-sided stencils at the ends).
template <typename T>
__global__ void __launch_bounds__(256) k_fd_deriv(FdArgs a) {
  long long total = 1;
  for (int b = 0; b < a.nd; ++b) total *= a.N[b];
  T* out = (T*)a.out;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    int c[3] = {0, 0, 0};
    long long r = e;
    for (int b = a.nd - 1; b >= 0; --b) {
      c[b] = (int)(r % a.N[b]);
      r /= a.N[b];
    }
    double acc = 0.0;
    for (int k = 0; k < a.nterm; ++k) {
      const FdTerm& t = a.t[k];
      const int ax = t.axis, n = a.N[ax], j = c[ax];
      long long s = 1;
      for (int b = ax + 1; b < a.nd; ++b) s *= a.N[b];
      const T* p = (const T*)t.psi;
      auto v = [&](int i) -> double { return (double)p[e + (long long)(i - j) * s]; };
      // face values at this point's position on the other axes
      long long fo = 0;
      for (int b = 0; b < a.nd; ++b)
        if (b != ax) fo = fo * a.N[b] + c[b];
      const double glo = (t.g_lo && j == 0) ? (double)((const T*)t.g_lo)[fo] : 0.0;
      const double ghi = (t.g_hi && j == n - 1) ? (double)((const T*)t.g_hi)[fo] : 0.0;
      const double h = a.h[ax];
      const int bc = a.bc[ax];
      double d;
      if (bc == FD_PERIODIC) {  // the grid wraps
        d = (v(j + 1 < n ? j + 1 : 0) - v(j > 0 ? j - 1 : n - 1)) / (2.0 * h);
      } else if (bc == FD_DIRICHLET && a.regular) {  // boundary nodes hold g; n >= 3
        if (j == 0) d = (-3.0 * v(0) + 4.0 * v(1) - v(2)) / (2.0 * h);
        else if (j == n - 1) d = (3.0 * v(n - 1) - 4.0 * v(n - 2) + v(n - 3)) / (2.0 * h);
        else d = (v(j + 1) - v(j - 1)) / (2.0 * h);
      } else if (bc == FD_DIRICHLET) {  // quadratic through the face value and two centres
        if (n == 1) d = (ghi - glo) / h;  // (both faces at this one point)
        else if (j == 0) d = (v(1) / 3.0 + v(0) - 4.0 * glo / 3.0) / h;
        else if (j == n - 1) d = (4.0 * ghi / 3.0 - v(n - 1) - v(n - 2) / 3.0) / h;
        else d = (v(j + 1) - v(j - 1)) / (2.0 * h);
      } else {  // Neumann ghosts: centred difference = g (REGULAR), face difference = g
        const double left = j > 0 ? v(j - 1) : (a.regular ? v(1) - 2.0 * h * glo : v(0) - h * glo);
        const double right =
            j < n - 1 ? v(j + 1) : (a.regular ? v(n - 2) + 2.0 * h * ghi : v(n - 1) + h * ghi);
        d = (right - left) / (2.0 * h);
      }
      acc += t.sign * d;
    }
    out[e] = (T)acc;
  }
}

hipError_t launch_fd_deriv(const FdArgs& a, int prec, hipStream_t s) {
  if (prec == 0) hipLaunchKernelGGL(k_fd_deriv<float>, dim3(1024), dim3(256), 0, s, a);
  else hipLaunchKernelGGL(k_fd_deriv<double>, dim3(1024), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_bounded(const PassArgs& a, int prec, hipStream_t s) {
  if (a.fast == FAST_GRAD_PREP)
    return prec == 0 ? launch_grad_prep<float>(a, s) : launch_grad_prep<double>(a, s);
  if (a.fast == FAST_ADD) return prec == 0 ? launch_add<float>(a, s) : launch_add<double>(a, s);
  if (a.fast == FAST_SMALL2D) return launch_small2d(a, prec, s);
  if (prec == 0) return launch_bounded_T<float>(a, s);
  return launch_bounded_T<double>(a, s);
}

}  // namespace hp
