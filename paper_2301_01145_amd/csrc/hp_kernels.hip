// General pencil-pass kernels of the spectral Poisson solve (gfx950).
//
// One launch transforms every pencil (1D line) of a field along one axis.  A
// workgroup of 256 threads takes a tile of P pencils: it loads the tile from
// HBM with unit-stride runs (along the pencil when the pencil is contiguous,
// across pencils otherwise), builds the complex FFT input in LDS, runs a
// mixed-radix (2/3/4/5/8, and any larger prime as a direct stage) Stockham
// FFT in LDS and writes the result with
// unit-stride runs again.  The strides of the input and output sides are
// independent, so a pass can also transpose.
//
// The sandwich pass (last axis of the forward transform) loads, transforms,
// multiplies by the spectral multiplier (Table 1 eigenvalues or the Green's
// spectrum, Section 2.2 step 2), applies the spectral derivative (step 3,
// eq. ft_sd), transforms back and stores, so the spectrum of that axis never
// leaves LDS.
#include <algorithm>
#include <mutex>

#include "hp_device.hpp"
#include "hp_faces.hpp"
#include "hp_internal.hpp"

namespace hp {

// ------------------------------------------------------------- Stockham FFT
// One radix-R stage over `nfft` transforms of length L stored contiguously in
// LDS.  Butterfly j of a transform reads x[j + t L/R] (t < R), twiddles input
// t by W_{Ns R}^{t k} (k = j mod Ns), and writes output t' to
// (j / Ns) Ns R + k + t' Ns.  All reads finish (barrier) before any write, so
// the stage is in place.
template <typename T, int R, int MAXE, bool INV>
__device__ __attribute__((noinline)) void fft_stage(C2<T>* Z, int L, int nfft, int Ns, int twstep,
                                          const C2<T>* __restrict__ tw) {
  constexpr int MB = (MAXE + R - 1) / R;
  const int nbl = L / R;
  const int total = nfft * nbl;
  C2<T> v[MB][R];
  int ob[MB];
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int idx = threadIdx.x + b * kThreads;
    ob[b] = -1;
    if (idx < total) {
      const int f = idx / nbl;
      const int j = idx - f * nbl;
      const int k = j % Ns;
      const C2<T>* src = Z + f * L + j;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        C2<T> x = src[t * nbl];
        if (t > 0 && k > 0) {
          C2<T> w = tw[t * k * twstep];
          if (INV) w.im = -w.im;
          x = cmul(x, w);
        }
        v[b][t] = x;
      }
      ob[b] = f * L + (j - k) * R + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    if (ob[b] >= 0) {
      dftR<T, R, INV>(v[b]);
#pragma unroll
      for (int t = 0; t < R; ++t) Z[ob[b] + t * Ns] = v[b][t];
    }
  }
  __syncthreads();
}

// One stage of a prime radix R > 5 (lengths with a prime factor that the fixed
// radices do not cover).  Output t' of butterfly j (k = j mod Ns) is the
// R-term sum  sum_t x[j + t L/R] W_{Ns R}^{t (k + t' Ns)}: the stage twiddle
// W_{Ns R}^{t k} and the R-point DFT factor W_R^{t t'} in one table entry.
// It costs R multiply-adds per output instead of O(log R), which is what a
// direct DFT of a prime length costs.  One output per thread slot (the tile
// holds at most kThreads * MAXE elements); all reads finish (barrier) before
// any write, so the stage is in place like the fixed-radix ones.
template <typename T, int MAXE, bool INV>
__device__ __attribute__((noinline)) void fft_stage_prime(C2<T>* Z, int L, int nfft, int R, int Ns,
                                                          int twstep, const C2<T>* __restrict__ tw) {
  const int nbl = L / R;
  const int total = nfft * L;
  C2<T> v[MAXE];
  int ob[MAXE];
#pragma unroll
  for (int b = 0; b < MAXE; ++b) {
    const int idx = threadIdx.x + b * kThreads;
    ob[b] = -1;
    if (idx < total) {
      const int f = idx / L;
      const int r = idx - f * L;
      const int j = r / R, tp = r - j * R;  // butterfly j, output t'
      const int k = j % Ns;
      const C2<T>* src = Z + f * L + j;
      // exponent of W_L for term t: t (k + t' Ns) twstep mod L, stepped by e1 < L
      const int e1 = (k + tp * Ns) * twstep;
      int e = 0;
      C2<T> acc = {(T)0, (T)0};
      for (int t = 0; t < R; ++t) {
        C2<T> w = tw[e];
        if (INV) w.im = -w.im;
        acc = cadd(acc, cmul(src[t * nbl], w));
        e += e1;
        if (e >= L) e -= L;
      }
      v[b] = acc;
      ob[b] = f * L + (j - k) * R + k + tp * Ns;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXE; ++b)
    if (ob[b] >= 0) Z[ob[b]] = v[b];
  __syncthreads();
}

// Complex elements per thread of one stage: BIG = 0 holds 16 (FP32) / 8
// (FP64), fewer registers and more resident waves; BIG = 1 holds 32 / 16 for
// tiles of long transforms.
template <typename T, int BIG>
struct Maxe {
  static constexpr int v = (BIG ? 32 : 16) / (sizeof(T) == 8 ? 2 : 1);
};

// Full FFT of nfft transforms in LDS (caller has synchronised the input).
template <typename T, int BIG, bool INV>
__device__ void fft_lds(C2<T>* Z, int nfft, const PassArgs& a) {
  constexpr int ME = Maxe<T, BIG>::v;
  const C2<T>* tw = (const C2<T>*)a.tw;
  const int L = a.L;
  int Ns = 1;
  for (int s = 0; s < a.nstage; ++s) {
    const int R = a.radix[s];
    const int twstep = L / (Ns * R);
    switch (R) {
      case 8: fft_stage<T, 8, ME, INV>(Z, L, nfft, Ns, twstep, tw); break;
      case 4: fft_stage<T, 4, ME, INV>(Z, L, nfft, Ns, twstep, tw); break;
      case 2: fft_stage<T, 2, ME, INV>(Z, L, nfft, Ns, twstep, tw); break;
      case 3: fft_stage<T, 3, ME, INV>(Z, L, nfft, Ns, twstep, tw); break;
      case 5: fft_stage<T, 5, ME, INV>(Z, L, nfft, Ns, twstep, tw); break;
      default: fft_stage_prime<T, ME, INV>(Z, L, nfft, R, Ns, twstep, tw); break;
    }
    Ns *= R;
  }
}

__device__ __forceinline__ bool xform_inverse_fft(int x) {
  return x == X_C2C_B || x == X_C2R || x == X_PAIR_B || x == X_DCT3 || x == X_DST3;
}
__device__ __forceinline__ bool xform_real_in(int x) {
  return x == X_R2C || x == X_PAIR_F || x == X_DST1 || x == X_DST2 || x == X_DST3 ||
         x == X_DCT1 || x == X_DCT2 || x == X_DCT3 || x == X_DHT;
}
__device__ __forceinline__ bool xform_real_out(int x) {
  return x == X_C2R || x == X_PAIR_B || x == X_DST1 || x == X_DST2 || x == X_DST3 ||
         x == X_DCT1 || x == X_DCT2 || x == X_DCT3 || x == X_DHT;
}

// ----------------------------------------------------------- tile addressing
struct Tile {
  int o, p0, np;
};

__device__ __forceinline__ Tile tile_of(const PassArgs& a) {
  const int tiles_p = (a.Np + a.P - 1) / a.P;
  Tile t;
  t.o = blockIdx.x / tiles_p;
  t.p0 = (blockIdx.x - t.o * tiles_p) * a.P;
  t.np = min(a.P, a.Np - t.p0);
  return t;
}

// Element e of a P x cnt tile -> (p, j), unit stride runs on the memory side.
__device__ __forceinline__ void tile_pj(int e, int P, int cnt, int jfast, int& p, int& j) {
  if (jfast) {
    p = e / cnt;
    j = e - p * cnt;
  } else {
    j = e / P;
    p = e - j * P;
  }
}

// ---------------------------------------------------------------- loading
// Each thread takes kLoadBatch elements per round and issues all their loads
// before the first is used, so a tile costs one memory latency per round
// instead of one per element.
constexpr int kLoadBatch = 4;

// Complex pencils straight into Z[p][m], zero beyond nin.
template <typename T>
__device__ void load_c2c(C2<T>* Z, const void* src, const PassArgs& a, const Tile& t) {
  const C2<T>* in = (const C2<T>*)src;
  const int cnt = a.nin;
  const int total = a.P * cnt;
  const long long obase = (long long)t.o * a.in_so + (long long)t.p0 * a.in_sp;
  for (int e0 = threadIdx.x; e0 < total; e0 += kLoadBatch * kThreads) {
    C2<T> v[kLoadBatch];
    int pp[kLoadBatch], jj[kLoadBatch];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int e = e0 + u * kThreads;
      tile_pj(min(e, total - 1), a.P, cnt, a.in_jfast, pp[u], jj[u]);
      // unconditional load from a clamped (in-tile) address; the pencils
      // beyond np are zeroed where the values are kept
      v[u] = in[obase + (long long)min(pp[u], t.np - 1) * a.in_sp + (long long)jj[u] * a.in_sj];
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u)
      if (e0 + u * kThreads < total) Z[pp[u] * a.L + jj[u]] = pp[u] < t.np ? v[u] : C2<T>{(T)0, (T)0};
  }
  for (int e = threadIdx.x; e < a.P * (a.L - cnt); e += kThreads) {
    const int p = e / (a.L - cnt);
    const int m = cnt + (e - p * (a.L - cnt));
    Z[p * a.L + m] = {(T)0, (T)0};
  }
}

// Real pencils into R[p][j] (j < nin), with boundary terms when present.
template <typename T>
__device__ void load_real(T* R, const void* src, const PassArgs& a, const Tile& t, bool faces) {
  const T* in = (const T*)src;
  const int cnt = a.nin;
  const int total = a.P * cnt;
  const long long obase = (long long)t.o * a.in_so + (long long)t.p0 * a.in_sp;
  for (int e0 = threadIdx.x; e0 < total; e0 += kLoadBatch * kThreads) {
    T v[kLoadBatch];
    int pp[kLoadBatch], jj[kLoadBatch];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int e = e0 + u * kThreads;
      tile_pj(min(e, total - 1), a.P, cnt, a.in_jfast, pp[u], jj[u]);
      v[u] = in[obase + (long long)min(pp[u], t.np - 1) * a.in_sp + (long long)jj[u] * a.in_sj];
    }
    if (faces) {
#pragma unroll
      for (int u = 0; u < kLoadBatch; ++u)
        if (e0 + u * kThreads < total && pp[u] < t.np)
          v[u] = (T)((double)v[u] + face_terms<T>(a, jj[u], t.p0 + pp[u], t.o));
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u)
      if (e0 + u * kThreads < total) R[pp[u] * cnt + jj[u]] = pp[u] < t.np ? v[u] : (T)0;
  }
}

// Half spectra (complex, nin = L/2 + 1) into R[p][k].
template <typename T>
__device__ void load_half(C2<T>* R, const void* src, const PassArgs& a, const Tile& t) {
  const C2<T>* in = (const C2<T>*)src;
  const int cnt = a.nin;
  const int total = a.P * cnt;
  const long long obase = (long long)t.o * a.in_so + (long long)t.p0 * a.in_sp;
  for (int e0 = threadIdx.x; e0 < total; e0 += kLoadBatch * kThreads) {
    C2<T> v[kLoadBatch];
    int pp[kLoadBatch], jj[kLoadBatch];
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u) {
      const int e = e0 + u * kThreads;
      tile_pj(min(e, total - 1), a.P, cnt, a.in_jfast, pp[u], jj[u]);
      v[u] = in[obase + (long long)min(pp[u], t.np - 1) * a.in_sp + (long long)jj[u] * a.in_sj];
    }
#pragma unroll
    for (int u = 0; u < kLoadBatch; ++u)
      if (e0 + u * kThreads < total) R[pp[u] * cnt + jj[u]] = pp[u] < t.np ? v[u] : C2<T>{(T)0, (T)0};
  }
}

// Build the complex FFT input Z[f][m] (f = pencil pair) from real pencils R.
// (XC: the transform type as a compile-time constant; build_from_real below
// branches once per call instead of once per element)
template <typename T, int XC>
__device__ void build_from_real_x(C2<T>* Z, const T* R, const PassArgs& a, int nfft) {
  constexpr int x = XC;
  const int L = a.L, n = a.n, cnt = a.nin;
  const C2<T>* q = (const C2<T>*)a.qtw;
  for (int e = threadIdx.x; e < nfft * L; e += kThreads) {
    const int f = e / L;
    const int m = e - f * L;
    const T* ra = R + (2 * f) * cnt;
    const T* rb = ra + cnt;
    C2<T> z = {(T)0, (T)0};
    switch (x) {
      case X_R2C:
      case X_PAIR_F:
      case X_DHT:
        if (m < cnt) z = {ra[m], rb[m]};
        break;
      case X_DST1:  // [0, x_0..x_{n-1}, 0, -x_{n-1}..-x_0]
        if (m >= 1 && m <= n) z = {ra[m - 1], rb[m - 1]};
        else if (m > n + 1) z = {-ra[L - m - 1], -rb[L - m - 1]};
        break;
      case X_DCT1: {  // [x_0..x_{n-1}, x_{n-2}..x_1]
        const int s = m < n ? m : L - m;
        z = {ra[s], rb[s]};
      } break;
      case X_DCT2:
      case X_DST2: {  // [x_0..x_{n-1}, x_{n-1}..x_0], DST-II with (-1)^j
        const int s = m < n ? m : L - 1 - m;
        z = {ra[s], rb[s]};
        if (x == X_DST2 && (s & 1)) z = {-z.re, -z.im};
      } break;
      case X_DCT3:
      case X_DST3: {  // e^{+i pi j/2n} (a_j + i b_j), j < n; 0 at n; conjugate twist above
        if (m == n) break;
        const int s = m < n ? m : L - m;
        const int src = (x == X_DST3) ? n - 1 - s : s;
        C2<T> v = {ra[src], rb[src]};
        C2<T> w = q[s];  // e^{-i pi s / 2n}
        if (m < n) w.im = -w.im;
        z = cmul(v, w);
      } break;
      default:
        break;
    }
    Z[e] = z;
  }
}

template <typename T>
__device__ void build_from_real(C2<T>* Z, const T* R, int x, const PassArgs& a, int nfft) {
  switch (x) {
    case X_R2C: build_from_real_x<T, X_R2C>(Z, R, a, nfft); break;
    case X_PAIR_F: build_from_real_x<T, X_PAIR_F>(Z, R, a, nfft); break;
    case X_DST1: build_from_real_x<T, X_DST1>(Z, R, a, nfft); break;
    case X_DST2: build_from_real_x<T, X_DST2>(Z, R, a, nfft); break;
    case X_DST3: build_from_real_x<T, X_DST3>(Z, R, a, nfft); break;
    case X_DCT1: build_from_real_x<T, X_DCT1>(Z, R, a, nfft); break;
    case X_DCT2: build_from_real_x<T, X_DCT2>(Z, R, a, nfft); break;
    case X_DCT3: build_from_real_x<T, X_DCT3>(Z, R, a, nfft); break;
    case X_DHT: build_from_real_x<T, X_DHT>(Z, R, a, nfft); break;
    default: build_from_real_x<T, -1>(Z, R, a, nfft); break;
  }
}

// Build Z[f][m] from two half spectra R[2f], R[2f+1] (Hermitian completion).
template <typename T>
__device__ void build_from_half(C2<T>* Z, const C2<T>* R, const PassArgs& a, int nfft) {
  const int L = a.L, cnt = a.nin, half = L / 2;
  for (int e = threadIdx.x; e < nfft * L; e += kThreads) {
    const int f = e / L;
    const int m = e - f * L;
    const C2<T>* ra = R + (2 * f) * cnt;
    const C2<T>* rb = ra + cnt;
    C2<T> A, B;
    if (m <= half) {
      A = ra[m];
      B = rb[m];
      if (m == 0 || 2 * m == L) {
        A.im = (T)0;
        B.im = (T)0;
      }
    } else {
      A = cconj(ra[L - m]);
      B = cconj(rb[L - m]);
    }
    Z[e] = {A.re - B.im, A.im + B.re};
  }
}

// ---------------------------------------------------------------- storing
// Value of output element (pencil p, index k) computed from the transformed Z.
template <typename T>
__device__ __forceinline__ T real_out(const C2<T>* Z, int x, const PassArgs& a, int p, int k) {
  const int f = p >> 1;
  const bool second = p & 1;
  const C2<T>* z = Z + f * a.L;
  switch (x) {
    case X_DST1: {
      C2<T> v = z[k + 1];
      return second ? v.re : -v.im;
    }
    case X_DCT1:
    case X_DCT3:
    case X_C2R:
    case X_PAIR_B: {
      C2<T> v = z[k];
      return second ? v.im : v.re;
    }
    case X_DST3: {
      C2<T> v = z[k];
      T r = second ? v.im : v.re;
      return (k & 1) ? -r : r;
    }
    case X_DCT2:
    case X_DST2: {
      const int kk = (x == X_DST2) ? a.n - 1 - k : k;
      C2<T> v = cmul(z[kk], ((const C2<T>*)a.qtw)[kk]);
      return second ? v.im : v.re;
    }
    case X_DHT: {
      // Z = X_a + i X_b with X_a, X_b Hermitian; H = Re X - Im X per pencil
      const C2<T> u = z[k], w = z[k == 0 ? 0 : a.L - k];
      return second ? (T)0.5 * ((u.im + w.im) + (u.re - w.re))
                    : (T)0.5 * ((u.re + w.re) - (u.im - w.im));
    }
    default:
      return (T)0;
  }
}

template <typename T>
__device__ __forceinline__ C2<T> half_out(const C2<T>* Z, const PassArgs& a, int p, int k) {
  const int f = p >> 1;
  const C2<T>* z = Z + f * a.L;
  C2<T> zk = z[k];
  C2<T> zc = cconj(z[k == 0 ? 0 : a.L - k]);
  if (p & 1) {  // (zk - zc) / (2 i)
    C2<T> d = csub(zk, zc);
    return {d.im * (T)0.5, -d.re * (T)0.5};
  }
  C2<T> s = cadd(zk, zc);
  return {s.re * (T)0.5, s.im * (T)0.5};
}

template <typename T, int XC>
__device__ void store_out_x(const C2<T>* Z, void* dst, const PassArgs& a, const Tile& t) {
  constexpr int x = XC;
  const int cnt = a.nout;
  const int total = a.P * cnt;
  const long long obase = (long long)t.o * a.out_so + (long long)t.p0 * a.out_sp;
  for (int e = threadIdx.x; e < total; e += kThreads) {
    int p, k;
    tile_pj(e, a.P, cnt, a.out_jfast, p, k);
    if (p >= t.np) continue;
    const long long off = obase + (long long)p * a.out_sp + (long long)k * a.out_sj;
    if (x == X_C2C_F || x == X_C2C_B) {
      ((C2<T>*)dst)[off] = Z[p * a.L + k];
    } else if (x == X_R2C) {
      ((C2<T>*)dst)[off] = half_out(Z, a, p, k);
    } else {
      ((T*)dst)[off] = real_out(Z, x, a, p, k);
    }
  }
}

template <typename T>
__device__ void store_out(const C2<T>* Z, int x, void* dst, const PassArgs& a, const Tile& t) {
  switch (x) {
    case X_C2C_F: store_out_x<T, X_C2C_F>(Z, dst, a, t); break;
    case X_C2C_B: store_out_x<T, X_C2C_B>(Z, dst, a, t); break;
    case X_R2C: store_out_x<T, X_R2C>(Z, dst, a, t); break;
    case X_C2R: store_out_x<T, X_C2R>(Z, dst, a, t); break;
    case X_PAIR_B: store_out_x<T, X_PAIR_B>(Z, dst, a, t); break;
    case X_DST1: store_out_x<T, X_DST1>(Z, dst, a, t); break;
    case X_DST2: store_out_x<T, X_DST2>(Z, dst, a, t); break;
    case X_DST3: store_out_x<T, X_DST3>(Z, dst, a, t); break;
    case X_DCT1: store_out_x<T, X_DCT1>(Z, dst, a, t); break;
    case X_DCT2: store_out_x<T, X_DCT2>(Z, dst, a, t); break;
    case X_DCT3: store_out_x<T, X_DCT3>(Z, dst, a, t); break;
    case X_DHT: store_out_x<T, X_DHT>(Z, dst, a, t); break;
    default: store_out_x<T, -1>(Z, dst, a, t); break;
  }
}

// -------------------------------------------------------- spectral multiply
template <typename T>
__device__ __forceinline__ T multiplier(const PassArgs& a, const int k[3]) {
  if (a.mult == M_EIGEN) {
    double lam = a.lam[0][k[0]];
    if (a.lam[1]) lam += a.lam[1][k[1]];
    if (a.lam[2]) lam += a.lam[2][k[2]];
    return lam == 0.0 ? (T)0 : (T)(a.norm / lam);
  }
  if (a.mult == M_GREEN) {
    const int i0 = min(k[0], a.gM[0] - k[0]);
    const int i1 = min(k[1], a.gM[1] - k[1]);
    return ((const T*)a.green)[(long long)i0 * a.g_s[0] + (long long)i1 * a.g_s[1] +
                               (long long)k[2] * a.g_s[2]];
  }
  return (T)1;
}

// Spectral indices of element m of pencil p (tile-relative pencils beyond the
// last one are clamped: their values are never stored).
__device__ __forceinline__ void spectral_index(const PassArgs& a, int m, int p, int o, int k[3]) {
  p = min(p, a.Np - 1);
  k[0] = k[1] = k[2] = 0;
  if (a.ax_j >= 0) k[a.ax_j] = m;
  if (a.ax_p >= 0) k[a.ax_p] = p;
  if (a.ax_o >= 0) k[a.ax_o] = o;
}

template <typename T>
__device__ __forceinline__ T kval(const PassArgs& a, int axis, const int k[3]) {
  return ((const T*)a.kvec[axis])[k[axis]];
}

// ------------------------------------------------------------ pass bodies
template <typename T, int BIG>
__device__ void oneway(const PassArgs& a, unsigned char* smem, const Tile& t, int field) {
  if (!a.in[field]) return;  // absent field (zero upstream gradient): uniform per block
  C2<T>* Z = (C2<T>*)smem;
  const int x = a.xf;
  const bool pair = xform_real_in(x) || x == X_C2R;
  const int nfft = pair ? a.P / 2 : a.P;
  const bool faces = a.face[0][0] || a.face[0][1] || a.face[1][0] || a.face[1][1] ||
                     a.face[2][0] || a.face[2][1];
  unsigned char* rbuf = smem + (size_t)nfft * a.L * sizeof(C2<T>);
  if (x == X_C2C_F || x == X_C2C_B) {
    load_c2c<T>(Z, a.in[field], a, t);
  } else if (x == X_C2R) {
    load_half<T>((C2<T>*)rbuf, a.in[field], a, t);
    __syncthreads();
    build_from_half<T>(Z, (const C2<T>*)rbuf, a, nfft);
  } else {
    load_real<T>((T*)rbuf, a.in[field], a, t, faces);
    __syncthreads();
    build_from_real<T>(Z, (const T*)rbuf, x, a, nfft);
  }
  __syncthreads();
  if (xform_inverse_fft(x)) fft_lds<T, BIG, true>(Z, nfft, a);
  else fft_lds<T, BIG, false>(Z, nfft, a);
  store_out<T>(Z, x, a.out[field], a, t);
}

// Real-to-real sandwich (Dirichlet / Neumann): forward R2R, multiply by the
// FD2 / PS multiplier, backward R2R, along the same axis.
template <typename T, int BIG>
__device__ void sandwich_r2r(const PassArgs& a, unsigned char* smem, const Tile& t, int field) {
  const int nfft = a.P / 2;
  C2<T>* Z = (C2<T>*)smem;
  T* R = (T*)(smem + (size_t)nfft * a.L * sizeof(C2<T>));
  const bool faces = a.face[0][0] || a.face[0][1] || a.face[1][0] || a.face[1][1] ||
                     a.face[2][0] || a.face[2][1];
  load_real<T>(R, a.in[field], a, t, faces);
  __syncthreads();
  build_from_real<T>(Z, R, a.xf, a, nfft);
  __syncthreads();
  if (xform_inverse_fft(a.xf)) fft_lds<T, BIG, true>(Z, nfft, a);
  else fft_lds<T, BIG, false>(Z, nfft, a);
  // spectral values times the multiplier, back into R (same [p][k] layout)
  for (int e = threadIdx.x; e < a.P * a.n; e += kThreads) {
    const int p = e / a.n;
    const int m = e - p * a.n;
    int k[3];
    spectral_index(a, m, t.p0 + p, t.o, k);
    R[e] = real_out<T>(Z, a.xf, a, p, m) * multiplier<T>(a, k);
  }
  __syncthreads();
  build_from_real<T>(Z, R, a.xb, a, nfft);
  __syncthreads();
  if (xform_inverse_fft(a.xb)) fft_lds<T, BIG, true>(Z, nfft, a);
  else fft_lds<T, BIG, false>(Z, nfft, a);
  store_out<T>(Z, a.xb, a.out[field], a, t);
}

// Complex sandwich (periodic after R2C, unbounded, 1D periodic pairs):
// every coupled field of the tile is resident: S_c (P x L each) plus a work
// buffer W for derivative outputs.
template <typename T, int BIG>
__device__ void sandwich_c2c(const PassArgs& a, unsigned char* smem, const Tile& t) {
  const bool pair = a.xf == X_PAIR_F;
  const int nfft = pair ? a.P / 2 : a.P;
  const int L = a.L;
  const int tileC = nfft * L;
  const bool adj = diff_is_adjoint(a.diff);
  const int nS = adj ? a.n_out : a.n_in;
  // independent fields (no derivative coupling) take their field from blockIdx.y
  const int fb = (a.diff == D_NONE) ? (int)blockIdx.y : 0;
  C2<T>* S = (C2<T>*)smem;
  C2<T>* W = S + (size_t)nS * tileC;
  T* R = (T*)W;  // raw real pencils (pair mode; W is free while loading)

  auto load_into = [&](C2<T>* dst, const void* src) {
    if (pair) {
      load_real<T>(R, src, a, t, false);
      __syncthreads();
      build_from_real<T>(dst, R, X_PAIR_F, a, nfft);
    } else {
      load_c2c<T>(dst, src, a, t);
    }
    __syncthreads();
    fft_lds<T, BIG, false>(dst, nfft, a);
  };

  for (int c = 0; c < nS; ++c) {
    if (a.in[fb + c]) {
      load_into(S + (size_t)c * tileC, a.in[fb + c]);
    } else {
      for (int e = threadIdx.x; e < tileC; e += kThreads) S[(size_t)c * tileC + e] = {(T)0, (T)0};
      __syncthreads();
    }
  }
  // spectral Laplacian: the first derivative i k_b (Nyquist zeroed) twice per axis
  auto lap_of = [&](const int k[3]) -> T {
    T s = (T)0;
    for (int b = 0; b < 3; ++b)
      if (a.kvec[b]) {
        const T kb = kval<T>(a, b, k);
        s -= kb * kb;
      }
    return s;
  };
  // Transposed derivative inputs: curl (symmetric), minus the divergence
  // (gradient), minus the gradient (divergence) or the Laplacian (symmetric).
  if (adj) {
    const int nextra = a.n_in - nS;
    for (int i = 0; i < nextra; ++i) {
      const void* src = a.in[nS + i];
      if (!src) continue;
      load_into(W, src);
      for (int e = threadIdx.x; e < tileC; e += kThreads) {
        const int f = e / L;
        const int m = e - f * L;
        int k[3];
        spectral_index(a, m, t.p0 + f, t.o, k);
        const C2<T> g = W[e];
        if (a.diff == D_ADJ_CURL && nS == 1) {
          // 2D curl of a scalar, (d_y, -d_x): its transpose is -d_y g_0 + d_x g_1
          const T kk = i == 0 ? -kval<T>(a, 1, k) : kval<T>(a, 0, k);
          S[e] = cadd(S[e], cscale(cmuli(g), kk));
        } else if (a.diff == D_ADJ_CURL) {
          // (C g)_c = i(k_{c+1} g_{c+2} - k_{c+2} g_{c+1}): g_i enters
          // component i+1 with +i k_{i+2} and component i+2 with -i k_{i+1}
          const int c1 = (i + 1) % 3, c2 = (i + 2) % 3;
          const T kc1 = kval<T>(a, c1, k), kc2 = kval<T>(a, c2, k);
          C2<T> ig = cmuli(g);
          S[(size_t)c1 * tileC + e] = cadd(S[(size_t)c1 * tileC + e], cscale(ig, kc2));
          S[(size_t)c2 * tileC + e] = csub(S[(size_t)c2 * tileC + e], cscale(ig, kc1));
        } else if (a.diff == D_ADJ_DIV) {
          const C2<T> ig = cmuli(g);
          for (int c = 0; c < nS; ++c)
            S[(size_t)c * tileC + e] = csub(S[(size_t)c * tileC + e], cscale(ig, kval<T>(a, c, k)));
        } else if (a.diff == D_ADJ_NABLA) {
          S[(size_t)i * tileC + e] = cadd(S[(size_t)i * tileC + e], cscale(g, lap_of(k)));
        } else {
          const T ka = kval<T>(a, i, k);
          S[e] = csub(S[e], cscale(cmuli(g), ka));
        }
      }
      __syncthreads();
    }
  }
  if (a.mult == M_GREEN_ROWS || a.mult == M_GREEN_ROWS_ODD) {
    // Paired real pencils 2f, 2f + 1 of the tile belong to different bounded
    // modes, so they take different real-even Green's rows G_a, G_b.  The FFT
    // Z of a + ib holds the Hermitian spectra X_a = (Z_m + conj Z_-m) / 2 and
    // X_b = (Z_m - conj Z_-m) / 2i; G_a X_a + i G_b X_b recombines to
    // Z'_m = A Z_m + B conj Z_-m with A = (G_a + G_b) / 2, B = (G_a - G_b) / 2,
    // the same A, B at -m.  One thread per bin pair (m, L - m).  Odd rows
    // (bins i b_a, i b_b, b odd in m): Z'_m = i (A Z_m + B conj Z_-m) and
    // Z'_-m = -i (A Z_-m + B conj Z_m), A, B from b_a, b_b at m.
    const int half = L / 2;
    const bool odd = a.mult == M_GREEN_ROWS_ODD;
    auto row = [&](int p, int m) -> T {
      p = min(p, a.Np - 1);
      long long off = (long long)m * a.g_s[a.ax_j] + (long long)p * a.g_s[a.ax_p];
      if (a.ax_o >= 0) off += (long long)t.o * a.g_s[a.ax_o];
      return ((const T*)a.green)[off];
    };
    for (int e = threadIdx.x; e < nfft * (half + 1); e += kThreads) {
      const int f = e / (half + 1);
      const int m = e - f * (half + 1);
      const int mm = m == 0 ? 0 : L - m;
      const T ga = row(t.p0 + 2 * f, m), gb = row(t.p0 + 2 * f + 1, m);
      const T A = (T)0.5 * (ga + gb), B = (T)0.5 * (ga - gb);
      C2<T>* z = S + (size_t)f * L;
      const C2<T> zm = z[m], zmm = z[mm];
      const C2<T> ym = cadd(cscale(zm, A), cscale(cconj(zmm), B));
      const C2<T> ymm = cadd(cscale(zmm, A), cscale(cconj(zm), B));
      if (odd) {
        z[m] = cmuli(ym);
        if (mm != m) z[mm] = cscale(cmuli(ymm), (T)-1);
      } else {
        z[m] = ym;
        if (mm != m) z[mm] = ymm;
      }
    }
  } else {
    // multiply by the spectral multiplier
    for (int e = threadIdx.x; e < tileC; e += kThreads) {
      const int f = e / L;
      const int m = e - f * L;
      int k[3];
      spectral_index(a, m, t.p0 + f, t.o, k);
      const T mu = multiplier<T>(a, k);
      for (int c = 0; c < nS; ++c) S[(size_t)c * tileC + e] = cscale(S[(size_t)c * tileC + e], mu);
    }
  }
  __syncthreads();
  const int xb = pair ? X_PAIR_B : X_C2C_B;
  // derivative outputs (forward GRAD / CURL) through W, then psi in place
  if (a.diff == D_GRAD || a.diff == D_CURL || a.diff == D_DIV || a.diff == D_NABLA) {
    const int nd = a.n_out - a.n_in;
    for (int d = 0; d < nd; ++d) {
      for (int e = threadIdx.x; e < tileC; e += kThreads) {
        const int f = e / L;
        const int m = e - f * L;
        int k[3];
        spectral_index(a, m, t.p0 + f, t.o, k);
        C2<T> v;
        if (a.diff == D_GRAD) {
          v = cscale(cmuli(S[e]), kval<T>(a, d, k));
        } else if (a.diff == D_DIV) {
          C2<T> acc = {(T)0, (T)0};
          for (int c = 0; c < a.n_in; ++c)
            acc = cadd(acc, cscale(S[(size_t)c * tileC + e], kval<T>(a, c, k)));
          v = cmuli(acc);
        } else if (a.diff == D_NABLA) {
          v = cscale(S[(size_t)d * tileC + e], lap_of(k));
        } else if (a.n_in == 1) {
          // 2D curl of a scalar: (d_y psi, -d_x psi)
          v = cscale(cmuli(S[e]), d == 0 ? kval<T>(a, 1, k) : -kval<T>(a, 0, k));
        } else {
          const int c1 = (d + 1) % 3, c2 = (d + 2) % 3;
          v = cmuli(csub(cscale(S[(size_t)c2 * tileC + e], kval<T>(a, c1, k)),
                         cscale(S[(size_t)c1 * tileC + e], kval<T>(a, c2, k))));
        }
        W[e] = v;
      }
      __syncthreads();
      fft_lds<T, BIG, true>(W, nfft, a);
      store_out<T>(W, xb, a.out[a.n_in + d], a, t);
      __syncthreads();
    }
  }
  for (int c = 0; c < nS; ++c) {
    fft_lds<T, BIG, true>(S + (size_t)c * tileC, nfft, a);
    store_out<T>(S + (size_t)c * tileC, xb, a.out[fb + c], a, t);
  }
}

template <typename T, int BIG>
__global__ void __launch_bounds__(kThreads) k_oneway(const PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  oneway<T, BIG>(a, smem, tile_of(a), blockIdx.y);
}

template <typename T, int BIG>
__global__ void __launch_bounds__(kThreads) k_sandwich_c2c(const PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  sandwich_c2c<T, BIG>(a, smem, tile_of(a));
}

template <typename T, int BIG>
__global__ void __launch_bounds__(kThreads) k_sandwich_r2r(const PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  sandwich_r2r<T, BIG>(a, smem, tile_of(a), blockIdx.y);
}

template <auto K>
static void allow_lds() {
  static bool done = false;  // one flag per kernel instantiation
  if (!done) {
    // ask for the whole 160 KB minus the kernel's static LDS; a refusal is
    // not an error here (the launch itself reports a size that does not fit),
    // so clear it instead of leaving it for the next hipGetLastError
    hipFuncAttributes fa{};
    size_t stat = 0;
    if (hipFuncGetAttributes(&fa, (const void*)K) == hipSuccess) stat = fa.sharedSizeBytes;
    else (void)hipGetLastError();
    if (hipFuncSetAttribute((const void*)K, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(160 * 1024 - stat)) != hipSuccess)
      (void)hipGetLastError();
    done = true;
  }
}

template <typename T, int BIG>
static void launch_t(const PassArgs& a, dim3 grid, hipStream_t s) {
  allow_lds<k_oneway<T, BIG>>();
  allow_lds<k_sandwich_c2c<T, BIG>>();
  allow_lds<k_sandwich_r2r<T, BIG>>();
  if (a.kind == PK_ONEWAY)
    hipLaunchKernelGGL((k_oneway<T, BIG>), grid, dim3(kThreads), a.lds_bytes, s, a);
  else if (a.xf == X_C2C_F || a.xf == X_PAIR_F)
    hipLaunchKernelGGL((k_sandwich_c2c<T, BIG>), grid, dim3(kThreads), a.lds_bytes, s, a);
  else
    hipLaunchKernelGGL((k_sandwich_r2r<T, BIG>), grid, dim3(kThreads), a.lds_bytes, s, a);
}

hipError_t launch_pass(const PassArgs& a, int prec, int grid_y, hipStream_t s) {
  const int tiles = ((a.Np + a.P - 1) / a.P) * a.No;
  dim3 grid(tiles, grid_y);
  if (prec == 0) {
    if (a.big) launch_t<float, 1>(a, grid, s);
    else launch_t<float, 0>(a, grid, s);
  } else {
    if (a.big) launch_t<double, 1>(a, grid, s);
    else launch_t<double, 0>(a, grid, s);
  }
  return hipGetLastError();
}

// ------------------------------------------------------- batched persistent
// Every workgroup pulls items (one tile of one pass of one problem) from a
// global queue in order, waits until the pass it depends on is complete,
// runs the tile with the same device code as the one-launch-per-pass path and
// publishes its completion.  Items are ordered pass by pass, so a workgroup
// only ever waits for items that running workgroups took earlier.
__global__ void k_zero_counters(unsigned* c, int n, int* err) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) c[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) err[0] = 0;
}

template <typename T, int BIG>
__global__ void __launch_bounds__(kThreads) k_batched(const PassArgs* passes, const BatchItem* items,
                                                      int nitems, unsigned* counters, int* err) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_item, s_ok;
  // The item index and the wait result are read back with readfirstlane so
  // that the compiler sees them as uniform: the loop then has one uniform
  // exit and every barrier is reached by all threads in every iteration.
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(&counters[0], 1u);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= nitems) break;
    const BatchItem bi = items[it];
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
      const PassArgs& a = passes[bi.pass];
      const int tiles_p = (a.Np + a.P - 1) / a.P;
      for (int k = 0; k < bi.ntile; ++k) {
        const int tile = bi.tile + k;
        Tile t;
        t.o = tile / tiles_p;
        t.p0 = (tile - t.o * tiles_p) * a.P;
        t.np = min(a.P, a.Np - t.p0);
        if (a.kind == PK_ONEWAY) oneway<T, BIG>(a, smem, t, 0);
        else sandwich_r2r<T, BIG>(a, smem, t, 0);
        __syncthreads();  // LDS reuse by the next tile
      }
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

int batched_blocks_per_cu(int lds, int prec, int big) {
  int n = 0;
  hipError_t e;
  if (prec == 0)
    e = big ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batched<float, 1>, kThreads, lds)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batched<float, 0>, kThreads, lds);
  else
    e = big ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batched<double, 1>, kThreads, lds)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batched<double, 0>, kThreads, lds);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return n > 0 ? n : 1;
}

template <typename T, int BIG>
static void launch_batched_t(const PassArgs* passes, const BatchItem* items, int nitems,
                             unsigned* counters, int* err, int grid, int lds, hipStream_t s) {
  allow_lds<k_batched<T, BIG>>();
  hipLaunchKernelGGL((k_batched<T, BIG>), dim3(grid), dim3(kThreads), lds, s, passes, items, nitems,
                     counters, err);
}

hipError_t launch_batched(const PassArgs* passes, const BatchItem* items, int nitems,
                          unsigned* counters, int ncounters, int* err, int grid, int lds,
                          int prec, int big, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_counters, dim3(1 + ncounters / 256), dim3(256), 0, s, counters,
                     ncounters, err);
  if (prec == 0) {
    if (big) launch_batched_t<float, 1>(passes, items, nitems, counters, err, grid, lds, s);
    else launch_batched_t<float, 0>(passes, items, nitems, counters, err, grid, lds, s);
  } else {
    if (big) launch_batched_t<double, 1>(passes, items, nitems, counters, err, grid, lds, s);
    else launch_batched_t<double, 0>(passes, items, nitems, counters, err, grid, lds, s);
  }
  return hipGetLastError();
}

// ------------------------------------------------------ plan-time kernels
// Tabulated integral of the spectral kernel at x >= 0: the nearest table node
// plus the Gauss-Legendre integral of the integrand over the rest (<= step/2).
template <class F>
__device__ double table_integral(double x, const GreenEval& e, F g) {
  int j = (int)(x / e.si_step + 0.5);
  j = min(j, e.si_n - 1);
  const double a = j * e.si_step;
  const double mid = 0.5 * (x + a), half = 0.5 * (x - a);
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) acc += e.gl_w[q] * g(mid + half * e.gl_x[q]);
  return e.si[j] + half * acc;
}

// ln(t) + E1(t), t >= 0 (the ln t singularities cancel): the power series
// -gamma - sum_k (-t)^k / (k k!) for t <= 2, else ln t + E1(t) with E1 from its
// continued fraction e^-t / (t + 1 - 1^2 / (t + 3 - 2^2 / (t + 5 - ...)))
// evaluated by the modified Lentz method.
__device__ double log_plus_e1(double t) {
  const double euler = 0.57721566490153286060651209008240243;
  if (t <= 2.0) {
    double term = 1.0, sum = 0.0;
    for (int k = 1; k <= 40; ++k) {
      term *= -t / k;  // (-t)^k / k!
      const double add = term / k;
      sum += add;
      if (fabs(add) < 1e-18 * fabs(sum)) break;
    }
    return -euler - sum;
  }
  const double tiny = 1e-300;
  double b = t + 1.0, c = 1.0 / tiny, d = 1.0 / b, h = d;
  for (int i = 1; i <= 200; ++i) {
    const double an = -(double)i * i;
    b += 2.0;
    d = 1.0 / (an * d + b);
    c = b + an / c;
    const double del = c * d;
    h *= del;
    if (fabs(del - 1.0) < 1e-16) break;
  }
  return log(t) + h * exp(-t);
}

// G(r) of a 2D or 1D free-space kernel (the readings beside the 3D ones).
__device__ double green_value_low(double r, const GreenEval& e) {
  const double pi = M_PI;
  if (e.dim == 2) {
    if (e.kind == 0) {
      const double euler = 0.57721566490153286060651209008240243;
      const double F = r == 0.0 ? 0.0 : table_integral(e.kc * r, e, [](double t) { return (1.0 - j0(t)) / t; });
      return (F - log(0.5 * e.kc) - euler) / (2.0 * pi);
    }
    // (1 / 2 pi) [ln sigma + (ln 2 + ln t + E1(t)) / 2 - e^-t sum_j L_{j-1}(t) / (2 j)], t = rho^2 / 2
    const double t = 0.5 * (r / e.sigma) * (r / e.sigma);
    double S = 0.0;
    switch (e.kind) {  // sum_{j=1}^{m-1} L_{j-1}(t) / (2 j), expanded
      case 4: S = 0.5; break;
      case 6: S = 0.5 + (1.0 - t) / 4.0; break;
      case 8: S = 0.5 + (1.0 - t) / 4.0 + ((0.5 * t - 2.0) * t + 1.0) / 6.0; break;
      case 10:
        S = 0.5 + (1.0 - t) / 4.0 + ((0.5 * t - 2.0) * t + 1.0) / 6.0 +
            (((-t / 6.0 + 1.5) * t - 3.0) * t + 1.0) / 8.0;
        break;
      default: break;
    }
    return (log(e.sigma) + 0.5 * (M_LN2 + log_plus_e1(t)) - exp(-t) * S) / (2.0 * pi);
  }
  // 1D: the spectral cutoff, or Gaussian order 2m: G2 plus
  // (sigma / sqrt(2 pi)) e^{-rho^2/2} sum_{j=1}^{m-1} (-1)^j He_{2j-2}(rho) / (2^j j!)
  // (the twice-integrated Hermite terms of the order-2m source), in t = rho^2
  const double x = fabs(r);
  if (e.kind == 0) {
    const double si = x == 0.0 ? 0.0 : table_integral(e.kc * x, e, [](double t) { return sin(t) / t; });
    return (x * si + cos(e.kc * x) / e.kc) / pi;
  }
  const double t = (x / e.sigma) * (x / e.sigma);
  double C = 1.0;
  switch (e.kind) {
    case 10: C += (((t - 15.0) * t + 45.0) * t - 15.0) / 384.0; [[fallthrough]];
    case 8: C -= ((t - 6.0) * t + 3.0) / 48.0; [[fallthrough]];
    case 6: C += (t - 1.0) / 8.0; [[fallthrough]];
    case 4: C -= 0.5; break;
    default: break;
  }
  return 0.5 * x * erf(x / (M_SQRT2 * e.sigma)) + e.sigma * exp(-0.5 * t) / sqrt(2.0 * pi) * C;
}

// G(r) of the free-space kernel (GreenEval); see the kernel list in hipoisson.h.
__device__ double green_value(double r, const GreenEval& e) {
  if (e.dim != 3) return green_value_low(r, e);
  if (e.kind == 0) {
    // spectral cutoff: -Si(kc r) / (2 pi^2 r); Si from the nearest table node
    // plus the Gauss-Legendre integral of sin(t) / t over the remaining stretch
    if (r == 0.0) return -e.kc / (2.0 * M_PI * M_PI);
    const double x = e.kc * r;
    int j = (int)(x / e.si_step + 0.5);
    j = min(j, e.si_n - 1);
    const double a = j * e.si_step;
    const double mid = 0.5 * (x + a), half = 0.5 * (x - a);
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double t = mid + half * e.gl_x[q];
      acc += e.gl_w[q] * sin(t) / t;
    }
    return -(e.si[j] + half * acc) / (2.0 * M_PI * M_PI * r);
  }
  // Gaussian order 2m: -(1 / (4 pi sigma)) [erf(rho / sqrt2) / rho
  //                    + sqrt(2 / pi) exp(-rho^2 / 2) S_m(rho^2)], with the
  // Hermite sum S_m expanded in t = rho^2
  const double rho = r / e.sigma, t = rho * rho;
  const double s2pi = 0.79788456080286535587989211986876;  // sqrt(2 / pi)
  const double E = rho == 0.0 ? s2pi : erf(rho / M_SQRT2) / rho;
  double S = 0.0;
  switch (e.kind) {
    case 4: S = 0.5; break;
    case 6: S = (7.0 - t) / 8.0; break;
    case 8: S = ((t - 16.0) * t + 57.0) / 48.0; break;
    case 10: S = (((29.0 - t) * t - 233.0) * t + 561.0) / 384.0; break;
    default: break;
  }
  return -(E + s2pi * exp(-0.5 * t) * S) / (4.0 * M_PI * e.sigma);
}

__global__ void k_green_eval(double* g, int M0, int M1, int M2, double h0, double h1,
                             double h2, const GreenEval e, double scale) {
  const long long total = (long long)M0 * M1 * M2;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int z = (int)(i % M2);
    const int y = (int)((i / M2) % M1);
    const int x = (int)(i / ((long long)M1 * M2));
    const double dx = min(x, M0 - x) * h0, dy = min(y, M1 - y) * h1, dz = min(z, M2 - z) * h2;
    g[i] = green_value(sqrt(dx * dx + dy * dy + dz * dz), e) * scale;
  }
}

hipError_t launch_green_eval(double* g, const int M[3], const double h[3], const GreenEval& ge,
                             double scale, hipStream_t s) {
  if (ge.kind == 0 && (!ge.si || ge.si_n < 1)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_green_eval, dim3(4096), dim3(256), 0, s, g, M[0], M[1], M[2], h[0], h[1],
                     h[2], ge, scale);
  return hipGetLastError();
}

// Weighted sum of the boundary-augmented source (zero-mode query): grid-stride
// accumulation in FP64, one partial per block.
template <typename T>
__global__ void __launch_bounds__(256) k_zero_mode(const PassArgs a, const T* f, int n0, int n1,
                                                   int n2, int t0, int t1, int t2, double* partial) {
  __shared__ double red[256];
  const long long total = (long long)n0 * n1 * n2;
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int i2 = (int)(i % n2), i1 = (int)((i / n2) % n1), i0 = (int)(i / ((long long)n1 * n2));
    double w = 1.0;
    if (t0 && (i0 == 0 || i0 == n0 - 1)) w *= 0.5;
    if (t1 && (i1 == 0 || i1 == n1 - 1)) w *= 0.5;
    if (t2 && (i2 == 0 || i2 == n2 - 1)) w *= 0.5;
    acc += w * ((double)f[i] + face_terms<T>(a, i0, i1, i2));
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

hipError_t launch_zero_mode(const PassArgs& a, const void* f, const int n[3], const int trap[3],
                            double* partial, int nb, int prec, hipStream_t s) {
  if (prec == 0)
    hipLaunchKernelGGL(k_zero_mode<float>, dim3(nb), dim3(256), 0, s, a, (const float*)f, n[0], n[1],
                       n[2], trap[0], trap[1], trap[2], partial);
  else
    hipLaunchKernelGGL(k_zero_mode<double>, dim3(nb), dim3(256), 0, s, a, (const double*)f, n[0],
                       n[1], n[2], trap[0], trap[1], trap[2], partial);
  return hipGetLastError();
}

// ------------------------------------------------- reference streaming copy
// A plain copy with 16-byte nontemporal loads and stores: every workgroup
// copies one contiguous 16 KiB chunk, four accesses in flight per thread (of
// the shapes measured, this one moved the most bytes per second; the
// nontemporal hint keeps the streamed data from displacing cache lines).  The
// bandwidth a kernel doing nothing but streaming reaches on the device: the
// measured ceiling beside the HBM specification.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyPer = 4;  // 16-byte accesses per thread

__global__ void __launch_bounds__(256) k_copy16(const u32x4* __restrict__ src,
                                                u32x4* __restrict__ dst, long long n16) {
  const long long base = (long long)blockIdx.x * (kCopyPer * 256) + threadIdx.x;
  u32x4 v[kCopyPer];
#pragma unroll
  for (int k = 0; k < kCopyPer; ++k) {
    const long long i = base + (long long)k * 256;
    if (i < n16) v[k] = __builtin_nontemporal_load(&src[i]);
  }
#pragma unroll
  for (int k = 0; k < kCopyPer; ++k) {
    const long long i = base + (long long)k * 256;
    if (i < n16) __builtin_nontemporal_store(v[k], &dst[i]);
  }
}

__global__ void k_copy_tail(const unsigned char* src, unsigned char* dst, long long n) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const long long n16 = (long long)(bytes / 16);
  if (n16 > 0) {
    const long long per = (long long)kCopyPer * 256;
    const long long grid = (n16 + per - 1) / per;
    if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)grid), dim3(256), 0, s, (const u32x4*)src,
                       (u32x4*)dst, n16);
  }
  const long long tail = (long long)(bytes - (size_t)n16 * 16);
  if (tail > 0)
    hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(64), 0, s, (const unsigned char*)src + n16 * 16,
                       (unsigned char*)dst + n16 * 16, tail);
  return hipGetLastError();
}

// ------------------------------------------ allocation-free zero-mode query
// The per-block partial sums of every component live in this file-scope
// device array instead of plan memory.  Each device holds its own copy (at
// its own address) until the process ends; in host code the name is only a
// stand-in, so host code uses the address that hipGetSymbolAddress returns
// for the device, never the name itself.
static __device__ __align__(256) double scratch[kZeroModeMaxComp * kZeroModeBlocks];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};
}  // namespace

hipError_t zero_mode_scratch(hipStream_t s, double** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipStreamGetDevice(s, &dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) {
      const hipError_t r = hipSetDevice(cur);
      if (e == hipSuccess) e = r;
    }
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = (double*)g_scratch_ptr[dev];
  return hipSuccess;
}

// out[c] = (partials of component c summed in block order) / W[c]; one
// thread per component, so the sum is the same as a host loop over them.
__global__ void k_zero_mode_finish(const double* partial, int nb, int ncomp, double W0, double W1,
                                   double W2, double* out) {
  const int c = threadIdx.x;
  if (c >= ncomp) return;
  const double W = c == 0 ? W0 : (c == 1 ? W1 : W2);
  double sum = 0.0;
  if (W != 0.0) {
    for (int i = 0; i < nb; ++i) sum += partial[(long long)c * nb + i];
    sum /= W;
  }
  out[c] = sum;
}

hipError_t launch_zero_mode_noalloc(const PassArgs* a, const void* const* f, int ncomp,
                                    const int n[3], const int trap[3], const double* W,
                                    double* out, int prec, hipStream_t s) {
  if (ncomp < 1 || ncomp > kZeroModeMaxComp) return hipErrorInvalidValue;
  double* partial = nullptr;
  hipError_t e = zero_mode_scratch(s, &partial);
  if (e != hipSuccess) return e;
  for (int c = 0; c < ncomp; ++c) {
    if (W[c] == 0.0) continue;  // no zero eigenvalue: the finish kernel writes 0
    e = launch_zero_mode(a[c], f[c], n, trap, partial + (long long)c * kZeroModeBlocks,
                         kZeroModeBlocks, prec, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_zero_mode_finish, dim3(1), dim3(64), 0, s, partial, kZeroModeBlocks, ncomp,
                     W[0], ncomp > 1 ? W[1] : 0.0, ncomp > 2 ? W[2] : 0.0, out);
  return hipGetLastError();
}

template <typename T>
__global__ void k_octant(const double* spec, int M0, int M1, int K2, double scale, T* out) {
  const int O0 = M0 / 2 + 1, O1 = M1 / 2 + 1;
  const long long total = (long long)O0 * O1 * K2;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % O0);
    const int y = (int)((i / O0) % O1);
    const int z = (int)(i / ((long long)O0 * O1));
    const long long src = ((long long)x * M1 + y) * K2 + z;
    out[i] = (T)(spec[2 * src] * scale);
  }
}

hipError_t launch_octant(const double* spec, const int M[3], double scale, void* out, int prec,
                         hipStream_t s) {
  const int K2 = M[2] / 2 + 1;
  if (prec == 0)
    hipLaunchKernelGGL(k_octant<float>, dim3(2048), dim3(256), 0, s, spec, M[0], M[1], K2, scale,
                       (float*)out);
  else
    hipLaunchKernelGGL(k_octant<double>, dim3(2048), dim3(256), 0, s, spec, M[0], M[1], K2, scale,
                       (double*)out);
  return hipGetLastError();
}

// Green's spectrum rows of the free axis (see launch_semi_green).  The DFT of
// the mirrored samples of G = -exp(-kappa x) / (2 kappa) sums two geometric
// series in q = exp(-kappa h); with s = (-1)^m q^n (n = M / 2) and
// theta = 2 pi m / M it is
//   -(1 - s)(1 - q^2) / (2 kappa ((1 - q)^2 + 4 q sin^2(theta / 2))),
// a sum of positive terms in the denominator (no cancellation).  kappa = 0
// (G = |x| / 2): h n^2 / 2 at m = 0, else -h (1 - (-1)^m) / (4 sin^2(theta / 2)).
// odd: G' = sign(x) exp(-kappa |x|) / 2 sampled at j = 1 .. n - 1 and with
// the opposite sign at M - j (0 at j = 0 and n); its bin m is -i times
// Im sum_{j=1}^{n-1} z^j, z = q e^{i theta}, a geometric series whose sum
// (z - s) / (1 - z) gives the stored b(m) (bin = i b):
//   -q sin(theta) (1 - s) / ((1 - q)^2 + 4 q sin^2(theta / 2)),
// for kappa = 0 (q = 1) -(1 - (-1)^m) cot(theta / 2) / 2, 0 at m = 0.
template <typename T>
__global__ void k_semi_green(T* out, const double* lam1, int n1, const double* lam2, int n2, int M,
                             double h, double scale, int odd) {
  const int K = M / 2 + 1, n = M / 2;
  const long long total = (long long)K * n1 * n2;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int m = (int)(i % K);
    const long long r = i / K;
    const int i1 = (int)(r % n1), i2 = (int)(r / n1);
    const double lam = lam1[i1] + (lam2 ? lam2[i2] : 0.0);
    const double sh = sinpi((double)m / (double)M);  // sin(theta / 2)
    const double sgn = (m & 1) ? -1.0 : 1.0;
    double v;
    if (odd) {
      const double st = sinpi(2.0 * (double)m / (double)M);  // sin(theta)
      if (lam < 0.0) {
        const double kappa = sqrt(-lam);
        const double q = exp(-kappa * h);
        const double omq = -expm1(-kappa * h);
        const double s = sgn * exp(-kappa * h * n);
        v = -q * st * (1.0 - s) / (omq * omq + 4.0 * q * sh * sh);
      } else {
        v = m == 0 ? 0.0 : -0.5 * (1.0 - sgn) * cospi((double)m / (double)M) / sh;
      }
    } else if (lam < 0.0) {
      const double kappa = sqrt(-lam);
      const double q = exp(-kappa * h);
      const double omq = -expm1(-kappa * h);       // 1 - q
      const double omq2 = -expm1(-2.0 * kappa * h);  // 1 - q^2
      const double s = sgn * exp(-kappa * h * n);
      v = -(1.0 - s) * omq2 / (2.0 * kappa * (omq * omq + 4.0 * q * sh * sh));
    } else if (m == 0) {
      v = 0.5 * h * (double)n * (double)n;
    } else {
      v = -h * (1.0 - sgn) / (4.0 * sh * sh);
    }
    out[i] = (T)(scale * v);
  }
}

hipError_t launch_semi_green(void* out, const double* lam1, int n1, const double* lam2, int n2,
                             int M, double h, double scale, int odd, int prec, hipStream_t s) {
  if (prec == 0)
    hipLaunchKernelGGL(k_semi_green<float>, dim3(1024), dim3(256), 0, s, (float*)out, lam1, n1, lam2,
                       n2, M, h, scale, odd);
  else
    hipLaunchKernelGGL(k_semi_green<double>, dim3(1024), dim3(256), 0, s, (double*)out, lam1, n1,
                       lam2, n2, M, h, scale, odd);
  return hipGetLastError();
}

struct FacePtrs {
  const void* f[3][2];
};

// Boundary nodes of the REGULAR Dirichlet axes (bit a of `axes`) of an
// output [N0][N1][N2]: block row blockIdx.y = 2 a + side walks face (a, side)
// only, one thread per node, the node's other two coordinates row-major (the
// face array's own index).  A node on several such faces is written once, by
// the face of its highest axis.  32-bit node indices within a face: the
// launch refuses faces of 2^30 nodes or more.
template <typename T>
__global__ void k_dirichlet_fill(T* out, int N0, int N1, int N2, int ndim, int axes, FacePtrs fp) {
  const int N[3] = {N0, N1, N2};
  const int a = blockIdx.y >> 1, side = blockIdx.y & 1;
  if (a >= ndim || !((axes >> a) & 1)) return;
  const int o0 = a == 0 ? 1 : 0, o1 = a == 2 ? 1 : 2;  // the other axes, in order
  const int n1 = N[o1], fsize = N[o0] * N[o1];
  const T* g = (const T*)fp.f[a][side];
  const long long st[3] = {(long long)N1 * N2, (long long)N2, 1LL};
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < fsize; j += gridDim.x * blockDim.x) {
    int c[3];
    c[a] = side ? N[a] - 1 : 0;
    c[o0] = j / n1;
    c[o1] = j - c[o0] * n1;
    bool own = true;
    for (int b = a + 1; b < ndim; ++b)
      if (((axes >> b) & 1) && (c[b] == 0 || c[b] == N[b] - 1)) own = false;
    if (!own) continue;
    out[c[0] * st[0] + c[1] * st[1] + c[2] * st[2]] = g ? g[j] : (T)0;
  }
}

hipError_t launch_dirichlet_fill(void* out, const int N[3], int ndim, int axes, const void* face[3][2],
                                 int prec, hipStream_t s) {
  FacePtrs fp;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 2; ++b) fp.f[a][b] = face[a][b];
  long long fmax = 1;
  for (int a = 0; a < 3; ++a) fmax = std::max(fmax, (long long)N[0] * N[1] * N[2] / std::max(N[a], 1));
  if (fmax >= (1LL << 30)) return hipErrorInvalidValue;
  const int bx = (int)std::min<long long>((fmax + 255) / 256, 1024);
  if (prec == 0)
    hipLaunchKernelGGL(k_dirichlet_fill<float>, dim3(bx, 6), dim3(256), 0, s, (float*)out, N[0],
                       N[1], N[2], ndim, axes, fp);
  else
    hipLaunchKernelGGL(k_dirichlet_fill<double>, dim3(bx, 6), dim3(256), 0, s, (double*)out, N[0],
                       N[1], N[2], ndim, axes, fp);
  return hipGetLastError();
}

}  // namespace hp
