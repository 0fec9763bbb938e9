// Free-space (doubled-domain) passes with one FFT per wavefront, for
// power-of-two doubled lengths L = 64 .. 1024.
//
// A pencil of length L is held by G = L / R0 lanes, R0 elements per lane:
// lane g holds x[g + G i], i < R0.  The first Stockham stage (radix R0) works
// on those registers directly; the following radix-8 (and a final radix-2/4)
// stages exchange data through a wavefront-private LDS slot, so no workgroup
// barrier is needed inside the FFT.  After the last stage lane g holds
// X[g + G i] again, which is also the input layout of the next FFT: the
// sandwich pass multiplies in registers and transforms back at once.
//
// Hockney-Eastwood pruning (Section 3, remark on the 2^(d-1) cost): only the
// physical half of every doubled axis is loaded (the other half is known to be
// zero, i >= R0/2 is a compile-time zero) and only the physical half of every
// backward transform is stored.
//
// Layouts (complex elements):  A1 [x][kz][y],  B2 [kz][ky][x];  user fields
// [x][y][z] real.  Passes whose pencil is strided in memory stage a tile of P
// pencils through LDS so that global accesses are runs of P elements.
#include "hp_device.hpp"
#include "hp_internal.hpp"

namespace hp {

template <int L>
struct WF {
  static constexpr int R0 = L >= 1024 ? 16 : 8;  // elements per lane
  static constexpr int G = L / R0;               // lanes per pencil
  static constexpr int PPW = 64 / G;             // pencils per wavefront
};

__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }

// One Stockham stage (radix R, NS = product of earlier radices) over the
// wavefront slot `buf` (element m at buf[m * bs]).
template <typename T, int L, int R, int NS, bool LAST, bool INV>
__device__ __forceinline__ void wstage(C2<T> (&x)[WF<L>::R0], C2<T>* buf, int bs, int g,
                                       const C2<T>* tw) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G, NB = R0 / R;
  C2<T> v[R0];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = g + G * b;
#pragma unroll
    for (int t = 0; t < R; ++t) v[b * R + t] = buf[(j + t * (L / R)) * bs];
  }
  wave_sync();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = g + G * b;
    const int k = j % NS;
#pragma unroll
    for (int t = 1; t < R; ++t) {
      C2<T> w = tw[t * k * (L / (NS * R))];
      if (INV) w.im = -w.im;
      v[b * R + t] = cmul(v[b * R + t], w);
    }
    dftN<T, R, INV>(&v[b * R]);
    if constexpr (LAST) {
#pragma unroll
      for (int t = 0; t < R; ++t) x[b + t * NB] = v[b * R + t];
    } else {
#pragma unroll
      for (int t = 0; t < R; ++t) buf[((j - k) * R + k + t * NS) * bs] = v[b * R + t];
    }
  }
  if constexpr (!LAST) wave_sync();
}

// In-place FFT of the pencil held as x[i] = x[g + G i]; on return x[i] = X[g + G i].
template <typename T, int L, bool INV>
__device__ __forceinline__ void wave_fft(C2<T> (&x)[WF<L>::R0], C2<T>* buf, int bs, int g,
                                         const C2<T>* tw) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G;
  dftN<T, R0, INV>(x);
  wave_sync();
#pragma unroll
  for (int t = 0; t < R0; ++t) buf[(g * R0 + t) * bs] = x[t];
  wave_sync();
  if constexpr (G == 8) {
    wstage<T, L, 8, R0, true, INV>(x, buf, bs, g, tw);
  } else {
    wstage<T, L, 8, R0, false, INV>(x, buf, bs, g, tw);
    wstage<T, L, G / 8, 8 * R0, true, INV>(x, buf, bs, g, tw);
  }
}

template <typename T, int L>
__device__ __forceinline__ void load_tw(C2<T>* tw_s, const void* tw) {
  const C2<T>* src = (const C2<T>*)tw;
  for (int m = threadIdx.x; m < L; m += kThreads) tw_s[m] = src[m];
}

// signed index m~ of m on an M-point grid, 0 at the Nyquist index
__device__ __forceinline__ int signed_index(int m, int M) {
  return (2 * m < M) ? m : ((2 * m == M) ? 0 : m - M);
}

// ------------------------------------------------------------ P1: R2C (z)
// Rows (x, y) of the real source, z < n2 of L = M2; pairs of rows (y, y+1)
// form one complex FFT; the half spectrum is untangled and written to
// A1[x][kz][y] through a [K2][P] tile.
template <typename T, int L, int P>
__global__ void __launch_bounds__(kThreads) kf_r2c(const PassArgs a) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G, PPW = WF<L>::PPW;
  constexpr int K2 = L / 2 + 1, TS = P + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  C2<T>* tw = (C2<T>*)smem;
  C2<T>* exch = tw + L;
  C2<T>* tile = exch + 4 * PPW * L;
  const T* in = (const T*)a.in[blockIdx.y];
  C2<T>* out = (C2<T>*)a.out[blockIdx.y];
  if (!in) return;
  const int n0 = a.un[0], n1 = a.un[1], n2 = a.un[2];
  const int ytiles = (n1 + P - 1) / P;
  const int x = blockIdx.x / ytiles, y0 = (blockIdx.x % ytiles) * P;
  load_tw<T, L>(tw, a.tw);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = lane / G, g = lane % G;
  C2<T>* buf = exch + (wave * PPW + q) * L;
  for (int pr0 = wave * PPW; pr0 < P / 2; pr0 += 4 * PPW) {
    const int pr = pr0 + q;
    const int ya = y0 + 2 * pr, yb = ya + 1;
    const bool va = pr < P / 2 && ya < n1, vb = pr < P / 2 && yb < n1;
    const T* ra = in + ((long long)x * n1 + ya) * n2;
    const T* rb = ra + n2;
    C2<T> v[R0];
#pragma unroll
    for (int i = 0; i < R0; ++i) {
      v[i] = {(T)0, (T)0};
      if (i < R0 / 2) {
        if (va) v[i].re = ra[g + G * i];
        if (vb) v[i].im = rb[g + G * i];
      }
    }
    wave_fft<T, L, false>(v, buf, 1, g, tw);
    wave_sync();
#pragma unroll
    for (int i = 0; i < R0; ++i) buf[g + G * i] = v[i];
    wave_sync();
    if (pr < P / 2) {
#pragma unroll
      for (int i = 0; i <= R0 / 2; ++i) {
        const int k = g + G * i;
        if (k > L / 2) break;
        const C2<T> zk = buf[k];
        const C2<T> zc = cconj(buf[(L - k) & (L - 1)]);
        const C2<T> s = cadd(zk, zc), d = csub(zk, zc);
        tile[k * TS + 2 * pr] = {s.re * (T)0.5, s.im * (T)0.5};
        tile[k * TS + 2 * pr + 1] = {d.im * (T)0.5, -d.re * (T)0.5};
      }
    }
    wave_sync();
  }
  __syncthreads();
  const long long obase = (long long)x * K2 * n1 + y0;
  for (int e = threadIdx.x; e < K2 * P; e += kThreads) {
    const int k = e / P, c = e - (e / P) * P;
    if (y0 + c < n1) out[obase + (long long)k * n1 + c] = tile[k * TS + c];
  }
  (void)n0;
}

// ------------------------------------------------------- P2: forward C2C (y)
// Pencils (x, kz) of A1, y < n1 of L = M1, written to B2[kz][ky][x] through a
// [L][P] tile whose columns double as the FFT exchange slots.
template <typename T, int L, int P>
__global__ void __launch_bounds__(kThreads) kf_fwd_y(const PassArgs a) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G, PPW = WF<L>::PPW;
  constexpr int TS = P + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  C2<T>* tw = (C2<T>*)smem;
  C2<T>* tile = tw + L;
  const C2<T>* in = (const C2<T>*)a.in[blockIdx.y];
  C2<T>* out = (C2<T>*)a.out[blockIdx.y];
  if (!in) return;
  const int n0 = a.un[0], n1 = a.un[1];
  const int K2 = a.gM[2] / 2 + 1;
  const int xtiles = (n0 + P - 1) / P;
  const int kz = blockIdx.x / xtiles, x0 = (blockIdx.x % xtiles) * P;
  load_tw<T, L>(tw, a.tw);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = lane / G, g = lane % G;
  for (int pp = wave * PPW; pp < P; pp += 4 * PPW) {
    const int p = pp + q;
    const bool valid = p < P && x0 + p < n0;
    const C2<T>* src = in + ((long long)(x0 + p) * K2 + kz) * n1;
    C2<T> v[R0];
#pragma unroll
    for (int i = 0; i < R0; ++i) {
      v[i] = {(T)0, (T)0};
      if (i < R0 / 2 && valid) v[i] = src[g + G * i];
    }
    C2<T>* col = tile + (p < P ? p : 0);
    wave_fft<T, L, false>(v, col, TS, g, tw);
    if (p < P) {
#pragma unroll
      for (int i = 0; i < R0; ++i) col[(g + G * i) * TS] = v[i];
    }
    wave_sync();
  }
  __syncthreads();
  const long long obase = (long long)kz * L * n0 + x0;
  for (int e = threadIdx.x; e < L * P; e += kThreads) {
    const int ky = e / P, c = e - (e / P) * P;
    if (x0 + c < n0) out[obase + (long long)ky * n0 + c] = tile[ky * TS + c];
  }
}

// --------------------------------------------------------- P3: sandwich (x)
// Pencils (ky, kz) of B2, x < n0 of L = M0: forward FFT, Ghat multiply,
// spectral derivative, backward FFT, x < n0 stored, all in registers.
template <typename T, int L>
__global__ void __launch_bounds__(kThreads) kf_sandwich(const PassArgs a) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G, PPW = WF<L>::PPW;
  extern __shared__ __align__(16) unsigned char smem[];
  C2<T>* tw = (C2<T>*)smem;
  C2<T>* exch = tw + L;
  const int n0 = a.un[0];
  const int M1 = a.gM[1], M2 = a.gM[2], K2 = M2 / 2 + 1;
  load_tw<T, L>(tw, a.tw);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = lane / G, g = lane % G;
  C2<T>* buf = exch + (wave * PPW + q) * L;
  const long long total = (long long)M1 * K2;
  const int fb = a.diff == D_NONE ? (int)blockIdx.y : 0;
  const T* gtab = (const T*)a.green;

  auto load = [&](C2<T> (&v)[R0], const void* src, long long base, bool valid) {
    const C2<T>* s = (const C2<T>*)src;
#pragma unroll
    for (int i = 0; i < R0; ++i) {
      v[i] = {(T)0, (T)0};
      if (i < R0 / 2 && valid) v[i] = s[base + g + G * i];
    }
  };
  auto store = [&](const C2<T> (&v)[R0], void* dst, long long base, bool valid) {
    C2<T>* d = (C2<T>*)dst;
    if (!valid) return;
#pragma unroll
    for (int i = 0; i < R0 / 2; ++i) d[base + g + G * i] = v[i];
  };

  for (long long grp = (long long)blockIdx.x * 4 + wave; grp * PPW < total;
       grp += (long long)gridDim.x * 4) {
    const long long pen = grp * PPW + q;
    const bool valid = pen < total;
    const int ky = valid ? (int)(pen % M1) : 0;
    const int kz = valid ? (int)(pen / M1) : 0;
    const long long base = ((long long)kz * M1 + ky) * n0;
    // Green's spectrum along the pencil and the wavenumbers
    const int i1 = min(ky, M1 - ky);
    const T* grow = gtab + (long long)kz * a.g_s[2] + (long long)i1 * a.g_s[1];
    T gv[R0], kx[R0];
#pragma unroll
    for (int i = 0; i < R0; ++i) {
      const int k0 = g + G * i;
      gv[i] = grow[min(k0, L - k0)];
      kx[i] = (T)(a.kc[0] * signed_index(k0, L));
    }
    const T kyv = (T)(a.kc[1] * signed_index(ky, M1));
    const T kzv = (T)(a.kc[2] * signed_index(kz, M2));
    auto kcomp = [&](int c, int i) -> T { return c == 0 ? kx[i] : (c == 1 ? kyv : kzv); };

    if (a.diff == D_NONE) {
      C2<T> v[R0];
      load(v, a.in[fb], base, valid);
      wave_fft<T, L, false>(v, buf, 1, g, tw);
#pragma unroll
      for (int i = 0; i < R0; ++i) v[i] = cscale(v[i], gv[i]);
      wave_fft<T, L, true>(v, buf, 1, g, tw);
      store(v, a.out[fb], base, valid);
    } else if (a.diff == D_CURL || a.diff == D_ADJ_CURL) {
      C2<T> S[3][R0];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (a.in[c]) {
          load(S[c], a.in[c], base, valid);
          wave_fft<T, L, false>(S[c], buf, 1, g, tw);
        } else {
#pragma unroll
          for (int i = 0; i < R0; ++i) S[c][i] = {(T)0, (T)0};
        }
      }
      if (a.diff == D_ADJ_CURL) {
        // the curl is symmetric: g_i enters S_{i+1} with +i k_{i+2}, S_{i+2} with -i k_{i+1}
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (!a.in[3 + c]) continue;
          C2<T> w[R0];
          load(w, a.in[3 + c], base, valid);
          wave_fft<T, L, false>(w, buf, 1, g, tw);
          const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
#pragma unroll
          for (int i = 0; i < R0; ++i) {
            const C2<T> iw = cmuli(w[i]);
            S[c1][i] = cadd(S[c1][i], cscale(iw, kcomp(c2, i)));
            S[c2][i] = csub(S[c2][i], cscale(iw, kcomp(c1, i)));
          }
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < R0; ++i) S[c][i] = cscale(S[c][i], gv[i]);
      if (a.diff == D_CURL) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const int c1 = (d + 1) % 3, c2 = (d + 2) % 3;
          C2<T> u[R0];
#pragma unroll
          for (int i = 0; i < R0; ++i)
            u[i] = cmuli(csub(cscale(S[c2][i], kcomp(c1, i)), cscale(S[c1][i], kcomp(c2, i))));
          wave_fft<T, L, true>(u, buf, 1, g, tw);
          store(u, a.out[3 + d], base, valid);
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        wave_fft<T, L, true>(S[c], buf, 1, g, tw);
        store(S[c], a.out[c], base, valid);
      }
    } else {  // D_GRAD / D_ADJ_GRAD on a scalar
      C2<T> S[R0];
      if (a.in[0]) {
        load(S, a.in[0], base, valid);
        wave_fft<T, L, false>(S, buf, 1, g, tw);
      } else {
#pragma unroll
        for (int i = 0; i < R0; ++i) S[i] = {(T)0, (T)0};
      }
      if (a.diff == D_ADJ_GRAD) {
        // transpose of the gradient: minus the divergence
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (!a.in[1 + c]) continue;
          C2<T> w[R0];
          load(w, a.in[1 + c], base, valid);
          wave_fft<T, L, false>(w, buf, 1, g, tw);
#pragma unroll
          for (int i = 0; i < R0; ++i) S[i] = csub(S[i], cscale(cmuli(w[i]), kcomp(c, i)));
        }
      }
#pragma unroll
      for (int i = 0; i < R0; ++i) S[i] = cscale(S[i], gv[i]);
      if (a.diff == D_GRAD) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          C2<T> u[R0];
#pragma unroll
          for (int i = 0; i < R0; ++i) u[i] = cscale(cmuli(S[i]), kcomp(c, i));
          wave_fft<T, L, true>(u, buf, 1, g, tw);
          store(u, a.out[1 + c], base, valid);
        }
      }
      wave_fft<T, L, true>(S, buf, 1, g, tw);
      store(S, a.out[0], base, valid);
    }
  }
}

// ------------------------------------------------------- P4: backward C2C (y)
// B2[kz][ky][x] -> B2[kz][y][x] (y < n1), in place, through a [L][P] tile.
template <typename T, int L, int P>
__global__ void __launch_bounds__(kThreads) kf_inv_y(const PassArgs a) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G, PPW = WF<L>::PPW;
  constexpr int TS = P + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  C2<T>* tw = (C2<T>*)smem;
  C2<T>* tile = tw + L;
  const C2<T>* in = (const C2<T>*)a.in[blockIdx.y];
  C2<T>* out = (C2<T>*)a.out[blockIdx.y];
  if (!in) return;
  const int n0 = a.un[0], n1 = a.un[1];
  const int xtiles = (n0 + P - 1) / P;
  const int kz = blockIdx.x / xtiles, x0 = (blockIdx.x % xtiles) * P;
  load_tw<T, L>(tw, a.tw);
  const long long base = (long long)kz * L * n0 + x0;
  for (int e = threadIdx.x; e < L * P; e += kThreads) {
    const int ky = e / P, c = e - (e / P) * P;
    C2<T> v = {(T)0, (T)0};
    if (x0 + c < n0) v = in[base + (long long)ky * n0 + c];
    tile[ky * TS + c] = v;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = lane / G, g = lane % G;
  for (int pp = wave * PPW; pp < P; pp += 4 * PPW) {
    const int p = pp + q;
    C2<T>* col = tile + (p < P ? p : 0);
    C2<T> v[R0];
#pragma unroll
    for (int i = 0; i < R0; ++i) v[i] = col[(g + G * i) * TS];
    wave_fft<T, L, true>(v, col, TS, g, tw);
    if (p < P) {
#pragma unroll
      for (int i = 0; i < R0 / 2; ++i) col[(g + G * i) * TS] = v[i];
    }
    wave_sync();
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n1 * P; e += kThreads) {
    const int y = e / P, c = e - (e / P) * P;
    if (x0 + c < n0) out[base + (long long)y * n0 + c] = tile[y * TS + c];
  }
}

// --------------------------------------------------------------- P5: C2R (z)
// Half spectra B2[kz][y][x] (kz < K2) of pencils (x, y) through a [K2][P]
// tile; pairs of pencils form one complex inverse FFT; z < n2 stored into the
// real output [x][y][z].
template <typename T, int L, int P>
__global__ void __launch_bounds__(kThreads) kf_c2r(const PassArgs a) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G, PPW = WF<L>::PPW;
  constexpr int K2 = L / 2 + 1, TS = P + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  C2<T>* tw = (C2<T>*)smem;
  C2<T>* exch = tw + L;
  C2<T>* tile = exch + 4 * PPW * L;
  const C2<T>* in = (const C2<T>*)a.in[blockIdx.y];
  T* out = (T*)a.out[blockIdx.y];
  if (!in) return;
  const int n0 = a.un[0], n1 = a.un[1], n2 = a.un[2];
  const int M1 = a.gM[1];
  const int xtiles = (n0 + P - 1) / P;
  const int y = blockIdx.x / xtiles, x0 = (blockIdx.x % xtiles) * P;
  load_tw<T, L>(tw, a.tw);
  const long long ibase = (long long)y * n0 + x0;
  for (int e = threadIdx.x; e < K2 * P; e += kThreads) {
    const int k = e / P, c = e - (e / P) * P;
    C2<T> v = {(T)0, (T)0};
    if (x0 + c < n0) v = in[ibase + (long long)k * M1 * n0 + c];
    tile[k * TS + c] = v;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = lane / G, g = lane % G;
  C2<T>* buf = exch + (wave * PPW + q) * L;
  for (int pr0 = wave * PPW; pr0 < P / 2; pr0 += 4 * PPW) {
    const int pr = pr0 + q;
    const int ca = 2 * (pr < P / 2 ? pr : 0), cb = ca + 1;
    C2<T> v[R0];
#pragma unroll
    for (int i = 0; i < R0; ++i) {
      const int m = g + G * i;
      C2<T> A, B;
      if (m <= L / 2) {
        A = tile[m * TS + ca];
        B = tile[m * TS + cb];
        if (m == 0 || m == L / 2) {
          A.im = (T)0;
          B.im = (T)0;
        }
      } else {
        A = cconj(tile[(L - m) * TS + ca]);
        B = cconj(tile[(L - m) * TS + cb]);
      }
      v[i] = {A.re - B.im, A.im + B.re};
    }
    wave_fft<T, L, true>(v, buf, 1, g, tw);
    const int xa = x0 + ca, xb = xa + 1;
    const bool va = pr < P / 2 && xa < n0, vb = pr < P / 2 && xb < n0;
    T* oa = out + ((long long)xa * n1 + y) * n2;
    T* ob = out + ((long long)xb * n1 + y) * n2;
#pragma unroll
    for (int i = 0; i < R0 / 2; ++i) {
      if (va) oa[g + G * i] = v[i].re;
      if (vb) ob[g + G * i] = v[i].im;
    }
  }
}

// ---------------------------------------------------------------- launch
int fast_lds_bytes(int fast, int L, int P, int K2, int prec) {
  const int cs = prec == 0 ? 8 : 16;
  const int R0 = L >= 1024 ? 16 : 8;
  const int exch = 4 * (64 / (L / R0)) * L;
  switch (fast) {
    case FAST_R2C:
    case FAST_C2R: return (L + exch + K2 * (P + 1)) * cs;
    case FAST_FWD_Y:
    case FAST_INV_Y: return (L + L * (P + 1)) * cs;
    case FAST_SANDWICH: return (L + exch) * cs;
    default: return 0;
  }
}

// Allow up to the full 160 KB of LDS for a kernel (once per instantiation).
template <auto K>
static void allow_lds() {
  static bool done = false;  // one flag per kernel instantiation
  if (!done) {
    (void)hipFuncSetAttribute((const void*)K, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    done = true;
  }
}

template <typename T, int L, int P>
static hipError_t launch_L(const PassArgs& a, int grid_y, hipStream_t s) {
  const int n0 = a.un[0], n1 = a.un[1];
  const int lds = a.lds_bytes;
  switch (a.fast) {
    case FAST_R2C: {
      dim3 grid(((n1 + P - 1) / P) * n0, grid_y);
      allow_lds<kf_r2c<T, L, P>>();
      hipLaunchKernelGGL((kf_r2c<T, L, P>), grid, dim3(kThreads), lds, s, a);
    } break;
    case FAST_FWD_Y: {
      dim3 grid(((n0 + P - 1) / P) * (a.gM[2] / 2 + 1), grid_y);
      allow_lds<kf_fwd_y<T, L, P>>();
      hipLaunchKernelGGL((kf_fwd_y<T, L, P>), grid, dim3(kThreads), lds, s, a);
    } break;
    case FAST_SANDWICH: {
      const long long total = (long long)a.gM[1] * (a.gM[2] / 2 + 1);
      const long long groups = (total + WF<L>::PPW - 1) / WF<L>::PPW;
      dim3 grid((unsigned)((groups + 3) / 4), grid_y);
      allow_lds<kf_sandwich<T, L>>();
      hipLaunchKernelGGL((kf_sandwich<T, L>), grid, dim3(kThreads), lds, s, a);
    } break;
    case FAST_INV_Y: {
      dim3 grid(((n0 + P - 1) / P) * (a.gM[2] / 2 + 1), grid_y);
      allow_lds<kf_inv_y<T, L, P>>();
      hipLaunchKernelGGL((kf_inv_y<T, L, P>), grid, dim3(kThreads), lds, s, a);
    } break;
    case FAST_C2R: {
      dim3 grid(((n0 + P - 1) / P) * n1, grid_y);
      allow_lds<kf_c2r<T, L, P>>();
      hipLaunchKernelGGL((kf_c2r<T, L, P>), grid, dim3(kThreads), lds, s, a);
    } break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int P>
static hipError_t launch_T(const PassArgs& a, int grid_y, hipStream_t s) {
  switch (a.L) {
    case 64: return launch_L<T, 64, P>(a, grid_y, s);
    case 128: return launch_L<T, 128, P>(a, grid_y, s);
    case 256: return launch_L<T, 256, P>(a, grid_y, s);
    case 512: return launch_L<T, 512, P>(a, grid_y, s);
    case 1024: return launch_L<T, 1024, P>(a, grid_y, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fast(const PassArgs& a, int prec, int grid_y, hipStream_t s) {
  if (prec == 0) {
    if (a.P != 16) return hipErrorInvalidValue;
    return launch_T<float, 16>(a, grid_y, s);
  }
  if (a.P != 8) return hipErrorInvalidValue;
  return launch_T<double, 8>(a, grid_y, s);
}

}  // namespace hp
