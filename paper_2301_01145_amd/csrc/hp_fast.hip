// Free-space (doubled-domain) passes with one FFT per wavefront
// (hp_wavefft.hpp), for power-of-two doubled lengths L = 64 .. 1024.  After
// an FFT lane g holds X[g + G i], which is also the input layout of the next
// FFT: the sandwich pass multiplies in registers and transforms back at once.
//
// Hockney-Eastwood pruning (Section 3, remark on the 2^(d-1) cost): only the
// physical half of every doubled axis is loaded (the other half is known to be
// zero, i >= R0/2 is a compile-time zero) and only the physical half of every
// backward transform is stored.
//
// Layouts (complex elements):  A1 [x][kz][y],  B2 [kz][ky][x];  user fields
// [x][y][z] real.  Passes whose pencil is strided in memory stage a tile of P
// pencils through LDS so that global accesses are runs of P elements.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "hp_device.hpp"
#include "hp_internal.hpp"
#include "hp_wavefft.hpp"

namespace hp {

constexpr int kC2RThreads = 256;  // workgroup of the C2R pass

template <typename T, int L>
__device__ __forceinline__ void load_tw(C2<T>* tw_s, const void* tw) {
  const C2<T>* src = (const C2<T>*)tw;
  for (int m = threadIdx.x; m < L; m += kC2RThreads) tw_s[m] = src[m];
}

// ------------------------------------------------------------ P1: R2C (z)
// Rows (x, y) of the real source, z < n2 of L = M2; pairs of rows (y, y+1)
// form one complex FFT; the half spectrum is untangled and written to
// A1[x][kz][y] through a [K2][P] tile.
template <int L, int P>
struct R2CShape {
  static constexpr int NW = (P / 2 + WF<L>::PPW - 1) / WF<L>::PPW;  // wavefronts
  static constexpr int NT = 64 * NW;
};

template <typename T, int L, int P, bool PAD>
__global__ void __launch_bounds__((R2CShape<L, P>::NT)) kf_r2c(const PassArgs a) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G, PPW = WF<L>::PPW;
  constexpr int NIN = PAD ? R0 / 2 : R0;  // elements per lane read from a row
  constexpr int K2 = L / 2 + 1, TS = P + 1;
  constexpr int NW = R2CShape<L, P>::NW, NT = R2CShape<L, P>::NT;
  extern __shared__ __align__(16) unsigned char smem[];
  C2<T>* tw = (C2<T>*)smem;
  C2<T>* exch = tw + L;
  C2<T>* tile = exch + NW * PPW * slot_len(L);
  const T* in = (const T*)a.in[blockIdx.y];
  C2<T>* out = (C2<T>*)a.out[blockIdx.y];
  if (!in) return;
  const int n0 = a.un[0], n1 = a.un[1], n2 = a.un[2];
  const int ytiles = (n1 + P - 1) / P;
  const int x = blockIdx.x / ytiles, y0 = (blockIdx.x % ytiles) * P;
  for (int m = threadIdx.x; m < L; m += NT) tw[m] = ((const C2<T>*)a.tw)[m];
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int q = lane / G, g = lane % G;
  C2<T>* buf = exch + (wave * PPW + q) * slot_len(L);
  for (int pr0 = wave * PPW; pr0 < P / 2; pr0 += NW * PPW) {
    const int pr = pr0 + q;
    const int ya = y0 + 2 * pr, yb = ya + 1;
    const bool va = pr < P / 2 && ya < n1, vb = pr < P / 2 && yb < n1;
    const T* ra = in + ((long long)x * n1 + ya) * n2;
    const T* rb = ra + n2;
    C2<T> v[R0];
#pragma unroll
    for (int i = 0; i < R0; ++i) {
      v[i] = {(T)0, (T)0};
      if (i < NIN) {
        if (va) v[i].re = ra[g + G * i];
        if (vb) v[i].im = rb[g + G * i];
      }
    }
    wave_fft<T, L, false, PAD>(v, buf, 1, g, tw);
    wave_sync();
#pragma unroll
    for (int i = 0; i < R0; ++i) buf[padrun<PadA, G>(g, i)] = v[i];
    wave_sync();
    if (pr < P / 2) {
#pragma unroll
      for (int i = 0; i <= R0 / 2; ++i) {
        const int k = g + G * i;
        if (k > L / 2) break;
        const C2<T> zk = buf[padrow(k)];
        const C2<T> zc = cconj(buf[padrow((L - k) & (L - 1))]);
        const C2<T> s = cadd(zk, zc), d = csub(zk, zc);
        tile[k * TS + 2 * pr] = {s.re * (T)0.5, s.im * (T)0.5};
        tile[k * TS + 2 * pr + 1] = {d.im * (T)0.5, -d.re * (T)0.5};
      }
    }
    wave_sync();
  }
  __syncthreads();
  const long long obase = (long long)x * K2 * n1 + y0;
  // a compile-time count: every LDS read of the thread is issued before the
  // first store waits for one (a run-time loop reads, waits and stores in turn)
#pragma unroll
  for (int r = 0; r < (K2 * P + NT - 1) / NT; ++r) {
    const int e = threadIdx.x + r * NT;
    const int k = e / P, c = e - (e / P) * P;
    if (e < K2 * P && y0 + c < n1) st_stream(&out[obase + (long long)k * n1 + c], tile[k * TS + c]);
  }
  (void)n0;
}

// ------------------------------------------------------- P2: forward C2C (y)
// Pencils (x, kz) of A1, y < n1 of L = M1, written to B2[kz][ky][x] through a
// [L][P] tile whose columns double as the FFT exchange slots.
template <typename T, int L, int P, bool PAD>
__global__ void __launch_bounds__(64 * (P / WF<L>::PPW)) kf_fwd_y(const PassArgs a) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G, PPW = WF<L>::PPW;
  constexpr int NIN = PAD ? R0 / 2 : R0;
  constexpr int TS = P + 1, NT = 64 * (P / PPW);
  extern __shared__ __align__(16) unsigned char smem[];
  C2<T>* tw = (C2<T>*)smem;
  C2<T>* tile = tw + L;
  const C2<T>* in = (const C2<T>*)a.in[blockIdx.y];
  C2<T>* out = (C2<T>*)a.out[blockIdx.y];
  if (!in) return;
  const int n0 = a.un[0], n1 = a.un[1];
  const int K2 = a.gM[2] / 2 + 1;
  const int xtiles = (n0 + P - 1) / P;
  const int kzl = blockIdx.x / xtiles, x0 = (blockIdx.x % xtiles) * P;
  const int kz = a.kz_base + kzl;  // global kz (A1); kzl indexes the B2 slab
  for (int m = threadIdx.x; m < L; m += NT) tw[m] = ((const C2<T>*)a.tw)[m];
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int q = lane / G, g = lane % G;
  {
    const int pp = wave * PPW;
    const int p = pp + q;
    const bool valid = p < P && x0 + p < n0;
    const C2<T>* src = in + ((long long)(x0 + p) * K2 + kz) * n1;
    C2<T> v[R0];
#pragma unroll
    for (int i = 0; i < R0; ++i) {
      v[i] = {(T)0, (T)0};
      if (i < NIN && valid) v[i] = src[g + G * i];
    }
    C2<T>* col = tile + (p < P ? p : 0);
    wave_fft<T, L, false, PAD>(v, col, TS, g, tw);
    wave_sync();
    if (p < P) {
#pragma unroll
      for (int i = 0; i < R0; ++i) col[padrun<PadA, G>(g, i) * TS] = v[i];
    }
    wave_sync();
  }
  __syncthreads();
  const long long obase = (long long)kzl * L * n0 + x0;
  static_assert((L * P) % NT == 0, "whole rounds of the tile store");
#pragma unroll
  for (int r = 0; r < L * P / NT; ++r) {
    const int e = threadIdx.x + r * NT;
    const int ky = e / P, c = e - (e / P) * P;
    if (x0 + c < n0) st_stream(&out[obase + (long long)ky * n0 + c], tile[padrow(ky) * TS + c]);
  }
}

// --------------------------------------------------------- P3: sandwich (x)
// A tile is P consecutive pencils (ky0 .. ky0+P-1, kz) of B2[kz][ky][x], one
// (or PPW) per wavefront, and one output group.  Each wavefront does the
// forward FFT (x < n0 nonzero of L = M0), the Green's multiply and the
// x-derivative in registers; every output field is transformed back and
// written, x < n0, to an LDS tile, then stored as runs of P along ky into
// C2[kz][x][ky] (the next pass reads its y-pencils contiguously).  Outputs:
// psi and, for the curl, A = -d_x psi_z and B = d_x psi_y (the y and z
// derivatives are applied by the y pass); for the gradient, psi and d_x psi.
//
// Persistent: a workgroup loads the twiddles once and walks tiles
// blockIdx-strided; the input pencil and Green's values of its next tile are
// loaded before the current one is processed, so their latency overlaps the
// FFTs and stores.  Tile order: kz slowest, then pairs of ky tiles
// (t, ytiles-1-t) whose wavenumbers +-ky share Green's function rows, then the
// output groups; the XCD-contiguous numbering keeps such tiles behind one L2.
// EXT: the divergence and the Laplacian (D_DIV, D_NABLA and their
// transposes) in instances of their own; the other instances keep the code
// of psi, the gradient and the curl only.
template <typename T, int L, int P, bool ADJ, bool DBL, bool PAD, bool EXT>
__global__ void __launch_bounds__(64 * (P / WF<L>::PPW),
                                  (sizeof(T) == 4 && P == 8 && L == 512 && !ADJ && !EXT) ? 4 : 1)
    kf_sandwich(const PassArgs a) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G, PPW = WF<L>::PPW;
  constexpr int NIN = PAD ? R0 / 2 : R0;  // elements per lane on the x < n0 side
  constexpr int NT = 64 * (P / PPW), TS = P + 1, NX = PAD ? L / 2 : L;
  extern __shared__ __align__(16) unsigned char smem[];
  // DBL: per-pencil exchange slots and two alternating [NX][P] output tiles
  // (one barrier per output field); otherwise one [slot_len(L)][P] tile whose
  // columns are the exchange slots (two barriers per output field).
  C2<T>* tw = (C2<T>*)smem;
  C2<T>* exch = tw + L;
  C2<T>* tiles = DBL ? exch + P * slot_len(L) : exch;
  const int M1 = a.gM[1], M2 = a.gM[2];
  const int ytiles = M1 / P;  // even: M1 is a power of two >= 64, P <= 16
  const int ngrp = a.ngrp;
  const int ntiles = ytiles * a.kz_count * ngrp;
  int lt = xcd_block(blockIdx.x, gridDim.x);
  if (lt >= ntiles) return;  // whole workgroup
  for (int m = threadIdx.x; m < L; m += NT) tw[m] = ((const C2<T>*)a.tw)[m];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int q = lane / G, g = lane % G;
  const int p = wave * PPW + q;
  C2<T>* col = DBL ? exch + p * slot_len(L) : tiles + p;
  constexpr int bs = DBL ? 1 : TS;
  // wavenumbers in the solve precision (the FP64 product rounded once was
  // three conversions and an FP64 multiply per bin)
  const T kc0 = (T)a.kc[0];
  auto kx = [&](int i) -> T { return kc0 * (T)signed_index(g + G * i, L); };

  struct TileIdx {
    int grp, kzl, ky0;
  };
  auto decode = [&](int l) {
    TileIdx t;
    t.grp = l % ngrp;
    l /= ngrp;
    const int mirror = l & 1;
    l >>= 1;
    const int tj = l % (ytiles / 2);
    t.kzl = l / (ytiles / 2);
    t.ky0 = (mirror ? ytiles - 1 - tj : tj) * P;
    return t;
  };
  auto in_ptr = [&](const TileIdx& t, const void* src) {
    return (const C2<T>*)src + ((long long)t.kzl * M1 + t.ky0 + p) * NX;
  };
  auto green_ptr = [&](const TileIdx& t) {
    const int ky = t.ky0 + p;
    return (const T*)a.green + (long long)(a.kz_base + t.kzl) * a.g_s[2] +
           (long long)min(ky, M1 - ky) * a.g_s[1];
  };
  // spectral multiplier of bin k0 along x: the Green's octant (free space) or
  // norm / (sum of the Table 1 eigenvalues) (periodic; 0 for the zero mode)
  auto mult_of = [&](const TileIdx& t, const T* gr, int k0) -> T {
    if constexpr (PAD) {
      return gr[min(k0, L - k0)];
    } else {
      const double lam = a.lam[0][k0] + a.lam[1][t.ky0 + p] + a.lam[2][a.kz_base + t.kzl];
      if (lam == 0.0) return (T)0;
      return (T)a.norm / (T)lam;
    }
  };
  // single-input groups (D_NONE, forward curl, forward Laplacian): prefetched
  // input and Green's values
  const bool pref = EXT ? (!ADJ && a.diff == D_NABLA) : (a.diff == D_NONE || (!ADJ && a.diff == D_CURL));
  auto src_of = [&](const TileIdx& t) {
    if constexpr (EXT) return a.in[t.grp];
    else return a.in[a.diff == D_NONE || a.diff == D_CURL ? t.grp : 0];
  };
  // GNOW (FP32): the Green's values of a tile are loaded at its start, ahead
  // of its forward transform, instead of a whole tile ahead with the input;
  // the eight registers that frees let the first output transform of a curl
  // group read its twiddles ahead of the exchanges too (A/B on one box:
  // 1.642 -> 1.636 ms; FP64 was 1.4 % slower that way and keeps the prefetch)
  constexpr bool GNOW = sizeof(T) == 4;
  C2<T> pf[NIN];
  T pg[GNOW ? 1 : R0];
  auto prefetch = [&](const TileIdx& t) {
    // an unbound field (adjoint with a zero upstream gradient) reads as zero
    const void* src = src_of(t);
    const T* gr = PAD ? green_ptr(t) : nullptr;
    if (src) {
      const C2<T>* sp = in_ptr(t, src);
#pragma unroll
      for (int i = 0; i < NIN; ++i) pf[i] = sp[g + G * i];
    } else {
#pragma unroll
      for (int i = 0; i < NIN; ++i) pf[i] = {(T)0, (T)0};
    }
    if constexpr (!GNOW) {
#pragma unroll
      for (int i = 0; i < R0; ++i) pg[i] = mult_of(t, gr, g + G * i);
    }
    (void)gr;
  };
  TileIdx cur = decode(lt);
  if (pref) prefetch(cur);
  __syncthreads();  // twiddles
  int tb = 0;
  for (;;) {
    const TileIdx t = cur;
    const int ky = t.ky0 + p;
    const int kz = a.kz_base + t.kzl;  // global kz (Ghat, k_z); t.kzl indexes the B2 / C2 slabs
    const T kyv = (T)(a.kc[1] * signed_index(ky, M1));
    const T kzv = (T)(a.kc[2] * signed_index(kz, M2));
    auto kcomp = [&](int c, int i) -> T { return c == 0 ? kx(i) : (c == 1 ? kyv : kzv); };
    const long long obase = (long long)t.kzl * NX * M1 + t.ky0;
    C2<T> v[R0];
    T gv[R0];
    if (pref) {
      const T* gr = PAD ? green_ptr(t) : nullptr;
      (void)gr;
#pragma unroll
      for (int i = 0; i < R0; ++i) {
        v[i] = i < NIN ? pf[i] : C2<T>{(T)0, (T)0};
        if constexpr (GNOW) gv[i] = mult_of(t, gr, g + G * i);
        else gv[i] = pg[i];
      }
    }
    const int nxt = lt + (int)gridDim.x;
    if (nxt < ntiles) {
      cur = decode(nxt);
      if (pref) prefetch(cur);
    }
    auto green = [&](C2<T> (&w)[R0]) {
      if (pref) {
#pragma unroll
        for (int i = 0; i < R0; ++i) w[i] = cscale(w[i], gv[i]);
      } else {
        const T* gr = PAD ? green_ptr(t) : nullptr;
#pragma unroll
        for (int i = 0; i < R0; ++i) w[i] = cscale(w[i], mult_of(t, gr, g + G * i));
      }
    };
    // forward FFT of the pencil of field `src` (x < n0 nonzero)
    auto load = [&](C2<T> (&w)[R0], const void* src) {
      const C2<T>* sp = in_ptr(t, src);
#pragma unroll
      for (int i = 0; i < R0; ++i) w[i] = i < NIN ? sp[g + G * i] : C2<T>{(T)0, (T)0};
      wave_fft<T, L, false, PAD>(w, col, bs, g, tw);
    };
    // backward FFT, x < n0 of every pencil to the tile, stored along ky
    // TW: the inverse transform's twiddles read ahead of each exchange; only
    // where no second field is live (with the curl's derivative output held
    // beside psi they do not fit the register budget)
    auto emit_tw = [&](auto tw_pre, C2<T> (&w)[R0], void* dst) {
      wave_fft<T, L, true, false, false, decltype(tw_pre)::value>(w, col, bs, g, tw);
      wave_sync();
      C2<T>* tile = DBL ? tiles + tb * NX * TS : tiles;
      auto row = [](int x) { return DBL ? x : padrow(x); };
#pragma unroll
      for (int i = 0; i < NIN; ++i) tile[row(g + G * i) * TS + p] = w[i];
      __syncthreads();
      C2<T>* d = (C2<T>*)dst + obase;
      // compile-time count (all LDS reads before the stores); offsets within
      // the kz slab, NX * M1 <= 2^20
      static_assert((NX * P) % NT == 0, "whole rounds of the tile store");
#pragma unroll
      for (int r = 0; r < NX * P / NT; ++r) {
        const int e = threadIdx.x + r * NT;
        const int x = e / P, c = e - (e / P) * P;
        st_stream(&d[x * M1 + c], tile[row(x) * TS + c]);
      }
      if (DBL) tb ^= 1;
      else __syncthreads();
    };
    auto emit = [&](C2<T> (&w)[R0], void* dst) { emit_tw(std::false_type{}, w, dst); };
    auto emit_last = [&](C2<T> (&w)[R0], void* dst) { emit_tw(std::true_type{}, w, dst); };

    // |k|^2 of bin i (every wavenumber with its Nyquist value zeroed)
    auto ksq = [&](int i) -> T { return kx(i) * kx(i) + kyv * kyv + kzv * kzv; };
    auto zero = [](C2<T> (&w)[R0]) {
#pragma unroll
      for (int i = 0; i < R0; ++i) w[i] = {(T)0, (T)0};
    };
    if constexpr (EXT) {
      const int nc = ngrp;  // components (Laplacian groups)
      if (!ADJ && a.diff == D_NABLA) {
        // psi_c and its Laplacian -|k|^2 psi_c (output nc + c)
        const int c = t.grp;
        wave_fft<T, L, false, PAD>(v, col, bs, g, tw);
        green(v);
        C2<T> u[R0];
#pragma unroll
        for (int i = 0; i < R0; ++i) u[i] = cscale(v[i], -ksq(i));
        emit(u, a.out[nc + c]);
        emit(v, a.out[c]);
      } else if (!ADJ) {
        // D_DIV: psi_0..2 and sum_c i k_c psi_c (output 3)
        C2<T> D[R0];
        zero(D);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          C2<T> w[R0];
          load(w, a.in[c]);
          green(w);
#pragma unroll
          for (int i = 0; i < R0; ++i) D[i] = cadd(D[i], cscale(cmuli(w[i]), kcomp(c, i)));
          emit(w, a.out[c]);
        }
        emit(D, a.out[3]);
      } else if (a.diff == D_ADJ_NABLA) {
        // the Laplacian is symmetric: S_c = g_psi_c - |k|^2 g_lap_c
        const int c = t.grp;
        C2<T> S[R0];
        if (a.in[c]) load(S, a.in[c]);
        else zero(S);
        if (a.in[nc + c]) {
          C2<T> w[R0];
          load(w, a.in[nc + c]);
#pragma unroll
          for (int i = 0; i < R0; ++i) S[i] = csub(S[i], cscale(w[i], ksq(i)));
        }
        green(S);
        emit(S, a.out[c]);
      } else {
        // D_ADJ_DIV, the transpose of the divergence (minus the gradient):
        // S_c = g_psi_c - i k_c g_div
        const bool hd = a.in[3] != nullptr;
        C2<T> Dv[R0];
        if (hd) load(Dv, a.in[3]);
        else zero(Dv);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          C2<T> S[R0];
          if (a.in[c]) load(S, a.in[c]);
          else zero(S);
          if (hd) {
#pragma unroll
            for (int i = 0; i < R0; ++i) S[i] = csub(S[i], cscale(cmuli(Dv[i]), kcomp(c, i)));
          }
          green(S);
          emit(S, a.out[c]);
        }
      }
    } else if (a.diff == D_NONE) {
      wave_fft<T, L, false, PAD>(v, col, bs, g, tw);
      green(v);
      emit_last(v, a.out[t.grp]);
    } else if (!ADJ && a.diff == D_CURL) {
      // one component per output group: psi_c, plus B = d_x psi_y (c = 1) or
      // A = -d_x psi_z (c = 2)
      const int c = t.grp;
      wave_fft<T, L, false, PAD>(v, col, bs, g, tw);
      green(v);
      if (c > 0) {
        C2<T> u[R0];
        const T sgn = c == 1 ? (T)1 : (T)-1;
#pragma unroll
        for (int i = 0; i < R0; ++i) u[i] = cscale(cmuli(v[i]), sgn * kx(i));
        emit_tw(std::integral_constant<bool, GNOW>{}, u, a.out[c == 1 ? 4 : 3]);
      }
      emit_last(v, a.out[c]);
    } else if (ADJ && a.diff == D_ADJ_CURL) {
      C2<T> S[3][R0];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (a.in[c]) {
          load(S[c], a.in[c]);
        } else {
#pragma unroll
          for (int i = 0; i < R0; ++i) S[c][i] = {(T)0, (T)0};
        }
      }
      // the curl is symmetric: g_i enters S_{i+1} with +i k_{i+2}, S_{i+2} with -i k_{i+1}
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (!a.in[3 + c]) continue;
        C2<T> w[R0];
        load(w, a.in[3 + c]);
        const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
#pragma unroll
        for (int i = 0; i < R0; ++i) {
          const C2<T> iw = cmuli(w[i]);
          S[c1][i] = cadd(S[c1][i], cscale(iw, kcomp(c2, i)));
          S[c2][i] = csub(S[c2][i], cscale(iw, kcomp(c1, i)));
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        green(S[c]);
        emit(S[c], a.out[c]);
      }
    } else {  // scalar gradient and its transpose
      C2<T> S[R0];
      if (a.in[0]) {
        load(S, a.in[0]);
      } else {
#pragma unroll
        for (int i = 0; i < R0; ++i) S[i] = {(T)0, (T)0};
      }
      if (ADJ) {
        // transpose of the gradient: minus the divergence
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (!a.in[1 + c]) continue;
          C2<T> w[R0];
          load(w, a.in[1 + c]);
#pragma unroll
          for (int i = 0; i < R0; ++i) S[i] = csub(S[i], cscale(cmuli(w[i]), kcomp(c, i)));
        }
      }
      green(S);
      if (!ADJ) {
        C2<T> u[R0];
#pragma unroll
        for (int i = 0; i < R0; ++i) u[i] = cscale(cmuli(S[i]), kx(i));
        emit(u, a.out[1]);
      }
      emit(S, a.out[0]);
    }
    lt = nxt;
    if (lt >= ntiles) break;
  }
}

// ------------------------------------------------------- P4: backward C2C (y)
// A workgroup takes P consecutive pencils (x, kz0 .. kz0+P-1) of C2[kz][x][ky]
// (each contiguous, all M1 wavenumbers), transforms them back along y and keeps
// y < n1, written through an [L][P] tile (columns = FFT exchange slots) as runs
// of P along kz into C1 ([x][y][kz]).  In curl mode the five inputs psi_x, psi_y,
// psi_z, A, B give psi and u = curl psi (u_x = d_y psi_z - d_z psi_y,
// u_y = d_z psi_x + A, u_z = B - d_y psi_x); in gradient mode psi, d_x psi give
// psi and grad psi.  At most two spectra are live per lane.
template <typename T, int L, int P, bool DBL, bool PAD>
__global__ void __launch_bounds__(64 * (P / WF<L>::PPW)) kf_inv_y(const PassArgs a) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G, PPW = WF<L>::PPW;
  constexpr int NIN = PAD ? R0 / 2 : R0;  // elements per lane stored (y < n1)
  constexpr int NT = 64 * (P / PPW), TS = P + 1, NY = PAD ? L / 2 : L;
  extern __shared__ __align__(16) unsigned char smem[];
  C2<T>* tw = (C2<T>*)smem;
  C2<T>* exch = tw + L;
  // non-double-buffered: the tile columns are the exchange slots, in the
  // short layout so that two workgroups of 16 pencils fit one CU
  constexpr bool SM = !DBL;
  C2<T>* tiles = DBL ? exch + P * slot_len(L) : exch;
  const int n0 = a.un[0];
  const int M2 = a.gM[2], K2 = M2 / 2 + 1;
  const int ztiles = (a.kz_count + P - 1) / P;
  const int x = blockIdx.x / ztiles, kzl0 = (blockIdx.x % ztiles) * P;
  const int kz0 = a.kz_base + kzl0;  // global kz (C1, k_z); kzl indexes the C2 slab
  for (int m = threadIdx.x; m < L; m += NT) tw[m] = ((const C2<T>*)a.tw)[m];
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int q = lane / G, g = lane % G;
  const int p = wave * PPW + q;
  const int kz = kz0 + p;
  const bool valid = kzl0 + p < a.kz_count;
  C2<T>* col = DBL ? exch + p * slot_len(L) : tiles + p;
  constexpr int bs = DBL ? 1 : TS;
  const long long ibase = ((long long)(valid ? kzl0 + p : 0) * n0 + x) * L;
  const long long obase = (long long)x * a.c1_sx + kz0;
  const int nvalid = min(P, a.kz_count - kzl0);
  const T kc1 = (T)a.kc[1];
  auto kyv = [&](int i) -> T { return kc1 * (T)signed_index(g + G * i, L); };
  const T kzv = (T)(a.kc[2] * signed_index(kz, M2));

  auto load = [&](C2<T> (&v)[R0], const void* src) {
    const C2<T>* sp = (const C2<T>*)src + ibase;
#pragma unroll
    // streaming loads here only: measured faster in this pass, slower in the others
    for (int i = 0; i < R0; ++i) v[i] = valid ? ld_stream(&sp[g + G * i]) : C2<T>{(T)0, (T)0};
  };
  int tb = 0;
  auto emit = [&](C2<T> (&v)[R0], void* dst) {
    wave_fft<T, L, true, false, SM>(v, col, bs, g, tw);
    wave_sync();
    C2<T>* tile = DBL ? tiles + tb * NY * TS : tiles;
    auto row = [](int y) { return DBL ? y : padrow(y); };
#pragma unroll
    for (int i = 0; i < NIN; ++i) tile[row(g + G * i) * TS + p] = v[i];
    __syncthreads();
    C2<T>* d = (C2<T>*)dst + obase;
    static_assert((NY * P) % NT == 0, "whole rounds of the tile store");
#pragma unroll
    for (int r = 0; r < NY * P / NT; ++r) {
      const int e = threadIdx.x + r * NT;
      const int y = e / P, c = e - (e / P) * P;
      if (c < nvalid) st_stream(&d[(long long)y * a.c1_sy + c], tile[row(y) * TS + c]);
    }
    if (DBL) tb ^= 1;
    else __syncthreads();
  };

  if (a.iy_mode == IY_PLAIN) {
    C2<T> v[R0];
    load(v, a.in[blockIdx.y]);
    emit(v, a.out[blockIdx.y]);
  } else if (a.iy_mode == IY_CURL5) {
    // two independent output groups (blockIdx.y), no input read twice:
    // {psi_z, u_x, psi_y} from psi_y, psi_z; {u_y, u_z, psi_x} from psi_x, A, B
    C2<T> s[R0], w[R0];
    if (blockIdx.y == 0) {
      load(s, a.in[2]);  // psi_z
#pragma unroll
      for (int i = 0; i < R0; ++i) w[i] = cscale(cmuli(s[i]), kyv(i));  // d_y psi_z
      emit(s, a.out[2]);
      load(s, a.in[1]);  // psi_y
#pragma unroll
      for (int i = 0; i < R0; ++i) w[i] = csub(w[i], cscale(cmuli(s[i]), kzv));  // - d_z psi_y
      emit(w, a.out[3]);
      emit(s, a.out[1]);
    } else {
      load(s, a.in[0]);  // psi_x
      load(w, a.in[3]);  // A
#pragma unroll
      for (int i = 0; i < R0; ++i) w[i] = cadd(w[i], cscale(cmuli(s[i]), kzv));  // d_z psi_x + A
      emit(w, a.out[4]);
      load(w, a.in[4]);  // B
#pragma unroll
      for (int i = 0; i < R0; ++i) w[i] = csub(w[i], cscale(cmuli(s[i]), kyv(i)));  // B - d_y psi_x
      emit(w, a.out[5]);
      emit(s, a.out[0]);
    }
  } else {  // IY_GRAD2
    C2<T> s[R0], w[R0];
    load(s, a.in[0]);
#pragma unroll
    for (int i = 0; i < R0; ++i) w[i] = cscale(cmuli(s[i]), kyv(i));
    emit(w, a.out[2]);
#pragma unroll
    for (int i = 0; i < R0; ++i) w[i] = cscale(cmuli(s[i]), kzv);
    emit(w, a.out[3]);
    emit(s, a.out[0]);
    load(w, a.in[1]);
    emit(w, a.out[1]);
  }
}

// --------------------------------------------------------------- P5: C2R (z)
// Half spectra C1 (kz < K2 contiguous; [x][y][kz]) of pencils (x, y) and
// (x, y + 1) form one complex inverse FFT (Hermitian completion); z < n2 of
// both rows is stored into the real output [x][y][z].
template <typename T, int L, bool PAD>
__global__ void __launch_bounds__(kC2RThreads) kf_c2r(const PassArgs a) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G, PPW = WF<L>::PPW;
  constexpr int NIN = PAD ? R0 / 2 : R0;  // elements per lane stored (z < n2)
  constexpr int K2 = L / 2 + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  C2<T>* tw = (C2<T>*)smem;
  C2<T>* exch = tw + L;
  const C2<T>* in = (const C2<T>*)a.in[blockIdx.y];
  T* out = (T*)a.out[blockIdx.y];
  if (!in) return;
  const int n0 = a.un[0], n1 = a.un[1], n2 = a.un[2];
  load_tw<T, L>(tw, a.tw);
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int q = lane / G, g = lane % G;
  C2<T>* buf = exch + (wave * PPW + q) * slot_len(L);
  const int ypairs = (n1 + 1) / 2;
  const long long total = (long long)n0 * ypairs;
  for (long long grp = (long long)blockIdx.x * 4 + wave; grp * PPW < total;
       grp += (long long)gridDim.x * 4) {
    const long long pr = grp * PPW + q;
    const bool valid = pr < total;
    const int x = valid ? (int)(pr / ypairs) : 0;
    const int ya = valid ? 2 * (int)(pr % ypairs) : 0, yb = ya + 1;
    const bool vb = valid && yb < n1;
    const C2<T>* pa = in + (long long)ya * a.c1_sy + (long long)x * a.c1_sx;
    const C2<T>* pb = pa + a.c1_sy;
    C2<T> v[R0];
#pragma unroll
    for (int i = 0; i < R0; ++i) {
      const int m = g + G * i;
      const int mm = m <= L / 2 ? m : L - m;
      C2<T> A = {(T)0, (T)0}, B = {(T)0, (T)0};
      if (valid) A = pa[mm];
      if (vb) B = pb[mm];
      if (m == 0 || m == L / 2) {
        A.im = (T)0;
        B.im = (T)0;
      } else if (m > L / 2) {
        A = cconj(A);
        B = cconj(B);
      }
      v[i] = {A.re - B.im, A.im + B.re};
    }
    wave_fft<T, L, true>(v, buf, 1, g, tw);
    T* oa = out + ((long long)x * n1 + ya) * n2;
    T* ob = oa + n2;
#pragma unroll
    for (int i = 0; i < NIN; ++i) {
      if (valid) st_stream(&oa[g + G * i], v[i].re);
      if (vb) st_stream(&ob[g + G * i], v[i].im);
    }
  }
}

// ---------------------------------------------------------------- launch
// Pencils per workgroup (runs of P elements on the strided side of a pass):
// FP32 8 or 16 per pass, FP64 8.  One-pencil kernels (C2R) take no tile.
int fast_tile(int fast, int L, int prec) {
  if (fast == FAST_C2R) return 2;
  if (prec != 0) return 8;
  if (L >= 1024) return 8;  // (16-pencil tiles are instantiated below 1024 only)
  static const char* env[] = {"", "HP_TILE_R2C", "HP_TILE_FWDY", "HP_TILE_SAND", "HP_TILE_INVY"};
  if (const char* t = std::getenv(env[fast])) {
    const int v = std::atoi(t);
    if (v == 8 || v == 16) return v;
  }
  // measured on MI355X at 256^3 (doubled 512^3): 8-pencil tiles in the x
  // pass (two workgroups per CU within its register budget), 16 elsewhere
  // (8 there cost 1 % of the solve in R2C and in the forward y pass)
  return fast == FAST_SANDWICH ? 8 : 16;
}

bool fast_tile_ok(int fast, int L, int P, int prec) {
  if (fast == FAST_C2R) return P == 2;
  if (fast < FAST_R2C || fast > FAST_INV_Y) return false;
  return P == 8 || (P == 16 && prec == 0 && L < 1024);
}

// Output-tile scheme of the x and backward-y passes: 1 = double-buffered
// tiles with separate exchange slots, 0 = one tile whose columns are the
// exchange slots (less LDS, two barriers per output field).  Measured at 256^3
// (doubled 512^3): 0 for FP32 (two workgroups per CU in the backward y pass),
// 1 for FP64.
int fast_emit_dbl(int fast, int prec) {
  const char* e = std::getenv(fast == FAST_INV_Y ? "HP_EMIT_INVY" : "HP_EMIT_SAND");
  if (e) return std::atoi(e) == 1 ? 1 : 0;
  return prec == 0 ? 0 : 1;
}

int fast_lds_bytes(int fast, int L, int P, int K2, int prec, int dbl, int pad) {
  const int cs = prec == 0 ? 8 : 16;
  const int R0 = L >= 1024 ? 16 : 8;
  const int ppw = 64 / (L / R0);
  const int SL = slot_len(L);
  const int NX = pad ? L / 2 : L;  // stored rows of the x / backward-y output tiles
  switch (fast) {
    case FAST_R2C: return (L + ((P / 2 + ppw - 1) / ppw) * ppw * SL + K2 * (P + 1)) * cs;
    case FAST_FWD_Y: return (L + SL * (P + 1)) * cs;
    case FAST_SANDWICH:
      if (dbl) return (L + P * SL + 2 * NX * (P + 1)) * cs;
      return (L + SL * (P + 1)) * cs;
    case FAST_INV_Y:
      if (dbl) return (L + P * SL + 2 * NX * (P + 1)) * cs;
      return (L + slot_len(L, true) * (P + 1)) * cs;
    case FAST_C2R: return (L + 4 * ppw * SL) * cs;
    default: return 0;
  }
}

template <typename T, int L, int P, bool PAD>
static hipError_t launch_LP(const PassArgs& a0, int grid_y, hipStream_t s) {
  PassArgs a = a0;
  a.ngrp = grid_y;
  const int n0 = a.un[0], n1 = a.un[1];
  const int lds = a.lds_bytes;
  switch (a.fast) {
    case FAST_R2C: {
      dim3 grid(((n1 + P - 1) / P) * n0, grid_y);
      allow_lds<kf_r2c<T, L, P, PAD>>();
      hipLaunchKernelGGL((kf_r2c<T, L, P, PAD>), grid, dim3(R2CShape<L, P>::NT), lds, s, a);
    } break;
    case FAST_FWD_Y: {
      dim3 grid(((n0 + P - 1) / P) * a.kz_count, grid_y);
      allow_lds<kf_fwd_y<T, L, P, PAD>>();
      hipLaunchKernelGGL((kf_fwd_y<T, L, P, PAD>), grid, dim3(64 * (P / WF<L>::PPW)), lds, s, a);
    } break;
    case FAST_SANDWICH: {
      constexpr int NT = 64 * (P / WF<L>::PPW);
      const int ntiles = (a.gM[1] / P) * a.kz_count * grid_y;
      const bool adj = diff_is_adjoint(a.diff);
      const bool ext = a.diff == D_DIV || a.diff == D_NABLA || a.diff == D_ADJ_DIV ||
                       a.diff == D_ADJ_NABLA;
      auto go = [&](auto kern) {
        allow_lds<decltype(kern)::value>();
        const int nb = persistent_grid<decltype(kern)::value>(NT, lds, ntiles);
        hipLaunchKernelGGL(decltype(kern)::value, dim3(nb), dim3(NT), lds, s, a);
      };
#define HP_SW(ADJ, DBL, EXT) \
  go(std::integral_constant<decltype(&kf_sandwich<T, L, P, ADJ, DBL, PAD, EXT>), \
                            &kf_sandwich<T, L, P, ADJ, DBL, PAD, EXT>>{})
#define HP_SW2(DBL, EXT) \
  do {                   \
    if (adj) HP_SW(true, DBL, EXT); \
    else HP_SW(false, DBL, EXT);    \
  } while (0)
      if (a.emit_dbl) {  // double-buffered output tiles
        if (ext) HP_SW2(true, true);
        else HP_SW2(true, false);
      } else {
        if (ext) HP_SW2(false, true);
        else HP_SW2(false, false);
      }
#undef HP_SW2
#undef HP_SW
    } break;
    case FAST_INV_Y: {
      constexpr int NT = 64 * (P / WF<L>::PPW);
      dim3 grid(((a.kz_count + P - 1) / P) * n0, grid_y);
      if (a.P > 64) return hipErrorInvalidValue;
      if (a.emit_dbl) {  // double-buffered output tiles
        allow_lds<kf_inv_y<T, L, P, true, PAD>>();
        hipLaunchKernelGGL((kf_inv_y<T, L, P, true, PAD>), grid, dim3(NT), lds, s, a);
      } else {
        allow_lds<kf_inv_y<T, L, P, false, PAD>>();
        hipLaunchKernelGGL((kf_inv_y<T, L, P, false, PAD>), grid, dim3(NT), lds, s, a);
      }
    } break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int L, bool PAD>
static hipError_t launch_LPAD(const PassArgs& a, int grid_y, hipStream_t s) {
  if (a.fast == FAST_C2R) {
    const int n0 = a.un[0], n1 = a.un[1];
    const long long pairs = (long long)n0 * ((n1 + 1) / 2);
    const long long groups = (pairs + WF<L>::PPW - 1) / WF<L>::PPW;
    dim3 grid((unsigned)((groups + 3) / 4), grid_y);
    allow_lds<kf_c2r<T, L, PAD>>();
    hipLaunchKernelGGL((kf_c2r<T, L, PAD>), grid, dim3(kC2RThreads), a.lds_bytes, s, a);
    return hipGetLastError();
  }
  if (a.P == 8) return launch_LP<T, L, 8, PAD>(a, grid_y, s);
  if constexpr (sizeof(T) == 4 && L < 1024) {
    if (a.P == 16) return launch_LP<T, L, 16, PAD>(a, grid_y, s);
  }
  return hipErrorInvalidValue;
}

// a.pad: free-space (doubled, half of every pencil physical) or periodic
template <typename T, int L>
static hipError_t launch_L(const PassArgs& a, int grid_y, hipStream_t s) {
  if (a.pad) return launch_LPAD<T, L, true>(a, grid_y, s);
  return launch_LPAD<T, L, false>(a, grid_y, s);
}

template <typename T>
static hipError_t launch_T(const PassArgs& a, int grid_y, hipStream_t s) {
  switch (a.L) {
    case 64: return launch_L<T, 64>(a, grid_y, s);
    case 128: return launch_L<T, 128>(a, grid_y, s);
    case 256: return launch_L<T, 256>(a, grid_y, s);
    case 512: return launch_L<T, 512>(a, grid_y, s);
    case 1024: return launch_L<T, 1024>(a, grid_y, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fast(const PassArgs& a, int prec, int grid_y, hipStream_t s) {
  if (prec == 0) return launch_T<float>(a, grid_y, s);
  return launch_T<double>(a, grid_y, s);
}

}  // namespace hp
