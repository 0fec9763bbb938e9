// Single-launch 2D periodic solve (Section 2.2: transform, divide by the
// eigenvalue sum of Table 1, transform back; Section 2.3.3: spectral GRAD,
// CURL of a scalar and NABLA) for grids whose half spectrum fits one
// workgroup's LDS.
//
// One workgroup runs the whole solve, so small problems pay one launch
// instead of three:
//   1. rows: the real transform along y (contiguous), two rows x, x + 1 as one
//      complex wavefront FFT, untangled into spec_c[ky][x], ky <= L1 / 2;
//   2. per output field: along x, per ky pencil, the forward FFT of the
//      component it derives from, the multiplier norm / (lam_x + lam_y) (0 for
//      the zero mode), the field's spectral factor (1, i k or -|k|^2) and the
//      backward FFT, into a spectral output buffer (in place for plain psi,
//      where every output is its own component);
//   3. per output field: the inverse real transform along y, two rows per
//      complex FFT (real part row x, imaginary part row x + 1), to global.
// Workgroup barriers separate the steps; inside a step every pencil is private
// to the lanes of one wavefront (hp_wavefft.hpp).
#include <algorithm>

#include "hp_device.hpp"
#include "hp_internal.hpp"
#include "hp_wavefft.hpp"

namespace hp {

namespace {

constexpr int kSmallWaves = 8, kSmallThreads = 64 * kSmallWaves;

// LDS layout (complex T): twiddles of L0 and L1, the exchange slots of every
// wavefront (PPW pencils of the FFT length in use), then the spectral buffers
// [L1 / 2 + 1][L0 + 1].
template <int L0, int L1>
struct SmallShape {
  static constexpr int K = L1 / 2 + 1;
  static constexpr int SR = L0 + 1;  // row stride: consecutive ky rows start on different banks
  static constexpr int W0 = WF<L0>::PPW * slot_len(L0), W1 = WF<L1>::PPW * slot_len(L1);
  static constexpr int WSLOT = W0 > W1 ? W0 : W1;  // per wavefront
  static constexpr int HEAD = L0 + L1 + kSmallWaves * WSLOT;
  static constexpr int BUF = K * SR;
};

template <typename T, int L0, int L1>
__global__ void __launch_bounds__(kSmallThreads) kf_small2d(const PassArgs a) {
  using S = SmallShape<L0, L1>;
  constexpr int K = S::K, SR = S::SR;
  extern __shared__ __align__(16) unsigned char smem[];
  C2<T>* tw0 = (C2<T>*)smem;
  C2<T>* tw1 = tw0 + L0;
  C2<T>* exch = tw1 + L1;
  C2<T>* spec = exch + kSmallWaves * S::WSLOT;
  for (int m = threadIdx.x; m < L0; m += kSmallThreads) tw0[m] = ((const C2<T>*)a.tw)[m];
  for (int m = threadIdx.x; m < L1; m += kSmallThreads) tw1[m] = ((const C2<T>*)a.qtw)[m];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int nin = a.n_in, nfo = a.n_out;
  const int diff = a.diff;
  const bool inplace = diff == D_NONE;
  C2<T>* obuf = spec + nin * S::BUF;
  __syncthreads();

  // 1. R2C along y of every input component: rows x, x + 1 of component c as
  // one complex FFT; X_a[k] = (Z[k] + conj Z[-k]) / 2, X_b[k] = (Z[k] - conj Z[-k]) / 2i
  {
    constexpr int R0 = WF<L1>::R0, G = WF<L1>::G, PPW = WF<L1>::PPW;
    const int q = lane / G, g = lane % G;
    C2<T>* buf = exch + wave * S::WSLOT + q * slot_len(L1);
    const int npair = nin * (L0 / 2);  // a multiple of PPW: every lane of a wave has work
    for (int j0 = wave * PPW; j0 < npair; j0 += kSmallWaves * PPW) {
      const int j = j0 + q;
      const int c = j / (L0 / 2), x = 2 * (j % (L0 / 2));
      const T* ra = (const T*)a.in[c] + (long long)x * L1;
      const T* rb = ra + L1;
      C2<T> v[R0];
#pragma unroll
      for (int i = 0; i < R0; ++i) v[i] = {ra[g + G * i], rb[g + G * i]};
      wave_fft<T, L1, false>(v, buf, 1, g, tw1);
      wave_sync();
#pragma unroll
      for (int i = 0; i < R0; ++i) buf[padrow(g + G * i)] = v[i];
      wave_sync();
      C2<T>* sc = spec + c * S::BUF;
#pragma unroll
      for (int i = 0; i <= R0 / 2; ++i) {
        const int k = g + G * i;
        if (k > L1 / 2) break;
        const C2<T> zk = buf[padrow(k)];
        const C2<T> zc = cconj(buf[padrow((L1 - k) & (L1 - 1))]);
        const C2<T> s = cadd(zk, zc), d = csub(zk, zc);
        sc[k * SR + x] = {s.re * (T)0.5, s.im * (T)0.5};
        sc[k * SR + x + 1] = {d.im * (T)0.5, -d.re * (T)0.5};
      }
      wave_sync();
    }
  }
  __syncthreads();

  for (int f = 0; f < nfo; ++f) {
    C2<T>* ob = inplace ? spec + f * S::BUF : obuf;
    // 2. along x, one pencil per ky (pencils past the last one recompute the
    // last and store nothing, so every lane of a wave runs the same code)
    {
      constexpr int R0 = WF<L0>::R0, G = WF<L0>::G, PPW = WF<L0>::PPW;
      const int q = lane / G, g = lane % G;
      C2<T>* buf = exch + wave * S::WSLOT + q * slot_len(L0);
      for (int p0 = wave * PPW; p0 < K; p0 += kSmallWaves * PPW) {
        const int ky = p0 + q;
        const int kyc = ky < K ? ky : K - 1;
        const double lam_y = a.lam[1][kyc];
        // wavenumber tables are bound only with derivative outputs
        const T kyv = f < nin ? (T)0 : ((const T*)a.kvec[1])[kyc];
        // psi-hat of component c on this pencil: forward FFT, then the multiplier
        auto psi_hat = [&](C2<T> (&w)[R0], int c) {
          const C2<T>* sc = spec + c * S::BUF + kyc * SR;
#pragma unroll
          for (int i = 0; i < R0; ++i) w[i] = sc[g + G * i];
          wave_fft<T, L0, false>(w, buf, 1, g, tw0);
#pragma unroll
          for (int i = 0; i < R0; ++i) {
            const double lam = a.lam[0][g + G * i] + lam_y;
            w[i] = cscale(w[i], lam == 0.0 ? (T)0 : (T)(a.norm / lam));
          }
        };
        C2<T> u[R0];
        if (f < nin) {
          psi_hat(u, f);  // psi_f
        } else {
          const int d = f - nin;
          if (diff == D_NABLA) {
            // -(k_x^2 + k_y^2) psi_d
            psi_hat(u, d);
#pragma unroll
            for (int i = 0; i < R0; ++i) {
              const T kxv = ((const T*)a.kvec[0])[g + G * i];
              u[i] = cscale(u[i], -(kxv * kxv) - kyv * kyv);
            }
          } else {
            // GRAD: i k_d psi; 2D CURL of a scalar: (i k_y psi, -i k_x psi)
            psi_hat(u, 0);
#pragma unroll
            for (int i = 0; i < R0; ++i) {
              const T kxv = ((const T*)a.kvec[0])[g + G * i];
              const T kk = diff == D_GRAD ? (d == 0 ? kxv : kyv) : (d == 0 ? kyv : -kxv);
              u[i] = cscale(cmuli(u[i]), kk);
            }
          }
        }
        wave_sync();
        wave_fft<T, L0, true>(u, buf, 1, g, tw0);
        if (ky < K) {
#pragma unroll
          for (int i = 0; i < R0; ++i) ob[ky * SR + g + G * i] = u[i];
        }
        wave_sync();
      }
    }
    __syncthreads();
    // 3. C2R along y, rows x, x + 1 as Z = X_a + i X_b (Hermitian extension
    // above L1 / 2; the k = 0 and L1 / 2 bins of a real row are real)
    {
      constexpr int R0 = WF<L1>::R0, G = WF<L1>::G, PPW = WF<L1>::PPW;
      const int q = lane / G, g = lane % G;
      C2<T>* buf = exch + wave * S::WSLOT + q * slot_len(L1);
      T* out = (T*)a.out[f];
      for (int j0 = wave * PPW; j0 < L0 / 2; j0 += kSmallWaves * PPW) {
        const int x = 2 * (j0 + q);
        C2<T> v[R0];
#pragma unroll
        for (int i = 0; i < R0; ++i) {
          const int k = g + G * i;
          const int kk = k <= L1 / 2 ? k : L1 - k;
          C2<T> xa = ob[kk * SR + x], xb = ob[kk * SR + x + 1];
          if (kk == 0 || kk == L1 / 2) xa.im = xb.im = (T)0;
          if (k > L1 / 2) { xa = cconj(xa); xb = cconj(xb); }
          v[i] = cadd(xa, cmuli(xb));
        }
        wave_fft<T, L1, true>(v, buf, 1, g, tw1);
#pragma unroll
        for (int i = 0; i < R0; ++i) {
          out[(long long)x * L1 + g + G * i] = v[i].re;
          out[(long long)(x + 1) * L1 + g + G * i] = v[i].im;
        }
        wave_sync();
      }
    }
    __syncthreads();  // the next field rewrites the output buffer
  }
}

template <typename T, int L0, int L1>
hipError_t small2d_go(const PassArgs& a, hipStream_t s) {
  allow_lds<kf_small2d<T, L0, L1>>();
  hipLaunchKernelGGL((kf_small2d<T, L0, L1>), dim3(1), dim3(kSmallThreads), a.lds_bytes, s, a);
  return hipGetLastError();
}

template <int L0, int L1>
int small2d_bytes(int prec, int nbuf) {
  using S = SmallShape<L0, L1>;
  return (S::HEAD + nbuf * S::BUF) * (prec == 0 ? 8 : 16);
}

}  // namespace

// LDS bytes of the single-launch solve with nbuf spectral buffers, or -1
// where the pair of lengths has no kernel instance.
int small2d_lds_bytes(int L0, int L1, int prec, int nbuf) {
#define HP_SMALL_CASE(A, B) \
  if (L0 == A && L1 == B) return small2d_bytes<A, B>(prec, nbuf);
  HP_SMALL_CASE(64, 64) HP_SMALL_CASE(64, 128) HP_SMALL_CASE(128, 64)
  if (prec == 0) { HP_SMALL_CASE(128, 128) HP_SMALL_CASE(64, 256) HP_SMALL_CASE(256, 64) }
#undef HP_SMALL_CASE
  return -1;
}

hipError_t launch_small2d(const PassArgs& a, int prec, hipStream_t s) {
  const int L0 = a.gM[0], L1 = a.gM[1];
#define HP_SMALL_CASE(A, B)                                                                 \
  if (L0 == A && L1 == B)                                                                   \
    return prec == 0 ? small2d_go<float, A, B>(a, s) : small2d_go<double, A, B>(a, s);
  HP_SMALL_CASE(64, 64) HP_SMALL_CASE(64, 128) HP_SMALL_CASE(128, 64)
#undef HP_SMALL_CASE
  if (prec == 0) {
    if (L0 == 128 && L1 == 128) return small2d_go<float, 128, 128>(a, s);
    if (L0 == 64 && L1 == 256) return small2d_go<float, 64, 256>(a, s);
    if (L0 == 256 && L1 == 64) return small2d_go<float, 256, 64>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace hp
