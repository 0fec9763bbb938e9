// Wavefront-level FFT of length L = 64 .. 1024 (powers of two) and
// L = 48, 96, 192 (3 times a power of two) (gfx950).
//
// A pencil of length L is held by G = L / R0 lanes, R0 elements per lane:
// lane g holds x[g + G i], i < R0.  The first Stockham stage (radix R0: 8 or
// 16 for powers of two, 12 = 4 x 3 otherwise) works on those registers
// directly; the following radix-8 (and a final radix-2/4) stages (after
// radix 12: radix 4, then 2 or 4) exchange data through a wavefront-private
// LDS slot, so no workgroup barrier is needed inside the FFT.  After the last
// stage lane g holds X[g + G i] again.
#pragma once

#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "hp_device.hpp"
#include "hp_internal.hpp"

namespace hp {

template <int L>
struct WF {
  static constexpr int R0 = wf_r0(L);  // elements per lane
  static constexpr int G = L / R0;     // lanes per pencil
  static constexpr int PPW = 64 / G;   // pencils per wavefront
  static_assert(R0 > 0 && G * R0 == L && 64 % G == 0, "wavefront FFT length");
};

__device__ __forceinline__ void wave_sync() { __builtin_amdgcn_wave_barrier(); }

// LDS layouts of the FFT exchange.  Element m of a pencil sits at row
// m + (m >> S) K of its slot.  The first exchange (stage-0 write, stride R0
// across lanes; stage-1 read, stride L/8) uses S = 4, K = 1; the second
// (stage-1 write, runs of 8 at stride 64; stage-2 read) uses S = 5, K = 4
// (S = 4, K = 2 for L = 128).  In a model of the LDS as 32 banks served 16
// lanes at a time every access of both exchanges is conflict-free (the first
// exchange's is within 2x in a 64-bank model).
template <int S, int K>
struct Pad {
  static constexpr int S_ = S, K_ = K;
  __host__ __device__ static constexpr int row(int m) { return m + (m >> S) * K; }
};
using PadA = Pad<4, 1>;
template <int L>
using PadB = typename std::conditional<(L >= 256), Pad<5, 4>, Pad<4, 2>>::type;

__host__ __device__ constexpr int padrow(int m) { return PadA::row(m); }
// rows of one exchange slot (both layouts; SMALL: the first layout only)
__host__ __device__ constexpr int slot_len(int L, bool small = false) {
  const int a = PadA::row(L - 1) + 1;
  const int b = (L >= 256 ? Pad<5, 4>::row(L - 1) : Pad<4, 2>::row(L - 1)) + 1;
  return small || a > b ? a : b;
}

// Rows of the elements a + t S' (t = 0, 1, ...) in layout PD: one base row
// plus a constant step when S' is a multiple of 2^S, so every access of a
// pattern shares one address and differs by an immediate offset.
template <typename PD, int SP>
__device__ __forceinline__ int padrun(int a, int t) {
  if constexpr (SP % (1 << PD::S_) == 0) return PD::row(a) + t * PD::row(SP);
  else return PD::row(a + t * SP);
}

// One Stockham stage (radix R, NS = product of earlier radices) over the
// wavefront slot `buf`: reads in layout PR, writes (unless LAST) in layout PW.
// twS holds this stage's twiddles as twS[(t - 1) NS + k] = W_{NS R}^{t k}.
// TWPRE: the stage's twiddles are read with the exchange, ahead of the wave
// barrier, so their LDS latency overlaps it (read at the multiply, each pair
// of them costs a wait of its own); it holds NB (R - 1) more complex values in
// registers across the exchange.
template <typename T, int L, int R, int NS, bool LAST, bool INV, typename PR, typename PW,
          bool TWPRE = true>
__device__ __forceinline__ void wstage(C2<T> (&x)[WF<L>::R0], C2<T>* buf, int bs, int g,
                                       const C2<T>* twS) {
  constexpr int R0 = WF<L>::R0, G = WF<L>::G, NB = R0 / R;
  C2<T> w[NB * (R - 1)];
  if constexpr (TWPRE) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int k = (g + G * b) % NS;
#pragma unroll
      for (int t = 1; t < R; ++t) w[b * (R - 1) + t - 1] = twS[(t - 1) * NS + k];
    }
  }
  C2<T> v[R0];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = g + G * b;
#pragma unroll
    for (int t = 0; t < R; ++t) v[b * R + t] = buf[padrun<PR, L / R>(j, t) * bs];
  }
  wave_sync();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = g + G * b;
    const int k = j % NS;
#pragma unroll
    for (int t = 1; t < R; ++t) {
      C2<T> tw1 = TWPRE ? w[b * (R - 1) + t - 1] : twS[(t - 1) * NS + k];
      if (INV) tw1.im = -tw1.im;
      v[b * R + t] = cmul(v[b * R + t], tw1);
    }
    dftN<T, R, INV>(&v[b * R]);
    if constexpr (LAST) {
#pragma unroll
      for (int t = 0; t < R; ++t) x[b + t * NB] = v[b * R + t];
    } else {
      // element (j - k) R + k + t NS; (j - k) R is a multiple of NS R >= 64
      const int m0 = (j - k) * R;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        int row;
        // NS and 2^S are powers of two and m0 is a multiple of 2^S: for
        // NS >= 2^S the step is constant; for NS < 2^S, k < NS keeps
        // k + NS t within the same 2^S block as NS t
        if constexpr (NS % (1 << PW::S_) == 0) row = PW::row(m0 + k) + t * PW::row(NS);
        else if constexpr ((NS & (NS - 1)) != 0) row = PW::row(m0 + k + NS * t);  // NS = 12
        else row = PW::row(m0) + k + NS * t + ((NS * t) >> PW::S_) * PW::K_;
        buf[row * bs] = v[b * R + t];
      }
    }
  }
  if constexpr (!LAST) wave_sync();
}

// In-place FFT of the pencil held as x[i] = x[g + G i]; on return x[i] = X[g + G i].
// HALF: x[i] is zero for i >= R0 / 2 (zero-padded input).  tw is the
// per-stage twiddle table (stage 1 at 0, stage 2 at 7 R0).
template <typename T, int L, bool INV, bool HALF = false, bool SMALL = false, bool TWPRE = true>
__device__ __forceinline__ void wave_fft(C2<T> (&x)[WF<L>::R0], C2<T>* buf, int bs, int g,
                                         const C2<T>* tw) {
  // SMALL: both exchanges in the first layout (a shorter slot, 2x conflicts
  // on the stage-1 writes)
  using PB = typename std::conditional<SMALL, PadA, PadB<L>>::type;
  constexpr int R0 = WF<L>::R0, G = WF<L>::G;
  if constexpr (HALF) dftN_half<T, R0, INV>(x);
  else dftN<T, R0, INV>(x);
  wave_sync();
  if constexpr (R0 % 16 == 0 || 16 % R0 == 0) {
    // element g R0 + t, t < R0 in {8, 16}: never crosses a multiple of 16
    const int r0 = PadA::row(g * R0);
#pragma unroll
    for (int t = 0; t < R0; ++t) buf[(r0 + t) * bs] = x[t];
  } else {
#pragma unroll
    for (int t = 0; t < R0; ++t) buf[PadA::row(g * R0 + t) * bs] = x[t];
  }
  wave_sync();
  if constexpr (G <= 8 && R0 % G == 0) {
    // one more stage, of radix G (R0 = 8, G = 8; R0 = 12, G = 4)
    wstage<T, L, G, R0, true, INV, PadA, PadA, TWPRE>(x, buf, bs, g, tw);
  } else if constexpr (R0 % 3 == 0) {
    // R0 = 12: a radix-4 stage, then radix G / 4 (2 or 4)
    wstage<T, L, 4, R0, false, INV, PadA, PadA, TWPRE>(x, buf, bs, g, tw);
    wstage<T, L, G / 4, 4 * R0, true, INV, PadA, PadA, TWPRE>(x, buf, bs, g, tw + 3 * R0);
  } else {
    static_assert((R0 & (R0 - 1)) == 0, "three stages: power-of-two lengths only");
    wstage<T, L, 8, R0, false, INV, PadA, PB, TWPRE>(x, buf, bs, g, tw);
    wstage<T, L, G / 8, 8 * R0, true, INV, PB, PB, TWPRE>(x, buf, bs, g, tw + 7 * R0);
  }
}

// Logical block index with the blocks of one XCD contiguous: workgroups are
// dealt to the 8 XCDs in turn, so workgroup b runs on XCD b % 8; numbering
// them XCD by XCD puts blocks with neighbouring logical indices (which read
// the same Green's function rows) behind one L2.  A bijection on [0, nb).
__device__ __forceinline__ int xcd_block(int bid, int nb) {
  const int xcd = bid & 7, local = bid >> 3;
  const int per = nb >> 3, rem = nb & 7;
  return xcd * per + min(xcd, rem) + local;
}

// signed index m~ of m on an M-point grid, 0 at the Nyquist index
__device__ __forceinline__ int signed_index(int m, int M) {
  return (2 * m < M) ? m : ((2 * m == M) ? 0 : m - M);
}

// ---------------------------------------------------------- launch helpers
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

// Workgroups that fit on the device at once (persistent launches), or the
// tile count when HP_PERSIST=0.
template <auto K>
static int persistent_grid(int nt, int lds, int ntiles) {
  static int cached_lds = -1, per_cu = 1;  // one cache per kernel instantiation
  if (cached_lds != lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, K, nt, lds) != hipSuccess || n < 1) {
      (void)hipGetLastError();
      n = 1;
    }
    per_cu = n;
    cached_lds = lds;
  }
  static int cus[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    dev = 0;
  }
  if (!cus[dev]) {
    int c = 0;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1) {
      (void)hipGetLastError();
      c = 1;
    }
    cus[dev] = c;
  }
  const char* e = std::getenv("HP_PERSIST");
  if (e && std::atoi(e) == 0) return ntiles;
  const long long g = (long long)per_cu * cus[dev];
  return (int)std::max(1LL, std::min<long long>(g, ntiles));
}

}  // namespace hp
