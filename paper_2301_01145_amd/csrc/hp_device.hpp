// Device-side complex arithmetic and small DFT kernels shared by the passes.
#pragma once

#include <hip/hip_runtime.h>

namespace hp {

template <typename T>
struct C2 {
  T re, im;
};

template <typename T>
__device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ C2<T> cscale(C2<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T>
__device__ __forceinline__ C2<T> cconj(C2<T> a) { return {a.re, -a.im}; }
// i * a
template <typename T>
__device__ __forceinline__ C2<T> cmuli(C2<T> a) { return {-a.im, a.re}; }
// Multiply by the rotation -i (forward transform) or +i (backward).
template <typename T, bool INV>
__device__ __forceinline__ C2<T> rot(C2<T> a) {
  return INV ? C2<T>{-a.im, a.re} : C2<T>{a.im, -a.re};
}

// Streaming (nontemporal) global stores: data written once per pass and not
// read again before it is evicted, so it is kept from displacing cache lines.
template <typename T>
__device__ __forceinline__ void st_stream(C2<T>* p, const C2<T>& v) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 w;
  w.x = v.re;
  w.y = v.im;
  __builtin_nontemporal_store(w, (v2*)p);
}
template <typename T>
__device__ __forceinline__ void st_stream(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}
// Streaming (nontemporal) global loads: data read once per pass.
template <typename T>
__device__ __forceinline__ C2<T> ld_stream(const C2<T>* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 w = __builtin_nontemporal_load((const v2*)p);
  return {w.x, w.y};
}
template <typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  return __builtin_nontemporal_load(p);
}

// ---------------------------------------------------------------- radix DFTs
template <typename T, bool INV>
__device__ __forceinline__ void dft2(C2<T>* v) {
  C2<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(C2<T>& x0, C2<T>& x1, C2<T>& x2, C2<T>& x3) {
  C2<T> s0 = cadd(x0, x2), s1 = csub(x0, x2), s2 = cadd(x1, x3), s3 = rot<T, INV>(csub(x1, x3));
  x0 = cadd(s0, s2);
  x2 = csub(s0, s2);
  x1 = cadd(s1, s3);
  x3 = csub(s1, s3);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4v(C2<T>* v) {
  C2<T> a = v[0], b = v[1], c = v[2], d = v[3];
  dft4<T, INV>(a, b, c, d);
  v[0] = a; v[1] = b; v[2] = c; v[3] = d;
}

// HALF: v[4..7] are known to be zero (zero-padded input), the first
// butterfly layer reduces to copies.
template <typename T, bool INV, bool HALF = false>
__device__ __forceinline__ void dft8(C2<T>* v) {
  const T r = (T)0.70710678118654752440084436210485;
  C2<T> a0, a1, a2, a3, b0, b1, b2, b3;
  if constexpr (HALF) {
    a0 = b0 = v[0]; a1 = b1 = v[1]; a2 = b2 = v[2]; a3 = b3 = v[3];
  } else {
    a0 = cadd(v[0], v[4]); a1 = cadd(v[1], v[5]); a2 = cadd(v[2], v[6]); a3 = cadd(v[3], v[7]);
    b0 = csub(v[0], v[4]); b1 = csub(v[1], v[5]); b2 = csub(v[2], v[6]); b3 = csub(v[3], v[7]);
  }
  // b_t *= W8^t (forward W8 = (1 - i)/sqrt2, backward its conjugate)
  if (INV) {
    b1 = {(b1.re - b1.im) * r, (b1.re + b1.im) * r};
    b3 = {(-b3.re - b3.im) * r, (b3.re - b3.im) * r};
  } else {
    b1 = {(b1.re + b1.im) * r, (b1.im - b1.re) * r};
    b3 = {(b3.im - b3.re) * r, (-b3.re - b3.im) * r};
  }
  b2 = rot<T, INV>(b2);
  dft4<T, INV>(a0, a1, a2, a3);
  dft4<T, INV>(b0, b1, b2, b3);
  v[0] = a0; v[2] = a1; v[4] = a2; v[6] = a3;
  v[1] = b0; v[3] = b1; v[5] = b2; v[7] = b3;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft3(C2<T>* v) {
  const T h = (T)0.86602540378443864676372317075294;  // sqrt(3)/2
  C2<T> A = cadd(v[1], v[2]), B = rot<T, INV>(csub(v[1], v[2]));
  C2<T> t = csub(v[0], cscale(A, (T)0.5));
  v[0] = cadd(v[0], A);
  v[1] = cadd(t, cscale(B, h));
  v[2] = csub(t, cscale(B, h));
}

template <typename T, bool INV>
__device__ __forceinline__ void dft5(C2<T>* v) {
  const T c1 = (T)0.30901699437494742410229341718282;   // cos(2 pi / 5)
  const T c2 = (T)-0.80901699437494742410229341718282;  // cos(4 pi / 5)
  const T s1 = (T)0.95105651629515357211643933337938;   // sin(2 pi / 5)
  const T s2 = (T)0.58778525229247312916870595463907;   // sin(4 pi / 5)
  C2<T> A1 = cadd(v[1], v[4]), B1 = csub(v[1], v[4]);
  C2<T> A2 = cadd(v[2], v[3]), B2 = csub(v[2], v[3]);
  C2<T> x0 = v[0];
  C2<T> t1 = cadd(x0, cadd(cscale(A1, c1), cscale(A2, c2)));
  C2<T> t2 = cadd(x0, cadd(cscale(A1, c2), cscale(A2, c1)));
  C2<T> u1 = rot<T, INV>(cadd(cscale(B1, s1), cscale(B2, s2)));
  C2<T> u2 = rot<T, INV>(csub(cscale(B1, s2), cscale(B2, s1)));
  v[0] = cadd(x0, cadd(A1, A2));
  v[1] = cadd(t1, u1);
  v[4] = csub(t1, u1);
  v[2] = cadd(t2, u2);
  v[3] = csub(t2, u2);
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dftR(C2<T>* v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 3) dft3<T, INV>(v);
  else if constexpr (R == 4) dft4v<T, INV>(v);
  else if constexpr (R == 5) dft5<T, INV>(v);
  else dft8<T, INV>(v);
}

// 16-point DFT as 4 x 4 with W16 twiddles between the two radix-4 layers.
// HALF: v[8..15] are known to be zero.
template <typename T, bool INV, bool HALF = false>
__device__ __forceinline__ void dft16(C2<T>* v) {
  // columns: a_n1[n2] = v[n1 + 4 n2]; DFT4 over n2 for each n1
  C2<T> a[4][4];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    C2<T> x0 = v[n1], x1 = v[n1 + 4];
    if constexpr (HALF) {
      const C2<T> r1 = rot<T, INV>(x1);
      a[n1][0] = cadd(x0, x1); a[n1][1] = cadd(x0, r1);
      a[n1][2] = csub(x0, x1); a[n1][3] = csub(x0, r1);
    } else {
      C2<T> x2 = v[n1 + 8], x3 = v[n1 + 12];
      dft4<T, INV>(x0, x1, x2, x3);
      a[n1][0] = x0; a[n1][1] = x1; a[n1][2] = x2; a[n1][3] = x3;
    }
  }
  // twiddle W16^(n1 k2)
  const T c1 = (T)0.92387953251128675612818318939679;  // cos(pi/8)
  const T s1 = (T)0.38268343236508977172845998403040;  // sin(pi/8)
  const T r2 = (T)0.70710678118654752440084436210485;
  const T cs[4][2] = {{(T)1, (T)0}, {c1, s1}, {r2, r2}, {s1, c1}};  // cos, sin of pi m / 8
#pragma unroll
  for (int n1 = 1; n1 < 4; ++n1) {
#pragma unroll
    for (int k2 = 1; k2 < 4; ++k2) {
      const int m = n1 * k2;  // 1..9
      // exp(-+ i pi m / 8)
      T c, sn;
      if (m <= 3) { c = cs[m][0]; sn = cs[m][1]; }
      else if (m == 4) { c = (T)0; sn = (T)1; }
      else if (m <= 7) { c = -cs[8 - m][0]; sn = cs[8 - m][1]; }
      else if (m == 8) { c = (T)-1; sn = (T)0; }
      else { c = -cs[m - 8][0]; sn = -cs[m - 8][1]; }
      C2<T> w = {c, INV ? sn : -sn};
      a[n1][k2] = cmul(a[n1][k2], w);
    }
  }
  // DFT4 over n1 for each k2: output index k2 + 4 k1
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    C2<T> x0 = a[0][k2], x1 = a[1][k2], x2 = a[2][k2], x3 = a[3][k2];
    dft4<T, INV>(x0, x1, x2, x3);
    v[k2] = x0; v[k2 + 4] = x1; v[k2 + 8] = x2; v[k2 + 12] = x3;
  }
}

// cos(pi m / 12) for any integer m, from the exact first-quadrant values
// (m = 0..6: 1, cos 15, cos 30, cos 45, 1/2, cos 75 degrees, 0).
__host__ __device__ constexpr double cospi12(int m) {
  m %= 24;
  if (m < 0) m += 24;
  const int r = m <= 6 ? m : (m <= 12 ? 12 - m : (m <= 18 ? m - 12 : 24 - m));
  const double c = r == 0 ? 1.0
                 : r == 1 ? 0.96592582628906828674974319972890
                 : r == 2 ? 0.86602540378443864676372317075294
                 : r == 3 ? 0.70710678118654752440084436210485
                 : r == 4 ? 0.5
                 : r == 5 ? 0.25881904510252076234889883762405
                          : 0.0;
  return (m > 6 && m < 18) ? -c : c;
}

// N = N1 N2 point DFT (N divides 24) by one Cooley-Tukey split: with
// x[N2 n1 + n2], N1-point DFTs over n1 for every n2, the twiddles
// W_N^(n2 k1), then N2-point DFTs over n2, giving X[k1 + N1 k2].
template <typename T, int N1, int N2, bool INV>
__device__ __forceinline__ void dft_split(C2<T>* v) {
  constexpr int N = N1 * N2;
  static_assert(24 % N == 0, "split DFT for lengths dividing 24");
  C2<T> a[N2][N1];
#pragma unroll
  for (int n2 = 0; n2 < N2; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) a[n2][n1] = v[N2 * n1 + n2];
    dftR<T, N1, INV>(a[n2]);
  }
#pragma unroll
  for (int n2 = 1; n2 < N2; ++n2) {
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) {
      const int m = (n2 * k1 * (24 / N)) % 24;  // W_N^(n2 k1) = exp(-+ i pi m / 12)
      const T c = (T)cospi12(m), sn = (T)cospi12(m - 6);
      a[n2][k1] = cmul(a[n2][k1], C2<T>{c, INV ? sn : -sn});
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) {
    C2<T> b[N2];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) b[n2] = a[n2][k1];
    dftR<T, N2, INV>(b);
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) v[k1 + N1 * k2] = b[k2];
  }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dftN(C2<T>* v) {
  if constexpr (R == 16) dft16<T, INV>(v);
  else if constexpr (R == 24) dft_split<T, 8, 3, INV>(v);
  else if constexpr (R == 12) dft_split<T, 4, 3, INV>(v);
  else dftR<T, R, INV>(v);
}

// First-stage DFT of a zero-padded pencil: the upper half of v is zero.
template <typename T, int R, bool INV>
__device__ __forceinline__ void dftN_half(C2<T>* v) {
  static_assert(R == 8 || R == 16, "half-input DFT for radix 8 and 16");
  if constexpr (R == 16) dft16<T, INV, true>(v);
  else dft8<T, INV, true>(v);
}

}  // namespace hp
