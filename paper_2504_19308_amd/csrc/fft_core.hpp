// Radix-2/4/8/16 DFT butterflies and Stockham stages for gfx950.
//
// Transforms are unnormalised: sign -1 is  X[k] = sum_j x[j] exp(-2 pi i jk/n)
// (the paper's sqrt(n) W), sign +1 the conjugate kernel; callers fold the 1/n
// of the inverse into their final store.
//
// A Stockham stage combines R already-transformed sub-sequences of length Ns
// into sequences of length Ns*R:  butterfly j reads x[j + r n/R], multiplies
// input r by exp(sign 2 pi i r (j mod Ns) / (Ns R)), takes a length-R DFT and
// writes output r to y[(j / Ns) Ns R + (j mod Ns) + r Ns].  Output comes out in
// natural order, so no bit reversal is needed.
#pragma once

#include <hip/hip_runtime.h>

namespace amm {

template <typename S> struct vec2;
template <> struct vec2<float> { using type = float2; };
template <> struct vec2<double> { using type = double2; };

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename V> __device__ __forceinline__ V cconj(V a) { return V{a.x, -a.y}; }
// multiply by sign*i :  (a + ib) * (s i) = -s b + i s a
template <int SIGN, typename V> __device__ __forceinline__ V mul_si(V a) {
  return SIGN < 0 ? V{a.y, -a.x} : V{-a.y, a.x};
}
template <typename V, typename S> __device__ __forceinline__ V cscale(V a, S s) {
  return V{a.x * s, a.y * s};
}

// exact constants of the 16th roots of unity
#define AMM_C8 0.92387953251128675613
#define AMM_S8 0.38268343236508977173
#define AMM_R2 0.70710678118654752440

template <int SIGN, typename V>
__device__ __forceinline__ void dft2(V& a, V& b) {
  V t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int SIGN, typename V>
__device__ __forceinline__ void dft4(V& x0, V& x1, V& x2, V& x3) {
  V t0 = cadd(x0, x2), t1 = csub(x0, x2);
  V t2 = cadd(x1, x3), t3 = mul_si<SIGN>(csub(x1, x3));
  x0 = cadd(t0, t2);
  x2 = csub(t0, t2);
  x1 = cadd(t1, t3);
  x3 = csub(t1, t3);
}

// w^m for w = exp(SIGN 2 pi i / 16), m in {0..15}, as compile-time algebra
template <int SIGN, int M, typename V>
__device__ __forceinline__ V rot16(V a) {
  using S = decltype(a.x);
  constexpr int m = M & 15;
  if constexpr (m == 0) return a;
  else if constexpr (m == 4) return mul_si<SIGN>(a);
  else if constexpr (m == 8) return V{-a.x, -a.y};
  else if constexpr (m == 12) return mul_si<-SIGN>(a);
  else {
    // cos and sin of 2 pi m / 16
    constexpr double c = (m == 1 || m == 15) ? AMM_C8 : (m == 2 || m == 14) ? AMM_R2
                       : (m == 3 || m == 13) ? AMM_S8 : (m == 5 || m == 11) ? -AMM_S8
                       : (m == 6 || m == 10) ? -AMM_R2 : -AMM_C8;   // 7, 9
    constexpr double s0 = (m == 1 || m == 7) ? AMM_S8 : (m == 2 || m == 6) ? AMM_R2
                        : (m == 3 || m == 5) ? AMM_C8 : (m == 9 || m == 15) ? -AMM_S8
                        : (m == 10 || m == 14) ? -AMM_R2 : -AMM_C8;  // 11, 13
    constexpr double s = SIGN < 0 ? -s0 : s0;
    return V{a.x * (S)c - a.y * (S)s, a.x * (S)s + a.y * (S)c};
  }
}

template <int SIGN, typename V>
__device__ __forceinline__ void dft8(V* x) {
  // even / odd split: E = DFT4(x0,x2,x4,x6), O = DFT4(x1,x3,x5,x7)
  dft4<SIGN>(x[0], x[2], x[4], x[6]);
  dft4<SIGN>(x[1], x[3], x[5], x[7]);
  V o1 = rot16<SIGN, 2>(x[3]);
  V o2 = rot16<SIGN, 4>(x[5]);
  V o3 = rot16<SIGN, 6>(x[7]);
  V e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
  x[0] = cadd(e0, x[1]); x[4] = csub(e0, x[1]);
  x[1] = cadd(e1, o1);   x[5] = csub(e1, o1);
  x[2] = cadd(e2, o2);   x[6] = csub(e2, o2);
  x[3] = cadd(e3, o3);   x[7] = csub(e3, o3);
}

template <int SIGN, typename V>
__device__ __forceinline__ void dft16(V* x) {
  // index j = 4 j1 + j2, frequency k = k1 + 4 k2
  dft4<SIGN>(x[0], x[4], x[8], x[12]);
  dft4<SIGN>(x[1], x[5], x[9], x[13]);
  dft4<SIGN>(x[2], x[6], x[10], x[14]);
  dft4<SIGN>(x[3], x[7], x[11], x[15]);
  // after this x[4 k1 + j2] holds the j2-th sub-DFT at k1; twiddle w16^(j2 k1)
  x[5] = rot16<SIGN, 1>(x[5]);
  x[6] = rot16<SIGN, 2>(x[6]);
  x[7] = rot16<SIGN, 3>(x[7]);
  x[9] = rot16<SIGN, 2>(x[9]);
  x[10] = rot16<SIGN, 4>(x[10]);
  x[11] = rot16<SIGN, 6>(x[11]);
  x[13] = rot16<SIGN, 3>(x[13]);
  x[14] = rot16<SIGN, 6>(x[14]);
  x[15] = rot16<SIGN, 9>(x[15]);
  dft4<SIGN>(x[0], x[1], x[2], x[3]);
  dft4<SIGN>(x[4], x[5], x[6], x[7]);
  dft4<SIGN>(x[8], x[9], x[10], x[11]);
  dft4<SIGN>(x[12], x[13], x[14], x[15]);
  // now x[4 k1 + k2] = X[k1 + 4 k2]: transpose the 4x4 index
  V t;
  t = x[1]; x[1] = x[4]; x[4] = t;
  t = x[2]; x[2] = x[8]; x[8] = t;
  t = x[3]; x[3] = x[12]; x[12] = t;
  t = x[6]; x[6] = x[9]; x[9] = t;
  t = x[7]; x[7] = x[13]; x[13] = t;
  t = x[11]; x[11] = x[14]; x[14] = t;
}

template <int R, int SIGN, typename V>
__device__ __forceinline__ void dftR(V* x) {
  if constexpr (R == 2) dft2<SIGN>(x[0], x[1]);
  else if constexpr (R == 4) dft4<SIGN>(x[0], x[1], x[2], x[3]);
  else if constexpr (R == 8) dft8<SIGN>(x);
  else if constexpr (R == 16) dft16<SIGN>(x);
}

// Radix of stage `st` for n = 2^LOG2N: radix-16 stages first, remainder last.
__host__ __device__ constexpr int stage_count(int log2n) { return (log2n + 3) / 4; }
__host__ __device__ constexpr int stage_log2r(int log2n, int st) {
  return (st < log2n / 4) ? 4 : (log2n % 4);
}

}  // namespace amm
