// Register-resident DFTs of small 3/5-smooth lengths and the four-step
// decomposition used by the fused passes.
//
// A length M = A * B transform of one line is split over threads:
//   step 1: thread n2 (< B) holds x[B n1 + n2], n1 < A, and computes the
//           A-point DFT over n1 in registers, then multiplies by w_M^(n2 k1);
//   exchange through LDS (one write, one read per element);
//   step 2: thread k1 (< A) holds the B values of column k1 and computes the
//           B-point DFT, giving X[k1 + A k2] in register k2.
// Register DFTs of composite length are themselves four-step products of
// radix-3/5 butterflies with compile-time twiddles, so every index is a
// constant after unrolling.
#pragma once
#include "hom_internal.hpp"

namespace hom {
namespace rf {

// cos(2 pi p / q) and sin(2 pi p / q) at compile time (Taylor series after
// reduction to [-pi, pi]; |error| < 1e-16 for the small q used here).
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double reduce(int p, int q) {
  int r = p % q;
  if (r < 0) r += q;
  double x = 2.0 * kPi * (double)r / (double)q;
  if (x > kPi) x -= 2.0 * kPi;
  return x;
}
constexpr double ccos(int p, int q) {
  const double x = reduce(p, q);
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
constexpr double csin(int p, int q) {
  const double x = reduce(p, q);
  double term = x, sum = x;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}

template <typename R>
__device__ __forceinline__ Cx<R> mk(R a, R b) {
  Cx<R> c;
  c.x = a;
  c.y = b;
  return c;
}
template <typename R>
__device__ __forceinline__ Cx<R> add(Cx<R> a, Cx<R> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename R>
__device__ __forceinline__ Cx<R> sub(Cx<R> a, Cx<R> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename R>
__device__ __forceinline__ Cx<R> scl(Cx<R> a, R s) { return mk(a.x * s, a.y * s); }
template <typename R>
__device__ __forceinline__ Cx<R> mul(Cx<R> a, Cx<R> b) { return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
// multiply by exp(S 2 pi i p / q) with compile-time p, q
template <typename R, int S, int p, int q>
__device__ __forceinline__ Cx<R> rot(Cx<R> a) {
  if constexpr (p % q == 0) {
    return a;
  } else {
    constexpr double c = ccos(p, q), s = S * csin(p, q);
    return mk((R)(a.x * (R)c - a.y * (R)s), (R)(a.x * (R)s + a.y * (R)c));
  }
}

// ---- compile-time zero tracking.  ZC<R, true> is a value known to be zero
// when the kernel is compiled (an input of a pruned transform): operations on
// it fold away instead of adding or scaling zeros, which the compiler may not
// remove itself (x + 0 is not x for x = -0).
template <typename R, bool Z>
struct ZC {
  Cx<R> v;
};
template <typename R, bool A, bool B>
__device__ __forceinline__ ZC<R, A && B> zadd(ZC<R, A> a, ZC<R, B> b) {
  if constexpr (A && B) return {};
  else if constexpr (A) return {b.v};
  else if constexpr (B) return {a.v};
  else return {add(a.v, b.v)};
}
template <typename R, bool A, bool B>
__device__ __forceinline__ ZC<R, A && B> zsub(ZC<R, A> a, ZC<R, B> b) {
  if constexpr (A && B) return {};
  else if constexpr (A) return {mk(-b.v.x, -b.v.y)};
  else if constexpr (B) return {a.v};
  else return {sub(a.v, b.v)};
}
template <typename R>
__device__ __forceinline__ R fmx(R a, R b, R c) {
  if constexpr (sizeof(R) == 4) return __builtin_fmaf(a, b, c);
  else return __builtin_fma(a, b, c);
}
// acc + c t, as one fused multiply-add per component
template <typename R, bool A, bool B>
__device__ __forceinline__ ZC<R, A && B> zaxpy(ZC<R, A> acc, R c, ZC<R, B> t) {
  if constexpr (B) return {acc.v};
  else if constexpr (A) return {scl(t.v, c)};
  else return {mk(fmx(c, t.v.x, acc.v.x), fmx(c, t.v.y, acc.v.y))};
}
// acc + i c t, as one fused multiply-add per component
template <typename R, bool A, bool B>
__device__ __forceinline__ ZC<R, A && B> zaxpyi(ZC<R, A> acc, R c, ZC<R, B> t) {
  if constexpr (B) return {acc.v};
  else if constexpr (A) return {mk(-c * t.v.y, c * t.v.x)};
  else return {mk(fmx(-c, t.v.y, acc.v.x), fmx(c, t.v.x, acc.v.y))};
}
template <typename R, bool A>
__device__ __forceinline__ Cx<R> zval(ZC<R, A> a) {
  if constexpr (A) return mk((R)0, (R)0);
  else return a.v;
}

// ---- prime radices, in place, natural order; S = -1 forward, +1 inverse.
// Z: bit j set when input j is known to be zero.
template <typename R, int S, int Z = 0>
__device__ __forceinline__ void dft3(Cx<R>& a0, Cx<R>& a1, Cx<R>& a2) {
  const R s3 = (R)(S * 0.86602540378443864676);
  const ZC<R, (Z & 1) != 0> x0{a0};
  const ZC<R, (Z & 2) != 0> x1{a1};
  const ZC<R, (Z & 4) != 0> x2{a2};
  const auto t = zadd(x1, x2);
  const auto m = zaxpy(x0, (R)-0.5, t);
  const auto u = zsub(x1, x2);
  a0 = zval(zadd(x0, t));
  a1 = zval(zaxpyi(m, s3, u));    // m + i s3 (x1 - x2)
  a2 = zval(zaxpyi(m, -s3, u));
}

// The odd part i (s1 t3 + s2 t4) is formed as i s1 (t3 + (s2/s1) t4) and its
// scale folded into the final sums, so every multiplication is part of an FMA.
template <typename R, int S, int Z = 0>
__device__ __forceinline__ void dft5(Cx<R>& a0, Cx<R>& a1, Cx<R>& a2, Cx<R>& a3, Cx<R>& a4) {
  const R c1 = (R)0.30901699437494742410, c2 = (R)-0.80901699437494742410;
  const R s1 = (R)(S * 0.95105651629515357212), s2 = (R)(S * 0.58778525229247312917);
  const R r21 = (R)0.61803398874989484820, r12 = (R)1.61803398874989484820;   // s2 / s1, s1 / s2
  const ZC<R, (Z & 1) != 0> x0{a0};
  const ZC<R, (Z & 2) != 0> x1{a1};
  const ZC<R, (Z & 4) != 0> x2{a2};
  const ZC<R, (Z & 8) != 0> x3{a3};
  const ZC<R, (Z & 16) != 0> x4{a4};
  const auto t1 = zadd(x1, x4);
  const auto t2 = zadd(x2, x3);
  const auto t3 = zsub(x1, x4);
  const auto t4 = zsub(x2, x3);
  const auto b1 = zaxpy(zaxpy(x0, c1, t1), c2, t2);
  const auto b2 = zaxpy(zaxpy(x0, c2, t1), c1, t2);
  const auto u1 = zaxpy(t3, r21, t4);    // (s1 t3 + s2 t4) / s1
  const auto u2 = zaxpy(t3, -r12, t4);   // (s2 t3 - s1 t4) / s2
  a0 = zval(zadd(x0, zadd(t1, t2)));
  a1 = zval(zaxpyi(b1, s1, u1));
  a4 = zval(zaxpyi(b1, -s1, u1));
  a2 = zval(zaxpyi(b2, s2, u2));
  a3 = zval(zaxpyi(b2, -s2, u2));
}

// Dft<R, N, S>::run(v): in-place DFT of v[0..N-1]; run_z<Z>: the same with
// the inputs of mask Z known to be zero (their registers are not read).
template <typename R, int N, int S>
struct Dft;

template <typename R, int S>
struct Dft<R, 1, S> {
  template <int Z = 0>
  static __device__ __forceinline__ void run_z(Cx<R>* v) {
    if constexpr (Z & 1) v[0] = mk((R)0, (R)0);
  }
  static __device__ __forceinline__ void run(Cx<R>* v) { (void)v; }
};
template <typename R, int S>
struct Dft<R, 3, S> {
  template <int Z = 0>
  static __device__ __forceinline__ void run_z(Cx<R>* v) { dft3<R, S, Z>(v[0], v[1], v[2]); }
  static __device__ __forceinline__ void run(Cx<R>* v) { run_z<0>(v); }
};
template <typename R, int S>
struct Dft<R, 5, S> {
  template <int Z = 0>
  static __device__ __forceinline__ void run_z(Cx<R>* v) { dft5<R, S, Z>(v[0], v[1], v[2], v[3], v[4]); }
  static __device__ __forceinline__ void run(Cx<R>* v) { run_z<0>(v); }
};

// bits n1 < N1 of mask Z at positions N2 n1 + n2 (the inputs of one first-step DFT)
template <int Z, int N1, int N2, int n2>
constexpr int sub_mask() {
  int m = 0;
  for (int n1 = 0; n1 < N1; ++n1)
    if ((Z >> (N2 * n1 + n2)) & 1) m |= 1 << n1;
  return m;
}

// composite N = N1 * N2: n = N2 n1 + n2, k = k1 + N1 k2
template <typename R, int N1, int N2, int S>
struct DftComp {
  template <int n2, int k1>
  static __device__ __forceinline__ void twid(Cx<R>* a) {
    a[k1] = rot<R, S, n2 * k1, N1 * N2>(a[k1]);
    if constexpr (k1 + 1 < N1) twid<n2, k1 + 1>(a);
  }
  template <int n2, int Z>
  static __device__ __forceinline__ void step1(const Cx<R>* v, Cx<R>* t) {
    Cx<R> a[N1];
    constexpr int zm = sub_mask<Z, N1, N2, n2>();
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) a[n1] = ((zm >> n1) & 1) ? mk((R)0, (R)0) : v[N2 * n1 + n2];
    Dft<R, N1, S>::template run_z<zm>(a);
    twid<n2, 0>(a);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) t[n2 * N1 + k1] = a[k1];
    if constexpr (n2 + 1 < N2) step1<n2 + 1, Z>(v, t);
  }
  template <int Z = 0>
  static __device__ __forceinline__ void run_z(Cx<R>* v) {
    Cx<R> t[N1 * N2];
    step1<0, Z>(v, t);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      Cx<R> b[N2];
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) b[n2] = t[n2 * N1 + k1];
      Dft<R, N2, S>::run(b);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) v[k1 + N1 * k2] = b[k2];
    }
  }
  static __device__ __forceinline__ void run(Cx<R>* v) { run_z<0>(v); }
};

template <typename R, int S>
struct Dft<R, 9, S> : DftComp<R, 3, 3, S> {};
template <typename R, int S>
struct Dft<R, 15, S> : DftComp<R, 3, 5, S> {};
template <typename R, int S>
struct Dft<R, 25, S> : DftComp<R, 5, 5, S> {};
template <typename R, int S>
struct Dft<R, 27, S> : DftComp<R, 3, 9, S> {};

// Factorisation M = A * B used by the fused passes (A: registers in step 1).
template <int M>
struct Split;
template <>
struct Split<9> { static constexpr int A = 3, B = 3; };
template <>
struct Split<25> { static constexpr int A = 5, B = 5; };
template <>
struct Split<27> { static constexpr int A = 9, B = 3; };
template <>
struct Split<45> { static constexpr int A = 9, B = 5; };
template <>
struct Split<75> { static constexpr int A = 15, B = 5; };
template <>
struct Split<81> { static constexpr int A = 9, B = 9; };
template <>
struct Split<125> { static constexpr int A = 25, B = 5; };
template <>
struct Split<225> { static constexpr int A = 15, B = 15; };
template <>
struct Split<243> { static constexpr int A = 27, B = 9; };
template <>
struct Split<375> { static constexpr int A = 25, B = 15; };
template <>
struct Split<625> { static constexpr int A = 25, B = 25; };
template <>
struct Split<675> { static constexpr int A = 27, B = 25; };

}  // namespace rf
}  // namespace hom
