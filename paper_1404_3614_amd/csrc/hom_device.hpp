// Device helpers shared by the pipeline kernels: complex arithmetic, index
// maps between Z_N and the doubled grid, fixed-order reductions, the basis
// T(k) of the projected spaces and the symmetric coefficient product.
#pragma once
#include "hom_internal.hpp"

namespace hom {

// ------------------------------------------------------------------ complex
template <typename R>
__device__ __forceinline__ Cx<R> cx(R a, R b) {
  Cx<R> c;
  c.x = a;
  c.y = b;
  return c;
}
template <typename R>
__device__ __forceinline__ Cx<R> operator+(Cx<R> a, Cx<R> b) { return cx(a.x + b.x, a.y + b.y); }
template <typename R>
__device__ __forceinline__ Cx<R> operator-(Cx<R> a, Cx<R> b) { return cx(a.x - b.x, a.y - b.y); }
template <typename R>
__device__ __forceinline__ Cx<R> operator*(Cx<R> a, R s) { return cx(a.x * s, a.y * s); }
template <typename R>
__device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
  return cx(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// i * s * a
template <typename R>
__device__ __forceinline__ Cx<R> imul(Cx<R> a, R s) { return cx(-a.y * s, a.x * s); }

// ------------------------------------------------------------------ indices
// FFT-order index <-> signed frequency for an odd length n.
__device__ __forceinline__ int fr(int i, int n) { return i <= (n - 1) / 2 ? i : i - n; }
__device__ __forceinline__ int ixn(int k, int n) { return k >= 0 ? k : k + n; }
// Position on the length-M axis of frequency index i of a length-N axis (zero padding).
__device__ __forceinline__ int padpos(int i, int N, int M) { return i <= (N - 1) / 2 ? i : i + (M - N); }
// Index on the length-N axis kept by truncation of position j of a length-M axis, or -1.
__device__ __forceinline__ int truncidx(int j, int N, int M) {
  const int h = (N - 1) / 2;
  if (j <= h) return j;
  if (j >= M - h) return j - (M - N);
  return -1;
}

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum_arr(const double* __restrict__ p, int n) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int i = lane; i < n; i += 64) s += p[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  return __shfl(s, 0, 64);
}

// wave_sum_arr over L rows of n values each (row w at p + w * stride), the
// result of row w in s[w] on every lane.  Each lane's loads of one trip (four
// per row) are all issued before the first add, so a short row costs one
// memory round trip instead of one per element; the additions keep
// wave_sum_arr's order, so the sums are the same to the bit.
template <int L>
__device__ __forceinline__ void wave_sum_rows(const double* __restrict__ p, size_t stride, int n, double (&s)[L]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int w = 0; w < L; ++w) s[w] = 0.0;
  for (int base = 0; base < n; base += 256) {
    double v[L][4];
#pragma unroll
    for (int w = 0; w < L; ++w)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = base + lane + 64 * j;
        v[w][j] = i < n ? p[w * stride + i] : 0.0;
      }
#pragma unroll
    for (int w = 0; w < L; ++w)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (base + lane + 64 * j < n) s[w] += v[w][j];
  }
#pragma unroll
  for (int w = 0; w < L; ++w) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s[w] += __shfl_down(s[w], off, 64);
    s[w] = __shfl(s[w], 0, 64);
  }
}

// Sum over the block in a fixed order; every thread must call it.
__device__ __forceinline__ double block_sum(double v, double* sred) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sred[w] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < kBlock / 64; ++i) r += sred[i];
  __syncthreads();
  return r;
}

// ------------------------------------------------------------------ basis T(k)
// Orthonormal basis of the range of G^E(k) (primal, one column xi/|xi|) or of
// G^J(k) (dual: d = 2 the rotated normal, d = 3 two tangents), Def. projection.
__device__ __forceinline__ void basis(const Geo& g, int k0, int k1, int k2, double T[3][2]) {
  // loops unrolled and axes selected, so every private array has constant indices
  double n[3] = {0.0, 0.0, 0.0};
  double n2 = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c >= g.d) continue;
    const int a = g.phys_axis[c];
    const int ka = a == 0 ? k0 : (a == 1 ? k1 : k2);
    const double iy = a == 0 ? g.iY[0] : (a == 1 ? g.iY[1] : g.iY[2]);
    n[c] = ka * iy;
    n2 += n[c] * n[c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) T[c][0] = T[c][1] = 0.0;
  if (n2 == 0.0) return;
  const double inv = 1.0 / sqrt(n2);
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if (c < g.d) n[c] *= inv;
  if (!g.dual) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (c < g.d) T[c][0] = n[c];
  } else if (g.d == 2) {
    T[0][0] = -n[1];
    T[1][0] = n[0];
  } else {
    int a = 0;
    double na = n[0];
    if (fabs(n[1]) < fabs(na)) {
      a = 1;
      na = n[1];
    }
    if (fabs(n[2]) < fabs(na)) {
      a = 2;
      na = n[2];
    }
    double t1[3] = {-na * n[0], -na * n[1], -na * n[2]};
    if (a == 0)
      t1[0] += 1.0;
    else if (a == 1)
      t1[1] += 1.0;
    else
      t1[2] += 1.0;
    const double in1 = 1.0 / sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
    t1[0] *= in1;
    t1[1] *= in1;
    t1[2] *= in1;
    const double t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T[c][0] = t1[c];
      T[c][1] = t2[c];
    }
  }
}

// Symmetric coefficient times vector: w = A u, A given by nc components.
template <typename R>
__device__ __forceinline__ void coef_mul(int d, int nc, const R* a, const R* u, R* w) {
  if (nc == 1) {
    for (int c = 0; c < d; ++c) w[c] = a[0] * u[c];
  } else if (d == 2) {  // xx, yy, xy
    w[0] = a[0] * u[0] + a[2] * u[1];
    w[1] = a[2] * u[0] + a[1] * u[1];
  } else {  // xx, yy, zz, xy, xz, yz
    w[0] = a[0] * u[0] + a[3] * u[1] + a[4] * u[2];
    w[1] = a[3] * u[0] + a[1] * u[1] + a[5] * u[2];
    w[2] = a[4] * u[0] + a[5] * u[1] + a[2] * u[2];
  }
}

__device__ __forceinline__ void decode_pair(const Geo& g, int q, int& h0, int& k1) {
  const int half1 = (g.N[1] + 1) / 2;
  if (q < half1) {
    h0 = 0;
    k1 = q;
  } else {
    const int q2 = q - half1;
    h0 = 1 + q2 / g.N[1];
    k1 = fr(q2 % g.N[1], g.N[1]);
  }
}

__host__ __device__ __forceinline__ size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }


// Energy rule.  A CG step x += alpha p lowers the energy a(E + x, E + x) of
// the iterate by alpha gamma (gamma = <r, r>), so the energy of every iterate
// (an upper bound on the primal side, on B on the dual side) is known from the
// recurrence: energy0 - esum.  The remaining decrease is extrapolated from the
// last four decrements as a geometric tail (ratio rho from the first and last
// of them), with a factor 2 of margin; the rule stops when it is below etol
// times the current energy.  It is an extra exit beside the residual rule,
// which still ends solves that are exact from the start.
// Copy of the CG states of L consecutive loads into shared memory, read by
// every thread of the block at once (one word each); the block synchronises
// before using it.
template <int L>
__device__ __forceinline__ void copy_states(const CgScal* __restrict__ src, CgScal* dst, int tid, int nthr) {
  static_assert(sizeof(CgScal) % 8 == 0, "CG state is a whole number of 8-byte words");
  constexpr int W = (int)(sizeof(CgScal) / 8);
  const unsigned long long* s = reinterpret_cast<const unsigned long long*>(src);
  unsigned long long* d = reinterpret_cast<unsigned long long*>(dst);
  for (int i = tid; i < L * W; i += nthr) d[i] = s[i];
}

// The state is read from r and written to w (the same record, or a copy of it
// taken before the writes).
__device__ __forceinline__ void energy_record(const CgScal* r, CgScal* w, int j, double dec) {
  w->edec[j & 3] = dec;
  w->esum = r->esum + dec;
}

__device__ __forceinline__ bool energy_converged(const CgScal* sc, int it) {
  if (it < 5) return false;
  const double d1 = sc->edec[(it - 1) & 3], d4 = sc->edec[(it - 4) & 3];
  if (!(d1 >= 0.0) || !(d4 > 0.0)) return false;
  const double rho = cbrt(d1 / d4);
  if (!(rho < 0.99)) return false;
  const double rem = 2.0 * d1 * rho / (1.0 - rho);
  return rem <= sc->etol * (sc->energy0 - sc->esum);
}

// Guaranteed rule.  For a lower bound mu on the spectrum of the operator,
// the Gauss-Radau quadrature of the CG Lanczos process bounds the remaining
// energy decrease of iterate j from above by gamma_j phi_j, with phi_0 = 1/mu
// and phi_j = t / (mu t + gamma_j / gamma_{j-1}), t = phi_{j-1} - alpha_{j-1}
// (Meurant and Tichy, Numer. Algorithms 2019).  gamma / mu bounds it as well,
// so phi never exceeds 1/mu, and 1/mu replaces a value that rounding has made
// meaningless.
__device__ __forceinline__ double radau_phi(const CgScal* sc, int it, double gam) {
  if (!(sc->mu > 0.0)) return INFINITY;
  const double inv = 1.0 / sc->mu;
  if (it == 0) return inv;
  const double t = sc->phi[(it - 1) & 1] - sc->alpha[(it - 1) & 1];
  const double ph = t / (sc->mu * t + gam / sc->gamma[(it - 1) & 1]);
  return (t > 0.0 && ph > 0.0 && ph < inv) ? ph : inv;
}

// Gap rule.  For a load E the primal energy U of the iterate bounds E.A_H E
// from above and L = |E|^4 / V, V the dual energy for J = E, from below
// (Cauchy-Schwarz with V >= E.A_H^-1 E).  With the Gauss-Radau bounds R on
// U - U* and R' = |E|^4 R_V / (V (V - R_V)) on L* - L (infinite unless
// V > R_V), the converged gap D* = U* - L* of this entry (eq.
// approx_homog_with_error) is at least (U - R) - (L + R').  A side stops when
// its own bound is at most etol (theta) times that: its algebraic error is
// then below theta D* (Convergence-criteria remark, Sec. 7.2).  The partner's
// (energy, bound) is its state at the last iterate of the previous chunk of
// iterations (start energy with an infinite bound during the first chunk):
// any iterate's values are valid, and the chunk-lockstep launch order of the
// two solves makes the decision deterministic.
__device__ __forceinline__ bool gap_converged(const CgScal* sc, int it, double own_rem) {
  const CgScal* o = sc->partner;
  if (!o) return false;
  const int slot = ((it / sc->chunk) + 1) & 1;          // the partner's previous chunk
  const double oe = o->snap_e[slot], orem = o->snap_r[slot];
  const double own_e = sc->energy0 - sc->esum;
  const double n2 = sc->normE * sc->normE, n4 = n2 * n2;
  double U, RU, V, RV;
  if (sc->side == 0) {
    U = own_e, RU = own_rem, V = oe, RV = orem;
  } else {
    U = oe, RU = orem, V = own_e, RV = own_rem;
  }
  const double L = n4 / V;
  const double RL = (V - RV > 0.0) ? n4 * RV / (V * (V - RV)) : INFINITY;
  const double dlow = (U - RU) - (L + RL);
  const double own = sc->side == 0 ? RU : RL;
  return dlow > 0.0 && own <= sc->etol * dlow;
}

// Stopping test of iteration it with gamma = gam, on the state sc; the writer
// thread (w not null) keeps the state of the guaranteed and gap rules in w
// (parity-buffered: other blocks of the same launch read the previous
// iteration's entry).
__device__ __forceinline__ bool stop_test(const CgScal* sc, CgScal* w, int it, double gam) {
  bool conv = sqrt(gam) <= sc->tol * sc->normE;
  if (sc->stop == 1) {
    conv = conv || energy_converged(sc, it);
  } else if (sc->stop == 2) {
    const double ph = radau_phi(sc, it, gam);
    if (w) w->phi[it & 1] = ph;
    conv = conv || gam * ph <= sc->etol * (sc->energy0 - sc->esum);
  } else if (sc->stop == 3) {
    const double ph = radau_phi(sc, it, gam);
    if (w) {
      w->phi[it & 1] = ph;
      w->rem = gam * ph;
    }
    conv = conv || gap_converged(sc, it, gam * ph);
  }
  return conv;
}

}  // namespace hom
