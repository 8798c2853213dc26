// Fused passes with register-resident four-step FFTs for the doubled-grid
// lengths of the benchmark configurations (M = 25, 81, 125, 625), FP32.
//
// Same arithmetic as the generic passes in hom_kernels.hip (same maps between
// Z_N and the doubled grid, same packing of two real fields per complex line,
// same CG recurrences), but every line FFT is M = A * B with A- and B-point
// DFTs held in registers and a single LDS exchange, all sizes compile-time.
// Launchers return false when no specialisation exists; the caller then uses
// the generic pass.
#include "hom_device.hpp"
#include "hom_regfft.hpp"

#include <hip/hip_ext.h>

#include <cstdlib>

namespace hom {

namespace {

constexpr int round64(int v) { return (v + 63) / 64 * 64; }

template <int M>
struct Cfg {
  static constexpr int A = rf::Split<M>::A, B = rf::Split<M>::B;
  static constexpr int T = A > B ? A : B;       // threads per line
  static constexpr int N = (M + 1) / 2, H = (N - 1) / 2;
};

__device__ __forceinline__ bool any_active(const UnitDev& U, int L) {
  bool a = false;
  for (int l = 0; l < L; ++l) a |= (U.sc[l].status == 0);
  return a;
}

// doubled-grid position -> kept index on Z_N (FFT order), or -1
template <int M>
__device__ __forceinline__ int kept(int pos) {
  constexpr int N = Cfg<M>::N, H = Cfg<M>::H;
  return pos <= H ? pos : (pos >= M - H ? pos - (M - N) : -1);
}

}  // namespace

// ============================================================== column pass
// TP points per block, T threads per point; every thread keeps all P packs.
template <typename R, int M, int D, int P, int NC, int TP>
__global__ __launch_bounds__(TP * Cfg<M>::T) void k_apply_fast(Geo g, const UnitDev* __restrict__ units, int cg) {
  constexpr int A = Cfg<M>::A, B = Cfg<M>::B, T = Cfg<M>::T, N = Cfg<M>::N;
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<R>* tw = reinterpret_cast<Cx<R>*>(smem);   // [M]
  Cx<R>* ex = tw + M;                           // [M][TP]
  const UnitDev& U = units[blockIdx.z];
  if (cg && !any_active(U, g.L)) return;
  const int npts = g.M[1] * g.M[2];
  const size_t Mtot = (size_t)M * npts;
  const int p0 = blockIdx.x * TP;
  const int tid = threadIdx.x, pt = tid % TP, q = tid / TP;
  const bool ok = (p0 + pt) < npts;
  const Cx<R>* twg = reinterpret_cast<const Cx<R>*>(g.tw[0]);
  for (int i = tid; i < M; i += blockDim.x) tw[i] = twg[i];
  Cx<R>* data = reinterpret_cast<Cx<R>*>(g.N[1] > 1 ? U.bufB : U.bufA);
  const size_t col = (size_t)(p0 + pt) * P;
  const size_t rowstride = (size_t)npts * P;

  Cx<R> v[P][T];
  // inverse, step 1: thread n2 = q holds x[B n1 + n2] (zero-padded N -> M)
#pragma unroll
  for (int n1 = 0; n1 < A; ++n1) {
    const int n = B * n1 + q;
    const int i0 = (q < B && ok) ? kept<M>(n) : -1;
#pragma unroll
    for (int pk = 0; pk < P; ++pk) v[pk][n1] = i0 >= 0 ? data[i0 * rowstride + col + pk] : rf::mk<R>(0, 0);
  }
  __syncthreads();
#pragma unroll
  for (int pk = 0; pk < P; ++pk) {
    if (q < B) {
      rf::Dft<R, A, 1>::run(v[pk]);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) {
        Cx<R> w = tw[q * k1];
        w.y = -w.y;
        ex[(q * A + k1) * TP + pt] = rf::mul(v[pk][k1], w);
      }
    }
    __syncthreads();
    if (q < A) {
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) v[pk][n2] = ex[(n2 * A + q) * TP + pt];
      rf::Dft<R, B, 1>::run(v[pk]);
    }
    __syncthreads();
  }
  // thread k1 = q holds u at x0 = q + A k2: apply the coefficient on the doubled grid
  if (q < A && ok) {
    const R* coef = reinterpret_cast<const R*>(U.coef);
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) {
      const size_t ci = (size_t)(q + A * k2) * npts + p0 + pt;
      R a[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) a[c] = coef[c * Mtot + ci];
      R u[2 * P], w[2 * P];
#pragma unroll
      for (int pk = 0; pk < P; ++pk) {
        u[2 * pk] = v[pk][k2].x;
        u[2 * pk + 1] = v[pk][k2].y;
      }
#pragma unroll
      for (int f = 0; f < 2 * P; ++f) w[f] = (R)0;
#pragma unroll
      for (int l = 0; l < (2 * P) / D; ++l) coef_mul<R>(D, NC, a, u + l * D, w + l * D);
#pragma unroll
      for (int pk = 0; pk < P; ++pk) v[pk][k2] = rf::mk<R>(w[2 * pk], w[2 * pk + 1]);
    }
  }
  // forward: step A over n2 in registers (thread n1 = q), exchange, step B over n1
#pragma unroll
  for (int pk = 0; pk < P; ++pk) {
    if (q < A) {
      rf::Dft<R, B, -1>::run(v[pk]);
#pragma unroll
      for (int m2 = 0; m2 < B; ++m2) ex[(q * B + m2) * TP + pt] = rf::mul(v[pk][m2], tw[q * m2]);
    }
    __syncthreads();
    if (q < B) {
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) v[pk][n1] = ex[(n1 * B + q) * TP + pt];
      rf::Dft<R, A, -1>::run(v[pk]);
    }
    __syncthreads();
  }
  // thread m2 = q holds X[q + B m1]: store the Z_N0 part
  if (q < B && ok) {
#pragma unroll
    for (int m1 = 0; m1 < A; ++m1) {
      const int i0 = kept<M>(q + B * m1);
      if (i0 >= 0)
#pragma unroll
        for (int pk = 0; pk < P; ++pk) data[i0 * rowstride + col + pk] = v[pk][m1];
    }
  }
  (void)N;
}

// ============================================================== row passes
// G row pairs per block; line A = (h0, k1, .), line B = (-h0, -k1, .).  The
// packed fields of both lines are staged in LDS in natural position order
// ([2G lines][P packs][M]); the four-step FFT runs one pack at a time and
// reuses the staging area for its exchange.
// T(k) of the field layout with compile-time dimension and problem type.
template <int D, int DUAL>
__device__ __forceinline__ void basis_t(const Geo& g, int k0, int k1, int k2, double T[3][2]) {
  const int kk[3] = {k0, k1, k2};
  double n[3] = {0.0, 0.0, 0.0};
  double n2 = 0.0;
#pragma unroll
  for (int c = 0; c < D; ++c) {
    const int a = (D == 2) ? (c == 0 ? 0 : 2) : c;
    n[c] = kk[a] * g.iY[a];
    n2 += n[c] * n[c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) T[c][0] = T[c][1] = 0.0;
  if (n2 == 0.0) return;
  const double inv = 1.0 / sqrt(n2);
#pragma unroll
  for (int c = 0; c < D; ++c) n[c] *= inv;
  if constexpr (!DUAL) {
#pragma unroll
    for (int c = 0; c < D; ++c) T[c][0] = n[c];
  } else if constexpr (D == 2) {
    T[0][0] = -n[1];
    T[1][0] = n[0];
  } else {
    const double a0 = fabs(n[0]), a1 = fabs(n[1]), a2 = fabs(n[2]);
    const int a = (a1 < a0) ? ((a2 < a1) ? 2 : 1) : ((a2 < a0) ? 2 : 0);
    double t1[3] = {-n[a] * n[0], -n[a] * n[1], -n[a] * n[2]};
    t1[0] += (a == 0);
    t1[1] += (a == 1);
    t1[2] += (a == 2);
    const double in1 = 1.0 / sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
    t1[0] *= in1;
    t1[1] *= in1;
    t1[2] *= in1;
    T[0][0] = t1[0];
    T[1][0] = t1[1];
    T[2][0] = t1[2];
    T[0][1] = n[1] * t1[2] - n[2] * t1[1];
    T[1][1] = n[2] * t1[0] - n[0] * t1[2];
    T[2][1] = n[0] * t1[1] - n[1] * t1[0];
  }
}

struct RowInfo {
  int valid, h0, k1, rowB, self, i1A, i1B, i0B;
};

__device__ __forceinline__ void row_info(const Geo& g, int qpair, RowInfo& ri) {
  ri.valid = qpair < g.Q;
  int h0 = 0, k1 = 0;
  if (ri.valid) decode_pair(g, qpair, h0, k1);
  ri.h0 = h0;
  ri.k1 = k1;
  ri.self = (h0 == 0 && k1 == 0);
  ri.rowB = (h0 == 0 && k1 != 0);
  ri.i1A = ixn(k1, g.N[1]);
  ri.i1B = ixn(-k1, g.N[1]);
  ri.i0B = ixn(-h0, g.N[0]);
}

template <typename R, int M, int D, int L, int DUAL, int G>
__global__ __launch_bounds__(round64(2 * G * Cfg<M>::T)) void k_first_fast(Geo g, const UnitDev* __restrict__ units,
                                                                         int mode, int jstep,
                                                                         const int* __restrict__ iter_base) {
  constexpr int A = Cfg<M>::A, B = Cfg<M>::B, T = Cfg<M>::T, N2 = Cfg<M>::N, H2 = Cfg<M>::H;
  constexpr int P = (L * D + 1) / 2, m = DUAL ? D - 1 : 1, d = D;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_alpha[kMaxLoads];
  __shared__ int s_act[kMaxLoads];
  __shared__ double s_red[16];
  __shared__ RowInfo s_row[G];
  const UnitDev& U = units[blockIdx.z];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int N1 = g.N[1];
  const int it = iter_base ? (*iter_base + jstep) : 0;
  Cx<R>* tw = reinterpret_cast<Cx<R>*>(smem);                          // [M]
  Cx<R>* stage = reinterpret_cast<Cx<R>*>(smem + align16(M * sizeof(Cx<R>)));  // [2G][P][M]

  if (tid < 64) {
    const int lane = tid;
    for (int w = 0; w < L; ++w) {
      int act = 1;
      double alpha = 0.0;
      if (mode == FIRST_CG) {
        CgScal* sc = U.sc + w;
        act = (sc->status == 0);
        if (act && it > 0) {
          const double delta = wave_sum_arr(U.part_d + (size_t)w * g.nbL, g.nbL);
          const double gam = sc->gamma[(it - 1) & 1];
          double den = delta;
          if (it > 1) den = delta - sc->beta[(it - 1) & 1] * gam / sc->alpha[(it - 2) & 1];
          if (!(den > 0.0)) {
            act = 0;
            if (blockIdx.x == 0 && lane == 0) {
              sc->status = -3;
              sc->iters = it - 1;
              sc->gamma_last = gam;
            }
          } else {
            alpha = gam / den;
            if (blockIdx.x == 0 && lane == 0) sc->alpha[(it - 1) & 1] = alpha;
          }
        }
      }
      if (lane == 0) {
        s_alpha[w] = alpha;
        s_act[w] = act;
      }
    }
  }
  if (tid < G) row_info(g, blockIdx.x * G + tid, s_row[tid]);
  const Cx<R>* twg = reinterpret_cast<const Cx<R>*>(g.tw[2]);
  for (int i = tid; i < M; i += nthr) tw[i] = twg[i];
  for (int i = tid; i < 2 * G * P * M; i += nthr) stage[i] = rf::mk<R>(0, 0);
  __syncthreads();
  if (mode == FIRST_CG) {
    int any = 0;
    for (int l = 0; l < L; ++l) any |= s_act[l];
    if (!any) return;
  }

  // ---- CG update of the stored entries; packed fields of row A into the staging area
  double gp0 = 0.0, gp1 = 0.0, gp2 = 0.0;
  for (int t = tid; t < G * 2 * N2; t += nthr) {
    const int gp = t / (2 * N2), rem = t - gp * 2 * N2;
    const int row = rem / N2, i2 = rem - row * N2;
    const RowInfo& ri = s_row[gp];
    if (!ri.valid || (row == 1 && !ri.rowB)) continue;
    const int h0 = ri.h0;
    const int i1 = row ? ri.i1B : ri.i1A;
    const double wt = h0 == 0 ? 1.0 : 2.0;
    Cx<double> rv[L][m];
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
      for (int c = 0; c < m; ++c) {
        const size_t idx = ((size_t)(c * g.H0 + h0) * N1 + i1) * N2 + i2;
        Cx<double> v = cx(0.0, 0.0);
        if (mode != FIRST_CG) {
          v = U.x[l][idx];
        } else if (s_act[l]) {
          v = U.r[l][idx];
          if (it > 0) {
            const double a = s_alpha[l];
            const Cx<double> xv = U.x[l][idx], pv = U.p[l][idx], sv = U.s[l][idx];
            v = v - sv * a;
            U.x[l][idx] = xv + pv * a;
            U.r[l][idx] = v;
          }
          const double e = wt * (v.x * v.x + v.y * v.y);
          if (l == 0) gp0 += e;
          else if (l == 1) gp1 += e;
          else gp2 += e;
        }
        rv[l][c] = v;
      }
    if (row == 1) continue;
    // fields x_hat_{l,gam}(k) = sum_c T_{gam c}(k) r_{l,c}(k) on line A at k2 and their conjugates on line B at -k2
    const int k2 = fr(i2, N2);
    double Tb[3][2];
    basis_t<D, DUAL>(g, h0, ri.k1, k2, Tb);
    const int posA = padpos(i2, N2, M), posB = padpos(ixn(-k2, N2), N2, M);
    Cx<R>* sA = stage + (size_t)(2 * gp) * P * M;
    Cx<R>* sB = stage + (size_t)(2 * gp + 1) * P * M;
#pragma unroll
    for (int pk = 0; pk < P; ++pk) {
      Cx<double> X[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int f = 2 * pk + s;
        X[s] = cx(0.0, 0.0);
        if (f < L * d) {
          const int lf = f / d, gam = f - (f / d) * d;
#pragma unroll
          for (int c = 0; c < m; ++c) X[s] = X[s] + rv[lf][c] * Tb[gam][c];
          if (mode == FIRST_BOUNDS && ri.self && k2 == 0) X[s].x += U.E[lf][gam];
        }
      }
      sA[pk * M + posA] = rf::mk<R>((R)(X[0].x - X[1].y), (R)(X[0].y + X[1].x));
      if (!ri.self) sB[pk * M + posB] = rf::mk<R>((R)(X[0].x + X[1].y), (R)(-X[0].y + X[1].x));
    }
  }
  if (mode == FIRST_CG) {
    for (int l = 0; l < L; ++l) {
      double v = l == 0 ? gp0 : (l == 1 ? gp1 : gp2);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if ((tid & 63) == 0) s_red[tid >> 6] = v;
      __syncthreads();
      if (tid == 0) {
        double s = 0.0;
        for (int i = 0; i < (nthr + 63) / 64; ++i) s += s_red[i];
        U.part_g[(size_t)l * g.nbF + blockIdx.x] = s;
      }
      __syncthreads();
    }
  }
  __syncthreads();

  // ---- inverse four-step FFT of every (line, pack), one pack at a time
  const int grp = tid / T, q = tid - (tid / T) * T;
  const int gp = grp >> 1, line = grp & 1;
  bool live = grp < 2 * G;
  RowInfo ri;
  if (live) {
    ri = s_row[gp];
    live = ri.valid && !(line == 1 && ri.self);
  }
  Cx<R>* out = reinterpret_cast<Cx<R>*>(U.bufA);
  const int i0 = live ? (line ? ri.i0B : ri.h0) : 0;
  const int i1 = live ? (line ? ri.i1B : ri.i1A) : 0;
  Cx<R> v[T];
#pragma unroll
  for (int pk = 0; pk < P; ++pk) {
    Cx<R>* sp = stage + ((size_t)grp * P + pk) * M;
    if (live && q < B) {
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) v[n1] = sp[B * n1 + q];
    }
    __syncthreads();
    if (live && q < B) {
      rf::Dft<R, A, 1>::run(v);
#pragma unroll
      for (int k1r = 0; k1r < A; ++k1r) {
        Cx<R> w = tw[q * k1r];
        w.y = -w.y;
        sp[q * A + k1r] = rf::mul(v[k1r], w);
      }
    }
    __syncthreads();
    if (live && q < A) {
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) v[n2] = sp[n2 * A + q];
      rf::Dft<R, B, 1>::run(v);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) out[(((size_t)i0 * N1 + i1) * M + (q + A * k2)) * P + pk] = v[k2];
    }
  }
  (void)H2;
}

template <typename R, int M, int D, int L, int DUAL, int G>
__global__ __launch_bounds__(round64(2 * G * Cfg<M>::T)) void k_last_fast(Geo g, const UnitDev* __restrict__ units,
                                                                        int mode, int jstep,
                                                                        const int* __restrict__ iter_base) {
  constexpr int A = Cfg<M>::A, B = Cfg<M>::B, T = Cfg<M>::T, N2 = Cfg<M>::N;
  constexpr int P = (L * D + 1) / 2, m = DUAL ? D - 1 : 1, d = D;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_beta[kMaxLoads];
  __shared__ int s_act[kMaxLoads];
  __shared__ double s_red[16];
  __shared__ RowInfo s_row[G];
  const UnitDev& U = units[blockIdx.z];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int N1 = g.N[1];
  const int it = iter_base ? (*iter_base + jstep) : 0;
  Cx<R>* tw = reinterpret_cast<Cx<R>*>(smem);                                   // [M]
  Cx<R>* stage = reinterpret_cast<Cx<R>*>(smem + align16(M * sizeof(Cx<R>)));  // [2G][P][M]

  if (tid < 64) {
    const int lane = tid;
    for (int w = 0; w < L; ++w) {
      int act = 1;
      double beta = 0.0;
      if (mode == LAST_CG) {
        CgScal* sc = U.sc + w;
        act = (sc->status == 0);
        if (act) {
          const double gam = wave_sum_arr(U.part_g + (size_t)w * g.nbF, g.nbF);
          const bool bad = !(gam == gam) || gam > 1e300;
          const bool conv = sqrt(gam) <= sc->tol * sc->normE;
          if (bad || conv || it >= sc->maxit) {
            act = 0;
            if (blockIdx.x == 0 && lane == 0) {
              sc->status = bad ? -1 : (conv ? 1 : 2);
              sc->iters = it;
              sc->gamma_last = gam;
              if (it == 0) sc->gamma0 = gam;
            }
          } else {
            beta = (it == 0) ? 0.0 : gam / sc->gamma[(it - 1) & 1];
            if (blockIdx.x == 0 && lane == 0) {
              sc->gamma[it & 1] = gam;
              sc->beta[it & 1] = beta;
              if (it == 0) sc->gamma0 = gam;
            }
          }
        }
      }
      if (lane == 0) {
        s_beta[w] = beta;
        s_act[w] = act;
      }
    }
  }
  if (tid < G) row_info(g, blockIdx.x * G + tid, s_row[tid]);
  const Cx<R>* twg = reinterpret_cast<const Cx<R>*>(g.tw[2]);
  for (int i = tid; i < M; i += nthr) tw[i] = twg[i];
  __syncthreads();
  {
    int any = 0;
    for (int l = 0; l < L; ++l) any |= s_act[l];
    if (!any) return;
  }

  // ---- forward four-step FFT of every (line, pack); natural-order result in the staging area
  const int grp = tid / T, q = tid - (tid / T) * T;
  const int gp = grp >> 1, line = grp & 1;
  bool live = grp < 2 * G;
  RowInfo ri;
  if (live) {
    ri = s_row[gp];
    live = ri.valid && !(line == 1 && ri.self);
  }
  const Cx<R>* in = reinterpret_cast<const Cx<R>*>(U.bufA);
  const int i0 = live ? (line ? ri.i0B : ri.h0) : 0;
  const int i1 = live ? (line ? ri.i1B : ri.i1A) : 0;
  Cx<R> v[P][T];
  if (live && q < A) {
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2)
#pragma unroll
      for (int pk = 0; pk < P; ++pk) v[pk][n2] = in[(((size_t)i0 * N1 + i1) * M + (q + A * n2)) * P + pk];
  }
#pragma unroll
  for (int pk = 0; pk < P; ++pk) {
    Cx<R>* sp = stage + ((size_t)grp * P + pk) * M;
    if (live && q < A) {
      rf::Dft<R, B, -1>::run(v[pk]);
#pragma unroll
      for (int m2 = 0; m2 < B; ++m2) sp[q * B + m2] = rf::mul(v[pk][m2], tw[q * m2]);
    }
    __syncthreads();
    if (live && q < B) {
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) v[pk][n1] = sp[n1 * B + q];
      rf::Dft<R, A, -1>::run(v[pk]);
    }
    __syncthreads();
    if (live && q < B) {
#pragma unroll
      for (int m1 = 0; m1 < A; ++m1) sp[q + B * m1] = v[pk][m1];
    }
  }
  __syncthreads();

  // ---- epilogue: unpack, project (T^T), CG direction update, <r, C r>
  double dp0 = 0.0, dp1 = 0.0, dp2 = 0.0;
  const double sc_m = g.invM * 0.5;
  for (int t = tid; t < G * 2 * N2; t += nthr) {
    const int gpe = t / (2 * N2), rem = t - gpe * 2 * N2;
    const int row = rem / N2, i2 = rem - row * N2;
    const RowInfo& re = s_row[gpe];
    if (!re.valid || (row == 1 && !re.rowB)) continue;
    const int k2 = fr(i2, N2);
    const int lineK = re.self ? 0 : row, lineM = re.self ? 0 : 1 - row;
    const Cx<R>* zK = stage + (size_t)(2 * gpe + lineK) * P * M;
    const Cx<R>* zM = stage + (size_t)(2 * gpe + lineM) * P * M;
    const int jK = padpos(i2, N2, M), jM = padpos(ixn(-k2, N2), N2, M);
    const int kk0 = row ? 0 : re.h0, kk1 = row ? -re.k1 : re.k1;
    const int ii1 = row ? re.i1B : re.i1A;
    const double wt = (re.h0 == 0) ? 1.0 : 2.0;
    double Tb[3][2];
    basis_t<D, DUAL>(g, kk0, kk1, k2, Tb);
#pragma unroll
    for (int l = 0; l < L; ++l) {
      if (mode == LAST_CG && !s_act[l]) continue;
      Cx<double> rv[m], pv[m], sv[m], bv[m];
#pragma unroll
      for (int c = 0; c < m; ++c) {
        const size_t idx = ((size_t)(c * g.H0 + kk0) * N1 + ii1) * N2 + i2;
        if (mode == LAST_CG) {
          rv[c] = U.r[l][idx];
          if (it > 0) {
            pv[c] = U.p[l][idx];
            sv[c] = U.s[l][idx];
          }
        } else if (mode == LAST_RESID) {
          bv[c] = U.b[l][idx];
        }
      }
      Cx<double> wv[D];
#pragma unroll
      for (int gam = 0; gam < d; ++gam) {
        const int f = l * d + gam, pk = f >> 1;
        const Cx<R> za = zK[pk * M + jK];
        const Cx<R> zb = zM[pk * M + jM];
        if ((f & 1) == 0)
          wv[gam] = cx(((double)za.x + (double)zb.x) * sc_m, ((double)za.y - (double)zb.y) * sc_m);
        else
          wv[gam] = cx(((double)za.y + (double)zb.y) * sc_m, -((double)za.x - (double)zb.x) * sc_m);
      }
#pragma unroll
      for (int c = 0; c < m; ++c) {
        Cx<double> w = cx(0.0, 0.0);
#pragma unroll
        for (int gam = 0; gam < d; ++gam) w = w + wv[gam] * Tb[gam][c];
        const size_t idx = ((size_t)(c * g.H0 + kk0) * N1 + ii1) * N2 + i2;
        double e;
        if (mode == LAST_CG) {
          const double b = s_beta[l];
          if (it == 0) {
            U.p[l][idx] = rv[c];
            U.s[l][idx] = w;
          } else {
            U.p[l][idx] = rv[c] + pv[c] * b;
            U.s[l][idx] = w + sv[c] * b;
          }
          e = wt * (rv[c].x * w.x + rv[c].y * w.y);
        } else if (mode == LAST_RESID) {
          const Cx<double> rn = bv[c] - w;
          U.r[l][idx] = rn;
          e = wt * (rn.x * rn.x + rn.y * rn.y);
        } else {
          U.s[l][idx] = w;
          e = wt * (w.x * w.x + w.y * w.y);
        }
        if (l == 0) dp0 += e;
        else if (l == 1) dp1 += e;
        else dp2 += e;
      }
    }
  }
  for (int l = 0; l < L; ++l) {
    double v2 = l == 0 ? dp0 : (l == 1 ? dp1 : dp2);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v2 += __shfl_down(v2, off, 64);
    if ((tid & 63) == 0) s_red[tid >> 6] = v2;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int i = 0; i < (nthr + 63) / 64; ++i) s += s_red[i];
      U.part_d[(size_t)l * g.nbL + blockIdx.x] = s;
    }
    __syncthreads();
  }
}

// ============================================================== dispatch
template <typename K>
static hipError_t launch_k(K kern, dim3 grid, int threads, size_t lds, hipStream_t st, const Geo& g,
                           const UnitDev* units, int a, int b, const int* c) {
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (g_ext_timing.on)
    hipExtLaunchKernelGGL(kern, grid, dim3(threads), lds, st, g_ext_timing.start, g_ext_timing.stop, 0, g, units, a, b,
                          c);
  else
    hipLaunchKernelGGL(kern, grid, dim3(threads), lds, st, g, units, a, b, c);
  return hipGetLastError();
}

template <int M, int D, int P, int NC>
static hipError_t run_apply(const Geo& g, const UnitDev* units, int n, int cg, hipStream_t st) {
  constexpr int T = Cfg<M>::T;
  constexpr int TP = (M >= 625) ? 8 : (256 / T);
  const int npts = g.M[1] * g.M[2];
  const size_t lds = (size_t)M * sizeof(Cx<float>) * (1 + TP);
  auto kern = k_apply_fast<float, M, D, P, NC, TP>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const dim3 grid((npts + TP - 1) / TP, 1, n);
  if (g_ext_timing.on)
    hipExtLaunchKernelGGL(kern, grid, dim3(TP * T), lds, st, g_ext_timing.start, g_ext_timing.stop, 0, g, units, cg);
  else
    hipLaunchKernelGGL(kern, grid, dim3(TP * T), lds, st, g, units, cg);
  return hipGetLastError();
}

// Returns true when a specialised column pass handled the launch (*err set).
bool fast_apply(const Geo& g, const UnitDev* units, int n, int cg, hipStream_t st, hipError_t* err) {
  if (std::getenv("HOM_NO_FAST")) return false;
  const int M = g.M[0], D = g.d, P = g.P, NC = g.nc;
#define HOM_AP(MM, DD, PP, CC)                                      \
  if (M == MM && D == DD && P == PP && NC == CC) {                 \
    *err = run_apply<MM, DD, PP, CC>(g, units, n, cg, st);         \
    return true;                                                   \
  }
  HOM_AP(625, 2, 1, 1) HOM_AP(625, 2, 2, 1) HOM_AP(625, 2, 1, 3) HOM_AP(625, 2, 2, 3)
  HOM_AP(125, 2, 1, 1) HOM_AP(125, 2, 2, 1) HOM_AP(125, 2, 1, 3) HOM_AP(125, 2, 2, 3)
  HOM_AP(81, 2, 1, 1) HOM_AP(81, 2, 2, 1) HOM_AP(81, 2, 1, 3) HOM_AP(81, 2, 2, 3)
  HOM_AP(25, 2, 1, 1) HOM_AP(25, 2, 2, 1) HOM_AP(25, 2, 1, 3) HOM_AP(25, 2, 2, 3)
  HOM_AP(81, 3, 2, 1) HOM_AP(81, 3, 3, 1) HOM_AP(81, 3, 5, 1)
  HOM_AP(81, 3, 2, 6) HOM_AP(81, 3, 3, 6) HOM_AP(81, 3, 5, 6)
#undef HOM_AP
  return false;
}

template <int M>
static constexpr int pairs_per_block() {
  return (M >= 625) ? 2 : ((M >= 125) ? 4 : (256 / (2 * Cfg<M>::T)));
}

static bool row_supported(int M, int D, int L) {
  if (D == 2) return (M == 625 || M == 125 || M == 81 || M == 25) && (L == 1 || L == 2);
  return M == 81 && L >= 1 && L <= 3;
}

// Row pairs per block of the specialised row passes, or 0 when no
// specialisation exists (then the generic passes run).
int fast_row_pairs(int M, int D, int L) {
  if (std::getenv("HOM_NO_FAST")) return 0;
  if (!row_supported(M, D, L)) return 0;
  if (M == 625) return pairs_per_block<625>();
  if (M == 125) return pairs_per_block<125>();
  if (M == 81) return pairs_per_block<81>();
  return pairs_per_block<25>();
}

template <int M, int D, int L, int DUAL>
static hipError_t run_row(bool first, const Geo& g, const UnitDev* units, int n, int mode, int jstep,
                          const int* iter_base, hipStream_t st) {
  constexpr int G = pairs_per_block<M>();
  constexpr int T = Cfg<M>::T, P = (L * D + 1) / 2;
  const int nb = (g.Q + G - 1) / G;
  const size_t lds = align16(M * sizeof(Cx<float>)) + (size_t)2 * G * P * M * sizeof(Cx<float>);
  if (first)
    return launch_k(k_first_fast<float, M, D, L, DUAL, G>, dim3(nb, 1, n), round64(2 * G * T), lds, st, g, units,
                    mode, jstep, iter_base);
  return launch_k(k_last_fast<float, M, D, L, DUAL, G>, dim3(nb, 1, n), round64(2 * G * T), lds, st, g, units, mode,
                  jstep, iter_base);
}

template <int M, int D, int L>
static hipError_t run_row_d(bool first, const Geo& g, const UnitDev* units, int n, int mode, int jstep,
                            const int* iter_base, hipStream_t st) {
  return g.dual ? run_row<M, D, L, 1>(first, g, units, n, mode, jstep, iter_base, st)
                : run_row<M, D, L, 0>(first, g, units, n, mode, jstep, iter_base, st);
}

bool fast_row(bool first, const Geo& g, const UnitDev* units, int n, int mode, int jstep, const int* iter_base,
              hipStream_t st, hipError_t* err) {
  if (!fast_row_pairs(g.M[2], g.d, g.L)) return false;
  const int M = g.M[2], D = g.d, L = g.L;
#define HOM_RW(MM, DD, LL)                                                          \
  if (M == MM && D == DD && L == LL) {                                             \
    *err = run_row_d<MM, DD, LL>(first, g, units, n, mode, jstep, iter_base, st);  \
    return true;                                                                   \
  }
  HOM_RW(625, 2, 1) HOM_RW(625, 2, 2) HOM_RW(125, 2, 1) HOM_RW(125, 2, 2) HOM_RW(81, 2, 1) HOM_RW(81, 2, 2)
  HOM_RW(25, 2, 1) HOM_RW(25, 2, 2) HOM_RW(81, 3, 1) HOM_RW(81, 3, 2) HOM_RW(81, 3, 3)
#undef HOM_RW
  return false;
}

}  // namespace hom
