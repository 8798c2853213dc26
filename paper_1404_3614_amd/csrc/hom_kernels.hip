// HIP kernels of libhom for gfx950 (CDNA4, wave64).
//
// One CG iteration of the Galerkin method without numerical integration
// (Sec. 6-7) is a chain of line-FFT passes over the doubled grid M = 2N - 1:
//
//   k_first  (rows, last axis)  CG update x += a p, r -= a s; <r,r> partial;
//                               r_hat(k) -> x_hat(k) = T(k) r(k) packed two real
//                               fields per complex line; inverse FFT (zero-padded N -> M)
//   k_mid    (3D, axis 1)       inverse FFT of the middle axis (N1 -> M1)
//   k_apply  (columns, axis 0)  inverse FFT (N0 -> M0), coefficient apply
//                               w = A_M(x) u(x) on the doubled grid (eq. MBA_GA),
//                               forward FFT, truncation to Z_N0 (operator P_N)
//   k_mid    (3D, axis 1)       forward FFT with truncation (M1 -> N1)
//   k_last   (rows, last axis)  forward FFT with truncation, unpacking, projection
//                               onto range G^E / G^J by T(k)^T, CG direction update,
//                               <r, C r> partial
//
// FFTs are self-sorting (Stockham) radix-2/3/4/5 passes on lines staged in LDS,
// in place with register staging: every stage loads its butterfly inputs into
// registers, synchronises, then stores the outputs.  The doubled-grid field
// never goes to HBM: only the intermediates with one pruned axis do.
#include <cstdlib>
#include "hom_device.hpp"

#include <hip/hip_ext.h>

namespace hom {

thread_local ExtTiming g_ext_timing;

// ------------------------------------------------------------------ FFT
template <typename R>
__device__ __forceinline__ void bfly2(Cx<R>* v) {
  const Cx<R> a = v[0];
  v[0] = a + v[1];
  v[1] = a - v[1];
}

// X_k = sum_n x_n w^(n k), w = exp(sgn 2 pi i / 4) = sgn i
template <typename R>
__device__ __forceinline__ void bfly4(Cx<R>* v, R sgn) {
  const Cx<R> a = v[0] + v[2], b = v[0] - v[2], c = v[1] + v[3], e = imul(v[1] - v[3], sgn);
  v[0] = a + c;
  v[2] = a - c;
  v[1] = b + e;
  v[3] = b - e;
}

template <typename R>
__device__ __forceinline__ void bfly3(Cx<R>* v, R sgn) {
  const R s3 = (R)0.86602540378443864676;
  Cx<R> t = v[1] + v[2];
  Cx<R> dl = v[1] - v[2];
  Cx<R> m = v[0] - t * (R)0.5;
  Cx<R> j = imul(dl, sgn * s3);
  v[0] = v[0] + t;
  v[1] = m + j;
  v[2] = m - j;
}

template <typename R>
__device__ __forceinline__ void bfly5(Cx<R>* v, R sgn) {
  const R c1 = (R)0.30901699437494742410, c2 = (R)-0.80901699437494742410;
  const R s1 = (R)0.95105651629515357212, s2 = (R)0.58778525229247312917;
  Cx<R> t1 = v[1] + v[4], t2 = v[2] + v[3], t3 = v[1] - v[4], t4 = v[2] - v[3];
  Cx<R> a1 = v[0] + t1 * c1 + t2 * c2;
  Cx<R> a2 = v[0] + t1 * c2 + t2 * c1;
  Cx<R> b1 = t3 * s1 + t4 * s2;
  Cx<R> b2 = t3 * s2 - t4 * s1;
  v[0] = v[0] + t1 + t2;
  Cx<R> ib1 = imul(b1, sgn), ib2 = imul(b2, sgn);
  v[1] = a1 + ib1;
  v[4] = a1 - ib1;
  v[2] = a2 + ib2;
  v[3] = a2 - ib2;
}

// In-place Stockham FFT of nl interleaved lines of length M held in LDS as
// buf[j * nl + l] (element j of line l).  The whole block participates.
// Stage with radix R after Ns points done: butterfly j reads elements
// j + r M/R, twiddles by w^(r (j mod Ns) M/(Ns R)) and writes
// (j / Ns) Ns R + (j mod Ns) + r Ns.
template <typename R, int MAXB>
__device__ void lds_fft(Cx<R>* buf, int nl, int M, const Plan& pl, const Cx<R>* __restrict__ tw, bool inv) {
  const int tid = threadIdx.x;
  const R sgn = inv ? (R)1 : (R)-1;
  int Ns = 1;
  for (int s = 0; s < pl.n; ++s) {
    const int Rr = pl.r[s];
    const int nb = M / Rr;
    const int total = nb * nl;
    const int tstride = M / (Ns * Rr);
    Cx<R> v[MAXB][5];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
      const int t = tid + i * kBlock;
      if (t < total) {
        const int l = t % nl, j = t / nl;
#pragma unroll
        for (int r = 0; r < 5; ++r)
          if (r < Rr) v[i][r] = buf[(j + r * nb) * nl + l];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
      const int t = tid + i * kBlock;
      if (t < total) {
        const int l = t % nl, j = t / nl;
        const int k = j % Ns;
        if (k) {
#pragma unroll
          for (int r = 1; r < 5; ++r)
            if (r < Rr) {
              Cx<R> w = tw[r * k * tstride];
              if (inv) w.y = -w.y;
              v[i][r] = cmul(v[i][r], w);
            }
        }
        if (Rr == 5)
          bfly5(v[i], sgn);
        else if (Rr == 3)
          bfly3(v[i], sgn);
        else if (Rr == 4)
          bfly4(v[i], sgn);
        else
          bfly2(v[i]);
        const int base = (j / Ns) * Ns * Rr + k;
#pragma unroll
        for (int r = 0; r < 5; ++r)
          if (r < Rr) buf[(base + r * Ns) * nl + l] = v[i][r];
      }
    }
    __syncthreads();
    Ns *= Rr;
  }
}


// ============================================================== first pass
template <typename R, int MAXB>
__global__ __launch_bounds__(kBlock) void k_first(Geo g, const UnitDev* __restrict__ units, int mode, int jstep,
                                                  const int* __restrict__ iter_base) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_alpha[kMaxLoads];
  __shared__ int s_act[kMaxLoads];
  __shared__ double s_red[kBlock / 64];
  const UnitDev& U = units[blockIdx.z];
  const int tid = threadIdx.x;
  const int N0 = g.N[0], N1 = g.N[1], N2 = g.N[2], M2 = g.M[2];
  const int L = g.L, m = g.m, P = g.P, d = g.d;
  int h0, k1;
  decode_pair(g, blockIdx.x, h0, k1);
  const bool self = (h0 == 0 && k1 == 0);
  const bool rowB = (h0 == 0 && k1 != 0);
  const int i1A = ixn(k1, N1), i1B = ixn(-k1, N1);
  const int it = iter_base ? (*iter_base + jstep) : 0;
  const int nl = (self ? 1 : 2) * P;

  Cx<double>* rA = reinterpret_cast<Cx<double>*>(smem);
  Cx<R>* buf = reinterpret_cast<Cx<R>*>(smem + align16((size_t)L * m * N2 * sizeof(Cx<double>)));

  // ---- scalars of the step: alpha_{it-1} from <r, C r> partials of the last pass
  if (tid < kMaxLoads * 64) {
    const int w = tid >> 6, lane = tid & 63;
    if (w < L) {
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
            if (blockIdx.x == 0 && lane == 0) {
              sc->alpha[(it - 1) & 1] = alpha;
              energy_record(sc, sc, it - 1, alpha * gam);
            }
          }
        }
      }
      if (lane == 0) {
        s_alpha[w] = alpha;
        s_act[w] = act;
      }
    }
  }
  __syncthreads();
  if (mode == FIRST_CG) {
    int any = 0;
    for (int l = 0; l < L; ++l) any |= s_act[l];
    if (!any) return;  // uniform over the block
  }

  // ---- phase 1: CG update of the stored rows, stage row A in LDS
  double gp0 = 0.0, gp1 = 0.0, gp2 = 0.0;
  const int per_row = L * m * N2;
  const int nrows = rowB ? 2 : 1;
  const double wt = (h0 == 0) ? 1.0 : 2.0;
  for (int t = tid; t < nrows * per_row; t += kBlock) {
    const int row = t / per_row, rem = t - row * per_row;
    const int l = rem / (m * N2), c = (rem / N2) % m, i2 = rem % N2;
    const int i1 = row ? i1B : i1A;
    const size_t idx = ((size_t)(c * g.H0 + h0) * N1 + i1) * N2 + i2;
    Cx<double> val = cx(0.0, 0.0);
    if (mode == FIRST_CG) {
      if (s_act[l]) {
        Cx<double> rv = U.r[l][idx];
        if (it > 0) {
          const double a = s_alpha[l];
          Cx<double> xv = U.x[l][idx];
          const Cx<double> pv = U.p[l][idx], sv = U.s[l][idx];
          xv = xv + pv * a;
          rv = rv - sv * a;
          U.x[l][idx] = xv;
          U.r[l][idx] = rv;
        }
        const double e = wt * (rv.x * rv.x + rv.y * rv.y);
        if (l == 0) gp0 += e;
        else if (l == 1) gp1 += e;
        else gp2 += e;
        val = rv;
      }
    } else {
      val = U.x[l][idx];
    }
    if (row == 0) rA[(l * m + c) * N2 + i2] = val;
  }
  if (mode == FIRST_CG) {
    for (int l = 0; l < L; ++l) {
      const double s = block_sum(l == 0 ? gp0 : (l == 1 ? gp1 : gp2), s_red);
      if (tid == 0) U.part_g[(size_t)l * g.nbF + blockIdx.x] = s;
    }
  }
  __syncthreads();

  // ---- phase 2: fields of both lines, two real fields per complex pack
  const int hN2 = (N2 - 1) / 2;
  for (int t = tid; t < M2 * nl; t += kBlock) {
    const int j = t / nl, l = t - (t / nl) * nl;
    const int line = l / P, pk = l - line * P;
    Cx<R> o = cx((R)0, (R)0);
    int k2 = 0;
    bool has = true;
    if (j <= hN2) k2 = j;
    else if (j >= M2 - hN2) k2 = j - M2;
    else has = false;
    if (has) {
      const int sk2 = line ? -k2 : k2;     // line B at k2 is conj of row A at -k2
      const int src = ixn(sk2, N2);
      double T[3][2];
      basis(g, h0, k1, sk2, T);
      Cx<double> X[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int f = 2 * pk + s;
        X[s] = cx(0.0, 0.0);
        if (f < L * d) {
          const int lf = f / d, gam = f - (f / d) * d;
          // row gam of T by selection (constant indices keep T in registers)
          const double t0 = gam == 0 ? T[0][0] : (gam == 1 ? T[1][0] : T[2][0]);
          const double t1 = gam == 0 ? T[0][1] : (gam == 1 ? T[1][1] : T[2][1]);
          Cx<double> xv = rA[(lf * m) * N2 + src] * t0;
          if (m > 1) xv = xv + rA[(lf * m + 1) * N2 + src] * t1;
          if (line) xv.y = -xv.y;
          if (mode == FIRST_BOUNDS && self && k2 == 0) xv.x += U.E[lf][gam];
          X[s] = xv;
        }
      }
      o = cx((R)(X[0].x - X[1].y), (R)(X[0].y + X[1].x));
    }
    if constexpr (MAXB == 0) {
      // long lines: the row transform runs afterwards over HBM (k_unit_lines)
      const int i0 = line ? ixn(-h0, N0) : h0, i1 = line ? i1B : i1A;
      reinterpret_cast<Cx<R>*>(U.bufA)[(((size_t)i0 * N1 + i1) * M2 + j) * P + pk] = o;
    } else {
      buf[j * nl + l] = o;
    }
  }
  if constexpr (MAXB > 0) {
    __syncthreads();
    lds_fft<R, MAXB>(buf, nl, M2, g.pl[2], reinterpret_cast<const Cx<R>*>(g.tw[2]), true);

    Cx<R>* out = reinterpret_cast<Cx<R>*>(U.bufA);
    const int i0A = h0, i0B = ixn(-h0, N0);
    for (int t = tid; t < M2 * nl; t += kBlock) {
      const int j = t / nl, l = t - (t / nl) * nl;
      const int line = l / P, pk = l - line * P;
      const int i0 = line ? i0B : i0A, i1 = line ? i1B : i1A;
      out[(((size_t)i0 * N1 + i1) * M2 + j) * P + pk] = buf[j * nl + l];
    }
  }
}

// ============================================================== last pass
template <typename R, int MAXB>
__global__ __launch_bounds__(kBlock) void k_last(Geo g, const UnitDev* __restrict__ units, int mode, int jstep,
                                                 const int* __restrict__ iter_base) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_beta[kMaxLoads];
  __shared__ int s_act[kMaxLoads];
  __shared__ double s_red[kBlock / 64];
  const UnitDev& U = units[blockIdx.z];
  const int tid = threadIdx.x;
  const int N0 = g.N[0], N1 = g.N[1], N2 = g.N[2], M2 = g.M[2];
  const int L = g.L, m = g.m, P = g.P, d = g.d;
  int h0, k1;
  decode_pair(g, blockIdx.x, h0, k1);
  const bool self = (h0 == 0 && k1 == 0);
  const bool rowB = (h0 == 0 && k1 != 0);
  const int i1A = ixn(k1, N1), i1B = ixn(-k1, N1);
  const int it = iter_base ? (*iter_base + jstep) : 0;
  const int nl = (self ? 1 : 2) * P;
  Cx<R>* buf = reinterpret_cast<Cx<R>*>(smem);

  // ---- scalars: gamma_it from the first-pass partials, convergence, beta_it
  if (tid < kMaxLoads * 64) {
    const int w = tid >> 6, lane = tid & 63;
    if (w < L) {
      int act = 1;
      double beta = 0.0;
      if (mode == LAST_CG) {
        CgScal* sc = U.sc + w;
        act = (sc->status == 0);
        if (act) {
          const double gam = wave_sum_arr(U.part_g + (size_t)w * g.nbF, g.nbF);
          const bool bad = !(gam == gam) || gam > 1e300;
          const bool conv = stop_test(sc, blockIdx.x == 0 && lane == 0 ? sc : nullptr, it, gam);
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
  __syncthreads();
  int any = 0;
  for (int l = 0; l < L; ++l) any |= s_act[l];
  if (!any) return;  // uniform over the block

  // ---- load both lines and transform forward (long lines: transformed in HBM
  // beforehand by k_unit_lines, read in place)
  const Cx<R>* in = reinterpret_cast<const Cx<R>*>(U.bufA);
  const int i0A = h0, i0B = ixn(-h0, N0);
  if constexpr (MAXB > 0) {
    for (int t = tid; t < M2 * nl; t += kBlock) {
      const int j = t / nl, l = t - (t / nl) * nl;
      const int line = l / P, pk = l - line * P;
      const int i0 = line ? i0B : i0A, i1 = line ? i1B : i1A;
      buf[j * nl + l] = in[(((size_t)i0 * N1 + i1) * M2 + j) * P + pk];
    }
    __syncthreads();
    lds_fft<R, MAXB>(buf, nl, M2, g.pl[2], reinterpret_cast<const Cx<R>*>(g.tw[2]), false);
  }
  auto line_at = [&](int pos, int line, int pk) -> Cx<R> {
    if constexpr (MAXB > 0) {
      return buf[pos * nl + line * P + pk];
    } else {
      const int i0 = line ? i0B : i0A, i1 = line ? i1B : i1A;
      return in[(((size_t)i0 * N1 + i1) * M2 + pos) * P + pk];
    }
  };

  // ---- epilogue on the stored entries of row A (and of row B when it is stored)
  double dp0 = 0.0, dp1 = 0.0, dp2 = 0.0;
  const int nrows = rowB ? 2 : 1;
  const double wt = (h0 == 0) ? 1.0 : 2.0;
  const double sc_m = g.invM * 0.5;
  for (int t = tid; t < nrows * N2; t += kBlock) {
    const int row = t / N2, i2 = t - row * N2;
    const int k2 = fr(i2, N2);
    const int lineK = self ? 0 : row, lineM = self ? 0 : 1 - row;
    const int posK = padpos(i2, N2, M2), posM = padpos(ixn(-k2, N2), N2, M2);
    const int kk0 = row ? 0 : h0, kk1 = row ? -k1 : k1;
    const int i1 = row ? i1B : i1A;
    double T[3][2];
    basis(g, kk0, kk1, k2, T);
    for (int l = 0; l < L; ++l) {
      if (mode == LAST_CG && !s_act[l]) continue;
      Cx<double> wv[3] = {cx(0.0, 0.0), cx(0.0, 0.0), cx(0.0, 0.0)};
#pragma unroll
      for (int gam = 0; gam < 3; ++gam) {
        if (gam >= d) continue;
        const int f = l * d + gam, pk = f >> 1;
        const Cx<R> za = line_at(posK, lineK, pk);
        const Cx<R> zb = line_at(posM, lineM, pk);
        if ((f & 1) == 0)
          wv[gam] = cx(((double)za.x + (double)zb.x) * sc_m, ((double)za.y - (double)zb.y) * sc_m);
        else
          wv[gam] = cx(((double)za.y + (double)zb.y) * sc_m, -((double)za.x - (double)zb.x) * sc_m);
      }
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        if (c >= m) continue;
        Cx<double> w = cx(0.0, 0.0);
#pragma unroll
        for (int gam = 0; gam < 3; ++gam)
          if (gam < d) w = w + wv[gam] * T[gam][c];
        const size_t idx = ((size_t)(c * g.H0 + kk0) * N1 + i1) * N2 + i2;
        double e;
        if (mode == LAST_CG) {
          const Cx<double> rv = U.r[l][idx];
          const double b = s_beta[l];
          if (it == 0) {
            U.p[l][idx] = rv;
            U.s[l][idx] = w;
          } else {
            U.p[l][idx] = rv + U.p[l][idx] * b;
            U.s[l][idx] = w + U.s[l][idx] * b;
          }
          e = wt * (rv.x * w.x + rv.y * w.y);
        } else if (mode == LAST_RESID) {
          const Cx<double> rn = U.b[l][idx] - w;
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
    const double s = block_sum(l == 0 ? dp0 : (l == 1 ? dp1 : dp2), s_red);
    if (tid == 0) U.part_d[(size_t)l * g.nbL + blockIdx.x] = s;
  }
}

// Per-point coefficient product and FP64 quadrature with the dimension fixed
// at compile time and the load loops unrolled, so that the per-point arrays
// are indexed by constants and stay in registers.
template <typename R, int D>
__device__ __forceinline__ void point_coef(int nc, int L, const R* a, const R* u, R* w) {
#pragma unroll
  for (int l = 0; l < kMaxLoads; ++l)
    if (l < L) coef_mul<R>(D, nc, a, u + l * D, w + l * D);
}

template <typename R, int D>
__device__ __forceinline__ void point_quad(int nc, int L, const R* a, const R* u, double* acc) {
#pragma unroll
  for (int la = 0; la < kMaxLoads; ++la) {
    if (la >= L) continue;
    R w[D];
    coef_mul<R>(D, nc, a, u + la * D, w);
#pragma unroll
    for (int lb = 0; lb < kMaxLoads; ++lb) {
      if (lb >= L) continue;
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) s += (double)u[lb * D + c] * (double)w[c];
      acc[la * kMaxLoads + lb] += s;
    }
  }
}

// ============================================================== middle axis (3D)
template <typename R, int MAXB>
__global__ __launch_bounds__(kBlock) void k_mid(Geo g, const UnitDev* __restrict__ units, int flags) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<R>* buf = reinterpret_cast<Cx<R>*>(smem);
  const UnitDev& U = units[blockIdx.z];
  const int inverse = flags & 1;
  if (flags & MID_CG) {
    bool any = false;
    for (int l = 0; l < g.L; ++l) any |= (U.sc[l].status == 0);
    if (!any) return;
  }
  const int tid = threadIdx.x;
  const int N1 = g.N[1], M1 = g.M[1];
  const int inner = g.M[2] * g.P;
  const int tile = g.tileM;
  const int e0 = blockIdx.x * tile;
  const int te = min(tile, inner - e0);
  const int i0 = blockIdx.y;
  const Cx<R>* in = reinterpret_cast<const Cx<R>*>(inverse ? U.bufA : U.bufB);
  Cx<R>* out = reinterpret_cast<Cx<R>*>(inverse ? U.bufB : U.bufA);
  const int Lin = inverse ? N1 : M1, Lout = inverse ? M1 : N1;
  for (int t = tid; t < M1 * tile; t += kBlock) {
    const int j = t / tile, e = t - (t / tile) * tile;
    Cx<R> v = cx((R)0, (R)0);
    if (e < te) {
      int src = j;
      if (inverse) src = truncidx(j, N1, M1);
      if (src >= 0) v = in[((size_t)i0 * Lin + src) * inner + e0 + e];
    }
    buf[j * tile + e] = v;
  }
  __syncthreads();
  lds_fft<R, MAXB>(buf, tile, M1, g.pl[1], reinterpret_cast<const Cx<R>*>(g.tw[1]), inverse != 0);
  for (int t = tid; t < Lout * tile; t += kBlock) {
    const int j = t / tile, e = t - (t / tile) * tile;
    if (e < te) {
      const int pos = inverse ? j : padpos(j, N1, M1);
      out[((size_t)i0 * Lout + j) * inner + e0 + e] = buf[pos * tile + e];
    }
  }
}

// ============================================================== axis 0 + coefficient
template <typename R, int MAXB>
__global__ __launch_bounds__(kBlock) void k_apply(Geo g, const UnitDev* __restrict__ units, int mode) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_red[kBlock / 64];
  Cx<R>* buf = reinterpret_cast<Cx<R>*>(smem);
  const UnitDev& U = units[blockIdx.z];
  const int tid = threadIdx.x;
  const int N0 = g.N[0], M0 = g.M[0], P = g.P, d = g.d, L = g.L, nc = g.nc;
  const int npts = g.M[1] * g.M[2];
  const size_t Mtot = (size_t)M0 * npts;
  const int tileA = g.tileA;
  // XCD-aware tile order: workgroups go round-robin to the 8 XCDs, so XCD x (blocks x, x + 8, ...)
  // takes the contiguous tiles [x nb8, (x + 1) nb8) and its L2 serves the neighbouring tiles' lines
  const int nb8 = (g.nbA + 7) / 8;
  const int tb = (int)(blockIdx.x % 8) * nb8 + (int)(blockIdx.x / 8);
  if (tb >= g.nbA) return;  // uniform over the block
  const int p0 = tb * tileA;
  const int tp = min(tileA, npts - p0);
  const int nl = tileA * P;
  Cx<R>* data = reinterpret_cast<Cx<R>*>(g.N[1] > 1 ? U.bufB : U.bufA);
  const R* coef = reinterpret_cast<const R*>(U.coef);
  if (mode == APPLY_COEF_CG) {
    bool any = false;
    for (int l = 0; l < L; ++l) any |= (U.sc[l].status == 0);
    if (!any) return;
    mode = APPLY_COEF;
  }

  if (mode == APPLY_FWD) {
    // real fields on the full doubled grid, two per complex pack
    for (int t = tid; t < M0 * nl; t += kBlock) {
      const int j = t / nl, l = t - (t / nl) * nl;
      const int pt = l / P, pk = l - pt * P;
      Cx<R> v = cx((R)0, (R)0);
      if (pt < tp) {
        const int f0 = 2 * pk, f1 = 2 * pk + 1;
        const size_t gi = (size_t)j * npts + p0 + pt;
        if (f0 < L * d) v.x = (R)U.grid[f0 * Mtot + gi];
        if (f1 < L * d) v.y = (R)U.grid[f1 * Mtot + gi];
      }
      buf[j * nl + l] = v;
    }
    __syncthreads();
  } else {
    for (int t = tid; t < M0 * nl; t += kBlock) {
      const int j = t / nl, l = t - (t / nl) * nl;
      const int i0 = truncidx(j, N0, M0);
      Cx<R> v = cx((R)0, (R)0);
      if (i0 >= 0 && l < tp * P) v = data[((size_t)i0 * npts + p0) * P + l];
      buf[j * nl + l] = v;
    }
    __syncthreads();
    lds_fft<R, MAXB>(buf, nl, M0, g.pl[0], reinterpret_cast<const Cx<R>*>(g.tw[0]), true);
  }
  if (mode == APPLY_GRID) {
    for (int t = tid; t < M0 * tileA; t += kBlock) {
      const int j = t / tileA, pt = t - (t / tileA) * tileA;
      if (pt >= tp) continue;
      const size_t gi = (size_t)j * npts + p0 + pt;
      for (int pk = 0; pk < P; ++pk) {
        const Cx<R> z = buf[j * nl + pt * P + pk];
        if (2 * pk < L * d) U.grid[(2 * pk) * Mtot + gi] = (float)z.x;
        if (2 * pk + 1 < L * d) U.grid[(2 * pk + 1) * Mtot + gi] = (float)z.y;
      }
    }
    return;
  }

  if (mode == APPLY_COEF || mode == APPLY_FWD) {
    for (int t = tid; t < M0 * tileA && mode == APPLY_COEF; t += kBlock) {
      const int j = t / tileA, pt = t - (t / tileA) * tileA;
      if (pt >= tp) continue;
      const size_t ci = (size_t)j * npts + p0 + pt;
      R a[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) a[c] = c < nc ? coef[c * Mtot + ci] : (R)0;
      R u[2 * kMaxPacks], w[2 * kMaxPacks];
#pragma unroll
      for (int pk = 0; pk < kMaxPacks; ++pk) {
        const Cx<R> z = pk < P ? buf[j * nl + pt * P + pk] : cx((R)0, (R)0);
        u[2 * pk] = z.x;
        u[2 * pk + 1] = z.y;
        w[2 * pk] = w[2 * pk + 1] = (R)0;
      }
      if (d == 2)
        point_coef<R, 2>(nc, L, a, u, w);
      else
        point_coef<R, 3>(nc, L, a, u, w);
#pragma unroll
      for (int pk = 0; pk < kMaxPacks; ++pk)
        if (pk < P) buf[j * nl + pt * P + pk] = cx(w[2 * pk], w[2 * pk + 1]);
    }
    __syncthreads();
    lds_fft<R, MAXB>(buf, nl, M0, g.pl[0], reinterpret_cast<const Cx<R>*>(g.tw[0]), false);
    for (int t = tid; t < N0 * nl; t += kBlock) {
      const int i0 = t / nl, l = t - (t / nl) * nl;
      if (l < tp * P) data[((size_t)i0 * npts + p0) * P + l] = buf[padpos(i0, N0, M0) * nl + l];
    }
  } else {
    // FP64 quadrature of the bilinear forms: sum_x v_b(x) . A(x) v_a(x)
    double acc[kMaxLoads * kMaxLoads];
#pragma unroll
    for (int i = 0; i < kMaxLoads * kMaxLoads; ++i) acc[i] = 0.0;
    for (int t = tid; t < M0 * tileA; t += kBlock) {
      const int j = t / tileA, pt = t - (t / tileA) * tileA;
      if (pt >= tp) continue;
      const size_t ci = (size_t)j * npts + p0 + pt;
      R a[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) a[c] = c < nc ? coef[c * Mtot + ci] : (R)0;
      R u[2 * kMaxPacks];
#pragma unroll
      for (int pk = 0; pk < kMaxPacks; ++pk) {
        const Cx<R> z = pk < P ? buf[j * nl + pt * P + pk] : cx((R)0, (R)0);
        u[2 * pk] = z.x;
        u[2 * pk + 1] = z.y;
      }
      if (d == 2)
        point_quad<R, 2>(nc, L, a, u, acc);
      else
        point_quad<R, 3>(nc, L, a, u, acc);
    }
#pragma unroll
    for (int i = 0; i < kMaxLoads * kMaxLoads; ++i) {
      if (i / kMaxLoads >= L || i % kMaxLoads >= L) continue;  // uniform over the block
      const double s = block_sum(acc[i], s_red);
      if (tid == 0) U.part_q[(size_t)tb * 9 + i] = s;
    }
  }
}

// Streaming copy of n 16-byte words (the bandwidth probe): each block moves
// contiguous chunks of 4 kBlock words, four loads in flight per thread before
// the stores; the tail word by word.
__global__ void k_stream_copy(const float4* __restrict__ src, float4* __restrict__ dst, size_t n) {
  constexpr int U = 4;
  const size_t chunk = (size_t)U * blockDim.x;
  const size_t nfull = n / chunk;
  for (size_t c = blockIdx.x; c < nfull; c += gridDim.x) {
    const size_t base = c * chunk + threadIdx.x;
    float4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = src[base + (size_t)u * blockDim.x];
#pragma unroll
    for (int u = 0; u < U; ++u) dst[base + (size_t)u * blockDim.x] = v[u];
  }
  for (size_t t = nfull * chunk + blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.x * blockDim.x)
    dst[t] = src[t];
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 16;
  size_t nb = (n + 4 * kBlock - 1) / (4 * kBlock);
  if (nb > 256 * 16) nb = 256 * 16;   // 16 blocks per CU
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)nb), dim3(kBlock), 0, st, reinterpret_cast<const float4*>(src),
                     reinterpret_cast<float4*>(dst), n);
  return hipGetLastError();
}

// out = sum_a w_a x_a over n complex entries (d <= 3 fields).
__global__ void k_combine(FieldTriple x, int d, double w0, double w1, double w2, Cx<double>* __restrict__ out,
                          size_t n) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
    Cx<double> s = x.p[0][t] * w0;
    if (d > 1) s = s + x.p[1][t] * w1;
    if (d > 2) s = s + x.p[2][t] * w2;
    out[t] = s;
  }
}

// ============================================================== setup FFT
template <typename R, int MAXB>
__global__ __launch_bounds__(kBlock) void k_line_fft(Cx<R>* data, int outer, int Lm, int inner, int tile, Plan pl,
                                                     const Cx<R>* tw, int inverse) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<R>* buf = reinterpret_cast<Cx<R>*>(smem);
  const int tid = threadIdx.x;
  const int e0 = blockIdx.x * tile;
  const int te = min(tile, inner - e0);
  const size_t base = (size_t)blockIdx.y * Lm * inner;
  for (int t = tid; t < Lm * tile; t += kBlock) {
    const int j = t / tile, e = t - (t / tile) * tile;
    buf[j * tile + e] = (e < te) ? data[base + (size_t)j * inner + e0 + e] : cx((R)0, (R)0);
  }
  __syncthreads();
  lds_fft<R, MAXB>(buf, tile, Lm, pl, tw, inverse != 0);
  for (int t = tid; t < Lm * tile; t += kBlock) {
    const int j = t / tile, e = t - (t / tile) * tile;
    if (e < te) data[base + (size_t)j * inner + e0 + e] = buf[j * tile + e];
  }
}

// Row transform (length M2) of every row of each unit's line buffer
// [N0][N1][M2][P], in place: blocks of `tile` packs of one row; grid.x = rows *
// ceil(P / tile), grid.z = unit.  Used by the row passes when their lines do not
// fit in LDS.
template <typename R, int MAXB>
__global__ __launch_bounds__(kBlock) void k_unit_lines(Geo g, const UnitDev* __restrict__ units, int tile, int nbi,
                                                       int inverse) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<R>* buf = reinterpret_cast<Cx<R>*>(smem);
  const UnitDev& U = units[blockIdx.z];
  Cx<R>* data = reinterpret_cast<Cx<R>*>(U.bufA);
  const int M2 = g.M[2], P = g.P, tid = threadIdx.x;
  const int row = blockIdx.x / nbi, e0 = (blockIdx.x - row * nbi) * tile;
  const int te = min(tile, P - e0);
  const size_t base = (size_t)row * M2 * P;
  for (int t = tid; t < M2 * tile; t += kBlock) {
    const int j = t / tile, e = t - (t / tile) * tile;
    buf[j * tile + e] = (e < te) ? data[base + (size_t)j * P + e0 + e] : cx((R)0, (R)0);
  }
  __syncthreads();
  lds_fft<R, MAXB>(buf, tile, M2, g.pl[2], reinterpret_cast<const Cx<R>*>(g.tw[2]), inverse != 0);
  for (int t = tid; t < M2 * tile; t += kBlock) {
    const int j = t / tile, e = t - (t / tile) * tile;
    if (e < te) data[base + (size_t)j * P + e0 + e] = buf[j * tile + e];
  }
}

// ============================================================== small kernels
// Right-hand side b(k) = -T(k)^T A_hat(k) E on the stored half of Z_N
// (the Z_N part of A_M E is exactly A_hat(k) E since E is constant).
__global__ void k_rhs(Geo g, const UnitDev* __restrict__ units) {
  const UnitDev& U = units[blockIdx.z];
  const int d = g.d, nc = g.nc;
  const int S = g.S;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < S; t += gridDim.x * blockDim.x) {
    const int i2 = t % g.N[2], i1 = (t / g.N[2]) % g.N[1], h0 = t / (g.N[2] * g.N[1]);
    const int k1 = fr(i1, g.N[1]), k2 = fr(i2, g.N[2]);
    double T[3][2];
    basis(g, h0, k1, k2, T);
    // loops unrolled with guards: constant indices keep a, v and T in registers
    Cx<double> a[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) a[c] = c < nc ? U.ahat[(size_t)c * S + t] : cx(0.0, 0.0);
    for (int l = 0; l < g.L; ++l) {
      Cx<double> v[3] = {cx(0.0, 0.0), cx(0.0, 0.0), cx(0.0, 0.0)};
#pragma unroll
      for (int gam = 0; gam < 3; ++gam) {
        if (gam >= d) continue;
        Cx<double> s = cx(0.0, 0.0);
#pragma unroll
        for (int dl = 0; dl < 3; ++dl) {
          if (dl >= d) continue;
          Cx<double> A;
          if (nc == 1) A = (gam == dl) ? a[0] : cx(0.0, 0.0);
          else if (d == 2) A = (gam == dl) ? a[gam] : a[2];
          else {
            if (gam == dl) A = a[gam];
            else {
              const int lo = min(gam, dl), hi = max(gam, dl);
              A = (lo == 0 && hi == 1) ? a[3] : ((lo == 0 && hi == 2) ? a[4] : a[5]);
            }
          }
          s = s + A * U.E[l][dl];
        }
        v[gam] = s;
      }
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        if (c >= g.m) continue;
        Cx<double> s = cx(0.0, 0.0);
#pragma unroll
        for (int gam = 0; gam < 3; ++gam)
          if (gam < d) s = s + v[gam] * T[gam][c];
        U.b[l][(size_t)c * S + t] = cx(-s.x, -s.y);
      }
    }
  }
}

// x = 0 or untouched (given x0), r = b (x0 = 0).
__global__ void k_start(Geo g, const UnitDev* __restrict__ units, int have_x0) {
  const UnitDev& U = units[blockIdx.z];
  const size_t n = (size_t)g.m * g.S;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
    for (int l = 0; l < g.L; ++l) {
      if (!have_x0) {
        U.x[l][t] = cx(0.0, 0.0);
        U.r[l][t] = U.b[l][t];
      }
      U.p[l][t] = cx(0.0, 0.0);
      U.s[l][t] = cx(0.0, 0.0);
    }
  }
}

// Energy of a given start field x0 relative to the zero field.  With
// a(E + x, E + x) = e0 - 2 <x, b> + <x, C x> (b = -G A E, so that a(E, x) =
// -<x, b>), the energy is e0 - <x, b + r> for r = b - C x.  The decrease
// <x0, b + r0> is stored as the starting sum of the decrements, so energy0 -
// esum is the energy of the iterate from the start on.  One block per unit,
// loads in turn, sums in a fixed order.
__global__ void k_start_energy(Geo g, const UnitDev* __restrict__ units) {
  __shared__ double s_red[kBlock / 64];
  const UnitDev& U = units[blockIdx.x];
  const size_t n = (size_t)g.m * g.S;
  const int plane = g.N[1] * g.N[2];
  for (int l = 0; l < g.L; ++l) {
    double acc = 0.0;
    for (size_t t = threadIdx.x; t < n; t += kBlock) {
      const int h0 = (int)((t / plane) % g.H0);
      const Cx<double> xv = U.x[l][t], bv = U.b[l][t], rv = U.r[l][t];
      acc += ((h0 == 0) ? 1.0 : 2.0) * (xv.x * (bv.x + rv.x) + xv.y * (bv.y + rv.y));
    }
    const double s = block_sum(acc, s_red);
    if (threadIdx.x == 0) {
      U.sc[l].esum = s;
      U.sc[l].snap_e[0] = U.sc[l].snap_e[1] = U.sc[l].energy0 - s;
    }
  }
}

// Smallest eigenvalue of a symmetric coefficient matrix (component order xx,
// yy(, zz), xy(, xz, yz)), lowered by a small multiple of its scale so that
// rounding keeps it below the exact value.  3x3: trigonometric solution of
// the characteristic cubic (Smith 1961), whose angle loses up to half the
// digits near a double eigenvalue, hence the larger margin there.
__device__ double sym_min_eig(const double* c, int nc, int d) {
  if (nc == 1) return c[0] - 1e-14 * fabs(c[0]);
  if (d == 2) {
    const double m = 0.5 * (c[0] + c[1]), h = 0.5 * (c[0] - c[1]);
    const double r = sqrt(h * h + c[2] * c[2]);
    return m - r - 1e-12 * (fabs(m) + r);
  }
  const double q = (c[0] + c[1] + c[2]) / 3.0;
  const double a = c[0] - q, b = c[1] - q, e = c[2] - q;
  const double off = c[3] * c[3] + c[4] * c[4] + c[5] * c[5];
  const double p = sqrt((a * a + b * b + e * e + 2.0 * off) / 6.0);
  if (!(p > 0.0)) return q - 1e-12 * fabs(q);
  const double ip = 1.0 / p;
  const double B00 = a * ip, B11 = b * ip, B22 = e * ip, B01 = c[3] * ip, B02 = c[4] * ip, B12 = c[5] * ip;
  double r = 0.5 * (B00 * (B11 * B22 - B12 * B12) - B01 * (B01 * B22 - B12 * B02) + B02 * (B01 * B12 - B11 * B02));
  r = fmin(1.0, fmax(-1.0, r));
  const double ang = acos(r) / 3.0;
  return q + 2.0 * p * cos(ang + 2.0943951023931957) - 1e-6 * (fabs(q) + 3.0 * p);
}

template <typename R>
__global__ void k_coef_min_eig(Geo g, const UnitDev* __restrict__ units) {
  __shared__ double s_min[kBlock / 64];
  const UnitDev& U = units[blockIdx.z];
  const R* __restrict__ coef = static_cast<const R*>(U.coef);
  const size_t npts = (size_t)g.M[0] * g.M[1] * g.M[2];
  double mn = INFINITY;
  for (size_t t = blockIdx.x * (size_t)kBlock + threadIdx.x; t < npts; t += (size_t)gridDim.x * kBlock) {
    double c[6];
    for (int k = 0; k < g.nc; ++k) c[k] = (double)coef[(size_t)k * npts + t];
    mn = fmin(mn, sym_min_eig(c, g.nc, g.d));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mn = fmin(mn, __shfl_down(mn, off, 64));
  if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = mn;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = s_min[0];
    for (int i = 1; i < kBlock / 64; ++i) r = fmin(r, s_min[i]);
    U.part_q[blockIdx.x] = r;
  }
}

__global__ void k_init_scal(Geo g, const UnitDev* __restrict__ units, int nunits, int* iter_base, int chunk,
                            double tol, int maxit, int stop, double etol, int mu_parts, double mu_user) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u == 0 && iter_base) *iter_base = 0;
  if (u >= nunits) return;
  const UnitDev& U = units[u];
  for (int l = 0; l < g.L; ++l) {
    CgScal* sc = U.sc + l;
    double e2 = 0.0;
    for (int c = 0; c < g.d; ++c) e2 += U.E[l][c] * U.E[l][c];
    sc->normE = sqrt(e2);
    sc->status = 0;
    sc->iters = 0;
    sc->gamma[0] = sc->gamma[1] = 0.0;
    sc->beta[0] = sc->beta[1] = 0.0;
    sc->alpha[0] = sc->alpha[1] = 1.0;
    sc->gamma0 = sc->gamma_last = 0.0;
    sc->tol = tol;
    sc->maxit = maxit;
    sc->stop = stop;
    sc->etol = etol;
    // E^T <C> E from the zero frequency of the coefficient series (component order
    // xx, yy(, zz), xy(, xz, yz) for symmetric matrices)
    double c0[6];
    for (int c = 0; c < g.nc; ++c) c0[c] = U.ahat[(size_t)c * g.S].x;
    const double* E = U.E[l];
    double en = 0.0;
    if (g.nc == 1) {
      en = c0[0] * e2;
    } else if (g.d == 2) {
      en = c0[0] * E[0] * E[0] + c0[1] * E[1] * E[1] + 2.0 * c0[2] * E[0] * E[1];
    } else {
      en = c0[0] * E[0] * E[0] + c0[1] * E[1] * E[1] + c0[2] * E[2] * E[2] +
           2.0 * (c0[3] * E[0] * E[1] + c0[4] * E[0] * E[2] + c0[5] * E[1] * E[2]);
    }
    sc->energy0 = en;
    sc->esum = 0.0;
    for (int j = 0; j < 4; ++j) sc->edec[j] = 0.0;
    // both the caller's bound and the doubled-grid minimum bound the spectrum from below
    double mu = mu_user;
    if (mu_parts > 0) {
      double gm = INFINITY;
      for (int q = 0; q < mu_parts; ++q) gm = fmin(gm, U.part_q[q]);
      mu = fmax(mu, gm);
    }
    sc->mu = (mu > 0.0) ? mu : 0.0;
    sc->phi[0] = sc->phi[1] = (mu > 0.0) ? 1.0 / mu : INFINITY;
    // gap rule: the state before the first chunk is the start (infinite bound)
    sc->partner = U.partner_sc ? U.partner_sc + l : nullptr;
    sc->snap_e[0] = sc->snap_e[1] = en;
    sc->snap_r[0] = sc->snap_r[1] = INFINITY;
    sc->rem = INFINITY;
    sc->chunk = chunk;
    sc->side = g.dual;
  }
}

// Symmetrise a field on the k0 = 0 plane so that it is the spectrum of a real
// field: x_hat(k) <- (x_hat(k) + conj(x_hat(-k))) / 2, and zero the mean.
__device__ __forceinline__ void symmetrize_field(const Geo& g, const Cx<double>* __restrict__ src,
                                                 Cx<double>* __restrict__ dst, int m) {
  const int S = g.S;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < S; t += gridDim.x * blockDim.x) {
    const int i2 = t % g.N[2], i1 = (t / g.N[2]) % g.N[1], h0 = t / (g.N[2] * g.N[1]);
    if (h0 > 0) {
      for (int c = 0; c < m; ++c) dst[(size_t)c * S + t] = src[(size_t)c * S + t];
      continue;
    }
    const int k1 = fr(i1, g.N[1]), k2 = fr(i2, g.N[2]);
    const int tm = (ixn(-k1, g.N[1])) * g.N[2] + ixn(-k2, g.N[2]);
    double Tk[3][2], Tm[3][2];
    basis(g, 0, k1, k2, Tk);
    basis(g, 0, -k1, -k2, Tm);
    Cx<double> xs[3];
    for (int gam = 0; gam < g.d; ++gam) {
      Cx<double> a = cx(0.0, 0.0), b = cx(0.0, 0.0);
      for (int c = 0; c < m; ++c) {
        a = a + src[(size_t)c * S + t] * Tk[gam][c];
        b = b + src[(size_t)c * S + tm] * Tm[gam][c];
      }
      xs[gam] = cx(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    }
    for (int c = 0; c < m; ++c) {
      Cx<double> s = cx(0.0, 0.0);
      for (int gam = 0; gam < g.d; ++gam) s = s + xs[gam] * Tk[gam][c];
      dst[(size_t)c * S + t] = s;
    }
  }
}
__global__ void k_symmetrize(Geo g, const Cx<double>* __restrict__ src, Cx<double>* __restrict__ dst, int m) {
  symmetrize_field(g, src, dst, m);
}
// One field per grid row: jobs[blockIdx.y].
__global__ void k_symmetrize_jobs(Geo g, const SymJob* __restrict__ jobs, int m) {
  const SymJob j = jobs[blockIdx.y];
  symmetrize_field(g, j.src, j.dst, m);
}

// After a chunk of iterations: advance the iteration base, count active loads
// and record every load's energy and Gauss-Radau bound at the chunk's last
// iterate (read by the partner solve under the gap rule during the next chunk).
__global__ void k_advance(Geo g, const UnitDev* __restrict__ units, int nunits, int* iter_base, int step,
                          int* active_out) {
  __shared__ int cnt[kBlock];
  int c = 0;
  const int slot = (*iter_base / step) & 1;
  for (int u = threadIdx.x; u < nunits; u += blockDim.x)
    for (int l = 0; l < g.L; ++l) {
      CgScal* sc = units[u].sc + l;
      c += (sc->status == 0);
      sc->snap_e[slot] = sc->energy0 - sc->esum;
      sc->snap_r[slot] = sc->rem;
    }
  cnt[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int i = 0; i < (int)blockDim.x; ++i) s += cnt[i];
    *active_out = s;
    *iter_base += step;
  }
}

// Twiddle tables exp(-2 pi i t / M), t < M, from sincospi in FP64.
__global__ void k_twiddles(Cx<double>* t64, Cx<float>* t32, int M) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < M; t += gridDim.x * blockDim.x) {
    double s, c;
    sincospi(-2.0 * (double)t / (double)M, &s, &c);
    t64[t] = cx(c, s);
    if (t32) t32[t] = cx((float)c, (float)s);
  }
}

__global__ void k_coef_real(const Cx<double>* __restrict__ full, double* __restrict__ c64, float* __restrict__ c32,
                            long n) {
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const double v = full[t].x;
    c64[t] = v;
    if (c32) c32[t] = (float)v;
  }
}

// Z_N part of a Z_M array (stored half), component-major.
__global__ void k_extract_half(Geo g, const Cx<double>* __restrict__ full, Cx<double>* __restrict__ half, int nc) {
  const int S = g.S;
  const size_t Mt = (size_t)g.M[0] * g.M[1] * g.M[2];
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < S * nc; t += gridDim.x * blockDim.x) {
    const int c = t / S, s = t - c * S;
    const int i2 = s % g.N[2], i1 = (s / g.N[2]) % g.N[1], h0 = s / (g.N[2] * g.N[1]);
    const int j0 = h0, j1 = padpos(i1, g.N[1], g.M[1]), j2 = padpos(i2, g.N[2], g.M[2]);
    half[t] = full[c * Mt + ((size_t)j0 * g.M[1] + j1) * g.M[2] + j2];
  }
}

// The same for the A and B data of every cell of a batch: grid (blocks, 2, cell).
__global__ void k_extract_half_jobs(Geo g, const CoefJob* __restrict__ jobs, int nc) {
  const CoefJob& J = jobs[blockIdx.z];
  const Cx<double>* full = blockIdx.y ? J.B : J.A;
  Cx<double>* half = J.half[blockIdx.y];
  const int S = g.S;
  const size_t Mt = (size_t)g.M[0] * g.M[1] * g.M[2];
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < S * nc; t += gridDim.x * blockDim.x) {
    const int c = t / S, s = t - c * S;
    const int i2 = s % g.N[2], i1 = (s / g.N[2]) % g.N[1], h0 = s / (g.N[2] * g.N[1]);
    const int j0 = h0, j1 = padpos(i1, g.N[1], g.M[1]), j2 = padpos(i2, g.N[2], g.M[2]);
    half[t] = full[c * Mt + ((size_t)j0 * g.M[1] + j1) * g.M[2] + j2];
  }
}

struct InclDev {
  int kind;         // 0 box, 1 ball
  double c[3];      // centre (internal axes)
  double h[3];      // box sides (internal axes) or radius in h[0]
  double A[6];      // coefficient difference in nc components
};

// A_hat(n) = A0 delta_n0 + sum_j A_j f_hat_j(n) exp(-2 pi i sum n_a x_a / Y_a) on Z_M
// (eq. A_with_inclusions, Remark inclusion; ball: textbook transform of a ball).
__global__ void k_coef_incl(int d, int M0, int M1, int M2, double iY0, double iY1, double iY2, int nc,
                            const double* __restrict__ A0c, int n_incl, const InclDev* __restrict__ inc,
                            Cx<double>* __restrict__ out) {
  const size_t Mt = (size_t)M0 * M1 * M2;
  const double iY[3] = {iY0, iY1, iY2};
  const double vol_inv = iY0 * iY1 * iY2;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < Mt; t += (size_t)gridDim.x * blockDim.x) {
    const int j2 = t % M2, j1 = (t / M2) % M1, j0 = t / ((size_t)M1 * M2);
    const int n[3] = {fr(j0, M0), fr(j1, M1), fr(j2, M2)};
    double acc_re[6] = {0, 0, 0, 0, 0, 0}, acc_im[6] = {0, 0, 0, 0, 0, 0};
    if (n[0] == 0 && n[1] == 0 && n[2] == 0)
      for (int c = 0; c < nc; ++c) acc_re[c] = A0c[c];
    for (int j = 0; j < n_incl; ++j) {
      const InclDev& I = inc[j];
      double f;
      if (I.kind == 0) {
        f = 1.0;
        for (int a = 0; a < 3; ++a) {
          const double hy = I.h[a] * iY[a];
          const double x = hy * n[a];
          f *= hy * (x == 0.0 ? 1.0 : sinpi(x) / (M_PI * x));
        }
      } else {
        double xi2 = 0.0;
        for (int a = 0; a < 3; ++a) xi2 += (n[a] * iY[a]) * (n[a] * iY[a]);
        const double kap = 2.0 * M_PI * sqrt(xi2);
        const double R = I.h[0];
        const double tt = kap * R;
        if (tt < 1e-2)
          f = (4.0 / 3.0) * M_PI * R * R * R * (1.0 - tt * tt / 10.0 + tt * tt * tt * tt / 280.0);
        else
          f = 4.0 * M_PI * (sin(tt) - tt * cos(tt)) / (kap * kap * kap);
        f *= vol_inv;
      }
      double ph = 0.0;
      for (int a = 0; a < 3; ++a) ph += n[a] * I.c[a] * iY[a];
      double sn, cs;
      sincospi(-2.0 * ph, &sn, &cs);
      for (int c = 0; c < nc; ++c) {
        acc_re[c] += I.A[c] * f * cs;
        acc_im[c] += I.A[c] * f * sn;
      }
    }
    for (int c = 0; c < nc; ++c) out[c * Mt + t] = cx(acc_re[c], acc_im[c]);
  }
}

// Pixel images: A_hat(n) = prod_a [sinc(n_a/P_a)/P_a exp(-2 pi i n_a (1/(2P_a) - 1/2))] * D(n mod P),
// D the unnormalised forward DFT of the image.
__global__ void k_pixel_factor(int M0, int M1, int M2, int P0, int P1, int P2, int nc, const Cx<double>* __restrict__ D,
                               Cx<double>* __restrict__ out) {
  const size_t Mt = (size_t)M0 * M1 * M2, Pt = (size_t)P0 * P1 * P2;
  const int Mv[3] = {M0, M1, M2}, Pv[3] = {P0, P1, P2};
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < Mt; t += (size_t)gridDim.x * blockDim.x) {
    const int j[3] = {(int)(t / ((size_t)M1 * M2)), (int)((t / M2) % M1), (int)(t % M2)};
    Cx<double> fac = cx(1.0, 0.0);
    size_t di = 0;
    for (int a = 0; a < 3; ++a) {
      const int n = fr(j[a], Mv[a]);
      const double x = (double)n / Pv[a];
      const double sc = (n == 0 ? 1.0 : sinpi(x) / (M_PI * x)) / Pv[a];
      double sn, cs;
      sincospi(-2.0 * n * (0.5 / Pv[a] - 0.5), &sn, &cs);
      fac = cmul(fac, cx(sc * cs, sc * sn));
      int nm = n % Pv[a];
      if (nm < 0) nm += Pv[a];
      di = di * Pv[a] + nm;
    }
    for (int c = 0; c < nc; ++c) out[c * Mt + t] = cmul(fac, D[c * Pt + di]);
  }
}

// ============================================================== launchers
static int pow2_at_least(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

static int max_butterflies(const Plan& pl, int M, int nl) {
  int mx = 0;
  for (int s = 0; s < pl.n; ++s) mx = max(mx, (M / pl.r[s]) * nl);
  return mx;
}

#define HOM_LAUNCH1(K, GRID, LDS, ...)                                                                   \
  do {                                                                                                 \
    if (g_ext_timing.on)                                                                               \
      hipExtLaunchKernelGGL(K, GRID, dim3(kBlock), LDS, st, g_ext_timing.start, g_ext_timing.stop, 0,  \
                            __VA_ARGS__);                                                             \
    else                                                                                               \
      hipLaunchKernelGGL(K, GRID, dim3(kBlock), LDS, st, __VA_ARGS__);                                 \
  } while (0)

#define HOM_DISPATCH(KERN, MAXB_NEEDED, LDS, GRID, ...)                                               \
  do {                                                                                               \
    const int mb_ = pow2_at_least((MAXB_NEEDED + kBlock - 1) / kBlock);                              \
    const void* fn_ = nullptr;                                                                       \
    switch (mb_) {                                                                                   \
      case 1: fn_ = (const void*)KERN<R, 1>; break;                                                  \
      case 2: fn_ = (const void*)KERN<R, 2>; break;                                                  \
      case 4: fn_ = (const void*)KERN<R, 4>; break;                                                  \
      case 8: fn_ = (const void*)KERN<R, 8>; break;                                                  \
      case 16: fn_ = (const void*)KERN<R, 16>; break;                                                \
      default: return hipErrorInvalidValue;                                                          \
    }                                                                                                \
    if ((LDS) > kLdsMax) return hipErrorInvalidValue;                                                \
    hipError_t e_ = hipFuncSetAttribute(fn_, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(LDS)); \
    if (e_ != hipSuccess) return e_;                                                                 \
    switch (mb_) {                                                                                   \
      case 1: HOM_LAUNCH1((KERN<R, 1>), GRID, LDS, __VA_ARGS__); break;                              \
      case 2: HOM_LAUNCH1((KERN<R, 2>), GRID, LDS, __VA_ARGS__); break;                              \
      case 4: HOM_LAUNCH1((KERN<R, 4>), GRID, LDS, __VA_ARGS__); break;                              \
      case 8: HOM_LAUNCH1((KERN<R, 8>), GRID, LDS, __VA_ARGS__); break;                              \
      case 16: HOM_LAUNCH1((KERN<R, 16>), GRID, LDS, __VA_ARGS__); break;                            \
    }                                                                                                \
    return hipGetLastError();                                                                        \
  } while (0)

// The fused row passes hold both lines of a row pair (2P complex lines of M2)
// in LDS; beyond the LDS size or the butterfly registers they run as a gather
// (or epilogue) kernel plus a separate row transform over HBM.
template <typename R>
static bool rows_fit(const Geo& g, size_t extra) {
  if (std::getenv("HOM_LONG_ROWS")) return false;  // the split form at any size (tests)
  const int nl = 2 * g.P;
  const size_t lds = extra + (size_t)g.M[2] * nl * sizeof(Cx<R>);
  return lds <= kLdsMax && (max_butterflies(g.pl[2], g.M[2], nl) + kBlock - 1) / kBlock <= 16;
}

template <typename R>
static hipError_t launch_unit_lines(const Geo& g, const UnitDev* units, int nunits, int inverse, hipStream_t st) {
  int tile = 1;
  while (tile * 2 <= g.P && (size_t)g.M[2] * tile * 2 * sizeof(Cx<R>) <= 48 * 1024) tile *= 2;
  const int nbi = (g.P + tile - 1) / tile;
  const long rows = (long)g.N[0] * g.N[1];
  if (rows * nbi > 0x7fffffffL) return hipErrorInvalidValue;
  const size_t lds = (size_t)g.M[2] * tile * sizeof(Cx<R>);
  HOM_DISPATCH(k_unit_lines, max_butterflies(g.pl[2], g.M[2], tile), lds, dim3((unsigned)(rows * nbi), 1, nunits), g,
               units, tile, nbi, inverse);
}

template <typename R>
static hipError_t launch_first_long(const Geo& g, const UnitDev* units, int nunits, int mode, int jstep,
                                    const int* iter_base, size_t lds, hipStream_t st) {
  if (lds > kLdsMax) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void*)k_first<R, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  HOM_LAUNCH1((k_first<R, 0>), dim3(g.Q, 1, nunits), lds, g, units, mode, jstep, iter_base);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_unit_lines<R>(g, units, nunits, 1, st);
}

template <typename R>
static hipError_t launch_last_long(const Geo& g, const UnitDev* units, int nunits, int mode, int jstep,
                                   const int* iter_base, hipStream_t st) {
  hipError_t e = launch_unit_lines<R>(g, units, nunits, 0, st);
  if (e != hipSuccess) return e;
  HOM_LAUNCH1((k_last<R, 0>), dim3(g.Q, 1, nunits), 0, g, units, mode, jstep, iter_base);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_first(const Geo& g, const UnitDev* units, int nunits, int mode, int jstep, const int* iter_base,
                        hipStream_t st) {
  if constexpr (sizeof(R) == 4) {
    hipError_t e;
    if (fast_row(true, g, units, nunits, mode, jstep, iter_base, st, &e)) return e;
  }
  const int nl = 2 * g.P;
  const size_t staged = align16((size_t)g.L * g.m * g.N[2] * sizeof(Cx<double>));
  if (!rows_fit<R>(g, staged)) return launch_first_long<R>(g, units, nunits, mode, jstep, iter_base, staged, st);
  const size_t lds = staged + (size_t)g.M[2] * nl * sizeof(Cx<R>);
  HOM_DISPATCH(k_first, max_butterflies(g.pl[2], g.M[2], nl), lds, dim3(g.Q, 1, nunits), g, units, mode, jstep,
               iter_base);
}

template <typename R>
hipError_t launch_last(const Geo& g, const UnitDev* units, int nunits, int mode, int jstep, const int* iter_base,
                       hipStream_t st) {
  if constexpr (sizeof(R) == 4) {
    hipError_t e;
    if (fast_row(false, g, units, nunits, mode, jstep, iter_base, st, &e)) return e;
  }
  const int nl = 2 * g.P;
  if (!rows_fit<R>(g, 0)) return launch_last_long<R>(g, units, nunits, mode, jstep, iter_base, st);
  const size_t lds = (size_t)g.M[2] * nl * sizeof(Cx<R>);
  HOM_DISPATCH(k_last, max_butterflies(g.pl[2], g.M[2], nl), lds, dim3(g.Q, 1, nunits), g, units, mode, jstep,
               iter_base);
}

template <typename R>
hipError_t launch_apply(const Geo& g, const UnitDev* units, int nunits, int mode, hipStream_t st) {
  if constexpr (sizeof(R) == 4) {
    hipError_t e;
    // a plane geometry has skipped the middle passes: only the plane pass fits its buffers
    if (g.plane && (mode == APPLY_COEF || mode == APPLY_COEF_CG))
      return fast_plane(g, units, nunits, mode == APPLY_COEF_CG ? 1 : 0, st, &e) ? e : hipErrorNotSupported;
    if (mode != APPLY_QUAD && fast_apply(g, units, nunits, mode == APPLY_COEF_CG ? 1 : 0, st, &e)) return e;
  }
  const int nl = g.tileA * g.P;
  const size_t lds = (size_t)g.M[0] * nl * sizeof(Cx<R>);
  HOM_DISPATCH(k_apply, max_butterflies(g.pl[0], g.M[0], nl), lds, dim3(8 * ((g.nbA + 7) / 8), 1, nunits), g, units,
               mode);
}

template <typename R>
hipError_t launch_mid(const Geo& g, const UnitDev* units, int nunits, int inverse, hipStream_t st) {
  if constexpr (sizeof(R) == 4) {
    hipError_t e;
    if (fast_mid(g, units, nunits, inverse, st, &e)) return e;
  }
  const int inner = g.M[2] * g.P;
  const int nb = (inner + g.tileM - 1) / g.tileM;
  const size_t lds = (size_t)g.M[1] * g.tileM * sizeof(Cx<R>);
  HOM_DISPATCH(k_mid, max_butterflies(g.pl[1], g.M[1], g.tileM), lds, dim3(nb, g.N[0], nunits), g, units, inverse);
}

template <typename R>
hipError_t launch_line_fft(Cx<R>* data, int outer, int Lm, int inner, const Plan& pl, const Cx<R>* tw, int inverse,
                           hipStream_t st) {
  int tile = 1;
  while (tile * 2 <= inner && (size_t)Lm * tile * 2 * sizeof(Cx<R>) <= 48 * 1024 && tile < 64) tile *= 2;
  const int nb = (inner + tile - 1) / tile;
  const size_t lds = (size_t)Lm * tile * sizeof(Cx<R>);
  HOM_DISPATCH(k_line_fft, max_butterflies(pl, Lm, tile), lds, dim3(nb, outer, 1), data, outer, Lm, inner, tile, pl,
               tw, inverse);
}

template hipError_t launch_first<float>(const Geo&, const UnitDev*, int, int, int, const int*, hipStream_t);
template hipError_t launch_first<double>(const Geo&, const UnitDev*, int, int, int, const int*, hipStream_t);
template hipError_t launch_last<float>(const Geo&, const UnitDev*, int, int, int, const int*, hipStream_t);
template hipError_t launch_last<double>(const Geo&, const UnitDev*, int, int, int, const int*, hipStream_t);
template hipError_t launch_apply<float>(const Geo&, const UnitDev*, int, int, hipStream_t);
template hipError_t launch_apply<double>(const Geo&, const UnitDev*, int, int, hipStream_t);
template hipError_t launch_mid<float>(const Geo&, const UnitDev*, int, int, hipStream_t);
template hipError_t launch_mid<double>(const Geo&, const UnitDev*, int, int, hipStream_t);
template hipError_t launch_line_fft<double>(Cx<double>*, int, int, int, const Plan&, const Cx<double>*, int,
                                            hipStream_t);

static int grid_for(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
}

hipError_t launch_rhs(const Geo& g, const UnitDev* units, int nunits, hipStream_t st) {
  hipLaunchKernelGGL(k_rhs, dim3(grid_for(g.S), 1, nunits), dim3(kBlock), 0, st, g, units);
  return hipGetLastError();
}

hipError_t launch_start_energy(const Geo& g, const UnitDev* units, int nunits, hipStream_t st) {
  hipLaunchKernelGGL(k_start_energy, dim3(nunits), dim3(kBlock), 0, st, g, units);
  return hipGetLastError();
}

hipError_t launch_start_vectors(const Geo& g, const UnitDev* units, int nunits, int have_x0, hipStream_t st) {
  hipLaunchKernelGGL(k_start, dim3(grid_for((size_t)g.m * g.S), 1, nunits), dim3(kBlock), 0, st, g, units, have_x0);
  return hipGetLastError();
}

hipError_t launch_init_scal(const Geo& g, const UnitDev* units, int nunits, int* iter_base, int chunk, double tol,
                            int maxit, int stop, double etol, int mu_parts, double mu_user, hipStream_t st) {
  hipLaunchKernelGGL(k_init_scal, dim3((nunits + kBlock - 1) / kBlock), dim3(kBlock), 0, st, g, units, nunits,
                     iter_base, chunk, tol, maxit, stop, etol, mu_parts, mu_user);
  return hipGetLastError();
}

hipError_t launch_coef_min_eig(bool fp32, const Geo& g, const UnitDev* units, int nunits, int nparts,
                               hipStream_t st) {
  if (nparts < 1) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_coef_min_eig<float>, dim3(nparts, 1, nunits), dim3(kBlock), 0, st, g, units);
  else
    hipLaunchKernelGGL(k_coef_min_eig<double>, dim3(nparts, 1, nunits), dim3(kBlock), 0, st, g, units);
  return hipGetLastError();
}

hipError_t launch_symmetrize(const Geo& g, const Cx<double>* src, Cx<double>* dst, int m, hipStream_t st) {
  hipLaunchKernelGGL(k_symmetrize, dim3(grid_for(g.S)), dim3(kBlock), 0, st, g, src, dst, m);
  return hipGetLastError();
}
hipError_t launch_symmetrize_jobs(const Geo& g, const SymJob* jobs, int njobs, int m, hipStream_t st) {
  if (njobs < 1) return hipSuccess;
  const int gx = std::max(1, std::min(grid_for(g.S), std::max(1, 2048 / njobs)));
  for (int j0 = 0; j0 < njobs; j0 += 65535)
    hipLaunchKernelGGL(k_symmetrize_jobs, dim3(gx, std::min(65535, njobs - j0)), dim3(kBlock), 0, st, g, jobs + j0,
                       m);
  return hipGetLastError();
}

hipError_t launch_advance(const Geo& g, const UnitDev* units, int nunits, int* iter_base, int step, int* active_out,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(kBlock), 0, st, g, units, nunits, iter_base, step, active_out);
  return hipGetLastError();
}

__global__ void k_collect_solve(const UnitDev* __restrict__ units, int n, int L, int nbL, SolveOut* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * L) return;
  const int u = t / L, l = t - u * L;
  const UnitDev& U = units[u];
  double s = 0.0;
  for (int q = 0; q < nbL; ++q) s += U.part_d[(size_t)l * nbL + q];
  out[t].rres = s;
  out[t].sc = U.sc[l];
}

__global__ void k_collect_bounds(const UnitDev* __restrict__ units, int n, int nbA, double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * 9) return;
  const int u = t / 9, j = t - u * 9;
  const double* p = units[u].part_q;
  double s = 0.0;
  // the host's order (q = 0, 1, ...), with the loads of eight terms in flight
#pragma unroll 8
  for (int q = 0; q < nbA; ++q) s += p[(size_t)q * 9 + j];
  out[t] = s;
}

hipError_t launch_collect_solve(const UnitDev* units, int n, int L, int nbL, SolveOut* out, hipStream_t st) {
  hipLaunchKernelGGL(k_collect_solve, dim3((n * L + 63) / 64), dim3(64), 0, st, units, n, L, nbL, out);
  return hipGetLastError();
}

hipError_t launch_collect_bounds(const UnitDev* units, int n, int nbA, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_collect_bounds, dim3((n * 9 + 63) / 64), dim3(64), 0, st, units, n, nbA, out);
  return hipGetLastError();
}

hipError_t launch_combine(const FieldTriple& x, int d, const double* w, Cx<double>* out, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_combine, dim3(grid_for(n)), dim3(kBlock), 0, st, x, d, w[0], d > 1 ? w[1] : 0.0,
                     d > 2 ? w[2] : 0.0, out, n);
  return hipGetLastError();
}

hipError_t launch_twiddles(Cx<double>* t64, Cx<float>* t32, int M, hipStream_t st) {
  hipLaunchKernelGGL(k_twiddles, dim3(grid_for(M)), dim3(kBlock), 0, st, t64, t32, M);
  return hipGetLastError();
}

// Network input: a/<a> and log(max(a, 1e-3 <a>)/<a>), a = trace(A_M)/d, <a> = trace(A_hat(0))/d.
// weight_only: one channel max(a, 1e-3 <a>)/<a> (the pointwise weight of the
// quadrature of the energy, kept positive where the truncated series of a
// discontinuous coefficient overshoots below zero).
__device__ __forceinline__ void net_input_cell(const double* __restrict__ c, int nc, int d, long Mt,
                                               const Cx<double>* __restrict__ ahat0, long S, float* __restrict__ out,
                                               int weight_only) {
  const int nd = (nc == 1) ? 1 : d;
  double mean = 0.0;
  for (int k = 0; k < nd; ++k) mean += ahat0[(size_t)k * S].x;
  mean /= nd;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < Mt; t += (long)gridDim.x * blockDim.x) {
    double a = 0.0;
    for (int k = 0; k < nd; ++k) a += c[(size_t)k * Mt + t];
    a /= nd;
    if (weight_only) {
      out[t] = (float)(fmax(a, 1e-3 * mean) / mean);
    } else {
      out[t] = (float)(a / mean);
      out[Mt + t] = (float)log(fmax(a, 1e-3 * mean) / mean);
    }
  }
}
__global__ void k_net_input(const double* __restrict__ c, int nc, int d, long Mt, const Cx<double>* __restrict__ ahat0,
                            long S, float* __restrict__ out, int weight_only) {
  net_input_cell(c, nc, d, Mt, ahat0, S, out, weight_only);
}
// Cell blockIdx.y of a batch into out + cell stride; with weights, blockIdx.z
// = k selects the primal (0) or dual (1) coefficient and its channel.
__global__ void k_net_input_jobs(const NetJob* __restrict__ jobs, int nc, int d, long Mt, long S, float* __restrict__ out,
                                 size_t stride, int weights) {
  const NetJob j = jobs[blockIdx.y];
  const int k = blockIdx.z;
  net_input_cell(j.coef64[k], nc, d, Mt, j.ahat0[k], S, out + blockIdx.y * stride + (size_t)k * Mt, weights);
}

hipError_t launch_net_input_jobs(const NetJob* jobs, int n, int nc, int d, long Mt, long S, float* out, size_t stride,
                                 int weights, hipStream_t st) {
  const int gx = std::max(1, std::min(grid_for(Mt), std::max(1, 4096 / n)));
  for (int i0 = 0; i0 < n; i0 += 65535)
    hipLaunchKernelGGL(k_net_input_jobs, dim3(gx, std::min(65535, n - i0), weights ? 2 : 1), dim3(kBlock), 0, st,
                       jobs + i0, nc, d, Mt, S, out + (size_t)i0 * stride, stride, weights);
  return hipGetLastError();
}
hipError_t launch_net_input(const double* coef64, int nc, int d, long Mt, const Cx<double>* ahat0, long S, float* out,
                            int weight_only, hipStream_t st) {
  hipLaunchKernelGGL(k_net_input, dim3(grid_for(Mt)), dim3(kBlock), 0, st, coef64, nc, d, Mt, ahat0, S, out,
                     weight_only);
  return hipGetLastError();
}

__global__ void k_coef_planes(const float* __restrict__ c32, float* __restrict__ cp, int nc, int M0, int M1, int M2) {
  const size_t total = (size_t)nc * M0 * M1 * M2;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    // t = ((m2 nc + c) M0 + m0) M1 + m1
    const size_t m1 = t % M1;
    size_t r = t / M1;
    const size_t m0 = r % M0;
    r /= M0;
    const size_t c = r % nc, m2 = r / nc;
    cp[t] = c32[((c * M0 + m0) * M1 + m1) * M2 + m2];
  }
}

hipError_t launch_coef_planes(const float* c32, float* cp, int nc, const int* Mz, hipStream_t st) {
  const size_t total = (size_t)nc * Mz[0] * Mz[1] * Mz[2];
  hipLaunchKernelGGL(k_coef_planes, dim3(grid_for(total)), dim3(kBlock), 0, st, c32, cp, nc, Mz[0], Mz[1], Mz[2]);
  return hipGetLastError();
}

hipError_t launch_coef_real(const Cx<double>* full, double* c64, float* c32, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_coef_real, dim3(grid_for(n)), dim3(kBlock), 0, st, full, c64, c32, n);
  return hipGetLastError();
}

hipError_t launch_extract_half(const Geo& g, const Cx<double>* full, Cx<double>* half, int nc, hipStream_t st) {
  hipLaunchKernelGGL(k_extract_half, dim3(grid_for((size_t)g.S * nc)), dim3(kBlock), 0, st, g, full, half, nc);
  return hipGetLastError();
}

hipError_t launch_extract_half_jobs(const Geo& g, const CoefJob* jobs, int n, int nc, hipStream_t st) {
  if (n < 1 || n > 65535) return hipErrorInvalidValue;
  const unsigned nb = (unsigned)std::min<size_t>(grid_for((size_t)g.S * nc), 1024);
  hipLaunchKernelGGL(k_extract_half_jobs, dim3(nb, 2, n), dim3(kBlock), 0, st, g, jobs, nc);
  return hipGetLastError();
}

hipError_t launch_coef_incl(int d, const int* Mint, const double* iY, int nc, const double* A0c, int n_incl,
                            const void* dev_incl, Cx<double>* out, hipStream_t st) {
  const size_t Mt = (size_t)Mint[0] * Mint[1] * Mint[2];
  hipLaunchKernelGGL(k_coef_incl, dim3(grid_for(Mt)), dim3(kBlock), 0, st, d, Mint[0], Mint[1], Mint[2], iY[0], iY[1],
                     iY[2], nc, A0c, n_incl, reinterpret_cast<const InclDev*>(dev_incl), out);
  return hipGetLastError();
}

hipError_t launch_pixel_factor(int d, const int* Mint, const int* Pint, int nc, const Cx<double>* dft, Cx<double>* out,
                               hipStream_t st) {
  (void)d;
  const size_t Mt = (size_t)Mint[0] * Mint[1] * Mint[2];
  hipLaunchKernelGGL(k_pixel_factor, dim3(grid_for(Mt)), dim3(kBlock), 0, st, Mint[0], Mint[1], Mint[2], Pint[0],
                     Pint[1], Pint[2], nc, dft, out);
  return hipGetLastError();
}

size_t incl_dev_size() { return sizeof(InclDev); }

// ---- point values on the N grid (GaNi, eq. FD_A_GaNi)
// Grid point x_a = Y_a k_a / N_a, k in Z_N (eq. grid_points).  A point is in a
// box inclusion iff |x_a - c_a| < h_a / 2 on every axis, in a ball iff
// |x - c|^2 < R^2, with periodic minimum-image differences (open sets: a point
// on an interface belongs to the matrix; closed = 1 puts box faces inside).
__global__ void k_sample_incl(int N0, int N1, int N2, double Y0, double Y1, double Y2, int nc,
                              const double* __restrict__ A0c, int n_incl, const InclDev* __restrict__ inc,
                              int closed, double* __restrict__ out) {
  const size_t Nt = (size_t)N0 * N1 * N2;
  const int Nn[3] = {N0, N1, N2};
  const double Y[3] = {Y0, Y1, Y2};
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < Nt; t += (size_t)gridDim.x * blockDim.x) {
    const int j[3] = {(int)(t / ((size_t)N1 * N2)), (int)((t / N2) % N1), (int)(t % N2)};
    double x[3];
    for (int a = 0; a < 3; ++a) x[a] = Y[a] * (double)fr(j[a], Nn[a]) / (double)Nn[a];
    double v[6];
    for (int c = 0; c < nc; ++c) v[c] = A0c[c];
    for (int q = 0; q < n_incl; ++q) {
      const InclDev& I = inc[q];
      double dl[3];
      for (int a = 0; a < 3; ++a) {
        const double u = x[a] - I.c[a];
        dl[a] = u - Y[a] * rint(u / Y[a]);
      }
      bool inside;
      if (I.kind == 0) {
        inside = true;
        for (int a = 0; a < 3; ++a) inside = inside && (closed ? fabs(dl[a]) <= 0.5 * I.h[a] : fabs(dl[a]) < 0.5 * I.h[a]);
      } else {
        inside = ((0.0 + dl[0] * dl[0]) + dl[1] * dl[1]) + dl[2] * dl[2] < I.h[0] * I.h[0];
      }
      if (inside)
        for (int c = 0; c < nc; ++c) v[c] = A0c[c] + I.A[c];
    }
    for (int c = 0; c < nc; ++c) out[c * Nt + t] = v[c];
  }
}

// Pixel i_a along axis a covers [-Y_a/2 + i_a Y_a/P_a, -Y_a/2 + (i_a+1) Y_a/P_a).
__global__ void k_sample_pixels(int N0, int N1, int N2, double Y0, double Y1, double Y2, int P0, int P1, int P2,
                                int nc, const double* __restrict__ img, double* __restrict__ out) {
  const size_t Nt = (size_t)N0 * N1 * N2, Pt = (size_t)P0 * P1 * P2;
  const int Nn[3] = {N0, N1, N2}, Pp[3] = {P0, P1, P2};
  const double Y[3] = {Y0, Y1, Y2};
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < Nt; t += (size_t)gridDim.x * blockDim.x) {
    const int j[3] = {(int)(t / ((size_t)N1 * N2)), (int)((t / N2) % N1), (int)(t % N2)};
    long ip[3];
    for (int a = 0; a < 3; ++a) {
      const double x = Y[a] * (double)fr(j[a], Nn[a]) / (double)Nn[a];
      long i = (long)floor((x / Y[a] + 0.5) * (double)Pp[a]);
      ip[a] = i < 0 ? 0 : (i > Pp[a] - 1 ? Pp[a] - 1 : i);
    }
    const size_t pix = ((size_t)ip[0] * P1 + ip[1]) * P2 + ip[2];
    for (int c = 0; c < nc; ++c) out[c * Nt + t] = img[c * Pt + pix];
  }
}

__global__ void k_real_to_cx(const double* __restrict__ in, Cx<double>* __restrict__ out, size_t n, double s) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
    out[t] = cx(in[t] * s, 0.0);
}

__global__ void k_scale_cx(Cx<double>* __restrict__ a, size_t n, double s) {
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
    a[t] = cx(a[t].x * s, a[t].y * s);
}

hipError_t launch_sample_incl(const int* Nint, const double* Yint, int nc, const double* A0c, int n_incl,
                              const void* dev_incl, bool closed, double* out, hipStream_t st) {
  const size_t Nt = (size_t)Nint[0] * Nint[1] * Nint[2];
  hipLaunchKernelGGL(k_sample_incl, dim3(grid_for(Nt)), dim3(kBlock), 0, st, Nint[0], Nint[1], Nint[2], Yint[0],
                     Yint[1], Yint[2], nc, A0c, n_incl, (const InclDev*)dev_incl, closed ? 1 : 0, out);
  return hipGetLastError();
}

hipError_t launch_sample_pixels(const int* Nint, const double* Yint, const int* Pint, int nc, const double* img,
                                double* out, hipStream_t st) {
  const size_t Nt = (size_t)Nint[0] * Nint[1] * Nint[2];
  hipLaunchKernelGGL(k_sample_pixels, dim3(grid_for(Nt)), dim3(kBlock), 0, st, Nint[0], Nint[1], Nint[2], Yint[0],
                     Yint[1], Yint[2], Pint[0], Pint[1], Pint[2], nc, img, out);
  return hipGetLastError();
}

// Smoothing filter of a 2D characteristic image (periodic 3 x 3 stencil with
// weights 4 / 2 / 1 sixteenths): out = 16 f_smoothed, in integers.
__global__ void k_smooth2d(int P0, int P1, const int* __restrict__ f, int* __restrict__ out) {
  const size_t n = (size_t)P0 * P1;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(t / P1), j = (int)(t % P1);
    const int im = i == 0 ? P0 - 1 : i - 1, ip = i == P0 - 1 ? 0 : i + 1;
    const int jm = j == 0 ? P1 - 1 : j - 1, jp = j == P1 - 1 ? 0 : j + 1;
    auto at = [&](int a, int b) { return f[(size_t)a * P1 + b]; };
    out[t] = 4 * at(i, j) + 2 * (at(ip, j) + at(im, j) + at(i, jp) + at(i, jm)) +
             (at(ip, jp) + at(im, jm) + at(im, jp) + at(ip, jm));
  }
}

hipError_t launch_smooth2d(int P0, int P1, const int* f, int* out, hipStream_t st) {
  hipLaunchKernelGGL(k_smooth2d, dim3(grid_for((size_t)P0 * P1)), dim3(kBlock), 0, st, P0, P1, f, out);
  return hipGetLastError();
}

hipError_t launch_real_to_cx(const double* in, Cx<double>* out, size_t n, double s, hipStream_t st) {
  hipLaunchKernelGGL(k_real_to_cx, dim3(grid_for(n)), dim3(kBlock), 0, st, in, out, n, s);
  return hipGetLastError();
}

hipError_t launch_scale_cx(Cx<double>* a, size_t n, double s, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_cx, dim3(grid_for(n)), dim3(kBlock), 0, st, a, n, s);
  return hipGetLastError();
}

}  // namespace hom
