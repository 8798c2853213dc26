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
#include <functional>

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

// Rows n1 of the four-step layout (positions B n1 + q, q < B) that lie
// outside Z_N for every thread q: the first register DFT of an inverse
// transform reads zeros there, and the last register DFT of a forward
// transform produces values that are dropped.  Both are known when the
// kernel is compiled, so the pruned work is removed.
template <int M>
constexpr bool dead_row(int n1) {
  return Cfg<M>::B * n1 > Cfg<M>::H && Cfg<M>::B * n1 + Cfg<M>::B - 1 < M - Cfg<M>::H;
}
// Global-memory access at a 32-bit byte offset from a block-uniform base:
// the base stays in scalar registers and the access is a global (not flat)
// instruction with a 32-bit vector offset.  Callers keep every buffer so
// accessed below 4 GiB.
typedef __attribute__((address_space(1))) unsigned char gbyte;
template <typename T>
__device__ __forceinline__ T gld(const void* base, unsigned boff) {
  return *reinterpret_cast<const __attribute__((address_space(1))) T*>((const gbyte*)base + boff);
}
template <typename T>
__device__ __forceinline__ void gst(void* base, unsigned boff, T v) {
  *reinterpret_cast<__attribute__((address_space(1))) T*>((gbyte*)base + boff) = v;
}
// complex FP32 values move as one 64-bit word
__device__ __forceinline__ Cx<float> gldc(const void* base, unsigned boff) {
  return __builtin_bit_cast(Cx<float>, gld<unsigned long long>(base, boff));
}
__device__ __forceinline__ void gstc(void* base, unsigned boff, Cx<float> v) {
  gst<unsigned long long>(base, boff, __builtin_bit_cast(unsigned long long, v));
}

// Element i of a buffer through a global (address space 1) pointer.  FLAT
// instructions (the default for pointers read from the unit table) count
// against the LDS counter as well, so every barrier after them waits until
// they complete; global instructions leave barriers to LDS traffic and let
// stores drain in the background.
typedef double gdbl2 __attribute__((ext_vector_type(2)));
typedef float gflt2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ Cx<double> gload(const Cx<double>* p, size_t i) {
  return __builtin_bit_cast(Cx<double>, ((const __attribute__((address_space(1))) gdbl2*)p)[i]);
}
__device__ __forceinline__ void gstore(Cx<double>* p, size_t i, Cx<double> v) {
  ((__attribute__((address_space(1))) gdbl2*)p)[i] = __builtin_bit_cast(gdbl2, v);
}
__device__ __forceinline__ Cx<float> gload(const Cx<float>* p, size_t i) {
  return __builtin_bit_cast(Cx<float>, ((const __attribute__((address_space(1))) gflt2*)p)[i]);
}
__device__ __forceinline__ void gstore(Cx<float>* p, size_t i, Cx<float> v) {
  ((__attribute__((address_space(1))) gflt2*)p)[i] = __builtin_bit_cast(gflt2, v);
}
__device__ __forceinline__ float gload(const float* p, size_t i) {
  return ((const __attribute__((address_space(1))) float*)p)[i];
}
__device__ __forceinline__ void gstore(double* p, size_t i, double v) {
  ((__attribute__((address_space(1))) double*)p)[i] = v;
}

// Element i through a global pointer (G) or the default flat one: the row
// passes measure faster with flat loads in 2D and global loads in 3D.
template <bool G, typename T>
__device__ __forceinline__ T pick_load(const T* p, size_t i) {
  if constexpr (G)
    return gload(p, i);
  else
    return p[i];
}

// rows whose positions B n1 + q lie in Z_N for every q < B
template <int M>
constexpr bool full_row(int n1) {
  return Cfg<M>::B * n1 + Cfg<M>::B - 1 <= Cfg<M>::H || Cfg<M>::B * n1 >= M - Cfg<M>::H;
}
template <int M>
constexpr int dead_mask() {
  int m = 0;
  for (int n1 = 0; n1 < Cfg<M>::A; ++n1)
    if (dead_row<M>(n1)) m |= 1 << n1;
  return m;
}

}  // namespace

// ============================================================== column pass
// Exchange of register lines between the two steps of a four-step FFT
// through LDS.  Threads with `wr` store their NW values of group q (the
// slots q G + j, j < NW), threads with `rd` load NR values of column q (the
// slots q + j G, j < NR); a slot holds TP points.  Groups of slots are laid
// out RS = G TP + pad elements apart, with RS = TP modulo the bank count, so
// that lane (q, pt) of a wave, lane number q TP + pt, touches bank
// (q TP + pt + j TP) mod banks on both sides: no bank conflicts for the 64
// lanes (HX, 4-byte words, 64 banks) or 32 lanes (complex words).  HX = 1
// moves the real parts and then the imaginary parts through a real-valued
// buffer of half the size (more blocks per CU for the same LDS).
template <int G, int TP, int HX>
constexpr int xpad() {
  constexpr int W = HX ? 64 : 32;
  return ((TP - G * TP) % W + W) % W;
}
// elements of one thread group's exchange area for M = A B
template <int A, int B, int TP, int HX>
constexpr int xarea() {
  constexpr int e1 = B * (A * TP + xpad<A, TP, HX>()), e2 = A * (B * TP + xpad<B, TP, HX>());
  return e1 > e2 ? e1 : e2;
}
template <typename R, int NW, int NR, int G, int TP, int HX>
__device__ __forceinline__ void xchg(Cx<R>* ex, Cx<R>* v, bool wr, bool rd, int q, int pt) {
  constexpr int RS = G * TP + xpad<G, TP, HX>();
  const int wb = q * RS + pt, rb = q * TP + pt;
  if constexpr (!HX) {
    if (wr) {
#pragma unroll
      for (int j = 0; j < NW; ++j) ex[wb + j * TP] = v[j];
    }
    __syncthreads();
    if (rd) {
#pragma unroll
      for (int j = 0; j < NR; ++j) v[j] = ex[rb + j * RS];
    }
    __syncthreads();
  } else {
    // the real parts are stored before they are overwritten by the loads
    R* e = reinterpret_cast<R*>(ex);
    if (wr) {
#pragma unroll
      for (int j = 0; j < NW; ++j) e[wb + j * TP] = v[j].x;
    }
    __syncthreads();
    if (rd) {
#pragma unroll
      for (int j = 0; j < NR; ++j) v[j].x = e[rb + j * RS];
    }
    __syncthreads();
    if (wr) {
#pragma unroll
      for (int j = 0; j < NW; ++j) e[wb + j * TP] = v[j].y;
    }
    __syncthreads();
    if (rd) {
#pragma unroll
      for (int j = 0; j < NR; ++j) v[j].y = e[rb + j * RS];
    }
    __syncthreads();
  }
}

// 2D column pass: the packs are independent (pack l holds the two components
// of load l, and the coefficient couples only those), so a group of TP x T
// threads takes one pack of TP points, T threads per point, one line per
// thread group in registers.  PB = 1: one pack per block; PB = P: the packs of
// the same points in one block, one thread group each, so the coefficient
// lines fetched for one pack serve the others from the CU's cache.  Block
// order is XCD-aware: blocks b and b + 8 run on the same XCD (round-robin
// dispatch), so each XCD takes a contiguous range of point blocks and, within
// it, the packs of one point block back to back.
// Below M = 625 the compiler's default allocation (about 110 VGPRs at M = 125,
// four waves per SIMD) shrinks without spills when asked for five waves: it
// then fits six (74-80 VGPRs), and the 125-point pass runs 19 % faster.  At
// M = 625 the same request spills to scratch (and runs 35 % slower).
template <typename R, int M, int P, int NC, int TP, int HX, int PB>
__global__ __launch_bounds__(PB * TP * Cfg<M>::T) __attribute__((amdgpu_waves_per_eu(M == 625 ? 1 : 5)))
void k_apply2_fast(Geo g, const UnitDev* __restrict__ units, int cg) {
  constexpr int A = Cfg<M>::A, B = Cfg<M>::B, T = Cfg<M>::T, NT = TP * Cfg<M>::T;
  static_assert(PB == 1 || PB == P, "a block holds one pack or all packs");
  static_assert(sizeof(R) == 4, "FP32 pass");
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<R>* tw = reinterpret_cast<Cx<R>*>(smem);   // [M]
  const UnitDev& U = units[blockIdx.z];
  if (cg && !any_active(U, g.L)) return;
  const int npts = g.M[2];
  const size_t Mtot = (size_t)M * npts;
  const int nbx = (npts + TP - 1) / TP, nbx8 = (nbx + 7) / 8;
  const int xcd = blockIdx.x % 8, w8 = blockIdx.x / 8;
  const int cbl = (PB == P) ? w8 : w8 / P, cb = xcd * nbx8 + cbl;
  if (cbl >= nbx8 || cb >= nbx) return;
  const int grp = (PB == 1) ? 0 : (int)threadIdx.x / NT, tid = (int)threadIdx.x - grp * NT;
  const int pk = (PB == P) ? grp : w8 % P;
  // exchange area of this thread group (complex, or real with HX)
  Cx<R>* ex = reinterpret_cast<Cx<R>*>(smem + (size_t)M * sizeof(Cx<R>) +
                                       (size_t)grp * xarea<A, B, TP, HX>() * (HX ? sizeof(R) : sizeof(Cx<R>)));
  const int p0 = cb * TP;
  const int pt = tid % TP, q = tid / TP;
  const bool ok = (p0 + pt) < npts;
  const Cx<R>* twg = reinterpret_cast<const Cx<R>*>(g.tw[0]);
  for (int i = threadIdx.x; i < M; i += blockDim.x) tw[i] = twg[i];
  void* data = U.bufA;
  // byte offset of element (row i0, point p0 + pt, pack pk): pack-major [P][N0][npts] or packs interleaved
  constexpr unsigned es = sizeof(Cx<R>);
  const unsigned rs = es * (g.pmaj ? (unsigned)npts : (unsigned)npts * P);
  // threads past the last point load from the last one (nothing of theirs is stored)
  const int pc = ok ? p0 + pt : npts - 1;
  const unsigned dbase = es * (g.pmaj ? (unsigned)pc + (unsigned)pk * g.N[0] * npts : (unsigned)pc * P + (unsigned)pk);
  const void* coef = U.coef;
  __syncthreads();

  Cx<R> v[T];
  // inverse, step 1: thread n2 = q holds x[B n1 + n2] (zero-padded N -> M); rows
  // wholly inside or outside Z_N0 need no per-thread test
  constexpr int N = Cfg<M>::N, H = Cfg<M>::H;
#pragma unroll
  for (int n1 = 0; n1 < A; ++n1) {
    const int pos = B * n1 + q;
    if (dead_row<M>(n1)) {
      v[n1] = rf::mk<R>(0, 0);
    } else if (full_row<M>(n1)) {
      const int i0 = (B * n1 <= H) ? pos : pos - (M - N);
      v[n1] = (T == B || q < B) ? gldc(data, (unsigned)i0 * rs + dbase) : rf::mk<R>(0, 0);
    } else {
      const int i0 = q < B ? kept<M>(pos) : -1;
      v[n1] = i0 >= 0 ? gldc(data, (unsigned)i0 * rs + dbase) : rf::mk<R>(0, 0);
    }
  }
  if (q < B) {
    rf::Dft<R, A, 1>::template run_z<dead_mask<M>()>(v);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      Cx<R> w = tw[q * k1];
      w.y = -w.y;
      v[k1] = rf::mul(v[k1], w);
    }
  }
  xchg<R, A, B, A, TP, HX>(ex, v, q < B, q < A, q, pt);
  if (q < A) {
    rf::Dft<R, B, 1>::run(v);
    // thread k1 = q holds u at x0 = q + A k2: the coefficient on the doubled grid
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) {
      const unsigned ci = (unsigned)((q + A * k2) * npts + pc) * (unsigned)sizeof(R);
      R a[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) a[c] = gld<R>(coef, (unsigned)(c * Mtot * sizeof(R)) + ci);
      const R u[2] = {v[k2].x, v[k2].y};
      R w[2];
      coef_mul<R>(2, NC, a, u, w);
      v[k2] = rf::mk<R>(w[0], w[1]);
    }
    // forward: step over n2 in registers (thread n1 = q), exchange, step over n1
    rf::Dft<R, B, -1>::run(v);
#pragma unroll
    for (int m2 = 0; m2 < B; ++m2) v[m2] = rf::mul(v[m2], tw[q * m2]);
  }
  xchg<R, B, A, B, TP, HX>(ex, v, q < A, q < B, q, pt);
  if (q < B) {
    rf::Dft<R, A, -1>::run(v);
    // thread m2 = q holds X[q + B m1]: store the Z_N0 part
    if (ok) {
#pragma unroll
      for (int m1 = 0; m1 < A; ++m1) {
        const int pos = q + B * m1;
        if (dead_row<M>(m1)) continue;
        if (full_row<M>(m1)) {
          gstc(data, (unsigned)((B * m1 <= H) ? pos : pos - (M - N)) * rs + dbase, v[m1]);
        } else {
          const int i0 = kept<M>(pos);
          if (i0 >= 0) gstc(data, (unsigned)i0 * rs + dbase, v[m1]);
        }
      }
    }
  }
}

// 3D column pass: TP points per block, T threads per point, all packs of a
// point held together (a load's three components straddle packs and the
// coefficient couples them).
template <typename R, int M, int D, int P, int NC, int TP>
__global__ __launch_bounds__(TP * Cfg<M>::T) void k_apply_fast(Geo g, const UnitDev* __restrict__ units, int cg) {
  constexpr int A = Cfg<M>::A, B = Cfg<M>::B, T = Cfg<M>::T;
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
  const R* coef = reinterpret_cast<const R*>(U.coef);

  Cx<R> v[P][T];
#pragma unroll
  for (int n1 = 0; n1 < A; ++n1) {
    const int i0 = (q < B && ok && !dead_row<M>(n1)) ? kept<M>(B * n1 + q) : -1;
#pragma unroll
    for (int pk = 0; pk < P; ++pk) v[pk][n1] = i0 >= 0 ? data[i0 * rowstride + col + pk] : rf::mk<R>(0, 0);
  }
  __syncthreads();
#pragma unroll
  for (int pk = 0; pk < P; ++pk) {
    if (q < B) {
      rf::Dft<R, A, 1>::template run_z<dead_mask<M>()>(v[pk]);
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
  if (q < A && ok) {
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
  if (q < B && ok) {
#pragma unroll
    for (int m1 = 0; m1 < A; ++m1) {
      if (dead_row<M>(m1)) continue;
      const int i0 = kept<M>(q + B * m1);
      if (i0 >= 0)
#pragma unroll
        for (int pk = 0; pk < P; ++pk) data[i0 * rowstride + col + pk] = v[pk][m1];
    }
  }
}

// ============================================================== middle pass (3D, axis 1)
// Lines along axis 1 of the flattened [M2][pack] elements: TP consecutive
// elements per block (contiguous in memory), T threads per line, grid
// (element blocks, N0 rows, units).  INV = 1: zero-padded N1 -> M1 inverse
// transform from the row-pass buffer to the column-pass buffer; INV = 0:
// forward transform back, keeping the Z_N1 part.
template <int M, int TP, int INV>
__global__ __launch_bounds__(TP * Cfg<M>::T) void k_mid_fast(Geo g, const UnitDev* __restrict__ units, int cg) {
  constexpr int A = Cfg<M>::A, B = Cfg<M>::B, T = Cfg<M>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<float>* tw = reinterpret_cast<Cx<float>*>(smem);  // [M]
  Cx<float>* ex = tw + M;                              // [M][TP]
  const UnitDev& U = units[blockIdx.z];
  if (cg && !any_active(U, g.L)) return;
  const int W = g.M[2] * g.P, N1 = g.N[1];
  const size_t i0 = blockIdx.y;
  const int tid = threadIdx.x, pt = tid % TP, q = tid / TP;
  const int f = blockIdx.x * TP + pt;
  const bool ok = f < W;
  const Cx<float>* twg = reinterpret_cast<const Cx<float>*>(g.tw[1]);
  for (int i = tid; i < M; i += blockDim.x) tw[i] = twg[i];
  const Cx<float>* in = reinterpret_cast<const Cx<float>*>(INV ? U.bufA : U.bufB);
  Cx<float>* out = reinterpret_cast<Cx<float>*>(INV ? U.bufB : U.bufA);
  Cx<float> v[T];
  if constexpr (INV) {
    // thread n2 = q holds x[B n1 + n2]
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) {
      const int i1 = (q < B && ok && !dead_row<M>(n1)) ? kept<M>(B * n1 + q) : -1;
      v[n1] = i1 >= 0 ? in[(i0 * N1 + i1) * W + f] : rf::mk<float>(0, 0);
    }
    __syncthreads();
    if (q < B) {
      rf::Dft<float, A, 1>::template run_z<dead_mask<M>()>(v);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) {
        Cx<float> w = tw[q * k1];
        w.y = -w.y;
        ex[(q * A + k1) * TP + pt] = rf::mul(v[k1], w);
      }
    }
    __syncthreads();
    if (q < A) {
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) v[n2] = ex[(n2 * A + q) * TP + pt];
      rf::Dft<float, B, 1>::run(v);
      if (ok) {
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) out[(i0 * M + q + A * k2) * W + f] = v[k2];
      }
    }
  } else {
    // thread n1 = q holds x[q + A n2]
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) v[n2] = (q < A && ok) ? in[(i0 * M + q + A * n2) * W + f] : rf::mk<float>(0, 0);
    __syncthreads();
    if (q < A) {
      rf::Dft<float, B, -1>::run(v);
#pragma unroll
      for (int m2 = 0; m2 < B; ++m2) ex[(q * B + m2) * TP + pt] = rf::mul(v[m2], tw[q * m2]);
    }
    __syncthreads();
    if (q < B) {
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) v[n1] = ex[(n1 * B + q) * TP + pt];
      rf::Dft<float, A, -1>::run(v);
      if (ok) {
#pragma unroll
        for (int m1 = 0; m1 < A; ++m1) {
          if (dead_row<M>(m1)) continue;
          const int i1 = kept<M>(q + B * m1);
          if (i1 >= 0) out[(i0 * N1 + i1) * W + f] = v[m1];
        }
      }
    }
  }
}

template <int M, int INV>
static hipError_t run_mid(const Geo& g, const UnitDev* units, int n, int cg, hipStream_t st) {
  constexpr int T = Cfg<M>::T, TP = (256 / T) > 64 ? 64 : (256 / T);
  const int W = g.M[2] * g.P;
  const size_t lds = (size_t)M * sizeof(Cx<float>) * (1 + TP);
  auto kern = k_mid_fast<M, TP, INV>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const dim3 grid((W + TP - 1) / TP, g.N[0], n);
  if (g_ext_timing.on)
    hipExtLaunchKernelGGL(kern, grid, dim3(TP * T), lds, st, g_ext_timing.start, g_ext_timing.stop, 0, g, units, cg);
  else
    hipLaunchKernelGGL(kern, grid, dim3(TP * T), lds, st, g, units, cg);
  return hipGetLastError();
}

// 3D middle pass for M1 in {25, 81, 125}; false when no specialisation exists.
bool fast_mid(const Geo& g, const UnitDev* units, int n, int flags, hipStream_t st, hipError_t* err) {
  if (std::getenv("HOM_NO_FAST")) return false;
  if (g.d != 3 || g.M[1] != 2 * g.N[1] - 1) return false;
  const int inv = flags & 1, cg = (flags & MID_CG) ? 1 : 0;
  switch (g.M[1]) {
    case 81: *err = inv ? run_mid<81, 1>(g, units, n, cg, st) : run_mid<81, 0>(g, units, n, cg, st); return true;
    case 125: *err = inv ? run_mid<125, 1>(g, units, n, cg, st) : run_mid<125, 0>(g, units, n, cg, st); return true;
    case 25: *err = inv ? run_mid<25, 1>(g, units, n, cg, st) : run_mid<25, 0>(g, units, n, cg, st); return true;
    default: return false;
  }
}

// ============================================================== coefficient setup (2D, FP64)
// A and A^-1 on the doubled grid in one complex transform: both Fourier
// series are Hermitian, so F_M^-1 (A_hat + i s B_hat) = A_M + i s B_M with real
// A_M, B_M.  s is the power of two nearest to <A>/<A^-1> (component 0 of the
// zero frequency), so both parts carry similar magnitudes through the
// rounding, and dividing by s is exact.
__device__ __forceinline__ double coef_pair_scale(const Cx<double>* A, const Cx<double>* Bh) {
  const double a = fabs(A[0].x), b = fabs(Bh[0].x);
  if (!(a > 0.0) || !(b > 0.0)) return 1.0;
  return ldexp(1.0, (int)rint(log2(a / b)));
}

// Inverse transform along axis 0 (columns of the [M][M] plane): TP columns
// per block, T threads per column; grid (column blocks, component[, cell]).
template <int M, int TP>
__device__ __forceinline__ void coef_cols(const Cx<double>* __restrict__ Ah, const Cx<double>* __restrict__ Bh,
                                          Cx<double>* __restrict__ out, const Cx<double>* __restrict__ twg) {
  constexpr int A = Cfg<M>::A, B = Cfg<M>::B, T = Cfg<M>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<double>* tw = reinterpret_cast<Cx<double>*>(smem);  // [M]
  Cx<double>* ex = tw + M;                               // [M][TP]
  const int tid = threadIdx.x, pt = tid % TP, q = tid / TP;
  const int p = blockIdx.x * TP + pt;
  const bool ok = p < M;
  const size_t base = (size_t)blockIdx.y * M * M;
  const double sc = coef_pair_scale(Ah, Bh);
  for (int i = tid; i < M; i += blockDim.x) tw[i] = twg[i];
  Cx<double> v[T];
#pragma unroll
  for (int n1 = 0; n1 < A; ++n1) {
    v[n1] = rf::mk<double>(0.0, 0.0);
    if (q < B && ok) {
      const size_t i = base + (size_t)(B * n1 + q) * M + p;
      const Cx<double> a = Ah[i], b = Bh[i];
      v[n1] = rf::mk<double>(a.x - sc * b.y, a.y + sc * b.x);
    }
  }
  __syncthreads();
  if (q < B) {
    rf::Dft<double, A, 1>::run(v);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      Cx<double> w = tw[q * k1];
      w.y = -w.y;
      ex[(q * A + k1) * TP + pt] = rf::mul(v[k1], w);
    }
  }
  __syncthreads();
  if (q < A) {
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) v[n2] = ex[(n2 * A + q) * TP + pt];
    rf::Dft<double, B, 1>::run(v);
    if (ok) {
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) out[base + (size_t)(q + A * k2) * M + p] = v[k2];
    }
  }
}

template <int M, int TP>
__global__ __launch_bounds__(TP * Cfg<M>::T) void k_coef_cols(const Cx<double>* __restrict__ Ah,
                                                              const Cx<double>* __restrict__ Bh,
                                                              Cx<double>* __restrict__ out,
                                                              const Cx<double>* __restrict__ twg) {
  coef_cols<M, TP>(Ah, Bh, out, twg);
}

template <int M, int TP>
__global__ __launch_bounds__(TP * Cfg<M>::T) void k_coef_cols_jobs(const CoefJob* __restrict__ jobs,
                                                                   const Cx<double>* __restrict__ twg) {
  const CoefJob& J = jobs[blockIdx.z];
  coef_cols<M, TP>(J.A, J.B, J.scratch, twg);
}

// Inverse transform along axis 2 (rows), G rows per block, T threads per row,
// then the real and imaginary parts split into A_M and B_M (FP64 and FP32).
template <int M, int G>
__device__ __forceinline__ void coef_rows(const Cx<double>* __restrict__ in, const Cx<double>* __restrict__ Ah,
                                          const Cx<double>* __restrict__ Bh, double* __restrict__ a64,
                                          float* __restrict__ a32, double* __restrict__ b64, float* __restrict__ b32,
                                          const Cx<double>* __restrict__ twg) {
  constexpr int A = Cfg<M>::A, B = Cfg<M>::B, T = Cfg<M>::T;
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<double>* tw = reinterpret_cast<Cx<double>*>(smem);  // [M]
  Cx<double>* ex = tw + M;                               // [G][M]
  const int tid = threadIdx.x, gr = tid / T, q = tid - gr * T;
  const int row = blockIdx.x * G + gr;
  const bool ok = row < M;
  const size_t base = (size_t)blockIdx.y * M * M + (size_t)(ok ? row : 0) * M;
  const double inv = 1.0 / coef_pair_scale(Ah, Bh);
  for (int i = tid; i < M; i += blockDim.x) tw[i] = twg[i];
  Cx<double>* e = ex + (size_t)gr * M;
  Cx<double> v[T];
#pragma unroll
  for (int n1 = 0; n1 < A; ++n1) v[n1] = (q < B && ok) ? in[base + B * n1 + q] : rf::mk<double>(0.0, 0.0);
  __syncthreads();
  if (q < B && ok) {
    rf::Dft<double, A, 1>::run(v);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      Cx<double> w = tw[q * k1];
      w.y = -w.y;
      e[q * A + k1] = rf::mul(v[k1], w);
    }
  }
  __syncthreads();
  if (q < A && ok) {
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) v[n2] = e[n2 * A + q];
    rf::Dft<double, B, 1>::run(v);
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) {
      const size_t i = base + q + A * k2;
      const double av = v[k2].x, bv = v[k2].y * inv;
      a64[i] = av;
      b64[i] = bv;
      if (a32) a32[i] = (float)av;
      if (b32) b32[i] = (float)bv;
    }
  }
}

template <int M, int G>
__global__ __launch_bounds__(G * Cfg<M>::T) void k_coef_rows(const Cx<double>* __restrict__ in,
                                                             const Cx<double>* __restrict__ Ah,
                                                             const Cx<double>* __restrict__ Bh,
                                                             double* __restrict__ a64, float* __restrict__ a32,
                                                             double* __restrict__ b64, float* __restrict__ b32,
                                                             const Cx<double>* __restrict__ twg) {
  coef_rows<M, G>(in, Ah, Bh, a64, a32, b64, b32, twg);
}

template <int M, int G>
__global__ __launch_bounds__(G * Cfg<M>::T) void k_coef_rows_jobs(const CoefJob* __restrict__ jobs,
                                                                  const Cx<double>* __restrict__ twg) {
  const CoefJob& J = jobs[blockIdx.z];
  coef_rows<M, G>(J.scratch, J.A, J.B, J.a64, J.a32, J.b64, J.b32, twg);
}

template <int M>
struct CoefTiles;
template <>
struct CoefTiles<625> { static constexpr int TP = 4, G = 4; };
template <>
struct CoefTiles<125> { static constexpr int TP = 8, G = 8; };
template <>
struct CoefTiles<81> { static constexpr int TP = 16, G = 16; };
template <>
struct CoefTiles<25> { static constexpr int TP = 32, G = 32; };

template <int M>
static hipError_t run_coef_setup(int nc, const Cx<double>* Ah, const Cx<double>* Bh, Cx<double>* scratch, double* a64,
                                 float* a32, double* b64, float* b32, const Cx<double>* tw, hipStream_t st) {
  constexpr int T = Cfg<M>::T, TP = CoefTiles<M>::TP, G = CoefTiles<M>::G;
  const size_t lds1 = (size_t)M * sizeof(Cx<double>) * (1 + TP);
  const size_t lds2 = (size_t)M * sizeof(Cx<double>) * (1 + G);
  auto k1 = k_coef_cols<M, TP>;
  auto k2 = k_coef_rows<M, G>;
  hipError_t e = hipFuncSetAttribute((const void*)k1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds1);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k1, dim3((M + TP - 1) / TP, nc), dim3(TP * T), lds1, st, Ah, Bh, scratch, tw);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k2, dim3((M + G - 1) / G, nc), dim3(G * T), lds2, st, scratch, Ah, Bh, a64, a32, b64, b32, tw);
  return hipGetLastError();
}

template <int M>
static hipError_t run_coef_setup_jobs(int nc, const CoefJob* jobs, int n, const Cx<double>* tw, hipStream_t st) {
  constexpr int T = Cfg<M>::T, TP = CoefTiles<M>::TP, G = CoefTiles<M>::G;
  const size_t lds1 = (size_t)M * sizeof(Cx<double>) * (1 + TP);
  const size_t lds2 = (size_t)M * sizeof(Cx<double>) * (1 + G);
  auto k1 = k_coef_cols_jobs<M, TP>;
  auto k2 = k_coef_rows_jobs<M, G>;
  hipError_t e = hipFuncSetAttribute((const void*)k1, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds1);
  if (e == hipSuccess) e = hipFuncSetAttribute((const void*)k2, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k1, dim3((M + TP - 1) / TP, nc, n), dim3(TP * T), lds1, st, jobs, tw);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k2, dim3((M + G - 1) / G, nc, n), dim3(G * T), lds2, st, jobs, tw);
  return hipGetLastError();
}

bool fast_coef_setup_jobs(int d, const int* Mz, int nc, const CoefJob* jobs, int n, const Cx<double>* tw,
                          hipStream_t st, hipError_t* err) {
  if (std::getenv("HOM_NO_FAST")) return false;
  if (d != 2 || Mz[0] != Mz[2] || n < 1 || n > 65535) return false;
  switch (Mz[0]) {
    case 625: *err = run_coef_setup_jobs<625>(nc, jobs, n, tw, st); return true;
    case 125: *err = run_coef_setup_jobs<125>(nc, jobs, n, tw, st); return true;
    case 81: *err = run_coef_setup_jobs<81>(nc, jobs, n, tw, st); return true;
    case 25: *err = run_coef_setup_jobs<25>(nc, jobs, n, tw, st); return true;
    default: return false;
  }
}

// 2D problems with M0 = M2 in {25, 81, 125, 625}: both coefficients on the
// doubled grid in two launches; false when no specialisation exists.
bool fast_coef_setup(int d, const int* Mz, int nc, const Cx<double>* Ah, const Cx<double>* Bh, Cx<double>* scratch,
                     double* a64, float* a32, double* b64, float* b32, const Cx<double>* tw, hipStream_t st,
                     hipError_t* err) {
  if (std::getenv("HOM_NO_FAST")) return false;
  if (d != 2 || Mz[0] != Mz[2]) return false;
  switch (Mz[0]) {
    case 625: *err = run_coef_setup<625>(nc, Ah, Bh, scratch, a64, a32, b64, b32, tw, st); return true;
    case 125: *err = run_coef_setup<125>(nc, Ah, Bh, scratch, a64, a32, b64, b32, tw, st); return true;
    case 81: *err = run_coef_setup<81>(nc, Ah, Bh, scratch, a64, a32, b64, b32, tw, st); return true;
    case 25: *err = run_coef_setup<25>(nc, Ah, Bh, scratch, a64, a32, b64, b32, tw, st); return true;
    default: return false;
  }
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

// A block handles the loads lo .. lo + L - 1 (lo = blockIdx.y * L): in 2D one
// load per block (its pack is independent of the others), in 3D all loads.
// P packs of the block start at pack po of the Pg packs of the field buffers.
template <typename R, int M, int D, int L, int DUAL, int G>
__global__ __launch_bounds__(256, D == 2 ? 6 : 1) void k_first_fast(Geo g, const UnitDev* __restrict__ units, int mode, int jstep,
                                                    const int* __restrict__ iter_base) {
  constexpr int A = Cfg<M>::A, B = Cfg<M>::B, T = Cfg<M>::T, N2 = Cfg<M>::N, H2 = Cfg<M>::H;
  constexpr int P = (L * D + 1) / 2, m = DUAL ? D - 1 : 1, d = D;
  const int lo = blockIdx.y * L, po = (lo * D) / 2, Pg = g.P;
  const bool cgm = (mode == FIRST_CG || mode == FIRST_PROF);
  // strides of the row-pass buffer between positions and between packs
  const size_t lstr = g.pmaj ? 1 : (size_t)Pg, pstr = g.pmaj ? (size_t)g.N[0] * g.N[1] * M : 1;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_alpha[kMaxLoads];
  __shared__ int s_act[kMaxLoads];
  __shared__ double s_red[16];
  __shared__ RowInfo s_row[G];
  __shared__ CgScal s_sc[L];
  const UnitDev& U = units[blockIdx.z];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int N1 = g.N[1];
  const int it = (mode == FIRST_PROF) ? 1 : (iter_base ? (*iter_base + jstep) : 0);
  Cx<R>* tw = reinterpret_cast<Cx<R>*>(smem);                          // [M]
  Cx<R>* stage = reinterpret_cast<Cx<R>*>(smem + align16(M * sizeof(Cx<R>)));  // [2G][P][M]

  // CG scalars of the step: the states of the block's loads and the sums of the
  // <p, C p> partials of the last pass are read at once, ahead of the set-up
  double delta[L];
#pragma unroll
  for (int w = 0; w < L; ++w) delta[w] = 0.0;
  if (mode == FIRST_CG) {
    copy_states<L>(U.sc + lo, s_sc, tid, nthr);
    if (tid < 64) wave_sum_rows<L>(U.part_d + (size_t)lo * g.nbL, g.nbL, g.nbL, delta);
  }
  if (tid < G) row_info(g, blockIdx.x * G + tid, s_row[tid]);
  const Cx<R>* twg = reinterpret_cast<const Cx<R>*>(g.tw[2]);
  for (int i = tid; i < M; i += nthr) tw[i] = twg[i];
  for (int i = tid; i < 2 * G * P * M; i += nthr) stage[i] = rf::mk<R>(0, 0);
  __syncthreads();
  // alpha_{it-1} = gamma_{it-1} / delta_{it-1} per load, from the shared copy of
  // its state; block 0 records the step in the state itself
  if (tid < 64) {
    const int lane = tid;
#pragma unroll
    for (int w = 0; w < L; ++w) {
      int act = 1;
      double alpha = 0.0;
      if (mode == FIRST_CG) {
        const CgScal* sc = &s_sc[w];
        CgScal* out = (blockIdx.x == 0 && lane == 0) ? U.sc + lo + w : nullptr;
        act = (sc->status == 0);
        if (act && it > 0) {
          const double gam = sc->gamma[(it - 1) & 1];
          double den = delta[w];
          if (it > 1) den = delta[w] - sc->beta[(it - 1) & 1] * gam / sc->alpha[(it - 2) & 1];
          if (!(den > 0.0)) {
            act = 0;
            if (out) {
              out->status = -3;
              out->iters = it - 1;
              out->gamma_last = gam;
            }
          } else {
            alpha = gam / den;
            if (out) {
              out->alpha[(it - 1) & 1] = alpha;
              energy_record(sc, out, it - 1, alpha * gam);
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
        if (!cgm) {
          v = U.x[lo + l][idx];
        } else if (s_act[l]) {
          v = U.r[lo + l][idx];
          if (it > 0) {
            const double a = s_alpha[l];
            const Cx<double> xv = U.x[lo + l][idx], pv = U.p[lo + l][idx], sv = U.s[lo + l][idx];
            v = v - sv * a;
            gstore(U.x[lo + l], idx, xv + pv * a);
            gstore(U.r[lo + l], idx, v);
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
          if (mode == FIRST_BOUNDS && ri.self && k2 == 0) X[s].x += U.E[lo + lf][gam];
        }
      }
      sA[pk * M + posA] = rf::mk<R>((R)(X[0].x - X[1].y), (R)(X[0].y + X[1].x));
      if (!ri.self) sB[pk * M + posB] = rf::mk<R>((R)(X[0].x + X[1].y), (R)(-X[0].y + X[1].x));
    }
  }
  if (cgm) {
    for (int l = 0; l < L; ++l) {
      double v = l == 0 ? gp0 : (l == 1 ? gp1 : gp2);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
      if ((tid & 63) == 0) s_red[tid >> 6] = v;
      __syncthreads();
      if (tid == 0) {
        double s = 0.0;
        for (int i = 0; i < (nthr + 63) / 64; ++i) s += s_red[i];
        U.part_g[(size_t)(lo + l) * g.nbF + blockIdx.x] = s;
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
      for (int n1 = 0; n1 < A; ++n1) v[n1] = dead_row<M>(n1) ? rf::mk<R>(0, 0) : sp[B * n1 + q];
    }
    __syncthreads();
    if (live && q < B) {
      rf::Dft<R, A, 1>::template run_z<dead_mask<M>()>(v);
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
      if constexpr (D == 2) {
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2)
          gstore(out, (((size_t)i0 * N1 + i1) * M + (q + A * k2)) * lstr + (po + pk) * pstr, v[k2]);
      }
    }
    if constexpr (D == 3) {
      // the exchange of this pack has been read: its slots take the results, in position order
      __syncthreads();
      if (live && q < A) {
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) sp[q + A * k2] = v[k2];
      }
    }
  }
  if constexpr (D == 3) {
    // 3D buffers interleave the packs of a position ([N0][N1][M2][P]): a block writes each line's
    // positions with all their packs back to back, so every cache line is filled at once (pack by
    // pack, the partial lines were evicted between the packs and written about 1.6 times)
    __syncthreads();
    for (int t = tid; t < 2 * G * M; t += nthr) {
      const int ln = t / M, pos = t - ln * M;
      const RowInfo& rr = s_row[ln >> 1];
      const int lb = ln & 1;
      if (!rr.valid || (lb == 1 && rr.self)) continue;
      const int a0 = lb ? rr.i0B : rr.h0, a1 = lb ? rr.i1B : rr.i1A;
      const size_t base = (((size_t)a0 * N1 + a1) * M + pos) * lstr + po * pstr;
#pragma unroll
      for (int pk = 0; pk < P; ++pk) gstore(out, base + pk * pstr, stage[((size_t)ln * P + pk) * M + pos]);
    }
  }
  (void)H2;
}

template <typename R, int M, int D, int L, int DUAL, int G>
__global__ __launch_bounds__(256, D == 2 ? 6 : 1) void k_last_fast(Geo g, const UnitDev* __restrict__ units, int mode, int jstep,
                                                   const int* __restrict__ iter_base) {
  constexpr int A = Cfg<M>::A, B = Cfg<M>::B, T = Cfg<M>::T, N2 = Cfg<M>::N;
  constexpr int P = (L * D + 1) / 2, m = DUAL ? D - 1 : 1, d = D;
  const int lo = blockIdx.y * L, po = (lo * D) / 2, Pg = g.P;
  const bool cgm = (mode == LAST_CG || mode == LAST_PROF);
  const size_t lstr = g.pmaj ? 1 : (size_t)Pg, pstr = g.pmaj ? (size_t)g.N[0] * g.N[1] * M : 1;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_beta[kMaxLoads];
  __shared__ int s_act[kMaxLoads];
  __shared__ double s_red[16];
  __shared__ RowInfo s_row[G];
  __shared__ CgScal s_sc[L];
  const UnitDev& U = units[blockIdx.z];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int N1 = g.N[1];
  const int it = (mode == LAST_PROF) ? 1 : (iter_base ? (*iter_base + jstep) : 0);
  Cx<R>* tw = reinterpret_cast<Cx<R>*>(smem);                                   // [M]
  Cx<R>* stage = reinterpret_cast<Cx<R>*>(smem + align16(M * sizeof(Cx<R>)));  // [2G][P][M]

  // the states of the block's loads and the sums of the <r, r> partials of the
  // first pass, read at once
  double gsum[L];
#pragma unroll
  for (int w = 0; w < L; ++w) gsum[w] = 0.0;
  if (mode == LAST_CG) {
    copy_states<L>(U.sc + lo, s_sc, tid, nthr);
    if (tid < 64) wave_sum_rows<L>(U.part_g + (size_t)lo * g.nbF, g.nbF, g.nbF, gsum);
  }
  if (tid < G) row_info(g, blockIdx.x * G + tid, s_row[tid]);
  const Cx<R>* twg = reinterpret_cast<const Cx<R>*>(g.tw[2]);
  for (int i = tid; i < M; i += nthr) tw[i] = twg[i];
  __syncthreads();
  // convergence and beta_it per load, from the shared copy of its state; block 0
  // records them in the state itself
  if (tid < 64) {
    const int lane = tid;
#pragma unroll
    for (int w = 0; w < L; ++w) {
      int act = 1;
      double beta = 0.0;
      if (mode == LAST_CG) {
        const CgScal* sc = &s_sc[w];
        CgScal* out = (blockIdx.x == 0 && lane == 0) ? U.sc + lo + w : nullptr;
        act = (sc->status == 0);
        if (act) {
          const double gam = gsum[w];
          const bool bad = !(gam == gam) || gam > 1e300;
          const bool conv = stop_test(sc, out, it, gam);
          if (bad || conv || it >= sc->maxit) {
            act = 0;
            if (out) {
              out->status = bad ? -1 : (conv ? 1 : 2);
              out->iters = it;
              out->gamma_last = gam;
              if (it == 0) out->gamma0 = gam;
            }
          } else {
            beta = (it == 0) ? 0.0 : gam / sc->gamma[(it - 1) & 1];
            if (out) {
              out->gamma[it & 1] = gam;
              out->beta[it & 1] = beta;
              if (it == 0) out->gamma0 = gam;
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
      for (int pk = 0; pk < P; ++pk)
        v[pk][n2] = pick_load<D == 3>(in, (((size_t)i0 * N1 + i1) * M + (q + A * n2)) * lstr + (po + pk) * pstr);
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
      for (int m1 = 0; m1 < A; ++m1)
        if (!dead_row<M>(m1)) sp[q + B * m1] = v[pk][m1];
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
        if (cgm) {
          rv[c] = pick_load<D == 3>((const Cx<double>*)U.r[lo + l], idx);
          if (it > 0) {
            pv[c] = pick_load<D == 3>((const Cx<double>*)U.p[lo + l], idx);
            sv[c] = pick_load<D == 3>((const Cx<double>*)U.s[lo + l], idx);
          }
        } else if (mode == LAST_RESID) {
          bv[c] = pick_load<D == 3>((const Cx<double>*)U.b[lo + l], idx);
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
        if (cgm) {
          const double b = s_beta[l];
          if (it == 0) {
            gstore(U.p[lo + l], idx, rv[c]);
            gstore(U.s[lo + l], idx, w);
          } else {
            gstore(U.p[lo + l], idx, rv[c] + pv[c] * b);
            gstore(U.s[lo + l], idx, w + sv[c] * b);
          }
          e = wt * (rv[c].x * w.x + rv[c].y * w.y);
        } else if (mode == LAST_RESID) {
          const Cx<double> rn = bv[c] - w;
          gstore(U.r[lo + l], idx, rn);
          e = wt * (rn.x * rn.x + rn.y * rn.y);
        } else {
          gstore(U.s[lo + l], idx, w);
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
      gstore(U.part_d, (size_t)(lo + l) * g.nbL + blockIdx.x, s);
    }
    __syncthreads();
  }
}

// ============================================================== dispatch
// Candidate tile shapes per FFT length (the first entry is the default).
// Row passes: pairs per block (2 G T <= 256 threads); column pass: points per block.
// 2D column pass: (points per thread group, half exchange, all packs in one block).
struct ApC {
  int tp, hx, all;
};
constexpr int kAp2 = 6;  // column-pass candidates per length
template <int M>
struct Cands;
template <>
struct Cands<625> {
  static constexpr int NG = 3;
  static constexpr int G[3] = {2, 1, 4};
  static constexpr int TP[2] = {8, 4};
  static constexpr ApC AP2[6] = {{8, 0, 0}, {10, 1, 0}, {20, 1, 0}, {5, 1, 0}, {10, 1, 1}, {5, 1, 1}};
};
template <>
struct Cands<125> {
  static constexpr int NG = 3;
  static constexpr int G[3] = {4, 2, 1};
  static constexpr int TP[2] = {10, 5};
  static constexpr ApC AP2[6] = {{10, 0, 0}, {5, 0, 0}, {10, 1, 0}, {5, 1, 0}, {5, 0, 1}, {5, 1, 1}};
};
template <>
struct Cands<81> {
  static constexpr int NG = 4;
  static constexpr int G[4] = {14, 7, 4, 2};
  static constexpr int TP[2] = {28, 14};
  static constexpr ApC AP2[6] = {{28, 0, 0}, {14, 0, 0}, {28, 1, 0}, {14, 1, 0}, {14, 0, 1}, {14, 1, 1}};
};
template <>
struct Cands<25> {
  static constexpr int NG = 3;
  static constexpr int G[3] = {25, 12, 6};
  static constexpr int TP[2] = {51, 25};
  static constexpr ApC AP2[6] = {{51, 0, 0}, {25, 0, 0}, {51, 1, 0}, {25, 1, 0}, {25, 0, 1}, {25, 1, 1}};
};

static bool apply_supported(int M, int D, int P, int NC) {
  if (D == 2) return (M == 625 || M == 125 || M == 81 || M == 25) && (P == 1 || P == 2) && (NC == 1 || NC == 3);
  return M == 81 && (P == 2 || P == 3 || P == 5) && (NC == 1 || NC == 6);
}

// Whether (tp, hx) is a column-pass shape of the specialised kernels (0, 0: default).
bool fast_apply_shape_ok(int M, int D, int tp, int hx, int all) {
  if (tp == 0 && hx == 0 && all == 0) return true;
  auto in2 = [&](const ApC* c) {
    for (int i = 0; i < kAp2; ++i)
      if (c[i].tp == tp && c[i].hx == hx && c[i].all == all) return true;
    return false;
  };
  auto in3 = [&](const int* c) { return hx == 0 && all == 0 && (c[0] == tp || c[1] == tp); };
  switch (M) {
    case 625: return D == 2 ? in2(Cands<625>::AP2) : in3(Cands<625>::TP);
    case 125: return D == 2 ? in2(Cands<125>::AP2) : in3(Cands<125>::TP);
    case 81: return D == 2 ? in2(Cands<81>::AP2) : in3(Cands<81>::TP);
    case 25: return D == 2 ? in2(Cands<25>::AP2) : in3(Cands<25>::TP);
    default: return false;
  }
}

bool fast_apply_supported(int M, int D, int P, int NC) {
  return !std::getenv("HOM_NO_FAST") && apply_supported(M, D, P, NC);
}

static bool row_supported(int M, int D, int L) {
  if (D == 2) return (M == 625 || M == 125 || M == 81 || M == 25) && L >= 1 && L <= kMaxLoads;
  return M == 81 && L >= 1 && L <= 3;
}

template <int M>
static int pick(const int* c, int n, int req) {
  for (int i = 0; i < n; ++i)
    if (c[i] == req) return req;
  return c[0];
}

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

template <int M, int D, int P, int NC, int TP>
static hipError_t run_apply_tp(const Geo& g, const UnitDev* units, int n, int cg, hipStream_t st) {
  constexpr int T = Cfg<M>::T;
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

template <int M, int P, int NC, int TP, int HX, int ALL>
static hipError_t run_apply2_tp(const Geo& g, const UnitDev* units, int n, int cg, hipStream_t st) {
  constexpr int T = Cfg<M>::T, PB = ALL ? P : 1;
  const int npts = g.M[2];
  const size_t lds = (size_t)M * sizeof(Cx<float>) +
                     (size_t)PB * xarea<Cfg<M>::A, Cfg<M>::B, TP, HX>() * (HX ? sizeof(float) : sizeof(Cx<float>));
  auto kern = k_apply2_fast<float, M, P, NC, TP, HX, PB>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int nbx = (npts + TP - 1) / TP;
  const dim3 grid(8 * ((nbx + 7) / 8) * (P / PB), 1, n);
  if (g_ext_timing.on)
    hipExtLaunchKernelGGL(kern, grid, dim3(PB * TP * T), lds, st, g_ext_timing.start, g_ext_timing.stop, 0, g, units,
                          cg);
  else
    hipLaunchKernelGGL(kern, grid, dim3(PB * TP * T), lds, st, g, units, cg);
  return hipGetLastError();
}

template <int M, int P, int NC, int I = 0>
static hipError_t run_apply2(const Geo& g, const UnitDev* units, int n, int cg, hipStream_t st) {
  constexpr ApC c = Cands<M>::AP2[I];
  if (g.apTP == c.tp && g.apHX == c.hx && g.apAll == c.all)
    return run_apply2_tp<M, P, NC, c.tp, c.hx, c.all>(g, units, n, cg, st);
  if constexpr (I + 1 < kAp2) {
    return run_apply2<M, P, NC, I + 1>(g, units, n, cg, st);
  } else {
    constexpr ApC c0 = Cands<M>::AP2[0];  // default
    return run_apply2_tp<M, P, NC, c0.tp, c0.hx, c0.all>(g, units, n, cg, st);
  }
}

template <int M, int D, int P, int NC>
static hipError_t run_apply(const Geo& g, const UnitDev* units, int n, int cg, hipStream_t st) {
  if constexpr (D == 2) {
    return run_apply2<M, P, NC>(g, units, n, cg, st);
  } else {
    constexpr int TP0 = Cands<M>::TP[0], TP1 = Cands<M>::TP[1];
    if (g.apTP == TP1) return run_apply_tp<M, D, P, NC, TP1>(g, units, n, cg, st);
    return run_apply_tp<M, D, P, NC, TP0>(g, units, n, cg, st);
  }
}

// Returns true when a specialised column pass handled the launch (*err set).
bool fast_apply(const Geo& g, const UnitDev* units, int n, int cg, hipStream_t st, hipError_t* err) {
  if (std::getenv("HOM_NO_FAST")) return false;
  const int M = g.M[0], D = g.d, P = g.P, NC = g.nc;
  if (M != 2 * g.N[0] - 1) return false;  // the register transforms keep Z_N of the doubled grid
  if (!apply_supported(M, D, P, NC)) return false;
  // the 2D column pass addresses its buffers with 32-bit byte offsets
  if (D == 2 && ((size_t)g.N[0] * g.M[2] * P * sizeof(Cx<float>) >= (size_t(1) << 32) ||
                 (size_t)NC * M * g.M[2] * sizeof(float) >= (size_t(1) << 32)))
    return false;
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

// ============================================================== plane pass (3D)
// The middle and column passes of a 3D operator application in one kernel.  A
// block takes one plane m2 of a unit's row-pass buffer ([N0][N1][M2][P]) and,
// one pack at a time, runs the zero-padded inverse transform along axis 1, the
// inverse transform along axis 0, the product with the coefficient on the
// doubled grid (Sec. 4, the quadrature of the Ga scheme), the forward
// transform along axis 0 and the truncated forward transform along axis 1;
// the result replaces the plane in place, where the last pass reads it.
// Every transform is the one of the separate passes operation for operation,
// so both routes give the same bits; the intermediate N0 x M1 plane stays in
// LDS instead of making two round trips through HBM.  The coefficient comes
// from its copy in plane order [M2][nc][M0][M1].
//
// Each four-step transform belongs to T = 9 lanes of one wave (seven groups
// per wave, lane 63 idle), so its exchange needs no block barrier: a line's
// exchange runs in its own column of the plane, a column's in its wave's
// exchange area.  Block barriers only separate the line and column steps
// (two per pack).  Twelve waves give 84 groups, one per column of the plane
// in a single round (the 41 lines take the first six waves); at 96.6 KB of
// LDS one block fills a CU (twelve waves, three per SIMD).  With six waves
// two blocks would fit the LDS, but a second one was never resident beside
// the first: the twelve-wave block is the same occupancy with half the
// column rounds.  Workgroup x runs on XCD x % 8: each XCD takes a run of
// consecutive planes, whose rows share cache lines of the row-pass buffer in
// that XCD's L2.
constexpr int kPlaneThreads = 768;

template <int M>
struct PlaneShape {
  static constexpr int T = Cfg<M>::T, N = Cfg<M>::N;
  static constexpr int GW = 64 / T;                     // thread groups per wave
  static constexpr int NW = kPlaneThreads / 64;         // waves per block
  static constexpr int NG = GW * NW;                    // thread groups per block
  static constexpr int R = (M + NG - 1) / NG;           // rounds of the column step
  // slots per exchange row: GW groups, padded so that the writes of a half-wave (slot 9 q + k of
  // group g at 8-byte address EX (9 q + k) + g) fall on distinct banks but for pairs (EX = 7 gave
  // four-way conflicts)
  static constexpr int EX = GW + 2;
  static constexpr size_t lds = ((size_t)M * N + (size_t)NW * EX * M) * sizeof(Cx<float>);
};

// Order of the LDS accesses of one wave (lanes exchange through LDS without a block barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int M, int P>
__global__ __launch_bounds__(kPlaneThreads) void k_plane_fast(Geo g, const UnitDev* __restrict__ units, int cg) {
  using S = PlaneShape<M>;
  constexpr int A = Cfg<M>::A, B = Cfg<M>::B, T = S::T, N = S::N, GW = S::GW, NG = S::NG;
  constexpr int PPX = (M + 7) / 8;  // planes per XCD
  static_assert(A == T && B == T, "square four-step split");
  static_assert(N <= NG, "one thread group per line of the plane");
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<float>* Y = reinterpret_cast<Cx<float>*>(smem);    // [M1][N0] the plane after the axis-1 transform
  const UnitDev& U = units[blockIdx.z];
  if (cg && !any_active(U, g.L)) return;
  const int m2 = (int)(blockIdx.x & 7) * PPX + (int)(blockIdx.x >> 3);
  if (m2 >= M) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int gi = lane / T, q = lane - gi * T;
  const int grp = wave * GW + gi;                       // line i0 / first column of this thread group
  const bool gv = gi < GW;                              // lane 63 (and beyond 7 T) idle
  constexpr int EX = S::EX;
  Cx<float>* ex = Y + (size_t)M * N + (size_t)wave * EX * M;  // this wave's exchange area [M][EX]
  // the twiddles omega_M^(q k) of every four-step transform of this lane, k < T, in registers: both
  // axes have the same length, hence the same table (the separate passes read the same values)
  Cx<float> tw[T];
  {
    const Cx<float>* t0 = reinterpret_cast<const Cx<float>*>(g.tw[0]);
#pragma unroll
    for (int k = 0; k < T; ++k) tw[k] = gload(t0, (size_t)(gv ? q * k : 0));
  }
  Cx<float>* buf = reinterpret_cast<Cx<float>*>(U.bufA);
  const size_t W = (size_t)M * P;                  // elements per (i0, i1) row of the buffer
  const int fields = g.L * g.d;                    // fields past the last load's are padding
  const bool lt = gv && grp < N;                   // this group owns line i0 = grp
  // the plane's inputs for every pack: row i1 = kept(B n1 + q) of line i0
  Cx<float> in[A][P];
#pragma unroll
  for (int n1 = 0; n1 < A; ++n1) {
    const int i1 = (lt && !dead_row<M>(n1)) ? kept<M>(B * n1 + q) : -1;
#pragma unroll
    for (int pk = 0; pk < P; ++pk)
      in[n1][pk] = i1 >= 0 ? gload(buf, ((size_t)grp * N + i1) * W + (size_t)m2 * P + pk) : rf::mk<float>(0, 0);
  }
  // the coefficient at the spatial points m0 = q + A k2 of this group's columns (nc = 1)
  const float* cp = U.coefp + (size_t)m2 * M * M;  // [M0][M1] of this plane
  float a[S::R][B];
#pragma unroll
  for (int r = 0; r < S::R; ++r) {
    const int m1 = grp + r * NG;
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) a[r][k2] = (gv && m1 < M) ? gload(cp, (size_t)(q + A * k2) * M + m1) : 0.f;
  }
  __syncthreads();
#pragma unroll
  for (int pk = 0; pk < P; ++pk) {
    Cx<float> v[T];
    // (1) axis 1, inverse, zero-padded N1 -> M1 (the middle pass, INV); exchange in column i0 of Y
    if (lt) {
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) v[n1] = in[n1][pk];
      rf::Dft<float, A, 1>::template run_z<dead_mask<M>()>(v);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) {
        Cx<float> w = tw[k1];
        w.y = -w.y;
        Y[(q * A + k1) * N + grp] = rf::mul(v[k1], w);
      }
    }
    wave_sync();
    if (lt) {
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) v[n2] = Y[(n2 * A + q) * N + grp];
    }
    wave_sync();
    if (lt) {
      rf::Dft<float, B, 1>::run(v);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) Y[(q + A * k2) * N + grp] = v[k2];
    }
    __syncthreads();
    // (2) axis 0 on the columns m1 of the plane: inverse, coefficient, forward (the column pass)
    const bool f0 = 2 * pk < fields, f1 = 2 * pk + 1 < fields;
#pragma unroll
    for (int r = 0; r < S::R; ++r) {
      const int m1 = grp + r * NG;
      const bool ok = gv && m1 < M;
      if (ok) {
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) {
          const int i0 = !dead_row<M>(n1) ? kept<M>(B * n1 + q) : -1;
          v[n1] = i0 >= 0 ? Y[m1 * N + i0] : rf::mk<float>(0, 0);
        }
        rf::Dft<float, A, 1>::template run_z<dead_mask<M>()>(v);
#pragma unroll
        for (int k1 = 0; k1 < A; ++k1) {
          Cx<float> w = tw[k1];
          w.y = -w.y;
          ex[(q * A + k1) * EX + gi] = rf::mul(v[k1], w);
        }
      }
      wave_sync();
      if (ok) {
#pragma unroll
        for (int n2 = 0; n2 < B; ++n2) v[n2] = ex[(n2 * A + q) * EX + gi];
        rf::Dft<float, B, 1>::run(v);
        // spatial values at m0 = q + A k2
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) v[k2] = rf::mk<float>(f0 ? a[r][k2] * v[k2].x : 0.f, f1 ? a[r][k2] * v[k2].y : 0.f);
        rf::Dft<float, B, -1>::run(v);
      }
      wave_sync();
      if (ok) {
#pragma unroll
        for (int mm = 0; mm < B; ++mm) ex[(q * B + mm) * EX + gi] = rf::mul(v[mm], tw[mm]);
      }
      wave_sync();
      if (ok) {
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) v[n1] = ex[(n1 * B + q) * EX + gi];
        rf::Dft<float, A, -1>::run(v);
#pragma unroll
        for (int mm = 0; mm < A; ++mm) {
          if (dead_row<M>(mm)) continue;
          const int i0 = kept<M>(q + B * mm);
          if (i0 >= 0) Y[m1 * N + i0] = v[mm];
        }
      }
      wave_sync();
    }
    __syncthreads();
    // (3) axis 1, forward, truncated M1 -> N1 (the middle pass, forward), into the buffer
    if (lt) {
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) v[n2] = Y[(q + A * n2) * N + grp];
    }
    wave_sync();
    if (lt) {
      rf::Dft<float, B, -1>::run(v);
#pragma unroll
      for (int mm = 0; mm < B; ++mm) Y[(q * B + mm) * N + grp] = rf::mul(v[mm], tw[mm]);
    }
    wave_sync();
    if (lt) {
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) v[n1] = Y[(n1 * B + q) * N + grp];
      rf::Dft<float, A, -1>::run(v);
      // the result of position q + B mm takes the register of the consumed input of position B n1 + q
#pragma unroll
      for (int mm = 0; mm < A; ++mm) in[mm][pk] = v[mm];
    }
    wave_sync();
  }
  // every pack of an element in one run (the buffer interleaves the packs of a position)
  if (lt) {
#pragma unroll
    for (int mm = 0; mm < A; ++mm) {
      if (dead_row<M>(mm)) continue;
      const int i1 = kept<M>(q + B * mm);
      if (i1 >= 0) {
#pragma unroll
        for (int pk = 0; pk < P; ++pk) gstore(buf, ((size_t)grp * N + i1) * W + (size_t)m2 * P + pk, in[mm][pk]);
      }
    }
  }
}

template <int M, int P>
static hipError_t run_plane(const Geo& g, const UnitDev* units, int n, int cg, hipStream_t st) {
  constexpr size_t lds = PlaneShape<M>::lds;
  auto kern = k_plane_fast<M, P>;
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const dim3 grid(8 * ((M + 7) / 8), 1, n);
  if (g_ext_timing.on)
    hipExtLaunchKernelGGL(kern, grid, dim3(kPlaneThreads), lds, st, g_ext_timing.start, g_ext_timing.stop, 0, g, units,
                          cg);
  else
    hipLaunchKernelGGL(kern, grid, dim3(kPlaneThreads), lds, st, g, units, cg);
  return hipGetLastError();
}

bool fast_plane_supported(int d, const int* Mz, const int* Nz, int nc) {
  if (std::getenv("HOM_NO_FAST") || std::getenv("HOM_NO_PLANE")) return false;
  return d == 3 && nc == 1 && Mz[0] == 81 && Mz[1] == 81 && Mz[2] == 81 && Nz[0] == 41 && Nz[1] == 41 && Nz[2] == 41;
}

// The middle, column and middle passes of a 3D application as one plane pass
// (g.plane set); false when the geometry has no plane pass.
bool fast_plane(const Geo& g, const UnitDev* units, int n, int cg, hipStream_t st, hipError_t* err) {
  if (!g.plane || !fast_plane_supported(g.d, g.M, g.N, g.nc) || n < 1 || n > 65535) return false;
  switch (g.P) {
    case 2: *err = run_plane<81, 2>(g, units, n, cg, st); return true;
    case 3: *err = run_plane<81, 3>(g, units, n, cg, st); return true;
    case 5: *err = run_plane<81, 5>(g, units, n, cg, st); return true;
    default: return false;
  }
}

template <int M>
static int row_pairs_for(int requested) {
  return pick<M>(Cands<M>::G, Cands<M>::NG, requested);
}

// Row pairs per block of the specialised row passes, or 0 when no
// specialisation exists (then the generic passes run).
int fast_row_pairs(int M, int N, int D, int L, int requested) {
  if (std::getenv("HOM_NO_FAST")) return 0;
  if (M != 2 * N - 1) return 0;  // the register transforms keep Z_N of the doubled grid
  if (!row_supported(M, D, L)) return 0;
  if (M == 625) return row_pairs_for<625>(requested);
  if (M == 125) return row_pairs_for<125>(requested);
  if (M == 81) return row_pairs_for<81>(requested);
  return row_pairs_for<25>(requested);
}

// Threads per block of a row pass: the requested count when it is a multiple
// of 64 that covers the 2 G T threads of the FFT phase and is at most 256.
static int row_threads(int G, int T, int requested) {
  const int need = round64(2 * G * T);
  if (requested >= need && requested <= 256 && requested % 64 == 0) return requested;
  return need;
}

template <int M, int D, int L, int DUAL, int G>
static hipError_t run_row_g(bool first, const Geo& g, const UnitDev* units, int n, int mode, int jstep,
                            const int* iter_base, hipStream_t st) {
  constexpr int T = Cfg<M>::T, P = (L * D + 1) / 2;
  static_assert(2 * G * T <= 256, "row pass needs at most 256 threads");
  const int nb = (g.Q + G - 1) / G;
  const int thr = row_threads(G, T, g.rowThreads);
  const size_t lds = align16(M * sizeof(Cx<float>)) + (size_t)2 * G * P * M * sizeof(Cx<float>);
  const dim3 grid(nb, D == 2 ? g.L / L : 1, n);
  if (first)
    return launch_k(k_first_fast<float, M, D, L, DUAL, G>, grid, thr, lds, st, g, units, mode, jstep, iter_base);
  return launch_k(k_last_fast<float, M, D, L, DUAL, G>, grid, thr, lds, st, g, units, mode, jstep, iter_base);
}

template <int M, int D, int L, int DUAL>
static hipError_t run_row(bool first, const Geo& g, const UnitDev* units, int n, int mode, int jstep,
                          const int* iter_base, hipStream_t st) {
  constexpr int G0 = Cands<M>::G[0], G1 = Cands<M>::G[1], G2 = Cands<M>::G[2];
  const int G = row_pairs_for<M>(g.rowG);
  if (G == G1) return run_row_g<M, D, L, DUAL, G1>(first, g, units, n, mode, jstep, iter_base, st);
  if (G == G2) return run_row_g<M, D, L, DUAL, G2>(first, g, units, n, mode, jstep, iter_base, st);
  if constexpr (Cands<M>::NG > 3) {
    constexpr int G3 = Cands<M>::G[Cands<M>::NG > 3 ? 3 : 0];
    if (G == G3) return run_row_g<M, D, L, DUAL, G3>(first, g, units, n, mode, jstep, iter_base, st);
  }
  return run_row_g<M, D, L, DUAL, G0>(first, g, units, n, mode, jstep, iter_base, st);
}

template <int M, int D, int L>
static hipError_t run_row_d(bool first, const Geo& g, const UnitDev* units, int n, int mode, int jstep,
                            const int* iter_base, hipStream_t st) {
  return g.dual ? run_row<M, D, L, 1>(first, g, units, n, mode, jstep, iter_base, st)
                : run_row<M, D, L, 0>(first, g, units, n, mode, jstep, iter_base, st);
}

bool fast_row(bool first, const Geo& g, const UnitDev* units, int n, int mode, int jstep, const int* iter_base,
              hipStream_t st, hipError_t* err) {
  if (!fast_row_pairs(g.M[2], g.N[2], g.d, g.L, g.rowG)) return false;
  const int M = g.M[2], D = g.d, L = g.L;
  // 2D: one load per block (grid y = load); 3D: every load in one block
#define HOM_RW2(MM)                                                                     \
  if (M == MM && D == 2) {                                                             \
    *err = run_row_d<MM, 2, 1>(first, g, units, n, mode, jstep, iter_base, st);        \
    return true;                                                                       \
  }
#define HOM_RW3(MM, LL)                                                                 \
  if (M == MM && D == 3 && L == LL) {                                                  \
    *err = run_row_d<MM, 3, LL>(first, g, units, n, mode, jstep, iter_base, st);       \
    return true;                                                                       \
  }
  HOM_RW2(625) HOM_RW2(125) HOM_RW2(81) HOM_RW2(25)
  HOM_RW3(81, 1) HOM_RW3(81, 2) HOM_RW3(81, 3)
#undef HOM_RW2
#undef HOM_RW3
  return false;
}

// ============================================================== tile tuning
static hipError_t time_ms(hipStream_t st, int reps, float* ms, const std::function<hipError_t()>& body) {
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return e;
  }
  e = body();  // untimed: first-launch costs
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = body();
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  if (e == hipSuccess) *ms /= (float)reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e;
}

template <int M>
static hipError_t tune_m(const Geo& g0, const UnitDev* units, int n, hipStream_t st, int reps, Tuning* best) {
  constexpr int T = Cfg<M>::T;
  Tuning t = *best;
  int cand = 0;
  hipError_t e = hipSuccess;
  if (row_supported(M, g0.d, g0.L)) {
    double bms = 1e30;
    for (int gi = 0; gi < Cands<M>::NG && e == hipSuccess; ++gi) {
      const int G = Cands<M>::G[gi];
      const int base = round64(2 * G * T);
      for (int thr = base; thr <= 256 && e == hipSuccess; thr = (thr == 256 ? 512 : 256)) {
        Geo g = g0;
        g.rowG = G;
        g.rowThreads = thr;
        g.nbF = g.nbL = (g.Q + G - 1) / G;
        float ms = 0.f;
        e = time_ms(st, reps, &ms, [&]() -> hipError_t {
          hipError_t x = hipSuccess;
          if (!fast_row(true, g, units, n, FIRST_PROF, 0, nullptr, st, &x)) return hipErrorInvalidValue;
          if (x != hipSuccess) return x;
          if (!fast_row(false, g, units, n, LAST_PROF, 0, nullptr, st, &x)) return hipErrorInvalidValue;
          return x;
        });
        ++cand;
        if (e == hipSuccess && ms < bms) {
          bms = ms;
          t.rowG = G;
          t.rowThreads = thr;
          t.row_ms = ms;
        }
      }
    }
  }
  if (e == hipSuccess && apply_supported(M, g0.d, g0.P, g0.nc) && g0.M[0] == M) {
    double bms = 1e30;
    const int ncand = g0.d == 2 ? kAp2 : 2;
    // 2D: each candidate is timed after the row pass that writes its input (in the chosen row
    // shape), as in a solve; timed alone, the column pass finds its input in the caches and
    // ranks the shapes differently.  The row pass's own time is subtracted.
    const bool with_first = g0.d == 2 && row_supported(M, g0.d, g0.L) && t.rowG > 0;
    Geo gr = g0;
    float first_ms = 0.f;
    if (with_first) {
      gr.rowG = t.rowG;
      gr.rowThreads = t.rowThreads;
      gr.nbF = gr.nbL = (gr.Q + gr.rowG - 1) / gr.rowG;
      e = time_ms(st, reps, &first_ms, [&]() -> hipError_t {
        hipError_t x = hipSuccess;
        if (!fast_row(true, gr, units, n, FIRST_PROF, 0, nullptr, st, &x)) return hipErrorInvalidValue;
        return x;
      });
    }
    for (int ci = 0; ci < ncand && e == hipSuccess; ++ci) {
      Geo g = g0;
      g.apTP = g0.d == 2 ? Cands<M>::AP2[ci].tp : Cands<M>::TP[ci];
      g.apHX = g0.d == 2 ? Cands<M>::AP2[ci].hx : 0;
      g.apAll = g0.d == 2 ? Cands<M>::AP2[ci].all : 0;
      if (g.apAll && g0.P == 1) continue;  // one pack: same kernel as one pack per block
      float ms = 0.f;
      e = time_ms(st, reps, &ms, [&]() -> hipError_t {
        hipError_t x = hipSuccess;
        if (with_first && !fast_row(true, gr, units, n, FIRST_PROF, 0, nullptr, st, &x)) return hipErrorInvalidValue;
        if (x != hipSuccess) return x;
        if (!fast_apply(g, units, n, 0, st, &x)) return hipErrorInvalidValue;
        return x;
      });
      ms -= first_ms;
      ++cand;
      if (e == hipSuccess && ms < bms) {
        bms = ms;
        t.apTP = g.apTP;
        t.apHX = g.apHX;
        t.apAll = g.apAll;
        t.apply_ms = ms;
      }
    }
  }
  if (e == hipSuccess) {
    t.candidates = cand;
    *best = t;
  }
  return e;
}

hipError_t tune_fast(const Geo& g, const UnitDev* units, int n, hipStream_t st, int reps, Tuning* best) {
  if (std::getenv("HOM_NO_FAST")) return hipSuccess;
  const int M = g.M[2];
  if (g.M[0] != M) return hipSuccess;  // tuned shapes cover equal row and column lengths
  if (M != 2 * g.N[2] - 1 || g.M[0] != 2 * g.N[0] - 1) return hipSuccess;
  if (M == 625) return tune_m<625>(g, units, n, st, reps, best);
  if (M == 125) return tune_m<125>(g, units, n, st, reps, best);
  if (M == 81) return tune_m<81>(g, units, n, st, reps, best);
  if (M == 25) return tune_m<25>(g, units, n, st, reps, best);
  return hipSuccess;
}

}  // namespace hom
