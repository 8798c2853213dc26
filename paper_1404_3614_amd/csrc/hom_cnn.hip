// Surrogate network for the CG initial guess: a periodic U-Net in FP32 with
// hand-written forward and backward kernels, sequenced by a small native
// runtime (hom_unet_*).  The prediction only has to be cheap and close: it is
// projected onto E_N / J_N by the solver, so any output gives an admissible
// starting field and the bounds stay guaranteed.
//
// Tensors are [B][C][Z][H][W] (Z = 1 in 2D), FP32.  A "view" addresses the
// channel slice [off, off + C) of a buffer with Ctot channels, so skip
// connections are concatenated in place.
//
// Architecture (levels L, base width c, widths c_l = c 2^l, sizes s_0 = input,
// s_{l+1} = ceil(s_l / 2)):
//   encoder l < L-1: conv3(in_l -> c_l) relu, conv3(c_l -> c_l) relu = skip_l,
//                    in_{l+1} = avgpool2(skip_l) (periodic, ceil)
//   bottleneck     : conv3(in_{L-1} -> c_{L-1}) relu, conv3 relu = dec_{L-1}
//   decoder l      : up = nearest-upsample(dec_{l+1}) to s_l, conv3(c_{l+1} -> c_l) relu,
//                    concat [that, skip_l], conv3(2 c_l -> c_l) relu, conv3 relu = dec_l
//   head           : conv1(c_0 -> cout)
// Parameters: one flat FP32 array, per conv layer in this order w[cout][cin][taps]
// then b[cout] (taps = 3^d, row-major over (z, y, x) offsets -1..1).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/hom.h"
#include "hom_internal.hpp"

namespace hom {
namespace cnn {

struct View {
  float* p;
  int C, Ctot, off;
};

// ------------------------------------------------------------------ convolution
// out[b, off_o + co, q] = act( bias[co] + sum_ci sum_tap w[co, ci, tap] in[b, off_i + ci, q + tap] )
// with periodic neighbours, KS = 3 (or 1), as implicit GEMMs on the matrix cores:
// M = output channels, N = points, K = input channels x taps, FP32 operands and
// accumulation (v_mfma_f32_16x16x4f32; lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and holds D[4 (l / 16) + r][l % 16], r < 4).
constexpr int CT = 256;      // threads per block (4 waves)
constexpr int COT = 32;      // output channels per block
constexpr int CIC = 8;       // input channels per LDS stage (forward)
constexpr int WCI = 16;      // input channels per block (weight gradient)
constexpr int kWgradBlocks = 2048;      // weight-gradient blocks a layer aims for (chunks of point tiles)
constexpr int kMaxWgradChunks = 1024;   // weight-gradient partials per layer at most (summed in a fixed order)

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Point tile of a block: 128 points, 2D 16 x 8, 3D 8 x 4 x 4 (x fastest)
template <int D>
struct Tile {
  static constexpr int X = D == 2 ? 16 : 8, Y = D == 2 ? 8 : 4, Z = D == 2 ? 1 : 4;
  static constexpr int NP = X * Y * Z;
};

// Smallest s >= n with s = want (mod 32): LDS channel strides that spread the
// channels read by one half-wave over distinct banks.
constexpr int pad_to(int n, int want) { return n + (((want - n % 32) % 32) + 32) % 32; }

template <int D, int KS>
struct Halo {
  static constexpr int R = KS / 2;
  static constexpr int X = Tile<D>::X + 2 * R, Y = Tile<D>::Y + 2 * R, Z = D == 3 ? Tile<D>::Z + 2 * R : 1;
  static constexpr int N = X * Y * Z;
  static constexpr int TAPS = D == 3 ? KS * KS * KS : KS * KS;
};

// Packed weights of a convolution, in the order the forward kernel stages them:
// wp[co block][ci stage][tap][c][COT] = w[co][ci][tap] (co = COT block + j,
// ci = CIC stage + c), zero past Cout and Cin, so that a stage's weights are one
// contiguous run of TAPS CIC COT floats, copied to LDS without re-indexing.
constexpr int kMaxPack = 32;
static_assert(5 * 6 - 2 <= kMaxPack, "a U-Net of 6 levels has 28 convolutions");
struct PackEntry {
  size_t src, dst;      // offsets of w in the parameters and of its packed copy
  int co, ci, taps;     // as seen by the packed convolution
  int flip;             // 1: the adjoint, w'[co][ci][tap] = w[ci][co][taps - 1 - tap]
};
struct PackTable {
  int n;
  PackEntry e[kMaxPack];
};

__host__ __device__ inline size_t packed_floats(int co, int ci, int taps) {
  return (size_t)((co + COT - 1) / COT) * ((ci + CIC - 1) / CIC) * taps * CIC * COT;
}

// One layer per grid row.
__global__ void k_pack_w(const float* __restrict__ params, PackTable tab, float* __restrict__ wp) {
  const PackEntry e = tab.e[blockIdx.y];
  const int nst = (e.ci + CIC - 1) / CIC;
  const size_t n = packed_floats(e.co, e.ci, e.taps);
  for (unsigned t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const int j = t % COT;
    unsigned r = t / COT;
    const int c = r % CIC;
    r /= CIC;
    const int tap = r % (unsigned)e.taps;
    r /= (unsigned)e.taps;
    const int st = r % (unsigned)nst, cob = r / (unsigned)nst;
    const int co = cob * COT + j, ci = st * CIC + c;
    float v = 0.f;
    if (co < e.co && ci < e.ci)
      v = e.flip ? params[e.src + ((size_t)ci * e.co + co) * e.taps + (e.taps - 1 - tap)]
                 : params[e.src + ((size_t)co * e.ci + ci) * e.taps + tap];
    wp[e.dst + t] = v;
  }
}

// One stage of the forward convolution (the halo of CIC input channels and
// their packed weights), loaded into registers while the previous stage is
// multiplied, then stored to LDS: the global loads' latency hides behind the
// matrix-core work.  Thread t holds halo points t, t + CT, ... of every channel
// (the channel offset is the same for the whole block) and float4s t, t + CT,
// ... of the weights; both land in LDS as contiguous runs (no bank conflicts).
template <int D, int KS>
struct Stage {
  using H = Halo<D, KS>;
  static constexpr int NJ = (H::N + CT - 1) / CT;           // halo points per thread and channel
  static constexpr int WQ = H::TAPS * CIC * COT / 4;        // float4s of a stage's weights
  static constexpr int NW = (WQ + CT - 1) / CT;
  int goff[NJ];                                             // point offsets in a channel plane, -1 past the halo
  float h[CIC][NJ];
  float4 w[NW];

  __device__ __forceinline__ void init(int tx0, int ty0, int tz0, int Zs, int Hs, int Ws) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int r = (int)threadIdx.x + j * CT;
      const int hx = r % H::X, hy = (r / H::X) % H::Y, hz = r / (H::X * H::Y);
      const int gx = wrap(tx0 + hx - H::R, Ws), gy = wrap(ty0 + hy - H::R, Hs);
      const int gz = (D == 3) ? wrap(tz0 + hz - H::R, Zs) : 0;
      goff[j] = r < H::N ? (gz * Hs + gy) * Ws + gx : -1;
    }
  }

  // in_c: channel ci0 of the image; nvalid channels of the stage exist; ws: the stage's packed weights
  __device__ __forceinline__ void load(const float* __restrict__ in_c, size_t plane, int nvalid,
                                       const float4* __restrict__ ws) {
#pragma unroll
    for (int c = 0; c < CIC; ++c)
#pragma unroll
      for (int j = 0; j < NJ; ++j) h[c][j] = (c < nvalid && goff[j] >= 0) ? in_c[c * plane + goff[j]] : 0.f;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const int f = (int)threadIdx.x + i * CT;
      w[i] = (WQ % CT == 0 || f < WQ) ? ws[f] : float4{0.f, 0.f, 0.f, 0.f};
    }
  }

  template <int HS>
  __device__ __forceinline__ void store(float* s_in, float* s_w) const {
#pragma unroll
    for (int c = 0; c < CIC; ++c)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        if (goff[j] >= 0) s_in[c * HS + (int)threadIdx.x + j * CT] = h[c][j];
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      const int f = (int)threadIdx.x + i * CT;
      if (WQ % CT == 0 || f < WQ) {
        const int row = f / (COT / 4), co = (f % (COT / 4)) * 4;
        *reinterpret_cast<float4*>(s_w + row * COT + ((co + 16 * (row & 1)) & (COT - 1))) = w[i];
      }
    }
  }
};

template <int D>
__device__ __forceinline__ void tile_origin(int tile, int Hs, int Ws, int* tx0, int* ty0, int* tz0) {
  const int tiles_x = (Ws + Tile<D>::X - 1) / Tile<D>::X, tiles_y = (Hs + Tile<D>::Y - 1) / Tile<D>::Y;
  *tx0 = (tile % tiles_x) * Tile<D>::X;
  tile /= tiles_x;
  *ty0 = (tile % tiles_y) * Tile<D>::Y;
  *tz0 = (tile / tiles_y) * Tile<D>::Z;
}

// Forward convolution (also the data gradient with flipped, transposed weights),
// weights packed by k_pack_w.
// Block: 128 points x 32 output channels; wave w: points 32 w .. 32 w + 31 (two
// tiles of 16) x the 32 channels (two tiles of 16).  K runs tap-major over
// stages of CIC input channels, so the four k of an MFMA step share a tap.
// Split K: grid.y = co tiles x nsplit; split s of a block sums the input
// channels [s cps, (s + 1) cps).  With nsplit > 1 the block writes its raw
// partial sums to part[s][b][co][q] and k_splitk_sum adds the splits in a fixed
// order and applies the epilogue (bias, activation, accumulation).
template <int D, int KS>
__global__ __launch_bounds__(CT) void k_conv_fwd(const float* __restrict__ in, int Cin, int inCtot, int inOff,
                                                 const float* __restrict__ wp, const float* __restrict__ bias,
                                                 float* __restrict__ out, int Cout, int outCtot, int outOff, int Zs,
                                                 int Hs, int Ws, int relu, int accumulate, int cps,
                                                 float* __restrict__ part) {
  using H = Halo<D, KS>;
  constexpr int TX = Tile<D>::X, TY = Tile<D>::Y;
  constexpr int TAPS = H::TAPS;
  constexpr int HS = pad_to(H::N, 16);     // channel stride: lanes 16..31 read the next channel 16 banks away
  __shared__ float s_in[CIC * HS];
  // [tap][c][co]: rows of COT = 32 channels, odd rows rotated by 16 so that the
  // two rows read by a half-wave fall on different banks
  static_assert(COT == 32 && CIC % 2 == 0, "row swizzle");
  __shared__ __align__(16) float s_w[TAPS * CIC * COT];
  int tx0, ty0, tz0;
  tile_origin<D>(blockIdx.x, Hs, Ws, &tx0, &ty0, &tz0);
  const int cot = (Cout + COT - 1) / COT;
  const int split = blockIdx.y / cot;
  const int co0 = (blockIdx.y - split * cot) * COT;
  const int ci_lo = split * cps, ci_hi = min(Cin, ci_lo + cps);
  const int b = blockIdx.z;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lk = lane >> 4, ln = lane & 15;
  const size_t plane = (size_t)Zs * Hs * Ws;
  const int wo0 = (ln + 16 * (lk & 1)) & (COT - 1), wo1 = wo0 ^ 16;   // swizzled channels ln, ln + 16
  // the two points of this lane (one per point tile of the wave), as halo offsets of their centres
  int hoff[2];
#pragma unroll
  for (int pt = 0; pt < 2; ++pt) {
    const int p = wave * 32 + pt * 16 + ln;
    const int px = p % TX, py = (p / TX) % TY, pz = p / (TX * TY);
    hoff[pt] = (pz * H::Y + py) * H::X + px;
  }
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  // ci_lo is a multiple of CIC: stage s of the packed weights holds channels [s CIC, (s + 1) CIC)
  const float* in_b = in + ((size_t)b * inCtot + inOff) * plane;
  const float4* w_blk = reinterpret_cast<const float4*>(wp) +
                        (size_t)(co0 / COT) * ((Cin + CIC - 1) / CIC) * (Stage<D, KS>::WQ);
  Stage<D, KS> stg;
  stg.init(tx0, ty0, tz0, Zs, Hs, Ws);
  if (ci_lo < ci_hi) stg.load(in_b + (size_t)ci_lo * plane, plane, ci_hi - ci_lo, w_blk + (size_t)(ci_lo / CIC) * Stage<D, KS>::WQ);
  for (int ci0 = ci_lo; ci0 < ci_hi; ci0 += CIC) {
    __syncthreads();                       // the previous stage's reads of LDS are done
    stg.template store<HS>(s_in, s_w);
    __syncthreads();
    const int nx = ci0 + CIC;
    if (nx < ci_hi)                        // the next stage's loads fly during this stage's products
      stg.load(in_b + (size_t)nx * plane, plane, ci_hi - nx, w_blk + (size_t)(nx / CIC) * Stage<D, KS>::WQ);
#pragma unroll 3
    for (int tap = 0; tap < TAPS; ++tap) {
      const int kx = tap % KS, ky = (tap / KS) % KS, kz = tap / (KS * KS);
      const int toff = (kz * H::Y + ky) * H::X + kx;
#pragma unroll
      for (int c0 = 0; c0 < CIC; c0 += 4) {
        const int c = c0 + lk;
        const float* wr = s_w + (tap * CIC + c) * COT;
        const float a0 = wr[wo0], a1 = wr[wo1];
        const float* ir = s_in + c * HS + toff;
        const float b0 = ir[hoff[0]], b1 = ir[hoff[1]];
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int pt = 0; pt < 2; ++pt) {
    const int p = wave * 32 + pt * 16 + ln;
    const int gx = tx0 + p % TX, gy = ty0 + (p / TX) % TY, gz = tz0 + p / (TX * TY);
    if (gx >= Ws || gy >= Hs || gz >= Zs) continue;
    const size_t q = ((size_t)gz * Hs + gy) * Ws + gx;
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int co = co0 + ct * 16 + 4 * lk + r;
        if (co >= Cout) continue;
        if (part) {
          part[(((size_t)split * gridDim.z + b) * Cout + co) * plane + q] = acc[ct][pt][r];
          continue;
        }
        float v = acc[ct][pt][r] + (bias ? bias[co] : 0.f);
        if (relu) v = fmaxf(v, 0.f);
        float* o = out + ((size_t)b * outCtot + outOff + co) * plane + q;
        if (accumulate) v += *o;
        *o = v;
      }
  }
}

// Sum of the split-K partials in split order, then the epilogue of k_conv_fwd.
__global__ void k_splitk_sum(const float* __restrict__ part, int nsplit, int B, int Cout, size_t plane,
                             const float* __restrict__ bias, float* __restrict__ out, int outCtot, int outOff, int relu,
                             int accumulate) {
  const size_t n = (size_t)B * Cout * plane;
  const int npl = (int)plane;
  for (int bc = blockIdx.y; bc < B * Cout; bc += gridDim.y) {
    const int b = bc / Cout, co = bc - b * Cout;
    const float* pp = part + (size_t)bc * plane;
    float* o = out + ((size_t)b * outCtot + outOff + co) * plane;
    const float bv = bias ? bias[co] : 0.f;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < npl; q += gridDim.x * blockDim.x) {
      float v = 0.f;
      for (int s = 0; s < nsplit; ++s) v += pp[(size_t)s * n + q];
      v += bv;
      if (relu) v = fmaxf(v, 0.f);
      if (accumulate) v += o[q];
      o[q] = v;
    }
  }
}

// One point tile of the weight gradient (the halo of WCI input channels and the
// output gradient of COT channels at the tile's points), loaded into registers
// while the previous tile is multiplied, then stored to LDS.  Thread t holds
// halo points t, t + CT, ... of every channel and point t % NP of channels
// t / NP + i CT / NP of the gradient; channel offsets are the same for the
// whole block.
template <int D, int KS>
struct WStage {
  using H = Halo<D, KS>;
  static constexpr int NP = Tile<D>::NP;
  static_assert(CT % NP == 0, "whole gradient rows per pass");
  static constexpr int NJ = (H::N + CT - 1) / CT;
  static constexpr int NG = COT * NP / CT;
  int b;
  int goff[NJ];   // halo point offsets in a channel plane, -1 past the halo
  int gq;         // this thread's tile point in a channel plane, -1 outside the grid
  float h[WCI][NJ];
  float gv[NG];

  __device__ __forceinline__ void init(int tile, int tiles_img, int Zs, int Hs, int Ws) {
    b = tile / tiles_img;
    int tx0, ty0, tz0;
    tile_origin<D>(tile - b * tiles_img, Hs, Ws, &tx0, &ty0, &tz0);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int r = (int)threadIdx.x + j * CT;
      const int hx = r % H::X, hy = (r / H::X) % H::Y, hz = r / (H::X * H::Y);
      const int gx = wrap(tx0 + hx - H::R, Ws), gy = wrap(ty0 + hy - H::R, Hs);
      const int gz = (D == 3) ? wrap(tz0 + hz - H::R, Zs) : 0;
      goff[j] = r < H::N ? (gz * Hs + gy) * Ws + gx : -1;
    }
    const int p = (int)threadIdx.x % NP;
    const int gx = tx0 + p % Tile<D>::X, gy = ty0 + (p / Tile<D>::X) % Tile<D>::Y, gz = tz0 + p / (Tile<D>::X * Tile<D>::Y);
    gq = (gx < Ws && gy < Hs && gz < Zs) ? (gz * Hs + gy) * Ws + gx : -1;
  }

  // in_c: channel ci0 of image b (nci channels exist); g_c: channel co0 of image b (nco exist)
  __device__ __forceinline__ void load(const float* __restrict__ in_c, int nci, const float* __restrict__ g_c, int nco,
                                       size_t plane) {
#pragma unroll
    for (int c = 0; c < WCI; ++c)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        h[c][j] = (c < nci && goff[j] >= 0) ? in_c[(unsigned)c * (unsigned)plane + (unsigned)goff[j]] : 0.f;
    const int co_t = (int)threadIdx.x / NP;
    const unsigned gbase = (unsigned)co_t * (unsigned)plane + (unsigned)gq;
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const int co = co_t + i * (CT / NP);
      gv[i] = (co < nco && gq >= 0) ? g_c[gbase + (unsigned)(i * (CT / NP)) * (unsigned)plane] : 0.f;
    }
  }

  template <int HS, int PS>
  __device__ __forceinline__ void store(float* s_in, float* s_g) const {
#pragma unroll
    for (int c = 0; c < WCI; ++c)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        if (goff[j] >= 0) s_in[c * HS + (int)threadIdx.x + j * CT] = h[c][j];
    const int co_t = (int)threadIdx.x / NP, p = (int)threadIdx.x % NP;
#pragma unroll
    for (int i = 0; i < NG; ++i) s_g[(co_t + i * (CT / NP)) * PS + p] = gv[i];
  }
};

// Weight gradient partials: dW[co][ci][tap] = sum over points q of
// g[co, q] in[ci, q + tap], as GEMMs with M = output channels, N = input
// channels (WCI per block), K = points, one per tap.  Block (chunk, co tile,
// ci tile) sums the point tiles tile0 .. tile1 of the whole batch (b-major)
// and writes part[chunk][co][ci][tap]; the chunks are summed in a fixed order
// later.  The 2 x TAPS output tiles (co half, tap) of a block are dealt to
// the 4 waves in turn.
template <int D, int KS>
__global__ __launch_bounds__(CT) void k_conv_wgrad(const float* __restrict__ in, int Cin, int inCtot, int inOff,
                                                   const float* __restrict__ g, int Cout, int gCtot, int gOff, int Zs,
                                                   int Hs, int Ws, int ntiles, int per_chunk, float* __restrict__ part) {
  using H = Halo<D, KS>;
  constexpr int TX = Tile<D>::X, TY = Tile<D>::Y, NP = Tile<D>::NP;
  constexpr int TAPS = H::TAPS;
  constexpr int HS = pad_to(H::N, 2);      // channel stride: the 16 channels of a k row on even banks, the next point odd
  constexpr int PS = pad_to(NP, 2);        // point stride of s_g: a half-wave reads 16 channels x 2 points conflict-free
  constexpr int NT = 2 * TAPS;             // output tiles (co half, tap)
  constexpr int TPW = (NT + 3) / 4;        // tiles per wave
  __shared__ float s_in[WCI * HS];
  __shared__ float s_g[COT * PS];          // [co][point]
  const int co0 = blockIdx.y * COT, ci0 = blockIdx.z * WCI;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lk = lane >> 4, ln = lane & 15;
  const size_t plane = (size_t)Zs * Hs * Ws;
  const int tiles_img = ((Ws + TX - 1) / TX) * ((Hs + TY - 1) / TY) * ((Zs + Tile<D>::Z - 1) / Tile<D>::Z);
  v4f acc[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) acc[i] = v4f{0.f, 0.f, 0.f, 0.f};
  const int t0 = blockIdx.x * per_chunk, t1 = min(t0 + per_chunk, ntiles);
  const int nci = min(WCI, Cin - ci0), nco = min(COT, Cout - co0);
  WStage<D, KS> stg;
  auto fetch = [&](int tile) {
    stg.init(tile, tiles_img, Zs, Hs, Ws);
    stg.load(in + ((size_t)stg.b * inCtot + inOff + ci0) * plane, nci,
             g + ((size_t)stg.b * gCtot + gOff + co0) * plane, nco, plane);
  };
  if (t0 < t1) fetch(t0);
  for (int tt = t0; tt < t1; ++tt) {
    __syncthreads();                       // the previous tile's reads of LDS are done
    stg.template store<HS, PS>(s_in, s_g);
    __syncthreads();
    if (tt + 1 < t1) fetch(tt + 1);        // the next tile's loads fly during this tile's products
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int j = wave + 4 * i;
      if (j >= NT) break;
      const int ct = j & 1, tap = j >> 1;
      const int kx = tap % KS, ky = (tap / KS) % KS, kz = tap / (KS * KS);
      const int toff = (kz * H::Y + ky) * H::X + kx;
#pragma unroll 4
      for (int k0 = 0; k0 < NP; k0 += 4) {
        const int p = k0 + lk;
        const int px = p % TX, py = (p / TX) % TY, pz = p / (TX * TY);
        const float a = s_g[(ct * 16 + ln) * PS + p];
        const float bv = s_in[ln * HS + (pz * H::Y + py) * H::X + px + toff];
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc[i], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int j = wave + 4 * i;
    if (j >= NT) break;
    const int ct = j & 1, tap = j >> 1;
    const int ci = ci0 + ln;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int co = co0 + ct * 16 + 4 * lk + r;
      if (co < Cout && ci < Cin) part[(((size_t)blockIdx.x * Cout + co) * Cin + ci) * TAPS + tap] = acc[i][r];
    }
  }
}

// Fixed-order sum of partials.  Block (x, s) covers the 64 values t in
// [64 x, 64 x + 64) and the chunks [s cs, min((s + 1) cs, nchunk)) of part[c][t]
// (n values per chunk); wave w sums the w-th quarter of those chunks in order,
// and the four quarters are added in order.  The result is added to dst[t]
// (accumulate) or written to dst[s n + t] (the partials of a second pass).
constexpr int kSumLanes = 64;
__global__ __launch_bounds__(CT) void k_sum_chunks(const float* __restrict__ part, int nchunk, int cs, size_t n,
                                                   float* __restrict__ dst, int accumulate) {
  __shared__ float red[CT / 64][kSumLanes];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const size_t t = (size_t)blockIdx.x * kSumLanes + lane;
  const int c_lo = blockIdx.y * cs, len = min(cs, nchunk - c_lo);
  const int q = (len + 3) / 4;
  const int a = c_lo + min(len, wave * q), e = c_lo + min(len, (wave + 1) * q);
  float sum = 0.f;
  if (t < n) {
    const float* p = part + t;
    int c = a;
    for (; c + 8 <= e; c += 8) {
      float v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = p[(size_t)(c + k) * n];
#pragma unroll
      for (int k = 0; k < 8; ++k) sum += v[k];
    }
    for (; c < e; ++c) sum += p[(size_t)c * n];
  }
  red[wave][lane] = sum;
  __syncthreads();
  if (wave == 0 && t < n) {
    const float v = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
    if (accumulate)
      dst[t] += v;
    else
      dst[(size_t)blockIdx.y * n + t] = v;
  }
}

// Bias gradient partials: bpart[s][co] = sum of g[b, co, q] over every image b
// and the points q of segment s (len consecutive points of a plane), in a fixed
// order; k_sum_chunks then adds the segments in order.  Grid (segments, Cout).
__global__ void k_bias_part(const float* __restrict__ g, int Cout, int gCtot, int gOff, size_t plane, int B,
                            int len, float* __restrict__ bpart) {
  __shared__ float red[CT];
  const int co = blockIdx.y;
  const int q0 = blockIdx.x * len, q1 = min((int)plane, q0 + len);
  float s = 0.f;
  for (int b = 0; b < B; ++b) {
    const float* gp = g + ((size_t)b * gCtot + gOff + co) * plane;
    for (int q = q0 + (int)threadIdx.x; q < q1; q += CT) s += gp[q];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = CT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) bpart[(size_t)blockIdx.x * Cout + co] = red[0];
}

// g <- g * (y > 0) on a view (relu derivative; y is the relu output)
__global__ void k_relu_mask(float* g, const float* y, int C, int gCtot, int gOff, int yCtot, int yOff, size_t plane,
                            int B) {
  const int npl = (int)plane;
  for (int bc = blockIdx.y; bc < B * C; bc += gridDim.y) {
    const int b = bc / C, c = bc - b * C;
    const float* yp = y + ((size_t)b * yCtot + yOff + c) * plane;
    float* gp = g + ((size_t)b * gCtot + gOff + c) * plane;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < npl; q += gridDim.x * blockDim.x)
      if (!(yp[q] > 0.f)) gp[q] = 0.f;
  }
}

// 2x2(x2) periodic average pooling with ceil sizes; output point j covers inputs (2j + o) mod n.
template <int D>
__global__ void k_pool(const float* __restrict__ in, int inCtot, int inOff, float* __restrict__ out, int outCtot,
                       int outOff, int C, int Z, int H, int W, int Zo, int Ho, int Wo, int B) {
  const float sc = D == 3 ? 0.125f : 0.25f;
  const int npo = Zo * Ho * Wo;
  for (int bc = blockIdx.y; bc < B * C; bc += gridDim.y) {
    const int b = bc / C, c = bc - b * C;
    const float* src = in + ((size_t)b * inCtot + inOff + c) * ((size_t)Z * H * W);
    float* dst = out + ((size_t)b * outCtot + outOff + c) * (size_t)npo;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < npo; q += gridDim.x * blockDim.x) {
      const int x = q % Wo, y = (q / Wo) % Ho, z = q / (Wo * Ho);
      float s = 0.f;
      for (int dz = 0; dz < (D == 3 ? 2 : 1); ++dz)
        for (int dy = 0; dy < 2; ++dy)
          for (int dx = 0; dx < 2; ++dx) {
            const int gz = D == 3 ? (2 * z + dz) % Z : 0;
            s += src[((size_t)gz * H + (2 * y + dy) % H) * W + (2 * x + dx) % W];
          }
      dst[q] = s * sc;
    }
  }
}

// adjoint of k_pool, accumulated into gin: gin[q] += sc * sum over outputs covering q
template <int D>
__global__ void k_pool_bwd(const float* __restrict__ gout, int goCtot, int goOff, float* __restrict__ gin,
                           int giCtot, int giOff, int C, int Z, int H, int W, int Zo, int Ho, int Wo, int B) {
  const float sc = D == 3 ? 0.125f : 0.25f;
  const int npi = Z * H * W;
  // output indices j along an axis of length nn (ceil(nn/2) outputs) covering input i
  auto cands = [](int i, int nn, int no, int* js) {
    int k = 0;
    js[k++] = i / 2;
    if ((nn & 1) && i == 0) js[k++] = no - 1;
    return k;
  };
  for (int bc = blockIdx.y; bc < B * C; bc += gridDim.y) {
    const int b = bc / C, c = bc - b * C;
    const float* g = gout + ((size_t)b * goCtot + goOff + c) * ((size_t)Zo * Ho * Wo);
    float* dst = gin + ((size_t)b * giCtot + giOff + c) * (size_t)npi;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < npi; q += gridDim.x * blockDim.x) {
      const int x = q % W, y = (q / W) % H, z = q / (W * H);
      int jx[2], jy[2], jz[2] = {0, 0};
      const int nx = cands(x, W, Wo, jx), ny = cands(y, H, Ho, jy);
      const int nz = D == 3 ? cands(z, Z, Zo, jz) : 1;
      float s = 0.f;
      for (int a = 0; a < nz; ++a)
        for (int bq = 0; bq < ny; ++bq)
          for (int e = 0; e < nx; ++e) s += g[((size_t)jz[a] * Ho + jy[bq]) * Wo + jx[e]];
      dst[q] += s * sc;
    }
  }
}

// nearest upsampling to (Z, H, W): out[q] = in[q / 2]
template <int D>
__global__ void k_up(const float* __restrict__ in, int inCtot, int inOff, float* __restrict__ out, int outCtot,
                     int outOff, int C, int Zi, int Hi, int Wi, int Z, int H, int W, int B) {
  const int npo = Z * H * W;
  for (int bc = blockIdx.y; bc < B * C; bc += gridDim.y) {
    const int b = bc / C, c = bc - b * C;
    const float* src = in + ((size_t)b * inCtot + inOff + c) * ((size_t)Zi * Hi * Wi);
    float* dst = out + ((size_t)b * outCtot + outOff + c) * (size_t)npo;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < npo; q += gridDim.x * blockDim.x) {
      const int x = q % W, y = (q / W) % H, z = q / (W * H);
      const int zi = D == 3 ? z / 2 : 0;
      dst[q] = src[(zi * Hi + y / 2) * Wi + x / 2];
    }
  }
}

// adjoint of k_up: gin[j] = sum of gout over the (up to 2^d) outputs mapping to j
template <int D>
__global__ void k_up_bwd(const float* __restrict__ gout, int goCtot, int goOff, float* __restrict__ gin, int giCtot,
                         int giOff, int C, int Zi, int Hi, int Wi, int Z, int H, int W, int B) {
  const int npi = Zi * Hi * Wi;
  for (int bc = blockIdx.y; bc < B * C; bc += gridDim.y) {
    const int b = bc / C, c = bc - b * C;
    const float* g = gout + ((size_t)b * goCtot + goOff + c) * ((size_t)Z * H * W);
    float* dst = gin + ((size_t)b * giCtot + giOff + c) * (size_t)npi;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < npi; q += gridDim.x * blockDim.x) {
      const int x = q % Wi, y = (q / Wi) % Hi, z = q / (Wi * Hi);
      float s = 0.f;
      for (int dz = 0; dz < (D == 3 ? 2 : 1); ++dz)
        for (int dy = 0; dy < 2; ++dy)
          for (int dx = 0; dx < 2; ++dx) {
            const int oz = D == 3 ? 2 * z + dz : 0, oy = 2 * y + dy, ox = 2 * x + dx;
            if (oz < Z && oy < H && ox < W) s += g[(oz * H + oy) * W + ox];
          }
      dst[q] = s;
    }
  }
}

// (Weighted) MSE: partial sums of w (o - t)^2 per block, gradient 2 w (o - t) / n.
// Element i = ((b * cout + c) * plane + q) takes weight channel c * wch / cout of
// weight[b][wch][plane]; weight == nullptr means w = 1.
__global__ void k_mse(const float* __restrict__ o, const float* __restrict__ t, size_t n, const float* __restrict__ weight,
                      int wch, int cout, size_t plane, float* __restrict__ grad, double* __restrict__ part) {
  __shared__ double red[CT];
  double s = 0.0;
  const float sc = 2.0f / (float)n;
  for (size_t i = blockIdx.x * (size_t)CT + threadIdx.x; i < n; i += (size_t)gridDim.x * CT) {
    const float dv = o[i] - t[i];
    float w = 1.f;
    if (weight) {
      const size_t q = i % plane, r = i / plane;
      const int c = (int)(r % cout);
      const size_t b = r / cout;
      w = weight[(b * wch + (size_t)c * wch / cout) * plane + q];
    }
    s += (double)w * dv * dv;
    if (grad) grad[i] = sc * w * dv;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = CT / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, size_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float gv = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gv;
    const float b = b2 * m2[i] + (1.f - b2) * gv * gv;
    m1[i] = a;
    m2[i] = b;
    p[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
  }
}

__global__ void k_fill(float* p, size_t n, float v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

static int gridn(size_t n) {
  size_t b = (n + CT - 1) / CT;
  return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

// Grid of the per-plane elementwise kernels: x over the points of a plane, y over the planes.
static dim3 plane_grid(size_t pts, int planes) {
  const size_t bx = std::max<size_t>(1, std::min<size_t>((pts + CT - 1) / CT, 1024));
  return dim3((unsigned)bx, (unsigned)std::max(1, std::min(planes, 65535)));
}

// ------------------------------------------------------------------ runtime
struct Conv {
  int cin, cout, ks;
  size_t w, b;          // offsets into the parameter array
  size_t pk, pkf;       // offsets of the packed weights and of the packed adjoint weights
  int lvl;              // spatial level of input and output
  View in, out;         // activations
  View gin, gout;       // gradients
  bool relu;
  bool accumulate_gin;  // gradient of the input is shared with another consumer
};

struct Net {
  hom_unet_desc desc;
  hipStream_t st;
  float* params;
  float* grads;
  float* m1;
  float* m2;
  size_t nparams;
  char* work;
  size_t work_bytes;
  int levels;
  int sz[8][3];         // per level (Z, H, W)
  std::vector<Conv> convs;
  // buffers per level (activations and gradients)
  float* in0;           // input copy
  float* out;           // network output
  float* gout;          // gradient of the output
  float* wpk;           // packed weights of every layer (k_pack_w), refreshed by each forward
  float* wpkf;          // packed adjoint weights (data gradients), refreshed by each backward
  PackTable fwd_pack, bwd_pack;
  size_t pack_max;      // largest packed layer (floats)
  float* wpart;         // weight-gradient partials
  float* bpart;         // bias-gradient partials
  float* rpart;         // second-level partials of the fixed-order sums
  float* tgt;           // loss targets gathered from sample pointers [batch][cout][plane]
  float* spart;         // split-K partial sums of the forward convolutions
  size_t spart_floats;
  float* wgt;           // loss weights gathered from sample pointers [batch][cout][plane]
  size_t wpart_floats;
  double* lpart;        // loss partials
  std::vector<float*> act_bufs;
  // views for the non-conv ops
  struct Pool { View in, out, gin, gout; int lvl; };
  struct Up { View in, out, gin, gout; int lvl; };
  std::vector<Pool> pools;
  std::vector<Up> ups;
};

static size_t plane(const Net& n, int l) { return (size_t)n.sz[l][0] * n.sz[l][1] * n.sz[l][2]; }

// point tiles of one image at level l
static int tiles_at(const Net& n, int l) {
  if (n.desc.d == 3)
    return ((n.sz[l][2] + Tile<3>::X - 1) / Tile<3>::X) * ((n.sz[l][1] + Tile<3>::Y - 1) / Tile<3>::Y) *
           ((n.sz[l][0] + Tile<3>::Z - 1) / Tile<3>::Z);
  return ((n.sz[l][2] + Tile<2>::X - 1) / Tile<2>::X) * ((n.sz[l][1] + Tile<2>::Y - 1) / Tile<2>::Y);
}

// Chunks of point tiles of a weight gradient: about kWgradBlocks blocks in all,
// at most kMaxWgradChunks partials, none empty.
static void wgrad_chunks(const Net& n, const Conv& c, int* nchunk, int* per_chunk) {
  const int ntiles = tiles_at(n, c.lvl) * n.desc.batch;
  const int blocks = ((c.cout + COT - 1) / COT) * ((c.cin + WCI - 1) / WCI);
  int want = (kWgradBlocks + blocks - 1) / blocks;
  want = std::max(1, std::min(std::min(want, kMaxWgradChunks), ntiles));
  *per_chunk = (ntiles + want - 1) / want;
  *nchunk = (ntiles + *per_chunk - 1) / *per_chunk;
}

// Chunks per segment of a fixed-order sum of nchunk partials of n values: about
// 2048 blocks in all, at least 8 chunks per segment, the segments' partials
// within kRpartFloats.
constexpr size_t kRpartFloats = 1 << 18;
static int sum_segment_chunks(int nchunk, size_t n) {
  const size_t bx = (n + kSumLanes - 1) / kSumLanes;
  size_t ns = bx >= 2048 ? 1 : (2048 + bx - 1) / bx;
  ns = std::min(ns, (size_t)(nchunk + 7) / 8);
  ns = std::min(ns, kRpartFloats / n);
  ns = std::max<size_t>(ns, 1);
  const int cs = (int)((nchunk + ns - 1) / ns);
  return cs;
}

// grad[t] += sum over c < nchunk of part[c n + t], in a fixed order.
static void sum_partials(const Net& n, const float* part, int nchunk, size_t nv, float* grad) {
  const int cs = sum_segment_chunks(nchunk, nv), ns = (nchunk + cs - 1) / cs;
  const int bx = (int)((nv + kSumLanes - 1) / kSumLanes);
  if (ns == 1) {
    hipLaunchKernelGGL(k_sum_chunks, dim3(bx, 1), dim3(CT), 0, n.st, part, nchunk, cs, nv, grad, 1);
    return;
  }
  hipLaunchKernelGGL(k_sum_chunks, dim3(bx, ns), dim3(CT), 0, n.st, part, nchunk, cs, nv, n.rpart, 0);
  hipLaunchKernelGGL(k_sum_chunks, dim3(bx, 1), dim3(CT), 0, n.st, n.rpart, ns, ns, nv, grad, 1);
}

// Segments of a plane for a bias gradient: about 2048 values each (over the
// batch), at most 256.
static int bias_segments(const Net& n, const Conv& c, int* len) {
  const size_t pl = plane(n, c.lvl), tot = (size_t)n.desc.batch * pl;
  const size_t ns = std::min<size_t>(std::min<size_t>(256, pl), std::max<size_t>(1, (tot + 2047) / 2048));
  *len = (int)((pl + ns - 1) / ns);
  return (int)((pl + *len - 1) / *len);
}

// Input-channel splits of a forward convolution with `blocks` blocks: enough for
// kSplitBlocks blocks, at most kMaxSplit, at least CIC channels per split, and
// the partials (nsplit x outputs floats) within the scratch.
constexpr int kSplitBlocks = 1024, kMaxSplit = 8;
static int splitk_factor(int blocks, int cin, size_t outputs, size_t scratch_floats) {
  int ns = 1;
  while (ns < kMaxSplit && blocks * ns < kSplitBlocks && cin >= 2 * ns * CIC &&
         (size_t)(2 * ns) * outputs <= scratch_floats)
    ns *= 2;
  // with few channels per split the last one may be empty: use as many as the channels fill
  const int cps = ((cin + ns - 1) / ns + CIC - 1) / CIC * CIC;
  return (cin + cps - 1) / cps;
}

// Build the layer list; with base == nullptr only sizes are computed.
static size_t build_net(Net& n, char* base, size_t* nparams) {
  const hom_unet_desc& ds = n.desc;
  const int d = ds.d, L = ds.levels, c0 = ds.base, B = ds.batch;
  n.levels = L;
  n.sz[0][0] = d == 3 ? ds.size[0] : 1;
  n.sz[0][1] = d == 3 ? ds.size[1] : ds.size[0];
  n.sz[0][2] = d == 3 ? ds.size[2] : ds.size[1];
  for (int l = 1; l < L; ++l)
    for (int a = 0; a < 3; ++a) n.sz[l][a] = (a == 0 && d == 2) ? 1 : (n.sz[l - 1][a] + 1) / 2;
  size_t off = 0;
  auto take = [&](size_t floats) -> float* {
    float* p = base ? reinterpret_cast<float*>(base + off) : nullptr;
    off += ((floats * sizeof(float) + 255) / 256) * 256;
    return p;
  };
  size_t poff = 0;
  auto conv = [&](int cin, int cout, int ks, int lvl, View in, View out, View gin, View gout, bool relu, bool acc) {
    Conv c;
    c.cin = cin;
    c.cout = cout;
    c.ks = ks;
    c.lvl = lvl;
    c.in = in;
    c.out = out;
    c.gin = gin;
    c.gout = gout;
    c.relu = relu;
    c.accumulate_gin = acc;
    const int taps = ks == 3 ? (d == 3 ? 27 : 9) : 1;
    c.w = poff;
    poff += (size_t)cout * cin * taps;
    c.b = poff;
    poff += cout;
    n.convs.push_back(c);
  };
  auto buf = [&](int C, int l) -> View {
    View v;
    v.p = take((size_t)B * C * plane(n, l));
    v.C = C;
    v.Ctot = C;
    v.off = 0;
    if (base) n.act_bufs.push_back(v.p);
    return v;
  };
  auto slice = [](View v, int off, int C) {
    v.off += off;
    v.C = C;
    return v;
  };
  n.convs.clear();
  n.pools.clear();
  n.ups.clear();
  std::vector<View> skip(L), gskip(L), cat(L), gcat(L);
  View in = buf(ds.cin, 0), gin_dummy = buf(ds.cin, 0);
  n.in0 = in.p;
  View cur = in, gcur = gin_dummy;
  int cprev = ds.cin;
  for (int l = 0; l < L; ++l) {
    const int cl = c0 << l;
    View a = buf(cl, l), ga = buf(cl, l);
    conv(cprev, cl, 3, l, cur, a, gcur, ga, true, false);
    if (l < L - 1) {
      cat[l] = buf(2 * cl, l);
      gcat[l] = buf(2 * cl, l);
      skip[l] = slice(cat[l], cl, cl);
      gskip[l] = slice(gcat[l], cl, cl);
      conv(cl, cl, 3, l, a, skip[l], ga, gskip[l], true, false);
      View p = buf(cl, l + 1), gp = buf(cl, l + 1);
      Net::Pool pl;
      pl.in = skip[l];
      pl.out = p;
      pl.gin = gskip[l];
      pl.gout = gp;
      pl.lvl = l;
      n.pools.push_back(pl);
      cur = p;
      gcur = gp;
      cprev = cl;
    } else {
      View bb = buf(cl, l), gbb = buf(cl, l);
      conv(cl, cl, 3, l, a, bb, ga, gbb, true, false);
      cur = bb;
      gcur = gbb;
      cprev = cl;
    }
  }
  for (int l = L - 2; l >= 0; --l) {
    const int cl = c0 << l, cu = c0 << (l + 1);
    View u = buf(cu, l), gu = buf(cu, l);
    Net::Up up;
    up.in = cur;
    up.out = u;
    up.gin = gcur;
    up.gout = gu;
    up.lvl = l;
    n.ups.push_back(up);
    conv(cu, cl, 3, l, u, slice(cat[l], 0, cl), gu, slice(gcat[l], 0, cl), true, false);
    View a = buf(cl, l), ga = buf(cl, l);
    conv(2 * cl, cl, 3, l, cat[l], a, gcat[l], ga, true, false);
    View bb = buf(cl, l), gbb = buf(cl, l);
    conv(cl, cl, 3, l, a, bb, ga, gbb, true, false);
    cur = bb;
    gcur = gbb;
  }
  View o = buf(ds.cout, 0), go = buf(ds.cout, 0);
  conv(c0, ds.cout, 1, 0, cur, o, gcur, go, false, false);
  n.out = o.p;
  n.gout = go.p;
  // packed weights, forward and adjoint (the first layer's adjoint is never used)
  size_t pk = 0, pkf = 0;
  n.fwd_pack.n = n.bwd_pack.n = 0;
  n.pack_max = 0;
  for (size_t i = 0; i < n.convs.size(); ++i) {
    Conv& c = n.convs[i];
    const int taps = c.ks == 3 ? (d == 3 ? 27 : 9) : 1;
    c.pk = pk;
    const size_t f = packed_floats(c.cout, c.cin, taps), g = packed_floats(c.cin, c.cout, taps);
    n.fwd_pack.e[n.fwd_pack.n++] = PackEntry{c.w, pk, c.cout, c.cin, taps, 0};
    pk += (f + 63) / 64 * 64;
    n.pack_max = std::max(n.pack_max, f);
    c.pkf = pkf;
    if (i > 0) {
      n.bwd_pack.e[n.bwd_pack.n++] = PackEntry{c.w, pkf, c.cin, c.cout, taps, 1};
      pkf += (g + 63) / 64 * 64;
      n.pack_max = std::max(n.pack_max, g);
    }
  }
  n.wpk = take(pk);
  n.wpkf = take(pkf);
  // scratch: weight-gradient partials (largest layer), loss partials
  size_t wp = 0, bp = 0;
  for (auto& c : n.convs) {
    int nchunk, per, len;
    wgrad_chunks(n, c, &nchunk, &per);
    const int taps = c.ks == 3 ? (d == 3 ? 27 : 9) : 1;
    wp = std::max(wp, (size_t)nchunk * c.cout * c.cin * taps);
    bp = std::max(bp, (size_t)bias_segments(n, c, &len) * c.cout);
  }
  n.wpart_floats = wp;
  n.wpart = take(n.wpart_floats);
  n.bpart = take(bp);
  n.rpart = take(kRpartFloats);
  n.tgt = take((size_t)B * ds.cout * plane(n, 0));
  // split-K partials: the largest output (B x cout x plane) of a conv whose level gives it fewer
  // than kSplitBlocks blocks, times kMaxSplit
  size_t sp = 0;
  for (auto& c : n.convs) {
    const int tiles = ((n.sz[c.lvl][2] + Tile<3>::X - 1) / Tile<3>::X) * ((n.sz[c.lvl][1] + Tile<3>::Y - 1) / Tile<3>::Y) *
                      ((n.sz[c.lvl][0] + Tile<3>::Z - 1) / Tile<3>::Z);
    const int tiles2 = ((n.sz[c.lvl][2] + Tile<2>::X - 1) / Tile<2>::X) * ((n.sz[c.lvl][1] + Tile<2>::Y - 1) / Tile<2>::Y);
    const int t = d == 3 ? tiles : tiles2;
    for (int dir = 0; dir < 2; ++dir) {          // forward (cout outputs) and data gradient (cin outputs)
      const int co = dir ? c.cin : c.cout;
      if (t * ((co + COT - 1) / COT) * B < kSplitBlocks)
        sp = std::max(sp, (size_t)kMaxSplit * B * co * plane(n, c.lvl));
    }
  }
  n.spart_floats = sp;
  n.spart = sp ? take(sp) : nullptr;
  n.wgt = take((size_t)B * ds.cout * plane(n, 0));
  n.lpart = reinterpret_cast<double*>(take(2 * 8192));
  *nparams = poff;
  return off;
}

template <int D>
// w: the layer's packed weights (k_pack_w)
static hipError_t conv_fwd_launch(const Net& n, const View& in, const float* w, const float* b, const View& out,
                                  int cin, int cout, int ks, int lvl, bool relu, bool acc) {
  const int Z = n.sz[lvl][0], H = n.sz[lvl][1], W = n.sz[lvl][2];
  const int tiles = ((W + Tile<D>::X - 1) / Tile<D>::X) * ((H + Tile<D>::Y - 1) / Tile<D>::Y) *
                    ((Z + Tile<D>::Z - 1) / Tile<D>::Z);
  const int cot = (cout + COT - 1) / COT, B = n.desc.batch;
  const size_t pl = (size_t)Z * H * W;
  const int ns = splitk_factor(tiles * cot * B, cin, (size_t)B * cout * pl, n.spart_floats);
  const int cps = ((cin + ns - 1) / ns + CIC - 1) / CIC * CIC;
  float* part = ns > 1 ? n.spart : nullptr;
  dim3 grid(tiles, cot * ns, B);
  if (ks == 3)
    hipLaunchKernelGGL((k_conv_fwd<D, 3>), grid, dim3(CT), 0, n.st, in.p, cin, in.Ctot, in.off, w, b, out.p, cout,
                       out.Ctot, out.off, Z, H, W, relu ? 1 : 0, acc ? 1 : 0, cps, part);
  else
    hipLaunchKernelGGL((k_conv_fwd<D, 1>), grid, dim3(CT), 0, n.st, in.p, cin, in.Ctot, in.off, w, b, out.p, cout,
                       out.Ctot, out.off, Z, H, W, relu ? 1 : 0, acc ? 1 : 0, cps, part);
  if (ns > 1)
    hipLaunchKernelGGL(k_splitk_sum, plane_grid(pl, B * cout), dim3(CT), 0, n.st, part, ns, B, cout, pl, b,
                       out.p, out.Ctot, out.off, relu ? 1 : 0, acc ? 1 : 0);
  return hipGetLastError();
}

static void pack_weights(const Net& n, const PackTable& t, float* wp) {
  if (t.n > 0)
    hipLaunchKernelGGL(k_pack_w, dim3(std::min(gridn(n.pack_max), 512), t.n), dim3(CT), 0, n.st, n.params, t, wp);
}

template <int D>
static hipError_t forward(Net& n) {
  pack_weights(n, n.fwd_pack, n.wpk);
  for (size_t i = 0, pi = 0, ui = 0; i < n.convs.size(); ++i) {
    const Conv& c = n.convs[i];
    // decoder upsampling precedes the first conv of each decoder level
    if (ui < n.ups.size() && c.in.p == n.ups[ui].out.p) {
      const auto& u = n.ups[ui++];
      const int lo = u.lvl, li = lo + 1;
      hipLaunchKernelGGL(k_up<D>, plane_grid(plane(n, lo), n.desc.batch * u.out.C), dim3(CT), 0, n.st, u.in.p, u.in.Ctot, u.in.off, u.out.p,
                         u.out.Ctot, u.out.off, u.out.C, n.sz[li][0], n.sz[li][1], n.sz[li][2], n.sz[lo][0],
                         n.sz[lo][1], n.sz[lo][2], n.desc.batch);
    }
    hipError_t e = conv_fwd_launch<D>(n, c.in, n.wpk + c.pk, n.params + c.b, c.out, c.cin, c.cout, c.ks, c.lvl,
                                      c.relu, false);
    if (e != hipSuccess) return e;
    // pooling follows the second conv of each encoder level
    if (pi < n.pools.size() && c.out.p == n.pools[pi].in.p && c.out.off == n.pools[pi].in.off) {
      const auto& p = n.pools[pi++];
      const int li = p.lvl, lo = li + 1;
      hipLaunchKernelGGL(k_pool<D>, plane_grid(plane(n, lo), n.desc.batch * p.out.C), dim3(CT), 0, n.st, p.in.p, p.in.Ctot, p.in.off, p.out.p,
                         p.out.Ctot, p.out.off, p.in.C, n.sz[li][0], n.sz[li][1], n.sz[li][2], n.sz[lo][0],
                         n.sz[lo][1], n.sz[lo][2], n.desc.batch);
    }
  }
  return hipGetLastError();
}

template <int D>
static hipError_t backward(Net& n) {
  const int B = n.desc.batch;
  const int d = n.desc.d;
  pack_weights(n, n.bwd_pack, n.wpkf);
  for (int i = (int)n.convs.size() - 1; i >= 0; --i) {
    const Conv& c = n.convs[i];
    const int l = c.lvl;
    const size_t pl = plane(n, l);
    const int taps = c.ks == 3 ? (d == 3 ? 27 : 9) : 1;
    if (c.relu) {
      hipLaunchKernelGGL(k_relu_mask, plane_grid(pl, B * c.cout), dim3(CT), 0, n.st, c.gout.p, c.out.p, c.cout, c.gout.Ctot,
                         c.gout.off, c.out.Ctot, c.out.off, pl, B);
    }
    // weight gradient: partials over chunks of point tiles, then a fixed-order sum
    const int ntiles = tiles_at(n, l) * B;
    int nchunk, per_chunk;
    wgrad_chunks(n, c, &nchunk, &per_chunk);
    const size_t nw = (size_t)c.cout * c.cin * taps;
    dim3 gw(nchunk, (c.cout + COT - 1) / COT, (c.cin + WCI - 1) / WCI);
    if (c.ks == 3)
      hipLaunchKernelGGL((k_conv_wgrad<D, 3>), gw, dim3(CT), 0, n.st, c.in.p, c.cin, c.in.Ctot, c.in.off, c.gout.p,
                         c.cout, c.gout.Ctot, c.gout.off, n.sz[l][0], n.sz[l][1], n.sz[l][2], ntiles, per_chunk,
                         n.wpart);
    else
      hipLaunchKernelGGL((k_conv_wgrad<D, 1>), gw, dim3(CT), 0, n.st, c.in.p, c.cin, c.in.Ctot, c.in.off, c.gout.p,
                         c.cout, c.gout.Ctot, c.gout.off, n.sz[l][0], n.sz[l][1], n.sz[l][2], ntiles, per_chunk,
                         n.wpart);
    sum_partials(n, n.wpart, nchunk, nw, n.grads + c.w);
    int len;
    const int nseg = bias_segments(n, c, &len);
    hipLaunchKernelGGL(k_bias_part, dim3(nseg, c.cout), dim3(CT), 0, n.st, c.gout.p, c.cout, c.gout.Ctot, c.gout.off,
                       pl, B, len, n.bpart);
    sum_partials(n, n.bpart, nseg, (size_t)c.cout, n.grads + c.b);
    // data gradient (not needed for the input of the network)
    if (i > 0) {
      hipError_t e = conv_fwd_launch<D>(n, c.gout, n.wpkf + c.pkf, nullptr, c.gin, c.cout, c.cin, c.ks, l, false,
                                        c.accumulate_gin);
      if (e != hipSuccess) return e;
    }
    // adjoint of the pooling / upsampling that produced this conv's input
    for (const auto& p : n.pools)
      if (p.out.p == c.in.p) {
        const int li = p.lvl, lo = li + 1;
        hipLaunchKernelGGL(k_pool_bwd<D>, plane_grid(plane(n, li), B * p.in.C), dim3(CT), 0, n.st, p.gout.p, p.gout.Ctot, p.gout.off,
                           p.gin.p, p.gin.Ctot, p.gin.off, p.in.C, n.sz[li][0], n.sz[li][1], n.sz[li][2],
                           n.sz[lo][0], n.sz[lo][1], n.sz[lo][2], B);
      }
    for (const auto& u : n.ups)
      if (u.out.p == c.in.p) {
        const int lo = u.lvl, li = lo + 1;
        hipLaunchKernelGGL(k_up_bwd<D>, plane_grid(plane(n, li), B * u.in.C), dim3(CT), 0, n.st, u.gout.p, u.gout.Ctot, u.gout.off,
                           u.gin.p, u.gin.Ctot, u.gin.off, u.in.C, n.sz[li][0], n.sz[li][1], n.sz[li][2],
                           n.sz[lo][0], n.sz[lo][1], n.sz[lo][2], B);
      }
  }
  return hipGetLastError();
}

}  // namespace cnn
}  // namespace hom

using hom::cnn::Net;

struct hom_unet {
  Net net;
  hipGraphExec_t fwd_graph = nullptr;   // the forward kernels, captured on the first forward of a stream
  ~hom_unet() {
    if (fwd_graph) (void)hipGraphExecDestroy(fwd_graph);
  }
};

namespace {
hom_status check_udesc(const hom_unet_desc* d) {
  if (!d) return HOM_E_INVALID;
  if (d->d != 2 && d->d != 3) return HOM_E_INVALID;
  if (d->levels < 1 || d->levels > 6 || d->base < 1 || d->base > 256 || d->cin < 1 || d->cout < 1 || d->batch < 1)
    return HOM_E_INVALID;
  long long pts = 1;
  for (int a = 0; a < d->d; ++a) {
    if (d->size[a] < 2) return HOM_E_INVALID;
    pts *= d->size[a];
  }
  // the kernels index a channel plane, and 32 planes of it, with 32-bit offsets
  if (pts > (1LL << 24)) return HOM_E_INVALID;
  return HOM_OK;
}
}  // namespace

extern "C" {

hom_status hom_unet_sizes(const hom_unet_desc* desc, size_t* n_params, size_t* work_bytes) {
  hom_status s = check_udesc(desc);
  if (s != HOM_OK) return s;
  if (!n_params || !work_bytes) return HOM_E_INVALID;
  Net n;
  n.desc = *desc;
  *work_bytes = hom::cnn::build_net(n, nullptr, n_params);
  return HOM_OK;
}

hom_status hom_unet_create(const hom_unet_desc* desc, float* params, float* grads, float* adam_m, float* adam_v,
                           void* work, size_t work_bytes, void* stream, hom_unet** out) {
  hom_status s = check_udesc(desc);
  if (s != HOM_OK) return s;
  if (!params || !grads || !adam_m || !adam_v || !work || !out) return HOM_E_INVALID;
  if (((uintptr_t)work) % 256) return HOM_E_WORKSPACE;
  hom_unet* u = new hom_unet();
  u->net.desc = *desc;
  size_t np = 0;
  const size_t need = hom::cnn::build_net(u->net, nullptr, &np);
  if (work_bytes < need) {
    delete u;
    return HOM_E_WORKSPACE;
  }
  u->net = Net();
  u->net.desc = *desc;
  hom::cnn::build_net(u->net, (char*)work, &np);
  u->net.nparams = np;
  u->net.params = params;
  u->net.grads = grads;
  u->net.m1 = adam_m;
  u->net.m2 = adam_v;
  u->net.work = (char*)work;
  u->net.work_bytes = work_bytes;
  u->net.st = reinterpret_cast<hipStream_t>(stream);
  *out = u;
  return HOM_OK;
}

}  // extern "C"

namespace {
// The forward kernels from the network's own input copy: replayed from a
// graph captured on the first call (a stream is needed), direct otherwise.
hom_status run_forward(hom_unet* u) {
  Net& n = u->net;
  if (!n.st) {
    hipError_t e = n.desc.d == 3 ? hom::cnn::forward<3>(n) : hom::cnn::forward<2>(n);
    return e == hipSuccess ? HOM_OK : HOM_E_DEVICE;
  }
  if (!u->fwd_graph) {
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(n.st, hipStreamCaptureModeThreadLocal) != hipSuccess) return HOM_E_DEVICE;
    hipError_t e = n.desc.d == 3 ? hom::cnn::forward<3>(n) : hom::cnn::forward<2>(n);
    hipError_t e2 = hipStreamEndCapture(n.st, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return HOM_E_DEVICE;
    }
    e = hipGraphInstantiate(&u->fwd_graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return HOM_E_DEVICE;
  }
  return hipGraphLaunch(u->fwd_graph, n.st) == hipSuccess ? HOM_OK : HOM_E_DEVICE;
}

// Copies of `count` samples of `each` floats from sample pointers into dst (device to device).
hom_status gather(float* dst, const float* const* src, int count, size_t each, hipStream_t st) {
  for (int i = 0; i < count; ++i) {
    if (!src[i]) return HOM_E_INVALID;
    if (hipMemcpyAsync(dst + (size_t)i * each, src[i], each * sizeof(float), hipMemcpyDeviceToDevice, st) !=
        hipSuccess)
      return HOM_E_DEVICE;
  }
  return HOM_OK;
}
}  // namespace

extern "C" {

hom_status hom_unet_forward_samples(hom_unet* u, const float* const* in, float* out) {
  if (!u || !in) return HOM_E_INVALID;
  Net& n = u->net;
  hom_status s = gather(n.in0, in, n.desc.batch, (size_t)n.desc.cin * hom::cnn::plane(n, 0), n.st);
  if (s != HOM_OK) return s;
  s = run_forward(u);
  if (s != HOM_OK) return s;
  if (out) {
    const size_t no = (size_t)n.desc.batch * n.desc.cout * hom::cnn::plane(n, 0);
    if (hipMemcpyAsync(out, n.out, no * sizeof(float), hipMemcpyDeviceToDevice, n.st) != hipSuccess)
      return HOM_E_DEVICE;
  }
  return HOM_OK;
}

hom_status hom_unet_forward(hom_unet* u, const float* in, float* out) {
  if (!u || !in) return HOM_E_INVALID;
  Net& n = u->net;
  const size_t nin = (size_t)n.desc.batch * n.desc.cin * hom::cnn::plane(n, 0);
  if (hipMemcpyAsync(n.in0, in, nin * sizeof(float), hipMemcpyDeviceToDevice, n.st) != hipSuccess)
    return HOM_E_DEVICE;
  hom_status s = run_forward(u);
  if (s != HOM_OK) return s;
  if (out) {
    const size_t no = (size_t)n.desc.batch * n.desc.cout * hom::cnn::plane(n, 0);
    if (hipMemcpyAsync(out, n.out, no * sizeof(float), hipMemcpyDeviceToDevice, n.st) != hipSuccess)
      return HOM_E_DEVICE;
  }
  return HOM_OK;
}

hom_status hom_unet_loss_weighted(hom_unet* u, const float* target, const float* weight, int32_t wch,
                                  double* loss) {
  if (!u || !target || !loss) return HOM_E_INVALID;
  Net& n = u->net;
  if (weight && (wch < 1 || wch > n.desc.cout || n.desc.cout % wch != 0)) return HOM_E_INVALID;
  const size_t pl = hom::cnn::plane(n, 0);
  const size_t no = (size_t)n.desc.batch * n.desc.cout * pl;
  const int nb = std::min(hom::cnn::gridn(no), 1024);
  hipLaunchKernelGGL(hom::cnn::k_mse, dim3(nb), dim3(hom::cnn::CT), 0, n.st, n.out, target, no, weight,
                     weight ? wch : 1, n.desc.cout, pl, n.gout, n.lpart);
  if (hipGetLastError() != hipSuccess) return HOM_E_DEVICE;
  std::vector<double> part(nb);
  if (hipMemcpyAsync(part.data(), n.lpart, nb * sizeof(double), hipMemcpyDeviceToHost, n.st) != hipSuccess ||
      hipStreamSynchronize(n.st) != hipSuccess)
    return HOM_E_DEVICE;
  double s = 0.0;
  for (double v : part) s += v;
  *loss = s / (double)no;
  return HOM_OK;
}

hom_status hom_unet_loss(hom_unet* u, const float* target, double* loss) {
  return hom_unet_loss_weighted(u, target, nullptr, 1, loss);
}

hom_status hom_unet_loss_samples(hom_unet* u, const float* const* target, const float* const* weight, int32_t wch,
                                 double* loss) {
  if (!u || !target || !loss) return HOM_E_INVALID;
  Net& n = u->net;
  if (weight && (wch < 1 || wch > n.desc.cout || n.desc.cout % wch != 0)) return HOM_E_INVALID;
  const size_t pl = hom::cnn::plane(n, 0);
  hom_status s = gather(n.tgt, target, n.desc.batch, (size_t)n.desc.cout * pl, n.st);
  if (s == HOM_OK && weight) s = gather(n.wgt, weight, n.desc.batch, (size_t)wch * pl, n.st);
  if (s != HOM_OK) return s;
  return hom_unet_loss_weighted(u, n.tgt, weight ? n.wgt : nullptr, wch, loss);
}

hom_status hom_unet_backward(hom_unet* u, const float* gout) {
  if (!u) return HOM_E_INVALID;
  Net& n = u->net;
  const size_t no = (size_t)n.desc.batch * n.desc.cout * hom::cnn::plane(n, 0);
  if (gout && hipMemcpyAsync(n.gout, gout, no * sizeof(float), hipMemcpyDeviceToDevice, n.st) != hipSuccess)
    return HOM_E_DEVICE;
  // zero parameter gradients and every activation-gradient buffer except the output gradient
  hipLaunchKernelGGL(hom::cnn::k_fill, dim3(hom::cnn::gridn(n.nparams)), dim3(hom::cnn::CT), 0, n.st, n.grads,
                     n.nparams, 0.f);
  for (const auto& c : n.convs) {
    if (c.gin.p && c.gin.p != n.gout) {
      const size_t tot = (size_t)n.desc.batch * c.gin.Ctot * hom::cnn::plane(n, c.lvl);
      hipLaunchKernelGGL(hom::cnn::k_fill, dim3(hom::cnn::gridn(tot)), dim3(hom::cnn::CT), 0, n.st, c.gin.p, tot,
                         0.f);
    }
  }
  for (const auto& p : n.pools) {
    const size_t tot = (size_t)n.desc.batch * p.gout.Ctot * hom::cnn::plane(n, p.lvl + 1);
    hipLaunchKernelGGL(hom::cnn::k_fill, dim3(hom::cnn::gridn(tot)), dim3(hom::cnn::CT), 0, n.st, p.gout.p, tot, 0.f);
  }
  hipError_t e = n.desc.d == 3 ? hom::cnn::backward<3>(n) : hom::cnn::backward<2>(n);
  return e == hipSuccess ? HOM_OK : HOM_E_DEVICE;
}

hom_status hom_unet_adam(hom_unet* u, float lr, float beta1, float beta2, float eps, int32_t step) {
  if (!u || step < 1) return HOM_E_INVALID;
  Net& n = u->net;
  const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
  hipLaunchKernelGGL(hom::cnn::k_adam, dim3(hom::cnn::gridn(n.nparams)), dim3(hom::cnn::CT), 0, n.st, n.params,
                     n.grads, n.m1, n.m2, n.nparams, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? HOM_OK : HOM_E_DEVICE;
}

void hom_unet_destroy(hom_unet* u) { delete u; }

}  // extern "C"
