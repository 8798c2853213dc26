// C ABI of libhom (declared in include/hom.h): validation, workspace carving,
// coefficient setup on the device, and the host loop that enqueues CG
// iterations (captured into a HIP graph per chunk of iterations).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/hom.h"
#include "hom_internal.hpp"

using namespace hom;

namespace {

constexpr size_t kAlign = 256;

size_t up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

bool smooth35(int M, Plan* pl) {
  int n = 0;
  int v = M;
  while (v % 5 == 0 && n < kMaxStages) {
    pl->r[n++] = 5;
    v /= 5;
  }
  while (v % 3 == 0 && n < kMaxStages) {
    pl->r[n++] = 3;
    v /= 3;
  }
  pl->n = n;
  return v == 1;
}

// Plan for lengths 2^a 3^b 5^c (the transforms of even GaNi grids): radix-4
// stages for pairs of twos, one radix-2 stage for an odd power, then 5s and 3s.
bool smooth235(int M, Plan* pl) {
  int n = 0;
  int v = M;
  while (v % 4 == 0 && n < kMaxStages) {
    pl->r[n++] = 4;
    v /= 4;
  }
  if (v % 2 == 0 && n < kMaxStages) {
    pl->r[n++] = 2;
    v /= 2;
  }
  while (v % 5 == 0 && n < kMaxStages) {
    pl->r[n++] = 5;
    v /= 5;
  }
  while (v % 3 == 0 && n < kMaxStages) {
    pl->r[n++] = 3;
    v /= 3;
  }
  pl->n = n;
  return v == 1;
}

int env_int(const char* name, int def) {
  const char* s = std::getenv(name);
  return s ? std::atoi(s) : def;
}

// ---- tile tuning of the specialised FP32 passes
// One entry per geometry and load count, shared by every problem and batch of
// the process: the first solve of a geometry times the candidates, later ones
// reuse the choice, so a batch and single-cell solves of the same geometry run
// the same kernels (and the same reduction order).
struct TuneKey {
  int M0, M1, M2, d, L, dual, nc, P;
  bool operator<(const TuneKey& o) const {
    return std::tie(M0, M1, M2, d, L, dual, nc, P) < std::tie(o.M0, o.M1, o.M2, o.d, o.L, o.dual, o.nc, o.P);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, Tuning> g_tune_cache;
int g_tune_mode = -1;  // -1: not read yet (HOM_TUNE, default 1)
bool g_tune_file_read = false;   // HOM_TUNE_CACHE read into the cache (once per process)

// ---- the tuner cache on disk: one JSON object per line, per device architecture
// (the gcnArchName up to its first ':'), so that later processes skip the timing.

// Architecture of the current device, or "" without one.
std::string device_arch() {
  int dev = -1;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
  std::string a = prop.gcnArchName;
  return a.substr(0, a.find(':'));
}

bool json_num(const std::string& line, const char* key, double* v) {
  const std::string k = std::string("\"") + key + "\":";
  const size_t at = line.find(k);
  if (at == std::string::npos) return false;
  const char* p = line.c_str() + at + k.size();
  char* end = nullptr;
  *v = std::strtod(p, &end);
  return end != p;
}

bool json_str(const std::string& line, const char* key, std::string* v) {
  const std::string k = std::string("\"") + key + "\":";
  size_t at = line.find(k);
  if (at == std::string::npos) return false;
  at = line.find('"', at + k.size());
  if (at == std::string::npos) return false;
  const size_t e = line.find('"', at + 1);
  if (e == std::string::npos) return false;
  *v = line.substr(at + 1, e - at - 1);
  return true;
}

// Entries of `arch` from the file into the cache (caller holds g_tune_mu);
// false when the file cannot be read or a line does not parse.
bool tune_file_read(const char* path, const std::string& arch, int* loaded) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  bool ok = true;
  int cnt = 0;
  char buf[1024];
  while (std::fgets(buf, sizeof(buf), f)) {
    std::string line(buf);
    if (line.find('{') == std::string::npos) continue;
    std::string a;
    double v[16];
    const char* keys[16] = {"M0", "M1", "M2", "d", "loads", "dual", "nc", "packs", "row_pairs", "row_threads",
                            "apply_points", "apply_half_exchange", "apply_all_packs", "row_ms", "apply_ms",
                            "candidates"};
    bool good = json_str(line, "arch", &a);
    for (int i = 0; i < 16 && good; ++i) good = json_num(line, keys[i], &v[i]);
    if (!good) {
      ok = false;
      break;
    }
    if (a != arch) continue;
    TuneKey k{(int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4], (int)v[5], (int)v[6], (int)v[7]};
    Tuning t;
    t.rowG = (int)v[8];
    t.rowThreads = (int)v[9];
    t.apTP = (int)v[10];
    t.apHX = (int)v[11];
    t.apAll = (int)v[12];
    t.row_ms = v[13];
    t.apply_ms = v[14];
    t.candidates = (int)v[15];
    g_tune_cache[k] = t;
    ++cnt;
  }
  std::fclose(f);
  if (loaded) *loaded = cnt;
  return ok;
}

// The whole cache, tagged with `arch`, to the file (caller holds g_tune_mu).
bool tune_file_write(const char* path, const std::string& arch) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  for (const auto& kv : g_tune_cache) {
    const TuneKey& k = kv.first;
    const Tuning& t = kv.second;
    std::fprintf(f,
                 "{\"arch\": \"%s\", \"M0\": %d, \"M1\": %d, \"M2\": %d, \"d\": %d, \"loads\": %d, \"dual\": %d, "
                 "\"nc\": %d, \"packs\": %d, \"row_pairs\": %d, \"row_threads\": %d, \"apply_points\": %d, "
                 "\"apply_half_exchange\": %d, \"apply_all_packs\": %d, \"row_ms\": %.9g, \"apply_ms\": %.9g, "
                 "\"candidates\": %d}\n",
                 arch.c_str(), k.M0, k.M1, k.M2, k.d, k.L, k.dual, k.nc, k.P, t.rowG, t.rowThreads, t.apTP, t.apHX,
                 t.apAll, t.row_ms, t.apply_ms, t.candidates);
  }
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

bool tuning_on() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_tune_mode < 0) g_tune_mode = env_int("HOM_TUNE", 1) != 0 ? 1 : 0;
  return g_tune_mode == 1;
}

struct SlotBufs {
  Cx<double>* r[kMaxLoads] = {};
  Cx<double>* p[kMaxLoads] = {};
  Cx<double>* s[kMaxLoads] = {};
  Cx<double>* b[kMaxLoads] = {};
  Cx<double>* tmp[kMaxLoads] = {};
  void* bufA = nullptr;
  void* bufB = nullptr;
  double* part_g = nullptr;
  double* part_d = nullptr;
  double* part_q = nullptr;
  CgScal* sc = nullptr;
  UnitDev* unit = nullptr;
  int* iter_base = nullptr;
  int* active = nullptr;
};

// Byte sizes of everything carved from the workspace.
struct Sizes {
  int d, nc, L;
  int N[3], M[3];
  int H0, S, Q;
  size_t Mt;
};

}  // namespace

// GaNi mode of a problem (Def. GaNi, the paper's Algorithm): solves use the
// trapezoidal rule on the N grid, i.e. point values of A and A^-1 there and
// N-point transforms; the bounds keep the exact quadrature.  Buffers live in a
// caller-owned workspace (hom_set_gani).  GaNi solves run in FP64 in either
// precision mode: the exact bounds of a GaNi minimiser are first order in its
// algebraic error (it does not minimise the exact form), so FP32 transforms
// would cost their rounding error at full strength; in mixed problems the FP64
// intermediates use the problem's (FP64) bound-evaluation buffers.
struct GaniData {
  bool on = false;
  double* coef64[2] = {};          // [nc][Nt] point values of A (primal) and A^-1 (dual)
  Cx<double>* ahat[2] = {};        // [nc][S] N-point DFT of the point values, stored half
  Cx<double>* tw64[3] = {};
  Cx<float>* tw32[3] = {};
  Cx<double>* scratch = nullptr;   // [nc][Nt] complex
  Plan plan[3] = {};
  int grid[3] = {};                // GaNi grid on internal axes: N (odd) or N + 1 (even; fields on Z_N = its Z^r)
  hipGraphExec_t graph[2][kMaxLoads + 1] = {};
};

struct hom_problem {
  hom_desc desc;
  int max_loads;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  Sizes z;
  Plan plan[3];
  double* coef64[2];
  float* coef32[2];
  float* coefp[2];      // FP32 coefficient in plane order (3D plane pass), or null
  Cx<double>* ahat_half[2];
  Cx<double>* tw64[3];
  Cx<float>* tw32[3];
  Cx<double>* scratch;  // setup: nc * Mt complex
  SlotBufs slot[2];     // primal, dual
  // bounds (FP64, L = d)
  void* bbufA;
  void* bbufB;
  void* bbufA2;         // the dual side's bound buffers (batched bounds run both sides at once)
  void* bbufB2;
  double* bpart_q[2];
  UnitDev* bunit[2];
  UnitDev host_unit[2];
  UnitDev host_bunit[2];
  int* pinned_active;
  hipGraphExec_t graph[2][kMaxLoads + 1];
  int graph_chunk;
  Tuning tune[2][kMaxLoads + 1];        // tile shapes of the single-problem solves
  bool tuned[2][kMaxLoads + 1];
  StopCfg stop;                         // stopping rule of later solves (hom_problem_set_stop)
  GaniData gani;
};

namespace {

bool fill_sizes(const hom_desc* desc, int max_loads, Sizes* z, Plan* plan) {
  if (!desc) return false;
  const int d = desc->d;
  if (d != 2 && d != 3) return false;
  z->d = d;
  z->nc = desc->ncoef;
  z->L = max_loads;
  int Nphys[3] = {desc->N[0], desc->N[1], d == 3 ? desc->N[2] : 1};
  if (d == 2) {
    z->N[0] = Nphys[0];
    z->N[1] = 1;
    z->N[2] = Nphys[1];
  } else {
    for (int a = 0; a < 3; ++a) z->N[a] = Nphys[a];
  }
  // quadrature grid: the doubled grid 2N - 1 unless the caller gives a larger one
  int Mphys[3] = {desc->M[0], desc->M[1], d == 3 ? desc->M[2] : 0};
  if (d == 2) {
    z->M[0] = Mphys[0] ? Mphys[0] : 2 * z->N[0] - 1;
    z->M[1] = 1;
    z->M[2] = Mphys[1] ? Mphys[1] : 2 * z->N[2] - 1;
  } else {
    for (int a = 0; a < 3; ++a) z->M[a] = Mphys[a] ? Mphys[a] : 2 * z->N[a] - 1;
  }
  for (int a = 0; a < 3; ++a) {
    if (a == 1 && d == 2) {
      plan[a].n = 0;
      continue;
    }
    if (!smooth35(z->M[a], &plan[a])) return false;
  }
  z->H0 = (z->N[0] + 1) / 2;
  z->S = z->H0 * z->N[1] * z->N[2];
  z->Q = (z->N[1] + 1) / 2 + (z->H0 - 1) * z->N[1];
  z->Mt = (size_t)z->M[0] * z->M[1] * z->M[2];
  return true;
}

int packs(int L, int d) { return (L * d + 1) / 2; }

hom_status validate_desc(const hom_desc* desc, int max_loads) {
  if (!desc) return HOM_E_INVALID;
  if (desc->d != 2 && desc->d != 3) return HOM_E_INVALID;
  if (max_loads < 1 || max_loads > kMaxLoads) return HOM_E_INVALID;
  if (desc->precision != HOM_FP64 && desc->precision != HOM_MIXED) return HOM_E_INVALID;
  const int d = desc->d;
  if (desc->ncoef != 1 && desc->ncoef != d * (d + 1) / 2) return HOM_E_INVALID;
  for (int a = 0; a < d; ++a) {
    if (!(desc->Y[a] > 0.0) || !std::isfinite(desc->Y[a])) return HOM_E_INVALID;
    if (desc->N[a] < 3 || desc->N[a] % 2 == 0) return HOM_E_UNSUPPORTED_SIZE;
    if (desc->N[a] > 4097) return HOM_E_UNSUPPORTED_SIZE;
    const int Ma = desc->M[a] ? desc->M[a] : 2 * desc->N[a] - 1;
    if (Ma < 2 * desc->N[a] - 1 || Ma % 2 == 0 || Ma > 8193) return HOM_E_UNSUPPORTED_SIZE;
    Plan pl;
    if (!smooth35(Ma, &pl)) return HOM_E_UNSUPPORTED_SIZE;
  }
  // LDS of the generic passes: the column pass holds one column of every pack
  // (FP64 for the bounds, whose packs carry d loads), the row passes stage the
  // stored rows of every load
  const int M0 = desc->M[0] ? desc->M[0] : 2 * desc->N[0] - 1;
  const int Nlast = desc->N[d - 1];
  const size_t cs = desc->precision == HOM_MIXED ? sizeof(float) * 2 : sizeof(double) * 2;
  const int L = std::max(max_loads, d);
  if ((size_t)M0 * packs(d, d) * 2 * sizeof(double) > kLdsMax) return HOM_E_UNSUPPORTED_SIZE;
  if ((size_t)M0 * packs(max_loads, d) * cs > kLdsMax) return HOM_E_UNSUPPORTED_SIZE;
  if ((size_t)L * std::max(1, d - 1) * Nlast * 2 * sizeof(double) > kLdsMax) return HOM_E_UNSUPPORTED_SIZE;
  return HOM_OK;
}


// Points per apply-pass block: largest count with LDS within budget and the
// per-thread butterfly registers within 16 sets.
int choose_tileA(int M0, int npts, int P, size_t csize, int min_radix) {
  // FP64 blocks are twice the bytes per line: half the budget keeps more of them per CU
  const size_t budget = (size_t)env_int("HOM_LDS_BUDGET", csize > sizeof(Cx<float>) ? 40 * 1024 : 80 * 1024);
  int best = 1;
  for (int t = 1; t <= 64 && t <= npts; ++t) {
    const size_t lds = (size_t)M0 * t * P * csize;
    const int bf = (M0 / min_radix) * t * P;
    if (lds <= budget && (bf + kBlock - 1) / kBlock <= 16) best = t;
  }
  return best;
}

int choose_tileM(int M1, int inner, size_t csize, int min_radix) {
  int best = 1;
  for (int t = 1; t <= 256 && t <= inner; ++t) {
    const size_t lds = (size_t)M1 * t * csize;
    const int bf = (M1 / min_radix) * t;
    if (lds <= 48 * 1024 && (bf + kBlock - 1) / kBlock <= 8) best = t;
  }
  return best;
}

int min_radix(const Plan& p) {
  int r = 5;
  for (int i = 0; i < p.n; ++i) r = std::min(r, p.r[i]);
  return p.n ? r : 5;
}

// Layout of the workspace; with pb == nullptr only the total is computed.
size_t carve(const hom_desc* desc, int max_loads, const Sizes& z, hom_problem* pb) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> size_t {
    const size_t o = off;
    off = up(off + bytes);
    return o;
  };
  char* base = pb ? pb->ws : nullptr;
  auto ptr = [&](size_t o) -> char* { return base ? base + o : nullptr; };
  const int d = z.d, nc = z.nc, L = max_loads;
  const bool mixed = desc->precision == HOM_MIXED;
  const size_t cs = mixed ? sizeof(Cx<float>) : sizeof(Cx<double>);
  for (int k = 0; k < 2; ++k) {
    size_t o = take(nc * z.Mt * sizeof(double));
    if (pb) pb->coef64[k] = (double*)ptr(o);
    if (mixed) {
      o = take(nc * z.Mt * sizeof(float));
      if (pb) pb->coef32[k] = (float*)ptr(o);
    } else if (pb) {
      pb->coef32[k] = nullptr;
    }
    if (mixed && fast_plane_supported(d, z.M, z.N, nc)) {
      o = take(nc * z.Mt * sizeof(float));
      if (pb) pb->coefp[k] = (float*)ptr(o);
    } else if (pb) {
      pb->coefp[k] = nullptr;
    }
    o = take(nc * (size_t)z.S * sizeof(Cx<double>));
    if (pb) pb->ahat_half[k] = (Cx<double>*)ptr(o);
  }
  for (int a = 0; a < 3; ++a) {
    size_t o = take(z.M[a] * sizeof(Cx<double>));
    if (pb) pb->tw64[a] = (Cx<double>*)ptr(o);
    o = take(z.M[a] * sizeof(Cx<float>));
    if (pb) pb->tw32[a] = (Cx<float>*)ptr(o);
  }
  {
    size_t o = take(nc * z.Mt * sizeof(Cx<double>));
    if (pb) pb->scratch = (Cx<double>*)ptr(o);
  }
  const size_t npts = (size_t)z.M[1] * z.M[2];
  for (int k = 0; k < 2; ++k) {
    const int m = k == 0 ? 1 : d - 1;
    const int P = packs(L, d);
    SlotBufs sb;
    const size_t vec = (size_t)m * z.S * sizeof(Cx<double>);
    for (int l = 0; l < L; ++l) {
      sb.r[l] = (Cx<double>*)ptr(take(vec));
      sb.p[l] = (Cx<double>*)ptr(take(vec));
      sb.s[l] = (Cx<double>*)ptr(take(vec));
      sb.b[l] = (Cx<double>*)ptr(take(vec));
      sb.tmp[l] = (Cx<double>*)ptr(take(vec));
    }
    sb.bufA = ptr(take((size_t)z.N[0] * z.N[1] * z.M[2] * P * cs));
    if (d == 3) sb.bufB = ptr(take((size_t)z.N[0] * z.M[1] * z.M[2] * P * cs));
    sb.part_g = (double*)ptr(take((size_t)L * z.Q * sizeof(double)));
    sb.part_d = (double*)ptr(take((size_t)L * z.Q * sizeof(double)));
    sb.part_q = (double*)ptr(take(npts * 9 * sizeof(double)));
    sb.sc = (CgScal*)ptr(take(L * sizeof(CgScal)));
    sb.unit = (UnitDev*)ptr(take(sizeof(UnitDev)));
    sb.iter_base = (int*)ptr(take(sizeof(int)));
    sb.active = (int*)ptr(take(sizeof(int)));
    if (pb) pb->slot[k] = sb;
  }
  {
    const int P = packs(std::max(d, L), d);
    void* a = ptr(take((size_t)z.N[0] * z.N[1] * z.M[2] * P * sizeof(Cx<double>)));
    void* b = d == 3 ? ptr(take((size_t)z.N[0] * z.M[1] * z.M[2] * P * sizeof(Cx<double>))) : nullptr;
    void* a2 = ptr(take((size_t)z.N[0] * z.N[1] * z.M[2] * P * sizeof(Cx<double>)));
    void* b2 = d == 3 ? ptr(take((size_t)z.N[0] * z.M[1] * z.M[2] * P * sizeof(Cx<double>))) : nullptr;
    double* q0 = (double*)ptr(take(npts * 9 * sizeof(double)));
    double* q1 = (double*)ptr(take(npts * 9 * sizeof(double)));
    UnitDev* u0 = (UnitDev*)ptr(take(sizeof(UnitDev)));
    UnitDev* u1 = (UnitDev*)ptr(take(sizeof(UnitDev)));
    if (pb) {
      pb->bbufA = a;
      pb->bbufB = b;
      pb->bbufA2 = a2;
      pb->bbufB2 = b2;
      pb->bpart_q[0] = q0;
      pb->bpart_q[1] = q1;
      pb->bunit[0] = u0;
      pb->bunit[1] = u1;
    }
  }
  return off;
}

Geo make_geo(const hom_problem* pb, int dual, int L, bool fp32, int P_override = 0, const Tuning* tune = nullptr) {
  const Sizes& z = pb->z;
  Geo g;
  std::memset(&g, 0, sizeof(g));
  g.d = z.d;
  for (int a = 0; a < 3; ++a) {
    g.N[a] = z.N[a];
    g.M[a] = z.M[a];
    g.pl[a] = pb->plan[a];
    g.tw[a] = fp32 ? (const void*)pb->tw32[a] : (const void*)pb->tw64[a];
  }
  g.H0 = z.H0;
  g.S = z.S;
  g.m = dual ? z.d - 1 : 1;
  g.L = L;
  g.P = P_override ? P_override : packs(L, z.d);
  g.nc = z.nc;
  g.dual = dual;
  g.Q = z.Q;
  g.nbF = z.Q;
  g.nbL = z.Q;
  if (fp32) {
    if (tune) {
      g.rowG = tune->rowG;
      g.rowThreads = tune->rowThreads;
      g.apTP = tune->apTP;
      g.apHX = tune->apHX;
      g.apAll = tune->apAll;
    }
    const int G = fast_row_pairs(z.M[2], z.N[2], z.d, L, g.rowG);
    if (G > 0) g.nbF = g.nbL = (z.Q + G - 1) / G;
    g.pmaj = (z.d == 2 && G > 0 && z.M[0] == 2 * z.N[0] - 1 && fast_apply_supported(z.M[0], z.d, g.P, z.nc)) ? 1 : 0;
    g.plane = (pb->coefp[dual] && fast_plane_supported(z.d, z.M, z.N, z.nc)) ? 1 : 0;
  }
  const size_t cs = fp32 ? sizeof(Cx<float>) : sizeof(Cx<double>);
  const int npts = z.M[1] * z.M[2];
  g.tileA = choose_tileA(z.M[0], npts, g.P, cs, min_radix(pb->plan[0]));
  g.nbA = (npts + g.tileA - 1) / g.tileA;
  g.tileM = z.d == 3 ? choose_tileM(z.M[1], z.M[2] * g.P, cs, min_radix(pb->plan[1])) : 1;
  if (z.d == 2) {
    g.phys_axis[0] = 0;
    g.phys_axis[1] = 2;
    g.phys_axis[2] = 1;
    g.iY[0] = 1.0 / pb->desc.Y[0];
    g.iY[1] = 1.0;
    g.iY[2] = 1.0 / pb->desc.Y[1];
  } else {
    for (int a = 0; a < 3; ++a) {
      g.phys_axis[a] = a;
      g.iY[a] = 1.0 / pb->desc.Y[a];
    }
  }
  g.invM = 1.0 / (double)z.Mt;
  return g;
}

// Geometry of the GaNi operator: the N grid takes the place of the
// quadrature grid (no padding, no truncation), N-point plans and twiddles;
// the specialised passes never apply (they keep Z_N of a doubled grid).
Geo make_geo_gani(const hom_problem* pb, int dual, int L, bool fp32, int P_override = 0) {
  Geo g = make_geo(pb, dual, L, fp32, P_override, nullptr);
  const Sizes& z = pb->z;
  size_t Nt = 1;
  for (int a = 0; a < 3; ++a) {
    g.M[a] = pb->gani.grid[a];
    g.pl[a] = pb->gani.plan[a];
    g.tw[a] = fp32 ? (const void*)pb->gani.tw32[a] : (const void*)pb->gani.tw64[a];
    Nt *= (size_t)g.M[a];
  }
  g.rowG = g.rowThreads = g.apTP = g.apHX = g.apAll = 0;
  g.pmaj = 0;
  g.plane = 0;
  g.nbF = g.nbL = z.Q;
  const size_t cs = fp32 ? sizeof(Cx<float>) : sizeof(Cx<double>);
  const int npts = g.M[1] * g.M[2];
  g.tileA = choose_tileA(g.M[0], npts, g.P, cs, min_radix(g.pl[0]));
  g.nbA = (npts + g.tileA - 1) / g.tileA;
  g.tileM = z.d == 3 ? choose_tileM(g.M[1], g.M[2] * g.P, cs, min_radix(g.pl[1])) : 1;
  g.invM = 1.0 / (double)Nt;
  return g;
}

#define HIPCHK(x)                      \
  do {                                 \
    if ((x) != hipSuccess) return HOM_E_DEVICE; \
  } while (0)

template <typename R>
hipError_t enqueue_matvec_passes(const Geo& g, const UnitDev* u, int nu, int first_mode, int last_mode, int jstep,
                                 const int* iter_base, hipStream_t st) {
  const bool cg = first_mode == FIRST_CG;
  hipError_t e = launch_first<R>(g, u, nu, first_mode, jstep, iter_base, st);
  if (e != hipSuccess) return e;
  if (g.d == 3 && !g.plane) {
    e = launch_mid<R>(g, u, nu, 1 | (cg ? MID_CG : 0), st);
    if (e != hipSuccess) return e;
  }
  e = launch_apply<R>(g, u, nu, cg ? APPLY_COEF_CG : APPLY_COEF, st);
  if (e != hipSuccess) return e;
  if (g.d == 3 && !g.plane) {
    e = launch_mid<R>(g, u, nu, cg ? MID_CG : 0, st);
    if (e != hipSuccess) return e;
  }
  return launch_last<R>(g, u, nu, last_mode, jstep, iter_base, st);
}

// One operator application from a primal-layout field to a dual-layout one: the
// first passes expand E + T^E(k) x (primal basis, E at k = 0), the column pass
// applies the coefficient on the quadrature grid, the last pass projects onto
// the dual basis T^J(k).
template <typename R>
hipError_t enqueue_cross_passes(const Geo& gin, const Geo& gout, const UnitDev* u, hipStream_t st) {
  hipError_t e = launch_first<R>(gin, u, 1, FIRST_BOUNDS, 0, nullptr, st);
  if (e != hipSuccess) return e;
  if (gin.d == 3 && !gin.plane) {
    e = launch_mid<R>(gin, u, 1, 1, st);
    if (e != hipSuccess) return e;
  }
  e = launch_apply<R>(gin, u, 1, APPLY_COEF, st);
  if (e != hipSuccess) return e;
  if (gin.d == 3 && !gin.plane) {
    e = launch_mid<R>(gin, u, 1, 0, st);
    if (e != hipSuccess) return e;
  }
  return launch_last<R>(gout, u, 1, LAST_MATVEC, 0, nullptr, st);
}

hipError_t enqueue_passes(bool fp32, const Geo& g, const UnitDev* u, int fm, int lm, int j, const int* ib,
                          hipStream_t st, int nu = 1) {
  return fp32 ? enqueue_matvec_passes<float>(g, u, nu, fm, lm, j, ib, st)
              : enqueue_matvec_passes<double>(g, u, nu, fm, lm, j, ib, st);
}

// gani: the coefficients of the GaNi operator (solves and operator application in GaNi mode)
void fill_unit(hom_problem* pb, int k, int L, const double* E, double* const* x, UnitDev* hu, bool gani = false) {
  std::memset(hu, 0, sizeof(*hu));
  SlotBufs& sb = pb->slot[k];
  const bool mixed = pb->desc.precision == HOM_MIXED;
  const GaniData& gn = pb->gani;
  if (gani) {
    hu->coef = gn.coef64[k];
    hu->ahat = gn.ahat[k];
  } else {
    hu->coef = mixed ? (const void*)pb->coef32[k] : (const void*)pb->coef64[k];
    hu->coefp = mixed ? pb->coefp[k] : nullptr;
    hu->ahat = pb->ahat_half[k];
  }
  for (int l = 0; l < L; ++l) {
    hu->x[l] = x ? reinterpret_cast<Cx<double>*>(x[l]) : sb.tmp[l];
    hu->r[l] = sb.r[l];
    hu->p[l] = sb.p[l];
    hu->s[l] = sb.s[l];
    hu->b[l] = sb.b[l];
    for (int c = 0; c < 3; ++c) hu->E[l][c] = (E && c < pb->desc.d) ? E[l * pb->desc.d + c] : 0.0;
  }
  // GaNi runs FP64 (see GaniData): the FP32-sized pass buffers of a mixed
  // problem are too small for it, the FP64 bound buffers hold its N-grid lines
  hu->bufA = (gani && mixed) ? pb->bbufA : sb.bufA;
  hu->bufB = (gani && mixed) ? pb->bbufB : sb.bufB;
  hu->part_g = sb.part_g;
  hu->part_d = sb.part_d;
  hu->part_q = sb.part_q;
  hu->sc = sb.sc;
}

// Validate loads and output pointers of one problem.
hom_status check_solve_args(const hom_problem* pb, int nload, const double* E, double* const* x_out, double tol,
                            int maxit) {
  if (!pb || !E || !x_out) return HOM_E_INVALID;
  if (nload < 1 || nload > pb->max_loads) return HOM_E_INVALID;
  if (!(tol > 0.0) || maxit < 0) return HOM_E_INVALID;
  for (int l = 0; l < nload; ++l) {
    if (!x_out[l]) return HOM_E_INVALID;
    double e2 = 0.0;
    for (int c = 0; c < pb->desc.d; ++c) {
      if (!std::isfinite(E[l * pb->desc.d + c])) return HOM_E_INVALID;
      e2 += E[l * pb->desc.d + c] * E[l * pb->desc.d + c];
    }
    if (e2 == 0.0) return HOM_E_INVALID;
  }
  return HOM_OK;
}

// Copy/symmetrise initial guesses into the outputs of one problem; returns whether any was given.
hom_status prepare_x0(hom_problem* pb, int k, int nload, const Geo& g, const double* const* x0,
                      double* const* x_out, bool* have) {
  hipStream_t st = pb->stream;
  SlotBufs& sb = pb->slot[k];
  *have = false;
  const size_t vbytes = (size_t)g.m * g.S * sizeof(Cx<double>);
  for (int l = 0; l < nload; ++l) {
    const double* src = x0 ? x0[l] : nullptr;
    if (!src) continue;
    *have = true;
    const Cx<double>* s = reinterpret_cast<const Cx<double>*>(src);
    if (src == x_out[l]) {
      HIPCHK(hipMemcpyAsync(sb.tmp[l], src, vbytes, hipMemcpyDeviceToDevice, st));
      s = sb.tmp[l];
    }
    HIPCHK(launch_symmetrize(g, s, reinterpret_cast<Cx<double>*>(x_out[l]), g.m, st));
  }
  return HOM_OK;
}

hom_status zero_missing_x0(hom_problem* pb, int k, int nload, const Geo& g, const double* const* x0,
                           double* const* x_out) {
  const size_t vbytes = (size_t)g.m * g.S * sizeof(Cx<double>);
  for (int l = 0; l < nload; ++l)
    if (!x0 || !x0[l]) HIPCHK(hipMemsetAsync(x_out[l], 0, vbytes, pb->stream));
  (void)k;
  return HOM_OK;
}

// CG over n units in lockstep (one unit = one problem's coefficient with nload loads).
struct SolveRun {
  hipStream_t st;
  Geo g;
  bool fp32;
  const UnitDev* units;       // device array of n units
  int n;
  int* iter_base;             // device
  int* active;                // device
  int* pinned_active;         // host, pinned
  hipGraphExec_t* graph;      // cache slot
  int chunk;
  std::vector<const double*> part_d;   // per unit, device
  std::vector<const CgScal*> sc;       // per unit, device
  // batches: end-of-solve summaries reduced on the device (n * L entries), one copy to pinned memory
  SolveOut* collect_dev = nullptr;
  SolveOut* collect_host = nullptr;
  // optional per-kernel timing: events recorded around every launch of the chunk
  std::vector<hipEvent_t>* events = nullptr;
  bool use_graph = false;              // set by start_run
  bool capture = true;                 // start_run captures the run's own chunk graph (groups capture theirs)
  StopCfg stop;                        // stopping rule
  int types[5] = {0, 0, 0, 0, 0};     // pass types of one iteration
  double* tsum = nullptr;              // [5] accumulated ms per pass type
  long long* tcnt = nullptr;           // [5] launches per pass type
};

// Pass types in launch order within one operator application (a plane pass
// counts as the column pass).
static int pass_types(const Geo& g, int* types) {
  const bool mid = g.d == 3 && !g.plane;
  int n = 0;
  types[n++] = 0;
  if (mid) types[n++] = 1;
  types[n++] = 2;
  if (mid) types[n++] = 3;
  types[n++] = 4;
  return n;
}

// One CG iteration with every kernel timed by its own start/stop event pair
// (hipExtLaunchKernelGGL); ev holds 2 events per pass.
template <typename R>
static hipError_t enqueue_timed_passes(const Geo& g, const UnitDev* u, int nu, int jstep, const int* iter_base,
                                       hipStream_t st, hipEvent_t* ev) {
  int k = 0;
  auto arm = [&]() {
    g_ext_timing.on = true;
    g_ext_timing.start = ev[2 * k];
    g_ext_timing.stop = ev[2 * k + 1];
    ++k;
  };
  hipError_t e;
  arm();
  e = launch_first<R>(g, u, nu, FIRST_CG, jstep, iter_base, st);
  if (e == hipSuccess && g.d == 3 && !g.plane) {
    arm();
    e = launch_mid<R>(g, u, nu, 1 | MID_CG, st);
  }
  if (e == hipSuccess) {
    arm();
    e = launch_apply<R>(g, u, nu, APPLY_COEF_CG, st);
  }
  if (e == hipSuccess && g.d == 3 && !g.plane) {
    arm();
    e = launch_mid<R>(g, u, nu, MID_CG, st);
  }
  if (e == hipSuccess) {
    arm();
    e = launch_last<R>(g, u, nu, LAST_CG, jstep, iter_base, st);
  }
  g_ext_timing.on = false;
  return e;
}

// One chunk of CG iterations of a run (direct launches, or the body of its graph).
hipError_t enqueue_chunk(SolveRun& R) {
  const Geo& g = R.g;
  hipStream_t st = R.st;
  const int npass = pass_types(g, R.types);
  for (int j = 0; j < R.chunk; ++j) {
    hipError_t e;
    if (R.events) {
      hipEvent_t* ev = R.events->data() + (size_t)j * 2 * npass;
      e = R.fp32 ? enqueue_timed_passes<float>(g, R.units, R.n, j, R.iter_base, st, ev)
                 : enqueue_timed_passes<double>(g, R.units, R.n, j, R.iter_base, st, ev);
    } else {
      e = enqueue_passes(R.fp32, g, R.units, FIRST_CG, LAST_CG, j, R.iter_base, st, R.n);
    }
    if (e != hipSuccess) return e;
  }
  hipError_t e = launch_advance(g, R.units, R.n, R.iter_base, R.chunk, R.active, st);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(R.pinned_active, R.active, sizeof(int), hipMemcpyDeviceToHost, st);
}

// Stage 1 of a solve: scalars, right-hand sides, start vectors (residual of a
// given start) and, for graph runs, the captured graph of one chunk.
hom_status start_run(SolveRun& R, int nload, double tol, int maxit, bool have_x0) {
  (void)nload;
  hipStream_t st = R.st;
  const Geo& g = R.g;
  // the guaranteed rule needs a lower bound on the spectrum of the operator: the
  // smallest eigenvalue of the coefficient over the doubled grid, per unit
  int mu_parts = 0;
  double mu_user = 0.0;
  R.chunk = std::max(1, R.chunk);
  if (R.stop.rule == 2 || R.stop.rule == 3) {
    const size_t npts = (size_t)g.M[0] * g.M[1] * g.M[2];
    mu_parts = (int)std::min<size_t>(64, (npts + kBlock - 1) / kBlock);
    HIPCHK(launch_coef_min_eig(R.fp32, g, R.units, R.n, mu_parts, st));
    mu_user = g.dual ? (R.stop.a_max > 0.0 ? 1.0 / R.stop.a_max : 0.0) : R.stop.a_min;
  }
  HIPCHK(launch_init_scal(g, R.units, R.n, R.iter_base, R.chunk, tol, maxit, R.stop.rule, R.stop.etol, mu_parts,
                          mu_user, st));
  HIPCHK(launch_rhs(g, R.units, R.n, st));
  HIPCHK(launch_start_vectors(g, R.units, R.n, have_x0 ? 1 : 0, st));
  if (have_x0) {
    HIPCHK(enqueue_passes(R.fp32, g, R.units, FIRST_FIELD, LAST_RESID, 0, nullptr, st, R.n));
    HIPCHK(launch_start_energy(g, R.units, R.n, st));
  }
  // events recorded inside a captured graph cannot be timed, so timing runs launch directly
  R.use_graph = st != nullptr && env_int("HOM_NO_GRAPH", 0) == 0 && R.events == nullptr;
  const int npass = pass_types(g, R.types);
  // event pairs for every pass of a chunk (a batch's chunk is longer in a group's single graph)
  if (R.events && R.events->size() < (size_t)R.chunk * 2 * npass) {
    const size_t have = R.events->size();
    R.events->resize((size_t)R.chunk * 2 * npass, nullptr);
    for (size_t i = have; i < R.events->size(); ++i) HIPCHK(hipEventCreate(&(*R.events)[i]));
  }
  hipGraphExec_t& gx = *R.graph;
  if (R.use_graph && R.capture && !gx) {
    hipGraph_t graph;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_chunk(R);
    hipError_t e2 = hipStreamEndCapture(st, &graph);
    if (e != hipSuccess || e2 != hipSuccess) return HOM_E_DEVICE;
    HIPCHK(hipGraphInstantiate(&gx, graph, nullptr, nullptr, 0));
    HIPCHK(hipGraphDestroy(graph));
  }
  return HOM_OK;
}

// Stage 2 of graph runs: the chunk graphs of several runs (on their own
// streams) replayed side by side until each has stopped.  One chunk per run
// stays in flight while the host reads the active count of the one before:
// the count is monotone and every pass of a finished unit returns at once, so
// a chunk enqueued after the last unit stopped changes nothing.
// partner (optional, per run: index of the partner run or -1): chunk c of a
// run starts after chunk c - 1 of its partner has ended (the partner's last
// chunk once it has stopped), so under the gap rule each reads the other's
// state at the end of the previous chunk, never a chunk being written.
// on_fin (optional; not for a run with a partner): called with ctx and the
// run's index as soon as the host sees the run stop, to enqueue its closing
// work on its stream while the other runs still iterate.
typedef hom_status (*RunFinHook)(void* ctx, int r);
hom_status loop_runs(SolveRun* const* runs, int nr, int maxit, const int* partner = nullptr,
                     RunFinHook on_fin = nullptr, void* ctx = nullptr) {
  std::vector<hipEvent_t> ev((size_t)2 * nr, nullptr);
  hom_status hs = HOM_OK;
  std::vector<int> it(nr, 0), done(nr, 0), fin(nr, 0), launched(nr, 0);
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < ev.size() && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
  auto launch = [&](int r) {
    const int c = launched[r];
    const int p = partner ? partner[r] : -1;
    if (p >= 0 && c > 0) {
      // the partner's chunk c - 1, or its last one: slot parity of that chunk
      const int pc = std::min(c - 1, launched[p] - 1);
      if (pc >= 0) e = hipStreamWaitEvent(runs[r]->st, ev[2 * p + (pc & 1)], 0);
    }
    if (e == hipSuccess) e = hipGraphLaunch(*runs[r]->graph, runs[r]->st);
    if (e == hipSuccess) e = hipEventRecord(ev[2 * r + (c & 1)], runs[r]->st);
    ++launched[r];
  };
  for (int r = 0; r < nr && e == hipSuccess; ++r) launch(r);
  int left = nr;
  while (e == hipSuccess && left > 0) {
    for (int r = 0; r < nr && e == hipSuccess; ++r) {
      if (fin[r]) continue;
      launch(r);
    }
    for (int r = 0; r < nr && e == hipSuccess; ++r) {
      if (fin[r]) continue;
      e = hipEventSynchronize(ev[2 * r + (it[r] & 1)]);
      if (e != hipSuccess) break;
      done[r] += runs[r]->chunk;
      ++it[r];
      if (*runs[r]->pinned_active == 0 || done[r] > maxit + runs[r]->chunk) {
        fin[r] = 1;
        --left;
        if (on_fin && !(partner && partner[r] >= 0)) {
          hs = on_fin(ctx, r);
          if (hs != HOM_OK) break;
        }
      }
    }
    if (hs != HOM_OK) break;
  }
  for (int r = 0; r < nr && e == hipSuccess; ++r) e = hipStreamSynchronize(runs[r]->st);
  for (auto x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) return HOM_E_DEVICE;
  return hs;
}

// Per-kernel event times of the chunk just completed, into the run's sums.
hom_status collect_events(SolveRun& R) {
  if (!R.events) return HOM_OK;
  const int npass = pass_types(R.g, R.types);
  for (int j = 0; j < R.chunk; ++j) {
    hipEvent_t* ev = R.events->data() + (size_t)j * 2 * npass;
    for (int p = 0; p < npass; ++p) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ev[2 * p], ev[2 * p + 1]));
      R.tsum[R.types[p]] += ms;
      R.tcnt[R.types[p]] += 1;
    }
  }
  return HOM_OK;
}

// Stage 2 of direct runs (no graph, optionally with per-kernel events): the
// runs advance one chunk each in turn (for partners, chunk c of each after
// chunk c - 1 of the other, as in loop_runs), each chunk waited for.
hom_status loop_direct(SolveRun* const* runs, int nr, int maxit) {
  std::vector<int> done(nr, 0), fin(nr, 0);
  int left = nr;
  while (left > 0) {
    for (int r = 0; r < nr; ++r) {
      if (fin[r]) continue;
      SolveRun& R = *runs[r];
      HIPCHK(enqueue_chunk(R));
      HIPCHK(hipStreamSynchronize(R.st));
      hom_status s = collect_events(R);
      if (s != HOM_OK) return s;
      done[r] += R.chunk;
      if (*R.pinned_active == 0 || done[r] > maxit + R.chunk) {
        fin[r] = 1;
        --left;
      }
    }
  }
  return HOM_OK;
}

// Stage 3: true residual b - C x of the returned iterates (in the precision
// mode of the solve) and the per-load summaries.  finish_enqueue puts the
// residual passes (and, with a summary workspace, its collection and copy to
// the host) on the run's stream; finish_run waits for them and reads.  Runs on
// different streams enqueue first and read afterwards, so their residual
// passes overlap.
static hom_status finish_enqueue(SolveRun& R, int nload) {
  hipStream_t st = R.st;
  const Geo& g = R.g;
  HIPCHK(enqueue_passes(R.fp32, g, R.units, FIRST_FIELD, LAST_RESID, 0, nullptr, st, R.n));
  if (R.collect_dev) {
    HIPCHK(launch_collect_solve(R.units, R.n, nload, g.nbL, R.collect_dev, st));
    HIPCHK(hipMemcpyAsync(R.collect_host, R.collect_dev, (size_t)R.n * nload * sizeof(SolveOut),
                          hipMemcpyDeviceToHost, st));
  }
  return HOM_OK;
}

hom_status finish_run(SolveRun& R, int nload, int maxit, hom_info* info, bool enqueued = false) {
  if (!enqueued) {
    hom_status s = finish_enqueue(R, nload);
    if (s != HOM_OK) return s;
  }
  hipStream_t st = R.st;
  const Geo& g = R.g;
  // partial sums of the residual pass ([load][nbL] per unit) and the CG scalars
  const size_t nbl = (size_t)g.nbL;
  std::vector<double> rres((size_t)R.n * nload);
  std::vector<CgScal> sc((size_t)R.n * nload);
  if (R.collect_dev) {
    HIPCHK(hipStreamSynchronize(st));
    for (size_t ul = 0; ul < (size_t)R.n * nload; ++ul) {
      rres[ul] = R.collect_host[ul].rres;
      sc[ul] = R.collect_host[ul].sc;
    }
  } else {
    std::vector<double> part((size_t)R.n * nload * nbl);
    for (int u = 0; u < R.n; ++u) {
      HIPCHK(hipMemcpyAsync(part.data() + (size_t)u * nload * nbl, R.part_d[u], (size_t)nload * nbl * sizeof(double),
                            hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(sc.data() + (size_t)u * nload, R.sc[u], nload * sizeof(CgScal), hipMemcpyDeviceToHost,
                            st));
    }
    HIPCHK(hipStreamSynchronize(st));
    for (size_t ul = 0; ul < (size_t)R.n * nload; ++ul) {
      double s = 0.0;
      for (size_t q = 0; q < nbl; ++q) s += part[ul * nbl + q];
      rres[ul] = s;
    }
  }
  hom_status worst = HOM_OK;
  for (int u = 0; u < R.n; ++u)
    for (int l = 0; l < nload; ++l) {
      const size_t ul = (size_t)u * nload + l;
      const double s = rres[ul];
      hom_info& in = info[ul];
      in.iters = sc[ul].iters;
      in.rel_res_recur = std::sqrt(std::max(sc[ul].gamma_last, 0.0)) / sc[ul].normE;
      in.rel_res_true = std::sqrt(std::max(s, 0.0)) / sc[ul].normE;
      in.energy = sc[ul].energy0 - sc[ul].esum;
      const int stt = sc[ul].status;
      hom_status h;
      if (stt == 1) h = HOM_OK;
      else if (stt == 2 || stt == 0) h = HOM_NOT_CONVERGED;
      else if (stt == -3) h = HOM_E_NOT_SPD;
      else h = HOM_E_INVALID;
      if (stt == 0) in.iters = maxit;
      in.status = h;
      if (h < 0 && (worst >= 0 || h < worst)) worst = h;
      else if (h == HOM_NOT_CONVERGED && worst == HOM_OK) worst = h;
    }
  return worst;
}

hom_status solve_units(SolveRun& R, int nload, double tol, int maxit, bool have_x0, hom_info* info) {
  hom_status s = start_run(R, nload, tol, maxit, have_x0);
  if (s != HOM_OK) return s;
  SolveRun* one = &R;
  s = R.use_graph ? loop_runs(&one, 1, maxit) : loop_direct(&one, 1, maxit);
  if (s != HOM_OK) return s;
  return finish_run(R, nload, maxit, info);
}

// Tile shapes for solves of nload loads over the problems pbs (one unit each in
// the device array units): the process-wide choice for this geometry, timed
// on first use with the units pointed at the problems' scratch vectors.
hom_status solve_tuning(hom_problem* const* pbs, int n, int k, int nload, UnitDev* units, hipStream_t st,
                        Tuning* out) {
  hom_problem* p0 = pbs[0];
  *out = Tuning();
  if (p0->desc.precision != HOM_MIXED || !tuning_on()) return HOM_OK;
  const Geo g = make_geo(p0, k, nload, true);
  const TuneKey key{g.M[0], g.M[1], g.M[2], g.d, nload, k, g.nc, g.P};
  const char* file = std::getenv("HOM_TUNE_CACHE");
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (file && *file && !g_tune_file_read) {
      g_tune_file_read = true;
      (void)tune_file_read(file, device_arch(), nullptr);    // a missing or foreign file only costs the timing
    }
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      *out = it->second;
      return HOM_OK;
    }
  }
  std::vector<UnitDev> hu(n);
  for (int i = 0; i < n; ++i) fill_unit(pbs[i], k, nload, nullptr, nullptr, &hu[i]);
  HIPCHK(hipMemcpyAsync(units, hu.data(), (size_t)n * sizeof(UnitDev), hipMemcpyHostToDevice, st));
  Tuning t;
  HIPCHK(tune_fast(g, units, n, st, std::max(1, env_int("HOM_TUNE_REPS", 3)), &t));
  HIPCHK(hipStreamSynchronize(st));
  std::lock_guard<std::mutex> lk(g_tune_mu);
  *out = g_tune_cache.emplace(key, t).first->second;
  if (file && *file) (void)tune_file_write(file, device_arch());
  return HOM_OK;
}

hom_status solve_impl(hom_problem* pb, int k, int nload, const double* E, const double* const* x0, double tol,
                      int maxit, double* const* x_out, hom_info* info) {
  hom_status s = check_solve_args(pb, nload, E, x_out, tol, maxit);
  if (s != HOM_OK) return s;
  if (!info || pb->stop.rule == 3) return HOM_E_INVALID;   // the gap rule needs the pair solve
  hipStream_t st = pb->stream;
  const bool gani = pb->gani.on;
  const bool fp32 = pb->desc.precision == HOM_MIXED && !gani;
  SlotBufs& sb = pb->slot[k];
  if (!gani && !pb->tuned[k][nload]) {
    s = solve_tuning(&pb, 1, k, nload, sb.unit, st, &pb->tune[k][nload]);
    if (s != HOM_OK) return s;
    pb->tuned[k][nload] = true;
  }
  Geo g = gani ? make_geo_gani(pb, k, nload, fp32) : make_geo(pb, k, nload, fp32, 0, &pb->tune[k][nload]);
  UnitDev* hu = &pb->host_unit[k];
  fill_unit(pb, k, nload, E, x_out, hu, gani);
  HIPCHK(hipMemcpyAsync(sb.unit, hu, sizeof(UnitDev), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  bool have_x0 = false;
  s = prepare_x0(pb, k, nload, g, x0, x_out, &have_x0);
  if (s != HOM_OK) return s;
  if (have_x0) {
    s = zero_missing_x0(pb, k, nload, g, x0, x_out);
    if (s != HOM_OK) return s;
  }
  SolveRun R;
  R.st = st;
  R.g = g;
  R.fp32 = fp32;
  R.units = sb.unit;
  R.n = 1;
  R.iter_base = sb.iter_base;
  R.active = sb.active;
  R.pinned_active = pb->pinned_active;
  R.graph = gani ? &pb->gani.graph[k][nload] : &pb->graph[k][nload];
  R.chunk = pb->graph_chunk;
  R.stop = pb->stop;
  R.part_d.push_back(sb.part_d);
  R.sc.push_back(sb.sc);
  return solve_units(R, nload, tol, maxit, have_x0, info);
}

void inv_small(int d, const double* A, double* X) {
  if (d == 2) {
    const double det = A[0] * A[3] - A[1] * A[2];
    X[0] = A[3] / det;
    X[1] = -A[1] / det;
    X[2] = -A[2] / det;
    X[3] = A[0] / det;
  } else {
    const double a = A[0], b = A[1], c = A[2], dd = A[3], e = A[4], f = A[5], g = A[6], h = A[7], i = A[8];
    const double C00 = e * i - f * h, C01 = -(dd * i - f * g), C02 = dd * h - e * g;
    const double det = a * C00 + b * C01 + c * C02;
    X[0] = C00 / det;
    X[1] = -(b * i - c * h) / det;
    X[2] = (b * f - c * e) / det;
    X[3] = C01 / det;
    X[4] = (a * i - c * g) / det;
    X[5] = -(a * f - c * dd) / det;
    X[6] = C02 / det;
    X[7] = -(a * h - b * g) / det;
    X[8] = (a * e - b * dd) / det;
  }
}

void fill_result(int d, const double Ebar[2][9], const bool have[2], hom_result* out) {
  std::memset(out, 0, sizeof(*out));
  for (int i = 0; i < 9; ++i)
    out->A_up[i] = out->B_up[i] = out->A_low[i] = out->A_mean[i] = out->D[i] = (i < d * d) ? NAN : 0.0;
  for (int i = 0; i < d * d; ++i) {
    out->A_up[i] = Ebar[0][i];
    out->B_up[i] = Ebar[1][i];
  }
  if (have[1]) inv_small(d, Ebar[1], out->A_low);
  for (int i = 0; i < d * d; ++i) {
    out->A_mean[i] = 0.5 * (out->A_up[i] + out->A_low[i]);
    out->D[i] = 0.5 * (out->A_up[i] - out->A_low[i]);
  }
}

void coef_components(int d, int nc, const double* A, double* out) {
  if (nc == 1) {
    out[0] = A[0];
  } else if (d == 2) {
    out[0] = A[0];
    out[1] = A[3];
    out[2] = A[1];
  } else {
    out[0] = A[0];
    out[1] = A[4];
    out[2] = A[8];
    out[3] = A[1];
    out[4] = A[2];
    out[5] = A[5];
  }
}

void twiddles(int M, std::vector<Cx<double>>& t64, std::vector<Cx<float>>& t32) {
  t64.resize(M);
  t32.resize(M);
  for (int t = 0; t < M; ++t) {
    // exp(-2 pi i t / M) from the DFT definition, evaluated in double
    const double a = -2.0 * M_PI * (double)t / (double)M;
    t64[t].x = std::cos(a);
    t64[t].y = std::sin(a);
    t32[t].x = (float)t64[t].x;
    t32[t].y = (float)t64[t].y;
  }
}

// Coefficient on the doubled grid, A_M(x^k) = sum_n omega^{kn} A_hat(n) (eq. MBA_GA), in FP64 on the
// device, its FP32 copy, and the Z_N part of A_hat; stream-ordered, no host synchronisation.
hom_status setup_coefficients(hom_problem* pb, const void* Ahat, const void* Bhat) {
  const Sizes& z = pb->z;
  hipStream_t st = pb->stream;
  Geo g = make_geo(pb, 0, 1, false);
  const int nc = z.nc;
  {
    const Cx<double>* A = reinterpret_cast<const Cx<double>*>(Ahat);
    const Cx<double>* B = reinterpret_cast<const Cx<double>*>(Bhat);
    hipError_t e = hipSuccess;
    if (fast_coef_setup(z.d, z.M, nc, A, B, pb->scratch, pb->coef64[0], pb->coef32[0], pb->coef64[1], pb->coef32[1],
                        pb->tw64[0], st, &e)) {
      HIPCHK(e);
      HIPCHK(launch_extract_half(g, A, pb->ahat_half[0], nc, st));
      HIPCHK(launch_extract_half(g, B, pb->ahat_half[1], nc, st));
      return HOM_OK;
    }
  }
  for (int k = 0; k < 2; ++k) {
    const void* src = k == 0 ? Ahat : Bhat;
    HIPCHK(hipMemcpyAsync(pb->scratch, src, nc * z.Mt * sizeof(Cx<double>), hipMemcpyDeviceToDevice, st));
    HIPCHK(launch_extract_half(g, pb->scratch, pb->ahat_half[k], nc, st));
    HIPCHK(launch_line_fft<double>(pb->scratch, nc, z.M[0], z.M[1] * z.M[2], pb->plan[0], pb->tw64[0], 1, st));
    if (z.M[1] > 1)
      HIPCHK(launch_line_fft<double>(pb->scratch, nc * z.M[0], z.M[1], z.M[2], pb->plan[1], pb->tw64[1], 1, st));
    HIPCHK(launch_line_fft<double>(pb->scratch, nc * z.M[0] * z.M[1], z.M[2], 1, pb->plan[2], pb->tw64[2], 1, st));
    HIPCHK(launch_coef_real(pb->scratch, pb->coef64[k], pb->coef32[k], (long)(nc * z.Mt), st));
    if (pb->coefp[k]) HIPCHK(launch_coef_planes(pb->coef32[k], pb->coefp[k], nc, z.M, st));
  }
  return HOM_OK;
}

}  // namespace

extern "C" {

const char* hom_status_str(int32_t s) {
  switch (s) {
    case HOM_OK: return "HOM_OK";
    case HOM_NOT_CONVERGED: return "HOM_NOT_CONVERGED";
    case HOM_E_INVALID: return "HOM_E_INVALID";
    case HOM_E_UNSUPPORTED_SIZE: return "HOM_E_UNSUPPORTED_SIZE";
    case HOM_E_NOT_SPD: return "HOM_E_NOT_SPD";
    case HOM_E_DEVICE: return "HOM_E_DEVICE";
    case HOM_E_WORKSPACE: return "HOM_E_WORKSPACE";
    default: return "HOM_UNKNOWN";
  }
}

hom_status hom_field_len(const hom_desc* desc, int32_t dual, size_t* n) {
  // depends on N only: S = ((N0 + 1) / 2) N1 (N2) stored frequencies per component
  if (!desc || !n || (desc->d != 2 && desc->d != 3)) return HOM_E_INVALID;
  const int d = desc->d;
  size_t S = 1;
  for (int a = 0; a < d; ++a) {
    if (desc->N[a] < 1 || desc->N[a] % 2 == 0) return HOM_E_UNSUPPORTED_SIZE;
    S *= (size_t)(a == 0 ? (desc->N[0] + 1) / 2 : desc->N[a]);
  }
  *n = (size_t)(dual ? d - 1 : 1) * S;
  return HOM_OK;
}

hom_status hom_workspace_bytes(const hom_desc* desc, int32_t max_loads, size_t* bytes) {
  hom_status s = validate_desc(desc, max_loads);
  if (s != HOM_OK) return s;
  if (!bytes) return HOM_E_INVALID;
  Sizes z;
  Plan pl[3];
  fill_sizes(desc, max_loads, &z, pl);
  *bytes = carve(desc, max_loads, z, nullptr);
  return HOM_OK;
}

hom_status hom_setup(const hom_desc* desc, int32_t max_loads, const void* Ahat, const void* Bhat, void* ws,
                     size_t ws_bytes, void* stream, hom_problem** out) {
  hom_status s = validate_desc(desc, max_loads);
  if (s != HOM_OK) return s;
  if (!Ahat || !Bhat || !ws || !out) return HOM_E_INVALID;
  if (((uintptr_t)ws) % kAlign) return HOM_E_WORKSPACE;
  Sizes z;
  Plan pl[3];
  fill_sizes(desc, max_loads, &z, pl);
  const size_t need = carve(desc, max_loads, z, nullptr);
  if (ws_bytes < need) return HOM_E_WORKSPACE;
  hom_problem* pb = new hom_problem();
  std::memset((void*)pb, 0, sizeof(*pb));
  pb->desc = *desc;
  pb->max_loads = max_loads;
  pb->stream = reinterpret_cast<hipStream_t>(stream);
  pb->ws = (char*)ws;
  pb->ws_bytes = ws_bytes;
  pb->z = z;
  for (int a = 0; a < 3; ++a) pb->plan[a] = pl[a];
  // iterations per captured chunk: a 3D iteration is long enough (about a millisecond on a batch) that
  // the host can poll every second one, so a solve that stops is seen sooner and its closing work
  // starts sooner; 2D iterations are far shorter
  pb->graph_chunk = env_int("HOM_CHUNK", z.d == 3 ? 2 : 8);
  carve(desc, max_loads, z, pb);
  if (hipHostMalloc((void**)&pb->pinned_active, sizeof(int), hipHostMallocDefault) != hipSuccess) {
    delete pb;
    return HOM_E_DEVICE;
  }
  hipStream_t st = pb->stream;
  for (int a = 0; a < 3; ++a)
    if (launch_twiddles(pb->tw64[a], pb->tw32[a], z.M[a], st) != hipSuccess) {
      (void)hipHostFree(pb->pinned_active);
      delete pb;
      return HOM_E_DEVICE;
    }
  hom_status rc = setup_coefficients(pb, Ahat, Bhat);
  if (rc != HOM_OK) {
    (void)hipStreamSynchronize(st);
    (void)hipHostFree(pb->pinned_active);
    delete pb;
    return rc;
  }
  *out = pb;
  return HOM_OK;
}

hom_status hom_update_coefficients(hom_problem* pb, const void* Ahat, const void* Bhat) {
  if (!pb || !Ahat || !Bhat) return HOM_E_INVALID;
  return setup_coefficients(pb, Ahat, Bhat);
}

hom_status hom_solve_primal(hom_problem* pb, int32_t nload, const double* E, const double* const* x0, double tol,
                            int32_t maxit, double* const* x_out, hom_info* info) {
  return solve_impl(pb, 0, nload, E, x0, tol, maxit, x_out, info);
}

hom_status hom_solve_dual(hom_problem* pb, int32_t nload, const double* J, const double* const* x0, double tol,
                          int32_t maxit, double* const* x_out, hom_info* info) {
  return solve_impl(pb, 1, nload, J, x0, tol, maxit, x_out, info);
}

hom_status hom_apply(hom_problem* pb, int32_t dual, const double* x, double* y) {
  if (!pb || !x || !y || (dual != 0 && dual != 1)) return HOM_E_INVALID;
  const int k = dual;
  hipStream_t st = pb->stream;
  const bool fp32 = pb->desc.precision == HOM_MIXED && !pb->gani.on;
  Geo g = pb->gani.on ? make_geo_gani(pb, k, 1, fp32) : make_geo(pb, k, 1, fp32);
  SlotBufs& sb = pb->slot[k];
  UnitDev* hu = &pb->host_unit[k];
  fill_unit(pb, k, 1, nullptr, nullptr, hu, pb->gani.on);
  hu->x[0] = reinterpret_cast<Cx<double>*>(const_cast<double*>(x));
  hu->s[0] = reinterpret_cast<Cx<double>*>(y);
  HIPCHK(hipMemcpyAsync(sb.unit, hu, sizeof(UnitDev), hipMemcpyHostToDevice, st));
  HIPCHK(enqueue_passes(fp32, g, sb.unit, FIRST_FIELD, LAST_MATVEC, 0, nullptr, st));
  HIPCHK(hipStreamSynchronize(st));
  return HOM_OK;
}

hom_status hom_probe_copy(const void* src, void* dst, size_t bytes, int32_t reps, void* stream, double* gbs) {
  if (!src || !dst || !gbs || reps < 1 || bytes < 16 || bytes % 16) return HOM_E_INVALID;
  if (((uintptr_t)src) % 16 || ((uintptr_t)dst) % 16) return HOM_E_INVALID;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return HOM_E_DEVICE;
  }
  hipError_t e = launch_stream_copy(src, dst, bytes, st);   // untimed: first-launch costs
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_stream_copy(src, dst, bytes, st);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess || !(ms > 0.f)) return HOM_E_DEVICE;
  *gbs = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;   // bytes read plus bytes written
  return HOM_OK;
}

hom_status hom_dual_start(hom_problem* pb, const double* const* primal, const double* Abar, double* const* x0_dual) {
  if (!pb || !primal || !Abar || !x0_dual) return HOM_E_INVALID;
  const int d = pb->desc.d;
  for (int a = 0; a < d; ++a)
    if (!primal[a] || !x0_dual[a]) return HOM_E_INVALID;
  // E^(b) = Abar^-1 e_b, column b of the inverse of the (symmetric positive definite) homogenised matrix
  double Am[9], Ai[9];
  for (int i = 0; i < d * d; ++i) {
    Am[i] = Abar[i];
    if (!std::isfinite(Am[i])) return HOM_E_INVALID;
  }
  for (int a = 0; a < d; ++a) {
    if (!(Am[a * d + a] > 0.0)) return HOM_E_INVALID;
    for (int b = 0; b < a; ++b)
      if (std::fabs(Am[a * d + b] - Am[b * d + a]) > 1e-12 * (std::fabs(Am[a * d + a]) + std::fabs(Am[b * d + b])))
        return HOM_E_INVALID;
  }
  inv_small(d, Am, Ai);
  for (int i = 0; i < d * d; ++i)
    if (!std::isfinite(Ai[i])) return HOM_E_INVALID;
  hipStream_t st = pb->stream;
  const bool gani = pb->gani.on;
  const bool fp32 = pb->desc.precision == HOM_MIXED && !gani;
  const Geo gin = gani ? make_geo_gani(pb, 0, 1, fp32) : make_geo(pb, 0, 1, fp32);
  const Geo gout = gani ? make_geo_gani(pb, 1, 1, fp32) : make_geo(pb, 1, 1, fp32);
  SlotBufs& sb = pb->slot[0];
  const size_t n = (size_t)gin.m * gin.S;   // complex entries of a primal field
  FieldTriple xt{};
  for (int a = 0; a < d; ++a) xt.p[a] = reinterpret_cast<const Cx<double>*>(primal[a]);
  UnitDev* hu = &pb->host_unit[0];
  for (int b = 0; b < d; ++b) {
    double w[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < d; ++a) w[a] = Ai[a * d + b];
    // the combined fluctuation sum_a E_a x^(a) (linear in the fields), and E itself at k = 0
    HIPCHK(launch_combine(xt, d, w, sb.tmp[0], n, st));
    fill_unit(pb, 0, 1, w, nullptr, hu, gani);
    hu->s[0] = reinterpret_cast<Cx<double>*>(x0_dual[b]);
    HIPCHK(hipMemcpyAsync(sb.unit, hu, sizeof(UnitDev), hipMemcpyHostToDevice, st));
    HIPCHK(fp32 ? enqueue_cross_passes<float>(gin, gout, sb.unit, st)
                : enqueue_cross_passes<double>(gin, gout, sb.unit, st));
    HIPCHK(hipStreamSynchronize(st));   // the host unit record is reused for the next load
  }
  return HOM_OK;
}

// Energy matrices a(e_b + x^(b), e_a + x^(a)) of primal and dual fields by the
// FP64 quadrature of a geometry: the exact form on the quadrature grid (gani =
// false, the bounds), or the trapezoidal rule on the N grid with the point
// values of the coefficient (gani = true, the GaNi matrices).
static hom_status energies(hom_problem* pb, const double* const* primal, const double* const* dual, bool gani,
                           double Ebar[2][9], bool have[2]) {
  const int d = pb->desc.d;
  for (int k = 0; k < 2; ++k) {
    const double* const* f = k == 0 ? primal : dual;
    if (f)
      for (int a = 0; a < d; ++a)
        if (!f[a]) return HOM_E_INVALID;
  }
  hipStream_t st = pb->stream;
  const int P = packs(d, d);
  have[0] = primal != nullptr;
  have[1] = dual != nullptr;
  std::vector<double> part[2];
  Geo g[2];
  for (int k = 0; k < 2; ++k) {
    if (!have[k]) continue;
    const double* const* f = k == 0 ? primal : dual;
    g[k] = gani ? make_geo_gani(pb, k, d, false, P) : make_geo(pb, k, d, false, P);
    UnitDev* hu = &pb->host_bunit[k];
    std::memset(hu, 0, sizeof(*hu));
    hu->coef = gani ? pb->gani.coef64[k] : pb->coef64[k];
    hu->ahat = gani ? pb->gani.ahat[k] : pb->ahat_half[k];
    for (int l = 0; l < d; ++l) {
      hu->x[l] = reinterpret_cast<Cx<double>*>(const_cast<double*>(f[l]));
      hu->E[l][l] = 1.0;
    }
    hu->bufA = pb->bbufA;
    hu->bufB = pb->bbufB;
    hu->part_q = pb->bpart_q[k];
    HIPCHK(hipMemcpyAsync(pb->bunit[k], hu, sizeof(UnitDev), hipMemcpyHostToDevice, st));
    HIPCHK(launch_first<double>(g[k], pb->bunit[k], 1, FIRST_BOUNDS, 0, nullptr, st));
    if (d == 3) HIPCHK(launch_mid<double>(g[k], pb->bunit[k], 1, 1, st));
    HIPCHK(launch_apply<double>(g[k], pb->bunit[k], 1, APPLY_QUAD, st));
    part[k].resize((size_t)g[k].nbA * 9);
    HIPCHK(hipMemcpyAsync(part[k].data(), pb->bpart_q[k], part[k].size() * sizeof(double), hipMemcpyDeviceToHost,
                          st));
  }
  HIPCHK(hipStreamSynchronize(st));
  for (int k = 0; k < 2; ++k) {
    for (int i = 0; i < 9; ++i) Ebar[k][i] = NAN;
    if (!have[k]) continue;
    for (int a = 0; a < d; ++a)
      for (int b = 0; b < d; ++b) {
        double s = 0.0;
        for (int q = 0; q < g[k].nbA; ++q) s += part[k][(size_t)q * 9 + a * kMaxLoads + b];
        Ebar[k][a * d + b] = s * g[k].invM;
      }
  }
  return HOM_OK;
}

hom_status hom_bounds(hom_problem* pb, const double* const* primal, const double* const* dual, hom_result* out) {
  if (!pb || !out) return HOM_E_INVALID;
  double Ebar[2][9];
  bool have[2];
  hom_status s = energies(pb, primal, dual, false, Ebar, have);
  if (s != HOM_OK) return s;
  fill_result(pb->desc.d, Ebar, have, out);
  return HOM_OK;
}

hom_status hom_gani_matrices(hom_problem* pb, const double* const* primal, const double* const* dual,
                             double* A_HN, double* B_HN) {
  if (!pb || !pb->gani.on || !A_HN || !B_HN) return HOM_E_INVALID;
  double Ebar[2][9];
  bool have[2];
  hom_status s = energies(pb, primal, dual, true, Ebar, have);
  if (s != HOM_OK) return s;
  const int d = pb->desc.d;
  for (int i = 0; i < d * d; ++i) {
    A_HN[i] = have[0] ? Ebar[0][i] : NAN;
    B_HN[i] = have[1] ? Ebar[1][i] : NAN;
  }
  return HOM_OK;
}

size_t gani_carve(const hom_desc* desc, const Sizes& z, const int* grid, GaniData* gd, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> size_t {
    const size_t o = off;
    off = up(off + bytes);
    return o;
  };
  auto ptr = [&](size_t o) -> char* { return base ? base + o : nullptr; };
  const int nc = z.nc;
  const size_t Nt = (size_t)grid[0] * grid[1] * grid[2];
  (void)desc;
  for (int k = 0; k < 2; ++k) {
    size_t o = take(nc * Nt * sizeof(double));
    if (gd) gd->coef64[k] = (double*)ptr(o);
    o = take(nc * (size_t)z.S * sizeof(Cx<double>));
    if (gd) gd->ahat[k] = (Cx<double>*)ptr(o);
  }
  for (int a = 0; a < 3; ++a) {
    size_t o = take(grid[a] * sizeof(Cx<double>));
    if (gd) gd->tw64[a] = (Cx<double>*)ptr(o);
    o = take(grid[a] * sizeof(Cx<float>));
    if (gd) gd->tw32[a] = (Cx<float>*)ptr(o);
  }
  size_t o = take(nc * Nt * sizeof(Cx<double>));
  if (gd) gd->scratch = (Cx<double>*)ptr(o);
  return off;
}

hom_status hom_smooth_pixels(const int32_t* P, const int32_t* f, int32_t* out, int32_t d, const double* A01,
                             double* table, void* stream) {
  if (!P || !f || !out || P[0] < 1 || P[1] < 1) return HOM_E_INVALID;
  if (table && (d != 2 || !A01)) return HOM_E_INVALID;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (launch_smooth2d(P[0], P[1], f, out, st) != hipSuccess) return HOM_E_DEVICE;
  if (table)       // phase k of the smoothed medium: A0 + (k/16)(A1 - A0), k = 0..16
    for (int k = 0; k <= 16; ++k)
      for (int i = 0; i < d * d; ++i) table[k * d * d + i] = A01[i] + (k / 16.0) * (A01[d * d + i] - A01[i]);
  return hipStreamSynchronize(st) == hipSuccess ? HOM_OK : HOM_E_DEVICE;
}

// GaNi grid on internal axes from the caller's physical grid (NULL: N); every
// grid[a] is N_a or the even N_a + 1 with factors 2, 3 and 5 only.
hom_status gani_grid(const hom_desc* desc, const Sizes& z, const int32_t* grid, int* gi, Plan* plans) {
  const int d = desc->d;
  int phys[3] = {0, 0, 0};
  for (int a = 0; a < d; ++a) phys[a] = grid ? grid[a] : desc->N[a];
  if (d == 2) {
    gi[0] = phys[0];
    gi[1] = 1;
    gi[2] = phys[1];
  } else {
    for (int a = 0; a < 3; ++a) gi[a] = phys[a];
  }
  for (int a = 0; a < 3; ++a) {
    if (gi[a] != z.N[a] && gi[a] != z.N[a] + 1) return HOM_E_UNSUPPORTED_SIZE;
    if (gi[a] > z.M[a]) return HOM_E_UNSUPPORTED_SIZE;  // the passes' buffers hold the quadrature grid
    if (gi[a] == 1) {
      plans[a].n = 0;
    } else if (!smooth235(gi[a], &plans[a])) {
      return HOM_E_UNSUPPORTED_SIZE;
    }
  }
  return HOM_OK;
}

hom_status hom_gani_workspace_bytes(const hom_desc* desc, const int32_t* grid, size_t* bytes) {
  if (!bytes) return HOM_E_INVALID;
  hom_status s = validate_desc(desc, 1);
  if (s != HOM_OK) return s;
  Sizes z;
  Plan pl[3];
  if (!fill_sizes(desc, 1, &z, pl)) return HOM_E_INVALID;
  int gi[3];
  Plan gp[3];
  s = gani_grid(desc, z, grid, gi, gp);
  if (s != HOM_OK) return s;
  *bytes = gani_carve(desc, z, gi, nullptr, nullptr);
  return HOM_OK;
}

hom_status hom_set_gani(hom_problem* pb, const int32_t* grid, const double* AN, const double* BN, void* ws,
                        size_t ws_bytes) {
  if (!pb || !AN || !BN || !ws) return HOM_E_INVALID;
  if (((uintptr_t)ws) % kAlign) return HOM_E_WORKSPACE;
  size_t need = 0;
  hom_status s = hom_gani_workspace_bytes(&pb->desc, grid, &need);
  if (s != HOM_OK) return s;
  if (ws_bytes < need) return HOM_E_WORKSPACE;
  GaniData& gd = pb->gani;
  const Sizes& z = pb->z;
  hipStream_t st = pb->stream;
  HIPCHK(hipStreamSynchronize(st));
  for (int k = 0; k < 2; ++k)
    for (int l = 0; l <= kMaxLoads; ++l)
      if (gd.graph[k][l]) {
        (void)hipGraphExecDestroy(gd.graph[k][l]);
        gd.graph[k][l] = nullptr;
      }
  gd.on = false;
  s = gani_grid(&pb->desc, z, grid, gd.grid, gd.plan);
  if (s != HOM_OK) return s;
  gani_carve(&pb->desc, z, gd.grid, &gd, (char*)ws);
  for (int a = 0; a < 3; ++a) HIPCHK(launch_twiddles(gd.tw64[a], gd.tw32[a], gd.grid[a], st));
  const int nc = z.nc;
  const int* G = gd.grid;
  const size_t Nt = (size_t)G[0] * G[1] * G[2];
  Geo g = make_geo_gani(pb, 0, 1, false);
  for (int k = 0; k < 2; ++k) {
    const double* src = k == 0 ? AN : BN;
    HIPCHK(hipMemcpyAsync(gd.coef64[k], src, nc * Nt * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(launch_real_to_cx(gd.coef64[k], gd.scratch, nc * Nt, 1.0, st));
    // Fourier coefficients of the point values: the grid DFT over the number of points, kept on
    // Z_N (the Nyquist frequencies of an even grid are dropped with the truncation)
    if (G[0] > 1) HIPCHK(launch_line_fft<double>(gd.scratch, nc, G[0], G[1] * G[2], gd.plan[0], gd.tw64[0], 0, st));
    if (G[1] > 1) HIPCHK(launch_line_fft<double>(gd.scratch, nc * G[0], G[1], G[2], gd.plan[1], gd.tw64[1], 0, st));
    if (G[2] > 1) HIPCHK(launch_line_fft<double>(gd.scratch, nc * G[0] * G[1], G[2], 1, gd.plan[2], gd.tw64[2], 0, st));
    HIPCHK(launch_scale_cx(gd.scratch, nc * Nt, 1.0 / (double)Nt, st));
    HIPCHK(launch_extract_half(g, gd.scratch, gd.ahat[k], nc, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  gd.on = true;
  return HOM_OK;
}

hom_status hom_clear_gani(hom_problem* pb) {
  if (!pb) return HOM_E_INVALID;
  pb->gani.on = false;
  return HOM_OK;
}

}  // extern "C"

namespace {

struct InclHost {
  int kind;
  double c[3];
  double h[3];
  double A[6];
};

// Inclusion table on internal axes: differences A_j - A0 (or of the inverses)
// in coefficient components, and A0's components.
hom_status incl_table(const hom_desc* desc, const double* A0, int32_t n_incl, const int32_t* kind,
                      const double* center, const double* size, const double* A_in, int32_t inverse,
                      InclHost* inc, double* A0c) {
  const int d = desc->d, nc = desc->ncoef;
  double A0m[9], A0i[9];
  std::memcpy(A0m, A0, sizeof(double) * d * d);
  inv_small(d, A0m, A0i);
  const double* base0 = inverse ? A0i : A0m;
  if (incl_dev_size() != sizeof(InclHost)) return HOM_E_INVALID;
  for (int j = 0; j < n_incl; ++j) {
    InclHost& I = inc[j];
    std::memset(&I, 0, sizeof(I));
    I.kind = kind[j];
    if (I.kind == 1 && d != 3) return HOM_E_INVALID;
    if (I.kind != 0 && I.kind != 1) return HOM_E_INVALID;
    const double* c = center + (size_t)j * d;
    const double* h = size + (size_t)j * d;
    if (d == 2) {
      I.c[0] = c[0];
      I.c[1] = 0.0;
      I.c[2] = c[1];
      I.h[0] = h[0];
      I.h[1] = 1.0;
      I.h[2] = h[1];
    } else {
      for (int a = 0; a < 3; ++a) {
        I.c[a] = c[a];
        I.h[a] = h[a];
      }
    }
    double Am[9], Ai[9], Dm[9];
    std::memcpy(Am, A_in + (size_t)j * d * d, sizeof(double) * d * d);
    if (inverse) inv_small(d, Am, Ai);
    for (int i = 0; i < d * d; ++i) Dm[i] = (inverse ? Ai[i] : Am[i]) - base0[i];
    coef_components(d, nc, Dm, I.A);
  }
  coef_components(d, nc, base0, A0c);
  return HOM_OK;
}

// Checks of a descriptor for point values on the N grid (no transform sizes
// involved) and the internal N.
hom_status sample_sizes(const hom_desc* desc, int* Nint) {
  if (!desc || (desc->d != 2 && desc->d != 3)) return HOM_E_INVALID;
  const int d = desc->d;
  if (desc->ncoef != 1 && desc->ncoef != d * (d + 1) / 2) return HOM_E_INVALID;
  for (int a = 0; a < d; ++a) {
    if (!(desc->Y[a] > 0.0) || !std::isfinite(desc->Y[a])) return HOM_E_INVALID;
    if (desc->N[a] < 1 || desc->N[a] > 8193) return HOM_E_UNSUPPORTED_SIZE;
  }
  Nint[0] = desc->N[0];
  Nint[1] = d == 3 ? desc->N[1] : 1;
  Nint[2] = d == 3 ? desc->N[2] : desc->N[1];
  return HOM_OK;
}

// Device bytes of the inclusion table: A0's components (64 bytes), then the records.
size_t incl_scratch_bytes(int n_incl) { return 64 + sizeof(InclHost) * (size_t)std::max(n_incl, 1); }

// Copies A0's components and the inclusion table into the device buffer dev
// (incl_scratch_bytes(n) bytes) and waits for the copies: the host table may
// be released when this returns.
hom_status incl_upload(const InclHost* inc, int n, const double* A0c, void* dev, hipStream_t st) {
  if (hipMemcpyAsync(dev, A0c, 6 * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
      (n > 0 && hipMemcpyAsync((char*)dev + 64, inc, sizeof(InclHost) * n, hipMemcpyHostToDevice, st) != hipSuccess) ||
      hipStreamSynchronize(st) != hipSuccess)
    return HOM_E_DEVICE;
  return HOM_OK;
}

// Bytes of the pixel-image scratch: the complex image (nc * Pt) and the
// twiddles of the three axes, each 256-byte aligned; offsets in tw_off.
size_t pixel_scratch_layout(int nc, const int* Pint, size_t* tw_off) {
  const size_t Pt = (size_t)Pint[0] * Pint[1] * Pint[2];
  size_t off = up(nc * Pt * sizeof(Cx<double>));
  for (int a = 0; a < 3; ++a) {
    if (tw_off) tw_off[a] = off;
    off = up(off + Pint[a] * sizeof(Cx<double>));
  }
  return off;
}

// Physical pixel counts to internal axes (2D embeds as (P0, 1, P1)).
bool pixel_axes(int d, const int32_t* P, int* Pint) {
  Pint[0] = P[0];
  Pint[1] = d == 3 ? P[1] : 1;
  Pint[2] = d == 3 ? P[2] : P[1];
  for (int a = 0; a < 3; ++a)
    if (Pint[a] < 1 || Pint[a] > (1 << 16)) return false;
  return true;
}

// Coefficient components of every phase (nc per phase, stride 6).
void phase_components(int d, int nc, int nphase, const double* phase_A, int32_t inverse, double* comp) {
  for (int q = 0; q < nphase; ++q) {
    double Am[9], Ai[9];
    std::memcpy(Am, phase_A + (size_t)q * d * d, sizeof(double) * d * d);
    if (inverse) inv_small(d, Am, Ai);
    coef_components(d, nc, inverse ? Ai : Am, comp + (size_t)q * 6);
  }
}

// Eigenvalues of a symmetric 3x3 matrix by cyclic Jacobi rotations (host).
void sym3_eigs(const double* A, double* ev) {
  double a[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) a[i][j] = 0.5 * (A[3 * i + j] + A[3 * j + i]);
  for (int sweep = 0; sweep < 50; ++sweep) {
    const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (off <= 1e-34 * dia) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (a[p][q] == 0.0) continue;
        const double th = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < 3; ++k) {       // columns p, q
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - sn * akq;
          a[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {       // rows p, q
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - sn * aqk;
          a[q][k] = sn * apk + c * aqk;
        }
      }
  }
  for (int i = 0; i < 3; ++i) ev[i] = a[i][i];
}

}  // namespace

extern "C" {

hom_status hom_coef_scratch_bytes(const hom_desc* desc, int32_t n_incl, const int32_t* P, size_t* bytes) {
  if (!desc || !bytes || (desc->d != 2 && desc->d != 3)) return HOM_E_INVALID;
  const int nc = desc->ncoef;
  if (nc != 1 && nc != desc->d * (desc->d + 1) / 2) return HOM_E_INVALID;
  if (!P) {
    if (n_incl < 0) return HOM_E_INVALID;
    *bytes = incl_scratch_bytes(n_incl);
    return HOM_OK;
  }
  int Pint[3];
  if (!pixel_axes(desc->d, P, Pint)) return HOM_E_INVALID;
  *bytes = pixel_scratch_layout(nc, Pint, nullptr);
  return HOM_OK;
}

hom_status hom_coef_inclusions(const hom_desc* desc, const double* A0, int32_t n_incl, const int32_t* kind,
                               const double* center, const double* size, const double* A_in, int32_t inverse,
                               void* out, void* scratch, size_t scratch_bytes, void* stream) {
  hom_status s = validate_desc(desc, 1);
  if (s != HOM_OK) return s;
  if (!A0 || !out || !scratch || n_incl < 0 || (n_incl > 0 && (!kind || !center || !size || !A_in)))
    return HOM_E_INVALID;
  if (scratch_bytes < incl_scratch_bytes(n_incl)) return HOM_E_WORKSPACE;
  const int d = desc->d, nc = desc->ncoef;
  Sizes z;
  Plan pl[3];
  fill_sizes(desc, 1, &z, pl);
  std::vector<InclHost> inc(std::max(n_incl, 1));
  double A0c[6] = {0, 0, 0, 0, 0, 0};
  s = incl_table(desc, A0, n_incl, kind, center, size, A_in, inverse, inc.data(), A0c);
  if (s != HOM_OK) return s;
  double iY[3] = {1.0 / desc->Y[0], 1.0, 1.0 / desc->Y[1]};
  if (d == 3) iY[1] = 1.0 / desc->Y[1], iY[2] = 1.0 / desc->Y[2];
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  s = incl_upload(inc.data(), n_incl, A0c, scratch, st);
  if (s != HOM_OK) return s;
  if (launch_coef_incl(d, z.M, iY, nc, (const double*)scratch, n_incl, (char*)scratch + 64,
                       reinterpret_cast<Cx<double>*>(out), st) != hipSuccess)
    return HOM_E_DEVICE;
  return HOM_OK;
}

}  // extern "C"

// ---- allocation-free variant of hom_coef_inclusions: the inclusion table goes
// to a fixed device array of the library instead of caller scratch.

namespace {
constexpr int kStaticMaxIncl = 512;
constexpr size_t kStaticInclBytes = (64 + sizeof(InclHost) * kStaticMaxIncl + 255) & ~size_t(255);
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};
}  // namespace

// One copy per GPU; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (static_table below).
static __device__ __align__(256) unsigned char scratch[kStaticInclBytes];

namespace {
// Device address of this GPU's copy of the array, looked up once per device
// with that device current.
hom_status static_table(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return HOM_E_DEVICE;
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HOM_E_DEVICE;
    g_static_ptr[dev] = p;
  }
  *out = g_static_ptr[dev];
  return HOM_OK;
}
}  // namespace

extern "C" {

hom_status hom_coef_inclusions_static(const hom_desc* desc, const double* A0, int32_t n_incl, const int32_t* kind,
                                      const double* center, const double* size, const double* A_in, int32_t inverse,
                                      void* out, void* stream) {
  hom_status s = validate_desc(desc, 1);
  if (s != HOM_OK) return s;
  if (!A0 || !out || n_incl < 0 || (n_incl > 0 && (!kind || !center || !size || !A_in))) return HOM_E_INVALID;
  if (n_incl > kStaticMaxIncl) return HOM_E_UNSUPPORTED_SIZE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return HOM_E_DEVICE;
  if (st) {
    hipDevice_t sdev = -1;
    if (hipStreamGetDevice(st, &sdev) != hipSuccess) return HOM_E_DEVICE;
    if (sdev != dev) return HOM_E_INVALID;
  }
  void* table = nullptr;
  s = static_table(&table);
  if (s != HOM_OK) return s;
  const int d = desc->d, nc = desc->ncoef;
  Sizes z;
  Plan pl[3];
  fill_sizes(desc, 1, &z, pl);
  InclHost inc[kStaticMaxIncl];          // host staging on the stack: no heap either
  double A0c[6] = {0, 0, 0, 0, 0, 0};
  s = incl_table(desc, A0, n_incl, kind, center, size, A_in, inverse, inc, A0c);
  if (s != HOM_OK) return s;
  double iY[3] = {1.0 / desc->Y[0], 1.0, 1.0 / desc->Y[1]};
  if (d == 3) iY[1] = 1.0 / desc->Y[1], iY[2] = 1.0 / desc->Y[2];
  // every word the kernel reads (A0's components, n_incl records) is written here
  s = incl_upload(inc, n_incl, A0c, table, st);
  if (s != HOM_OK) return s;
  if (launch_coef_incl(d, z.M, iY, nc, (const double*)table, n_incl, (char*)table + 64,
                       reinterpret_cast<Cx<double>*>(out), st) != hipSuccess)
    return HOM_E_DEVICE;
  // the next call may overwrite the table: finish reading it first
  return hipStreamSynchronize(st) == hipSuccess ? HOM_OK : HOM_E_DEVICE;
}

hom_status hom_sample_inclusions(const hom_desc* desc, const double* A0, int32_t n_incl, const int32_t* kind,
                                 const double* center, const double* size, const double* A_in, int32_t inverse,
                                 int32_t closed, double* out, void* scratch, size_t scratch_bytes, void* stream) {
  int Nint[3];
  hom_status s = sample_sizes(desc, Nint);
  if (s != HOM_OK) return s;
  if (!A0 || !out || !scratch || n_incl < 0 || (n_incl > 0 && (!kind || !center || !size || !A_in)))
    return HOM_E_INVALID;
  if (scratch_bytes < incl_scratch_bytes(n_incl)) return HOM_E_WORKSPACE;
  const int d = desc->d, nc = desc->ncoef;
  std::vector<InclHost> inc(std::max(n_incl, 1));
  double A0c[6] = {0, 0, 0, 0, 0, 0};
  s = incl_table(desc, A0, n_incl, kind, center, size, A_in, inverse, inc.data(), A0c);
  if (s != HOM_OK) return s;
  double Yint[3] = {desc->Y[0], 1.0, desc->Y[1]};
  if (d == 3) Yint[1] = desc->Y[1], Yint[2] = desc->Y[2];
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  s = incl_upload(inc.data(), n_incl, A0c, scratch, st);
  if (s != HOM_OK) return s;
  if (launch_sample_incl(Nint, Yint, nc, (const double*)scratch, n_incl, (char*)scratch + 64, closed != 0, out, st) !=
      hipSuccess)
    return HOM_E_DEVICE;
  return HOM_OK;
}

hom_status hom_sample_pixels(const hom_desc* desc, const int32_t* P, const int32_t* phase, int32_t nphase,
                             const double* phase_A, int32_t inverse, double* out, void* scratch, size_t scratch_bytes,
                             void* stream) {
  int Nint[3];
  hom_status s = sample_sizes(desc, Nint);
  if (s != HOM_OK) return s;
  if (!P || !phase || nphase < 1 || !phase_A || !out || !scratch) return HOM_E_INVALID;
  const int d = desc->d, nc = desc->ncoef;
  int Pint[3];
  if (!pixel_axes(d, P, Pint)) return HOM_E_INVALID;
  if (scratch_bytes < pixel_scratch_layout(nc, Pint, nullptr)) return HOM_E_WORKSPACE;
  const size_t Pt = (size_t)Pint[0] * Pint[1] * Pint[2];
  std::vector<double> comp((size_t)nphase * 6);
  phase_components(d, nc, nphase, phase_A, inverse, comp.data());
  std::vector<double> img(nc * Pt);
  for (size_t t = 0; t < Pt; ++t) {
    const int q = phase[t];
    if (q < 0 || q >= nphase) return HOM_E_INVALID;
    for (int c = 0; c < nc; ++c) img[c * Pt + t] = comp[(size_t)q * 6 + c];
  }
  double Yint[3] = {desc->Y[0], 1.0, desc->Y[1]};
  if (d == 3) Yint[1] = desc->Y[1], Yint[2] = desc->Y[2];
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  double* dev = reinterpret_cast<double*>(scratch);
  if (hipMemcpyAsync(dev, img.data(), img.size() * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess || launch_sample_pixels(Nint, Yint, Pint, nc, dev, out, st) != hipSuccess)
    return HOM_E_DEVICE;
  return HOM_OK;
}

hom_status hom_coef_pixels(const hom_desc* desc, const int32_t* P, const int32_t* phase, int32_t nphase,
                           const double* phase_A, int32_t inverse, void* out, void* scratch, size_t scratch_bytes,
                           void* stream) {
  hom_status s = validate_desc(desc, 1);
  if (s != HOM_OK) return s;
  if (!P || !phase || nphase < 1 || !phase_A || !out || !scratch) return HOM_E_INVALID;
  const int d = desc->d, nc = desc->ncoef;
  Sizes z;
  Plan pl[3];
  fill_sizes(desc, 1, &z, pl);
  int Pint[3];
  if (!pixel_axes(d, P, Pint)) return HOM_E_INVALID;
  Plan pp[3];
  for (int a = 0; a < 3; ++a) {
    if (Pint[a] == 1) {
      pp[a].n = 0;
      continue;
    }
    if (!smooth235(Pint[a], &pp[a])) return HOM_E_UNSUPPORTED_SIZE;
  }
  size_t twoff[3];
  if (scratch_bytes < pixel_scratch_layout(nc, Pint, twoff)) return HOM_E_WORKSPACE;
  const size_t Pt = (size_t)Pint[0] * Pint[1] * Pint[2];
  std::vector<double> comp((size_t)nphase * 6);
  phase_components(d, nc, nphase, phase_A, inverse, comp.data());
  std::vector<Cx<double>> img(nc * Pt);
  for (size_t t = 0; t < Pt; ++t) {
    const int q = phase[t];
    if (q < 0 || q >= nphase) return HOM_E_INVALID;
    for (int c = 0; c < nc; ++c) {
      img[c * Pt + t].x = comp[(size_t)q * 6 + c];
      img[c * Pt + t].y = 0.0;
    }
  }
  std::vector<Cx<double>> tw[3];
  std::vector<Cx<float>> tw32;
  for (int a = 0; a < 3; ++a) twiddles(Pint[a], tw[a], tw32);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* dev = reinterpret_cast<char*>(scratch);
  Cx<double>* D = reinterpret_cast<Cx<double>*>(dev);
  hipError_t e = hipMemcpyAsync(D, img.data(), img.size() * sizeof(Cx<double>), hipMemcpyHostToDevice, st);
  for (int a = 0; a < 3 && e == hipSuccess; ++a)
    e = hipMemcpyAsync(dev + twoff[a], tw[a].data(), Pint[a] * sizeof(Cx<double>), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);     // the host staging vectors end with this call
  // unnormalised forward DFT of the image along each axis
  if (e == hipSuccess && Pint[0] > 1)
    e = launch_line_fft<double>(D, nc, Pint[0], Pint[1] * Pint[2], pp[0], (const Cx<double>*)(dev + twoff[0]), 0, st);
  if (e == hipSuccess && Pint[1] > 1)
    e = launch_line_fft<double>(D, nc * Pint[0], Pint[1], Pint[2], pp[1], (const Cx<double>*)(dev + twoff[1]), 0, st);
  if (e == hipSuccess && Pint[2] > 1)
    e = launch_line_fft<double>(D, nc * Pint[0] * Pint[1], Pint[2], 1, pp[2], (const Cx<double>*)(dev + twoff[2]), 0,
                                st);
  if (e == hipSuccess) e = launch_pixel_factor(d, z.M, Pint, nc, D, reinterpret_cast<Cx<double>*>(out), st);
  return e == hipSuccess ? HOM_OK : HOM_E_DEVICE;
}

hom_status hom_phase_eig_range(int32_t d, int32_t nphase, const double* phase_A, double* range) {
  if ((d != 2 && d != 3) || nphase < 1 || !phase_A || !range) return HOM_E_INVALID;
  double lo = INFINITY, hi = -INFINITY;
  for (int q = 0; q < nphase; ++q) {
    const double* A = phase_A + (size_t)q * d * d;
    for (int i = 0; i < d * d; ++i)
      if (!std::isfinite(A[i])) return HOM_E_INVALID;
    double ev[3];
    if (d == 2) {
      const double a = A[0], c = A[3], b = 0.5 * (A[1] + A[2]);
      const double m = 0.5 * (a + c), r = std::hypot(0.5 * (a - c), b);
      ev[0] = m - r;
      ev[1] = m + r;
    } else {
      sym3_eigs(A, ev);
    }
    for (int i = 0; i < d; ++i) {
      lo = std::min(lo, ev[i]);
      hi = std::max(hi, ev[i]);
    }
  }
  range[0] = lo;
  range[1] = hi;
  return lo > 0.0 ? HOM_OK : HOM_E_NOT_SPD;
}

// Average per-launch time of each operator pass over n units (HIP events on the stream).
static hom_status profile_units(const Geo& g, const UnitDev* units, int n, bool fp32, hipStream_t st, int reps,
                                double* ms_out) {
  hipEvent_t ev[6];
  for (int i = 0; i < 6; ++i) HIPCHK(hipEventCreate(&ev[i]));
  hom_status rc = HOM_OK;
  auto run = [&](int which) -> hipError_t {
    for (int r = 0; r < reps; ++r) {
      hipError_t e = hipSuccess;
      if (which == 0)
        e = fp32 ? launch_first<float>(g, units, n, FIRST_FIELD, 0, nullptr, st)
                 : launch_first<double>(g, units, n, FIRST_FIELD, 0, nullptr, st);
      if (which == 1 && g.d == 3 && !g.plane)
        e = fp32 ? launch_mid<float>(g, units, n, 1, st) : launch_mid<double>(g, units, n, 1, st);
      if (which == 2)
        e = fp32 ? launch_apply<float>(g, units, n, APPLY_COEF, st) : launch_apply<double>(g, units, n, APPLY_COEF, st);
      if (which == 3 && g.d == 3 && !g.plane)
        e = fp32 ? launch_mid<float>(g, units, n, 0, st) : launch_mid<double>(g, units, n, 0, st);
      if (which == 4)
        e = fp32 ? launch_last<float>(g, units, n, LAST_MATVEC, 0, nullptr, st)
                 : launch_last<double>(g, units, n, LAST_MATVEC, 0, nullptr, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  for (int w = 0; w < 5 && rc == HOM_OK; ++w)
    if (run(w) != hipSuccess) rc = HOM_E_DEVICE;  // untimed round: first-launch costs excluded
  for (int w = 0; w < 5 && rc == HOM_OK; ++w)
    if (hipEventRecord(ev[w], st) != hipSuccess || run(w) != hipSuccess || hipEventRecord(ev[w + 1], st) != hipSuccess)
      rc = HOM_E_DEVICE;
  if (rc == HOM_OK && hipEventSynchronize(ev[5]) != hipSuccess) rc = HOM_E_DEVICE;
  for (int w = 0; w < 5 && rc == HOM_OK; ++w) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev[w], ev[w + 1]) != hipSuccess) rc = HOM_E_DEVICE;
    const bool skipped = (w == 1 || w == 3) && (g.d != 3 || g.plane);
    ms_out[w] = skipped ? 0.0 : (double)ms / reps;
  }
  for (int i = 0; i < 6; ++i) (void)hipEventDestroy(ev[i]);
  return rc;
}

// Point a unit at scratch vectors for a timing run (input tmp = 0, output p).
static hom_status profile_unit_setup(hom_problem* pb, int k, int nload, const Geo& g, UnitDev* hu) {
  SlotBufs& sb = pb->slot[k];
  fill_unit(pb, k, nload, nullptr, nullptr, hu);
  for (int l = 0; l < nload; ++l) hu->s[l] = sb.p[l];
  const size_t vbytes = (size_t)g.m * g.S * sizeof(Cx<double>);
  for (int l = 0; l < nload; ++l) HIPCHK(hipMemsetAsync(sb.tmp[l], 0, vbytes, pb->stream));
  return HOM_OK;
}

hom_status hom_profile_passes(hom_problem* pb, int32_t dual, int32_t nload, int32_t reps, double* ms_out) {
  if (!pb || !ms_out || (dual != 0 && dual != 1) || nload < 1 || nload > pb->max_loads || reps < 1)
    return HOM_E_INVALID;
  const int k = dual;
  hipStream_t st = pb->stream;
  const bool fp32 = pb->desc.precision == HOM_MIXED;
  Geo g = make_geo(pb, k, nload, fp32, 0, pb->tuned[k][nload] ? &pb->tune[k][nload] : nullptr);
  SlotBufs& sb = pb->slot[k];
  UnitDev* hu = &pb->host_unit[k];
  hom_status s = profile_unit_setup(pb, k, nload, g, hu);
  if (s != HOM_OK) return s;
  HIPCHK(hipMemcpyAsync(sb.unit, hu, sizeof(UnitDev), hipMemcpyHostToDevice, st));
  return profile_units(g, sb.unit, 1, fp32, st, reps, ms_out);
}

// Unit for the FP64 grid transfers of one problem (bounds buffers, nload loads).
static void grid_unit(hom_problem* pb, int k, int nload, UnitDev* hu) {
  std::memset(hu, 0, sizeof(*hu));
  SlotBufs& sb = pb->slot[k];
  hu->coef = pb->coef64[k];
  hu->ahat = pb->ahat_half[k];
  for (int l = 0; l < nload; ++l) {
    hu->r[l] = sb.r[l];
    hu->p[l] = sb.p[l];
    hu->s[l] = sb.s[l];
    hu->b[l] = sb.b[l];
    hu->x[l] = sb.tmp[l];
  }
  hu->bufA = pb->bbufA;
  hu->bufB = pb->bbufB;
  hu->part_g = sb.part_g;
  hu->part_d = sb.part_d;
  hu->part_q = pb->bpart_q[k];
  hu->sc = sb.sc;
}

hom_status hom_field_to_grid(hom_problem* pb, int32_t dual, int32_t nload, const double* const* fields, float* out) {
  if (!pb || !fields || !out || (dual != 0 && dual != 1) || nload < 1 || nload > pb->max_loads) return HOM_E_INVALID;
  for (int l = 0; l < nload; ++l)
    if (!fields[l]) return HOM_E_INVALID;
  const int k = dual;
  hipStream_t st = pb->stream;
  Geo g = make_geo(pb, k, nload, false);
  UnitDev* hu = &pb->host_bunit[k];
  grid_unit(pb, k, nload, hu);
  for (int l = 0; l < nload; ++l) hu->x[l] = reinterpret_cast<Cx<double>*>(const_cast<double*>(fields[l]));
  hu->grid = out;
  HIPCHK(hipMemcpyAsync(pb->bunit[k], hu, sizeof(UnitDev), hipMemcpyHostToDevice, st));
  HIPCHK(launch_first<double>(g, pb->bunit[k], 1, FIRST_FIELD, 0, nullptr, st));
  if (g.d == 3) HIPCHK(launch_mid<double>(g, pb->bunit[k], 1, 1, st));
  HIPCHK(launch_apply<double>(g, pb->bunit[k], 1, APPLY_GRID, st));
  HIPCHK(hipStreamSynchronize(st));
  return HOM_OK;
}

hom_status hom_grid_to_field(hom_problem* pb, int32_t dual, int32_t nload, const float* in, double* const* out) {
  if (!pb || !in || !out || (dual != 0 && dual != 1) || nload < 1 || nload > pb->max_loads) return HOM_E_INVALID;
  for (int l = 0; l < nload; ++l)
    if (!out[l]) return HOM_E_INVALID;
  const int k = dual;
  hipStream_t st = pb->stream;
  Geo g = make_geo(pb, k, nload, false);
  UnitDev* hu = &pb->host_bunit[k];
  grid_unit(pb, k, nload, hu);
  for (int l = 0; l < nload; ++l) hu->s[l] = reinterpret_cast<Cx<double>*>(out[l]);
  hu->grid = const_cast<float*>(in);
  HIPCHK(hipMemcpyAsync(pb->bunit[k], hu, sizeof(UnitDev), hipMemcpyHostToDevice, st));
  HIPCHK(launch_apply<double>(g, pb->bunit[k], 1, APPLY_FWD, st));
  if (g.d == 3) HIPCHK(launch_mid<double>(g, pb->bunit[k], 1, 0, st));
  HIPCHK(launch_last<double>(g, pb->bunit[k], 1, LAST_MATVEC, 0, nullptr, st));
  HIPCHK(hipStreamSynchronize(st));
  return HOM_OK;
}

hom_status hom_net_input(hom_problem* pb, float* out) {
  if (!pb || !out) return HOM_E_INVALID;
  HIPCHK(launch_net_input(pb->coef64[0], pb->z.nc, pb->z.d, (long)pb->z.Mt, pb->ahat_half[0], (long)pb->z.S, out, 0,
                          pb->stream));
  return HOM_OK;
}

hom_status hom_net_weights(hom_problem* pb, float* out) {
  if (!pb || !out) return HOM_E_INVALID;
  for (int k = 0; k < 2; ++k)
    HIPCHK(launch_net_input(pb->coef64[k], pb->z.nc, pb->z.d, (long)pb->z.Mt, pb->ahat_half[k], (long)pb->z.S,
                            out + (size_t)k * pb->z.Mt, 1, pb->stream));
  return HOM_OK;
}

struct hom_batch {
  int n;
  std::vector<hom_problem*> pbs;
  hipStream_t stream;
  UnitDev* units[2];
  UnitDev* bunits[2];
  int* iter_base[2];
  int* active[2];
  std::vector<UnitDev> host_units[2];
  std::vector<UnitDev> host_bunits[2];
  hipGraphExec_t graph[2][kMaxLoads + 1];
  hipGraphExec_t tgraph[2][kMaxLoads + 1];      // variants with event records
  std::vector<hipEvent_t> tevents[2][kMaxLoads + 1];
  int timing = 0;
  Tuning tune[2][kMaxLoads + 1];
  bool tuned[2][kMaxLoads + 1] = {};
  StopCfg stop;                        // as in hom_problem
  SolveOut* collect_dev = nullptr;     // [2][n][kMaxLoads] end-of-solve summaries (workspace)
  hipStream_t stream2 = nullptr;       // library stream of the dual in side-by-side solves
  int* pinned = nullptr;               // [2] active counts of the primal and dual loops (pinned; the
                                       // captured chunk graphs copy into these)
  hipEvent_t order_ev = nullptr;       // orders the library stream after the caller's
  double* bcollect_dev = nullptr;      // [2][n][9] bounds quadrature sums (workspace)
  CoefJob* jobs_dev = nullptr;         // [n] coefficient set-up table (workspace)
  std::vector<CoefJob> host_jobs;
  SymJob* xjobs_dev[2] = {nullptr, nullptr};   // [n kMaxLoads] starting-field symmetrisations per side (workspace)
  std::vector<SymJob> host_xjobs[2];
  NetJob* njobs_dev = nullptr;         // [n] network-input table (workspace), uploaded once
  bool njobs_ready = false;
  SolveOut* collect_host = nullptr;    // pinned mirrors
  double* bcollect_host = nullptr;
  double tsum[5] = {0, 0, 0, 0, 0};
  long long tcnt[5] = {0, 0, 0, 0, 0};
};

static size_t batch_layout(int n, char* base, hom_batch* b) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off = up(off + bytes);
    return p;
  };
  for (int k = 0; k < 2; ++k) {
    char* u = take((size_t)n * sizeof(UnitDev));
    char* bu = take((size_t)n * sizeof(UnitDev));
    char* ib = take(sizeof(int));
    char* ac = take(sizeof(int));
    if (b) {
      b->units[k] = (UnitDev*)u;
      b->bunits[k] = (UnitDev*)bu;
      b->iter_base[k] = (int*)ib;
      b->active[k] = (int*)ac;
    }
  }
  char* cs = take((size_t)2 * n * kMaxLoads * sizeof(SolveOut));
  char* cb = take((size_t)n * 2 * 9 * sizeof(double));
  char* cj = take((size_t)n * sizeof(CoefJob));
  char* xj0 = take((size_t)n * kMaxLoads * sizeof(SymJob));
  char* xj1 = take((size_t)n * kMaxLoads * sizeof(SymJob));
  char* nj = take((size_t)n * sizeof(NetJob));
  if (b) {
    b->collect_dev = (SolveOut*)cs;
    b->bcollect_dev = (double*)cb;
    b->jobs_dev = (CoefJob*)cj;
    b->xjobs_dev[0] = (SymJob*)xj0;
    b->xjobs_dev[1] = (SymJob*)xj1;
    b->njobs_dev = (NetJob*)nj;
  }
  return off;
}

hom_status hom_batch_workspace_bytes(int32_t n, size_t* bytes) {
  if (n < 1 || !bytes) return HOM_E_INVALID;
  *bytes = batch_layout(n, nullptr, nullptr);
  return HOM_OK;
}

hom_status hom_batch_create(hom_problem* const* pbs, int32_t n, void* ws, size_t ws_bytes, hom_batch** out) {
  if (!pbs || n < 1 || !ws || !out) return HOM_E_INVALID;
  if (((uintptr_t)ws) % kAlign) return HOM_E_WORKSPACE;
  if (ws_bytes < batch_layout(n, nullptr, nullptr)) return HOM_E_WORKSPACE;
  for (int i = 0; i < n; ++i) {
    if (!pbs[i]) return HOM_E_INVALID;
    const hom_desc& a = pbs[0]->desc;
    const hom_desc& c = pbs[i]->desc;
    if (std::memcmp(&a, &c, sizeof(hom_desc)) != 0 || pbs[i]->max_loads != pbs[0]->max_loads ||
        pbs[i]->stream != pbs[0]->stream)
      return HOM_E_INVALID;
  }
  hom_batch* b = new hom_batch();
  b->n = n;
  b->pbs.assign(pbs, pbs + n);
  b->stream = pbs[0]->stream;
  std::memset(b->graph, 0, sizeof(b->graph));
  std::memset(b->tgraph, 0, sizeof(b->tgraph));
  batch_layout(n, (char*)ws, b);
  for (int k = 0; k < 2; ++k) {
    b->host_units[k].resize(n);
    b->host_bunits[k].resize(n);
  }
  if (hipHostMalloc((void**)&b->collect_host, (size_t)2 * n * kMaxLoads * sizeof(SolveOut), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void**)&b->bcollect_host, (size_t)n * 2 * 9 * sizeof(double), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void**)&b->pinned, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    if (b->collect_host) (void)hipHostFree(b->collect_host);
    if (b->bcollect_host) (void)hipHostFree(b->bcollect_host);
    delete b;
    return HOM_E_DEVICE;
  }
  *out = b;
  return HOM_OK;
}

// Batches solve the exact (Ga) operator only.
static bool batch_has_gani(const hom_batch* b) {
  for (const hom_problem* p : b->pbs)
    if (p->gani.on) return true;
  return false;
}

// Iterations per chunk of a batch's solve.  Per-kernel timing launches every
// pass directly and waits for each chunk, so it takes chunks of at least 8
// iterations (the host waits, between which the GPU idles, would otherwise
// lengthen the measured kernels); not under the gap rule, whose stops depend
// on the chunk boundaries.
static int batch_chunk(const hom_batch* b, const hom_problem* p0) {
  int c = p0->graph_chunk;
  if (b->timing && b->stop.rule != 3) c = std::max(c, 8);
  return c;
}

hom_status hom_batch_solve(hom_batch* b, int32_t dual, int32_t nload, const double* E, const double* const* x0,
                           double tol, int32_t maxit, double* const* x_out, hom_info* info) {
  if (!b || !info || (dual != 0 && dual != 1)) return HOM_E_INVALID;
  if (batch_has_gani(b) || b->stop.rule == 3) return HOM_E_INVALID;   // the gap rule needs the pair solve
  const int k = dual, n = b->n;
  for (int i = 0; i < n; ++i) {
    hom_status s = check_solve_args(b->pbs[i], nload, E, x_out + (size_t)i * nload, tol, maxit);
    if (s != HOM_OK) return s;
  }
  hom_problem* p0 = b->pbs[0];
  hipStream_t st = b->stream;
  const bool fp32 = p0->desc.precision == HOM_MIXED;
  if (!b->tuned[k][nload]) {
    hom_status s = solve_tuning(b->pbs.data(), n, k, nload, b->units[k], st, &b->tune[k][nload]);
    if (s != HOM_OK) return s;
    b->tuned[k][nload] = true;
  }
  Geo g = make_geo(p0, k, nload, fp32, 0, &b->tune[k][nload]);
  bool have_x0 = false;
  for (int i = 0; i < n; ++i) {
    fill_unit(b->pbs[i], k, nload, E, x_out + (size_t)i * nload, &b->host_units[k][i]);
    if (x0) {
      bool h = false;
      hom_status s = prepare_x0(b->pbs[i], k, nload, g, x0 + (size_t)i * nload, x_out + (size_t)i * nload, &h);
      if (s != HOM_OK) return s;
      have_x0 = have_x0 || h;
    }
  }
  if (have_x0)
    for (int i = 0; i < n; ++i) {
      hom_status s = zero_missing_x0(b->pbs[i], k, nload, g, x0 + (size_t)i * nload, x_out + (size_t)i * nload);
      if (s != HOM_OK) return s;
    }
  HIPCHK(hipMemcpyAsync(b->units[k], b->host_units[k].data(), (size_t)n * sizeof(UnitDev), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  SolveRun R;
  R.st = st;
  R.g = g;
  R.fp32 = fp32;
  R.units = b->units[k];
  R.n = n;
  R.iter_base = b->iter_base[k];
  R.active = b->active[k];
  R.pinned_active = b->pinned + k;
  R.graph = &b->graph[k][nload];
  R.chunk = batch_chunk(b, p0);
  R.stop = b->stop;
  if (b->timing) {
    R.events = &b->tevents[k][nload];
    R.tsum = b->tsum;
    R.tcnt = b->tcnt;
  }
  for (int i = 0; i < n; ++i) {
    R.part_d.push_back(b->pbs[i]->slot[k].part_d);
    R.sc.push_back(b->pbs[i]->slot[k].sc);
  }
  R.collect_dev = b->collect_dev + (size_t)k * n * kMaxLoads;
  R.collect_host = b->collect_host + (size_t)k * n * kMaxLoads;
  return solve_units(R, nload, tol, maxit, have_x0, info);
}

// The batch's second library stream (the dual side's) and the event that
// orders it against the first, created on first use.
static bool side_stream(hom_batch* b) {
  if (!b->stream2 && hipStreamCreateWithFlags(&b->stream2, hipStreamNonBlocking) != hipSuccess) {
    b->stream2 = nullptr;
    return false;
  }
  if (!b->order_ev && hipEventCreateWithFlags(&b->order_ev, hipEventDisableTiming) != hipSuccess) {
    b->order_ev = nullptr;
    return false;
  }
  return true;
}

static hom_status upload_batch_bounds(hom_batch* b, int k, const double* const* f, hipStream_t st);
static hom_status launch_batch_bounds(hom_batch* b, int k, hipStream_t st);
static hom_status read_batch_bounds(hom_batch* b, const bool have[2], hom_result* out);

// Closing work of one side of a pair solve: the residual passes and, when
// bounds are asked for, the side's FP64 bound passes on its fields (their
// unit tables are uploaded before the iterations start).
struct PairClose {
  hom_batch* b;
  SolveRun* R;
  int nload;
  bool bounds;
  bool queued[2];
};

static hom_status pair_close(void* ctx, int k) {
  PairClose& c = *static_cast<PairClose*>(ctx);
  if (c.queued[k]) return HOM_OK;
  hom_status s = finish_enqueue(c.R[k], c.nload);
  if (s == HOM_OK && c.bounds) s = launch_batch_bounds(c.b, k, c.R[k].st);
  if (s == HOM_OK) c.queued[k] = true;
  return s;
}

// Primal and dual solves side by side; with bounds (unit loads only) each
// side's bound passes start as soon as that side has stopped, beside the
// other side's remaining iterations.
static hom_status solve_pair(hom_batch* b, int32_t nload, const double* E, const double* const* x0_primal,
                             const double* const* x0_dual, double tol, int32_t maxit, double* const* x_primal,
                             double* const* x_dual, hom_info* info_primal, hom_info* info_dual, hom_result* bounds) {
  if (!b || !info_primal || !info_dual || !x_primal || !x_dual) return HOM_E_INVALID;
  if (batch_has_gani(b)) return HOM_E_INVALID;
  const int n = b->n;
  for (int i = 0; i < n; ++i) {
    hom_status s = check_solve_args(b->pbs[i], nload, E, x_primal + (size_t)i * nload, tol, maxit);
    if (s == HOM_OK) s = check_solve_args(b->pbs[i], nload, E, x_dual + (size_t)i * nload, tol, maxit);
    if (s != HOM_OK) return s;
  }
  hom_problem* p0 = b->pbs[0];
  const bool gap_rule = b->stop.rule == 3;
  const bool fp32 = p0->desc.precision == HOM_MIXED;
  if (!side_stream(b)) return HOM_E_DEVICE;
  hipStream_t st[2] = {b->stream, b->stream2};
  for (int k = 0; k < 2; ++k)
    if (!b->tuned[k][nload]) {
      hom_status s = solve_tuning(b->pbs.data(), n, k, nload, b->units[k], b->stream, &b->tune[k][nload]);
      if (s != HOM_OK) return s;
      b->tuned[k][nload] = true;
    }
  SolveRun R[2];
  bool have_x0[2] = {false, false};
  for (int k = 0; k < 2; ++k) {
    double* const* xo = k == 0 ? x_primal : x_dual;
    const double* const* x0 = k == 0 ? x0_primal : x0_dual;
    const Geo gk = make_geo(p0, k, nload, fp32, 0, &b->tune[k][nload]);
    for (int i = 0; i < n; ++i) {
      fill_unit(b->pbs[i], k, nload, E, xo + (size_t)i * nload, &b->host_units[k][i]);
      // gap rule: each load reads the same load of the other solve of its cell
      if (gap_rule) b->host_units[k][i].partner_sc = b->pbs[i]->slot[1 - k].sc;
    }
    // starting fields: every given one symmetrised into its output in one launch (a field given
    // in place goes through the problem's scratch first)
    if (x0) {
      auto& jobs = b->host_xjobs[k];
      jobs.clear();
      const size_t vbytes = (size_t)gk.m * gk.S * sizeof(Cx<double>);
      for (int i = 0; i < n; ++i)
        for (int l = 0; l < nload; ++l) {
          const double* src = x0[(size_t)i * nload + l];
          if (!src) continue;
          double* dst = xo[(size_t)i * nload + l];
          const Cx<double>* sp = reinterpret_cast<const Cx<double>*>(src);
          if (src == dst) {
            Cx<double>* tmp = b->pbs[i]->slot[k].tmp[l];
            HIPCHK(hipMemcpyAsync(tmp, src, vbytes, hipMemcpyDeviceToDevice, b->stream));
            sp = tmp;
          }
          jobs.push_back(SymJob{sp, reinterpret_cast<Cx<double>*>(dst)});
        }
      have_x0[k] = !jobs.empty();
      if (have_x0[k]) {
        HIPCHK(hipMemcpyAsync(b->xjobs_dev[k], jobs.data(), jobs.size() * sizeof(SymJob), hipMemcpyHostToDevice,
                              b->stream));
        HIPCHK(launch_symmetrize_jobs(gk, b->xjobs_dev[k], (int)jobs.size(), gk.m, b->stream));
      }
    }
    if (have_x0[k])
      for (int i = 0; i < n; ++i) {
        hom_status s = zero_missing_x0(b->pbs[i], k, nload, gk, x0 + (size_t)i * nload, xo + (size_t)i * nload);
        if (s != HOM_OK) return s;
      }
    HIPCHK(hipMemcpyAsync(b->units[k], b->host_units[k].data(), (size_t)n * sizeof(UnitDev), hipMemcpyHostToDevice,
                          b->stream));
    R[k].st = st[k];
    R[k].g = make_geo(p0, k, nload, fp32, 0, &b->tune[k][nload]);
    R[k].fp32 = fp32;
    R[k].units = b->units[k];
    R[k].n = n;
    R[k].iter_base = b->iter_base[k];
    R[k].active = b->active[k];
    R[k].pinned_active = b->pinned + k;
    R[k].graph = &b->graph[k][nload];
    R[k].chunk = batch_chunk(b, p0);
    R[k].stop = b->stop;
    for (int i = 0; i < n; ++i) {
      R[k].part_d.push_back(b->pbs[i]->slot[k].part_d);
      R[k].sc.push_back(b->pbs[i]->slot[k].sc);
    }
    R[k].collect_dev = b->collect_dev + (size_t)k * n * kMaxLoads;
    R[k].collect_host = b->collect_host + (size_t)k * n * kMaxLoads;
    // per-kernel timing measures kernels one at a time (the runs then advance chunk by chunk in turn)
    if (b->timing) {
      R[k].events = &b->tevents[k][nload];
      R[k].tsum = b->tsum;
      R[k].tcnt = b->tcnt;
    }
  }
  // the second stream starts after everything the caller's stream holds (coefficient setup, unit tables)
  HIPCHK(hipEventRecord(b->order_ev, b->stream));
  HIPCHK(hipStreamWaitEvent(b->stream2, b->order_ev, 0));
  hom_status s = HOM_OK;
  for (int k = 0; k < 2 && s == HOM_OK && bounds; ++k)
    s = upload_batch_bounds(b, k, k == 0 ? x_primal : x_dual, st[k]);
  for (int k = 0; k < 2 && s == HOM_OK; ++k) s = start_run(R[k], nload, tol, maxit, have_x0[k]);
  if (s != HOM_OK) return s;
  SolveRun* runs[2] = {&R[0], &R[1]};
  const int partners[2] = {1, 0};
  PairClose close{b, R, nload, bounds != nullptr, {false, false}};
  if (R[0].use_graph && R[1].use_graph)
    s = loop_runs(runs, 2, maxit, gap_rule ? partners : nullptr, pair_close, &close);
  else
    s = loop_direct(runs, 2, maxit);
  if (s != HOM_OK) return s;
  for (int k = 0; k < 2; ++k) {
    s = pair_close(&close, k);
    if (s != HOM_OK) return s;
  }
  hom_status s0 = finish_run(R[0], nload, maxit, info_primal, true);
  hom_status s1 = finish_run(R[1], nload, maxit, info_dual, true);
  // later work on the caller's stream comes after the second stream's
  HIPCHK(hipStreamSynchronize(b->stream2));
  if (bounds) {
    const bool have[2] = {true, true};
    s = read_batch_bounds(b, have, bounds);
    if (s != HOM_OK) return s;
  }
  if (s0 < 0) return s0;
  if (s1 < 0) return s1;
  return s0 != HOM_OK ? s0 : s1;
}

hom_status hom_batch_solve_pair(hom_batch* b, int32_t nload, const double* E, const double* const* x0_primal,
                                const double* const* x0_dual, double tol, int32_t maxit, double* const* x_primal,
                                double* const* x_dual, hom_info* info_primal, hom_info* info_dual) {
  return solve_pair(b, nload, E, x0_primal, x0_dual, tol, maxit, x_primal, x_dual, info_primal, info_dual, nullptr);
}

hom_status hom_batch_solve_bounds(hom_batch* b, const double* const* x0_primal, const double* const* x0_dual,
                                  double tol, int32_t maxit, double* const* x_primal, double* const* x_dual,
                                  hom_info* info_primal, hom_info* info_dual, hom_result* out) {
  if (!b || !out) return HOM_E_INVALID;
  const int d = b->pbs[0]->desc.d;
  if (b->pbs[0]->max_loads < d) return HOM_E_INVALID;
  double E[9] = {};
  for (int l = 0; l < d; ++l) E[l * d + l] = 1.0;
  return solve_pair(b, d, E, x0_primal, x0_dual, tol, maxit, x_primal, x_dual, info_primal, info_dual, out);
}

// ---- grid transfers and network inputs of every problem of a batch (one launch per pass)

// Units of the bound-evaluation buffers of every problem, with grid[i] = base + i * stride.
static hom_status batch_grid_units(hom_batch* b, int k, int nload, float* base, size_t stride) {
  for (int i = 0; i < b->n; ++i) {
    grid_unit(b->pbs[i], k, nload, &b->host_bunits[k][i]);
    b->host_bunits[k][i].grid = base + (size_t)i * stride;
  }
  return HOM_OK;
}

hom_status hom_batch_field_to_grid(hom_batch* b, int32_t dual, int32_t nload, const double* const* fields, float* out,
                                   size_t stride) {
  if (!b || !fields || !out || (dual != 0 && dual != 1)) return HOM_E_INVALID;
  hom_problem* p0 = b->pbs[0];
  if (nload < 1 || nload > p0->max_loads) return HOM_E_INVALID;
  if (stride < (size_t)nload * p0->z.d * p0->z.Mt) return HOM_E_INVALID;
  for (size_t i = 0; i < (size_t)b->n * nload; ++i)
    if (!fields[i]) return HOM_E_INVALID;
  const int k = dual;
  hipStream_t st = b->stream;
  Geo g = make_geo(p0, k, nload, false);
  batch_grid_units(b, k, nload, out, stride);
  for (int i = 0; i < b->n; ++i)
    for (int l = 0; l < nload; ++l)
      b->host_bunits[k][i].x[l] = reinterpret_cast<Cx<double>*>(const_cast<double*>(fields[(size_t)i * nload + l]));
  HIPCHK(hipMemcpyAsync(b->bunits[k], b->host_bunits[k].data(), (size_t)b->n * sizeof(UnitDev), hipMemcpyHostToDevice,
                        st));
  HIPCHK(launch_first<double>(g, b->bunits[k], b->n, FIRST_FIELD, 0, nullptr, st));
  if (g.d == 3) HIPCHK(launch_mid<double>(g, b->bunits[k], b->n, 1, st));
  HIPCHK(launch_apply<double>(g, b->bunits[k], b->n, APPLY_GRID, st));
  HIPCHK(hipStreamSynchronize(st));   // the host unit table is reused by the next call
  return HOM_OK;
}

hom_status hom_batch_grid_to_field(hom_batch* b, int32_t dual, int32_t nload, const float* in, size_t stride,
                                   double* const* out) {
  if (!b || !in || !out || (dual != 0 && dual != 1)) return HOM_E_INVALID;
  hom_problem* p0 = b->pbs[0];
  if (nload < 1 || nload > p0->max_loads) return HOM_E_INVALID;
  if (stride < (size_t)nload * p0->z.d * p0->z.Mt) return HOM_E_INVALID;
  for (size_t i = 0; i < (size_t)b->n * nload; ++i)
    if (!out[i]) return HOM_E_INVALID;
  const int k = dual;
  hipStream_t st = b->stream;
  Geo g = make_geo(p0, k, nload, false);
  batch_grid_units(b, k, nload, const_cast<float*>(in), stride);
  for (int i = 0; i < b->n; ++i)
    for (int l = 0; l < nload; ++l)
      b->host_bunits[k][i].s[l] = reinterpret_cast<Cx<double>*>(out[(size_t)i * nload + l]);
  HIPCHK(hipMemcpyAsync(b->bunits[k], b->host_bunits[k].data(), (size_t)b->n * sizeof(UnitDev), hipMemcpyHostToDevice,
                        st));
  HIPCHK(launch_apply<double>(g, b->bunits[k], b->n, APPLY_FWD, st));
  if (g.d == 3) HIPCHK(launch_mid<double>(g, b->bunits[k], b->n, 0, st));
  HIPCHK(launch_last<double>(g, b->bunits[k], b->n, LAST_MATVEC, 0, nullptr, st));
  HIPCHK(hipStreamSynchronize(st));   // the host unit table is reused by the next call
  return HOM_OK;
}

hom_status hom_batch_net_input(hom_batch* b, float* out, size_t stride, int32_t weights) {
  if (!b || !out || (weights != 0 && weights != 1)) return HOM_E_INVALID;
  const size_t Mt = b->pbs[0]->z.Mt;
  if (stride < 2 * Mt) return HOM_E_INVALID;
  if (!b->njobs_ready) {     // the coefficient pointers of the cells never change: one upload
    std::vector<NetJob> h(b->n);
    for (int i = 0; i < b->n; ++i)
      for (int k = 0; k < 2; ++k) {
        h[i].coef64[k] = b->pbs[i]->coef64[k];
        h[i].ahat0[k] = b->pbs[i]->ahat_half[k];
      }
    HIPCHK(hipMemcpyAsync(b->njobs_dev, h.data(), (size_t)b->n * sizeof(NetJob), hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    b->njobs_ready = true;
  }
  const hom_problem* p0 = b->pbs[0];
  HIPCHK(launch_net_input_jobs(b->njobs_dev, b->n, p0->z.nc, p0->z.d, (long)Mt, (long)p0->z.S, out, stride, weights,
                               b->stream));
  return HOM_OK;
}

// ---- groups: the primal and dual solves of several batches in one captured graph

struct hom_group {
  std::vector<hom_batch*> bs;
  hipGraphExec_t graph = nullptr;      // `chunks` chunks of every solve of every batch
  std::vector<Tuning> graph_tiles;     // tile shapes the graph was captured with
  int graph_rule = -1;
  int chunks = 1;                      // chunks of iterations per graph launch (HOM_GROUP_CHUNKS; 1 under
                                       // the gap rule, whose partners exchange state between launches)
  int graph_chunks = 0;                // chunks per launch of the captured graph
  int launch = 0;                      // 0: one graph for all solves; 1: each solve's own chunk graph, one host loop
  std::vector<hipEvent_t> evs;         // fork, joins, per-batch order events, chunk-end pair
};

}  // extern "C"

namespace {
// Fill the units of both sides of a batch (unit loads), partner pointers for the gap rule.
hom_status group_units(hom_batch* b, double* const* xp, double* const* xd) {
  const int n = b->n, d = b->pbs[0]->desc.d;
  double E[kMaxLoads * 3] = {};
  for (int l = 0; l < d; ++l) E[l * d + l] = 1.0;
  for (int k = 0; k < 2; ++k) {
    double* const* xo = k == 0 ? xp : xd;
    for (int i = 0; i < n; ++i) {
      fill_unit(b->pbs[i], k, d, E, xo + (size_t)i * d, &b->host_units[k][i]);
      if (b->stop.rule == 3) b->host_units[k][i].partner_sc = b->pbs[i]->slot[1 - k].sc;
    }
    HIPCHK(hipMemcpyAsync(b->units[k], b->host_units[k].data(), (size_t)n * sizeof(UnitDev), hipMemcpyHostToDevice,
                          b->stream));
  }
  return HOM_OK;
}

void group_run(hom_batch* b, int k, SolveRun& R) {
  hom_problem* p0 = b->pbs[0];
  const int n = b->n, d = p0->desc.d;
  R.st = k == 0 ? b->stream : b->stream2;
  R.g = make_geo(p0, k, d, p0->desc.precision == HOM_MIXED, 0, &b->tune[k][d]);
  R.fp32 = p0->desc.precision == HOM_MIXED;
  R.units = b->units[k];
  R.n = n;
  R.iter_base = b->iter_base[k];
  R.active = b->active[k];
  R.pinned_active = b->pinned + k;
  R.graph = &b->graph[k][d];
  R.capture = false;
  R.chunk = batch_chunk(b, p0);
  R.stop = b->stop;
  for (int i = 0; i < n; ++i) {
    R.part_d.push_back(b->pbs[i]->slot[k].part_d);
    R.sc.push_back(b->pbs[i]->slot[k].sc);
  }
  R.collect_dev = b->collect_dev + (size_t)k * n * kMaxLoads;
  R.collect_host = b->collect_host + (size_t)k * n * kMaxLoads;
  if (b->timing) {
    R.events = &b->tevents[k][d];
    R.tsum = b->tsum;
    R.tcnt = b->tcnt;
  }
}

// `chunks` chunks of every run captured on the root stream: a fork event, each
// run's chunks on its own stream, each joined back.
hom_status group_capture(std::vector<SolveRun>& runs, hipStream_t root, std::vector<hipEvent_t>& evs, int chunks,
                         hipGraphExec_t* out) {
  const size_t nr = runs.size();
  hipEvent_t fork = evs[0];
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(root, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipEventRecord(fork, root);
  for (size_t r = 0; r < nr && e == hipSuccess; ++r)
    if (runs[r].st != root) e = hipStreamWaitEvent(runs[r].st, fork, 0);
  for (int c = 0; c < chunks && e == hipSuccess; ++c)
    for (size_t r = 0; r < nr && e == hipSuccess; ++r) e = enqueue_chunk(runs[r]);
  for (size_t r = 0; r < nr && e == hipSuccess; ++r) {
    if (runs[r].st != root) {
      e = hipEventRecord(evs[1 + r], runs[r].st);
      if (e == hipSuccess) e = hipStreamWaitEvent(root, evs[1 + r], 0);
    }
  }
  hipError_t e2 = hipStreamEndCapture(root, &graph);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return HOM_E_DEVICE;
  }
  e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  return e == hipSuccess ? HOM_OK : HOM_E_DEVICE;
}
}  // namespace

extern "C" {

hom_status hom_group_create(hom_batch* const* batches, int32_t n, hom_group** out) {
  if (!batches || n < 1 || !out) return HOM_E_INVALID;
  for (int i = 0; i < n; ++i) {
    if (!batches[i] || batch_has_gani(batches[i])) return HOM_E_INVALID;
    for (int j = 0; j < i; ++j)
      if (batches[j] == batches[i]) return HOM_E_INVALID;
  }
  hom_group* g = new hom_group();
  g->bs.assign(batches, batches + n);
  g->chunks = std::max(1, std::min(16, env_int("HOM_GROUP_CHUNKS", 1)));
  // fork, one join per run (2 per batch), one order event per batch
  g->evs.assign((size_t)1 + 2 * n + n, nullptr);
  for (auto& ev : g->evs)
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      for (auto x : g->evs)
        if (x) (void)hipEventDestroy(x);
      delete g;
      return HOM_E_DEVICE;
    }
  *out = g;
  return HOM_OK;
}

// Closing work of the runs of a group (run 2 bi + k: side k of batch bi), as
// for a pair solve.
struct GroupClose {
  hom_group* grp;
  std::vector<SolveRun>* runs;
  bool bounds;
  std::vector<char> queued;
};

static hom_status group_close(void* ctx, int r) {
  GroupClose& c = *static_cast<GroupClose*>(ctx);
  if (c.queued[r]) return HOM_OK;
  hom_batch* b = c.grp->bs[r / 2];
  SolveRun& R = (*c.runs)[r];
  hom_status s = finish_enqueue(R, b->pbs[0]->desc.d);
  if (s == HOM_OK && c.bounds) s = launch_batch_bounds(b, r & 1, R.st);
  if (s == HOM_OK) c.queued[r] = 1;
  return s;
}

static hom_status group_solve(hom_group* grp, double tol, int32_t maxit, double* const* x_primal,
                              double* const* x_dual, hom_info* info_primal, hom_info* info_dual, hom_result* bounds) {
  if (!grp || !x_primal || !x_dual || !info_primal || !info_dual) return HOM_E_INVALID;
  const int nb = (int)grp->bs.size();
  // validation of every batch before anything is launched
  size_t off = 0;
  for (hom_batch* b : grp->bs) {
    const int d = b->pbs[0]->desc.d;
    double E[9] = {};
    for (int l = 0; l < d; ++l) E[l * d + l] = 1.0;
    if (batch_has_gani(b) || b->pbs[0]->max_loads < d) return HOM_E_INVALID;
    for (int i = 0; i < b->n; ++i) {
      hom_status s = check_solve_args(b->pbs[i], d, E, x_primal + off + (size_t)i * d, tol, maxit);
      if (s == HOM_OK) s = check_solve_args(b->pbs[i], d, E, x_dual + off + (size_t)i * d, tol, maxit);
      if (s != HOM_OK) return s;
    }
    off += (size_t)b->n * d;
  }
  std::vector<SolveRun> runs(2 * (size_t)nb);
  hipStream_t root = grp->bs[0]->stream;
  bool timing = false;
  off = 0;
  for (int bi = 0; bi < nb; ++bi) {
    hom_batch* b = grp->bs[bi];
    const int d = b->pbs[0]->desc.d;
    if (!side_stream(b)) return HOM_E_DEVICE;
    for (int k = 0; k < 2; ++k)
      if (!b->tuned[k][d]) {
        hom_status s = solve_tuning(b->pbs.data(), b->n, k, d, b->units[k], b->stream, &b->tune[k][d]);
        if (s != HOM_OK) return s;
        b->tuned[k][d] = true;
      }
    hom_status s = group_units(b, x_primal + off, x_dual + off);
    if (s != HOM_OK) return s;
    off += (size_t)b->n * d;
    group_run(b, 0, runs[2 * bi]);
    group_run(b, 1, runs[2 * bi + 1]);
    timing = timing || b->timing;
    // everything on this batch's stream so far (the caller's setup, the unit tables) before the group's work
    HIPCHK(hipEventRecord(grp->evs[1 + 2 * nb + bi], b->stream));
  }
  for (int bi = 0; bi < nb; ++bi) {
    hom_batch* b = grp->bs[bi];
    for (int bj = 0; bj < nb; ++bj)
      for (hipStream_t st : {b->stream, b->stream2})
        if (bj != bi || st != b->stream) HIPCHK(hipStreamWaitEvent(st, grp->evs[1 + 2 * nb + bj], 0));
  }
  // bound-pass unit tables of both sides of every batch, on the sides' streams
  off = 0;
  for (int bi = 0; bi < nb && bounds; ++bi) {
    hom_batch* b = grp->bs[bi];
    for (int k = 0; k < 2; ++k) {
      hom_status s = upload_batch_bounds(b, k, (k == 0 ? x_primal : x_dual) + off, runs[2 * bi + k].st);
      if (s != HOM_OK) return s;
    }
    off += (size_t)b->n * b->pbs[0]->desc.d;
  }
  // one graph launch advances every solve by its chunk and waits for the slowest, so in launch
  // mode 0 every solve takes the longest chunk of the group (a 3D batch's short chunks would
  // multiply the launches of the whole graph); not under the gap rule, whose stops depend on the
  // chunk boundaries, so that every launch mode stops where the batch's own solves do
  int chunk_max = 1;
  bool any_gap = false;
  for (auto& R : runs) {
    chunk_max = std::max(chunk_max, R.chunk);
    any_gap = any_gap || R.stop.rule == 3;
  }
  for (auto& R : runs) {
    R.capture = grp->launch == 1;      // launch mode 1 replays each solve's own chunk graph
    if (grp->launch == 0 && !any_gap) R.chunk = chunk_max;
    hom_status s = start_run(R, R.g.L, tol, maxit, false);
    if (s != HOM_OK) return s;
  }
  hom_status s = HOM_OK;
  GroupClose close{grp, &runs, bounds != nullptr, std::vector<char>(runs.size(), 0)};
  const bool graphs = !timing && std::all_of(runs.begin(), runs.end(), [](const SolveRun& R) { return R.use_graph; });
  if (graphs && grp->launch == 1) {
    // every solve's chunk graph on its own stream, one host loop over all of them; the
    // primal and dual of a batch are partners under the gap rule
    std::vector<SolveRun*> rp;
    std::vector<int> partner(runs.size(), -1);
    for (size_t r = 0; r < runs.size(); ++r) {
      rp.push_back(&runs[r]);
      if (grp->bs[r / 2]->stop.rule == 3) partner[r] = (int)(r ^ 1);
    }
    s = loop_runs(rp.data(), (int)rp.size(), maxit, partner.data(), group_close, &close);
    if (s != HOM_OK) return s;
  } else if (graphs) {
    // the captured graph holds the geometry (tile shapes) and the stopping rule of every run
    std::vector<Tuning> tiles;
    for (hom_batch* b : grp->bs)
      for (int k = 0; k < 2; ++k) tiles.push_back(b->tune[k][b->pbs[0]->desc.d]);
    const int rule = grp->bs[0]->stop.rule;
    bool gap = false;
    for (hom_batch* b : grp->bs) gap = gap || b->stop.rule == 3;
    // under the gap rule a chunk must see its partner's previous chunk complete: one chunk per launch
    const int chunks = gap ? 1 : grp->chunks;
    bool same = grp->graph && grp->graph_rule == rule && grp->graph_chunks == chunks &&
                tiles.size() == grp->graph_tiles.size();
    for (size_t i = 0; same && i < tiles.size(); ++i) same = std::memcmp(&tiles[i], &grp->graph_tiles[i], sizeof(Tuning)) == 0;
    if (!same) {
      if (grp->graph) (void)hipGraphExecDestroy(grp->graph);
      grp->graph = nullptr;
      // the start kernels of every run come before the capture's fork on the root stream
      for (size_t r = 0; r < runs.size(); ++r)
        if (runs[r].st != root) {
          HIPCHK(hipEventRecord(grp->evs[1 + r], runs[r].st));
          HIPCHK(hipStreamWaitEvent(root, grp->evs[1 + r], 0));
        }
      s = group_capture(runs, root, grp->evs, chunks, &grp->graph);
      if (s != HOM_OK) return s;
      grp->graph_tiles = tiles;
      grp->graph_rule = rule;
      grp->graph_chunks = chunks;
    } else {
      for (size_t r = 0; r < runs.size(); ++r)
        if (runs[r].st != root) {
          HIPCHK(hipEventRecord(grp->evs[1 + r], runs[r].st));
          HIPCHK(hipStreamWaitEvent(root, grp->evs[1 + r], 0));
        }
    }
    // one launch advances every solve by a chunk; one chunk stays in flight while the
    // host reads the active counts of the one before
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
    int it = 0, done = 0;
    // the iteration guard counts the shortest chunk (runs of 2D and 3D batches differ)
    int chunk = runs[0].chunk;
    for (auto& R : runs) chunk = std::min(chunk, R.chunk);
    chunk *= grp->graph_chunks;
    if (e == hipSuccess) e = hipGraphLaunch(grp->graph, root);
    if (e == hipSuccess) e = hipEventRecord(ev[0], root);
    while (e == hipSuccess) {
      e = hipGraphLaunch(grp->graph, root);
      if (e == hipSuccess) e = hipEventRecord(ev[(it + 1) & 1], root);
      if (e == hipSuccess) e = hipEventSynchronize(ev[it & 1]);
      if (e != hipSuccess) break;
      done += chunk;
      ++it;
      bool any = false;
      for (auto& R : runs) any = any || *R.pinned_active != 0;
      if (!any || done > maxit + chunk) break;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(root);
    for (auto x : ev)
      if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) return HOM_E_DEVICE;
  } else {
    std::vector<SolveRun*> rp;
    for (auto& R : runs) rp.push_back(&R);
    s = loop_direct(rp.data(), (int)rp.size(), maxit);
    if (s != HOM_OK) return s;
  }
  // per-run residual checks and summaries, worst status over the group (every
  // run's residual passes are enqueued before the first is read)
  for (size_t r = 0; r < runs.size(); ++r) {
    s = group_close(&close, (int)r);
    if (s != HOM_OK) return s;
  }
  hom_status worst = HOM_OK;
  off = 0;
  for (int bi = 0; bi < nb; ++bi) {
    const int d = grp->bs[bi]->pbs[0]->desc.d;
    for (int k = 0; k < 2; ++k) {
      hom_info* info = (k == 0 ? info_primal : info_dual) + off;
      hom_status r = finish_run(runs[2 * bi + k], d, maxit, info, true);
      if (r < 0 && (worst >= 0 || r < worst)) worst = r;
      else if (r == HOM_NOT_CONVERGED && worst == HOM_OK) worst = r;
    }
    off += (size_t)grp->bs[bi]->n * d;
  }
  for (hom_batch* b : grp->bs) HIPCHK(hipStreamSynchronize(b->stream2));
  if (bounds) {
    const bool have[2] = {true, true};
    for (hom_batch* b : grp->bs) {
      s = read_batch_bounds(b, have, bounds);
      if (s != HOM_OK) return s;
      bounds += b->n;
    }
  }
  return worst;
}

hom_status hom_group_solve_pair(hom_group* grp, double tol, int32_t maxit, double* const* x_primal,
                                double* const* x_dual, hom_info* info_primal, hom_info* info_dual) {
  return group_solve(grp, tol, maxit, x_primal, x_dual, info_primal, info_dual, nullptr);
}

hom_status hom_group_solve_bounds(hom_group* grp, double tol, int32_t maxit, double* const* x_primal,
                                  double* const* x_dual, hom_info* info_primal, hom_info* info_dual,
                                  hom_result* out) {
  if (!out) return HOM_E_INVALID;
  return group_solve(grp, tol, maxit, x_primal, x_dual, info_primal, info_dual, out);
}

hom_status hom_group_set_launch(hom_group* grp, int32_t mode) {
  if (!grp || (mode != 0 && mode != 1)) return HOM_E_INVALID;
  grp->launch = mode;
  return HOM_OK;
}

void hom_group_destroy(hom_group* grp) {
  if (!grp) return;
  if (grp->graph) (void)hipGraphExecDestroy(grp->graph);
  for (auto x : grp->evs)
    if (x) (void)hipEventDestroy(x);
  delete grp;
}

hom_status hom_batch_update_coefficients(hom_batch* b, const void* const* Ahat, const void* const* Bhat) {
  if (!b || !Ahat || !Bhat) return HOM_E_INVALID;
  for (int i = 0; i < b->n; ++i)
    if (!Ahat[i] || !Bhat[i]) return HOM_E_INVALID;
  // every cell in two transform launches and one extraction launch where the
  // specialised set-up exists, else cell by cell
  hom_problem* p0 = b->pbs[0];
  const Sizes& z = p0->z;
  const int n = b->n;
  b->host_jobs.resize(n);
  for (int i = 0; i < n; ++i) {
    const hom_problem* pb = b->pbs[i];
    CoefJob& J = b->host_jobs[i];
    J.A = reinterpret_cast<const Cx<double>*>(Ahat[i]);
    J.B = reinterpret_cast<const Cx<double>*>(Bhat[i]);
    J.scratch = pb->scratch;
    J.a64 = pb->coef64[0];
    J.a32 = pb->coef32[0];
    J.b64 = pb->coef64[1];
    J.b32 = pb->coef32[1];
    J.half[0] = pb->ahat_half[0];
    J.half[1] = pb->ahat_half[1];
  }
  hipStream_t st = b->stream;
  HIPCHK(hipMemcpyAsync(b->jobs_dev, b->host_jobs.data(), (size_t)n * sizeof(CoefJob), hipMemcpyHostToDevice, st));
  hipError_t e = hipSuccess;
  if (fast_coef_setup_jobs(z.d, z.M, z.nc, b->jobs_dev, n, p0->tw64[0], st, &e)) {
    HIPCHK(e);
    HIPCHK(launch_extract_half_jobs(make_geo(p0, 0, 1, false), b->jobs_dev, n, z.nc, st));
    return HOM_OK;
  }
  for (int i = 0; i < n; ++i) {
    hom_status s = setup_coefficients(b->pbs[i], Ahat[i], Bhat[i]);
    if (s != HOM_OK) return s;
  }
  return HOM_OK;
}

// FP64 bound passes of one side (k = 0 primal, 1 dual) of every problem of a
// batch, enqueued on st: the side's own bound buffers (so the two sides may
// run on different streams at once) and its quadrature sums in the batch
// workspace.  upload_batch_bounds copies the side's unit table (f: n * d
// device pointers, problem-major, unit loads); launch_batch_bounds enqueues
// the passes that read it.
static hom_status upload_batch_bounds(hom_batch* b, int k, const double* const* f, hipStream_t st) {
  const int n = b->n;
  const int d = b->pbs[0]->desc.d;
  for (int i = 0; i < n; ++i) {
    hom_problem* pb = b->pbs[i];
    UnitDev* hu = &b->host_bunits[k][i];
    std::memset(hu, 0, sizeof(*hu));
    hu->coef = pb->coef64[k];
    hu->ahat = pb->ahat_half[k];
    for (int l = 0; l < d; ++l) {
      hu->x[l] = reinterpret_cast<Cx<double>*>(const_cast<double*>(f[(size_t)i * d + l]));
      hu->E[l][l] = 1.0;
    }
    hu->bufA = k == 0 ? pb->bbufA : pb->bbufA2;
    hu->bufB = k == 0 ? pb->bbufB : pb->bbufB2;
    hu->part_q = pb->bpart_q[k];
  }
  HIPCHK(hipMemcpyAsync(b->bunits[k], b->host_bunits[k].data(), (size_t)n * sizeof(UnitDev), hipMemcpyHostToDevice,
                        st));
  return HOM_OK;
}

static hom_status launch_batch_bounds(hom_batch* b, int k, hipStream_t st) {
  const int n = b->n;
  hom_problem* p0 = b->pbs[0];
  const int d = p0->desc.d;
  const Geo g = make_geo(p0, k, d, false, packs(d, d));
  HIPCHK(launch_first<double>(g, b->bunits[k], n, FIRST_BOUNDS, 0, nullptr, st));
  if (d == 3) HIPCHK(launch_mid<double>(g, b->bunits[k], n, 1, st));
  HIPCHK(launch_apply<double>(g, b->bunits[k], n, APPLY_QUAD, st));
  HIPCHK(launch_collect_bounds(b->bunits[k], n, g.nbA, b->bcollect_dev + (size_t)k * n * 9, st));
  return HOM_OK;
}

// Copies both sides' quadrature sums to the host on the batch stream (after
// the work on it), waits, and fills the results (sides not in have: NaN).
static hom_status read_batch_bounds(hom_batch* b, const bool have[2], hom_result* out) {
  const int n = b->n;
  hom_problem* p0 = b->pbs[0];
  const int d = p0->desc.d;
  HIPCHK(hipMemcpyAsync(b->bcollect_host, b->bcollect_dev, (size_t)2 * n * 9 * sizeof(double), hipMemcpyDeviceToHost,
                        b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  const double invM = make_geo(p0, 0, d, false, packs(d, d)).invM;
  for (int i = 0; i < n; ++i) {
    double Ebar[2][9];
    for (int k = 0; k < 2; ++k) {
      for (int j = 0; j < 9; ++j) Ebar[k][j] = NAN;
      if (!have[k]) continue;
      const double* sums = b->bcollect_host + ((size_t)k * n + i) * 9;
      for (int a = 0; a < d; ++a)
        for (int c = 0; c < d; ++c) Ebar[k][a * d + c] = sums[a * kMaxLoads + c] * invM;
    }
    fill_result(d, Ebar, have, &out[i]);
  }
  return HOM_OK;
}

hom_status hom_batch_bounds(hom_batch* b, const double* const* primal, const double* const* dual, hom_result* out) {
  if (!b || !out) return HOM_E_INVALID;
  const int n = b->n;
  const int d = b->pbs[0]->desc.d;
  for (int k = 0; k < 2; ++k) {
    const double* const* f = k == 0 ? primal : dual;
    if (f)
      for (int i = 0; i < n * d; ++i)
        if (!f[i]) return HOM_E_INVALID;
  }
  const bool have[2] = {primal != nullptr, dual != nullptr};
  // with both sides the dual's passes run on the second stream, beside the
  // primal's, and the batch stream waits for them before the copy
  hipStream_t sts[2] = {b->stream, b->stream};
  if (have[0] && have[1]) {
    if (!side_stream(b)) return HOM_E_DEVICE;
    HIPCHK(hipEventRecord(b->order_ev, b->stream));
    HIPCHK(hipStreamWaitEvent(b->stream2, b->order_ev, 0));
    sts[1] = b->stream2;
  }
  for (int k = 0; k < 2; ++k) {
    if (!have[k]) continue;
    hom_status s = upload_batch_bounds(b, k, k == 0 ? primal : dual, sts[k]);
    if (s == HOM_OK) s = launch_batch_bounds(b, k, sts[k]);
    if (s != HOM_OK) return s;
  }
  if (sts[1] != b->stream) {
    HIPCHK(hipEventRecord(b->order_ev, b->stream2));
    HIPCHK(hipStreamWaitEvent(b->stream, b->order_ev, 0));
  }
  return read_batch_bounds(b, have, out);
}

hom_status hom_batch_profile_passes(hom_batch* b, int32_t dual, int32_t nload, int32_t reps, double* ms_out) {
  if (!b || !ms_out || (dual != 0 && dual != 1) || reps < 1) return HOM_E_INVALID;
  hom_problem* p0 = b->pbs[0];
  if (nload < 1 || nload > p0->max_loads) return HOM_E_INVALID;
  const int k = dual, n = b->n;
  const bool fp32 = p0->desc.precision == HOM_MIXED;
  Geo g = make_geo(p0, k, nload, fp32, 0, b->tuned[k][nload] ? &b->tune[k][nload] : nullptr);
  for (int i = 0; i < n; ++i) {
    hom_status s = profile_unit_setup(b->pbs[i], k, nload, g, &b->host_units[k][i]);
    if (s != HOM_OK) return s;
  }
  HIPCHK(hipMemcpyAsync(b->units[k], b->host_units[k].data(), (size_t)n * sizeof(UnitDev), hipMemcpyHostToDevice,
                        b->stream));
  return profile_units(g, b->units[k], n, fp32, b->stream, reps, ms_out);
}

hom_status hom_batch_set_timing(hom_batch* b, int32_t on) {
  if (!b) return HOM_E_INVALID;
  b->timing = on ? 1 : 0;
  for (int i = 0; i < 5; ++i) {
    b->tsum[i] = 0.0;
    b->tcnt[i] = 0;
  }
  return HOM_OK;
}

hom_status hom_batch_get_timing(hom_batch* b, double* ms_sum, int64_t* launches) {
  if (!b || !ms_sum || !launches) return HOM_E_INVALID;
  for (int i = 0; i < 5; ++i) {
    ms_sum[i] = b->tsum[i];
    launches[i] = b->tcnt[i];
  }
  return HOM_OK;
}

static void tuning_report(const hom_problem* p0, int k, int nload, const Tuning& t, hom_tuning* out) {
  const Geo g = make_geo(p0, k, nload, p0->desc.precision == HOM_MIXED, 0, &t);
  out->row_pairs = p0->desc.precision == HOM_MIXED ? fast_row_pairs(g.M[2], g.N[2], g.d, nload, t.rowG) : 0;
  out->row_threads = t.rowThreads;
  out->apply_points = t.apTP;
  out->apply_half_exchange = t.apHX;
  out->apply_all_packs = t.apAll;
  out->candidates = t.candidates;
  out->row_ms = t.row_ms;
  out->apply_ms = t.apply_ms;
}

static bool stop_args_ok(int32_t rule, double etol, double a_min, double a_max) {
  if (rule < 0 || rule > 3) return false;
  if (rule > 0 && !(etol > 0.0 && etol < 1.0)) return false;
  if (!(a_min >= 0.0 && a_min < INFINITY) || !(a_max >= 0.0 && a_max < INFINITY)) return false;
  return !(a_min > 0.0 && a_max > 0.0 && a_min > a_max);
}

static StopCfg make_stop(int32_t rule, double etol, double a_min, double a_max) {
  StopCfg c;
  c.rule = rule;
  c.etol = rule ? etol : 0.0;
  c.a_min = a_min;
  c.a_max = a_max;
  return c;
}

hom_status hom_problem_set_stop(hom_problem* pb, int32_t rule, double etol, double a_min, double a_max) {
  if (!pb || !stop_args_ok(rule, etol, a_min, a_max)) return HOM_E_INVALID;
  pb->stop = make_stop(rule, etol, a_min, a_max);
  return HOM_OK;
}

hom_status hom_batch_set_stop(hom_batch* b, int32_t rule, double etol, double a_min, double a_max) {
  if (!b || !stop_args_ok(rule, etol, a_min, a_max)) return HOM_E_INVALID;
  b->stop = make_stop(rule, etol, a_min, a_max);
  return HOM_OK;
}

hom_status hom_tune_cache_load(const char* path, const char* arch, int32_t* loaded) {
  if (!path) return HOM_E_INVALID;
  const std::string a = arch ? std::string(arch) : device_arch();
  if (a.empty()) return HOM_E_DEVICE;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  int n = 0;
  const bool ok = tune_file_read(path, a, &n);
  if (loaded) *loaded = n;
  return ok ? HOM_OK : HOM_E_INVALID;
}

hom_status hom_tune_cache_save(const char* path, const char* arch) {
  if (!path) return HOM_E_INVALID;
  const std::string a = arch ? std::string(arch) : device_arch();
  if (a.empty()) return HOM_E_DEVICE;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return tune_file_write(path, a) ? HOM_OK : HOM_E_INVALID;
}

hom_status hom_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache.clear();
  return HOM_OK;
}

hom_status hom_set_tuning(int32_t mode) {
  if (mode != 0 && mode != 1) return HOM_E_INVALID;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_mode = mode;
  return HOM_OK;
}

// Validate a caller-chosen tile shape for solves of (dual, nload) of problem p0.
static bool tiles_ok(const hom_problem* p0, int nload, const hom_tuning* t) {
  if (p0->desc.precision != HOM_MIXED) return false;
  const Sizes& z = p0->z;
  if (t->row_pairs != 0 && fast_row_pairs(z.M[2], z.N[2], z.d, nload, t->row_pairs) != t->row_pairs) return false;
  if (t->row_threads != 0 && (t->row_threads % 64 != 0 || t->row_threads > 256)) return false;
  return fast_apply_shape_ok(z.M[0], z.d, t->apply_points, t->apply_half_exchange, t->apply_all_packs);
}

static Tuning tiles_from(const hom_tuning* t) {
  Tuning u;
  u.rowG = t->row_pairs;
  u.rowThreads = t->row_threads;
  u.apTP = t->apply_points;
  u.apHX = t->apply_half_exchange;
  u.apAll = t->apply_all_packs;
  return u;
}

hom_status hom_problem_set_tiles(hom_problem* pb, int32_t dual, int32_t nload, const hom_tuning* t) {
  if (!pb || !t || (dual != 0 && dual != 1) || nload < 1 || nload > pb->max_loads) return HOM_E_INVALID;
  if (!tiles_ok(pb, nload, t)) return HOM_E_INVALID;
  const int k = dual;
  HIPCHK(hipStreamSynchronize(pb->stream));
  if (pb->graph[k][nload]) {
    (void)hipGraphExecDestroy(pb->graph[k][nload]);
    pb->graph[k][nload] = nullptr;
  }
  pb->tune[k][nload] = tiles_from(t);
  pb->tuned[k][nload] = true;
  return HOM_OK;
}

hom_status hom_batch_set_tiles(hom_batch* b, int32_t dual, int32_t nload, const hom_tuning* t) {
  if (!b || !t || (dual != 0 && dual != 1) || nload < 1 || nload > b->pbs[0]->max_loads) return HOM_E_INVALID;
  if (!tiles_ok(b->pbs[0], nload, t)) return HOM_E_INVALID;
  const int k = dual;
  HIPCHK(hipStreamSynchronize(b->stream));
  if (b->graph[k][nload]) {
    (void)hipGraphExecDestroy(b->graph[k][nload]);
    b->graph[k][nload] = nullptr;
  }
  b->tune[k][nload] = tiles_from(t);
  b->tuned[k][nload] = true;
  return HOM_OK;
}

hom_status hom_problem_tuning(hom_problem* pb, int32_t dual, int32_t nload, hom_tuning* out) {
  if (!pb || !out || (dual != 0 && dual != 1) || nload < 1 || nload > pb->max_loads) return HOM_E_INVALID;
  const int k = dual;
  if (!pb->tuned[k][nload]) {
    hom_status s = solve_tuning(&pb, 1, k, nload, pb->slot[k].unit, pb->stream, &pb->tune[k][nload]);
    if (s != HOM_OK) return s;
    pb->tuned[k][nload] = true;
  }
  tuning_report(pb, k, nload, pb->tune[k][nload], out);
  return HOM_OK;
}

hom_status hom_batch_tuning(hom_batch* b, int32_t dual, int32_t nload, hom_tuning* out) {
  if (!b || !out || (dual != 0 && dual != 1) || nload < 1 || nload > b->pbs[0]->max_loads) return HOM_E_INVALID;
  const int k = dual;
  if (!b->tuned[k][nload]) {
    hom_status s = solve_tuning(b->pbs.data(), b->n, k, nload, b->units[k], b->stream, &b->tune[k][nload]);
    if (s != HOM_OK) return s;
    b->tuned[k][nload] = true;
  }
  tuning_report(b->pbs[0], k, nload, b->tune[k][nload], out);
  return HOM_OK;
}

void hom_batch_destroy(hom_batch* b) {
  if (!b) return;
  for (int k = 0; k < 2; ++k)
    for (int l = 0; l <= kMaxLoads; ++l) {
      if (b->graph[k][l]) (void)hipGraphExecDestroy(b->graph[k][l]);
      if (b->tgraph[k][l]) (void)hipGraphExecDestroy(b->tgraph[k][l]);
      for (auto ev : b->tevents[k][l]) (void)hipEventDestroy(ev);
    }
  if (b->collect_host) (void)hipHostFree(b->collect_host);
  if (b->bcollect_host) (void)hipHostFree(b->bcollect_host);
  if (b->pinned) (void)hipHostFree(b->pinned);
  if (b->order_ev) (void)hipEventDestroy(b->order_ev);
  if (b->stream2) {
    (void)hipStreamSynchronize(b->stream2);
    (void)hipStreamDestroy(b->stream2);
  }
  delete b;
}

void hom_destroy(hom_problem* pb) {
  if (!pb) return;
  for (int k = 0; k < 2; ++k)
    for (int l = 0; l <= kMaxLoads; ++l) {
      if (pb->graph[k][l]) (void)hipGraphExecDestroy(pb->graph[k][l]);
      if (pb->gani.graph[k][l]) (void)hipGraphExecDestroy(pb->gani.graph[k][l]);
    }
  if (pb->pinned_active) (void)hipHostFree(pb->pinned_active);
  delete pb;
}

}  // extern "C"
