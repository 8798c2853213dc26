// Internal types shared by the kernels and the C ABI layer of libhom.
//
// Internal geometry always has three axes.  A 2D problem (N0, N1) is
// embedded as (N0, 1, N1): the middle axis has one point, so its FFT pass is
// skipped and every kernel is written once.  Physical axis g of the problem
// is internal axis phys_axis[g].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hom {

constexpr int kMaxLoads = 3;      // loads solved together per coefficient field
constexpr int kMaxPacks = 5;      // ceil(3 loads * 3 components / 2)
constexpr size_t kLdsMax = 160 * 1024;  // LDS bytes per workgroup (gfx950)
constexpr int kMaxStages = 12;    // radix-3/5 stages per FFT length
constexpr int kBlock = 256;       // threads per block of every pipeline kernel

template <typename R>
struct __align__(2 * sizeof(R)) Cx {
  R x, y;
};

// Radix schedule of one FFT length (product of r[0..n-1]).
struct Plan {
  int n;
  int r[kMaxStages];
};

// Per-load CG scalars (Chronopoulos-Gear recurrence), double-buffered by iteration parity.
struct CgScal {
  double gamma[2];   // <r_i, r_i>
  double beta[2];    // gamma_i / gamma_{i-1}
  double alpha[2];   // step length alpha_i
  double normE;      // ||E||
  double gamma0;     // <r_0, r_0>
  double gamma_last; // <r, r> at exit
  int32_t status;    // 0 active, 1 converged, 2 maxit, -3 not SPD, -1 invalid (NaN)
  int32_t iters;     // iteration index at exit
  double tol;
  int32_t maxit;
  int32_t stop;      // 0: residual rule ||r|| <= tol ||E||; 1: energy rule (below)
  double etol;       // energy rule: stop when the extrapolated remaining energy decrease <= etol * energy
  double energy0;    // energy of the zero field: E^T <A> E (primal) or E^T <A^-1> E (dual)
  double esum;       // energy0 minus the energy of the iterate: decrease to a given x0 plus the
                     // decrements alpha_j gamma_j so far
  double edec[4];    // the last four decrements
  double mu;         // guaranteed rule: lower bound on the spectrum of the operator (0: none)
  double phi[2];     // guaranteed rule: Gauss-Radau factor, remaining energy <= gamma phi
  // gap rule (3): the partner solve of the same load (the dual of a primal solve and the
  // reverse) and, per chunk of iterations, this solve's energy and Gauss-Radau bound at the
  // chunk's last iterate (slot c & 1 for chunk c; slot 1 holds the start, bound infinite)
  const CgScal* partner;
  double snap_e[2];
  double snap_r[2];
  double rem;        // Gauss-Radau bound of the latest tested iterate
  int32_t chunk;     // iterations per chunk
  int32_t side;      // 0 primal, 1 dual
};

// Stopping rule of a solve: 0 residual; 1 residual or extrapolated energy;
// 2 residual or guaranteed energy bound; 3 residual or the gap rule (primal
// and dual side by side, etol = theta).  a_min / a_max: bounds on the
// pointwise eigenvalues of the coefficient given by the caller (0: none).
struct StopCfg {
  int rule = 0;
  double etol = 0.0, a_min = 0.0, a_max = 0.0;
};

// End-of-solve summary of one (unit, load): sum of the residual partials and the CG scalars.
struct SolveOut {
  double rres;
  CgScal sc;
};

// One coefficient field with L loads: device-resident pointers.
struct UnitDev {
  const void* coef;                  // R-typed [nc][M0*M1*M2] on the doubled grid
  const Cx<double>* ahat;            // [nc][S] Fourier coefficients on the stored half of Z_N
  Cx<double>* x[kMaxLoads];
  Cx<double>* r[kMaxLoads];
  Cx<double>* p[kMaxLoads];
  Cx<double>* s[kMaxLoads];
  Cx<double>* b[kMaxLoads];
  void* bufA;                        // [N0][N1][M2][P]
  void* bufB;                        // [N0][M1][M2][P] (3D only)
  double* part_g;                    // [L][nbF]
  double* part_d;                    // [L][nbL]
  double* part_q;                    // [nbApply][9]
  CgScal* sc;                        // [L]
  double E[kMaxLoads][3];            // loads (physical components)
  CgScal* partner_sc;                // [L] CG scalars of the partner solve (gap rule), or null
  float* grid;                       // real fields on the doubled grid [L*d][M^d] (grid transfers)
  const float* coefp;                // FP32 coefficient in plane order [M2][nc][M0][M1] (plane pass), or null
};

// Shape information shared by every unit of a launch (passed by value).
struct Geo {
  int d;               // physical dimension
  int N[3], M[3];      // internal sizes (N[1] = M[1] = 1 for d = 2)
  int H0;              // (N0 + 1) / 2 stored k0 values
  int S;               // H0 * N1 * N2 stored frequencies per component
  int m;               // components of the unknown per load (1 primal, d - 1 dual)
  int L;               // loads per unit
  int P;               // complex packs = ceil(L * d / 2)
  int nc;              // coefficient components
  int dual;            // 0 primal (G^E), 1 dual (G^J)
  int Q;               // stored row pairs handled by the first/last pass
  int nbF, nbL, nbA;   // blocks per unit of first / last / apply pass
  int tileA;           // points per apply-pass block
  int tileM;           // complex elements per middle-pass block
  int rowG;            // row pairs per block of the specialised row passes (0: default)
  int rowThreads;      // threads per block of the specialised row passes (0: default)
  int apTP;            // points per block of the specialised column pass (0: default)
  int apHX;            // 2D column pass: exchange real and imaginary parts separately
  int apAll;           // 2D column pass: all packs of a point block in one block
  int pmaj;            // 2D, both specialised passes: row-pass buffer pack-major [P][N0][M2]
                       // (otherwise [N0][N1][M2][P], packs interleaved)
  int plane;           // 3D: the coefficient product runs as one plane pass (fast_plane), no middle passes
  int phys_axis[3];
  double iY[3];        // 1 / Y_a (internal axes)
  double invM;         // 1 / (M0 M1 M2)
  Plan pl[3];
  const void* tw[3];   // R-typed twiddles exp(-2 pi i t / M_a), t < M_a
};

// *_PROF: the memory traffic of a CG iteration with zero step lengths and no
// scalar updates, on scratch vectors (tile tuning of the specialised passes).
enum FirstMode { FIRST_CG = 0, FIRST_FIELD = 1, FIRST_BOUNDS = 2, FIRST_PROF = 3 };
enum LastMode { LAST_CG = 0, LAST_RESID = 1, LAST_MATVEC = 2, LAST_PROF = 3 };
enum ApplyMode { APPLY_COEF = 0, APPLY_QUAD = 1, APPLY_COEF_CG = 2, APPLY_GRID = 3, APPLY_FWD = 4 };
constexpr int MID_CG = 2;  // flag or-ed into the inverse argument of launch_mid

// Host-side switch of the calling thread: when `on`, its next pipeline kernel launch is issued with
// hipExtLaunchKernelGGL and these start/stop events (kernel-execution
// timestamps), used by the timing mode of batched solves.
struct ExtTiming {
  bool on = false;
  hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local ExtTiming g_ext_timing;

// Launch wrappers (hom_kernels.hip).  All return hipError_t of the launch.
template <typename R>
hipError_t launch_first(const Geo& g, const UnitDev* units, int nunits, int mode, int jstep,
                        const int* iter_base, hipStream_t st);
template <typename R>
hipError_t launch_last(const Geo& g, const UnitDev* units, int nunits, int mode, int jstep,
                       const int* iter_base, hipStream_t st);
template <typename R>
hipError_t launch_apply(const Geo& g, const UnitDev* units, int nunits, int mode, hipStream_t st);
template <typename R>
hipError_t launch_mid(const Geo& g, const UnitDev* units, int nunits, int inverse, hipStream_t st);

// Generic strided complex FFT pass over [outer][L][inner] arrays, full length (setup).
template <typename R>
hipError_t launch_line_fft(Cx<R>* data, int outer, int Lm, int inner, const Plan& pl, const Cx<R>* tw,
                           int inverse, hipStream_t st);

hipError_t launch_rhs(const Geo& g, const UnitDev* units, int nunits, hipStream_t st);
hipError_t launch_init_scal(const Geo& g, const UnitDev* units, int nunits, int* iter_base, int chunk, double tol, int maxit,
                            int stop, double etol, int mu_parts, double mu_user, hipStream_t st);
// Per unit: partial minima over the doubled grid of the smallest eigenvalue of
// the coefficient (the unit's own, primal or dual), nparts of them in part_q.
hipError_t launch_coef_min_eig(bool fp32, const Geo& g, const UnitDev* units, int nunits, int nparts,
                               hipStream_t st);
hipError_t launch_start_vectors(const Geo& g, const UnitDev* units, int nunits, int have_x0, hipStream_t st);
// After the residual of a given start field: the energy decrease from the zero field to it (CgScal::esum).
hipError_t launch_start_energy(const Geo& g, const UnitDev* units, int nunits, hipStream_t st);
hipError_t launch_symmetrize(const Geo& g, const Cx<double>* src, Cx<double>* dst, int m, hipStream_t st);
// The same for many fields of one geometry, one launch.
struct SymJob {
  const Cx<double>* src;
  Cx<double>* dst;
};
hipError_t launch_symmetrize_jobs(const Geo& g, const SymJob* jobs, int njobs, int m, hipStream_t st);
hipError_t launch_advance(const Geo& g, const UnitDev* units, int nunits, int* iter_base, int step,
                          int* active_out, hipStream_t st);
hipError_t launch_twiddles(Cx<double>* t64, Cx<float>* t32, int M, hipStream_t st);
// Per (unit, load): residual partials summed in index order, and the CG scalars.
hipError_t launch_collect_solve(const UnitDev* units, int n, int L, int nbL, SolveOut* out, hipStream_t st);
// Per (unit, entry < 9): bounds quadrature partials summed in index order.
hipError_t launch_collect_bounds(const UnitDev* units, int n, int nbA, double* out, hipStream_t st);
// Network inputs of n cells of one geometry, cell i at out + i stride (weights:
// the primal and dual weight channels, k Mt apart), one launch.
struct NetJob {
  const double* coef64[2];
  const Cx<double>* ahat0[2];
};
hipError_t launch_net_input_jobs(const NetJob* jobs, int n, int nc, int d, long Mt, long S, float* out, size_t stride,
                                 int weights, hipStream_t st);
hipError_t launch_net_input(const double* coef64, int nc, int d, long Mt, const Cx<double>* ahat0, long S, float* out,
                            int weight_only, hipStream_t st);
hipError_t launch_coef_real(const Cx<double>* full, double* c64, float* c32, long n, hipStream_t st);
// FP32 coefficient [nc][M0][M1][M2] copied into plane order [M2][nc][M0][M1] (the 3D plane pass).
hipError_t launch_coef_planes(const float* c32, float* cp, int nc, const int* Mz, hipStream_t st);
hipError_t launch_extract_half(const Geo& g, const Cx<double>* full, Cx<double>* half, int nc, hipStream_t st);
hipError_t launch_coef_incl(int d, const int* Mint, const double* iY, int nc, const double* A0c, int n_incl,
                            const void* dev_incl, Cx<double>* out, hipStream_t st);
hipError_t launch_pixel_factor(int d, const int* Mint, const int* Pint, int nc, const Cx<double>* dft,
                               Cx<double>* out, hipStream_t st);
size_t incl_dev_size();
// Point values of the coefficient on the N grid (internal axes, [nc][N0 N1 N2]).
hipError_t launch_sample_incl(const int* Nint, const double* Yint, int nc, const double* A0c, int n_incl,
                              const void* dev_incl, bool closed, double* out, hipStream_t st);
hipError_t launch_sample_pixels(const int* Nint, const double* Yint, const int* Pint, int nc, const double* img,
                                double* out, hipStream_t st);
// out = s * in as complex values with zero imaginary part; a *= s.
hipError_t launch_real_to_cx(const double* in, Cx<double>* out, size_t n, double s, hipStream_t st);
hipError_t launch_scale_cx(Cx<double>* a, size_t n, double s, hipStream_t st);
// 16 x the smoothed 2D characteristic image (periodic 3 x 3 stencil 4 / 2 / 1).
hipError_t launch_smooth2d(int P0, int P1, const int* f, int* out, hipStream_t st);

// Specialised FP32 passes (hom_fast.hip); false/0 when no specialisation exists.
bool fast_apply(const Geo& g, const UnitDev* units, int n, int cg, hipStream_t st, hipError_t* err);
bool fast_row(bool first, const Geo& g, const UnitDev* units, int n, int mode, int jstep, const int* iter_base,
              hipStream_t st, hipError_t* err);
// Row pairs per block for a requested value (0 or an unsupported value: the default).
int fast_row_pairs(int M, int N, int D, int L, int requested);
bool fast_apply_supported(int M, int D, int P, int NC);
// 3D middle pass (axis 1) for M1 in {25, 81, 125}; flags as launch_mid.
bool fast_mid(const Geo& g, const UnitDev* units, int n, int flags, hipStream_t st, hipError_t* err);
// 3D plane pass (middle, column and middle passes in one kernel) for M = 81 on
// every axis and an isotropic coefficient; *_supported is the host-side test
// (workspace layout, geometry flag), fast_plane the launch (g.plane set).
bool fast_plane_supported(int d, const int* Mz, const int* Nz, int nc);
bool fast_plane(const Geo& g, const UnitDev* units, int n, int cg, hipStream_t st, hipError_t* err);
bool fast_apply_shape_ok(int M, int D, int tp, int hx, int all);
// Both coefficients on the doubled grid (FP64 and, when given, FP32 copies) for
// 2D problems with equal doubled-grid lengths 25, 81, 125 or 625.
bool fast_coef_setup(int d, const int* Mz, int nc, const Cx<double>* Ah, const Cx<double>* Bh, Cx<double>* scratch,
                     double* a64, float* a32, double* b64, float* b32, const Cx<double>* tw, hipStream_t st,
                     hipError_t* err);
// Per-cell pointers of a batched coefficient set-up (a device table, one entry
// per cell): the Fourier data on Z_M, the transform scratch, the grid values
// of A and A^-1, and the stored halves of their Z_N parts.
struct CoefJob {
  const Cx<double>* A;
  const Cx<double>* B;
  Cx<double>* scratch;
  double* a64;
  float* a32;
  double* b64;
  float* b32;
  Cx<double>* half[2];
};
// The same set-up for n cells of one geometry in two launches (grid z = cell).
bool fast_coef_setup_jobs(int d, const int* Mz, int nc, const CoefJob* jobs, int n, const Cx<double>* tw,
                          hipStream_t st, hipError_t* err);
hipError_t launch_extract_half_jobs(const Geo& g, const CoefJob* jobs, int n, int nc, hipStream_t st);
// Device-to-device copy of `bytes` (a multiple of 16, 16-byte aligned pointers).
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t st);
// Up to three device field vectors, passed by value to a kernel.
struct FieldTriple {
  const Cx<double>* p[3];
};
// out = sum_a w[a] x.p[a] over n complex entries.
hipError_t launch_combine(const FieldTriple& x, int d, const double* w, Cx<double>* out, size_t n, hipStream_t st);

// Tile shapes of the specialised passes: row pairs and threads per block of the
// row passes, points per block of the column pass (0 = default).
struct Tuning {
  int rowG = 0, rowThreads = 0, apTP = 0, apHX = 0, apAll = 0;
  double row_ms = 0.0, apply_ms = 0.0;   // measured per first+last pair and per column pass
  int candidates = 0;                    // configurations timed
};
// Times every candidate tile shape of the specialised passes on the given
// units (profile modes, scratch vectors) and returns the fastest in *best.
// g.nbF / g.nbL need not be set.  Returns hipSuccess with best untouched when
// no specialisation applies.
hipError_t tune_fast(const Geo& g, const UnitDev* units, int n, hipStream_t st, int reps, Tuning* best);

}  // namespace hom
