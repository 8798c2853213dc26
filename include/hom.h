/*
 * hom.h -- C ABI of libhom: guaranteed upper/lower bounds on homogenized
 * coefficients by the FFT-based Galerkin method (Vondrejc, Zeman, Marek,
 * "Guaranteed upper-lower bounds on homogenized properties by FFT-based
 * Galerkin method"), hot path on AMD MI355X (gfx950).
 *
 * What is computed.  For a Y-periodic SPD coefficient field A (Sec. 3, eq. A)
 * and an odd grid N (eq. N_odd), the library solves the Galerkin problems of
 * Def. homog_problem restricted to trigonometric polynomials of degree N:
 *   primal  min_{e in E_N} a(E + e, E + e),     a(u,v)    = (A u, v)_{L2}
 *   dual    min_{j in J_N} a^-1(J + j, J + j),  a^-1(u,v) = (A^-1 u, v)_{L2}
 * by conjugate gradients (Sec. 7.1), where the bilinear forms are integrated
 * exactly by the double-grid quadrature (Lemma integral_eval_double_grid):
 * every operator application goes to the doubled grid M = 2N - 1, applies the
 * coefficient there (eq. MBA_GA) and comes back.  The energies of the
 * minimisers are the guaranteed bounds of Def. upper_lower_bounds and
 * Lemma bounds:  Bbar^-1 <= A_H <= Abar.
 *
 * Conventions shared by all entry points
 *  - Every pointer documented as "device" is a HIP device pointer owned by
 *    the caller; the library never frees caller memory.  "host" pointers are
 *    read or written synchronously.
 *  - All device work is ordered on the hipStream_t given at setup (passed as
 *    void*; NULL means the default stream).  Entry points that return host
 *    results (solves, bounds) synchronise that stream before returning.
 *  - No exception crosses the ABI; every entry point returns hom_status.
 *    Arguments are validated before anything is launched.
 *  - Grid sizes N_a must be odd (3 <= N_a <= 4097) and the quadrature grid
 *    M_a (2 N_a - 1, or hom_desc.M) odd with factors 3 and 5 only (the FFT
 *    radices of the solve), M_a <= 8193; sizes whose passes cannot hold a
 *    column of every pack in LDS (2D FP64: M_0 above 5120) are refused too,
 *    with HOM_E_UNSUPPORTED_SIZE.  Even grids enter only as GaNi grids
 *    (hom_set_gani) and as sampling grids (hom_sample_*).
 *
 * Spectral layout of a solution ("field") vector.
 *   A field x in E_N (primal) or J_N (dual) is stored by its Fourier
 *   coefficients on the half index set k0 in [0, (N0-1)/2], k1 in Z_N1,
 *   (k2 in Z_N2), frequencies k_a < 0 stored at index k_a + N_a; the other
 *   half follows from x_hat(-k) = conj(x_hat(k)) (real fields).  At each k
 *   the coefficient is expanded in an orthonormal basis T(k) of the range of
 *   the projection G^E(k) (primal: T = xi/|xi|, xi_a = k_a/Y_a) or G^J(k)
 *   (dual, d = 2: T = (-n_2, n_1); d = 3: t1 = normalised e_a - n_a n with a
 *   the axis of smallest |n_a| (first on ties), t2 = n x t1), so
 *   x_hat(k) = T(k) c(k).  The vector holds c as complex double (re, im
 *   interleaved), m components (primal 1, dual d - 1) outermost:
 *     index = ((c * H0 + k0) * N1 + (k1 mod N1)) [* N2 + (k2 mod N2)],
 *   H0 = (N0 + 1)/2.  The entry k = 0 is zero.  hom_field_len() returns the
 *   number of complex entries.
 */
#ifndef HOM_H
#define HOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HOM_OK = 0,
  HOM_NOT_CONVERGED = 1,        /* warning: maxit reached; outputs are valid, the bounds still guaranteed */
  HOM_E_INVALID = -1,           /* bad argument (null pointer, d, tolerance, ...) */
  HOM_E_UNSUPPORTED_SIZE = -2,  /* even N, M not odd 3/5-smooth, a size beyond the LDS of the passes, or a
                                   GaNi grid without a 2/3/5 transform */
  HOM_E_NOT_SPD = -3,           /* CG met <p, C p> <= 0: the coefficient is not SPD */
  HOM_E_DEVICE = -4,            /* a HIP call failed */
  HOM_E_WORKSPACE = -5          /* workspace too small or misaligned */
} hom_status;

enum { HOM_FP64 = 0, HOM_MIXED = 1 };   /* hom_desc.precision */

typedef struct {
  int32_t d;          /* 2 or 3 */
  int32_t N[3];       /* odd grid sizes per axis (N[2] ignored for d = 2) */
  double  Y[3];       /* cell side lengths Y_a > 0 (cell = prod (-Y_a/2, Y_a/2)) */
  int32_t precision;  /* HOM_FP64: everything FP64.  HOM_MIXED: FFTs and the coefficient
                         apply in FP32; CG vectors, inner products, residual recurrence,
                         right-hand side and the bound quadrature in FP64 */
  int32_t ncoef;      /* 1: isotropic a(x) I.  d(d+1)/2: symmetric matrix, components
                         ordered xx, yy, (zz), xy, (xz, yz) */
  int32_t M[3];       /* quadrature grid per axis.  0: the doubled grid 2N - 1 of Lemma
                         integral_eval_double_grid.  Otherwise an odd M >= 2N - 1 whose
                         factors are 3 and 5: the product of two trigonometric polynomials
                         of Z_N with the series of A on Z_M has no frequency that aliases
                         onto Z_N on such a grid either, so the quadrature stays exact; it
                         serves grids N whose 2N - 1 has other factors (M[2] ignored for
                         d = 2).  Every "doubled grid" below means this grid. */
} hom_desc;

typedef struct {
  int32_t iters;          /* CG iterations performed */
  int32_t status;         /* hom_status of this load */
  double  rel_res_recur;  /* ||r|| / ||E|| from the CG recurrence at exit */
  double  rel_res_true;   /* ||b - C x|| / ||E|| recomputed at exit (FP64 path of the precision mode) */
  double  energy;         /* energy a(E + x, E + x) of the returned field from the CG energy
                             decrements (and, from a given x0, the energy of x0): primal, an upper
                             bound on E^T A_H E; dual, J^T A_H^-1 J is bounded by it. */
} hom_info;

typedef struct {
  double A_up[9];    /* Abar (upper bound), row-major d x d */
  double B_up[9];    /* Bbar (dual energies) */
  double A_low[9];   /* Bbar^{-1} (lower bound) */
  double A_mean[9];  /* (Abar + Bbar^{-1}) / 2 */
  double D[9];       /* (Abar - Bbar^{-1}) / 2, the guaranteed error */
} hom_result;

typedef struct hom_problem hom_problem;

/* Human-readable name of a status code (static string). */
const char* hom_status_str(int32_t status);

/* Number of complex entries of one solution vector (layout above) for the
 * primal (dual = 0) or the dual (dual = 1) problem. */
hom_status hom_field_len(const hom_desc* desc, int32_t dual, size_t* n_complex);

/* Bytes of device workspace hom_setup needs for up to max_loads simultaneous
 * loads (1 <= max_loads <= 3).  Alignment required: 256 bytes. */
hom_status hom_workspace_bytes(const hom_desc* desc, int32_t max_loads, size_t* bytes);

/* Build a problem (Sec. 6, Lemma integral_eval_double_grid, Lemma
 * bounds_for_matrix-inclusion).  Ahat, Bhat: device, complex double
 * (re, im interleaved), ncoef x M0 x M1 (x M2), the Fourier coefficients of A
 * and of A^{-1} on Z_M (M = 2N - 1), frequency n_a stored at n_a mod M_a.
 * The library evaluates the coefficient on the doubled grid,
 * A_M(x^k) = sum_n omega_M^{kn} A_hat(n), in FP64 on the device (plus an
 * FP32 copy for HOM_MIXED), and keeps the Z_N part of A_hat for the
 * right-hand side.  The work is enqueued on the stream without host
 * synchronisation: Ahat/Bhat must stay valid until the stream has passed it
 * (every solve and bounds call synchronises the stream).
 * ws: device workspace of at least hom_workspace_bytes(); it must stay
 * allocated until hom_destroy.  stream: hipStream_t or NULL.
 * On success *out receives a handle (host memory owned by the library). */
hom_status hom_setup(const hom_desc* desc, int32_t max_loads, const void* Ahat, const void* Bhat,
                     void* ws, size_t ws_bytes, void* stream, hom_problem** out);

/* Replace the coefficient of an existing problem (same desc) by new Fourier
 * data, as hom_setup does; keeps the handle, its workspace and any batch or
 * captured graph built on it.  Same lifetime rule for Ahat/Bhat. */
hom_status hom_update_coefficients(hom_problem* pb, const void* Ahat, const void* Bhat);

/* Primal solves (Sec. 7.1, eq. linear_system_primal with the exact form):
 * for each of nload loads E (host, nload x d doubles) find x in E_N with
 * G^E K x = -G^E K E by CG, K the exact Galerkin operator on the doubled
 * grid.  x0: host array of nload device pointers (field layout) or NULL for
 * x0 = 0; an initial guess is symmetrised on the k0 = 0 plane (real field)
 * and is admissible by construction of the layout.  Stopping rule
 * (Convergence-criteria remark, Sec. 7.2): ||r_i|| <= tol ||E||, r the
 * residual in the L2 norm (Parseval).  x_out: host array of nload device
 * pointers, each hom_field_len(primal) complex doubles; may alias x0.
 * info: host array of nload entries.  Returns HOM_NOT_CONVERGED if any load
 * hit maxit (its iterate is still returned), HOM_E_NOT_SPD on breakdown. */
hom_status hom_solve_primal(hom_problem* pb, int32_t nload, const double* E, const double* const* x0,
                            double tol, int32_t maxit, double* const* x_out, hom_info* info);

/* Dual solves (eq. linear_system_dual): G^J K' j = -G^J K' J with K' the
 * exact Galerkin operator of the series of A^{-1}; arguments as above,
 * fields in the dual layout. */
hom_status hom_solve_dual(hom_problem* pb, int32_t nload, const double* J, const double* const* x0,
                          double tol, int32_t maxit, double* const* x_out, hom_info* info);

/* Guaranteed bounds (Def. upper_lower_bounds, eq. approx_homog_with_error):
 * Abar_ab = a(e_b + x^(b), e_a + x^(a)), Bbar_ab = a^-1(e_b + j^(b), e_a + j^(a)),
 * each by the FP64 double-grid quadrature; A_low = Bbar^-1, A_mean, D.
 * primal, dual: host arrays of d device pointers to fields for the unit loads
 * e_1..e_d (any admissible fields give guaranteed bounds).  Either array may
 * be NULL, in which case the corresponding outputs are NaN. */
hom_status hom_bounds(hom_problem* pb, const double* const* primal, const double* const* dual,
                      hom_result* out);

/* Apply the Galerkin operator once: y = T^T G K (T x) (primal, dual = 0) or
 * the dual analogue, in the precision mode of the problem.  x, y: device
 * field vectors.  Used to check the operator against a reference. */
hom_status hom_apply(hom_problem* pb, int32_t dual, const double* x, double* y);

/* Bandwidth probe: copies `bytes` (a multiple of 16) from src to dst (device,
 * 16-byte aligned, not overlapping) reps times after one untimed copy, on
 * `stream`, and returns the rate in GB/s of bytes read plus bytes written
 * (HIP events).  The measured streaming peak beside the published HBM one. */
hom_status hom_probe_copy(const void* src, void* dst, size_t bytes, int32_t reps, void* stream, double* gbs);

/* Dual start from the primal minimisers (Proposition FD_odd_problem (ii), eq.
 * FD_superposition_odd_A, and the remark on avoiding the dual solution): for
 * each dual load J = e_b, with E = Abar^-1 e_b,
 *     J + j0 = A sum_a E_a (e_a + x^(a)),  projected onto J_N,
 * the product taken by the problem's operator (the exact form on the
 * quadrature grid, or the GaNi form in GaNi mode, where the relation is exact
 * for exact GaNi minimisers on odd grids).  primal: host array of d device
 * primal fields for the unit loads e_1..e_d; Abar: host d x d row-major,
 * symmetric with a positive diagonal (the upper bound of those fields, or
 * A_{H,N} in GaNi mode); x0_dual: host array of d device dual fields (outputs,
 * the fluctuations j0 in the dual layout), a valid x0 of hom_solve_dual.
 * Synchronises the stream.  HOM_E_INVALID for null pointers or a non-finite,
 * non-symmetric or singular Abar. */
hom_status hom_dual_start(hom_problem* pb, const double* const* primal, const double* Abar, double* const* x0_dual);

/* Device scratch bytes of the coefficient and sampling helpers below: P NULL
 * gives the size for n_incl inclusions (hom_coef_inclusions,
 * hom_sample_inclusions), P (host, d pixel counts) the size for that image
 * (hom_coef_pixels, hom_sample_pixels), for desc->d and desc->ncoef.
 * HOM_E_INVALID for a bad descriptor, n_incl < 0 or a pixel count outside
 * [1, 65536]. */
hom_status hom_coef_scratch_bytes(const hom_desc* desc, int32_t n_incl, const int32_t* P, size_t* bytes);

/* Device-side Fourier coefficients of a matrix-inclusion medium (eq.
 * A_with_inclusions, Remark inclusion): A_hat(n) = A0 delta_n0 +
 * sum_j (A_j - A0) f_hat_j(n) phi_{-n}(x_j) on Z_M, written in the Ahat layout of
 * hom_setup (ncoef components).  inverse = 1 gives the series of A^{-1}
 * (valid for non-overlapping inclusions: A0^{-1} and A_j^{-1} - A0^{-1}).
 * Host inputs: A0 (d x d), n_incl inclusions with kind[j] (0 box, 1 ball (d = 3)),
 * center[j*d + a], size[j*d + a] (box sides; ball radius in size[j*d]),
 * A_in[j*d*d ...] (coefficient inside, d x d row-major).  out: device.
 * scratch: device, caller-owned, at least hom_coef_scratch_bytes(desc, n_incl,
 * NULL) bytes (HOM_E_WORKSPACE if smaller): it receives the inclusion table.
 * The host inputs are copied into scratch before the call returns (the call
 * waits for the stream's earlier work and that copy); the transform itself
 * runs asynchronously on stream, so scratch must stay allocated until the
 * stream has passed it.  The library allocates no device memory here. */
hom_status hom_coef_inclusions(const hom_desc* desc, const double* A0, int32_t n_incl, const int32_t* kind,
                               const double* center, const double* size, const double* A_in,
                               int32_t inverse, void* out, void* scratch, size_t scratch_bytes, void* stream);

/* hom_coef_inclusions without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments and result as hom_coef_inclusions, without the
 * scratch: the inclusion table goes to a device array of the library, one
 * fixed copy of 53,504 bytes per GPU, held until the process ends, which
 * limits n_incl to 512 (HOM_E_UNSUPPORTED_SIZE above that, before anything is
 * launched).  stream must belong to the current device (HOM_E_INVALID
 * otherwise).  The call synchronises the stream before returning, so calls
 * made one after another from one host thread never overlap; calls that
 * overlap on one GPU (concurrent host threads) race on the shared table and
 * must be serialised by the caller.  No hipMalloc, hipFree or allocating
 * library routine is called; the host table is staged on the stack. */
hom_status hom_coef_inclusions_static(const hom_desc* desc, const double* A0, int32_t n_incl, const int32_t* kind,
                                      const double* center, const double* size, const double* A_in,
                                      int32_t inverse, void* out, void* stream);

/* Device-side Fourier coefficients of a pixel/voxel image (Remark inclusion
 * summed over pixels): pixel i_a along axis a covers
 * [-Y_a/2 + i_a Y_a/P_a, -Y_a/2 + (i_a+1) Y_a/P_a); P_a must have factors 2, 3 and 5
 * only (a P-point transform of the image).
 * phase: host int32 array (P0 x P1 (x P2), row-major) of phase ids;
 * phase_A: host nphase x d x d.  inverse = 1 uses the inverse phase matrices.
 * out: device, Ahat layout of hom_setup.  scratch: device, caller-owned, at
 * least hom_coef_scratch_bytes(desc, 0, P) bytes (the image and its
 * transforms); staging and asynchrony as hom_coef_inclusions. */
hom_status hom_coef_pixels(const hom_desc* desc, const int32_t* P, const int32_t* phase, int32_t nphase,
                           const double* phase_A, int32_t inverse, void* out, void* scratch, size_t scratch_bytes,
                           void* stream);

/* Smallest and largest eigenvalue over nphase symmetric d x d phase
 * matrices (host, row-major): range[0] = a_min, range[1] = a_max (host), the
 * spectrum bounds of the coefficient (Sec. 3: A is uniformly elliptic and
 * bounded, which bounds the spectrum of the Galerkin operators), as taken by
 * hom_problem_set_stop / hom_batch_set_stop.  HOM_E_NOT_SPD if a_min <= 0,
 * HOM_E_INVALID for non-finite entries. */
hom_status hom_phase_eig_range(int32_t d, int32_t nphase, const double* phase_A, double* range);

/* ---- GaNi: Galerkin approximation with numerical integration (Def. GaNi,
 * Lemma FD_of_GaNi) and the paper's Algorithm (Sec. 7.2): the minimisers are
 * computed with the trapezoidal rule on the N grid, whose fully discrete
 * coefficient is the block-diagonal matrix of point values A(x_N^k)
 * (eq. FD_A_GaNi; the dual uses A^-1(x_N^k), eq. FD_inverse_matrix_equality),
 * and step (iii) evaluates the guaranteed bounds of those minimisers exactly
 * (hom_bounds, unchanged).  The GaNi grid G is the problem's N (odd grids) or
 * the even N + 1 (general grids, Sec. 4.4): on an even grid the spaces E_N =
 * G^E_{N,0}[X_N] and J_N drop the Nyquist frequencies, so their fields are the
 * trigonometric polynomials of the reduced set, which is the problem's odd Z_N,
 * and the solve truncates the grid's Nyquist content after each product.  G_a
 * must have factors 2, 3 and 5 only (e.g. the paper's N = 5 3^j or 2^j); the
 * bounds need the quadrature grid of hom_desc.M (any odd 3/5-smooth
 * M >= 2N - 1).
 *
 * Point values on a grid of hom_desc.N points per axis (odd or even here),
 * x_a = Y_a k_a / N_a with -N_a/2 <= k_a < N_a/2 (eqs. grid_points,
 * index_sets), of a matrix-inclusion cell (arguments as hom_coef_inclusions)
 * or of a pixel image (as hom_coef_pixels).  A point belongs to a box iff
 * |x_a - c_a| < h_a / 2 on every axis (<= with closed = 1: the paper's closed
 * square of its even-grid experiment), to a ball iff |x - c| < R, with
 * periodic minimum-image differences: otherwise interfaces belong to the matrix.
 * out: device FP64 [ncoef][N0][N1]([N2]), row-major over the physical axes
 * (2D: [ncoef][N0][N1]); components as hom_desc.ncoef; inverse = 1 gives the
 * values of A^-1.  scratch: device, caller-owned, at least
 * hom_coef_scratch_bytes bytes for these inputs; staging and asynchrony as
 * hom_coef_inclusions. */
hom_status hom_sample_inclusions(const hom_desc* desc, const double* A0, int32_t n_incl, const int32_t* kind,
                                 const double* center, const double* size, const double* A_in, int32_t inverse,
                                 int32_t closed, double* out, void* scratch, size_t scratch_bytes, void* stream);
hom_status hom_sample_pixels(const hom_desc* desc, const int32_t* P, const int32_t* phase, int32_t nphase,
                             const double* phase_A, int32_t inverse, double* out, void* scratch, size_t scratch_bytes,
                             void* stream);

/* The coefficient smoothing filter of the paper's fly-ash example (Sec. 8.3):
 * each value of a 2D characteristic image f (device int32, P[0] x P[1]
 * row-major, values 0 / 1) becomes 4/16 of itself plus 2/16 of each of its
 * four axis neighbours and 1/16 of each of its four diagonal neighbours,
 * periodically.  out (device int32, same shape) receives 16 f_smoothed, exact
 * in integers; a pixel image with the phases k = 0..16 of coefficient
 * A0 + (k/16)(A1 - A0) is the smoothed medium (hom_coef_pixels, hom_sample_pixels).
 * table (host, 17 x d x d, may be NULL) receives those phase matrices from
 * A01 (host, 2 x d x d: A0 then A1; d = 2).  Synchronises the stream. */
hom_status hom_smooth_pixels(const int32_t* P, const int32_t* f, int32_t* out, int32_t d, const double* A01,
                             double* table, void* stream);

/* Device workspace bytes of hom_set_gani for the GaNi grid `grid` (host,
 * d entries, each N_a or N_a + 1; NULL: N), alignment 256. */
hom_status hom_gani_workspace_bytes(const hom_desc* desc, const int32_t* grid, size_t* bytes);

/* Switch later solves and hom_apply of pb to GaNi on the grid `grid` (as
 * above): AN, BN are the point values of A and of A^-1 on that grid (layout
 * of hom_sample_*, device, read during the call).  ws: device workspace of hom_gani_workspace_bytes bytes, kept until
 * hom_clear_gani or hom_destroy (it holds the values, the N-point DFT of the
 * values on the stored half of Z_N, which gives the right-hand side, and
 * twiddles).  The solves then stop and report as before; the energy in
 * hom_info is the GaNi energy.  GaNi solves, hom_apply and hom_dual_start run
 * in FP64 whatever hom_desc.precision says: the exact bounds of a GaNi
 * minimiser (step (iii)) are first order in its algebraic error, because it
 * does not minimise the exact form, so FP32 transforms would enter the bounds
 * at full strength.  Batches reject GaNi problems (HOM_E_INVALID).
 * HOM_E_UNSUPPORTED_SIZE when an N_a has other factors. */
hom_status hom_set_gani(hom_problem* pb, const int32_t* grid, const double* AN, const double* BN, void* ws,
                        size_t ws_bytes);

/* Back to the exact (Ga) operator for later solves. */
hom_status hom_clear_gani(hom_problem* pb);

/* GaNi homogenized matrices A_{H,N}, B_{H,N} (eq. GaNi): the trapezoidal-rule
 * energies of primal and dual fields of the unit loads (host arrays of d
 * device pointers, as hom_bounds), row-major d x d into A_HN and B_HN (host).
 * Either array may be NULL: its matrix is then NaN.
 * For odd grids A_{H,N} = B_{H,N}^-1 at the GaNi minimisers; on even grids
 * B_{H,N}^-1 <= A_{H,N} (Proposition FD_even_problem).  Requires GaNi mode. */
hom_status hom_gani_matrices(hom_problem* pb, const double* const* primal, const double* const* dual,
                             double* A_HN, double* B_HN);

/* Per-kernel timing of one operator application (measurement support).
 * Enqueues `reps` launches of each pass of the operator of the primal
 * (dual = 0) or dual problem with nload loads, in the launch configuration of
 * the solver, bracketing each batch of launches with HIP events on the
 * problem's stream.  ms_out (host, 5 doubles) receives the average duration
 * per launch in milliseconds of: row inverse pass, middle inverse pass (3D,
 * else 0), column pass with the coefficient, middle forward pass (3D, else 0),
 * row forward pass.  The slot's scratch vectors are overwritten. */
hom_status hom_profile_passes(hom_problem* pb, int32_t dual, int32_t nload, int32_t reps, double* ms_out);

/* Release the handle (host memory only; the workspace stays with the caller). */
void hom_destroy(hom_problem* pb);

/* ---- Batched solves.  A batch groups n problems with identical hom_desc and
 * max_loads that were set up on the same stream; every kernel launch of a CG
 * iteration then covers all n problems (one grid slice per problem), and
 * chunks of iterations are replayed from one captured HIP graph.  Each
 * problem keeps its own CG scalars and stopping decision; converged problems
 * skip their work.  The bounds are still computed per problem exactly as in
 * hom_bounds. */
typedef struct hom_batch hom_batch;

/* Device workspace bytes for a batch of n problems (alignment 256). */
hom_status hom_batch_workspace_bytes(int32_t n, size_t* bytes);

/* pbs: host array of n handles (n >= 1), all with the same desc, max_loads
 * and stream, else HOM_E_INVALID.  ws: device workspace of
 * hom_batch_workspace_bytes(n) bytes, kept until hom_batch_destroy.  The
 * problems must outlive the batch. */
hom_status hom_batch_create(hom_problem* const* pbs, int32_t n, void* ws, size_t ws_bytes, hom_batch** out);

/* Lockstep primal (dual = 0) or dual (dual = 1) solves of all problems for
 * the same nload loads E (host, nload x d).  x0: NULL or host array of
 * n * nload device pointers (entries may be NULL); x_out: host array of
 * n * nload device pointers, problem-major; info: host array of n * nload.
 * Same return convention as hom_solve_primal (worst status over the batch). */
hom_status hom_batch_solve(hom_batch* b, int32_t dual, int32_t nload, const double* E, const double* const* x0,
                           double tol, int32_t maxit, double* const* x_out, hom_info* info);

/* Primal and dual solves of the same nload loads for every problem, side by
 * side: the dual runs on a stream of the library (default priority), so the
 * kernels of the two solves share the GPU.  Same results as hom_batch_solve
 * with dual = 0 and dual = 1; x0_primal, x0_dual (each NULL or as x0 there:
 * re-projected starting fields), x_primal, x_dual and the info arrays as
 * there.  Synchronises the caller's stream on entry and both
 * streams on return.  With per-kernel timing on, the two solves advance one
 * chunk of iterations each in turn.  Under the gap rule (stop rule 3) each
 * load of one solve reads the same load of the other at the end of the
 * previous chunk, so the two advance in chunk lockstep (cross-stream waits). */
hom_status hom_batch_solve_pair(hom_batch* b, int32_t nload, const double* E, const double* const* x0_primal,
                                const double* const* x0_dual, double tol, int32_t maxit, double* const* x_primal,
                                double* const* x_dual, hom_info* info_primal, hom_info* info_dual);

/* hom_update_coefficients for every problem of the batch (Ahat[i], Bhat[i]
 * for problem i, same layout and ownership; host arrays of n device
 * pointers), enqueued in one call.  2D problems with equal doubled-grid
 * lengths 25, 81, 125 or 625 are set up together (three launches over all
 * cells, the pointer table in the batch workspace); others cell by cell.
 * The results are bitwise those of per-problem updates. */
hom_status hom_batch_update_coefficients(hom_batch* b, const void* const* Ahat, const void* const* Bhat);

/* Bounds of every problem (as hom_bounds): primal, dual: host arrays of
 * n * d device pointers (problem-major, unit loads e_1..e_d), either may be
 * NULL; out: host array of n results. */
hom_status hom_batch_bounds(hom_batch* b, const double* const* primal, const double* const* dual, hom_result* out);

/* Primal and dual solves of the unit loads e_1..e_d for every problem
 * (eq. linear_system_primal and eq. linear_system_dual, as
 * hom_batch_solve_pair with nload = d and E = I) followed by their guaranteed
 * bounds (Def. upper_lower_bounds, as hom_batch_bounds on the returned
 * fields).  The bound passes of a side are enqueued on its stream as soon as
 * that side has stopped, so they run beside the other side's remaining
 * iterations (without per-kernel timing and outside the gap rule; otherwise
 * after both have stopped).  The fields, infos and results are those of
 * hom_batch_solve_pair followed by hom_batch_bounds.  x0_primal, x0_dual,
 * x_primal, x_dual: as in hom_batch_solve_pair with nload = d; out: host array
 * of n results.  HOM_E_INVALID if the problems hold fewer than d loads.
 * Synchronises as hom_batch_solve_pair; returns its status. */
hom_status hom_batch_solve_bounds(hom_batch* b, const double* const* x0_primal, const double* const* x0_dual,
                                  double tol, int32_t maxit, double* const* x_primal, double* const* x_dual,
                                  hom_info* info_primal, hom_info* info_dual, hom_result* out);

/* As hom_profile_passes, for the launch configuration of the batch (every
 * launch covers all n problems). */
hom_status hom_batch_profile_passes(hom_batch* b, int32_t dual, int32_t nload, int32_t reps, double* ms_out);

/* Per-kernel timing of the CG iterations of later hom_batch_solve calls
 * (measurement support): with on = 1 the iterations are launched directly
 * (not from the captured graph, whose event records cannot be timed) with a
 * HIP event recorded around every kernel on the problem stream, and the
 * elapsed times are accumulated per pass type (same five types as
 * hom_profile_passes).  Turning it on or off resets the accumulators. */
hom_status hom_batch_set_timing(hom_batch* b, int32_t on);
/* ms_sum[5]: accumulated milliseconds; launches[5]: number of launches. */
hom_status hom_batch_get_timing(hom_batch* b, double* ms_sum, int64_t* launches);

void hom_batch_destroy(hom_batch* b);

/* ---- groups: several batches (size classes, e.g. of a mixed batch of uneven
 * N and d) solved together.  hom_group_solve_pair runs the primal and dual
 * solves of the unit loads e_1..e_d of every problem of every batch with one
 * captured HIP graph: a fork on the first batch's stream, one branch per solve
 * on the batch's own stream (primal) and library stream (dual), a join.  One
 * hipGraphLaunch advances every solve of every batch by one chunk of
 * iterations, and the host reads the active counts once per chunk (one chunk
 * in flight); finished units return at once.  Results equal those of
 * hom_batch_solve_pair on each batch (same kernels, same reduction order).
 * The graph is captured on the first call and again when a batch's tile
 * shapes change.  batches: host array of n distinct batch handles (no GaNi
 * problems), which must outlive the group. */
typedef struct hom_group hom_group;
hom_status hom_group_create(hom_batch* const* batches, int32_t n, hom_group** out);

/* x_primal, x_dual: host arrays of device field pointers, batch-major, then
 * problem, then load (d_b loads for batch b, d_b its dimension); info_primal,
 * info_dual: host arrays of the same length.  Stopping rule and tile shapes
 * are each batch's own (hom_batch_set_stop, hom_batch_set_tiles).  Waits for
 * the work already on every batch's stream, synchronises every stream before
 * returning; with per-kernel timing on in any batch, the solves advance one
 * chunk each in turn without graphs.  Returns the worst status over the group
 * (as hom_solve_primal). */
hom_status hom_group_solve_pair(hom_group* g, double tol, int32_t maxit, double* const* x_primal,
                                double* const* x_dual, hom_info* info_primal, hom_info* info_dual);
/* hom_group_solve_pair followed by the guaranteed bounds of every problem
 * (Def. upper_lower_bounds, as hom_batch_bounds on each batch's returned
 * fields), in one call.  In launch mode 1 the bound passes of a solve are
 * enqueued on its stream as soon as it has stopped (outside the gap rule),
 * beside the solves still iterating; otherwise after all have stopped.  Same
 * fields, infos and results as the two calls.  out: host array of the total
 * problem count, batch-major. */
hom_status hom_group_solve_bounds(hom_group* g, double tol, int32_t maxit, double* const* x_primal,
                                  double* const* x_dual, hom_info* info_primal, hom_info* info_dual,
                                  hom_result* out);
/* Launch mode of later hom_group_solve_pair calls: 0 (default) one captured
 * graph advances every solve by a chunk per launch, as above; 1 each solve
 * replays its own captured chunk graph on its own stream and one host loop
 * polls them all, so that no solve waits for the chunks of another batch (the
 * primal and dual of a batch still advance in chunk lockstep under the gap
 * rule).  Results are the same in both modes.  HOM_E_INVALID for other modes. */
hom_status hom_group_set_launch(hom_group* g, int32_t mode);
void hom_group_destroy(hom_group* g);

/* ---- Tile tuning of the FP32 passes.
 * The specialised FP32 kernels (doubled-grid lengths 25, 81, 125, 625) have
 * several tile shapes: row pairs and threads per block of the row passes,
 * points per block, the LDS exchange width and the packs per block of the
 * column pass.  With tuning on (the default; the
 * environment variable HOM_TUNE=0 turns it off at start-up), the first
 * mixed-precision solve of a geometry (grid, loads, primal/dual, coefficient
 * components) in the process times every candidate on that solve's own units,
 * with zero step lengths on scratch vectors, and keeps the fastest for every
 * later solve of the geometry, single or batched.  The shape changes the
 * blocking of the CG reductions, hence rounding in the last bits; within a
 * process all solves of a geometry use one shape.  Off: fixed defaults. */
typedef struct {
  int32_t row_pairs;     /* row pairs per block of the row passes (0: generic passes) */
  int32_t row_threads;   /* threads per row block (0: the smallest that covers the FFT) */
  int32_t apply_points;  /* points per column-pass block (0: default) */
  int32_t apply_half_exchange; /* 1: the column pass exchanges real and imaginary parts in turn */
  int32_t apply_all_packs; /* 1: a column-pass block holds every pack of its points (2D) */
  int32_t candidates;    /* configurations timed (0: defaults, not tuned) */
  double row_ms;         /* measured time of one row-pass pair (first + last), ms */
  double apply_ms;       /* measured time of one column pass, ms */
} hom_tuning;

/* Stopping rule of later solves.  The Convergence-criteria remark (Sec. 7.2)
 * picks a residual tolerance small enough that the algebraic error stays
 * below the discretisation error; rules 1 and 2 measure the algebraic error
 * of the bounds themselves, so a solve can stop once it is small beside the
 * guaranteed error D (eq. GaNi_error) or a requested accuracy.  Each
 * CG step lowers the energy a(E + x, E + x) of the iterate by alpha gamma, so
 * the energy of every iterate, the primal upper bound on E^T A_H E (dual: the
 * bound on J^T A_H^-1 J), is known from the recurrence.
 *   rule 0 (default): the residual rule of the Convergence-criteria remark,
 *     ||r|| <= tol ||E|| with the tol of each solve call.
 *   rule 1: rule 0 or, whichever holds first, a heuristic energy rule: the
 *     remaining decrease, extrapolated from the last four decrements as a
 *     geometric tail with a factor 2 of margin, is below etol times the
 *     current energy.  Irregular convergence can end it early.
 *   rule 2: rule 0 or a guaranteed energy rule: the Gauss-Radau upper bound
 *     on the remaining decrease (from a lower bound mu on the spectrum of the
 *     operator) is below etol times the current energy, so the returned
 *     energy exceeds the converged one by at most a relative etol / (1 - etol)
 *     (in exact arithmetic; FP32 operators add their own rounding).  mu is the
 *     larger of the smallest eigenvalue of the coefficient over the doubled
 *     grid (the operator's quadratic form is a mean over those points) and
 *     a_min (dual: 1 / a_max) when the caller gives one (> 0); a caller's
 *     value must bound the coefficient's eigenvalues, or the guarantee is lost.
 *   rule 3: rule 0 or the gap rule, relative to the discretisation error
 *     (Convergence-criteria remark of Sec. 7.2; eq. approx_homog_with_error):
 *     for a load E the primal energy U bounds E.A_H E from above and
 *     |E|^4 / V, V the dual energy for J = E, from below; with the
 *     Gauss-Radau bounds R (on U - U*) and R' = |E|^4 R_V / (V (V - R_V)) (on
 *     L* - L, infinite unless V > R_V, mu as in rule 2), the converged gap
 *     D* = U* - L* of the entry is at least (U - R) - (L + R'), and each side
 *     stops when its own bound is at most etol (theta) times that, so that its
 *     algebraic error is below theta D*.  The partner's state is the one at
 *     the last iterate of the previous chunk of iterations (start energy,
 *     infinite bound, during the first).  Only the side-by-side solves
 *     (hom_batch_solve_pair, hom_group_solve_pair) run it; other solves
 *     return HOM_E_INVALID under rule 3.
 * 0 < etol < 1 for rules 1 to 3; a_min, a_max >= 0 (0: not given).  Every
 * iterate is admissible, so the bounds stay guaranteed under every rule.
 * HOM_E_INVALID for other values. */
hom_status hom_problem_set_stop(hom_problem* pb, int32_t rule, double etol, double a_min, double a_max);
hom_status hom_batch_set_stop(hom_batch* b, int32_t rule, double etol, double a_min, double a_max);

/* mode 1: tune geometries not seen yet; 0: defaults for geometries not seen
 * yet.  Choices already made stay in use.  HOM_E_INVALID for other modes. */
hom_status hom_set_tuning(int32_t mode);
/* Tile shapes the solves of (dual, nload) use; tunes now when no solve of
 * this problem / batch has chosen them yet. */
hom_status hom_problem_tuning(hom_problem* pb, int32_t dual, int32_t nload, hom_tuning* out);
hom_status hom_batch_tuning(hom_batch* b, int32_t dual, int32_t nload, hom_tuning* out);
/* The tuner's choices on disk, so that later processes skip the timing.  One
 * JSON object per line: the device architecture (gcnArchName up to its first
 * ':'), the geometry key (doubled grid M0 M1 M2 on internal axes, d, loads,
 * dual, coefficient components, packs) and the shape with its measured
 * times; shapes are shared by every batch size of a geometry, so that batches
 * and single solves run the same kernels.  hom_tune_cache_load merges the
 * entries of `arch` (NULL: the current device's) into the process cache
 * (*loaded, may be NULL: their count; HOM_E_INVALID for an unreadable file or
 * a line that does not parse, entries read before it stay); hom_tune_cache_save
 * writes the whole process cache tagged with `arch` (replacing the file);
 * hom_tune_cache_clear empties the process cache.  With the environment
 * variable HOM_TUNE_CACHE set to a path, the first tuning of the process
 * loads that file and every new choice rewrites it.  HOM_E_DEVICE when arch
 * is NULL and no device is present. */
hom_status hom_tune_cache_load(const char* path, const char* arch, int32_t* loaded);
hom_status hom_tune_cache_save(const char* path, const char* arch);
hom_status hom_tune_cache_clear(void);

/* Pin the tile shape of the solves of (dual, nload): row_pairs, row_threads,
 * apply_points, apply_half_exchange and apply_all_packs of *t (all 0 =
 * default; the timing fields are ignored).  For bitwise-reproducible results
 * across processes, or to compare shapes.  Mixed precision only;
 * HOM_E_INVALID for a shape the specialised kernels do not have.
 * Synchronises the problem's stream. */
hom_status hom_problem_set_tiles(hom_problem* pb, int32_t dual, int32_t nload, const hom_tuning* t);
hom_status hom_batch_set_tiles(hom_batch* b, int32_t dual, int32_t nload, const hom_tuning* t);

/* ---- Learned initial guess (measurement-independent helper of the solver).
 * Fields on the doubled grid M = 2N - 1, real FP32, [nload][d][M0][M1](M2):
 * component g of the fluctuation field of load l. */

/* Values on the doubled grid of nload field vectors (primal dual = 0 or dual
 * dual = 1 layout): u_l = F_M^-1 pad_M(T c_l) (eq. trig_connection), FP64
 * arithmetic, written as FP32.  fields: host array of nload device pointers;
 * out: device. */
hom_status hom_field_to_grid(hom_problem* pb, int32_t dual, int32_t nload, const double* const* fields,
                             float* out);

/* Admissible field vectors from arbitrary real fields on the doubled grid:
 * c_l = T(k)^T [F_M u_l](k) for k in Z_N (truncation P_N and projection on
 * E_N or J_N, Def. projection), FP64 arithmetic.  in: device [nload][d][M^d];
 * out: host array of nload device pointers (field layout). */
hom_status hom_grid_to_field(hom_problem* pb, int32_t dual, int32_t nload, const float* in, double* const* out);

/* Network input channels of a problem on the doubled grid, FP32 [2][M^d]:
 * a(x)/<a> and log(max(a(x), 1e-3 <a>)/<a>), with a = trace(A_M)/d the
 * coefficient on the doubled grid and <a> its mean.  out: device. */
hom_status hom_net_input(hom_problem* pb, float* out);

/* The three transfers above for every problem of a batch at once (one launch
 * per pass covers all cells), on the batch's stream.  Cell i's grid block
 * starts at in / out + i * stride floats (stride >= nload d M^d, or 2 M^d
 * for the network inputs, so that a cell's block may sit inside a larger
 * sample record); fields / out: host arrays of n * nload device pointers,
 * problem-major.  hom_batch_field_to_grid and hom_batch_grid_to_field
 * synchronise the stream (their unit table is reused); hom_batch_net_input
 * writes the input channels (weights = 0) or the energy weights (weights = 1)
 * of every cell and returns without synchronising. */
hom_status hom_batch_field_to_grid(hom_batch* b, int32_t dual, int32_t nload, const double* const* fields, float* out,
                                   size_t stride);
hom_status hom_batch_grid_to_field(hom_batch* b, int32_t dual, int32_t nload, const float* in, size_t stride,
                                   double* const* out);
hom_status hom_batch_net_input(hom_batch* b, float* out, size_t stride, int32_t weights);

/* Pointwise energy weights on the doubled grid, FP32 [2][M^d]: channel 0
 * max(a, 1e-3 <a>)/<a> for a = trace(A_M)/d (primal), channel 1 the same for
 * b = trace((A^-1)_M)/d (dual): the weights of the double-grid quadrature of
 * the energies (Lemma integral_eval_double_grid), kept positive.  out: device. */
hom_status hom_net_weights(hom_problem* pb, float* out);

/* U-Net surrogate (FP32, hand-written kernels): levels (1..6), base width
 * (1..256), input and output channels, spatial size (2D: H, W; 3D: Z, H, W;
 * each at least 2, at most 2^24 points in all) and batch.  Other values:
 * HOM_E_INVALID. */
typedef struct {
  int32_t d;
  int32_t levels;
  int32_t base;
  int32_t cin;
  int32_t cout;
  int32_t size[3];
  int32_t batch;
} hom_unet_desc;

typedef struct hom_unet hom_unet;

/* Number of parameters and bytes of device work memory (activations,
 * gradients, scratch) of a network. */
hom_status hom_unet_sizes(const hom_unet_desc* desc, size_t* n_params, size_t* work_bytes);
/* params, grads, adam_m, adam_v: device FP32 arrays of n_params each (caller
 * owned; params initialised by the caller).  work: device, 256-byte aligned. */
hom_status hom_unet_create(const hom_unet_desc* desc, float* params, float* grads, float* adam_m, float* adam_v,
                           void* work, size_t work_bytes, void* stream, hom_unet** out);
/* in: device [batch][cin][size]; out: device [batch][cout][size] or NULL.
 * With a stream the forward kernels are captured into a HIP graph on the
 * first call and replayed after (the input is copied into the network's own
 * buffer first, so the graph serves every input). */
hom_status hom_unet_forward(hom_unet* u, const float* in, float* out);
/* The same with the batch's samples gathered from `batch` device pointers
 * (host array), each [cin][size]: a minibatch of stored samples without a
 * separate gather. */
hom_status hom_unet_forward_samples(hom_unet* u, const float* const* in, float* out);
/* Mean squared error of the last forward output against target (device); sets
 * the output gradient; *loss on the host (synchronises the stream). */
hom_status hom_unet_loss(hom_unet* u, const float* target, double* loss);
/* Weighted mean squared error: sum_i w_i (out_i - target_i)^2 / n, output
 * channel c taking weight channel c * wch / cout of weight [batch][wch][size]
 * (device; cout must be a multiple of wch, 1 <= wch <= cout; NULL = unit
 * weights).  Used with the coefficient as weight to approximate the energy
 * norm of the field error. */
hom_status hom_unet_loss_weighted(hom_unet* u, const float* target, const float* weight, int32_t wch,
                                  double* loss);
/* hom_unet_loss_weighted with the targets ([cout][size] each) and the weights
 * ([wch][size] each, or NULL) gathered from `batch` device pointers (host arrays). */
hom_status hom_unet_loss_samples(hom_unet* u, const float* const* target, const float* const* weight, int32_t wch,
                                 double* loss);
/* Parameter gradients of the last forward pass for the output gradient gout
 * (device) or, when gout is NULL, the gradient set by hom_unet_loss. */
hom_status hom_unet_backward(hom_unet* u, const float* gout);
/* One Adam step (step >= 1 is the 1-based step count for bias correction). */
hom_status hom_unet_adam(hom_unet* u, float lr, float beta1, float beta2, float eps, int32_t step);
void hom_unet_destroy(hom_unet* u);

#ifdef __cplusplus
}
#endif
#endif /* HOM_H */
