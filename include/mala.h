/*
 * mala.h -- C ABI of the MI355X (gfx950) grid-inference library.
 *
 * The library computes, for every point of a real-space grid around a
 * periodic atomic snapshot, the path of the MALA method (arXiv:2411.19617):
 *   bispectrum descriptors B(r, j)                 (Sec. 3.2.2, Eqs. ionicdensity,
 *                                                   SNAPExpansion, snap_dim)
 *   -> feed-forward network to the LDOS d(r, e)     (Sec. 2.4, Eq. ffnn)
 *   -> DOS D(e) = integral of d over space          (Sec. 2.3, Eq. DOS.from.ldos)
 *   -> Fermi level from N_e = int f D               (Sec. 3.4, Eq. NumberElectrons_from_DOS)
 *   -> band energy E_b = int f e D                  (Sec. 2.3, Eq. band.energy)
 *   -> density n(r) = int f d                       (Sec. 2.3, Eq. density.from.ldos)
 * with the energy integrals done exactly for a piecewise-linear D through
 * Fermi-Dirac weights (Sec. 3.4, Eqs. ldosintegralsummation, fermidiracspecial).
 *
 * Conventions shared by every call
 *  - Units: Angstrom, eV, Kelvin; k_B = 8.617333262e-5 eV/K.  LDOS in
 *    1/(eV A^3), DOS in 1/eV, density in 1/A^3.
 *  - Cell: orthorhombic, edges L[3]; grid N[3]; point (i,j,k) sits at
 *    (i Lx/Nx, j Ly/Ny, k Lz/Nz) and has flat index p = (i*Ny + j)*Nz + k.
 *  - Descriptor order: for j1 = 0..twojmax, j2 = 0..j1, j = j1-j2 .. min(twojmax,
 *    j1+j2) step 2, keep j >= j1 (all doubled); n_B = mala_n_descriptors(twojmax).
 *  - Neighbours: every periodic image within rcut; cosine cutoff
 *    f_c = (cos(pi r/rcut)+1)/2; theta0 = 0.99363 pi r/rcut; self weight 1.
 *  - Buffers named "device" are device pointers (hipMalloc'd or torch CUDA
 *    tensors) owned by the caller; "host" pointers are ordinary host memory
 *    that is read before the call returns.  The library owns contexts and
 *    weights and the scratch memory inside a context.
 *  - Every compute call is asynchronous on the context's stream; outputs are
 *    valid after the stream has been synchronised.  Calls on one context
 *    must not overlap (they share its scratch).
 *  - Errors: a negative status; mala_last_error() gives a message for the
 *    calling thread.  Nothing is thrown across the ABI.  Argument errors are
 *    detected before any work is enqueued.  Capacity overflows found on the
 *    device (too many neighbours of one point) are reported by the next
 *    call of mala_check_device_errors().
 */
#ifndef MALA_H
#define MALA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mala_status;
#define MALA_OK 0
#define MALA_E_INVALID_ARG (-1)  /* bad pointer, size, or parameter            */
#define MALA_E_UNSUPPORTED (-2)  /* valid but not supported by the library (e.g. twojmax) */
#define MALA_E_OOM (-3)          /* device allocation failed                   */
#define MALA_E_NO_ROOT (-4)      /* N_e outside [N(e_0), N(e_last)]            */
#define MALA_E_HIP (-5)          /* a HIP runtime call failed                  */
#define MALA_E_BUSY (-6)         /* serving: result not ready yet              */
#define MALA_E_CAPACITY (-7)     /* a fixed per-tile capacity was exceeded      */

#define MALA_PREC_FP32 0         /* network in FP32 on MFMA                    */
#define MALA_PREC_BF16 1         /* network in BF16 on MFMA, FP32 accumulate    */

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* mala_last_error(void);
const char* mala_version(void);

/* Number of bispectrum components for twojmax (Eq. snap_dim with J_max =
 * twojmax/2): (twojmax+2)(twojmax+3)(twojmax+4)/24.  -1 if twojmax < 0.     */
int32_t mala_n_descriptors(int32_t twojmax);

/* ---------------------------------------------------------------- context */
typedef struct mala_ctx mala_ctx;

/* Create a context on HIP device `device`, enqueueing on `stream` (a
 * hipStream_t; NULL = the legacy default stream).  *out receives the handle. */
mala_status mala_create(int32_t device, void* stream, mala_ctx** out);
mala_status mala_destroy(mala_ctx* ctx);
mala_status mala_set_stream(mala_ctx* ctx, void* stream);
/* Blocks until the context's stream is idle. */
mala_status mala_synchronize(mala_ctx* ctx);
/* Synchronises, then returns MALA_E_CAPACITY if any kernel since the last
 * check flagged a capacity overflow (and clears the flag), else MALA_OK.    */
mala_status mala_check_device_errors(mala_ctx* ctx);

/* ---------------------------------------------------------------- weights
 * Weights blob (little endian, as written by the input generator):
 *   char     magic[8] = "MALANET1"
 *   int32    version (=1), n_layers, output_activation (1 = activation also on
 *            the output layer, as in Eq. ffnn; 0 = identity), reserved
 *   float64  leaky_slope                 (LeakyReLU negative slope)
 *   int32    widths[n_layers+1], padded with one int32 if n_layers+1 is odd
 *   float64  in_mean[w0], in_std[w0]     (x0 = (B - mean)/std)
 *   per layer l: float64 W[w(l+1)][w(l)] row-major, float64 b[w(l+1)]
 *   float64  out_scale[wL], out_shift[wL] (LDOS = out_scale*y + out_shift)
 *   uint64   seed
 * The library supports n_layers = 3, w0 <= 128, hidden widths <= 512 and
 * wL <= 256.  The blob is copied; the caller may free it after the call.
 * Weights live on the context's device but do not depend on the context
 * afterwards; mala_weights_free synchronises that device before freeing.    */
typedef struct mala_weights mala_weights;
mala_status mala_weights_load(mala_ctx* ctx, const void* blob, size_t bytes,
                              int32_t precision, mala_weights** out);
mala_status mala_weights_free(mala_weights* w);

typedef struct {
    double L[3];      /* orthorhombic cell edges, Angstrom */
    int32_t N[3];     /* grid points per edge              */
} mala_cell_grid;

typedef struct {
    double e0;        /* first energy, eV   */
    double de;        /* spacing, eV (> 0)  */
    int32_t n;        /* number of energies */
} mala_egrid;

/* Device-resident result record written by mala_integrate / mala_predict. */
typedef struct {
    double e_fermi;       /* eV                                   */
    double e_band;        /* eV (total; divide by N_atoms for per-atom) */
    double n_found;       /* N(E_F) from the weights              */
    double n_target;      /* requested N_e                        */
    int32_t iterations;   /* root-finder steps (Newton or bisection) */
    int32_t status;       /* MALA_OK or MALA_E_NO_ROOT            */
    int32_t density_from_window; /* mala_predict: 1 if the density came from
                                    the stored energy window, 0 otherwise */
    int32_t reserved;
    double entropy;       /* S_s / k_B (Eq. electronicentropyDOS):
                             int -[f ln f + (1-f) ln(1-f)] D de       */
    double e_entropy;     /* -tau S_s in eV, the entropy term of the
                             free energy (Eq. KSfreeenergy)           */
} mala_result;

/* ---------------------------------------------------------------- compute */

/* Bispectrum descriptors (Sec. 3.2.2) of grid points [pt_begin, pt_end).
 *  positions: host float64 [n_atoms][3] (any values; wrapped into the cell)
 *  rcut > 0; twojmax in {2, 4, 6, 8, 10}
 *  B_out: device float32 [pt_end - pt_begin][n_B], row = point.
 * Empty ranges are a no-op.                                                  */
mala_status mala_descriptors(mala_ctx* ctx, const double* positions, int32_t n_atoms,
                             const mala_cell_grid* cg, double rcut, int32_t twojmax,
                             int64_t pt_begin, int64_t pt_end, float* B_out);

/* Vector-Jacobian product of the descriptors: the descriptor factor of the
 * force expression (Eq. forcesmala) applied to weights gB over the
 * components, i.e. the gradient of L = sum_p sum_l gB[p][l] B_l(p) over the
 * grid points p in [pt_begin, pt_end) with respect to every atom position
 * (the force contribution is its negative):
 *   dLdR_out[a][d] = dL / dR_{a,d}, summed over every periodic image.
 *  positions, cg, rcut, twojmax as for mala_descriptors;
 *  gB: device float32 [pt_end - pt_begin][n_B] (row = point);
 *  dLdR_out: device float64 [n_atoms][3] (caller-owned), overwritten.
 * An atom sitting exactly on a grid point is left out of that point's
 * gradient (the descriptors have no derivative there).  The per-atom sums
 * are FP64 atomic additions whose order is not fixed, so repeated calls can
 * differ in the last bits.  An empty range writes zeros.  Capacity overflows
 * are reported by mala_check_device_errors as for mala_descriptors.        */
mala_status mala_descriptors_vjp(mala_ctx* ctx, const double* positions, int32_t n_atoms,
                                 const mala_cell_grid* cg, double rcut, int32_t twojmax,
                                 int64_t pt_begin, int64_t pt_end, const float* gB, double* dLdR_out);

/* Grid-centred atomic cluster expansion descriptors (Sec. 3.2.3, Eqs.
 * unweighted_ionicdensity, gridatom_basis, grid_base, product_grid_basis,
 * ace_grid) of grid points [pt_begin, pt_end), one chemical element:
 *   A_nlm = R_n(0) Y_0^0 delta_l0 + sum over atom images within rcut of
 *           R_n(r) Y_l^m(d/r),  R_n(r) = T_n(2 r / rcut - 1) fc(r)
 *   (Chebyshev polynomials, cosine cutoff, orthonormal complex spherical
 *   harmonics with the Condon-Shortley phase, n < nmax, l <= lmax);
 *   rank 1: A_n00 for n < nmax;
 *   rank 2: sum_m (-1)^m A_{n1 l m} A_{n2 l -m} for l = 0..lmax, n1 <= n2;
 *   rank 3: sum (l1 l2 l3; m1 m2 m3) A_{n1 l1 m1} A_{n2 l2 m2} A_{n3 l3 m3}
 *   (Wigner 3j) over multisets of three (n, l) pairs in the order of the key
 *   p = n (lmax+1) + l, p1 <= p2 <= p3, with l1+l2+l3 even and triangle.
 *  nmax in 1..4, lmax in 0..4 (MALA_E_UNSUPPORTED otherwise); positions,
 *  cg, rcut as for mala_descriptors;
 *  layout MALA_LAYOUT_POINT_MAJOR: out is device float32
 *  [pt_end - pt_begin][mala_ace_count(nmax, lmax)]; MALA_LAYOUT_DESCRIPTOR_MAJOR:
 *  [mala_ace_count(nmax, lmax)][pt_end - pt_begin] (one plane per descriptor,
 *  written with coalesced stores: faster when the consumer can take planes).
 * Empty ranges are a no-op.                                                  */
#define MALA_LAYOUT_POINT_MAJOR 0
#define MALA_LAYOUT_DESCRIPTOR_MAJOR 1
int32_t mala_ace_count(int32_t nmax, int32_t lmax);   /* descriptors per point, or < 0 */
mala_status mala_ace_descriptors(mala_ctx* ctx, const double* positions, int32_t n_atoms,
                                 const mala_cell_grid* cg, double rcut, int32_t nmax, int32_t lmax,
                                 int64_t pt_begin, int64_t pt_end, int32_t layout, float* out);

/* Grid ACE descriptors of rank 4 (Sec. 3.2.3, Eq. ace_grid with four
 * factors and one intermediate coupling L, the generalized Clebsch-Gordan
 * coefficient of the coupling tree ((l1 l2) L, (l3 l4) L) -> 0):
 *   B = sum_m <l1 m1 l2 m2|L M> <l3 m3 l4 m4|L -M> (-1)^(L-M)/sqrt(2L+1)
 *       A_{n1 l1 m1} A_{n2 l2 m2} A_{n3 l3 m3} A_{n4 l4 m4},  M = m1 + m2,
 * with A, the radial basis and the self term as for mala_ace_descriptors.
 * The set: for keys p = n (lmax4+1) + l (n < nmax4, l <= lmax4), every
 * multiset p1 <= p2 <= p3 <= p4 with an even l-sum and, for it, the
 * couplings L in increasing order whose coefficients (summed over the
 * permutations that exchange equal keys) are linearly independent of those
 * kept before: the non-redundant rank-4 descriptors the paper requires.
 *  nmax4 in 1..3, lmax4 in 0..3 (MALA_E_UNSUPPORTED otherwise);
 *  out: device float32 [pt_end - pt_begin][mala_ace4_count(nmax4, lmax4)]
 *  (MALA_LAYOUT_POINT_MAJOR) or its transpose (MALA_LAYOUT_DESCRIPTOR_MAJOR),
 *  descriptors in the order of mala_ace4_list.
 * Point-major output goes through descriptor planes of 65,536-point chunks
 * in a context buffer (65,536 x count floats, 246 MB at nmax4 = lmax4 = 3).
 * mala_ace4_list writes (p1, p2, p3, p4, L) per descriptor into out[5 n]
 * (host int32, cap entries of five) and returns the count, or < 0 if the
 * sizes are unsupported or cap is too small.  Empty ranges are a no-op.    */
int32_t mala_ace4_count(int32_t nmax4, int32_t lmax4);
int32_t mala_ace4_list(int32_t nmax4, int32_t lmax4, int32_t* out, int32_t cap);
mala_status mala_ace4_descriptors(mala_ctx* ctx, const double* positions, int32_t n_atoms,
                                  const mala_cell_grid* cg, double rcut, int32_t nmax4, int32_t lmax4,
                                  int64_t pt_begin, int64_t pt_end, int32_t layout, float* out);

/* Gaussian descriptors of grid points [pt_begin, pt_end): the Gaussian
 * representation of the ionic positions behind the structure factor
 * (Eq. structurefactor_gaussian), a Gaussian of width sigma normalised to
 * unit integral on every atom and periodic image within the cutoff:
 *   G(r) = (2 pi sigma^2)^(-3/2) sum_{|r-R| < cutoff} exp(-|r-R|^2 / (2 sigma^2)).
 *  positions: host float64 [n_atoms][3]; cg as for mala_descriptors;
 *  sigma > 0 and cutoff > 0 in Angstrom (cutoff = 8 sigma leaves e^-32 of
 *  each Gaussian out); G_out: device float32 [pt_end - pt_begin].
 * Empty ranges are a no-op.  More than 1024 atom images near one 64-point
 * tile is reported by mala_check_device_errors (MALA_E_CAPACITY).          */
mala_status mala_gaussian_descriptors(mala_ctx* ctx, const double* positions, int32_t n_atoms,
                                      const mala_cell_grid* cg, double sigma, double cutoff,
                                      int64_t pt_begin, int64_t pt_end, float* G_out);

/* LDOS of n_pts points through the network (Eq. ffnn) and the output
 * transform.  B: device float32 [n_pts][w0]; ldos_out: device float32
 * [n_pts][wL].                                                                */
mala_status mala_ldos_infer(mala_ctx* ctx, const mala_weights* w, const float* B,
                            int64_t n_pts, float* ldos_out);

/* Vector-Jacobian product of the network: the network factor of the force
 * expression (Eq. forcesmala) applied to a vector over the energies,
 *   g(p) = (dd(p)/dB(p))^T v(p),  d = LDOS of mala_ldos_infer,
 * by backpropagation (sigma'(z) = 1 for z > 0, slope otherwise; the network
 * is piecewise linear and g jumps where a unit crosses its kink).
 *  B: device float32 [n_pts][w0]; v: device float32 [n_pts][wL];
 *  g_out: device float32 [n_pts][w0] (caller-owned).
 * FP32 weights only (MALA_E_UNSUPPORTED for BF16 weights: rounding there
 * moves units across their kinks often enough to change g by percent).
 * n_pts = 0 is a no-op.                                                      */
mala_status mala_ldos_vjp(mala_ctx* ctx, const mala_weights* w, const float* B, const float* v,
                          int64_t n_pts, float* g_out);

/* Observables from a stored LDOS (Sec. 3.4): DOS, Fermi level, band
 * energy, electronic entropy (Eq. electronicentropyDOS) and density.
 *  ldos: device float32 [n_pts][eg->n]; dV = cell volume / N_points;
 *  T_kelvin > 0; n_electrons > 0.
 *  dos_out: device float64 [eg->n]; density_out: device float64 [n_pts] or
 *  NULL; result: device mala_result.  If N_e has no root, result->status is
 *  MALA_E_NO_ROOT, E_F/E_b/entropy are NaN and the density is not written. */
mala_status mala_integrate(mala_ctx* ctx, const float* ldos, int64_t n_pts, double dV,
                           const mala_egrid* eg, double T_kelvin, double n_electrons,
                           double* dos_out, double* density_out, mala_result* result);

/* mala_integrate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, kernels and results (bit for bit) as mala_integrate, but
 * its scratch (2048 FP64 partial rows of 256 energies plus 256 FP64 weights,
 * 4 MiB + 2 KiB) is a fixed device array of the library, one per GPU, held
 * until the process ends and looked up once per device by mala_create.  It
 * calls no hipMalloc/hipFree and records no profiling events.  Every n_pts
 * fits (points are split over at most 2048 partial rows); eg->n above 256 is
 * rejected (MALA_E_UNSUPPORTED) as in mala_integrate.  All calls on one GPU
 * share that scratch: calls that overlap on one GPU (different streams or
 * contexts without ordering between them) race and give wrong results.     */
mala_status mala_integrate_noalloc(mala_ctx* ctx, const float* ldos, int64_t n_pts, double dV,
                                   const mala_egrid* eg, double T_kelvin, double n_electrons,
                                   double* dos_out, double* density_out, mala_result* result);

/* Whole path, fused: descriptors of every grid point (cached as B in
 * device memory), network with the DOS reduced in the epilogue (the full
 * LDOS is never stored), Fermi level, band energy, entropy and density.
 * The density needs E_F, which needs every point.  In the default mode a
 * network pass over every 61st point first estimates E_F; the main pass then
 * keeps per point only the FP64 sum of the fully occupied part below the
 * window and the LDOS inside the window E_est +- (40 kT + 0.3 eV); once E_F
 * is solved, the density is finished from those.  If the window does not
 * contain E_F +- 40 kT, a second network pass recomputes the density
 * (decided on the device, no host round trip).
 *  result->status is MALA_E_CAPACITY (and the density is not written) when
 *  the context's capacity flags are set: a fixed neighbour capacity was
 *  exceeded by this call's descriptors or by an earlier call since the last
 *  mala_check_device_errors (which reports and clears them).
 *  B_cache: device float32 [N_points][n_B] or NULL (then context scratch).
 *  Outputs as in mala_integrate; density_out may be NULL.                   */
mala_status mala_predict(mala_ctx* ctx, const mala_weights* w, const double* positions,
                         int32_t n_atoms, const mala_cell_grid* cg, double rcut,
                         int32_t twojmax, const mala_egrid* eg, double T_kelvin,
                         double n_electrons, double* dos_out, double* density_out,
                         mala_result* result, float* B_cache);

/* How mala_predict obtains the density: from the stored energy window with
 * recompute as fallback (default), or always by the recompute pass.         */
#define MALA_DENSITY_WINDOW 0
#define MALA_DENSITY_RECOMPUTE 1
mala_status mala_set_density_mode(mala_ctx* ctx, int32_t mode);

/* ---------------------------------------------------------------- serving
 * A request loop for streams of snapshots of different sizes (MD-trajectory
 * style use of the method).  The server owns the weights and max_inflight
 * slots; each slot is a context with its own HIP stream and device state, so
 * the work of requests in different slots overlaps on the device.  Requests
 * are admitted strictly in arrival order whenever a slot is free and the
 * device memory held by all slots plus what the request needs stays within
 * hbm_budget (idle slots release cached buffers first).  A request that can
 * never fit is rejected by submit with MALA_E_OOM.  Each request runs the
 * single-snapshot path of mala_predict with its own fixed work partition, so
 * its result is bitwise the same alone and among other requests.
 *  - submit copies the positions; dos_out (and density_out, if not NULL) are
 *    host buffers the server fills when the ticket completes; they must stay
 *    valid until poll/wait has returned for the ticket.
 *  - poll returns MALA_E_BUSY until the ticket is done, then the request's
 *    status (MALA_OK, or its error) once, and forgets the ticket.
 *  - times[3] = submit, start (admission), done, in seconds since creation.
 *  - destroy waits for running requests and drops queued ones.             */
typedef struct mala_server mala_server;
typedef struct {
    const double* positions;   /* host float64 [n_atoms][3]         */
    int32_t n_atoms;
    mala_cell_grid cell_grid;
    double rcut;
    int32_t twojmax;
    mala_egrid egrid;
    double T_kelvin;
    double n_electrons;
    double* dos_out;           /* host float64 [egrid.n]            */
    double* density_out;       /* host float64 [N_points] or NULL   */
} mala_request;

mala_status mala_server_create(int32_t device, const void* weights_blob, size_t bytes,
                               int32_t precision, size_t hbm_budget, int32_t max_inflight,
                               mala_server** out);
/* Host-only executor (a timer of ns_per_point per grid point per request)
 * behind the same scheduler: exercises admission and ordering without a
 * device.  Its "results" are the ticket number in dos_out/density_out.      */
mala_status mala_server_create_mock(int32_t slots, size_t hbm_budget, double ns_per_point,
                                    mala_server** out);
mala_status mala_server_submit(mala_server* s, const mala_request* req, uint64_t* ticket);
mala_status mala_server_poll(mala_server* s, uint64_t ticket, mala_result* result, double* times);
mala_status mala_server_wait(mala_server* s, uint64_t ticket, double timeout_s,
                             mala_result* result, double* times);
/* Sizes every slot once, before a stream of requests, for the element-wise
 * largest of the given requests (points, atoms, cell list, energy window of
 * the hottest one): afterwards a request within those sizes makes no device
 * or pinned allocation.  The server must be idle (MALA_E_BUSY otherwise);
 * MALA_E_OOM if all slots at that size would exceed the HBM budget.  Only
 * the shapes of the requests are read (positions are not).                 */
mala_status mala_server_reserve(mala_server* s, const mala_request* reqs, int32_t n);
/* Concurrency by work: a request is admitted next to running ones only if
 * the grid points in flight would stay within max_points (a request larger
 * than that runs alone; 0, the default, admits up to max_inflight requests
 * whatever their size).  Requests that fill the GPU on their own then do
 * not share it, which shortens their latency at the same throughput.      */
mala_status mala_server_set_inflight_points(mala_server* s, int64_t max_points);
/* stats[7] = queued, running, device bytes held by the slots, peak bytes
 * held, budget, allocations (device and pinned) made by the slots so far,
 * reserved bytes per slot (0 without mala_server_reserve).                 */
mala_status mala_server_stats(mala_server* s, double* stats);
const char* mala_server_last_error(void);
mala_status mala_server_destroy(mala_server* s);

/* ---------------------------------------------------------------- timing
 * Per-stage instrumentation (the method's cost breakdown by stage): while
 * enabled, every kernel group is bracketed by HIP events recorded on the
 * context stream (no synchronisation is added).  mala_profile_read()
 * synchronises the stream and returns, per stage, the summed event time in
 * milliseconds, the number of launches and the grid points they processed.
 * Enabling (on != 0) resets the accumulators.                               */
#define MALA_STAGE_BIN 0          /* atom cell list                          */
#define MALA_STAGE_UI 1           /* neighbour gather + u expansion          */
#define MALA_STAGE_ZB 2           /* Z/B contraction (bispectrum)            */
#define MALA_STAGE_MLP_LDOS 3     /* network, LDOS stored                    */
#define MALA_STAGE_MLP_DOS 4      /* network, DOS reduced in the epilogue    */
#define MALA_STAGE_FERMI 5        /* DOS sum, E_F root, E_band, weights */
#define MALA_STAGE_MLP_DENSITY 6  /* network, density in the epilogue        */
#define MALA_STAGE_INTEGRATE 7    /* stored-LDOS column sums and density     */
#define MALA_STAGE_ESTIMATE 8     /* E_F estimate on a point subsample       */
#define MALA_STAGE_DENSITY_WINDOW 9 /* density from the stored energy window */
#define MALA_STAGE_GAUSS 10       /* Gaussian descriptors                    */
#define MALA_STAGE_MLP_VJP 11     /* network vector-Jacobian product         */
#define MALA_STAGE_ADJ_Y 12       /* descriptor adjoint: dL/du               */
#define MALA_STAGE_ADJ_DEDR 13    /* descriptor adjoint: dL/dR               */
#define MALA_STAGE_ACE 14         /* grid ACE descriptors                    */
#define MALA_STAGE_ACE4 15        /* grid ACE descriptors of rank 4          */
#define MALA_N_STAGES 16
mala_status mala_profile_enable(mala_ctx* ctx, int32_t on);
mala_status mala_profile_read(mala_ctx* ctx, double* ms, int64_t* launches, int64_t* points);

#ifdef __cplusplus
}
#endif

#endif /* MALA_H */
