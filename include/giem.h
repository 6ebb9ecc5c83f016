/*
 * giem.h -- C-ABI of the MI355X (gfx950) Galerkin integral-equation solver.
 *
 * The library solves the discrete contracting integral equation (CIE) of
 * Kruglyakov & Bloshanskaya, "High-performance parallel solver for integral
 * equations of electromagnetics based on Galerkin method" (arXiv:1512.06126):
 *
 *   Problem (Sect. 2.1): Maxwell's equations with time factor exp(-i w t),
 *   layered background conductivity sigma_b(z), anomalous conductivity
 *   sigma_a in a rectangular domain split into Nx x Ny x Nz cells of uniform
 *   lateral size hx x hy (Sect. 3.1), magnetotelluric plane-wave source.
 *
 *   System (Sect. 2.2, linear system for U_n): A U = U^0 with
 *     A = S + R1 B R2   (Sect. 3.1, factorised form),
 *     S = 1 - gamma, R1 = -2 sqrt(Re sb) / V, R2 = sqrt(Re sb) gamma,
 *     gamma = (sa - sb) / (sa + conj sb), U^0 = sqrt(Re sb) <E^N>,
 *   B the block-Toeplitz matrix of Galerkin coefficients B_n^m (double
 *   volume integrals of the electric Green's tensor), E = U / a with
 *   a = (sa + conj sb) / (2 sqrt(Re sb)).
 *
 *   Operator apply (Sect. 3.3, three-step algorithm): forward 2-D FFT of the
 *   3 Nz zero-padded planes, Nz-order block products with the stored
 *   spectra of the packed table, inverse FFT.  Solver: GMRES with restarts
 *   (Sect. 3.3 names flexible GMRES; with no preconditioner it is GMRES).
 *
 * Conventions
 *   complex numbers are interleaved (re, im) doubles ("c128") unless stated;
 *   "device" pointers are HIP device memory (e.g. torch tensors' data_ptr),
 *   "host" pointers are ordinary host memory;
 *   every call is ordered on the caller's hipStream_t passed as `stream`
 *   (NULL = the default stream);
 *   cell vectors use the layout [nrhs][3][Nz][Ny][Nx] (component x, y, z;
 *   x index fastest); per-cell scalars use [Nz][Ny][Nx];
 *   SI units, mu0 = 4 pi 1e-7, omega = 2 pi f.
 *
 * Ownership: the caller owns every array it passes.  The library owns only
 * the giem_handle with its device tables and workspace, released by
 * giem_free.  No pointer is retained after a call returns.
 *
 * Errors: 0 = success; negative = error (outputs untouched unless stated),
 * with a message from giem_last_error() (thread-local); GIEM_ENOCONV is a
 * warning: the output holds the last iterate and the statistics are valid.
 * One handle must not be used by two threads at once.
 */
#ifndef GIEM_H
#define GIEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GIEM_OK 0
#define GIEM_EINVAL (-1)  /* bad argument, shape or pointer                   */
#define GIEM_EDOMAIN (-2) /* physics outside the method's domain (see calls)  */
#define GIEM_ENOMEM (-3)  /* device or host allocation failed                 */
#define GIEM_EHIP (-4)    /* a HIP runtime call failed                        */
#define GIEM_ENOCONV 1    /* iteration limit reached before the tolerance     */

/* operator modes for giem_apply */
#define GIEM_MODE_A 0u  /* y = A x   = S x + R1 B R2 x                            */
#define GIEM_MODE_AT 1u /* y = A^T x = S x + R2 B R1 x (B = B^T by reciprocity)  */
#define GIEM_MODE_B 2u  /* y = B x   (the raw convolution with the coefficients) */

/* arithmetic of the FFT convolution */
#define GIEM_FP64 0u /* complex128 FFTs, FP64 block products                     */
#define GIEM_FP32 1u /* complex64 FFTs and tables, FP32-accumulated products      */

/* giem_tables flags */
#define GIEM_TABLES_C64 1u /* also keep complex64 spectra for GIEM_FP32 applies */

/* Model of the medium (Sect. 2.1 and Appendix B).  All pointers are host. */
typedef struct {
  int32_t nlay;           /* number of interfaces d_1 < ... < d_nlay            */
  const double *d;        /* [nlay] interface depths, d_1 = 0 (surface), m, z down */
  const double *sigma_b;  /* c128 [nlay+1]: [0] air (0 allowed), [k] the layer
                             below d_k, [nlay] the lower half-space; Re >= 0     */
  int32_t nx, ny, nz;     /* anomaly grid (Sect. 3.1)                           */
  double hx, hy;          /* lateral cell size, m                               */
  double x0, y0;          /* position of the grid corner, m                     */
  const double *z_edges;  /* [nz+1] increasing depths of the cell faces, m; no
                             cell may straddle an interface (Appendix A)        */
} giem_model;

typedef struct giem_handle giem_handle; /* opaque: tables, workspace */

/* GMRES options.  precision: GIEM_FP64, or GIEM_FP32 = complex64 convolution
   inside an inner GMRES, corrected by FP64 residual refinement (outer loop). */
typedef struct {
  double tol;          /* stop when ||b - A x|| <= tol ||b|| (weighted norm)   */
  int32_t restart;     /* Krylov dimension m of GMRES(m), 1..64               */
  int32_t max_iter;    /* limit on operator applies of the (inner) GMRES      */
  int32_t precision;   /* GIEM_FP64 or GIEM_FP32                              */
  double inner_tol;    /* GIEM_FP32: relative tolerance of each inner solve
                          (default 1e-3); looser where a looser one already
                          meets tol (the last refinement step)            */
  int32_t max_outer;   /* GIEM_FP32: limit on refinement steps                */
  int32_t weighted_ip; /* nonzero: volume-weighted L2 inner product (Sect. 2.1) */
  int32_t warm_start;  /* nonzero: E_cells holds the initial guess on entry    */
  int32_t graph;       /* nonzero: each restart cycle runs as one captured HIP
                          graph with the Arnoldi step on the device (one host
                          wait per cycle); giem_solve_multi always does      */
} giem_solve_opts;

#define GIEM_HISTORY 64
typedef struct {
  int32_t iters;       /* operator applies in GMRES (all RHS, max over RHS)    */
  int32_t outer_iters; /* refinement steps (GIEM_FP32), else restarts          */
  int32_t converged;   /* 1 if every RHS met tol                              */
  double rel_residual; /* max over RHS of the final true ||b - A x|| / ||b||   */
  double ms;           /* wall time of the call, ms                           */
  int32_t n_history;   /* entries of history                                  */
  double history[GIEM_HISTORY];
                       /* the true ||b - A x|| / ||b|| (max over the RHS, one
                          that stopped earlier counting with its final
                          value) at the start of every restart cycle
                          (GIEM_FP64) or after every refinement step
                          (GIEM_FP32), the last entry being the final one;
                          with more than GIEM_HISTORY entries the first
                          GIEM_HISTORY - 1 and the last are kept              */
} giem_solve_stats;

/*
 * giem_tables -- compute the Galerkin coefficient tables B_n^m (Sect. 3.2,
 * Appendices A-C) for nfreq frequencies in FP64 and keep their packed spectra
 * (Sect. 3.3) on the device, together with the packed spatial tables
 * (Nx Ny 2Nz(2Nz+1) complex128 per frequency, read by giem_tables_export).
 * The vertical functions and the geometry-only quadrature matrices are built
 * on the host; the Hankel and horizontal contractions run as FP64 GEMMs on
 * the device.  Synchronises the stream.
 *   freq_hz: host [nfreq], > 0.  flags: GIEM_TABLES_C64 or 0.
 *   *out receives a new handle.
 * Errors: EINVAL (shapes), EDOMAIN (a cell straddles an interface,
 * Re sigma_b <= 0 in a layer holding cells), ENOMEM, EHIP.
 */
int giem_tables(const giem_model *model, int32_t nfreq, const double *freq_hz,
                uint32_t flags, void *stream, giem_handle **out);

/*
 * giem_tables_import -- build a handle from caller-supplied packed spatial
 * tables (Sect. 3.1, storage after Lemmas 1-2) instead of computing them.
 *   host_packed_spatial: host c128 [nfreq][Ny][Nx][E], E = 2 Nz (2 Nz + 1);
 *   block (i, j) holds Q(i, j) for y-offset i, x-offset j (observation minus
 *   source cell), classes in the order
 *     [xx upper][xy upper][yy upper][zz upper][xz full][yz full]
 *   (upper triangles row-major over iz <= jz, full blocks row-major [iz][jz];
 *   iz = depth index of the observation cell).  Entries of classes odd in x
 *   (xy, xz) at j = 0 and odd in y (xy, yz) at i = 0 are taken as zero.
 *   The spectra are computed on the device (packed even/odd 2-D transforms).
 */
int giem_tables_import(const giem_model *model, int32_t nfreq, const double *freq_hz,
                       const void *host_packed_spatial, uint32_t flags, void *stream,
                       giem_handle **out);

/* giem_tables_export -- copy the packed spatial table of frequency ifreq
   (layout as in giem_tables_import) to host memory [Ny][Nx][E] c128. */
int giem_tables_export(const giem_handle *t, int32_t ifreq, void *host_packed_spatial);

/* giem_tables_bytes -- device bytes held by the packed spectral tables of one
   frequency: (Nx+1)(Ny+1) 2 Nz (2 Nz + 1) complex (c128 and, if kept, c64). */
int giem_tables_bytes(const giem_handle *t, int64_t *bytes_c128, int64_t *bytes_c64);

/*
 * giem_apply -- one application of the operator (Sect. 3.3, three steps).
 *   sigma_a: device c128 [Nz][Ny][Nx] (ignored for GIEM_MODE_B);
 *   x, y:    device c128 [nrhs][3][Nz][Ny][Nx], 1 <= nrhs <= 8; x and y must
 *            not overlap;
 *   mode:    GIEM_MODE_A, GIEM_MODE_AT or GIEM_MODE_B; prec: GIEM_FP64 or
 *            GIEM_FP32 (needs GIEM_TABLES_C64).
 * Never synchronises the stream.  Errors: EINVAL, EDOMAIN (Re sigma_b <= 0),
 * EHIP.
 */
int giem_apply(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs,
               const void *x, void *y, uint32_t mode, uint32_t prec, void *stream);

/*
 * giem_apply_noalloc -- giem_apply for callers that cannot allocate device
 * memory during the call (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, kernels and results as
 * giem_apply; the two spectra buffers of the three steps live in a fixed
 * 64 MiB device array of the library instead of the handle's workspace, so
 * the call makes no hipMalloc, hipFree or other allocation (the handle and its
 * tables come from giem_tables as before).  Limit: 2 x 4 Nx Ny x 3 Nz x nrhs
 * complex (16 bytes in GIEM_FP64, 8 in GIEM_FP32) must fit in 64 MiB, e.g.
 * 64 x 64 x 16 with 2 right-hand sides in FP64; larger calls return EINVAL
 * before any kernel runs.  The array is one per device and shared by every
 * call on it, so calls that overlap in time on one device race (issue them on
 * one stream, or serialise them).  The handle's device must be current.
 * Never synchronises the stream.  Errors: EINVAL, EDOMAIN, EHIP.
 */
int giem_apply_noalloc(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs,
                       const void *x, void *y, uint32_t mode, uint32_t prec, void *stream);

/*
 * giem_apply_batch -- giem_apply for several frequencies of the handle at
 * once, one launch per kernel for all of them: y[f][r] = op_{ifreqs[f]}
 * x[f][r].  The frequencies share sigma_a (the diagonal scalings of
 * Sect. 3.1 do not depend on frequency); the spectra of all vectors are
 * transformed together and the block product runs over (frequency, point)
 * pairs, each with its own table.
 *   ifreqs:  host int32 [nf], 1 <= nf <= 16, indices of the handle's
 *            frequencies (repeats allowed);
 *   x, y:    device c128 [nf][nrhs][3][Nz][Ny][Nx], 1 <= nrhs <= 8,
 *            nf * nrhs <= 32; x and y must not overlap;
 *   sigma_a, mode, prec: as for giem_apply.
 * The result equals nf separate giem_apply calls.  The spectra workspace
 * grows to 2 x 4 Nx Ny x 3 Nz x 16 bytes per vector of the batch.  Never
 * synchronises the stream.  Errors: EINVAL, EDOMAIN, ENOMEM, EHIP.
 */
int giem_apply_batch(giem_handle *t, int32_t nf, const int32_t *ifreqs, const void *sigma_a,
                     int32_t nrhs, const void *x, void *y, uint32_t mode, uint32_t prec,
                     void *stream);

/* giem_apply_timed -- giem_apply with HIP events around each of the five
   kernels (x-FFT, y-FFT, block product, inverse y-FFT, inverse x-FFT); waits
   for the stream and writes their durations in ms to stage_ms[5]. */
int giem_apply_timed(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs,
                     const void *x, void *y, uint32_t mode, uint32_t prec, void *stream,
                     double *stage_ms);

/* giem_profile -- switch per-kernel event recording on or off for every
   later operator apply on this handle, including those inside giem_solve and
   giem_adjoint, and discard what was recorded.  enable: 0 off; 1 all five
   kernels (six hipEventRecord calls per apply); 2 + k, k = 0 .. 4, only
   kernel k in the order of giem_apply_timed (two calls per apply, which
   perturbs a solve less: the six events cost about 2% of a GMRES solve on a
   128 x 128 x 32 grid).  The events only time: they are recorded without a
   system-scope fence.  Never synchronises.  Errors: EINVAL (null handle or
   enable outside 0 .. 6). */
int giem_profile(giem_handle *t, int32_t enable);

/* giem_tune -- choose launch shapes of the apply for this handle by timing
   (Sect. 3.3): for the four FFT passes (x forward, y forward, y inverse, x
   inverse) every instantiated (sequences per workgroup, threads per
   workgroup) pair that fits the local data share, and for the block product
   the variants of giem_set_block_buffers; each candidate is run on
   nrhs right-hand sides of frequency ifreq for every precision whose tables
   exist, and the fastest median is kept on the handle for all later applies.
   The FFT shapes and block variants 1 and 2 do not change any result bit;
   variant 3 sums each contraction in another order (rounding-level
   differences).
     sigma_a: device c128 [Nz][Ny][Nx] (the diagonals of mode A are used);
     chosen:  host int32 [2][5][2] or NULL: per precision (0 = FP64,
              1 = FP32) the (sequences, threads) of the four passes, then
              (block-product variant, 0), as now in effect.
   The choice is also kept for the process and given to handles created
   later for the same grid (Nx, Ny, Nz) on the same device.
   Allocates and frees two vectors of nrhs right-hand sides; synchronises.
   Errors: EINVAL, ENOMEM, EHIP. */
int giem_tune(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs, void *stream,
              int32_t *chosen);

/* giem_set_fft_shape -- set the FFT launch shape of one precision (0 = FP64,
   1 = FP32) directly, e.g. to reuse a result of giem_tune on another handle
   of the same grid.  shape: host int32 [4][2], (sequences per workgroup,
   threads per workgroup) for x forward, y forward, y inverse, x inverse;
   threads must be 256 or 512 and the pass must fit the local data share and
   at most 16 elements per thread.  NULL restores the built-in choice.  Every
   shape gives the same result bits.
   Errors: EINVAL (nothing is changed). */
int giem_set_fft_shape(giem_handle *t, uint32_t prec, const int32_t *shape);

/* giem_set_block_buffers -- variant of the block product (Sect. 3.3 step 2)
   for one precision (0 = FP64, 1 = FP32): 1 or 2 register sets of prefetched
   points in one workgroup per CU (2 keeps the next point's loads in flight
   while a point is staged into local memory), 3 = two workgroups per CU,
   each wavefront doing a whole 16-row contraction (one workgroup's matrix
   products overlap the other's staging; where two do not fit the local data
   share, 1 is used), 4 = the row of the next point written from registers
   into a second local-memory buffer during the current point's matrix
   products (Nz <= 32 and at most 2 right-hand sides in FP64, else 2 is
   used), 0 for the built-in choice (1).  Where a point's packed row and
   input vectors do not fit the local data share (Nz > 32 at 2 right-hand
   sides) every variant runs the band-pair kernel, which stages the row by
   pairs of 16-level bands.  Results agree to rounding whichever variant
   runs.  Errors: EINVAL. */
int giem_set_block_buffers(giem_handle *t, uint32_t prec, int32_t nbuf);

/* giem_profile_read -- wait for the last recorded apply and report what was
   recorded since giem_profile or the previous read, then clear it:
     stage_ms[2][5]: summed kernel durations (ms) per precision (0 = FP64,
                     1 = FP32) and per kernel in the order of giem_apply_timed
                     (zero for kernels that were not bracketed);
     applies[2]: number of applies (all launched ones);
     rhs[2]:     right-hand sides in them whose results were used: GMRES
                 queues each step's apply before the host has finished the
                 previous step, and the vectors of a system that stops at
                 that step, or of a step whose Gram-Schmidt pass is repeated,
                 are discarded and not counted here.
   All pointers are host memory owned by the caller.  Errors: EINVAL, EHIP. */
int giem_profile_read(giem_handle *t, double *stage_ms, int64_t *applies, int64_t *rhs);

/*
 * giem_solve -- solve A U = U^0 by GMRES(m) (Sect. 2.2 system, Sect. 3.3
 * solver) and return the cell-averaged field E = U / a.
 *   sigma_a: device c128 [Nz][Ny][Nx] with Re >= 0 and no NaN;
 *   rhs:     device c128 [nrhs][3][Nz][Ny][Nx] holding U^0, or NULL for the
 *            plane-wave source: RHS 0 = x polarisation, RHS 1 = y
 *            polarisation (E^N horizontal, 1 V/m at z = 0);
 *   E_cells: device c128 [nrhs][3][Nz][Ny][Nx] output (input if warm_start);
 *   opts, stats: host; stats may be NULL.
 * Synchronises once per Arnoldi step.  Returns GIEM_ENOCONV if the
 * iteration limit is reached.
 */
int giem_solve(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs,
               const void *rhs, void *E_cells, const giem_solve_opts *opts,
               giem_solve_stats *stats, void *stream);

/*
 * giem_solve_batch -- giem_solve for nf frequencies of one model at once.
 * The operators of one model at several frequencies share sigma_a and the
 * diagonal scalings of Sect. 3.1 and differ only in their tables, so the
 * nf x nrhs systems run GMRES (Sect. 3.3, item (ii)) in lockstep: one host
 * synchronisation per Arnoldi step for all of them, applies grouped per
 * frequency.  Each system follows its own Krylov process, so the results are
 * those of nf separate giem_solve calls up to rounding.
 *   ifreqs:  host int32 [nf], frequency indices of the handle;
 *   rhs:     host [nf] device pointers to [nrhs][3][Nz][Ny][Nx] c128, or
 *            NULL (or NULL entries) for the plane-wave source;
 *   E_cells: host [nf] device pointers to [nrhs][3][Nz][Ny][Nx] c128 outputs
 *            (inputs if warm_start);
 *   stats:   host [nf] or NULL; iters and outer_iters count the whole batch,
 *            ms is the wall time of the call.
 * nf * nrhs <= 96.  Returns GIEM_ENOCONV if any system stops at the
 * iteration limit.  Errors as giem_solve.
 */
int giem_solve_batch(giem_handle *t, int32_t nf, const int32_t *ifreqs, const void *sigma_a,
                     int32_t nrhs, const void *const *rhs, void *const *E_cells,
                     const giem_solve_opts *opts, giem_solve_stats *stats, void *stream);

/*
 * giem_solve_multi -- the systems of several models (handles, grids of any
 * size) at several frequencies each, solved together: Sect. 3.3 item (ii)
 * GMRES for every (model, frequency, right-hand side) system, each restart
 * cycle of m Arnoldi steps recorded once as a HIP graph and replayed.  Inside
 * a cycle nothing returns to the host: the applies, both Gram-Schmidt passes
 * (the second one gated on the device by the same cancellation test as
 * giem_solve), the Hessenberg column, the Givens rotation and the residual
 * estimate run on the device, and the kernels of different models run on
 * separate branches of the graph.  The host waits once per cycle (Krylov
 * solution update, true residual, convergence).  A system that converges
 * inside a cycle keeps its Krylov length at that step.  With GIEM_FP32 the
 * FP64 residual refinement runs on the host and every inner solve is such a
 * cycle of complex64 graphs.
 *   groups:  host [ngroups]; group g solves handle t (each handle in one
 *            group) at its frequency indices ifreqs[nf] with its sigma_a,
 *            right-hand sides rhs[nf] (or NULL / NULL entries: plane waves,
 *            nrhs <= 2) into E_cells[nf] (as giem_solve_batch);
 *   stats:   host [sum of nf] in group order, or NULL.
 * At most 96 systems in total; every handle on the current device.  Errors
 * and ENOCONV as giem_solve.
 */
typedef struct {
  giem_handle *t;
  int32_t nf;
  const int32_t *ifreqs;      /* host [nf]                                    */
  const void *sigma_a;        /* device c128 [Nz][Ny][Nx] of this model       */
  const void *const *rhs;     /* host [nf] device pointers, or NULL           */
  void *const *E_cells;       /* host [nf] device pointers [nrhs][3][N] c128  */
} giem_solve_group;

int giem_solve_multi(int32_t ngroups, const giem_solve_group *groups, int32_t nrhs,
                     const giem_solve_opts *opts, giem_solve_stats *stats, void *stream);

/*
 * giem_adjoint -- gradient of J = sum_r Re( sum_n g_r[n] . E_r[n] ) with
 * respect to log sigma_a of every cell for real conductivities, from one
 * solve with A^T = S + R2 B R1.  B = B^T for the full 3N x 3N matrix: Lemma 1
 * (Sect. 3.1: yx = xy, zx = -xz^T, zy = -yz^T at a fixed lateral offset)
 * with the mirror parities of Lemma 2, which is the reciprocity
 * G(M, M0) = G(M0, M)^T of the Green's tensor of Appendix A.
 *   adj_src: device c128 [nrhs][3][Nz][Ny][Nx], g above;
 *   E_fwd:   device c128 [nrhs][3][Nz][Ny][Nx], the forward solution E;
 *   grad_log_sigma: device double [Nz][Ny][Nx], accumulated (+=).
 */
int giem_adjoint(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs,
                 const void *adj_src, const void *E_fwd, void *grad_log_sigma,
                 const giem_solve_opts *opts, giem_solve_stats *stats, void *stream);

/*
 * giem_fields -- electric and magnetic fields at receivers in the earth
 * above or below the anomaly grid from the cell field (Sect. 2.2, the representation
 * of the fields through G^E and G^H integrated over the cells, which holds
 * for any observation point; Appendix A):
 *   e(r) = E^N(r) + sum_n (sa_n - sb_n) [int_{cell n} G^E(r, M0) dM0] E_n,
 *   h(r) = H^N(r) + sum_n (sa_n - sb_n) [int_{cell n} G^H(r, M0) dM0] E_n,
 * with G^H = curl G^E / (i w mu0).  The horizontal E and all of H are
 * continuous across the surface; E_z is the value at the surface on the
 * earth side when the air is insulating (there sigma E_z + j_z = 0).
 *   sigma_a: device c128 [Nz][Ny][Nx];
 *   E_cells: device c128 [nrhs][3][Nz][Ny][Nx] (E = U / a, as from giem_solve);
 *   rec_xyz: host [nrec][3] receiver positions (x, y, z) in m, z positive
 *            down; all receivers of a call at one depth z0 with
 *            d[0] <= z0 <= z_edges[0] (the earth's surface, any depth in
 *            the earth above the grid, or the top face of the grid's first
 *            cells) or z0 > z_edges[Nz] (below the grid), each above or
 *            below the centre of a cell of the grid;
 *   E_rec, H_rec: device c128 [nrhs][nrec][3] outputs.
 * E^N, H^N at depth z0 of the plane wave of 1 V/m at the surface are added
 * for RHS 0 (x polarisation) and RHS 1 (y polarisation); further RHS get the
 * anomalous fields only (giem_fields_anomalous: none added, for any source).
 * The cell integrals for every receiver offset are computed on the first
 * call for a frequency and depth and kept on the handle.  Synchronises the
 * stream.  Errors: EINVAL, EDOMAIN (receivers not at one depth in those
 * ranges or not over cell centres), ENOMEM, EHIP.
 */
int giem_fields(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs,
                const void *E_cells, int32_t nrec, const double *rec_xyz, void *E_rec,
                void *H_rec, void *stream);

/*
 * giem_fields_anomalous -- giem_fields without the plane-wave normal fields:
 * e - E^N and h - H^N of every RHS (Sect. 2.2), for solves whose source is
 * not the plane wave (giem_dipole_source).  Same arguments and errors.
 */
int giem_fields_anomalous(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs,
                          const void *E_cells, int32_t nrec, const double *rec_xyz, void *E_rec,
                          void *H_rec, void *stream);

/*
 * giem_dipole_source -- right-hand side of electric dipole sources (Sect.
 * 2.1: an external current J_ext = p delta(r - r_s); Sect. 2.2: the source
 * enters the scaled system only through the cell averages of its normal
 * field, U0_n = sqrt(Re sigma_b) <E^0>_n).  By reciprocity of the layered
 * background (Appendix A: G^E(r, r') = G^E(r', r)^T) the cell integral of
 * the dipole's normal field is the transposed receiver kernel of a receiver
 * at the source point: int_{cell n} E^0 = [int_{cell n} G^E(r_s, M0) dM0]^T p.
 *   src_xyz: host [nsrc][3] source positions, 1 <= nsrc <= 8, with the
 *            constraints of giem_fields' receivers (one depth z0 above
 *            or below the grid, over or under cell centres);
 *   moments: host c128 [nsrc][3] dipole moments p (A m);
 *   rhs:     device c128 [nsrc][3][Nz][Ny][Nx] output, one right-hand side
 *            per source, to be passed as giem_solve's rhs; the solve gives
 *            the total cell field, and at receivers giem_fields_anomalous
 *            gives the anomalous part (the dipole's own normal field at the
 *            receivers is not computed).
 * Shares the receiver kernels of giem_fields (built on first use for the
 * depth).  Synchronises the stream.  Errors: EINVAL, EDOMAIN, ENOMEM, EHIP.
 */
int giem_dipole_source(giem_handle *t, int32_t ifreq, int32_t nsrc, const double *src_xyz,
                       const double *moments, void *rhs, void *stream);

/*
 * giem_impedance -- impedance tensor at every receiver from the fields of the
 * x and the y polarisation (Sect. 4, the apparent resistivity of the
 * benchmark is computed from it): with Eh[c][p] = e_c of polarisation p and
 * Hh[c][p] = h_c of polarisation p (c, p in {x, y}), Z = Eh Hh^-1.
 *   E_rec, H_rec: device c128 [2][nrec][3] (as written by giem_fields with
 *                 nrhs = 2: RHS 0 = x, RHS 1 = y polarisation);
 *   Z:            device c128 [nrec][2][2] output, row-major (Zxx Zxy Zyx Zyy).
 * Asynchronous on the stream.  A receiver whose Hh is singular gets inf/NaN.
 * Errors: EINVAL, EHIP.
 */
int giem_impedance(int32_t nrec, const void *E_rec, const void *H_rec, void *Z, void *stream);

/*
 * giem_impedance_adjoint -- reverse mode of giem_impedance.  gZ holds the
 * gradient of a real function L with respect to Z in the convention
 * dL = Re sum conj(gZ) dZ (the gradient torch stores for complex tensors).
 * Writes wE, wH such that dL = Re sum_{p,q,c} (wE[p][q][c] de + wH[p][q][c] dh)
 * for perturbations de, dh of E_rec, H_rec.
 *   E_rec, H_rec: device c128 [2][nrec][3];  gZ: device c128 [nrec][2][2];
 *   wE, wH:       device c128 [2][nrec][3] outputs (z components zero).
 * Asynchronous on the stream.  Errors: EINVAL, EHIP.
 */
int giem_impedance_adjoint(int32_t nrec, const void *E_rec, const void *H_rec, const void *gZ,
                           void *wE, void *wH, void *stream);

/*
 * giem_fields_adjoint -- transpose of giem_fields (Sect. 2.2 field
 * representation).  For weights wE, wH on the receiver fields,
 * dL = Re sum (wE . de + wH . dh), it writes the source of the adjoint solve
 * and adds the explicit part of the gradient:
 *   v_n      = sum_q wE_q^T [int_{cell n} G^E(r_q, M0) dM0]
 *            + wH_q^T [int_{cell n} G^H(r_q, M0) dM0]          (per RHS),
 *   adj_src  = (sa_n - sb_n) v_n            (device c128 [nrhs][3][Nz][Ny][Nx]),
 *   grad_log_sigma[n] += Re sum_r sa_n v_n . E_n  (device double [Nz][Ny][Nx]).
 * Passing adj_src and E_cells to giem_adjoint then adds the part of the
 * gradient that flows through the cell field, so that grad_log_sigma ends as
 * dL / d log sa for real conductivities.  Receivers, E_cells and the kernel
 * cache are as in giem_fields; nrec = 0 gives adj_src = 0.  Synchronises.
 * Errors: EINVAL, EDOMAIN, ENOMEM, EHIP.
 */
int giem_fields_adjoint(giem_handle *t, int32_t ifreq, const void *sigma_a, int32_t nrhs,
                        const void *E_cells, int32_t nrec, const double *rec_xyz, const void *wE,
                        const void *wH, void *adj_src, void *grad_log_sigma, void *stream);

void giem_free(giem_handle *t);
const char *giem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GIEM_H */
