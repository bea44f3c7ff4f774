/*
 * rpb.h -- C ABI of librpb: the wall-corrected Rotne-Prager ("Rotne-Prager-Blake")
 * mobility of N equal spheres above a no-slip wall, and its three consumers, on one
 * AMD Instinct MI355X (gfx950).
 *
 * Paper: F. Balboa Usabiaga, B. Delmotte, A. Donev, "Brownian dynamics of confined
 * suspensions of active microrollers", J. Chem. Phys. 146, 134104 (2017), arXiv:1612.00474.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Units are the caller's; reduced units a = eta = kT = 1 are typical.  The wall is
 *    the plane z = 0 and the fluid fills z > 0.
 *  - Every array argument is a DEVICE pointer to contiguous row-major [n][3] float64
 *    (x, y, z per sphere), 8-byte aligned, owned by the caller.  The library never
 *    frees or keeps them after the call returns.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream).  Calls
 *    that must read device scalars (Lanczos convergence, validation flags)
 *    synchronise `stream` before returning; host out-parameters are valid on return.
 *    The single-system Lanczos solves of small systems (3 n <= 1536) run their
 *    eigensolve on a second stream owned by the context, beside the next product; before
 *    returning they make `stream` wait for all of it, so work enqueued later on `stream`
 *    is ordered after the whole solve.  That stream's work is enqueued by a helper thread
 *    that the context starts on the first such solve and rpb_destroy() stops; it makes HIP
 *    calls on the context's device only while a solve is in progress.
 *  - Return value: RPB_OK (0) or a negative rpb_status.  rpb_last_error() then holds
 *    a message.  No C++ exception crosses this interface.
 *  - n == 0 is a no-op that returns RPB_OK.  RPB_EINVAL for n < 0, a NULL required
 *    pointer, a, eta or kT <= 0, an unknown precision, an output that overlaps an
 *    input, or an argument outside the documented range.
 *  - RPB_ENONFINITE when a position holds NaN or Inf (checked on the device before any
 *    product is formed).
 *  - One context per host thread; calls on one context must not overlap.  A context
 *    owns its device workspace, which grows on demand (hipMalloc) and is released by
 *    rpb_destroy().
 *  - Results are deterministic: no floating-point atomics, fixed reduction orders.
 */
#ifndef RPB_H
#define RPB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rpb_ctx rpb_ctx;     /* opaque: device, workspace, tuning table, timers */
typedef void *rpb_stream_t;         /* a hipStream_t */

typedef enum {
  RPB_OK = 0,
  RPB_EINVAL = -1,      /* invalid argument */
  RPB_ENOMEM = -2,      /* device allocation failed */
  RPB_EDEVICE = -3,     /* a HIP call failed (message in rpb_last_error) */
  RPB_ENOCONV = -4,     /* Lanczos tolerance not reached within max_iter; output = last iterate */
  RPB_ENOTSPD = -5,     /* a Ritz value of the Lanczos tridiagonal is negative */
  RPB_ENONFINITE = -6   /* NaN or Inf in the positions */
} rpb_status;

typedef enum {
  RPB_FP64 = 0,         /* pair terms and sums in float64 */
  RPB_MIXED = 1         /* pair terms in float32 with compensated (Kahan) float32 sums per
                           target, positions split into float32 hi/lo; vectors, Lanczos
                           recurrence, eigensolve and norms stay float64 */
} rpb_precision;

typedef struct {
  double a;             /* sphere radius (> 0) */
  double eta;           /* fluid viscosity (> 0) */
  double kT;            /* thermal energy k_B T (> 0) */
  int precision;        /* rpb_precision */
  int wall;             /* 1: no-slip wall at z = 0 (Rotne-Prager-Blake tensors, heights clamped
                           and weighted as in App. A, soft wall repulsion in rpb_forces);
                           0: free space (unbounded RPY tensors of Sec. II.B alone, no
                           clamping, no wall force), the contrast of Sec. II.C / Fig. 1 */
  double lx, ly;        /* both > 0: pseudo-periodic boundaries in x and y with these box
                           lengths (App. B): pair forces by the minimum image convention,
                           hydrodynamics summed over the minimum image and its images in the
                           eight neighbour cells; both 0: unbounded.  Single-system calls only
                           (the batched entry points return RPB_EINVAL); rpb_forces needs
                           lx, ly > 2 (2a + 40 b) so that the minimum image holds every pair
                           within its cutoff. */
} rpb_params;

/* Context ---------------------------------------------------------------------------- */

/* Create a context on HIP device `hip_device`.  *out receives the handle. */
int rpb_create(int hip_device, rpb_ctx **out);
/* Release the context and its device workspace (NULL is ignored). */
void rpb_destroy(rpb_ctx *ctx);
/* Message of the last failure on this context ("" if none).  Valid until the next call. */
const char *rpb_last_error(const rpb_ctx *ctx);
/* Library version string. */
const char *rpb_version(void);

/* Mobility product --------------------------------------------------------------------
 *
 * U = M F + M_C T for spheres at `pos`, with
 *   M    the translation mobility (paper, Sec. II.B, eq. mobilityDifferential for separated
 *        spheres, eq. mobilityOverlap for overlapping spheres: unbounded RPY part plus the
 *        Faxen-applied image part of Blake's wall Green's function; self block included),
 *   M_C  the translation-rotation mobility (Sec. III, eq. mobilityDifferentialTR),
 * both regularised as M = B M~ B (App. A, eq. effMob): B_ii = H0(z_i/a) with
 * H0(x) = clamp(x, 0, 1), and M~ evaluated with heights clamped to max(z, a).  The same
 * B is applied to M_C, so spheres at or below the wall neither move nor move others.
 * Direct O(N^2) summation over all ordered pairs (Sec. II.B).
 *
 * force, torque: [n][3] device arrays, either may be NULL (treated as zero; not both).
 * vel_out: [n][3] device array, overwritten; must not overlap pos, force or torque.
 */
int rpb_mobility_matvec(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                        const double *force, const double *torque, double *vel_out,
                        rpb_stream_t stream);

/* The same whole-system product for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc).  It calls no
 * hipMalloc, hipFree or other allocating routine: every intermediate (packed geometry, packed
 * sources, partial sums of the ordered pair kernel over source chunks) lives in a 32 MiB
 * static device array that each GPU the library runs on holds until the process ends
 * (resolved once per device by rpb_create).  It also never synchronises the stream and does
 * not check the positions (a NaN or Inf position gives a non-finite velocity, not
 * RPB_ENONFINITE); the opt-in output check and timing records do not apply.
 * Limit: the packed geometry and sources plus one source chunk of partial sums must fit,
 * about (32 + 48 + 24) n bytes in float64 and (28 + 24 + 24) n in mixed precision, so n up to
 * about 322,000 (RPB_FP64) or 441,000 (RPB_MIXED); larger n returns RPB_EINVAL.  Below the limit the
 * sources are split into as many chunks (workgroups) as the launch shape asks for and fit.
 * The result agrees with rpb_mobility_matvec to rounding (another summation order).
 * All calls on one GPU share its array, which keeps the last call's contents: calls that
 * overlap in time on one GPU (several streams or host threads) race and must be serialised
 * by the caller.  Arguments and other errors as for rpb_mobility_matvec. */
int rpb_mobility_matvec_noalloc(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                                const double *force, const double *torque, double *vel_out,
                                rpb_stream_t stream);

/* Rows [row_begin, row_end) of the same product (all n spheres are sources).  vel_out
 * then holds (row_end - row_begin) rows: the per-GPU share of a row-sharded product.  Row
 * ranges take the ordered kernel (target tiles x source chunks, chunking fixed by n), so
 * the results of any partition of [0, n) concatenate bitwise to one another and to a
 * whole-system product taken with that kernel; the default whole-system product (one
 * evaluation per unordered pair, other summation order) agrees with them to rounding. */
int rpb_mobility_matvec_rows(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                             const double *force, const double *torque, int64_t row_begin,
                             int64_t row_end, double *vel_out, rpb_stream_t stream);

/* Brownian increment ------------------------------------------------------------------
 *
 * out ~ M^{1/2} w by the Krylov/Lanczos method of Ando et al. (paper, Sec. II.C): m Lanczos
 * steps on K_m(M, w) with full re-orthogonalisation, T_m = Q L Q^T on the device (updated
 * each step from T_{m-1}'s eigendecomposition, as lanczos_tridiag_sqrt below),
 * g_m = |w| V_m Q L^{1/2} Q^T e_1.  Stops at the first m >= 2
 * with eps_m = |g_m - g_{m-1}| / |g_{m-1}| < tol (evaluated in the orthonormal basis), or
 * when the Krylov space is invariant (exact result, RPB_OK), or at max_iter
 * (RPB_ENOCONV, out = g_max_iter).  Only M (not M_C) enters.
 *
 * w, out: [n][3] device arrays (out must not overlap pos or w).  tol > 0 (use a tiny tol
 * with max_iter = m for a fixed number of steps).  1 <= max_iter <= 64.
 * iters_out, eps_out: host pointers (may be NULL) for m and eps_m (0 when m = 1).
 */
int lanczos_sqrt_apply(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                       const double *w, double tol, int max_iter, double *out,
                       int *iters_out, double *eps_out, rpb_stream_t stream);

/* Block-diagonal preconditioned Lanczos (the preconditioning tried in Sec. II.C): with L the
 * diagonal whose square is the diagonal of the self blocks M_ii (the wall self-mobilities
 * mu_par, mu_par, mu_perp times H_i^2; L = 1 where H_i = 0), Lanczos runs on
 * B = L^-1 M L^-1 and returns out = L B^{1/2} w.  That is a square root of M in the sense
 * out out^T ~ M over w (covariance L B L = M), not the symmetric root M^{1/2} w, so it is a
 * valid Brownian increment.  The stopping test applies to the B-space iterates.  Arguments,
 * errors and iteration semantics as for lanczos_sqrt_apply. */
int lanczos_sqrt_apply_precond(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                               const double *w, double tol, int max_iter, double *out,
                               int *iters_out, double *eps_out, rpb_stream_t stream);

/* The small dense step of the same method (Sec. II.C) on its own: for the symmetric
 * tridiagonal T with diagonal alpha[0..m-1] and off-diagonal beta[0..m-2], the vectors
 * y_k = wnorm T_k^{1/2} e_1 of its leading k x k blocks T_k, k = 1..m, in the order and by the
 * device code of the Lanczos solves: T_k = Q L Q^T from the arrowhead matrix that T_{k-1}'s
 * eigenvectors make of T_k (secular equation, one root per lane, deflation of negligible
 * couplings, eigenvectors from the recomputed coupling of Gu and Eisenstat), then
 * y_k = wnorm Q L^{1/2} Q^T e_1 with negative eigenvalues taken as zero.
 * alpha, beta: host arrays (beta may be NULL when m = 1), finite; wnorm finite, >= 0.
 * y_out: host array of m * m doubles, row k - 1 holding y_k in its first k entries and zeros
 * after.  1 <= m <= 64.  Synchronises the stream.  RPB_EDEVICE if an eigenvalue iteration
 * does not converge. */
int lanczos_tridiag_sqrt(rpb_ctx *ctx, int32_t m, const double *alpha, const double *beta,
                         double wnorm, double *y_out, rpb_stream_t stream);

/* Stochastic drift --------------------------------------------------------------------
 *
 * Centred random finite difference (paper, Sec. II.A, last term of eq. EM / eq. AB):
 *   drift = (kT/delta) [ M(q + delta/2 w~) w~ - M(q - delta/2 w~) w~ ],
 * equal in expectation to kT div_q . M up to O(delta^2).  delta > 0.
 * The two products use `rfd_precision` (RPB_FP64 or RPB_MIXED); in float32 the
 * difference of two O(1) products is divided by delta, so float64 is the default
 * choice for small delta.
 */
int rfd_drift(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
              const double *w_tilde, double delta, int rfd_precision, double *drift_out,
              rpb_stream_t stream);

/* One-sided random finite difference (Sec. II.A: the paper allows a one-sided difference in
 * place of the centred one):
 *   drift = (kT/delta) [ M(q + delta w~) w~ - M(q) w~ ],
 * equal in expectation to kT div_q . M up to O(delta); its truncation/round-off balance is
 * delta/a ~ eps^{1/2} against eps^{1/3} for the centred form.  Arguments and errors as for
 * rfd_drift. */
int rfd_drift_one_sided(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                        const double *w_tilde, double delta, int rfd_precision,
                        double *drift_out, rpb_stream_t stream);

/* Forces --------------------------------------------------------------------------------
 *
 * Soft steric repulsion of the paper (Sec. III, eq. soft_potential) between all pairs
 * (d = 2a, r = centre distance) and with the wall (d = a, r = z), plus gravity f_grav_z
 * along z:  f(r) = U0/b for r < d, (U0/b) exp(-(r-d)/b) for r >= d, repulsive.  Pairs with
 * r - d > 40 b are skipped (their force is below 4.3e-18 U0/b).  u0 >= 0, b > 0.
 * The pairs are found with a cell list (cells of side >= 2a + 40 b, O(N) work); a box with
 * fewer than three such cells per side takes an all-pairs search.  Results are bitwise
 * reproducible.  The workspace grows by about 100 bytes per sphere.
 */
int rpb_forces(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
               double f_grav_z, double u0, double b, double *force_out, rpb_stream_t stream);

/* Counter-based normal variates: Philox4x64-10 (Salmon et al., SC'11) with key
 * (seed, stream_id) and counter (block, step, 0, 0); block k gives variates 4k..4k+3;
 * uniforms ((x >> 12) + 1/2) 2^-52, normals by Box-Muller on (u0,u1) and (u2,u3).
 * out: `count` float64 values on the device. */
int rpb_normals(rpb_ctx *ctx, int64_t count, uint64_t seed, uint64_t stream_id,
                uint64_t step, double *out, rpb_stream_t stream);

/* Time step -------------------------------------------------------------------------------
 *
 * One step of eq. BD with the active torque term of Sec. III:
 *   u^n     = M^n F^n + M_C^n T                         (forces from rpb_forces, T constant)
 *   SAB (eq. AB): q^{n+1} = q^n + dt (3/2 u^n - 1/2 u^{n-1}) + sqrt(2 kT dt) g^n + dt D^n
 *   EM  (eq. EM): q^{n+1} = q^n + dt u^n + sqrt(2 kT dt) g^n + dt D^n
 * with g^n = lanczos_sqrt_apply(W^n) (or lanczos_sqrt_apply_precond) and D^n = rfd_drift(W~^n)
 * (or rfd_drift_one_sided).  The first SAB step (have_prev == 0) is an EM step.  On return
 * state->pos holds q^{n+1}, state->u_prev holds u^n, state->step is incremented and
 * state->have_prev = 1.
 */
typedef struct {
  double dt;            /* time step (> 0) */
  double delta;         /* RFD length (> 0) */
  double lanczos_tol;   /* Lanczos relative tolerance (> 0) */
  int lanczos_max_iter; /* 1..64 */
  int scheme;           /* 0 = stochastic Adams-Bashforth, 1 = Euler-Maruyama */
  int rfd_precision;    /* rpb_precision of the two RFD products */
  int rfd_scheme;       /* 0 = centred RFD (rfd_drift), 1 = one-sided (rfd_drift_one_sided) */
  int lanczos_precond;  /* 1: block-diagonal preconditioned Lanczos (lanczos_sqrt_apply_precond) */
  double f_grav_z;      /* gravity force on each sphere along z */
  double torque[3];     /* constant torque on every sphere */
  double steric_u0;     /* U0 of eq. soft_potential */
  double steric_b;      /* b of eq. soft_potential */
  uint64_t seed;        /* noise seed: W = normals(seed, 0, step), W~ = normals(seed, 1, step) */
} rpb_sab_config;

typedef struct {
  int64_t n;            /* number of spheres */
  double *pos;          /* [n][3] device, in/out */
  double *u_prev;       /* [n][3] device, caller-owned storage for u^{n-1} (in/out) */
  int64_t step;         /* step counter n (in/out) */
  int have_prev;        /* 1 when u_prev holds u^{n-1} (in/out) */
} rpb_sab_state;

/* w, w_tilde: optional [n][3] device arrays of the normals W^n, W~^n; NULL draws them
 * with rpb_normals(seed, 0 or 1, step).  iters_out / eps_out: optional host pointers for
 * the Lanczos iteration count and last eps.  RPB_ENOCONV from Lanczos does not stop the
 * step (the last iterate is used) but is returned after the update. */
int sab_step(rpb_ctx *ctx, const rpb_params *p, const rpb_sab_config *cfg, rpb_sab_state *state,
             const double *w, const double *w_tilde, int *iters_out, double *eps_out,
             rpb_stream_t stream);

/* Batched suspensions -----------------------------------------------------------------------
 *
 * nsys independent suspensions, concatenated: sphere i of system s is row offs[s] + i of
 * every [n_total][3] device array, n_total = offs[nsys].  `offs` is a HOST array of nsys + 1
 * non-decreasing int64 with offs[0] = 0 (empty systems allowed).  Spheres of different systems
 * do not interact.  One persistent launch of the pair kernel serves all systems: work items
 * (system, target tile, source chunk) are sorted by cost, largest first, and pulled from a
 * device counter by a fixed grid of workgroups, so uneven sizes share the whole GPU.
 * Each system's result equals the single-system call on its own rows (same arithmetic, the
 * summation order over sources may differ).  1 <= nsys <= 4096 for the Lanczos and step
 * calls. */
int rpb_mobility_matvec_batched(rpb_ctx *ctx, const rpb_params *p, int32_t nsys,
                                const int64_t *offs, const double *pos, const double *force,
                                const double *torque, double *vel_out, rpb_stream_t stream);

/* One Lanczos process per system (tolerance test per system; a converged system is frozen
 * while the others continue).  iters_out, eps_out: optional HOST arrays of nsys entries.
 * Returns RPB_ENOCONV if any system missed tol (its output is its last iterate). */
int lanczos_sqrt_apply_batched(rpb_ctx *ctx, const rpb_params *p, int32_t nsys,
                               const int64_t *offs, const double *pos, const double *w,
                               double tol, int max_iter, double *out, int *iters_out,
                               double *eps_out, rpb_stream_t stream);

/* One SAB / EM step of every system (sab_step per system, all in the same launches).  The
 * step number `step` selects the device noise (w / w_tilde NULL); have_prev = 0 makes it an
 * EM step.  pos and u_prev ([n_total][3], device) are updated in place; the caller advances
 * its step counter.  iters_out, eps_out: optional HOST arrays of nsys entries. */
int sab_step_batched(rpb_ctx *ctx, const rpb_params *p, const rpb_sab_config *cfg, int32_t nsys,
                     const int64_t *offs, double *pos, double *u_prev, int64_t step,
                     int have_prev, const double *w, const double *w_tilde, int *iters_out,
                     double *eps_out, rpb_stream_t stream);

/* Several source vectors, one configuration ------------------------------------------------
 *
 * vel[v] = M force[v] for v < nvec: force and vel are [nvec][n][3] float64 device arrays
 * (vector-major), pos [n][3].  The products the Lanczos method needs (Sec. II.C) for several
 * independent noise vectors of one configuration share the pair coefficients: each unordered
 * pair's coefficients are evaluated once and applied to four vectors in the same launch
 * (the symmetric tile-pair kernel, diagonal tiles as ordered pairs).  Forces only (no
 * torques), wall or free space, no pseudo-periodic box (RPB_EINVAL).  Each result agrees with
 * rpb_mobility_matvec on that vector to rounding (summation order differs).  The partial sums
 * of one launch are held to 512 MiB: larger systems walk the triangle of tile pairs in chunks,
 * each followed by its reduction into vel, so the workspace stays bounded for any n. */
int rpb_mobility_matvec_multi(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                              int32_t nvec, const double *force, double *vel,
                              rpb_stream_t stream);

/* nvec independent Lanczos processes (Sec. II.C) for M^{1/2} w[v], one configuration: every
 * Krylov iteration takes one multi-vector product of the processes still running; a process
 * stops on its own tolerance test.  w, out: [nvec][n][3] device; iters_out, eps_out: optional
 * HOST arrays of nvec entries; 0 <= nvec <= 4096.  Returns RPB_ENOCONV if any process missed
 * tol (its output is its last iterate). */
int lanczos_sqrt_apply_multi(rpb_ctx *ctx, const rpb_params *p, int64_t n, const double *pos,
                             int32_t nvec, const double *w, double tol, int max_iter,
                             double *out, int *iters_out, double *eps_out, rpb_stream_t stream);

/* A batched step captured in a hipGraph.  Creation runs one warm-up step on scratch copies
 * (the caller's arrays are not modified), then captures the step bound to `pos` and `u_prev`
 * with the Lanczos budget cfg->lanczos_max_iter (converged systems are frozen on the device;
 * no host synchronisation inside the step).  Each rpb_step_graph_launch advances pos, u_prev
 * and the device step counter (starting at `step`, with `have_prev`) by one step on `stream`.
 * The graph owns a private context and workspace; it must be destroyed before the arrays are
 * freed.  rpb_step_graph_status synchronises `stream` and reports the step counter and the
 * per-system Lanczos iterations / eps of the last step. */
typedef struct rpb_graph rpb_graph;
int rpb_step_graph_create(rpb_ctx *ctx, const rpb_params *p, const rpb_sab_config *cfg,
                          int32_t nsys, const int64_t *offs, double *pos, double *u_prev,
                          int64_t step, int have_prev, rpb_graph **out, rpb_stream_t stream);
int rpb_step_graph_launch(rpb_graph *g, rpb_stream_t stream);
int rpb_step_graph_status(rpb_graph *g, int64_t *step_out, int *iters_out, double *eps_out,
                          rpb_stream_t stream);
void rpb_step_graph_destroy(rpb_graph *g);

/* Launch-shape tuning ---------------------------------------------------------------------
 *
 * One shape per precision.  Single-system products: tpt, targets per lane of the pair kernels
 * (1, 2 or 4; 4 applies to the symmetric kernel, the ordered kernel then takes 2); target_wgs,
 * workgroups the ordered kernel aims for when splitting the sources into chunks; symmetric,
 * whole-system products use the symmetric tile-pair kernel (M_ij = M_ji^T: each unordered pair
 * evaluated once, both directions applied; with torques both coupling directions come from the
 * shared geometry).  The symmetric kernel's partial sums (float32 in mixed precision) are held to
 * 512 MiB per launch: larger systems walk the triangle of tile pairs in several launches, so any n
 * takes it.  Row ranges (rpb_mobility_matvec_rows) always take the ordered kernel.  Batched
 * products: batch_tpt (1 or 2); batch_symmetric, the
 * persistent kernel works on (system, tile pair) items of the symmetric kernel instead of
 * (system, target tile, source chunk) items (a batch whose symmetric partials would exceed 4 GiB
 * takes the ordered items); batch_chunk, sources per ordered work item
 * (multiple of 256); batch_wgs, persistent workgroups.  rpb_autotune times the candidates for
 * p->precision on the given configuration (force-only products, `reps` launches each, HIP
 * events on `stream`); nsys = 1 tunes the single-system fields, nsys > 1 the batched ones.
 * The fastest is kept in the context and cached per (precision, single/batched,
 * floor(log2 n_total)); a cached shape is reused without timing (best_ms_out = -1 then).
 * Results depend on the shape only through the order of the floating-point summation. */
typedef struct {
  int tpt;
  int target_wgs;
  int batch_chunk;
  int batch_wgs;
  int symmetric;        /* 1: whole-system products evaluate each unordered pair once */
  int batch_tpt;
  int batch_symmetric;  /* 1: batched products evaluate each unordered pair once */
} rpb_shape;
typedef struct {
  rpb_shape fp64;
  rpb_shape mixed;
} rpb_tuning;
int rpb_get_tuning(const rpb_ctx *ctx, rpb_tuning *out);
int rpb_set_tuning(rpb_ctx *ctx, const rpb_tuning *t);
int rpb_autotune(rpb_ctx *ctx, const rpb_params *p, int32_t nsys, const int64_t *offs,
                 const double *pos, int reps, rpb_tuning *out, double *best_ms_out,
                 rpb_stream_t stream);

/* Output check (debug aid) ---------------------------------------------------------------------
 *
 * Off by default.  When enabled on a context, rpb_mobility_matvec, rpb_mobility_matvec_rows,
 * rpb_mobility_matvec_batched, lanczos_sqrt_apply (and its preconditioned form), rfd_drift,
 * rfd_drift_one_sided and sab_step scan their result (the velocity, the increment, the drift,
 * the new positions) for NaN or Inf once it is computed, synchronise the stream and return
 * RPB_ENONFINITE if one is found.  The result is left as computed (for sab_step the state has
 * advanced).  Inputs other than positions (forces, torques, noise) are not checked, so this is
 * how a non-finite force shows up.  Costs one pass over the result and a synchronisation per
 * call.  Returns RPB_EINVAL for a NULL context. */
int rpb_output_check_enable(rpb_ctx *ctx, int enable);

/* Timing ------------------------------------------------------------------------------------
 *
 * When enabled, the library brackets every launch of the O(N^2) pair kernel with HIP
 * events on the stream it is launched on.  rpb_timing_read() synchronises, returns the
 * summed kernel time in milliseconds, the number of launches and the number of ordered
 * pair interactions of the launches of kernel variant `kind`, and removes them from the
 * record.  kind = 2 * (precision == RPB_MIXED) + (torque present), plus 4 for the batched
 * kernel; 8 + 2 * (precision == RPB_MIXED) for the multi-vector kernel, whose pair count is
 * n^2 times the vectors of the launch; kind = -1 takes all.  A single-system Lanczos solve
 * enqueues one iteration past its stop before it reads the stop flag; that iteration's
 * launches return at once and are dropped from the record. */
int rpb_timing_enable(rpb_ctx *ctx, int enable);
int rpb_timing_read(rpb_ctx *ctx, int kind, double *ms_out, int64_t *launches_out,
                    double *pairs_out);

#ifdef __cplusplus
}
#endif

#endif /* RPB_H */
