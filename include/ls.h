/*
 * ls.h -- C ABI of the MI355X two-level Lippmann-Schwinger solver.
 *
 * Method: Zepeda-Nunez & Zhao, "Fast alternating bi-directional
 * preconditioner for the 2D high-frequency Lippmann-Schwinger equation"
 * (arXiv 1602.07652).  The discrete problem is H u = f with
 * H = I + omega^2 G D and f = -omega^2 G D u_I (Section 2, eq.
 * discrete_Lipmann-Schwinger); the preconditioner is Alg. 3 (Section 4):
 * an inner GMRES on the sparsified system C v = A r (Section 2, eq.
 * preconditioner) preconditioned by the bi-directional sweep, Alg. 2
 * (Section 3.5), built from Alg. 1 (Section 3.4) on horizontal and vertical
 * slabs.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Grid: n x n points x_{i,j} = (h (i+1), h (j+1)), 0 <= i, j < n
 *   (Section 2, 0-based).  A grid vector is stored row by row, x fastest:
 *   element (i, j) at index j*n + i (the global ordering of Section 3.2).
 * - Complex vectors are interleaved (re, im) doubles: a grid vector is
 *   2*n*n doubles; a batch of `batch` vectors is contiguous, stride 2*n*n.
 * - Unless stated otherwise pointers are DEVICE pointers (HIP device memory
 *   on the plan's device).  The caller owns them; the library never keeps
 *   them after the call returns.
 * - All device work is enqueued on the plan's stream (a hipStream_t passed
 *   as void*, NULL for the default stream).  ls_apply, ls_stencil_*,
 *   ls_slab_solve, ls_sweep and ls_bidirectional return without
 *   synchronising; ls_precond_apply and ls_solve synchronise (GMRES needs
 *   the inner products on the host).
 * - A plan is not re-entrant: one host thread and one stream per plan.
 * - Return value: LS_OK or an error code; on error ls_last_error() gives a
 *   message (per thread).  No C++ exception crosses this ABI.  Outputs are
 *   unspecified after an error other than LS_ENOCONV.
 */
#ifndef LS_MI355X_H
#define LS_MI355X_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ls_plan ls_plan;

typedef enum {
  LS_OK = 0,
  LS_EINVAL = 1,      /* bad argument (size, pointer, option) */
  LS_ENOMEM = 2,      /* device allocation failed */
  LS_EDEVICE = 3,     /* a HIP call failed */
  LS_ENOCONV = 4,     /* GMRES hit its iteration limit; outputs hold the last iterate */
  LS_ESINGULAR = 5,   /* a zero or non-finite pivot in a slab factorisation */
  LS_EUNSUPPORTED = 6 /* valid request outside what the library implements */
} ls_status;

/* Arithmetic of the on-line stage.
 * LS_FP64: everything in FP64.
 * LS_FP32_REFINE: FP32 FFT convolution, stencils, slab solves and sweeps
 *   (slab factors computed in FP64, stored in FP32), FP64 inner products and
 *   Hessenberg least squares, and an FP64 iterative-refinement loop around
 *   an FP32 flexible GMRES (residuals f - H u in FP64).  The flexible outer
 *   loop the paper suggests (Section 6) is what lets the preconditioned
 *   solve run in reduced precision. */
enum { LS_FP64 = 0, LS_FP32_REFINE = 1 };

/* Inner preconditioner used inside Alg. 3. */
enum {
  LS_PREC_BD = 0,   /* Alg. 2, bi-directional sweep (the paper's choice) */
  LS_PREC_PT1 = 1,  /* Alg. 1 on horizontal slabs only (one direction) */
  LS_PREC_NONE = 2  /* inner GMRES without preconditioner */
};

typedef struct {
  int slabs;             /* L, number of layers per direction; 0 = n/64 (at least 1) */
  int ext;               /* extension of each layer in grid rows (Section 5: 10) */
  double inner_tol;      /* inner GMRES relative tolerance (Alg. 3: 1e-3) */
  int max_outer;         /* outer flexible-GMRES iteration limit (no restart) */
  int max_inner;         /* inner GMRES iteration limit */
  double shift_c;        /* complex shift in the cut-off region, omega^2 sigma = shift_c*omega (Section 3.3) */
  int precision;         /* LS_FP64 or LS_FP32_REFINE */
  int precond;           /* LS_PREC_* */
  int inner_fixed_iters; /* > 0: inner GMRES runs exactly this many iterations;
                          * 1 (Section 6: the inner solve relaxed under the
                          * flexible outer loop) is computed in closed form on
                          * the device, z = (w^H g / w^H w) M g, w = C M g */
  int max_batch;         /* largest `batch` passed to ls_apply / ls_rhs_from_incident */
  double lowp_tol;       /* LS_FP32_REFINE: relative tolerance of each FP32 correction solve */
  int max_refine;        /* refinement sweeps limit (LS_FP32_REFINE) / FP64 restarts limit (LS_FP64) */
  int use_graphs;        /* 1: the inner preconditioner runs as a captured hipGraph */
  int autotune;          /* 1: time the FFT column-pass tile variants at plan creation */
  int fft_variant;       /* autotune 0: FFT column-pass variant to use, 0..7 (0: radix-16 register passes) */
  int sweep;             /* LS_SWEEP_SEQUENTIAL or LS_SWEEP_DECOUPLED (how Alg. 1 runs, one right-hand side) */
  int level0;            /* LS_LEVEL0_AUTO or LS_LEVEL0_DENSE (the one-right-hand-side slab solves' level-0 odd blocks) */
} ls_options;

/* How one application of Alg. 1 (Section 3.4) runs for one right-hand side
 * (ls_options.sweep); both are the same linear operator.
 * LS_SWEEP_SEQUENTIAL: as written, 2L - 1 local solves one after the other,
 *   each waiting for the traces of its neighbour.
 * LS_SWEEP_DECOUPLED: every layer's local solve of its own right-hand side
 *   first (independent), then the traces the sweeps pass between layers by
 *   two short chains of dense products with precomputed trace-transfer maps
 *   (each the restriction of a local Green's function to the two lines a
 *   neighbour reads -- the reduction of the sweep to interface unknowns the
 *   paper's Section 6 names as future work), then every layer's solve with
 *   its trace sources added (independent again): 2L local solves with no
 *   dependence between layers, plus the chains.  Plan creation then also
 *   builds the maps: 4n local solves per layer, three 2n x 2n maps per layer
 *   (n = 1024: 64 MB each in FP64).  Batches of several right-hand sides use
 *   the sequential sweep. */
enum { LS_SWEEP_SEQUENTIAL = 0, LS_SWEEP_DECOUPLED = 1 };

/* The level-0 odd blocks of a slab's block cyclic reduction (Section 3.2's
 * local matrices, built from Section 2's 9-point stencils) are tridiagonal:
 * a point of a grid column couples only to its two vertical neighbours in
 * that column.  LS_LEVEL0_AUTO: the one-right-hand-side solves take those
 * blocks' steps as tridiagonal solves (3q numbers per block read instead of
 * the q^2 of the dense inverse) when every block's solve agrees with its
 * dense inverse at plan creation (relative difference <= 1e-9), else by the
 * dense inverses; LS_LEVEL0_DENSE: always by the dense inverses.
 * ls_plan_info reports which the plan uses. */
enum { LS_LEVEL0_AUTO = 0, LS_LEVEL0_DENSE = 1 };

typedef struct {
  int outer_its;          /* outer flexible-GMRES iterations */
  int inner_its_total;    /* inner GMRES iterations summed over all outer iterations */
  double relres_est;      /* least-squares residual estimate at exit */
  double relres_true;     /* ||f - H u|| / ||f|| recomputed in FP64 at exit */
  int converged;          /* 1 if relres_true <= tol (the recomputed FP64 residual, not the estimate) */
  double t_ms;            /* wall time of this right-hand side */
  int fno_flags;          /* ls_solve_fno only: LS_FNO_* bits of ls_fno.h, else 0 */
} ls_solve_info;

/* Defaults: slabs 0 (n/64), ext 10, inner_tol 1e-3, max_outer 100,
 * max_inner 50, shift_c 0, LS_FP64, LS_PREC_BD, inner_fixed_iters 0,
 * max_batch 1, lowp_tol 1e-5, max_refine 10, use_graphs 1, autotune 1,
 * fft_variant 0, sweep LS_SWEEP_SEQUENTIAL, level0 LS_LEVEL0_AUTO.
 * Never fails. */
void ls_options_default(ls_options* opt);

/* Off-line stage (Section 4.1): builds everything that depends on the
 * medium.  n >= 8 with 2n-1 <= 4096 (the padded FFT side P is the power of
 * two >= 2n-1); h > 0; omega > 0; m: DEVICE pointer to n*n doubles
 * (m(x_{i,j}) at index j*n + i), copied -- the caller keeps ownership.
 * Each extended layer must satisfy q = thickness + extensions <= 96
 * (LS_EUNSUPPORTED otherwise) and each layer must be at least ext rows thick.  opt may be NULL (defaults).
 * stream: hipStream_t as void*; NULL makes the plan create its own blocking
 * stream (ordered with the null stream, and capturable into graphs).  On
 * success *out owns all device memory of the plan.  Steps: kernel samples w and the circulant spectrum (Section 2),
 * stencils alpha/beta (Section 2), slab matrices (Section 3.3) and their
 * block-cyclic-reduction factors (Section 4.1). */
ls_status ls_plan_create(ls_plan** out, int n, double h, double omega, const double* m,
                         const ls_options* opt, void* stream);

/* The off-line stage for another medium on the same grid and frequency:
 * like ls_plan_create with (n, h, omega) taken from src, but the kernel
 * samples, the spectrum and the stencils -- which depend only on (n, h,
 * omega) (Section 2) -- are copied from src instead of recomputed, and
 * src's autotuned FFT variants are reused (when both plans autotune and
 * have the same precision).  Only the medium-dependent part runs: slab
 * assembly and factorisation (Section 4.1, done once per medium).  src must
 * live on the current device; it is only read and may be destroyed
 * afterwards.  m, opt, stream as for ls_plan_create. */
ls_status ls_plan_create_like(ls_plan** out, const ls_plan* src, const double* m, const ls_options* opt,
                              void* stream);

/* Wall times in ms of the off-line stage of this plan (Section 4.1), by
 * step: ms[0] kernel samples and circulant embedding, ms[1] stencils,
 * ms[2] spectrum (2-D FFT and quarter extraction; for ls_plan_create_like
 * the copies from the source plan), ms[3] slab assembly, ms[4] slab
 * factorisation, ms[5] top-of-reduction operators, ms[6] trace-transfer
 * maps (LS_SWEEP_DECOUPLED), ms[7] FFT autotuning, ms[8] the whole plan
 * creation.  Steps are timed with the stream drained between them.  count
 * <= 9 entries are written (more are zeroed).  HOST array. */
ls_status ls_plan_timings(const ls_plan* plan, double* ms, int count);

/* Choices the plan made at creation (Section 4.1 off-line stage): info[0]
 * = 1 when the one-right-hand-side slab solves take the level-0 odd
 * blocks' steps by the tridiagonal elimination (those blocks are
 * tridiagonal: the local matrices of Section 3.2, built from Section 2's
 * 9-point stencils, couple a point of a column only to its two vertical
 * neighbours in that column; every block's elimination agreed with its
 * dense inverse), 0 when they use the dense inverses;
 * info[1] = blocks of the dense top-of-reduction operator of the first slab
 * (0: none); info[2] = the FFT column-pass variant the FP64 operator uses
 * (the autotuner's choice, or opt.fft_variant without autotuning; Section
 * 4.2: the FFT dominates the cost of H); info[3] = the FP32 operator's
 * (-1 on an FP64 plan).  count entries are written (beyond 4: zeros).
 * HOST array; LS_EINVAL for a null plan or array or count < 1. */
ls_status ls_plan_info(const ls_plan* plan, int* info, int count);

/* Frees the plan (synchronises its stream first).  NULL is accepted. */
ls_status ls_plan_destroy(ls_plan* plan);

/* Hv = v + omega^2 G (m . v) for `batch` vectors (Section 2; Section 4.2:
 * zero-padded 2-D FFT convolution with the precomputed spectrum).
 * 1 <= batch <= opt.max_batch.  v == Hv (in place) is allowed. */
ls_status ls_apply(ls_plan* plan, const double* v, double* Hv, int batch);

/* f = -omega^2 G (m . u_I) (Section 2). */
ls_status ls_rhs_from_incident(ls_plan* plan, const double* uI, double* f, int batch);

/* z ~= C^{-1} A r by Alg. 3: inner GMRES on C v = A r, x0 = 0, right-
 * preconditioned by opt.precond, stopping at relative residual inner_tol
 * (or after inner_fixed_iters iterations).  Synchronises.  Returns
 * LS_ENOCONV if the inner limit was hit (z then holds the last iterate). */
ls_status ls_precond_apply(ls_plan* plan, const double* r, double* z, int batch);

/* v ~= C^{-1} g: the sparsified system alone, solved by GMRES (x0 = 0, no
 * restart) right-preconditioned by opt.precond -- Alg. 2 (LS_PREC_BD), Alg. 1
 * one direction (LS_PREC_PT1) or none -- until the least-squares residual
 * estimate is <= tol or after max_its iterations.  This is the solve whose
 * iteration counts and times Section 5.1 compares for the one-directional
 * and bi-directional preconditioners (its Table 2, tol 1e-6).  g, v: DEVICE
 * arrays of `batch` grid vectors, g != v.  info: HOST array of `batch`
 * records or NULL: outer_its = iterations, relres_est = the estimate,
 * relres_true = ||g - C v|| / ||g|| recomputed in FP64, converged = the
 * estimate met tol.  FP32 plans run the iteration in FP32 (inner products
 * in FP64).  Synchronises.  LS_ENOCONV if some right-hand side hit max_its
 * (v then holds the last iterate). */
ls_status ls_sparse_solve(ls_plan* plan, const double* g, double* v, int batch, double tol, int max_its,
                          ls_solve_info* info);

/* u ~= H^{-1} f: the on-line stage of Section 4 -- the outer GMRES on the
 * discrete Lippmann-Schwinger system H u = f of Section 2, preconditioned by
 * Alg. 3 (ls_precond_apply), run as the flexible GMRES that Section 6
 * proposes (x0 = 0, no restart) until the least-squares residual estimate
 * is <= tol.  The FP64 residual ||f - H u|| / ||f|| is then recomputed; a
 * right-hand side whose estimate met tol but whose recomputed residual did
 * not is restarted from its iterate (FP64 corrections d ~ H^{-1}(f - H u),
 * at most max_refine).
 * LS_FP32_REFINE plans: FP64 refinement sweeps r = f - H u, each solving
 * H d = r with the FP32 flexible GMRES to max(lowp_tol, tol/||r||) and
 * adding d, until ||f - H u|| / ||f|| <= tol; f and u stay FP64.
 * f, u: DEVICE arrays of `batch` grid vectors, f != u; batch >= 1 (worked
 * through max_batch at a time); tol > 0.
 * info: HOST array of `batch` records or NULL; info[b].converged is 1 iff
 * the recomputed residual is <= tol.  Synchronises.
 * LS_ENOCONV if some right-hand side ends above tol (max_outer or
 * max_refine reached); u then holds the last iterate. */
ls_status ls_solve(ls_plan* plan, const double* f, double* u, int batch, double tol,
                   ls_solve_info* info);

/* Several independent media (plans, possibly of different n) solved at
 * once: one host thread per plan calls ls_solve on that plan's stream, so
 * the GPU runs the plans' kernels concurrently (the paper solves 64
 * incident waves per medium, Section 5).  Plans must be distinct and use
 * distinct streams.  f[i], u[i]: DEVICE arrays of batch[i] grid vectors of
 * plans[i]; info[i]: HOST arrays or info == NULL.  Returns the first
 * error other than LS_ENOCONV, else LS_ENOCONV if any plan did not
 * converge, else LS_OK. */
ls_status ls_solve_multi(ls_plan* const* plans, int count, const double* const* f,
                         double* const* u, const int* batch, double tol,
                         ls_solve_info* const* info);

const char* ls_status_str(ls_status s);
const char* ls_last_error(void);

/* ------------------------------------------------------------------------
 * Step-level entry points.  Each exposes one step of the path above on the
 * plan's device data, so it can be checked on its own.
 * ---------------------------------------------------------------------- */

/* Geometry: P (padded FFT side), L (slabs per direction), the padded side
 * and the number of complex entries of the stored spectrum. */
ls_status ls_plan_dims(const ls_plan* plan, int* P, int* L, int* spec_side);

/* Quadrature weights w_q, q in [-(n-1), n-1]^2 (Section 2: h^2 G(h|q|) off
 * the diagonal, the modified trapezoidal weight at q = 0), written to the
 * DEVICE array w of (2n-1)^2 complex, w[(qz+n-1)*(2n-1) + qx+n-1]. */
ls_status ls_get_kernel_samples(ls_plan* plan, double* w);

/* Stored spectrum: S[ky][kx] for 0 <= kx, ky <= P/2 (spec_side = P/2+1),
 * S = (omega^2 / P^2) * FFT2(circulant embedding of w) (Section 2).  The
 * full spectrum is even in kx and ky and symmetric in (kx, ky), so this
 * quarter holds all of it.  DEVICE array of spec_side^2 complex. */
ls_status ls_get_spectrum(ls_plan* plan, double* S);

/* Stencil tables alpha and beta (Section 2), HOST arrays of 81 complex each,
 * index ((tz*3 + tx)*3 + dz+1)*3 + dx+1 with the type per axis
 * 0 = low edge (index 0), 1 = interior, 2 = high edge (index n-1). */
ls_status ls_get_stencils(ls_plan* plan, double* alpha, double* beta);

/* y = A r and y = C v (Section 2: C = A + omega^2 B D on A's pattern). */
ls_status ls_stencil_A(ls_plan* plan, const double* r, double* y, int batch);
ls_status ls_stencil_C(ls_plan* plan, const double* v, double* y, int batch);

/* Layer geometry (Section 3.1): orient 0 = horizontal layers (rows of
 * constant z), 1 = vertical layers (columns).  Writes lims[4] = {a, b, z0,
 * z1}: layer lines [a, b], extended lines [z0, z1] along the slab's short
 * axis.  HOST array. */
ls_status ls_slab_info(const ls_plan* plan, int orient, int slab, int* lims);

/* FP32 operator of an LS_FP32_REFINE plan: Hv = v + omega^2 G (m . v) with
 * interleaved complex FP32 vectors [batch][n][n] (Section 2; the
 * refinement loop's low-precision operator).  LS_EINVAL on FP64 plans. */
ls_status ls_apply_c64(ls_plan* plan, const float* v, float* Hv, int batch);

/* x = (C^l)^{-1} b for one extended slab (Section 3.3 matrix, factored off
 * line).  b, x: DEVICE arrays of n*q complex in the slab frame
 * [long][short]: element (i, r) at index i*q + r is the grid point at long
 * coordinate i and short coordinate z0 + r (horizontal: x = i, z = z0 + r;
 * vertical: z = i, x = z0 + r).  b == x allowed.  LS_FP32_REFINE plans
 * solve with the FP32 factors (b, x stay FP64 arrays); the same holds for
 * ls_sweep, ls_bidirectional and ls_precond_apply. */
ls_status ls_slab_solve(ls_plan* plan, int orient, int slab, const double* b, double* x);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * slab solve as ls_slab_solve, same arguments, layout and results (the same
 * kernels), but the call allocates nothing.  Its scratch -- the eliminated
 * right-hand sides, plus the FP32 copies of b and x on LS_FP32_REFINE plans
 * or the copy of b when b == x -- lives in one static device array of
 * ls_noalloc_scratch_bytes() bytes (6 MiB, enough for every slab a plan can
 * have: n * q <= 2048 * 96) that each GPU holds until the process ends; its
 * device address is taken once per device by ls_plan_create.  Every call on
 * one GPU shares that array, so calls that overlap on one GPU (other
 * streams, other host threads) race: serialise them.  A slab larger than
 * the array gives LS_EINVAL; the plan's own scratch is not touched. */
ls_status ls_slab_solve_noalloc(ls_plan* plan, int orient, int slab, const double* b, double* x);
size_t ls_noalloc_scratch_bytes(void);

/* v = Preconditioner(g) (Alg. 1) on horizontal (orient 0) or vertical
 * (orient 1) layers; g, v grid vectors, g != v. */
ls_status ls_sweep(ls_plan* plan, int orient, const double* g, double* v);

/* v = BiDirectionalPreconditioner(g) (Alg. 2); g != v. */
ls_status ls_bidirectional(ls_plan* plan, const double* g, double* v);

#ifdef __cplusplus
}
#endif
#endif /* LS_MI355X_H */
