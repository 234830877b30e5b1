/*
 * gevd.h -- C interface of the MI355X (gfx950) dense generalized
 * Hermitian eigensolver  H C = eps S C.
 *
 * The problem is the paper's Eq. (2): H and S are the Hamiltonian and
 * overlap matrices of a non-orthogonal basis, S is Hermitian positive
 * definite, C holds eigenvectors as columns and eps the eigenvalues.  The
 * solve follows the paper's section "Solving the generalized eigenproblem":
 * Cholesky S = U^H U (step 1), inversion U -> U^{-1} (step 2), the two
 * products A = U^{-H} H U^{-1} (step 3), the standard eigenproblem of A, and
 * the back-transformation C = U^{-1} C~.  The standard eigenproblem uses the
 * two-stage route (full -> band -> tridiagonal) that the paper names for
 * subsets of eigenvectors (section "ELPA - Usability"), a divide-and-conquer
 * tridiagonal solver, and back-transformation of only the wanted vectors.
 * Per-step entry points exist because the paper's library offers an
 * interface for each transformation step (section "ELPA").
 *
 * Conventions for every call below
 *  - Matrices are column-major: element (i, j) at p[i + j*ld], ld >= n.
 *  - Real problems use double; complex problems use interleaved
 *    (re, im) doubles, layout-compatible with C99 double _Complex.
 *  - Matrix and vector pointers are DEVICE pointers on the handle's device,
 *    owned by the caller; the library never frees them.
 *  - Work is enqueued on the handle's stream.  Calls that return an info
 *    value computed on the device (positive definiteness) synchronise that
 *    stream before returning; the others return after enqueueing.
 *  - Workspace is owned by the handle: allocated on first use, grown when a
 *    larger problem arrives, released by gevd_destroy.
 *  - Return value: 0 on success; -i when argument i (1-based) is invalid
 *    (checked on the host before any launch); j > 0 when S is not positive
 *    definite at leading minor j (paper: S must not be numerically
 *    singular); or one of the GEVD_E_* codes.
 */
#ifndef GEVD_H
#define GEVD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GEVD_OK 0
#define GEVD_E_NONFINITE (-1001) /* NaN or Inf found in H or S */
#define GEVD_E_NOCONV (-1002)    /* tridiagonal solver failed to converge */
#define GEVD_E_NOMEM (-1003)     /* device memory exhausted */
#define GEVD_E_HIP (-1004)       /* a HIP runtime call failed */
#define GEVD_E_STATE (-1005)     /* call order violated (e.g. no overlap set) */
#define GEVD_E_HANG (-1006)      /* a device-side wait exceeded its bound */
#define GEVD_E_SCRATCH (-1007)   /* request exceeds the fixed scratch of gevd_solve_batched_noalloc */
#define GEVD_E_RANK (-1008)      /* gevd_solve_reduced: fewer retained overlap eigenvectors than nev */

/* Warning bits (gevd_get_warnings): the result is complete and returned.
 * GEVD_W_ILLCOND: the Cholesky factor's diagonal gives cond(S) >=
 * (max |U_ii| / min |U_ii|)^2 > GEVD_ILLCOND_KAPPA.  The paper requires the
 * condition number of S to stay inside the range double precision resolves
 * (about 1e12) for the Cholesky route, and otherwise moves to the basis of
 * S's eigenvectors (gevd_solve_reduced). */
#define GEVD_W_ILLCOND 1
#define GEVD_ILLCOND_KAPPA 1e12

/* Scalar type of a problem. */
#define GEVD_REAL 0    /* real symmetric, double */
#define GEVD_COMPLEX 1 /* complex Hermitian, interleaved double pairs */

/* Options for gevd_set_option. */
#define GEVD_OPT_BAND 1     /* half-bandwidth b of the intermediate band (0 = auto) */
#define GEVD_OPT_TIMING 2   /* 1: record per-phase device times (events) */
#define GEVD_OPT_LEAF 3     /* divide-and-conquer leaf size (0 = auto) */
#define GEVD_OPT_KSTATS 4   /* 1: time kernel families with HIP events (see gevd_get_kernel_stats) */
#define GEVD_OPT_PRECISION 5 /* GEVD_PREC_FP64 (default) or GEVD_PREC_FP32_REFINE */
#define GEVD_OPT_REFINE 6   /* refinement sweeps of the reduced-precision form (0..10, default 2) */
/* GEVD_OPT_PANEL: 1 (default) asks for the persistent full -> band panel
 * kernel (one launch per panel, at most 64 workgroups that synchronise per
 * column and so must all be resident at once).  Within a process, one handle
 * per device holds that route at a time: a call whose handle cannot take it
 * (another handle's solve is using it) runs with one launch per panel
 * column instead, which needs no co-residency, and the owner keeps the route
 * until its work on the device has finished.  0 always uses the per-column
 * launches (set it when several processes share a device).  0 or 1. */
#define GEVD_OPT_PANEL 7
/* GEVD_OPT_GEMM_TILE: -1 (default) picks each matrix product's workgroup
 * tile from its shape; 0..8 forces one tile on every product of this
 * handle's calls (0 = 64x64, 4 = 64x32, 5 = 32x64 with four waves;
 * 6 = 128x128, 7 = 128x64, 8 = 64x128 with eight waves, complex products on
 * eight-wave tiles in the three-product form; 1-3 are four-wave 128x64,
 * 64x128, 128x128).  Results differ only by rounding; meant for tests and
 * measurements. */
#define GEVD_OPT_GEMM_TILE 8
/* GEVD_OPT_STAGES: how the standard eigenproblem is tridiagonalised.  2 (and
 * 0, the default) full -> band -> tridiagonal (two stages, back-transformed
 * through both); 1 one-stage Householder tridiagonalisation (the route the
 * paper ran on GPUs for full spectra, section "ELPA - Usability"): every
 * reflector computed from the panel-corrected column and a memory-bound
 * product with the trailing matrix, rank-2x32 MFMA updates per panel, and a
 * single back-transformation.  The one-stage route always runs in FP64 (the
 * precision form applies to the two-stage route). */
#define GEVD_OPT_STAGES 9

/* Precision forms (GEVD_OPT_PRECISION) of gevd_solve, gevd_solve_resident
 * and gevd_eigh.  FP32_REFINE: the products of the full -> band reduction
 * and of the stage-1 back-transformation run on the FP32 matrix cores
 * (operands rounded to FP32, FP32 accumulation; A itself stays FP64); the
 * Cholesky, inversion, the two products forming A, band -> tridiagonal, the
 * divide-and-conquer solve and the bulge-reflector back-transformation stay
 * FP64; then the nev wanted pairs are refined in FP64 against A by the
 * Ogita-Aishima correction restricted to their subspace (G = X^H X,
 * M = X^H A X, X <- X + X E), GEVD_OPT_REFINE sweeps.  eval[0..nev) holds the
 * refined values (ascending); eval[nev..n) the values of the reduced-
 * precision stages.  The refinement cannot restore components that the
 * FP32 stages lost outside the wanted subspace: for an ill-conditioned S
 * (large ||A||, eigenvalues clustered relative to it) the result stays near
 * FP32 accuracy. */
#define GEVD_PREC_FP64 0
#define GEVD_PREC_FP32_REFINE 1

/* Kernel families reported by gevd_get_kernel_stats. */
#define GEVD_K_GEMM 0       /* MFMA matrix products (all shapes, both scalar types) */
#define GEVD_K_PANEL 1      /* full -> band panel columns */
#define GEVD_K_CHASE 2      /* band -> tridiagonal bulge chasing */
#define GEVD_K_BACKCHASE 3  /* back-transformation through the bulge reflectors */
#define GEVD_K_DC 4         /* divide-and-conquer (leaves, merge steps; merge products count as GEMM) */
#define GEVD_K_OTHER 5      /* everything else (Cholesky diagonal blocks, T factors, copies) */
#define GEVD_K_SMALL 6      /* batched small problems (one fused persistent launch per group) */
#define GEVD_K_GEMM32 7     /* matrix products of the reduced-precision form (FP32 matrix cores) */
#define GEVD_NKFAM 8

/* Phases reported by gevd_get_timings (milliseconds, last solve). */
#define GEVD_PH_CHOLESKY 0  /* S = U^H U */
#define GEVD_PH_INVERT 1    /* U -> U^{-1} */
#define GEVD_PH_MULTIPLY 2  /* A = U^{-H} H U^{-1} */
#define GEVD_PH_BAND 3      /* full -> band */
#define GEVD_PH_TRIDIAG 4   /* band -> tridiagonal */
#define GEVD_PH_SOLVE 5     /* tridiagonal divide-and-conquer */
#define GEVD_PH_BACK2 6     /* back-transform through band -> tridiagonal */
#define GEVD_PH_BACK1 7     /* back-transform through full -> band */
#define GEVD_PH_MULT 8      /* C = U^{-1} C~ */
#define GEVD_NPHASE 9

typedef struct gevd_ctx *gevd_handle;

/* Create a handle bound to HIP device `device`, using the default stream.
 * *h receives the handle.  Errors: -1 (h NULL), GEVD_E_HIP. */
int gevd_create(gevd_handle *h, int device);

/* Release the handle and all workspace it owns (synchronises its stream). */
int gevd_destroy(gevd_handle h);

/* Use `stream` (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream)
 * for all following work of this handle. */
int gevd_set_stream(gevd_handle h, void *stream);

/* Set an integer option (GEVD_OPT_*).  Band width must be 0 or in [8, 64]. */
int gevd_set_option(gevd_handle h, int option, int value);

/* Human-readable text for a return code (static storage). */
const char *gevd_strerror(int code);

/* Bytes of device workspace the handle holds for a (dtype, n, nev) solve;
 * a caller admitting work by memory footprint adds its own n x n H, S and
 * n x nev C.  Host-only computation.  gevd_workspace_bytes assumes the
 * default options; gevd_handle_workspace_bytes uses the handle's (band
 * width, leaf size, precision form: FP32_REFINE adds a copy of A and the
 * refinement blocks). */
size_t gevd_workspace_bytes(int dtype, int n, int nev);
size_t gevd_handle_workspace_bytes(gevd_handle h, int dtype, int n, int nev);

/* Whole generalized solve (paper Eq. (2) by its three reduction steps and
 * the back-transformation).
 *  dtype     GEVD_REAL or GEVD_COMPLEX
 *  n         order of H and S (>= 1)
 *  nev       number of wanted eigenpairs, the nev algebraically smallest
 *            (1 <= nev <= n)
 *  H, ldh    upper triangle read (the strictly lower part is ignored);
 *            overwritten (used as workspace)
 *  S, lds    upper triangle read; on return its upper triangle holds U with
 *            S = U^H U; the strictly lower part is clobbered
 *  eval      n doubles: all eigenvalues in ascending order
 *  C, ldc    n x nev: eigenvectors of the nev smallest eigenvalues, with
 *            C^H S C = I
 * Synchronises the stream.  Returns 0, -i, j > 0 (S not positive definite
 * at minor j; nothing else is computed), or GEVD_E_*. */
int gevd_solve(gevd_handle h, int dtype, int n, int nev, void *H, int ldh, void *S, int lds,
               double *eval, void *C, int ldc);

/* Warning bits (GEVD_W_*) of the last gevd_solve or gevd_set_overlap, and
 * through kappa_lower (may be NULL) the lower bound of cond(S) it computed
 * from the Cholesky factor (0 before any).  Host-only. */
int gevd_get_warnings(gevd_handle h, double *kappa_lower);

/* Generalized solve for an ill-conditioned overlap: the route the paper
 * describes at the end of its section "Solving the generalized
 * eigenproblem".  S = D diag(sigma) D^H is diagonalised; the eigenvectors
 * with sigma_i < delta (the paper: typically delta <= 1e-5) are omitted; in
 * the basis X = D_r diag(sigma_r)^(-1/2) of the m retained ones the problem
 * becomes the standard eigenproblem of X^H H X (order m), solved by the
 * two-stage route; C = X c~ (so C^H S C = I).
 *  dtype, n, nev  as gevd_solve; nev <= m is required
 *  delta     retention threshold (> 0, finite)
 *  H, ldh    upper triangle read; clobbered
 *  S, lds    upper triangle read; not modified
 *  eval      n doubles: eval[0..m) the m eigenvalues of the reduced problem
 *            ascending; eval[m..n) is not written
 *  C, ldc    n x nev S-orthonormal eigenvectors of the nev smallest
 *  m         host int (may be NULL): number of retained eigenvectors
 *  sigma     device, n doubles (may be NULL): the eigenvalues of S
 *            ascending (for the caller's condition report)
 * Synchronises.  Returns 0, -i, GEVD_E_RANK (m < nev; m and sigma are
 * still written), or GEVD_E_*. */
int gevd_solve_reduced(gevd_handle h, int dtype, int n, int nev, double delta, void *H, int ldh, const void *S,
                       int lds, double *eval, void *C, int ldc, int *m, double *sigma);

/* Density matrix from the eigenvectors (the paper's density-matrix
 * section: P_ij = sum_l f_l conj(c_li) c_lj, with c_l the l-th eigenvector,
 * i.e. column l of C, and f_l its occupation number) and, if Q is not NULL,
 * its energy-weighted counterpart Q_ij = sum_l f_l eps_l conj(c_li) c_lj
 * (the two matrices ELSI returns to DFT codes).
 *  C, ldc   n x k eigenvectors (device), e.g. gevd_solve's C
 *  f        device, k occupation numbers
 *  eval     device, k eigenvalues (read only when Q is not NULL)
 *  P, ldp   n x n Hermitian result, both triangles written
 *  Q, ldq   n x n (or NULL)
 * P = conj(C) diag(f) C^T is formed on the matrix cores from its upper
 * tiles and mirrored.  Returns after enqueueing; 0 or -i. */
int gevd_density(gevd_handle h, int dtype, int n, int k, const void *C, int ldc, const double *f,
                 const double *eval, void *P, int ldp, void *Q, int ldq);

/* SCF residency.  In a self-consistent-field loop S is fixed while H changes
 * every iteration, so the overlap is factored once: gevd_set_overlap reads
 * the upper triangle of S (not modified), computes U (S = U^H U) and keeps
 * U^{-1} in device memory owned by the handle (n*n scalars, released by
 * gevd_destroy or the next gevd_set_overlap).  Synchronises; returns 0, -i,
 * j > 0 if S is not positive definite at minor j, or GEVD_E_*. */
int gevd_set_overlap(gevd_handle h, int dtype, int n, const void *S, int lds);

/* Generalized solve with the overlap of the last gevd_set_overlap: the
 * steps of gevd_solve after the inversion (the two products, the standard
 * eigenproblem, C = U^{-1} C~).  H (upper triangle read) is clobbered.
 * Returns GEVD_E_STATE if no overlap is set.  Synchronises. */
int gevd_solve_resident(gevd_handle h, int nev, void *H, int ldh, double *eval, void *C, int ldc);

/* Step 1: Cholesky factorisation S = U^H U in place (upper triangle read
 * and overwritten with U; the strictly lower triangle is clobbered).
 * Synchronises the stream; returns 0 or j > 0 for a non positive definite
 * leading minor j. */
int gevd_cholesky(gevd_handle h, int dtype, int n, void *S, int lds);

/* Step 2: Uinv = U^{-1} for the upper triangular U (upper triangle of U
 * read).  Uinv receives the full n x n matrix with exact zeros below the
 * diagonal.  U and Uinv must not overlap. */
int gevd_invert_upper(gevd_handle h, int dtype, int n, const void *U, int ldu, void *Uinv, int ldi);

/* Step 3: A = Uinv^H H Uinv (the paper's two products), H read from its
 * upper triangle and clobbered (its diagonal is halved: the products are
 * formed as A = Z + Z^H, Z = Uinv^H (M Uinv), M = triu(H) - diag(H)/2, which
 * takes n^3 real flops instead of the 4n^3/3 of H Uinv then Uinv^H (H Uinv)),
 * Uinv upper triangular (lower part ignored).  A receives the full
 * Hermitian matrix; it may be H itself but must not overlap Uinv. */
int gevd_reduce(gevd_handle h, int dtype, int n, void *H, int ldh, const void *Uinv, int ldi, void *A,
                int lda);

/* Standard Hermitian eigenproblem A z = eps z by full -> band ->
 * tridiagonal -> divide-and-conquer -> back-transformation.
 *  A, lda   full Hermitian matrix (both triangles read); clobbered
 *  eval     n doubles, all eigenvalues ascending
 *  Z, ldz   n x nev orthonormal eigenvectors of the nev smallest */
int gevd_eigh(gevd_handle h, int dtype, int n, int nev, void *A, int lda, double *eval, void *Z, int ldz);

/* Back-transformation C = Uinv Ct (n x nev), Uinv upper triangular. */
int gevd_backtransform(gevd_handle h, int dtype, int n, int nev, const void *Uinv, int ldi, const void *Ct,
                       int ldct, void *C, int ldc);

/* First stage only: full Hermitian A (clobbered) -> band of half-bandwidth
 * b (the handle's band option, see gevd_get_band).  The band is returned
 * in lower band storage: Bd[(i - j) + j*ldb] = B[i, j] for 0 <= i-j <= b,
 * ldb >= b + 1. */
int gevd_band(gevd_handle h, int dtype, int n, void *A, int lda, void *Bd, int ldb);

/* Half-bandwidth the handle uses for order n and dtype. */
int gevd_get_band(gevd_handle h, int dtype, int n);

/* Both reduction stages: full Hermitian A (clobbered) -> real symmetric
 * tridiagonal (d: n diagonal, e: n-1 subdiagonal), device doubles. */
int gevd_tridiagonalize(gevd_handle h, int dtype, int n, void *A, int lda, double *d, double *e);

/* Real symmetric tridiagonal eigenproblem by divide-and-conquer.
 *  d, e     device doubles (n, n-1); not modified
 *  eval     n eigenvalues ascending
 *  Z, ldz   n x nev real orthonormal eigenvectors of the nev smallest */
int gevd_stedc(gevd_handle h, int n, int nev, const double *d, const double *e, double *eval, double *Z,
               int ldz);

/* Per-phase device times (ms) of the last gevd_solve or gevd_eigh when
 * GEVD_OPT_TIMING is on; ms must hold nphase doubles.  Synchronises. */
int gevd_get_timings(gevd_handle h, double *ms, int nphase);

/* Accumulated accounting of one kernel family (GEVD_K_*) since the option
 * GEVD_OPT_KSTATS was enabled or the last gevd_reset_kernel_stats: number
 * of launches, their summed device time in ms (HIP events recorded on the
 * launch stream around each launch), and the algorithmic flops those
 * launches perform (real-arithmetic count, a complex multiply-add counting
 * 8; triangular operands counted by their nonzeros).  Synchronises. */
int gevd_get_kernel_stats(gevd_handle h, int family, long long *launches, double *ms, double *flops);
int gevd_reset_kernel_stats(gevd_handle h);

/* ------------------------------------------------------------------
 * Batched small problems.  The paper's k-points and spin channels are
 * independent generalized problems of the same kind (introduction; section
 * "ELPA - Usability"); when each has order n <= 512 one GPU solves many of
 * them at once.  A batch is grouped by scalar type and order bucket
 * (n <= 64, 128, 256, 512); each group is one launch of a persistent fused
 * kernel whose workgroups take problems from a queue and run the whole
 * solve of gevd_solve on each one (Cholesky, the reduction by two
 * triangular solves, one-stage Householder tridiagonalisation, all
 * eigenvalues by bisection and the wanted eigenvectors by twisted
 * factorisations, implicit QL with all vectors as the fallback,
 * back-transformation).  Launch shapes (lanes per workgroup, workgroups
 * per CU) come from the handle's table (gevd_set_batch_shape /
 * gevd_tune_batched) or a default table (the shapes the tuner chose on
 * MI355X, bounded by the occupancy the device reports).
 */
typedef struct {
    int dtype;     /* GEVD_REAL or GEVD_COMPLEX */
    int n;         /* order, 1 <= n <= 512 */
    int nev;       /* wanted eigenpairs (the smallest), 1 <= nev <= n */
    void *H;       /* device, n x n, upper triangle read; clobbered */
    int ldh;       /* >= n */
    void *S;       /* device, n x n, upper triangle read; on return it holds U
                      (S = U^H U) and the strictly lower triangle U^H */
    int lds;       /* >= n */
    double *eval;  /* device, n eigenvalues ascending */
    void *C;       /* device, n x nev eigenvectors, C^H S C = I */
    int ldc;       /* >= n */
    int flags;     /* 0 or GEVD_PROBLEM_FACTORED */
} gevd_problem;

/* S already holds U (upper) and U^H (strictly lower) from an earlier solve
 * of this same S by the batched entry points: the Cholesky step is skipped
 * (SCF iterations with a fixed overlap reuse the factor). */
#define GEVD_PROBLEM_FACTORED 1

typedef struct gevd_batch_s *gevd_batch;

/* Solve `count` problems (array of descriptors in host memory) and write
 * each problem's status to info[i] (host array of count ints): 0, j > 0 if
 * S is not positive definite at minor j, GEVD_E_NONFINITE, or
 * GEVD_E_NOCONV; a failed problem leaves its eval and C undefined and does
 * not affect the others.  Allocates and frees a small plan (descriptors,
 * per-workgroup n x n scratch), synchronises.  Returns 0 when the launches
 * ran, -3 if any descriptor is invalid (nothing is launched), or GEVD_E_*. */
int gevd_solve_batched(gevd_handle h, int count, const gevd_problem *probs, int *info);

/* A reusable batch for repeated solves on the same buffers (an SCF loop
 * rewrites H in place each iteration): the descriptors are uploaded and the
 * launches captured into a HIP graph once; gevd_batch_run replays the graph
 * on the handle's current stream.  If info is not NULL it receives the
 * per-problem status (as above) and the call synchronises; otherwise it
 * returns after enqueueing.  The launch shapes are those of the handle when
 * the batch was created.  Errors: as gevd_solve_batched. */
int gevd_batch_create(gevd_handle h, int count, const gevd_problem *probs, gevd_batch *b);
int gevd_batch_run(gevd_batch b, int *info);
/* gevd_batch_run without any host synchronisation: replays the graph on the
 * handle's current stream, then copies the per-problem status (count ints,
 * problem i at info_dev[i], values as for gevd_solve_batched) into the
 * caller's device array on the same stream.  Returns once both are
 * enqueued; the statuses, eigenvalues and vectors are valid when the stream
 * reaches that point (an event, or any later work on the stream, may consume
 * them).  info_dev is the caller's, count ints in device memory.  Errors: -1
 * null batch, -2 null info_dev, GEVD_E_HIP. */
int gevd_batch_run_async(gevd_batch b, int *info_dev);
int gevd_batch_destroy(gevd_batch b);

/* Launch shape of the bucket holding order n: threads per workgroup (64,
 * 128, 256, 512 or 1024; 0 restores the default) and workgroups per CU. */
int gevd_set_batch_shape(gevd_handle h, int dtype, int n, int threads, int wg_per_cu);
int gevd_get_batch_shape(gevd_handle h, int dtype, int n, int *threads, int *wg_per_cu);

/* Tune the bucket holding order n: time every candidate shape on `count`
 * synthetic problems of the bucket's largest order (device-generated,
 * diagonally dominant S) and keep the fastest in the handle's table; the
 * chosen shape is returned through threads / wg_per_cu (either may be NULL).
 * Allocates its own buffers; synchronises. */
int gevd_tune_batched(gevd_handle h, int dtype, int n, int count, int *threads, int *wg_per_cu);

/* ------------------------------------------------------------------
 * For callers that cannot allocate device memory while they run (tight
 * serving loops, harnesses that forbid hipMalloc): gevd_solve_batched with
 * no allocation.  Same arguments, results and per-problem status as
 * gevd_solve_batched (the same fused kernel; a problem's result does not
 * depend on the launch shape, so both give identical bits), but every
 * device buffer it needs beyond the caller's H, S, eval and C (descriptors,
 * status words, queue counters, per-workgroup Z slots) lives in one fixed
 * array of GEVD_NOALLOC_SCRATCH_BYTES per device, resolved by gevd_create
 * and held until the process ends; host staging lives in the handle.  It
 * calls no hipMalloc/hipFree and creates no streams or events.
 *  - count must not exceed GEVD_NOALLOC_MAX_COUNT: otherwise GEVD_E_SCRATCH
 *    is returned before anything is launched.
 *  - The scalar types run one after the other on the handle's stream, and a
 *    group's persistent grid is bounded by the Z slots that fit (n <= 512:
 *    2 MiB per slot), so large orders run on fewer workgroups than in
 *    gevd_solve_batched.
 *  - Calls on one device share that device's array: the library serialises
 *    them within a process (a host lock held until the call has
 *    synchronised), and each call rewrites every part of the array it
 *    reads (counters are cleared by a kernel before use).
 * Returns 0 when the launches ran (per-problem status in info), -i for an
 * invalid argument i (-3: a descriptor), GEVD_E_SCRATCH, or GEVD_E_*. */
#define GEVD_NOALLOC_SCRATCH_BYTES (64u << 20)
#define GEVD_NOALLOC_MAX_COUNT 2048
int gevd_solve_batched_noalloc(gevd_handle h, int count, const gevd_problem *probs, int *info);

#ifdef __cplusplus
}
#endif
#endif /* GEVD_H */
