/*
 * ks.h -- C-ABI of the MI355X (gfx950) generalized Kohn-Sham eigensolver and
 * density build.
 *
 * The library solves, per k-point, the generalized Hermitian-definite
 * eigenproblem H C = S C eps of a numerical-atomic-orbital Hamiltonian
 * (paper Sec. 2, the equation after the basis expansion, and its Bloch form
 * per k-point), in the collinear form (real symmetric or complex Hermitian,
 * order n) and in the noncollinear spinor form (complex Hermitian H of order
 * 2n in spin blocks [[aa, ab], [ba, bb]], overlap diag(S, S) with S of order
 * n; paper Sec. 2 end and the definitions of H_NC, C_NC, S_NC in Sec. 3.2).
 * It then forms the Fermi-Dirac occupations, the chemical potential (one mu
 * common to all k-points, from the electron count), the band energy and the
 * density matrix (paper Sec. 2 density-matrix equation and its spinor form;
 * Parts 3-4 of the collinear flow of Sec. 3.1, Parts 4-5 of Sec. 3.2).
 *
 * Route: Cholesky S = L L^H; A = L^-1 H L^-H (spinor form: with L applied to
 * each spin block, i.e. (I2 (x) L)); blocked Householder tridiagonalisation
 * A = Q T Q^H; divide-and-conquer eigensolver of T; back-transform
 * C = L^-H Q Z.  Plans created with KS_PLAN_LOWDIN take the paper's own route
 * instead (eigen-decomposition of S, V = U s^-1/2, H' = V^H H V, C = V C'),
 * optionally dropping the near-null directions of an overcomplete basis.
 * Further entry points form the energy-density matrix C diag(f eps) C^H and
 * the Bloch sums H(k), S(k) of real-space blocks for a batch of k-points.
 * Everything runs in HIP kernels on the device, asynchronously on the plan's
 * stream; the host only validates arguments and enqueues.
 *
 * Conventions shared by all entry points
 *   - Matrices are row-major with a row stride ("leading dimension") in
 *     elements; complex matrices interleave (re, im) doubles exactly like
 *     C99 double complex and torch.complex128.
 *   - Every matrix/vector pointer is DEVICE memory owned by the caller, unless
 *     a parameter says "host".  The library never frees caller memory.
 *   - H and S must be Hermitian; only their LOWER triangle (diagonal included)
 *     is read.  Outputs rho, grad_H, grad_S are written full (both triangles).
 *   - Eigenvectors are the COLUMNS of C (C[:, i] belongs to eps[i]), eps is
 *     ascending per k-point, and C^H S_NC C = I.
 *   - Batches of k-points are contiguous: matrix b of H/C/rho/grad_H starts at
 *     b * order * ld_h elements, of S/grad_S at b * n * ld_s, vectors at
 *     b * order.
 *   - The density convention is rho = C f C^H, i.e. rho_lm = sum_i f_i c_li
 *     conj(c_mi); the paper's n_lm = sum_i f_i conj(c_li) c_mi equals conj(rho_lm)
 *     (spinor blocks likewise).  Occupations include the spin factor g
 *     (g = 2 collinear, g = 1 noncollinear), so 0 <= f <= g and
 *     sum_k w_k tr(rho_k S_NC,k) = n_electrons.
 *   - Argument errors are returned synchronously BEFORE any device work.
 *     Numerical failures found on the device (non-positive pivot of S,
 *     non-finite input, no convergence, occupied states outside the computed
 *     window) are recorded in the plan's device info word and read back with
 *     ks_plan_get_info; outputs are undefined after such a failure.
 *   - A plan is used by one host thread at a time.
 */
#ifndef KS_H
#define KS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KS_OK = 0,
    KS_ERR_INVALID_ARG = 1,     /* bad pointer, size, stride, flag or range       */
    KS_ERR_NOT_POSDEF = 2,      /* S has a non-positive pivot (info = column)     */
    KS_ERR_NO_CONVERGENCE = 3,  /* an iterative step hit its iteration cap        */
    KS_ERR_ELECTRON_COUNT = 4,  /* n_electrons <= 0 or above g * order            */
    KS_ERR_WINDOW = 5,          /* occupied states outside the eigenvector window */
    KS_ERR_NONFINITE = 6,       /* NaN or Inf in H or S                           */
    KS_ERR_ALLOC = 7,           /* workspace does not fit in device memory        */
    KS_ERR_HIP = 8,             /* a HIP runtime call failed                      */
    KS_ERR_NOT_SUPPORTED = 9    /* valid but unsupported combination              */
} ks_status;

enum { KS_REAL64 = 0, KS_COMPLEX128 = 1 };           /* element type of H, S, C, rho */
enum { KS_COLLINEAR = 0, KS_NONCOLLINEAR = 1 };      /* spin form                    */
enum { KS_FP64 = 0, KS_MIXED = 1 };                  /* arithmetic of the solve      */
/* Plan flags.  KS_PLAN_GRAPH: ks_gevd captures its launch sequence from the
 * plan stream into a HIP graph the first time it sees an argument set (H, S,
 * eps, C, il, iu, flags) and replays the graph while the same set repeats; a
 * different set is captured afresh.  Needs a non-NULL stream.  The batched
 * launches (all k-points of the plan in each kernel) are the same either way,
 * so results do not depend on the flag. */
enum { KS_PLAN_GRAPH = 1u,
       /* KS_PLAN_AUTOTUNE: at ks_plan_create, time the candidate tile shapes of
        * the tridiagonalisation's symmetric product (tiles per workgroup) on the
        * plan's own order and batch, and keep the fastest (synchronous, a few
        * milliseconds; without the flag a fixed default is used).  The choice
        * changes only the grouping of partial sums, not the algorithm. */
       KS_PLAN_AUTOTUNE = 2u,
       /* KS_PLAN_LOWDIN: ks_gevd takes the paper's own route (Sec. 3.1 Parts
        * 2-1..2-5, Sec. 3.2 Parts 3-1..3-6) instead of the Cholesky one:
        * U^H S U = s by the same Hermitian eigensolver (tridiagonalisation,
        * divide and conquer, back-transform) on S, V = U s^-1/2,
        * H' = V_NC^H H V_NC with V_NC = diag(V, V), H' C' = C' eps, C = V_NC C'.
        * KS_REUSE_S keeps V (cycles 2 onwards skip Parts 2-1 and 2-2).  A
        * non-positive eigenvalue of S gives KS_ERR_NOT_POSDEF with info = the
        * number of eigenvalues <= 0.  Spinor plans hold a second, collinear
        * plan of order n for the eigenproblem of S (its workspace is included
        * in ks_plan_workspace_bytes).  Not with KS_MIXED (KS_ERR_NOT_SUPPORTED).
        * Results equal the Cholesky route's up to rounding: eps, rho and the
        * occupied subspace do not depend on the S-orthonormal basis. */
       KS_PLAN_LOWDIN = 4u,
       /* KS_PLAN_TWOSTAGE: the reduced matrix is brought to tridiagonal form in
        * two stages (the two-stage scheme of the paper's CPU solver, Sec. 4, in
        * place of the one-stage Householder reduction whose bandwidth-bound
        * matrix-vector products Sec. 6 names as the limit): panels of 32 columns
        * are factored by Householder QR and the trailing matrix takes two-sided
        * rank-64 updates on the matrix cores, leaving a band of half-bandwidth
        * 32; bulge chasing then reduces the band to tridiagonal form, and the
        * eigenvectors take the chasing reflectors (in groups of 32 sweeps, 16
        * for complex data) before the panel reflectors.  Same outputs as the
        * one-stage route up to rounding.  FP64 only (with KS_MIXED:
        * KS_ERR_NOT_SUPPORTED); the Loewdin route uses it for H' (the
        * eigen-decomposition of S stays one-stage).  Its kernels wait for each
        * other across workgroups, so a plan asks for at most one workgroup per
        * compute unit per waiting launch (orders up to 512 times the compute
        * units, 256 times for complex data, else KS_ERR_NOT_SUPPORTED); a wait
        * that never completes (in the band reduction, the bulge chasing or the
        * chasing reflectors' back-transform) gives up after seconds with
        * KS_ERR_NO_CONVERGENCE. */
       KS_PLAN_TWOSTAGE = 8u,
       /* KS_PLAN_REAL_OVERLAP: on a KS_COMPLEX128 plan, S (still passed in
        * complex storage) is real, as the overlap of real orbitals at the
        * Gamma point is, also in the spinor form diag(S, S) of Sec. 3.2 whose
        * H carries the complex spin-orbit blocks.  The Cholesky factor and its
        * inverse are then formed in real arithmetic, and the products with
        * them (the reduction L^-1 H L^-H, the Cholesky form of Sec. 3.1 Part
        * 2-3, and C = L^-H X, Part 2-5) take the complex matrices as real ones of twice the
        * columns: two real products per complex one instead of three.  An
        * imaginary part other than zero in the lower triangle of S (diagonal
        * included) gives KS_ERR_INVALID_ARG with info = its 1-based row.  No
        * effect on KS_REAL64 plans; the Loewdin route ignores it.  Results
        * equal the complex route's up to rounding. */
       KS_PLAN_REAL_OVERLAP = 16u };
enum { KS_REUSE_S = 1u };                            /* ks_gevd flags                */

typedef struct ks_plan ks_plan; /* opaque: workspace, cached Cholesky factor, info */

typedef struct {
    int32_t n;          /* orbitals per spin block; order = n (collinear) or 2n   */
    int32_t batch;      /* k-points solved together (>= 1, <= 64): every kernel of  */
                        /* the solve takes all of them in one launch, except the   */
                        /* tridiagonalisation (two halves on two streams)          */
    int32_t dtype;      /* KS_REAL64 or KS_COMPLEX128; noncollinear needs complex  */
    int32_t spin;       /* KS_COLLINEAR (g = 2) or KS_NONCOLLINEAR (g = 1)         */
    int32_t precision;  /* KS_FP64 or KS_MIXED (FP32 trailing updates, refined)    */
    int32_t ld_h;       /* row stride of H, C, rho, grad_H; >= order               */
    int32_t ld_s;       /* row stride of S, grad_S; >= n                           */
    void*   stream;     /* hipStream_t every call is enqueued on (NULL = default)  */
    uint32_t flags;     /* plan flags                                              */
} ks_plan_desc;

/* Validate the descriptor, size the workspace for it and allocate it on the
 * current device.  KS_ERR_INVALID_ARG for a bad descriptor (no allocation is
 * attempted), KS_ERR_NOT_SUPPORTED for a valid but unsupported one,
 * KS_ERR_ALLOC if the workspace does not fit.  On success *out owns the
 * workspace until ks_plan_destroy.  A plan for a batch of two or more also
 * owns a side stream (non-blocking, default priority) and two events: the
 * tridiagonalisation runs half of the batch there, forked from and joined
 * back to the plan's stream within each ks_gevd call, so callers order work
 * on the plan's stream alone (KS_ERR_HIP if they cannot be created). */
ks_status ks_plan_create(const ks_plan_desc* desc, ks_plan** out);

/* Free the plan's workspace, side stream and events (synchronizes its streams
 * first).  NULL is a no-op. */
void ks_plan_destroy(ks_plan* plan);

/* Generalized eigen-decomposition of every k-point (paper Sec. 2, H C = S C eps;
 * Sec. 3.2 for the spinor form).
 *   H    [batch][order][ld_h]  lower triangle read
 *   S    [batch][n][ld_s]      lower triangle read; ignored when flags has
 *                              KS_REUSE_S and a previous call factored it
 *   eps  [batch][order]        all eigenvalues, ascending
 *   C    [batch][order][ld_h]  columns 0 .. iu-il hold eigenvectors il .. iu
 *   il, iu  1-based inclusive eigenvector range, 1 <= il <= iu <= order
 *   flags   KS_REUSE_S: S is unchanged since the last call on this plan, reuse
 *           its cached Cholesky factor (the self-consistent cycle after the
 *           first, paper Sec. 5, cycles 2 onwards reuse the overlap work).
 * Device failures: KS_ERR_NOT_POSDEF (info = failing column, 1-based; under
 * KS_PLAN_LOWDIN the number of eigenvalues of S that are <= 0),
 * KS_ERR_NONFINITE, KS_ERR_NO_CONVERGENCE, and under KS_PLAN_REAL_OVERLAP
 * KS_ERR_INVALID_ARG (info = row of an imaginary entry of S) via
 * ks_plan_get_info. */
ks_status ks_gevd(ks_plan* plan, const void* H, const void* S, double* eps, void* C,
                  int32_t il, int32_t iu, uint32_t flags);

/* Occupations, chemical potential, band energy and density matrix (paper Sec. 2
 * density-matrix equation; Part 3 and Part 4 of Sec. 3.1).
 *   eps       [batch][order] eigenvalues from ks_gevd
 *   C         [batch][order][ld_h], columns 0 .. iu-il = eigenvectors il .. iu
 *   n_electrons  total electron count per cell, 0 < n_electrons <= g*order
 *   kT        Fermi-Dirac temperature (Ha), > 0;  f = g / (1 + exp((eps-mu)/kT))
 *   kweights  HOST array [batch] of k weights (sum 1), NULL = uniform 1/batch
 *   rho       [batch][order][ld_h] output, rho_k = C_k f_k C_k^H
 *   mu, eband DEVICE scalars: the common chemical potential (bisection on the
 *             weighted electron count) and sum_k w_k sum_i f_ik eps_ik
 *   occ       DEVICE [batch][order] occupations f_ik, or NULL
 * Device failure KS_ERR_WINDOW if some f_ik > g*1e-15 lies outside [il, iu]. */
ks_status ks_density(ks_plan* plan, const double* eps, const void* C, int32_t il, int32_t iu,
                     double n_electrons, double kT, const double* kweights, void* rho,
                     double* mu, double* eband, double* occ);

/* ks_density for callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation with the same kernels, so the same results bit for bit, but it
 * takes the descriptor the eigenvectors were computed under instead of a plan
 * and allocates nothing.  Its scratch (the occupied-window count, and the
 * occupations and the failure word when occ / info are NULL) is a static
 * device array of 1 MiB per GPU, held until the process ends.
 *   desc     n, batch, dtype, spin, ld_h, stream as for the plan (precision,
 *            ld_s and flags are not used)
 *   info     device int32[2] or NULL: info[0] = ks_status of a failure found on
 *            the device (KS_ERR_WINDOW), 0 if none; info[1] = its detail.  The
 *            call clears it first.  With NULL the word lives in the scratch and
 *            cannot be read back.
 *   other arguments as for ks_density.
 * KS_ERR_ALLOC, before any device work, if occ is NULL and batch * order
 * exceeds 131008 (the occupations would not fit the scratch); argument errors
 * as for ks_density.  All calls on one GPU share its scratch: calls that overlap
 * in time on one GPU (two streams, two host threads) race and must not be
 * issued; consecutive calls on one stream are safe. */
ks_status ks_density_noalloc(const ks_plan_desc* desc, const double* eps, const void* C, int32_t il, int32_t iu,
                             double n_electrons, double kT, const double* kweights, void* rho, double* mu,
                             double* eband, double* occ, int32_t* info);

/* Energy-density matrix E_k = C_k diag(f_k eps_k) C_k^H (paper Sec. 3.1, the
 * Part 4 quantity needed for forces; with H C = S C eps it equals
 * S^-1 H rho, and tr(E S) = E_band per k).  Not positive semi-definite, so it
 * is a scaled product rather than a square-root factorisation.
 *   eps  [batch][order] eigenvalues, C as for ks_density (window il .. iu)
 *   occ  DEVICE [batch][order] occupations f_ik (from ks_density)
 *   edm  [batch][order][ld_h] output, both triangles (exactly Hermitian)
 * Argument errors (null pointers, window outside 1..order) return before any
 * device work; the call is asynchronous on the plan's stream. */
ks_status ks_energy_density(ks_plan* plan, const double* eps, const void* C, int32_t il, int32_t iu,
                            const double* occ, void* edm);

/* Bloch sums X(k) = sum_R X_R exp(i k.R) for every k-point of a plan (paper
 * Sec. 2, the Bloch-sum equations for H(k) and S(k)); complex collinear plans
 * only (KS_ERR_NOT_SUPPORTED otherwise).
 *   nR    number of lattice vectors, 1 <= nR <= 64
 *   R     DEVICE [nR][3] lattice vectors (Bohr)
 *   kvec  DEVICE [batch][3] k-points (1/Bohr)
 *   XR    DEVICE [nR][n][ld_r] real blocks X_R (row-major), ld_r >= n
 *   Xk    DEVICE [batch][n][ld_k] complex128 output, ld_k >= n
 * Only the lower triangle is summed; the upper one is written as its conjugate
 * transpose and the diagonal as its real part, which is X(k) itself when the
 * set of R is closed under negation with X_-R = X_R^T (then X(k) is
 * Hermitian).  Argument errors return before any device work. */
ks_status ks_bloch_sum(ks_plan* plan, int32_t nR, const double* R, const double* kvec, const double* XR,
                       int32_t ld_r, void* Xk, int32_t ld_k);

/* Adjoint of (rho, E_band) with respect to (H, S): given dL/drho (grad_rho,
 * full, may be NULL for zero) and dL/dE_band (grad_eband, DEVICE scalar or
 * NULL for zero), writes grad_H [batch][order][ld_h] and grad_S [batch][n][ld_s]
 * such that dL = sum_k Re tr(grad_H^H dH) + Re tr(grad_S^H dS).  Needs ALL
 * eigenvectors (C from ks_gevd with il = 1, iu = order) and mu, occ from
 * ks_density.  The k weights w_k (which enter E_band and the common mu) are
 * those of the last ks_density call on this plan (uniform 1/batch before the
 * first); nothing else is kept from the forward calls.  Spinor form: grad_S
 * is the sum of the two diagonal spin blocks of the gradient of diag(S, S). */
ks_status ks_density_backward(ks_plan* plan, const double* eps, const void* C, const double* mu,
                              const double* occ, double kT, const void* grad_rho,
                              const double* grad_eband, void* grad_H, void* grad_S);

/* Per-part timing, the analogue of the paper's per-Part GPU time tables (Sec. 5,
 * e.g. the breakdown of Parts 2-1 .. 4 per SCF cycle).  With profiling enabled the
 * plan records HIP events on its stream around each phase below and around every
 * `stride`-th launch of the tridiagonalisation's trailing matrix-vector kernel
 * (the bandwidth-bound half of the eigensolver, Sec. 6).  Profiling adds a few
 * event records per phase; keep it off for plain timing. */
enum {
    KS_PHASE_CHOLESKY = 0, KS_PHASE_REDUCE = 1, KS_PHASE_TRIDIAG = 2, KS_PHASE_DC = 3,
    KS_PHASE_BACKTR = 4, KS_PHASE_DENSITY = 5, KS_PHASE_ADJOINT = 6,
    KS_PHASE_REFINE = 7,      /* KS_MIXED: correction sweeps + subspace step        */
    KS_NPHASE = 8
};
typedef struct {
    double phase_ms[8];       /* summed over the calls since the last read          */
    int64_t phase_calls[8];
    double hemv_ms;           /* summed duration of the sampled kernel launches     */
    int64_t hemv_launches;    /* sampled launches                                   */
    double hemv_bytes;        /* their algorithmic bytes: the lower triangle of the  */
                              /* trailing matrix, read once per launch              */
} ks_profile;

/* enable != 0 turns recording on (stride >= 1), 0 turns it off.  Host-only. */
ks_status ks_plan_set_profiling(ks_plan* plan, int32_t enable, int32_t stride);

/* Synchronize the plan's stream, fill *out with what was recorded since the last
 * read, and clear it. */
ks_status ks_plan_get_profile(ks_plan* plan, ks_profile* out);

/* The tuning knobs of a plan and, under KS_PLAN_AUTOTUNE, what was measured
 * at plan creation on the plan's own buffers and shapes.
 *
 * Symmetric product of the one-stage tridiagonalisation: ms[i] is the time of
 * the timing launches with cand[i] tiles per workgroup summed over the sampled
 * columns, and tiles_per_workgroup the candidate with the least total.  The
 * tridiagonalisation uses, for columns k from seg_first[i] up to
 * seg_first[i+1] - 1 (the last segment up to the end), the candidate
 * seg_tiles[i] that was fastest at the column sampled in that segment.
 *
 * Back-transform and GEMM tiles: backtr_block is the number of reflectors per
 * compact-WY block of the back-transform (128 or 256) and gemm_big_min_k the
 * smallest inner dimension for which a large product takes the 128 x 128
 * tiles (KS_TUNE_NEVER: never, 64 x 64 tiles only).  backtr_ms[b][g] is the
 * time of one back-transform of all eigenvectors with backtr_block = 128 << b
 * and gemm_big_min_k = 256 (g = 0) or KS_TUNE_NEVER (g = 1).
 *
 * Divide and conquer: dc_leaf is the largest leaf of the tear tree (16 or 32),
 * dc_ms[l] the time of one solve of a synthetic tridiagonal of the plan's
 * order with dc_leaf = 16 << l.
 *
 * Without autotuning nseg = 1, every column uses tiles_per_workgroup, the
 * other knobs take their defaults (backtr_block 256 from order 4096 up, 128
 * below; gemm_big_min_k 256; dc_leaf 32) and the times are 0.  from_cache is
 * 1 when the knobs were set by ks_plan_set_tuning, 0 otherwise. */
#define KS_TUNE_SEGMENTS 8
#define KS_TUNE_NEVER 0x7fffffff
typedef struct {
    int32_t tiles_per_workgroup;
    int32_t ncand;
    int32_t cand[4];
    double  ms[4];
    int32_t nseg;
    int32_t seg_first[KS_TUNE_SEGMENTS];
    int32_t seg_tiles[KS_TUNE_SEGMENTS];
    int32_t backtr_block;
    int32_t gemm_big_min_k;
    double  backtr_ms[2][2];
    int32_t dc_leaf;
    double  dc_ms[2];
    int32_t from_cache;
} ks_tuning;
ks_status ks_plan_get_tuning(ks_plan* plan, ks_tuning* out);

/* Set a plan's knobs from a ks_tuning filled by ks_plan_get_tuning on a plan
 * of the same descriptor (for instance one kept in a tuning cache), without
 * timing anything.  Only the knobs are read: tiles_per_workgroup, nseg,
 * seg_first, seg_tiles, backtr_block, gemm_big_min_k and dc_leaf; the measured
 * times are copied for reporting.  KS_ERR_INVALID_ARG (plan unchanged) if a
 * knob is outside its candidates (tiles 2, 4 or 8; 1 <= nseg <=
 * KS_TUNE_SEGMENTS with seg_first[0] = 0 and increasing; backtr_block 128 or
 * 256; gemm_big_min_k >= 16 or KS_TUNE_NEVER; dc_leaf 16 or 32).  Host-side
 * except for re-uploading the divide-and-conquer tree (synchronous); a
 * captured graph of the plan is dropped and captured again on the next call. */
ks_status ks_plan_set_tuning(ks_plan* plan, const ks_tuning* t);

/* KS_MIXED plans: the number of correction sweeps (0 .. 4, default 1) applied
 * to the window's FP32 eigenvectors before the FP64 subspace step.  Each sweep
 * shrinks the window subspace's components along the other eigenvectors by
 * about u32 ||A|| / gap (u32 the FP32 unit roundoff, gap the distance from the
 * window's eigenvalues to the rest of the spectrum).  The subspace step then
 * solves the window's eigenproblem inside the corrected subspace,
 * G = X^H A X with B = X^H X, by two refinement passes on the M x M matrices
 * (a first-order orthonormalising and diagonalising correction between
 * groups of eigenvalues more than 2e-6 max|eps| apart, an exact Jacobi solve
 * inside each closer group, groups of more than 64 taken in pieces of 64);
 * its eigenvalues carry the square of what the sweeps leave.  Host-only;
 * KS_ERR_INVALID_ARG outside the range, KS_ERR_NOT_SUPPORTED on an FP64 plan. */
ks_status ks_plan_set_refinement(ks_plan* plan, int32_t sweeps);

/* KS_PLAN_LOWDIN plans: canonical orthogonalisation of an overcomplete basis
 * (the Loewdin route with the eigenvectors of S whose eigenvalue s_j is at
 * most tau * max(s) left out, so that H' is solved on the span of the rest).
 * 0 <= tau < 1; tau = 0 (the default) keeps every s_j and requires all of
 * them positive, as in the paper.  With tau > 0 the dropped directions stay
 * in the fixed-order solve as placeholders: per matrix, the last
 * nsp * (n - nkeep) eigenvalues all equal sigma = 2 |H'|_F + 1 (above every
 * kept one), their eigenvectors are zero and their occupation is zero; the
 * caller reads nkeep with ks_plan_get_overlap_rank.  Takes effect at the next
 * ks_gevd that decomposes S (not under KS_REUSE_S).  While the V in use was
 * formed with tau > 0, ks_density_backward returns KS_ERR_NOT_SUPPORTED (its
 * formulas assume a complete S-orthonormal eigenbasis).  Host-only;
 * KS_ERR_INVALID_ARG outside the range, KS_ERR_NOT_SUPPORTED on a plan
 * without KS_PLAN_LOWDIN. */
ks_status ks_plan_set_overlap_cutoff(ks_plan* plan, double tau);

/* KS_PLAN_LOWDIN plans: the number of eigenvectors of S kept by the last
 * decomposition of S, per k-point, into the HOST array nkeep[batch]
 * (synchronizes the plan's stream).  KS_ERR_INVALID_ARG before S has been
 * decomposed or for NULL, KS_ERR_NOT_SUPPORTED without KS_PLAN_LOWDIN. */
ks_status ks_plan_get_overlap_rank(ks_plan* plan, int32_t* nkeep);

/* Graph use under KS_PLAN_GRAPH: how many argument sets were captured and how
 * many ks_gevd calls replayed a captured graph.  Host-only. */
ks_status ks_plan_get_graph_stats(ks_plan* plan, int64_t* captures, int64_t* replays);

/* Synchronize the plan's stream and read its info word: 0 if no device failure
 * was recorded since the last call, else the failing Cholesky column (>0) for
 * KS_ERR_NOT_POSDEF, the row (>0) of an imaginary overlap entry for
 * KS_ERR_INVALID_ARG under KS_PLAN_REAL_OVERLAP, or -status for other device
 * failures.  Clears the word.  Returns KS_OK or the status of the recorded
 * failure. */
ks_status ks_plan_get_info(ks_plan* plan, int32_t* info);

/* Static, never NULL. */
const char* ks_status_string(ks_status s);

/* Bytes of device workspace ks_plan_create would allocate for desc
 * (0 if desc is invalid).  Host-only, no device call. */
uint64_t ks_plan_workspace_bytes(const ks_plan_desc* desc);

#ifdef __cplusplus
}
#endif

#endif /* KS_H */
