/*
 * fiohss — approximate inversion of discrete Fourier integral operators on AMD
 * Instinct MI355X (gfx950): butterfly-factorization (BF) apply, randomized HSS
 * construction of G~ ~ K~^* K~, ULV factorization and solve, and the online
 * solve f^ = F K~^* u (Li & Liu, "Approximate Inversion of Discrete Fourier
 * Integral Operators via Hierarchically Semiseparable Matrices").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Complex data are complex128 stored as interleaved (re, im) doubles.
 *  - Blocks of vectors are column-major: element (i, j) of an N x k block with
 *    leading dimension ld >= N is at offset i + j * ld (in complex elements).
 *  - Pointers documented as "device" must point to GPU memory allocated by
 *    the caller; the caller owns them.  Pointers documented as "host" are
 *    ordinary CPU memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *    are stream-ordered and asynchronous unless stated otherwise.  Argument
 *    errors are returned synchronously, before anything is enqueued.
 *  - Handles (fio_bf_t, hss_t, hss_ulv_t) are created by the library, are
 *    immutable once built and are released by the matching *_destroy.  Applies
 *    and solves on one handle may run concurrently on different streams when
 *    each call gets its own workspace.
 *  - Vector ordering of the discrete FIO (Section 1, eq. fio): spatial entry i
 *    is x_i = i / N, frequency entry j is xi_j = j - N/2.
 */
#ifndef FIOHSS_H
#define FIOHSS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FIO_OK = 0,
    FIO_ERR_ARG = -1,            /* invalid argument (bad size, NULL pointer, workspace too small) */
    FIO_ERR_OOM = -2,            /* a device allocation failed; no handle was created */
    FIO_ERR_HIP = -3,            /* a HIP runtime call failed */
    FIO_ERR_NOT_HPD = -4,        /* a Cholesky pivot of the ULV factorization was not positive */
    FIO_ERR_NOT_CONVERGED = -5,  /* refinement did not reach the requested residual */
    FIO_ERR_UNSUPPORTED = -6,    /* valid request outside what the library implements */
    FIO_ERR_CALLBACK = -7,       /* a caller callback returned non-zero */
    FIO_WARN_RANK_CAP = 1        /* HSS ranks hit the cap; the result is valid but less accurate */
} fio_status;

typedef enum {
    FIO_PREC_FP64 = 0,           /* complex128 factors and coefficients */
    FIO_PREC_FP32 = 1,           /* complex64 factors and coefficients, complex128 input/output */
    FIO_PREC_SPLIT_FP16 = 2      /* transfer blocks and coefficients split into hi + lo fp16 halves,
                                    MFMA with fp32 accumulation (see fio_bf_apply) */
} fio_prec;

typedef enum { FIO_AMP_ONE = 0, FIO_AMP_GAUSSIAN_SUM = 1, FIO_AMP_HANKEL = 2 } fio_amp_kind;
typedef enum { FIO_PHASE2_ANISO = 0, FIO_PHASE2_ISO = 1 } fio_phase2_kind;

typedef struct fio_bf_s *fio_bf_t;
typedef struct hss_s *hss_t;
typedef struct hss_ulv_s *hss_ulv_t;

/* ---------------------------------------------------------------------------
 * Butterfly factorization (Section 2.2, eq. bf):
 *   K~ = U^[L'] B^[L'] ... B^[h+1] M^[h] C^[h+1] ... C^[L'] V^[L'],
 * with q first-kind Chebyshev points per box and dimension on the closed box,
 * L' = max(L - level_offset, h) (the outer level of Section 5.2's implementation
 * note), amplitude a (see amp_kind below; 1 by default), and
 *
 * dim = 1: N = n = 2^L points (L even), h = L/2, phase
 *     Phi(x, xi) = x xi + (c0 + c1 sin(2 pi x)) |xi|;
 *   (c0, c1) = (0, 0) is the shifted DFT; (1/8, 1/16) is c(x) = (2 + sin 2 pi x)/16.
 *
 * dim = 2: n = 2^L points per dimension, N = n^2, quadtrees in space and
 *   frequency, h = ceil(L/2) (odd L: the U and V sides both stop at level h and
 *   M couples each U pair with the 4 V pairs of its parent spatial box and the
 *   frequency children of its box), phase of Section 5.2
 *     Phi(x, xi) = x.xi + sqrt(c1(x)^2 xi1^2 + c2(x)^2 xi2^2),
 *     c1(x) = c0 + c1 sin(2 pi x1) sin(2 pi x2),  c2(x) = c0 + c1 cos(2 pi x1) cos(2 pi x2);
 *   (c0, c1) = (1/8, 1/16) is the paper's 2D workload, (0, 0) the 2D DFT.
 *   Vectors are in the user order of the 2D grid: entry i1 n + i2 is
 *   x = (i1/n, i2/n) or xi = (i1 - n/2, i2 - n/2).  Only L - level_offset <= h
 *   is built (no B or C factor; n <= 128 at level_offset 3), leaf boxes of at most
 *   128 points and q^2 <= 128: other descriptors return FIO_ERR_UNSUPPORTED.
 * ------------------------------------------------------------------------- */
typedef struct {
    int dim;                 /* 1 or 2 */
    long n;                  /* points per dimension: 2^L (1D: L even, n >= 64; 2D: 4 <= n <= 2^15) */
    double c0, c1;           /* phase parameters, see above */
    int q;                   /* Chebyshev points per box and dimension, 2 <= q <= 16 */
    int level_offset;        /* L' = max(L - level_offset, h); 3 gives leaf boxes of 8 points per dimension */
    unsigned prec_mask;      /* bit p set: keep a copy of the factors in fio_prec p resident;
                                FIO_PREC_SPLIT_FP16 (dim 1, q = 9 only, else FIO_ERR_UNSUPPORTED
                                at build/import) also keeps the FP32 copy */
    /* 2D phase (fio_phase2_kind; must be 0 for dim 1, else FIO_ERR_UNSUPPORTED):
     * FIO_PHASE2_ANISO is Section 5.2's family above; FIO_PHASE2_ISO is Section 5.3's
     *   Phi(x, xi) = x.xi + c(x) ||xi||,  c(x) = c0 + c1 sin(2 pi x1) sin(2 pi x2)
     * (the family with c2 = c1), (c0, c1) = (3/8, 1/8) there.  FIO_ERR_ARG for other values. */
    int phase_kind;
    /* Amplitude (fio_amp_kind).  The interpolation factors U, B, C, V do not depend on it; it
     * enters the middle factor only, M = k(Z, Gamma) with k = a exp(2 pi i Phi)
     * (eq. bf_kernel_func_low_rank), so every apply path and precision serves it unchanged.
     * FIO_AMP_ONE: a = 1; the other amplitude fields are ignored.
     * FIO_AMP_GAUSSIAN_SUM (dim 1 only): Section 5.1's
     *   a(x, xi) = sum_k exp(-((x - x_k)^2 + ((xi - xi_k) / N)^2) / amp_sigma2),
     *   k = 1 .. amp_terms (at most 16), with the centers in HOST memory at amp_centers
     *   (x_1 .. x_m, then xi_1 .. xi_m), copied when the descriptor is planned (build, import,
     *   factor count).  FIO_ERR_ARG for amp_terms outside 1..16, amp_sigma2 <= 0 or a NULL
     *   amp_centers.
     * FIO_AMP_HANKEL (dim 2 only): Section 5.3's a(x, xi) = H0^(1)(2 pi rho) exp(-2 pi i rho),
     *   rho = Phi(x, xi) - x.xi, H0^(1) the Hankel function of the first kind of order 0.  It
     *   is infinite at xi = 0; the butterfly evaluates it at Chebyshev points only, which never
     *   fall on xi = 0, so K~ is finite there.
     * A kind not valid for the dimension returns FIO_ERR_UNSUPPORTED, other values FIO_ERR_ARG. */
    int amp_kind;
    int amp_terms;
    double amp_sigma2;
    const double *amp_centers;
} fio_bf_desc;

/* Number of complex entries of the explicit factors of `desc`, in the layout
 * read by fio_bf_import and written by fio_bf_export (0 on an invalid desc). */
size_t fio_bf_factor_count(const fio_bf_desc *desc);

/* Builds the factors on the GPU from the definitions of Section 2.2: every
 * entry of U, B, M, C, V is evaluated by a kernel from Phi, the Chebyshev
 * points and the Lagrange basis (each exponent is a phase difference between nearby
 * points, evaluated as such, so it stays accurate at any N).  Synchronizes `stream`
 * before returning. */
fio_status fio_bf_build(const fio_bf_desc *desc, void *stream, fio_bf_t *out);

/* Creates a handle from explicit factors held in HOST memory, `count`
 * complex128 entries laid out as
 *   V[sigma][tau][j][s]                 2^L' x 2^(L-L') x q x b
 *   C^[L'], C^[L'-1], ..., C^[h+1]       each (N/2) x 2q x 2q
 *   M[p][i][j]                          N x q x q
 *   B^[h+1], ..., B^[L']                each (N/2) x 2q x 2q
 *   U[tau][sigma][s][i]                 2^L' x 2^(L-L') x b x q
 * with b = N / 2^L' and the pair/group numbering
 *   U-side level l:  pair (tau at spatial level l, sigma at frequency level L-l) -> tau 2^(L-l) + sigma
 *   V-side level l:  pair (tau at spatial level L-l, sigma at frequency level l) -> tau 2^l + sigma
 *   B^[l+1] group (alpha at spatial level l, sigma at frequency level L-l-1) -> alpha 2^(L-l-1) + sigma
 *   C^[l+1] group (alpha at spatial level L-l-1, sigma at frequency level l) -> alpha 2^l + sigma
 *   block row c_out q + i (output pair tau = 2 alpha + c_out), column c_in q + t (input pair
 *   beta = 2 sigma + c_in), entries as defined in Section 2.2 (eq. bf_left_func_low_rank and
 *   its frequency-side mirror).
 * For dim = 2 the layout is V, M, U with column-major blocks:
 *   V block p = tau' 4^h + sigma (tau' at spatial level L-h, sigma at frequency level h),
 *     q^2 x b^2, entry (i, s) at p q^2 b^2 + s q^2 + i;
 *   M block u 4^h + sigma (both at level h), q^2 x q^2, entry (i, j) at blk q^4 + j q^2 + i,
 *     equal to k(z_u,i, gamma_sigma,j);
 *   U block p = tau 4^(L-h) + sigma' (tau at spatial level h, sigma' at frequency level L-h),
 *     b^2 x q^2, entry (s, i) at p q^2 b^2 + i b^2 + s;
 * with b = n / 2^h, box indices the Morton codes of the box coordinates (bit k of
 * the first coordinate at position 2k + 1, of the second at 2k), s the Morton
 * code of a point inside its box and i = i1 q + i2.  The conjugate-transposed
 * copies used by fio_bf_apply_adj are derived on the device.
 * Used to apply factors produced elsewhere (e.g. to test the apply kernels on
 * factors of a reference implementation).  Synchronous. */
fio_status fio_bf_import(const fio_bf_desc *desc, const void *host_factors, size_t count,
                         void *stream, fio_bf_t *out);

/* Copies the FP64 factors of `bf` to HOST memory in the import layout.  Synchronous. */
fio_status fio_bf_export(fio_bf_t bf, void *host_out, size_t count, void *stream);

/* Bytes of device workspace fio_bf_apply / fio_bf_apply_adj need for nrhs columns. */
fio_status fio_bf_workspace_size(fio_bf_t bf, int nrhs, fio_prec prec, size_t *bytes);

/* Y = K~ X (N x nrhs blocks, device).  `prec` selects the factor copy; the
 * input and output are complex128 in every precision.  `ws` is device memory
 * of at least fio_bf_workspace_size bytes, or NULL to use a workspace owned
 * by the handle (then calls on the handle must not overlap).  X and Y must
 * not overlap.
 * FIO_PREC_SPLIT_FP16 (the growth direction of the refinement's low-precision
 * K~^*): every transfer block a and its input coefficients x are split into
 * half-precision parts a_hi + a_lo, x_hi + x_lo, and a x is formed on the matrix
 * cores as a_hi x_hi + a_hi x_lo + a_lo x_hi with FP32 accumulation; each
 * column is scaled by a power of two per pass so that its entries sit well
 * inside half range (any FP32-representable input scale works).  The middle
 * factor is folded into the neighbouring transfer level (FP64 products before
 * the split); leaf factors and the coefficient buffers between passes are
 * FP32.  Accuracy is that of FP32 (about 1e-6 relative per apply).  A
 * FIO_ERR_ARG is returned when the handle holds no such copy. */
fio_status fio_bf_apply(fio_bf_t bf, const void *X, long ldx, void *Y, long ldy, int nrhs,
                        fio_prec prec, void *ws, size_t ws_bytes, void *stream);

/* Y = K~^* X: the factors of eq. bf in reverse order, conjugate-transposed
 * (Section 2.2, last paragraph).  Arguments as fio_bf_apply. */
fio_status fio_bf_apply_adj(fio_bf_t bf, const void *X, long ldx, void *Y, long ldy, int nrhs,
                            fio_prec prec, void *ws, size_t ws_bytes, void *stream);

/* Tile autotuner of the applies.  For `nrhs` columns in precision `prec`, times every candidate
 * tile configuration of fio_bf_apply and of fio_bf_apply_adj on the caller's X (one warm-up
 * and `reps` timed applies each, HIP events on `stream`) and keeps the fastest per direction
 * in the handle; later applies whose column count falls in the same bucket (the next power of
 * two of nrhs, all counts >= 64 in one bucket) and precision use it.  Candidates: for dim = 2
 * the column chunk of the workgroups (8 or 16) times the reduction split of the U and V^*
 * steps (4, 8, 16 dividing the partner count); for dim = 1 (q = 9) the number of transfer
 * levels per fused pass (1, 2, 3), with 3 levels the first leaf factor folded into the first pass
 * or run as its own kernel, and for FIO_PREC_SPLIT_FP16 each of these with the transfer passes
 * on the matrix cores (split FP16) or on the vector units (FP32); the built-in default is always
 * a candidate (fio_tile describes a candidate).  Every candidate applies the same operator
 * (results differ at most by rounding order, and the FP32 engine is the more accurate one of a
 * split-precision request).  Y (ldy >= N)
 * receives the last apply; `ws` as for fio_bf_apply (NULL: the handle's workspace).  When
 * `report` is not NULL, a NUL-terminated summary of the timings and the choices is written to
 * it (at most report_len bytes).  Synchronous.  Must not run concurrently with applies on the
 * same handle (the candidates are installed in turn).  Errors as fio_bf_apply; FIO_ERR_ARG
 * also for nrhs < 1 or reps < 1. */
fio_status fio_bf_autotune(fio_bf_t bf, const void *X, long ldx, void *Y, long ldy, int nrhs, fio_prec prec,
                           int reps, void *ws, size_t ws_bytes, void *stream, char *report, size_t report_len);

/* Pins the tile configuration of one direction (adj != 0: fio_bf_apply_adj), precision and
 * column bucket (as fio_bf_autotune), e.g. to reproduce a tuned choice: kc in {0, 8, 16},
 * nsplit 0 or a power of two dividing the 2D partner count (at most 16), kmax in 0..3 (1D
 * levels per pass); 0 keeps the built-in default.  Values a descriptor does not use are
 * ignored.  FIO_ERR_ARG for other values.  Host-side only; must not run concurrently with
 * applies on the same handle. */
fio_status fio_bf_set_tile(fio_bf_t bf, int adj, fio_prec prec, int nrhs, int kc, int nsplit, int kmax);

/* One tile configuration of an apply (fio_bf_autotune's candidates).  0 everywhere is the
 * built-in default. */
typedef struct {
    int kc;        /* dim 2: column chunk of the workgroups, 0, 8 or 16 */
    int nsplit;    /* dim 2: reduction split of the U and V^* steps, 0 or a power of two dividing the
                      partner count, at most 16 */
    int kmax;      /* dim 1: transfer levels per fused pass, 0 (as many as the LDS tile holds) or 1..3 */
    int leaf_sep;  /* dim 1: 1 runs the first leaf factor as its own kernel instead of folding it into a
                      first pass of 3 levels */
    int valu;      /* dim 1, FIO_PREC_SPLIT_FP16 only: 1 runs the transfer passes as FP32 structured
                      passes on the vector units instead of split FP16 on the matrix cores */
} fio_tile;

/* fio_bf_set_tile with every field of fio_tile; FIO_ERR_ARG for values outside the ranges above
 * (valu = 1 with another precision included).  Host-side only, as fio_bf_set_tile. */
fio_status fio_bf_set_tile_cfg(fio_bf_t bf, int adj, fio_prec prec, int nrhs, const fio_tile *t);

/* The configuration later applies of that direction, precision and column bucket use (all zero:
 * the built-in default). */
fio_status fio_bf_get_tile_cfg(fio_bf_t bf, int adj, fio_prec prec, int nrhs, fio_tile *t);

/* The handle's tuned table as NUL-terminated text, so that a tuning can be kept and reused by
 * another process: a header line "fiohss-tune 1 dim=<d> n=<n> q=<q> level_offset=<o>", then one
 * line "adj=<0|1> prec=<p> cols=<bucket> kc=.. nsplit=.. kmax=.. leaf_sep=.. valu=.." per tuned
 * (direction, precision, column bucket).  *needed (if not NULL) receives the size including the
 * NUL; buf == NULL only queries it; FIO_ERR_ARG when len is smaller. */
fio_status fio_bf_tune_export(fio_bf_t bf, char *buf, size_t len, size_t *needed);

/* Loads a table written by fio_bf_tune_export into the handle (entries it names replace the
 * handle's; others are kept).  FIO_ERR_ARG, with the handle unchanged, for malformed text, a
 * header of another operator shape (dim, n, q, level_offset) or an invalid configuration. */
fio_status fio_bf_tune_import(fio_bf_t bf, const char *text);

void fio_bf_destroy(fio_bf_t bf);

/* Index map of the 2D grids: reorders the rows of X (n^2 x nrhs, device) into Y
 * between the user's lexicographic order (row i1 n + i2) and the Morton order
 * (row = Morton code of (i1, i2), bit k of i1 at position 2k + 1), in which every
 * dyadic box is a contiguous run of rows; the HSS representation of
 * K~^* K~ built by fio_hss_build for dim = 2 uses the binary tree over this
 * order.  to_internal != 0: Y[morton(i1, i2)] = X[i1 n + i2]; else the inverse.
 * n a power of two <= 2^15; X and Y must not overlap. */
fio_status fio_permute2d(long n, int to_internal, const void *X, long ldx, void *Y, long ldy, int nrhs,
                         void *stream);

/* Selects the apply kernels: on != 0 (default) runs consecutive transfer factors
 * as fused multi-level passes on closed sub-butterflies held in LDS, with the
 * middle factor folded into the pass that ends at level h; on == 0 runs one
 * kernel per factor.  Both give the same result up to rounding order.  Not
 * thread-safe with respect to concurrent applies. */
void fio_set_fused(int on);

/* With fused passes on: on != 0 (default) folds the first leaf factor of an apply (V^[L']
 * forward, U^[L']* adjoint) into its first pass of transfer factors when that pass holds 3
 * levels (FP64 and FP32 structured factors, 2^L' >= 64; the pass then reads the input vectors
 * instead of the leaf coefficients); on == 0 runs the leaf factor as its own kernel.  Both give
 * bitwise identical results.  Not thread-safe with respect to concurrent applies. */
void fio_set_leaf_fused(int on);

/* Selects how the HSS construction (hss_build_from_samples, fio_hss_build) runs the node
 * algebra of a level: levels whose largest node has at least `rows` rows run every
 * reflector and pivot step as its own launch spread over many workgroups; smaller levels
 * run one workgroup per node.  Both give the same result up to rounding order.  rows <= 0
 * restores the default (256).  Not thread-safe with respect to concurrent constructions. */
void fio_hss_set_big_node(int rows);

/* The same choice for the basis elimination of hss_ulv_factor (QL of each node's basis and
 * the explicit Q): levels whose largest node has at least `rows` rows apply every reflector
 * in its own launch over many workgroups.  rows <= 0 restores the default (256). */
void fio_ulv_set_big_node(int rows);

/* ---------------------------------------------------------------------------
 * Randomized black-box HSS construction of a Hermitian matrix (Section 3).
 * The tree is binary over rows 0..N-1, leaves of `leaf` rows (N = leaf 2^Lh);
 * ranks are per node; the effective leaf size of a nonleaf node is the sum of
 * its children's ranks, and level l uses s_l = m_max + rhat + p samples with
 * m_max the largest effective leaf size of the level (rhat <= 0: rhat = m_max).
 * A column of the QRCP of the sample block is kept while |R_jj| > tol * g,
 * g = norm_est if > 0, else ||Y^[L]||_F / ||Omega^[L]||_F from the leaf level.
 * ------------------------------------------------------------------------- */
typedef struct {
    int leaf;           /* leaf size m_L (64) */
    double tol;         /* relative truncation tolerance */
    int p;              /* oversampling */
    int rhat;           /* rank guess added to the sample count; <= 0: m_max */
    double norm_est;    /* scale of the tolerance; <= 0: estimated from the leaf samples */
    int rank_cap;       /* <= 0: no cap; else ranks are truncated at rank_cap (FIO_WARN_RANK_CAP) */
    int sample_prec;    /* fio_hss_build only: fio_prec of the K~^* K~ sample applies, FIO_PREC_FP64
                           (0, default) or FIO_PREC_FP32 (needs the handle's FP32 copy, else FIO_ERR_ARG;
                           its ~1e-6 relative rounding sits far below the truncation tolerances the
                           construction is used with); ignored by hss_build_from_samples */
    int adaptive;       /* 0: s_l = m_max + rhat + p at every level.  1: Section 3.1's s_l = m_l + r_l + p
                           with the rank r_l guessed as the largest rank of level l + 1 (rhat, or m_max,
                           at the leaf level); a level where some node's rank exceeds the guess is
                           sampled again with the guess m_max, which always suffices (a second call of
                           omega for that level, with more columns) */
} hss_opts;

/* Y = H X for ncols columns (device, column-major).  Return 0 on success. */
typedef int (*hss_matvec_fn)(void *ctx, const void *X, long ldx, void *Y, long ldy, int ncols,
                             void *stream);
/* Fills the rows x cols test matrix Omega^[level] (device, column-major, ld = rows)
 * with i.i.d. standard complex Gaussians.  Return 0 on success. */
typedef int (*hss_omega_fn)(void *ctx, int level, long rows, long cols, void *out, void *stream);

/* Section 3.1-3.3 with a caller-supplied matvec and test-matrix source.  The
 * level loop runs on the host (each level's sizes depend on the ranks found
 * below it); all per-node algebra runs in batched kernels.  Synchronous. */
fio_status hss_build_from_samples(long n, const hss_opts *opts, hss_matvec_fn matvec, void *matvec_ctx,
                                  hss_omega_fn omega, void *omega_ctx, void *stream, hss_t *out);

/* Algorithm alg:fio_inv step 2: hss_build_from_samples with the matvec
 * X -> K~^* (K~ X) applied by this library's BF kernels, in opts->sample_prec. */
fio_status fio_hss_build(fio_bf_t bf, const hss_opts *opts, hss_omega_fn omega, void *omega_ctx,
                         void *stream, hss_t *out);

/* Tree shape of an HSS handle: *levels = Lh; ranks (host, may be NULL) receives
 * the 2^(Lh+1) - 2 node ranks level by level from level 1 to Lh. */
fio_status hss_shape(hss_t h, int *levels, int *leaf, long *n, int *ranks, size_t nranks);

/* HSS generators to/from HOST memory, packed level by level:
 *   for l = 1..Lh, node j: U_(l,j) column-major m x r;
 *   for l = 0..Lh-1, node j: B_(l,j) = B_{a2,a1} column-major r_a2 x r_a1;
 *   for leaves j: D_j column-major leaf x leaf.
 * `ranks` lists the node ranks as hss_shape does.  hss_generator_count gives
 * the number of complex entries.  Synchronous. */
size_t hss_generator_count(long n, int leaf, const int *ranks);
fio_status hss_export(hss_t h, void *host_out, size_t count, void *stream);
fio_status hss_import(long n, int leaf, const int *ranks, const void *host_gen, size_t count,
                      void *stream, hss_t *out);

/* Y = H X with the telescoping form (eq. hss_telescoping_factorization). */
fio_status hss_matvec(hss_t h, const void *X, long ldx, void *Y, long ldy, int nrhs, void *stream);

void hss_destroy(hss_t h);

/* ---------------------------------------------------------------------------
 * ULV factorization (Section 2.4): per node, QL basis elimination, Cholesky
 * of the eliminated block, Schur complement, merge; root Cholesky.  The
 * factors are stored per node as the m x m matrix W = [L11^-1 Q1^*;
 * Q2^* - Dhat21 L11^-1 Q1^*], so that the bottom-up solve step is
 * [bhat1; yhat2] = W y and the top-down step is c = W^* [bhat1; chat2]
 * (algebraically the same steps as Section 2.4).  Synchronous; returns
 * FIO_ERR_NOT_HPD when a pivot is not positive.
 * ------------------------------------------------------------------------- */
fio_status hss_ulv_factor(hss_t h, void *stream, hss_ulv_t *out);

/* Bytes of device workspace hss_ulv_solve needs for nrhs columns. */
fio_status hss_ulv_workspace_size(hss_ulv_t f, int nrhs, size_t *bytes);

/* C = G~^{-1} Y (N x nrhs, device).  In-place (C == Y, ldc == ldy) is allowed. */
fio_status hss_ulv_solve(hss_ulv_t f, const void *Y, long ldy, void *C, long ldc, int nrhs,
                         void *ws, size_t ws_bytes, void *stream);

void hss_ulv_destroy(hss_ulv_t f);

/* ---------------------------------------------------------------------------
 * Online solve (Section 4.1, eq. fio_inv_approx): F ~ K^{-1} U.
 *   mode DIRECT: F = G~^{-1} K~^* U (K~^* in `prec`, ULV in FP64).
 *   mode IR:     F0 = G~^{-1} K~^*_prec U; then up to max_ir times
 *                R = U - K~ F (FP64), F += G~^{-1} K~^*_prec R, stopping when the
 *                largest column ratio ||R_j|| / ||U_j|| <= rel_res_tol
 *                (rel_res_tol <= 0: exactly max_ir steps, no host sync).
 *   mode PCG:    conjugate gradients on K~^* K~ F = K~^* U (Section 4.1, eq.
 *                fio_approx_normal_eq) preconditioned by G~^{-1}, from F = 0, each
 *                column its own recurrence, every apply in FP64 (prec must be
 *                FP64); at most max_ir iterations, stopping when the largest column
 *                ratio ||B_j - K~^* K~ F_j|| / ||B_j|| <= rel_res_tol with B = K~^* U
 *                (rel_res_tol <= 0: exactly max_ir iterations, no host sync).
 *                FIO_ERR_NOT_CONVERGED when the limit is reached first.
 * ------------------------------------------------------------------------- */
typedef enum { FIO_SOLVE_DIRECT = 0, FIO_SOLVE_IR = 1, FIO_SOLVE_PCG = 2 } fio_solve_mode;

typedef struct {
    int mode;             /* fio_solve_mode */
    int prec;             /* fio_prec of the K~^* applies */
    double rel_res_tol;   /* IR stopping rule, see above */
    int max_ir;           /* IR step limit */
} fio_solve_opts;

typedef struct {
    int ir_steps;         /* refinement steps (IR) or iterations (PCG) taken */
    double rel_res;       /* largest column relative residual after the last step (IR and PCG
                             with rel_res_tol > 0 only; -1 otherwise) */
} fio_solve_info;

fio_status fio_solve_workspace_size(fio_bf_t bf, hss_ulv_t f, int nrhs, const fio_solve_opts *opts,
                                    size_t *bytes);

/* `info` is host memory (may be NULL).  With mode IR and rel_res_tol > 0 the
 * call synchronizes `stream` once per step to read the residual norms. */
fio_status fio_approx_solve(fio_bf_t bf, hss_ulv_t f, const void *U, long ldu, void *F, long ldf,
                            int nrhs, const fio_solve_opts *opts, fio_solve_info *info,
                            void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate (code under hipGraph capture, tight serving loops,
 * harnesses that forbid hipMalloc): fio_approx_solve with the workspace taken from a
 * file-scope device array of fio_approx_solve_static_max_bytes() bytes (64 MiB), one per
 * GPU, held until the process ends; the call allocates nothing, on the device or the host.
 * Same arguments and results as fio_approx_solve without ws / ws_bytes; the array of the
 * current device is used, so the current device must be the one that `stream` runs on.
 * Returns FIO_ERR_ARG (with a message on stderr) when the solve needs more workspace than
 * the array holds (fio_solve_workspace_size tells the need), and for the residual-checked
 * forms (IR or PCG with rel_res_tol > 0, which read norms back into host memory).  Every
 * call on a GPU shares that GPU's array: calls that overlap in time on one GPU (other
 * streams, other threads) race; the array's contents left by a call are not used by the
 * next (nothing in it must start at zero). */
size_t fio_approx_solve_static_max_bytes(void);
fio_status fio_approx_solve_static(fio_bf_t bf, hss_ulv_t f, const void *U, long ldu, void *F, long ldf,
                                   int nrhs, const fio_solve_opts *opts, fio_solve_info *info, void *stream);

const char *fio_status_str(fio_status s);

/* ---------------------------------------------------------------------------
 * Solve server (continuous batching).  Operators (a BF handle and the ULV
 * factors of its HSS approximation) stay resident.  fio_server_submit queues a
 * request (nrhs columns for one operator) and returns at once; a dispatcher
 * thread forms a batch whenever one of `streams` slots is free: the oldest
 * waiting request plus later requests for the same operator, in arrival order,
 * while the batch fits the slot's memory.  Each slot owns one device arena,
 * allocated at the first submission and shared by all operators: mem_budget /
 * streams bytes (0: the largest batch of any operator at max_batch_rhs
 * columns).  A batch of w columns needs its input and output blocks (2 N w
 * complex entries) plus the solve workspace for w columns; the widest w that
 * fits the arena bounds every batch of that operator (memory-based admission),
 * and the arenas take at most mem_budget bytes of device memory (captured
 * graphs add the runtime's own bookkeeping, a few MB each).  A request wider than
 * that returns FIO_ERR_ARG at submission, as does a budget too small for one
 * column.  The batch runs as one fio_approx_solve on the slot's stream
 * (replayed from a captured hipGraph when use_graphs != 0; the arena addresses
 * depend only on the slot, operator and width, so the graphs stay valid).
 * U must be complete (the work producing it finished) when it is submitted;
 * batches on different slots overlap on the device.  Every column is solved
 * independently, so with a fixed refinement step count (solve mode DIRECT, or
 * IR with rel_res_tol <= 0, which add_operator requires) a request's result is
 * bitwise the same alone and in any batch.  U must stay valid and F untouched
 * until the request completes (fio_server_wait_all).  Times are seconds since
 * fio_server_create.  add_operator is accepted only before the first submission.
 * ------------------------------------------------------------------------- */
typedef struct fio_server_s *fio_server_t;
typedef struct {
    int max_batch_rhs;     /* columns per batch */
    int streams;           /* concurrent batch slots (1..8) */
    size_t mem_budget;     /* device bytes of all slot arenas; 0 = one widest batch per slot */
    int use_graphs;        /* replay captured hipGraphs per (operator, batch width) */
    int width_bucket;      /* > 1: batch widths rounded up to a multiple (zero columns appended), and
                              with use_graphs every (slot, operator, width) graph is captured when the
                              first request arrives; <= 1: exact widths, graphs captured on first use */
} fio_server_opts;

fio_status fio_server_create(const fio_server_opts *opts, fio_server_t *out);
fio_status fio_server_add_operator(fio_server_t s, fio_bf_t bf, hss_ulv_t f, const fio_solve_opts *opts,
                                   int *op_id);
fio_status fio_server_submit(fio_server_t s, int op_id, const void *U, long ldu, void *F, long ldf, int nrhs,
                             long long *req_id);
fio_status fio_server_wait_all(fio_server_t s);
fio_status fio_server_request_info(fio_server_t s, long long req_id, double *t_submit, double *t_start,
                                   double *t_done, int *batch, int *status);
fio_status fio_server_stats(fio_server_t s, long *completed, long *batches, long *max_queue,
                            size_t *peak_bytes);
double fio_server_now(fio_server_t s);
void fio_server_destroy(fio_server_t s);

/* ---------------------------------------------------------------------------
 * Measurement hooks.  While enabled, the library brackets each of its hot
 * kernel launches (BF levels, ULV levels) with HIP events recorded on the
 * launch stream and accumulates the durations per kernel name
 * ("bf_transfer_f64", "bf_transfer_f32", "bf_middle_f64", "bf_leaf_in_f64",
 * "bf_leaf_out_f64", ..., "ulv_up", "ulv_down", "ulv_root").
 * fio_timing_query and fio_timing_names wait for the pending events; they
 * return FIO_OK / the length of the comma-separated name list.
 * ------------------------------------------------------------------------- */
void fio_timing_enable(int on);
void fio_timing_reset(void);
int fio_timing_query(const char *kernel, long *launches, double *total_ms);
int fio_timing_names(char *buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif
