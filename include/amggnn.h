/*
 * amggnn.h -- C ABI of the MI355X (gfx950) GNN-smoothed algebraic multigrid solve phase.
 *
 * Problem (paper Sec. 2.1, Eq. 1): A u = f with A sparse, symmetric, zero row sums
 * for all-Neumann problems. The library stores A with a POSITIVE diagonal: a caller
 * holding the paper's negative semi-definite form passes -A and -f (same solution).
 *
 * Conventions for every matrix argument
 *   CSR, int32 rowptr[n+1] (rowptr[0] == 0), int32 col[nnz] strictly ascending within
 *   a row, float64 val[nnz]. Square level matrices store their diagonal.
 *
 * Memory
 *   Pointers documented as "device" point to GPU memory owned by the caller (for
 *   example PyTorch tensors); the context keeps NON-OWNING views of the hierarchy
 *   arrays handed to amgg_load_level / amgg_load_prolong, which must outlive it.
 *   Everything the solver derives (R = P^T, FP32 copies, smoother values, dense
 *   coarse inverse, level vectors, reduction scratch) lives in ONE caller-allocated
 *   device workspace of amgg_workspace_bytes() bytes. The library never allocates
 *   device memory; host-side results (amgg_rs_*) are allocated and freed by it.
 *
 * Streams
 *   Every device call takes `void* stream` (a hipStream_t; NULL = default stream) and
 *   is ordered on it. Calls returning host results synchronise that stream.
 *
 * Errors
 *   0 = success; negative = error (nothing is left half-done on the host side; the
 *   message is in amgg_last_error(), per thread); positive = solver outcome of
 *   amgg_solve (not an error). No C++ exception crosses this interface. A context
 *   is not thread-safe; distinct contexts are independent.
 */
#ifndef AMGGNN_H
#define AMGGNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AMGG_OK 0
#define AMGG_EINVAL (-1)     /* invalid argument, shape or pattern */
#define AMGG_EWORKSPACE (-2) /* workspace missing or too small */
#define AMGG_EHIP (-3)       /* HIP runtime error */
#define AMGG_ESTATE (-4)     /* call out of order (e.g. vcycle before smoothers are set) */
#define AMGG_ENONFINITE (-5) /* non-finite input or coefficient */

#define AMGG_MAXIT 1     /* solve: iteration limit reached */
#define AMGG_DIVERGED 2  /* solve: ||r|| > div_factor ||b|| or non-finite */
#define AMGG_STAGNATED 3 /* solve: reduction over stag_window iterations worse than stag_ratio */
#define AMGG_BREAKDOWN 4 /* solve: flexible CG lost positive definiteness (z^T r <= 0 or p^T A p <= 0) */

#define AMGG_MAX_LEVELS 16
#define AMGG_MAX_DEGREE 4
#define AMGG_MAX_COARSE_DENSE 4096 /* largest coarsest level solved by the dense inverse */

/* ------------------------------------------------------------------------------------
 * Host setup: classical Ruge-Stueben hierarchy {A_l, P_l} (paper Sec. 2.2 and Sec. 4:
 * classical RS coarsening, strength threshold theta = 0.25; App. B.1, Tab. 7: at most
 * 10 levels; Alg. 1, step 2). The paper names the method only; this implementation
 * fixes: negative-coupling strength, RS first pass with ties to the smallest index,
 * direct interpolation with positive couplings lumped on the diagonal, Galerkin
 * A_c = P^T (A P) by row-wise accumulation in ascending column order with exact zeros
 * dropped off the diagonal. Coarsening stops at max_levels, at n <= max_coarse, when
 * no C point exists or when 10 n_c > 9 n.
 * ------------------------------------------------------------------------------------ */
typedef struct amgg_rs amgg_rs;

/* Build the hierarchy of the host CSR matrix (n rows). theta in (0,1); max_levels in
 * [1, AMGG_MAX_LEVELS]; max_coarse >= 1. On success *out owns host memory released by
 * amgg_rs_free. Also detects the all-Neumann case (|row sum| <= 1e-12 a_ii everywhere).
 * Errors: AMGG_EINVAL for a bad pattern (unsorted columns, missing or non-positive
 * diagonal, out-of-range column). */
int amgg_rs_setup(const int32_t* rowptr, const int32_t* col, const double* val, int32_t n,
                  double theta, int max_levels, int32_t max_coarse, amgg_rs** out);
/* Number of levels and the singular (constant null space) flag. */
int amgg_rs_info(const amgg_rs* h, int* nlevels, int* singular);
/* Sizes of level lvl: n rows, nnz of A_l, and P_l's column count and nnz (0 on the coarsest). */
int amgg_rs_level_size(const amgg_rs* h, int lvl, int32_t* n, int32_t* nnz, int32_t* p_ncols, int32_t* p_nnz);
/* Copy level lvl into caller-allocated host arrays sized by amgg_rs_level_size; the P
 * arguments are ignored (may be NULL) on the coarsest level. cf (may be NULL) receives
 * 1 for C points and 0 for F points (all 0 on the coarsest level). */
int amgg_rs_copy_level(const amgg_rs* h, int lvl, int32_t* rowptr, int32_t* col, double* val,
                       int32_t* p_rowptr, int32_t* p_col, double* p_val, int8_t* cf);
void amgg_rs_free(amgg_rs* h);

/* The same setup into caller-allocated host buffers, in two calls: amgg_rs_setup_query reports
 * the hierarchy's sizes; amgg_rs_setup_fill, with the same inputs, writes every level into the
 * caller's arrays, sized as the query reported (each call runs the whole setup, so a caller that
 * wants it once keeps an amgg_rs handle instead). Errors as amgg_rs_setup, plus AMGG_EINVAL
 * when a fill pointer is NULL where the level needs it. */
typedef struct {
    int nlevels;
    int singular;
    int32_t n[AMGG_MAX_LEVELS], nnz[AMGG_MAX_LEVELS];      /* A_l: rows, stored entries */
    int32_t p_ncols[AMGG_MAX_LEVELS], p_nnz[AMGG_MAX_LEVELS]; /* P_l (0 on the coarsest level) */
} amgg_hier_sizes;
typedef struct {
    int32_t* rowptr[AMGG_MAX_LEVELS]; /* n + 1 */
    int32_t* col[AMGG_MAX_LEVELS];    /* nnz */
    double* val[AMGG_MAX_LEVELS];     /* nnz */
    int32_t* p_rowptr[AMGG_MAX_LEVELS]; /* n + 1 (levels above the coarsest) */
    int32_t* p_col[AMGG_MAX_LEVELS];    /* p_nnz */
    double* p_val[AMGG_MAX_LEVELS];     /* p_nnz */
    int8_t* cf[AMGG_MAX_LEVELS];        /* n, may be NULL: 1 for C points */
} amgg_hier_host;
int amgg_rs_setup_query(const int32_t* rowptr, const int32_t* col, const double* val, int32_t n, double theta,
                        int max_levels, int32_t max_coarse, amgg_hier_sizes* sizes_out);
int amgg_rs_setup_fill(const int32_t* rowptr, const int32_t* col, const double* val, int32_t n, double theta,
                       int max_levels, int32_t max_coarse, const amgg_hier_host* out);

/* Stepwise form of amgg_rs_setup for callers that form the Galerkin products elsewhere
 * (amgg_galerkin_device). amgg_rs_begin validates the matrix as amgg_rs_setup does and
 * holds it as level 0. amgg_rs_coarsen works on the last level: it applies the stopping
 * rules and, unless coarsening stops (*more = 0; further calls keep returning 0), computes
 * the level's C/F split and interpolation P (*more = 1; amgg_rs_level_size and
 * amgg_rs_copy_level then report P). The next level's matrix must then be supplied,
 * either by amgg_rs_galerkin (host product, as in amgg_rs_setup) or by amgg_rs_push_level
 * (host CSR arrays, n = P's column count, validated like the input), before coarsening
 * again. With host products throughout the result equals amgg_rs_setup's.
 * Errors: AMGG_EINVAL (bad argument or pattern), AMGG_ESTATE (call out of sequence). */
int amgg_rs_begin(const int32_t* rowptr, const int32_t* col, const double* val, int32_t n,
                  double theta, int max_levels, int32_t max_coarse, amgg_rs** out);
int amgg_rs_coarsen(amgg_rs* h, int* more);
int amgg_rs_galerkin(amgg_rs* h);
int amgg_rs_push_level(amgg_rs* h, int32_t n, const int32_t* rowptr, const int32_t* col, const double* val);
/* The same coarsening step with the strength of connection and the interpolation formed elsewhere
 * (amgg_strength_device, amgg_interp_device); the C/F split, a sequential greedy, stays here.
 * amgg_rs_split with strong = NULL applies the level-count and size stopping rules to the last
 * level: *more = 1 means the level is to be coarsened and its strength flags are wanted. Called
 * again with strong (host, one byte per stored entry of the level's matrix in stored order, 1 =
 * strong, as amgg_strength_device writes them) it computes the split: *more = 0 if coarsening
 * stops there (no C point, or 10 n_c > 9 n), else *more = 1 and cf_out (host, n bytes) receives
 * 1 for C points and 0 for F points. amgg_rs_push_interp then supplies the level's P (host CSR,
 * n rows, nc = the number of C points, ascending columns; e.g. from amgg_interp_device), after
 * which the next level's matrix is supplied as after amgg_rs_coarsen. With flags and P equal to
 * the host setup's the result equals amgg_rs_setup's. Errors: AMGG_EINVAL, AMGG_ESTATE. */
int amgg_rs_split(amgg_rs* h, const uint8_t* strong, int8_t* cf_out, int* more);
int amgg_rs_push_interp(amgg_rs* h, int32_t nc, const int32_t* rowptr, const int32_t* col, const double* val);

/* ------------------------------------------------------------------------------------
 * Device setup of one level: strength of connection, direct interpolation and the Galerkin
 * product (paper Sec. 2.2: the coarse operator is R A P with R = P^T; Sec. 4: classical
 * Ruge-Stueben; Alg. 1, step 2).
 * ------------------------------------------------------------------------------------ */
typedef void* (*amgg_alloc_fn)(size_t bytes, void* user); /* device memory, or NULL */
typedef void (*amgg_release_fn)(void* ptr, void* user);

/* Strength of connection of one level on device `device` (Sec. 4: classical Ruge-Stueben with
 * threshold theta), bitwise the host setup's: strong[p] = 1 when stored entry p of row i (column
 * j != i) satisfies -a_ij >= theta max_{k != i}(-a_ik) with that max positive, else 0 (positive
 * couplings are weak). A: device CSR (n rows, nnz entries, ascending columns, checked on the
 * device), read only; strong: device, nnz bytes, written. alloc / release as for
 * amgg_galerkin_device (one temporary). Synchronises the stream once. Errors: AMGG_EINVAL
 * (NULL, bad size or pattern, theta outside (0, 1)), AMGG_EWORKSPACE, AMGG_EHIP. */
int amgg_strength_device(int device, int32_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                         int32_t nnz, double theta, uint8_t* strong, amgg_alloc_fn alloc, amgg_release_fn release,
                         void* user, void* stream);
/* Direct interpolation of one level on device `device` (Sec. 2.2: the prolongation of classical
 * Ruge-Stueben AMG), bitwise the host setup's: C points (cf[i] != 0) are numbered in ascending
 * order and their rows of P are the identity; an F row with strong C neighbours C_i (strong,
 * as amgg_strength_device writes it) gets w_ik = -(alpha_i a_ik) / (a_ii + sum of the row's
 * positive off-diagonals), alpha_i = (sum of its negative off-diagonals) / (sum of a_ik over
 * C_i), every sum in ascending column order; other F rows are empty. A, strong and cf (n bytes)
 * are device arrays, read only. On success *nc is the number of C points and *p_rowptr (n + 1
 * entries), *p_col, *p_val (*p_nnz entries) were obtained from alloc and belong to the caller;
 * temporaries are released before the call returns, also on error. Synchronises the stream.
 * Errors: AMGG_EINVAL (NULL, bad size or pattern, no C point), AMGG_EWORKSPACE, AMGG_EHIP. */
int amgg_interp_device(int device, int32_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                       int32_t nnz, const uint8_t* strong, const int8_t* cf, amgg_alloc_fn alloc,
                       amgg_release_fn release, void* user, int32_t* nc, int32_t** p_rowptr, int32_t** p_col,
                       double** p_val, int32_t* p_nnz, void* stream);

/* A_c = P^T (A P) on device `device`, bitwise equal to the host product of amgg_rs_setup:
 * R = P^T is the exact transpose, and each entry of A P and of R (A P) is accumulated over
 * the left operand's row in ascending column order, starting from 0.0, with products and
 * sums rounded separately; exact zeros off the diagonal are then dropped (zeros of A P are
 * kept). A (n x n, a_nnz entries) and P (n x nc, p_nnz entries) are device CSR arrays
 * with int32 strictly ascending columns and FP64 values, read only; their patterns are
 * checked on the device before use. Device memory comes from alloc(bytes, user); temporaries are
 * handed back through release(ptr, user) before the call returns, also on error. On
 * success *ac_rowptr (nc + 1 entries), *ac_col and *ac_val (*ac_nnz entries) were obtained
 * from alloc and belong to the caller. chunk_products bounds the expanded products sorted
 * at once, which sets the temporary memory (about 24 bytes per product); 0 selects 2^27.
 * Work is queued on `stream` (hipStream_t), which the call synchronises to read sizes.
 * Errors: AMGG_EINVAL (NULL, bad sizes or pattern, more than 2^31 - 1 result entries),
 * AMGG_EWORKSPACE (alloc returned NULL), AMGG_EHIP (runtime error). */
int amgg_galerkin_device(int device, int32_t n, int32_t nc, const int32_t* a_rowptr, const int32_t* a_col,
                         const double* a_val, int32_t a_nnz, const int32_t* p_rowptr, const int32_t* p_col,
                         const double* p_val, int32_t p_nnz, amgg_alloc_fn alloc, amgg_release_fn release,
                         void* user, int64_t chunk_products, int32_t** ac_rowptr, int32_t** ac_col,
                         double** ac_val, int32_t* ac_nnz, void* stream);


/* ------------------------------------------------------------------------------------
 * Device context: hierarchy load (Alg. 1, step 2) and derived data.
 * ------------------------------------------------------------------------------------ */
typedef struct amgg_ctx amgg_ctx;

/* Context on HIP device `device` for a hierarchy of `nlevels` levels (1..AMGG_MAX_LEVELS). */
int amgg_create(amgg_ctx** out, int device, int nlevels);
int amgg_destroy(amgg_ctx* ctx);
/* Message of the last failing call on this thread ("" if none). */
const char* amgg_last_error(void);

/* Level matrix A_l (device CSR, n x n, diagonal stored and positive). */
int amgg_load_level(amgg_ctx* ctx, int lvl, int32_t n, int32_t nnz, const int32_t* rowptr,
                    const int32_t* col, const double* val);
/* Prolongation P_l (device CSR, n_f x n_c) between level lvl and lvl+1; lvl < nlevels-1. */
int amgg_load_prolong(amgg_ctx* ctx, int lvl, int32_t n_f, int32_t n_c, int32_t nnz,
                      const int32_t* rowptr, const int32_t* col, const double* val);
/* Workspace size for the loaded hierarchy (all levels and prolongations must be loaded). */
int amgg_workspace_bytes(const amgg_ctx* ctx, size_t* bytes);
/* Bind the workspace (device, 256-byte aligned, >= amgg_workspace_bytes) and derive on the
 * GPU: R_l = P_l^T as CSR (exact transpose, sorted columns), correctly rounded FP32 copies
 * of A_l, P_l, R_l, the diagonal and s_l = max |offdiag(A_l)| (Sec. 3.1, Eq. 5), and the
 * dense FP64 inverse of the coarsest matrix by LU with partial pivoting (Sec. 2.2: direct
 * solve on the coarsest level). singular != 0 factors A_L + alpha 1 1^T with
 * alpha = mean(diag A_L)/n_L so that the coarse correction of a consistent right-hand
 * side has zero mean. Synchronises the stream. Errors: AMGG_EINVAL if the coarsest level
 * exceeds AMGG_MAX_COARSE_DENSE or a pivot is zero; AMGG_EWORKSPACE. */
int amgg_finalize(amgg_ctx* ctx, int singular, void* workspace, size_t ws_bytes, void* stream);

/* Device views into the workspace for inspection (any argument may be NULL). */
typedef struct {
    int32_t n, nnz, n_coarse, p_nnz;
    const int32_t* r_rowptr; /* R = P^T: n_coarse + 1 */
    const int32_t* r_col;    /* p_nnz */
    const double* r_val;     /* p_nnz */
    const float* a_val32;    /* nnz */
    const float* p_val32;    /* p_nnz */
    const float* r_val32;    /* p_nnz */
    const double* q_val;     /* nnz, smoother values on A's pattern */
    const float* q_val32;    /* nnz */
    const double* diag;      /* n */
    const double* scale;     /* 1 value: s_l (of the whole level; block scales are internal) */
    const double* coarse_inv;/* n*n row-major on the coarsest level, else NULL; on a
                                block-diagonal level the blocks' n_b*n_b inverses in turn */
    int32_t fused_rows;      /* rows per block of the fused smoothing kernels, 0 = not fused */
    /* Packed columns of A_l (shared by Q_l), P_l and R_l, in this order: rows per block of the
     * packing (0: the kernels read the 4-byte columns) and its far entries (columns outside the
     * 16-bit window of their block, listed separately). */
    int32_t pack_rows[3];
    int64_t pack_far[3];
    /* Products the CSR-stream kernels hold in LDS per workgroup for A_l (and Q_l), P_l and R_l:
     * the largest row block rounded up to whole rounds of 2048, at most 4096. */
    int32_t stream_cap[3];
} amgg_level_view;
int amgg_level_view_get(const amgg_ctx* ctx, int lvl, amgg_level_view* out);
/* Copy level lvl's FP64 smoother values Q^-1 (nnz entries on A_l's pattern, as assembled from
 * Eq. 5; Sec. 3.1) into the caller's device buffer q_out (nnz doubles), ordered on `stream`.
 * Errors: AMGG_EINVAL (bad level or NULL), AMGG_ESTATE (not finalized or no smoother set). */
int amgg_get_smoother_values(const amgg_ctx* ctx, int lvl, double* q_out, void* stream);

/* ------------------------------------------------------------------------------------
 * Smoother: sparse pseudo-inverse Q^{-1} on A_l's pattern (Sec. 3.1, Eq. 5; Alg. 1 step 8)
 *   q_ii = f_d(a_ii/s)/a_ii,  q_ij = f_o(a_ij/s)/(a_ii + a_jj),  s = max |offdiag(A_l)|
 *   f_d(x) = d0 + x(d1 + x(d2 + ...)),  f_o(x) = x(o1 + x(o2 + ...))   (Horner, FP64,
 *   every operation rounded separately, IEEE division).
 * coeffs = (d0..d_deg, o1..o_deg): 2*degree+1 values, degree in [1, AMGG_MAX_DEGREE].
 * ------------------------------------------------------------------------------------ */
/* Host coefficients. When every o_k is zero the smoother is diagonal and the cycle uses
 * the one-pass diagonal (Jacobi-type) step. */
int amgg_set_smoother_coeffs(amgg_ctx* ctx, int lvl, int degree, const double* coeffs, void* stream);
/* Device coefficients (FP32, 2*degree+1 values, e.g. straight from the GCIN output):
 * always assembled as a general sparse smoother; no host synchronisation. */
int amgg_set_smoother_coeffs_device(amgg_ctx* ctx, int lvl, int degree, const float* coeffs_dev, void* stream);
/* The diagonal form of Eq. 5 from device coefficients (diagonal != 0): f_o is taken as 0 whatever
 * the off-diagonal coefficients hold, so Q^{-1} is the diagonal q_ii = f_d(a_ii/s)/a_ii, the cycle
 * uses the one-pass diagonal step on the level, and the coefficient gradients of
 * amgg_vcycle_loss_adjoint(_blocks) for o1..o_deg are 0 there (they are no parameters of the
 * level). A member of the Eq. 5 family chosen for cost: on the large levels the sparse Q^{-1}
 * adds a second pass over the level's matrix to every smoothing step. diagonal == 0 is
 * amgg_set_smoother_coeffs_device. */
int amgg_set_smoother_coeffs_device_form(amgg_ctx* ctx, int lvl, int degree, const float* coeffs_dev, int diagonal,
                                         void* stream);
/* omega-Jacobi, the paper's baseline (Sec. 2.3, Eq. 4; Sec. 4: omega = 2/3) = coeffs (omega, 0, ..). */
int amgg_set_smoother_jacobi(amgg_ctx* ctx, int lvl, double omega, void* stream);

/* ------------------------------------------------------------------------------------
 * Solve phase (Sec. 2.2; Alg. 1, steps 9-10)
 * ------------------------------------------------------------------------------------ */
/* One V(nu1, nu2) cycle u <- V(u, f) on the fine level. f and u are device FP64 vectors of
 * n_0 entries; u is read and overwritten. precision 64 runs the whole cycle in FP64;
 * precision 32 casts f and u to FP32, runs the cycle in FP32 (coarse solve in FP64) and
 * casts back. Pre-smooth nu1 steps u <- u + Q^{-1}(f - A u), restrict r with R = P^T,
 * recurse from a zero guess, prolongate and correct, post-smooth nu2 steps; the coarsest
 * level is solved directly. nu1, nu2 in [0, 8]. */
int amgg_vcycle(amgg_ctx* ctx, int nu1, int nu2, int precision, const double* f, double* u, void* stream);

/* One level operator on its own (the building blocks of the cycle), e.g. to time a kernel
 * or check an operator. Vectors are device arrays of the given precision (float* for 32,
 * double* for 64) sized by the level: x, y, f of n_lvl entries except where noted.
 *   AMGG_OP_SPMV      y = A_l x
 *   AMGG_OP_RESIDUAL  y = f - A_l x
 *   AMGG_OP_SMOOTH    y = y + Q_l^{-1} x        (smoother values on A_l's pattern)
 *   AMGG_OP_JACOBI    y = x + diag(Q_l^{-1}) (f - A_l x)   (the one-pass diagonal step)
 *   AMGG_OP_RESTRICT  y = R_l x, y of n_{l+1} entries          (lvl < nlevels-1)
 *   AMGG_OP_PROLONG   y = y + P_l x, x of n_{l+1} entries      (lvl < nlevels-1)
 *   AMGG_OP_COARSE    y = A_L^{-1} x by the dense inverse       (lvl == nlevels-1)
 * SMOOTH and JACOBI need the level's smoother to be set. */
#define AMGG_OP_SPMV 0
#define AMGG_OP_RESIDUAL 1
#define AMGG_OP_SMOOTH 2
#define AMGG_OP_JACOBI 3
#define AMGG_OP_RESTRICT 4
#define AMGG_OP_PROLONG 5
#define AMGG_OP_COARSE 6
int amgg_level_apply(amgg_ctx* ctx, int lvl, int op, int precision, const void* x, void* y, const void* f,
                     void* stream);
/* Kernel fusion switch (diagnostics and tests). With enable = 1 (the default) the cycle
 * fuses, on every level that admits it, the first pre-smoothing step from u = 0 with the
 * residual after it, and each later smoothing step u <- u + Q^{-1}(f - A u) into one
 * kernel (the residual of a row block and of its halo rows is kept in LDS). Every row sum
 * keeps its order, so the results are bitwise the same as with enable = 0, where each
 * operator is its own pass. Drops the captured solve graphs. */
int amgg_set_fusion(amgg_ctx* ctx, int enable);

/* Column packing of the CSR-stream kernels. amgg_finalize packs the columns of every level
 * matrix, prolongation and restriction as 2-byte offsets from a base column per row block, the
 * few columns outside a block's 16-bit window kept in a per-block list (a matrix with more
 * than 1/8 of its entries outside keeps its plain 4-byte columns). mode 1 (the default) reads
 * the packed columns of matrices with at least 2^24 entries, which stream from HBM (smaller
 * ones stay in the last-level cache, where the packing does not pay); mode 2 reads them for
 * every matrix whose packing fits; mode 0 never. The products and their order are those of
 * the plain CSR walk, so results are bitwise the same in every mode. Drops the captured
 * solve graphs. */
int amgg_set_packed_columns(amgg_ctx* ctx, int mode);

/* The same operator, launched so that the kernel itself records start_event when it begins
 * and stop_event when it ends (both hipEvent_t created by the caller with timing enabled;
 * neither may be NULL): hipEventElapsedTime(start, stop) after completion is that kernel's
 * own execution time, without queueing or launch gaps. Errors as amgg_level_apply. */
int amgg_level_apply_timed(amgg_ctx* ctx, int lvl, int op, int precision, const void* x, void* y, const void* f,
                           void* start_event, void* stop_event, void* stream);

#define AMGG_OUTER_STATIONARY 0 /* u <- V(u, f) repeated (FP64 cycles only) */
#define AMGG_OUTER_IR 1         /* x <- x + V(0, b - A x): iterative refinement, FP64 residual */
#define AMGG_OUTER_FCG 2        /* flexible preconditioned CG, FP64, z = V(0, r) */

typedef struct {
    int outer;            /* AMGG_OUTER_* */
    int inner_precision;  /* 64 or 32 (32 not allowed with STATIONARY) */
    int nu1, nu2;         /* smoothing steps */
    int maxit;            /* iteration limit (Sec. 4 uses 500) */
    double tol;           /* stop when ||b - A x|| <= tol ||b|| */
    int fallback;         /* nonzero: on divergence, stagnation or breakdown switch every
                             level to omega-Jacobi (omega = 2/3) and continue from x */
    double div_factor;    /* diverged if ||r|| > div_factor ||b||; <= 0 means 1e3 */
    double stag_ratio;    /* stagnated if ||r_k|| > stag_ratio ||r_{k-w}||; <= 0 means 0.99 */
    int stag_window;      /* w; <= 0 means 10 */
    int graphs;           /* nonzero: replay each IR / flexible-CG iteration as one captured HIP
                             graph (captured on first use per configuration, kept in the context) */
} amgg_solve_opts;

typedef struct {
    int iterations; /* outer iterations */
    int vcycles;    /* V-cycles applied */
    double relres;  /* final ||b - A x|| / ||b|| as tracked by the method */
    int status;     /* 0 converged, else AMGG_MAXIT / DIVERGED / STAGNATED / BREAKDOWN */
    int fell_back;  /* 1 if the Jacobi fallback was taken */
} amgg_solve_info;

/* Solve A x = b from x = 0 (Sec. 4: V-cycles until the relative residual reaches tol).
 * b, x: device FP64 n_0-vectors (x is overwritten). For a singular hierarchy b is
 * projected to zero mean first. history (host, may be NULL) receives up to history_cap
 * relative residuals, entry 0 being 1. Returns 0 on convergence, a positive outcome code
 * otherwise, negative on error. The host waits for each iteration's scalars (residual norm,
 * flags) while up to two further iterations are already enqueued on the stream; iterations
 * enqueued past the one that stops the solve leave x as it is. Returns with the stream idle. */
int amgg_solve(amgg_ctx* ctx, const amgg_solve_opts* opts, const double* b, double* x,
               amgg_solve_info* info, double* history, int history_cap, void* stream);

/* Judge of the learned smoother. The plain omega-Jacobi AMG is the baseline the learned
 * coefficients must beat in solve time (Sec. 4: acceleration = mean Jacobi solve time over the
 * mean learned-smoother solve time); this call takes that decision on the matrix at hand.
 * It sets the learned smoother on every level (coeffs_dev: device FP32 [nlevels][2*degree+1],
 * e.g. the GCIN output; the diag_levels finest levels in the diagonal form of Eq. 5, as
 * amgg_set_smoother_coeffs_device_form), runs `iters` iterations of the outer loop `opts`
 * (its tol is the target; maxit and fallback are ignored) on b from x = 0, then the same with
 * omega = 2/3 Jacobi on every level. Each run is preceded by an untimed two-iteration run
 * (graph capture) and timed by the host clock around its synchronous iterations. A run that
 * reached tol predicts its own time; otherwise the prediction is ms_per_iter * (iterations +
 * (log10(tol) - log10_relres) / log10_rate), log10_rate being the log10 residual reduction per
 * iteration over the second half of the run (the first iterations fall faster than the rest of
 * a solve will), and infinite when the run diverged, broke down, stagnated or stopped reducing
 * the residual. The context keeps the smoother with the smaller prediction (ties keep
 * Jacobi): learned_wins = 1 leaves the learned coefficients set, 0 leaves omega-Jacobi on every
 * level. b, x: device FP64 n_0-vectors; x is scratch (overwritten; a later amgg_solve with the
 * same b and x replays the graphs captured here). iters in [1, 100]; about 12 separate the
 * solvers' rates on the benchmark meshes. Synchronises the stream. Not available on a
 * block-diagonal context (-4). The decision rests on measured times, so two calls may decide
 * differently when the predictions are close. */
typedef struct {
    int learned_wins;       /* 1: learned smoother kept; 0: omega-Jacobi kept */
    int iterations[2];      /* iterations run by the probe: [0] learned, [1] Jacobi */
    int status[2];          /* the probes' amgg_solve outcomes (0: reached tol) */
    double log10_relres[2]; /* log10 of the relative residual at the end of the probe */
    double log10_rate[2];   /* log10 residual reduction per iteration, second half of the probe */
    double ms_per_iter[2];  /* wall-clock milliseconds per iteration */
    double predicted_ms[2]; /* predicted solve time to tol (INFINITY when unusable) */
} amgg_judge_info;

int amgg_judge_smoother(amgg_ctx* ctx, const amgg_solve_opts* opts, int iters, int degree,
                        const float* coeffs_dev, int diag_levels, const double* b, double* x,
                        amgg_judge_info* info, void* stream);

/* ------------------------------------------------------------------------------------
 * Learning: residual-reduction loss (Sec. 3.3, Eq. 11) of nvc V-cycles from u0 and its
 * gradient with respect to every level's smoother coefficients, by a hand-written adjoint
 * of the cycle that recomputes each level's smoothing iterates from the level's stored
 * entry vector (no per-step storage).
 * ------------------------------------------------------------------------------------ */
/* Coefficients must have been set (all levels, same degree) with amgg_set_smoother_coeffs
 * or amgg_set_smoother_coeffs_device. f, u0: device FP64 (u0 may be NULL for 0).
 * precision 64 or 32. loss_dev: device FP64 scalar; dcoeffs_dev: device FP64
 * [nlevels][2*degree+1] (coarsest row zero). No host synchronisation. */
int amgg_vcycle_loss_adjoint(amgg_ctx* ctx, int nu1, int nu2, int precision, int nvc,
                             const double* f, const double* u0, double* loss_dev,
                             double* dcoeffs_dev, void* stream);

/* ------------------------------------------------------------------------------------
 * Block-diagonal (batched) hierarchies: the independent problems of a training mini-batch
 * (Sec. 3.3-3.4; Alg. 1, steps 7-12) in one context, so that each kernel of a V-cycle and
 * of its adjoint serves all of them at once.
 * ------------------------------------------------------------------------------------ */
/* Declare level lvl (loaded, before amgg_finalize) block-diagonal with nblk blocks: block b
 * holds rows [offsets[b], offsets[b+1]) (host array of nblk+1 entries from 0 to n, no empty
 * block) and is coupled to no other block. Every level needs the same nblk, and P_l must map
 * block b of level l into block b of level l+1 (amgg_finalize checks both). coeff_rows
 * (host, nblk entries; NULL means 0..nblk-1): the row of the coefficient array that block
 * b reads in amgg_set_smoother_coeffs_blocks and whose gradient it receives in
 * amgg_vcycle_loss_adjoint_blocks; -1 means no smoother on that block (Q = 0: with an
 * identity P this passes a problem whose own hierarchy is shallower through the level
 * unchanged). Rows >= 0 must differ within a level. singular (host, nblk entries, may be
 * NULL): on the coarsest level, the blocks whose dense solve takes the rank-one fix of an
 * all-Neumann problem. Each block gets its own off-diagonal scale s of Eq. 5 and its own
 * dense coarsest inverse; amgg_set_smoother_coeffs / _jacobi apply the same coefficients to
 * every block with a coefficient row. amgg_solve is not available on such a context. */
int amgg_set_level_blocks(amgg_ctx* ctx, int lvl, int32_t nblk, const int32_t* offsets,
                          const int32_t* coeff_rows, const int32_t* singular);
/* Eq. 5 smoother of a block-diagonal level: block b uses the degree-`degree` coefficients at
 * coeffs_dev + coeff_rows[b] * stride (device FP32, e.g. the GCIN output for all levels of
 * all problems, one row per level graph; stride >= 2*degree+1). */
int amgg_set_smoother_coeffs_blocks(amgg_ctx* ctx, int lvl, int degree, const float* coeffs_dev,
                                    int32_t stride, void* stream);
/* The same with the form of amgg_set_smoother_coeffs_device_form for every block of the level. */
int amgg_set_smoother_coeffs_blocks_form(amgg_ctx* ctx, int lvl, int degree, const float* coeffs_dev,
                                         int32_t stride, int diagonal, void* stream);
/* amgg_vcycle_loss_adjoint of every block at once: loss_dev[b] (device FP64, nblk) is block
 * b's loss, and the gradient of block b's loss with respect to the coefficients of level l
 * is added to row coeff_rows_l[b] of dcoeffs_dev (device FP64, dcoeff_rows x (2*degree+1),
 * zeroed first; rows no block uses stay 0). f and u0 (may be NULL) hold the blocks' fine
 * vectors one after the other. Sums over a block run in a different order than in
 * amgg_vcycle_loss_adjoint (differences at rounding level). No host synchronisation. */
int amgg_vcycle_loss_adjoint_blocks(amgg_ctx* ctx, int nu1, int nu2, int precision, int nvc,
                                    const double* f, const double* u0, double* loss_dev,
                                    double* dcoeffs_dev, int32_t dcoeff_rows, void* stream);

/* Chain rule through the per-problem losses (Sec. 3.3, Eq. 11; Alg. 1, step 12): with dcoeffs the
 * gradient of each problem's loss with respect to the coefficient rows it owns (device FP64
 * nrows x ncols, as amgg_vcycle_loss_adjoint(_blocks) write it), row_problem[r] the problem that
 * owns row r (device int32, NULL: problem 0 owns every row) and dloss[p] the derivative of an
 * outer objective with respect to problem p's loss (device FP64), writes the objective's
 * gradient out[r][k] = (float)(dcoeffs[r][k] * dloss[row_problem[r]]) (device FP32), which the
 * predictor backward takes. No host synchronisation. */
int amgg_chain_loss_grad(int32_t nrows, int32_t ncols, const double* dcoeffs, const int32_t* row_problem,
                         const double* dloss, float* out, void* stream);

/* Validation metric of Sec. 3.3, Eq. 13 over n held-out problems: out[0] = mean_i (loss[i] -
 * loss_jacobi[i]), where loss[i] and loss_jacobi[i] are the Eq. 11 losses of the same cycles from
 * the same start with the learned and with the omega-Jacobi smoother, so that each difference is
 * log10(||r_n|| / ||r_n^omega-J||); negative means better than Jacobi. Device FP64 arrays, summed
 * in index order. No host synchronisation. */
int amgg_validation_metric(int32_t n, const double* loss, const double* loss_jacobi, double* out, void* stream);

/* out[i] = (float)(in[i] * scale) for i < n (device arrays): hands the FP64 coefficient
 * gradients of amgg_vcycle_loss_adjoint, scaled by 1/|batch| (Alg. 1, step 12: batch-mean
 * loss), to the FP32 predictor backward. */
int amgg_cast_scale_f64_f32(const double* in, float* out, int64_t n, double scale, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* AMGGNN_H */
