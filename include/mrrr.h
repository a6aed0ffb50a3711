/*
 * mrrr.h -- C ABI of libmrrr, an MRRR (Multiple Relatively Robust
 * Representations) eigensolver for real symmetric tridiagonal matrices on
 * AMD Instinct MI355X (gfx950).
 *
 * The problem is the one the thesis states for its MRRR driver (Alg. 3.2 and
 * Sec. 3.2.1): given the diagonal d (alpha_1..alpha_n) and off-diagonal e
 * (beta_1..beta_{n-1}) of T, compute the eigenpairs (lambda_i, z_i) for all
 * i, for the indices il..iu, or for the eigenvalues in the half-open value
 * interval [vl, vu).  Eigenvalues are returned in ascending order; Z holds
 * the matching orthonormal eigenvectors column by column (column-major).
 *
 * Conventions shared by every entry point:
 *  - Pointers marked "device" are HIP device pointers; "host" ones are host
 *    memory.  The caller owns every buffer it passes; the library never
 *    modifies inputs and never frees caller memory.
 *  - All GPU work is enqueued on the handle's stream (mrrr_set_stream); a call
 *    returns after its work is enqueued and, where stated, after a
 *    synchronisation needed to report host-side results.
 *  - Return value: 0 on success; a positive mrrr_status_t on failure or
 *    warning; -(k) when the k-th argument (1-based, handle = 1) is invalid.
 *    Arguments are validated before anything is launched.
 *  - Eigenvector sign: when opts->sign_convention is 1 (default), the entry
 *    of largest magnitude of each vector is positive (ties: lowest index).
 *  - One handle per host thread; calls on one handle must not overlap.
 */
#ifndef MRRR_H
#define MRRR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mrrr_handle_s *mrrr_handle_t;

/* Status codes (positive).  Negative returns name an invalid argument. */
typedef enum {
    MRRR_OK = 0,
    /* A new representation was accepted although its element growth was
     * above the threshold (Alg. 3.8 keeps the candidate of least growth when
     * none passes) and the check of conditional element growth after the tree
     * did not clear it (see stats->n_cond_checked), or a cluster hit the depth
     * limit.  Outputs are filled;
     * stats->n_unverified_rrr says how often, and the columns of such
     * clusters are checked for orthogonality (and corrected when needed)
     * after the tree, with stats->n_check_failed counting the ones that could
     * not be.  The status reports the untested acceptance instead of hiding
     * it (Sec. 3.2.3, remark (6) on the shift selection). */
    MRRR_WARN_UNVERIFIED = 1,
    MRRR_ENOMEM = 2,     /* device allocation or a work-queue capacity failed */
    MRRR_ENOCONV = 3,    /* an eigenvalue failed to converge */
    MRRR_EHIP = 4,       /* a HIP runtime call failed */
                         /* 5 is not used */
    MRRR_ETIMEOUT = 6,   /* the device watchdog stopped the solve */
    MRRR_EINTERNAL = 7   /* an internal consistency check failed */
} mrrr_status_t;

typedef enum {
    MRRR_RANGE_ALL = 0,    /* all n eigenpairs */
    MRRR_RANGE_VALUE = 1,  /* eigenvalues in [vl, vu) (Sec. 3.2.1) */
    MRRR_RANGE_INDEX = 2   /* eigenvalues il..iu, 1-based (Sec. 3.2.1) */
} mrrr_range_t;

/* Tunables.  Defaults from mrrr_default_options follow the thesis. */
typedef struct {
    int32_t jobz;            /* 0: eigenvalues only; 1: eigenvalues and vectors */
    int32_t sign_convention; /* 1: largest-magnitude entry positive; 0: as computed */
    double gaptol;           /* relative gap separating singletons, 1e-3 (Sec. 4.1.4) */
    double rtol_class;       /* classification accuracy, 1e-2*gaptol (Sec. 3.2.2) */
    double perturb_xi;       /* root perturbation bound in units of eps, 8 (Alg. 3.2) */
    uint64_t seed;           /* seed of the root perturbation */
    int32_t max_rqi;         /* Rayleigh-quotient steps before bisection, 10 */
    int32_t max_shift_tries; /* back-off levels per side for a new RRR, 16 (Alg. 3.8) */
    int32_t max_depth;       /* deepest representation tree allowed, 64 */
    int32_t workers;         /* persistent-kernel wavefronts; 0 = fill the GPU */
    int32_t slice_min;       /* smallest refinement slice (eigenvalues), 2 */
    int32_t slice_max;       /* largest refinement slice (eigenvalues), 64 */
    double timeout_s;        /* device watchdog for one solve, seconds (30) */
    double arena_scale;      /* node-pool size factor (1.0); grows on ENOMEM */
    void *trace;             /* device, optional: trace_cap mrrr_trace_t records */
    int64_t trace_cap;       /* 0 = no trace */
    int32_t lanes_per_eig;   /* most lanes one refinement gives one eigenvalue
                                (multisection points, a power of two 1..64);
                                64 by default */
    int32_t bundle;          /* singletons per task (1..64), 64 by default */
    const int32_t *tune;     /* host, optional, batched calls only: for matrix
                                b, tune[3b..3b+2] = lanes_per_eig, bundle,
                                slice_max (an entry <= 0 keeps the value
                                above); read during the call only */
    double check_tol;        /* columns of a cluster whose representation
                                passed no growth test are corrected when
                                max |Z^T Z - I| over them exceeds
                                check_tol * n * eps (20); 0 corrects every
                                checked cluster */
    double cond_growth_k;    /* k_elg of the check of conditional element
                                growth after the tree (Sec. 3.1.2), 10; the
                                bound is (k_elg / 3) n spdiam; 0 switches the
                                check off (every representation that failed the
                                element-growth bound then stays unverified) */
    int32_t bundle_helpers;  /* 1 (default): the worker of a singleton bundle on
                                a representation of 4096 rows or more takes an
                                idle worker, when there is one, to share its
                                twisted factorisations and eigenvector solve
                                (the results are the same bit for bit);
                                0: never */
    int32_t pass_helpers;    /* 1 (default): on a representation of 4096 rows
                                or more, idle workers, when there are any, count
                                multisection points for the refinement of a
                                cluster's end eigenvalues and of the root's
                                extremal eigenvalues (Sec. 4.1.3 R-tasks; the
                                brackets, and so the results, are the same bit
                                for bit); 0: never */
} mrrr_options_t;

/* One record per executed device task (the per-task timeline of the
 * thesis' execution traces, Sec. 4.1.4).  Written in completion order;
 * stats->n_tasks tells how many tasks ran (records beyond trace_cap are
 * dropped). */
typedef struct {
    int32_t type;    /* 1 root, 2 refinement slice, 3 cluster, 4 singleton bundle,
                        5 helper of a cluster's end refinement, 6 helper of a
                        singleton bundle */
    int32_t worker;  /* workgroup (wavefront) index */
    int32_t node;    /* representation the task worked on (root: block) */
    int32_t depth;   /* its depth in the representation tree */
    int32_t a, b;    /* member range (inclusive) or bundle offset and size */
    int64_t t0, t1;  /* device wall-clock ticks (hipDeviceAttributeWallClockRate) */
    double x0, x1;   /* cluster: chosen shift tau and element growth max|D+|;
                        root: shift mu and spectral diameter */
    int32_t flags;   /* cluster: 1 = accepted without passing the growth test */
    int32_t child;   /* cluster: id of the new representation */
} mrrr_trace_t;

/* Per-call statistics (host struct, filled after the work completes). */
typedef struct {
    int64_t m;                 /* eigenpairs computed */
    int64_t n_blocks;          /* irreducible blocks after splitting */
    int64_t n_nodes;           /* representations: roots + clusters */
    int64_t largest_cluster;   /* biggest cluster at any depth */
    int32_t dmax;              /* depth of the representation tree */
    int32_t pad;
    int64_t n_unverified_rrr;  /* RRRs accepted without passing the element-
                                  growth bound of Alg. 3.8 (see n_cond_checked:
                                  those shown afterwards to exhibit conditional
                                  element growth no longer set
                                  MRRR_WARN_UNVERIFIED) */
    int64_t n_bisect_fallback; /* singletons that fell back to bisection */
    int64_t n_nan_retry;       /* twisted-factorisation and eigenvector passes that one
                                  worker redid in IEEE form after a NaN */
    int64_t qd_steps;          /* lane-steps of the qd / Sturm recurrences */
    int64_t n_tasks;           /* device tasks executed */
    int64_t n_singleton_tasks; /* singleton bundles executed */
    int64_t n_rqi_iters;       /* lane Rayleigh-quotient iterations */
    int64_t arena_bytes;       /* node-pool bytes used */
    double ms;                 /* device time of the solve (hipEvent), ms */
    double tree_ms;            /* device time of the persistent tree kernel
                                  alone (hipEvents on the handle's stream
                                  around its launch); 0 for batched calls */
    int64_t n_sturm_guarded;   /* Sturm-count passes that one worker redid in the
                                  guarded quotient form: a zero pivot, an overflow,
                                  or data outside the range of the division-free
                                  count (App. B) */
    int64_t n_checked;         /* clusters whose representation passed no growth
                                  test (at most 64 wanted columns, outermost in
                                  their subtree): Z^T Z of their columns checked
                                  after the tree (remark (6) on Alg. 3.8) */
    int64_t n_reorthogonalized;/* of those, re-orthogonalised because
                                  max |Z^T Z - I| exceeded 20 n eps */
    int64_t n_check_failed;    /* unverified clusters left unchecked (no record
                                  slot) or too far from orthogonal to correct */
    int64_t n_check_wide;      /* unverified clusters with more than 64 wanted
                                  columns: not checked as a whole; those of
                                  their descendants that are unverified and
                                  hold at most 64 wanted columns are */
    int64_t n_cond_checked;    /* representations counted in n_unverified_rrr
                                  that were checked after the tree for
                                  conditional element growth (Sec. 3.1.2):
                                  || |L||D||L^T| |z| || <= (k/3) n spdiam ||z||,
                                  k = opts->cond_growth_k
                                  for the computed vector z of every wanted
                                  member (of 512 evenly spread ones, both ends
                                  included, in a cluster of more; needs
                                  jobz = 1) */
    int64_t n_cond_failed;     /* of those, representations with a vector above
                                  the bound */
    double max_cond_growth;    /* largest || |L||D||L^T| |z| || / (||z|| spdiam)
                                  found by that check */
    int64_t n_factor_quotient; /* shift selections (Alg. 3.8) that one worker
                                  redid in the quotient form of the stationary
                                  transform: data, shift or pivots outside the
                                  range of the division-free form, or no
                                  candidate within the growth bound while one
                                  overflowed */
} mrrr_stats_t;

/* Creates a handle on HIP device `device`.  The handle owns a workspace that
 * grows on demand and is released by mrrr_destroy.  Errors: -1 (h NULL),
 * -2 (bad device), MRRR_EHIP. */
int mrrr_create(mrrr_handle_t *h, int device);

/* Releases the handle and its workspace (synchronises its stream first). */
int mrrr_destroy(mrrr_handle_t h);

/* Sets the stream (a hipStream_t; NULL = the legacy default stream) on which
 * all later work of this handle is enqueued. */
int mrrr_set_stream(mrrr_handle_t h, void *stream);

/* Fills *o with the defaults. */
void mrrr_default_options(mrrr_options_t *o);

/* Human-readable text for a status code (static storage). */
const char *mrrr_status_string(int status);

/* mrrr_dstemr: eigenpairs of T = tridiag(e, d, e) (Alg. 3.2 on each block
 * left by the splitting of Sec. 3.2.1).
 *   n        matrix order, n >= 0.
 *   d        device, n doubles: diagonal alpha_1..alpha_n.
 *   e        device, n-1 doubles: off-diagonal beta_1..beta_{n-1} (may be
 *            NULL when n <= 1).
 *   range    MRRR_RANGE_ALL / _VALUE ([vl, vu), vl < vu) / _INDEX
 *            (1 <= il <= iu+1, iu <= n; il = iu+1 asks for nothing).
 *   opts     host, may be NULL for the defaults.
 *   m        host, out: number of eigenpairs found.  For ALL and INDEX it
 *            is known without waiting; for VALUE the call synchronises.
 *   w        device, >= m doubles, out: ascending eigenvalues.
 *   Z        device, out (ignored when opts->jobz == 0): n x m column-major
 *            with leading dimension ldz >= max(1, n).  For VALUE ranges size
 *            Z for the largest possible m (e.g. n columns).
 *   stats    host, may be NULL.  When non-NULL the call synchronises and
 *            fills it.
 * The call always waits for the device to finish (it must read back the
 * device status word, so that a failure is reported, never hidden).
 * An INDEX range over a matrix that splits into several blocks selects by
 * rank in the direct sum of the blocks; eigenvalues of different blocks that
 * agree to working accuracy are ranked in block order.
 * Errors: negative argument index, MRRR_ENOMEM, MRRR_ETIMEOUT, MRRR_EHIP.
 * MRRR_WARN_UNVERIFIED still fills all outputs. */
int mrrr_dstemr(mrrr_handle_t h, int64_t n, const double *d, const double *e,
                int range, double vl, double vu, int64_t il, int64_t iu,
                const mrrr_options_t *opts, int64_t *m, double *w, double *Z,
                int64_t ldz, mrrr_stats_t *stats);

/* Fills *o with the defaults of the single/double form (Sec. 5.1.1 and the
 * single/double settings of Sec. 5.2.1): gaptol 1e-5, rtol_class 1e-7
 * (1e-2 gaptol), perturb_xi 2^29 (the root's data perturbed by up to
 * eps_single = 2^-24 relative); everything else as mrrr_default_options. */
void mrrr_default_options_mixed(mrrr_options_t *o);

/* mrrr_sstemr: the mixed-precision MRRR of Ch. 5 for single-precision data
 * (single/double): input and output in FP32, every step inside in FP64.
 * The arguments mean what they mean for mrrr_dstemr, with float in place of
 * double for d, e, vl, vu, w and Z (device pointers, Z column-major with
 * ldz >= max(1, n)); opts NULL means mrrr_default_options_mixed.  The data
 * are widened exactly, the matrix splits where |beta_i| <= eps_s sqrt(n)
 * ||T|| (eps_s = 2^-24), the Rayleigh-quotient iteration stops once the local
 * residual is below eps_s sqrt(n) times the gap, and the results are rounded
 * to nearest FP32 as they are written.  The goal is residual and
 * orthogonality of order eps_s sqrt(n).
 * Workspace: the handle keeps FP64 copies of d, e, w and of Z (n x m
 * doubles), grown on demand.
 * Errors: as mrrr_dstemr. */
int mrrr_sstemr(mrrr_handle_t h, int64_t n, const float *d, const float *e,
                int range, float vl, float vu, int64_t il, int64_t iu,
                const mrrr_options_t *opts, int64_t *m, float *w, float *Z,
                int64_t ldz, mrrr_stats_t *stats);

/* mrrr_dsyevr: eigenpairs of a dense real symmetric matrix A by the three
 * stages of Sec. 2.3.2 -- reduction to tridiagonal form A = Q T Q^T, MRRR on
 * T (as mrrr_dstemr), back-transformation Z := Q Z_T.  The reduction and the
 * back-transformation are the library routines of rocSOLVER (Householder
 * tridiagonalisation of the lower triangle, and the application of its
 * reflectors).
 *   A        device, n x n column-major with leading dimension lda >= max(1, n);
 *            only the lower triangle is read; A is not modified (the handle
 *            keeps a reduced copy).
 *   range .. ldz, stats: as mrrr_dstemr, at the same argument positions (A
 *            and lda take the places of d and e).  The sign convention is
 *            applied to the vectors of A.  stats describe the tridiagonal
 *            solve.
 * Workspace: the handle keeps n^2 + 3n doubles and a rocBLAS handle, both
 * created on first use; rocSOLVER allocates its own scratch.
 * The call synchronises the handle's stream before returning.
 * Errors: negative argument index, MRRR_ENOMEM, MRRR_EHIP (including a
 * failure of the reduction or the back-transformation), and those of
 * mrrr_dstemr. */
int mrrr_dsyevr(mrrr_handle_t h, int64_t n, const double *A, int64_t lda,
                int range, double vl, double vu, int64_t il, int64_t iu,
                const mrrr_options_t *opts, int64_t *m, double *w, double *Z,
                int64_t ldz, mrrr_stats_t *stats);

/* Batched form: all eigenpairs of `batch` independent tridiagonals, solved
 * by one persistent launch (no counterpart in the thesis; tridiagonals from
 * many Lanczos runs are the motivating case of Sec. 2.4).
 *   n_offsets host, batch+1 int64: matrix b occupies rows
 *             [n_offsets[b], n_offsets[b+1]) of d_cat and e_cat.
 *   d_cat     device, n_offsets[batch] doubles.
 *   e_cat     device, n_offsets[batch] doubles; e_cat[n_offsets[b]+i] is
 *             beta_{i+1} of matrix b for i < n_b - 1; the last slot of each
 *             matrix is padding and is ignored.
 *   w_cat     device, out: n_offsets[batch] doubles, matrix b's eigenvalues
 *             ascending at [n_offsets[b], n_offsets[b+1]).
 *   Z_cat     device, out: matrix b's n_b x n_b eigenvector matrix
 *             (column-major, ld n_b) starts at z_offsets[b] (host int64 array
 *             of batch entries; NULL means packed: sum over c < b of n_c^2).
 * The first call with a given (batch, sizes, options) builds a plan and
 * captures the launch sequence in a hipGraph; later calls replay it. */
int mrrr_dstemr_batched(mrrr_handle_t h, int64_t batch, const int64_t *n_offsets,
                        const double *d_cat, const double *e_cat,
                        const int64_t *z_offsets, const mrrr_options_t *opts,
                        double *w_cat, double *Z_cat, mrrr_stats_t *stats);

/* Reverse-mode derivative of a loss L(w, Z) through the eigendecomposition
 * of T = tridiag(e, d, e) (all n eigenpairs, as returned by mrrr_dstemr).
 *   w, Z       device: eigenvalues (n) and eigenvectors (n x n, ld ldz).
 *   wbar       device, n doubles: dL/dw (NULL = zero).
 *   Zbar       device, n x n (ld ldzbar): dL/dZ (NULL = zero).
 *   gap_mask_rel  pairs with |w_b - w_a| < gap_mask_rel*||T|| (||T|| =
 *              max|w|) are left out of the eigenvector term and counted.
 *   dbar       device, out, n doubles: dL/dd_j = (Z M Z^T)_jj.
 *   ebar       device, out, n-1 doubles: dL/de_j = (ZMZ^T)_{j,j+1} +
 *              (ZMZ^T)_{j+1,j}, with M = diag(wbar) + F o (Z^T Zbar),
 *              F_ab = 1/(w_b - w_a) off the diagonal.
 *   n_masked   host, out, may be NULL: number of masked (a, b) pairs; the call
 *              synchronises when it is non-NULL.
 * The two products with Z run on FP64 matrix cores. */
int mrrr_dstemr_backward(mrrr_handle_t h, int64_t n, const double *w,
                         const double *Z, int64_t ldz, const double *wbar,
                         const double *Zbar, int64_t ldzbar, double gap_mask_rel,
                         double *dbar, double *ebar, int64_t *n_masked);

/* Batched backward over the layout of mrrr_dstemr_batched: w_cat, wbar_cat,
 * dbar_cat and ebar_cat use n_offsets (ebar keeps one pad slot per matrix,
 * written as 0); Z_cat and Zbar_cat use z_offsets (NULL = packed).  wbar_cat
 * or Zbar_cat may be NULL. */
int mrrr_dstemr_backward_batched(mrrr_handle_t h, int64_t batch,
                                 const int64_t *n_offsets, const double *w_cat,
                                 const double *Z_cat, const int64_t *z_offsets,
                                 const double *wbar_cat, const double *Zbar_cat,
                                 double gap_mask_rel, double *dbar_cat,
                                 double *ebar_cat, int64_t *n_masked);

/* Largest n that mrrr_dstemr_backward_noalloc accepts with an eigenvector
 * cotangent (Zbar non-NULL). */
#define MRRR_BACKWARD_NOALLOC_MAX_N 2048

/* mrrr_dstemr_backward without any device allocation, for callers that
 * cannot allocate: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Arguments, layout and results are those
 * of mrrr_dstemr_backward (same kernels, same values bit for bit).  Instead
 * of the handle's growing workspace it uses one fixed device array per GPU
 * (about 36 MB, held by every GPU the library runs on until the process
 * ends): the problem record, the mask counter, M and the partial sums.
 * Its address is taken once per handle at mrrr_create.
 *   n        with Zbar non-NULL, 0 <= n <= MRRR_BACKWARD_NOALLOC_MAX_N, else
 *            -2 is returned before anything is launched; without Zbar any n.
 * Every call on one GPU shares that GPU's array and overwrites it (the
 * counter is cleared by the call itself): calls that overlap on one GPU,
 * from any handle or stream, race and must be serialised by the caller.
 * The call launches kernels only (no memset, no host-to-device copy); with
 * n_masked non-NULL and Zbar non-NULL it copies the count back and
 * synchronises the stream.
 * Errors: negative argument index, MRRR_EHIP (includes a device on which the
 * array's address could not be taken). */
int mrrr_dstemr_backward_noalloc(mrrr_handle_t h, int64_t n, const double *w,
                                 const double *Z, int64_t ldz, const double *wbar,
                                 const double *Zbar, int64_t ldzbar, double gap_mask_rel,
                                 double *dbar, double *ebar, int64_t *n_masked);

/* Diagnostic: q[i] = a[i] / b[i] by the quotient the kernels use where the
 * shift selection of Alg. 3.8 and a new representation's rows need
 * quotients (the hardware reciprocal, one Newton step and Markstein's
 * residual correction).  For finite, nonzero operands whose IEEE quotient is
 * finite the result is faithful (one of the two doubles next to the exact
 * quotient) and equals IEEE division except where the exact quotient lies
 * within about 2^-70 (relative) of the midpoint between two doubles, since
 * the reciprocal itself is only accurate to 2^-24.  A zero, infinite or NaN
 * divisor, an infinite or NaN dividend, and possibly a quotient within about
 * 2^-24 of overflow, give NaN (the kernels then redo that pass with IEEE
 * division).  a, b, q: device, n doubles each; enqueued on the handle's
 * stream, no synchronisation.
 * Errors: negative argument index, MRRR_EHIP. */
int mrrr_diag_quotient(mrrr_handle_t h, int64_t n, const double *a, const double *b, double *q);

#ifdef __cplusplus
}
#endif

#endif /* MRRR_H */
