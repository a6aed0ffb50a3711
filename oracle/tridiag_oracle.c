/*
 * CPU oracle for the symmetric tridiagonal eigenproblem -- TEST
 * INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and bench.py's
 * cpu_baseline leg may load it; the GPU library never does.
 *
 * What it computes is the plain definition of the result: the wanted
 * eigenvalues of T = tridiag(e, d, e) in ascending order and orthonormal
 * eigenvectors with small residuals.  It gets there the slow, obvious way:
 * bisection followed by inverse iteration (Sec. 2.2, method BI; the LAPACK
 * pair DSTEBZ/DSTEIN):
 *
 *   1. Gershgorin interval (App. B, Alg. B.3), with |beta_1| in the first row.
 *   2. Splitting where |e_i| <= eps*sqrt(n)*bnorm (Sec. 3.2.1, eq. tolsplit).
 *   3. Each eigenvalue by bisection (Alg. 3.3) on the Sturm count of T
 *      (App. B, Alg. B.1) with a pivmin guard, down to the last ulp.
 *   4. Each eigenvector by inverse iteration with a partially pivoted LU of
 *      T - lambda I; eigenvalues closer than orfac*bnorm (orfac = 1e-3) form a
 *      cluster whose vectors are Gram-Schmidt orthogonalised against the
 *      earlier members at every iteration (Sec. 2.2's BI discussion).
 *   5. Sign convention: the entry of largest magnitude is positive (ties to
 *      the lowest index).
 *
 * Plus a cyclic Jacobi solver for dense symmetric matrices (Sec. 2.3's Jacobi
 * method), used as brute force for small n.
 *
 * eps = 2^-53 is the unit roundoff ("half the distance between one and the
 * next larger float", Sec. 1.x notation).  Column-major storage throughout.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EPS 0x1p-53
#define ORC_SAFMIN DBL_MIN

enum { ORC_ALL = 0, ORC_VALUE = 1, ORC_INDEX = 2 };

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ---------------------------------------------------------------------- */
/* App. B, Alg. B.3: Gershgorin interval.  out = {g_l, g_u, bnorm}.        */
/* The printed first row omits |.| on beta_1; the disc radius needs it.    */
void orc_gershgorin(int64_t n, const double *d, const double *e, double *out)
{
    double gl, gu;
    if (n <= 0) { out[0] = out[1] = out[2] = 0.0; return; }
    if (n == 1) {
        gl = gu = d[0];
    } else {
        gl = d[0] - fabs(e[0]);
        gu = d[0] + fabs(e[0]);
        for (int64_t i = 1; i < n - 1; ++i) {
            double r = fabs(e[i - 1]) + fabs(e[i]);
            if (d[i] - r < gl) gl = d[i] - r;
            if (d[i] + r > gu) gu = d[i] + r;
        }
        if (d[n - 1] - fabs(e[n - 2]) < gl) gl = d[n - 1] - fabs(e[n - 2]);
        if (d[n - 1] + fabs(e[n - 2]) > gu) gu = d[n - 1] + fabs(e[n - 2]);
    }
    double bnorm = fmax(fabs(gl), fabs(gu));
    double slack = (2.0 * (double)n + 10.0) * bnorm * ORC_EPS;
    out[0] = gl - slack;
    out[1] = gu + slack;
    out[2] = bnorm;
}

/* Sec. 3.2.1: split where |beta_i| <= eps*sqrt(n)*bnorm.  Writes the block
 * start rows to starts[0..nb) and starts[nb] = n; returns nb. */
int64_t orc_split(int64_t n, const double *e, double bnorm, int64_t *starts)
{
    int64_t nb = 0;
    if (n <= 0) { starts[0] = 0; return 0; }
    double tol = ORC_EPS * sqrt((double)n) * bnorm;
    starts[nb++] = 0;
    for (int64_t i = 0; i < n - 1; ++i)
        if (fabs(e[i]) <= tol) starts[nb++] = i + 1;
    starts[nb] = n;
    return nb;
}

/* pivmin as in the Sturm-count literature: smallest safe pivot magnitude. */
static double orc_pivmin(int64_t n, const double *e)
{
    double m = 1.0;
    for (int64_t i = 0; i < n - 1; ++i) if (e[i] * e[i] > m) m = e[i] * e[i];
    return ORC_SAFMIN * m;
}

/* App. B, Alg. B.1: number of eigenvalues of T smaller than sigma.  A pivot
 * of magnitude below pivmin is replaced by -pivmin (the usual guard that
 * keeps the count exact for a tiny perturbation of T). */
int64_t orc_negcount(int64_t n, const double *d, const double *e,
                     double sigma, double pivmin)
{
    int64_t count = 0;
    if (n <= 0) return 0;
    double piv = d[0] - sigma;
    if (fabs(piv) < pivmin) piv = -pivmin;
    count += (piv < 0.0);
    for (int64_t i = 1; i < n; ++i) {
        piv = (d[i] - sigma) - (e[i - 1] * e[i - 1]) / piv;
        if (fabs(piv) < pivmin) piv = -pivmin;
        count += (piv < 0.0);
    }
    return count;
}

/* Alg. B.1 at many shifts: counts[j] = number of eigenvalues of T below
 * shifts[j], with the pivmin guard of orc_negcount. */
void orc_negcount_many(int64_t n, const double *d, const double *e,
                       int64_t nshift, const double *shifts, int64_t *counts)
{
    double pivmin = orc_pivmin(n, e);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < nshift; ++j)
        counts[j] = orc_negcount(n, d, e, shifts[j], pivmin);
}

/* Alg. 3.3 (bisection) for the k-th (1-based) eigenvalue of one block,
 * starting from [lo, hi] with count(lo) < k <= count(hi).  It runs to full
 * accuracy: until the width is at most max(2*omega, 2*eps*max(|lo|,|hi|)) or
 * no double lies strictly inside (the printed loop test, read as "stop when
 * either tolerance is met"). */
static double orc_bisect_k(int64_t n, const double *d, const double *e,
                           int64_t k, double lo, double hi, double pivmin)
{
    for (int it = 0; it < 4096; ++it) {
        double w = hi - lo;
        double tol = fmax(2.0 * ORC_SAFMIN, 2.0 * ORC_EPS * fmax(fabs(lo), fabs(hi)));
        if (w <= tol) break;
        double mid = lo + 0.5 * w;
        if (!(mid > lo && mid < hi)) break;
        if (orc_negcount(n, d, e, mid, pivmin) < k) lo = mid; else hi = mid;
    }
    return lo + 0.5 * (hi - lo);
}

/* All eigenvalues of one block with local 1-based indices [k0, k1]. */
static void orc_block_eigs(int64_t n, const double *d, const double *e,
                           int64_t k0, int64_t k1, double *w)
{
    if (n == 1) { w[0] = d[0]; return; }   /* 1x1: the eigenvalue is d_1 */
    double g[3];
    orc_gershgorin(n, d, e, g);
    double pivmin = orc_pivmin(n, e);
    /* make sure the bracket is valid for every index */
    double lo = g[0], hi = g[1];
    for (int t = 0; t < 64 && orc_negcount(n, d, e, lo, pivmin) > 0; ++t)
        lo -= fmax(fabs(lo), 1.0);
    for (int t = 0; t < 64 && orc_negcount(n, d, e, hi, pivmin) < n; ++t)
        hi += fmax(fabs(hi), 1.0);
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = k0; k <= k1; ++k)
        w[k - k0] = orc_bisect_k(n, d, e, k, lo, hi, pivmin);
}

/* ---------------------------------------------------------------------- */
/* Counter-based uniform(-1,1) for inverse-iteration start vectors:        */
/* splitmix64 (Steele, Lea, Flood 2014).                                   */
static uint64_t orc_splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

static double orc_uniform(uint64_t seed, uint64_t a, uint64_t b)
{
    uint64_t h = orc_splitmix64(seed ^ orc_splitmix64(a * 0x100000001B3ull + b));
    return ((double)(h >> 11) * 0x1p-53) * 2.0 - 1.0;
}

/* LU factorisation with partial pivoting of the tridiagonal T - shift*I
 * (n >= 1).  U has three diagonals u0 (diag), u1, u2; mult[i] and swp[i]
 * describe the elimination of row i+1.  Pivots below tiny in magnitude are
 * replaced by +-tiny. */
typedef struct {
    double *u0, *u1, *u2, *mult;
    unsigned char *swp;
} orc_lu;

static void orc_lu_factor(int64_t n, const double *d, const double *e,
                          double shift, double tiny, orc_lu *f)
{
    double p = d[0] - shift, q = (n > 1) ? e[0] : 0.0, r = 0.0;
    for (int64_t i = 0; i < n - 1; ++i) {
        double s = e[i];
        double t = d[i + 1] - shift;
        double v = (i + 1 < n - 1) ? e[i + 1] : 0.0;
        if (fabs(p) >= fabs(s)) {
            if (fabs(p) < tiny) p = (p < 0.0) ? -tiny : tiny;
            double m = s / p;
            f->u0[i] = p; f->u1[i] = q; f->u2[i] = r;
            f->mult[i] = m; f->swp[i] = 0;
            p = t - m * q;
            q = v - m * r;
            r = 0.0;
        } else {
            double m = p / s;
            f->u0[i] = s; f->u1[i] = t; f->u2[i] = v;
            f->mult[i] = m; f->swp[i] = 1;
            double np = q - m * t;
            double nq = r - m * v;
            p = np; q = nq; r = 0.0;
        }
    }
    if (fabs(p) < tiny) p = (p < 0.0) ? -tiny : tiny;
    f->u0[n - 1] = p;
    f->u1[n - 1] = 0.0;
    f->u2[n - 1] = 0.0;
}

/* Solve (T - shift I) x = b in place with the factorisation. */
static void orc_lu_solve(int64_t n, const orc_lu *f, double *x)
{
    for (int64_t i = 0; i < n - 1; ++i) {
        if (f->swp[i]) {
            double a = x[i];
            x[i] = x[i + 1];
            x[i + 1] = a - f->mult[i] * x[i];
        } else {
            x[i + 1] -= f->mult[i] * x[i];
        }
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = x[i];
        if (i + 1 < n) s -= f->u1[i] * x[i + 1];
        if (i + 2 < n) s -= f->u2[i] * x[i + 2];
        x[i] = s / f->u0[i];
    }
}

static double orc_nrm2(int64_t n, const double *x)
{
    double scale = 0.0, ssq = 1.0;
    for (int64_t i = 0; i < n; ++i) {
        if (x[i] != 0.0) {
            double a = fabs(x[i]);
            if (scale < a) { ssq = 1.0 + ssq * (scale / a) * (scale / a); scale = a; }
            else ssq += (a / scale) * (a / scale);
        }
    }
    return scale * sqrt(ssq);
}

/* ||T x - lambda x||_2 on one block */
static double orc_resid(int64_t n, const double *d, const double *e,
                        double lambda, const double *x)
{
    double scale = 0.0, ssq = 1.0;
    for (int64_t i = 0; i < n; ++i) {
        double r = (d[i] - lambda) * x[i];
        if (i > 0) r += e[i - 1] * x[i - 1];
        if (i + 1 < n) r += e[i] * x[i + 1];
        if (r != 0.0) {
            double a = fabs(r);
            if (scale < a) { ssq = 1.0 + ssq * (scale / a) * (scale / a); scale = a; }
            else ssq += (a / scale) * (a / scale);
        }
    }
    return scale * sqrt(ssq);
}

/* Sign convention shared with the GPU path: the entry of largest magnitude
 * becomes positive; among entries of equal magnitude the lowest row decides
 * (the strict comparison keeps the first maximum). */
void orc_sign_fix(int64_t n, double *x)
{
    int64_t im = 0;
    double am = -1.0;
    for (int64_t i = 0; i < n; ++i)
        if (fabs(x[i]) > am) { am = fabs(x[i]); im = i; }
    if (x[im] < 0.0)
        for (int64_t i = 0; i < n; ++i) x[i] = -x[i];
}

/* Gram-Schmidt of x against columns Q[:, 0..m) (each length n, ld = ldq),
 * applied twice (a second sweep restores what rounding lost in the first);
 * inner products in parallel when big. */
static void orc_gs(int64_t n, double *x, const double *Q, int64_t ldq, int64_t m,
                   int par)
{
    for (int pass = 0; pass < 2; ++pass) {
        for (int64_t j = 0; j < m; ++j) {
            const double *q = Q + j * ldq;
            double dot = 0.0;
            if (par) {
                #pragma omp parallel for reduction(+:dot) schedule(static)
                for (int64_t i = 0; i < n; ++i) dot += q[i] * x[i];
                #pragma omp parallel for schedule(static)
                for (int64_t i = 0; i < n; ++i) x[i] -= dot * q[i];
            } else {
                for (int64_t i = 0; i < n; ++i) dot += q[i] * x[i];
                for (int64_t i = 0; i < n; ++i) x[i] -= dot * q[i];
            }
        }
    }
}

/* Inverse iteration for the members [c0, c1) of one cluster of one block.
 * lam[] ascending, Zb has ld ldz and row 0 = first row of the block. */
static void orc_cluster_vectors(int64_t n, const double *d, const double *e,
                                double bnorm, const double *lam, int64_t c0,
                                int64_t c1, const int64_t *gidx, double *Zb,
                                int64_t ldz, uint64_t seed, int par)
{
    orc_lu f;
    double *buf = (double *)malloc(sizeof(double) * (size_t)(4 * n + 1));
    f.u0 = buf; f.u1 = buf + n; f.u2 = buf + 2 * n; f.mult = buf + 3 * n;
    f.swp = (unsigned char *)malloc((size_t)n + 1);
    double tiny = ORC_EPS * bnorm;
    if (tiny == 0.0) tiny = ORC_SAFMIN;
    double tol = 2.0 * (double)n * ORC_EPS * bnorm;
    double prev_shift = -INFINITY;
    for (int64_t j = c0; j < c1; ++j) {
        double *x = Zb + j * ldz;
        double lambda = lam[j];
        /* members equal to working precision get distinct shifts so that
         * their factorisations differ (then Gram-Schmidt separates them) */
        double shift = lambda;
        double pertol = 10.0 * fabs(2.0 * ORC_EPS * shift) + 10.0 * ORC_SAFMIN;
        if (j > c0 && shift - prev_shift < pertol) shift = prev_shift + pertol;
        prev_shift = shift;
        if (n == 1) { x[0] = 1.0; continue; }
        orc_lu_factor(n, d, e, shift, tiny, &f);
        for (int64_t i = 0; i < n; ++i) x[i] = orc_uniform(seed, (uint64_t)gidx[j], (uint64_t)i);
        double nr = orc_nrm2(n, x);
        for (int64_t i = 0; i < n; ++i) x[i] /= nr;
        for (int it = 0; it < 10; ++it) {
            orc_lu_solve(n, &f, x);
            if (j > c0) orc_gs(n, x, Zb + c0 * ldz, ldz, j - c0, par);
            nr = orc_nrm2(n, x);
            if (!(nr > 0.0) || !isfinite(nr)) {
                /* restart from a fresh vector (degenerate solve) */
                for (int64_t i = 0; i < n; ++i) x[i] = orc_uniform(seed + 1 + (uint64_t)it, (uint64_t)gidx[j], (uint64_t)i);
                nr = orc_nrm2(n, x);
            }
            for (int64_t i = 0; i < n; ++i) x[i] /= nr;
            if (it >= 2 && orc_resid(n, d, e, lambda, x) <= tol) break;
        }
    }
    free(f.swp);
    free(buf);
}

/* All vectors of one block for the ascending eigenvalues lam[0..m).  Z has
 * ld ldz; rows [0, n) of the given columns are written (block rows). */
static void orc_block_vectors(int64_t n, const double *d, const double *e,
                              double bnorm, const double *lam, int64_t m,
                              const int64_t *gidx, double *Zb, int64_t ldz,
                              uint64_t seed, double orfac)
{
    if (m <= 0) return;
    int64_t *cs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    int64_t nc = 0;
    cs[nc++] = 0;
    for (int64_t j = 1; j < m; ++j)
        if (lam[j] - lam[j - 1] > orfac * bnorm) cs[nc++] = j;
    cs[nc] = m;
    /* large clusters: serial over members (inner products in parallel only
     * when the vectors are long enough to pay for it) */
    for (int64_t c = 0; c < nc; ++c)
        if (cs[c + 1] - cs[c] >= 32)
            orc_cluster_vectors(n, d, e, bnorm, lam, cs[c], cs[c + 1], gidx, Zb, ldz, seed, n >= 8192);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < nc; ++c)
        if (cs[c + 1] - cs[c] < 32)
            orc_cluster_vectors(n, d, e, bnorm, lam, cs[c], cs[c + 1], gidx, Zb, ldz, seed, 0);
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j) orc_sign_fix(n, Zb + j * ldz);
    free(cs);
}

/* ---------------------------------------------------------------------- */
/* The whole solve.  range: 0 all, 1 values in [vl, vu), 2 indices il..iu  */
/* (1-based, of the whole matrix).  w must hold n entries, Z (if non-null) */
/* n x n with ld ldz.  Returns m (number of eigenpairs) or -1 on bad args. */
int64_t orc_solve(int64_t n, const double *d, const double *e, int range,
                  double vl, double vu, int64_t il, int64_t iu, double *w,
                  double *Z, int64_t ldz, uint64_t seed, double orfac)
{
    if (n < 0) return -1;
    if (n == 0) return 0;
    double g[3];
    orc_gershgorin(n, d, e, g);
    int64_t *starts = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t nb = orc_split(n, e, g[2], starts);
    /* effective off-diagonal with the split entries zeroed */
    double *es = (double *)malloc(sizeof(double) * (size_t)(n > 1 ? n - 1 : 1));
    for (int64_t i = 0; i < n - 1; ++i) es[i] = e[i];
    for (int64_t b = 1; b < nb; ++b) es[starts[b] - 1] = 0.0;

    /* per block: wanted local index range */
    int64_t *k0 = (int64_t *)calloc((size_t)nb, sizeof(int64_t));
    int64_t *k1 = (int64_t *)calloc((size_t)nb, sizeof(int64_t));
    int64_t m = 0;
    if (range == ORC_ALL || range == ORC_VALUE) {
        for (int64_t b = 0; b < nb; ++b) {
            int64_t nb_ = starts[b + 1] - starts[b];
            const double *db = d + starts[b], *eb = es + starts[b];
            if (range == ORC_ALL) { k0[b] = 1; k1[b] = nb_; }
            else {
                double pm = orc_pivmin(nb_, eb);
                k0[b] = orc_negcount(nb_, db, eb, vl, pm) + 1;
                k1[b] = orc_negcount(nb_, db, eb, vu, pm);
            }
            if (k1[b] >= k0[b]) m += k1[b] - k0[b] + 1;
        }
    } else if (range == ORC_INDEX) {
        if (il < 1 || iu > n || il > iu + 1) { free(starts); free(es); free(k0); free(k1); return -1; }
        if (nb == 1) { k0[0] = il; k1[0] = iu; m = iu - il + 1; }
        else {
            /* all eigenvalues of every block, then select by global rank */
            for (int64_t b = 0; b < nb; ++b) { k0[b] = 1; k1[b] = starts[b + 1] - starts[b]; }
            m = n;
        }
    } else {
        free(starts); free(es); free(k0); free(k1); return -1;
    }
    /* eigenvalues per block */
    double *lam = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    int64_t *blk = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    int64_t *loc = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    int64_t pos = 0;
    for (int64_t b = 0; b < nb; ++b) {
        if (k1[b] < k0[b]) continue;
        int64_t nb_ = starts[b + 1] - starts[b];
        orc_block_eigs(nb_, d + starts[b], es + starts[b], k0[b], k1[b], lam + pos);
        for (int64_t k = k0[b]; k <= k1[b]; ++k) { blk[pos] = b; loc[pos] = k; ++pos; }
    }
    /* global ascending order (stable insertion by value, then block) */
    int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    for (int64_t i = 0; i < m; ++i) ord[i] = i;
    if (nb > 1) {
        /* merge sort of ord by lam */
        int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
        for (int64_t width = 1; width < m; width *= 2) {
            for (int64_t lo = 0; lo < m; lo += 2 * width) {
                int64_t mid = lo + width < m ? lo + width : m;
                int64_t hi = lo + 2 * width < m ? lo + 2 * width : m;
                int64_t a = lo, c = mid, o = lo;
                while (a < mid && c < hi) tmp[o++] = (lam[ord[c]] < lam[ord[a]]) ? ord[c++] : ord[a++];
                while (a < mid) tmp[o++] = ord[a++];
                while (c < hi) tmp[o++] = ord[c++];
            }
            memcpy(ord, tmp, sizeof(int64_t) * (size_t)m);
        }
        free(tmp);
    }
    int64_t first = 0, mout = m;
    if (range == ORC_INDEX && nb > 1) { first = il - 1; mout = iu - il + 1; }
    for (int64_t i = 0; i < mout; ++i) w[i] = lam[ord[first + i]];

    if (Z != NULL && mout > 0) {
        for (int64_t j = 0; j < mout; ++j) memset(Z + j * ldz, 0, sizeof(double) * (size_t)n);
        /* per block: collect its selected eigenvalues (ascending), solve
         * into a scratch block, scatter to output columns */
        for (int64_t b = 0; b < nb; ++b) {
            int64_t nb_ = starts[b + 1] - starts[b];
            int64_t cnt = 0;
            for (int64_t i = 0; i < mout; ++i) if (blk[ord[first + i]] == b) ++cnt;
            if (cnt == 0) continue;
            double *lb = (double *)malloc(sizeof(double) * (size_t)cnt);
            int64_t *col = (int64_t *)malloc(sizeof(int64_t) * (size_t)cnt);
            int64_t *gid = (int64_t *)malloc(sizeof(int64_t) * (size_t)cnt);
            int64_t c = 0;
            for (int64_t i = 0; i < mout; ++i) {
                int64_t s = ord[first + i];
                if (blk[s] == b) { lb[c] = lam[s]; col[c] = i; gid[c] = starts[b] + loc[s]; ++c; }
            }
            double *Zs = (double *)malloc(sizeof(double) * (size_t)(nb_ * cnt));
            orc_block_vectors(nb_, d + starts[b], es + starts[b], g[2], lb, cnt, gid, Zs, nb_, seed, orfac);
            for (int64_t j = 0; j < cnt; ++j)
                memcpy(Z + col[j] * ldz + starts[b], Zs + j * nb_, sizeof(double) * (size_t)nb_);
            free(Zs); free(lb); free(col); free(gid);
        }
    }
    free(ord); free(lam); free(blk); free(loc);
    free(starts); free(es); free(k0); free(k1);
    return mout;
}

/* Single eigenvalue by global index (1-based), to full accuracy, for
 * sampling large problems one eigenvalue at a time.  The same steps as the
 * whole solve: Gershgorin interval (Alg. B.3), the splitting of Sec. 3.2.1
 * (entries at or below eps*sqrt(n)*bnorm set to zero), an interval checked
 * to hold the whole spectrum, then bisection (Alg. 3.3) on the Sturm count
 * of the split matrix.  With the split entries zero the count of T is the
 * sum of the blocks' counts, so the k-th eigenvalue of T is the k-th of the
 * direct sum of the blocks. */
double orc_eigval_index(int64_t n, const double *d, const double *e, int64_t k)
{
    if (n <= 0 || k < 1 || k > n) return NAN;
    if (n == 1) return d[0];
    double g[3];
    orc_gershgorin(n, d, e, g);
    int64_t *starts = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t nb = orc_split(n, e, g[2], starts);
    double *es = (double *)malloc(sizeof(double) * (size_t)(n - 1));
    for (int64_t i = 0; i < n - 1; ++i) es[i] = e[i];
    for (int64_t b = 1; b < nb; ++b) es[starts[b] - 1] = 0.0;
    double pivmin = orc_pivmin(n, es);
    double lo = g[0], hi = g[1];
    for (int t = 0; t < 64 && orc_negcount(n, d, es, lo, pivmin) > 0; ++t)
        lo -= fmax(fabs(lo), 1.0);
    for (int t = 0; t < 64 && orc_negcount(n, d, es, hi, pivmin) < n; ++t)
        hi += fmax(fabs(hi), 1.0);
    double lam = orc_bisect_k(n, d, es, k, lo, hi, pivmin);
    free(es);
    free(starts);
    return lam;
}

/* ---------------------------------------------------------------------- */
/* Cyclic Jacobi (Sec. 2.3) for a dense symmetric A (n x n, ld lda, it is  */
/* overwritten).  w ascending, V the matching orthonormal eigenvectors     */
/* (sign convention applied).  Returns the number of sweeps.               */
int orc_jacobi(int64_t n, double *A, int64_t lda, double *w, double *V, int64_t ldv)
{
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) V[i + j * ldv] = (i == j) ? 1.0 : 0.0;
    double fro = 0.0;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) fro += A[i + j * lda] * A[i + j * lda];
    fro = sqrt(fro);
    int sweep;
    for (sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i)
                if (i != j) off += A[i + j * lda] * A[i + j * lda];
        if (sqrt(off) <= ORC_EPS * fro) break;
        for (int64_t p = 0; p < n - 1; ++p) {
            for (int64_t q = p + 1; q < n; ++q) {
                double apq = A[p + q * lda];
                if (apq == 0.0) continue;
                double app = A[p + p * lda], aqq = A[q + q * lda];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                /* A <- J^T A J with J the rotation in (p, q) */
                for (int64_t k = 0; k < n; ++k) {
                    double akp = A[k + p * lda], akq = A[k + q * lda];
                    A[k + p * lda] = c * akp - s * akq;
                    A[k + q * lda] = s * akp + c * akq;
                }
                for (int64_t k = 0; k < n; ++k) {
                    double apk = A[p + k * lda], aqk = A[q + k * lda];
                    A[p + k * lda] = c * apk - s * aqk;
                    A[q + k * lda] = s * apk + c * aqk;
                }
                A[p + q * lda] = 0.0;
                A[q + p * lda] = 0.0;
                for (int64_t k = 0; k < n; ++k) {
                    double vkp = V[k + p * ldv], vkq = V[k + q * ldv];
                    V[k + p * ldv] = c * vkp - s * vkq;
                    V[k + q * ldv] = s * vkp + c * vkq;
                }
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) w[i] = A[i + i * lda];
    /* selection sort ascending, permuting V's columns */
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = i;
        for (int64_t j = i + 1; j < n; ++j) if (w[j] < w[k]) k = j;
        if (k != i) {
            double t = w[i]; w[i] = w[k]; w[k] = t;
            for (int64_t r = 0; r < n; ++r) {
                double a = V[r + i * ldv]; V[r + i * ldv] = V[r + k * ldv]; V[r + k * ldv] = a;
            }
        }
    }
    for (int64_t j = 0; j < n; ++j) orc_sign_fix(n, V + j * ldv);
    return sweep;
}
