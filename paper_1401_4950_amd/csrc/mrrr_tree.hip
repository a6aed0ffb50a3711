// MRRR for symmetric tridiagonal matrices on gfx950: the device side.
//
// One wavefront (64 lanes, one workgroup) is one worker.  Workers drain three
// device-side task queues in priority order refine > root/cluster >
// singleton (the R > C > S order of the thesis' task-based MRRR, Sec. 4.1,
// Algs. 4.1-4.3).  Every sweep over a representation stages the rows in LDS
// (D, and the derived D*L and D*L*L of Sec. 4.1.3) so that all 64 lanes read
// the same row from one broadcast; the lanes carry different shifts
// (multisection) or different eigenvalues (singleton bundles).
//
// Numerical kernels, all in FP64:
//   negcount_rep   NegCount on L D L^T (App. B, Alg. B.2): the sign count of
//                  the stationary qd transform.
//   negcount_T     NegCount on T (App. B, Alg. B.1), for the root.
//   dstqds_select  the stationary transform (Alg. 3.5) for the candidate shifts
//   dstqds_values  of Alg. 3.8, one per lane, and the winner's rows, 64-row
//                  tiles in parallel from the selection's checkpoints.
//   twisted        dstqds + the progressive transform (Alg. 3.6) + gamma_k
//                  and the twist index r = argmin |gamma_k| (Alg. 3.7), with
//                  the norm of the solution of N_r^T z = e_r accumulated as
//                  nested sums so that no O(n) per-lane scratch is needed:
//                  the forward pass keeps (s, h) every 16 rows, the backward
//                  pass recomputes each 16-row block in registers.
//   solve_vector   N_r^T z = e_r (Alg. 3.7, lower half) from the same
//                  checkpoints, written straight into Z, normalised.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "mrrr_internal.h"

namespace mrrr {

#define DEV __device__ __forceinline__

constexpr double kEps = 0x1p-53;               // unit roundoff
constexpr double kSafmin = 2.2250738585072014e-308;
constexpr int kMaxPass = 400;

// ---------------------------------------------------------------- helpers

DEV int lane_id() { return (int)threadIdx.x; }

// IEEE sign bit, so that -0 counts as negative (App. B, remark on SignBit).
DEV int sbit(double x) { return (int)((unsigned long long)__double_as_longlong(x) >> 63); }

// The guarded quotient of Algs. 3.5, 3.6 and B.2: q := 1 when both numerator
// and denominator are infinite, else num / den.
DEV double qd_q(double num, double den) {
    return (__builtin_isinf(num) && __builtin_isinf(den)) ? 1.0 : num / den;
}

// Quotients from the hardware reciprocal (relative error below 2^-24 on
// gfx950): with r ~ 1/b and e = 1 - b r, q1 = q0 (1 + e) for q0 = a r leaves
// a relative error of order e^2, and the residual step q1 + (a - b q1) r
// (Markstein's correction) brings it to the last bit.  A zero, infinite or
// NaN operand, where the recurrences need IEEE semantics and the guard of
// qd_q, always leaves a NaN here (0 * inf in e, inf - inf in the residual);
// callers then recompute that quotient with qd_q.  One reciprocal serves all
// quotients by the same pivot.
struct Recip {
    double b, r, e;
};
DEV Recip recip(double b) {
    Recip o;
    o.b = b;
    o.r = __builtin_amdgcn_rcp(b);
    o.e = __builtin_fma(-b, o.r, 1.0);
    return o;
}
DEV double quot(const Recip& x, double a) {
    const double q0 = a * x.r;
    const double q1 = __builtin_fma(q0, x.e, q0);
    const double rem = __builtin_fma(-x.b, q1, a);
    return __builtin_fma(rem, x.r, q1);
}
// Whole-pass forms: G = false takes the reciprocal quotient with no per-row
// test (the caller checks for a NaN once the pass is over and then runs the
// pass again with G = true, the IEEE quotient and the guard).
template <bool G>
DEV double qq(double num, const Recip& x) {
    return G ? qd_q(num, x.b) : quot(x, num);
}
template <bool G>
DEV double dq(double num, const Recip& x) {
    return G ? num / x.b : quot(x, num);
}

DEV int64_t ld_rlx_i64(int64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV int32_t ld_rlx_i32(int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Brackets of other workers' eigenvalues are read and written with relaxed
// agent-scope atomics (a stale value is a wider, still valid bracket).
DEV double ld_rlx_d(double* p) {
    unsigned long long v = __hip_atomic_load((unsigned long long*)p, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)v);
}
DEV void st_rlx_d(double* p, double x) {
    __hip_atomic_store((unsigned long long*)p, (unsigned long long)__double_as_longlong(x),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

DEV void set_error(const Params& P, int code) {
    if (lane_id() == 0) {
        int32_t expect = 0;
        __hip_atomic_compare_exchange_strong(&P.ctl->error, &expect, code, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

DEV void add_stat(int64_t* p, int64_t v) {
    if (lane_id() == 0 && v != 0)
        __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

DEV double wave_min(double x) {
    for (int o = 32; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o));
    return x;
}
DEV double wave_max(double x) {
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
    return x;
}
DEV int wave_or(int x) {
    return __ballot(x != 0) != 0ull;
}

// splitmix64 (Steele, Lea and Flood, 2014): a counter-based generator for the
// pseudo-random relative perturbation of the root (Alg. 3.2).
DEV uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
DEV double unit_pm1(uint64_t seed, uint64_t idx) {
    uint64_t h = splitmix64(seed ^ splitmix64(idx));
    return ((double)(h >> 11) * 0x1p-53) * 2.0 - 1.0;
}

// ---------------------------------------------------------------- LDS

// A worker claims up to kPopMax consecutive tasks of a long queue at once.
constexpr int kPopMax = 8;
// A node's refinement slices are listed in LDS before they are pushed.
constexpr int kMaxSlices = 1024;

// One staged row of a representation or of T, read by all lanes:
//   N-representation (D, L): d = d_i, dll = d_i l_i^2, dl = d_i l_i;
//   T:                       d = alpha_i, dll = beta_{i-1}^2, dl = beta_{i-1}.
// The two values the Sturm counts need come first (one 16-byte LDS read).
struct alignas(32) QRow {
    double d, dll, dl, dl2;   // dl2 = (d l)^2 (representations only)
};
typedef double dv2 __attribute__((ext_vector_type(2)));
// (d, dll) of staged row k in one 16-byte LDS read
#define QROW_DDLL(S, k) (*reinterpret_cast<const dv2*>(&(S).tr[(k)].d))
// rows of three values read ahead of the recurrence (registers for two groups)
constexpr int kAhead = 4;

struct Shared {
    QRow tr[kTile];                           // staged rows
    double m_lo[kWave], m_hi[kWave];          // multisection members
    double m_sig[kWave];
    int64_t m_slot[kWave];
    int32_t m_j[kWave];
    int32_t m_flag[kWave];                    // bit0 lo verified, bit1 hi verified
    int32_t m_cnt[kWave];
    int32_t ulist[kWave];
    Task task[kPopMax];                       // tasks claimed by one pop
    int32_t ibc[8];
    double dbc[8];
    // what the finished task reports to the trace: depth, flags, child, x0, x1
    int32_t info_i[4];
    double info_d[2];
    int32_t redo;                             // twisted / Getvec passes redone in IEEE form
    int32_t redo_sturm;                       // Sturm counts redone in guarded form
    int32_t redo_fac;                         // shift selections redone in quotient form
    int32_t sl_a[kMaxSlices];                 // refinement slices being pushed: first member,
    int8_t sl_q[kMaxSlices];                  //   log2 of the size
};

// Rows [base, base + 64) of an N-representation (D, L): each lane fetches one
// row (rep_fetch, issued one tile ahead so the loads overlap the previous
// tile's arithmetic) and stages D, D*L and D*L*L in LDS (rep_commit) -- the
// derived data that all lanes share.
struct RepRow {
    double d, l;
};

DEV RepRow rep_fetch(const double* D, const double* L, int64_t base, int64_t n) {
    const int64_t r = base + lane_id();
    RepRow f;
    f.d = 0.0;
    f.l = 0.0;
    if (r < n) {
        f.d = D[r];
        if (r < n - 1) f.l = L[r];
    }
    return f;
}

// Returns whether the lane's row is in the range the division-free count
// accepts (kHomData below); the other callers ignore it.
DEV bool rep_commit(Shared& S, const RepRow& f) {
    const int l = lane_id();
    const double dl = f.d * f.l;
    __syncthreads();
    QRow x;
    x.d = f.d;
    x.dll = dl * f.l;
    x.dl = dl;
    x.dl2 = dl * dl;
    S.tr[l] = x;
    __syncthreads();
    return (f.d == 0.0 && f.l == 0.0) ||
           (fabs(x.d) >= 0x1p-150 && fabs(x.d) <= 0x1p150 &&
            (f.l == 0.0 || (fabs(x.dll) >= 0x1p-150 && fabs(x.dll) <= 0x1p150)));
}

// Rows of T (row i couples to row i-1), multiplied by the problem's
// power-of-two scale (exact; see mrrr_setup_kernel).
DEV RepRow T_fetch(const double* d, const double* e, int64_t base, int64_t n, double sc) {
    const int64_t r = base + lane_id();
    RepRow f;
    f.d = 0.0;
    f.l = 0.0;
    if (r < n) {
        f.d = d[r] * sc;
        if (r >= 1) f.l = e[r - 1] * sc;
    }
    return f;
}

// Returns whether the lane's row is in the range the division-free count
// accepts (as rep_commit).
DEV bool T_commit(Shared& S, const RepRow& f) {
    const int l = lane_id();
    __syncthreads();
    QRow x;
    x.d = f.d;
    x.dll = f.l * f.l;
    x.dl = f.l;
    x.dl2 = 0.0;
    S.tr[l] = x;
    __syncthreads();
    return (f.d == 0.0 || (fabs(f.d) >= 0x1p-150 && fabs(f.d) <= 0x1p150)) &&
           (f.l == 0.0 || (fabs(x.dll) >= 0x1p-150 && fabs(x.dll) <= 0x1p150));
}

// ------------------------------------------------------------ Sturm counts

// NegCount(L D L^T, sigma) for one shift per lane (App. B, Alg. B.2).
// Guarded: the quotient is 1 where both operands are infinite.
DEV int negcount_rep_guarded(Shared& S, const double* D, const double* L, int64_t n, double sigma) {
    double s = -sigma;
    int cnt = 0;
    RepRow f = rep_fetch(D, L, 0, n);
    for (int64_t base = 0; base < n; base += kTile) {
        rep_commit(S, f);
        if (base + kTile < n) f = rep_fetch(D, L, base + kTile, n);
        const int lim = (int)((n - base) < kTile ? (n - base) : kTile);
        for (int t = 0; t < lim; ++t) {
            const dv2 x = QROW_DDLL(S, t);
            const double dp = s + x.x;
            cnt += sbit(dp);
            s = qd_q(s, dp) * x.y - sigma;
        }
    }
    return cnt;
}

// The same count without divisions.  With s_i = u_i / v_i the recurrence of
// Alg. B.2 reads
//     w_i = d_i v_i + u_i            (d+_i = w_i / v_i)
//     u_{i+1} = u_i (d_i l_i^2) - sigma w_i,   v_{i+1} = w_i,
// so that sign(d+_i) = sign(w_i) xor sign(w_{i-1}) (v_0 = 1, u_0 = -sigma).
// Each quantity carries one rounding as in the quotient form (one fewer: there
// is no quotient), so the count is that of the same nearby representation the
// error analysis of the stationary transform allows.  The pair (u, v) is
// scaled by a power of two every 8 rows, which changes no sign and no
// rounding.
//
// The relative-error argument needs every rounded result to carry a relative
// error of one rounding (or an absolute one far below it).  It holds when the
// data d_i, d_i l_i^2 and sigma lie in [2^-150, 2^150] (or are zero) and every
// w met, and every v after a rescaling, is at least kHomState = 2^-800:
//   * d_i v_i and u_i lie on the 2^-1074 grid (ulp(d) ulp(v) >= 2^-1054), so
//     their sum w_i is exact when subnormal and zero only when exactly zero;
//     a tiny w fails the check;
//   * |sigma w_i| >= 2^-950, so u_{i+1} is a normal result, or an exact one
//     after a cancellation (then u_i l l d is normal and on the grid), and the
//     at most 2^-1075 that a subnormal product u_i (d l^2) or a rescaled tiny u
//     can be off is below 2^-120 of |u_{i+1}| (|d l^2| <= 2^150).
// A lane outside these bounds, or with a non-finite (u, v) at the end (an
// overflow persists as inf or NaN), counts again with the guarded quotient
// form.  One row costs two dependent fused multiply-adds instead of a
// reciprocal and four corrections; the sign bits of 32 rows are shifted into
// one word and counted with one popcount.
constexpr double kHomData = 0x1p-150;
constexpr double kHomState = 0x1p-800;
// s_waitcnt lgkmcnt(8) (vmcnt and expcnt left at their maxima): the LDS reads
// of the group before the last 8 are complete
constexpr int kWaitLds8 = 0xC87F;

DEV unsigned hi32(double x) { return (unsigned)((unsigned long long)__double_as_longlong(x) >> 32); }

DEV bool hom_sigma_ok(double sigma) {
    return sigma == 0.0 || (fabs(sigma) >= kHomData && fabs(sigma) <= 0x1p150);
}

DEV void hom_rescale(double& u, double& v, double& mw) {
    const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(u), fabs(v)));
    u = __builtin_ldexp(u, -ex);
    v = __builtin_ldexp(v, -ex);
    mw = fmin(mw, fabs(v));
}

DEV int negcount_rep(Shared& S, const double* D, const double* L, int64_t n, double sigma) {
    double u = -sigma, v = 1.0;
    double mw = 1.0;             // smallest |w| met (and |v| after rescaling)
    unsigned B = 0, Bold = 0;    // sign bits of the last rows, newest in bit 0
    int cnt = 0;
    bool data_ok = true;
    RepRow f = rep_fetch(D, L, 0, n);
    for (int64_t base = 0; base < n; base += kTile) {
        data_ok &= (__ballot(!rep_commit(S, f)) == 0ull);
        if (base + kTile < n) f = rep_fetch(D, L, base + kTile, n);
        const int lim = (int)((n - base) < kTile ? (n - base) : kTile);
        if (lim == kTile) {
            dv2 cur[8], nxt[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) cur[k] = QROW_DDLL(S, k);
#pragma unroll
            for (int g = 0; g < kTile / 8; ++g) {
                if (g + 1 < kTile / 8) {
#pragma unroll
                    for (int k = 0; k < 8; ++k) nxt[k] = QROW_DDLL(S, (g + 1) * 8 + k);
                }
                // the next group's LDS reads stay ahead of this group's rows,
                // and one wait covers the 8 rows of this group
                __builtin_amdgcn_sched_barrier(0);
                if (g + 1 < kTile / 8) __builtin_amdgcn_s_waitcnt(kWaitLds8);
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const double w = __builtin_fma(cur[k].x, v, u);
                    const double p = u * cur[k].y;
                    B = __builtin_amdgcn_alignbit(B, hi32(w), 31);
                    u = __builtin_fma(-sigma, w, p);
                    v = w;
                    mw = fmin(mw, fabs(w));
                }
                if ((g & 3) == 3) {
                    // 32 sign bits: a sign change between neighbouring rows
                    // (and between the block's first row and the row before)
                    cnt += __builtin_popcount(B ^ __builtin_amdgcn_alignbit(Bold, B, 1));
                    Bold = B;
                }
                hom_rescale(u, v, mw);
#pragma unroll
                for (int k = 0; k < 8; ++k) cur[k] = nxt[k];
            }
        } else {
            for (int t = 0; t < lim; ++t) {
                const dv2 x = QROW_DDLL(S, t);
                const double w = __builtin_fma(x.x, v, u);
                cnt += sbit(w) ^ sbit(v);
                const double p = u * x.y;
                u = __builtin_fma(-sigma, w, p);
                v = w;
                mw = fmin(mw, fabs(w));
                hom_rescale(u, v, mw);
            }
        }
    }
    // sigma = 0 keeps u = 0 exactly (then w_i = d_i v_i)
    const bool bad = !data_ok || !hom_sigma_ok(sigma) || !(mw >= kHomState) ||
                     !__builtin_isfinite(u) || !__builtin_isfinite(v);
    if (wave_or(bad ? 1 : 0)) {
        const int c2 = negcount_rep_guarded(S, D, L, n, sigma);
        if (bad) cnt = c2;
        if (lane_id() == 0) S.redo_sturm += 1;
    }
    return cnt;
}

// NegCount(T, sigma) for one shift per lane (App. B, Alg. B.1), IEEE form:
// a zero pivot turns the next one into -inf and the count stays right.
DEV int negcount_T_ieee(Shared& S, const double* d, const double* e, int64_t n, double sc, double sigma) {
    double piv = 1.0;
    int cnt = 0;
    RepRow f = T_fetch(d, e, 0, n, sc);
    for (int64_t base = 0; base < n; base += kTile) {
        T_commit(S, f);
        if (base + kTile < n) f = T_fetch(d, e, base + kTile, n, sc);
        const int lim = (int)((n - base) < kTile ? (n - base) : kTile);
        for (int t = 0; t < lim; ++t) {
            const int64_t i = base + t;
            const dv2 x = QROW_DDLL(S, t);
            piv = (i == 0) ? (x.x - sigma) : ((x.x - sigma) - x.y / piv);
            cnt += sbit(piv);
        }
    }
    return cnt;
}

// The same count without divisions: with the leading minors P_i of T - sigma I
// (P_{-1} = 1, P_{-2} = 0) the pivots of Alg. B.1 are q_i = P_i / P_{i-1} and
//     P_i = (alpha_i - sigma) P_{i-1} - beta_{i-1}^2 P_{i-2},
// one fused multiply-add on the dependence chain per row.  The roundings are
// those of the pivot form (the difference, the product with beta^2, the final
// subtraction), with the quotient's rounding gone; (P_{i-1}, P_{i-2}) is
// scaled by a power of two every 8 rows, and the same bounds as for
// negcount_rep (data, sigma, every P met) keep every rounded result normal or
// an exact zero -- the difference alpha_i - sigma is exact or rounded with a
// last bit no finer than 2^-202, so its products stay on the 2^-1074 grid.
// A lane outside them counts again in IEEE form.
DEV int negcount_T(Shared& S, const double* d, const double* e, int64_t n, double sc, double sigma) {
    double a = 1.0, b = 0.0;     // P_{i-1}, P_{i-2}
    double mw = 1.0;
    unsigned B = 0, Bold = 0;
    int cnt = 0;
    bool data_ok = true;
    RepRow f = T_fetch(d, e, 0, n, sc);
    for (int64_t base = 0; base < n; base += kTile) {
        data_ok &= (__ballot(!T_commit(S, f)) == 0ull);
        if (base + kTile < n) f = T_fetch(d, e, base + kTile, n, sc);
        const int lim = (int)((n - base) < kTile ? (n - base) : kTile);
        if (lim == kTile) {
            dv2 cur[8], nxt[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) cur[k] = QROW_DDLL(S, k);
#pragma unroll
            for (int g = 0; g < kTile / 8; ++g) {
                if (g + 1 < kTile / 8) {
#pragma unroll
                    for (int k = 0; k < 8; ++k) nxt[k] = QROW_DDLL(S, (g + 1) * 8 + k);
                }
                __builtin_amdgcn_sched_barrier(0);
                if (g + 1 < kTile / 8) __builtin_amdgcn_s_waitcnt(kWaitLds8);
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const double c = cur[k].x - sigma;
                    const double m = cur[k].y * b;
                    const double pn = __builtin_fma(c, a, -m);
                    B = __builtin_amdgcn_alignbit(B, hi32(pn), 31);
                    b = a;
                    a = pn;
                    mw = fmin(mw, fabs(pn));
                }
                if ((g & 3) == 3) {
                    cnt += __builtin_popcount(B ^ __builtin_amdgcn_alignbit(Bold, B, 1));
                    Bold = B;
                }
                hom_rescale(b, a, mw);
                mw = fmin(mw, fabs(b));
#pragma unroll
                for (int k = 0; k < 8; ++k) cur[k] = nxt[k];
            }
        } else {
            for (int t = 0; t < lim; ++t) {
                const dv2 x = QROW_DDLL(S, t);
                const double pn = __builtin_fma(x.x - sigma, a, -(x.y * b));
                cnt += sbit(pn) ^ sbit(a);
                b = a;
                a = pn;
                mw = fmin(mw, fabs(pn));
                hom_rescale(b, a, mw);
                mw = fmin(mw, fabs(b));
            }
        }
    }
    const bool bad = !data_ok || !hom_sigma_ok(sigma) || !(mw >= kHomState) || !__builtin_isfinite(a) ||
                     !__builtin_isfinite(b);
    if (wave_or(bad ? 1 : 0)) {
        const int c2 = negcount_T_ieee(S, d, e, n, sc, sigma);
        if (bad) cnt = c2;
        if (lane_id() == 0) S.redo_sturm += 1;
    }
    return cnt;
}

// ----------------------------------------------------- multisection engine
//
// Refines the brackets [lo, hi] of up to 64 eigenvalues of one
// representation (members m = 0..M-1 in S.m_*).  Each pass gives every
// unconverged member L = 64 / (#unconverged) lanes (a power of two), each
// lane counting at one interior point; the bracket shrinks to the two
// neighbouring points whose counts straddle the index (Alg. 3.3 with L
// points instead of one).  Bracket ends that were never confirmed by a count
// are checked before a member is declared converged; a failed check widens
// the bracket (as an implementation of Alg. 3.3 must, Sec. 3.2.2).
struct MemberCtx {
    int mode;            // kModeClass: rtol_class, kModeFull: full accuracy
    int32_t na, nb;      // member range of the node (neighbour tests)
    int64_t slot_base;   // slot = slot_base + j
    bool publish;        // write brackets to global memory after every pass
    int lanes;           // most lanes per unconverged member (power of two)
};

DEV double dist0(double a, double b) {   // distance of [a, b] from zero
    return a > 0.0 ? a : (b < 0.0 ? -b : 0.0);
}

// True when reldist(j, j+1) < gaptol for every refinement of the current
// brackets (Sec. 3.2.3 classification): then j and j+1 end up in one cluster
// whatever more bisection does.
DEV bool surely_clustered(double lo1, double hi1, double lo2, double hi2, double gaptol) {
    const double num = hi2 - lo1;
    const double den = fmax(dist0(lo1, hi1), dist0(lo2, hi2));
    return num < gaptol * den;
}

DEV bool bracket_done(const Params& P, int mode, double lo, double hi) {
    const double w = hi - lo;
    const double mx = fmax(fabs(lo), fabs(hi));
    const double mid = lo + 0.5 * w;
    if (!(mid > lo && mid < hi)) return true;          // no double strictly inside
    if (mode == kModeFull) return (w <= 2.0 * kEps * mx) || (w <= 2.0 * kSafmin);
    return w <= fmax(P.rtol * mx, 2.0 * kSafmin);       // Alg. 3.3 stopping rule
}

// The t-th of L multisection points inside (lo, hi), increasing in t.
// Equally spaced, except where the bracket reaches (to within 2^-8 of its
// extent) to zero, where an eigenvalue of the representation may be tiny
// (an eigenvalue next to the root's or a cluster's shift): then half of the
// points are spaced geometrically toward zero, down to 2^-120 of the first
// equally spaced point (and not below 2^-140), so that one pass finds the
// eigenvalue's binade.
// (no geometric point below 2^-140: the division-free count sends shifts
// below 2^-150 to the guarded form; an eigenvalue that small is still found,
// by equally spaced points)
constexpr double kGeoFloor = 0x1p-140;
DEV double geo_point(double a, double x1, int k, int h) {   // k-th of h in (a, x1)
    const double fr = (double)(k + 1) / (double)(h + 1);
    if (!(a >= kGeoFloor && x1 > a)) return x1 * fr;   // too close to zero: equally spaced
    return a * exp2(log2(x1 / a) * fr);
}
DEV double msec_point_pos(double lo, double hi, int t, int L) {   // 0 <= lo < hi
    const int h = L / 2, nl = L - h;
    const double w = hi - lo;
    const double x1 = lo + w / (double)(nl + 1);
    if (t >= h) return lo + w * (double)(t - h + 1) / (double)(nl + 1);
    const double a = fmax(lo, fmax(x1 * 0x1p-120, kGeoFloor));
    return geo_point(a, x1, t, h);
}
DEV double msec_point(double lo, double hi, int t, int L) {
    const double w = hi - lo;
    if (L >= 4 && w > 0.0) {
        if (lo >= 0.0 && lo < hi * 0x1p-8) return msec_point_pos(lo, hi, t, L);
        if (hi <= 0.0 && -hi < -lo * 0x1p-8) return -msec_point_pos(-hi, -lo, L - 1 - t, L);
        if (lo < 0.0 && hi > 0.0) {
            // equally spaced points, and in the gap that holds zero, zero
            // and geometric points toward it on both sides
            const int nl = L / 2, hg = (L - nl - 1) / 2, hp = L - nl - 1 - hg;
            const int k0 = (int)((-lo / w) * (double)(nl + 1));   // equally spaced points below zero
            const int kb = k0 < nl ? k0 : nl;
            if (t < kb) return lo + w * (double)(t + 1) / (double)(nl + 1);
            int u = t - kb;
            const double xl = lo + w * (double)kb / (double)(nl + 1);       // last point below zero (or lo)
            const double xr = lo + w * (double)(kb + 1) / (double)(nl + 1); // first point above zero (or hi)
            if (u < hg) {
                const double m = -fmin(xl, 0.0);
                return -geo_point(fmax(m * 0x1p-120, kGeoFloor), m, hg - 1 - u, hg);
            }
            u -= hg;
            if (u == 0) return 0.0;
            u -= 1;
            if (u < hp) {
                const double m = fmax(xr, 0.0);
                return geo_point(fmax(m * 0x1p-120, kGeoFloor), m, u, hp);
            }
            u -= hp;
            return lo + w * (double)(kb + 1 + u) / (double)(nl + 1);
        }
    }
    return lo + w * (double)(t + 1) / (double)(L + 1);
}

DEV void refine_members(Shared& S, const Params& P, const double* D, const double* L, int64_t n,
                        int M, const MemberCtx& C, int64_t& steps) {
    const int l = lane_id();
    // a joint first pass when all members share one bracket (a fresh root):
    // 64 points spread over the common interval place every member at once
    bool joint = M > 1;
    if (joint) {
        int same = 1;
        if (l < M) same = (S.m_lo[l] == S.m_lo[0] && S.m_hi[l] == S.m_hi[0]) ? 1 : 0;
        joint = __ballot(same == 0) == 0ull;
    }
    if (joint) {
        const double lo = S.m_lo[0], hi = S.m_hi[0];
        const double sig = msec_point(lo, hi, l, kWave);
        const int c = negcount_rep(S, D, L, n, sig);
        steps += (int64_t)n * kWave;
        __syncthreads();
        S.m_cnt[l] = c;
        S.m_sig[l] = sig;
        __syncthreads();
        if (l < M) {
            const int j = S.m_j[l];
            int a = 0, b = kWave;   // first sample whose count reaches j
            while (a < b) {
                const int mid = (a + b) >> 1;
                if (S.m_cnt[mid] >= j) b = mid; else a = mid + 1;
            }
            // only points with a confirmed count become bracket ends
            if (a < kWave && S.m_cnt[a] >= j) { S.m_hi[l] = S.m_sig[a]; S.m_flag[l] |= 2; }
            if (a > 0 && S.m_cnt[a - 1] < j) { S.m_lo[l] = S.m_sig[a - 1]; S.m_flag[l] |= 1; }
        }
        __syncthreads();
    }
    for (int pass = 0; pass < kMaxPass; ++pass) {
        // need: 0 done, 1 bisect the interior, 2 confirm an unverified end
        int need = 0;
        if (l < M) {
            const double lo = S.m_lo[l], hi = S.m_hi[l];
            bool conv = bracket_done(P, C.mode, lo, hi);
            if (!conv && C.mode == kModeClass && C.na >= 0) {
                // neighbours inside the slice: their current brackets (LDS);
                // outside: the brackets the node started with.  Both are
                // fixed by the slice's own inputs, so the outcome does not
                // depend on how other slices are scheduled.
                const int j = S.m_j[l];
                if (j > C.na && j < C.nb) {
                    const int64_t sl = C.slot_base + j;
                    double llo, lhi, rlo, rhi;
                    if (l > 0) { llo = S.m_lo[l - 1]; lhi = S.m_hi[l - 1]; }
                    else { llo = P.lo0[sl - 1]; lhi = P.hi0[sl - 1]; }
                    if (l + 1 < M) { rlo = S.m_lo[l + 1]; rhi = S.m_hi[l + 1]; }
                    else { rlo = P.lo0[sl + 1]; rhi = P.hi0[sl + 1]; }
                    conv = surely_clustered(llo, lhi, lo, hi, P.gaptol) &&
                           surely_clustered(lo, hi, rlo, rhi, P.gaptol);
                }
            }
            need = !conv ? 1 : ((S.m_flag[l] & 3) != 3 ? 2 : 0);
            S.m_cnt[l] = need;
        }
        const uint64_t um = __ballot(need != 0);
        const int nu = __popcll(um);
        if (nu == 0) break;
        if (need != 0) S.ulist[__popcll(um & ((1ull << l) - 1ull))] = l;
        __syncthreads();
        int Lg = 1;
        while (Lg * 2 * nu <= kWave && Lg * 2 <= C.lanes) Lg *= 2;
        const int u = l / Lg;
        const int t = l % Lg;
        const bool valid = (u < nu);
        const int m = valid ? S.ulist[u] : 0;
        const double lo = S.m_lo[m], hi = S.m_hi[m];
        const int j = S.m_j[m];
        const int fm = S.m_flag[m];
        const int needm = S.m_cnt[m];
        const double w = hi - lo;
        int role = 0;        // 0 interior point, 1 confirm lo, 2 confirm hi
        double sig;
        if (needm == 2) {
            const bool vlo = !(fm & 1), vhi = !(fm & 2);
            if (vlo && vhi) role = (Lg >= 2 && (t & 1)) ? 2 : 1;
            else role = vlo ? 1 : 2;
            sig = (role == 1) ? lo : hi;
        } else {
            sig = msec_point(lo, hi, t, Lg);
        }
        if (!valid) sig = 0.0;
        const int c = negcount_rep(S, D, L, n, sig);
        steps += (int64_t)n * (int64_t)__popcll(__ballot(valid));
        // interior points: the first one of the group whose count reaches j
        const int gb = u * Lg;
        const uint64_t gmask = (Lg == 64) ? ~0ull : (((1ull << Lg) - 1ull) << (gb & 63));
        const uint64_t ge = __ballot(valid && role == 0 && c >= j) & gmask;
        const int tstar = ge ? (__ffsll((unsigned long long)ge) - 1 - gb) : Lg;
        const double s_hi = __shfl(sig, gb + (tstar < Lg ? tstar : Lg - 1));
        const double s_lo = __shfl(sig, gb + (tstar > 0 ? tstar - 1 : 0));
        const uint64_t lo_good = __ballot(valid && role == 1 && c < j) & gmask;
        const uint64_t lo_bad = __ballot(valid && role == 1 && c >= j) & gmask;
        const uint64_t hi_good = __ballot(valid && role == 2 && c >= j) & gmask;
        const uint64_t hi_bad = __ballot(valid && role == 2 && c < j) & gmask;
        __syncthreads();
        if (valid && t == 0) {
            double nlo = lo, nhi = hi;
            int nf = fm;
            if (needm != 2) {
                if (tstar < Lg) { nhi = s_hi; nf |= 2; }
                if (tstar > 0) { nlo = s_lo; nf |= 1; }
            } else {
                // a bracket end that fails its count is moved outward by a
                // step that quadruples with every failure (bits 2.. of the
                // flag count them), so any misplaced bracket is recovered in
                // a few dozen passes
                const double mx = fmax(fabs(lo), fabs(hi));
                const int fails = (fm >> 2) & 63;
                const double wid = ldexp(fmax(fmax(w, 4.0 * kEps * mx), 4.0 * kSafmin), 2 * fails);
                if (lo_good) nf |= 1;
                if (hi_good) nf |= 2;
                if (lo_bad) { nlo = lo - wid; nhi = lo; nf = (nf & ~1) | 2; }
                else if (hi_bad) { nhi = hi + wid; nlo = hi; nf = (nf & ~2) | 1; }
                if (lo_bad || hi_bad) nf = (nf & 3) | (((fails < 63 ? fails + 1 : 63)) << 2);
            }
            S.m_lo[m] = nlo;
            S.m_hi[m] = nhi;
            S.m_flag[m] = nf;
        }
        __syncthreads();
        if (C.publish && l < M) {
            st_rlx_d(P.lo + S.m_slot[l], S.m_lo[l]);
            st_rlx_d(P.hi + S.m_slot[l], S.m_hi[l]);
        }
    }
}

// --------------------------------------------- twisted factorisation (RQI)
//
// Per lane: the twisted factorisations N_k Delta_k N_k^T = L D L^T - lam I of
// Alg. 3.7 for its own lam.  Forward: the stationary transform (Alg. 3.5),
// s_i and the running h_i = sum_{k<=i} z_k^2 of the solution with z_i = 1
// (h_{i+1} = 1 + lplus_i^2 h_i), checkpointed every kCkb rows.  Backward: the
// progressive transform (Alg. 3.6, read with omega^-(i+1) := p(i+1) +
// d(i)l(i)^2 on its first line), g_i = 1 + uminus_i^2 g_{i+1}, and
// gamma_i = s_i + d_i * p_{i+1}/omega_{i+1}; r = argmin |gamma_i| (lowest i on
// ties).  Then ||z||^2 = h_r + g_r - 1 for the solution of N_r^T z = e_r.
struct CkPtr {
    double* base;       // this lane's column of the checkpoint region
    int64_t stride;     // distance between checkpoint rows
    DEV double& at(int64_t c, int k) const { return base[(c * kCkSlots + k) * stride]; }
};

struct TwistOut {
    int neg;       // NegCount(lam) = #negative d+
    int r;         // twist index (0-based row)
    double gam;    // gamma_r
    double nrm2;   // ||z||^2 with z_r = 1
    int bad;       // reciprocal pass met a special operand (redo guarded)
    int guarded;   // the result (and the lane's checkpoints) came from the IEEE pass
};

template <bool G>
DEV TwistOut twisted_impl(Shared& S, const double* D, const double* L, int64_t n, double lam, bool live,
                          const CkPtr& ck, int64_t& steps) {
    TwistOut o;
    // ---- forward: dstqds with checkpoints of (s, h); rows read from LDS
    //      in groups of kAhead, one group ahead of the arithmetic
    double s = -lam, h = 1.0, dplast = 0.0;
    int cnt = 0;
    auto row = [&](int64_t i, const QRow& x) {
        if ((i & (kCkb - 1)) == 0 && live) {
            ck.at(i / kCkb, 0) = s;
            ck.at(i / kCkb, 1) = h;
        }
        const double dp = s + x.d;
        cnt += sbit(dp);
        const Recip rc = recip(dp);
        const double q = qq<G>(s, rc);
        const double lp = dq<G>(x.dl, rc);
        h = 1.0 + (lp * lp) * h;
        dplast = dp;
        s = q * x.dll - lam;
    };
    RepRow f = rep_fetch(D, L, 0, n);
    for (int64_t base = 0; base < n; base += kTile) {
        rep_commit(S, f);
        if (base + kTile < n) f = rep_fetch(D, L, base + kTile, n);
        const int lim = (int)((n - base) < kTile ? (n - base) : kTile);
        if (lim == kTile) {
            QRow cur[kAhead], nxt[kAhead];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) cur[u] = S.tr[u];
#pragma unroll
            for (int g = 0; g < kTile / kAhead; ++g) {
                if (g + 1 < kTile / kAhead) {
#pragma unroll
                    for (int u = 0; u < kAhead; ++u) nxt[u] = S.tr[(g + 1) * kAhead + u];
                }
#pragma unroll
                for (int u = 0; u < kAhead; ++u) row(base + g * kAhead + u, cur[u]);
#pragma unroll
                for (int u = 0; u < kAhead; ++u) cur[u] = nxt[u];
            }
        } else {
            for (int t = 0; t < lim; ++t) row(base + t, S.tr[t]);
        }
    }
    steps += n;
    // ---- backward: dqds (progressive) with argmin |gamma|
    const int64_t cl = (n - 1) / kCkb;
    double p = D[n - 1] - lam;
    double g = 1.0;
    double best = fabs(dplast);
    int r = (int)(n - 1);
    double gam_r = dplast, g_r = 1.0;
    if (live) ck.at(cl, 2) = p;
    const int64_t last_tile = ((n - 1) / kTile) * kTile;
    RepRow fb_ = rep_fetch(D, L, last_tile, n);
    // the forward checkpoint of the block after the current one is loaded a
    // block ahead, so that its latency hides behind the current block
    double s_next = live ? ck.at(cl, 0) : 0.0;
    for (int64_t tb = last_tile; tb >= 0; tb -= kTile) {
        rep_commit(S, fb_);
        if (tb - kTile >= 0) fb_ = rep_fetch(D, L, tb - kTile, n);
        const int64_t cfirst = tb / kCkb;
        const int64_t clast = ((tb + kTile - 1) < (n - 1) ? (tb + kTile - 1) : (n - 1)) / kCkb;
        for (int64_t c = clast; c >= cfirst; --c) {
            const double s_blk = s_next;
            s_next = (live && c >= 1) ? ck.at(c - 1, 0) : 0.0;
            const int64_t b0 = c * kCkb;
            const int64_t b1 = (b0 + kCkb) < (n - 1) ? (b0 + kCkb) : (n - 1);   // rows [b0, b1)
            if (b0 >= b1) continue;
            if (c < cl && live) ck.at(c, 2) = p;      // p_{b1}
            // recompute s_i for the block from the forward checkpoint
            double sreg[kCkb];
            QRow xr[kCkb];
#pragma unroll
            for (int t = 0; t < kCkb; ++t) {
                const int k = (int)(b0 + t - tb);
                xr[t] = S.tr[k < kTile ? k : kTile - 1];
            }
            double sr = s_blk;
#pragma unroll
            for (int t = 0; t < kCkb; ++t) {
                sreg[t] = sr;
                if (b0 + t < b1) {
                    const double dp = sr + xr[t].d;
                    sr = qq<G>(sr, recip(dp)) * xr[t].dll - lam;
                }
            }
#pragma unroll
            for (int t = kCkb - 1; t >= 0; --t) {
                if (b0 + t < b1) {
                    const double om = p + xr[t].dll;
                    const Recip rc = recip(om);
                    const double q = qq<G>(p, rc);
                    const double um = dq<G>(xr[t].dl, rc);
                    const double gam = sreg[t] + xr[t].d * q;
                    p = q * xr[t].d - lam;
                    g = 1.0 + (um * um) * g;
                    if (fabs(gam) <= best) {
                        best = fabs(gam);
                        r = (int)(b0 + t);
                        gam_r = gam;
                        g_r = g;
                    }
                }
            }
        }
    }
    steps += 2 * n;
    // ---- h_r from the nearest forward checkpoint (<= kCkb - 1 rows)
    double hr = 1.0;
    if (live) {
        const int64_t c = r / kCkb;
        double sr = ck.at(c, 0);
        hr = ck.at(c, 1);
        for (int64_t i = c * kCkb; i < r; ++i) {
            const double dv = D[i], lv = L[i];
            const double dl = dv * lv, dll = dl * lv;
            const double dp = sr + dv;
            const double q = qd_q(sr, dp);
            const double lp = dl / dp;
            hr = 1.0 + (lp * lp) * hr;
            sr = q * dll - lam;
        }
    }
    o.neg = cnt;
    o.r = r;
    o.gam = gam_r;
    o.nrm2 = hr + g_r - 1.0;
    // a zero or infinite pivot anywhere leaves a NaN in the last s or p
    o.bad = (__builtin_isnan(s) || __builtin_isnan(p)) ? 1 : 0;
    return o;
}

// ------------------------------ division-free twisted factorisation (RQI)
//
// The transforms of Algs. 3.5 and 3.6 in the homogeneous form of negcount_rep:
// forward s_i = u_i / v_i with
//     w_i = d_i v_i + u_i (d+_i = w_i / v_i),  u_{i+1} = (d l^2)_i u_i - lam w_i,  v_{i+1} = w_i,
// backward p_i = x_i / y_i with
//     Om_{i+1} = (d l^2)_i y_{i+1} + x_{i+1} (omega_{i+1} = Om / y_{i+1}),
//     x_i = d_i x_{i+1} - lam Om_{i+1},  y_i = Om_{i+1}.
// Telescoping the products of lplus_i = (d l)_i v_i / w_i and
// uminus_i = (d l)_i y_{i+1} / y_i gives the running sums of Alg. 3.7's
// solution without quotients: h_i = E_i / v_i^2 with
// E_{i+1} = (d l)_i^2 E_i + w_i^2 (E_0 = 1), and g_i = F_i / y_i^2 with
// F_i = (d l)_i^2 F_{i+1} + y_i^2 (F_{n-1} = 1).  The twist index minimises
// |gamma_i| = |u_i Om_{i+1} + d_i x_{i+1} v_i| / |v_i Om_{i+1}|, ranked with the
// hardware reciprocal; gamma_r, h_r and g_r are then recomputed at r alone
// with IEEE quotients.  The eigenvector is division-free too: below r,
// z_i = v_i Y_i with Y_i = -(d l)_i Y_{i+1}; above r, z_k = yh_k X_k with
// X_k = -(d l)_{k-1} X_{k-1}, where yh_k is y_k before its rescaling.
//
// (u, v, E) is scaled by a power of two (v into [1/2, 1)) after every row
// i = 7 mod 8, (x, y, F) after every row i = 0 mod 8, always at the same rows,
// so that the checkpoints -- (u, v, E) entering row 16c and (x, y, F) at the
// top of block c, 6 doubles per 16 rows -- restart either recurrence exactly.
// The range checks of negcount_rep (data, lam, every w and Om at least
// 2^-800, finite states, h and g at least 1/2) send a lane to the guarded
// quotient form, for its factorisation and its eigenvector both.

DEV void hom_fwd_scale(double& u, double& v, double& E) {
    const int ex = __builtin_amdgcn_frexp_exp(v);
    u = __builtin_ldexp(u, -ex);
    v = __builtin_ldexp(v, -ex);
    E = __builtin_ldexp(E, -2 * ex);
}
DEV int hom_bwd_scale(double& x, double& y, double& F) {
    const int ex = __builtin_amdgcn_frexp_exp(y);
    x = __builtin_ldexp(x, -ex);
    y = __builtin_ldexp(y, -ex);
    F = __builtin_ldexp(F, -2 * ex);
    return ex;
}
DEV void row_data(const double* D, const double* L, int64_t n, int64_t i, double& d, double& dll, double& dl,
                  double& dl2) {
    d = D[i];
    const double l = (i < n - 1) ? L[i] : 0.0;
    dl = d * l;
    dll = dl * l;
    dl2 = dl * dl;
}

// The forward half of twisted_hom: the stationary transform over all rows
// with its checkpoints (u, v, E every kCkb rows), the sign count, the
// smallest |w| and the last row's w and v.
struct TwFwd {
    double u, v, E, mw, wl, vl;
    int cnt;
    bool data_ok;
};
DEV TwFwd tw_forward(Shared& S, const double* D, const double* L, int64_t n, double lam, bool live, const CkPtr& ck,
                     int64_t& steps) {
    double u = -lam, v = 1.0, E = 1.0, mw = 1.0;
    double wl = 0.0, vl = 1.0;     // w_{n-1}, v_{n-1}
    unsigned B = 0, Bold = 0;
    int cnt = 0;
    bool data_ok = true;
    RepRow f = rep_fetch(D, L, 0, n);
    for (int64_t base = 0; base < n; base += kTile) {
        data_ok &= (__ballot(!rep_commit(S, f)) == 0ull);
        if (base + kTile < n) f = rep_fetch(D, L, base + kTile, n);
        if (base + kTile < n) {
            // a whole tile that does not hold the last row
            QRow cur[kAhead], nxt[kAhead];
#pragma unroll
            for (int k = 0; k < kAhead; ++k) cur[k] = S.tr[k];
#pragma unroll
            for (int g = 0; g < kTile / kAhead; ++g) {
                if (g + 1 < kTile / kAhead) {
#pragma unroll
                    for (int k = 0; k < kAhead; ++k) nxt[k] = S.tr[(g + 1) * kAhead + k];
                }
#pragma unroll
                for (int k = 0; k < kAhead; ++k) {
                    const int t = g * kAhead + k;
                    if ((t & (kCkb - 1)) == 0 && live) {
                        const int64_t c = (base + t) / kCkb;
                        ck.at(c, 0) = u;
                        ck.at(c, 1) = v;
                        ck.at(c, 2) = E;
                    }
                    const double w = __builtin_fma(cur[k].d, v, u);
                    const double p = u * cur[k].dll;
                    B = __builtin_amdgcn_alignbit(B, hi32(w), 31);
                    u = __builtin_fma(-lam, w, p);
                    E = __builtin_fma(cur[k].dl2, E, w * w);
                    v = w;
                    mw = fmin(mw, fabs(w));
                    if ((t & 7) == 7) hom_fwd_scale(u, v, E);
                    if ((t & 31) == 31) {
                        cnt += __builtin_popcount(B ^ __builtin_amdgcn_alignbit(Bold, B, 1));
                        Bold = B;
                    }
                }
#pragma unroll
                for (int k = 0; k < kAhead; ++k) cur[k] = nxt[k];
            }
        } else {
            const int lim = (int)(n - base);
            for (int t = 0; t < lim; ++t) {
                const int64_t i = base + t;
                const QRow x = S.tr[t];
                if ((i & (kCkb - 1)) == 0 && live) {
                    ck.at(i / kCkb, 0) = u;
                    ck.at(i / kCkb, 1) = v;
                    ck.at(i / kCkb, 2) = E;
                }
                const double w = __builtin_fma(x.d, v, u);
                cnt += sbit(w) ^ sbit(v);
                mw = fmin(mw, fabs(w));
                if (i == n - 1) {
                    wl = w;
                    vl = v;
                } else {
                    const double p = u * x.dll;
                    u = __builtin_fma(-lam, w, p);
                    E = __builtin_fma(x.dl2, E, w * w);
                    v = w;
                    if ((i & 7) == 7) hom_fwd_scale(u, v, E);
                }
            }
        }
    }
    steps += n;
    TwFwd o;
    o.u = u;
    o.v = v;
    o.E = E;
    o.mw = mw;
    o.wl = wl;
    o.vl = vl;
    o.cnt = cnt;
    o.data_ok = data_ok;
    return o;
}

// The end of twisted_hom: gamma_r, h_r and g_r at the twist index r alone
// (IEEE quotients), from the checkpoints of both transforms; `bfin` tells
// whether the backward transform's final state was finite, `mw` is the
// smallest |w| and |omega| of both.
DEV TwistOut tw_at_r(const double* D, const double* L, int64_t n, double lam, bool live, const CkPtr& ck, int r,
                     const TwFwd& f, bool bfin, double mw) {
    TwistOut o;
    const double wl = f.wl, vl = f.vl, E = f.E;
    double gam = wl / vl, hr = E / (vl * vl), gr = 1.0;
    if (live && r < n - 1) {
        const int64_t c = r / kCkb;
        double uu = ck.at(c, 0), vv = ck.at(c, 1), EE = ck.at(c, 2);
        double d, dll, dl, dl2;
        for (int64_t i = c * kCkb; i < r; ++i) {
            row_data(D, L, n, i, d, dll, dl, dl2);
            const double w = __builtin_fma(d, vv, uu);
            const double p = uu * dll;
            uu = __builtin_fma(-lam, w, p);
            EE = __builtin_fma(dl2, EE, w * w);
            vv = w;
            if ((i & 7) == 7) hom_fwd_scale(uu, vv, EE);
        }
        const int64_t b1 = (c * kCkb + kCkb) < (n - 1) ? (c * kCkb + kCkb) : (n - 1);
        double xx = ck.at(c, 3), yy = ck.at(c, 4), FF = ck.at(c, 5);
        for (int64_t i = b1 - 1; i > r; --i) {
            row_data(D, L, n, i, d, dll, dl, dl2);
            const double om = __builtin_fma(dll, yy, xx);
            xx = __builtin_fma(-lam, om, d * xx);
            FF = __builtin_fma(dl2, FF, om * om);
            yy = om;
            if ((i & 7) == 0) hom_bwd_scale(xx, yy, FF);
        }
        row_data(D, L, n, r, d, dll, dl, dl2);
        const double om = __builtin_fma(dll, yy, xx);
        const double m = d * xx;
        gam = __builtin_fma(uu, om, m * vv) / (vv * om);
        hr = EE / (vv * vv);
        gr = __builtin_fma(dl2, FF, om * om) / (om * om);
    }
    o.neg = f.cnt;
    o.r = r;
    o.gam = gam;
    o.nrm2 = hr + gr - 1.0;
    const bool fin = __builtin_isfinite(f.u) && __builtin_isfinite(f.v) && __builtin_isfinite(E) && bfin &&
                     __builtin_isfinite(o.nrm2) && __builtin_isfinite(gam);
    o.bad = (live && (!f.data_ok || !hom_sigma_ok(lam) || !(mw >= kHomState) || !fin || !(hr >= 0.5) ||
                      !(gr >= 0.5))) ? 1 : 0;
    o.guarded = 0;
    return o;
}

DEV TwistOut twisted_hom(Shared& S, const double* D, const double* L, int64_t n, double lam, bool live,
                         const CkPtr& ck, int64_t& steps) {
    const TwFwd fw = tw_forward(S, D, L, n, lam, live, ck, steps);
    const double wl = fw.wl, vl = fw.vl;
    double mw = fw.mw;
    // ---- backward, with the argmin of |gamma|
    const int64_t cl = (n - 1) / kCkb;
    double x = D[n - 1] - lam, y = 1.0, F = 1.0;
    if (live) {
        ck.at(cl, 3) = x;
        ck.at(cl, 4) = y;
        ck.at(cl, 5) = F;
    }
    double best = fabs(wl) * __builtin_amdgcn_rcp(fabs(vl));   // gamma_{n-1} = d+_{n-1}
    int r = (int)(n - 1);
    const int64_t last_tile = ((n - 1) / kTile) * kTile;
    RepRow fb_ = rep_fetch(D, L, last_tile, n);
    double u_next = live ? ck.at(cl, 0) : 0.0, v_next = live ? ck.at(cl, 1) : 1.0;
    for (int64_t tb = last_tile; tb >= 0; tb -= kTile) {
        rep_commit(S, fb_);
        if (tb - kTile >= 0) fb_ = rep_fetch(D, L, tb - kTile, n);
        const int64_t cfirst = tb / kCkb;
        const int64_t clast = ((tb + kTile - 1) < (n - 1) ? (tb + kTile - 1) : (n - 1)) / kCkb;
        for (int64_t c = clast; c >= cfirst; --c) {
            double uu = u_next, vv = v_next;
            u_next = (live && c >= 1) ? ck.at(c - 1, 0) : 0.0;
            v_next = (live && c >= 1) ? ck.at(c - 1, 1) : 1.0;
            const int64_t b0 = c * kCkb;
            const int64_t b1 = (b0 + kCkb) < (n - 1) ? (b0 + kCkb) : (n - 1);   // rows [b0, b1)
            if (b0 >= b1) continue;
            if (c < cl && live) {
                ck.at(c, 3) = x;
                ck.at(c, 4) = y;
                ck.at(c, 5) = F;
            }
            // a whole block (every block but the last) runs without row tests
            const int nb = (int)(b1 - b0);
            auto run = [&](auto full_t) {
                constexpr bool kFull = decltype(full_t)::value;
                const int kb = (int)(b0 - tb);
                QRow xr[kCkb];
#pragma unroll
                for (int t = 0; t < kCkb; ++t) xr[t] = S.tr[kFull ? kb + t : (kb + t < kTile ? kb + t : kTile - 1)];
                // the block's forward states, entering each row
                double ur[kCkb], vr[kCkb];
#pragma unroll
                for (int t = 0; t < kCkb; ++t) {
                    ur[t] = uu;
                    vr[t] = vv;
                    if (kFull || t < nb) {
                        const double w = __builtin_fma(xr[t].d, vv, uu);
                        const double p = uu * xr[t].dll;
                        uu = __builtin_fma(-lam, w, p);
                        vv = w;
                        if ((t & 7) == 7) {
                            const int ex = __builtin_amdgcn_frexp_exp(vv);
                            uu = __builtin_ldexp(uu, -ex);
                            vv = __builtin_ldexp(vv, -ex);
                        }
                    }
                }
                int rt = -1;
#pragma unroll
                for (int t = kCkb - 1; t >= 0; --t) {
                    if (kFull || t < nb) {
                        const double om = __builtin_fma(xr[t].dll, y, x);
                        const double m = xr[t].d * x;
                        const double num = __builtin_fma(ur[t], om, m * vr[t]);
                        const double den = vr[t] * om;
                        const double ga = fabs(num) * __builtin_amdgcn_rcp(fabs(den));
                        const bool take = ga <= best;
                        best = take ? ga : best;
                        rt = take ? t : rt;
                        x = __builtin_fma(-lam, om, m);
                        F = __builtin_fma(xr[t].dl2, F, om * om);
                        y = om;
                        mw = fmin(mw, fabs(om));
                        if ((t & 7) == 0) hom_bwd_scale(x, y, F);
                    }
                }
                if (rt >= 0) r = (int)b0 + rt;
            };
            if (nb == kCkb) run(std::true_type{});
            else run(std::false_type{});
        }
    }
    steps += 2 * n;
    return tw_at_r(D, L, n, lam, live, ck, r, fw,
                   __builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(F), mw);
}

// Alg. 3.7's N_r^T z = e_r in the division-free form (see twisted_hom), from
// the checkpoints of the lane's accepted factorisation: z_r = 1; per 16-row
// block the states are recomputed in registers, then the solution runs
// through the block.  Values scaled by `scale` go to zcol[row] when `write`;
// the sum of squares is returned.
// `part`: 0 the whole vector; 1 the rows below the twist (r+1 .. n-1) alone;
// 2 the rows above it and z_r (the two parts are independent; a bundle's
// helper takes part 1).
DEV double solve_vector_hom(Shared& S, const double* D, const double* L, int64_t n, double lam, bool live, int r,
                            double scale, const CkPtr& ck, double* zcol, bool write, int part, int64_t& steps) {
    // The rows of one block run without branches that depend on r: every lane
    // steps through every row and keeps its running product only on the rows
    // of its own half; the stores and the sum of squares are masked.
    double ss = (live && part != 1) ? 1.0 : 0.0;
    const int64_t cl = (n - 1) / kCkb;
    // ---- upward: z_k = yh_k X_k for k = r+1 .. n-1
    double X = 0.0, dlprev = 0.0;
    if (part != 2) {
        double x_next = live ? ck.at(0, 3) : 0.0, y_next = live ? ck.at(0, 4) : 1.0;
        RepRow fu = rep_fetch(D, L, 0, n);
        for (int64_t tb = 0; tb < n; tb += kTile) {
            rep_commit(S, fu);
            if (tb + kTile < n) fu = rep_fetch(D, L, tb + kTile, n);
            const int64_t cfirst = tb / kCkb;
            const int64_t clast = ((tb + kTile - 1) < (n - 1) ? (tb + kTile - 1) : (n - 1)) / kCkb;
            for (int64_t c = cfirst; c <= clast; ++c) {
                double xx = x_next, yy = y_next;
                x_next = (live && c + 1 <= cl) ? ck.at(c + 1, 3) : 0.0;
                y_next = (live && c + 1 <= cl) ? ck.at(c + 1, 4) : 1.0;
                const int64_t b0 = c * kCkb;
                const int64_t b1 = (b0 + kCkb) < (n - 1) ? (b0 + kCkb) : (n - 1);
                if (b0 >= b1) continue;
                const int rt = r - (int)b0, nb = (int)(b1 - b0);
                // a whole block (every block but the last) runs without row tests
                auto run = [&](auto full_t) {
                    constexpr bool kFull = decltype(full_t)::value;
                    const int kb = (int)(b0 - tb);
                    QRow xr[kCkb];
#pragma unroll
                    for (int t = 0; t < kCkb; ++t) xr[t] = S.tr[kFull ? kb + t : (kb + t < kTile ? kb + t : kTile - 1)];
                    // the block's y before rescaling, and the exponents removed
                    double yh[kCkb];
                    int ex[kCkb];
                    double yr = 1.0;
#pragma unroll
                    for (int t = kCkb - 1; t >= 0; --t) {
                        yh[t] = 1.0;
                        ex[t] = 0;
                        if (kFull || t < nb) {
                            const double om = __builtin_fma(xr[t].dll, yy, xx);
                            xx = __builtin_fma(-lam, om, xr[t].d * xx);
                            yy = om;
                            yh[t] = om;
                            if ((t & 7) == 0) {
                                ex[t] = __builtin_amdgcn_frexp_exp(yy);
                                xx = __builtin_ldexp(xx, -ex[t]);
                                yy = __builtin_ldexp(yy, -ex[t]);
                            }
                        }
                        yr = (t == rt) ? yh[t] : yr;
                    }
                    if (live && rt >= 0 && rt < nb) X = 1.0 / yr;   // X_r
#pragma unroll
                    for (int t = 0; t < kCkb; ++t) {
                        if (kFull || t < nb) {
                            const bool act = live && t > rt;
                            const double Xm = -dlprev * X;
                            const double Xn = ((t & 7) == 0) ? __builtin_ldexp(Xm, -ex[t]) : Xm;
                            X = act ? Xn : X;
                            const double z = act ? yh[t] * X : 0.0;
                            ss = __builtin_fma(z, z, ss);
                            if (write && act) zcol[b0 + t] = z * scale;
                            dlprev = xr[t].dl;
                        }
                    }
                };
                if (nb == kCkb) run(std::true_type{});
                else run(std::false_type{});
            }
        }
        // the last row: yh_{n-1} = y_{n-1} = 1, no rescaling
        if (live && r < n - 1) {
            X = -dlprev * X;
            ss = __builtin_fma(X, X, ss);
            if (write) zcol[n - 1] = X * scale;
        }
    }
    // ---- downward: z_i = v_i Y_i for i = r-1 .. 0
    if (part != 1) {
        double Y = 0.0;
        double u_next = live ? ck.at(cl, 0) : 0.0, v_next = live ? ck.at(cl, 1) : 1.0;
        const int64_t last_tile = ((n - 1) / kTile) * kTile;
        RepRow fb_ = rep_fetch(D, L, last_tile, n);
        for (int64_t tb = last_tile; tb >= 0; tb -= kTile) {
            rep_commit(S, fb_);
            if (tb - kTile >= 0) fb_ = rep_fetch(D, L, tb - kTile, n);
            const int64_t cfirst = tb / kCkb;
            const int64_t clast = ((tb + kTile - 1) < (n - 1) ? (tb + kTile - 1) : (n - 1)) / kCkb;
            for (int64_t c = clast; c >= cfirst; --c) {
                double uu = u_next, vv = v_next;
                u_next = (live && c >= 1) ? ck.at(c - 1, 0) : 0.0;
                v_next = (live && c >= 1) ? ck.at(c - 1, 1) : 1.0;
                const int64_t b0 = c * kCkb;
                const int64_t b1 = (b0 + kCkb) < (n - 1) ? (b0 + kCkb) : (n - 1);
                if (b0 >= b1) {
                    // block cl is empty when n - 1 = 16 cl: v_{n-1} is its checkpoint
                    if (live && r == n - 1) Y = 1.0 / vv;
                    continue;
                }
                const int rt = r - (int)b0, nb = (int)(b1 - b0);
                auto run = [&](auto full_t) {
                    constexpr bool kFull = decltype(full_t)::value;
                    const int kb = (int)(b0 - tb);
                    QRow xr[kCkb];
#pragma unroll
                    for (int t = 0; t < kCkb; ++t) xr[t] = S.tr[kFull ? kb + t : (kb + t < kTile ? kb + t : kTile - 1)];
                    double vr[kCkb];
                    int ex[kCkb];
                    double vrr = 1.0;
#pragma unroll
                    for (int t = 0; t < kCkb; ++t) {
                        vr[t] = vv;
                        ex[t] = 0;
                        vrr = (t == rt) ? vv : vrr;
                        if (kFull || t < nb) {
                            const double w = __builtin_fma(xr[t].d, vv, uu);
                            const double p = uu * xr[t].dll;
                            uu = __builtin_fma(-lam, w, p);
                            vv = w;
                            if ((t & 7) == 7) {
                                ex[t] = __builtin_amdgcn_frexp_exp(vv);
                                uu = __builtin_ldexp(uu, -ex[t]);
                                vv = __builtin_ldexp(vv, -ex[t]);
                            }
                        }
                    }
                    // r == n - 1 with no empty last block: v_{n-1} is the state
                    // after this block's last row
                    const bool rlast = rt == nb && b1 == n - 1 && (n - 1) % kCkb != 0;
                    if (rlast) vrr = vv;
                    if (live && ((rt >= 0 && rt < nb) || rlast)) Y = 1.0 / vrr;   // Y_r
#pragma unroll
                    for (int t = kCkb - 1; t >= 0; --t) {
                        if (kFull || t < nb) {
                            const bool act = live && t < rt;
                            const double Ym = -xr[t].dl * Y;
                            const double Yn = ((t & 7) == 7) ? __builtin_ldexp(Ym, -ex[t]) : Ym;
                            Y = act ? Yn : Y;
                            const double z = act ? vr[t] * Y : 0.0;
                            ss = __builtin_fma(z, z, ss);
                            if (write && act) zcol[b0 + t] = z * scale;
                        }
                    }
                };
                if (nb == kCkb) run(std::true_type{});
                else run(std::false_type{});
            }
        }
    }
    if (live && write && part != 1) zcol[r] = scale;
    steps += (part == 0) ? 2 * n : n;
    return ss;
}

// The twisted factorisation with reciprocal quotients; the lanes that met a
// zero or infinite pivot repeat it with IEEE quotients and the guard.  Only
// those lanes are redone: a lane's eigenvector must later be solved with the
// same arithmetic that produced its checkpoints, because near a tiny pivot
// the rounding of one quotient cancels only against that of its neighbours
// in the same computation.
DEV TwistOut twisted(Shared& S, const double* D, const double* L, int64_t n, double lam, bool live,
                     const CkPtr& ck, int64_t& steps) {
    TwistOut o = twisted_hom(S, D, L, n, lam, live, ck, steps);
    const bool redo = live && o.bad;
    if (wave_or(redo ? 1 : 0)) {
        const TwistOut g = twisted_impl<true>(S, D, L, n, lam, redo, ck, steps);
        if (lane_id() == 0) S.redo += 1;
        if (redo) {
            o = g;
            o.guarded = 1;
        }
    }
    return o;
}


// Solve N_r^T z = e_r (Alg. 3.7): z_r = 1; z_{i+1} = -uminus_i z_i above r;
// z_i = -lplus_i z_{i+1} below r; the zero-pivot rules of Alg. 3.7 where a
// pivot vanished (an index outside the matrix gives 0).  uminus / lplus are
// recomputed per 16-row block from the checkpoints of the accepted
// factorisation.  Each value is scaled by `scale` and stored to zcol[row]
// when `write`; sum of squares returned.
template <bool G>
DEV double solve_vector_impl(Shared& S, const double* D, const double* L, int64_t n, double lam,
                             bool live, int r, double scale, const CkPtr& ck, double* zcol, bool write,
                             int64_t& steps) {
    double ss = live ? 1.0 : 0.0;
    if (live && write) zcol[r] = scale;
    // ---- upward: rows r+1 .. n-1
    double zc = 1.0, zm1 = 0.0, zr1 = 0.0;   // z_i, z_{i-1}, saved z_{r+1}
    const int64_t cl = (n - 1) / kCkb;
    double p_next = live ? ck.at(0, 2) : 0.0;   // checkpoints loaded a block ahead
    RepRow fu = rep_fetch(D, L, 0, n);
    for (int64_t tb = 0; tb < n; tb += kTile) {
        rep_commit(S, fu);
        if (tb + kTile < n) fu = rep_fetch(D, L, tb + kTile, n);
        const int64_t cfirst = tb / kCkb;
        const int64_t clast = ((tb + kTile - 1) < (n - 1) ? (tb + kTile - 1) : (n - 1)) / kCkb;
        for (int64_t c = cfirst; c <= clast; ++c) {
            const double p_blk = p_next;
            p_next = (live && c + 1 <= cl) ? ck.at(c + 1, 2) : 0.0;
            const int64_t b0 = c * kCkb;
            const int64_t b1 = (b0 + kCkb) < (n - 1) ? (b0 + kCkb) : (n - 1);
            if (b0 >= b1) continue;
            double ureg[kCkb];
            QRow xr[kCkb];
#pragma unroll
            for (int t = 0; t < kCkb; ++t) {
                const int k = (int)(b0 + t - tb);
                xr[t] = S.tr[k < kTile ? k : kTile - 1];
            }
            double pr = p_blk;
#pragma unroll
            for (int t = kCkb - 1; t >= 0; --t) {
                ureg[t] = 0.0;
                if (b0 + t < b1) {
                    const double om = pr + xr[t].dll;
                    const Recip rc = recip(om);
                    ureg[t] = (!G || om != 0.0) ? dq<G>(xr[t].dl, rc) : __builtin_inf();
                    pr = qq<G>(pr, rc) * xr[t].d - lam;
                }
            }
#pragma unroll
            for (int t = 0; t < kCkb; ++t) {
                const int64_t i = b0 + t;
                if (i < b1 && i >= r) {
                    double zn;
                    if (!__builtin_isinf(ureg[t])) {
                        zn = -ureg[t] * zc;
                    } else {
                        // omega(i+1) = 0: z_{i+1} = -(d_{i-1} l_{i-1} / d_i l_i) z_{i-1}
                        const int k = (int)(i - tb);
                        zn = 0.0;
                        if (i - 1 >= r && i >= 1) {
                            const double dlm = D[i - 1] * L[i - 1];
                            zn = -(dlm / S.tr[k].dl) * zm1;
                        }
                    }
                    if (i == r) zr1 = zn;
                    zm1 = zc;
                    zc = zn;
                    ss += zn * zn;
                    if (live && write) zcol[i + 1] = zn * scale;
                }
            }
        }
    }
    // ---- downward: rows r-1 .. 0
    zc = 1.0;                // z_{i+1}
    double zp2 = zr1;        // z_{i+2}
    const int64_t last_tile = ((n - 1) / kTile) * kTile;
    double s_next = live ? ck.at(cl, 0) : 0.0;
    RepRow fb_ = rep_fetch(D, L, last_tile, n);
    for (int64_t tb = last_tile; tb >= 0; tb -= kTile) {
        rep_commit(S, fb_);
        if (tb - kTile >= 0) fb_ = rep_fetch(D, L, tb - kTile, n);
        const int64_t cfirst = tb / kCkb;
        const int64_t clast = ((tb + kTile - 1) < (n - 1) ? (tb + kTile - 1) : (n - 1)) / kCkb;
        for (int64_t c = clast; c >= cfirst; --c) {
            const double s_blk = s_next;
            s_next = (live && c >= 1) ? ck.at(c - 1, 0) : 0.0;
            const int64_t b0 = c * kCkb;
            const int64_t b1 = (b0 + kCkb) < (n - 1) ? (b0 + kCkb) : (n - 1);
            if (b0 >= b1) continue;
            double lreg[kCkb];
            QRow xr[kCkb];
#pragma unroll
            for (int t = 0; t < kCkb; ++t) {
                const int k = (int)(b0 + t - tb);
                xr[t] = S.tr[k < kTile ? k : kTile - 1];
            }
            double sr = s_blk;
#pragma unroll
            for (int t = 0; t < kCkb; ++t) {
                lreg[t] = 0.0;
                if (b0 + t < b1) {
                    const double dp = sr + xr[t].d;
                    const Recip rc = recip(dp);
                    lreg[t] = (!G || dp != 0.0) ? dq<G>(xr[t].dl, rc) : __builtin_inf();
                    sr = qq<G>(sr, rc) * xr[t].dll - lam;
                }
            }
#pragma unroll
            for (int t = kCkb - 1; t >= 0; --t) {
                const int64_t i = b0 + t;
                if (i < b1 && i < r) {
                    double zn;
                    if (!__builtin_isinf(lreg[t])) {
                        zn = -lreg[t] * zc;
                    } else {
                        // d+(i) = 0: z_i = -(d_{i+1} l_{i+1} / d_i l_i) z_{i+2}
                        const int k = (int)(i - tb);
                        zn = 0.0;
                        if (i + 1 <= n - 2) {
                            const double dlp = D[i + 1] * L[i + 1];
                            zn = -(dlp / S.tr[k].dl) * zp2;
                        }
                    }
                    zp2 = zc;
                    zc = zn;
                    ss += zn * zn;
                    if (live && write) zcol[i] = zn * scale;
                }
            }
        }
    }
    steps += 2 * n;
    return ss;
}

// Getvec in the arithmetic of the lane's accepted factorisation: reciprocal
// quotients, or IEEE quotients with the guard for lanes whose factorisation
// needed them (`guarded`); a NaN from the reciprocal pass (the zero-pivot
// rules of Alg. 3.7 need IEEE infinities) also sends a lane to the IEEE
// pass, which rewrites every entry of its column.
DEV double solve_vector(Shared& S, const double* D, const double* L, int64_t n, double lam, bool live, int r,
                        double scale, const CkPtr& ck, double* zcol, bool write, bool guarded, int64_t& steps) {
    double ss = solve_vector_hom(S, D, L, n, lam, live && !guarded, r, scale, ck, zcol, write, 0, steps);
    const bool redo = live && (guarded || __builtin_isnan(ss));
    if (wave_or(redo ? 1 : 0)) {
        const double sg = solve_vector_impl<true>(S, D, L, n, lam, redo, r, scale, ck, zcol, write, steps);
        if (redo) ss = sg;
        if (lane_id() == 0) S.redo += 1;
    }
    return ss;
}

// ------------------------------------------------------------- queues
//
// Bounded multi-producer multi-consumer rings, one per priority class.  Each
// cell carries a sequence number: pos when free for the producer of ticket
// pos, pos + 1 when it holds that producer's task, pos + cap once consumed.

// Claims tasks at the head of queue q into out[]; returns how many (0 when
// the queue is empty).  A consumer first takes a share of the count of
// published, unclaimed tasks (one fetch-and-add; a share the count did not
// cover is given back), then its tickets at the head (a second
// fetch-and-add).  Neither step can fail and be retried, so a burst of
// claims costs two atomic operations each however many workers contend; a
// compare-and-swap on the head would let only one of them through per round
// trip.  Every ticket taken this way has been reserved by a producer, since
// the claims never exceed the tasks published.  One task per claim while the
// queue is short, so that parallel work spreads over the workers; about
// (queued / workers) tasks, up to kPopMax, when it is long.  A claimed cell
// that its producer has reserved but not yet published is waited for.
DEV int try_pop(const Params& P, int q, Task* out) {   // one lane
    // Polling uses relaxed loads only: an acquire at agent scope invalidates
    // the L2, and idle workers poll often.  The acquire follows a claim.
    const uint64_t cap = P.qcap[q];
    int64_t* av = P.ctl->avail(q);
    const int64_t seen = __hip_atomic_load(av, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (seen <= 0) return 0;
    const int64_t nw = P.nworkers;
    int64_t k = (seen + nw - 1) / nw;
    k = k < 1 ? 1 : (k > kPopMax ? kPopMax : k);
    if (k > 1 && seen < 2 * nw) k = 1;
    const int64_t old = __hip_atomic_fetch_add(av, -k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t got = old >= k ? k : (old > 0 ? old : 0);
    if (got < k) __hip_atomic_fetch_add(av, k - got, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (got == 0) return 0;
    const uint64_t pos = __hip_atomic_fetch_add(P.ctl->head(q), (uint64_t)got, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    // every claimed cell published (relaxed polls), then one acquire for the
    // cells and the data their tasks refer to
    for (int64_t i = 0; i < got; ++i) {
        const uint64_t c = (pos + i) % cap;
        int wait = 0;
        while (__hip_atomic_load(&P.seq[q][c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != pos + i + 1) {
            // a producer whose push failed never publishes: the error ends the wait
            if (++wait > (1 << 24) ||
                ((wait & 1023) == 0 && __hip_atomic_load(&P.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                set_error(P, kErrInternal);
                return 0;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    for (int64_t i = 0; i < got; ++i) out[i] = P.q[q][(pos + i) % cap];
    // the cells go back to the producers once the loads are done
    __builtin_amdgcn_s_waitcnt(0);
    for (int64_t i = 0; i < got; ++i)
        __hip_atomic_store(&P.seq[q][(pos + i) % cap], pos + i + cap, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (int)got;
}

// Lane 0 reserves `count` tickets; every lane fills some of the cells.  One
// agent-scope release after all cells are written publishes them together
// with everything this wave wrote before (a release writes back the XCD's L2,
// so it is paid once per push, not once per cell); the sequence numbers then
// go out as relaxed stores.
DEV uint64_t push_reserve(const Params& P, int q, int count) {
    uint64_t first = 0;
    if (lane_id() == 0) {
        __hip_atomic_fetch_add(&P.ctl->pending, (int64_t)count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        first = __hip_atomic_fetch_add(P.ctl->tail(q), (uint64_t)count, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
    }
    return __shfl(first, 0);
}

// Waits (bounded) until the cell of ticket `pos` is free, then writes it.
DEV bool push_fill(const Params& P, int q, uint64_t pos, const Task& t) {
    const uint64_t cell = pos % P.qcap[q];
    int spin = 0;
    while (__hip_atomic_load(&P.seq[q][cell], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != pos) {
        if (++spin > (1 << 22) || __hip_atomic_load(&P.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return false;
        __builtin_amdgcn_s_sleep(1);
    }
    P.q[q][cell] = t;
    return true;
}

DEV bool push_publish(const Params& P, int q, uint64_t first, int count, bool ok) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (ok) {
        for (int k = lane_id(); k < count; k += kWave) {
            const uint64_t pos = first + (uint64_t)k;
            __hip_atomic_store(&P.seq[q][pos % P.qcap[q]], pos + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // the tasks become claimable (consumers wait for the cells themselves)
    if (__ballot(!ok) == 0ull && lane_id() == 0)
        __hip_atomic_fetch_add(P.ctl->avail(q), (int64_t)count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__ballot(!ok) != 0ull) {
        set_error(P, kErrNoMem);
        return false;
    }
    return true;
}

template <class Gen>
DEV bool push_batch(const Params& P, int q, int count, Gen gen) {
    if (count <= 0) return true;
    const uint64_t first = push_reserve(P, q, count);
    bool ok = true;
    for (int k = lane_id(); k < count && ok; k += kWave) ok = push_fill(P, q, first + (uint64_t)k, gen(k));
    return push_publish(P, q, first, count, ok);
}

DEV bool push_one(const Params& P, int q, Task t) {
    return push_batch(P, q, 1, [&](int) { return t; });
}

// Refinement slices of members [a, b] of a node (R-tasks of Sec. 4.1.3),
// sized by the work each member still needs.  A member whose bracket must
// shrink by 2^bits to reach the accuracy of `mode` needs bits / log2(L + 1)
// multisection passes with L points; a slice of s members gives each
// L = 64 / s points (at most `lanes`).  For a pass budget Pb every member has
// a capacity -- the largest power-of-two slice that still finishes it in Pb
// passes -- and each 64-member chunk is cut into the largest aligned
// power-of-two blocks whose members all fit.  Pb starts at what the hardest
// member needs alone and grows until the slices number at most the node's
// share of the workers (the workers times the share of all rows that the
// block has), so that one round of slices finishes the node: the
// refinement's critical path is the hardest member's passes, not a fixed
// slice size's.  Slices are at least slice_min (a power of two) and at most
// smax members.
DEV int member_bits(const Params& P, int mode, double lo, double hi) {
    const double w = hi - lo;
    const double mx = fmax(fabs(lo), fabs(hi));
    const double tgt = (mode == kModeFull) ? fmax(2.0 * kEps * mx, 2.0 * kSafmin) : fmax(P.rtol * mx, 2.0 * kSafmin);
    if (!(w > tgt)) return 0;
    const double ratio = w / tgt;
    int bits = __builtin_isfinite(ratio) ? __builtin_amdgcn_frexp_exp(ratio) : 1100;
    // a bracket that reaches zero may hold a tiny eigenvalue: the binade
    // search costs about one more pass (a larger estimate sizes the other
    // slices for more passes than the level takes; none leaves the hard
    // member alone on the critical path)
    const bool reach = (lo <= 0.0 && hi >= 0.0) || (lo > 0.0 && lo < hi * 0x1p-8) || (hi < 0.0 && hi > lo * 0x1p-8);
    if (reach) bits += 6;
    return bits < 255 ? bits : 255;
}

DEV double slice_bpp(int s, int lanes) {   // bits per pass of an s-member slice
    int lg = kWave / s;
    if (lg > lanes) lg = lanes;
    return log2((double)lg + 1.0);
}

// The cut of a 64-member chunk.  mb[q] = the most bits any member of the
// lane's aligned block of 2^q members needs (members past the node's end
// need none); a block of s members fits the pass budget Pb when
// Pb * (bits per pass of an s-member slice) covers its mb.  The lane's slice
// is its largest fitting block (between 2^qmin and 2^qmax members).
DEV void chunk_maxbits(int bits, int* mb) {
    int m = bits;
    mb[0] = m;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        m = max(m, __shfl_xor(m, 1 << q));
        mb[q + 1] = m;
    }
}
// The most bits a member of an aligned block of 2^k members can still get
// within the pass budget Pb, cap[k] = floor((Pb - cf) * bpp) for k = 1..6
// (bpp[i] and cf[i] are for slices of 64 >> i members, i.e. q = 6 - i; cf
// passes confirm the members' unverified bracket ends first).  An integer
// need fits exactly when it is at most cap[k].
DEV void slice_caps(double Pb, const double* bpp, const int* cf, int* cap) {
    cap[0] = 0;
#pragma unroll
    for (int k = 1; k <= 6; ++k) cap[k] = (int)floor((Pb - (double)cf[6 - k]) * bpp[6 - k]);
}
DEV int slice_q(const int* mb, const int* cap, int qmin, int qmax) {
    // the largest fitting q in (qmin, qmax], else qmin; every block size is
    // tested (constant indices keep the arrays in registers)
    int q = qmin;
#pragma unroll
    for (int k = 1; k <= 6; ++k) {
        const bool fit = mb[k] <= cap[k];
        q = (k > qmin && k <= qmax && fit) ? k : q;
    }
    return q;
}

// The members' needs are in P.need (written with their brackets, see
// member_bits); maxbits is the largest.  Eight pass budgets are counted in one
// sweep over the members.
DEV void push_slices(Shared& S, const Params& P, int node_id, int a, int b, int mode, double share, int smax,
                     int64_t sb, int lanes, int maxbits) {
    const int l = lane_id();
    const int budget = share < 1.0 ? 1 : (int)share;
    int qmin = 0, qmax = 0;
    while ((1 << (qmin + 1)) <= P.slice_min && qmin < 6) ++qmin;
    while ((1 << (qmax + 1)) <= smax && qmax < 6) ++qmax;
    if (qmax < qmin) qmax = qmin;
    double bpp[6];   // bits per pass of slices of 64 >> k members
    int cf[6];       // passes that confirm unverified ends: one, or two with one lane a member
    for (int k = 0; k < 6; ++k) {
        bpp[k] = slice_bpp(kWave >> k, lanes);
        cf[k] = ((1 << k) < lanes ? (1 << k) : lanes) >= 2 ? 1 : 2;
    }
    const double best_bpp = slice_bpp(1 << qmin, lanes);
    const int best_cf = ((kWave >> qmin) < lanes ? (kWave >> qmin) : lanes) >= 2 ? 1 : 2;
    int P0 = best_cf + (int)ceil((double)maxbits / best_bpp);
    if (P0 < 1) P0 = 1;
    constexpr int kTry = 8;
    constexpr int kAheadChunks = 4;   // chunks whose needs are loaded together
    int Pb = 0, ns = 0;
    for (int round = 0; round < 4 && Pb == 0; ++round) {
        int pbk[kTry], nsk[kTry], capk[kTry][7];
#pragma unroll
        for (int t = 0; t < kTry; ++t) {
            pbk[t] = P0 + (P0 * t) / 4 + t;
            nsk[t] = 0;
            slice_caps((double)pbk[t], bpp, cf, capk[t]);
        }
        for (int base = a; base <= b; base += kAheadChunks * kWave) {
            int nd[kAheadChunks];
#pragma unroll
            for (int k = 0; k < kAheadChunks; ++k) {
                const int j = base + k * kWave + l;
                nd[k] = (j <= b) ? (int)P.need[sb + j] : 0;
            }
#pragma unroll
            for (int k = 0; k < kAheadChunks; ++k) {
                if (base + k * kWave > b) break;
                const bool in = base + k * kWave + l <= b;
                int mb[7];
                chunk_maxbits(nd[k], mb);
#pragma unroll
                for (int t = 0; t < kTry; ++t) {
                    const int q = slice_q(mb, capk[t], qmin, qmax);
                    nsk[t] += __popcll(__ballot(in && (l & ((1 << q) - 1)) == 0));
                }
            }
        }
        for (int t = 0; t < kTry && Pb == 0; ++t) {
            if (nsk[t] <= budget || (round == 3 && t == kTry - 1)) {
                Pb = pbk[t];
                ns = nsk[t];
            }
        }
        P0 = pbk[kTry - 1] + 1 + pbk[kTry - 1] / 4;
    }
    if (l == 0) __hip_atomic_store(&P.nodes[node_id].pending, ns, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // list the slices in LDS and push the list whenever it fills (one wait
    // for free cells per 64 slices instead of one per 64-member chunk)
    int capf[7];
    slice_caps((double)Pb, bpp, cf, capf);
    int listed = 0;
    int nd[kAheadChunks];
    for (int base = a; base <= b; base += kWave) {
        const int kc = ((base - a) / kWave) % kAheadChunks;
        if (kc == 0) {
#pragma unroll
            for (int u = 0; u < kAheadChunks; ++u) {
                const int ju = base + u * kWave + l;
                nd[u] = (ju <= b) ? (int)P.need[sb + ju] : 0;
            }
        }
        const int j = base + l;
        const bool in = j <= b;
        int mb[7];
        int ndk = nd[0];
#pragma unroll
        for (int u = 1; u < kAheadChunks; ++u) ndk = (kc == u) ? nd[u] : ndk;
        chunk_maxbits(ndk, mb);
        const int q = slice_q(mb, capf, qmin, qmax);
        const bool st = in && (l & ((1 << q) - 1)) == 0;
        const uint64_t sm = __ballot(st);
        if (st) {
            const int k = listed + __popcll(sm & ((1ull << l) - 1ull));
            S.sl_a[k] = j;
            S.sl_q[k] = (int8_t)q;
        }
        listed += __popcll(sm);
        if (listed > kMaxSlices - kWave || base + kWave > b) {
            __syncthreads();
            push_batch(P, kQRefine, listed, [&](int k) {
                Task t;
                t.type = kTaskRefine;
                t.node = node_id;
                t.a = S.sl_a[k];
                const int e = t.a + (1 << S.sl_q[k]) - 1;
                t.b = (e < b ? e : b) | (mode << 30);
                return t;
            });
            __syncthreads();
            listed = 0;
        }
    }
}

DEV int new_node(const Params& P) {   // all lanes get the id
    int id = 0;
    if (lane_id() == 0)
        id = __hip_atomic_fetch_add(&P.ctl->node_top, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    id = __shfl(id, 0);
    if (id >= P.max_nodes) {
        set_error(P, kErrNoMem);
        return -1;
    }
    return id;
}

// ------------------------------------- cooperative refinement
//
// The refinement of a cluster's end eigenvalues to full accuracy (the first
// step of Alg. 3.8) lies on the critical path of a deep cluster tree while most
// workers are idle.  The worker that owns it (the leader) then lends its
// passes to idle workers without changing them: the leader counts one pass
// of the sequential multisection schedule (the one refine_members follows:
// each unfinished member gets Lg points inside its bracket), and each helper
// counts, for some of the Lg + 1 brackets that pass can leave a member in,
// the next pass's points inside that bracket.  When every member's outcome
// was covered and no member finished, the round advances two passes, else
// one; either way the brackets are exactly those of the sequential schedule,
// so the results do not depend on how many helpers joined (even where counts
// are not monotone at the rounding level, as inside glued Wilkinson's tight
// clusters).  The leader waits only for helpers counted in the current
// round, which are already running; a helper that joins late waits for the
// next round or, finding the refinement finished, returns at once.
constexpr int kCoopMax = 66;                // workers per round, the leader included
constexpr int64_t kCoopMinRows = 4096;      // shorter passes are not worth sharing
// The three-pass rounds of a cluster whose children have most of the workers
// (a chain of representations, as in 1-2-1): both ends refined with 16
// points each and pass, every member on its own (Lg fixed); helpers count the
// second pass inside each of the 17 brackets the first can leave a member in,
// and the third inside each of the 17 x 17 the first two can.
constexpr int kDeepLg = 16;
constexpr double kDeepShare = 256.0;        // a child's share of the workers from which the ends go deep
constexpr int kCoopMaxDeep = 1 + (2 * (kDeepLg + 1) * (kDeepLg + 2) + kWave / kDeepLg - 1) / (kWave / kDeepLg);
enum CoopWord : int {
    kCbGen = 0,     // (round << 8) | M while a round runs; -1 once finished
    kCbJoined,      // helpers that have joined (their ranks are 1, 2, ...)
    kCbArrive,      // helpers done with the current round
    kCbNode,        // the node whose representation is refined
    kCbAct,         // bit m: member m unfinished (64-bit mask)
    kCbLg,          // points per member in this round's passes
    kCbLv,          // passes a round can advance (2, or 3 for the deep rounds)
    kCbLo = 8,      // [64] the round's brackets
    kCbHi = kCbLo + kWave,
    kCbJ = kCbHi + kWave,          // [64] the members' indices
    // per second-pass branch (member, bracket), then per third-pass branch
    // (member, bracket, bracket): 1 + first point reaching j; 0 not counted
    kCbRes = kCbJ + kWave,
    kCbWords = kCbRes + 2 * (kDeepLg + 1) * (kDeepLg + 2)
};
constexpr int64_t kCbDone = -1;
static_assert(128 + kCbWords <= kNodeExtra, "a representation's node-pool share holds the cooperation block");
static_assert(2 * (32 + 1) <= 2 * (kDeepLg + 1) * (kDeepLg + 2), "the result words hold the two-pass rounds too");
static_assert(kCoopMaxDeep <= 255, "the round word holds the workers of a round");

DEV int64_t cb_ld(int64_t* cb, int w) {
    return __hip_atomic_load(cb + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV void cb_st(int64_t* cb, int w, int64_t v) {
    __hip_atomic_store(cb + w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
DEV int coop_lg(int nu, int lanes) {   // refine_members' points per member for nu members
    int Lg = 1;
    while (Lg * 2 * nu <= kWave && Lg * 2 <= lanes) Lg *= 2;
    return Lg;
}

// What the counts run on: a node's representation (D, L), or, for the
// extremal eigenvalues of a root, the block's T itself (d non-null), whose
// multisection points are equally spaced.
struct CoopSrc {
    const double* D;
    const double* L;
    const double* d;
    const double* e;
    double sc;
};
DEV double coop_point(bool onT, double lo, double hi, int t, int Lg) {
    return onT ? lo + (hi - lo) * (double)(t + 1) / (double)(Lg + 1) : msec_point(lo, hi, t, Lg);
}

// A helper's share of a round: branch g = (rank - 1) * (64 / Lg) + l / Lg.
// The first nu (Lg + 1) branches are (a, b): bracket b of the a-th
// unfinished member after the first pass; in rounds of three passes the next
// nu (Lg + 1)^2 are (a, b, c): bracket c inside that one after the second.
// Lane k of the branch counts point k of the next pass inside its bracket.
DEV void coop_branches(Shared& S, int64_t* cb, const CoopSrc& src, int64_t n, int rank, uint64_t act, int Lg,
                       int lv, int64_t& steps) {
    const int l = lane_id();
    const int nu = __popcll(act);
    if ((act >> l) & 1ull) S.ulist[__popcll(act & ((1ull << l) - 1ull))] = l;
    __syncthreads();
    const int bp = kWave / Lg, w1 = Lg + 1, nbr2 = nu * w1, nbr = nbr2 + (lv >= 3 ? nu * w1 * w1 : 0);
    const int g = (rank - 1) * bp + l / Lg, k = l % Lg;
    const bool on = g < nbr;
    int a = 0, b = 0, c3 = -1;
    if (on && g < nbr2) {
        a = g / w1;
        b = g % w1;
    } else if (on) {
        const int h = g - nbr2;
        a = h / (w1 * w1);
        b = (h / w1) % w1;
        c3 = h % w1;
    }
    const int m = S.ulist[a];
    const double lo = __longlong_as_double((long long)cb_ld(cb, kCbLo + m));
    const double hi = __longlong_as_double((long long)cb_ld(cb, kCbHi + m));
    const int j = (int)cb_ld(cb, kCbJ + m);
    const bool onT = src.d != nullptr;
    double lob = (b == 0) ? lo : coop_point(onT, lo, hi, b - 1, Lg);
    double hib = (b == Lg) ? hi : coop_point(onT, lo, hi, b, Lg);
    if (c3 >= 0) {
        const double l2 = (c3 == 0) ? lob : coop_point(onT, lob, hib, c3 - 1, Lg);
        const double h2 = (c3 == Lg) ? hib : coop_point(onT, lob, hib, c3, Lg);
        lob = l2;
        hib = h2;
    }
    const double sig = on ? coop_point(onT, lob, hib, k, Lg) : 0.0;
    const int c = onT ? negcount_T(S, src.d, src.e, n, src.sc, sig) : negcount_rep(S, src.D, src.L, n, sig);
    steps += n * (int64_t)__popcll(__ballot(on));
    const int gb = (l / Lg) * Lg;
    const uint64_t gmask = (Lg == 64) ? ~0ull : (((1ull << Lg) - 1ull) << (gb & 63));
    const uint64_t ge = __ballot(on && c >= j) & gmask;
    const int tstar = ge ? (__ffsll((unsigned long long)ge) - 1 - gb) : Lg;
    if (on && k == 0) cb_st(cb, kCbRes + g, tstar + 1);
    __syncthreads();
}

// A helper task: join the refinement whose block is at `cboff` and take a
// share of every round that counts it, until the leader marks it finished.
DEV void task_help(Shared& S, const Params& P, int64_t cboff, int64_t& steps) {
    const int l = lane_id();
    int64_t* cb = reinterpret_cast<int64_t*>(P.arena + cboff);
    int64_t rank = 0;
    if (l == 0 && cb_ld(cb, kCbGen) != kCbDone)
        rank = 1 + __hip_atomic_fetch_add(cb + kCbJoined, (int64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    rank = __shfl(rank, 0);
    if (rank == 0) return;
    // a node's representation, or (a negative word: -1 - block) a root's T
    const int pid = (int)cb_ld(cb, kCbNode);
    CoopSrc src;
    int64_t n;
    if (pid >= 0) {
        const Node nd = P.nodes[pid];
        n = P.blocks[nd.block].n;
        src.D = P.arena + nd.data;
        src.L = src.D + n;
        src.d = nullptr;
        src.e = nullptr;
        src.sc = 1.0;
    } else {
        const Block blk = P.blocks[-1 - pid];
        n = blk.n;
        src.D = nullptr;
        src.L = nullptr;
        src.d = P.d + blk.row0;
        src.e = P.e + blk.row0;
        src.sc = P.probs[blk.prob].tscale;
    }
    const uint64_t t0 = wall_clock64();
    int64_t last = 0;
    for (;;) {
        int64_t gen = 0;
        if (l == 0) {
            for (;;) {
                gen = __hip_atomic_load(cb + kCbGen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                if (gen != last) break;
                if (__hip_atomic_load(&P.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                    wall_clock64() - t0 > P.timeout_ticks) {
                    gen = kCbDone;
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
        }
        gen = __shfl(gen, 0);
        if (gen == kCbDone) return;
        last = gen;
        const int M = (int)(gen & 0xff);
        if (rank >= M) continue;   // joined after this round was laid out
        const uint64_t act = (uint64_t)cb_ld(cb, kCbAct);
        const int Lg = (int)cb_ld(cb, kCbLg);
        const int lv = (int)cb_ld(cb, kCbLv);
        coop_branches(S, cb, src, n, (int)rank, act, Lg, lv, steps);
        // the results out (every lane's stores are complete), then the arrival
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (l == 0) __hip_atomic_fetch_add(cb + kCbArrive, (int64_t)1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The leader's side, for the nm members whose verified brackets are in
// S.m_lo / m_hi and indices in S.m_j: refine_members' schedule in `mode`
// with `lanes` points at most per member, to the end.  False when the
// brackets share one interval (refine_members then starts with a joint
// pass) or on an error; the brackets are then valid for refine_members to
// finish.  `publish` writes the final brackets to the members' slots.
// `lg_fix` > 0: the deep schedule -- every unfinished member gets lg_fix
// points per pass whatever the others do, so each advances on its own, up to
// three passes a round.
DEV bool coop_refine(Shared& S, const Params& P, int pid, const double* D, const double* L, int64_t n, int nm,
                     int mode, int lanes, int64_t* cb, int64_t cboff, int helpers, bool publish, int lg_fix,
                     int64_t& steps) {
    const int l = lane_id();
    {
        int same = 1;
        if (l < nm) same = (S.m_lo[l] == S.m_lo[0] && S.m_hi[l] == S.m_hi[0]) ? 1 : 0;
        if (nm > 1 && __ballot(same == 0) == 0ull) return false;
    }
    if (l == 0) {
        cb_st(cb, kCbGen, 0);
        cb_st(cb, kCbJoined, 0);
        cb_st(cb, kCbArrive, 0);
        cb_st(cb, kCbNode, pid);
    }
    if (l < nm) cb_st(cb, kCbJ + l, S.m_j[l]);
    // the push's release publishes the block with the tasks
    if (!push_batch(P, kQRefine, helpers, [&](int) {
            Task t;
            t.type = kTaskHelp;
            t.node = pid;
            t.a = (int32_t)(uint32_t)((uint64_t)cboff & 0xffffffffull);
            t.b = (int32_t)(uint32_t)((uint64_t)cboff >> 32);
            return t;
        }))
        return false;
    // a short wait lets the first round start with the helpers that idle
    // workers pick up at once (they poll every few microseconds)
    const uint64_t tw = wall_clock64();
    int64_t joined = 0;
    if (l == 0) {
        for (;;) {
            joined = cb_ld(cb, kCbJoined);
            if (joined >= helpers || wall_clock64() - tw > 4000) break;   // 40 us of the 100 MHz clock
            __builtin_amdgcn_s_sleep(8);
        }
    }
    bool ok = true;
    for (int round = 1; round < kMaxPass; ++round) {
        const double lo = (l < nm) ? S.m_lo[l] : 0.0, hi = (l < nm) ? S.m_hi[l] : 0.0;
        const uint64_t act = __ballot(l < nm && !bracket_done(P, mode, lo, hi));
        if (act == 0ull) break;
        const int nu = __popcll(act);
        const int Lg = lg_fix > 0 ? lg_fix : coop_lg(nu, lanes);
        const int lv = lg_fix > 0 ? 3 : 2;
        const int nbr = nu * (Lg + 1) + (lv >= 3 ? nu * (Lg + 1) * (Lg + 1) : 0);
        if (l == 0) joined = cb_ld(cb, kCbJoined);
        joined = __shfl(joined, 0);
        const int M = 1 + (int)(joined < helpers ? joined : helpers);
        if (l < nm) {
            cb_st(cb, kCbLo + l, __double_as_longlong(lo));
            cb_st(cb, kCbHi + l, __double_as_longlong(hi));
        }
        for (int g = l; g < nbr; g += kWave) cb_st(cb, kCbRes + g, 0);
        if (l == 0) {
            cb_st(cb, kCbArrive, 0);
            cb_st(cb, kCbAct, (int64_t)act);
            cb_st(cb, kCbLg, Lg);
            cb_st(cb, kCbLv, lv);
        }
        // every lane's stores out before the round is published
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (l == 0) __hip_atomic_store(cb + kCbGen, ((int64_t)round << 8) | M, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        // this round's first pass, as refine_members counts it
        if ((act >> l) & 1ull) S.ulist[__popcll(act & ((1ull << l) - 1ull))] = l;
        __syncthreads();
        const int u = l / Lg, t = l % Lg;
        const bool valid = u < nu;
        const int m = valid ? S.ulist[u] : 0;
        const double mlo = S.m_lo[m], mhi = S.m_hi[m];
        const int j = S.m_j[m];
        const double sig = valid ? msec_point(mlo, mhi, t, Lg) : 0.0;
        const int c = negcount_rep(S, D, L, n, sig);
        steps += n * (int64_t)__popcll(__ballot(valid));
        const int gb = u * Lg;
        const uint64_t gmask = (Lg == 64) ? ~0ull : (((1ull << Lg) - 1ull) << (gb & 63));
        const uint64_t ge = __ballot(valid && c >= j) & gmask;
        const int tstar = ge ? (__ffsll((unsigned long long)ge) - 1 - gb) : Lg;
        const double s_hi = __shfl(sig, gb + (tstar < Lg ? tstar : Lg - 1));
        const double s_lo = __shfl(sig, gb + (tstar > 0 ? tstar - 1 : 0));
        // the helpers counted in M are running: each arrives after one count
        int stop = 0;
        if (l == 0) {
            const uint64_t t1 = wall_clock64();
            while (__hip_atomic_load(cb + kCbArrive, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < M - 1) {
                if (__hip_atomic_load(&P.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                    wall_clock64() - t1 > P.timeout_ticks) {
                    stop = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        if (__shfl(stop, 0)) {
            ok = false;
            break;
        }
        // lane t == 0 of each member's group: the bracket after the first
        // pass, and after the second where every member's outcome was counted
        // and no member finished (else the second pass runs next round)
        double nlo = mlo, nhi = mhi;
        if (valid && t == 0) {
            if (tstar < Lg) nhi = s_hi;
            if (tstar > 0) nlo = s_lo;
        }
        const bool lead = valid && t == 0;
        const bool fin1 = lead && bracket_done(P, mode, nlo, nhi);
        int64_t res = 0;
        if (lead) res = cb_ld(cb, kCbRes + u * (Lg + 1) + tstar);
        if (lg_fix == 0) {
            const bool two = __ballot(fin1) == 0ull && __ballot(lead && res == 0) == 0ull;
            if (lead && two) {
                const int t2 = (int)res - 1;
                const double a2 = (t2 > 0) ? msec_point(nlo, nhi, t2 - 1, Lg) : nlo;
                const double b2 = (t2 < Lg) ? msec_point(nlo, nhi, t2, Lg) : nhi;
                nlo = a2;
                nhi = b2;
            }
        } else if (lead && !fin1 && res != 0) {
            // the deep schedule: the second pass where it was counted, and
            // the third where the member is still unfinished and it was too
            const int t2 = (int)res - 1;
            const double a2 = (t2 > 0) ? msec_point(nlo, nhi, t2 - 1, Lg) : nlo;
            const double b2 = (t2 < Lg) ? msec_point(nlo, nhi, t2, Lg) : nhi;
            nlo = a2;
            nhi = b2;
            if (!bracket_done(P, mode, nlo, nhi)) {
                const int64_t r3 =
                    cb_ld(cb, kCbRes + nu * (Lg + 1) + (u * (Lg + 1) + tstar) * (Lg + 1) + t2);
                if (r3 != 0) {
                    const int t3 = (int)r3 - 1;
                    const double a3 = (t3 > 0) ? msec_point(nlo, nhi, t3 - 1, Lg) : nlo;
                    const double b3 = (t3 < Lg) ? msec_point(nlo, nhi, t3, Lg) : nhi;
                    nlo = a3;
                    nhi = b3;
                }
            }
        }
        __syncthreads();
        if (lead) {
            S.m_lo[m] = nlo;
            S.m_hi[m] = nhi;
        }
        __syncthreads();
    }
    if (l == 0) __hip_atomic_store(cb + kCbGen, kCbDone, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (publish && l < nm) {
        st_rlx_d(P.lo + S.m_slot[l], S.m_lo[l]);
        st_rlx_d(P.hi + S.m_slot[l], S.m_hi[l]);
    }
    return ok;
}

// Helpers from workers that are idle now: tasks pushed and not yet finished
// occupy (or wait for) the others.  0 when too few are idle to be worth it.
DEV int coop_helpers(const Params& P, int cap = kCoopMax) {
    int64_t pend = 0;
    if (lane_id() == 0) pend = __hip_atomic_load(&P.ctl->pending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    pend = __shfl(pend, 0);
    const int64_t idle = (int64_t)P.nworkers - pend;
    const int h = (int)(idle / 4 < cap - 1 ? idle / 4 : cap - 1);
    return h >= 3 ? h : 0;
}

// The extremal eigenvalues of a long block's T with idle workers' help.  The
// root's own schedule (each pass 32 equally spaced points inside each of the
// two brackets, both ends every pass until both are delta wide) advances two
// passes a round as in coop_refine: the leader counts the first, helpers the
// second inside every bracket the first can leave an end in.  The brackets
// are those of the sequential passes, bit for bit, with any number of
// helpers.  False on an error or a time-out; the brackets are then valid for
// the sequential passes to continue.
constexpr int kRootCoopHelpers = 33;   // 2 ends x 33 brackets, 2 branches a helper
DEV bool root_extremal_coop(Shared& S, const Params& P, int bid, const double* d, const double* e, int64_t n,
                            double sc, double delta, double& lo1, double& hi1, double& lon, double& hin, int64_t* cb,
                            int64_t cboff, int helpers, int64_t& steps) {
    const int l = lane_id();
    constexpr int Lg = 32;
    if (l == 0) {
        cb_st(cb, kCbGen, 0);
        cb_st(cb, kCbJoined, 0);
        cb_st(cb, kCbArrive, 0);
        cb_st(cb, kCbNode, -1 - bid);
        cb_st(cb, kCbJ + 0, 1);
        cb_st(cb, kCbJ + 1, n);
    }
    if (!push_batch(P, kQRefine, helpers, [&](int) {
            Task t;
            t.type = kTaskHelp;
            t.node = 0;
            t.a = (int32_t)(uint32_t)((uint64_t)cboff & 0xffffffffull);
            t.b = (int32_t)(uint32_t)((uint64_t)cboff >> 32);
            return t;
        }))
        return false;
    const uint64_t tw = wall_clock64();
    int64_t joined = 0;
    if (l == 0) {
        for (;;) {
            joined = cb_ld(cb, kCbJoined);
            if (joined >= helpers || wall_clock64() - tw > 4000) break;   // 40 us of the 100 MHz clock
            __builtin_amdgcn_s_sleep(8);
        }
    }
    bool ok = true;
    const int half = l >> 5, t = l & 31;
    for (int round = 1; round < 200; ++round) {
        if (hi1 - lo1 <= delta && hin - lon <= delta) break;
        if (l == 0) joined = cb_ld(cb, kCbJoined);
        joined = __shfl(joined, 0);
        const int M = 1 + (int)(joined < helpers ? joined : helpers);
        if (l == 0) {
            cb_st(cb, kCbLo + 0, __double_as_longlong(lo1));
            cb_st(cb, kCbHi + 0, __double_as_longlong(hi1));
            cb_st(cb, kCbLo + 1, __double_as_longlong(lon));
            cb_st(cb, kCbHi + 1, __double_as_longlong(hin));
            cb_st(cb, kCbArrive, 0);
            cb_st(cb, kCbAct, 3);
            cb_st(cb, kCbLg, Lg);
            cb_st(cb, kCbLv, 2);
        }
        for (int g = l; g < 2 * (Lg + 1); g += kWave) cb_st(cb, kCbRes + g, 0);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (l == 0) __hip_atomic_store(cb + kCbGen, ((int64_t)round << 8) | M, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        // the first pass, as the sequential loop counts it
        const double lo = half ? lon : lo1, hi = half ? hin : hi1;
        const double sig = coop_point(true, lo, hi, t, Lg);
        const int c = negcount_T(S, d, e, n, sc, sig);
        steps += n * kWave;
        const uint64_t ge = __ballot(c >= (half ? (int)n : 1));
        const uint64_t g0 = ge & 0xffffffffull, g1 = ge >> 32;
        const int t0 = g0 ? __ffsll((unsigned long long)g0) - 1 : 32;
        const int t1 = g1 ? __ffsll((unsigned long long)g1) - 1 : 32;
        const double h0 = __shfl(sig, t0 < 32 ? t0 : 31), l0 = __shfl(sig, t0 > 0 ? t0 - 1 : 0);
        const double h1 = __shfl(sig, 32 + (t1 < 32 ? t1 : 31)), l1 = __shfl(sig, 32 + (t1 > 0 ? t1 - 1 : 0));
        int stop = 0;
        if (l == 0) {
            const uint64_t t2 = wall_clock64();
            while (__hip_atomic_load(cb + kCbArrive, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < M - 1) {
                if (__hip_atomic_load(&P.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                    wall_clock64() - t2 > P.timeout_ticks) {
                    stop = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        // the first pass's brackets (kept even when the round stops here)
        if (t0 < 32) hi1 = h0;
        if (t0 > 0) lo1 = l0;
        if (t1 < 32) hin = h1;
        if (t1 > 0) lon = l1;
        if (__shfl(stop, 0)) {
            ok = false;
            break;
        }
        // the second pass, where both outcomes were counted and the
        // sequential loop would run it (not both ends delta wide yet)
        const int64_t r0 = cb_ld(cb, kCbRes + t0), r1 = cb_ld(cb, kCbRes + (Lg + 1) + t1);
        if (r0 != 0 && r1 != 0 && !(hi1 - lo1 <= delta && hin - lon <= delta)) {
            const int u0 = (int)r0 - 1, u1 = (int)r1 - 1;
            const double a0 = (u0 > 0) ? coop_point(true, lo1, hi1, u0 - 1, Lg) : lo1;
            const double b0 = (u0 < Lg) ? coop_point(true, lo1, hi1, u0, Lg) : hi1;
            const double a1 = (u1 > 0) ? coop_point(true, lon, hin, u1 - 1, Lg) : lon;
            const double b1 = (u1 < Lg) ? coop_point(true, lon, hin, u1, Lg) : hin;
            lo1 = a0;
            hi1 = b0;
            lon = a1;
            hin = b1;
        }
        __syncthreads();
    }
    if (l == 0) __hip_atomic_store(cb + kCbGen, kCbDone, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    return ok;
}

DEV int64_t arena_alloc(const Params& P, int64_t count) {
    uint64_t off = 0;
    if (lane_id() == 0)
        off = __hip_atomic_fetch_add(&P.ctl->arena_top, (uint64_t)count, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
    off = __shfl(off, 0);
    if (off + (uint64_t)count > P.arena_cap) {
        set_error(P, kErrNoMem);
        return -1;
    }
    return (int64_t)off;
}

DEV void stat_max(int64_t* p, int64_t v) {
    if (lane_id() == 0) __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ new RRRs

struct FacOut {
    int ok;
    double growth;
};

// L+ D+ L+^T = L D L^T - tau I by the differential stationary qd transform
// (Alg. 3.5), in two passes.  dstqds_select: the shift selection of Alg. 3.8
// without writing any candidate -- one candidate shift tau per lane runs the
// transform (quotients from the reciprocal, see quot), recording whether the
// factorisation exists (every d+ and l+ finite, every d+ nonzero; a zero or
// infinite pivot turns the reciprocal form into NaN, which fails the test as
// well) and its element growth max |d+_i|, and keeping the state s entering
// every 64-row tile ([tile][lane]) so that dstqds_values can recompute the
// winner's rows tile by tile in parallel, bit for bit as one sequential pass
// computes them.
DEV FacOut dstqds_select(Shared& S, const double* D, const double* L, int64_t n, double tau, double* cks) {
    const int l = lane_id();
    double s = -tau, gmax = 0.0;
    int ok = 1;
    auto row = [&](const QRow& x) {
        const double dp = s + x.d;
        ok &= (__builtin_isfinite(dp) && dp != 0.0) ? 1 : 0;
        gmax = fmax(gmax, fabs(dp));
        const Recip rc = recip(dp);
        // l+ = (d l) / d+ overflows exactly when (d l) times the reciprocal
        // does (up to the reciprocal's 2^-24)
        ok &= __builtin_isfinite(x.dl * rc.r) ? 1 : 0;
        s = quot(rc, s) * x.dll - tau;
    };
    RepRow f = rep_fetch(D, L, 0, n);
    int64_t tile = 0;
    for (int64_t base = 0; base < n; base += kTile, ++tile) {
        rep_commit(S, f);
        cks[tile * kWave + l] = s;
        if (base + kTile < n) f = rep_fetch(D, L, base + kTile, n);
        const int lim = (int)((n - base) < kTile ? (n - base) : kTile);
        if (lim == kTile) {
            QRow cur[kAhead], nxt[kAhead];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) cur[u] = S.tr[u];
#pragma unroll
            for (int g = 0; g < kTile / kAhead; ++g) {
                if (g + 1 < kTile / kAhead) {
#pragma unroll
                    for (int u = 0; u < kAhead; ++u) nxt[u] = S.tr[(g + 1) * kAhead + u];
                }
#pragma unroll
                for (int u = 0; u < kAhead; ++u) row(cur[u]);
#pragma unroll
                for (int u = 0; u < kAhead; ++u) cur[u] = nxt[u];
            }
        } else {
            for (int t = 0; t < lim; ++t) row(S.tr[t]);
        }
    }
    FacOut o;
    o.ok = ok;
    o.growth = gmax;
    return o;
}

// The rows of the candidate that lane c ran in dstqds_select, written to
// (Dp, Lp): the 64-row tiles go round the lanes, each lane restarting the
// transform from the s its tile was entered with, in the arithmetic of
// dstqds, so the result is bit for bit that of one sequential pass.  Rows are
// read eight ahead of the recurrence.
DEV void dstqds_values(const double* D, const double* L, int64_t n, double tau, const double* cks, int c,
                       double* Dp, double* Lp) {
    const int l = lane_id();
    const int64_t ntiles = (n + kTile - 1) / kTile;
    for (int64_t tile = l; tile < ntiles; tile += kWave) {
        double s = cks[tile * kWave + c];
        const int64_t base = tile * kTile;
        const int lim = (int)((n - base) < kTile ? (n - base) : kTile);
        for (int t0 = 0; t0 < lim; t0 += 8) {
            double dd[8], ll[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int64_t i = base + t0 + k;
                dd[k] = (t0 + k < lim) ? D[i] : 0.0;
                ll[k] = (t0 + k < lim && i < n - 1) ? L[i] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (t0 + k < lim) {
                    const int64_t i = base + t0 + k;
                    const double dl = dd[k] * ll[k];
                    const double dll = dl * ll[k];
                    const double dp = s + dd[k];
                    Dp[i] = dp;
                    const Recip rc = recip(dp);
                    Lp[i] = quot(rc, dl);
                    s = quot(rc, s) * dll - tau;
                }
            }
        }
    }
}

// Division-free forms of both passes, with the pair (u, v) of negcount_rep
// (s_i = u_i / v_i):
//     w_i = d_i v_i + u_i,   d+_i = w_i / v_i,
//     u_{i+1} = u_i (d_i l_i^2) - tau w_i,   v_{i+1} = w_i,
// two dependent fused multiply-adds per row where the quotient form has a
// reciprocal and four corrections on the chain.  The recurrence carries the
// roundings of the quotient form's s, less the quotient's; the values pass
// rounds d+ = w / v and l+ = (d l) / d+ once each as it writes them, a
// relative change of one unit roundoff in each output element, inside what
// the mixed relative error analysis of the transform (Sec. 3.2.3) allows.  A
// lane's element growth max |d+| (and the smallest |d+|) come from the
// hardware reciprocal of v, off the chain, good to about 2^-22 -- ample to
// compare candidates.  (u, v) entering each 64-row tile is kept, u and v in
// two [tile][lane] arrays, and the pair is scaled by a power of two after
// every 8 rows of a full tile and after every row of the last, partial one:
// the same schedule in both passes, so that the values pass reproduces the
// winner's w and v bit for bit.
//
// A lane's result holds within the bounds of negcount_rep (data and tau,
// every |w| and every rescaled |v| at least 2^-800) and with every |d+| at
// least 2^-850 (so |l+| <= 2^1000).  A state that overflowed (|w| or |u|
// past 2^1024 within 8 rows of a rescaling) means some |d+| >= 2^100: that
// candidate is rejected.  Any other lane outside the bounds makes the caller
// run the quotient form for the whole wave.
struct HomFac {
    int ok;          // the candidate exists (within the bounds)
    int unknown;     // outside the bounds: only the quotient form can tell
    double growth;   // max |d+|, about (ok lanes)
};
constexpr double kHomPivot = 0x1p-850;

DEV void hom_rescale2(double& u, double& v) {
    const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(u), fabs(v)));
    u = __builtin_ldexp(u, -ex);
    v = __builtin_ldexp(v, -ex);
}

DEV HomFac dstqds_select_hom(Shared& S, const double* D, const double* L, int64_t n, double tau, double* cku,
                             double* ckv) {
    const int l = lane_id();
    double u = -tau, v = 1.0;
    double mw = 1.0, gmax = 0.0, gmin = __builtin_inf();
    bool data_ok = true;
    auto row = [&](double d, double dll) {
        const double w = __builtin_fma(d, v, u);
        const double g = fabs(w) * __builtin_amdgcn_rcp(fabs(v));
        gmax = fmax(gmax, g);
        gmin = fmin(gmin, g);
        const double p = u * dll;
        u = __builtin_fma(-tau, w, p);
        v = w;
        mw = fmin(mw, fabs(w));
    };
    RepRow f = rep_fetch(D, L, 0, n);
    int64_t tile = 0;
    for (int64_t base = 0; base < n; base += kTile, ++tile) {
        data_ok &= (__ballot(!rep_commit(S, f)) == 0ull);
        cku[tile * kWave + l] = u;
        ckv[tile * kWave + l] = v;
        if (base + kTile < n) f = rep_fetch(D, L, base + kTile, n);
        const int lim = (int)((n - base) < kTile ? (n - base) : kTile);
        if (lim == kTile) {
            dv2 cur[8], nxt[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) cur[k] = QROW_DDLL(S, k);
#pragma unroll
            for (int g = 0; g < kTile / 8; ++g) {
                if (g + 1 < kTile / 8) {
#pragma unroll
                    for (int k = 0; k < 8; ++k) nxt[k] = QROW_DDLL(S, (g + 1) * 8 + k);
                }
                __builtin_amdgcn_sched_barrier(0);
                if (g + 1 < kTile / 8) __builtin_amdgcn_s_waitcnt(kWaitLds8);
#pragma unroll
                for (int k = 0; k < 8; ++k) row(cur[k].x, cur[k].y);
                hom_rescale(u, v, mw);
#pragma unroll
                for (int k = 0; k < 8; ++k) cur[k] = nxt[k];
            }
        } else {
            for (int t = 0; t < lim; ++t) {
                const dv2 x = QROW_DDLL(S, t);
                row(x.x, x.y);
                hom_rescale(u, v, mw);
            }
        }
    }
    const bool ovf = !__builtin_isfinite(u) || !__builtin_isfinite(v) || !(gmax < 0x1p1000);
    HomFac o;
    o.unknown = (!data_ok || !hom_sigma_ok(tau) || (!ovf && (!(mw >= kHomState) || !(gmin >= kHomPivot)))) ? 1 : 0;
    o.ok = (!o.unknown && !ovf) ? 1 : 0;
    o.growth = o.ok ? gmax : __builtin_inf();
    return o;
}

// The rows of the candidate that lane c ran in dstqds_select_hom, written to
// (Dp, Lp), the 64-row tiles going round the lanes from the kept (u, v).
DEV void dstqds_values_hom(const double* D, const double* L, int64_t n, double tau, const double* cku,
                           const double* ckv, int c, double* Dp, double* Lp) {
    const int l = lane_id();
    const int64_t ntiles = (n + kTile - 1) / kTile;
    for (int64_t tile = l; tile < ntiles; tile += kWave) {
        double u = cku[tile * kWave + c], v = ckv[tile * kWave + c];
        const int64_t base = tile * kTile;
        const int lim = (int)((n - base) < kTile ? (n - base) : kTile);
        for (int t0 = 0; t0 < lim; t0 += 8) {
            double dd[8], ll[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int64_t i = base + t0 + k;
                dd[k] = (t0 + k < lim) ? D[i] : 0.0;
                ll[k] = (t0 + k < lim && i < n - 1) ? L[i] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (t0 + k < lim) {
                    const int64_t i = base + t0 + k;
                    // the staged values of rep_commit
                    const double dl = dd[k] * ll[k];
                    const double dll = dl * ll[k];
                    const double w = __builtin_fma(dd[k], v, u);
                    const double dp = quot(recip(v), w);
                    Dp[i] = dp;
                    Lp[i] = quot(recip(dp), dl);
                    const double p = u * dll;
                    u = __builtin_fma(-tau, w, p);
                    v = w;
                    if (lim < kTile) hom_rescale2(u, v);
                }
            }
            if (lim == kTile) hom_rescale2(u, v);
        }
    }
}

// T - mu I = L D L^T by Gaussian elimination without pivoting; sgn > 0
// requires every pivot positive, sgn < 0 every pivot negative (a definite
// root, Sec. 3.1.2).  In two passes, as for dstqds: factor_select runs one
// candidate mu per lane without writing (quotients from the reciprocal), and
// keeps the pivot entering every 64-row tile, [tile][lane]; factor_values
// recomputes the winner's rows tile by tile across the lanes, bit for bit.
DEV FacOut factor_select(Shared& S, const double* d, const double* e, int64_t n, double sc, double mu, int sgn,
                         double* ckp) {
    const int l = lane_id();
    double dprev = 1.0, gmax = 0.0;
    int ok = 1;
    // row 0 has beta = 0 staged, and dprev = 1 makes the quotient term an
    // exact zero there: d_0 = alpha_0 - mu
    auto row = [&](const QRow& x) {
        const double dv = (x.d - mu) - quot(recip(dprev), x.dl) * x.dl;
        ok &= (__builtin_isfinite(dv) && (sgn > 0 ? dv > 0.0 : dv < 0.0)) ? 1 : 0;
        gmax = fmax(gmax, fabs(dv));
        dprev = dv;
    };
    RepRow f = T_fetch(d, e, 0, n, sc);
    int64_t tile = 0;
    for (int64_t base = 0; base < n; base += kTile, ++tile) {
        T_commit(S, f);
        ckp[tile * kWave + l] = dprev;
        if (base + kTile < n) f = T_fetch(d, e, base + kTile, n, sc);
        const int lim = (int)((n - base) < kTile ? (n - base) : kTile);
        if (lim == kTile) {
            // rows read kAhead ahead of the recurrence, as in dstqds_select
            QRow cur[kAhead], nxt[kAhead];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) cur[u] = S.tr[u];
#pragma unroll
            for (int g = 0; g < kTile / kAhead; ++g) {
                if (g + 1 < kTile / kAhead) {
#pragma unroll
                    for (int u = 0; u < kAhead; ++u) nxt[u] = S.tr[(g + 1) * kAhead + u];
                }
#pragma unroll
                for (int u = 0; u < kAhead; ++u) row(cur[u]);
#pragma unroll
                for (int u = 0; u < kAhead; ++u) cur[u] = nxt[u];
            }
        } else {
            for (int t = 0; t < lim; ++t) row(S.tr[t]);
        }
    }
    FacOut o;
    o.ok = ok;
    o.growth = gmax;
    return o;
}

// The rows of the chosen root factorization, each tile from its checkpoint
// (lanes run tiles side by side); what is stored is each datum times its
// pseudo-random relative perturbation 1 + amp u (Alg. 3.2; u from the seed
// and the global row g: 2g for d, 2g + 1 for l), while the recurrence goes on
// with the unperturbed value.
DEV void factor_values(const double* d, const double* e, int64_t n, double sc, double mu, const double* ckp, int c,
                       double* Dd, double* Ld, uint64_t seed, double amp, int64_t row0) {
    const int l = lane_id();
    const int64_t ntiles = (n + kTile - 1) / kTile;
    for (int64_t tile = l; tile < ntiles; tile += kWave) {
        double dprev = ckp[tile * kWave + c];
        const int64_t base = tile * kTile;
        const int lim = (int)((n - base) < kTile ? (n - base) : kTile);
        for (int t0 = 0; t0 < lim; t0 += 8) {
            double dd[8], ee[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int64_t i = base + t0 + k;
                dd[k] = (t0 + k < lim) ? d[i] * sc : 0.0;
                ee[k] = (t0 + k < lim && i >= 1) ? e[i - 1] * sc : 0.0;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (t0 + k < lim) {
                    const int64_t i = base + t0 + k;
                    double dv;
                    if (i == 0) {
                        dv = dd[k] - mu;
                    } else {
                        const double lv = quot(recip(dprev), ee[k]);
                        const uint64_t gl = (uint64_t)(row0 + i - 1);
                        Ld[i - 1] = lv * (1.0 + amp * unit_pm1(seed, 2 * gl + 1));
                        dv = (dd[k] - mu) - lv * ee[k];
                    }
                    const uint64_t g = (uint64_t)(row0 + i);
                    Dd[i] = dv * (1.0 + amp * unit_pm1(seed, 2 * g));
                    dprev = dv;
                }
            }
        }
    }
}

// ---------------------------------------------------------- classification

DEV bool pair_split(double lo1, double hi1, double lo2, double hi2, double gaptol) {
    // reldist(j, j+1) >= gaptol (Sec. 3.2.3); a zero scale means an infinite
    // relative gap
    const double den = fmax(fmax(fabs(lo1), fabs(hi1)), fmax(fabs(lo2), fabs(hi2)));
    return (lo2 - hi1) >= gaptol * den;
}

// Partition a node's members into singletons and clusters (Alg. 4.2,
// ClassifyEigenvalues) and enqueue the resulting S- and C-tasks.
DEV void classify(Shared& S, const Params& P, int node_id) {
    const int l = lane_id();
    const Node nd = P.nodes[node_id];
    const Block blk = P.blocks[nd.block];
    const int64_t sb = blk.row0 - 1;
    const int a = nd.a, b = nd.b;
    const bool depth_cap = (nd.depth + 1 >= P.max_depth);
    // pass 1: count singletons, and the members in clusters (whose tasks
    // divide this node's share of the workers among them)
    int nsing = 0, nclu = 0;
    for (int base = a; base <= b; base += kWave) {
        const int j = base + l;
        bool single = false, clu = false;
        if (j <= b) {
            const double lo = ld_rlx_d(P.lo + sb + j), hi = ld_rlx_d(P.hi + sb + j);
            bool sbf = (j == a), saf = (j == b);
            if (!sbf) sbf = pair_split(ld_rlx_d(P.lo + sb + j - 1), ld_rlx_d(P.hi + sb + j - 1), lo, hi, P.gaptol);
            if (!saf) saf = pair_split(lo, hi, ld_rlx_d(P.lo + sb + j + 1), ld_rlx_d(P.hi + sb + j + 1), P.gaptol);
            if (depth_cap) sbf = saf = true;
            single = sbf && saf && j >= blk.w0 && j <= blk.w1;
            clu = !(sbf && saf);
        }
        nsing += __popcll(__ballot(single));
        nclu += __popcll(__ballot(clu));
    }
    // read by the cluster tasks (published by their push)
    if (l == 0) P.nodes[node_id].clustered = nclu;
    int64_t off = 0;
    if (l == 0 && nsing > 0)
        off = __hip_atomic_fetch_add(&P.ctl->slist_top, (int64_t)nsing, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    off = __shfl(off, 0);
    if (off + nsing > P.slist_cap) {
        set_error(P, kErrNoMem);
        return;
    }
    // pass 2: write the singleton list, gaps, and enqueue clusters.  A
    // cluster pushed in one chunk may be taken at once, and its task rewrites
    // its members' brackets in the child's coordinates; the one member of an
    // earlier chunk that a later chunk needs (its left neighbour) is therefore
    // carried in registers instead of being read again.
    int pos = 0;
    int open = -1;           // start of the cluster being scanned
    double open_lg = 0.0;    // its gap to the left neighbour
    double carry_lo = 0.0, carry_hi = 0.0;
    int64_t largest = 0;
    int ncl = 0, nunv = 0;
    for (int base = a; base <= b; base += kWave) {
        const int j = base + l;
        bool sbf = false, saf = false;
        double lo = 0.0, hi = 0.0, llo = 0.0, lhi = 0.0, rlo = 0.0, rhi = 0.0;
        if (j <= b) {
            lo = ld_rlx_d(P.lo + sb + j);
            hi = ld_rlx_d(P.hi + sb + j);
            sbf = (j == a);
            saf = (j == b);
            if (!sbf) {
                if (l == 0) {
                    llo = carry_lo;
                    lhi = carry_hi;
                } else {
                    llo = ld_rlx_d(P.lo + sb + j - 1);
                    lhi = ld_rlx_d(P.hi + sb + j - 1);
                }
                sbf = pair_split(llo, lhi, lo, hi, P.gaptol);
            }
            if (!saf) {
                rlo = ld_rlx_d(P.lo + sb + j + 1);
                rhi = ld_rlx_d(P.hi + sb + j + 1);
                saf = pair_split(lo, hi, rlo, rhi, P.gaptol);
            }
            if (depth_cap && !(sbf && saf)) {
                sbf = saf = true;
                nunv += 1;
            }
        }
        carry_lo = __shfl(lo, kWave - 1);
        carry_hi = __shfl(hi, kWave - 1);
        const bool in = (j <= b);
        const bool single = in && sbf && saf && j >= blk.w0 && j <= blk.w1;
        const uint64_t sm = __ballot(single);
        const double lg = (j == a) ? nd.lgap : (lo - lhi);
        const double rg = (j == b) ? nd.rgap : (rlo - hi);
        if (single) {
            const int k = pos + __popcll(sm & ((1ull << l) - 1ull));
            P.slist[off + k] = (int32_t)(sb + j);
            P.gap[sb + j] = fmin(lg, rg);
        }
        pos += __popcll(sm);
        // cluster boundaries, in order
        const uint64_t starts = __ballot(in && sbf && !saf);
        const uint64_t ends = __ballot(in && !sbf && saf);
        uint64_t ev = starts | ends;
        while (ev) {
            const int t = __ffsll((unsigned long long)ev) - 1;
            ev &= ev - 1ull;
            const int jj = base + t;
            const double lg_t = __shfl(lg, t), rg_t = __shfl(rg, t);
            if ((starts >> t) & 1ull) {
                open = jj;
                open_lg = lg_t;
            } else if (open >= 0) {
                const int p = open, q = jj;
                open = -1;
                if ((int64_t)(q - p + 1) > largest) largest = q - p + 1;
                if (q >= blk.w0 && p <= blk.w1) {
                    ++ncl;
                    // the cluster's gaps to its outside neighbours travel in
                    // gap[] at its end slots (published by the push)
                    if (l == 0) {
                        P.gap[sb + p] = open_lg;
                        P.gap[sb + q] = rg_t;
                    }
                    Task tk;
                    tk.type = kTaskCluster;
                    tk.node = node_id;
                    tk.a = p;
                    tk.b = q;
                    push_one(P, kQCluster, tk);
                }
            }
        }
    }
    // singleton bundles of the matrix's bundle size (at most one per lane)
    const int bs = P.probs[blk.prob].bundle;
    const int nb = (nsing + bs - 1) / bs;
    push_batch(P, kQSingle, nb, [&](int k) {
        Task t;
        t.type = kTaskSingle;
        t.node = node_id;
        t.a = (int)(off + (int64_t)k * bs);
        const int rem = nsing - k * bs;
        t.b = rem < bs ? rem : bs;
        return t;
    });
    stat_max(&P.ctl->largest_cluster, largest);
    add_stat(&P.ctl->n_unverified, nunv > 0 ? 1 : 0);
    (void)ncl;
}

// ---------------------------------------------------------------- tasks

DEV void task_root(Shared& S, const Params& P, int bid, int64_t& steps) {
    const int l = lane_id();
    const Block blk = P.blocks[bid];
    const int64_t n = blk.n;
    const double* d = P.d + blk.row0;
    const double* e = P.e + blk.row0;
    const double sc = P.probs[blk.prob].tscale;
    // Gershgorin interval of the block (App. B, Alg. B.3), of the scaled T
    double gl = __builtin_inf(), gu = -__builtin_inf();
    for (int64_t i = l; i < n; i += kWave) {
        const double r = (i > 0 ? fabs(e[i - 1] * sc) : 0.0) + (i < n - 1 ? fabs(e[i] * sc) : 0.0);
        gl = fmin(gl, d[i] * sc - r);
        gu = fmax(gu, d[i] * sc + r);
    }
    gl = wave_min(gl);
    gu = wave_max(gu);
    const double bnorm = fmax(fabs(gl), fabs(gu));
    const double slack = (2.0 * (double)n + 10.0) * bnorm * kEps;
    gl -= slack;
    gu += slack;
    const double spdiam = gu - gl;
    // extremal eigenvalues by multisection on NegCount(T): lanes 0-31 lambda_1,
    // lanes 32-63 lambda_n, until the brackets are 4 n eps bnorm wide
    double delta = 4.0 * (double)n * kEps * fmax(bnorm, kSafmin);
    double lo1 = gl, hi1 = gu, lon = gl, hin = gu;
    // the root's representation, the selection's checkpoints and (at
    // 4n + 128) the block of the cooperative passes
    const int64_t off = arena_alloc(P, 4 * n + kNodeExtra);
    if (off < 0) return;
    if (n >= kCoopMinRows && P.coop) {
        // long blocks: with idle workers' help (the same brackets either way)
        const int h = coop_helpers(P);
        if (h > 0)
            root_extremal_coop(S, P, bid, d, e, n, sc, delta, lo1, hi1, lon, hin,
                               reinterpret_cast<int64_t*>(P.arena + off + 4 * n + 128), off + 4 * n + 128,
                               h < kRootCoopHelpers ? h : kRootCoopHelpers, steps);
    }
    const int half = l >> 5, t = l & 31;
    for (int pass = 0; pass < 200; ++pass) {
        if (hi1 - lo1 <= delta && hin - lon <= delta) break;
        const double lo = half ? lon : lo1, hi = half ? hin : hi1;
        const double sig = coop_point(true, lo, hi, t, 32);
        const int c = negcount_T(S, d, e, n, sc, sig);
        steps += n * kWave;
        const uint64_t ge = __ballot(c >= (half ? (int)n : 1));
        const uint64_t g0 = ge & 0xffffffffull, g1 = ge >> 32;
        const int t0 = g0 ? __ffsll((unsigned long long)g0) - 1 : 32;
        const int t1 = g1 ? __ffsll((unsigned long long)g1) - 1 : 32;
        const double h0 = __shfl(sig, t0 < 32 ? t0 : 31), l0 = __shfl(sig, t0 > 0 ? t0 - 1 : 0);
        const double h1 = __shfl(sig, 32 + (t1 < 32 ? t1 : 31)), l1 = __shfl(sig, 32 + (t1 > 0 ? t1 - 1 : 0));
        if (t0 < 32) hi1 = h0;
        if (t0 > 0) lo1 = l0;
        if (t1 < 32) hin = h1;
        if (t1 > 0) lon = l1;
    }
    // root shift mu: just outside either end, so that T - mu I is definite
    // (lane 0 the left candidate, lane 1 the right one)
    double* C0 = P.arena + off;
    double* ckp = P.arena + off + 2 * n;   // the selection's checkpoints
    double mul = lo1 - delta, mur = hin + delta;
    int side = -1;
    for (int tr = 0; tr < 16 && side < 0; ++tr) {
        const double mu = (l == 0) ? mul : mur;
        const FacOut f = factor_select(S, d, e, n, sc, mu, (l == 0) ? 1 : -1, ckp);
        steps += 2 * n;
        const int ok0 = __shfl(f.ok, 0), ok1 = __shfl(f.ok, 1);
        const double g0 = __shfl(f.growth, 0), g1 = __shfl(f.growth, 1);
        if (ok0 && ok1) side = (g1 < g0) ? 1 : 0;
        else if (ok0) side = 0;
        else if (ok1) side = 1;
        else {
            delta *= 2.0;
            mul = lo1 - delta;
            mur = hin + delta;
        }
    }
    if (side < 0) {
        set_error(P, kErrInternal);
        return;
    }
    const double mu = side ? mur : mul;
    __syncthreads();
    // the rows, each datum perturbed by a pseudo-random relative amount of at
    // most xi*eps (Alg. 3.2)
    factor_values(d, e, n, sc, mu, ckp, side, C0, C0 + n, P.seed, P.xi * kEps, blk.row0);
    double* Dr = C0;
    double* Lr = Dr + n;
    // this wave reads the perturbed rows next; other workers get them through
    // the release of the pushes below
    __threadfence_block();
    __syncthreads();
    // root brackets: the definite root's spectrum lies between 0 and the
    // shifted Gershgorin end; confirm both ends by counts, widen if needed
    double rlo, rhi;
    double pad = 16.0 * (double)n * (P.xi + 1.0) * kEps;
    for (int tr = 0; tr < 12; ++tr) {
        if (side == 0) { rlo = 0.0; rhi = (gu - mu) * (1.0 + pad) + kSafmin; }
        else { rhi = 0.0; rlo = (gl - mu) * (1.0 + pad) - kSafmin; }
        const double sig = (l == 0) ? rlo : rhi;
        const int c = negcount_rep(S, Dr, Lr, n, sig);
        steps += 2 * n;
        const int c0 = __shfl(c, 0), c1 = __shfl(c, 1);
        if (c0 == 0 && c1 == (int)n) break;
        pad *= 16.0;
    }
    const int id = new_node(P);
    if (id < 0) return;
    // the block's share of the launch's workers (its part of all rows)
    const double root_share = (double)P.nworkers * (double)n / (double)(P.total_rows > 0 ? P.total_rows : 1);
    if (l == 0) {
        Node nd;
        nd.data = off;
        nd.block = bid;
        nd.depth = 0;
        nd.a = (int32_t)blk.k0;
        nd.b = (int32_t)blk.k1;
        nd.parent = -1;
        nd.pending = 0;
        nd.sigma = mu;
        nd.lgap = __builtin_inf();
        nd.rgap = __builtin_inf();
        nd.spdiam = spdiam;
        nd.checked = 0.0;
        nd.share = root_share;
        nd.clustered = 0;
        nd.pad = 0;
        P.nodes[id] = nd;
        P.blocks[bid].root = id;
    }
    const int64_t sb = blk.row0 - 1;
    // one multisection pass over the root bracket (64 points) places every
    // member between two counted points, so that the refinement slices can
    // be sized by the work each member still needs
    {
        const double sig = msec_point(rlo, rhi, l, kWave);
        const int c = negcount_rep(S, Dr, Lr, n, sig);
        steps += n * kWave;
        __syncthreads();
        S.m_cnt[l] = c;
        S.m_sig[l] = sig;
        __syncthreads();
    }
    int maxbits = 0;
    for (int64_t j = blk.k0 + l; j <= blk.k1; j += kWave) {
        int a = 0, b = kWave;   // first point whose count reaches j
        while (a < b) {
            const int mid = (a + b) >> 1;
            if (S.m_cnt[mid] >= j) b = mid; else a = mid + 1;
        }
        double lo = rlo, hi = rhi;
        // only points whose own count confirms them become bracket ends
        if (a < kWave && S.m_cnt[a] >= j) hi = S.m_sig[a];
        if (a > 0 && S.m_cnt[a - 1] < j) lo = S.m_sig[a - 1];
        P.lo[sb + j] = lo;
        P.hi[sb + j] = hi;
        P.lo0[sb + j] = lo;
        P.hi0[sb + j] = hi;
        P.vflag[sb + j] = 3;
        const int bits = member_bits(P, P.jobz ? kModeClass : kModeFull, lo, hi);
        P.need[sb + j] = (uint8_t)bits;
        maxbits = max(maxbits, bits);
    }
    for (int o = 32; o > 0; o >>= 1) maxbits = max(maxbits, __shfl_xor(maxbits, o));
    if (l == 0) {
        S.info_i[2] = id;
        S.info_d[0] = mu;
        S.info_d[1] = spdiam;
    }
    add_stat(&P.ctl->n_nodes, 1);
    push_slices(S, P, id, (int)blk.k0, (int)blk.k1, P.jobz ? kModeClass : kModeFull, root_share,
                P.probs[blk.prob].slice_max, sb, P.probs[blk.prob].lanes, maxbits);
}

DEV void load_members(Shared& S, const Params& P, int64_t sb, int a, int M) {
    const int l = lane_id();
    if (l < M) {
        const int j = a + l;
        const int64_t slot = sb + j;
        S.m_j[l] = j;
        S.m_slot[l] = slot;
        S.m_lo[l] = ld_rlx_d(P.lo + slot);
        S.m_hi[l] = ld_rlx_d(P.hi + slot);
        S.m_flag[l] = P.vflag[slot];
    }
    __syncthreads();
}

DEV void task_refine(Shared& S, const Params& P, int node_id, int a, int braw, int64_t& steps) {
    const int l = lane_id();
    const int mode = (braw >> 30) & 1;
    const int b = braw & 0x3fffffff;
    const Node nd = P.nodes[node_id];
    const Block blk = P.blocks[nd.block];
    const int64_t n = blk.n;
    const double* D = P.arena + nd.data;
    const double* L = D + n;
    const int M = b - a + 1;
    const int64_t sb = blk.row0 - 1;
    load_members(S, P, sb, a, M);
    MemberCtx C;
    C.mode = mode;
    C.na = nd.a;
    C.nb = nd.b;
    C.slot_base = sb;
    C.publish = true;
    C.lanes = P.probs[blk.prob].lanes;
    refine_members(S, P, D, L, n, M, C, steps);
    if (l < M) P.vflag[S.m_slot[l]] = (uint8_t)(S.m_flag[l] & 3);
    if (mode == kModeFull && !P.jobz && l < M) {
        // eigenvalues only: the root's bisection result is final
        const int j = S.m_j[l];
        if (j >= blk.w0 && j <= blk.w1) {
            const Problem& pr = P.probs[blk.prob];
            const int64_t col = blk.col0 + (j - blk.w0);
            P.w[pr.woff + col] = (nd.sigma + (S.m_lo[l] + 0.5 * (S.m_hi[l] - S.m_lo[l]))) * pr.tscale_inv;
        }
    }
    // the slice's writes go out with the count (release); the last slice
    // sees every other slice's writes (acquire)
    int last = 0;
    if (l == 0)
        last = (__hip_atomic_fetch_add(&P.nodes[node_id].pending, -1, __ATOMIC_ACQ_REL,
                                       __HIP_MEMORY_SCOPE_AGENT) == 1) ? 1 : 0;
    last = __shfl(last, 0);
    if (last && mode == kModeClass) classify(S, P, node_id);
}

DEV double grow_lo(double x, double nu) { return x - nu * fabs(x); }
DEV double grow_hi(double x, double nu) { return x + nu * fabs(x); }

DEV void task_cluster(Shared& S, const Params& P, int pid, int p, int q, int64_t& steps) {
    const int l = lane_id();
    const Node par = P.nodes[pid];
    const Block blk = P.blocks[par.block];
    const int64_t n = blk.n;
    const double* D = P.arena + par.data;
    // the child's share of the workers: twice its part of the parent's
    // clustered members, at most the parent's share.  Clusters of one parent
    // refine side by side; a share of exactly their part left workers idle
    // while they waited for each other's slower levels (glued Wilkinson), the
    // parent's whole share for each made their slices queue behind each
    // other's (1.3x the time)
    const double frac = (double)(q - p + 1) / (double)(par.clustered > 0 ? par.clustered : 1);
    const double child_share = fmin(par.share, 2.0 * par.share * frac);
    const double* L = D + n;
    const int64_t sb = blk.row0 - 1;
    // the new representation's D+ and L+, then the selection's checkpoints
    // (u and v, n + 64 doubles each), then the block of the cooperative end
    // refinement
    const int64_t off = arena_alloc(P, 4 * n + kNodeExtra);
    if (off < 0) return;
    double* Cn = P.arena + off;
    double* cku = Cn + 2 * n;
    double* ckv = Cn + 3 * n + 64;
    const int64_t cboff = off + 4 * n + 128;
    // 1. the cluster's end eigenvalues to full accuracy (Alg. 3.8, first step)
    if (l < 2) {
        const int j = (l == 0) ? p : q;
        const int64_t slot = sb + j;
        S.m_j[l] = j;
        S.m_slot[l] = slot;
        S.m_lo[l] = ld_rlx_d(P.lo + slot);
        S.m_hi[l] = ld_rlx_d(P.hi + slot);
        S.m_flag[l] = P.vflag[slot];
    }
    __syncthreads();
    MemberCtx C;
    C.mode = kModeFull;
    C.na = -1;
    C.nb = -1;
    C.slot_base = sb;
    C.publish = true;
    C.lanes = P.probs[blk.prob].lanes;
    // long representations: with idle workers' help when there are any (the
    // brackets are those of the sequential schedule either way)
    // A cluster whose child gets most of the workers (a chain of
    // representations) takes the deep schedule, with or without helpers.
    bool ends_done = false;
    const bool deep = n >= kCoopMinRows && child_share >= kDeepShare && C.lanes >= kDeepLg;
    if (n >= kCoopMinRows && (S.m_flag[0] & 3) == 3 && (S.m_flag[1] & 3) == 3 &&
        !(bracket_done(P, C.mode, S.m_lo[0], S.m_hi[0]) && bracket_done(P, C.mode, S.m_lo[1], S.m_hi[1]))) {
        if (deep) {
            ends_done = coop_refine(S, P, pid, D, L, n, 2, C.mode, C.lanes,
                                    reinterpret_cast<int64_t*>(P.arena + cboff), cboff,
                                    P.coop ? coop_helpers(P, kCoopMaxDeep) : 0, true, kDeepLg, steps);
        } else if (P.coop) {
            const int helpers = coop_helpers(P);
            if (helpers > 0)
                ends_done = coop_refine(S, P, pid, D, L, n, 2, C.mode, C.lanes,
                                        reinterpret_cast<int64_t*>(P.arena + cboff), cboff, helpers, true, 0, steps);
        }
    }
    if (!ends_done) refine_members(S, P, D, L, n, 2, C, steps);
    const double lo_p = S.m_lo[0], hi_p = S.m_hi[0];
    const double lo_q = S.m_lo[1], hi_q = S.m_hi[1];
    // gaps to the neighbours outside the cluster (shift invariant), as the
    // parent's classification measured them: the neighbours' brackets may be
    // rewritten meanwhile by their own tasks
    const double lgap = ld_rlx_d(P.gap + sb + p);
    const double rgap = ld_rlx_d(P.gap + sb + q);
    // 2. shifts just outside both ends; keep the candidate with the smaller
    //    element growth; back off while the growth is too large (Alg. 3.8)
    // All back-off levels of Alg. 3.8 are tried at once: lane 2t uses
    // tau_l(t) and lane 2t+1 tau_r(t).  Level 0 sits 100 eps |lambda|
    // outside the cluster; levels 1..T-1 back off geometrically from
    // 100 eps |lambda| up to a quarter of the gap to the nearest eigenvalue
    // outside the cluster on that side, so that no level moves the shift past
    // the cluster's neighbours (which would keep the cluster from being
    // broken).  The selection below is the algorithm's sequential rule: the
    // first level whose better candidate passes the growth test wins;
    // otherwise the least growth seen.  Only the winner's rows are written.
    const double spd = par.spdiam;
    const double thresh = 8.0 * spd;    // ||D+|| = O(spdiam): accept at once
    const int T = P.max_tries < 32 ? P.max_tries : 32;
    const int tt = l >> 1, side = l & 1;
    const double tau_l0 = lo_p - 100.0 * kEps * fabs(lo_p);
    const double tau_r0 = hi_q + 100.0 * kEps * fabs(hi_q);
    double mytau = side ? tau_r0 : tau_l0;
    // the gap between the end member and its inner neighbour: the child can
    // split the end member off only if the shift stays within about
    // gap / gaptol of it
    const double gin_l = fmax(ld_rlx_d(P.lo + sb + p + 1) - hi_p, 0.0);
    const double gin_r = fmax(lo_q - ld_rlx_d(P.hi + sb + q - 1), 0.0);
    if (tt >= 1 && T >= 2) {
        // relative steps only: an absolute floor (say eps * spdiam) would stop
        // a deep node, whose eigenvalues are tiny, from ever getting closer
        const double dmin = fmax(100.0 * kEps * (side ? fmax(fabs(lo_q), fabs(hi_q))
                                                       : fmax(fabs(lo_p), fabs(hi_p))),
                                 64.0 * kSafmin);
        const double g = side ? rgap : lgap;
        const double gin = side ? gin_r : gin_l;
        const double dmax = fmax(dmin, fmin(0.25 * fmin(__builtin_isfinite(g) ? g : spd, spd),
                                             gin / (2.0 * P.gaptol)));
        const double frac = (T > 2) ? (double)(tt - 1) / (double)(T - 2) : 0.0;
        const double del = dmin * pow(dmax / dmin, frac);
        mytau = side ? tau_r0 + del : tau_l0 - del;
    }
    // the division-free form first; the quotient form when it cannot tell for
    // some candidate, or when no candidate passed and one was rejected for an
    // overflow (the least growth must then be known for every candidate)
    const bool mine = l < 2 * T;
    const HomFac hf = dstqds_select_hom(S, D, L, n, mytau, cku, ckv);
    FacOut f;
    f.ok = hf.ok;
    f.growth = hf.growth;
    bool quot_form = wave_or((mine && hf.unknown) ? 1 : 0) != 0;
    if (quot_form) f = dstqds_select(S, D, L, n, mytau, cku);
    steps += 2 * n * T;
    double best, best_tau;
    int chosen, best_lane;
    double tau, chosen_growth;
    auto pick = [&]() {
        best = __builtin_inf();
        best_tau = 0.0;
        chosen = -1;
        best_lane = 0;
        tau = 0.0;
        chosen_growth = 0.0;
        for (int t = 0; t < T; ++t) {
            const int ok0 = __shfl(f.ok, 2 * t), ok1 = __shfl(f.ok, 2 * t + 1);
            const double g0 = __shfl(f.growth, 2 * t), g1 = __shfl(f.growth, 2 * t + 1);
            const double t0 = __shfl(mytau, 2 * t), t1 = __shfl(mytau, 2 * t + 1);
            int pk = -1;
            if (ok0 && ok1) pk = (g1 < g0) ? 1 : 0;
            else if (ok0) pk = 0;
            else if (ok1) pk = 1;
            if (pk < 0) continue;
            const double g = pk ? g1 : g0;
            const double tp = pk ? t1 : t0;
            if (g < best) { best = g; best_tau = tp; best_lane = 2 * t + pk; }
            if (g <= thresh && chosen < 0) {
                chosen = 2 * t + pk;
                tau = tp;
                chosen_growth = g;
            }
        }
    };
    pick();
    if (chosen < 0 && !quot_form && wave_or((mine && !hf.ok) ? 1 : 0)) {
        quot_form = true;
        f = dstqds_select(S, D, L, n, mytau, cku);
        steps += 2 * n * T;
        pick();
    }
    if (quot_form && l == 0) S.redo_fac += 1;
    int unverified = 0;
    if (chosen < 0) {
        if (!(best < __builtin_inf())) {
            set_error(P, kErrNoConv);
            return;
        }
        // no candidate passed: the least element growth (Alg. 3.8, last resort)
        chosen = best_lane;
        tau = best_tau;
        chosen_growth = best;
        unverified = 1;
    }
    // the checkpoints of lane `chosen` go to every lane
    __syncthreads();
    if (quot_form) dstqds_values(D, L, n, tau, cku, chosen, Cn, Cn + n);
    else dstqds_values_hom(D, L, n, tau, cku, ckv, chosen, Cn, Cn + n);
    steps += n;
    const int id = new_node(P);
    if (id < 0) return;
    if (l == 0) {
        // an unverified representation's columns are checked after the tree,
        // unless an ancestor's check already covers them
        double checked = par.checked;
        if (unverified && checked == 0.0 && P.jobz) {
            const int c0 = max(p, blk.w0), c1 = min(q, blk.w1);
            const int64_t m = (int64_t)c1 - c0 + 1;
            if (m >= 2 && m <= kCheckMax) {
                const int64_t k = __hip_atomic_fetch_add(&P.ctl->chk_top, (int64_t)1, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                if (k < P.chk_cap) {
                    const Problem pr = P.probs[blk.prob];
                    CheckRec rc;
                    rc.z = pr.zoff + (blk.col0 + (c0 - blk.w0)) * pr.ldz + (blk.row0 - pr.row0);
                    rc.ldz = pr.ldz;
                    rc.n = n;
                    rc.m = m;
                    rc.loss[0] = rc.loss[1] = 0.0;
                    rc.pad[0] = rc.pad[1] = 0;
                    P.chk[k] = rc;
                    checked = 1.0;
                } else {
                    add_stat(&P.ctl->n_check_failed, 1);
                }
            } else if (m > kCheckMax) {
                add_stat(&P.ctl->n_check_wide, 1);
            }
        }
        // every unverified representation with wanted members: checked after
        // the tree for conditional element growth against their vectors
        if (unverified && P.jobz && P.cond_k > 0.0) {
            const int c0 = max(p, blk.w0), c1 = min(q, blk.w1);
            const int64_t m = (int64_t)c1 - c0 + 1;
            if (m >= 1) {
                const int64_t k = __hip_atomic_fetch_add(&P.ctl->grw_top, (int64_t)1, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                if (k < P.grw_cap) {
                    const Problem pr = P.probs[blk.prob];
                    GrowthRec g;
                    g.rep = off;
                    g.z = pr.zoff + (blk.col0 + (c0 - blk.w0)) * pr.ldz + (blk.row0 - pr.row0);
                    g.ldz = pr.ldz;
                    g.n = n;
                    g.m = m;
                    g.mc = m < kGrowthSample ? m : kGrowthSample;
                    g.col0 = 0;
                    g.bound = (P.cond_k / 3.0) * (double)n * spd;   // see mrrr_growth_kernel
                    g.spdiam = spd;
                    g.flag = 0;
                    g.pad = 0;
                    P.grw[k] = g;
                }
            }
        }
        Node nd;
        nd.data = off;
        nd.block = par.block;
        nd.depth = par.depth + 1;
        nd.a = p;
        nd.b = q;
        nd.parent = pid;
        nd.pending = 0;
        nd.sigma = par.sigma + tau;
        nd.lgap = lgap;
        nd.rgap = rgap;
        nd.spdiam = spd;
        nd.checked = checked;
        nd.share = child_share;
        nd.clustered = 0;
        nd.pad = 0;
        P.nodes[id] = nd;
    }
    // 3. child brackets: (lambda(1 -+ nu) - tau)(1 -+ nu), nu = 10 k_rr n eps
    //    with k_rr = 10, widened outward (Sec. 3.2.3)
    //    (eight 64-member chunks' loads in flight at once: the members'
    //    brackets are stable since the parent was classified, and the pop
    //    that brought this task cleared this CU's cache)
    const double nu = 100.0 * (double)n * kEps;
    int maxbits = 0;
    constexpr int kChunks = 8;
    for (int base = p; base <= q; base += kChunks * kWave) {
        double lo4[kChunks], hi4[kChunks];
#pragma unroll
        for (int k = 0; k < kChunks; ++k) {
            const int j = base + k * kWave + l;
            lo4[k] = (j <= q) ? P.lo[sb + j] : 0.0;
            hi4[k] = (j <= q) ? P.hi[sb + j] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kChunks; ++k) {
            const int j = base + k * kWave + l;
            if (j <= q) {
                const int64_t slot = sb + j;
                double lo = lo4[k], hi = hi4[k];
                if (j == p) { lo = lo_p; hi = hi_p; }
                if (j == q) { lo = lo_q; hi = hi_q; }
                const double clo = grow_lo(grow_lo(lo, nu) - tau, nu);
                const double chi = grow_hi(grow_hi(hi, nu) - tau, nu);
                st_rlx_d(P.lo + slot, clo);
                st_rlx_d(P.hi + slot, chi);
                P.lo0[slot] = clo;
                P.hi0[slot] = chi;
                P.vflag[slot] = 0;
                const int bits = member_bits(P, kModeClass, clo, chi);
                P.need[slot] = (uint8_t)bits;
                maxbits = max(maxbits, bits);
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) maxbits = max(maxbits, __shfl_xor(maxbits, o));
    if (l == 0) {
        S.info_i[0] = par.depth;
        S.info_i[1] = unverified;
        S.info_i[2] = id;
        S.info_d[0] = tau;
        S.info_d[1] = chosen_growth;
    }
    add_stat(&P.ctl->n_nodes, 1);
    add_stat(&P.ctl->n_unverified, unverified);
    if (l == 0) {
        __hip_atomic_fetch_max(&P.ctl->dmax, par.depth + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    push_slices(S, P, id, p, q, kModeClass, child_share, P.probs[blk.prob].slice_max, sb, P.probs[blk.prob].lanes,
                maxbits);
}

// ------------------------------------- a helper for a singleton bundle
//
// When idle workers are about (the last bundles of a solve), a bundle's
// worker (the leader) takes one of them as a helper, and the two waves share
// each twisted factorisation and the eigenvector solve, in the same arithmetic
// as the one-wave forms, so that every value comes out bit for bit the same:
//   1. the leader runs the forward transform (tw_forward) while the helper
//      runs the backward one over all rows, keeping its checkpoints
//      (tw_backward_plain);
//   2. the 16-row blocks are split at a tile boundary: each wave replays both
//      transforms of its blocks from the checkpoints and ranks |gamma| there
//      (tw_gamma_blocks); the lower index wins ties, as in the one-wave scan;
//   3. the eigenvector's part below the twist and its part above it are
//      written by the two waves (solve_vector_hom's two halves).
// The leader publishes its lanes' data in a block of the node pool and a
// command word; the helper answers with an acknowledgement (release /
// acquire at agent scope).
constexpr int64_t kAssistMinRows = 4096;   // shorter transforms are not worth sharing
enum AsWord : int {
    kAsGen = 0,     // (sequence << 8) | command; kAsDone once the leader is finished
    kAsJoin,        // 0 open, 1 a helper joined, 2 closed without one
    kAsAck,         // the helper's last finished sequence << 8 | command
    kAsNode,        // the node whose representation is used
    kAsLive,        // lanes that take part (64-bit mask)
    kAsHalf,        // the first block of the helper's share (a multiple of 4)
    kAsStride,      // checkpoint stride of the bundle's problem
    kAsLam = 8,                 // [64] shifts (bits of doubles)
    kAsCk = kAsLam + kWave,     // [64] checkpoint column offsets in P.ck
    kAsR = kAsCk + kWave,       // [64] twist indices
    kAsScale = kAsR + kWave,    // [64] eigenvector scales
    kAsZ = kAsScale + kWave,    // [64] column offsets in P.Z
    kAsBest = kAsZ + kWave,     // [64] best |gamma| (in: gamma_{n-1}; out: the helper's)
    kAsRb = kAsBest + kWave,    // [64] its row
    kAsMw = kAsRb + kWave,      // [64] the helper's smallest |omega| / its sum of squares
    kAsFin = kAsMw + kWave,     // [64] the helper's final backward state finite
    kAsWords = kAsFin + kWave
};
enum AsCmd : int { kCmdBwd = 1, kCmdGamma = 2, kCmdVecUp = 3 };
constexpr int64_t kAsDone = -1;

struct Assist {
    int64_t* cb;
    int64_t gen;
    bool on;
};

DEV double as_ldd(int64_t* cb, int w) { return __longlong_as_double((long long)cb_ld(cb, w)); }
DEV void as_std(int64_t* cb, int w, double x) { cb_st(cb, w, (int64_t)__double_as_longlong(x)); }

// Every lane's stores out, then the command (release).
DEV void as_issue(Assist& as, int cmd) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    as.gen = (((as.gen >> 8) + 1) << 8) | cmd;
    if (lane_id() == 0) __hip_atomic_store(as.cb + kAsGen, as.gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Until the helper has acknowledged the last command (acquire); false on an
// error or the watchdog.
DEV bool as_wait(const Params& P, Assist& as) {
    int stop = 0;
    if (lane_id() == 0) {
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(as.cb + kAsAck, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != as.gen) {
            if (__hip_atomic_load(&P.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                wall_clock64() - t0 > P.timeout_ticks) {
                stop = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __syncthreads();
    if (__shfl(stop, 0)) {
        set_error(P, kErrTimeout);
        return false;
    }
    return true;
}

// Takes a helper for a bundle of node `node_id` if an idle worker joins
// within 40 us (the lanes' checkpoint columns at ck_off).  Tried at the start
// of every Rayleigh-quotient step and before the eigenvector solve until one
// joins: the result does not depend on when it does.  The block comes from
// the node pool once per bundle and serves every try.
DEV void assist_try(const Params& P, Assist& as, int node_id, int64_t n, int64_t ck_stride, int64_t ck_off) {
    if (as.on || !P.assist || n < kAssistMinRows || coop_helpers(P) <= 0) return;
    if (as.cb == nullptr) {
        const int64_t off = arena_alloc(P, kAsWords);
        if (off < 0) return;
        as.cb = reinterpret_cast<int64_t*>(P.arena + off);
    }
    int64_t* cb = as.cb;
    if (lane_id() == 0) {
        cb_st(cb, kAsGen, 0);
        cb_st(cb, kAsAck, 0);
        cb_st(cb, kAsNode, node_id);
        cb_st(cb, kAsStride, ck_stride);
        cb_st(cb, kAsJoin, 0);
    }
    cb_st(cb, kAsCk + lane_id(), ck_off);
    as.gen = 0;
    const int64_t off = reinterpret_cast<double*>(cb) - P.arena;
    Task t;
    t.type = kTaskAssist;
    t.node = node_id;
    t.a = (int32_t)(uint32_t)((uint64_t)off & 0xffffffffull);
    t.b = (int32_t)(uint32_t)((uint64_t)off >> 32);
    if (!push_one(P, kQRefine, t)) return;   // its release publishes the block
    int64_t st = 0;
    if (lane_id() == 0) {
        const uint64_t t0 = wall_clock64();
        for (;;) {
            st = cb_ld(cb, kAsJoin);
            if (st != 0) break;
            if (wall_clock64() - t0 > 4000) {   // 40 us of the 100 MHz clock: close it
                int64_t expect = 0;
                __hip_atomic_compare_exchange_strong(cb + kAsJoin, &expect, (int64_t)2, __ATOMIC_ACQ_REL,
                                                     __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                st = (expect == 0) ? 2 : expect;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    as.on = (__shfl(st, 0) == 1);
}

DEV void assist_close(Assist& as) {
    if (as.on && lane_id() == 0)
        __hip_atomic_store(as.cb + kAsGen, kAsDone, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    as.on = false;
}

// The backward (progressive) transform over all rows with its checkpoints,
// in twisted_hom's arithmetic, without the ranking of gamma.  Returns the
// smallest |omega|; `fin` whether the final state is finite.
DEV double tw_backward_plain(Shared& S, const double* D, const double* L, int64_t n, double lam, bool live,
                             const CkPtr& ck, bool& fin, int64_t& steps) {
    const int64_t cl = (n - 1) / kCkb;
    double x = D[n - 1] - lam, y = 1.0, F = 1.0, mw = 1.0;
    if (live) {
        ck.at(cl, 3) = x;
        ck.at(cl, 4) = y;
        ck.at(cl, 5) = F;
    }
    const int64_t last_tile = ((n - 1) / kTile) * kTile;
    RepRow fb_ = rep_fetch(D, L, last_tile, n);
    for (int64_t tb = last_tile; tb >= 0; tb -= kTile) {
        rep_commit(S, fb_);
        if (tb - kTile >= 0) fb_ = rep_fetch(D, L, tb - kTile, n);
        const int64_t cfirst = tb / kCkb;
        const int64_t clast = ((tb + kTile - 1) < (n - 1) ? (tb + kTile - 1) : (n - 1)) / kCkb;
        for (int64_t c = clast; c >= cfirst; --c) {
            const int64_t b0 = c * kCkb;
            const int64_t b1 = (b0 + kCkb) < (n - 1) ? (b0 + kCkb) : (n - 1);   // rows [b0, b1)
            if (b0 >= b1) continue;
            if (c < cl && live) {
                ck.at(c, 3) = x;
                ck.at(c, 4) = y;
                ck.at(c, 5) = F;
            }
            const int nb = (int)(b1 - b0);
            auto run = [&](auto full_t) {
                constexpr bool kFull = decltype(full_t)::value;
                const int kb = (int)(b0 - tb);
                QRow xr[kCkb];
#pragma unroll
                for (int t = 0; t < kCkb; ++t) xr[t] = S.tr[kFull ? kb + t : (kb + t < kTile ? kb + t : kTile - 1)];
#pragma unroll
                for (int t = kCkb - 1; t >= 0; --t) {
                    if (kFull || t < nb) {
                        const double om = __builtin_fma(xr[t].dll, y, x);
                        const double m = xr[t].d * x;
                        x = __builtin_fma(-lam, om, m);
                        F = __builtin_fma(xr[t].dl2, F, om * om);
                        y = om;
                        mw = fmin(mw, fabs(om));
                        if ((t & 7) == 0) hom_bwd_scale(x, y, F);
                    }
                }
            };
            if (nb == kCkb) run(std::true_type{});
            else run(std::false_type{});
        }
    }
    steps += n;
    fin = __builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(F);
    return mw;
}

// twisted_hom's ranking of |gamma| over the blocks [c0, c1] (c0 a multiple
// of 4), both transforms replayed from their checkpoints; best and r come in
// as the ranking stands above block c1 and go out as it stands after c0.
DEV void tw_gamma_blocks(Shared& S, const double* D, const double* L, int64_t n, double lam, bool live,
                         const CkPtr& ck, int64_t c0, int64_t c1, double& best, int& r, int64_t& steps) {
    if (c1 < c0) return;
    const int64_t t_hi = (c1 * kCkb / kTile) * kTile, t_lo = c0 * kCkb;
    RepRow fb_ = rep_fetch(D, L, t_hi, n);
    // both transforms' states entering each block, loaded a block ahead
    double un = live ? ck.at(c1, 0) : 0.0, vn = live ? ck.at(c1, 1) : 1.0;
    double xn = live ? ck.at(c1, 3) : 0.0, yn = live ? ck.at(c1, 4) : 1.0;
    for (int64_t tb = t_hi; tb >= t_lo; tb -= kTile) {
        rep_commit(S, fb_);
        if (tb - kTile >= t_lo) fb_ = rep_fetch(D, L, tb - kTile, n);
        const int64_t cfirst = tb / kCkb;
        const int64_t clast0 = ((tb + kTile - 1) < (n - 1) ? (tb + kTile - 1) : (n - 1)) / kCkb;
        const int64_t clast = clast0 < c1 ? clast0 : c1;
        for (int64_t c = clast; c >= cfirst; --c) {
            double uu = un, vv = vn, x = xn, y = yn, F = 0.0;
            const bool ahead = live && c - 1 >= c0;
            un = ahead ? ck.at(c - 1, 0) : 0.0;
            vn = ahead ? ck.at(c - 1, 1) : 1.0;
            xn = ahead ? ck.at(c - 1, 3) : 0.0;
            yn = ahead ? ck.at(c - 1, 4) : 1.0;
            const int64_t b0 = c * kCkb;
            const int64_t b1 = (b0 + kCkb) < (n - 1) ? (b0 + kCkb) : (n - 1);   // rows [b0, b1)
            if (b0 >= b1) continue;
            const int nb = (int)(b1 - b0);
            auto run = [&](auto full_t) {
                constexpr bool kFull = decltype(full_t)::value;
                const int kb = (int)(b0 - tb);
                QRow xr[kCkb];
#pragma unroll
                for (int t = 0; t < kCkb; ++t) xr[t] = S.tr[kFull ? kb + t : (kb + t < kTile ? kb + t : kTile - 1)];
                double ur[kCkb], vr[kCkb];
#pragma unroll
                for (int t = 0; t < kCkb; ++t) {
                    ur[t] = uu;
                    vr[t] = vv;
                    if (kFull || t < nb) {
                        const double w = __builtin_fma(xr[t].d, vv, uu);
                        const double p = uu * xr[t].dll;
                        uu = __builtin_fma(-lam, w, p);
                        vv = w;
                        if ((t & 7) == 7) {
                            const int ex = __builtin_amdgcn_frexp_exp(vv);
                            uu = __builtin_ldexp(uu, -ex);
                            vv = __builtin_ldexp(vv, -ex);
                        }
                    }
                }
                int rt = -1;
#pragma unroll
                for (int t = kCkb - 1; t >= 0; --t) {
                    if (kFull || t < nb) {
                        const double om = __builtin_fma(xr[t].dll, y, x);
                        const double m = xr[t].d * x;
                        const double num = __builtin_fma(ur[t], om, m * vr[t]);
                        const double den = vr[t] * om;
                        const double ga = fabs(num) * __builtin_amdgcn_rcp(fabs(den));
                        const bool take = ga <= best;
                        best = take ? ga : best;
                        rt = take ? t : rt;
                        x = __builtin_fma(-lam, om, m);
                        y = om;
                        if ((t & 7) == 0) hom_bwd_scale(x, y, F);
                    }
                }
                if (rt >= 0) r = (int)b0 + rt;
            };
            if (nb == kCkb) run(std::true_type{});
            else run(std::false_type{});
        }
    }
    steps += (c1 - c0 + 1) * kCkb;
}

// twisted_hom shared with the helper (see above); the same result.
DEV TwistOut twisted_split(Shared& S, const Params& P, const double* D, const double* L, int64_t n, double lam,
                           bool live, const CkPtr& ck, Assist& as, int64_t& steps) {
    const int l = lane_id();
    const int64_t cl = (n - 1) / kCkb;
    as_std(as.cb, kAsLam + l, lam);
    const uint64_t lm = __ballot(live);   // (by every lane, outside the branch)
    if (l == 0) cb_st(as.cb, kAsLive, (int64_t)lm);
    as_issue(as, kCmdBwd);
    const TwFwd fw = tw_forward(S, D, L, n, lam, live, ck, steps);
    if (!as_wait(P, as)) {
        TwistOut o;
        o.neg = 0; o.r = 0; o.gam = 0.0; o.nrm2 = 1.0; o.bad = 0; o.guarded = 0;
        return o;
    }
    const double mwb = as_ldd(as.cb, kAsMw + l);
    const bool bfin = cb_ld(as.cb, kAsFin + l) != 0;
    // the helper ranks the upper blocks from gamma_{n-1} on, the leader the
    // lower ones from scratch
    const int64_t half = ((cl + 1) / 8) * 4;
    as_std(as.cb, kAsBest + l, fabs(fw.wl) * __builtin_amdgcn_rcp(fabs(fw.vl)));   // gamma_{n-1} = d+_{n-1}
    if (l == 0) cb_st(as.cb, kAsHalf, half);
    as_issue(as, kCmdGamma);
    double best = __builtin_inf();
    int r = -1;
    tw_gamma_blocks(S, D, L, n, lam, live, ck, 0, half - 1, best, r, steps);
    if (!as_wait(P, as)) {
        TwistOut o;
        o.neg = 0; o.r = 0; o.gam = 0.0; o.nrm2 = 1.0; o.bad = 0; o.guarded = 0;
        return o;
    }
    const double best_h = as_ldd(as.cb, kAsBest + l);
    const int r_h = (int)cb_ld(as.cb, kAsRb + l);
    if (!(r >= 0 && best <= best_h)) r = r_h;
    return tw_at_r(D, L, n, lam, live, ck, r, fw, bfin, fmin(fw.mw, mwb));
}

// The helper's side: join the bundle whose block is at `off`, then answer
// its commands until the leader is finished.
DEV void task_assist(Shared& S, const Params& P, int64_t off, int64_t& steps) {
    const int l = lane_id();
    int64_t* cb = reinterpret_cast<int64_t*>(P.arena + off);
    int joined = 0;
    if (l == 0) {
        int64_t expect = 0;
        joined = __hip_atomic_compare_exchange_strong(cb + kAsJoin, &expect, (int64_t)1, __ATOMIC_ACQ_REL,
                                                      __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) ? 1 : 0;
    }
    if (!__shfl(joined, 0)) return;
    const int node_id = (int)cb_ld(cb, kAsNode);
    const Node nd = P.nodes[node_id];
    const Block blk = P.blocks[nd.block];
    const int64_t n = blk.n;
    const double* D = P.arena + nd.data;
    const double* L = D + n;
    const int64_t stride = cb_ld(cb, kAsStride);
    const int64_t cl = (n - 1) / kCkb;
    const uint64_t t0 = wall_clock64();
    int64_t last = 0;
    for (;;) {
        int64_t gen = 0;
        if (l == 0) {
            for (;;) {
                gen = __hip_atomic_load(cb + kAsGen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                if (gen != last) break;
                if (__hip_atomic_load(&P.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                    wall_clock64() - t0 > P.timeout_ticks) {
                    gen = kAsDone;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        gen = __shfl(gen, 0);
        if (gen == kAsDone) return;
        last = gen;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int cmd = (int)(gen & 0xff);
        const bool live = ((uint64_t)cb_ld(cb, kAsLive) >> l) & 1ull;
        const double lam = as_ldd(cb, kAsLam + l);
        CkPtr ck;
        ck.base = P.ck + cb_ld(cb, kAsCk + l);
        ck.stride = stride;
        if (cmd == kCmdBwd) {
            bool fin = true;
            const double mw = tw_backward_plain(S, D, L, n, lam, live, ck, fin, steps);
            as_std(cb, kAsMw + l, mw);
            cb_st(cb, kAsFin + l, fin ? 1 : 0);
        } else if (cmd == kCmdGamma) {
            double best = as_ldd(cb, kAsBest + l);
            int r = (int)(n - 1);
            tw_gamma_blocks(S, D, L, n, lam, live, ck, cb_ld(cb, kAsHalf), cl, best, r, steps);
            as_std(cb, kAsBest + l, best);
            cb_st(cb, kAsRb + l, r);
        } else if (cmd == kCmdVecUp) {
            const int r = (int)cb_ld(cb, kAsR + l);
            const double scale = as_ldd(cb, kAsScale + l);
            double* zcol = P.Z + cb_ld(cb, kAsZ + l);
            const double ss = solve_vector_hom(S, D, L, n, lam, live, r, scale, ck, zcol, true, 1, steps);
            as_std(cb, kAsMw + l, ss);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (l == 0) __hip_atomic_store(cb + kAsAck, gen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// twisted() with the helper: the shared transforms, then the guarded form for
// the lanes that need it, on the leader alone.
DEV TwistOut twisted_assisted(Shared& S, const Params& P, const double* D, const double* L, int64_t n, double lam,
                              bool live, const CkPtr& ck, Assist& as, int64_t& steps) {
    TwistOut o = twisted_split(S, P, D, L, n, lam, live, ck, as, steps);
    const bool redo = live && o.bad;
    if (wave_or(redo ? 1 : 0)) {
        const TwistOut g = twisted_impl<true>(S, D, L, n, lam, redo, ck, steps);
        if (lane_id() == 0) S.redo += 1;
        if (redo) {
            o = g;
            o.guarded = 1;
        }
    }
    return o;
}

// solve_vector() with the helper: it writes the rows below the twist, the
// leader the rest; a NaN in either part, or a guarded lane, goes to the
// guarded form on the leader alone.
DEV void solve_vector_assisted(Shared& S, const Params& P, const double* D, const double* L, int64_t n, double lam,
                               bool live, int r, double scale, const CkPtr& ck, double* zcol, bool guarded,
                               Assist& as, int64_t& steps) {
    const int l = lane_id();
    const bool hl = live && !guarded;
    as_std(as.cb, kAsLam + l, lam);
    cb_st(as.cb, kAsR + l, r);
    as_std(as.cb, kAsScale + l, scale);
    cb_st(as.cb, kAsZ + l, (int64_t)(zcol - P.Z));
    const uint64_t lm = __ballot(hl);   // (by every lane, outside the branch)
    if (l == 0) cb_st(as.cb, kAsLive, (int64_t)lm);
    as_issue(as, kCmdVecUp);
    const double ss = solve_vector_hom(S, D, L, n, lam, hl, r, scale, ck, zcol, true, 2, steps);
    if (!as_wait(P, as)) return;
    const double ssh = as_ldd(as.cb, kAsMw + l);
    const bool redo = live && (guarded || __builtin_isnan(ss) || __builtin_isnan(ssh));
    if (wave_or(redo ? 1 : 0)) {
        solve_vector_impl<true>(S, D, L, n, lam, redo, r, scale, ck, zcol, true, steps);
        if (lane_id() == 0) S.redo += 1;
    }
}

// A bundle of singletons of one node, one per lane (Alg. 4.3): Rayleigh
// quotient iteration on twisted factorisations with the inertia of Delta_r
// guarding the direction; bisection to full accuracy plus one more Getvec as
// the fallback; then the eigenvector (Alg. 3.7) straight into Z.
DEV void task_single(Shared& S, const Params& P, int node_id, int off, int cnt, int64_t& steps) {
    const int l = lane_id();
    const Node nd = P.nodes[node_id];
    const Block blk = P.blocks[nd.block];
    const Problem pr = P.probs[blk.prob];
    const int64_t n = blk.n;
    const double* D = P.arena + nd.data;
    const double* L = D + n;
    const int64_t sb = blk.row0 - 1;
    const bool act = l < cnt;
    const int64_t slot = P.slist[off + (act ? l : 0)];
    const int j = (int)(slot - sb);
    double lo = ld_rlx_d(P.lo + slot), hi = ld_rlx_d(P.hi + slot);
    const double gap = P.gap[slot];
    int vf = P.vflag[slot];
    double lam = lo + 0.5 * (hi - lo);
    CkPtr ck;
    ck.base = P.ck + pr.ck_base + (blk.col0 + (j - blk.w0));   // one column per output column
    ck.stride = pr.ck_stride;
    // a helper for long representations when a worker is idle
    Assist as;
    as.cb = nullptr;
    as.gen = 0;
    as.on = false;
    const int64_t ck_off = (int64_t)(ck.base - P.ck);
    // tol1: the local residual may stop at n eps gap in FP64; with data in a
    // coarser format (unit roundoff eps_x) the orthogonality goal is
    // eps_x sqrt(n), and the iteration stops at eps_x sqrt(n) gap (Sec. 5.1.1)
    const double tol1 = (P.io_eps > 0.0) ? P.io_eps * sqrt((double)n) : (double)n * kEps, tol2 = 2.0 * kEps;
    // Alg. 4.3: Rayleigh-quotient steps while the correction improves the
    // eigenvalue -- right sign, inside the bracket, and at most half the
    // previous correction (a correction that stops shrinking is at the
    // rounding floor of the representation); otherwise bisection to full
    // accuracy.  Lanes that need bisection wait, so that one refinement
    // round serves all of them; one more factorisation at the refined value
    // is then accepted.
    bool done = !act, need_fb = false, force = false, tg = false;
    double prev = __builtin_inf();
    int r = 0;
    double nrm2 = 1.0;
    int64_t nrqi = 0, nfb = 0;
    for (int it = 0; it < P.max_rqi + 4; ++it) {
        const bool live = !done && !need_fb;
        if (__ballot(live) == 0ull) {
            const uint64_t fm = __ballot(need_fb);
            if (fm == 0ull) break;
            const int k = __popcll(fm & ((1ull << l) - 1ull));
            if (need_fb) {
                S.m_j[k] = j;
                S.m_slot[k] = slot;
                S.m_lo[k] = lo;
                S.m_hi[k] = hi;
                S.m_flag[k] = vf;
            }
            __syncthreads();
            MemberCtx C;
            C.mode = kModeFull;
            C.na = -1;
            C.nb = -1;
            C.slot_base = sb;
            C.publish = false;
            C.lanes = kWave;
            refine_members(S, P, D, L, n, __popcll(fm), C, steps);
            if (need_fb) {
                lo = S.m_lo[k];
                hi = S.m_hi[k];
                vf = S.m_flag[k];
                lam = lo + 0.5 * (hi - lo);
                force = true;
                need_fb = false;
            }
            nfb += __popcll(fm);
            __syncthreads();
            continue;
        }
        assist_try(P, as, node_id, n, pr.ck_stride, ck_off);
        const TwistOut tw = as.on ? twisted_assisted(S, P, D, L, n, lam, live, ck, as, steps)
                                  : twisted(S, D, L, n, lam, live, ck, steps);
        nrqi += __popcll(__ballot(live));
        if (live) {
            const bool below = tw.neg >= j;       // lambda_j < lam
            if (below) { hi = fmin(hi, lam); vf |= 2; }
            else { lo = fmax(lo, lam); vf |= 1; }
            const bool fin = __builtin_isfinite(tw.nrm2) && tw.nrm2 > 0.0;
            const double resid = fin ? fabs(tw.gam) / sqrt(tw.nrm2) : __builtin_inf();
            const double rqc = fin ? tw.gam / tw.nrm2 : 0.0;
            if (force || (fin && (resid <= tol1 * gap || fabs(rqc) <= tol2 * fabs(lam)))) {
                done = true;
                r = tw.r;
                nrm2 = tw.nrm2;
                tg = tw.guarded != 0;
            } else {
                const bool sign_ok = below ? (rqc <= 0.0) : (rqc >= 0.0);
                const double cand = lam + rqc;
                if (fin && sign_ok && cand >= lo && cand <= hi && fabs(rqc) <= 0.5 * prev && it < P.max_rqi) {
                    lam = cand;
                    prev = fabs(rqc);
                } else {
                    need_fb = true;
                    // The bisection starts next to lam, which the count has
                    // just confirmed as one end.  The other end is put at four
                    // times the rejected correction (a correction that stopped
                    // shrinking still measures the distance), or, when its
                    // sign was wrong, at twice the last accepted one; it is
                    // checked by a count before the bracket can converge, and
                    // moved outward if the check fails.  Without such a scale
                    // the bracket stays as it is.
                    double w2 = __builtin_inf();
                    if (fin && sign_ok && cand >= lo && cand <= hi) w2 = 4.0 * fabs(rqc);
                    else if (fin) w2 = 2.0 * prev;
                    w2 = fmax(w2, 8.0 * kEps * fabs(lam));
                    if (below) {
                        const double e2 = lam - w2;
                        if (e2 > lo) { lo = e2; vf &= ~1; }
                    } else {
                        const double e2 = lam + w2;
                        if (e2 < hi) { hi = e2; vf &= ~2; }
                    }
                }
            }
        }
    }
    if (__ballot(act && !done) != 0ull) {
        assist_close(as);
        set_error(P, kErrNoConv);
        return;
    }
    const int64_t col = blk.col0 + (j - blk.w0);
    if (P.jobz) {
        double* zcol = P.Z + pr.zoff + (act ? col : 0) * pr.ldz + (blk.row0 - pr.row0);
        const bool fin = __builtin_isfinite(nrm2) && nrm2 > 0.0;
        if (__ballot(act && !fin) != 0ull) {
            // a zero pivot spoiled the nested norm: sum the squares directly
            const double ss = solve_vector(S, D, L, n, lam, act, r, 1.0, ck, zcol, false, tg, steps);
            if (!fin) nrm2 = ss;
        }
        const double scale = 1.0 / sqrt(nrm2);
        assist_try(P, as, node_id, n, pr.ck_stride, ck_off);
        if (as.on) solve_vector_assisted(S, P, D, L, n, lam, act, r, scale, ck, zcol, tg, as, steps);
        else solve_vector(S, D, L, n, lam, act, r, scale, ck, zcol, true, tg, steps);
        if (pr.flags & 1) {
            // several blocks: the rest of each column is zero, written column
            // by column with the wave's lanes on consecutive rows
            const int64_t r0 = blk.row0 - pr.row0;
            uint64_t am = __ballot(act);
            while (am) {
                const int c = __ffsll((unsigned long long)am) - 1;
                am &= am - 1ull;
                double* zc = P.Z + pr.zoff + __shfl(col, c) * pr.ldz;
                for (int64_t i = l; i < r0; i += kWave) zc[i] = 0.0;
                for (int64_t i = r0 + n + l; i < pr.n; i += kWave) zc[i] = 0.0;
            }
        }
    }
    if (act) P.w[pr.woff + col] = (nd.sigma + lam) * pr.tscale_inv;
    assist_close(as);
    add_stat(&P.ctl->n_rqi, nrqi);
    add_stat(&P.ctl->n_fallback, nfb);
}

}  // namespace mrrr

// ---------------------------------------------------------------- kernels

using namespace mrrr;

// The persistent worker: one wavefront per workgroup, looping over the task
// queues until no task is pending (or an error / the watchdog stops it).
extern "C" __global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 1))) void mrrr_tree_kernel(Params P) {
    __shared__ Shared S;
    const int l = lane_id();
    const uint64_t t0 = wall_clock64();
    int64_t steps = 0, ntask = 0, nsingle = 0;
    if (l == 0) {
        S.redo = 0;
        S.redo_sturm = 0;
        S.redo_fac = 0;
    }
    for (;;) {
        if (l == 0) {
            int status = 0, got = 0;
            int nap = 1;
            for (;;) {
                if (__hip_atomic_load(&P.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { status = 2; break; }
                for (int qq = 0; qq < kNumQ && got == 0; ++qq) got = try_pop(P, qq, S.task);
                if (got > 0) { status = 1; break; }
                if (__hip_atomic_load(&P.ctl->pending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) { status = 2; break; }
                if (wall_clock64() - t0 > P.timeout_ticks) {
                    int32_t expect = 0;
                    __hip_atomic_compare_exchange_strong(&P.ctl->error, &expect, (int32_t)kErrTimeout,
                                                         __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    status = 2;
                    break;
                }
                // back off while the queues are empty (up to ~4 us between polls)
                for (int z = 0; z < nap; ++z) __builtin_amdgcn_s_sleep(127);
                if (nap < 8) nap *= 2;
            }
            S.ibc[0] = status;
            S.ibc[1] = got;
        }
        __syncthreads();
        const int status = S.ibc[0];
        const int ngot = S.ibc[1];
        __syncthreads();
        // tasks claimed before an error still count as finished below
        for (int bi = 0; bi < ngot; ++bi) {
            const Task tk = S.task[bi];
            const uint64_t ts = wall_clock64();
            if (l == 0) {
                S.info_i[0] = 0; S.info_i[1] = 0; S.info_i[2] = -1; S.info_i[3] = 0;
                S.info_d[0] = 0.0; S.info_d[1] = 0.0;
            }
            __syncthreads();
            if (status == 1) {
                switch (tk.type) {
                    case kTaskRoot: task_root(S, P, tk.node, steps); break;
                    case kTaskRefine: task_refine(S, P, tk.node, tk.a, tk.b, steps); break;
                    case kTaskCluster: task_cluster(S, P, tk.node, tk.a, tk.b, steps); break;
                    case kTaskSingle: task_single(S, P, tk.node, tk.a, tk.b, steps); ++nsingle; break;
                    case kTaskHelp:
                        task_help(S, P, (int64_t)((uint64_t)(uint32_t)tk.a | ((uint64_t)(uint32_t)tk.b << 32)), steps);
                        break;
                    case kTaskAssist:
                        task_assist(S, P, (int64_t)((uint64_t)(uint32_t)tk.a | ((uint64_t)(uint32_t)tk.b << 32)),
                                    steps);
                        break;
                    default: set_error(P, kErrInternal); break;
                }
            }
            __syncthreads();
            if (P.trace && l == 0 && status == 1) {
                const int64_t k = __hip_atomic_fetch_add(&P.ctl->trace_top, (int64_t)1, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                if (k < P.trace_cap) {
                    TraceRec r;
                    r.type = tk.type;
                    r.worker = (int32_t)blockIdx.x;
                    r.node = tk.node;
                    r.depth = S.info_i[0];
                    r.a = tk.a;
                    r.b = tk.b;
                    r.t0 = (int64_t)ts;
                    r.t1 = (int64_t)wall_clock64();
                    r.x0 = S.info_d[0];
                    r.x1 = S.info_d[1];
                    r.flags = S.info_i[1];
                    r.child = S.info_i[2];
                    P.trace[k] = r;
                }
            }
            ++ntask;
        }
        // pending only detects the end of the work (a task's results reach
        // other workers through the pushes and node counters above)
        if (l == 0 && ngot > 0)
            __hip_atomic_fetch_add(&P.ctl->pending, (int64_t)-ngot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (status != 1) break;
    }
    add_stat(&P.ctl->qd_steps, steps);
    add_stat(&P.ctl->n_tasks, ntask);
    add_stat(&P.ctl->n_single, nsingle);
    add_stat(&P.ctl->n_nan, (int64_t)S.redo);
    add_stat(&P.ctl->n_sturm, (int64_t)S.redo_sturm);
    add_stat(&P.ctl->n_fac_quot, (int64_t)S.redo_fac);
}

// Resets the control block and the queue cells (no memset nodes, so that the
// sequence can be captured in a graph).
extern "C" __global__ void mrrr_init_kernel(Params P) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    if (tid == 0) {
        Ctl c;
        uint64_t* raw = (uint64_t*)&c;
        for (size_t k = 0; k < sizeof(Ctl) / 8; ++k) raw[k] = 0;
        *P.ctl = c;
    }
    for (int qq = 0; qq < kNumQ; ++qq)
        for (int64_t i = tid; i < (int64_t)P.qcap[qq]; i += nth) P.seq[qq][i] = (uint64_t)i;
}

// Per problem: splitting into irreducible blocks (Sec. 3.2.1), index ranges
// per block, trivial 1x1 blocks, and one root task per remaining block.
extern "C" __global__ __launch_bounds__(64) void mrrr_setup_kernel(Params P) {
    __shared__ Shared S;
    const int l = lane_id();
    const int p = blockIdx.x;
    Problem* pr = P.probs + p;
    const int64_t n = pr->n;
    if (n <= 0) {
        if (l == 0) { pr->m = 0; pr->nblocks = 0; }
        return;
    }
    const double* d = P.d + pr->row0;
    const double* e = P.e + pr->row0;
    // Gershgorin interval and the finiteness test in one sweep, four rows
    // per lane in flight (min and max do not depend on the order)
    constexpr int U = 4;
    double gl = __builtin_inf(), gu = -__builtin_inf();
    int bad_d = 0, bad_e = 0;
    for (int64_t i0 = l; i0 < n; i0 += (int64_t)kWave * U) {
        double dv[U], ev[U], em[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + (int64_t)u * kWave;
            dv[u] = (i < n) ? d[i] : 0.0;
            ev[u] = (i < n - 1) ? e[i] : 0.0;
            em[u] = (i > 0 && i < n) ? e[i - 1] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + (int64_t)u * kWave;
            if (i < n) {
                const double r = fabs(em[u]) + fabs(ev[u]);
                gl = fmin(gl, dv[u] - r);
                gu = fmax(gu, dv[u] + r);
                bad_d |= __builtin_isfinite(dv[u]) ? 0 : 1;
                if (i < n - 1) bad_e |= __builtin_isfinite(ev[u]) ? 0 : 1;
            }
        }
    }
    gl = wave_min(gl);
    gu = wave_max(gu);
    if (wave_or(bad_d) || wave_or(bad_e)) {
        if (l == 0) { pr->m = 0; pr->nblocks = 0; }
        set_error(P, wave_or(bad_d) ? kErrBadD : kErrBadE);
        return;
    }
    const double bnorm = fmax(fabs(gl), fabs(gu));
    // splitting (Sec. 3.2.1): |beta_i| <= eps sqrt(n) ||T||, with eps the
    // unit roundoff of the caller's data format (Sec. 5.1.1 for single/double)
    const double tol = (P.io_eps > 0.0 ? P.io_eps : kEps) * sqrt((double)n) * bnorm;
    // The tree works on 2^-k T with the Gershgorin bound in [1/2, 1): a
    // power of two changes no rounding, keeps squares of the entries and the
    // products of the division-free Sturm counts away from overflow and
    // underflow, and is undone exactly on the eigenvalues.
    const int kexp = (bnorm > 0.0 && __builtin_isfinite(bnorm)) ? __builtin_amdgcn_frexp_exp(bnorm) : 0;
    const double tsc = __builtin_ldexp(1.0, -kexp);
    Block* B = P.blocks + pr->row0;
    int nb = 0;
    int64_t start = 0;
    // split points in increasing order, four 64-row chunks loaded at once
    for (int64_t base0 = 0; base0 < n - 1; base0 += (int64_t)kWave * U) {
        double ev[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = base0 + (int64_t)u * kWave + l;
            ev[u] = (i < n - 1) ? e[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t base = base0 + (int64_t)u * kWave;
            const int64_t i = base + l;
            const bool sp = (i < n - 1) && fabs(ev[u]) <= tol;
            uint64_t mk = __ballot(sp);
            while (mk) {
                const int t = __ffsll((unsigned long long)mk) - 1;
                mk &= mk - 1ull;
                const int64_t is = base + t;
                if (l == 0) {
                    B[nb].prob = p;
                    B[nb].root = -1;
                    B[nb].row0 = pr->row0 + start;
                    B[nb].n = is - start + 1;
                }
                ++nb;
                start = is + 1;
            }
        }
    }
    if (l == 0) {
        B[nb].prob = p;
        B[nb].root = -1;
        B[nb].row0 = pr->row0 + start;
        B[nb].n = n - start;
    }
    ++nb;
    __threadfence_block();
    __syncthreads();
    // index ranges per block
    int64_t m = 0;
    int err = 0;
    // An index range over several blocks (Sec. 3.2.1): the il-th and iu-th
    // eigenvalues of the direct sum are bracketed to full accuracy by
    // multisection on the Sturm count of T with the split entries zero (the
    // sum of the blocks' counts; lanes 0-31 for il, 32-63 for iu).  A block
    // then keeps its eigenvalues above the il bracket and below the iu
    // bracket; of the ones inside a bracket (equal to working accuracy) the
    // lower blocks' come first, as in a stable merge by value.
    const bool split_index = (pr->range == 2 && nb > 1);
    double ta[2] = {0.0, 0.0}, tb[2] = {0.0, 0.0};   // brackets [a, b) of the two targets (scaled)
    int64_t na[2] = {0, 0};                           // N(a) of each target
    int64_t quota[2] = {0, 0};
    if (split_index) {
        const double slack = (2.0 * (double)n + 10.0) * bnorm * kEps;
        const int t = l >> 5, j = l & 31;
        const int64_t kt = t ? pr->iu : pr->il;
        double a = (gl - slack) * tsc, bb = (gu + slack) * tsc;
        int64_t ca = 0;
        for (int pass = 0; pass < 2200; ++pass) {
            const double wid = bb - a;
            const bool done = !(wid > 2.0 * kEps * fmax(fabs(a), fabs(bb))) || !(a + 0.5 * wid > a && a + 0.5 * wid < bb);
            if (__ballot(!done) == 0ull) break;
            const double x = done ? a : a + wid * ((double)(j + 1) / 33.0);
            int64_t c = 0;
            for (int q = 0; q < nb; ++q) c += negcount_T(S, P.d + B[q].row0, P.e + B[q].row0, B[q].n, tsc, x);
            // new bracket of this half: the highest point with N < k, the
            // lowest with N >= k (points increase with the lane)
            const bool below = !done && c < kt && x > a;
            const bool above = !done && c >= kt && x < bb;
            double na_x = below ? x : -__builtin_inf();
            int64_t na_c = below ? c : -1;
            double nb_x = above ? x : __builtin_inf();
            int64_t nb_c = above ? c : INT64_MAX;
            for (int o = 16; o > 0; o >>= 1) {
                const double ox = __shfl_xor(na_x, o);
                const int64_t oc = __shfl_xor(na_c, o);
                if (ox > na_x) { na_x = ox; na_c = oc; }
                const double px = __shfl_xor(nb_x, o);
                const int64_t pc = __shfl_xor(nb_c, o);
                if (px < nb_x) { nb_x = px; nb_c = pc; }
            }
            if (na_c >= 0) { a = na_x; ca = na_c; }
            if (nb_c != INT64_MAX) bb = nb_x;
        }
        for (int u = 0; u < 2; ++u) {
            ta[u] = __shfl(a, 32 * u);
            tb[u] = __shfl(bb, 32 * u);
            na[u] = __shfl(ca, 32 * u);
        }
        quota[0] = pr->il - 1 - na[0];   // of the il bracket's eigenvalues, these lie below il
        quota[1] = pr->iu - na[1];       // of the iu bracket's eigenvalues, these lie up to iu
    }
    for (int b = 0; b < nb && !err; ++b) {
        const int64_t nbk = B[b].n;
        int64_t w0, w1;
        if (pr->range == 0) {
            w0 = 1;
            w1 = nbk;
        } else if (pr->range == 1) {
            const double sig = ((l == 0) ? pr->vl : pr->vu) * tsc;
            const int c = negcount_T(S, P.d + B[b].row0, P.e + B[b].row0, nbk, tsc, sig);
            w0 = (int64_t)__shfl(c, 0) + 1;
            w1 = (int64_t)__shfl(c, 1);
        } else if (split_index) {
            const double sig = (l == 0) ? ta[0] : (l == 1) ? tb[0] : (l == 2) ? ta[1] : tb[1];
            const int c = negcount_T(S, P.d + B[b].row0, P.e + B[b].row0, nbk, tsc, sig);
            const int64_t c0 = __shfl(c, 0), c1 = __shfl(c, 1), c2 = __shfl(c, 2), c3 = __shfl(c, 3);
            const int64_t x = max((int64_t)0, min(c1 - c0, quota[0]));
            const int64_t y = max((int64_t)0, min(c3 - c2, quota[1]));
            quota[0] -= x;
            quota[1] -= y;
            w0 = min(c0 + x + 1, nbk + 1);
            w1 = min(c2 + y, nbk);
        } else {
            w0 = pr->il;
            w1 = pr->iu;
        }
        if (l == 0) {
            B[b].w0 = w0;
            B[b].w1 = w1;
            B[b].k0 = w0 > 1 ? w0 - 1 : 1;
            B[b].k1 = w1 < nbk ? w1 + 1 : nbk;
            B[b].col0 = (pr->range == 0) ? (B[b].row0 - pr->row0) : m;
        }
        if (w1 >= w0) m += w1 - w0 + 1;
    }
    if (split_index && !err && m != pr->iu - pr->il + 1) err = kErrInternal;
    __threadfence_block();
    __syncthreads();
    if (l == 0) {
        pr->m = err ? 0 : m;
        pr->nblocks = nb;
        pr->bnorm = bnorm;
        pr->tscale = tsc;
        pr->tscale_inv = __builtin_ldexp(1.0, kexp);
        pr->flags = (nb > 1) ? 1 : 0;
        __hip_atomic_fetch_add(&P.ctl->n_blocks, (int64_t)nb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (err) {
        set_error(P, err);
        return;
    }
    for (int b = 0; b < nb; ++b) {
        const Block bk = B[b];
        if (bk.w1 < bk.w0) continue;
        if (bk.n == 1) {
            // a 1x1 block: its eigenpair is (d_i, e_i)
            if (l == 0) P.w[pr->woff + bk.col0] = P.d[bk.row0];
            if (P.jobz) {
                double* zc = P.Z + pr->zoff + bk.col0 * pr->ldz;
                for (int64_t i = l; i < n; i += kWave) zc[i] = (i == bk.row0 - pr->row0) ? 1.0 : 0.0;
            }
            continue;
        }
        Task t;
        t.type = kTaskRoot;
        t.node = (int)(pr->row0 + b);
        t.a = 0;
        t.b = 0;
        push_one(P, kQCluster, t);
    }
}

// After the tree: eigenvalues of several blocks, or values of one tight
// cluster computed from different representations, may come out of
// ascending order.  mrrr_sort_kernel (one workgroup per problem) leaves a
// sorted problem alone; otherwise it sorts (w, column) pairs by a bitonic
// network in scratch (keys at colbuf + 2 row0, columns at perm + 2 row0,
// padded to a power of two <= 2 n), writes the sorted w, and marks the
// problem (flags bit 1) for mrrr_permute_kernel, which moves Z's columns.
extern "C" __global__ __launch_bounds__(1024) void mrrr_sort_kernel(Params P) {
    __shared__ int unsorted;
    Problem* prp = P.probs + blockIdx.x;
    const int64_t m = prp->m;
    const int tid = threadIdx.x, nt = blockDim.x;
    // a solve that failed (and will be retried or reported) has no output
    if (m < 2 || __hip_atomic_load(&P.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    double* w = P.w + prp->woff;
    if (tid == 0) unsorted = 0;
    __syncthreads();
    int u = 0;
    for (int64_t i = tid; i + 1 < m; i += nt) u |= (w[i] > w[i + 1]) ? 1 : 0;
    if (u) atomicOr(&unsorted, 1);
    __syncthreads();
    if (!unsorted) return;
    int64_t p2 = 1;
    while (p2 < m) p2 <<= 1;
    double* key = P.colbuf + 2 * prp->row0;
    int32_t* col = P.perm + 2 * prp->row0;
    for (int64_t i = tid; i < p2; i += nt) {
        key[i] = (i < m) ? w[i] : __builtin_inf();
        col[i] = (i < m) ? (int32_t)i : INT32_MAX;
    }
    __syncthreads();
    for (int64_t k = 2; k <= p2; k <<= 1) {
        for (int64_t j = k >> 1; j > 0; j >>= 1) {
            for (int64_t i = tid; i < p2; i += nt) {
                const int64_t x = i ^ j;
                if (x <= i) continue;
                const double ki = key[i], kx = key[x];
                const int32_t ci = col[i], cx = col[x];
                const bool gt = (ki > kx) || (ki == kx && ci > cx);   // (key, column) order
                const bool up = (i & k) == 0;
                if (up ? gt : !gt) {
                    key[i] = kx; key[x] = ki;
                    col[i] = cx; col[x] = ci;
                }
            }
            __syncthreads();
        }
    }
    for (int64_t i = tid; i < m; i += nt) w[i] = key[i];
    if (tid == 0) prp->flags |= 2;
}

// Cycle leaders of a marked problem's permutation by pointer jumping: after
// round 0 (lead = p, jump = col[p]) each round sets lead = min(lead,
// lead[jump]) and jump = jump[jump], so after ceil(log2 m) rounds lead[p] is
// the smallest index on p's cycle -- O(m log m) work whatever the cycle
// lengths (the columns of split blocks interleave into long cycles).  Two
// buffers of (lead, jump) alternate in the colbuf scratch, which the sort's
// keys no longer need: int32 at colbuf + 16 row0 bytes, 4 m entries.
DEV int32_t* cycle_buf(const Params& P, const Problem& pr, int which) {   // which: 0 = A, 1 = B
    return reinterpret_cast<int32_t*>(P.colbuf) + 4 * pr.row0 + 2 * pr.m * which;
}

extern "C" __global__ __launch_bounds__(256) void mrrr_cycle_kernel(Params P, int round) {
    const Problem pr = P.probs[blockIdx.y];
    if (!(pr.flags & 2) || !P.jobz) return;
    const int64_t m = pr.m;
    const int32_t* col = P.perm + 2 * pr.row0;
    int32_t* src = cycle_buf(P, pr, (round & 1) ? 0 : 1);   // round r reads the buffer round r-1 wrote
    int32_t* dst = cycle_buf(P, pr, (round & 1) ? 1 : 0);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x) {
        if (round == 0) {
            dst[p] = (int32_t)p;
            dst[m + p] = col[p];
        } else {
            const int32_t jp = src[m + p];
            const int32_t a = src[p], b = src[jp];
            dst[p] = a < b ? a : b;
            dst[m + p] = src[m + jp];
        }
    }
}

// Position i of a marked problem receives column col[i].  The permutation is
// applied in place cycle by cycle: for the cycle whose smallest index (its
// leader, from mrrr_cycle_kernel) is p, the rows of each 64-row chunk move
// along the cycle independently of the other chunks, so a wave takes one
// (leader, chunk) item at a time and a long cycle is spread over as many
// waves as it has chunks (columns of split blocks with equal spectra
// interleave into cycles of thousands).
extern "C" __global__ __launch_bounds__(64) void mrrr_permute_kernel(Params P, int rounds) {   // rounds: index of the last round
    const int l = lane_id();
    const Problem pr = P.probs[blockIdx.y];
    if (!(pr.flags & 2) || !P.jobz) return;
    const int64_t m = pr.m, n = pr.n, ldz = pr.ldz;
    const int64_t nch = (n + kWave - 1) / kWave;
    const int32_t* col = P.perm + 2 * pr.row0;
    const int32_t* lead = cycle_buf(P, pr, (rounds & 1) ? 1 : 0);   // written by round `rounds`
    double* Z = P.Z + pr.zoff;
    for (int64_t it = blockIdx.x; it < m * nch; it += gridDim.x) {
        const int64_t p = it / nch;
        if (col[p] == p || lead[p] != p) continue;
        const int64_t r = (it - p * nch) * kWave + l;
        const bool in = r < n;
        const double keep = in ? Z[p * ldz + r] : 0.0;
        int64_t pp = p;
        for (int64_t guard = 0; guard <= m; ++guard) {
            const int64_t sidx = col[pp];
            if (sidx == p) {
                if (in) Z[pp * ldz + r] = keep;
                break;
            }
            if (in) Z[pp * ldz + r] = Z[sidx * ldz + r];
            pp = sidx;
        }
    }
}

// Sign convention: the entry of largest magnitude of each column positive
// (ties to the lowest row).  One wavefront per column.
extern "C" __global__ __launch_bounds__(64) void mrrr_sign_kernel(Params P, int64_t ncols_total) {
    const int l = lane_id();
    if (__hip_atomic_load(&P.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    for (int64_t g = blockIdx.x; g < ncols_total; g += gridDim.x) {
        // column g is slot-ordered: find its problem
        int a = 0, b = P.nprob - 1;
        while (a < b) {
            const int mid = (a + b + 1) >> 1;
            if (P.probs[mid].row0 <= g) a = mid; else b = mid - 1;
        }
        const Problem& pr = P.probs[a];
        const int64_t col = g - pr.row0;
        if (col >= pr.m) continue;
        double* z = P.Z + pr.zoff + col * pr.ldz;
        // each lane visits its rows l, l + 64, ... in increasing order (so a
        // later equal entry never wins), eight loads in flight
        constexpr int U = 8;
        double best = -1.0;
        int64_t bi = 0;
        for (int64_t i0 = l; i0 < pr.n; i0 += (int64_t)kWave * U) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = i0 + (int64_t)u * kWave;
                v[u] = (i < pr.n) ? fabs(z[i]) : -1.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (v[u] > best) { best = v[u]; bi = i0 + (int64_t)u * kWave; }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(best, o);
            const int64_t oi = __shfl_xor(bi, o);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        const bool neg = z[bi] < 0.0;
        if (neg) {
            for (int64_t i0 = l; i0 < pr.n; i0 += (int64_t)kWave * U) {
                double v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t i = i0 + (int64_t)u * kWave;
                    v[u] = (i < pr.n) ? z[i] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t i = i0 + (int64_t)u * kWave;
                    if (i < pr.n) z[i] = -v[u];
                }
            }
        }
    }
}

// The reciprocal-based quotient (quot) element by element, for checking it
// against IEEE division on the device that runs the kernels.
extern "C" __global__ void mrrr_quot_kernel(const double* a, const double* b, double* q, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) q[i] = quot(recip(b[i]), a[i]);
}

// Single/double form (Sec. 5.1.1): the caller's FP32 data in, FP64 inside,
// FP32 results out.  Widening is exact; narrowing rounds to nearest.
extern "C" __global__ void mrrr_widen_kernel(const float* __restrict__ x, double* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (double)x[i];
}

// dst(i, j) = src(i, j) for i < rows, j < cols; one 256-thread block covers
// 256 consecutive rows of one column (blockIdx.y), so reads and writes are
// contiguous along the column.
extern "C" __global__ void mrrr_narrow_kernel(const double* __restrict__ src, int64_t lds, float* __restrict__ dst,
                                              int64_t ldd, int64_t rows, int64_t cols) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t j = blockIdx.y; j < cols; j += gridDim.y)
        if (i < rows) dst[j * ldd + i] = (float)src[j * lds + i];
}

// ------------------------------------------------------------ launchers

namespace mrrr {

hipError_t launch_quot(const double* a, const double* b, double* q, int64_t n, hipStream_t s) {
    const int64_t grid = (n + 255) / 256;
    if (grid > 0) hipLaunchKernelGGL(mrrr_quot_kernel, dim3((unsigned)grid), dim3(256), 0, s, a, b, q, n);
    return hipGetLastError();
}

hipError_t launch_widen(const float* x, double* y, int64_t n, hipStream_t s) {
    const int64_t grid = (n + 255) / 256;
    if (grid > 0) hipLaunchKernelGGL(mrrr_widen_kernel, dim3((unsigned)grid), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

hipError_t launch_narrow(const double* src, int64_t lds, float* dst, int64_t ldd, int64_t rows, int64_t cols,
                         hipStream_t s) {
    const int64_t gx = (rows + 255) / 256;
    const int64_t gy = cols < 65535 ? cols : 65535;
    if (gx > 0 && gy > 0)
        hipLaunchKernelGGL(mrrr_narrow_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, src, lds, dst, ldd,
                           rows, cols);
    return hipGetLastError();
}

hipError_t launch_init(const Params& P, hipStream_t s) {
    uint64_t mx = 1;
    for (int q = 0; q < kNumQ; ++q) mx = P.qcap[q] > mx ? P.qcap[q] : mx;
    int grid = (int)((mx + 255) / 256);
    if (grid > 4096) grid = 4096;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(mrrr_init_kernel, dim3(grid), dim3(256), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_setup(const Params& P, hipStream_t s) {
    hipLaunchKernelGGL(mrrr_setup_kernel, dim3(P.nprob), dim3(kWave), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_tree(const Params& P, hipStream_t s) {
    hipLaunchKernelGGL(mrrr_tree_kernel, dim3(P.nworkers), dim3(kWave), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_finalize(const Params& P, hipStream_t s) {
    hipLaunchKernelGGL(mrrr_sort_kernel, dim3(P.nprob), dim3(1024), 0, s, P);
    // rounds of pointer jumping: enough for the longest possible cycle
    int rounds = 1;
    while ((int64_t)1 << (rounds - 1) < std::max<int64_t>(P.total_rows, 2)) ++rounds;
    const unsigned gc = (unsigned)std::max(1, std::min(256, 65536 / std::max(1, (int)P.nprob)));
    for (int r = 0; r < rounds; ++r) hipLaunchKernelGGL(mrrr_cycle_kernel, dim3(gc, P.nprob), dim3(256), 0, s, P, r);
    const unsigned gx = (unsigned)std::max(1, std::min(8192, 262144 / std::max(1, (int)P.nprob)));
    hipLaunchKernelGGL(mrrr_permute_kernel, dim3(gx, P.nprob), dim3(kWave), 0, s, P, rounds - 1);
    return hipGetLastError();
}

hipError_t launch_sign(const Params& P, int64_t ncols_total, hipStream_t s) {
    int64_t g = ncols_total < 65536 ? ncols_total : 65536;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(mrrr_sign_kernel, dim3((unsigned)g), dim3(kWave), 0, s, P, ncols_total);
    return hipGetLastError();
}

hipError_t tree_occupancy(int* blocks_per_cu) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, mrrr_tree_kernel, kWave, 0);
}

}  // namespace mrrr
