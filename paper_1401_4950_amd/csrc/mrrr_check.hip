// Orthogonality check of the clusters whose representation passed no
// element-growth test, and their repair.
//
// When no candidate shift of a cluster yields a representation with small
// element growth, the candidate with the least growth is kept (Alg. 3.8, last
// resort), and nothing then guarantees the relative robustness that the
// orthogonality of the cluster's eigenvectors rests on.  Remark (6) on the
// shift selection of Sec. 3.2.3 suggests checking the accuracy of such a
// cluster's eigenpairs explicitly.  The tree records each such cluster of at
// most kCheckMax wanted columns (the outermost one of a subtree); after the
// tree, one workgroup per record forms the Gram matrix G = Z_c^T Z_c of those
// columns (mrrr_check_small_kernel: up to kSmallM columns by plain FMAs;
// mrrr_check_wide_kernel: wider clusters on the matrix cores); where
// max |G - I| exceeds check_tol n eps (an option, 20 by default),
// mrrr_repair_kernel replaces Z_c by the first-order symmetric (Loewdin)
// orthogonalisation Z_c (I - E / 2), E = G - I, twice: the columns move as
// little as possible, and after the second pass the loss is of the order of
// |E|^4.
//
// Gram blocks run on the FP64 matrix cores (v_mfma_f64_16x16x4f64; lane
// layout: A(i, k) from lane i + 16 k, B(k, j) from lane j + 16 k, result
// register r of lane l holds C(4 r + l / 16, l % 16)).  With A = Z_gi^T and
// B = Z_gj both operands of lane (c, k) are column c of their group at one
// row.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mrrr_internal.h"

namespace mrrr {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kGroups = kCheckMax / 16;                   // 16-column groups
constexpr int kPairs = kGroups * (kGroups + 1) / 2;       // Gram blocks gi <= gj
constexpr double kEpsC = 1.1102230246251565e-16;          // 2^-53
constexpr double kRepairMax = 1e-3;   // m max |G - I| above this: not repaired
constexpr int kEStride = kCheckMax + 1;

__device__ __forceinline__ void stat_add(int64_t* p, int64_t v) {
    if (v) __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// |G_ij - delta_ij|, with a NaN counted as infinite
__device__ __forceinline__ double loss_term(double g, bool diag) {
    const double a = fabs(g - (diag ? 1.0 : 0.0));
    return (a <= 1e300) ? a : __builtin_inf();
}

__device__ __forceinline__ double check_threshold(const Params& P, int64_t n) {
    return P.check_tol * (double)n * kEpsC;
}

// Gram blocks (gi, gj), gi <= gj < TT, of the m columns at Z (stride ldz)
// over rows [b, e) by one wavefront, 4 U rows per step: lane (c, k) loads
// rows base + 4 u + k of column c of every group, so that the 4 lanes of a
// column read 32 contiguous bytes and a step uses every line it touches.
template <int TT>
__device__ void gram_blocks(const double* __restrict__ Z, int64_t ldz, int64_t b, int64_t e, int m,
                            dbl4 (&acc)[kPairs]) {
    constexpr int U = TT == 1 ? 16 : (TT == 2 ? 8 : 4);
    const int lane = threadIdx.x & 63;
    const int c = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int p = 0; p < kPairs; ++p) acc[p] = dbl4{0.0, 0.0, 0.0, 0.0};
    for (int64_t base = b; base < e; base += 4 * U) {
        double v[U][TT];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int g = 0; g < TT; ++g) {
                const int col = g * 16 + c;
                const int64_t i = base + 4 * u + kq;
                v[u][g] = (col < m && i < e) ? Z[(int64_t)col * ldz + i] : 0.0;
            }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int p = 0;
#pragma unroll
            for (int gi = 0; gi < kGroups; ++gi)
#pragma unroll
                for (int gj = gi; gj < kGroups; ++gj, ++p)
                    if (gj < TT)
                        acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[u][gi], v[u][gj], acc[p], 0, 0, 0);
        }
    }
}

__device__ void gram(const double* Z, int64_t ldz, int64_t b, int64_t e, int m, dbl4 (&acc)[kPairs]) {
    switch ((m + 15) >> 4) {
        case 1: gram_blocks<1>(Z, ldz, b, e, m, acc); break;
        case 2: gram_blocks<2>(Z, ldz, b, e, m, acc); break;
        case 3: gram_blocks<3>(Z, ldz, b, e, m, acc); break;
        default: gram_blocks<4>(Z, ldz, b, e, m, acc); break;
    }
}

// Calls f(i, j, g) for the upper triangle i <= j < m of G = sum of the
// blocks, each entry once over the wavefront.
template <class F>
__device__ __forceinline__ void for_upper(const dbl4 (&acc)[kPairs], int m, F f) {
    const int lane = threadIdx.x & 63;
    int p = 0;
#pragma unroll
    for (int gi = 0; gi < kGroups; ++gi)
#pragma unroll
        for (int gj = gi; gj < kGroups; ++gj, ++p)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = gi * 16 + 4 * r + (lane >> 4), j = gj * 16 + (lane & 15);
                if (i < m && j < m && i <= j) f(i, j, acc[p][r]);
            }
}

// max |G - I| over the wavefront (a NaN counts as infinite)
__device__ double gram_loss(const dbl4 (&acc)[kPairs], int m) {
    double lm = 0.0;
    for_upper(acc, m, [&](int i, int j, double g) { lm = fmax(lm, loss_term(g, i == j)); });
    for (int o = 32; o > 0; o >>= 1) lm = fmax(lm, __shfl_xor(lm, o));
    return lm;
}

constexpr int kChkThreads = 256;                          // 4 waves per record
constexpr int kSmallM = 8;
constexpr int kRedWords = 2 * kPairs * 4 * 64;            // two waves' blocks

// max |G - I| of M <= kSmallM columns by plain FMAs: thread t takes rows
// t, t + 256, ... (coalesced), the M (M + 1) / 2 sums stay in registers,
// are reduced by a fixed butterfly per wave and then over the waves in order.
template <int M>
__device__ double small_loss(const double* __restrict__ Z, int64_t ldz, int64_t n, double* red) {
    constexpr int U = M <= 3 ? 8 : (M <= 5 ? 4 : 2);   // rows in flight per thread
    constexpr int K = M * (M + 1) / 2;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    for (int64_t r0 = tid; r0 < n; r0 += kChkThreads * U) {
        double x[U][M];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < M; ++i) {
                const int64_t r = r0 + kChkThreads * u;
                x[u][i] = (r < n) ? Z[(int64_t)i * ldz + r] : 0.0;
            }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int k = 0;
#pragma unroll
            for (int i = 0; i < M; ++i)
#pragma unroll
                for (int j = i; j < M; ++j, ++k) acc[k] = fma(x[u][i], x[u][j], acc[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double g = acc[k];
        for (int o = 32; o > 0; o >>= 1) g += __shfl_xor(g, o);
        if (lane == 0) red[wave * K + k] = g;
    }
    __syncthreads();
    // entry k = (i, j) of the upper triangle, row by row, on thread k of wave 0
    double lm = 0.0;
    if (tid < K) {
        int i = 0, kk = tid;
        while (kk >= M - i) {
            kk -= M - i;
            ++i;
        }
        const double g = ((red[tid] + red[K + tid]) + red[2 * K + tid]) + red[3 * K + tid];
        lm = loss_term(g, kk == 0);
    }
    for (int o = 32; o > 0; o >>= 1) lm = fmax(lm, __shfl_xor(lm, o));
    return lm;   // valid in wave 0
}

// max |G - I| of 8 < m <= kCheckMax columns: wave w forms the blocks over
// the w-th quarter of the rows; the four sets are summed pairwise through LDS,
// (w0 + w2) + (w1 + w3), a fixed order.
__device__ __forceinline__ void blocks_to_lds(const dbl4 (&acc)[kPairs], double* slot, int lane) {
#pragma unroll
    for (int p = 0; p < kPairs; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) slot[(p * 4 + r) * 64 + lane] = acc[p][r];
}
__device__ __forceinline__ void blocks_from_lds(dbl4 (&acc)[kPairs], const double* slot, int lane) {
#pragma unroll
    for (int p = 0; p < kPairs; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[p][r] += slot[(p * 4 + r) * 64 + lane];
}
// The blocks of all n rows by the four waves of a workgroup; the sums end in
// wave 0's acc.
__device__ void gram4(const double* Z, int64_t ldz, int64_t n, int m, double* red, dbl4 (&acc)[kPairs]) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t q = (n + 3) / 4;
    const int64_t b = (int64_t)wave * q < n ? (int64_t)wave * q : n;
    const int64_t e = (b + q < n) ? b + q : n;
    gram(Z, ldz, b, e, m, acc);
    constexpr int kSlot = kPairs * 4 * 64;
    if (wave >= 2) blocks_to_lds(acc, red + (wave - 2) * kSlot, lane);
    __syncthreads();
    if (wave < 2) blocks_from_lds(acc, red + wave * kSlot, lane);
    __syncthreads();
    if (wave == 1) blocks_to_lds(acc, red, lane);
    __syncthreads();
    if (wave == 0) blocks_from_lds(acc, red, lane);
}

__device__ double wide_loss(const double* Z, int64_t ldz, int64_t n, int m, double* red) {
    dbl4 acc[kPairs];
    gram4(Z, ldz, n, m, red, acc);
    double lm = 0.0;
    if ((threadIdx.x >> 6) == 0) lm = gram_loss(acc, m);
    return lm;   // valid in wave 0
}

}  // namespace

}  // namespace mrrr

using namespace mrrr;

// The loss of orthogonality of each record's columns, and the count of
// records too far gone to be corrected: one workgroup of four waves per
// record (grid-stride).  Clusters of at most kSmallM columns and wider ones
// go to two kernels, so that the first, which needs few registers, keeps many
// records in flight.
__device__ __forceinline__ void check_done(const Params& P, int64_t rec, const CheckRec& rc, double loss) {
    if (threadIdx.x == 0) {
        P.chk[rec].loss[0] = loss;
        stat_add(&P.ctl->n_checked, 1);
        const bool failed = loss > check_threshold(P, rc.n) && !((double)rc.m * loss <= kRepairMax);
        stat_add(&P.ctl->n_check_failed, failed ? 1 : 0);
    }
}

extern "C" __global__ __launch_bounds__(kChkThreads) __attribute__((amdgpu_waves_per_eu(4)))
void mrrr_check_small_kernel(Params P) {
    __shared__ double red[4 * kSmallM * (kSmallM + 1) / 2];
    // after a failed tree (the host retries or reports it) Z is incomplete
    int64_t nrec = (P.ctl->error == kErrNone) ? P.ctl->chk_top : 0;
    if (nrec > P.chk_cap) nrec = P.chk_cap;
    for (int64_t rec = blockIdx.x; rec < nrec; rec += gridDim.x) {
        const CheckRec rc = P.chk[rec];
        const int m = (int)rc.m;
        if (m > kSmallM) continue;
        const double* Z = P.Z + rc.z;
        double loss;
        __syncthreads();   // the previous record's partial sums are read
        switch (m) {
            case 2: loss = small_loss<2>(Z, rc.ldz, rc.n, red); break;
            case 3: loss = small_loss<3>(Z, rc.ldz, rc.n, red); break;
            case 4: loss = small_loss<4>(Z, rc.ldz, rc.n, red); break;
            case 5: loss = small_loss<5>(Z, rc.ldz, rc.n, red); break;
            case 6: loss = small_loss<6>(Z, rc.ldz, rc.n, red); break;
            case 7: loss = small_loss<7>(Z, rc.ldz, rc.n, red); break;
            default: loss = small_loss<8>(Z, rc.ldz, rc.n, red); break;
        }
        check_done(P, rec, rc, loss);
    }
}

extern "C" __global__ __launch_bounds__(kChkThreads) __attribute__((amdgpu_waves_per_eu(2)))
void mrrr_check_wide_kernel(Params P) {
    __shared__ double red[kRedWords];
    // after a failed tree (the host retries or reports it) Z is incomplete
    int64_t nrec = (P.ctl->error == kErrNone) ? P.ctl->chk_top : 0;
    if (nrec > P.chk_cap) nrec = P.chk_cap;
    for (int64_t rec = blockIdx.x; rec < nrec; rec += gridDim.x) {
        const CheckRec rc = P.chk[rec];
        const int m = (int)rc.m;
        if (m <= kSmallM) continue;
        __syncthreads();   // the previous record's partial sums are read
        const double loss = wide_loss(P.Z + rc.z, rc.ldz, rc.n, m, red);
        check_done(P, rec, rc, loss);
    }
}

constexpr int kRepThreads = 256;

// Z_c <- Z_c (I - E / 2) for m <= KM columns, one row per thread: the row
// is copied into registers first; x_j is read again from memory (a register
// array cannot be indexed by j), one column ahead of its use, and so is
// column j + 1 of E (for KM <= 32, where the registers allow it).
template <int KM>
__device__ void apply_rows(double* __restrict__ Z, int64_t ldz, int64_t n, int m, const double* E) {
    for (int64_t row = threadIdx.x; row < n; row += kRepThreads) {
        double x[KM];
#pragma unroll
        for (int i = 0; i < KM; ++i) x[i] = (i < m) ? Z[(int64_t)i * ldz + row] : 0.0;
        double xn = Z[row];
        if constexpr (KM <= 32) {
            double ec[KM];
#pragma unroll
            for (int i = 0; i < KM; ++i) ec[i] = E[i * kEStride];
            for (int j = 0; j < m; ++j) {
                const double xj = xn;
                const int jn = (j + 1 < m) ? j + 1 : j;
                xn = Z[(int64_t)jn * ldz + row];
                double en[KM];
#pragma unroll
                for (int i = 0; i < KM; ++i) en[i] = E[i * kEStride + jn];
                double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
                for (int i = 0; i < KM; i += 4) {
                    s0 = fma(ec[i + 0], x[i + 0], s0);
                    s1 = fma(ec[i + 1], x[i + 1], s1);
                    s2 = fma(ec[i + 2], x[i + 2], s2);
                    s3 = fma(ec[i + 3], x[i + 3], s3);
                }
                Z[(int64_t)j * ldz + row] = fma(-0.5, (s0 + s1) + (s2 + s3), xj);
#pragma unroll
                for (int i = 0; i < KM; ++i) ec[i] = en[i];
            }
        } else {
            for (int j = 0; j < m; ++j) {
                const double xj = xn;
                if (j + 1 < m) xn = Z[(int64_t)(j + 1) * ldz + row];
                double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
                for (int i = 0; i < KM; i += 4) {
                    s0 = fma(E[(i + 0) * kEStride + j], x[i + 0], s0);
                    s1 = fma(E[(i + 1) * kEStride + j], x[i + 1], s1);
                    s2 = fma(E[(i + 2) * kEStride + j], x[i + 2], s2);
                    s3 = fma(E[(i + 3) * kEStride + j], x[i + 3], s3);
                }
                Z[(int64_t)j * ldz + row] = fma(-0.5, (s0 + s1) + (s2 + s3), xj);
            }
        }
    }
}

// One workgroup per record whose loss exceeds the tolerance (and is small
// enough to correct): Z_c <- Z_c (I - E / 2) twice, the second time with the
// E of the corrected columns.  The four waves form the Gram blocks, wave 0
// stages E in LDS; every thread then owns rows of Z_c and rewrites them from
// a copy in registers.
extern "C" __global__ __launch_bounds__(kRepThreads) void mrrr_repair_kernel(Params P) {
    __shared__ double E[kCheckMax * kEStride];
    __shared__ double red[kRedWords];
    const int tid = threadIdx.x;
    // after a failed tree (the host retries or reports it) Z is incomplete
    int64_t nrec = (P.ctl->error == kErrNone) ? P.ctl->chk_top : 0;
    if (nrec > P.chk_cap) nrec = P.chk_cap;
    for (int64_t rec = blockIdx.x; rec < nrec; rec += gridDim.x) {
        const CheckRec rc = P.chk[rec];
        const int m = (int)rc.m;
        const int64_t n = rc.n, ldz = rc.ldz;
        const double loss0 = rc.loss[0];
        if (!(loss0 > check_threshold(P, n)) || !((double)m * loss0 <= kRepairMax)) continue;
        double* Z = P.Z + rc.z;
        for (int pass = 0; pass < 2; ++pass) {
            __syncthreads();   // the previous E is no longer read
            for (int idx = tid; idx < kCheckMax * kEStride; idx += kRepThreads) E[idx] = 0.0;
            __syncthreads();
            dbl4 acc[kPairs];
            gram4(Z, ldz, n, m, red, acc);
            if (tid < 64) {
                if (pass == 1) {
                    const double loss1 = gram_loss(acc, m);
                    if (tid == 0) P.chk[rec].loss[1] = loss1;
                }
                // upper triangle only, mirrored: E is exactly symmetric
                for_upper(acc, m, [&](int i, int j, double g) {
                    const double v = g - (i == j ? 1.0 : 0.0);
                    E[i * kEStride + j] = v;
                    E[j * kEStride + i] = v;
                });
            }
            __syncthreads();
            switch ((m + 15) >> 4) {
                case 1: apply_rows<16>(Z, ldz, n, m, E); break;
                case 2: apply_rows<32>(Z, ldz, n, m, E); break;
                case 3: apply_rows<48>(Z, ldz, n, m, E); break;
                default: apply_rows<64>(Z, ldz, n, m, E); break;
            }
        }
        if (tid == 0) stat_add(&P.ctl->n_repaired, 1);
    }
}

namespace mrrr {

// ------------------------------------------------ conditional element growth
//
// A representation M = L D L^T whose element growth max |D| failed the test
// of Alg. 3.8 may still exhibit conditional element growth for its members
// (Sec. 3.1.2): for every relative perturbation M~ of its data bounded by xi,
// ||(M~ - M) z_i|| <= k_elg n xi spdiam for the computed eigenvectors z_i.  To
// first order the entries of M~ - M are bounded by 3 xi times those of
// |L||D||L^T| (tridiagonal: |d_{j-1} l_{j-1}|, |d_j| + |d_{j-1}| l_{j-1}^2,
// |d_j l_j|), so the test taken here is
//     || |L||D||L^T| |z| || <= (k_elg / 3) n spdiam ||z||,   k_elg = 10 (option),
// for the wanted members' final vectors (computed from this representation or
// from a descendant), over all rows of the block: every member of a cluster of
// up to kGrowthSample wanted members, else kGrowthSample members spread evenly
// over the cluster with both ends included (a chain of nested clusters of
// thousands would otherwise cost a pass over Z per level).  (The first condition
// of the definition, ||M~ - M|| <= spdiam, holds for xi = O(n eps) unless the
// growth exceeds 1e11 spdiam, where this test fails as well.)

// Exclusive prefix sum of the records' column counts (one workgroup).
extern "C" __global__ __launch_bounds__(1024) void mrrr_growth_prefix_kernel(Params P) {
    __shared__ int64_t part[1024];
    if (__hip_atomic_load(&P.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int64_t top = P.ctl->grw_top;
    const int64_t nrec = top < P.grw_cap ? top : P.grw_cap;
    const int t = threadIdx.x, nt = blockDim.x;
    const int64_t chunk = (nrec + nt - 1) / nt;
    const int64_t a = (int64_t)t * chunk, b = (a + chunk < nrec) ? a + chunk : nrec;
    int64_t sum = 0;
    for (int64_t r = a; r < b; ++r) sum += P.grw[r].mc;
    part[t] = sum;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int k = 0; k < nt; ++k) {
            const int64_t v = part[k];
            part[k] = acc;
            acc += v;
        }
        P.ctl->grw_cols = acc;
    }
    __syncthreads();
    int64_t acc = part[t];
    for (int64_t r = a; r < b; ++r) {
        P.grw[r].col0 = acc;
        acc += P.grw[r].mc;
    }
}

// One wavefront per column of a record: sum over the block's rows of
// w_j^2, w = |L||D||L^T| |z|, and of z_j^2.  Each step covers 4 x 64 rows
// with all twelve loads of a lane in flight at once; the neighbours z_{j-1},
// z_{j+1}, d_{j-1}, l_{j-1} come by shuffles within a 64-row group, from the
// adjacent group's edge lane, or (at the step's two ends) by the edge lanes'
// own loads.
extern "C" __global__ __launch_bounds__(256) void mrrr_growth_kernel(Params P) {
    constexpr int U = 4;
    if (__hip_atomic_load(&P.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int64_t top = P.ctl->grw_top;
    const int64_t nrec = top < P.grw_cap ? top : P.grw_cap;
    const int64_t ncol = P.ctl->grw_cols;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int64_t g = (int64_t)blockIdx.x * 4 + wv; g < ncol; g += (int64_t)gridDim.x * 4) {
        int64_t lo = 0, hi = nrec - 1;                 // the record holding column g
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (P.grw[mid].col0 <= g) lo = mid; else hi = mid - 1;
        }
        GrowthRec* rec = P.grw + lo;
        const int64_t n = rec->n;
        const double* D = P.arena + rec->rep;
        const double* L = D + n;
        const int64_t k = g - rec->col0;                // k-th checked column of mc
        const int64_t c = (rec->mc == rec->m) ? k : (k * (rec->m - 1)) / (rec->mc - 1);
        const double* z = P.Z + rec->z + c * rec->ldz;
        double ss = 0.0, zz = 0.0;
        for (int64_t base = 0; base < n; base += (int64_t)U * 64) {
            double zv[U], dv[U], lv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t j = base + 64 * u + lane;
                zv[u] = (j < n) ? z[j] : 0.0;
                dv[u] = (j < n) ? D[j] : 0.0;
                lv[u] = (j < n - 1) ? L[j] : 0.0;
            }
            // the rows just outside the step, by its edge lanes
            const int64_t jb = base - 1, je = base + (int64_t)U * 64;
            double zb = 0.0, db = 0.0, lb = 0.0, ze = 0.0;
            if (lane == 0 && jb >= 0) { zb = z[jb]; db = D[jb]; lb = L[jb]; }
            if (lane == 63 && je < n) ze = z[je];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t j = base + 64 * u + lane;
                double zp = __shfl_up(zv[u], 1), dp = __shfl_up(dv[u], 1), lp = __shfl_up(lv[u], 1);
                double zn = __shfl_down(zv[u], 1);
                // group edges: the neighbouring group's edge lane, or the step's ends
                const double zpe = (u > 0) ? __shfl(zv[u > 0 ? u - 1 : 0], 63) : zb;
                const double dpe = (u > 0) ? __shfl(dv[u > 0 ? u - 1 : 0], 63) : db;
                const double lpe = (u > 0) ? __shfl(lv[u > 0 ? u - 1 : 0], 63) : lb;
                const double zne = (u + 1 < U) ? __shfl(zv[u + 1 < U ? u + 1 : u], 0) : ze;
                if (lane == 0) { zp = zpe; dp = dpe; lp = lpe; }
                if (lane == 63) zn = zne;
                if (j < n) {
                    const double w = fabs(dp * lp) * fabs(zp) + (fabs(dv[u]) + fabs(dp * lp * lp)) * fabs(zv[u]) +
                                     fabs(dv[u] * lv[u]) * fabs(zn);
                    ss += w * w;
                    zz += zv[u] * zv[u];
                }
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            ss += __shfl_xor(ss, o);
            zz += __shfl_xor(zz, o);
        }
        if (lane == 0) {
            const double G = sqrt(ss / zz);
            if (!(G <= rec->bound)) {
                int32_t expect = 0;
                if (__hip_atomic_compare_exchange_strong(&rec->flag, &expect, (int32_t)1, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    stat_add(&P.ctl->n_grw_failed, 1);
            }
            const double ratio = G / rec->spdiam;
            const uint64_t bits = (ratio <= 1e300) ? (uint64_t)__double_as_longlong(ratio)
                                                   : (uint64_t)__double_as_longlong(__builtin_inf());
            __hip_atomic_fetch_max(&P.ctl->grw_max, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

hipError_t launch_growth(const Params& P, hipStream_t s) {
    if (!P.jobz || P.grw_cap <= 0 || !(P.cond_k > 0.0)) return hipSuccess;
    hipLaunchKernelGGL(mrrr_growth_prefix_kernel, dim3(1), dim3(1024), 0, s, P);
    hipLaunchKernelGGL(mrrr_growth_kernel, dim3(8192), dim3(256), 0, s, P);
    return hipGetLastError();
}

hipError_t launch_check(const Params& P, hipStream_t s) {
    if (!P.jobz || P.chk_cap <= 0) return hipSuccess;
    const int64_t g = P.chk_cap < 4096 ? P.chk_cap : 4096;
    hipLaunchKernelGGL(mrrr_check_small_kernel, dim3((unsigned)g), dim3(kChkThreads), 0, s, P);
    const int64_t gw = P.chk_cap < 1024 ? P.chk_cap : 1024;
    hipLaunchKernelGGL(mrrr_check_wide_kernel, dim3((unsigned)gw), dim3(kChkThreads), 0, s, P);
    const int64_t gr = P.chk_cap < 1024 ? P.chk_cap : 1024;
    hipLaunchKernelGGL(mrrr_repair_kernel, dim3((unsigned)gr), dim3(kRepThreads), 0, s, P);
    return hipGetLastError();
}

}  // namespace mrrr
