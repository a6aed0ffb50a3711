// Reverse mode through the tridiagonal eigendecomposition on gfx950.
//
// For T = tridiag(e, d, e) = Z diag(w) Z^T and a loss L(w, Z) with
// wbar = dL/dw and Zbar = dL/dZ:
//     M    = diag(wbar) + F o (Z^T Zbar),  F_ab = 1/(w_b - w_a) (a != b)
//     Tbar = Z M Z^T,  dbar_j = Tbar_jj,  ebar_j = Tbar_{j,j+1} + Tbar_{j+1,j}.
// The two products with Z are the only dense work and run on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64):
//     gemm_form_m : C = Z^T Zbar, epilogue writes M (gap mask, counts)
//     gemm_reduce : Y = Z M, epilogue reduces each row of Y against rows
//                   j-1, j, j+1 of Z, so Y itself is never stored.
// With Zbar absent the O(n^2) eigenvalue-only formulas are used directly.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/mrrr.h"

namespace mrrr {

typedef double dbl4 __attribute__((ext_vector_type(4)));

struct AdjProb {
    int64_t n;
    int64_t woff;   // w, wbar, dbar, ebar offset
    int64_t zoff, ldz;
    int64_t zboff, ldzb;
    int64_t moff;   // M scratch (n x n, ld n)
    int64_t poff;   // partial sums: 3 x n x ceil(n/32)
    double thresh;  // gap mask (absolute), set on the device
    int64_t epad;   // 1: ebar keeps a pad slot at n-1 (batched layout)
};

constexpr int kBM = 64, kBN = 64, kBK = 16;

// C(i, j) = sum_k A(i, k) B(k, j) over one 64 x 64 tile; A(i, k) =
// A[i*sai + k*sak], B(k, j) = B[k*sbk + j*sbj].  256 threads = 4 waves in a
// 2 x 2 arrangement, each wave 32 x 32 = 2 x 2 MFMA tiles of 16 x 16.
// Lane layout of v_mfma_f64_16x16x4f64 (measured on gfx950): A(i, k) from
// lane i + 16 k, B(k, j) from lane j + 16 k, and result register r of lane l
// holds C(4 r + l / 16, l % 16), r = 0..3.
template <class Epi>
__device__ __forceinline__ void mfma_tile(const double* __restrict__ A, int64_t sai, int64_t sak,
                                          const double* __restrict__ B, int64_t sbk, int64_t sbj,
                                          int64_t M, int64_t N, int64_t K, int64_t i0, int64_t j0,
                                          Epi epi) {
    __shared__ double As[kBK][kBM + 1];
    __shared__ double Bs[kBK][kBN + 1];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    dbl4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
    for (int64_t k0 = 0; k0 < K; k0 += kBK) {
        // stage A (64 x 16) and B (16 x 64); the faster-moving index follows
        // the contiguous dimension of each operand
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = tid + 256 * r;
            int ii, kk;
            if (sak == 1) { kk = e % kBK; ii = e / kBK; } else { ii = e % kBM; kk = e / kBM; }
            const int64_t gi = i0 + ii, gk = k0 + kk;
            As[kk][ii] = (gi < M && gk < K) ? A[gi * sai + gk * sak] : 0.0;
            int jj, kb;
            if (sbk == 1) { kb = e % kBK; jj = e / kBK; } else { jj = e % kBN; kb = e / kBN; }
            const int64_t gj = j0 + jj, gkb = k0 + kb;
            Bs[kb][jj] = (gj < N && gkb < K) ? B[gkb * sbk + gj * sbj] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kBK; ks += 4) {
            const int kr = ks + (lane >> 4);
            double av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = As[kr][wi + a * 16 + (lane & 15)];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = Bs[kr][wj + b * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    epi(acc, i0 + wi, j0 + wj, lane, wave);
}

// C = Z^T Zbar; M(a, b) = C(a, b) / (w_b - w_a) off the diagonal (0 and
// counted when |w_b - w_a| < thresh), wbar_a on the diagonal.
extern "C" __global__ __launch_bounds__(256) void mrrr_adj_form_m(const AdjProb* __restrict__ probs,
                                                                 const double* __restrict__ w,
                                                                 const double* __restrict__ Z,
                                                                 const double* __restrict__ Zb,
                                                                 const double* __restrict__ wbar,
                                                                 double* __restrict__ Mbuf,
                                                                 unsigned long long* __restrict__ masked) {
    const AdjProb pr = probs[blockIdx.z];
    const int64_t n = pr.n;
    const int64_t i0 = (int64_t)blockIdx.x * kBM, j0 = (int64_t)blockIdx.y * kBN;
    if (i0 >= n || j0 >= n) return;
    const double* Zp = Z + pr.zoff;
    const double* Zbp = Zb + pr.zboff;
    const double* wp = w + pr.woff;
    const double* wbp = wbar ? wbar + pr.woff : nullptr;
    double* Mp = Mbuf + pr.moff;
    const double thr = pr.thresh;
    mfma_tile(Zp, pr.ldz, 1, Zbp, 1, pr.ldzb, n, n, n, i0, j0,
              [&](dbl4 (&acc)[2][2], int64_t ib, int64_t jb, int lane, int) {
                  unsigned long long cnt = 0;
#pragma unroll
                  for (int a = 0; a < 2; ++a)
#pragma unroll
                      for (int b = 0; b < 2; ++b)
#pragma unroll
                          for (int r = 0; r < 4; ++r) {
                              const int64_t i = ib + a * 16 + 4 * r + (lane >> 4);
                              const int64_t j = jb + b * 16 + (lane & 15);
                              if (i < n && j < n) {
                                  double v;
                                  if (i == j) {
                                      v = wbp ? wbp[i] : 0.0;
                                  } else {
                                      const double diff = wp[j] - wp[i];
                                      if (fabs(diff) < thr) { v = 0.0; ++cnt; }
                                      else v = acc[a][b][r] / diff;
                                  }
                                  Mp[j * n + i] = v;
                              }
                          }
                  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
                  if (lane == 0 && cnt) atomicAdd(masked + blockIdx.z, cnt);
              });
}

// Y = Z M; for every row i of the tile: s0 = sum_a Z(i,a) Y(i,a),
// s1 = sum_a Z(i+1,a) Y(i,a), s2 = sum_a Z(i-1,a) Y(i,a) over the wave's 32
// columns, written to partial column (tile column * 2 + wave column).
extern "C" __global__ __launch_bounds__(256) void mrrr_adj_reduce(const AdjProb* __restrict__ probs,
                                                                 const double* __restrict__ Z,
                                                                 const double* __restrict__ Mbuf,
                                                                 double* __restrict__ part) {
    const AdjProb pr = probs[blockIdx.z];
    const int64_t n = pr.n;
    const int64_t i0 = (int64_t)blockIdx.x * kBM, j0 = (int64_t)blockIdx.y * kBN;
    if (i0 >= n || j0 >= n) return;
    const double* Zp = Z + pr.zoff;
    const double* Mp = Mbuf + pr.moff;
    const int64_t npc = (n + 31) / 32;
    double* pp = part + pr.poff;
    mfma_tile(Zp, 1, pr.ldz, Mp, 1, n, n, n, n, i0, j0,
              [&](dbl4 (&acc)[2][2], int64_t ib, int64_t jb, int lane, int wave) {
                  const int64_t pc = (j0 / 32) + (wave & 1);
                  if (j0 + 32 * (wave & 1) >= n) return;   // no columns here
#pragma unroll
                  for (int a = 0; a < 2; ++a)
#pragma unroll
                      for (int r = 0; r < 4; ++r) {
                          const int64_t i = ib + a * 16 + 4 * r + (lane >> 4);
                          double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
                          for (int b = 0; b < 2; ++b) {
                              const int64_t j = jb + b * 16 + (lane & 15);
                              if (i < n && j < n) {
                                  const double y = acc[a][b][r];
                                  const double* zc = Zp + j * pr.ldz;
                                  s0 += zc[i] * y;
                                  if (i + 1 < n) s1 += zc[i + 1] * y;
                                  if (i >= 1) s2 += zc[i - 1] * y;
                              }
                          }
                          // sum over the 16 lanes holding this row
                          for (int o = 8; o > 0; o >>= 1) {
                              s0 += __shfl_xor(s0, o);
                              s1 += __shfl_xor(s1, o);
                              s2 += __shfl_xor(s2, o);
                          }
                          if ((lane & 15) == 0 && i < n) {
                              pp[(0 * npc + pc) * n + i] = s0;
                              pp[(1 * npc + pc) * n + i] = s1;
                              pp[(2 * npc + pc) * n + i] = s2;
                          }
                      }
              });
}

// dbar_i = sum_pc s0; ebar_j = sum_pc s1(j) + s2(j+1).  Partial columns that
// no tile wrote (beyond n) are skipped by the column count.
extern "C" __global__ void mrrr_adj_finish(const AdjProb* __restrict__ probs, const double* __restrict__ part,
                                           double* __restrict__ dbar, double* __restrict__ ebar) {
    const AdjProb pr = probs[blockIdx.y];
    const int64_t n = pr.n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t npc = (n + 31) / 32;
    const double* pp = part + pr.poff;
    double s0 = 0.0, s1 = 0.0, s2n = 0.0;
    for (int64_t pc = 0; pc < npc; ++pc) {
        s0 += pp[(0 * npc + pc) * n + i];
        s1 += pp[(1 * npc + pc) * n + i];
        if (i + 1 < n) s2n += pp[(2 * npc + pc) * n + i + 1];
    }
    dbar[pr.woff + i] = s0;
    if (i + 1 < n) ebar[pr.woff + i] = s1 + s2n;
    else if (pr.epad) ebar[pr.woff + i] = 0.0;   // pad slot (batched layout)
}

// Eigenvalue-only loss: dbar_j = sum_a wbar_a z_ja^2, ebar_j = 2 sum_a wbar_a
// z_ja z_{j+1,a}; one thread per row, columns streamed (coalesced in j).
extern "C" __global__ void mrrr_adj_values(const AdjProb* __restrict__ probs, const double* __restrict__ Z,
                                           const double* __restrict__ wbar, double* __restrict__ dbar,
                                           double* __restrict__ ebar) {
    const AdjProb pr = probs[blockIdx.y];
    const int64_t n = pr.n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* Zp = Z + pr.zoff;
    const double* wb = wbar + pr.woff;
    double s0 = 0.0, s1 = 0.0;
    for (int64_t a = 0; a < n; ++a) {
        const double z = Zp[a * pr.ldz + i];
        const double c = wb[a] * z;
        s0 += c * z;
        if (i + 1 < n) s1 += c * Zp[a * pr.ldz + i + 1];
    }
    dbar[pr.woff + i] = s0;
    if (i + 1 < n) ebar[pr.woff + i] = 2.0 * s1;
    else if (pr.epad) ebar[pr.woff + i] = 0.0;
}

// ||T|| = max |w| per problem, and the absolute gap mask.
extern "C" __global__ void mrrr_adj_thresh(AdjProb* probs, const double* __restrict__ w, double rel) {
    AdjProb* pr = probs + blockIdx.x;
    const int64_t n = pr->n;
    double mx = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) mx = fmax(mx, fabs(w[pr->woff + i]));
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    __shared__ double sm[16];
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t = fmax(t, sm[k]);
        pr->thresh = rel * t;
    }
}

int adjoint_run(hipStream_t s, int64_t batch, const int64_t* noff, const int64_t* zoffs, const double* w,
                const double* Z, const double* wbar, const double* Zbar, double gap_mask_rel, double* dbar,
                double* ebar, int64_t* n_masked_h, int64_t ldz_single, int64_t ldzbar_single,
                void* (*alloc)(void*, size_t), void* ctx) {
    std::vector<AdjProb> pv((size_t)batch);
    int64_t zpack = 0, msz = 0, psz = 0, nmax = 0;
    for (int64_t b = 0; b < batch; ++b) {
        const int64_t n = noff[b + 1] - noff[b];
        AdjProb& p = pv[(size_t)b];
        p.n = n;
        p.woff = noff[b];
        p.zoff = zoffs ? zoffs[b] : zpack;
        p.ldz = (ldz_single > 0) ? ldz_single : (n > 0 ? n : 1);
        p.zboff = p.zoff;
        p.ldzb = (ldzbar_single > 0) ? ldzbar_single : p.ldz;
        if (ldz_single > 0) p.zboff = 0;
        p.moff = msz;
        p.poff = psz;
        p.thresh = 0.0;
        p.epad = (ldz_single > 0) ? 0 : 1;
        zpack += n * n;
        if (Zbar) {
            msz += n * n;
            psz += 3 * n * ((n + 31) / 32);
        }
        nmax = n > nmax ? n : nmax;
    }
    const size_t bytes_p = sizeof(AdjProb) * (size_t)batch;
    const size_t bytes_m = sizeof(double) * (size_t)msz;
    const size_t bytes_q = sizeof(double) * (size_t)psz;
    const size_t bytes_c = sizeof(unsigned long long) * (size_t)batch;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    char* base = (char*)alloc(ctx, al(bytes_p) + al(bytes_m) + al(bytes_q) + al(bytes_c));
    if (!base) return MRRR_ENOMEM;
    AdjProb* dprobs = (AdjProb*)base;
    double* Mb = (double*)(base + al(bytes_p));
    double* part = (double*)(base + al(bytes_p) + al(bytes_m));
    unsigned long long* cnt = (unsigned long long*)(base + al(bytes_p) + al(bytes_m) + al(bytes_q));
    if (hipMemcpyAsync(dprobs, pv.data(), bytes_p, hipMemcpyHostToDevice, s) != hipSuccess) return MRRR_EHIP;
    if (hipMemsetAsync(cnt, 0, bytes_c, s) != hipSuccess) return MRRR_EHIP;
    const unsigned rows_blocks = (unsigned)((nmax + 255) / 256);
    if (!Zbar) {
        if (wbar) {
            hipLaunchKernelGGL(mrrr_adj_values, dim3(rows_blocks, (unsigned)batch), dim3(256), 0, s, dprobs, Z, wbar,
                               dbar, ebar);
        } else {
            // no cotangent at all: zero gradient
            for (int64_t b = 0; b < batch; ++b) {
                const int64_t n = pv[(size_t)b].n;
                if (hipMemsetAsync(dbar + pv[(size_t)b].woff, 0, sizeof(double) * (size_t)n, s) != hipSuccess)
                    return MRRR_EHIP;
                const int64_t ne = (batch == 1) ? (n > 0 ? n - 1 : 0) : n;
                if (ne > 0 && hipMemsetAsync(ebar + pv[(size_t)b].woff, 0, sizeof(double) * (size_t)ne, s) != hipSuccess)
                    return MRRR_EHIP;
            }
        }
    } else {
        hipLaunchKernelGGL(mrrr_adj_thresh, dim3((unsigned)batch), dim3(256), 0, s, dprobs, w, gap_mask_rel);
        const unsigned tiles = (unsigned)((nmax + kBM - 1) / kBM);
        hipLaunchKernelGGL(mrrr_adj_form_m, dim3(tiles, tiles, (unsigned)batch), dim3(256), 0, s, dprobs, w, Z, Zbar,
                           wbar, Mb, cnt);
        hipLaunchKernelGGL(mrrr_adj_reduce, dim3(tiles, tiles, (unsigned)batch), dim3(256), 0, s, dprobs, Z, Mb,
                           part);
        hipLaunchKernelGGL(mrrr_adj_finish, dim3(rows_blocks, (unsigned)batch), dim3(256), 0, s, dprobs, part, dbar,
                           ebar);
    }
    if (hipGetLastError() != hipSuccess) return MRRR_EHIP;
    if (n_masked_h) {
        std::vector<unsigned long long> hc((size_t)batch);
        if (hipMemcpyAsync(hc.data(), cnt, bytes_c, hipMemcpyDeviceToHost, s) != hipSuccess) return MRRR_EHIP;
        if (hipStreamSynchronize(s) != hipSuccess) return MRRR_EHIP;
        int64_t t = 0;
        for (auto v : hc) t += (int64_t)v;
        *n_masked_h = t;
    }
    return MRRR_OK;
}


// ------------------------------------------------- backward without allocation
//
// A fixed device array holds everything the backward keeps besides its
// inputs and outputs: the problem record and the mask counter (first 512
// bytes), M (n x n) and the partial sums (3 n ceil(n/32)), for n up to
// MRRR_BACKWARD_NOALLOC_MAX_N.  Every call on one GPU uses that GPU's copy of
// the array, so calls that overlap on one GPU race.  Host code never names the
// array: it uses the address hipGetSymbolAddress returned for the device.

constexpr int64_t kNaMaxN = MRRR_BACKWARD_NOALLOC_MAX_N;
constexpr int64_t kNaHeader = 64;   // doubles: AdjProb at 0, counter at byte 256
constexpr int64_t kNaDoubles = kNaHeader + kNaMaxN * kNaMaxN + 3 * kNaMaxN * ((kNaMaxN + 31) / 32);
static_assert(sizeof(AdjProb) <= 256, "problem record must fit the header");

static __device__ __align__(256) double scratch[kNaDoubles];

// Called once per device at handle creation, with that device current.
int adjoint_scratch_address(void** ptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
        *ptr = nullptr;
        return MRRR_EHIP;
    }
    *ptr = p;
    return MRRR_OK;
}

// The record and the cleared counter are written by a kernel (its argument
// is copied at launch), so the call copies nothing from host memory.
extern "C" __global__ void mrrr_adj_na_setup(AdjProb p, AdjProb* dst, unsigned long long* cnt) {
    if (threadIdx.x == 0) {
        *dst = p;
        *cnt = 0ull;
    }
}

extern "C" __global__ void mrrr_adj_na_zero(double* __restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

int adjoint_run_noalloc(hipStream_t s, void* scr, int64_t n, const double* w, const double* Z, int64_t ldz,
                        const double* wbar, const double* Zbar, int64_t ldzbar, double gap_mask_rel,
                        double* dbar, double* ebar, int64_t* n_masked_h) {
    if (!scr) return MRRR_EHIP;
    if (Zbar && n > kNaMaxN) return -2;
    AdjProb pr{};
    pr.n = n;
    pr.ldz = ldz;
    pr.ldzb = Zbar ? ldzbar : ldz;
    pr.epad = 0;
    AdjProb* dprob = static_cast<AdjProb*>(scr);
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(static_cast<char*>(scr) + 256);
    double* Mb = static_cast<double*>(scr) + kNaHeader;
    double* part = Mb + n * n;
    const unsigned rows_blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(mrrr_adj_na_setup, dim3(1), dim3(64), 0, s, pr, dprob, cnt);
    if (!Zbar) {
        if (wbar) {
            hipLaunchKernelGGL(mrrr_adj_values, dim3(rows_blocks, 1), dim3(256), 0, s, dprob, Z, wbar, dbar, ebar);
        } else {
            hipLaunchKernelGGL(mrrr_adj_na_zero, dim3(rows_blocks), dim3(256), 0, s, dbar, n);
            if (n > 1)
                hipLaunchKernelGGL(mrrr_adj_na_zero, dim3(rows_blocks), dim3(256), 0, s, ebar, n - 1);
        }
    } else {
        hipLaunchKernelGGL(mrrr_adj_thresh, dim3(1), dim3(256), 0, s, dprob, w, gap_mask_rel);
        const unsigned tiles = (unsigned)((n + kBM - 1) / kBM);
        hipLaunchKernelGGL(mrrr_adj_form_m, dim3(tiles, tiles, 1), dim3(256), 0, s, dprob, w, Z, Zbar, wbar, Mb,
                           cnt);
        hipLaunchKernelGGL(mrrr_adj_reduce, dim3(tiles, tiles, 1), dim3(256), 0, s, dprob, Z, Mb, part);
        hipLaunchKernelGGL(mrrr_adj_finish, dim3(rows_blocks, 1), dim3(256), 0, s, dprob, part, dbar, ebar);
    }
    if (hipGetLastError() != hipSuccess) return MRRR_EHIP;
    if (n_masked_h) {
        unsigned long long hc = 0;
        if (Zbar) {
            if (hipMemcpyAsync(&hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, s) != hipSuccess) return MRRR_EHIP;
            if (hipStreamSynchronize(s) != hipSuccess) return MRRR_EHIP;
        }
        *n_masked_h = (int64_t)hc;
    }
    return MRRR_OK;
}

}  // namespace mrrr
