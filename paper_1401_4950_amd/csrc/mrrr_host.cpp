// Host runtime behind include/mrrr.h: handle, workspace, argument checks,
// launch sequence, status read-back, batched plans with hipGraph replay.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/mrrr.h"
#include "mrrr_internal.h"

static_assert(sizeof(mrrr::TraceRec) == sizeof(mrrr_trace_t), "trace record layout");
static_assert(sizeof(mrrr::CheckRec) == 64, "check record layout");

namespace mrrr {
hipError_t launch_init(const Params& P, hipStream_t s);
hipError_t launch_setup(const Params& P, hipStream_t s);
hipError_t launch_tree(const Params& P, hipStream_t s);
hipError_t launch_finalize(const Params& P, hipStream_t s);
hipError_t launch_sign(const Params& P, int64_t ncols_total, hipStream_t s);
hipError_t launch_check(const Params& P, hipStream_t s);
hipError_t launch_growth(const Params& P, hipStream_t s);
hipError_t tree_occupancy(int* blocks_per_cu);
hipError_t launch_quot(const double* a, const double* b, double* q, int64_t n, hipStream_t s);
hipError_t launch_widen(const float* x, double* y, int64_t n, hipStream_t s);
hipError_t launch_narrow(const double* src, int64_t lds, float* dst, int64_t ldd, int64_t rows, int64_t cols,
                         hipStream_t s);
int adjoint_run(hipStream_t s, int64_t batch, const int64_t* n_offsets_h, const int64_t* z_offsets_h,
                const double* w, const double* Z, const double* wbar, const double* Zbar,
                double gap_mask_rel, double* dbar, double* ebar, int64_t* n_masked_h, int64_t ldz_single,
                int64_t ldzbar_single, void* (*alloc)(void*, size_t), void* alloc_ctx);
int adjoint_scratch_address(void** ptr);
int adjoint_run_noalloc(hipStream_t s, void* scr, int64_t n, const double* w, const double* Z, int64_t ldz,
                        const double* wbar, const double* Zbar, int64_t ldzbar, double gap_mask_rel,
                        double* dbar, double* ebar, int64_t* n_masked_h);
}  // namespace mrrr

using namespace mrrr;

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t want) {
        if (want == 0) want = 8;
        if (bytes >= want) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) bytes = want;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

struct Workspace {
    DevBuf probs, blocks, nodes, q[kNumQ], seq[kNumQ], lo, hi, gap, lo0, hi0, vflag, need, slist, arena, ck, colbuf, perm, ctl, chk,
        grw;
    void release() {
        probs.release(); blocks.release(); nodes.release();
        for (int i = 0; i < kNumQ; ++i) { q[i].release(); seq[i].release(); }
        lo.release(); hi.release(); gap.release(); lo0.release(); hi0.release(); vflag.release(); need.release(); slist.release();
        arena.release(); ck.release(); colbuf.release(); perm.release(); ctl.release(); chk.release(); grw.release();
    }
};

struct Sizes {
    int64_t rows = 0, nprob = 0, max_nodes = 0, ck = 0;
    uint64_t qcap[kNumQ] = {0, 0, 0};
    uint64_t arena = 0;
};

}  // namespace

struct mrrr_batched_plan_s {
    int64_t batch = 0;
    std::vector<int64_t> noff, zoff;
    std::vector<int32_t> tune;   // copy of the per-matrix table (empty: none)
    mrrr_options_t opts{};
    const double *d = nullptr, *e = nullptr;
    double *w = nullptr, *Z = nullptr;
    Workspace ws;
    Params P{};
    Sizes sz;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<Problem> probs;
    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        ws.release();
    }
};

struct mrrr_handle_s {
    int device = 0;
    hipStream_t stream = nullptr;
    int ncu = 0;
    int occ = 0;
    double wall_khz = 100000.0;
    Workspace ws;
    hipEvent_t ev0 = nullptr, ev1 = nullptr, evt0 = nullptr, evt1 = nullptr;
    mrrr_batched_plan_s* plan = nullptr;   // most recent batched plan
    DevBuf adj;                            // backward scratch
    void* na_scratch = nullptr;            // this device's fixed backward scratch (no-allocation entry point)
    DevBuf mixed;                          // single/double form: FP64 copies of d, e, w, Z
    DevBuf dense;                          // dense driver: copy of A (reflectors), d, e, tau
    rocblas_handle rb = nullptr;           // dense driver: reduction and back-transformation
};

extern "C" void mrrr_default_options(mrrr_options_t* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->jobz = 1;
    o->sign_convention = 1;
    o->gaptol = 1e-3;
    o->rtol_class = 1e-5;
    o->perturb_xi = 8.0;
    o->seed = 0x5eed5eedull;
    o->max_rqi = 10;
    o->max_shift_tries = 16;
    o->max_depth = 64;
    o->workers = 0;
    o->slice_min = 2;
    o->slice_max = 64;
    o->lanes_per_eig = 64;
    o->bundle = 64;
    o->tune = nullptr;
    o->timeout_s = 30.0;
    o->arena_scale = 1.0;
    o->check_tol = 20.0;
    o->cond_growth_k = 10.0;
    o->bundle_helpers = 1;
    o->pass_helpers = 1;
}

extern "C" const char* mrrr_status_string(int s) {
    if (s < 0) return "invalid argument";
    switch (s) {
        case MRRR_OK: return "ok";
        case MRRR_WARN_UNVERIFIED: return "a representation was accepted without passing the element-growth test";
        case MRRR_ENOMEM: return "out of device memory or work-queue capacity";
        case MRRR_ENOCONV: return "an eigenvalue did not converge";
        case MRRR_EHIP: return "HIP runtime error";
        case MRRR_ETIMEOUT: return "device watchdog expired";
        case MRRR_EINTERNAL: return "internal consistency check failed";
        default: return "unknown status";
    }
}

extern "C" int mrrr_create(mrrr_handle_t* h, int device) {
    if (!h) return -1;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return MRRR_EHIP;
    if (device < 0 || device >= ndev) return -2;
    auto* H = new (std::nothrow) mrrr_handle_s;
    if (!H) return MRRR_ENOMEM;
    H->device = device;
    if (hipSetDevice(device) != hipSuccess) { delete H; return MRRR_EHIP; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete H; return MRRR_EHIP; }
    H->ncu = prop.multiProcessorCount;
    int rate = 0;
    if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, device) == hipSuccess && rate > 0)
        H->wall_khz = (double)rate;
    // the fixed scratch of the no-allocation backward: its address on this
    // device, taken once here with the device current (a failure is reported
    // by that entry point, the rest of the library does not need it)
    if (adjoint_scratch_address(&H->na_scratch) != MRRR_OK) H->na_scratch = nullptr;
    int occ = 0;
    if (tree_occupancy(&occ) != hipSuccess || occ < 1) occ = 1;
    H->occ = occ;
    if (hipEventCreate(&H->ev0) != hipSuccess || hipEventCreate(&H->ev1) != hipSuccess ||
        hipEventCreate(&H->evt0) != hipSuccess || hipEventCreate(&H->evt1) != hipSuccess) {
        for (hipEvent_t ev : {H->ev0, H->ev1, H->evt0, H->evt1})
            if (ev) (void)hipEventDestroy(ev);
        delete H;
        return MRRR_EHIP;
    }
    *h = H;
    return MRRR_OK;
}

extern "C" int mrrr_destroy(mrrr_handle_t h) {
    if (!h) return -1;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    if (h->plan) { h->plan->release(); delete h->plan; }
    h->ws.release();
    h->adj.release();
    h->mixed.release();
    h->dense.release();
    if (h->rb) (void)rocblas_destroy_handle(h->rb);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    if (h->evt0) (void)hipEventDestroy(h->evt0);
    if (h->evt1) (void)hipEventDestroy(h->evt1);
    delete h;
    return MRRR_OK;
}

extern "C" int mrrr_set_stream(mrrr_handle_t h, void* stream) {
    if (!h) return -1;
    h->stream = (hipStream_t)stream;
    return MRRR_OK;
}

namespace {

int map_device_error(int code) {
    switch (code) {
        case kErrNone: return MRRR_OK;
        case kErrNoMem: return MRRR_ENOMEM;
        case kErrNoConv: return MRRR_ENOCONV;
        case kErrTimeout: return MRRR_ETIMEOUT;
        case kErrBadD: return -3;
        case kErrBadE: return -4;
        default: return MRRR_EINTERNAL;
    }
}

// Allocates the workspace for `sz` and fills the pointer part of P.
hipError_t prepare(Workspace& ws, const Sizes& sz, Params& P) {
    hipError_t e;
#define ENS(buf, bytes) do { if ((e = (buf).ensure(bytes)) != hipSuccess) return e; } while (0)
    ENS(ws.probs, sizeof(Problem) * (size_t)sz.nprob);
    ENS(ws.blocks, sizeof(Block) * (size_t)std::max<int64_t>(sz.rows, 1));
    ENS(ws.nodes, sizeof(Node) * (size_t)sz.max_nodes);
    for (int q = 0; q < kNumQ; ++q) {
        ENS(ws.q[q], sizeof(Task) * sz.qcap[q]);
        ENS(ws.seq[q], sizeof(uint64_t) * sz.qcap[q]);
    }
    const size_t r = (size_t)std::max<int64_t>(sz.rows, 1);
    ENS(ws.lo, sizeof(double) * r);
    ENS(ws.hi, sizeof(double) * r);
    ENS(ws.gap, sizeof(double) * r);
    ENS(ws.lo0, sizeof(double) * r);
    ENS(ws.hi0, sizeof(double) * r);
    ENS(ws.vflag, r);
    ENS(ws.need, r);
    ENS(ws.slist, sizeof(int32_t) * r);
    ENS(ws.arena, sizeof(double) * sz.arena);
    ENS(ws.ck, sizeof(double) * (size_t)std::max<int64_t>(sz.ck, 1));
    ENS(ws.colbuf, sizeof(double) * 2 * r);
    ENS(ws.perm, sizeof(int32_t) * 2 * r);
    ENS(ws.ctl, sizeof(Ctl));
    // checked clusters are disjoint and hold two columns or more
    const int64_t nchk = std::max<int64_t>(sz.rows / 2, 1);
    ENS(ws.chk, sizeof(CheckRec) * (size_t)nchk);
    // cluster representations form a laminar family of member sets of two or
    // more: fewer than rows of them
    ENS(ws.grw, sizeof(GrowthRec) * r);
#undef ENS
    P.probs = ws.probs.as<Problem>();
    P.blocks = ws.blocks.as<Block>();
    P.nodes = ws.nodes.as<Node>();
    P.max_nodes = (int32_t)std::min<int64_t>(sz.max_nodes, INT32_MAX);
    for (int q = 0; q < kNumQ; ++q) {
        P.q[q] = ws.q[q].as<Task>();
        P.seq[q] = ws.seq[q].as<uint64_t>();
        P.qcap[q] = sz.qcap[q];
    }
    P.lo = ws.lo.as<double>();
    P.hi = ws.hi.as<double>();
    P.gap = ws.gap.as<double>();
    P.lo0 = ws.lo0.as<double>();
    P.hi0 = ws.hi0.as<double>();
    P.vflag = ws.vflag.as<uint8_t>();
    P.need = ws.need.as<uint8_t>();
    P.slist = ws.slist.as<int32_t>();
    P.slist_cap = sz.rows;
    P.arena = ws.arena.as<double>();
    P.arena_cap = sz.arena;
    P.ck = ws.ck.as<double>();
    P.colbuf = ws.colbuf.as<double>();
    P.perm = ws.perm.as<int32_t>();
    P.ctl = ws.ctl.as<Ctl>();
    P.chk = ws.chk.as<CheckRec>();
    P.chk_cap = nchk;
    P.grw = ws.grw.as<GrowthRec>();
    P.grw_cap = (int64_t)r;
    P.total_rows = sz.rows;
    return hipSuccess;
}

void set_options(Params& P, const mrrr_options_t& o, double wall_khz, int workers, double io_eps = 0.0) {
    P.jobz = o.jobz ? 1 : 0;
    P.gaptol = o.gaptol;
    P.rtol = o.rtol_class;
    P.xi = o.perturb_xi;
    P.seed = o.seed;
    P.max_rqi = o.max_rqi;
    P.max_tries = o.max_shift_tries;
    P.max_depth = o.max_depth;
    P.slice_min = std::max(1, o.slice_min);
    P.sign_conv = o.sign_convention;
    P.assist = o.bundle_helpers != 0 ? 1 : 0;
    P.coop = o.pass_helpers != 0 ? 1 : 0;
    P.nworkers = workers;
    P.timeout_ticks = (uint64_t)std::max(1.0, o.timeout_s * wall_khz * 1000.0);
    P.trace = (o.trace && o.trace_cap > 0) ? static_cast<TraceRec*>(o.trace) : nullptr;
    P.trace_cap = P.trace ? o.trace_cap : 0;
    P.check_tol = o.check_tol;
    P.io_eps = io_eps;
    P.cond_k = o.cond_growth_k;
}

int check_options(const mrrr_options_t& o) {
    if (!(o.gaptol > 0.0 && o.gaptol < 1.0)) return 1;
    if (!(o.rtol_class > 0.0 && o.rtol_class < 1.0)) return 1;
    if (!(o.perturb_xi >= 0.0 && o.perturb_xi <= 0x1p30)) return 1;
    if (o.max_rqi < 0 || o.max_shift_tries < 1 || o.max_depth < 1) return 1;
    if (!(o.timeout_s > 0.0)) return 1;
    if (o.trace_cap < 0) return 1;
    if (o.lanes_per_eig < 1 || o.lanes_per_eig > kWave || (o.lanes_per_eig & (o.lanes_per_eig - 1))) return 1;
    if (o.bundle < 1 || o.bundle > kWave) return 1;
    if (!(o.check_tol >= 0.0 && o.check_tol <= 1e15)) return 1;
    if (!(o.cond_growth_k >= 0.0 && o.cond_growth_k <= 1e300)) return 1;
    return 0;
}

// Launch shape of one matrix: the scalar options, or entry b of the
// per-matrix table where it is positive (lanes rounded down to a power of
// two, everything clamped to what the kernel supports).
void apply_tune(Problem& pr, const mrrr_options_t& o, const int32_t* tune, int64_t b) {
    int lanes = o.lanes_per_eig, bundle = o.bundle, smax = o.slice_max;
    if (tune) {
        if (tune[3 * b] > 0) lanes = tune[3 * b];
        if (tune[3 * b + 1] > 0) bundle = tune[3 * b + 1];
        if (tune[3 * b + 2] > 0) smax = tune[3 * b + 2];
    }
    lanes = std::min(kWave, std::max(1, lanes));
    int p2 = 1;
    while (p2 * 2 <= lanes) p2 *= 2;
    pr.lanes = (int16_t)p2;
    pr.bundle = (int16_t)std::min(kWave, std::max(1, bundle));
    pr.slice_max = std::min(kWave, std::max(std::max(1, o.slice_min), smax));
}

Sizes base_sizes(int64_t rows, int64_t nprob, int64_t kwork, int64_t nmax, double arena_scale) {
    Sizes sz;
    sz.rows = rows;
    sz.nprob = nprob;
    sz.max_nodes = (int64_t)((double)(rows + 2 * nprob + 1024) * std::max(1.0, arena_scale));
    sz.qcap[kQRefine] = (uint64_t)std::max<int64_t>(65536, 2 * rows + 1024);
    sz.qcap[kQCluster] = (uint64_t)std::max<int64_t>(16384, rows + 1024);
    sz.qcap[kQSingle] = (uint64_t)std::max<int64_t>(16384, rows + 1024);
    // node pool: 4 n + kNodeExtra doubles per representation (D and L of
    // the new representation, the checkpoints of the factorisation and the
    // cooperation block); start from a few hundred nodes of the largest block
    // size
    const double per_node = 4.0 * (double)nmax + (double)kNodeExtra;
    const double nodes = std::min<double>((double)kwork + 2.0 * nprob, 256.0 + (double)kwork / 4.0);
    double a = per_node * std::max(nodes, 8.0 * nprob) * std::max(arena_scale, 1e-3);
    const double cap = per_node * ((double)kwork + 2.0 * nprob + 8.0) * std::max(1.0, arena_scale);
    if (a > cap) a = cap;
    sz.arena = (uint64_t)std::max(a, per_node + 64.0);
    return sz;
}

int read_back(mrrr_handle_t h, const Params& P, Ctl* ctl_h, std::vector<Problem>* probs_h) {
    if (hipMemcpyAsync(ctl_h, P.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream) != hipSuccess) return MRRR_EHIP;
    if (probs_h && hipMemcpyAsync(probs_h->data(), P.probs, sizeof(Problem) * probs_h->size(),
                                  hipMemcpyDeviceToHost, h->stream) != hipSuccess)
        return MRRR_EHIP;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return MRRR_EHIP;
    return MRRR_OK;
}

// Representations accepted without passing a growth test: those that failed
// the element-growth bound of Alg. 3.8 and were not shown afterwards to
// exhibit conditional element growth for their members' vectors.
int64_t still_unverified(const Ctl& c) {
    const int64_t passed = c.grw_top - c.n_grw_failed;
    return c.n_unverified - (passed > 0 ? passed : 0);
}

void fill_stats(mrrr_stats_t* st, const Ctl& c, int64_t m, float ms, float tree_ms = 0.f) {
    if (!st) return;
    std::memset(st, 0, sizeof(*st));
    st->m = m;
    st->n_blocks = c.n_blocks;
    st->n_nodes = c.n_nodes;
    st->largest_cluster = c.largest_cluster;
    st->dmax = c.dmax;
    st->n_unverified_rrr = c.n_unverified;
    st->n_bisect_fallback = c.n_fallback;
    st->n_nan_retry = c.n_nan;
    st->n_sturm_guarded = c.n_sturm;
    st->n_factor_quotient = c.n_fac_quot;
    st->n_checked = c.n_checked;
    st->n_reorthogonalized = c.n_repaired;
    st->n_check_failed = c.n_check_failed;
    st->n_check_wide = c.n_check_wide;
    st->n_cond_checked = c.grw_top;
    st->n_cond_failed = c.n_grw_failed;
    {
        double g;
        std::memcpy(&g, &c.grw_max, sizeof(g));
        st->max_cond_growth = g;
    }
    st->qd_steps = c.qd_steps;
    st->n_tasks = c.n_tasks;
    st->n_singleton_tasks = c.n_single;
    st->n_rqi_iters = c.n_rqi;
    st->arena_bytes = (int64_t)(c.arena_top * sizeof(double));
    st->ms = ms;
    st->tree_ms = tree_ms;
}

// ev_tree: optional pair of events recorded around the tree kernel
hipError_t enqueue_solve(const Params& P, int64_t ncols_total, bool sign, hipStream_t s,
                         hipEvent_t* ev_tree = nullptr) {
    hipError_t e;
    if ((e = launch_init(P, s)) != hipSuccess) return e;
    if ((e = launch_setup(P, s)) != hipSuccess) return e;
    if (ev_tree && (e = hipEventRecord(ev_tree[0], s)) != hipSuccess) return e;
    if ((e = launch_tree(P, s)) != hipSuccess) return e;
    if (ev_tree && (e = hipEventRecord(ev_tree[1], s)) != hipSuccess) return e;
    if ((e = launch_growth(P, s)) != hipSuccess) return e;
    if ((e = launch_check(P, s)) != hipSuccess) return e;
    if ((e = launch_finalize(P, s)) != hipSuccess) return e;
    if (sign && P.jobz && (e = launch_sign(P, ncols_total, s)) != hipSuccess) return e;
    return hipSuccess;
}

int workers_for(mrrr_handle_t h, const mrrr_options_t& o) {
    if (o.workers > 0) return o.workers;
    return std::max(1, h->ncu * h->occ);
}

}  // namespace

namespace {

// Arguments of one single-matrix solve, validated by the caller's entry point.
int check_single(mrrr_handle_t h, int64_t n, const void* d, const void* e, int range, double vl, double vu,
                 int64_t il, int64_t iu, const mrrr_options_t& o, const int64_t* m, const void* w, const void* Z,
                 int64_t ldz) {
    if (!h) return -1;
    if (n < 0 || n > (int64_t)INT32_MAX / 2) return -2;
    if (n > 0 && !d) return -3;
    if (n > 1 && !e) return -4;
    if (range < 0 || range > 2) return -5;
    if (range == MRRR_RANGE_VALUE && !(std::isfinite(vl) && std::isfinite(vu) && vl < vu)) return -7;
    if (range == MRRR_RANGE_INDEX && (il < 1 || il > n + 1)) return -8;
    if (range == MRRR_RANGE_INDEX && (iu < il - 1 || iu > n)) return -9;
    if (check_options(o)) return -10;
    if (!m) return -11;
    if (n > 0 && !w) return -12;
    if (o.jobz && n > 0 && !Z) return -13;
    if (o.jobz && ldz < std::max<int64_t>(1, n)) return -14;
    return MRRR_OK;
}

// The solve of one matrix on device data already in FP64 (arguments checked).
int solve_single(mrrr_handle_t h, int64_t n, const double* d, const double* e, int range, double vl, double vu,
                 int64_t il, int64_t iu, const mrrr_options_t& o, double io_eps, int64_t* m, double* w, double* Z,
                 int64_t ldz, mrrr_stats_t* stats) {

    Problem pr{};
    pr.row0 = 0;
    pr.n = n;
    pr.zoff = 0;
    pr.ldz = o.jobz ? ldz : 1;
    pr.woff = 0;
    pr.il = il;
    pr.iu = iu;
    pr.vl = vl;
    pr.vu = vu;
    pr.range = range;
    apply_tune(pr, o, nullptr, 0);
    int64_t kwork = n;
    pr.ck_base = 0;
    pr.ck_stride = n;
    if (range == MRRR_RANGE_INDEX) {
        // work: the wanted indices and a guard on each side; checkpoint
        // columns: one per output column
        const int64_t k0 = std::max<int64_t>(il - 1, 1), k1 = std::min<int64_t>(iu + 1, n);
        kwork = k1 - k0 + 1;
        pr.ck_stride = iu - il + 1;
    }
    const int workers = workers_for(h, o);
    int status = MRRR_OK;
    double scale = o.arena_scale;
    for (int attempt = 0; attempt < 4; ++attempt) {
        Sizes sz = base_sizes(n, 1, kwork, n, scale);
        sz.ck = o.jobz ? kCkSlots * ((n + kCkb - 1) / kCkb) * pr.ck_stride : 1;
        Params P{};
        P.d = d;
        P.e = e ? e : d;
        P.w = w;
        P.Z = Z;
        P.nprob = 1;
        if (prepare(h->ws, sz, P) != hipSuccess) return MRRR_ENOMEM;
        set_options(P, o, h->wall_khz, workers, io_eps);
        if (hipMemcpyAsync(P.probs, &pr, sizeof(Problem), hipMemcpyHostToDevice, h->stream) != hipSuccess)
            return MRRR_EHIP;
        if (hipEventRecord(h->ev0, h->stream) != hipSuccess) return MRRR_EHIP;
        hipEvent_t evt[2] = {h->evt0, h->evt1};
        if (enqueue_solve(P, n, o.sign_convention != 0, h->stream, evt) != hipSuccess) return MRRR_EHIP;
        if (hipEventRecord(h->ev1, h->stream) != hipSuccess) return MRRR_EHIP;
        Ctl c{};
        std::vector<Problem> ph(1);
        if ((status = read_back(h, P, &c, &ph)) != MRRR_OK) return status;
        float ms = 0.f, tms = 0.f;
        (void)hipEventElapsedTime(&ms, h->ev0, h->ev1);
        (void)hipEventElapsedTime(&tms, h->evt0, h->evt1);
        status = map_device_error(c.error);
        if (status == MRRR_ENOMEM && attempt < 3) {
            scale *= 8.0;   // grow the node pool and retry
            continue;
        }
        *m = ph[0].m;
        fill_stats(stats, c, ph[0].m, ms, tms);
        if (status == MRRR_OK && still_unverified(c) > 0) status = MRRR_WARN_UNVERIFIED;
        break;
    }
    return status;
}

}  // namespace

extern "C" int mrrr_dstemr(mrrr_handle_t h, int64_t n, const double* d, const double* e, int range,
                           double vl, double vu, int64_t il, int64_t iu, const mrrr_options_t* opts,
                           int64_t* m, double* w, double* Z, int64_t ldz, mrrr_stats_t* stats) {
    mrrr_options_t o;
    mrrr_default_options(&o);
    if (opts) o = *opts;
    const int bad = check_single(h, n, d, e, range, vl, vu, il, iu, o, m, w, Z, ldz);
    if (bad != MRRR_OK) return bad;
    *m = 0;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (n == 0 || (range == MRRR_RANGE_INDEX && iu < il)) return MRRR_OK;
    if (hipSetDevice(h->device) != hipSuccess) return MRRR_EHIP;
    return solve_single(h, n, d, e, range, vl, vu, il, iu, o, 0.0, m, w, Z, ldz, stats);
}

extern "C" void mrrr_default_options_mixed(mrrr_options_t* o) {
    if (!o) return;
    mrrr_default_options(o);
    o->gaptol = 1e-5;            // Sec. 5.2.1: fixed at 1e-5 for single/double
    o->rtol_class = 1e-7;        // 1e-2 gaptol, for the first bisection and the refinements
    o->perturb_xi = 0x1p29;      // xi = eps_single = 2^-24 = 2^29 eps_double
}

extern "C" int mrrr_sstemr(mrrr_handle_t h, int64_t n, const float* d, const float* e, int range, float vl,
                           float vu, int64_t il, int64_t iu, const mrrr_options_t* opts, int64_t* m, float* w,
                           float* Z, int64_t ldz, mrrr_stats_t* stats) {
    mrrr_options_t o;
    mrrr_default_options_mixed(&o);
    if (opts) o = *opts;
    const int bad = check_single(h, n, d, e, range, (double)vl, (double)vu, il, iu, o, m, w, Z, ldz);
    if (bad != MRRR_OK) return bad;
    *m = 0;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (n == 0 || (range == MRRR_RANGE_INDEX && iu < il)) return MRRR_OK;
    if (hipSetDevice(h->device) != hipSuccess) return MRRR_EHIP;
    // FP64 working copies: d, e (n each), w (n), Z (n x kmax, ld n)
    const int64_t kmax = (range == MRRR_RANGE_INDEX) ? iu - il + 1 : n;
    const size_t need = sizeof(double) * (3 * (size_t)n + (o.jobz ? (size_t)n * (size_t)kmax : 0));
    if (h->mixed.ensure(need) != hipSuccess) return MRRR_ENOMEM;
    double* d64 = h->mixed.as<double>();
    double* e64 = d64 + n;
    double* w64 = e64 + n;
    double* Z64 = o.jobz ? w64 + n : nullptr;
    if (launch_widen(d, d64, n, h->stream) != hipSuccess) return MRRR_EHIP;
    if (n > 1 && launch_widen(e, e64, n - 1, h->stream) != hipSuccess) return MRRR_EHIP;
    const int st = solve_single(h, n, d64, e64, range, (double)vl, (double)vu, il, iu, o, 0x1p-24, m, w64, Z64,
                                std::max<int64_t>(n, 1), stats);
    if (st != MRRR_OK && st != MRRR_WARN_UNVERIFIED) return st;
    const int64_t mm = *m;
    if (mm > 0) {
        if (launch_narrow(w64, 1, w, 1, mm, 1, h->stream) != hipSuccess) return MRRR_EHIP;
        if (o.jobz && launch_narrow(Z64, n, Z, ldz, n, mm, h->stream) != hipSuccess) return MRRR_EHIP;
    }
    return st;
}

// ------------------------------------------------------------ dense driver

extern "C" int mrrr_dsyevr(mrrr_handle_t h, int64_t n, const double* A, int64_t lda, int range, double vl, double vu,
                           int64_t il, int64_t iu, const mrrr_options_t* opts, int64_t* m, double* w, double* Z,
                           int64_t ldz, mrrr_stats_t* stats) {
    if (!h) return -1;
    if (n < 0 || n > (int64_t)INT32_MAX / 2) return -2;
    if (n > 0 && !A) return -3;
    if (lda < std::max<int64_t>(1, n)) return -4;
    mrrr_options_t o;
    mrrr_default_options(&o);
    if (opts) o = *opts;
    // A and lda take the argument positions of d and e; the others are
    // checked as mrrr_dstemr checks them
    const int bad = check_single(h, n, A, A, range, vl, vu, il, iu, o, m, w, Z, ldz);
    if (bad != MRRR_OK) return bad;
    *m = 0;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (n == 0 || (range == MRRR_RANGE_INDEX && iu < il)) return MRRR_OK;
    if (hipSetDevice(h->device) != hipSuccess) return MRRR_EHIP;
    if (!h->rb && rocblas_create_handle(&h->rb) != rocblas_status_success) {
        h->rb = nullptr;
        return MRRR_EHIP;
    }
    if (rocblas_set_stream(h->rb, h->stream) != rocblas_status_success) return MRRR_EHIP;
    // workspace: the reduced matrix (its lower triangle holds the Householder
    // vectors of Q), the tridiagonal's d and e, and the reflectors' scalars
    const size_t nn = (size_t)n * (size_t)n;
    if (h->dense.ensure(sizeof(double) * (nn + 3 * (size_t)n)) != hipSuccess) return MRRR_ENOMEM;
    double* Aw = h->dense.as<double>();
    double* dd = Aw + nn;
    double* ee = dd + n;
    double* tau = ee + n;
    if (hipMemcpy2DAsync(Aw, sizeof(double) * (size_t)n, A, sizeof(double) * (size_t)lda, sizeof(double) * (size_t)n,
                         (size_t)n, hipMemcpyDeviceToDevice, h->stream) != hipSuccess)
        return MRRR_EHIP;
    // 1. A = Q T Q^T (Householder reduction of the lower triangle)
    if (rocsolver_dsytrd(h->rb, rocblas_fill_lower, (rocblas_int)n, Aw, (rocblas_int)n, dd, ee, tau) !=
        rocblas_status_success)
        return MRRR_EHIP;
    // 2. eigenpairs of T by MRRR (the sign convention waits for the vectors of A)
    mrrr_options_t ot = o;
    ot.sign_convention = 0;
    const int st = solve_single(h, n, dd, ee, range, vl, vu, il, iu, ot, 0.0, m, w, Z, ldz, stats);
    if (st != MRRR_OK && st != MRRR_WARN_UNVERIFIED) return st;
    const int64_t mm = *m;
    if (o.jobz && mm > 0) {
        // 3. Z := Q Z
        if (rocsolver_dormtr(h->rb, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none, (rocblas_int)n,
                             (rocblas_int)mm, Aw, (rocblas_int)n, tau, Z, (rocblas_int)ldz) != rocblas_status_success)
            return MRRR_EHIP;
        if (o.sign_convention) {
            // the problem record of the solve still describes Z (n rows, mm
            // columns, leading dimension ldz)
            Params P{};
            P.probs = h->ws.probs.as<Problem>();
            P.nprob = 1;
            P.Z = Z;
            P.ctl = h->ws.ctl.as<Ctl>();
            if (launch_sign(P, mm, h->stream) != hipSuccess) return MRRR_EHIP;
        }
    }
    if (hipStreamSynchronize(h->stream) != hipSuccess) return MRRR_EHIP;
    return st;
}

// ------------------------------------------------------------------ batched

namespace {

int build_plan(mrrr_handle_t h, mrrr_batched_plan_s* pl) {
    const int64_t batch = pl->batch;
    const int64_t rows = pl->noff[batch];
    int64_t nmax = 0, zpack = 0, ck = 0;
    pl->probs.assign((size_t)batch, Problem{});
    for (int64_t b = 0; b < batch; ++b) {
        const int64_t nb = pl->noff[b + 1] - pl->noff[b];
        nmax = std::max(nmax, nb);
        Problem& pr = pl->probs[(size_t)b];
        pr.row0 = pl->noff[b];
        pr.n = nb;
        pr.zoff = pl->zoff.empty() ? zpack : pl->zoff[(size_t)b];
        pr.ldz = std::max<int64_t>(1, nb);
        pr.woff = pl->noff[b];
        pr.il = 1;
        pr.iu = nb;
        pr.range = MRRR_RANGE_ALL;
        apply_tune(pr, pl->opts, pl->tune.empty() ? nullptr : pl->tune.data(), b);
        pr.ck_base = ck;
        pr.ck_stride = nb;
        ck += pl->opts.jobz ? kCkSlots * ((nb + kCkb - 1) / kCkb) * nb : 0;
        zpack += nb * nb;
    }
    Sizes sz = base_sizes(rows, batch, rows, nmax, pl->opts.arena_scale);
    // each block's root and clusters draw 4 n_b + kNodeExtra doubles; budget by sum n_b
    double arena = 0.0;
    for (int64_t b = 0; b < batch; ++b) {
        const double nb = (double)(pl->noff[b + 1] - pl->noff[b]);
        arena += (4.0 * nb + (double)kNodeExtra) * std::min(nb + 2.0, 64.0 + nb / 4.0);
    }
    sz.arena = (uint64_t)std::max(arena * std::max(pl->opts.arena_scale, 1e-3), 1024.0);
    sz.ck = std::max<int64_t>(ck, 1);
    pl->sz = sz;
    Params P{};
    P.d = pl->d;
    P.e = pl->e;
    P.w = pl->w;
    P.Z = pl->Z;
    P.nprob = (int32_t)batch;
    if (prepare(pl->ws, sz, P) != hipSuccess) return MRRR_ENOMEM;
    set_options(P, pl->opts, h->wall_khz, workers_for(h, pl->opts));
    if (hipMemcpy(P.probs, pl->probs.data(), sizeof(Problem) * (size_t)batch, hipMemcpyHostToDevice) != hipSuccess)
        return MRRR_EHIP;
    pl->P = P;
    // capture init -> setup -> tree -> finalize -> sign as one graph
    hipStream_t cs = nullptr;
    if (hipStreamCreate(&cs) != hipSuccess) return MRRR_EHIP;
    int st = MRRR_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) st = MRRR_EHIP;
    if (st == MRRR_OK && enqueue_solve(P, rows, pl->opts.sign_convention != 0, cs) != hipSuccess) st = MRRR_EHIP;
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(cs, &g) != hipSuccess) st = MRRR_EHIP;
    (void)hipStreamDestroy(cs);
    if (st != MRRR_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    pl->graph = g;
    if (hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0) != hipSuccess) return MRRR_EHIP;
    return MRRR_OK;
}

bool same_plan(const mrrr_batched_plan_s* pl, int64_t batch, const int64_t* noff, const int64_t* zoff,
               const mrrr_options_t& o, const double* d, const double* e, double* w, double* Z) {
    if (!pl || pl->batch != batch) return false;
    mrrr_options_t a = pl->opts, b = o;
    a.tune = nullptr;   // the table is compared by content below
    b.tune = nullptr;
    if (std::memcmp(&a, &b, sizeof(a)) != 0) return false;
    if ((o.tune == nullptr) != pl->tune.empty()) return false;
    if (o.tune && std::memcmp(pl->tune.data(), o.tune, sizeof(int32_t) * 3 * (size_t)batch) != 0) return false;
    if (pl->d != d || pl->e != e || pl->w != w || pl->Z != Z) return false;
    if (std::memcmp(pl->noff.data(), noff, sizeof(int64_t) * (size_t)(batch + 1)) != 0) return false;
    if ((zoff == nullptr) != pl->zoff.empty()) return false;
    if (zoff && std::memcmp(pl->zoff.data(), zoff, sizeof(int64_t) * (size_t)batch) != 0) return false;
    return true;
}

}  // namespace

extern "C" int mrrr_dstemr_batched(mrrr_handle_t h, int64_t batch, const int64_t* n_offsets,
                                   const double* d_cat, const double* e_cat, const int64_t* z_offsets,
                                   const mrrr_options_t* opts, double* w_cat, double* Z_cat,
                                   mrrr_stats_t* stats) {
    if (!h) return -1;
    if (batch < 0 || batch > (1 << 24)) return -2;
    if (batch > 0 && !n_offsets) return -3;
    if (batch > 0 && n_offsets[0] != 0) return -3;
    for (int64_t b = 0; b < batch; ++b)
        if (n_offsets[b + 1] < n_offsets[b]) return -3;
    const int64_t rows = batch > 0 ? n_offsets[batch] : 0;
    if (rows > (int64_t)INT32_MAX / 2) return -3;
    if (z_offsets)
        for (int64_t b = 0; b < batch; ++b)
            if (z_offsets[b] < 0) return -6;
    if (rows > 0 && !d_cat) return -4;
    if (rows > 0 && !e_cat) return -5;
    mrrr_options_t o;
    mrrr_default_options(&o);
    if (opts) o = *opts;
    if (check_options(o)) return -7;
    if (rows > 0 && !w_cat) return -8;
    if (o.jobz && rows > 0 && !Z_cat) return -9;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (rows == 0) return MRRR_OK;
    if (hipSetDevice(h->device) != hipSuccess) return MRRR_EHIP;
    double scale = o.arena_scale;
    for (int attempt = 0; attempt < 4; ++attempt) {
        mrrr_options_t oo = o;
        oo.arena_scale = scale;
        if (!same_plan(h->plan, batch, n_offsets, z_offsets, oo, d_cat, e_cat, w_cat, Z_cat)) {
            if (h->plan) { h->plan->release(); delete h->plan; h->plan = nullptr; }
            auto* pl = new (std::nothrow) mrrr_batched_plan_s;
            if (!pl) return MRRR_ENOMEM;
            pl->batch = batch;
            pl->noff.assign(n_offsets, n_offsets + batch + 1);
            if (z_offsets) pl->zoff.assign(z_offsets, z_offsets + batch);
            if (oo.tune) pl->tune.assign(oo.tune, oo.tune + 3 * batch);
            pl->opts = oo;
            pl->opts.tune = nullptr;   // never kept: the caller owns the table
            pl->d = d_cat;
            pl->e = e_cat;
            pl->w = w_cat;
            pl->Z = Z_cat;
            const int st = build_plan(h, pl);
            if (st != MRRR_OK) { pl->release(); delete pl; return st; }
            h->plan = pl;
        }
        mrrr_batched_plan_s* pl = h->plan;
        if (hipEventRecord(h->ev0, h->stream) != hipSuccess) return MRRR_EHIP;
        if (hipGraphLaunch(pl->exec, h->stream) != hipSuccess) return MRRR_EHIP;
        if (hipEventRecord(h->ev1, h->stream) != hipSuccess) return MRRR_EHIP;
        Ctl c{};
        int st = read_back(h, pl->P, &c, nullptr);
        if (st != MRRR_OK) return st;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, h->ev0, h->ev1);
        st = map_device_error(c.error);
        if (st == MRRR_ENOMEM && attempt < 3) {
            scale *= 8.0;
            continue;
        }
        fill_stats(stats, c, rows, ms);
        if (st == MRRR_OK && still_unverified(c) > 0) st = MRRR_WARN_UNVERIFIED;
        return st;
    }
    return MRRR_ENOMEM;
}

// ----------------------------------------------------------------- backward

namespace {
void* adj_alloc(void* ctx, size_t bytes) {
    DevBuf* b = static_cast<DevBuf*>(ctx);
    if (b->ensure(bytes) != hipSuccess) return nullptr;
    return b->p;
}
}  // namespace

extern "C" int mrrr_dstemr_backward(mrrr_handle_t h, int64_t n, const double* w, const double* Z,
                                    int64_t ldz, const double* wbar, const double* Zbar, int64_t ldzbar,
                                    double gap_mask_rel, double* dbar, double* ebar, int64_t* n_masked) {
    if (!h) return -1;
    if (n < 0 || n > (int64_t)INT32_MAX / 2) return -2;
    if (n > 0 && !w) return -3;
    if (n > 0 && !Z) return -4;
    if (ldz < std::max<int64_t>(1, n)) return -5;
    if (Zbar && ldzbar < std::max<int64_t>(1, n)) return -8;
    if (!(gap_mask_rel >= 0.0)) return -9;
    if (n > 0 && !dbar) return -10;
    if (n > 1 && !ebar) return -11;
    if (n_masked) *n_masked = 0;
    if (n == 0) return MRRR_OK;
    if (hipSetDevice(h->device) != hipSuccess) return MRRR_EHIP;
    const int64_t noff[2] = {0, n};
    return adjoint_run(h->stream, 1, noff, nullptr, w, Z, wbar, Zbar, gap_mask_rel, dbar, ebar, n_masked, ldz,
                       ldzbar, adj_alloc, &h->adj);
}

extern "C" int mrrr_dstemr_backward_noalloc(mrrr_handle_t h, int64_t n, const double* w, const double* Z,
                                            int64_t ldz, const double* wbar, const double* Zbar, int64_t ldzbar,
                                            double gap_mask_rel, double* dbar, double* ebar, int64_t* n_masked) {
    if (!h) return -1;
    if (n < 0 || n > (int64_t)INT32_MAX / 2) return -2;
    if (Zbar && n > MRRR_BACKWARD_NOALLOC_MAX_N) return -2;
    if (n > 0 && !w) return -3;
    if (n > 0 && !Z) return -4;
    if (ldz < std::max<int64_t>(1, n)) return -5;
    if (Zbar && ldzbar < std::max<int64_t>(1, n)) return -8;
    if (!(gap_mask_rel >= 0.0)) return -9;
    if (n > 0 && !dbar) return -10;
    if (n > 1 && !ebar) return -11;
    if (n_masked) *n_masked = 0;
    if (n == 0) return MRRR_OK;
    if (!h->na_scratch) return MRRR_EHIP;
    if (hipSetDevice(h->device) != hipSuccess) return MRRR_EHIP;
    return adjoint_run_noalloc(h->stream, h->na_scratch, n, w, Z, ldz, wbar, Zbar, ldzbar, gap_mask_rel, dbar, ebar,
                               n_masked);
}

extern "C" int mrrr_dstemr_backward_batched(mrrr_handle_t h, int64_t batch, const int64_t* n_offsets,
                                            const double* w_cat, const double* Z_cat, const int64_t* z_offsets,
                                            const double* wbar_cat, const double* Zbar_cat, double gap_mask_rel,
                                            double* dbar_cat, double* ebar_cat, int64_t* n_masked) {
    if (!h) return -1;
    if (batch < 0 || batch > (1 << 24)) return -2;
    if (batch > 0 && (!n_offsets || n_offsets[0] != 0)) return -3;
    for (int64_t b = 0; b < batch; ++b)
        if (n_offsets[b + 1] < n_offsets[b]) return -3;
    const int64_t rows = batch > 0 ? n_offsets[batch] : 0;
    if (rows > 0 && !w_cat) return -4;
    if (rows > 0 && !Z_cat) return -5;
    if (z_offsets)
        for (int64_t b = 0; b < batch; ++b)
            if (z_offsets[b] < 0) return -6;
    if (!(gap_mask_rel >= 0.0)) return -9;
    if (rows > 0 && !dbar_cat) return -10;
    if (rows > 0 && !ebar_cat) return -11;
    if (n_masked) *n_masked = 0;
    if (rows == 0) return MRRR_OK;
    if (hipSetDevice(h->device) != hipSuccess) return MRRR_EHIP;
    return adjoint_run(h->stream, batch, n_offsets, z_offsets, w_cat, Z_cat, wbar_cat, Zbar_cat, gap_mask_rel,
                       dbar_cat, ebar_cat, n_masked, -1, -1, adj_alloc, &h->adj);
}

// ---------------------------------------------------------------- diagnostics

extern "C" int mrrr_diag_quotient(mrrr_handle_t h, int64_t n, const double* a, const double* b, double* q) {
    if (!h) return -1;
    if (n < 0 || n > ((int64_t)1 << 40)) return -2;
    if (n > 0 && !a) return -3;
    if (n > 0 && !b) return -4;
    if (n > 0 && !q) return -5;
    if (n == 0) return MRRR_OK;
    if (hipSetDevice(h->device) != hipSuccess) return MRRR_EHIP;
    if (launch_quot(a, b, q, n, h->stream) != hipSuccess) return MRRR_EHIP;
    return MRRR_OK;
}
