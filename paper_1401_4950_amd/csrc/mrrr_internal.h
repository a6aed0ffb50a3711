// Internal data layout shared by the host runtime and the gfx950 kernels.
//
// One solve works on P "problems" (1 for mrrr_dstemr, B for the batched
// form).  Each problem is split into irreducible blocks (Sec. 3.2.1); each
// block gets a root representation and a tree of cluster representations
// (the representation tree of Sec. 3.1.2), processed as device tasks drawn
// from three queues (Sec. 4.1: refinement > cluster > singleton priority).
//
// Indexing: every eigenvalue of every block owns one "slot", its global row
// index row0(block) + j - 1 for the block-local index j (1-based).  Slots
// index the bracket arrays lo/hi/gap and the checkpoint rows.
#pragma once

#include <stdint.h>

namespace mrrr {

constexpr int kWave = 64;      // wavefront = one worker
constexpr int kTile = 64;      // rows of a representation staged in LDS at once
constexpr int kCkb = 16;       // rows between checkpoints of the twisted solver
constexpr int kCkSlots = 6;    // doubles per checkpoint and eigenvalue
constexpr int kNumQ = 3;       // 0: refine, 1: root + cluster, 2: singleton
// node pool doubles per representation of an n-row block: 4 n + kNodeExtra
// (D and L; the shift selection's two checkpoint arrays of n + 64; the block
// of the cooperative end refinement)
constexpr int64_t kNodeExtra = 1024;
constexpr int kQRefine = 0, kQCluster = 1, kQSingle = 2;

enum TaskType : int32_t {
    kTaskRoot = 1,     // build the root RRR of a block and start its refinement
    kTaskRefine = 2,   // refine a slice of one node's eigenvalue brackets
    kTaskCluster = 3,  // new RRR for a cluster (Alg. 3.8), then refine its members
    kTaskSingle = 4,   // bundle of singletons of one node (Alg. 4.3 + Alg. 3.7)
    kTaskHelp = 5,     // idle worker lending its lanes to a cluster's end refinement
    kTaskAssist = 6    // idle worker sharing a singleton bundle's passes
};

enum RefineMode : int32_t { kModeClass = 0, kModeFull = 1 };

enum ErrCode : int32_t {
    kErrNone = 0, kErrNoMem = 2, kErrNoConv = 3,
    kErrTimeout = 6, kErrInternal = 7,
    kErrBadD = 100, kErrBadE = 101   // non-finite input data
};

struct Task {
    int32_t type;
    int32_t node;   // node id (root: block id)
    int32_t a;      // first member (local index) or singleton-list offset
    int32_t b;      // last member (inclusive) or count; refine: mode in bit 30
};

struct Problem {
    int64_t row0;     // first row in d/e and first slot
    int64_t n;
    int64_t zoff;     // element offset of this problem's Z block
    int64_t ldz;
    int64_t woff;     // element offset of this problem's w
    int64_t il, iu;   // requested indices (INDEX range)
    double vl, vu;    // requested values (VALUE range)
    int32_t range;
    int32_t nblocks;  // device: number of irreducible blocks
    int64_t m;        // device: number of eigenpairs returned
    double bnorm;     // device: Gershgorin bound of the whole problem
    int64_t ck_base;  // checkpoint region (doubles) of this problem
    int64_t ck_stride;  // checkpoint columns: one per output column
    int32_t flags;    // device: bit0 several blocks; bit1 columns to permute
    int16_t lanes;    // most multisection lanes per eigenvalue (power of two)
    int16_t bundle;   // singletons per S-task
    int32_t slice_max;  // largest refinement slice
    int32_t pad;
    double tscale;    // device: the tree works on tscale * T (a power of two)
    double tscale_inv;
};

struct Block {
    int32_t prob;
    int32_t root;     // node id of the root representation (-1 = none)
    int64_t row0;     // global first row
    int64_t n;
    int64_t k0, k1;   // working local indices (wanted plus one guard each side)
    int64_t w0, w1;   // wanted local indices, 1-based inclusive
    int64_t col0;     // output column of local index w0 within the problem
};

struct Node {
    int64_t data;     // arena offset: D at data, L at data+n (N-representation)
    int32_t block;
    int32_t depth;
    int32_t a, b;     // member local indices, inclusive
    int32_t parent;
    int32_t pending;  // refinement slices still running
    double sigma;     // accumulated shift: lambda(T) = sigma + lambda(node)
    double lgap, rgap;  // absolute gaps to the neighbours outside [a, b]
    double spdiam;    // spectral diameter of the block's root
    double checked;   // nonzero: the columns of this node or of an ancestor
                      // are checked for orthogonality after the tree
    double share;     // workers its refinement slices may occupy: at a root the
                      // block's share of the launch, at a child its parent's
                      // share times its part of the parent's clustered members
    int32_t clustered;  // members in clusters, written by its classification
    int32_t pad;
};

// Columns of a cluster whose representation passed no element-growth test
// (Alg. 3.8, last resort), checked for orthogonality after the tree and
// re-orthogonalised when it is lost (remark (6) on the shift selection of
// Sec. 3.2.3: check the accuracy of the cluster's eigenpairs).
constexpr int kCheckMax = 64;   // widest cluster that is checked (columns)
struct CheckRec {
    int64_t z;        // offset in Z of the first column, at the block's first row
    int64_t ldz;
    int64_t n;        // rows of the block
    int64_t m;        // columns, 2..kCheckMax
    double loss[2];   // max |Z^T Z - I| found by the two passes (written on the device)
    int64_t pad[2];
};

// Representations that passed no element-growth test, checked after the tree
// for conditional element growth (Sec. 3.1.2, Definition of conditional
// element growth; the test of remark (3) on Alg. 3.8) against the computed
// eigenvectors of their wanted members.
constexpr int64_t kGrowthSample = 512;   // most member columns checked per representation
struct GrowthRec {
    int64_t rep;      // arena offset of D+ (L+ follows at rep + n)
    int64_t z;        // offset in Z of the first wanted member's column, at the block's first row
    int64_t ldz;
    int64_t n;        // rows of the block
    int64_t m;        // wanted member columns
    int64_t mc;       // columns checked: all m, or kGrowthSample spread evenly (both ends included)
    int64_t col0;     // device: first column of this record in the flattened list (prefix sum)
    double bound;     // the largest acceptable || |L+||D+||L+^T| |z| || / ||z||
    double spdiam;    // spectral diameter of the block's root (the same frame)
    int32_t flag;     // device: 1 once a column exceeded the bound
    int32_t pad;
};

// Words that many workers hit (queue heads and tails, the pending count, the
// error flag) each sit on a 256-byte line of their own, so that polling one
// does not contend with updates of another.
constexpr int kLineU64 = 32;

struct Ctl {
    uint64_t head_[kNumQ * kLineU64];   // head of queue q at head_[q * kLineU64]
    uint64_t tail_[kNumQ * kLineU64];
    int64_t avail_[kNumQ * kLineU64];  // published tasks no consumer has claimed yet
    int64_t pending;      // tasks pushed and not yet finished
    int64_t pad_p[kLineU64 - 1];
    int32_t error;        // first error code raised on the device
    int32_t dmax;
    int64_t pad_e[kLineU64 - 1];
    uint64_t arena_top;   // doubles handed out from the node arena
    int32_t node_top;
    int32_t pad2;
    int64_t slist_top;
    int64_t pad_a[kLineU64 - 3];
    int64_t n_nodes, largest_cluster, n_unverified, n_fallback, n_nan;
    int64_t qd_steps, n_tasks, n_single, n_rqi, n_blocks;
    int64_t trace_top;
    int64_t n_sturm;
    int64_t chk_top;      // records in Params::chk
    int64_t n_checked, n_repaired, n_check_failed;
    int64_t n_check_wide; // unverified clusters too wide to be checked themselves
    int64_t grw_top;      // records in Params::grw
    int64_t n_grw_failed; // of those, representations with a column above the bound
    uint64_t grw_max;     // largest ratio || |L||D||L^T| |z| || / (||z|| spdiam) seen (bits of a double)
    int64_t grw_cols;     // columns in all records (after the prefix sum)
    int64_t n_fac_quot;   // shift selections redone in quotient form
#ifdef __HIPCC__
    __device__ __host__ uint64_t* head(int q) { return head_ + q * kLineU64; }
    __device__ __host__ uint64_t* tail(int q) { return tail_ + q * kLineU64; }
    __device__ __host__ int64_t* avail(int q) { return avail_ + q * kLineU64; }
#endif
};

struct TraceRec {       // mirrors mrrr_trace_t
    int32_t type, worker, node, depth, a, b;
    int64_t t0, t1;
    double x0, x1;
    int32_t flags, child;
};

struct Params {
    const double* d;
    const double* e;
    double* w;
    double* Z;
    Problem* probs;
    int32_t nprob;
    int32_t jobz;
    Block* blocks;        // problem p's blocks live at blocks[row0(p) + b]
    Node* nodes;
    int32_t max_nodes;
    int32_t nworkers;
    Task* q[kNumQ];
    uint64_t* seq[kNumQ];
    uint64_t qcap[kNumQ];
    double* lo;           // per slot bracket, in the frame of its current node
    double* hi;
    double* gap;          // per slot absolute gap (singletons)
    double* lo0;          // per slot bracket as the current node received it
    double* hi0;          //   (a deterministic snapshot for neighbour tests)
    uint8_t* vflag;       // per slot: bit0 lo verified, bit1 hi verified
    uint8_t* need;        // per slot: bits its bracket must still shrink by (slicing)
    int32_t* slist;       // singleton lists
    int64_t slist_cap;
    double* arena;
    uint64_t arena_cap;   // doubles
    double* ck;           // checkpoints of the twisted solver
    double* colbuf;       // 2 doubles per slot: sort keys of the final merge
    int32_t* perm;        // 2 per slot: column order of the final merge
    Ctl* ctl;
    int64_t total_rows;
    double gaptol, rtol, xi;
    uint64_t seed;
    int32_t max_rqi, max_tries, max_depth, slice_min, sign_conv;
    int32_t assist;       // singleton bundles may take a helper (same results)
    int32_t coop;         // idle workers may share refinement passes (same results)
    uint64_t timeout_ticks;
    TraceRec* trace;
    int64_t trace_cap;
    CheckRec* chk;        // clusters checked after the tree (see CheckRec)
    int64_t chk_cap;
    double check_tol;     // correct when max |Z^T Z - I| > check_tol n eps
    double io_eps;        // unit roundoff of the caller's data format when it is
                          // coarser than FP64 (single/double: 2^-24), else 0
    GrowthRec* grw;       // representations checked for conditional element growth
    int64_t grw_cap;
    double cond_k;        // k_elg of that check; 0: no check
};

}  // namespace mrrr
