// Types shared by the kernels (pw_kernels.hip) and the host runtime (pw_host.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

namespace pw {

// One query as the device sees it (Algorithm 1 inputs and parameters).
struct QueryDesc {
    int32_t s, t;       // internal (storage) ids of the endpoints
    int32_t L;
    uint32_t uid;
    uint32_t K, R, B, G;
    uint32_t slot;      // row of the block-sum / done / result tables
    uint32_t seed_lo, seed_hi;  // 64-bit Philox key of this query
    uint32_t psum_base; // first per-probe accumulator of a query whose probes are split
    uint32_t share;     // walk-sharing group size M (1 = every probe has its own walks)
};

// A work-group chunk: replicas [p0, p0 + pc) of the walk-sharing groups
// [g0, g0 + gc) of query q, which hold probes [k0, k0 + kc). Groups number
// ceil(B/M) per block: group j of block b holds probes bB + jM .. up to M of
// them, never past the block. Either pc == R (whole groups), or gc == 1 and
// the group's replicas are split over several chunks whose partial sums meet
// in per-probe accumulators. With M = 1 a group is a probe (g0 = k0).
struct Chunk {
    uint32_t q;
    uint32_t k0;
    uint32_t kc;
    uint32_t p0;
    uint32_t pc;
    uint32_t g0;
    uint32_t gc;
    uint32_t pad;
};

struct DomainParams {
    uint32_t n, rb, mask, rsh, A, A8;
};

struct GraphTables {
    const uint4* node;
    const uint32_t* col;
    const uint4* adj;
    const uint32_t* rp;
    const uint32_t* col24;
    const uint2* node8;
    DomainParams dom;
};

// A finished query as posted by the work group that completed it.
struct Completion {
    uint32_t slot;
    uint32_t pad;
    double beta;
};

// Arguments of one walk launch.
struct WalkArgs {
    GraphTables g;
    const QueryDesc* qd;
    const Chunk* chunks;
    uint32_t nchunks;
    uint32_t gdim;                  // G (blocks per query) of this launch
    uint32_t* cursor;               // work-stealing cursor (persistent launches)
    unsigned long long* blocksum;   // [slot][G][2] int128 block sums of trunc(Q 2^64)
    uint32_t* done;                 // [slot] probes finished
    unsigned long long* psum;       // [probe][4] exact S1, S2 of split probes
    uint32_t* pcount;               // [probe] replicas finished of split probes
    double* beta;                   // [slot] results
    double* q_debug;                // optional: [K] per-probe Q of the (single) query
    double* ybar_debug;             // optional: [G] block means
    uint32_t* comp_count;           // optional (served mode): completions posted so far
    Completion* comp_ring;          // optional: ring of (slot, beta) completions
    uint32_t comp_cap;
    uint32_t recycle;               // clear a finished query's block sums and counter
    uint32_t persistent;
    // Persistent launches: the chunk table is cut into nqueues segments
    // [qoff[i], qoff[i+1]), each with its own cursor cursor[i]. A work group
    // starts on the queue of the XCD it runs on and moves to the next queue
    // when that one is empty, so chunks of one query share an XCD's L2.
    uint32_t nqueues;
    uint32_t qoff[9];
    // Optional abort flag in host memory mapped for the device (a watchdog on
    // the host sets it): a work group reads it before each chunk and, once it
    // is nonzero, takes no further chunk.
    const uint32_t* abort_flag;
};

// Largest walk-sharing group the kernels are built for.
constexpr uint32_t kMaxShare = 4;
// Kernel instance for a sharing factor M: 1, 2 or 4 probes per walk.
inline int share_class(uint32_t M) { return M <= 1 ? 1 : M <= 2 ? 2 : 4; }

constexpr int kBlockThreads = 256;
// Work-group size of the walk and gather kernels per layout code and walk
// sharing class. With one probe per walk the hubs-first layouts (codes 3, 4
// and 5) stage the node entries of the 8,192 highest-degree nodes (64 KB; the
// 16,384 row offsets with the probe on storage ids, code 5) in LDS
// once per 1,024-thread work group: two groups per CU keep 8 waves per SIMD
// within the 160 KB of LDS, and the staged nodes take 42% of the steps on a
// Chung-Lu n=1e5 graph (1,024 nodes per 256-thread group take 18%). The
// sharing kernels run 4-5 waves per SIMD, one such group per CU, and keep
// 256-thread groups with 1,024 staged nodes.
constexpr int block_threads(int layout, int share)
{
    return (layout == 3 || layout == 4 || layout == 5) && share <= 1 ? 1024 : kBlockThreads;
}
constexpr uint32_t kMaxQueues = 8;      // one chunk queue per XCD
constexpr int kMaxChunkProbes = 256;
constexpr int kMaxG = 128;
// Probes with at least this many replicas are run one probe per wave block
// (wave-uniform probe keys); fewer replicas use the per-lane mapping.
constexpr uint32_t kUniformMinR = 48;
// Batched and served launches split a probe whose R exceeds this many replicas
// into chunks of at most this size (a multiple of 64).
constexpr uint32_t kSplitReplicas = 4096;

// Launchers (defined in pw_kernels.hip). All return hipError_t of the launch.
// uniform: every chunk of the launch has R >= kUniformMinR.
// layout: 0 CSR, 1 fat, 2 compact.
hipError_t launch_walk(const WalkArgs& a, int layout, int uniform, int share, uint32_t grid, hipStream_t st);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_trace(const GraphTables& g, int layout, uint32_t count, const int32_t* start,
                        const uint32_t* uid, const uint32_t* k, const uint32_t* p,
                        const uint32_t* side, int32_t L, uint32_t seed_lo, uint32_t seed_hi,
                        int32_t* trace, float* acc, hipStream_t st);
hipError_t launch_probe_eval(const GraphTables& g, uint32_t seed_lo, uint32_t seed_hi, uint32_t uid,
                             uint32_t k, uint32_t count, const uint32_t* nodes, uint32_t* pi,
                             int8_t* z, hipStream_t st);
hipError_t build_fat_adjacency(const uint4* node, const uint32_t* col, uint4* adj, uint32_t nnz,
                               hipStream_t st);
// Gather-roofline microbenchmark: `chains` in {1, 2, 4, 8} chains per lane.
hipError_t launch_gather(const GraphTables& g, int layout, int chains, uint32_t grid, int32_t steps, uint32_t seed,
                         uint32_t* sink, hipStream_t st);
// Binary64 truncated series and spectral helpers (row offsets rp[0..n], and
// either col (32-bit ids) or col24 (packed 3-byte ids)).
hipError_t launch_spmv_step(const uint32_t* rp, const uint32_t* col, const uint32_t* col24, uint32_t n, uint32_t Q,
                            const double* V, double* Y, double* H, hipStream_t st);
hipError_t launch_colsum(const double* H, uint32_t n, uint32_t Q, double* sq, double* lin, hipStream_t st);
// v_0 = D^{-1} b_st columns (Q <= 64): entries s[q] = vs[q], t[q] = vt[q] of V and H,
// which the caller has zeroed.
hipError_t launch_series_seed(const uint32_t* s, const uint32_t* t, const double* vs, const double* vt, uint32_t Q,
                              double* V, double* H, hipStream_t st);
// Power iteration for lambda, all on the device: phi, x, y, z are n doubles,
// part 2 * 1024 doubles, scal 2 doubles; the estimate ends in scal[1].
hipError_t launch_lambda(const uint32_t* rp, const uint32_t* col, const uint32_t* col24, uint32_t n, uint32_t nnz,
                         int32_t iters, uint64_t seed, double* phi, double* x, double* y, double* z, double* part,
                         double* scal, hipStream_t st);
// Work groups of the walk kernel that fit on the device at once.
int walk_occupancy(int layout, int uniform, int share, int* wgs_per_cu);

// Bytes of the fixed device scratch array (pw_scratch.hip).
constexpr size_t kScratchBytes = size_t(64) << 20;
// Device address of `device`'s scratch array (resolved on first use, with that
// device current) and that device's scratch lock, held by *held on success.
int scratch_acquire(int device, void** base, std::unique_lock<std::mutex>* held);

}  // namespace pw
