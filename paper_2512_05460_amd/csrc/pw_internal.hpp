// Types shared by the kernels (pw_kernels.hip) and the host runtime (pw_host.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "pw_runs.hpp"

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
    const uint32_t* runtab;  // code 8: rp[0 .. run_h1], then the run records (run_words words)
    uint32_t run_h1, run_words, run_ninv;  // run_ninv: d_max + 1 reciprocals
    uint32_t run_shift;                    // log2 of the storage ids per run record
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

// Layout codes of the kernels (0-5 are the graph layouts bd_graph_get_info
// reports; 6 is a kernel variant of layout 1, 7 and 8 of layout 5), and the hub
// nodes they stage in LDS.
constexpr int kLayoutCsr = 0, kLayoutFat = 1, kLayoutCompact = 2, kLayoutCompactHub = 3, kLayoutHub32 = 4,
              kLayoutHubId = 5;
// The fat layout read with non-temporal loads (the same tables and results):
// for tables far larger than the Infinity Cache, where every step misses it
// anyway and keeping the entries out of the caches' replacement order leaves
// them to the node entries of the walks' start nodes.
constexpr int kLayoutFatNT = 6;
// Layout 5's tables with one 1,024-thread work group per CU: 36,864 hub row
// offsets (144 KB of LDS) and two replica pairs per lane, so four dependent
// load chains per lane keep as many loads in flight at four waves per SIMD as
// two chains at eight.
constexpr int kLayoutHubIdX2 = 7;
// Layout 5's tables with the row offset and degree of every node resolved in
// LDS, so that a walk step issues one global load (the neighbour id) instead
// of two. Storage order is descending degree: the first h1 storage ids (the
// high-degree nodes, whose degrees are nearly all distinct) keep their row
// offsets; past h1 the degrees form runs of equal value at least as long as
// a block (2^shift storage ids, shift from kRunShiftMin to kRunShiftMax: the
// smallest whose table fits), so each block holds at most two runs and one
// 8-byte record describes it: {row offset of its first node,
// dA | dB << 11 | bnd << 22}, its nodes before bnd having degree dA and the
// rest dB. After the table the LDS holds 1.0f/d for d = 0 .. d_max, so a step
// reads the reciprocal instead of dividing. The launch shape is code 7's; the
// results are layout 5's. The walk-sharing kernels (256-thread groups) hold a
// smaller copy (kRunWordsShared words); where the table does not fit it,
// walk sharing runs code 7's kernels on these tables (run_kernel).
constexpr int kLayoutHubRuns = 8;  // constants and builder: pw_runs.hpp
// The same table in two 1,024-thread work groups per CU, one replica pair per
// thread, 8 waves per SIMD (the table in at most 64 KB: BD_NARROW_HUBS).
constexpr int kLayoutHubRunsNarrow = 9;
constexpr bool runs_layout(int layout) { return layout == kLayoutHubRuns || layout == kLayoutHubRunsNarrow; }
// LDS words of the run table and reciprocals in the walk-sharing kernels of
// code 8 (24 KB: with their other LDS, four such groups per CU)
constexpr uint32_t kRunWordsShared = 6144;
constexpr bool hubid_layout(int layout)
{
    return layout == kLayoutHubId || layout == kLayoutHubIdX2 || runs_layout(layout);
}
// replica pairs a lane runs at once
constexpr int lane_pairs(int layout) { return layout == kLayoutHubIdX2 || layout == kLayoutHubRuns ? 2 : 1; }
constexpr bool hub_layout(int layout)
{
    return layout == kLayoutCompactHub || layout == kLayoutHub32 || hubid_layout(layout);
}
// hub entries staged per work group (64 KB in 1,024-thread groups, 8 KB in
// 256-thread ones): 8,192 / 1,024 node entries of 8 bytes, or 16,384 / 2,048
// row offsets of 4 bytes with the probe on storage ids; 36,864 offsets in the
// one-group-per-CU kernel of code 7
constexpr uint32_t hub_nodes(int threads, int layout)
{
    if (layout == kLayoutHubIdX2 && threads >= 1024) return 36864u;  // 144 KB: what the CU's 160 KB leaves
    // code 8: capacity in 32-bit words of the run table and the reciprocals
    if (layout == kLayoutHubRuns) return threads >= 1024 ? 36864u : kRunWordsShared - 1u;
    if (layout == kLayoutHubRunsNarrow) return threads >= 1024 ? 16383u : kRunWordsShared - 1u;
    return (threads >= 1024 ? 8192u : 1024u) * (layout == kLayoutHubIdX2 ? 4u : layout == kLayoutHubId ? 2u : 1u);
}
// 32-bit words of the LDS hub copy (entries 0 .. hub_nodes, inclusive)
constexpr uint32_t hub_words(int threads, int layout)
{
    return !hub_layout(layout) ? 2u : hubid_layout(layout) ? hub_nodes(threads, layout) + 1u
                                                            : 2u * (hub_nodes(threads, layout) + 1u);
}

constexpr int kBlockThreads = 256;
// Work-group size of the walk and gather kernels per layout code and walk
// sharing class. With one probe per walk the hubs-first kernels (codes 3, 4, 5,
// 7 and 8) run 1,024-thread work groups: codes 3 and 4 stage the node entries
// of the 8,192 highest-degree nodes (64 KB), code 5 their 16,384 row offsets,
// two groups per CU at 8 waves per SIMD; code 7 stages 36,864 offsets (144 KB)
// in one group per CU at 4 waves per SIMD with two replica pairs per thread,
// and code 8 the run table in the same shape. On the Chung-Lu n=1e5 graph the
// nodes resolved in LDS take 42%, 54%, 73% and 100% of the walk steps. The
// sharing kernels run 4-5 waves per SIMD, one such group per CU, and keep
// 256-thread groups.
constexpr int block_threads(int layout, int share) { return hub_layout(layout) && share <= 1 ? 1024 : kBlockThreads; }
// (probe, replica) pairs one work group runs at once: a pair per thread, two
// per thread in the kernels of layout codes 7 and 8
constexpr int group_pairs(int layout, int share)
{
    return block_threads(layout, share) * (share <= 1 ? lane_pairs(layout) : 1);
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
