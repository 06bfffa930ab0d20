/*
 * probewalk.h -- C ABI of the MI355X (gfx950) ProbeWalk library.
 *
 * ProbeWalk (Zheng & Zhang, arXiv 2512.05460) estimates the squared
 * biharmonic distance beta(s,t) = b_st^T (L^+)^2 b_st (Definition 2.1) of a
 * connected undirected graph under a relative-error target eps (Problem 2.2)
 * with Algorithm 1: K = B*G Paired-Sign Probes (Definition 3.1, generated on
 * the fly as in section 3.3), R replicas of two length-L walks per probe
 * (section 3.2, eq. for phi-hat), the U-statistic Q_R (Lemma 3.4) and the
 * median of G block means.
 *
 * Conventions shared by every entry point
 *   - Every function returns an int status: BD_OK (0) or a negative BD_E_*
 *     code. Nothing throws across the ABI. bd_strerror() names a code.
 *   - Pointers documented as "host" are ordinary host memory, borrowed for
 *     the duration of the call only; the library keeps no reference to them.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream). The
 *     calls enqueue work on it and synchronise it before they return, except
 *     where stated.
 *   - Device memory. The library holds the device memory of the graph tables,
 *     the per-graph work buffers (grown on demand) and the server arenas, and
 *     frees it in graph_free / bd_server_destroy. It takes that memory from
 *     the allocator installed with bd_set_allocator (for example PyTorch's
 *     caching allocator), else from hipMalloc; each buffer is returned to the
 *     allocator it came from. Inputs are never retained: graph_load_csr
 *     copies the caller's CSR (host arrays, or device arrays with
 *     BD_DEVICE_PTRS) into tables of its own.
 *   - Random streams depend only on (seed, uid, k, p, side, step): a query's
 *     result is bit-identical whatever batch, mode, chunking or server
 *     traffic it runs in.
 *   - Limits: 2 <= n <= 2^30, nnz < 2^31, max degree < 2^24, L <= 16383,
 *     K and R < 2^32.
 *   - Threads: calls on different graphs may run concurrently. The calls that
 *     use a graph's work buffers (bd_query_batch, bd_query_probes,
 *     bd_query_stabilized, bd_autotune, bd_truncated_beta, bd_graph_lambda)
 *     take that graph's lock and run one at a time; the validation entry
 *     points and servers have buffers of their own and run beside them.
 *     graph_free must not race with any other call on the graph.
 *   - Walk sharing (bd_policy.share > 1) is an extension of Algorithm 1;
 *     every other result follows the algorithm as the paper states it, with
 *     the readings fixed where the paper leaves freedom written out in the
 *     oracle's sources.
 */
#ifndef PROBEWALK_H
#define PROBEWALK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define BD_OK          0
#define BD_E_INVALID  -1  /* bad argument; per query: s == t, s or t out of range,
                             eps outside (0,1), L < 0 or L > 16383 */
#define BD_E_GRAPH    -2  /* graph is not simple, symmetric, sorted and connected */
#define BD_E_RANGE    -3  /* n, nnz or a degree beyond the limits above */
#define BD_E_BUDGET   -4  /* per query: walk steps (2*K*R*L without walk sharing) above the
                             policy cap, or K, R >= 2^32 */
#define BD_E_HIP      -5  /* a HIP runtime call failed */
#define BD_E_NOMEM    -6  /* device or host allocation failed */
#define BD_E_NODEVICE -7  /* no usable gfx950 device */
#define BD_E_NOTFOUND -8  /* unknown server request id */
#define BD_E_FULL     -9  /* server admission refused: request exceeds the caps */
#define BD_E_CANCELLED -10 /* server destroyed before the request finished */
#define BD_E_TIMEOUT  -11 /* bd_server_wait timed out (the request is still running); per
                             query: abandoned at the bd_exec deadline */
#define BD_E_SCRATCH  -12 /* bd_query_batch_noalloc: the batch needs more than the fixed
                             scratch array holds (BD_NOALLOC_SCRATCH_BYTES) */

/* ---- graph --------------------------------------------------------------- */
typedef struct bd_graph bd_graph;

/* graph_load_csr flags */
#define BD_LAYOUT_CSR       0u  /* node table {offset, degree, 1/degree} + neighbour ids:
                                   two dependent gathers per walk step */
#define BD_LAYOUT_FAT       1u  /* adds 16-byte adjacency entries {neighbour, its offset,
                                   its degree, its 1/degree}: one gather per walk step */
#define BD_SKIP_VALIDATION  2u  /* trust the caller: skip the symmetry, sortedness and
                                   connectivity checks (ranges are still checked) */
#define BD_RELABEL_DEGREE   4u  /* store nodes in descending-degree order (locality of the
                                   node table); ids at the ABI, neighbour order and every
                                   result are unchanged */
#define BD_LAYOUT_COMPACT   8u  /* 32-bit row offsets + 3-byte neighbour ids, 1/degree
                                   recomputed: the smallest footprint (n <= 2^24; not with
                                   BD_LAYOUT_FAT). With BD_RELABEL_DEGREE: 8-byte node
                                   entries {row offset, original id} in descending-degree
                                   order, the 8192 highest-degree ones staged in LDS by
                                   every work group (1024 in the walk-sharing kernels)
                                   (layout code 3); above 2^24 nodes the neighbour ids
                                   take 4 bytes (layout code 4) */
#define BD_WIDE_IDS        16u  /* with BD_LAYOUT_COMPACT | BD_RELABEL_DEGREE: 4-byte
                                   neighbour ids (layout code 4) at any n */
#define BD_PROBE_STORAGE_IDS 128u /* with BD_LAYOUT_COMPACT | BD_RELABEL_DEGREE (n <= 2^24; not
                                   with BD_WIDE_IDS): the probe is evaluated on the storage id,
                                   the node's rank in descending degree (ties by id), instead
                                   of the caller's id. Algorithm 1 on the relabelled graph:
                                   rows keep the caller's neighbour order, so the walks are
                                   the same, and a uniformly random probe composed with a
                                   fixed relabelling is again one, but the bits of every
                                   result follow the relabelled ids. A node entry is its
                                   4-byte row offset, and the walk kernels read every node's
                                   row offset and degree from LDS where the degree-run table
                                   fits (BD_DIRECT_HUBS). bd_walk_trace still reports caller
                                   ids */
#define BD_NONTEMPORAL    256u  /* with BD_LAYOUT_FAT: read the adjacency entries with
                                   non-temporal loads at any size (same results) */
#define BD_TEMPORAL       512u  /* with BD_LAYOUT_FAT: ordinary loads at any size. Without
                                   either flag the fat layout uses non-temporal loads when
                                   its tables take at least 4 GiB (16x the Infinity Cache:
                                   measured +9.5% at 20.7 GB, -3.5% at 2.2 GB) */
/* Kernels of the BD_PROBE_STORAGE_IDS layout (same tables, same results). By
 * default the walks resolve every node in LDS through the degree-run table:
 * the row offsets of the first h1 storage ids, past which every block of
 * storage ids holds nodes of at most two degrees (runs, in descending-degree
 * order), each at most 2,047, then one 8-byte record per block (64 to 512
 * storage ids, the smallest that fits) and 1/d for every degree; a walk step
 * then makes one global load instead of two (on the Chung-Lu n=1e5 graph
 * h1 = 1,571 and 22 KB). Where the table fits 64 KB two 1,024-thread work
 * groups per CU run one replica pair per thread (layout code 9); where it
 * fits 144 KB one group per CU runs two pairs per thread (code 8); else one
 * group per CU stages the row offsets of the 36,864 highest-degree nodes
 * (code 7). The flags below force a choice. */
#define BD_NARROW_HUBS   1024u  /* two work groups per CU, one pair per thread: the table
                                   where it fits 64 KB (code 9), else the 16,384
                                   highest-degree row offsets (code 5) */
#define BD_DIRECT_HUBS   2048u  /* no degree-run table: the highest-degree row offsets
                                   (code 7; code 5 with BD_NARROW_HUBS) */
#define BD_WIDE_HUBS     4096u  /* one work group per CU, two pairs per thread: the table
                                   where it fits 144 KB (code 8), else code 7. Not with
                                   BD_NARROW_HUBS */
#define BD_DEVICE_PTRS     64u  /* row_ptr and col_idx are device pointers on the current
                                   device (e.g. the data of PyTorch tensors) instead of host
                                   arrays; they are read once, on `stream`, and not kept.
                                   BD_E_INVALID if either is not device memory of the
                                   current device */
#define BD_LAYOUT_AUTO     32u  /* the library picks: BD_LAYOUT_COMPACT | BD_RELABEL_DEGREE
                                   when those tables take at most 12 MiB (measured
                                   crossover), else BD_LAYOUT_FAT (with BD_RELABEL_DEGREE only if
                                   given). Not with BD_LAYOUT_FAT, BD_LAYOUT_COMPACT or
                                   BD_WIDE_IDS (BD_E_INVALID). bd_graph_get_info reports
                                   the choice */

typedef struct {
    int64_t  n, nnz;
    int32_t  d_min, d_max;
    int32_t  bipartite;      /* 1 if the graph is bipartite (section 2.1 assumes not;
                                the estimator still targets beta^(L)) */
    int32_t  layout;         /* 0 CSR, 1 fat, 2 compact, 3 compact with hubs first,
                                4 hubs first with 4-byte neighbour ids, 5 hubs first with
                                the probe on storage ids */
    int64_t  device_bytes;   /* device memory held by the graph tables */
    int32_t  nontemporal;    /* 1 if the fat layout reads its entries with non-temporal loads */
    int32_t  lds_hubs;       /* nodes whose row offset and degree the walk kernels with one
                                probe per walk read from LDS (0 = none; n with the
                                degree-run table) */
} bd_graph_info;

/*
 * Load a graph (section 2.1: connected, undirected, simple) and keep it
 * resident on the current device.
 *   n        number of nodes.
 *   row_ptr  n+1 int64 offsets (host, or device with BD_DEVICE_PTRS),
 *            row_ptr[0] = 0, nondecreasing.
 *   col_idx  row_ptr[n] int32 neighbour ids (host, or device with
 *            BD_DEVICE_PTRS); each row ascending, no self-loops, no repeats,
 *            and the adjacency symmetric. The order of
 *            a row is part of the contract: the walk's neighbour index j
 *            selects col_idx[row_ptr[x] + j].
 *   flags    BD_LAYOUT_* | BD_RELABEL_DEGREE | BD_WIDE_IDS | BD_SKIP_VALIDATION |
 *            BD_DEVICE_PTRS | BD_PROBE_STORAGE_IDS | BD_NONTEMPORAL | BD_TEMPORAL.
 *   out      receives the handle; release with graph_free.
 * Errors: BD_E_GRAPH if a check fails (disconnected, asymmetric, unsorted,
 * self-loop), BD_E_RANGE for sizes beyond the limits, BD_E_INVALID for
 * conflicting layout flags, BD_E_NOMEM, BD_E_HIP.
 */
int  graph_load_csr(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                    uint32_t flags, void* stream, bd_graph** out);

/*
 * Device allocator of the library's buffers. alloc returns `bytes` of device
 * memory of the current device (NULL on failure, reported as BD_E_NOMEM);
 * free returns a pointer alloc gave, with its size. `stream` is passed as
 * NULL: the library synchronises its own work on a buffer before freeing it.
 * ctx is passed back unchanged. Both functions may be called from any thread
 * that calls into the library (not from the server's scheduler thread, which
 * allocates nothing).
 */
typedef struct {
    void* ctx;
    void* (*alloc)(void* ctx, size_t bytes, void* stream);
    void  (*free)(void* ctx, void* ptr, size_t bytes, void* stream);
} bd_allocator;

/*
 * Install the allocator for every device buffer allocated from now on (graph
 * tables, work buffers, server arenas, temporaries of the validation and
 * reference entry points); NULL restores hipMalloc/hipFree. Buffers already
 * allocated keep the allocator they came from, which must stay usable until
 * they are freed. BD_E_INVALID if a is not NULL and a function is missing.
 */
int  bd_set_allocator(const bd_allocator* a);

void graph_free(bd_graph* g);
int  bd_graph_get_info(const bd_graph* g, bd_graph_info* info);

/* ---- walk-count policy (Algorithm 1 parameters, Theorem 3.8) --------------- */
#define BD_POLICY_PAPER  0  /* B = ceil(448/eps^2), R = ceil(128 (L+1)^2 / (d_min^2 (1-eps/2) (1/d_s+1/d_t)^2)) */
#define BD_POLICY_SCALED 1  /* the same formulas with c_B, c_R in place of 448, 128 */
#define BD_POLICY_FIXED  2  /* B = B_fixed, R = R_fixed */

typedef struct {
    int32_t  kind;
    double   c_B, c_R;       /* BD_POLICY_SCALED */
    double   delta;          /* failure probability; G = ceil(8 ln(1/delta)); 0 -> 0.01 */
    int64_t  B_fixed, R_fixed;
    uint64_t max_steps_per_query;  /* 0 = no cap; a query above it gets BD_E_BUDGET */
    int32_t  share;          /* walk sharing, an extension of Algorithm 1 (0 or 1 = off,
                                at most 4): the probes of each median-of-means block are
                                taken in groups of `share` consecutive probes scored on
                                one set of R walk pairs, whose random streams are keyed
                                by the group's first probe. Groups never cross a block,
                                so the G block means stay independent and each Q_k stays
                                unbiased; walk steps drop by about that factor. */
} bd_policy;

typedef struct {
    double   beta;           /* beta-hat^(L)(s,t), binary64 */
    int64_t  K, R;           /* probes and replicas per probe */
    int32_t  B, G, L;
    int32_t  status;         /* BD_OK, BD_E_INVALID or BD_E_BUDGET for this query */
    int64_t  walk_steps;     /* 2*R*L transitions per walk pair, K*R pairs (G*ceil(B/share)*R
                                with walk sharing); saturates at INT64_MAX */
} bd_result;

/*
 * Plan only (Algorithm 1 parameters). Fills K, R, B, G, L, walk_steps and
 * status of out[0..nq); beta is set to 0. No device work. pol may be NULL
 * (BD_POLICY_PAPER, delta = 0.01).
 */
int bd_plan(const bd_graph* g, int64_t nq, const int32_t* s, const int32_t* t,
            const double* eps, const int32_t* L, const bd_policy* pol, bd_result* out);

/* ---- execution ------------------------------------------------------------ */
#define BD_MODE_PLAIN    0u  /* one query per launch, fixed tiling */
#define BD_MODE_BATCHED  1u  /* all queries in one persistent launch with work stealing */

typedef struct {
    uint32_t mode;
    int32_t  chunk_probes;   /* probes per work-group chunk; 0 = from chunk_pairs */
    int32_t  grid_wgs;       /* persistent grid size (BATCHED); 0 = resident capacity */
    int32_t  use_graph;      /* BATCHED: replay a captured hipGraph of the launch (work buffers
                                are reused; the graph is rebuilt when the batch shape changes) */
    int32_t  chunk_pairs;    /* (probe, replica) pairs per chunk, also the replica-part size of
                                a split probe (BATCHED); 0 = one per work-group thread (PLAIN:
                                256, or 2048 on the hubs-first layouts with two pairs per
                                thread, but at most the probes that give each compute unit a
                                chunk) / 4096 (BATCHED) */
    int32_t  queues;         /* BATCHED: chunk queues of the persistent launch, 1..8. A query's
                                chunks stay in one queue and a work group takes chunks from the
                                queue of the XCD it runs on before the others, so they share
                                that XCD's L2. 0 = 8. Results do not depend on it. */
    int32_t  uniform_min_r;  /* BATCHED: queries with at least this many replicas run on the
                                wave-uniform kernel (one probe per wave, probe keys in scalar
                                registers), the others on the general kernel (lanes over
                                (probe, replica) pairs). 0 = automatic: 48, and the general
                                kernel for all when the wave-uniform chunks could not fill
                                the device; < 0 = general kernel only. Results do not
                                depend on it. */
    double   deadline_ms;    /* > 0: a watchdog on the calling thread raises an abort flag
                                once the call has run this long; the walk kernels read it
                                before each chunk and take no further chunk, and queries
                                that had not finished get status BD_E_TIMEOUT (beta 0); the
                                finished ones keep their results, bit-identical to an
                                unbounded call. Ignored by bd_query_batch_noalloc.
                                0 = no deadline. */
} bd_exec;

typedef struct {
    double   walk_kernel_ms; /* summed HIP-event time of the walk kernel launches */
    double   total_ms;       /* wall time of the call */
    int64_t  launches;       /* walk kernel launches */
    int64_t  chunks;         /* work-group chunks processed */
    int64_t  walk_steps;     /* transitions executed (valid queries) */
    int64_t  walk_pairs;     /* (k, p) pairs executed */
} bd_stats;

/*
 * Estimate beta(s,t) for nq queries (Algorithm 1 for each).
 *   s, t, eps, L   host arrays of nq entries.
 *   uid            host array of nq query ids for the random streams, or
 *                  NULL for uid[i] = i. uid < 2^31.
 *   seed           64-bit Philox key.
 *   pol            walk-count policy (NULL = paper constants).
 *   exec           execution mode (NULL = BD_MODE_BATCHED, automatic sizes).
 *   out            host, nq results (caller-allocated).
 *   stats          host, optional (may be NULL).
 * Returns BD_OK when the batch ran; per-query failures are reported in
 * out[i].status and leave the other queries unaffected.
 */
int bd_query_batch(bd_graph* g, int64_t nq, const int32_t* s, const int32_t* t,
                   const double* eps, const int32_t* L, const uint32_t* uid,
                   uint64_t seed, const bd_policy* pol, const bd_exec* exec,
                   void* stream, bd_result* out, bd_stats* stats);

/*
 * For callers that cannot allocate device memory (code under hipGraph capture,
 * serving loops that must not call hipMalloc, harnesses that forbid it): the
 * same computation as bd_query_batch, bit for bit, with every work buffer
 * (query descriptors, chunk table, block sums, counters, split-probe
 * accumulators, results) carved out of a fixed device array of
 * BD_NOALLOC_SCRATCH_BYTES that the library holds on each device from the
 * time it is loaded there until the process ends. The call allocates no
 * device memory and creates no events or streams; the caller still passes its
 * inputs and outputs in host memory and the graph stays as loaded.
 *   Arguments, results and errors as bd_query_batch, and additionally:
 *   - BD_E_SCRATCH when the batch's buffers exceed the array (about 650 bytes
 *     per query plus 32 per chunk, and 36 per probe of queries whose probes
 *     are split in batched mode); nothing runs then;
 *   - BD_E_INVALID when the current device is not the graph's;
 *   - exec->use_graph is ignored (no hipGraph), and stats->walk_kernel_ms is
 *     0 (no timing events); the other stats are filled.
 * The array is shared by every call on a device and keeps the last call's
 * contents; each call clears the parts that must start at zero. Calls on one
 * device take a process-wide lock for the array and run one at a time: two
 * calls overlapping on one device would otherwise race on it.
 */
#define BD_NOALLOC_SCRATCH_BYTES (64u << 20)
int bd_query_batch_noalloc(bd_graph* g, int64_t nq, const int32_t* s, const int32_t* t,
                           const double* eps, const int32_t* L, const uint32_t* uid,
                           uint64_t seed, const bd_policy* pol, const bd_exec* exec,
                           void* stream, bd_result* out, bd_stats* stats);

/*
 * The truncated distance beta^(L)(s,t) = ||h||^2 - (1^T h)^2 / n with
 * h = sum_{i=0..L} P^i D^{-1} b_st (Lemma 2.3), in binary64 on the device by
 * L sparse products (the paper's PUSH series; a deterministic reference for
 * the estimator, which is unbiased for beta^(L) by Lemma 3.3).
 *   beta_L  host, nq doubles.
 * Up to 64 queries share one pass: three n x Q binary64 blocks (the series
 * term, the next term, the running sum), fewer queries per pass when those
 * would take more than half of the free device memory.
 */
int bd_truncated_beta(bd_graph* g, int64_t nq, const int32_t* s, const int32_t* t, int32_t L,
                      void* stream, double* beta_L);

/*
 * The mixing factor lambda = max(|lambda_2|, |lambda_n|) of P = D^{-1} A
 * (section 2.1), estimated by `iters` power iterations on D^{-1/2} A D^{-1/2}
 * (same spectrum) with the stationary direction projected out; the estimate
 * is ||N x|| for the unit iterate x, which converges to lambda from below.
 * The iteration runs on the device (four n-vectors of binary64, the start
 * vector a counter-based function of seed); only the estimate is copied back.
 */
int bd_graph_lambda(bd_graph* g, int32_t iters, uint64_t seed, void* stream, double* lambda);

/*
 * Truncation length of Theorem 3.8 (Algorithm 1, first line):
 * L = ceil(log(96 n / (eps (1-lambda)^2 (1/d_s + 1/d_t)^2)) / log(1/lambda)).
 * Host-only. BD_E_RANGE unless 0 < lambda < 1 (a bipartite graph has lambda = 1);
 * values above 16383 are reported as 16384.
 */
int bd_theorem_L(const bd_graph* g, int64_t nq, const int32_t* s, const int32_t* t, const double* eps,
                 double lambda, int32_t* L);

/*
 * Truncation length by the stabilization rule (section 4.3): starting at
 * L = L0 = 1, estimate at L and 2L; accept L_stop = 2L and beta-hat^(2L) when
 * |beta-hat^(2L) - beta-hat^(L)| <= (eps/2) |beta-hat^(2L)|, else double L.
 * Doubling stops at L_max (out[i] is then the estimate at L_max and
 * L_stop[i] = L_max). Each round runs every still-unstopped query in one
 * batched launch; estimates at a given L are the same as bd_query_batch's.
 *   L_max   cap on L (1 <= L_max <= 16383).
 *   L_stop  host, nq int32 (the accepted truncation length per query).
 * Other arguments as bd_query_batch (eps[] is the relative-error target).
 */
int bd_query_stabilized(bd_graph* g, int64_t nq, const int32_t* s, const int32_t* t,
                        const double* eps, int32_t L_max, const uint32_t* uid, uint64_t seed,
                        const bd_policy* pol, const bd_exec* exec, void* stream,
                        bd_result* out, int32_t* L_stop);

/*
 * Autotuner: runs the (small, representative) sample batch once per candidate
 * execution configuration and returns the fastest by walk-kernel time in *best:
 * chunk_pairs in {128, 256, ..., 16384} with 8 chunk queues, then (BATCHED)
 * the best of those with 1 queue. times_ms (host, may be NULL) receives the
 * kernel time of each of the n_candidates (<= 16) candidates in that order;
 * *n_candidates is set to the count.
 */
int bd_autotune(bd_graph* g, int64_t nq, const int32_t* s, const int32_t* t, const double* eps,
                const int32_t* L, uint64_t seed, const bd_policy* pol, uint32_t mode, void* stream,
                bd_exec* best, double* times_ms, int32_t* n_candidates);

/* ---- validation entry points (expose intermediate values for parity tests) -- */

/*
 * Node sequences X_0..X_L of `count` walks (the walk step of the production
 * kernels, section 3.2) and their binary32 sums of z/d.
 *   start, uid, k, p, side  host arrays of `count` entries (side 0 = s-walk,
 *                           1 = t-walk; selects the random stream).
 *   trace                   host, count*(L+1) int32, row-major; may be NULL.
 *   acc                     host, count floats; may be NULL.
 */
int bd_walk_trace(bd_graph* g, int64_t count, const int32_t* start, const uint32_t* uid,
                  const uint32_t* k, const uint32_t* p, const uint32_t* side, int32_t L,
                  uint64_t seed, void* stream, int32_t* trace, float* acc);

/*
 * pi_k(x) and z^(k)_x (section 3.3 stateless generator) for `count` nodes.
 *   nodes  host, count uint32 node ids (< n).
 *   pi     host, count uint32 (may be NULL); z host, count int8 (may be NULL).
 */
int bd_probe_eval(bd_graph* g, uint64_t seed, uint32_t uid, uint32_t k, int64_t count,
                  const uint32_t* nodes, void* stream, uint32_t* pi, int8_t* z);

/*
 * One query with its intermediate values: the K per-probe statistics Q_k
 * (Alg. 1 Q_R(z^(k))) and the G block means. q_out (K doubles) and ybar_out
 * (G doubles) are host arrays sized from bd_plan; either may be NULL.
 */
int bd_query_probes(bd_graph* g, int32_t s, int32_t t, double eps, int32_t L, uint32_t uid,
                    uint64_t seed, const bd_policy* pol, const bd_exec* exec, void* stream,
                    double* q_out, double* ybar_out, bd_result* out);

/* ---- measurement -------------------------------------------------------------- */
typedef struct {
    double  ms;               /* kernel time (HIP events) */
    double  steps_per_s;      /* transitions per second */
    double  gathers_per_s;    /* dependent loads per second (2 per step, or 1 with BD_LAYOUT_FAT) */
    int64_t steps;            /* transitions executed */
    int32_t chains_per_lane;
    int32_t work_groups;
} bd_roofline;

/*
 * Random-gather roofline of the loaded graph (measurement for section 3.2's walk
 * loop): lanes run `chains_per_lane` (1, 2, 4 or 8) independent chains of
 * `steps` transitions with exactly the walk kernel's dependent loads on the
 * same tables, but a cheap xorshift instead of Philox and no probe arithmetic.
 * work_groups = 0 picks 4x the resident capacity.
 */
int bd_gather_roofline(bd_graph* g, int32_t chains_per_lane, int32_t steps, int32_t work_groups,
                       void* stream, bd_roofline* out);

/* ---- served mode: continuous batching ---------------------------------------- */
typedef struct bd_server bd_server;

typedef struct {
    bd_policy policy;
    int64_t   max_queries_inflight;   /* admission cap on resident queries (0 = 65536) */
    uint64_t  max_steps_inflight;     /* admission cap on outstanding walk steps (0 = none) */
    int32_t   chunk_probes;           /* 0 = automatic */
    double    slice_ms;               /* least device time per scheduling slice (0 = 20); a slice
                                         also lasts at least four times its longest chunk */
    double    small_first;            /* share of each slice's work given first to the requests
                                         with the fewest walk steps left, smallest first (the rest
                                         is round-robin over requests): 0 = 0.5, < 0 = none */
} bd_server_cfg;

/*
 * Create a server over a loaded graph. The server owns a host scheduler thread
 * and device streams; requests submitted while others run are admitted at
 * the next slice boundary as capacity frees up, and their chunks share the
 * device with the running ones (part of each slice to the requests with the
 * least work left, the rest round-robin over requests; chunks of at most one
 * work group's pairs, so that no chunk holds a slice open for long). The
 * graph must outlive the server.
 */
int  bd_server_create(bd_graph* g, const bd_server_cfg* cfg, bd_server** out);
/* Submit nq queries (host arrays, copied). Returns a request id. BD_E_FULL if
 * the request alone exceeds the admission caps. uid as in bd_query_batch. */
int  bd_server_submit(bd_server* srv, int64_t nq, const int32_t* s, const int32_t* t,
                      const double* eps, const int32_t* L, const uint32_t* uid,
                      uint64_t seed, uint64_t* request_id);
/* Non-blocking poll: *done = 1 and out[0..nq) filled when the request finished. */
int  bd_server_poll(bd_server* srv, uint64_t request_id, bd_result* out, int* done,
                    double* latency_ms);
/* Block until the request finishes (timeout_ms <= 0: no timeout). */
int  bd_server_wait(bd_server* srv, uint64_t request_id, double timeout_ms, bd_result* out,
                    double* latency_ms);
/*
 * Cancel a request (failure handling of a serving loop: a client gone, a
 * deadline missed). A request still queued for admission is finished at once;
 * an admitted one gets no further chunk: the chunks already launched run to
 * their end (each is bounded work), then the slots of its unfinished queries
 * are cleared and freed for other requests. Its queries that finished before
 * keep their results; the others get status BD_E_CANCELLED (beta 0). Poll or
 * wait for the request as usual to collect it. BD_OK also when it had already
 * finished or been cancelled; BD_E_NOTFOUND for an unknown (or collected) id.
 */
int  bd_server_cancel(bd_server* srv, uint64_t request_id);
void bd_server_destroy(bd_server* srv);

/* ---- misc ------------------------------------------------------------------ */
const char* bd_strerror(int code);
/* Writes a one-line description of the current device into buf. */
int bd_device_info(char* buf, size_t len);

#ifdef __cplusplus
}
#endif

#endif /* PROBEWALK_H */
