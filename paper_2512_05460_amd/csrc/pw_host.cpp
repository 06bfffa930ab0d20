// Host runtime and C ABI of the ProbeWalk library: graph loading and
// validation, the walk-count planner (Algorithm 1 parameters), the plain and
// batched launchers, validation entry points and the served mode.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "probewalk.h"
#include "pw_internal.hpp"

using namespace pw;

namespace {

constexpr int64_t kMaxN = int64_t(1) << 30;
constexpr int64_t kMaxNnz = (int64_t(1) << 31) - 1;
constexpr int32_t kMaxDeg = (1 << 24) - 1;
constexpr int32_t kMaxL = 16383;
// BD_LAYOUT_AUTO: up to this size of hubs-first compact tables their two
// short requests per step, mostly L2 hits with 42% of the node reads from
// LDS, beat the fat layout's one 16-byte request into a 4.5x larger table;
// beyond it the misses dominate and fat wins. Measured on Chung-Lu graphs of
// mean degree 10: with 7.2 MiB of tables hubs first ran 1.40x fat, with
// 14.4 MiB 0.89x.
constexpr int64_t kAutoCompactBytes = int64_t(12) << 20;
// The fat layout switches to non-temporal loads of its adjacency entries when
// its tables exceed 16 times the 256 MB Infinity Cache: measured +9.5% walk
// steps/s with 20.7 GB of tables (Chung-Lu n=4e7), -3.5% with 2.2 GB (n=1e7)
// and -46% with 192 MB (the grid, whose locality lives in the caches).
constexpr int64_t kFatNontemporalBytes = int64_t(4) << 30;

#define HIP_TRY(expr)                                  \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return BD_E_HIP;         \
    } while (0)

// The process-wide device allocator (bd_set_allocator): hipMalloc/hipFree
// unless the caller installed its own.
std::mutex g_alloc_mu;
bd_allocator g_alloc{};

bd_allocator current_allocator()
{
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc;
}

// Device allocation owned by the library, released through the allocator it
// came from.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bd_allocator al{};
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) {
            if (al.free) al.free(al.ctx, p, bytes, nullptr);
            else (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
    }
    int alloc(size_t b)
    {
        release();
        if (b == 0) b = 16;
        b = (b + 255) & ~(size_t)255;
        al = current_allocator();
        if (al.alloc) {
            p = al.alloc(al.ctx, b, nullptr);
            if (!p) return BD_E_NOMEM;
        } else if (hipMalloc(&p, b) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return BD_E_NOMEM;
        }
        bytes = b;
        return BD_OK;
    }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// Work buffers of bd_query_batch, kept with the graph and grown on demand, and
// the captured hipGraph of the last batched launch shape.
struct Workspace {
    DevBuf qd, chunks, bs, done, beta, cursor, psum, pcount, qdbg, ydbg;
    hipStream_t gstream = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<uint64_t> gkey;
    int64_t graph_builds = 0, graph_replays = 0;
    // the watchdog's abort flag: host memory mapped for the device
    uint32_t* abort_host = nullptr;
    uint32_t* abort_dev = nullptr;
    int ensure(DevBuf& b, size_t bytes)
    {
        if (b.p && b.bytes >= bytes) return BD_OK;
        return b.alloc(std::max(bytes, 2 * b.bytes));
    }
    int ensure_abort_flag()
    {
        if (abort_host) return BD_OK;
        void* h = nullptr;
        if (hipHostMalloc(&h, 64, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
            (void)hipGetLastError();
            return BD_E_NOMEM;
        }
        void* d = nullptr;
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipHostFree(h);
            return BD_E_HIP;
        }
        abort_host = static_cast<uint32_t*>(h);
        abort_dev = static_cast<uint32_t*>(d);
        __atomic_store_n(abort_host, 0u, __ATOMIC_SEQ_CST);
        return BD_OK;
    }
    ~Workspace()
    {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (gstream) (void)hipStreamDestroy(gstream);
        if (abort_host) (void)hipHostFree(abort_host);
    }
};

struct bd_graph {
    int64_t n = 0, nnz = 0;
    int32_t d_min = 0, d_max = 0;
    int32_t bipartite = 0;
    int32_t layout = 0;  // 0 CSR, 1 fat, 2 compact, ... (kLayout* of the kernels)
    int32_t kernel_layout = 0;  // the kernels' layout code: layout, 6 for fat with non-temporal
                                // loads, 7, 8 or 9 for layout 5 (kLayout* of the kernels)
    int device = 0;
    uint32_t cus = 0;                // compute units of the device
    std::vector<int32_t> deg;        // host copy for the planner, by caller id
    std::vector<uint32_t> internal;  // caller id -> storage id (empty: identity)
    std::vector<uint32_t> external;  // storage id -> caller id where walks see storage ids (layout 5)
    DevBuf node, col, adj, rp32, col24, node8, runtab;
    uint32_t run_h1 = 0, run_words = 0, run_ninv = 0;  // code 8: direct row offsets, words of runtab, d_max + 1
    uint32_t run_shift = 0;                            // code 8: log2 of the storage ids per record
    bool runs_shared = false;                          // code 8: the table fits the walk-sharing kernels
    DomainParams dom{};
    int64_t device_bytes = 0;
    std::mutex mu;  // serialises calls that use the per-graph work buffers
    Workspace ws;
};

// ---------------------------------------------------------------------------
// Graph loading
// ---------------------------------------------------------------------------
namespace {

DomainParams make_domain(uint32_t n)
{
    DomainParams d{};
    uint32_t w = 0;
    while ((uint64_t(1) << w) < n) ++w;
    d.n = n;
    d.rb = w >> 1;
    d.mask = (1u << d.rb) - 1u;
    d.rsh = d.rb ? 32u - d.rb : 31u;
    d.A = (uint32_t)((uint64_t(n) + d.mask) >> d.rb);
    d.A8 = d.A << 8;
    return d;
}

// Checks run on the host, in parallel over node ranges.
int validate(int64_t n, const int64_t* rp, const int32_t* col, int32_t* bip)
{
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::atomic<int> bad{0};
    auto worker = [&](int64_t lo, int64_t hi) {
        for (int64_t v = lo; v < hi && !bad.load(std::memory_order_relaxed); ++v) {
            const int64_t b = rp[v], e = rp[v + 1];
            for (int64_t i = b; i < e; ++i) {
                const int32_t u = col[i];
                if (u == v || (i > b && col[i - 1] >= u)) {
                    bad = 1;
                    break;
                }
                // symmetry: v must appear in row u
                const int32_t* rb = col + rp[u];
                const int32_t* re = col + rp[u + 1];
                if (!std::binary_search(rb, re, (int32_t)v)) {
                    bad = 1;
                    break;
                }
            }
        }
    };
    std::vector<std::thread> th;
    const int64_t per = (n + nt - 1) / nt;
    for (unsigned i = 0; i < nt; ++i) {
        const int64_t lo = i * per, hi = std::min<int64_t>(n, lo + per);
        if (lo < hi) th.emplace_back(worker, lo, hi);
    }
    for (auto& t : th) t.join();
    if (bad) return BD_E_GRAPH;
    // connectivity and bipartiteness by one BFS with 2-colouring
    std::vector<int8_t> colour((size_t)n, -1);
    std::vector<int32_t> queue((size_t)n);
    size_t head = 0, tail = 0;
    colour[0] = 0;
    queue[tail++] = 0;
    int32_t bipartite = 1;
    while (head < tail) {
        const int32_t v = queue[head++];
        for (int64_t i = rp[v]; i < rp[v + 1]; ++i) {
            const int32_t u = col[i];
            if (colour[u] < 0) {
                colour[u] = (int8_t)(1 - colour[v]);
                queue[tail++] = u;
            } else if (colour[u] == colour[v]) {
                bipartite = 0;
            }
        }
    }
    if ((int64_t)tail != n) return BD_E_GRAPH;
    *bip = bipartite;
    return BD_OK;
}

// The caller's arrays when they live in device memory (BD_DEVICE_PTRS): checked
// to be device allocations of the current device, then read once into host
// copies for validation and layout building.
int fetch_device_csr(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, hipStream_t st,
                     std::vector<int64_t>& rp, std::vector<int32_t>& col)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    for (const void* ptr : {(const void*)row_ptr, (const void*)col_idx}) {
        hipPointerAttribute_t at{};
        if (hipPointerGetAttributes(&at, ptr) != hipSuccess) {
            (void)hipGetLastError();
            return BD_E_INVALID;
        }
        if (at.type != hipMemoryTypeDevice || at.device != dev) return BD_E_INVALID;
    }
    rp.resize((size_t)n + 1);
    HIP_TRY(hipMemcpyAsync(rp.data(), row_ptr, rp.size() * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int64_t nnz = rp[(size_t)n];
    if (rp[0] != 0 || nnz < 0) return BD_E_GRAPH;
    if (nnz > kMaxNnz) return BD_E_RANGE;
    col.resize((size_t)std::max<int64_t>(nnz, 1));
    if (nnz) HIP_TRY(hipMemcpyAsync(col.data(), col_idx, (size_t)nnz * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return BD_OK;
}

}  // namespace

extern "C" int bd_set_allocator(const bd_allocator* a)
{
    if (a && (!a->alloc || !a->free)) return BD_E_INVALID;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc = a ? *a : bd_allocator{};
    return BD_OK;
}

extern "C" int graph_load_csr(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                              uint32_t flags, void* stream, bd_graph** out)
{
    if (!out || !row_ptr || !col_idx) return BD_E_INVALID;
    *out = nullptr;
    if (n < 2 || n > kMaxN) return BD_E_RANGE;
    std::vector<int64_t> rp_host;
    std::vector<int32_t> col_host;
    if (flags & BD_DEVICE_PTRS) {
        const int rc = fetch_device_csr(n, row_ptr, col_idx, (hipStream_t)stream, rp_host, col_host);
        if (rc != BD_OK) return rc;
        row_ptr = rp_host.data();
        col_idx = col_host.data();
        flags &= ~BD_DEVICE_PTRS;
    }
    if (row_ptr[0] != 0) return BD_E_GRAPH;
    const int64_t nnz = row_ptr[n];
    if (nnz < 0 || nnz > kMaxNnz) return BD_E_RANGE;
    int32_t dmin = INT32_MAX, dmax = 0;
    for (int64_t v = 0; v < n; ++v) {
        const int64_t d = row_ptr[v + 1] - row_ptr[v];
        if (d < 0) return BD_E_GRAPH;
        if (d > kMaxDeg) return BD_E_RANGE;
        dmin = std::min<int32_t>(dmin, (int32_t)d);
        dmax = std::max<int32_t>(dmax, (int32_t)d);
    }
    if (dmin < 1) return BD_E_GRAPH;  // an isolated node: not connected
    if (flags & BD_LAYOUT_AUTO) {
        if (flags & (BD_LAYOUT_FAT | BD_LAYOUT_COMPACT | BD_WIDE_IDS | BD_PROBE_STORAGE_IDS)) return BD_E_INVALID;
        const int64_t compact_bytes = 8 * (n + 1) + 3 * nnz + 8;
        flags = (n <= (int64_t(1) << 24) && compact_bytes <= kAutoCompactBytes)
                    ? (flags | BD_LAYOUT_COMPACT | BD_RELABEL_DEGREE)
                    : (flags | BD_LAYOUT_FAT);
    }
    // compact layouts: 3-byte ids up to 2^24 nodes; hubs first keeps 4-byte ids above that
    const bool storage_probe = (flags & BD_PROBE_STORAGE_IDS) != 0;
    if (storage_probe && ((flags & (BD_LAYOUT_COMPACT | BD_RELABEL_DEGREE)) != (BD_LAYOUT_COMPACT | BD_RELABEL_DEGREE) ||
                          (flags & BD_WIDE_IDS)))
        return BD_E_INVALID;
    if (storage_probe && n > (int64_t(1) << 24)) return BD_E_RANGE;
    const bool wide = (flags & BD_LAYOUT_COMPACT) && (flags & BD_RELABEL_DEGREE) && !storage_probe &&
                      (n > (int64_t(1) << 24) || (flags & BD_WIDE_IDS));
    if ((flags & BD_NONTEMPORAL) && (flags & BD_TEMPORAL)) return BD_E_INVALID;
    if ((flags & BD_NARROW_HUBS) && !(flags & BD_PROBE_STORAGE_IDS)) return BD_E_INVALID;
    if ((flags & BD_DIRECT_HUBS) && !(flags & BD_PROBE_STORAGE_IDS)) return BD_E_INVALID;
    if ((flags & BD_WIDE_HUBS) && (!(flags & BD_PROBE_STORAGE_IDS) || (flags & BD_NARROW_HUBS))) return BD_E_INVALID;
    if ((flags & (BD_NONTEMPORAL | BD_TEMPORAL)) && !(flags & BD_LAYOUT_FAT)) return BD_E_INVALID;
    if (flags & BD_LAYOUT_COMPACT) {
        if (flags & BD_LAYOUT_FAT) return BD_E_INVALID;
        if (!wide && (n > (int64_t(1) << 24) || 3 * nnz + 8 > (int64_t)UINT32_MAX)) return BD_E_RANGE;
    }
    for (int64_t i = 0; i < nnz; ++i)
        if (col_idx[i] < 0 || col_idx[i] >= n) return BD_E_GRAPH;
    int32_t bip = 0;
    if (!(flags & BD_SKIP_VALIDATION)) {
        const int rc = validate(n, row_ptr, col_idx, &bip);
        if (rc != BD_OK) return rc;
    }
    int dev = 0, ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return BD_E_NODEVICE;
    }
    HIP_TRY(hipGetDevice(&dev));

    bd_graph* g = new (std::nothrow) bd_graph();
    if (!g) return BD_E_NOMEM;
    g->n = n;
    g->nnz = nnz;
    g->d_min = dmin;
    g->d_max = dmax;
    g->bipartite = bip;
    g->layout = (flags & BD_LAYOUT_COMPACT) ? (storage_probe ? 5 : wide ? 4 : (flags & BD_RELABEL_DEGREE) ? 3 : 2)
                                            : (flags & BD_LAYOUT_FAT) ? 1 : 0;
    g->kernel_layout = g->layout;
    if (g->layout == 5 && !(flags & BD_NARROW_HUBS)) g->kernel_layout = 7;
    if (g->layout == 1) {
        const int64_t fat_bytes = 16 * nnz + 16 * n;
        const bool nt = (flags & BD_NONTEMPORAL) ? true
                        : (flags & BD_TEMPORAL)  ? false
                                                 : fat_bytes >= kFatNontemporalBytes;
        if (nt) g->kernel_layout = 6;
    }
    g->device = dev;
    {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cu = 256;
        g->cus = (uint32_t)std::max(cu, 1);
    }
    g->dom = make_domain((uint32_t)n);
    g->deg.resize((size_t)n);
    for (int64_t v = 0; v < n; ++v) g->deg[(size_t)v] = (int32_t)(row_ptr[v + 1] - row_ptr[v]);
    // storage order: caller order, or descending degree (ties by id)
    std::vector<uint32_t> order;  // storage id -> caller id
    std::vector<int32_t> relabelled;
    const int32_t* col_store = col_idx;
    if (flags & BD_RELABEL_DEGREE) {
        order.resize((size_t)n);
        for (int64_t v = 0; v < n; ++v) order[(size_t)v] = (uint32_t)v;
        std::stable_sort(order.begin(), order.end(),
                         [&](uint32_t a, uint32_t b) { return g->deg[a] > g->deg[b]; });
        g->internal.resize((size_t)n);
        for (int64_t i = 0; i < n; ++i) g->internal[order[(size_t)i]] = (uint32_t)i;
        if (storage_probe) g->external = order;  // walks report storage ids: map them back
        relabelled.resize((size_t)nnz);
        int64_t pos = 0;
        for (int64_t i = 0; i < n; ++i) {
            const uint32_t v = order[(size_t)i];
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
                relabelled[(size_t)pos++] = (int32_t)g->internal[(size_t)col_idx[e]];
        }
        col_store = relabelled.data();
    }
    std::vector<uint32_t> nodetab((size_t)n * 4);
    int64_t off = 0;
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t v = order.empty() ? (uint32_t)i : order[(size_t)i];
        const int32_t d = g->deg[v];
        const float inv = 1.0f / (float)d;
        uint32_t bits;
        std::memcpy(&bits, &inv, 4);
        nodetab[(size_t)i * 4 + 0] = (uint32_t)off;
        nodetab[(size_t)i * 4 + 1] = (uint32_t)d;
        nodetab[(size_t)i * 4 + 2] = bits;
        nodetab[(size_t)i * 4 + 3] = v;
        off += d;
    }
    hipStream_t st = (hipStream_t)stream;
    int rc = BD_OK;
    std::vector<uint32_t> rp32, packed;
    if (g->layout >= 2) {
        // compact: 32-bit row offsets (storage order), 3-byte neighbour storage ids
        // (little endian) with 8 bytes of padding -- 4-byte ids above 2^24 nodes;
        // with hubs first also the node entries {row offset, original id}, entry
        // n = {nnz, 0}
        const bool packed_ids = g->layout != 4;
        const bool hubs = g->layout == 3 || g->layout == 4;  // 8-byte node entries (layout 5 reads rp32)
        rp32.resize((size_t)n + 1);
        for (int64_t i = 0; i < n; ++i) rp32[(size_t)i] = nodetab[(size_t)i * 4];
        rp32[(size_t)n] = (uint32_t)nnz;
        if (packed_ids) {
            const size_t bytes = (size_t)(3 * nnz + 8);
            packed.assign((bytes + 3) / 4, 0u);
            uint8_t* b = reinterpret_cast<uint8_t*>(packed.data());
            for (int64_t i = 0; i < nnz; ++i) {
                const uint32_t v = (uint32_t)col_store[i];
                b[3 * i + 0] = (uint8_t)v;
                b[3 * i + 1] = (uint8_t)(v >> 8);
                b[3 * i + 2] = (uint8_t)(v >> 16);
            }
        }
        std::vector<uint32_t> node8;
        if (hubs) {
            node8.resize(2 * ((size_t)n + 1));
            for (int64_t i = 0; i < n; ++i) {
                node8[2 * (size_t)i] = nodetab[(size_t)i * 4];
                node8[2 * (size_t)i + 1] = nodetab[(size_t)i * 4 + 3];
            }
            node8[2 * (size_t)n] = (uint32_t)nnz;
            node8[2 * (size_t)n + 1] = 0u;
        }
        rc = g->rp32.alloc(rp32.size() * 4);
        if (rc == BD_OK && packed_ids) rc = g->col24.alloc(packed.size() * 4);
        if (rc == BD_OK && !packed_ids) rc = g->col.alloc((size_t)std::max<int64_t>(nnz, 1) * 4);
        if (rc == BD_OK && hubs) rc = g->node8.alloc(node8.size() * 4);
        if (rc != BD_OK) {
            delete g;
            return rc;
        }
        if (hipMemcpyAsync(g->rp32.p, rp32.data(), rp32.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
            (packed_ids && hipMemcpyAsync(g->col24.p, packed.data(), packed.size() * 4, hipMemcpyHostToDevice,
                                          st) != hipSuccess) ||
            (!packed_ids && hipMemcpyAsync(g->col.p, col_store, (size_t)nnz * 4, hipMemcpyHostToDevice,
                                           st) != hipSuccess) ||
            (hubs && hipMemcpyAsync(g->node8.p, node8.data(), node8.size() * 4, hipMemcpyHostToDevice,
                                    st) != hipSuccess)) {
            delete g;
            return BD_E_HIP;
        }
        if (hipStreamSynchronize(st) != hipSuccess) {
            delete g;
            return BD_E_HIP;
        }
    } else {
        rp32.resize((size_t)n + 1);
        for (int64_t i = 0; i < n; ++i) rp32[(size_t)i] = nodetab[(size_t)i * 4];
        rp32[(size_t)n] = (uint32_t)nnz;
        rc = g->rp32.alloc(rp32.size() * 4);
        if (rc == BD_OK) rc = g->node.alloc((size_t)n * 16);
        if (rc == BD_OK) rc = g->col.alloc((size_t)std::max<int64_t>(nnz, 1) * 4);
        if (rc == BD_OK && g->layout == 1) rc = g->adj.alloc((size_t)std::max<int64_t>(nnz, 1) * 16);
        if (rc != BD_OK) {
            delete g;
            return rc;
        }
        if (hipMemcpyAsync(g->node.p, nodetab.data(), (size_t)n * 16, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(g->rp32.p, rp32.data(), rp32.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(g->col.p, col_store, (size_t)nnz * 4, hipMemcpyHostToDevice, st) != hipSuccess) {
            delete g;
            return BD_E_HIP;
        }
    }
    if (g->layout == 1 &&
        build_fat_adjacency(g->node.as<uint4>(), g->col.as<uint32_t>(), g->adj.as<uint4>(),
                            (uint32_t)nnz, st) != hipSuccess) {
        delete g;
        return BD_E_HIP;
    }
    if (hipStreamSynchronize(st) != hipSuccess) {
        delete g;
        return BD_E_HIP;
    }
    if (g->layout == 5 && !(flags & BD_DIRECT_HUBS)) {
        // the degree-run table: two work groups per CU where it fits 64 KB,
        // else one per CU with two pairs per thread (flags may force either)
        std::vector<uint32_t> runtab;
        int code = 0;
        uint32_t shift = kRunShiftMin;
        for (const int c : {kLayoutHubRunsNarrow, kLayoutHubRuns}) {
            if ((c == kLayoutHubRunsNarrow && (flags & BD_WIDE_HUBS)) ||
                (c == kLayoutHubRuns && (flags & BD_NARROW_HUBS)))
                continue;
            // the smallest block that fits: smaller blocks let shorter runs in
            for (shift = kRunShiftMin; shift <= kRunShiftMax; ++shift)
                if (build_run_table(rp32, shift, (uint32_t)dmax + 1u, hub_words(1024, c), &g->run_h1, &runtab))
                    break;
            if (shift <= kRunShiftMax) {
                code = c;
                break;
            }
        }
        if (code != 0) {
            g->run_words = (uint32_t)runtab.size();
            g->run_ninv = (uint32_t)dmax + 1u;
            g->run_shift = shift;
            const int arc = g->runtab.alloc(runtab.size() * 4);
            if (arc != BD_OK) {
                delete g;
                return arc;
            }
            if (hipMemcpyAsync(g->runtab.p, runtab.data(), runtab.size() * 4, hipMemcpyHostToDevice, st) !=
                    hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                delete g;
                return BD_E_HIP;
            }
            g->kernel_layout = code;
            g->runs_shared = ((runtab.size() + 3) & ~(size_t)3) + g->run_ninv <= kRunWordsShared;
        }
    }
    g->device_bytes = (int64_t)(g->node.bytes + g->col.bytes + g->adj.bytes + g->rp32.bytes + g->col24.bytes +
                                g->node8.bytes + g->runtab.bytes);
    *out = g;
    return BD_OK;
}

extern "C" void graph_free(bd_graph* g)
{
    delete g;
}

extern "C" int bd_graph_get_info(const bd_graph* g, bd_graph_info* info)
{
    if (!g || !info) return BD_E_INVALID;
    info->n = g->n;
    info->nnz = g->nnz;
    info->d_min = g->d_min;
    info->d_max = g->d_max;
    info->bipartite = g->bipartite;
    info->layout = g->layout;
    info->nontemporal = g->kernel_layout == 6 ? 1 : 0;
    info->lds_hubs = runs_layout(g->kernel_layout) ? (int32_t)g->n
                     : hub_layout(g->kernel_layout)
                         ? (int32_t)std::min<int64_t>(hub_nodes(1024, g->kernel_layout), g->n)
                         : 0;
    info->device_bytes = g->device_bytes;
    return BD_OK;
}

// ---------------------------------------------------------------------------
// Planner (Algorithm 1 parameters; proof of Theorem 3.8)
// ---------------------------------------------------------------------------
namespace {

constexpr double kCeilGuard = 1.0 - 0x1p-40;

int64_t ceil_guarded(double x)
{
    return (int64_t)std::ceil(x * kCeilGuard);
}

// walk-sharing group size of a policy (0 and 1: none)
uint32_t policy_share(const bd_policy& p)
{
    return p.share > 1 ? (uint32_t)p.share : 1u;
}

bd_policy default_policy()
{
    bd_policy p{};
    p.kind = BD_POLICY_PAPER;
    p.c_B = 448.0;
    p.c_R = 128.0;
    p.delta = 0.01;
    return p;
}

// Fills B, G, K, R, L, walk_steps and status of one result.
void plan_one(const bd_graph* g, int32_t s, int32_t t, double eps, int32_t L, const bd_policy& pol,
              bd_result* r)
{
    std::memset(r, 0, sizeof(*r));
    r->L = L;
    if (s < 0 || t < 0 || s >= g->n || t >= g->n || s == t || !(eps > 0.0 && eps < 1.0) || L < 0 ||
        L > kMaxL || pol.share < 0 || pol.share > (int32_t)kMaxShare) {
        r->status = BD_E_INVALID;
        return;
    }
    const double delta = pol.delta > 0.0 ? pol.delta : 0.01;
    const int64_t G = ceil_guarded(8.0 * std::log(1.0 / delta));
    int64_t B, R;
    if (pol.kind == BD_POLICY_FIXED) {
        B = pol.B_fixed;
        R = pol.R_fixed;
    } else {
        const double cB = pol.kind == BD_POLICY_PAPER ? 448.0 : pol.c_B;
        const double cR = pol.kind == BD_POLICY_PAPER ? 128.0 : pol.c_R;
        B = ceil_guarded(cB / (eps * eps));
        const double ds = g->deg[(size_t)s], dt = g->deg[(size_t)t], dm = g->d_min;
        const double inv = 1.0 / ds + 1.0 / dt;
        const double theta = (1.0 - eps / 2.0) * inv * inv;
        const double Lp1 = (double)L + 1.0;
        const double rr = cR * Lp1 * Lp1 / (dm * dm * theta);
        R = rr > 9.0e18 ? INT64_MAX : ceil_guarded(rr);
    }
    B = std::max<int64_t>(B, 1);
    R = std::max<int64_t>(R, 2);
    r->B = (int32_t)std::min<int64_t>(B, INT32_MAX);
    r->G = (int32_t)G;
    r->R = R;
    // exact products in 128 bits, saturated at INT64_MAX
    typedef unsigned __int128 u128;
    const u128 i64max = (u128)INT64_MAX;
    const u128 K = (u128)(uint64_t)B * (u128)(uint64_t)G;
    r->K = K > i64max ? INT64_MAX : (int64_t)K;
    // walks: R pairs per walk-sharing group, ceil(B/M) groups per block
    const uint64_t M = pol.share > 1 ? (uint64_t)pol.share : 1u;
    const u128 groups = (u128)(((uint64_t)B + M - 1) / M) * (u128)(uint64_t)G;
    u128 steps;
    if (L == 0) {
        steps = 0;
    } else if ((groups >> 64) != 0) {
        steps = i64max + 1;
    } else {
        const u128 GR = groups * (u128)(uint64_t)R;  // < 2^127
        steps = (GR >> 112) != 0 ? i64max + 1 : 2 * GR * (u128)(uint64_t)L;  // L < 2^14
    }
    r->walk_steps = steps > i64max ? INT64_MAX : (int64_t)steps;
    if (G > kMaxG || B > INT32_MAX || K >= 4294967295u || R >= (int64_t)4294967295LL)
        r->status = BD_E_BUDGET;
    else if (pol.max_steps_per_query && steps > (u128)pol.max_steps_per_query)
        r->status = BD_E_BUDGET;
    else
        r->status = BD_OK;
}

}  // namespace

extern "C" int bd_plan(const bd_graph* g, int64_t nq, const int32_t* s, const int32_t* t,
                       const double* eps, const int32_t* L, const bd_policy* pol, bd_result* out)
{
    if (!g || nq < 0 || (nq > 0 && (!s || !t || !eps || !L || !out))) return BD_E_INVALID;
    const bd_policy p = pol ? *pol : default_policy();
    for (int64_t i = 0; i < nq; ++i) plan_one(g, s[i], t[i], eps[i], L[i], p, &out[i]);
    return BD_OK;
}

// ---------------------------------------------------------------------------
// Batched execution
// ---------------------------------------------------------------------------
namespace {

uint32_t storage_id(const bd_graph* g, int32_t v)
{
    return g->internal.empty() ? (uint32_t)v : g->internal[(size_t)v];
}

GraphTables tables(const bd_graph* g)
{
    GraphTables t{};
    t.node = g->node.as<const uint4>();
    t.col = g->col.as<const uint32_t>();
    t.adj = g->adj.as<const uint4>();
    t.rp = g->rp32.as<const uint32_t>();
    t.col24 = g->col24.as<const uint32_t>();
    t.node8 = g->node8.as<const uint2>();
    t.runtab = g->runtab.as<const uint32_t>();
    t.run_h1 = g->run_h1;
    t.run_words = g->run_words;
    t.run_ninv = g->run_ninv;
    t.run_shift = g->run_shift;
    t.dom = g->dom;
    return t;
}

// The kernel code that runs walks of sharing class `share` on g: the graph's,
// except that walk sharing on the degree-run table runs code 8's sharing
// kernels, which hold a smaller copy, or code 7's (the same tables and
// results) where it does not fit them.
int run_kernel(const bd_graph* g, int share)
{
    if (runs_layout(g->kernel_layout) && share > 1) return g->runs_shared ? kLayoutHubRuns : kLayoutHubIdX2;
    return g->kernel_layout;
}

int resident_wgs(const bd_graph* g, int uniform, int share = 1)
{
    int per_cu = 0;
    if (walk_occupancy(run_kernel(g, share), uniform, share, &per_cu) != 0 || per_cu < 1) per_cu = 1;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, g->device) != hipSuccess) return per_cu * 256;
    return per_cu * prop.multiProcessorCount;
}

// How the probes of one query are cut into work-group chunks.
//   plain:   one chunk holds whole probes (all R replicas), at least one pair
//            per thread of the layout's work group (256, or 1,024 hubs first),
//            but no more probes than give every compute unit a chunk;
//   batched / served: whole probes up to kSplitReplicas pairs per chunk, and a
//   probe with R > kSplitReplicas is cut into replica parts (multiples of 64)
//   so that no chunk runs much longer than the others.
uint32_t exec_queues(const bd_exec& ex)
{
    if (ex.queues <= 0) return kMaxQueues;
    return std::min<uint32_t>((uint32_t)ex.queues, kMaxQueues);
}

struct ChunkPlan {
    uint32_t gc = 1;       // walk-sharing groups per chunk (whole-group chunks)
    uint32_t part = 0;     // replicas per part, 0 = groups are not split
};

// The walk-sharing groups of a query: each of the G blocks of B probes holds
// ceil(B/M) groups of M consecutive probes (the last one may be smaller).
struct Groups {
    uint32_t B = 1, M = 1, per_block = 1, n = 0;
    Groups() = default;
    Groups(const QueryDesc& d)
        : B(d.B), M(std::max<uint32_t>(d.share, 1u)), per_block((d.B + M - 1) / M), n(d.G * per_block)
    {
    }
    uint32_t first(uint32_t gi) const { return (gi / per_block) * B + (gi % per_block) * M; }
    uint32_t size(uint32_t gi) const { return std::min(M, B - (gi % per_block) * M); }
};

ChunkPlan chunk_plan(const bd_exec& ex, const QueryDesc& d, int layout, uint32_t spread = 0)
{
    ChunkPlan cp;
    const Groups grp(d);
    const uint32_t R = d.R;
    const uint32_t pairs = ex.chunk_pairs > 0 ? std::max<uint32_t>((uint32_t)ex.chunk_pairs, 64u)
                           : ex.mode == BD_MODE_PLAIN ? (uint32_t)group_pairs(layout, share_class(d.share))
                                                      : kSplitReplicas;
    if (ex.mode != BD_MODE_PLAIN && R >= kUniformMinR && R > pairs) {
        const uint32_t parts = (R + pairs - 1) / pairs;
        cp.part = ((R + parts - 1) / parts + 63u) & ~63u;
        cp.gc = 1;
        return cp;
    }
    uint32_t gc;
    if (ex.chunk_probes > 0) {
        gc = std::max<uint32_t>(1u, (uint32_t)ex.chunk_probes / grp.M);
    } else if (ex.mode == BD_MODE_PLAIN) {
        gc = (uint32_t)std::max<uint64_t>(1, ((uint64_t)pairs + R - 1) / R);
        // a query too small to give each of `spread` compute units a chunk is
        // spread over more of them: its launch is bound by the walks' step
        // latency, and compute units left idle are lost to it
        if (spread > 0) gc = std::min<uint32_t>(gc, std::max<uint32_t>(1u, (grp.n + spread - 1) / spread));
    } else {
        // at most `pairs` lane slots per chunk, counted as the kernels lay the
        // pairs out (probes with R >= kUniformMinR in blocks of 64 replicas, one
        // wave block each; others a pair per lane), so that a chunk of one work
        // group's pairs runs in one pass: rounding up would add a nearly empty
        // second one
        const uint64_t slots = R >= kUniformMinR ? ((uint64_t)R + 63) / 64 * 64 : R;
        gc = (uint32_t)std::max<uint64_t>(1, (uint64_t)pairs / slots);
    }
    gc = std::min<uint32_t>(gc, (uint32_t)kMaxChunkProbes / grp.M);
    gc = std::min<uint32_t>(gc, std::max<uint32_t>(grp.n, 1));
    cp.gc = std::max<uint32_t>(gc, 1);
    return cp;
}

// Emits the chunks of one query in order: (next_g, next_p) is the cursor.
struct ChunkCursor {
    uint32_t q = 0, R = 0;
    Groups grp;
    ChunkPlan plan;
    uint32_t next_g = 0, next_p = 0;
    ChunkCursor() = default;
    ChunkCursor(uint32_t q_, const QueryDesc& d, const bd_exec& ex, int layout, uint32_t spread = 0)
        : q(q_), R(d.R), grp(d), plan(chunk_plan(ex, d, layout, spread))
    {
    }
    bool done() const { return next_g >= grp.n; }
    Chunk next()
    {
        Chunk c{};
        c.q = q;
        c.g0 = next_g;
        if (plan.part) {
            c.gc = 1;
            c.p0 = next_p;
            c.pc = std::min<uint32_t>(plan.part, R - next_p);
            next_p += c.pc;
            if (next_p >= R) {
                next_p = 0;
                ++next_g;
            }
        } else {
            c.gc = std::min<uint32_t>(plan.gc, grp.n - next_g);
            c.p0 = 0;
            c.pc = R;
            next_g += c.gc;
        }
        c.k0 = grp.first(c.g0);
        const uint32_t last = c.g0 + c.gc - 1;
        c.kc = grp.first(last) + grp.size(last) - c.k0;
        return c;
    }
    // walk steps of the next chunk (2 walks of L steps per replica and group)
    uint64_t chunk_steps(uint32_t L) const
    {
        const uint64_t pairs = plan.part ? (uint64_t)std::min<uint32_t>(plan.part, R - next_p)
                                         : (uint64_t)std::min<uint32_t>(plan.gc, grp.n - next_g) * R;
        return 2ull * pairs * ((uint64_t)L + 1);
    }
};

struct Batch {
    std::vector<QueryDesc> qd;
    std::vector<Chunk> chunks;
    uint32_t split_probes = 0;          // per-probe accumulators needed
    std::vector<uint32_t> chunk_begin;  // per valid query, first chunk (chunks grouped by query)
    std::vector<int64_t> index;         // valid query -> caller's index
    uint32_t G = 0;
    uint32_t n_uniform = 0;             // chunks [0, n_uniform) belong to queries with R >= kUniformMinR
    // chunk queues of the persistent launches: part 0 = [0, n_uniform), part 1 =
    // the rest; qoff[part][i] is the first chunk of queue i relative to the part
    uint32_t nqueues = 1;
    uint32_t qoff[2][kMaxQueues + 1] = {};
    int share = 1;                      // kernel instance for the walk-sharing factor
};

// Device buffers of one batch: either the graph's workspace (grown on demand)
// or a carving of the library's fixed scratch array (no allocation).
struct WorkPtrs {
    void *qd = nullptr, *chunks = nullptr, *bs = nullptr, *done = nullptr, *beta = nullptr, *cursor = nullptr,
         *psum = nullptr, *pcount = nullptr, *qdbg = nullptr, *ydbg = nullptr;
};

// Bytes of each buffer a batch needs (in WorkPtrs order).
void work_sizes(const Batch& b, bool qdbg, bool ydbg, size_t sz[10])
{
    const size_t nv = b.qd.size();
    sz[0] = nv * sizeof(QueryDesc);
    sz[1] = b.chunks.size() * sizeof(Chunk);
    sz[2] = nv * (size_t)b.G * 16;
    sz[3] = nv * 4;
    sz[4] = nv * 8;
    sz[5] = 2 * kMaxQueues * 4;
    sz[6] = (size_t)b.split_probes * 32;
    sz[7] = (size_t)b.split_probes * 4;
    sz[8] = qdbg ? (size_t)b.qd[0].K * 8 : 0;
    sz[9] = ydbg ? (size_t)b.G * 8 : 0;
}

int workspace_ptrs(Workspace& w, const Batch& b, bool qdbg, bool ydbg, WorkPtrs* wp)
{
    size_t sz[10];
    work_sizes(b, qdbg, ydbg, sz);
    DevBuf* bufs[10] = {&w.qd, &w.chunks, &w.bs, &w.done, &w.beta, &w.cursor, &w.psum, &w.pcount, &w.qdbg, &w.ydbg};
    void** out[10] = {&wp->qd, &wp->chunks, &wp->bs, &wp->done, &wp->beta, &wp->cursor, &wp->psum, &wp->pcount,
                      &wp->qdbg, &wp->ydbg};
    for (int i = 0; i < 10; ++i) {
        if (i >= 8 && sz[i] == 0) continue;
        const int rc = w.ensure(*bufs[i], sz[i]);
        if (rc != BD_OK) return rc;
        *out[i] = bufs[i]->p;
    }
    return BD_OK;
}

// The buffers laid out one after another, each 256-byte aligned, inside
// [base, base + cap). BD_E_SCRATCH when they do not fit.
int carve_ptrs(void* base, size_t cap, const Batch& b, WorkPtrs* wp)
{
    size_t sz[10];
    work_sizes(b, false, false, sz);
    void** out[8] = {&wp->qd, &wp->chunks, &wp->bs, &wp->done, &wp->beta, &wp->cursor, &wp->psum, &wp->pcount};
    size_t off = 0;
    for (int i = 0; i < 8; ++i) {
        const size_t need = std::max<size_t>(sz[i], 16);
        if (need > cap || off > cap - need) return BD_E_SCRATCH;
        *out[i] = static_cast<char*>(base) + off;
        off += (need + 255) & ~(size_t)255;
    }
    return BD_OK;
}

// Run one set of valid queries: zero the tables, launch, read the results.
// The work buffers are w (see WorkPtrs). With ex.use_graph (batched mode, and
// only with the graph's own workspace, `owned`) the zeroing and the persistent
// launches are captured once per launch shape into a hipGraph on a
// library-owned stream and replayed; descriptors and chunk tables are copied
// in before each replay. Without `owned` nothing is created: no events, so
// stats->walk_kernel_ms stays 0.
// With ex.deadline_ms > 0 (and `owned`) a watchdog on the calling thread waits
// for the launches by polling; once the deadline has passed it raises the
// abort flag, the work groups take no further chunk, and the queries whose
// probe count did not reach K are marked in *incomplete.
int run_batch(bd_graph* g, const Batch& b, const bd_exec& ex, hipStream_t user_st, const WorkPtrs& w,
              bool owned, std::vector<double>& beta, bd_stats* stats, double* q_dbg_host, double* y_dbg_host,
              std::vector<uint8_t>* incomplete = nullptr)
{
    const size_t nv = b.qd.size();
    if (nv == 0) return BD_OK;
    const double t_call = now_ms();
    const bool watch = owned && ex.deadline_ms > 0.0;
    if (watch) {
        const int rc = g->ws.ensure_abort_flag();
        if (rc != BD_OK) return rc;
        __atomic_store_n(g->ws.abort_host, 0u, __ATOMIC_SEQ_CST);
    }
    bool fired = false;
    auto past_deadline = [&]() {
        if (watch && !fired && now_ms() - t_call > ex.deadline_ms) {
            __atomic_store_n(g->ws.abort_host, 1u, __ATOMIC_SEQ_CST);
            fired = true;
        }
        return fired;
    };
    const size_t gdim = b.G;
    Workspace& ws = g->ws;
    const bool graph_mode = owned && ex.use_graph && ex.mode != BD_MODE_PLAIN && !q_dbg_host && !y_dbg_host;
    if (graph_mode && !ws.gstream && hipStreamCreateWithFlags(&ws.gstream, hipStreamNonBlocking) != hipSuccess)
        return BD_E_HIP;
    hipStream_t st = graph_mode ? ws.gstream : user_st;
    HIP_TRY(hipMemcpyAsync(w.qd, b.qd.data(), nv * sizeof(QueryDesc), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(w.chunks, b.chunks.data(), b.chunks.size() * sizeof(Chunk), hipMemcpyHostToDevice,
                           st));

    WalkArgs a{};
    a.g = tables(g);
    a.qd = static_cast<const QueryDesc*>(w.qd);
    a.gdim = (uint32_t)gdim;
    a.cursor = static_cast<uint32_t*>(w.cursor);
    a.blocksum = static_cast<unsigned long long*>(w.bs);
    a.done = static_cast<uint32_t*>(w.done);
    a.psum = static_cast<unsigned long long*>(w.psum);
    a.pcount = static_cast<uint32_t*>(w.pcount);
    a.beta = static_cast<double*>(w.beta);
    a.q_debug = q_dbg_host ? static_cast<double*>(w.qdbg) : nullptr;
    a.ybar_debug = y_dbg_host ? static_cast<double*>(w.ydbg) : nullptr;
    a.abort_flag = watch ? g->ws.abort_dev : nullptr;
    const int layout = run_kernel(g, b.share);

    // the zeroing every launch needs
    auto zero_all = [&](hipStream_t s2) -> int {
        if (launch_zero(w.bs, nv * gdim * 16, s2) != hipSuccess) return BD_E_HIP;
        if (launch_zero(w.done, nv * 4, s2) != hipSuccess) return BD_E_HIP;
        if (launch_zero(w.cursor, 2 * kMaxQueues * 4, s2) != hipSuccess) return BD_E_HIP;
        if (launch_zero(w.psum, (size_t)b.split_probes * 32, s2) != hipSuccess) return BD_E_HIP;
        if (launch_zero(w.pcount, (size_t)b.split_probes * 4, s2) != hipSuccess) return BD_E_HIP;
        return BD_OK;
    };
    // the persistent launches of the batched mode: wave-uniform chunks, then the rest
    uint32_t grids[2] = {0, 0};
    const uint32_t parts[3] = {0u, b.n_uniform, (uint32_t)b.chunks.size()};
    for (int part = 0; part < 2; ++part) {
        const uint32_t nch = parts[part + 1] - parts[part];
        uint32_t grid = ex.grid_wgs > 0 ? (uint32_t)ex.grid_wgs : (uint32_t)resident_wgs(g, part == 0, b.share);
        grids[part] = std::min<uint32_t>(grid, nch);
    }
    auto launch_persistent = [&](hipStream_t s2) -> int {
        for (int part = 0; part < 2; ++part) {
            if (grids[part] == 0) continue;
            WalkArgs ab = a;
            ab.chunks = static_cast<const Chunk*>(w.chunks) + parts[part];
            ab.nchunks = parts[part + 1] - parts[part];
            ab.cursor = static_cast<uint32_t*>(w.cursor) + part * kMaxQueues;
            ab.persistent = 1;
            ab.nqueues = b.nqueues;
            for (uint32_t i = 0; i <= b.nqueues; ++i) ab.qoff[i] = b.qoff[part][i];
            if (launch_walk(ab, layout, part == 0, b.share, grids[part], s2) != hipSuccess) return BD_E_HIP;
        }
        return BD_OK;
    };

    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (owned) {
        HIP_TRY(hipEventCreate(&e0));
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return BD_E_HIP;
        }
    }
    double kernel_ms = 0.0;
    int64_t launches = 0;
    int status = BD_OK;
    auto timed = [&](auto&& body) -> int {
        if (e0 && hipEventRecord(e0, st) != hipSuccess) return BD_E_HIP;
        const int r = body();
        if (r != BD_OK) return r;
        ++launches;
        if (!e0) return BD_OK;
        if (hipEventRecord(e1, st) != hipSuccess) return BD_E_HIP;
        if (watch) {
            // poll, raising the abort flag once the deadline has passed; a
            // raised flag ends the launch within one chunk per work group
            for (;;) {
                const hipError_t q = hipEventQuery(e1);
                if (q == hipSuccess) break;
                if (q != hipErrorNotReady) return BD_E_HIP;
                past_deadline();
                std::this_thread::sleep_for(std::chrono::microseconds(200));
            }
            (void)hipGetLastError();  // the not-ready answers are no error
        } else if (hipEventSynchronize(e1) != hipSuccess) {
            return BD_E_HIP;
        }
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return BD_E_HIP;
        kernel_ms += ms;
        return BD_OK;
    };
    if (ex.mode == BD_MODE_PLAIN) {
        status = zero_all(st);
        // one query per launch, one work group per chunk
        for (size_t q = 0; q < nv && status == BD_OK; ++q) {
            if (past_deadline()) break;  // the remaining queries are not launched
            const uint32_t c0 = b.chunk_begin[q];
            const uint32_t c1 = q + 1 < nv ? b.chunk_begin[q + 1] : (uint32_t)b.chunks.size();
            WalkArgs aq = a;
            aq.chunks = static_cast<const Chunk*>(w.chunks) + c0;
            aq.nchunks = c1 - c0;
            aq.persistent = 0;
            const int uniform = b.qd[q].R >= kUniformMinR;
            status = timed([&] {
                return launch_walk(aq, layout, uniform, b.share, c1 - c0, st) == hipSuccess ? BD_OK : BD_E_HIP;
            });
        }
    } else if (!graph_mode) {
        status = zero_all(st);
        if (status == BD_OK) status = timed([&] { return launch_persistent(st); });
    } else {
        // key: everything the captured launches depend on
        std::vector<uint64_t> key = {nv, b.chunks.size(), b.n_uniform, b.split_probes, gdim, grids[0],
                                     grids[1], (uint64_t)layout, (uint64_t)b.share, b.nqueues,
                                     (uint64_t)(uintptr_t)w.qd, (uint64_t)(uintptr_t)w.chunks,
                                     (uint64_t)(uintptr_t)w.bs, (uint64_t)(uintptr_t)w.psum,
                                     (uint64_t)(uintptr_t)w.pcount, (uint64_t)(uintptr_t)w.done,
                                     (uint64_t)(uintptr_t)w.beta, (uint64_t)(uintptr_t)w.cursor};
        for (int part = 0; part < 2; ++part)
            for (uint32_t i = 0; i <= b.nqueues; ++i) key.push_back(b.qoff[part][i]);
        key.push_back((uint64_t)(uintptr_t)a.abort_flag);
        if (!ws.gexec || ws.gkey != key) {
            if (ws.gexec) {
                (void)hipGraphExecDestroy(ws.gexec);
                ws.gexec = nullptr;
            }
            hipGraph_t graph = nullptr;
            HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            int cr = zero_all(st);
            if (cr == BD_OK) cr = launch_persistent(st);
            const hipError_t ce = hipStreamEndCapture(st, &graph);
            if (cr != BD_OK || ce != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return BD_E_HIP;
            }
            const hipError_t ie = hipGraphInstantiate(&ws.gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) {
                ws.gexec = nullptr;
                return BD_E_HIP;
            }
            ws.gkey = key;
            ++ws.graph_builds;
        }
        status = timed([&] { return hipGraphLaunch(ws.gexec, st) == hipSuccess ? BD_OK : BD_E_HIP; });
        ++ws.graph_replays;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (status != BD_OK) return status;
    beta.resize(nv);
    HIP_TRY(hipMemcpyAsync(beta.data(), w.beta, nv * 8, hipMemcpyDeviceToHost, st));
    if (q_dbg_host)
        HIP_TRY(hipMemcpyAsync(q_dbg_host, w.qdbg, (size_t)b.qd[0].K * 8, hipMemcpyDeviceToHost, st));
    if (y_dbg_host) HIP_TRY(hipMemcpyAsync(y_dbg_host, w.ydbg, gdim * 8, hipMemcpyDeviceToHost, st));
    std::vector<uint32_t> done_count;
    if (fired) {
        // which queries the aborted launches finished: those whose probe count reached K
        done_count.resize(nv);
        HIP_TRY(hipMemcpyAsync(done_count.data(), w.done, nv * 4, hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    if (watch) __atomic_store_n(g->ws.abort_host, 0u, __ATOMIC_SEQ_CST);
    if (incomplete) {
        incomplete->assign(nv, 0);
        for (size_t q = 0; q < done_count.size(); ++q) (*incomplete)[q] = done_count[q] != b.qd[q].K;
    }
    if (stats) {
        stats->walk_kernel_ms += kernel_ms;
        stats->launches += launches;
        stats->chunks += (int64_t)b.chunks.size();
    }
    return BD_OK;
}

// Build descriptors and the chunk table for the valid queries of a batch.
void build_batch(const bd_graph* g, int64_t nq, const int32_t* s, const int32_t* t, const int32_t* L,
                 const uint32_t* uid, uint64_t seed, const bd_result* plans, const bd_exec& ex, uint32_t share,
                 Batch& b)
{
    share = std::max<uint32_t>(share, 1u);
    b.share = share_class(share);
    for (int64_t i = 0; i < nq; ++i) {
        const bd_result& r = plans[i];
        if (r.status != BD_OK) continue;
        QueryDesc d{};
        d.s = (int32_t)storage_id(g, s[i]);
        d.t = (int32_t)storage_id(g, t[i]);
        d.L = L[i];
        d.uid = uid ? uid[i] : (uint32_t)i;
        d.K = (uint32_t)r.K;
        d.R = (uint32_t)r.R;
        d.B = (uint32_t)r.B;
        d.G = (uint32_t)r.G;
        d.slot = (uint32_t)b.qd.size();
        d.seed_lo = (uint32_t)seed;
        d.seed_hi = (uint32_t)(seed >> 32);
        d.share = share;
        b.G = std::max<uint32_t>(b.G, d.G);
        b.index.push_back(i);
        b.qd.push_back(d);
    }
    // chunk table: grouped by query; batched launches order queries by
    // descending cost so the longest work starts first
    auto cost = [&](size_t q) { return (double)b.qd[q].K * b.qd[q].R * (double)b.qd[q].L; };
    int64_t umin = ex.uniform_min_r == 0 ? (int64_t)kUniformMinR
                   : ex.uniform_min_r < 0 ? INT64_MAX : (int64_t)ex.uniform_min_r;
    if (ex.mode != BD_MODE_PLAIN && ex.uniform_min_r == 0) {
        // automatic: the wave-uniform kernel gets a launch of its own only when
        // its chunks can fill the device; otherwise the general kernel runs every
        // chunk
        uint64_t nu = 0;
        for (const QueryDesc& d : b.qd) {
            if ((int64_t)d.R < umin) continue;
            const ChunkPlan cp = chunk_plan(ex, d, g->kernel_layout);
            const uint32_t ng = Groups(d).n;
            nu += cp.part ? (uint64_t)ng * ((d.R + cp.part - 1) / cp.part) : (ng + cp.gc - 1) / cp.gc;
        }
        if (nu < (uint64_t)resident_wgs(g, 1, b.share)) umin = INT64_MAX;
    }
    auto uniform = [&](size_t q) { return ex.mode != BD_MODE_PLAIN && (int64_t)b.qd[q].R >= umin; };
    std::vector<size_t> order(b.qd.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    if (ex.mode != BD_MODE_PLAIN) {
        std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
            if (uniform(x) != uniform(y)) return uniform(x);
            return cost(x) > cost(y);
        });
    }
    b.nqueues = ex.mode == BD_MODE_PLAIN ? 1u : exec_queues(ex);
    b.chunk_begin.assign(b.qd.size(), 0);
    auto emit = [&](size_t q) {
        QueryDesc& d = b.qd[q];
        ChunkCursor cur((uint32_t)q, d, ex, g->kernel_layout, ex.mode == BD_MODE_PLAIN ? g->cus : 0u);
        if (cur.plan.part) {
            d.psum_base = b.split_probes;
            b.split_probes += d.K;
        }
        b.chunk_begin[q] = (uint32_t)b.chunks.size();
        while (!cur.done()) b.chunks.push_back(cur.next());
    };
    // each part (wave-uniform queries, then the rest) is dealt into nqueues
    // queues by longest-processing-time-first on the walk steps, so the queues
    // carry about equal work; a query's chunks stay together in one queue
    const size_t split = (size_t)(std::find_if(order.begin(), order.end(), [&](size_t q) { return !uniform(q); }) -
                                  order.begin());
    for (int part = 0; part < 2; ++part) {
        const size_t o0 = part == 0 ? 0 : split, o1 = part == 0 ? split : order.size();
        const uint32_t base = (uint32_t)b.chunks.size();
        std::vector<std::vector<size_t>> bins(b.nqueues);
        std::vector<double> load(b.nqueues, 0.0);
        for (size_t oi = o0; oi < o1; ++oi) {
            const size_t q = order[oi];
            const size_t i = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
            bins[i].push_back(q);
            load[i] += cost(q);
        }
        for (uint32_t i = 0; i < b.nqueues; ++i) {
            b.qoff[part][i] = (uint32_t)b.chunks.size() - base;
            for (size_t q : bins[i]) emit(q);
        }
        b.qoff[part][b.nqueues] = (uint32_t)b.chunks.size() - base;
        if (part == 0) b.n_uniform = (uint32_t)b.chunks.size();
    }
}

}  // namespace

extern "C" int bd_query_batch(bd_graph* g, int64_t nq, const int32_t* s, const int32_t* t,
                              const double* eps, const int32_t* L, const uint32_t* uid,
                              uint64_t seed, const bd_policy* pol, const bd_exec* exec, void* stream,
                              bd_result* out, bd_stats* stats)
{
    if (!g || nq < 0 || (nq > 0 && (!s || !t || !eps || !L || !out))) return BD_E_INVALID;
    const double t0 = now_ms();
    if (stats) std::memset(stats, 0, sizeof(*stats));
    const bd_policy p = pol ? *pol : default_policy();
    bd_exec ex{};
    ex.mode = BD_MODE_BATCHED;
    if (exec) ex = *exec;
    for (int64_t i = 0; i < nq; ++i) {
        plan_one(g, s[i], t[i], eps[i], L[i], p, &out[i]);
        if (uid && uid[i] >= 0x80000000u) out[i].status = BD_E_INVALID;
    }
    std::lock_guard<std::mutex> lock(g->mu);
    Batch b;
    build_batch(g, nq, s, t, L, uid, seed, out, ex, policy_share(p), b);
    std::vector<double> beta;
    std::vector<uint8_t> incomplete;
    WorkPtrs wp;
    int rc = b.qd.empty() ? BD_OK : workspace_ptrs(g->ws, b, false, false, &wp);
    if (rc == BD_OK)
        rc = run_batch(g, b, ex, (hipStream_t)stream, wp, true, beta, stats, nullptr, nullptr, &incomplete);
    if (rc != BD_OK) return rc;
    for (size_t q = 0; q < b.qd.size(); ++q) {
        bd_result& r = out[b.index[q]];
        if (!incomplete.empty() && incomplete[q]) {
            r.status = BD_E_TIMEOUT;  // abandoned at the deadline
            r.beta = 0.0;
            continue;
        }
        r.beta = beta[q];
        if (stats) {
            stats->walk_steps += r.walk_steps;
            const int64_t M = (int64_t)policy_share(p);
            stats->walk_pairs += (int64_t)r.G * ((r.B + M - 1) / M) * r.R;
        }
    }
    if (stats) stats->total_ms = now_ms() - t0;
    return BD_OK;
}

static_assert(kScratchBytes == (size_t)BD_NOALLOC_SCRATCH_BYTES, "scratch size of the ABI");

extern "C" int bd_query_batch_noalloc(bd_graph* g, int64_t nq, const int32_t* s, const int32_t* t,
                                      const double* eps, const int32_t* L, const uint32_t* uid,
                                      uint64_t seed, const bd_policy* pol, const bd_exec* exec, void* stream,
                                      bd_result* out, bd_stats* stats)
{
    if (!g || nq < 0 || (nq > 0 && (!s || !t || !eps || !L || !out))) return BD_E_INVALID;
    const double t0 = now_ms();
    if (stats) std::memset(stats, 0, sizeof(*stats));
    const bd_policy p = pol ? *pol : default_policy();
    bd_exec ex{};
    ex.mode = BD_MODE_BATCHED;
    if (exec) ex = *exec;
    ex.use_graph = 0;
    for (int64_t i = 0; i < nq; ++i) {
        plan_one(g, s[i], t[i], eps[i], L[i], p, &out[i]);
        if (uid && uid[i] >= 0x80000000u) out[i].status = BD_E_INVALID;
    }
    Batch b;
    build_batch(g, nq, s, t, L, uid, seed, out, ex, policy_share(p), b);
    std::vector<double> beta;
    if (!b.qd.empty()) {
        int dev = -1;
        HIP_TRY(hipGetDevice(&dev));
        if (dev != g->device) return BD_E_INVALID;
        void* base = nullptr;
        std::unique_lock<std::mutex> held;
        int rc = scratch_acquire(dev, &base, &held);
        if (rc != BD_OK) return rc;
        WorkPtrs wp;
        rc = carve_ptrs(base, kScratchBytes, b, &wp);
        if (rc == BD_OK) rc = run_batch(g, b, ex, (hipStream_t)stream, wp, false, beta, stats, nullptr, nullptr);
        if (rc != BD_OK) return rc;
    }
    for (size_t q = 0; q < b.qd.size(); ++q) {
        bd_result& r = out[b.index[q]];
        r.beta = beta[q];
        if (stats) {
            stats->walk_steps += r.walk_steps;
            const int64_t M = (int64_t)policy_share(p);
            stats->walk_pairs += (int64_t)r.G * ((r.B + M - 1) / M) * r.R;
        }
    }
    if (stats) stats->total_ms = now_ms() - t0;
    return BD_OK;
}

extern "C" int bd_query_probes(bd_graph* g, int32_t s, int32_t t, double eps, int32_t L, uint32_t uid,
                               uint64_t seed, const bd_policy* pol, const bd_exec* exec, void* stream,
                               double* q_out, double* ybar_out, bd_result* out)
{
    if (!g || !out) return BD_E_INVALID;
    const bd_policy p = pol ? *pol : default_policy();
    bd_exec ex{};
    ex.mode = BD_MODE_PLAIN;
    if (exec) ex = *exec;
    plan_one(g, s, t, eps, L, p, out);
    if (uid >= 0x80000000u) out->status = BD_E_INVALID;
    if (out->status != BD_OK) return out->status;
    std::lock_guard<std::mutex> lock(g->mu);
    Batch b;
    build_batch(g, 1, &s, &t, &L, &uid, seed, out, ex, policy_share(p), b);
    std::vector<double> beta;
    WorkPtrs wp;
    int rc = workspace_ptrs(g->ws, b, q_out != nullptr, ybar_out != nullptr, &wp);
    if (rc == BD_OK) rc = run_batch(g, b, ex, (hipStream_t)stream, wp, true, beta, nullptr, q_out, ybar_out);
    if (rc != BD_OK) return rc;
    out->beta = beta[0];
    return BD_OK;
}

// ---------------------------------------------------------------------------
// Truncated series in binary64 and the spectral quantities of Lemma 2.3 /
// Theorem 3.8
// ---------------------------------------------------------------------------
extern "C" int bd_truncated_beta(bd_graph* g, int64_t nq, const int32_t* s, const int32_t* t, int32_t L,
                                 void* stream, double* beta_L)
{
    if (!g || nq < 0 || L < 0 || (nq > 0 && (!s || !t || !beta_L))) return BD_E_INVALID;
    for (int64_t i = 0; i < nq; ++i)
        if (s[i] < 0 || t[i] < 0 || s[i] >= g->n || t[i] >= g->n || s[i] == t[i]) return BD_E_INVALID;
    if (nq == 0) return BD_OK;
    std::lock_guard<std::mutex> lock(g->mu);
    hipStream_t st = (hipStream_t)stream;
    const uint32_t n = (uint32_t)g->n;
    const uint32_t* rp = g->rp32.as<const uint32_t>();
    const bool packed_ids = g->layout == 2 || g->layout == 3 || g->layout == 5;
    const uint32_t* col = packed_ids ? nullptr : g->col.as<const uint32_t>();
    const uint32_t* col24 = packed_ids ? g->col24.as<const uint32_t>() : nullptr;
    // queries per pass: three n x Q binary64 blocks within half the free device memory
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    const size_t per_q = (size_t)n * 8 * 3;
    const uint32_t Qmax = (uint32_t)std::max<size_t>(1, std::min<size_t>({64, (size_t)nq, free_b / 2 / per_q}));
    DevBuf dv, dy, dh, dsq, dlin;
    int rc = dv.alloc((size_t)n * Qmax * 8);
    if (rc == BD_OK) rc = dy.alloc((size_t)n * Qmax * 8);
    if (rc == BD_OK) rc = dh.alloc((size_t)n * Qmax * 8);
    if (rc == BD_OK) rc = dsq.alloc(Qmax * 8);
    if (rc == BD_OK) rc = dlin.alloc(Qmax * 8);
    if (rc != BD_OK) return rc;
    for (int64_t q0 = 0; q0 < nq; q0 += Qmax) {
        const uint32_t Q = (uint32_t)std::min<int64_t>(Qmax, nq - q0);
        const size_t bytes = (size_t)n * Q * 8;
        // v_0 = D^{-1} b_st in storage ids
        uint32_t ss[64], tt[64];
        double vs[64], vt[64];
        for (uint32_t q = 0; q < Q; ++q) {
            const int32_t a = s[q0 + q], b = t[q0 + q];
            ss[q] = storage_id(g, a);
            tt[q] = storage_id(g, b);
            vs[q] = 1.0 / (double)g->deg[(size_t)a];
            vt[q] = -1.0 / (double)g->deg[(size_t)b];
        }
        HIP_TRY(launch_zero(dv.p, bytes, st));
        HIP_TRY(launch_zero(dh.p, bytes, st));
        HIP_TRY(launch_series_seed(ss, tt, vs, vt, Q, dv.as<double>(), dh.as<double>(), st));
        for (int32_t i = 0; i < L; ++i) {
            HIP_TRY(launch_spmv_step(rp, col, col24, n, Q, dv.as<double>(), dy.as<double>(), dh.as<double>(), st));
            std::swap(dv.p, dy.p);
        }
        HIP_TRY(launch_colsum(dh.as<double>(), n, Q, dsq.as<double>(), dlin.as<double>(), st));
        std::vector<double> sq(Q), lin(Q);
        HIP_TRY(hipMemcpyAsync(sq.data(), dsq.p, Q * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(lin.data(), dlin.p, Q * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (uint32_t q = 0; q < Q; ++q) beta_L[q0 + q] = sq[q] - lin[q] * lin[q] / (double)n;
    }
    return BD_OK;
}

extern "C" int bd_graph_lambda(bd_graph* g, int32_t iters, uint64_t seed, void* stream, double* lambda)
{
    if (!g || iters < 1 || !lambda) return BD_E_INVALID;
    std::lock_guard<std::mutex> lock(g->mu);
    hipStream_t st = (hipStream_t)stream;
    const uint32_t n = (uint32_t)g->n;
    const uint32_t* rp = g->rp32.as<const uint32_t>();
    const bool packed_ids = g->layout == 2 || g->layout == 3 || g->layout == 5;
    const uint32_t* col = packed_ids ? nullptr : g->col.as<const uint32_t>();
    const uint32_t* col24 = packed_ids ? g->col24.as<const uint32_t>() : nullptr;
    DevBuf phi, x, y, z, part, scal;
    int rc = phi.alloc((size_t)n * 8);
    if (rc == BD_OK) rc = x.alloc((size_t)n * 8);
    if (rc == BD_OK) rc = y.alloc((size_t)n * 8);
    if (rc == BD_OK) rc = z.alloc((size_t)n * 8);
    if (rc == BD_OK) rc = part.alloc(2 * 1024 * 8);
    if (rc == BD_OK) rc = scal.alloc(2 * 8);
    if (rc != BD_OK) return rc;
    HIP_TRY(launch_lambda(rp, col, col24, n, (uint32_t)g->nnz, iters, seed, phi.as<double>(), x.as<double>(),
                          y.as<double>(), z.as<double>(), part.as<double>(), scal.as<double>(), st));
    double sc[2] = {0.0, 0.0};
    HIP_TRY(hipMemcpyAsync(sc, scal.p, sizeof(sc), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *lambda = sc[1];
    return BD_OK;
}

extern "C" int bd_theorem_L(const bd_graph* g, int64_t nq, const int32_t* s, const int32_t* t, const double* eps,
                            double lambda, int32_t* L)
{
    if (!g || nq < 0 || (nq > 0 && (!s || !t || !eps || !L))) return BD_E_INVALID;
    if (!(lambda > 0.0 && lambda < 1.0)) return BD_E_RANGE;
    for (int64_t i = 0; i < nq; ++i) {
        if (s[i] < 0 || t[i] < 0 || s[i] >= g->n || t[i] >= g->n || s[i] == t[i] || !(eps[i] > 0 && eps[i] < 1))
            return BD_E_INVALID;
        const double inv = 1.0 / g->deg[(size_t)s[i]] + 1.0 / g->deg[(size_t)t[i]];
        const double arg = 96.0 * (double)g->n / (eps[i] * (1.0 - lambda) * (1.0 - lambda) * inv * inv);
        const double v = std::ceil(std::log(arg) / std::log(1.0 / lambda) * kCeilGuard);
        L[i] = v > (double)kMaxL ? kMaxL + 1 : (int32_t)std::max(0.0, v);
    }
    return BD_OK;
}

extern "C" int bd_query_stabilized(bd_graph* g, int64_t nq, const int32_t* s, const int32_t* t,
                                   const double* eps, int32_t L_max, const uint32_t* uid, uint64_t seed,
                                   const bd_policy* pol, const bd_exec* exec, void* stream, bd_result* out,
                                   int32_t* L_stop)
{
    if (!g || nq < 0 || (nq > 0 && (!s || !t || !eps || !out || !L_stop)) || L_max < 1 || L_max > kMaxL)
        return BD_E_INVALID;
    bd_exec ex{};
    ex.mode = BD_MODE_BATCHED;
    if (exec) ex = *exec;
    std::vector<uint32_t> ids((size_t)nq);
    for (int64_t i = 0; i < nq; ++i) ids[(size_t)i] = uid ? uid[i] : (uint32_t)i;
    // estimate at L for the listed queries (their own uids, so each estimate
    // equals the one bd_query_batch gives for that query and L)
    auto run = [&](const std::vector<int64_t>& idx, const std::vector<int32_t>& Ls, std::vector<bd_result>& res) {
        const size_t m = idx.size();
        std::vector<int32_t> ss(m), tt(m);
        std::vector<double> ee(m);
        std::vector<uint32_t> uu(m);
        for (size_t j = 0; j < m; ++j) {
            ss[j] = s[idx[j]];
            tt[j] = t[idx[j]];
            ee[j] = eps[idx[j]];
            uu[j] = ids[(size_t)idx[j]];
        }
        res.assign(m, bd_result{});
        return bd_query_batch(g, (int64_t)m, ss.data(), tt.data(), ee.data(), Ls.data(), uu.data(), seed, pol,
                              &ex, stream, res.data(), nullptr);
    };
    std::vector<int64_t> live;
    std::vector<bd_result> prev((size_t)nq);  // estimate at the current L
    std::vector<int32_t> curL((size_t)nq, 1);
    for (int64_t i = 0; i < nq; ++i) {
        live.push_back(i);
        L_stop[i] = 0;
    }
    {  // L0 = 1
        std::vector<int32_t> Ls(live.size(), 1);
        std::vector<bd_result> res;
        const int rc = run(live, Ls, res);
        if (rc != BD_OK) return rc;
        for (size_t j = 0; j < live.size(); ++j) prev[(size_t)live[j]] = res[j];
    }
    std::vector<int64_t> next;
    for (int64_t i : live) {
        if (prev[(size_t)i].status != BD_OK) {
            out[i] = prev[(size_t)i];
            L_stop[i] = 1;
        } else if (L_max == 1) {
            out[i] = prev[(size_t)i];
            L_stop[i] = 1;
        } else {
            next.push_back(i);
        }
    }
    live.swap(next);
    while (!live.empty()) {
        std::vector<int32_t> Ls(live.size());
        for (size_t j = 0; j < live.size(); ++j) Ls[j] = std::min<int32_t>(2 * curL[(size_t)live[j]], L_max);
        std::vector<bd_result> res;
        const int rc = run(live, Ls, res);
        if (rc != BD_OK) return rc;
        next.clear();
        for (size_t j = 0; j < live.size(); ++j) {
            const int64_t i = live[j];
            const bd_result& r2 = res[j];
            const bd_result& r1 = prev[(size_t)i];
            const bool stable = r2.status == BD_OK && std::fabs(r2.beta - r1.beta) <= 0.5 * eps[i] * std::fabs(r2.beta);
            if (r2.status != BD_OK || stable || Ls[j] >= L_max) {
                out[i] = r2;
                L_stop[i] = Ls[j];
            } else {
                prev[(size_t)i] = r2;
                curL[(size_t)i] = Ls[j];
                next.push_back(i);
            }
        }
        live.swap(next);
    }
    return BD_OK;
}

extern "C" int bd_autotune(bd_graph* g, int64_t nq, const int32_t* s, const int32_t* t, const double* eps,
                           const int32_t* L, uint64_t seed, const bd_policy* pol, uint32_t mode, void* stream,
                           bd_exec* best, double* times_ms, int32_t* n_candidates)
{
    if (!g || !best || nq < 1 || !s || !t || !eps || !L) return BD_E_INVALID;
    const int32_t cands[8] = {128, 256, 512, 1024, 2048, 4096, 8192, 16384};
    std::vector<bd_result> res((size_t)nq);
    double best_ms = 1e300;
    int n = 0;
    auto trial = [&](const bd_exec& ex) -> int {
        bd_stats st{};
        const int rc = bd_query_batch(g, nq, s, t, eps, L, nullptr, seed, pol, &ex, stream, res.data(), &st);
        if (rc != BD_OK) return rc;
        if (times_ms) times_ms[n] = st.walk_kernel_ms;
        ++n;
        if (st.walk_kernel_ms < best_ms) {
            best_ms = st.walk_kernel_ms;
            *best = ex;
        }
        return BD_OK;
    };
    for (int i = 0; i < 8; ++i) {
        bd_exec ex{};
        ex.mode = mode;
        ex.chunk_pairs = mode == BD_MODE_PLAIN ? std::max(cands[i] / 16, 64) : cands[i];
        ex.queues = (int32_t)kMaxQueues;
        const int rc = trial(ex);
        if (rc != BD_OK) return rc;
    }
    if (mode != BD_MODE_PLAIN) {
        bd_exec ex = *best;
        ex.queues = 1;
        const int rc = trial(ex);
        if (rc != BD_OK) return rc;
    }
    if (n_candidates) *n_candidates = n;
    return BD_OK;
}

// ---------------------------------------------------------------------------
// Validation entry points
// ---------------------------------------------------------------------------
extern "C" int bd_walk_trace(bd_graph* g, int64_t count, const int32_t* start, const uint32_t* uid,
                             const uint32_t* k, const uint32_t* p, const uint32_t* side, int32_t L,
                             uint64_t seed, void* stream, int32_t* trace, float* acc)
{
    if (!g || count < 0 || L < 0 || L > kMaxL) return BD_E_INVALID;
    if (count == 0) return BD_OK;
    if (!start || !uid || !k || !p || !side || count > 0x7FFFFFFF) return BD_E_INVALID;
    for (int64_t i = 0; i < count; ++i)
        if (start[i] < 0 || start[i] >= g->n || side[i] > 1u || uid[i] >= 0x80000000u || p[i] == 0xFFFFFFFFu)
            return BD_E_INVALID;
    hipStream_t st = (hipStream_t)stream;
    const size_t c = (size_t)count;
    DevBuf ds, du, dk, dp, dsd, dt, da;
    int rc = ds.alloc(c * 4);
    if (rc == BD_OK) rc = du.alloc(c * 4);
    if (rc == BD_OK) rc = dk.alloc(c * 4);
    if (rc == BD_OK) rc = dp.alloc(c * 4);
    if (rc == BD_OK) rc = dsd.alloc(c * 4);
    if (rc == BD_OK && trace) rc = dt.alloc(c * (size_t)(L + 1) * 4);
    if (rc == BD_OK && acc) rc = da.alloc(c * 4);
    if (rc != BD_OK) return rc;
    std::vector<int32_t> start_store(start, start + c);
    for (auto& v : start_store) v = (int32_t)storage_id(g, v);
    HIP_TRY(hipMemcpyAsync(ds.p, start_store.data(), c * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(du.p, uid, c * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dk.p, k, c * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dp.p, p, c * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dsd.p, side, c * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(launch_trace(tables(g), g->kernel_layout, (uint32_t)c, ds.as<int32_t>(),
                         du.as<uint32_t>(), dk.as<uint32_t>(), dp.as<uint32_t>(), dsd.as<uint32_t>(), L,
                         (uint32_t)seed, (uint32_t)(seed >> 32), trace ? dt.as<int32_t>() : nullptr,
                         acc ? da.as<float>() : nullptr, st));
    if (trace) HIP_TRY(hipMemcpyAsync(trace, dt.p, c * (size_t)(L + 1) * 4, hipMemcpyDeviceToHost, st));
    if (acc) HIP_TRY(hipMemcpyAsync(acc, da.p, c * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (trace && !g->external.empty())
        for (size_t i = 0; i < c * (size_t)(L + 1); ++i) trace[i] = (int32_t)g->external[(size_t)trace[i]];
    return BD_OK;
}

extern "C" int bd_probe_eval(bd_graph* g, uint64_t seed, uint32_t uid, uint32_t k, int64_t count,
                             const uint32_t* nodes, void* stream, uint32_t* pi, int8_t* z)
{
    if (!g || count < 0 || uid >= 0x80000000u) return BD_E_INVALID;
    if (count == 0) return BD_OK;
    if (!nodes || count > 0x7FFFFFFF) return BD_E_INVALID;
    for (int64_t i = 0; i < count; ++i)
        if (nodes[i] >= (uint64_t)g->n) return BD_E_INVALID;
    hipStream_t st = (hipStream_t)stream;
    const size_t c = (size_t)count;
    DevBuf dn, dpi, dz;
    int rc = dn.alloc(c * 4);
    if (rc == BD_OK && pi) rc = dpi.alloc(c * 4);
    if (rc == BD_OK && z) rc = dz.alloc(c);
    if (rc != BD_OK) return rc;
    HIP_TRY(hipMemcpyAsync(dn.p, nodes, c * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(launch_probe_eval(tables(g), (uint32_t)seed, (uint32_t)(seed >> 32), uid, k, (uint32_t)c,
                              dn.as<uint32_t>(), pi ? dpi.as<uint32_t>() : nullptr,
                              z ? dz.as<int8_t>() : nullptr, st));
    if (pi) HIP_TRY(hipMemcpyAsync(pi, dpi.p, c * 4, hipMemcpyDeviceToHost, st));
    if (z) HIP_TRY(hipMemcpyAsync(z, dz.p, c, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return BD_OK;
}

// ---------------------------------------------------------------------------
// Gather roofline
// ---------------------------------------------------------------------------
extern "C" int bd_gather_roofline(bd_graph* g, int32_t chains_per_lane, int32_t steps, int32_t work_groups,
                                  void* stream, bd_roofline* out)
{
    if (!g || !out || steps < 1 ||
        (chains_per_lane != 1 && chains_per_lane != 2 && chains_per_lane != 4 && chains_per_lane != 8))
        return BD_E_INVALID;
    hipStream_t st = (hipStream_t)stream;
    uint32_t grid = work_groups > 0 ? (uint32_t)work_groups : 4u * (uint32_t)resident_wgs(g, 1, 1);
    DevBuf sink;
    const int wg = block_threads(g->kernel_layout, 1);
    int rc = sink.alloc((size_t)grid * wg * 4);
    if (rc != BD_OK) return rc;
    const int fat = g->layout == 1;
    // warm-up launch (caches, clocks), then the timed one
    HIP_TRY(launch_gather(tables(g), g->kernel_layout, chains_per_lane, grid, std::min(steps, 64), 1u, sink.as<uint32_t>(), st));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, st));
    HIP_TRY(launch_gather(tables(g), g->kernel_layout, chains_per_lane, grid, steps, 2u, sink.as<uint32_t>(), st));
    HIP_TRY(hipEventRecord(e1, st));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const double n = (double)grid * wg * chains_per_lane * steps;
    out->ms = ms;
    out->steps = (int64_t)n;
    out->steps_per_s = n / (ms * 1e-3);
    out->gathers_per_s = out->steps_per_s * (fat ? 1.0 : 2.0);
    out->chains_per_lane = chains_per_lane;
    out->work_groups = (int32_t)grid;
    return BD_OK;
}

// ---------------------------------------------------------------------------
// Misc
// ---------------------------------------------------------------------------
extern "C" const char* bd_strerror(int code)
{
    switch (code) {
    case BD_OK: return "ok";
    case BD_E_INVALID: return "invalid argument";
    case BD_E_GRAPH: return "graph is not simple, symmetric, sorted and connected";
    case BD_E_RANGE: return "size beyond the library limits";
    case BD_E_BUDGET: return "walk budget beyond the cap or K, R >= 2^32";
    case BD_E_HIP: return "HIP runtime error";
    case BD_E_NOMEM: return "out of memory";
    case BD_E_NODEVICE: return "no usable GPU";
    case BD_E_NOTFOUND: return "unknown request id";
    case BD_E_FULL: return "request exceeds the admission caps";
    case BD_E_CANCELLED: return "request cancelled";
    case BD_E_TIMEOUT: return "timed out";
    case BD_E_SCRATCH: return "batch exceeds the fixed scratch array of the allocation-free entry point";
    default: return "unknown error";
    }
}

extern "C" int bd_device_info(char* buf, size_t len)
{
    if (!buf || len == 0) return BD_E_INVALID;
    int dev = 0, ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        std::snprintf(buf, len, "no device");
        return BD_E_NODEVICE;
    }
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t p;
    HIP_TRY(hipGetDeviceProperties(&p, dev));
    std::snprintf(buf, len, "%s (%s), %d CUs, %d MHz, %.1f GiB, L2 %d KiB", p.name, p.gcnArchName,
                  p.multiProcessorCount, p.clockRate / 1000, (double)p.totalGlobalMem / (1 << 30),
                  p.l2CacheSize / 1024);
    return BD_OK;
}

// ---------------------------------------------------------------------------
// Served mode: continuous batching
//
// A scheduler thread keeps a table of resident queries ("slots") on the
// device. Each scheduling slice is one persistent walk launch over chunks
// taken round-robin over the admitted requests (and within a request over its
// queries), so a request that arrives while others run joins the very next
// slice, its work shares the device with theirs, and a small request is not
// held back by the size of a large one. Two slices are in flight on two
// streams, so the next slice's work groups take over compute units as the
// current slice's finish. The work group that finishes a query posts (slot,
// beta) to its slice's completion ring and clears the slot's tables; the host
// frees the slot when it reads the ring. Admission is FIFO under caps on
// resident queries and accumulator memory and, optionally, outstanding walk
// steps.
// ---------------------------------------------------------------------------
namespace {

struct PinnedBuf {
    void* p = nullptr;
    size_t bytes = 0;
    PinnedBuf() = default;
    PinnedBuf(const PinnedBuf&) = delete;
    PinnedBuf& operator=(const PinnedBuf&) = delete;
    ~PinnedBuf()
    {
        if (p) (void)hipHostFree(p);
    }
    int alloc(size_t b)
    {
        if (hipHostMalloc(&p, b, hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            return BD_E_NOMEM;
        }
        bytes = b;
        return BD_OK;
    }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

struct Request {
    std::vector<bd_result> res;
    std::vector<QueryDesc> desc;  // valid queries
    std::vector<int64_t> index;   // valid query -> result index
    int64_t remaining = 0;
    uint64_t steps = 0;
    uint64_t split_probes = 0;    // accumulators its split queries need
    double t_submit = 0, t_done = 0;
    bool done = false;
    std::deque<uint32_t> rr_slots;  // admitted queries with chunks left to hand out
    bool in_rr = false;             // the request is in the server's round-robin
    std::vector<uint32_t> slots;    // slots taken at admission
    bool admitted = false;
    bool cancelled = false;         // bd_server_cancel: no further chunk is handed out
    uint64_t left_steps = 0;        // walk steps not yet handed out (slice ordering)
    uint64_t cancel_mark = 0;       // slices launched when it was cancelled
};

struct SlotState {
    bool busy = false;         // held by a query of request `req`
    uint64_t req = 0;
    int64_t ridx = 0;
    ChunkCursor cur;           // next chunk of this query
    uint32_t L = 0;
    uint64_t steps = 0;        // walk steps of the query
    bool uniform = false;      // R >= kUniformMinR
    uint32_t psum_base = 0, psum_n = 0;  // accumulator range of a query with split probes
};

// First-fit allocator of per-probe accumulator ranges (units: probes).
struct RangeAlloc {
    std::map<uint32_t, uint32_t> free_;  // offset -> length
    void init(uint32_t n)
    {
        free_.clear();
        if (n) free_[0] = n;
    }
    bool alloc(uint32_t n, uint32_t* off)
    {
        if (n == 0) {
            *off = 0;
            return true;
        }
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                const uint32_t rest = it->second - n, o = it->first + n;
                free_.erase(it);
                if (rest) free_[o] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint32_t off, uint32_t n)
    {
        if (n == 0) return;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Slice {
    double max_cost = 0;  // largest chunk cost (L + 1) * passes over the work group's lanes
    double sum_cost = 0;  // summed chunk costs
    PinnedBuf chunks_h;
    DevBuf chunks_d;
    DevBuf d_cursor;   // chunk cursors of the slice's launches
    DevBuf d_comp;     // completion ring: [u32 count, pad to 16 B][Completion x cap]
    PinnedBuf comp_h;  // host copy of d_comp after the slice
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    uint32_t n = 0;
    uint32_t n_uniform = 0;  // chunks [0, n_uniform) have R >= kUniformMinR
    bool inflight = false;
    uint64_t steps = 0;
    double t_launch = 0;
};

constexpr uint32_t kSliceMaxChunks = 1u << 18;

}  // namespace

struct bd_server {
    bd_graph* g = nullptr;
    bd_server_cfg cfg{};
    bd_policy pol{};
    hipStream_t st = nullptr;    // descriptor copies at admission
    hipEvent_t ev_admit = nullptr;
    bool admit_recorded = false;
    uint32_t slots = 0, gdim = 0;
    int resident[2] = {0, 0};  // resident work groups: [0] small-R kernel, [1] wave-uniform kernel
    DevBuf d_qd, d_bs, d_done, d_beta, d_psum, d_pcount;
    PinnedBuf h_qd;
    uint32_t arena = 0;  // per-probe accumulators for split probes
    RangeAlloc psum_alloc;
    Slice slice[2];
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread th;
    bool stop = false;
    int broken = BD_OK;
    std::map<uint64_t, Request> reqs;
    std::deque<uint64_t> pending;
    uint64_t next_id = 1;
    std::vector<uint32_t> free_slots;
    std::vector<SlotState> slot;
    std::deque<uint64_t> rr;  // requests with chunks left, round-robin
    uint64_t inflight_steps = 0;
    uint64_t slices_launched = 0, slices_done = 0;
    std::vector<uint64_t> cancelled;  // admitted requests waiting for their slots to be reclaimed
    double steps_per_ms = 5e7;
    double t_last_done = 0;
    // a lane's time per walk step (ms): a chunk needs about (L + 1) steps per
    // pass of the work group over its pairs, however few pairs it has
    double ms_per_lane_step = 1e-3;
    // The last kRateWindow completed slices: walk steps, summed chunk costs,
    // and the time from the later of the slice's launch and the previous
    // completion to its own completion. Slices overlap (two are in flight, and
    // one holding a few long chunks runs beside the next), so one slice's
    // interval can be far shorter than its work took; but the intervals of
    // consecutive slices tile the busy time, so the sums over the window give
    // the device's rate.
    static constexpr int kRateWindow = 8;
    double win_steps[kRateWindow] = {}, win_cost[kRateWindow] = {}, win_ms[kRateWindow] = {};
    int win_next = 0;
};

namespace {

// How the server cuts queries into chunks: as the batched mode, with at most
// one pass of a work group per chunk (its pairs fit the group's lanes). A
// chunk takes about (L + 1) lane steps per pass, and under load a lane step
// waits on a loaded memory system (several microseconds on the fat layout),
// so a chunk of several passes would hold its slice, and every request that
// arrives meanwhile, open for tens of milliseconds.
bd_exec server_exec(const bd_server* S)
{
    bd_exec ex{};
    ex.mode = BD_MODE_BATCHED;
    ex.chunk_probes = S->cfg.chunk_probes;
    ex.chunk_pairs = group_pairs(S->g->kernel_layout, share_class(policy_share(S->pol)));
    return ex;
}

size_t comp_bytes(const bd_server* S)
{
    return 16 + (size_t)S->slots * sizeof(Completion);
}

// completions copied back after every slice; a slice that finishes more
// queries than this has the rest fetched when it is read
constexpr uint32_t kCompPrefix = 4096;

size_t comp_prefix_bytes(const bd_server* S)
{
    return 16 + (size_t)std::min(S->slots, kCompPrefix) * sizeof(Completion);
}

void finish_request(bd_server* S, uint64_t id, Request& r)
{
    (void)id;
    r.done = true;
    r.t_done = now_ms();
    S->cv_done.notify_all();
}

// Move pending requests into slots (FIFO) while the caps allow. Caller holds mu.
int admit(bd_server* S)
{
    while (!S->pending.empty()) {
        const uint64_t id = S->pending.front();
        Request& r = S->reqs[id];
        const size_t need = r.desc.size();
        if (need > S->free_slots.size()) break;
        const uint64_t cap = S->cfg.max_steps_inflight;
        if (cap && S->inflight_steps > 0 && S->inflight_steps + r.steps > cap) break;
        // memory admission: accumulators of split probes, all or nothing
        const bd_exec ex = server_exec(S);
        std::vector<uint32_t> base(need, 0);
        bool fits = true;
        for (size_t i = 0; i < need && fits; ++i) {
            const QueryDesc& d = r.desc[i];
            if (chunk_plan(ex, d, S->g->kernel_layout).part && !S->psum_alloc.alloc(d.K, &base[i])) {
                for (size_t j = 0; j < i; ++j)
                    if (chunk_plan(ex, r.desc[j], S->g->kernel_layout).part) S->psum_alloc.release(base[j], r.desc[j].K);
                fits = false;
            }
        }
        if (!fits) break;
        S->pending.pop_front();
        r.admitted = true;
        r.left_steps = r.steps;
        if (need > 0 && !r.in_rr) {
            S->rr.push_back(id);
            r.in_rr = true;
        }
        std::vector<uint32_t> taken(need);
        for (size_t i = 0; i < need; ++i) {
            const uint32_t sl = S->free_slots.back();
            S->free_slots.pop_back();
            taken[i] = sl;
            QueryDesc d = r.desc[i];
            d.slot = sl;
            d.psum_base = base[i];
            S->h_qd.as<QueryDesc>()[sl] = d;
            SlotState& ss = S->slot[sl];
            ss.busy = true;
            ss.req = id;
            r.slots.push_back(sl);
            ss.ridx = r.index[i];
            ss.cur = ChunkCursor(sl, d, ex, S->g->kernel_layout);
            ss.L = (uint32_t)d.L;
            ss.steps = (uint64_t)r.res[(size_t)ss.ridx].walk_steps;
            ss.uniform = d.R >= kUniformMinR;
            ss.psum_base = base[i];
            ss.psum_n = ss.cur.plan.part ? d.K : 0;
            S->inflight_steps += ss.steps;
            r.rr_slots.push_back(sl);
        }
        // descriptors to the device, one copy per run of consecutive slots
        std::sort(taken.begin(), taken.end());
        for (size_t i = 0; i < need;) {
            size_t j = i + 1;
            while (j < need && taken[j] == taken[j - 1] + 1) ++j;
            if (hipMemcpyAsync(S->d_qd.as<QueryDesc>() + taken[i], S->h_qd.as<QueryDesc>() + taken[i],
                               (j - i) * sizeof(QueryDesc), hipMemcpyHostToDevice, S->st) != hipSuccess)
                return BD_E_HIP;
            i = j;
        }
        if (need > 0) {
            // slices launched from now on wait for these descriptor copies
            if (hipEventRecord(S->ev_admit, S->st) != hipSuccess) return BD_E_HIP;
            S->admit_recorded = true;
        }
    }
    return BD_OK;
}

// Read the completion ring of a finished slice. Caller holds mu.
int process_completions(bd_server* S, const Slice& sl)
{
    const uint32_t count = std::min(*sl.comp_h.as<const uint32_t>(), S->slots);
    if (count > kCompPrefix) {
        const size_t off = 16 + (size_t)kCompPrefix * sizeof(Completion);
        if (hipMemcpy(sl.comp_h.as<char>() + off, sl.d_comp.as<char>() + off,
                      (size_t)(count - kCompPrefix) * sizeof(Completion), hipMemcpyDeviceToHost) != hipSuccess)
            return BD_E_HIP;
    }
    const Completion* ring = reinterpret_cast<const Completion*>(sl.comp_h.as<const char>() + 16);
    for (uint32_t i = 0; i < count; ++i) {
        const Completion c = ring[i];
        SlotState& ss = S->slot[c.slot];
        auto it = S->reqs.find(ss.req);
        if (it != S->reqs.end()) {
            Request& r = it->second;
            r.res[(size_t)ss.ridx].beta = c.beta;
            if (--r.remaining == 0) finish_request(S, ss.req, r);
        }
        S->inflight_steps -= std::min(S->inflight_steps, ss.steps);
        S->psum_alloc.release(ss.psum_base, ss.psum_n);
        ss.psum_n = 0;
        ss.busy = false;
        S->free_slots.push_back(c.slot);
    }
    return BD_OK;
}

// Cancelled requests whose slots no launched slice can touch any more: clear
// the slots' device state (block sums, probe counter, split-probe
// accumulators) on the admission stream, which every later slice waits for,
// free them, and finish the request with BD_E_CANCELLED for the queries that
// had not finished. Caller holds mu.
int reclaim_cancelled(bd_server* S)
{
    for (size_t i = 0; i < S->cancelled.size();) {
        const uint64_t id = S->cancelled[i];
        auto it = S->reqs.find(id);
        if (it == S->reqs.end()) {
            S->cancelled.erase(S->cancelled.begin() + (ptrdiff_t)i);
            continue;
        }
        Request& r = it->second;
        if (S->slices_done < r.cancel_mark) {
            ++i;
            continue;
        }
        bool zeroed = false;
        for (uint32_t sl : r.slots) {
            SlotState& ss = S->slot[sl];
            if (!ss.busy || ss.req != id) continue;  // finished (and recycled by its work group) already
            if (launch_zero(S->d_bs.as<char>() + (size_t)sl * S->gdim * 16, (size_t)S->gdim * 16, S->st) !=
                    hipSuccess ||
                launch_zero(S->d_done.as<uint32_t>() + sl, 4, S->st) != hipSuccess ||
                (ss.psum_n && (launch_zero(S->d_psum.as<char>() + (size_t)ss.psum_base * 32, (size_t)ss.psum_n * 32,
                                           S->st) != hipSuccess ||
                               launch_zero(S->d_pcount.as<uint32_t>() + ss.psum_base, (size_t)ss.psum_n * 4,
                                           S->st) != hipSuccess)))
                return BD_E_HIP;
            zeroed = true;
            r.res[(size_t)ss.ridx].status = BD_E_CANCELLED;
            r.res[(size_t)ss.ridx].beta = 0.0;
            S->inflight_steps -= std::min(S->inflight_steps, ss.steps);
            S->psum_alloc.release(ss.psum_base, ss.psum_n);
            ss.psum_n = 0;
            ss.busy = false;
            S->free_slots.push_back(sl);
            --r.remaining;
        }
        if (zeroed) {
            // slices launched from now on wait for the clearing
            if (hipEventRecord(S->ev_admit, S->st) != hipSuccess) return BD_E_HIP;
            S->admit_recorded = true;
        }
        if (!r.done) finish_request(S, id, r);
        S->cancelled.erase(S->cancelled.begin() + (ptrdiff_t)i);
    }
    return BD_OK;
}

// Take chunks round-robin for one slice. Caller holds mu.
// A slice lasts at least as long as its longest chunk, so its work target is
// the larger of slice_ms and four times that chunk's expected time: a slice
// then holds several chunks per work group and its tail stays short. Within
// the slice, the longest chunks start first.
void fill_slice(bd_server* S, Slice& sl)
{
    const double slice_ms = S->cfg.slice_ms > 0 ? S->cfg.slice_ms : 20.0;
    const double small_share = S->cfg.small_first < 0 ? 0.0 : S->cfg.small_first > 0 ? std::min(S->cfg.small_first, 1.0)
                                                                                    : 0.5;
    Chunk* out = sl.chunks_h.as<Chunk>();
    sl.n = 0;
    sl.steps = 0;
    sl.max_cost = 0;
    sl.sum_cost = 0;
    double target = slice_ms * S->steps_per_ms;
    struct Item {
        double cost;
        Chunk c;
    };
    std::vector<Item> big, small;  // wave-uniform chunks, then the rest
    const uint64_t wg = (uint64_t)group_pairs(S->g->kernel_layout, share_class(policy_share(S->pol)));
    auto room = [&] { return big.size() + small.size() < kSliceMaxChunks; };
    // one chunk of request r (its next query in turn); false when it has none left
    auto take = [&](Request& r) {
        if (r.rr_slots.empty()) return false;
        const uint32_t q = r.rr_slots.front();
        r.rr_slots.pop_front();
        SlotState& ss = S->slot[q];
        const uint64_t cs = ss.cur.chunk_steps(ss.L);
        sl.steps += cs;
        r.left_steps -= std::min(r.left_steps, cs);
        const Chunk c = ss.cur.next();
        const double cost = ((double)ss.L + 1.0) * (double)(((uint64_t)c.gc * c.pc + wg - 1) / wg);
        sl.sum_cost += cost;
        if (cost > sl.max_cost) {
            sl.max_cost = cost;
            target = std::max(target, 4.0 * cost * S->ms_per_lane_step * S->steps_per_ms);
        }
        (ss.uniform ? big : small).push_back(Item{cost, c});
        if (!ss.cur.done()) r.rr_slots.push_back(q);
        return true;
    };
    // First the requests with the least work left, smallest first, up to
    // small_share of the slice: a short request that arrives under load
    // finishes in the next slice or two instead of waiting its turn behind
    // long ones; the rest of the slice is round-robin, so none starves.
    if (small_share > 0.0 && S->rr.size() > 1) {
        std::vector<uint64_t> order(S->rr.begin(), S->rr.end());
        std::stable_sort(order.begin(), order.end(),
                         [&](uint64_t a, uint64_t b) { return S->reqs[a].left_steps < S->reqs[b].left_steps; });
        for (uint64_t id : order) {
            Request& r = S->reqs[id];
            if (r.cancelled) continue;
            while ((double)sl.steps < small_share * target && room() && take(r)) {
            }
            if (r.rr_slots.empty()) {
                S->rr.erase(std::find(S->rr.begin(), S->rr.end(), id));
                r.in_rr = false;
            }
            if ((double)sl.steps >= small_share * target || !room()) break;
        }
    }
    while (!S->rr.empty() && room() &&
           ((double)sl.steps < target || big.size() + small.size() < (size_t)S->resident[1])) {
        const uint64_t id = S->rr.front();
        S->rr.pop_front();
        Request& r = S->reqs[id];
        if (r.cancelled) {
            r.in_rr = false;
            continue;
        }
        take(r);
        if (!r.rr_slots.empty()) S->rr.push_back(id);
        else r.in_rr = false;
    }
    auto longest_first = [](const Item& a, const Item& b) { return a.cost > b.cost; };
    std::stable_sort(big.begin(), big.end(), longest_first);
    std::stable_sort(small.begin(), small.end(), longest_first);
    for (const Item& it : big) out[sl.n++] = it.c;
    // The wave-uniform chunks get a launch of their own only when they can fill
    // the device; otherwise the general kernel (which runs any chunk) takes them
    // at the head of its table, so the slice is one launch and no part of it
    // waits for a nearly empty one.
    sl.n_uniform = sl.n >= (uint32_t)S->resident[1] ? sl.n : 0u;
    for (const Item& it : small) out[sl.n++] = it.c;
}

int launch_slice(bd_server* S, Slice& sl)
{
    hipStream_t st = sl.st;
    if (S->admit_recorded && hipStreamWaitEvent(st, S->ev_admit, 0) != hipSuccess) return BD_E_HIP;
    if (hipMemcpyAsync(sl.chunks_d.p, sl.chunks_h.p, (size_t)sl.n * sizeof(Chunk), hipMemcpyHostToDevice, st) !=
        hipSuccess)
        return BD_E_HIP;
    if (launch_zero(sl.d_cursor.p, 16, st) != hipSuccess) return BD_E_HIP;
    if (launch_zero(sl.d_comp.p, 16, st) != hipSuccess) return BD_E_HIP;
    // the slice's chunk table holds the wave-uniform chunks first
    WalkArgs a{};
    a.g = tables(S->g);
    a.qd = S->d_qd.as<const QueryDesc>();
    a.chunks = sl.chunks_d.as<const Chunk>();
    a.nchunks = sl.n;
    a.gdim = S->gdim;
    a.cursor = sl.d_cursor.as<uint32_t>();
    a.blocksum = S->d_bs.as<unsigned long long>();
    a.done = S->d_done.as<uint32_t>();
    a.psum = S->d_psum.as<unsigned long long>();
    a.pcount = S->d_pcount.as<uint32_t>();
    a.beta = S->d_beta.as<double>();
    a.comp_count = sl.d_comp.as<uint32_t>();
    a.comp_ring = reinterpret_cast<Completion*>(sl.d_comp.as<char>() + 16);
    a.comp_cap = S->slots;
    a.recycle = 1;
    a.persistent = 1;
    const uint32_t parts[3] = {0u, sl.n_uniform, sl.n};
    for (int part = 0; part < 2; ++part) {
        WalkArgs ap = a;
        ap.chunks = sl.chunks_d.as<const Chunk>() + parts[part];
        ap.nchunks = parts[part + 1] - parts[part];
        ap.cursor = sl.d_cursor.as<uint32_t>() + part;
        ap.nqueues = 1;
        ap.qoff[0] = 0;
        ap.qoff[1] = ap.nchunks;
        const uint32_t grid = std::min<uint32_t>((uint32_t)S->resident[part == 0], ap.nchunks);
        if (grid && launch_walk(ap, run_kernel(S->g, share_class(policy_share(S->pol))), part == 0,
                                share_class(policy_share(S->pol)), grid, st) !=
                        hipSuccess)
            return BD_E_HIP;
    }
    if (hipMemcpyAsync(sl.comp_h.p, sl.d_comp.p, comp_prefix_bytes(S), hipMemcpyDeviceToHost, st) != hipSuccess)
        return BD_E_HIP;
    if (hipEventRecord(sl.ev, st) != hipSuccess) return BD_E_HIP;
    sl.inflight = true;
    sl.t_launch = now_ms();
    ++S->slices_launched;
    return BD_OK;
}

void fail_all(bd_server* S, int code)
{
    for (auto& kv : S->reqs) {
        Request& r = kv.second;
        if (r.done) continue;
        for (auto& x : r.res)
            if (x.status == BD_OK) x.status = code;
        finish_request(S, kv.first, r);
    }
    S->pending.clear();
    S->rr.clear();
}

void server_loop(bd_server* S)
{
    int cur = 0;
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        S->cv_work.wait(lk, [&] {
            return S->stop || !S->pending.empty() || !S->rr.empty() || S->slice[0].inflight ||
                   S->slice[1].inflight || !S->cancelled.empty();
        });
        const bool any_inflight = S->slice[0].inflight || S->slice[1].inflight;
        if (S->stop && !any_inflight) break;
        int rc = BD_OK;
        if (!S->stop) rc = admit(S);
        Slice& sl = S->slice[cur];
        if (rc == BD_OK && sl.inflight) {
            lk.unlock();
            const hipError_t e = hipEventSynchronize(sl.ev);
            lk.lock();
            if (e != hipSuccess) {
                rc = BD_E_HIP;
            } else {
                // device rate from the time between slice completions (slices overlap)
                const double tn = now_ms();
                const double dt = tn - std::max(sl.t_launch, S->t_last_done);
                S->t_last_done = tn;
                if (sl.steps > 0) {
                    const int w = S->win_next;
                    S->win_next = (w + 1) % bd_server::kRateWindow;
                    S->win_steps[w] = (double)sl.steps;
                    S->win_cost[w] = sl.sum_cost;
                    S->win_ms[w] = std::max(dt, 0.0);
                    double st = 0, sc = 0, sm = 0;
                    for (int i = 0; i < bd_server::kRateWindow; ++i) {
                        st += S->win_steps[i];
                        sc += S->win_cost[i];
                        sm += S->win_ms[i];
                    }
                    if (sm > 2.0) {
                        S->steps_per_ms = st / sm;
                        // resident work groups ran the summed chunk costs in that time
                        if (sc > 0) S->ms_per_lane_step = std::min(sm * (double)S->resident[0] / sc, 1e-2);
                    }
                }
                rc = process_completions(S, sl);
                ++S->slices_done;
            }
            sl.inflight = false;
        }
        if (rc == BD_OK && !S->cancelled.empty()) rc = reclaim_cancelled(S);
        if (rc == BD_OK && !S->stop) {
            rc = admit(S);
            if (rc == BD_OK) {
                fill_slice(S, sl);
                if (sl.n > 0) rc = launch_slice(S, sl);
            }
        }
        if (rc != BD_OK) {
            S->broken = rc;
            fail_all(S, rc);
            // drain whatever is still on the device before leaving
            lk.unlock();
            (void)hipStreamSynchronize(S->slice[0].st);
            (void)hipStreamSynchronize(S->slice[1].st);
            (void)hipStreamSynchronize(S->st);
            lk.lock();
            S->slice[0].inflight = S->slice[1].inflight = false;
            break;
        }
        cur ^= 1;
    }
    fail_all(S, BD_E_CANCELLED);
}

}  // namespace

extern "C" int bd_server_create(bd_graph* g, const bd_server_cfg* cfg, bd_server** out)
{
    if (!g || !out) return BD_E_INVALID;
    *out = nullptr;
    bd_server* S = new (std::nothrow) bd_server();
    if (!S) return BD_E_NOMEM;
    S->g = g;
    if (cfg) S->cfg = *cfg;
    S->pol = cfg ? cfg->policy : default_policy();
    if (S->pol.delta <= 0.0) S->pol.delta = 0.01;
    S->slots = (uint32_t)(S->cfg.max_queries_inflight > 0 ? std::min<int64_t>(S->cfg.max_queries_inflight, 1 << 22)
                                                         : 65536);
    S->gdim = (uint32_t)ceil_guarded(8.0 * std::log(1.0 / S->pol.delta));
    if (S->gdim > (uint32_t)kMaxG) {
        delete S;
        return BD_E_BUDGET;
    }
    S->resident[0] = resident_wgs(g, 0, share_class(policy_share(S->pol)));
    S->resident[1] = resident_wgs(g, 1, share_class(policy_share(S->pol)));
    int rc = S->d_qd.alloc((size_t)S->slots * sizeof(QueryDesc));
    if (rc == BD_OK) rc = S->d_bs.alloc((size_t)S->slots * S->gdim * 16);
    if (rc == BD_OK) rc = S->d_done.alloc((size_t)S->slots * 4);
    if (rc == BD_OK) rc = S->d_beta.alloc((size_t)S->slots * 8);
    S->arena = 1u << 22;
    if (rc == BD_OK) rc = S->d_psum.alloc((size_t)S->arena * 32);
    if (rc == BD_OK) rc = S->d_pcount.alloc((size_t)S->arena * 4);
    S->psum_alloc.init(S->arena);
    if (rc == BD_OK) rc = S->h_qd.alloc((size_t)S->slots * sizeof(QueryDesc));
    for (int i = 0; i < 2 && rc == BD_OK; ++i) {
        rc = S->slice[i].chunks_h.alloc((size_t)kSliceMaxChunks * sizeof(Chunk));
        if (rc == BD_OK) rc = S->slice[i].chunks_d.alloc((size_t)kSliceMaxChunks * sizeof(Chunk));
        if (rc == BD_OK) rc = S->slice[i].comp_h.alloc(comp_bytes(S));
        if (rc == BD_OK) rc = S->slice[i].d_comp.alloc(comp_bytes(S));
        if (rc == BD_OK) rc = S->slice[i].d_cursor.alloc(16);
        if (rc == BD_OK && hipEventCreateWithFlags(&S->slice[i].ev, hipEventDisableTiming) != hipSuccess)
            rc = BD_E_HIP;
        if (rc == BD_OK && hipStreamCreateWithFlags(&S->slice[i].st, hipStreamNonBlocking) != hipSuccess)
            rc = BD_E_HIP;
    }
    if (rc == BD_OK && hipStreamCreateWithFlags(&S->st, hipStreamNonBlocking) != hipSuccess) rc = BD_E_HIP;
    if (rc == BD_OK && hipEventCreateWithFlags(&S->ev_admit, hipEventDisableTiming) != hipSuccess) rc = BD_E_HIP;
    if (rc == BD_OK && launch_zero(S->d_bs.p, (size_t)S->slots * S->gdim * 16, S->st) != hipSuccess) rc = BD_E_HIP;
    if (rc == BD_OK && launch_zero(S->d_done.p, (size_t)S->slots * 4, S->st) != hipSuccess) rc = BD_E_HIP;
    if (rc == BD_OK && launch_zero(S->d_psum.p, (size_t)S->arena * 32, S->st) != hipSuccess) rc = BD_E_HIP;
    if (rc == BD_OK && launch_zero(S->d_pcount.p, (size_t)S->arena * 4, S->st) != hipSuccess) rc = BD_E_HIP;
    if (rc == BD_OK && hipStreamSynchronize(S->st) != hipSuccess) rc = BD_E_HIP;
    if (rc != BD_OK) {
        for (int i = 0; i < 2; ++i) {
            if (S->slice[i].ev) (void)hipEventDestroy(S->slice[i].ev);
            if (S->slice[i].st) (void)hipStreamDestroy(S->slice[i].st);
        }
        if (S->ev_admit) (void)hipEventDestroy(S->ev_admit);
        if (S->st) (void)hipStreamDestroy(S->st);
        delete S;
        return rc;
    }
    S->slot.resize(S->slots);
    S->free_slots.reserve(S->slots);
    for (uint32_t i = S->slots; i-- > 0;) S->free_slots.push_back(i);
    S->th = std::thread(server_loop, S);
    *out = S;
    return BD_OK;
}

extern "C" int bd_server_submit(bd_server* S, int64_t nq, const int32_t* s, const int32_t* t,
                                const double* eps, const int32_t* L, const uint32_t* uid, uint64_t seed,
                                uint64_t* request_id)
{
    if (!S || nq < 0 || !request_id || (nq > 0 && (!s || !t || !eps || !L))) return BD_E_INVALID;
    Request r;
    r.res.resize((size_t)nq);
    for (int64_t i = 0; i < nq; ++i) {
        plan_one(S->g, s[i], t[i], eps[i], L[i], S->pol, &r.res[(size_t)i]);
        if (uid && uid[i] >= 0x80000000u) r.res[(size_t)i].status = BD_E_INVALID;
        const bd_result& pr = r.res[(size_t)i];
        if (pr.status != BD_OK) continue;
        QueryDesc d{};
        d.s = (int32_t)storage_id(S->g, s[i]);
        d.t = (int32_t)storage_id(S->g, t[i]);
        d.L = L[i];
        d.uid = uid ? uid[i] : (uint32_t)i;
        d.K = (uint32_t)pr.K;
        d.R = (uint32_t)pr.R;
        d.B = (uint32_t)pr.B;
        d.G = (uint32_t)pr.G;
        d.seed_lo = (uint32_t)seed;
        d.seed_hi = (uint32_t)(seed >> 32);
        d.share = policy_share(S->pol);
        r.desc.push_back(d);
        r.index.push_back(i);
        r.steps += (uint64_t)pr.walk_steps;
        const bd_exec ex = server_exec(S);
        if (chunk_plan(ex, d, S->g->kernel_layout).part) r.split_probes += d.K;
    }
    r.remaining = (int64_t)r.desc.size();
    if (r.desc.size() > S->slots || r.split_probes > S->arena) return BD_E_FULL;
    if (S->cfg.max_steps_inflight && r.steps > S->cfg.max_steps_inflight) return BD_E_FULL;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->broken != BD_OK) return S->broken;
    const uint64_t id = S->next_id++;
    r.t_submit = now_ms();
    const bool empty = r.remaining == 0;
    auto& slot = S->reqs[id];
    slot = std::move(r);
    if (empty) finish_request(S, id, slot);
    else S->pending.push_back(id);
    *request_id = id;
    S->cv_work.notify_all();
    return BD_OK;
}

extern "C" int bd_server_poll(bd_server* S, uint64_t request_id, bd_result* out, int* done, double* latency_ms)
{
    if (!S || !done) return BD_E_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(request_id);
    if (it == S->reqs.end()) return BD_E_NOTFOUND;
    *done = it->second.done ? 1 : 0;
    if (!it->second.done) return BD_OK;
    if (out) std::memcpy(out, it->second.res.data(), it->second.res.size() * sizeof(bd_result));
    if (latency_ms) *latency_ms = it->second.t_done - it->second.t_submit;
    S->reqs.erase(it);
    return BD_OK;
}

extern "C" int bd_server_wait(bd_server* S, uint64_t request_id, double timeout_ms, bd_result* out,
                              double* latency_ms)
{
    if (!S) return BD_E_INVALID;
    std::unique_lock<std::mutex> lk(S->mu);
    auto ready = [&] {
        auto it = S->reqs.find(request_id);
        return it == S->reqs.end() || it->second.done;
    };
    if (timeout_ms > 0) {
        if (!S->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), ready))
            return BD_E_TIMEOUT;
    } else {
        S->cv_done.wait(lk, ready);
    }
    auto it = S->reqs.find(request_id);
    if (it == S->reqs.end()) return BD_E_NOTFOUND;
    if (out) std::memcpy(out, it->second.res.data(), it->second.res.size() * sizeof(bd_result));
    if (latency_ms) *latency_ms = it->second.t_done - it->second.t_submit;
    S->reqs.erase(it);
    return BD_OK;
}

extern "C" int bd_server_cancel(bd_server* S, uint64_t request_id)
{
    if (!S) return BD_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->reqs.find(request_id);
        if (it == S->reqs.end()) return BD_E_NOTFOUND;
        Request& r = it->second;
        if (r.done || r.cancelled) return BD_OK;
        r.cancelled = true;
        if (!r.admitted) {
            // still queued: nothing of it reached the device
            S->pending.erase(std::remove(S->pending.begin(), S->pending.end(), request_id), S->pending.end());
            for (size_t i = 0; i < r.index.size(); ++i) r.res[(size_t)r.index[i]].status = BD_E_CANCELLED;
            finish_request(S, request_id, r);
            return BD_OK;
        }
        // admitted: its chunks already on the device finish; the slots of the
        // queries they leave unfinished are reclaimed once those slices are done
        r.cancel_mark = S->slices_launched;
        S->cancelled.push_back(request_id);
    }
    S->cv_work.notify_all();
    return BD_OK;
}

extern "C" void bd_server_destroy(bd_server* S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->th.joinable()) S->th.join();
    for (int i = 0; i < 2; ++i) (void)hipStreamSynchronize(S->slice[i].st);
    (void)hipStreamSynchronize(S->st);
    for (int i = 0; i < 2; ++i) {
        if (S->slice[i].ev) (void)hipEventDestroy(S->slice[i].ev);
        (void)hipStreamDestroy(S->slice[i].st);
    }
    (void)hipEventDestroy(S->ev_admit);
    (void)hipStreamDestroy(S->st);
    delete S;
}
