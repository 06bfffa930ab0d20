// Chung-Lu power-law graph generator for the largest workload (seeded,
// multi-threaded, deterministic for any thread count).
//
// Same model as synth/graphs.py chung_lu: weights w_i proportional to
// (i+1)^(-1/(gamma-1)), scaled to the mean degree and capped at sqrt(sum w);
// round(n * mean / 2) edges with both endpoints drawn independently with
// probability proportional to w; self-loops and repeated edges dropped; node
// ids shuffled; the largest connected component kept. The random numbers come
// from a counter-based generator (the SplitMix64 output function of Steele,
// Lea and Flood applied to seed + index * 0x9E3779B97F4A7C15), so edge e is the
// same whatever thread draws it. The result is the canonical CSR: symmetric,
// rows ascending, no self-loops or repeats.
//
// This holds no part of the estimator; it only builds inputs.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// i-th value of the stream of `key`
inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * kGolden); }

inline double unit(uint64_t r) { return (double)(r >> 11) * 0x1p-53; }

template <class F>
void parallel_for(int64_t n, int threads, F&& f)
{
    if (threads <= 1 || n < 4096) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    const int64_t step = (n + threads - 1) / threads;
    for (int i = 0; i < threads; ++i) {
        const int64_t a = i * step, b = std::min<int64_t>(n, a + step);
        if (a >= b) break;
        th.emplace_back([&f, a, b] { f(a, b); });
    }
    for (auto& t : th) t.join();
}

// Rows processed in dynamically claimed blocks (rows differ widely in length).
template <class F>
void parallel_rows(int64_t n, int threads, F&& f)
{
    std::atomic<int64_t> next{0};
    const int64_t blk = 4096;
    auto work = [&] {
        for (;;) {
            const int64_t a = next.fetch_add(blk);
            if (a >= n) break;
            f(a, std::min<int64_t>(n, a + blk));
        }
    };
    if (threads <= 1) {
        work();
        return;
    }
    std::vector<std::thread> th;
    for (int i = 0; i < threads; ++i) th.emplace_back(work);
    for (auto& t : th) t.join();
}

struct Csr {
    int64_t n = 0;
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col;
};

struct Sampler {
    std::vector<double> cdf;        // cumulative weights, cdf[n-1] = 1
    std::vector<uint32_t> first;    // first[j] = #{i : cdf[i] <= j / nb}
    uint64_t nb = 0;
    // the index i with cdf[i-1] <= r < cdf[i] (entries <= r counted), clamped to n-1
    uint32_t operator()(double r) const
    {
        int64_t j = (int64_t)(r * (double)nb) - 1;
        if (j < 0) j = 0;
        uint64_t idx = first[(size_t)j];
        const uint64_t n = cdf.size();
        while (idx < n && cdf[idx] <= r) ++idx;
        return (uint32_t)std::min<uint64_t>(idx, n - 1);
    }
};

}  // namespace

extern "C" {

void* clg_generate(int64_t n, double mean_deg, double gamma, uint64_t seed, int threads, int lcc)
{
    if (n < 2 || n > 0x7FFFFFFF || !(mean_deg > 0) || !(gamma > 1)) return nullptr;
    if (threads < 1) threads = 1;
    Csr* out = new Csr();

    // weights and their cumulative distribution
    Sampler smp;
    std::vector<double> w((size_t)n);
    double sum = 0;
    for (int64_t i = 0; i < n; ++i) {
        w[(size_t)i] = std::pow((double)(i + 1), -1.0 / (gamma - 1.0));
        sum += w[(size_t)i];
    }
    const double scale = mean_deg * (double)n / sum;
    double tot = 0;
    for (auto& x : w) {
        x *= scale;
        tot += x;
    }
    const double cap = std::sqrt(tot);
    smp.cdf.resize((size_t)n);
    double acc = 0;
    for (int64_t i = 0; i < n; ++i) {
        acc += std::min(w[(size_t)i], cap);
        smp.cdf[(size_t)i] = acc;
    }
    for (auto& x : smp.cdf) x /= acc;
    smp.cdf[(size_t)n - 1] = 1.0;
    std::vector<double>().swap(w);
    smp.nb = 4 * (uint64_t)n;
    smp.first.resize(smp.nb);
    {
        uint64_t i = 0;
        for (uint64_t j = 0; j < smp.nb; ++j) {
            const double b = (double)j / (double)smp.nb;
            while (i < (uint64_t)n && smp.cdf[i] <= b) ++i;
            smp.first[j] = (uint32_t)i;
        }
    }

    // shuffled ids (Fisher-Yates on the stream seed ^ 1)
    std::vector<uint32_t> perm((size_t)n);
    for (int64_t i = 0; i < n; ++i) perm[(size_t)i] = (uint32_t)i;
    const uint64_t kperm = mix64(seed ^ 0x5045524Dull);
    for (int64_t i = n - 1; i > 0; --i) {
        const uint64_t r = draw(kperm, (uint64_t)i);
        const int64_t j = (int64_t)(((unsigned __int128)r * (unsigned __int128)(i + 1)) >> 64);
        std::swap(perm[(size_t)i], perm[(size_t)j]);
    }

    const int64_t m = (int64_t)std::llround((double)n * mean_deg / 2.0);
    const uint64_t kedge = mix64(seed ^ 0x45444745ull);
    auto endpoints = [&](int64_t e, uint32_t* a, uint32_t* b) {
        *a = perm[smp(unit(draw(kedge, 2 * (uint64_t)e)))];
        *b = perm[smp(unit(draw(kedge, 2 * (uint64_t)e + 1)))];
    };

    // pass 1: degrees with repeats; pass 2: fill
    std::vector<uint32_t> deg((size_t)n, 0);
    parallel_for(m, threads, [&](int64_t e0, int64_t e1) {
        for (int64_t e = e0; e < e1; ++e) {
            uint32_t a, b;
            endpoints(e, &a, &b);
            if (a == b) continue;
            __atomic_fetch_add(&deg[a], 1u, __ATOMIC_RELAXED);
            __atomic_fetch_add(&deg[b], 1u, __ATOMIC_RELAXED);
        }
    });
    std::vector<int64_t> rp((size_t)n + 1, 0);
    for (int64_t v = 0; v < n; ++v) rp[(size_t)v + 1] = rp[(size_t)v] + deg[(size_t)v];
    std::vector<uint32_t>().swap(deg);
    std::vector<int32_t> col((size_t)rp[(size_t)n]);
    std::vector<int64_t> cur(rp.begin(), rp.end() - 1);
    parallel_for(m, threads, [&](int64_t e0, int64_t e1) {
        for (int64_t e = e0; e < e1; ++e) {
            uint32_t a, b;
            endpoints(e, &a, &b);
            if (a == b) continue;
            col[(size_t)__atomic_fetch_add(&cur[a], 1, __ATOMIC_RELAXED)] = (int32_t)b;
            col[(size_t)__atomic_fetch_add(&cur[b], 1, __ATOMIC_RELAXED)] = (int32_t)a;
        }
    });
    std::vector<int64_t>().swap(cur);
    std::vector<uint32_t>().swap(perm);

    // sort rows, drop repeats, pack
    std::vector<int64_t> len((size_t)n);
    parallel_rows(n, threads, [&](int64_t v0, int64_t v1) {
        for (int64_t v = v0; v < v1; ++v) {
            int32_t* a = col.data() + rp[(size_t)v];
            int32_t* b = col.data() + rp[(size_t)v + 1];
            std::sort(a, b);
            len[(size_t)v] = std::unique(a, b) - a;
        }
    });
    int64_t pos = 0;
    for (int64_t v = 0; v < n; ++v) {
        const int64_t src = rp[(size_t)v];
        rp[(size_t)v] = pos;
        if (pos != src) std::memmove(col.data() + pos, col.data() + src, (size_t)len[(size_t)v] * 4);
        pos += len[(size_t)v];
    }
    rp[(size_t)n] = pos;
    std::vector<int64_t>().swap(len);

    // largest component: components by breadth-first search, keep the largest
    std::vector<int32_t> comp((size_t)n, -1);
    std::vector<int32_t> queue((size_t)n);
    int32_t ncomp = 0, best = -1;
    int64_t best_size = 0;
    for (int64_t s0 = 0; s0 < n && lcc; ++s0) {
        if (comp[(size_t)s0] >= 0) continue;
        int64_t qh = 0, qt = 0;
        queue[(size_t)qt++] = (int32_t)s0;
        comp[(size_t)s0] = ncomp;
        while (qh < qt) {
            const int32_t v = queue[(size_t)qh++];
            for (int64_t i = rp[(size_t)v]; i < rp[(size_t)v + 1]; ++i) {
                const int32_t u = col[(size_t)i];
                if (comp[(size_t)u] < 0) {
                    comp[(size_t)u] = ncomp;
                    queue[(size_t)qt++] = u;
                }
            }
        }
        if (qt > best_size) {
            best_size = qt;
            best = ncomp;
        }
        ++ncomp;
    }
    std::vector<int32_t>().swap(queue);
    if (lcc && best_size < n) {
        // increasing renaming of the kept nodes: rows stay in order and sorted
        std::vector<int32_t> nid((size_t)n, -1);
        int32_t k = 0;
        for (int64_t v = 0; v < n; ++v)
            if (comp[(size_t)v] == best) nid[(size_t)v] = k++;
        int64_t p = 0;
        int64_t r = 0;
        for (int64_t v = 0; v < n; ++v) {
            const int64_t a = rp[(size_t)v], b = rp[(size_t)v + 1];
            if (comp[(size_t)v] != best) continue;
            rp[(size_t)r++] = p;  // r <= v: the entry for v is read above before any later write
            for (int64_t i = a; i < b; ++i) col[(size_t)p++] = nid[(size_t)col[(size_t)i]];
        }
        rp[(size_t)r] = p;
        rp.resize((size_t)r + 1);
        col.resize((size_t)p);
        out->n = r;
    } else {
        out->n = n;
    }
    out->row_ptr.swap(rp);
    out->col.swap(col);
    out->col.shrink_to_fit();
    return out;
}

int64_t clg_n(void* h) { return static_cast<Csr*>(h)->n; }

int64_t clg_nnz(void* h) { return (int64_t)static_cast<Csr*>(h)->col.size(); }

void clg_copy(void* h, int64_t* row_ptr, int32_t* col)
{
    const Csr* c = static_cast<Csr*>(h);
    std::memcpy(row_ptr, c->row_ptr.data(), c->row_ptr.size() * sizeof(int64_t));
    std::memcpy(col, c->col.data(), c->col.size() * sizeof(int32_t));
}

void clg_free(void* h) { delete static_cast<Csr*>(h); }

}  // extern "C"
