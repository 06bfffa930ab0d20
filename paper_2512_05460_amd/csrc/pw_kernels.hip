// HIP kernels of the ProbeWalk hot path (gfx950).
//
// One work group runs one chunk: probes [k0, k0+kc) of one query with all R
// replicas each (Algorithm 1: the probe loop, the replica loop and the walk
// loop). Its lanes (256, or 1,024 on the hubs-first layouts with one probe
// per walk) stride over the kc*R (probe, replica) pairs; each lane
// runs the s-walk and the t-walk of its pair interleaved, so two independent
// dependent-gather chains are in flight per lane. Per-probe sums S1, S2 are
// exact 128-bit integers accumulated in LDS; at the end of the chunk each
// probe's Q_R (U-statistic, Lemma 3.4) is added as trunc(Q 2^64) to its
// median-of-means block in global memory. The work group that completes a
// query's last probe forms the G block means and their median.
//
// The same chunk routine serves one-query-per-launch (grid = chunks) and
// persistent launches (grid = resident capacity, chunks claimed from per-XCD
// atomic cursors until none are left, so every wave exits).
#include <algorithm>

#include "pw_device.hpp"
#include "pw_internal.hpp"

namespace pw {

__device__ __forceinline__ DevGraph make_graph(const GraphTables& g)
{
    DevGraph G;
    G.node = g.node;
    G.col = g.col;
    G.adj = g.adj;
    G.rp = g.rp;
    G.col24 = g.col24;
    G.node8 = g.node8;
    G.hub = nullptr;
    G.hub4 = nullptr;
    G.inv = nullptr;
    G.rec_word = 0;
    G.runtab = g.runtab;
    G.run_h1 = g.run_h1;
    G.run_words = g.run_words;
    G.run_ninv = g.run_ninv;
    G.run_shift = g.run_shift;
    G.nhub = 0;
    G.dom.n = g.dom.n;
    G.dom.rb = g.dom.rb;
    G.dom.mask = g.dom.mask;
    G.dom.rsh = g.dom.rsh;
    G.dom.A = g.dom.A;
    G.dom.A8 = g.dom.A8;
    return G;
}

// One transition followed by scoring the node just left: the gathers for the
// next node are issued before the probe arithmetic of the current node, so
// the ALU work overlaps the memory latency. Terms still enter the binary32
// sum in step order X_0, X_1, ..., X_L.
template <int kLayout>
__device__ __forceinline__ float advance(WalkState& w, float acc, uint32_t u, const DevGraph& G,
                                         const Probe& pr)
{
    const uint32_t xp = w.x;
    const float ip = w.inv;
    step<kLayout>(w, u, G);
    return add_term(acc, xp, ip, pr, G.dom);
}

// U_p = a - b for replica p of probe k (Algorithm 1 walk loop, eq. for phi-hat).
template <int kLayout>
__device__ __forceinline__ float walk_pair(const DevGraph& G, const Probe& pr, WalkState ws,
                                           WalkState wt, int L, uint32_t p, uint32_t k,
                                           uint32_t uid, uint32_t slo, uint32_t shi)
{
    float a = 0.0f, b = 0.0f;
    const uint32_t cs = uid << 1, ct = (uid << 1) | 1u;
    const int full = L >> 2;
    for (int blk = 0; blk < full; ++blk) {
        const U4 rs = philox10((uint32_t)blk, p, k, cs, slo, shi);
        const U4 rt = philox10((uint32_t)blk, p, k, ct, slo, shi);
        a = advance<kLayout>(ws, a, rs.x, G, pr);
        b = advance<kLayout>(wt, b, rt.x, G, pr);
        a = advance<kLayout>(ws, a, rs.y, G, pr);
        b = advance<kLayout>(wt, b, rt.y, G, pr);
        a = advance<kLayout>(ws, a, rs.z, G, pr);
        b = advance<kLayout>(wt, b, rt.z, G, pr);
        a = advance<kLayout>(ws, a, rs.w, G, pr);
        b = advance<kLayout>(wt, b, rt.w, G, pr);
    }
    const int rem = L & 3;
    if (rem) {
        const U4 rs = philox10((uint32_t)full, p, k, cs, slo, shi);
        const U4 rt = philox10((uint32_t)full, p, k, ct, slo, shi);
        a = advance<kLayout>(ws, a, rs.x, G, pr);
        b = advance<kLayout>(wt, b, rt.x, G, pr);
        if (rem > 1) {
            a = advance<kLayout>(ws, a, rs.y, G, pr);
            b = advance<kLayout>(wt, b, rt.y, G, pr);
        }
        if (rem > 2) {
            a = advance<kLayout>(ws, a, rs.z, G, pr);
            b = advance<kLayout>(wt, b, rt.z, G, pr);
        }
    }
    a = add_term(a, ws.x, ws.inv, pr, G.dom);
    b = add_term(b, wt.x, wt.inv, pr, G.dom);
    return __fsub_rn(a, b);
}

// Two replica pairs per lane (layout code 7): U_p1 of probe k1 and U_p2 of
// probe k2, the four walks interleaved step by step so that four dependent
// loads are in flight per lane. Each walk is the one walk_pair runs.
template <int kLayout>
__device__ __forceinline__ void walk_pair2(const DevGraph& G, const Probe& pr1, const Probe& pr2, WalkState s0,
                                           WalkState t0, int L, uint32_t p1, uint32_t k1, uint32_t p2, uint32_t k2,
                                           uint32_t uid, uint32_t slo, uint32_t shi, float* U1, float* U2)
{
    WalkState s1 = s0, t1 = t0, s2 = s0, t2 = t0;
    float a1 = 0.0f, b1 = 0.0f, a2 = 0.0f, b2 = 0.0f;
    const uint32_t cs = uid << 1, ct = (uid << 1) | 1u;
    const int full = L >> 2;
    for (int blk = 0; blk < full; ++blk) {
        const U4 rs1 = philox10((uint32_t)blk, p1, k1, cs, slo, shi);
        const U4 rt1 = philox10((uint32_t)blk, p1, k1, ct, slo, shi);
        const U4 rs2 = philox10((uint32_t)blk, p2, k2, cs, slo, shi);
        const U4 rt2 = philox10((uint32_t)blk, p2, k2, ct, slo, shi);
        a1 = advance<kLayout>(s1, a1, rs1.x, G, pr1);
        b1 = advance<kLayout>(t1, b1, rt1.x, G, pr1);
        a2 = advance<kLayout>(s2, a2, rs2.x, G, pr2);
        b2 = advance<kLayout>(t2, b2, rt2.x, G, pr2);
        a1 = advance<kLayout>(s1, a1, rs1.y, G, pr1);
        b1 = advance<kLayout>(t1, b1, rt1.y, G, pr1);
        a2 = advance<kLayout>(s2, a2, rs2.y, G, pr2);
        b2 = advance<kLayout>(t2, b2, rt2.y, G, pr2);
        a1 = advance<kLayout>(s1, a1, rs1.z, G, pr1);
        b1 = advance<kLayout>(t1, b1, rt1.z, G, pr1);
        a2 = advance<kLayout>(s2, a2, rs2.z, G, pr2);
        b2 = advance<kLayout>(t2, b2, rt2.z, G, pr2);
        a1 = advance<kLayout>(s1, a1, rs1.w, G, pr1);
        b1 = advance<kLayout>(t1, b1, rt1.w, G, pr1);
        a2 = advance<kLayout>(s2, a2, rs2.w, G, pr2);
        b2 = advance<kLayout>(t2, b2, rt2.w, G, pr2);
    }
    const int rem = L & 3;
    if (rem) {
        const U4 rs1 = philox10((uint32_t)full, p1, k1, cs, slo, shi);
        const U4 rt1 = philox10((uint32_t)full, p1, k1, ct, slo, shi);
        const U4 rs2 = philox10((uint32_t)full, p2, k2, cs, slo, shi);
        const U4 rt2 = philox10((uint32_t)full, p2, k2, ct, slo, shi);
        a1 = advance<kLayout>(s1, a1, rs1.x, G, pr1);
        b1 = advance<kLayout>(t1, b1, rt1.x, G, pr1);
        a2 = advance<kLayout>(s2, a2, rs2.x, G, pr2);
        b2 = advance<kLayout>(t2, b2, rt2.x, G, pr2);
        if (rem > 1) {
            a1 = advance<kLayout>(s1, a1, rs1.y, G, pr1);
            b1 = advance<kLayout>(t1, b1, rt1.y, G, pr1);
            a2 = advance<kLayout>(s2, a2, rs2.y, G, pr2);
            b2 = advance<kLayout>(t2, b2, rt2.y, G, pr2);
        }
        if (rem > 2) {
            a1 = advance<kLayout>(s1, a1, rs1.z, G, pr1);
            b1 = advance<kLayout>(t1, b1, rt1.z, G, pr1);
            a2 = advance<kLayout>(s2, a2, rs2.z, G, pr2);
            b2 = advance<kLayout>(t2, b2, rt2.z, G, pr2);
        }
    }
    a1 = add_term(a1, s1.x, s1.inv, pr1, G.dom);
    b1 = add_term(b1, t1.x, t1.inv, pr1, G.dom);
    a2 = add_term(a2, s2.x, s2.inv, pr2, G.dom);
    b2 = add_term(b2, t2.x, t2.inv, pr2, G.dom);
    *U1 = __fsub_rn(a1, b1);
    *U2 = __fsub_rn(a2, b2);
}

// Walk sharing: one walk scored against the m <= kShare probes of a group.
// The terms of each probe enter its own binary32 sum in step order, exactly as
// in advance/walk_pair.
template <int kLayout, int kShare>
__device__ __forceinline__ void advance_m(WalkState& w, float* acc, uint32_t m, uint32_t u, const DevGraph& G,
                                          const Probe* pr)
{
    const uint32_t xp = w.x;
    const float ip = w.inv;
    step<kLayout>(w, u, G);
#pragma unroll
    for (int j = 0; j < kShare; ++j)
        if ((uint32_t)j < m) acc[j] = add_term(acc[j], xp, ip, pr[j], G.dom);
}

// U_p for each probe of a group; the walks' streams are keyed by kw, the
// group's first probe.
template <int kLayout, int kShare>
__device__ __forceinline__ void walk_pair_m(const DevGraph& G, const Probe* pr, uint32_t m, WalkState ws,
                                            WalkState wt, int L, uint32_t p, uint32_t kw, uint32_t uid,
                                            uint32_t slo, uint32_t shi, float* U)
{
    float a[kShare], b[kShare];
#pragma unroll
    for (int j = 0; j < kShare; ++j) a[j] = b[j] = 0.0f;
    const uint32_t cs = uid << 1, ct = (uid << 1) | 1u;
    const int full = L >> 2;
    for (int blk = 0; blk < full; ++blk) {
        const U4 rs = philox10((uint32_t)blk, p, kw, cs, slo, shi);
        const U4 rt = philox10((uint32_t)blk, p, kw, ct, slo, shi);
        advance_m<kLayout, kShare>(ws, a, m, rs.x, G, pr);
        advance_m<kLayout, kShare>(wt, b, m, rt.x, G, pr);
        advance_m<kLayout, kShare>(ws, a, m, rs.y, G, pr);
        advance_m<kLayout, kShare>(wt, b, m, rt.y, G, pr);
        advance_m<kLayout, kShare>(ws, a, m, rs.z, G, pr);
        advance_m<kLayout, kShare>(wt, b, m, rt.z, G, pr);
        advance_m<kLayout, kShare>(ws, a, m, rs.w, G, pr);
        advance_m<kLayout, kShare>(wt, b, m, rt.w, G, pr);
    }
    const int rem = L & 3;
    if (rem) {
        const U4 rs = philox10((uint32_t)full, p, kw, cs, slo, shi);
        const U4 rt = philox10((uint32_t)full, p, kw, ct, slo, shi);
        advance_m<kLayout, kShare>(ws, a, m, rs.x, G, pr);
        advance_m<kLayout, kShare>(wt, b, m, rt.x, G, pr);
        if (rem > 1) {
            advance_m<kLayout, kShare>(ws, a, m, rs.y, G, pr);
            advance_m<kLayout, kShare>(wt, b, m, rt.y, G, pr);
        }
        if (rem > 2) {
            advance_m<kLayout, kShare>(ws, a, m, rs.z, G, pr);
            advance_m<kLayout, kShare>(wt, b, m, rt.z, G, pr);
        }
    }
#pragma unroll
    for (int j = 0; j < kShare; ++j) {
        if ((uint32_t)j < m) {
            a[j] = add_term(a[j], ws.x, ws.inv, pr[j], G.dom);
            b[j] = add_term(b[j], wt.x, wt.inv, pr[j], G.dom);
        }
        U[j] = __fsub_rn(a[j], b[j]);
    }
}

// Probes [*kf, *kf + *sz) of walk-sharing group gi: groups of M probes inside
// each block of B (the last group of a block may be smaller).
__device__ __forceinline__ void group_probes(uint32_t gi, uint32_t B, uint32_t M, uint32_t gpb, uint32_t* kf,
                                             uint32_t* sz)
{
    const uint32_t blk = gi / gpb;
    const uint32_t j = gi - blk * gpb;
    *kf = blk * B + j * M;
    *sz = min(M, B - j * M);
}

__device__ __forceinline__ void lds_add_i128(unsigned long long* p, i128 v)
{
    const unsigned long long lo = (unsigned long long)(u128)v;
    const unsigned long long hi = (unsigned long long)((u128)v >> 64);
    const unsigned long long old = atomicAdd(p, lo);
    const unsigned long long carry = (old + lo < old) ? 1ull : 0ull;
    atomicAdd(p + 1, hi + carry);
}

// Median of the G block means (section 3.2, Algorithm 1 final loop).
__device__ void finalize_query(const WalkArgs& A, const QueryDesc& d, double* ys)
{
    const uint32_t G = d.G;
    const unsigned long long* bs = A.blocksum + (size_t)d.slot * A.gdim * 2;
    for (uint32_t g = 0; g < G; ++g) {
        const double y = (i128_to_f64(load_i128(bs + 2 * g)) * 0x1p-64) / (double)d.B;
        ys[g] = y;
        if (A.ybar_debug) A.ybar_debug[g] = y;
    }
    for (uint32_t i = 1; i < G; ++i) {
        const double v = ys[i];
        uint32_t j = i;
        while (j > 0 && ys[j - 1] > v) {
            ys[j] = ys[j - 1];
            --j;
        }
        ys[j] = v;
    }
    const double med = (G & 1u) ? ys[G / 2] : 0.5 * (ys[G / 2 - 1] + ys[G / 2]);
    A.beta[d.slot] = med;
    if (A.recycle) {
        // every chunk of this query has finished: the slot can be cleared for reuse
        unsigned long long* w = A.blocksum + (size_t)d.slot * A.gdim * 2;
        for (uint32_t g = 0; g < 2 * A.gdim; ++g) w[g] = 0ull;
        A.done[d.slot] = 0u;
    }
    if (A.comp_ring) {
        const uint32_t i = atomicAdd(A.comp_count, 1u);
        Completion c;
        c.slot = d.slot;
        c.pad = 0u;
        c.beta = med;
        A.comp_ring[i % A.comp_cap] = c;
    }
    __threadfence();
}

template <int kLayout, int kUniform, int kShare>
__device__ void run_chunk(const WalkArgs& A, const DevGraph& G, uint32_t ci,
                          unsigned long long* acc, double* ys)
{
    const Chunk c = A.chunks[ci];
    const QueryDesc d = A.qd[c.q];
    constexpr int kT = block_threads(kLayout, kShare);
    const int tid = threadIdx.x;
    for (uint32_t j = tid; j < c.kc * 4u; j += kT) acc[j] = 0ull;
    __syncthreads();

    const WalkState s0 = start_at<kLayout>(G, (uint32_t)d.s);
    const WalkState t0 = start_at<kLayout>(G, (uint32_t)d.t);
    // walk sharing: M probes per group, ceil(B/M) groups per block
    const uint32_t M = kShare == 1 ? 1u : d.share;
    const uint32_t gpb = (d.B + M - 1) / M;
    constexpr bool kDual = lane_pairs(kLayout) == 2 && kShare == 1;
    if (kDual && kUniform) {
        // Two blocks of 64 replicas per wave pass: units u and u + nw, each of
        // one probe (wave-uniform keys). A lane whose replica lies past the
        // chunk walks a clamped in-range replica and drops the result, so the
        // wave never splits into the single- and two-pair paths.
        const uint32_t wave = __builtin_amdgcn_readfirstlane((uint32_t)tid >> 6);
        const uint32_t lane = (uint32_t)tid & 63u;
        const uint32_t nb = (c.pc + 63u) >> 6;
        const uint32_t units = c.gc * nb;
        const uint32_t pend = c.p0 + c.pc;
        constexpr uint32_t nw = (uint32_t)kT / 64u;
        for (uint32_t u = wave; u < units; u += 2u * nw) {
            const uint32_t gg1 = u / nb;
            const uint32_t q1 = c.p0 + (u - gg1 * nb) * 64u + lane;
            const uint32_t k1 = c.k0 + gg1;
            const Probe pr1 = make_probe(d.seed_lo, d.seed_hi, d.uid, k1, G.dom.n);
            const uint32_t u2 = u + nw;
            if (u2 < units) {
                const uint32_t gg2 = u2 / nb;
                const uint32_t q2 = c.p0 + (u2 - gg2 * nb) * 64u + lane;
                const uint32_t k2 = c.k0 + gg2;
                const Probe pr2 = make_probe(d.seed_lo, d.seed_hi, d.uid, k2, G.dom.n);
                float U1, U2;
                walk_pair2<kLayout>(G, pr1, pr2, s0, t0, d.L, min(q1, pend - 1u), k1, min(q2, pend - 1u), k2, d.uid,
                                    d.seed_lo, d.seed_hi, &U1, &U2);
                if (q1 < pend) {
                    lds_add_i128(acc + 4 * gg1, fix54(U1));
                    lds_add_i128(acc + 4 * gg1 + 2, (i128)sqfix64(U1));
                }
                if (q2 < pend) {
                    lds_add_i128(acc + 4 * gg2, fix54(U2));
                    lds_add_i128(acc + 4 * gg2 + 2, (i128)sqfix64(U2));
                }
            } else if (q1 < pend) {
                const float U = walk_pair<kLayout>(G, pr1, s0, t0, d.L, q1, k1, d.uid, d.seed_lo, d.seed_hi);
                lds_add_i128(acc + 4 * gg1, fix54(U));
                lds_add_i128(acc + 4 * gg1 + 2, (i128)sqfix64(U));
            }
        }
    } else if (kDual) {
        // Lanes over the chunk's (probe, replica) pairs, two per lane per pass
        // (items base + tid and base + kT + tid); as above, an item past the
        // end is replaced by the last one and its result dropped.
        const uint64_t total = (uint64_t)c.gc * c.pc;
        for (uint64_t base = 0; base < total; base += 2u * (uint64_t)kT) {
            const uint64_t w1 = base + (uint64_t)tid, w2 = w1 + (uint64_t)kT;
            if (base + (uint64_t)kT < total) {
                const uint64_t x1 = min(w1, total - 1u), x2 = min(w2, total - 1u);
                const uint32_t gg1 = (uint32_t)(x1 / c.pc), gg2 = (uint32_t)(x2 / c.pc);
                const uint32_t p1 = c.p0 + (uint32_t)(x1 - (uint64_t)gg1 * c.pc);
                const uint32_t p2 = c.p0 + (uint32_t)(x2 - (uint64_t)gg2 * c.pc);
                const uint32_t k1 = c.k0 + gg1, k2 = c.k0 + gg2;
                const Probe pr1 = make_probe(d.seed_lo, d.seed_hi, d.uid, k1, G.dom.n);
                const Probe pr2 = make_probe(d.seed_lo, d.seed_hi, d.uid, k2, G.dom.n);
                float U1, U2;
                walk_pair2<kLayout>(G, pr1, pr2, s0, t0, d.L, p1, k1, p2, k2, d.uid, d.seed_lo, d.seed_hi, &U1, &U2);
                if (w1 < total) {
                    lds_add_i128(acc + 4 * gg1, fix54(U1));
                    lds_add_i128(acc + 4 * gg1 + 2, (i128)sqfix64(U1));
                }
                if (w2 < total) {
                    lds_add_i128(acc + 4 * gg2, fix54(U2));
                    lds_add_i128(acc + 4 * gg2 + 2, (i128)sqfix64(U2));
                }
            } else if (w1 < total) {
                const uint32_t gg = (uint32_t)(w1 / c.pc);
                const uint32_t p = c.p0 + (uint32_t)(w1 - (uint64_t)gg * c.pc);
                const uint32_t k = c.k0 + gg;
                const Probe pr = make_probe(d.seed_lo, d.seed_hi, d.uid, k, G.dom.n);
                const float U = walk_pair<kLayout>(G, pr, s0, t0, d.L, p, k, d.uid, d.seed_lo, d.seed_hi);
                lds_add_i128(acc + 4 * gg, fix54(U));
                lds_add_i128(acc + 4 * gg + 2, (i128)sqfix64(U));
            }
        }
    } else if (kUniform) {
        // Each wave takes blocks of 64 consecutive replicas of one group, so the
        // group and every probe key are uniform across the wave (scalar
        // registers); only the last block of a group runs partially masked.
        const uint32_t wave = __builtin_amdgcn_readfirstlane((uint32_t)tid >> 6);
        const uint32_t lane = (uint32_t)tid & 63u;
        const uint32_t nb = (c.pc + 63u) >> 6;
        const uint32_t units = c.gc * nb;
        const uint32_t pend = c.p0 + c.pc;
        for (uint32_t u = wave; u < units; u += kT / 64) {
            const uint32_t gg = u / nb;
            const uint32_t p = c.p0 + (u - gg * nb) * 64u + lane;
            if (p < pend) {
                if constexpr (kShare == 1) {
                    const uint32_t k = c.k0 + gg;
                    const Probe pr = make_probe(d.seed_lo, d.seed_hi, d.uid, k, G.dom.n);
                    const float U = walk_pair<kLayout>(G, pr, s0, t0, d.L, p, k, d.uid, d.seed_lo, d.seed_hi);
                    lds_add_i128(acc + 4 * gg, fix54(U));
                    lds_add_i128(acc + 4 * gg + 2, (i128)sqfix64(U));
                } else {
                    uint32_t kf, sz;
                    group_probes(c.g0 + gg, d.B, M, gpb, &kf, &sz);
                    Probe pr[kShare];
#pragma unroll
                    for (int j = 0; j < kShare; ++j)
                        if ((uint32_t)j < sz) pr[j] = make_probe(d.seed_lo, d.seed_hi, d.uid, kf + j, G.dom.n);
                    float U[kShare];
                    walk_pair_m<kLayout, kShare>(G, pr, sz, s0, t0, d.L, p, kf, d.uid, d.seed_lo, d.seed_hi, U);
#pragma unroll
                    for (int j = 0; j < kShare; ++j) {
                        if ((uint32_t)j < sz) {
                            unsigned long long* a4 = acc + 4 * (kf + j - c.k0);
                            lds_add_i128(a4, fix54(U[j]));
                            lds_add_i128(a4 + 2, (i128)sqfix64(U[j]));
                        }
                    }
                }
            }
        }
    } else {
        // Any replica count: lanes stride over the chunk's (group, replica)
        // pairs, so one wave can cover several groups.
        const uint64_t total = (uint64_t)c.gc * c.pc;
        for (uint64_t base = 0; base < total; base += kT) {
            const uint64_t w = base + (uint64_t)tid;
            if (w < total) {
                const uint32_t gg = (uint32_t)(w / c.pc);
                const uint32_t p = c.p0 + (uint32_t)(w - (uint64_t)gg * c.pc);
                if constexpr (kShare == 1) {
                    const uint32_t k = c.k0 + gg;
                    const Probe pr = make_probe(d.seed_lo, d.seed_hi, d.uid, k, G.dom.n);
                    const float U = walk_pair<kLayout>(G, pr, s0, t0, d.L, p, k, d.uid, d.seed_lo, d.seed_hi);
                    lds_add_i128(acc + 4 * gg, fix54(U));
                    lds_add_i128(acc + 4 * gg + 2, (i128)sqfix64(U));
                } else {
                    uint32_t kf, sz;
                    group_probes(c.g0 + gg, d.B, M, gpb, &kf, &sz);
                    Probe pr[kShare];
#pragma unroll
                    for (int j = 0; j < kShare; ++j)
                        if ((uint32_t)j < sz) pr[j] = make_probe(d.seed_lo, d.seed_hi, d.uid, kf + j, G.dom.n);
                    float U[kShare];
                    walk_pair_m<kLayout, kShare>(G, pr, sz, s0, t0, d.L, p, kf, d.uid, d.seed_lo, d.seed_hi, U);
#pragma unroll
                    for (int j = 0; j < kShare; ++j) {
                        if ((uint32_t)j < sz) {
                            unsigned long long* a4 = acc + 4 * (kf + j - c.k0);
                            lds_add_i128(a4, fix54(U[j]));
                            lds_add_i128(a4 + 2, (i128)sqfix64(U[j]));
                        }
                    }
                }
            }
        }
    }
    __syncthreads();

    if (c.pc < d.R) {
        // Part of a split group: add each probe's partial sums to its
        // accumulator; the chunk that brings a probe's replica count to R forms
        // its Q_R.
        if (tid == 0) {
            for (uint32_t j = 0; j < c.kc; ++j) {
                const uint32_t k = c.k0 + j;
                const size_t pi = (size_t)d.psum_base + k;
                unsigned long long* ps = A.psum + pi * 4;
                atomic_add_i128(ps, (i128)(((u128)acc[4 * j + 1] << 64) | (u128)acc[4 * j]));
                atomic_add_i128(ps + 2, (i128)(((u128)acc[4 * j + 3] << 64) | (u128)acc[4 * j + 2]));
                __threadfence();
                const uint32_t prev = atomicAdd(A.pcount + pi, c.pc);
                if (prev + c.pc == d.R) {
                    __threadfence();
                    const i128 S1 = load_i128(ps);
                    const u128 S2 = (u128)load_i128(ps + 2);
                    const double Q = probe_q(S1, S2, d.R);
                    if (A.q_debug) A.q_debug[k] = Q;
                    atomic_add_i128(A.blocksum + ((size_t)d.slot * A.gdim + k / d.B) * 2,
                                    f64_to_i128_trunc(Q * 0x1p64));
                    // every part of this probe has been added: clear it for reuse
                    ps[0] = ps[1] = ps[2] = ps[3] = 0ull;
                    A.pcount[pi] = 0u;
                    __threadfence();
                    const uint32_t old = atomicAdd(A.done + d.slot, 1u);
                    if (old + 1u == d.K) {
                        __threadfence();
                        finalize_query(A, d, ys);
                    }
                }
            }
        }
        __syncthreads();
        return;
    }

    for (uint32_t j = tid; j < c.kc; j += kT) {
        const i128 S1 = (i128)(((u128)acc[4 * j + 1] << 64) | (u128)acc[4 * j]);
        const u128 S2 = ((u128)acc[4 * j + 3] << 64) | (u128)acc[4 * j + 2];
        const double Q = probe_q(S1, S2, d.R);
        const uint32_t k = c.k0 + j;
        if (A.q_debug) A.q_debug[k] = Q;
        atomic_add_i128(A.blocksum + ((size_t)d.slot * A.gdim + k / d.B) * 2,
                        f64_to_i128_trunc(Q * 0x1p64));
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        const uint32_t old = atomicAdd(A.done + d.slot, c.kc);
        if (old + c.kc == d.K) {
            __threadfence();
            finalize_query(A, d, ys);
        }
    }
    __syncthreads();
}

// The host watchdog's abort flag (host memory, read at system scope; the
// value is uniform over the work group once read by one thread, and a flag
// seen late only lets one more chunk run).
__device__ __forceinline__ bool abort_raised(const WalkArgs& A)
{
    return A.abort_flag != nullptr &&
           __hip_atomic_load(A.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u;
}

// kUniform: every chunk of the launch has R >= kUniformMinR (see run_chunk).
// Eight waves per SIMD where the kernel fits 64 VGPRs without spilling.
template <int kLayout, int kUniform, int kShare>
__global__ __launch_bounds__(block_threads(kLayout, kShare),
                             kShare == 1 && lane_pairs(kLayout) == 2                                         ? 4
                             : kShare == 1 && (kUniform || kLayout == kLayoutCompact || hub_layout(kLayout)) ? 8
                                                                                                            : 1) void
walk_kernel(WalkArgs A)
{
    __shared__ unsigned long long acc[kMaxChunkProbes * 4];
    __shared__ double ys[kMaxG];
    __shared__ uint32_t next;
    constexpr int kT = block_threads(kLayout, kShare);
    constexpr uint32_t kHubs = hub_nodes(kT, kLayout);
    __shared__ __align__(16) uint32_t hub_lds[hub_words(kT, kLayout)];
    DevGraph G = make_graph(A.g);
    stage_hubs<kLayout>(G, hub_lds, kHubs);
    if (!A.persistent) {
        // one read of the abort flag for the whole work group (run_chunk has barriers)
        if (threadIdx.x == 0) next = abort_raised(A) ? 1u : 0u;
        __syncthreads();
        if (blockIdx.x < A.nchunks && next == 0u) run_chunk<kLayout, kUniform, kShare>(A, G, blockIdx.x, acc, ys);
        return;
    }
    // Claim chunks from the queue of this XCD first, then from the others in
    // turn. A queue seen empty stays empty (its cursor only grows), so each
    // work group makes at most nqueues failed claims and every wave exits.
    // (thread 0 keeps the queue state in LDS, so it holds no registers while
    // the chunk runs)
    __shared__ uint32_t qstate[2];   // current queue, queues found empty
    if (threadIdx.x == 0) {
        uint32_t xcc = 0;
        if (A.nqueues > 1) asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
        qstate[0] = (xcc & 15u) % A.nqueues;
        qstate[1] = 0;
    }
    for (;;) {
        if (threadIdx.x == 0) {
            uint32_t ci = 0xFFFFFFFFu;
            uint32_t qi = qstate[0], tried = qstate[1];
            if (abort_raised(A)) tried = A.nqueues;  // take no further chunk
            while (tried < A.nqueues) {
                const uint32_t beg = A.qoff[qi];
                const uint32_t c = atomicAdd(A.cursor + qi, 1u);
                if (c < A.qoff[qi + 1] - beg) {
                    ci = beg + c;
                    break;
                }
                qi = qi + 1 == A.nqueues ? 0u : qi + 1;
                ++tried;
            }
            qstate[0] = qi;
            qstate[1] = tried;
            next = ci;
        }
        __syncthreads();
        const uint32_t ci = next;
        __syncthreads();
        if (ci >= A.nchunks) break;
        run_chunk<kLayout, kUniform, kShare>(A, G, ci, acc, ys);
    }
}

template <int kLayout>
static const void* walk_fn_l(int uniform, int share)
{
    if constexpr (kLayout != kLayoutHubRunsNarrow) {  // code 9 shares code 8's sharing kernels
        if (share == 4)
            return uniform ? (const void*)walk_kernel<kLayout, 1, 4> : (const void*)walk_kernel<kLayout, 0, 4>;
        if (share == 2)
            return uniform ? (const void*)walk_kernel<kLayout, 1, 2> : (const void*)walk_kernel<kLayout, 0, 2>;
    }
    return uniform ? (const void*)walk_kernel<kLayout, 1, 1> : (const void*)walk_kernel<kLayout, 0, 1>;
}

static const void* walk_fn(int layout, int uniform, int share)
{
    if (layout == kLayoutFat) return walk_fn_l<kLayoutFat>(uniform, share);
    if (layout == kLayoutFatNT) return walk_fn_l<kLayoutFatNT>(uniform, share);
    if (layout == kLayoutCompact) return walk_fn_l<kLayoutCompact>(uniform, share);
    if (layout == kLayoutCompactHub) return walk_fn_l<kLayoutCompactHub>(uniform, share);
    if (layout == kLayoutHub32) return walk_fn_l<kLayoutHub32>(uniform, share);
    if (layout == kLayoutHubId) return walk_fn_l<kLayoutHubId>(uniform, share);
    if (layout == kLayoutHubIdX2) return walk_fn_l<kLayoutHubIdX2>(uniform, share);
    if (layout == kLayoutHubRuns) return walk_fn_l<kLayoutHubRuns>(uniform, share);
    if (layout == kLayoutHubRunsNarrow) return walk_fn_l<kLayoutHubRunsNarrow>(uniform, share);
    return walk_fn_l<kLayoutCsr>(uniform, share);
}

template <int kLayout, int kUniform>
static void launch_l(const WalkArgs& a, int share, uint32_t grid, hipStream_t st)
{
    if constexpr (kLayout == kLayoutHubRunsNarrow) {  // code 9 shares code 8's sharing kernels
        (void)share;
        hipLaunchKernelGGL((walk_kernel<kLayout, kUniform, 1>), dim3(grid), dim3(block_threads(kLayout, 1)), 0, st, a);
    } else {
        if (share == 4)
            hipLaunchKernelGGL((walk_kernel<kLayout, kUniform, 4>), dim3(grid), dim3(block_threads(kLayout, 4)), 0, st,
                               a);
        else if (share == 2)
            hipLaunchKernelGGL((walk_kernel<kLayout, kUniform, 2>), dim3(grid), dim3(block_threads(kLayout, 2)), 0, st,
                               a);
        else
            hipLaunchKernelGGL((walk_kernel<kLayout, kUniform, 1>), dim3(grid), dim3(block_threads(kLayout, 1)), 0, st,
                               a);
    }
}

hipError_t launch_walk(const WalkArgs& a, int layout, int uniform, int share, uint32_t grid, hipStream_t st)
{
    if (grid == 0) return hipSuccess;
    if (layout == kLayoutFat) {
        if (uniform) launch_l<kLayoutFat, 1>(a, share, grid, st);
        else launch_l<kLayoutFat, 0>(a, share, grid, st);
    } else if (layout == kLayoutFatNT) {
        if (uniform) launch_l<kLayoutFatNT, 1>(a, share, grid, st);
        else launch_l<kLayoutFatNT, 0>(a, share, grid, st);
    } else if (layout == kLayoutCompact) {
        if (uniform) launch_l<kLayoutCompact, 1>(a, share, grid, st);
        else launch_l<kLayoutCompact, 0>(a, share, grid, st);
    } else if (layout == kLayoutCompactHub) {
        if (uniform) launch_l<kLayoutCompactHub, 1>(a, share, grid, st);
        else launch_l<kLayoutCompactHub, 0>(a, share, grid, st);
    } else if (layout == kLayoutHub32) {
        if (uniform) launch_l<kLayoutHub32, 1>(a, share, grid, st);
        else launch_l<kLayoutHub32, 0>(a, share, grid, st);
    } else if (layout == kLayoutHubId) {
        if (uniform) launch_l<kLayoutHubId, 1>(a, share, grid, st);
        else launch_l<kLayoutHubId, 0>(a, share, grid, st);
    } else if (layout == kLayoutHubIdX2) {
        if (uniform) launch_l<kLayoutHubIdX2, 1>(a, share, grid, st);
        else launch_l<kLayoutHubIdX2, 0>(a, share, grid, st);
    } else if (layout == kLayoutHubRuns) {
        if (uniform) launch_l<kLayoutHubRuns, 1>(a, share, grid, st);
        else launch_l<kLayoutHubRuns, 0>(a, share, grid, st);
    } else if (layout == kLayoutHubRunsNarrow) {
        if (uniform) launch_l<kLayoutHubRunsNarrow, 1>(a, share, grid, st);
        else launch_l<kLayoutHubRunsNarrow, 0>(a, share, grid, st);
    } else {
        if (uniform) launch_l<kLayoutCsr, 1>(a, share, grid, st);
        else launch_l<kLayoutCsr, 0>(a, share, grid, st);
    }
    return hipGetLastError();
}

int walk_occupancy(int layout, int uniform, int share, int* wgs_per_cu)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, walk_fn(layout, uniform, share),
                                                     block_threads(layout, share), 0) !=
        hipSuccess)
        return -1;
    *wgs_per_cu = nb;
    return 0;
}

// ---------------------------------------------------------------------------
// Small utility kernels
// ---------------------------------------------------------------------------
__global__ void zero_kernel(uint32_t* p, size_t words)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st)
{
    const size_t words = (bytes + 3) / 4;
    if (words == 0) return hipSuccess;
    size_t blocks = (words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(zero_kernel, dim3((uint32_t)blocks), dim3(256), 0, st, (uint32_t*)p, words);
    return hipGetLastError();
}

__global__ void fat_kernel(const uint4* node, const uint32_t* col, uint4* adj, uint32_t nnz)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += gridDim.x * blockDim.x) {
        const uint4 e = node[col[i]];
        adj[i] = make_uint4(e.w, e.x, e.y, e.z);
    }
}

hipError_t build_fat_adjacency(const uint4* node, const uint32_t* col, uint4* adj, uint32_t nnz,
                               hipStream_t st)
{
    if (nnz == 0) return hipSuccess;
    uint32_t blocks = (nnz + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fat_kernel, dim3(blocks), dim3(256), 0, st, node, col, adj, nnz);
    return hipGetLastError();
}

// One walk per thread, recording X_0..X_L and the binary32 sum of z/d; the
// transitions and the scoring are the production ones (advance / add_term).
template <int kLayout>
__global__ void trace_kernel(GraphTables gt, uint32_t count, const int32_t* start,
                             const uint32_t* uid, const uint32_t* kk, const uint32_t* pp,
                             const uint32_t* side, int32_t L, uint32_t slo, uint32_t shi,
                             int32_t* trace, float* acc_out)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    DevGraph G = make_graph(gt);
    if constexpr (runs_layout(kLayout)) {
        // the run table in LDS, as the walk kernels read it
        __shared__ __align__(16) uint32_t lds[hub_words(1024, kLayout)];
        stage_hubs<kLayout>(G, lds, hub_nodes(1024, kLayout));
    }
    if (i >= count) return;
    const uint32_t x0 = (uint32_t)start[i];
    const Probe pr = make_probe(slo, shi, uid[i], kk[i], G.dom.n);
    WalkState w = start_at<kLayout>(G, x0);
    const uint32_t c3 = (uid[i] << 1) | side[i];
    int32_t* tr = trace ? trace + (size_t)i * (L + 1) : nullptr;
    if (tr) tr[0] = (int32_t)w.x;
    float a = 0.0f;
    U4 r = U4{0, 0, 0, 0};
    for (int s = 0; s < L; ++s) {
        if ((s & 3) == 0) r = philox10((uint32_t)(s >> 2), pp[i], kk[i], c3, slo, shi);
        const uint32_t u = (s & 3) == 0 ? r.x : (s & 3) == 1 ? r.y : (s & 3) == 2 ? r.z : r.w;
        a = advance<kLayout>(w, a, u, G, pr);
        if (tr) tr[s + 1] = (int32_t)w.x;
    }
    a = add_term(a, w.x, w.inv, pr, G.dom);
    if (acc_out) acc_out[i] = a;
}

hipError_t launch_trace(const GraphTables& g, int layout, uint32_t count, const int32_t* start,
                        const uint32_t* uid, const uint32_t* k, const uint32_t* p,
                        const uint32_t* side, int32_t L, uint32_t slo, uint32_t shi,
                        int32_t* trace, float* acc, hipStream_t st)
{
    if (count == 0) return hipSuccess;
    const uint32_t blocks = (count + 127) / 128;
#define PW_TRACE(Lay) hipLaunchKernelGGL(trace_kernel<Lay>, dim3(blocks), dim3(128), 0, st, g, count, start, uid, k, p, side, L, slo, shi, trace, acc)
    if (layout == kLayoutFat) PW_TRACE(1);
    else if (layout == kLayoutFatNT) PW_TRACE(6);
    else if (layout == kLayoutCompact) PW_TRACE(2);
    else if (layout == kLayoutCompactHub) PW_TRACE(3);
    else if (layout == kLayoutHub32) PW_TRACE(4);
    else if (layout == kLayoutHubId) PW_TRACE(5);
    else if (layout == kLayoutHubIdX2) PW_TRACE(7);
    else if (layout == kLayoutHubRuns) PW_TRACE(8);
    else if (layout == kLayoutHubRunsNarrow) PW_TRACE(9);
    else PW_TRACE(0);
#undef PW_TRACE
    return hipGetLastError();
}

__global__ void probe_kernel(GraphTables gt, uint32_t slo, uint32_t shi, uint32_t uid, uint32_t k,
                             uint32_t count, const uint32_t* nodes, uint32_t* pi, int8_t* z)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const DevGraph G = make_graph(gt);
    const Probe pr = make_probe(slo, shi, uid, k, G.dom.n);
    uint32_t y = 0;
    const int v = probe_value(nodes[i], pr, G.dom, &y);
    if (pi) pi[i] = y;
    if (z) z[i] = (int8_t)v;
}

hipError_t launch_probe_eval(const GraphTables& g, uint32_t slo, uint32_t shi, uint32_t uid,
                             uint32_t k, uint32_t count, const uint32_t* nodes, uint32_t* pi,
                             int8_t* z, hipStream_t st)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(probe_kernel, dim3((count + 255) / 256), dim3(256), 0, st, g, slo, shi, uid, k,
                       count, nodes, pi, z);
    return hipGetLastError();
}

}  // namespace pw

namespace pw {

// Gather roofline: the walk's dependent loads over the loaded graph tables
// with a cheap xorshift in place of Philox and no probe arithmetic. Each lane
// runs kChains independent chains of `steps` transitions; the number of
// transitions per second is the memory-side ceiling of the walk kernel on
// this graph, layout and footprint.
template <int kLayout, int kChains>
__global__ __launch_bounds__(block_threads(kLayout, 1)) void gather_kernel(GraphTables gt, int32_t steps, uint32_t seed,
                                                               uint32_t* sink)
{
    constexpr int kT = block_threads(kLayout, 1);
    constexpr uint32_t kHubs = hub_nodes(kT, kLayout);
    __shared__ __align__(16) uint32_t hub_lds[hub_words(kT, kLayout)];
    DevGraph G = make_graph(gt);
    stage_hubs<kLayout>(G, hub_lds, kHubs);
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    WalkState w[kChains];
    uint32_t rng[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        uint32_t h = (gid * kChains + c) * 0x9E3779B1u ^ seed;
        h ^= h >> 16;
        h *= 0x85EBCA6Bu;
        h ^= h >> 13;
        rng[c] = h | 1u;
        w[c] = start_at<kLayout>(G, __umulhi(h, G.dom.n));
    }
    uint32_t acc = 0;
    for (int s = 0; s < steps; ++s) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            uint32_t x = rng[c];
            x ^= x << 13;
            x ^= x >> 17;
            x ^= x << 5;
            rng[c] = x;
            step<kLayout>(w[c], x, G);
        }
    }
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc ^= w[c].x ^ __float_as_uint(w[c].inv);
    sink[gid] = acc;
}

hipError_t launch_gather(const GraphTables& g, int layout, int chains, uint32_t grid, int32_t steps, uint32_t seed,
                         uint32_t* sink, hipStream_t st)
{
#define PW_GATHER(F, C) \
    hipLaunchKernelGGL((gather_kernel<F, C>), dim3(grid), dim3(block_threads(F, 1)), 0, st, g, steps, seed, sink)
#define PW_GATHER_C(F)                  \
    do {                                \
        if (chains == 1) PW_GATHER(F, 1); \
        else if (chains == 2) PW_GATHER(F, 2); \
        else if (chains == 4) PW_GATHER(F, 4); \
        else PW_GATHER(F, 8);           \
    } while (0)
    if (layout == kLayoutFat) PW_GATHER_C(1);
    else if (layout == kLayoutFatNT) PW_GATHER_C(6);
    else if (layout == kLayoutCompact) PW_GATHER_C(2);
    else if (layout == kLayoutCompactHub) PW_GATHER_C(3);
    else if (layout == kLayoutHub32) PW_GATHER_C(4);
    else if (layout == kLayoutHubId) PW_GATHER_C(5);
    else if (layout == kLayoutHubIdX2) PW_GATHER_C(7);
    else if (layout == kLayoutHubRuns) PW_GATHER_C(8);
    else if (layout == kLayoutHubRunsNarrow) PW_GATHER_C(9);
    else PW_GATHER_C(0);
#undef PW_GATHER_C
#undef PW_GATHER
    return hipGetLastError();
}

}  // namespace pw

namespace pw {

// ---------------------------------------------------------------------------
// Sparse products in binary64 for the truncated series (Lemma 2.3) and the
// mixing factor (section 2.1). V is n x Q row-major (Q <= 64 columns).
//
// One wave per row. Its lanes are J = 64/Qp neighbour slots times Qp columns
// (Qp = the power of two >= Q): lane (j, q) sums V[u][q] over the row's
// neighbours j, j + J, j + 2J, ..., and a butterfly over the J slots (the same
// value in every lane of a column, in a fixed order) completes the row sum. With
// Q = 64 a lane owns one column and walks the whole row; with Q = 1 the 64
// lanes share the row's neighbours.
//   kMode 0 (series step):     y[x][q] = (1/d_x) sum_u v[u][q];  h[x][q] += y[x][q]
//   kMode 1 (normalised A):    y[x]    = (1/sqrt d_x) sum_u v[u]  (v = x / sqrt d)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t nbr_at(const uint32_t* col, const uint32_t* col24, uint32_t i)
{
    if (col24) {
        const uint32_t o = i * 3u;
        return __builtin_amdgcn_alignbit(col24[(o >> 2) + 1], col24[o >> 2], (o & 3u) * 8u) & 0xFFFFFFu;
    }
    return col[i];
}

template <int kMode>
__global__ __launch_bounds__(256) void rowsum_kernel(const uint32_t* rp, const uint32_t* col, const uint32_t* col24,
                                                     uint32_t n, uint32_t Q, uint32_t qbits, const double* V,
                                                     double* Y, double* H)
{
    const uint32_t row = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (row >= n) return;  // wave-uniform: the whole wave leaves
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t Qp = 1u << qbits;
    const uint32_t q = lane & (Qp - 1u);
    const uint32_t j = lane >> qbits;
    const uint32_t J = 64u >> qbits;
    const uint32_t b = rp[row], e = rp[row + 1];
    double acc = 0.0;
    if (q < Q)
        for (uint32_t i = b + j; i < e; i += J) acc = __dadd_rn(acc, V[(size_t)nbr_at(col, col24, i) * Q + q]);
    for (uint32_t off = Qp; off < 64u; off <<= 1) acc = __dadd_rn(acc, __shfl_xor(acc, (int)off));
    if (j != 0 || q >= Q) return;
    const double d = (double)(e - b);
    if (kMode == 0) {
        const double y = __dmul_rn(acc, __ddiv_rn(1.0, d));
        const size_t at = (size_t)row * Q + q;
        Y[at] = y;
        H[at] = __dadd_rn(H[at], y);
    } else {
        Y[row] = __ddiv_rn(acc, sqrt(d));
    }
}

// v_0 = D^{-1} b_st for up to 64 queries: zero first, then the two entries of
// each column (storage ids and degrees in the argument block).
struct SeriesSeed {
    uint32_t s[64], t[64];
    double vs[64], vt[64];
};

__global__ void series_seed_kernel(SeriesSeed a, uint32_t Q, double* V, double* H)
{
    const uint32_t q = threadIdx.x;
    if (q >= Q) return;
    V[(size_t)a.s[q] * Q + q] = a.vs[q];
    V[(size_t)a.t[q] * Q + q] = a.vt[q];
    H[(size_t)a.s[q] * Q + q] = a.vs[q];
    H[(size_t)a.t[q] * Q + q] = a.vt[q];
}

// Per-query sums ||h||^2 and 1^T h in a fixed order: one work group per query,
// a strided partial per thread, then a fixed tree in LDS.
__global__ __launch_bounds__(256) void colsum_kernel(const double* H, uint32_t n, uint32_t Q, double* sq,
                                                     double* lin)
{
    __shared__ double a[256], c[256];
    const uint32_t q = blockIdx.x;
    double s2 = 0.0, s1 = 0.0;
    for (uint32_t x = threadIdx.x; x < n; x += 256u) {
        const double h = H[(size_t)x * Q + q];
        s2 = __dadd_rn(s2, __dmul_rn(h, h));
        s1 = __dadd_rn(s1, h);
    }
    a[threadIdx.x] = s2;
    c[threadIdx.x] = s1;
    __syncthreads();
    for (uint32_t w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            a[threadIdx.x] = __dadd_rn(a[threadIdx.x], a[threadIdx.x + w]);
            c[threadIdx.x] = __dadd_rn(c[threadIdx.x], c[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sq[q] = a[0];
        lin[q] = c[0];
    }
}

static uint32_t pow2_bits(uint32_t Q)
{
    uint32_t b = 0;
    while ((1u << b) < Q) ++b;
    return b;
}

hipError_t launch_spmv_step(const uint32_t* rp, const uint32_t* col, const uint32_t* col24, uint32_t n, uint32_t Q,
                            const double* V, double* Y, double* H, hipStream_t st)
{
    hipLaunchKernelGGL(rowsum_kernel<0>, dim3((n + 3) / 4), dim3(256), 0, st, rp, col, col24, n, Q, pow2_bits(Q), V,
                       Y, H);
    return hipGetLastError();
}

hipError_t launch_series_seed(const uint32_t* s, const uint32_t* t, const double* vs, const double* vt, uint32_t Q,
                              double* V, double* H, hipStream_t st)
{
    SeriesSeed a{};
    for (uint32_t q = 0; q < Q && q < 64; ++q) {
        a.s[q] = s[q];
        a.t[q] = t[q];
        a.vs[q] = vs[q];
        a.vt[q] = vt[q];
    }
    hipLaunchKernelGGL(series_seed_kernel, dim3(1), dim3(64), 0, st, a, Q, V, H);
    return hipGetLastError();
}

hipError_t launch_colsum(const double* H, uint32_t n, uint32_t Q, double* sq, double* lin, hipStream_t st)
{
    hipLaunchKernelGGL(colsum_kernel, dim3(Q), dim3(256), 0, st, H, n, Q, sq, lin);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Spectral radius of P off the stationary direction: power iteration on the
// symmetric N = D^{-1/2} A D^{-1/2} (same spectrum as P), whose top
// eigenvector is phi = sqrt(d)/||sqrt(d)|| = sqrt(d / nnz). Every iteration
// runs on the device: z = x / sqrt(d); y = N x (rowsum_kernel<1>); the two sums
// phi.y and y.y in a fixed order (per-block partials, then one block); and
// x = (y - (phi.y) phi) / ||y - (phi.y) phi||, whose norm
// sqrt(y.y - (phi.y)^2) (phi is a unit vector) is the estimate of lambda.
// ---------------------------------------------------------------------------
constexpr uint32_t kDotBlocks = 1024;

__global__ __launch_bounds__(256) void phi_kernel(const uint32_t* rp, uint32_t n, double nnz, double* phi)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        phi[i] = sqrt(__ddiv_rn((double)(rp[i + 1] - rp[i]), nnz));
}

// a counter-based start vector: the SplitMix64 output function of seed + i
// times the golden-ratio increment, mapped to [-1/2, 1/2)
__global__ __launch_bounds__(256) void start_vector_kernel(uint64_t seed, uint32_t n, double* x)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        x[i] = (double)(z >> 11) * 0x1p-53 - 0.5;
    }
}

__global__ __launch_bounds__(256) void scale_rsqrt_deg_kernel(const uint32_t* rp, uint32_t n, const double* x,
                                                              double* z)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        z[i] = __ddiv_rn(x[i], sqrt((double)(rp[i + 1] - rp[i])));
}

__device__ __forceinline__ void block_sum2(double* a, double* c)
{
    for (uint32_t w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            a[threadIdx.x] = __dadd_rn(a[threadIdx.x], a[threadIdx.x + w]);
            c[threadIdx.x] = __dadd_rn(c[threadIdx.x], c[threadIdx.x + w]);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void dot2_kernel(const double* phi, const double* y, uint32_t n, double* part)
{
    __shared__ double a[256], c[256];
    double py = 0.0, yy = 0.0;
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < n; i += gridDim.x * 256u) {
        py = __dadd_rn(py, __dmul_rn(phi[i], y[i]));
        yy = __dadd_rn(yy, __dmul_rn(y[i], y[i]));
    }
    a[threadIdx.x] = py;
    c[threadIdx.x] = yy;
    __syncthreads();
    block_sum2(a, c);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = a[0];
        part[2 * blockIdx.x + 1] = c[0];
    }
}

// scal[0] = phi.y, scal[1] = sqrt(max(y.y - (phi.y)^2, 0))
__global__ __launch_bounds__(256) void dot2_finish_kernel(const double* part, uint32_t nb, double* scal)
{
    __shared__ double a[256], c[256];
    double py = 0.0, yy = 0.0;
    for (uint32_t i = threadIdx.x; i < nb; i += 256u) {
        py = __dadd_rn(py, part[2 * i]);
        yy = __dadd_rn(yy, part[2 * i + 1]);
    }
    a[threadIdx.x] = py;
    c[threadIdx.x] = yy;
    __syncthreads();
    block_sum2(a, c);
    if (threadIdx.x == 0) {
        scal[0] = a[0];
        scal[1] = sqrt(fmax(__dsub_rn(c[0], __dmul_rn(a[0], a[0])), 0.0));
    }
}

__global__ __launch_bounds__(256) void project_kernel(const double* y, const double* phi, const double* scal,
                                                      uint32_t n, double* x)
{
    const double dot = scal[0], nrm = scal[1];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        x[i] = nrm > 0.0 ? __ddiv_rn(__dsub_rn(y[i], __dmul_rn(dot, phi[i])), nrm) : 0.0;
}

hipError_t launch_lambda(const uint32_t* rp, const uint32_t* col, const uint32_t* col24, uint32_t n, uint32_t nnz,
                         int32_t iters, uint64_t seed, double* phi, double* x, double* y, double* z, double* part,
                         double* scal, hipStream_t st)
{
    const dim3 grid(std::min<uint32_t>((n + 255) / 256, 16384u)), block(256);
    const uint32_t nb = std::min<uint32_t>(kDotBlocks, (n + 255) / 256);
    hipLaunchKernelGGL(phi_kernel, grid, block, 0, st, rp, n, (double)nnz, phi);
    hipLaunchKernelGGL(start_vector_kernel, grid, block, 0, st, seed, n, y);
    hipLaunchKernelGGL(dot2_kernel, dim3(nb), block, 0, st, phi, y, n, part);
    hipLaunchKernelGGL(dot2_finish_kernel, dim3(1), block, 0, st, part, nb, scal);
    hipLaunchKernelGGL(project_kernel, grid, block, 0, st, y, phi, scal, n, x);
    for (int32_t it = 0; it < iters; ++it) {
        hipLaunchKernelGGL(scale_rsqrt_deg_kernel, grid, block, 0, st, rp, n, x, z);
        hipLaunchKernelGGL(rowsum_kernel<1>, dim3((n + 3) / 4), block, 0, st, rp, col, col24, n, 1u, 0u, z, y,
                           (double*)nullptr);
        hipLaunchKernelGGL(dot2_kernel, dim3(nb), block, 0, st, phi, y, n, part);
        hipLaunchKernelGGL(dot2_finish_kernel, dim3(1), block, 0, st, part, nb, scal);
        hipLaunchKernelGGL(project_kernel, grid, block, 0, st, y, phi, scal, n, x);
    }
    return hipGetLastError();
}

}  // namespace pw
