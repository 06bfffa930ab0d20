// Device-side building blocks of the ProbeWalk hot path for gfx950.
//
//   * Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).
//   * The stateless Paired-Sign Probe of section 3.3: a keyed permutation pi_k
//     of [n] (alternating Feistel network on Z_A x Z_{2^rb}, cycle walking),
//     the parity zero set, and base signs from the 2-universal hash
//     h_k(u) = ((a_k u + b_k) mod (2^31-1)) mod 2.
//   * One walk transition (Algorithm 1 walk loop) for the two adjacency layouts.
//   * Exact fixed-point sums for the U-statistic (Algorithm 1 S1, S2, Q_R):
//     every per-replica difference U is an integer multiple of 2^-54, so S1 is
//     held as the 128-bit integer S1*2^54, S2 as sum floor(U^2 2^64), and
//     block sums of Q as sum trunc(Q 2^64). Summation order never matters.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pw_internal.hpp"

namespace pw {

typedef __int128 i128;
typedef unsigned __int128 u128;

constexpr uint32_t kHashP = 2147483647u;  // 2^31 - 1
constexpr uint32_t kProbeCtr = 0xFFFFFFFFu;  // counter word reserved for probe keys
constexpr int kFeistelRounds = 6;

// ---------------------------------------------------------------------------
// Philox4x32-10
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

// ---------------------------------------------------------------------------
// Probe domain (per graph) and probe keys (per query and probe index k)
// ---------------------------------------------------------------------------
struct Domain {
    uint32_t n;     // nodes
    uint32_t rb;    // bits of the XOR half
    uint32_t mask;  // 2^rb - 1
    uint32_t rsh;   // 32 - rb (31 when rb == 0; the mask then clears the result)
    uint32_t A;     // modulus of the additive half, A = ceil(n / 2^rb)
    uint32_t A8;    // A << 8
};

struct Probe {
    uint32_t K[kFeistelRounds];
    uint32_t a, b;
    uint32_t zlo;   // first zero position: pi_k(i) >= zlo  <=>  z_i = 0  (zlo = n - r)
};

__device__ __forceinline__ Probe make_probe(uint32_t seed_lo, uint32_t seed_hi, uint32_t uid,
                                            uint32_t k, uint32_t n)
{
    Probe pr;
    const U4 w0 = philox10(0u, kProbeCtr, k, uid << 1, seed_lo, seed_hi);
    const U4 w1 = philox10(1u, kProbeCtr, k, uid << 1, seed_lo, seed_hi);
    const U4 w2 = philox10(2u, kProbeCtr, k, uid << 1, seed_lo, seed_hi);
    pr.K[0] = w0.x;
    pr.K[1] = w0.y;
    pr.K[2] = w0.z;
    pr.K[3] = w0.w;
    pr.K[4] = w1.x;
    pr.K[5] = w1.y;
    pr.a = 1u + w1.z % (kHashP - 1u);
    pr.b = w1.w % kHashP;
    const uint32_t r = (n & 1u) ? 1u : 2u * (w2.x & 1u);
    pr.zlo = n - r;
    return pr;
}

__device__ __forceinline__ uint32_t umul24(uint32_t a, uint32_t b)
{
    return (uint32_t)((uint64_t)(a & 0xFFFFFFu) * (uint64_t)(b & 0xFFFFFFu));
}

__device__ __forceinline__ uint32_t umul24hi(uint32_t a, uint32_t b)
{
    return (uint32_t)(((uint64_t)(a & 0xFFFFFFu) * (uint64_t)(b & 0xFFFFFFu)) >> 32);
}

__device__ __forceinline__ uint32_t fmix(uint32_t v, uint32_t key)
{
    uint32_t h = umul24(v ^ key, 0x9E3779u);
    h ^= h >> 15;
    return umul24(h, 0x873593u);
}

// pi_k(x): Feistel rounds alternate L <- (L + F(R)) mod A and R <- R ^ top_rb(F(L));
// values that land in [n, A*2^rb) are walked again until they fall in [n].
__device__ __forceinline__ uint32_t feistel_pi(uint32_t x, const Probe& pr, const Domain& dm)
{
    do {
        uint32_t L = x >> dm.rb;
        uint32_t R = x & dm.mask;
#pragma unroll
        for (int r = 0; r < kFeistelRounds; r += 2) {
            const uint32_t f = umul24hi(fmix(R, pr.K[r]) >> 8, dm.A8);
            const uint32_t t = L + f;
            L = min(t, t - dm.A);  // (L + f) mod A, since L + f < 2A
            R ^= (fmix(L, pr.K[r + 1]) >> dm.rsh) & dm.mask;
        }
        x = (L << dm.rb) | R;
    } while (x >= dm.n);
    return x;
}

// ((a u + b) mod (2^31 - 1)) & 1 for u < 2^30, a, b < 2^31
__device__ __forceinline__ uint32_t hash_bit(const Probe& pr, uint32_t u)
{
    const uint64_t v = (uint64_t)pr.a * u + pr.b;  // < 2^62
    uint32_t t = ((uint32_t)v & kHashP) + (uint32_t)(v >> 31);
    t = (t & kHashP) + (t >> 31);
    t = min(t, t - kHashP);
    return t & 1u;
}

// acc + z^(k)_x * inv, skipping the term when z = 0
__device__ __forceinline__ float add_term(float acc, uint32_t x, float inv, const Probe& pr,
                                          const Domain& dm)
{
    const uint32_t y = feistel_pi(x, pr, dm);
    const uint32_t neg = hash_bit(pr, y >> 1) ^ (y & 1u);
    const float v = neg ? -inv : inv;
    const float s = __fadd_rn(acc, v);
    return (y >= pr.zlo) ? acc : s;
}

__device__ __forceinline__ int probe_value(uint32_t x, const Probe& pr, const Domain& dm,
                                           uint32_t* pi_out)
{
    const uint32_t y = feistel_pi(x, pr, dm);
    *pi_out = y;
    if (y >= pr.zlo) return 0;
    return (hash_bit(pr, y >> 1) ^ (y & 1u)) ? -1 : 1;
}

// ---------------------------------------------------------------------------
// Graph tables and one walk transition
// ---------------------------------------------------------------------------
// Node table entry, indexed by the internal (storage) id of a node:
//   {row offset, degree, bits of 1.0f/degree, original id}.
// Internal ids may be a relabelling of the caller's ids (hubs first, for
// locality); rows keep the caller's neighbour order, and the probe is always
// evaluated on the original id, so trajectories do not depend on the storage.
// Fat adjacency entry at position row_offset(x) + j:
//   {neighbour's original id, its row offset, its degree, bits of its 1.0f/degree}.
//
// Compact layout (ids as given, n <= 2^24): row offsets rp[0..n] as uint32 and
// neighbour ids packed in 3 bytes each; 1.0f/degree is recomputed (correctly
// rounded) at every step instead of stored.
// Compact layout with hubs first: storage ids in descending-degree order, node
// entries {row offset, original id} (8 bytes; entry n = {nnz, 0}), neighbour
// storage ids packed in 3 bytes; the entries of the first hub_nodes() storage ids
// (the highest-degree nodes, which the walks visit most) are staged in LDS.
// Above 2^24 nodes the same layout keeps 4-byte neighbour storage ids.
// Hubs first with the probe on storage ids: the same storage order, but the
// probe is evaluated on the storage id itself (the node's rank in descending
// degree), so a node entry is its 4-byte row offset alone (rp[x], rp[x + 1]:
// one 8-byte load) and twice as many hubs fit in the same LDS.
// (layout codes and hub counts: pw_internal.hpp)

struct DevGraph {
    const uint4* node;      // n entries (CSR and fat layouts)
    const uint32_t* col;    // nnz entries (CSR layout; hubs-first layout above 2^24 nodes)
    const uint4* adj;       // nnz entries (fat layout)
    const uint32_t* rp;     // n + 1 entries (compact layout)
    const uint32_t* col24;  // 3 nnz bytes + padding, read as aligned words (compact layouts)
    const uint2* node8;     // n + 1 entries {row offset, original id} (compact layout, hubs first)
    const uint2* hub;       // LDS copy of node8[0 .. nhub] (nhub = 0: none)
    const uint32_t* hub4;   // LDS copy of rp[0 .. nhub] (probe on storage ids)
    const uint32_t* runtab; // code 8: the run table (global memory), staged in LDS as hub4
    const float* inv;       // code 8: LDS table of 1.0f/d for d = 0 .. d_max
    uint32_t run_h1, run_words, run_ninv, run_shift;
    uint32_t rec_word;      // code 8: word index of the run records in hub4
    uint32_t nhub;
    Domain dom;
};

struct WalkState {
    uint32_t x, off, deg;
    float inv;
};

__device__ __forceinline__ WalkState start_state(uint4 e)
{
    return WalkState{e.w, e.x, e.y, __uint_as_float(e.z)};
}

// Row offset and degree of node x in the compact layout (one 8-byte load).
__device__ __forceinline__ void compact_row(const DevGraph& G, uint32_t x, WalkState& w)
{
    const uint32_t b = G.rp[x];
    const uint32_t e = G.rp[x + 1];
    w.x = x;
    w.off = b;
    w.deg = e - b;
    w.inv = __fdiv_rn(1.0f, (float)w.deg);
}

// Node x of the compact layout with hubs first: entries x and x + 1 (LDS for
// the staged hubs, else one 16-byte global load), the probe sees the original id.
__device__ __forceinline__ void hub_row(const DevGraph& G, uint32_t x, WalkState& w)
{
    uint2 a, b;
    if (x < G.nhub) {
        a = G.hub[x];
        b = G.hub[x + 1];
    } else {
        a = G.node8[x];
        b = G.node8[x + 1];
    }
    w.x = a.y;
    w.off = a.x;
    w.deg = b.x - a.x;
    w.inv = __fdiv_rn(1.0f, (float)w.deg);
}

// Node x with the probe on its storage id: rp[x], rp[x + 1] from LDS for the
// staged hubs, else one 8-byte global load.
__device__ __forceinline__ void hubid_row(const DevGraph& G, uint32_t x, WalkState& w)
{
    uint32_t b, e;
    if (x < G.nhub) {
        b = G.hub4[x];
        e = G.hub4[x + 1];
    } else {
        b = G.rp[x];
        e = G.rp[x + 1];
    }
    w.x = x;
    w.off = b;
    w.deg = e - b;
    w.inv = __fdiv_rn(1.0f, (float)w.deg);
}

// Node x with every node resolved from LDS (code 8): the row offsets of the
// first nhub storage ids, then one record per block of 2^run_shift storage ids
// past them (the layout is described with kLayoutHubRuns). Without the
// records (a kernel that did not stage them) the global row offsets give the
// same values.
__device__ __forceinline__ void runs_row(const DevGraph& G, uint32_t x, WalkState& w)
{
    // one two-word LDS read at either x (direct offsets: rp[x], rp[x + 1]) or
    // x's block record, both decoded and the right one selected
    const bool direct = x < G.nhub;
    const uint32_t i = x - G.nhub;
    const uint32_t at = direct ? x : G.rec_word + 2u * (i >> G.run_shift);
    const uint32_t w0 = G.hub4[at], w1 = G.hub4[at + 1];
    const uint32_t j = i & ((1u << G.run_shift) - 1u);
    const uint32_t dA = w1 & kRunMaxDeg, dB = (w1 >> 11) & kRunMaxDeg, bnd = w1 >> 22;
    const uint32_t ja = min(j, bnd);
    const uint32_t d = direct ? w1 - w0 : (j < bnd ? dA : dB);
    w.x = x;
    w.off = direct ? w0 : w0 + ja * dA + (j - ja) * dB;
    w.deg = d;
    w.inv = G.inv[d];
}

// Walk state at internal id x (the start of a walk).
template <int kLayout>
__device__ __forceinline__ WalkState start_at(const DevGraph& G, uint32_t x)
{
    if (kLayout == kLayoutCompact) {
        WalkState w;
        compact_row(G, x, w);
        return w;
    }
    if (kLayout == kLayoutCompactHub || kLayout == kLayoutHub32) {
        WalkState w;
        hub_row(G, x, w);
        return w;
    }
    if (runs_layout(kLayout)) {
        WalkState w;
        runs_row(G, x, w);
        return w;
    }
    if (hubid_layout(kLayout)) {
        WalkState w;
        hubid_row(G, x, w);
        return w;
    }
    return start_state(G.node[x]);
}

// Uniform neighbour: j = floor(u * d / 2^32) into the ascending neighbour list.
template <int kLayout>
__device__ __forceinline__ void step(WalkState& w, uint32_t u, const DevGraph& G)
{
    const uint32_t j = __umulhi(u, w.deg);
    const uint32_t pos = w.off + j;
    if (kLayout == kLayoutFat || kLayout == kLayoutFatNT) {
        uint4 e;
        if (kLayout == kLayoutFatNT) {
            typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
            const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(G.adj) + pos);
            e = make_uint4(v.x, v.y, v.z, v.w);
        } else {
            e = G.adj[pos];
        }
        w.x = e.x;
        w.off = e.y;
        w.deg = e.z;
        w.inv = __uint_as_float(e.w);
    } else if (kLayout == kLayoutCompact || kLayout == kLayoutCompactHub || hubid_layout(kLayout)) {
        // the 3 bytes at byte offset 3*pos lie in the aligned 8 bytes at word (3*pos)/4
        const uint32_t o = pos * 3u;
        const uint32_t wi = o >> 2;
        const uint32_t lo = G.col24[wi];
        const uint32_t hi = G.col24[wi + 1];
        const uint32_t x = __builtin_amdgcn_alignbit(hi, lo, (o & 3u) * 8u) & 0xFFFFFFu;
        if (kLayout == kLayoutCompact) compact_row(G, x, w);
        else if (runs_layout(kLayout)) runs_row(G, x, w);
        else if (hubid_layout(kLayout)) hubid_row(G, x, w);
        else hub_row(G, x, w);
    } else if (kLayout == kLayoutHub32) {
        hub_row(G, G.col[pos], w);
    } else {
        const uint4 e = G.node[G.col[pos]];
        w.x = e.w;
        w.off = e.x;
        w.deg = e.y;
        w.inv = __uint_as_float(e.z);
    }
}

// Copy the hub entries of the compact layout with hubs first into LDS (every
// thread of the block must call it); other layouts keep nhub = 0.
template <int kLayout>
__device__ __forceinline__ void stage_hubs(DevGraph& G, uint32_t* lds, uint32_t capacity)
{
    if constexpr (kLayout == kLayoutCompactHub || kLayout == kLayoutHub32) {
        const uint32_t nh = min(capacity, G.dom.n);
        uint2* l2 = reinterpret_cast<uint2*>(lds);
        for (uint32_t i = threadIdx.x; i <= nh; i += blockDim.x) l2[i] = G.node8[i];
        __syncthreads();
        G.hub = l2;
        G.nhub = nh;
    } else if constexpr (runs_layout(kLayout)) {
        // the run table, then 1.0f/d for every degree 0 .. d_max (the same
        // correctly rounded quotients a step would compute); the host takes
        // this layout only where both fit `capacity` + 1 words
        const uint32_t words = G.run_words;
        const uint32_t inv_at = (words + 3u) & ~3u;
        for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) lds[i] = G.runtab[i];
        for (uint32_t i = threadIdx.x; i < G.run_ninv; i += blockDim.x)
            lds[inv_at + i] = __float_as_uint(__fdiv_rn(1.0f, (float)max(i, 1u)));
        __syncthreads();
        G.hub4 = lds;
        G.nhub = G.run_h1;
        G.rec_word = run_records_at(G.run_h1);
        G.inv = reinterpret_cast<const float*>(lds + inv_at);
        (void)capacity;
    } else if constexpr (hubid_layout(kLayout)) {
        const uint32_t nh = min(capacity, G.dom.n);
        for (uint32_t i = threadIdx.x; i <= nh; i += blockDim.x) lds[i] = G.rp[i];
        __syncthreads();
        G.hub4 = lds;
        G.nhub = nh;
    }
}

// ---------------------------------------------------------------------------
// Exact fixed-point helpers
// ---------------------------------------------------------------------------
// U * 2^54 (exact: U is a multiple of 2^-54 with |U| < 2^15)
__device__ __forceinline__ i128 fix54(float U)
{
    const uint32_t b = __float_as_uint(U);
    const int e = (int)((b >> 23) & 0xFFu);
    if (e == 0) return 0;
    const uint64_t M = (uint64_t)((b & 0x7FFFFFu) | 0x800000u);
    const int sh = e - 96;  // (e - 127 - 23) + 54
    u128 mag;
    if (sh >= 0) mag = (u128)M << sh;
    else mag = (sh > -32) ? (u128)(M >> (-sh)) : (u128)0;
    return (b >> 31) ? -(i128)mag : (i128)mag;
}

// floor(U^2 * 2^64)
__device__ __forceinline__ u128 sqfix64(float U)
{
    const uint32_t b = __float_as_uint(U);
    const int e = (int)((b >> 23) & 0xFFu);
    if (e == 0) return 0;
    const uint64_t M = (uint64_t)((b & 0x7FFFFFu) | 0x800000u);
    const uint64_t M2 = M * M;  // < 2^48
    const int sh = 2 * e - 236;  // 2 (e - 150) + 64
    if (sh >= 0) return (u128)M2 << sh;
    if (sh > -64) return (u128)(M2 >> (-sh));
    return 0;
}

// Correctly rounded (round-to-nearest-even) conversions of 128-bit integers to
// binary64: normalise, keep the top 64 bits with a sticky bit in bit 0, and let
// the exact two-part u64 -> f64 conversion round once.
__device__ __forceinline__ double u128_to_f64(u128 m)
{
    const uint64_t hi = (uint64_t)(m >> 64);
    const uint64_t lo = (uint64_t)m;
    if (hi == 0) {
        // u64 -> f64: hi32 * 2^32 + lo32 is a single rounding of exact parts
        const double h = (double)(uint32_t)(lo >> 32) * 4294967296.0;
        return h + (double)(uint32_t)lo;
    }
    const int lz = __clzll(hi);
    const u128 n = m << lz;  // MSB at bit 127
    uint64_t top = (uint64_t)(n >> 64);
    top |= ((uint64_t)n != 0) ? 1ull : 0ull;
    const double h = (double)(uint32_t)(top >> 32) * 4294967296.0;
    const double t = h + (double)(uint32_t)top;
    return ldexp(t, 64 - lz);
}

__device__ __forceinline__ double i128_to_f64(i128 v)
{
    return v < 0 ? -u128_to_f64((u128)(-v)) : u128_to_f64((u128)v);
}

// trunc(d) for |d| < 2^126 as a 128-bit integer
__device__ __forceinline__ i128 f64_to_i128_trunc(double d)
{
    const double m = fabs(trunc(d));
    const double hi = floor(m * 0x1p-64);
    const double lo = m - hi * 0x1p64;
    const u128 mag = ((u128)(uint64_t)hi << 64) | (u128)(uint64_t)lo;
    return d < 0 ? -(i128)mag : (i128)mag;
}

// Q = (s1^2 - s2) / (R (R - 1)) with s1 = S1 2^-54, s2 = S2 2^-64
__device__ __forceinline__ double probe_q(i128 S1, u128 S2, uint32_t R)
{
    const double s1 = i128_to_f64(S1) * 0x1p-54;
    const double s2 = u128_to_f64(S2) * 0x1p-64;
    const double num = __dsub_rn(__dmul_rn(s1, s1), s2);
    const double den = __dmul_rn((double)R, (double)(R - 1u));
    return __ddiv_rn(num, den);
}

// 128-bit atomic add as two 64-bit atomics with an explicit carry: the low
// word's returned old value tells whether this addition wrapped, so the
// high word receives exactly the carries of all additions.
__device__ __forceinline__ void atomic_add_i128(unsigned long long* p, i128 v)
{
    const unsigned long long lo = (unsigned long long)(u128)v;
    const unsigned long long hi = (unsigned long long)((u128)v >> 64);
    const unsigned long long old = atomicAdd(p, lo);
    const unsigned long long carry = (old + lo < old) ? 1ull : 0ull;
    atomicAdd(p + 1, hi + carry);
}

__device__ __forceinline__ i128 load_i128(const unsigned long long* p)
{
    const unsigned long long lo = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long hi = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (i128)(((u128)hi << 64) | (u128)lo);
}

}  // namespace pw
