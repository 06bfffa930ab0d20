// The degree-run node table of kernel code 8 (host side, no HIP): the
// constants of its layout, the builder, and the decoding the kernels apply
// (runs_row in pw_device.hpp computes the same from its LDS copy).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

namespace pw {

constexpr uint32_t kRunShiftMin = 6, kRunShiftMax = 9;
constexpr uint32_t kRunMaxDeg = 0x7FFu;
// first 32-bit word of the run records in the table (8-byte aligned)
constexpr uint32_t run_records_at(uint32_t h1) { return (h1 + 2u) & ~1u; }

// The degree-run table of kernel code 8 from the row offsets rp[0..n] of a
// graph stored in descending-degree order, for blocks of 2^shift storage ids:
// h1 is the smallest start of a run of equal degree (or 0, or n) such that
// every block from h1 on holds at most two runs and no run past it has degree
// above kRunMaxDeg. The table is rp[0..h1], padding to an even word, then per
// block {rp of its first node, dA | dB << 11 | bnd << 22}. Its size grows
// with h1, so false if at that h1 it and the ninv reciprocals the kernels
// place after it (from a 4-word boundary) would exceed capacity_words.
inline bool build_run_table(const std::vector<uint32_t>& rp, uint32_t shift, uint32_t ninv, size_t capacity_words,
                            uint32_t* h1_out, std::vector<uint32_t>* out)
{
    const size_t n = rp.size() - 1, block = size_t(1) << shift;
    auto deg = [&](size_t i) { return rp[i + 1] - rp[i]; };
    // starts[i]: run starts among storage ids 1 .. i-1 (a start at j > 0 is a
    // change of degree between j - 1 and j)
    std::vector<uint32_t> starts(n + 1, 0u);
    size_t hmin = 0;
    for (size_t i = 1; i <= n; ++i) starts[i] = starts[i - 1] + (i - 1 > 0 && deg(i - 1) != deg(i - 2) ? 1u : 0u);
    for (size_t i = 0; i < n; ++i)
        if (deg(i) > kRunMaxDeg) hmin = i + 1;
    auto runs_in = [&](size_t f, size_t e) { return 1u + starts[e] - starts[f + 1]; };  // runs in [f, e)
    auto valid = [&](size_t h) {
        for (size_t f = h; f < n; f += block)
            if (runs_in(f, std::min(n, f + block)) > 2u) return false;
        return true;
    };
    size_t h1 = n;
    for (size_t h = hmin; h <= n; ++h) {
        if (h != hmin && h != n && deg(h) == deg(h - 1)) continue;  // candidates: run starts
        if (valid(h)) {
            h1 = h;
            break;
        }
    }
    const size_t blocks = (n - h1 + block - 1) / block;
    const size_t at = run_records_at((uint32_t)h1);
    const size_t words = at + 2 * blocks;
    if (((words + 3) & ~(size_t)3) + ninv > capacity_words) return false;
    out->assign(words, 0u);
    for (size_t i = 0; i <= h1; ++i) (*out)[i] = rp[i];
    for (size_t b = 0; b < blocks; ++b) {
        const size_t f = h1 + b * block, len = std::min<size_t>(block, n - f);
        const uint32_t dA = deg(f);
        size_t bnd = 0;
        while (bnd < len && deg(f + bnd) == dA) ++bnd;
        const uint32_t dB = bnd < len ? deg(f + bnd) : 0u;
        (*out)[at + 2 * b] = rp[f];
        (*out)[at + 2 * b + 1] = dA | (dB << 11) | ((uint32_t)bnd << 22);
    }
    *h1_out = (uint32_t)h1;
    return true;
}

// Row offset and degree of storage id x from the table (h1 and shift as built).
inline void run_table_row(const std::vector<uint32_t>& tab, uint32_t h1, uint32_t shift, uint32_t x, uint32_t* off,
                          uint32_t* deg)
{
    if (x < h1) {
        *off = tab[x];
        *deg = tab[x + 1] - tab[x];
        return;
    }
    const uint32_t i = x - h1, at = run_records_at(h1) + 2u * (i >> shift), j = i & ((1u << shift) - 1u);
    const uint32_t w0 = tab[at], w1 = tab[at + 1];
    const uint32_t dA = w1 & kRunMaxDeg, dB = (w1 >> 11) & kRunMaxDeg, bnd = w1 >> 22;
    const uint32_t ja = std::min(j, bnd);
    *off = w0 + ja * dA + (j - ja) * dB;
    *deg = j < bnd ? dA : dB;
}

}  // namespace pw
