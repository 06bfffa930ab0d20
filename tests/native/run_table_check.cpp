// Host check of the degree-run node table (pw_runs.hpp): reads cases from
// stdin, one per line: "shift ninv capacity_words n d_0 d_1 ... d_{n-1}" with
// the degrees of a graph in storage order (descending). For each it prints
// "ok h1 words" when the table was built and every node's row offset and
// degree decode to the row offsets', "nofit" when the builder declined, or
// "bad x" at the first node that decodes wrong.
#include <cstdio>
#include <vector>

#include "pw_runs.hpp"

int main()
{
    unsigned shift, ninv;
    size_t cap, n;
    while (std::scanf("%u %u %zu %zu", &shift, &ninv, &cap, &n) == 4) {
        std::vector<uint32_t> rp(n + 1, 0u);
        for (size_t i = 0; i < n; ++i) {
            unsigned d;
            if (std::scanf("%u", &d) != 1) return 2;
            rp[i + 1] = rp[i] + d;
        }
        uint32_t h1 = 0;
        std::vector<uint32_t> tab;
        if (!pw::build_run_table(rp, shift, ninv, cap, &h1, &tab)) {
            std::printf("nofit\n");
            continue;
        }
        size_t bad = n;
        for (size_t x = 0; x < n && bad == n; ++x) {
            uint32_t off = 0, deg = 0;
            pw::run_table_row(tab, h1, shift, (uint32_t)x, &off, &deg);
            if (off != rp[x] || deg != rp[x + 1] - rp[x]) bad = x;
        }
        if (bad < n) std::printf("bad %zu\n", bad);
        else std::printf("ok %u %zu\n", h1, tab.size());
    }
    return 0;
}
