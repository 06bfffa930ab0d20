"""Write cl100k_cg_reference.txt: exact beta for the first 128 query pairs of
the Chung-Lu n=100,000 workload.

Calls only the oracle (oracle.exact: CG with a second solve; the truncated
series beta^(L) at L = 1000 for the first 8 pairs) and the seeded generators.

    python tests/golden/make_cl100k_reference.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact  # noqa: E402
from synth import graphs, queries  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cl100k_cg_reference.txt")


def main():
    g = graphs.workload_graph("cl100k")
    s, t = queries.uniform_pairs(g.n, 4096, graphs.GRAPH_SEED + 1 + graphs.QUERY_SEED_OFFSET)
    lines = ["# Exact squared biharmonic distance, Chung-Lu n=100,000 mean degree 10 exponent 2.5 LCC",
             f"# graph: n={g.n} nnz={g.nnz}; pairs: synth.queries.uniform_pairs(n, 4096, seed) first 128",
             "# beta_cg = ||x||^2 with (L + 11^T/n) x = b (Jacobi PCG, rel. residual 1e-12);",
             "# beta_2nd = b^T y with (L + 11^T/n) y = x; beta_L1000 = truncated series (first 8 pairs, else nan)",
             "# index s t d_s d_t beta_cg beta_2nd beta_L1000"]
    for i in range(128):
        b1, b2, _ = exact.beta_cg(g, int(s[i]), int(t[i]))
        bl = exact.beta_truncated(g, int(s[i]), int(t[i]), 1000) if i < 8 else float("nan")
        lines.append(f"{i} {s[i]} {t[i]} {g.deg[s[i]]} {g.deg[t[i]]} {b1!r} {b2!r} {bl!r}")
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(OUT)


if __name__ == "__main__":
    main()
