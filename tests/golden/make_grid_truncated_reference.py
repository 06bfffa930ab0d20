"""Write grid1414_truncated_reference.txt: the truncated distance beta^(L)
(Lemma 2.3) for the first 32 query pairs of the 1,414 x 1,414 grid workload at
L = 500, 2000 and 5000.

The grid is bipartite, so the series does not converge to beta and beta^(L)
is the reference the estimator is measured against at a fixed L. Calls only the
oracle (oracle.exact.beta_truncated_multi: L binary64 sparse products) and the
seeded generators; about 20 minutes on one core.

    python tests/golden/make_grid_truncated_reference.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact  # noqa: E402
from synth import graphs, queries  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grid1414_truncated_reference.txt")
LS = (500, 2000, 5000)
PAIRS = 32


def main():
    g = graphs.workload_graph("grid1414")
    s, t, _, _ = queries.workload_batch("grid1414", g.n)
    s, t = s[:PAIRS], t[:PAIRS]
    out = exact.beta_truncated_multi(g, s, t, LS)
    lines = ["# Truncated squared biharmonic distance beta^(L) = ||h||^2 - (1^T h)^2 / n,",
             "# h = sum_{i<=L} P^i D^-1 b_st (binary64 sparse products), 1,414 x 1,414 grid, 5% of edges removed",
             f"# graph: n={g.n} nnz={g.nnz}; pairs: synth.queries.workload_batch('grid1414', n) first {PAIRS}",
             "# index s t d_s d_t " + " ".join(f"beta_L{L}" for L in LS)]
    for i in range(PAIRS):
        vals = " ".join(repr(float(out[j, i])) for j in range(len(LS)))
        lines.append(f"{i} {s[i]} {t[i]} {g.deg[s[i]]} {g.deg[t[i]]} {vals}")
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(OUT)


if __name__ == "__main__":
    main()
