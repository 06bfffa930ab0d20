"""Write the exact squared biharmonic distances of sampled query pairs of the
two large Chung-Lu workloads, by binary64 CG in plain torch on a GPU.

Calls only the oracle (oracle.cg_torch: many-pairs CG with a second solve, the
truncated series beta^(L) at L = 1000 for the first 8 pairs) and the seeded
generators.

  cl10m  Chung-Lu n=1e7, mean degree 10, exponent 2.3, LCC: the first 64 pairs
         of its query set (tests/golden/cl10m_cg_reference.txt)
  cl40m  Chung-Lu n=4e7, mean degree 25, exponent 2.2, LCC: the first 64 pairs
         of its 262,144-query set, with their L (tests/golden/cl40m_cg_reference.txt)

    python tests/golden/make_cg_reference.py cl10m [--out PATH] [--count 64]
"""
import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

from oracle import cg_torch  # noqa: E402
from synth import graphs, queries  # noqa: E402

DESC = {
    "cl10m": "Chung-Lu n=10,000,000 mean degree 10 exponent 2.3 LCC",
    "cl40m": "Chung-Lu n=40,000,000 mean degree 25 exponent 2.2 LCC",
}


def say(*a):
    print(*a, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(DESC))
    ap.add_argument("--out", default=None)
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--chunk", type=int, default=32)
    ap.add_argument("--truncated", type=int, default=8, help="pairs that also get beta^(1000)")
    a = ap.parse_args()
    out = a.out or os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{a.workload}_cg_reference.txt")
    t0 = time.time()
    g = graphs.workload_graph(a.workload)
    say(f"graph {a.workload}: n={g.n} nnz={g.nnz} ({time.time() - t0:.1f} s)")
    s, t, _, L = queries.workload_batch(a.workload, g.n, a.count)
    op = cg_torch.Laplacian(g, "cuda")
    say(f"laplacian on {op.device} ({time.time() - t0:.1f} s)")
    b1, b2, its, res = cg_torch.beta_cg_many(g, s, t, "cuda", chunk=a.chunk, op=op, log=say)
    say(f"cg done ({time.time() - t0:.1f} s)")
    m = min(a.truncated, a.count)
    bl = np.full(a.count, np.nan)
    if m:
        bl[:m] = cg_torch.beta_truncated_many(g, s[:m], t[:m], 1000, "cuda", op=op)
    say(f"truncated series done ({time.time() - t0:.1f} s)")
    lines = [f"# Exact squared biharmonic distance, {DESC[a.workload]}",
             f"# graph: n={g.n} nnz={g.nnz}; pairs: synth.queries.workload_batch('{a.workload}', n) first {a.count}",
             "# beta_cg = ||x||^2 with (L + 11^T/n) x = b (Jacobi PCG in binary64, plain torch on a GPU,",
             "# rel. residual 1e-12); beta_2nd = b^T y with (L + 11^T/n) y = x;",
             f"# beta_L1000 = truncated series at L = 1000 (first {m} pairs, else nan); L = the query's L",
             "# index s t d_s d_t L beta_cg beta_2nd beta_L1000 cg_iterations max_rel_residual"]
    for i in range(a.count):
        lines.append(f"{i} {s[i]} {t[i]} {g.deg[s[i]]} {g.deg[t[i]]} {L[i]} {float(b1[i])!r} {float(b2[i])!r} "
                     f"{float(bl[i])!r} {its[i]} {res[i]:.3e}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    rel = np.abs(b1 - b2) / b1
    say(f"wrote {out}: two-solve agreement max {rel.max():.2e}; gap to beta^(1000) "
        f"max {np.nanmax(np.abs(bl - b1) / b1) if m else float('nan'):.2e}")


if __name__ == "__main__":
    main()
