"""Calibration of the scaled walk-count policy against exact distances.

Algorithm 1 sets B = ceil(c_B / eps^2) and
R = ceil(c_R (L+1)^2 / (d_min^2 (1 - eps/2) (1/d_s + 1/d_t)^2)) with the
worst-case constants c_B = 448, c_R = 128 (proof of Theorem 3.8). The scaled
policy keeps both formulas and takes the cheapest (c_B, c_R) from a ladder
that puts at least a target fraction of reference queries within eps of their
exact distance (Problem 2.2's criterion), for one graph and one L.

One GPU run per c_R is enough for every c_B of the ladder: the per-probe
statistic Q_k of probe k depends only on (seed, uid, k, R, L), never on B, and
for a given B the estimate is the median of the G means of the consecutive
blocks [gB, (g+1)B) of Q_0, Q_1, ... So the run at the largest B returns
(bd_query_probes) every Q_k a smaller B would use, and the smaller B's
estimate is formed from them exactly as the kernel forms it: block sums of
trunc(Q_k 2^64) in exact integers, divided by 2^64 and by B in binary64, and
the middle block mean (the mean of the two middle ones for even G).

The exact distances are inputs (for the workloads of this repository they are
the stored CG references under tests/golden); nothing here computes them.

    python -m paper_2512_05460_amd.calibrate cl10m --ref tests/golden/cl10m_cg_reference.txt
"""

from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import binding as B

GUARD = 1.0 - 2.0 ** -40


def _ceil(x: float) -> int:
    return int(math.ceil(x * GUARD))


def median_of_means(q: np.ndarray, b: int, G: int) -> float:
    """The estimate from the per-probe values of probes 0 .. bG-1 (blocks of b)."""
    means = []
    for g in range(G):
        acc = 0
        for v in q[g * b:(g + 1) * b]:
            acc += int(float(v) * 2.0 ** 64)  # trunc(Q 2^64), exact
        means.append((float(acc) * 2.0 ** -64) / b)
    means.sort()
    return means[G // 2] if G % 2 else 0.5 * (means[G // 2 - 1] + means[G // 2])


def probe_values(dg, s, t, eps: float, L, seed: int, c_B: float, c_R: float, uid=None, log=None):
    """Per query: (Q_k for every probe at c_B, result) from one run each (batched
    mode, whose results are the plain mode's bit for bit)."""
    pol = B.policy("scaled", c_B=c_B, c_R=c_R)
    out = []
    L = np.broadcast_to(np.asarray(L), np.shape(s))
    t0 = time.time()
    for i in range(len(s)):
        u = i if uid is None else int(uid[i])
        res, q, _ = B.bd_query_probes(dg, int(s[i]), int(t[i]), eps, int(L[i]), u, seed, pol,
                                      B.exec_cfg("batched"))
        out.append((q, res))
        # a line per query where queries are long (each is one device call)
        if log is not None and ((i + 1) % 16 == 0 or int(L[i]) > 2000):
            log(f"    {i + 1}/{len(s)} queries, {time.time() - t0:.1f} s")
    return out


def calibrate(dg, s, t, beta_ref, eps: float, L, seed: int, c_B_ladder, c_R_ladder, target: float = 0.97,
              uid=None, log=None):
    """Evaluate every (c_B, c_R) of the ladders; return (best, table). best is the
    candidate with the fewest walk steps whose fraction within eps is >= target
    (None if none is)."""
    beta_ref = np.asarray(beta_ref, dtype=np.float64)
    c_B_ladder = sorted(c_B_ladder)
    table = []
    for c_R in c_R_ladder:
        t0 = time.time()
        runs = probe_values(dg, s, t, eps, L, seed, c_B_ladder[-1], c_R, uid, log)
        G = int(runs[0][1]["G"])
        for c_B in c_B_ladder:
            b = max(_ceil(c_B / (eps * eps)), 1)
            est = np.array([median_of_means(q, b, G) for q, _ in runs])
            err = np.abs(est - beta_ref) / beta_ref
            R = np.array([int(r["R"]) for _, r in runs])
            Ls = np.array([int(r["L"]) for _, r in runs])
            steps = float(np.sum(2.0 * b * G * R * Ls))
            table.append({"c_B": c_B, "c_R": c_R, "B": b, "R_median": float(np.median(R)),
                          "R_max": int(R.max()), "within": float(np.mean(err <= eps)),
                          "median_rel_err": float(np.median(err)), "walk_steps": steps})
        if log is not None:
            log(f"  c_R = {c_R:.4g}: {time.time() - t0:.1f} s; " +
                ", ".join(f"B={r['B']}: {r['within']:.3f}" for r in table[-len(c_B_ladder):]))
    ok = [r for r in table if r["within"] >= target]
    best = min(ok, key=lambda r: r["walk_steps"]) if ok else None
    return best, table


def load_reference(path: str) -> dict:
    """The columns of a reference file by name: its "# index s t ..." comment
    line names the whitespace-separated columns of the data rows."""
    with open(path) as f:
        names = [ln for ln in f if ln.startswith("# index")][0][1:].split()
    data = np.loadtxt(path, comments="#", ndmin=2)
    if data.shape[1] != len(names):
        raise ValueError(f"{path}: {len(names)} column names for {data.shape[1]} columns")
    return {name: data[:, i] for i, name in enumerate(names)}


def select_pairs(ref: dict, only_L: int = 0, offset: int = 0, pairs: int = 0) -> np.ndarray:
    """Rows of a reference file to use: those whose L column equals only_L
    (all when 0), skipping the first `offset` of them, then the first `pairs`
    (all when 0)."""
    sel = np.ones(ref["index"].size, dtype=bool)
    if only_L:
        sel &= ref["L"] == only_L
    idx = np.flatnonzero(sel)[offset:]
    return idx[:pairs] if pairs else idx


def main(argv=None):
    from synth import graphs  # seeded workload inputs

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("workload")
    ap.add_argument("--ref", required=True, help="reference file: index s t d_s d_t [L] beta ...")
    ap.add_argument("--eps", type=float, default=0.05)
    ap.add_argument("--L", type=int, default=0, help="run every pair at this L (0: the file's L column)")
    ap.add_argument("--pairs", type=int, default=0, help="use the first this many pairs (0: all)")
    ap.add_argument("--offset", type=int, default=0, help="skip this many of the selected pairs first")
    ap.add_argument("--only-L", type=int, default=0, help="use only the pairs whose L column equals this")
    ap.add_argument("--c-B", type=float, nargs="+", required=True)
    ap.add_argument("--c-R", type=float, nargs="+", required=True)
    ap.add_argument("--target", type=float, default=0.97)
    ap.add_argument("--seed", type=lambda x: int(x, 0), default=graphs.CALIBRATION_SEED)
    ap.add_argument("--layout", type=int, default=B.BD_LAYOUT_AUTO)
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)

    def log(*x):
        print(*x, flush=True)

    ref = load_reference(a.ref)
    idx = select_pairs(ref, a.only_L, a.offset, a.pairs)
    s = ref["s"][idx].astype(np.int32)
    t = ref["t"][idx].astype(np.int32)
    beta = ref["beta_cg"][idx]
    L = np.full(idx.size, a.L, dtype=np.int32) if a.L or "L" not in ref else ref["L"][idx].astype(np.int32)
    uid = ref["index"][idx].astype(np.int64)
    t0 = time.time()
    g = graphs.workload_graph(a.workload)
    dg = B.graph_load_csr(g.n, g.row_ptr, g.col, a.layout)
    log(f"{a.workload}: {idx.size} pairs, eps={a.eps}, L {sorted(set(L.tolist()))}, seed {a.seed:#x} "
        f"(graph {time.time() - t0:.1f} s); first pairs (s, t, beta): "
        f"{[(int(x), int(y), float(z)) for x, y, z in zip(s[:3], t[:3], beta[:3])]}")
    best, table = calibrate(dg, s, t, beta, a.eps, L, a.seed, a.c_B, a.c_R, a.target, uid=uid, log=log)
    log(json.dumps({"best": best}))
    if a.json:
        with open(a.json, "w") as f:
            json.dump({"workload": a.workload, "eps": a.eps, "seed": a.seed, "pairs": int(idx.size),
                       "L": sorted(set(L.tolist())), "target": a.target, "best": best, "table": table}, f, indent=1)
    dg.free()
    return 0 if best is not None else 1


if __name__ == "__main__":
    sys.exit(main())
