"""The degree-run node table of the storage-id layout's default kernel, on the
host (paper_2512_05460_amd/csrc/pw_runs.hpp, compiled with g++): every node's
row offset and degree decode from the table to the row offsets', h1 is the
smallest run start past which each block holds at most two runs, and the
builder declines a table that does not fit. (The kernels decode the same
table from LDS; tests/test_gpu_storage_probe.py checks them on the GPU.)"""

import os
import shutil
import subprocess

import numpy as np
import pytest

from synth import graphs

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2512_05460_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("runs") / "run_table_check")
    subprocess.run(["g++", "-O2", "-std=c++17", f"-I{CSRC}", os.path.join(HERE, "native", "run_table_check.cpp"),
                    "-o", exe], check=True)

    def run(cases):
        lines = [" ".join(str(v) for v in (sh, ninv, cap, len(d), *d)) for sh, ninv, cap, d in cases]
        out = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True)
        return [ln.split() for ln in out.stdout.splitlines()]
    return run


def storage_degrees(g):
    return np.sort(np.diff(g.row_ptr))[::-1].astype(int).tolist()


CAP = 36865  # the 1,024-thread kernels' LDS words


def test_workload_graphs_decode(checker):
    cases = []
    for key in ("ba1k", "cl100k"):
        d = storage_degrees(graphs.workload_graph(key))
        cases += [(sh, max(d) + 1, CAP, d) for sh in (6, 7, 8, 9)]
    res = checker(cases)
    assert all(r[0] == "ok" for r in res), res
    assert res[4][1] == "1571"  # cl100k, blocks of 64: the h1 the kernels use


def test_edge_cases(checker):
    long_tail = [9, 7, 7, 5] + [3] * 300 + [2] * 200 + [1] * 3
    cases = [
        (6, 10, CAP, [4] * 1000),                    # one run: h1 = 0
        (6, 10, CAP, [5, 4, 3, 2, 1]),               # five runs in one block: the last two after h1 = 3
        (6, 10, CAP, [9] + [4] * 100 + [1]),         # short runs at both ends
        (6, 10, CAP, long_tail),                     # a short run between long ones
        (6, 3000, CAP, [2500] * 70 + [3] * 200),     # degrees above 2,047 stay direct
        (6, 10, 8, [4] * 1000),                      # too large for the capacity
        (6, 10, CAP, [7]),                           # a single node
    ]
    res = checker(cases)
    assert [r[0] for r in res] == ["ok", "ok", "ok", "ok", "ok", "nofit", "ok"], res
    assert res[0][1] == "0" and res[1][1] == "3"
    assert int(res[4][1]) >= 70  # the runs of degree 2,500 lie before h1


def test_random_degree_sequences(checker):
    rng = np.random.default_rng(5)
    cases = []
    for _ in range(40):
        n = int(rng.integers(1, 5000))
        d = np.sort(rng.zipf(1.8, size=n).clip(1, 3000))[::-1].tolist()
        cases.append((int(rng.integers(6, 10)), max(d) + 1, CAP, d))
    res = checker(cases)
    assert all(r[0] in ("ok", "nofit") for r in res), res
    assert sum(r[0] == "ok" for r in res) > 30
