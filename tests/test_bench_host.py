"""Host logic of bench.py that needs no GPU: the one-GPU guard, the
kernel-source hash that ties committed counter summaries to the sources, and
the summary reader."""

import importlib.util
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def _copy_sources(bench, dst):
    os.makedirs(os.path.join(dst, "paper_2512_05460_amd", "csrc"))
    for f in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_2512_05460_amd", "csrc", f),
                    os.path.join(dst, "paper_2512_05460_amd", "csrc", f))


def test_hash_ignores_comments_not_code(bench, tmp_path, monkeypatch):
    h0 = bench.kernel_source_hash()
    _copy_sources(bench, str(tmp_path))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() == h0
    k = tmp_path / "paper_2512_05460_amd" / "csrc" / "pw_kernels.hip"
    src = k.read_text()
    k.write_text("// a comment line\n/* a block\n   comment */\n\n" + src.replace("\n", "  // tail\n", 3))
    assert bench.kernel_source_hash() == h0
    k.write_text(src + "\nstatic int pw_unused_probe_of_the_hash;\n")
    assert bench.kernel_source_hash() != h0


def test_read_counters(bench, tmp_path):
    good = tmp_path / "good.txt"
    good.write_text("# header = ignored\nkernel_source_sha256_16 = %s\nx = 1.5   (a note)\n"
                    % bench.kernel_source_hash())
    kv, why = bench.read_counters(str(good))
    assert why == "" and kv["x"] == "1.5"
    stale = tmp_path / "stale.txt"
    stale.write_text("kernel_source_sha256_16 = 0000000000000000\nx = 1\n")
    assert bench.read_counters(str(stale))[0] is None
    assert bench.read_counters(str(tmp_path / "missing.txt"))[0] is None

