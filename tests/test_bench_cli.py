"""Host-side checks of bench.py's command line (no GPU): the multi-GPU
refusal and the input dumps the native driver reads."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=600)


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "one MI355X" in r.stderr and r.stdout == ""


def test_dump_inputs_matches_meta(tmp_path):
    r = run_bench("--dump-inputs", str(tmp_path), "--n", "5000")
    assert r.returncode == 0, r.stderr
    N, d, m, eps, lam, seed = open(tmp_path / "meta.txt").read().split()
    N, d = int(N), int(d)
    assert N == 5000 and int(m) == 256 and float(eps) > 0 and float(lam) < 0 and int(seed) >= 0
    X = np.fromfile(tmp_path / "X.bin", dtype=np.float32)
    F = np.fromfile(tmp_path / "F.bin", dtype=np.float32)
    assert X.size == 3 * N and F.size == d * N
    assert np.isfinite(X).all() and np.isfinite(F).all()


def test_dump_batch_matches_meta(tmp_path):
    r = run_bench("--dump-batch", str(tmp_path))
    assert r.returncode == 0, r.stderr
    lines = open(tmp_path / "meta_batch.txt").read().splitlines()
    count, d, m, eps, lam = lines[0].split()
    count, d = int(count), int(d)
    rows = [tuple(int(v) for v in ln.split()) for ln in lines[1:]]
    assert count == 512 == len(rows) and d == 3 and int(m) == 128
    Ns = np.array([n for n, _ in rows])
    assert Ns.min() >= 1000 and Ns.max() <= 65536
    assert len({s for _, s in rows}) == count  # every cloud has its own seed
    total = int(Ns.sum())
    assert os.path.getsize(tmp_path / "Xb.bin") == 4 * 3 * total
    assert os.path.getsize(tmp_path / "Fb.bin") == 4 * d * total
