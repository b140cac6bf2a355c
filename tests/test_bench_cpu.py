"""Host logic of bench.py and studies.py (CPU): the algorithmic byte counts
behind the roofline figures, the parsing of time-to-tolerance variants
(storage, precision ladder, method), the committed reference lookup, and the
refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import paper_2607_24518_amd as sym  # noqa: E402
import studies  # noqa: E402


def test_algorithmic_bytes():
    # S once (n^2 entries of 4 / 2 / 1 bytes), H read once, S.H written once
    assert bench.stream_bytes(100000, 100000, 32, 4) == 40025600000
    assert bench.stream_bytes(100000, 100000, 32, 2) == 20025600000
    assert bench.stream_bytes(12500, 1000000, 64, 2) == 12500 * 1000000 * 2 + 1000000 * 64 * 4 + 12500 * 64 * 4
    # the update reads H_t, S.H, G and writes H_{t+1}, G: five n x k FP32 arrays
    assert bench.step_bytes(100000, 100000, 32, 4) - bench.stream_bytes(100000, 100000, 32, 4) == 5 * 100000 * 32 * 4


@pytest.mark.parametrize("variant,method,eta_scale", [
    ("fp32", sym.ADAGRAD, 1.0), ("fp8>bf16-piecewise", sym.PIECEWISE_ADAGRAD, 1.0),
    ("fp8>fp32-blocksvrg", sym.BLOCK_SVRG, 1.0), ("bf16-adam", sym.ADAM, 0.1), ("fp32-admm1000", sym.ADMM, 1.0),
    ("fp32-blocksvrg-eta0.5", sym.BLOCK_SVRG, 0.5), ("bf16-adam-eta3", sym.ADAM, 0.3)])
def test_variant_parsing(variant, method, eta_scale):
    p = studies.variant_params(variant, 0.05)
    assert p.method == method and p.eta == pytest.approx(0.05 * eta_scale)
    ladder = variant.split("-")[0].split(">")
    assert all(dt in sym.DTYPES for dt in ladder)
    if method == sym.ADMM:
        assert p.rho == 1000.0
    if method == sym.BLOCK_SVRG:
        assert p.block_rows == 1024 and p.phi0 == 0.75 and p.snapshot_s == 10


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_ttt_scan_finds_the_first_iterate_within_tolerance():
    """The scan behind every time-to-tolerance figure: a coarse pass every 32
    kept iterates, then bisection inside the first bracket that reaches the
    tolerance; on a decreasing sequence it returns exactly the first kept
    iterate with (f - f_ref)/f_ref <= tol, with its iteration count and time."""
    import numpy as np
    f_ref, every = 100.0, 2
    for first in (0, 5, 31, 32, 33, 700, 999):
        rel = np.where(np.arange(1000) < first, 1e-3 * (1000 - np.arange(1000)), 5e-5)
        f = f_ref * (1.0 + rel)
        times = [0.01 * (j + 1) for j in range(1000)]
        calls = []

        def objective_of(j):
            calls.append(j)
            return f[j]

        e = studies.ttt_scan(objective_of, list(range(1000)), 1000, f_ref, 1e-4, every, times)
        assert e["iters"] == (first + 1) * every and e["seconds"] == times[first]
        assert e["final_rel"] == pytest.approx(5e-5) and len(set(calls)) < 60
    # never within the tolerance: no time
    e = studies.ttt_scan(lambda j: 200.0, list(range(64)), 64, f_ref, 1e-4, every, [0.0] * 64)
    assert "iters" not in e and "seconds" not in e and e["final_rel"] == pytest.approx(1.0)


def test_committed_reference_lookup():
    # only a complete reference of exactly this workload is used
    assert studies.committed_reference(0, 100000, 2500, 32, 32, 1) is None
    d = studies.committed_reference(0, 100000, 2500, 32, 32, 0)
    assert d is not None, "the oracle reference of the n = 1e5 workload is committed"
    assert d["complete"] and d["f_ref"] > 0 and d["iterations"] >= 100
    # the reference is the lowest objective of the run, which decreases
    fs = [e["f"] for e in d["trace"]]
    assert d["f_ref"] <= min(fs) and all(b <= a * (1 + 1e-12) for a, b in zip(fs, fs[1:]))
    assert d["t_best"] == d["iterations"] - 1
