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
    ("fp8>fp32-blocksvrg", sym.BLOCK_SVRG, 1.0), ("bf16-adam", sym.ADAM, 0.1), ("fp32-admm1000", sym.ADMM, 1.0)])
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


def test_committed_reference_lookup():
    # only a complete reference of exactly this workload is used
    assert studies.committed_reference(0, 100000, 2500, 32, 32, 1) is None
    d = studies.committed_reference(0, 100000, 2500, 32, 32, 0)
    if d is not None:
        assert d["complete"] and d["f_ref"] > 0 and d["iterations"] >= 100
