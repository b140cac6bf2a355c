"""The TPDM at its full size: n = 100000 instruments, T = 20000 samples
(Student-t 2.5 factors with a near-dominant common factor, 32 groups, noise
0.3, generated on the device), lower tail, q = 5 % (1000 exceedances) - the
instance the TPDM time-to-tolerance runs use.

The oracle's rows come from oracle.tpdm_rows (the definition of section
"Empirical Estimation" taken a block of columns at a time: 16 GB of FP64
margins and an 80 GB matrix do not fit its host memory otherwise).  Checked
rows: two whole 256-row panels (rows 256-511 and the ragged last panel
99840-99999, so the FP8 panel scales can be derived by the oracle) and three
single rows.  Tolerances as for the n = 4096 TPDM: FP64 1e-12, FP32 3e-6
(FP32 products over the 1000 selected samples), BF16 half an ulp plus that,
FP8 one E4M3 step of S times the oracle's panel scale, the unit diagonal
exact."""
import time

import numpy as np
import pytest
import torch

import oracle as o
import paper_2607_24518_amd as sym
import synth

pytestmark = pytest.mark.gpu

from gpu_util import ctx, dev, stored_numpy, stored_rows  # noqa: E402

N, T, Q = 100000, 20000, 0.05
PANELS = (np.arange(256, 512), np.arange(99840, 100000))
SINGLES = np.array([12345, 50000, 77777])


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "bf16", "fp8"])
def test_row_reader_equals_the_whole_matrix_reader(dtype):
    """The row-wise decoder used below against the whole-matrix one, on a
    700-instrument TPDM (a ragged last tile, three 256-row panels)."""
    X = synth.tpdm_returns(1, T=4000, n=700, groups=5, nu=3.0).X
    S = sym.symnmf_build_S(ctx(), X.to(dev()), kind=sym.TPDM, dtype=sym.DTYPES[dtype], q=Q, lower_tail=1,
                           fp8_panel_rows=256)
    rows = np.array([0, 1, 255, 256, 300, 511, 512, 699])
    assert np.array_equal(stored_rows(S, rows), stored_numpy(S)[rows])


@pytest.fixture(scope="module")
def tpdm_big():
    t0 = time.time()
    X = synth.tpdm_returns(0, T=T, n=N, groups=32, nu=2.5, common=True, device=dev()).X
    Xh = X.cpu().numpy()
    print(f"[tpdm n=1e5] returns generated ({time.time() - t0:.1f} s); oracle rows ...", flush=True)
    rows = np.concatenate(PANELS + (SINGLES,))
    ref = o.tpdm_rows(Xh, Q, rows, lower_tail=True)
    del Xh
    print(f"[tpdm n=1e5] oracle rows done ({time.time() - t0:.1f} s)", flush=True)
    return X, rows, ref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype", ["fp64", "fp32", "bf16", "fp8"])
def test_tpdm_full_size_rows(tpdm_big, dtype):
    X, rows, ref = tpdm_big
    print(f"[tpdm n=1e5] build {dtype}", flush=True)
    S = sym.symnmf_build_S(ctx(), X, kind=sym.TPDM, dtype=sym.DTYPES[dtype], q=Q, lower_tail=1, fp8_panel_rows=256)
    M = stored_rows(S, rows)
    del S
    torch.cuda.empty_cache()
    if dtype == "fp64":
        assert np.max(np.abs(M - ref)) < 1e-12
    elif dtype == "fp32":
        assert np.max(np.abs(M - ref)) < 3e-6
    elif dtype == "bf16":
        ulp = 2.0 ** (np.floor(np.log2(np.maximum(np.abs(ref), 1e-30))) - 7)
        assert np.all(np.abs(M - ref) <= 0.5 * ulp + 3e-6)
    else:
        i = 0
        for panel in PANELS:
            Mp, Rp = M[i:i + panel.size], ref[i:i + panel.size]
            i += panel.size
            assert np.all(Mp[np.arange(panel.size), panel] == 1.0)
            scale = o.fp8_panel_scales(Rp, 256, row0=int(panel[0]))[0]
            off = np.ones(Mp.shape, dtype=bool)
            off[np.arange(panel.size), panel] = False
            bound = 2.0 ** -4 * np.abs(Rp) + 2.0 ** -9 / scale * 1.01 + 1e-7
            assert np.all((np.abs(Mp - Rp) <= bound)[off])
    # every checked row is a row of a unit-diagonal TPDM
    assert np.all(M[np.arange(rows.size), rows] == 1.0)
