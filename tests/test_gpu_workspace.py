"""Device scratch of the C ABI's calls: with a caller-owned workspace attached
(symnmf_set_workspace) the calls allocate nothing, succeed with exactly the
size the *_workspace queries report, fail with ENOMEM below it, and give the
same results as with the library's own pool; without one, the pool stops
allocating once it holds what the calls need."""
import numpy as np
import pytest
import torch

import oracle as o
import paper_2607_24518_amd as sym
import synth

pytestmark = pytest.mark.gpu

from gpu_util import dev, from_dev, to_dev  # noqa: E402


@pytest.fixture()
def fresh_ctx():
    c = sym.symnmf_create(0)
    yield c
    sym.symnmf_destroy(c)


def _calls(c, X, k):
    """Every pooled call once; returns their results."""
    S = sym.symnmf_build_S(c, X, dtype=sym.S_BF16)
    n = X.shape[1]
    H = to_dev(o.init_H(0.1, n, k, 3))
    f, _ = sym.symnmf_objective(c, S, H, k)
    g = to_dev(np.random.default_rng(2).normal(size=5001))
    med = sym.symnmf_median_sq(c, g)
    Y = torch.empty(n, 64, device=dev())
    sym.symnmf_sketch(c, S, 7, 64, Y)
    H0 = torch.empty(n, k, device=dev())
    sym.symnmf_warm_start(c, S, None, 64, k, 7, H0)
    se = sym.symnmf_subspace_error(c, H, H0)
    return S, f, med, from_dev(Y), from_dev(H0), se


def test_attached_workspace_of_the_queried_size(fresh_ctx):
    c = fresh_ctx
    X = to_dev(synth.c1_instance(1, T=500, n=700, groups=5).X.numpy())
    n, k = 700, 16
    ref = _calls(c, X, k)                                      # library pool
    S = ref[0]
    need = max(sym.symnmf_build_S_workspace(n, 500, dtype=sym.S_BF16), sym.symnmf_objective_workspace(c, S, k),
               sym.symnmf_median_workspace(), sym.symnmf_sketch_workspace(c, S, 64),
               sym.symnmf_warm_start_workspace(c, S, 64, k), sym.symnmf_subspace_error_workspace(n, k))
    assert need > 0
    ws = torch.empty(need, dtype=torch.uint8, device=dev())
    sym.symnmf_set_workspace(c, ws)
    held, allocs0 = sym.symnmf_workspace_info(c)
    assert held == need
    got = _calls(c, X, k)
    assert sym.symnmf_workspace_info(c) == (need, allocs0)    # nothing allocated
    assert torch.equal(got[0].buf, ref[0].buf)
    assert got[1] == ref[1] and got[2] == ref[2] and got[5] == ref[5]
    assert np.array_equal(got[3], ref[3]) and np.array_equal(got[4], ref[4])
    sym.symnmf_set_workspace(c, None)


@pytest.mark.parametrize("which", ["build", "objective", "median", "warm_start"])
def test_each_query_is_exact(fresh_ctx, which):
    c = fresh_ctx
    X = to_dev(synth.c1_instance(1, T=500, n=700, groups=5).X.numpy())
    n, k = 700, 16
    S = sym.symnmf_build_S(c, X, dtype=sym.S_FP32)
    H = to_dev(o.init_H(0.1, n, k, 3))
    g = to_dev(np.random.default_rng(2).normal(size=5001))
    call = {"build": (sym.symnmf_build_S_workspace(n, 500, dtype=sym.S_FP8),
                      lambda: sym.symnmf_build_S(c, X, dtype=sym.S_FP8)),
            "objective": (sym.symnmf_objective_workspace(c, S, k), lambda: sym.symnmf_objective(c, S, H, k)),
            "median": (sym.symnmf_median_workspace(), lambda: sym.symnmf_median_sq(c, g)),
            "warm_start": (sym.symnmf_warm_start_workspace(c, S, 64, k),
                           lambda: sym.symnmf_warm_start(c, S, None, 64, k, 7, torch.empty(n, k, device=dev())))}
    need, fn = call[which]
    small = torch.empty(need - 256, dtype=torch.uint8, device=dev())
    sym.symnmf_set_workspace(c, small)
    with pytest.raises(sym.SymnmfError) as e:
        fn()
    assert e.value.code == sym.ENOMEM and "workspace is too small" in str(e.value)
    exact = torch.empty(need, dtype=torch.uint8, device=dev())
    sym.symnmf_set_workspace(c, exact)
    fn()
    sym.symnmf_set_workspace(c, None)


def test_library_pool_stops_allocating(fresh_ctx):
    c = fresh_ctx
    X = to_dev(synth.c1_instance(1, T=500, n=700, groups=5).X.numpy())
    _calls(c, X, 16)
    held, allocs = sym.symnmf_workspace_info(c)
    assert held > 0 and allocs >= 1
    for _ in range(3):
        _calls(c, X, 16)
    assert sym.symnmf_workspace_info(c) == (held, allocs)
