"""The allocation-free median entry point against the allocating one, through
the C ABI: two calls in a row (the second on fewer values, so the library's
fixed scratch array holds the first call's state when the second starts), and
its size and argument checks."""
import numpy as np
import pytest
import torch

import oracle as o
import paper_2607_24518_amd as sym

pytestmark = pytest.mark.gpu

from gpu_util import ctx, dev, to_dev  # noqa: E402


def test_median_noalloc_equals_allocating_entry_point_on_two_calls():
    c = ctx()
    rng = np.random.default_rng(11)
    out = torch.full((2,), -1.0, dtype=torch.float64, device=dev())
    for m in (1_000_003, 4097, 1, 2):
        g = rng.normal(size=m).astype(np.float32)
        g[: m // 3] = 0.0                       # ties and zeros
        gd = to_dev(g)
        sym.symnmf_median_sq_noalloc(c, gd, out)
        torch.cuda.synchronize()
        got = out[0].item()
        ref = sym.symnmf_median_sq(c, gd)
        assert np.float32(got) == np.float32(ref) and got == float(np.float32(got)), m
        # and both are the lower median of the squares (same float32 squaring)
        g2 = (g * g).astype(np.float32).astype(np.float64)
        assert got == o.lower_median(g2), m
    assert out[1].item() == -1.0                # only out_dev[0] is written


def test_median_noalloc_on_the_stream_of_the_context_then_allocating_calls():
    c = ctx()
    g = to_dev(np.linspace(-3.0, 3.0, 10001).astype(np.float32))
    out = torch.empty(1, dtype=torch.float64, device=dev())
    sym.symnmf_median_sq_noalloc(c, g, out)
    sym.symnmf_median_sq_noalloc(c, g[:11], out)     # a smaller call right after, same stream
    torch.cuda.synchronize()
    assert np.float32(out.item()) == np.float32(sym.symnmf_median_sq(c, g[:11]))


def test_median_noalloc_rejects_bad_sizes():
    c = ctx()
    g = torch.zeros(16, device=dev())
    out = torch.empty(1, dtype=torch.float64, device=dev())
    for m in (0, -5, 2 ** 32):                       # refused on the host, before any kernel
        with pytest.raises(sym.SymnmfError) as e:
            sym.symnmf_median_sq_noalloc(c, g, out, m=m)
        assert e.value.code == sym.EINVAL
