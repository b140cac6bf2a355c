"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/symnmf.h declares, and its host-only entry points agree
with the oracle and the header."""
import os
import re

import numpy as np
import pytest

import oracle as o

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "symnmf.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(symnmf_[A-Za-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def binding():
    import paper_2607_24518_amd as b
    if not os.path.exists(b.LIB_PATH):
        pytest.skip("libsymnmf.so not built (run __graft_entry__.build())")
    b.lib()
    return b


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ["symnmf_build_S", "symnmf_init_H", "symnmf_step", "symnmf_objective",
                     "symnmf_solve_to_tol", "symnmf_create", "symnmf_state_create"]:
        assert required in names


def test_library_exports_every_declared_symbol(binding):
    import ctypes
    L = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in _declared_functions() if not hasattr(L, n)]
    assert missing == []
    # and the binding wraps each of them under the same name
    assert set(_declared_functions()) <= set(binding.SIGNATURES)
    for n in _declared_functions():
        assert callable(getattr(binding, n))


def test_struct_sizes_match_header_layout(binding):
    import ctypes
    assert ctypes.sizeof(binding.symnmf_sbuild_params) == 64
    assert ctypes.sizeof(binding.symnmf_S) == 8 * 3 + 8 * 6 + 4 * 2 + 8 * 4
    assert ctypes.sizeof(binding.symnmf_stats) == 8 * 7 + 4 * 4
    assert ctypes.sizeof(binding.symnmf_params) == 8 + 8 * 10 + 8 * 3 + 8 + 8 * 3 + 8 * 4 + 8 + 8 + 8 * 3
    assert ctypes.sizeof(binding.symnmf_control) == 8 * 4 + 4 * 2 + 8 * 2
    assert binding.symnmf_abi_version() == 4


def test_kmeans_seed_rows_are_bit_identical_to_the_oracle(binding):
    import oracle.kmeans_oracle as km
    for seed, n, K in [(0, 1000, 2), (5, 512, 8), (2**64 - 3, 100000, 316), (9, 64, 64), (1, 1, 1)]:
        assert binding.symnmf_kmeans_seed_rows(seed, n, K) == km.seed_rows(seed, n, K).tolist()
    with pytest.raises(binding.SymnmfError):
        binding.symnmf_kmeans_seed_rows(0, 5, 6)
    assert ctypes_sizeof(binding.symnmf_kmeans_stats) == 8 * 5 + 4 * 2


def ctypes_sizeof(t):
    import ctypes
    return ctypes.sizeof(t)


def test_params_default(binding):
    p = binding.symnmf_params_default()
    assert p.method == binding.ADAGRAD and p.delta == 10 and p.warmup == 50
    assert p.tau_E == 0.1 and p.tau_g_inf == 1e-4 and p.n_ref == 1e4 and p.tau_stag == 1e-5
    assert p.rho == 500.0
    assert (p.beta1, p.beta2, p.beta3) == (0.9, 0.999, 0.99)


def test_S_bytes(binding):
    assert binding.symnmf_S_bytes(512, 512, binding.S_FP32) == 512 * 512 * 4
    assert binding.symnmf_S_bytes(100000, 100000, binding.S_FP32, 256) == 100096 * 100096 * 4
    assert binding.symnmf_S_bytes(100000, 100000, binding.S_BF16, 256) == 100096 * 100096 * 2
    fp8 = binding.symnmf_S_bytes(1000, 1000, binding.S_FP8, 256)
    assert fp8 >= 1024 * 1024 + 4 * 4 + 1024 * 4
    assert binding.symnmf_S_bytes(0, 10, binding.S_FP32) == -1


def test_block_sampler_is_bit_identical_to_the_oracle(binding):
    for seed, t, stream, nb, m in [(0, 0, 0, 98, 74), (7, 13, 1, 98, 74), (2**63 + 5, 99, 0, 391, 200),
                                   (3, 1, 1, 5, 5), (11, 2, 0, 20, 1)]:
        ours = binding.symnmf_sample_blocks(seed, t, stream, nb, m)
        ref = o.sample_blocks(seed, t, stream, nb, m).tolist()
        assert ours == ref


def test_tiled_storage_offsets_match_the_documented_layout(binding):
    """symnmf_S_offset against an independent decoder of the tiled format."""
    import torch
    from gpu_util import untile
    rows_pad, ld = 512, 768
    for dtype, E in [(binding.S_FP32, 4), (binding.S_BF16, 8), (binding.S_FP8, 16)]:
        flat = torch.arange(rows_pad * ld, dtype=torch.float64)
        M = untile(flat, rows_pad, ld, E).numpy()      # M[r, c] = offset of (r, c)
        rng = np.random.default_rng(E)
        for r, c in zip(rng.integers(0, rows_pad, 300), rng.integers(0, ld, 300)):
            assert binding.symnmf_S_offset(int(r), int(c), rows_pad, ld, dtype) == int(M[r, c])
        assert sorted(M.ravel().astype(np.int64).tolist()) == list(range(rows_pad * ld))
    assert binding.symnmf_S_offset(3, 5, 512, 768, binding.S_FP64) == 3 * 768 + 5
    assert binding.symnmf_S_offset(512, 0, 512, 768, binding.S_FP32) == -1


@pytest.mark.parametrize("tiles,chunks,P", [(1, 1, 256), (2, 3, 256), (3, 3, 256), (391, 391, 256),
                                            (392, 391, 256), (49, 3907, 256), (49, 3907, 250), (50, 3907, 250),
                                            (7, 5, 512)])
def test_partial_slots_are_one_to_one(tiles, chunks, P):
    """Host check of the stream-K partial indexing: work-group w owns units
    [w U / Pe, (w+1) U / Pe); each maximal run of one tile (pair of tiles for
    the 8-wave kernel) writes slot w + a (2 (w + q) + h); the slots are
    distinct, fit the allocated buffer, and the update kernel's owner range of
    each tile is exactly its set of writers."""
    def owner(u, U, Pe):
        return ((u + 1) * Pe - 1) // U

    for tall in (False, True):
        na = (tiles + 1) // 2 if tall else tiles
        U = na * chunks
        Pe = min(U, P)
        slots, writers = {}, {}
        for w in range(Pe):
            lo, hi = w * U // Pe, (w + 1) * U // Pe
            assert hi > lo
            for a in range(lo // chunks, (hi - 1) // chunks + 1):
                halves = [(2 * a + h, 2 * (w + a) + h) for h in (0, 1) if 2 * a + h < tiles] if tall else [(a, w + a)]
                for tile, slot in halves:
                    assert slot not in slots
                    slots[slot] = tile
                    writers.setdefault(tile, set()).add(w)
        cap = 2 * (P + na) if tall else P + tiles
        assert max(slots) < cap
        for tile in range(tiles):
            a = tile // 2 if tall else tile
            w_lo, w_hi = owner(a * chunks, U, Pe), owner((a + 1) * chunks - 1, U, Pe)
            assert writers[tile] == set(range(w_lo, w_hi + 1))
