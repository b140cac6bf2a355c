"""Python binding of libsymnmf (the MI355X SymNMF hot path).

Argument marshalling only: every function below calls the C ABI declared in
``include/symnmf.h`` with the same name; all arithmetic runs in the library's
HIP kernels.  torch provides device memory (tensors' ``data_ptr``) and the
HIP stream.  If the shared library is missing the calls raise - there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsymnmf.so")

# enums (include/symnmf.h)
OK, EINVAL, ENOMEM, EDEVICE, ENUMERIC, ENOTCONV, EUNSUPPORTED = range(7)
S_FP32, S_BF16, S_FP8, S_FP64 = range(4)
ABS_CORR, TPDM = range(2)
ADAGRAD, RMSPROP, PIECEWISE_ADAGRAD, ROW_SVRG, BLOCK_SVRG, ADMM, ADAM, NADAM, ADAN, MU = range(10)
DTYPES = {"fp32": S_FP32, "bf16": S_BF16, "fp8": S_FP8, "fp64": S_FP64}

c_i32, c_i64, c_u64, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p


class symnmf_sbuild_params(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("dtype", c_i32), ("n", c_i64), ("T", c_i64), ("row0", c_i64),
                ("rows", c_i64), ("q", c_dbl), ("lower_tail", c_i32), ("raw_marginals", c_i32),
                ("fp8_panel_rows", c_i64)]


class symnmf_S(ctypes.Structure):
    _fields_ = [("data", c_vp), ("panel_scale", c_vp), ("diag", c_vp), ("n", c_i64), ("row0", c_i64),
                ("rows", c_i64), ("ld", c_i64), ("rows_pad", c_i64), ("fp8_panel_rows", c_i64),
                ("dtype", c_i32), ("kind", c_i32), ("fro2", c_dbl), ("fro2_stored", c_dbl),
                ("sum", c_dbl), ("mean", c_dbl)]


class symnmf_params(ctypes.Structure):
    _fields_ = [("method", c_i32), ("softplus", c_i32), ("eta", c_dbl), ("eps", c_dbl), ("alpha", c_dbl),
                ("mu", c_dbl), ("c", c_dbl), ("c_r", c_dbl), ("eps_med", c_dbl), ("row_frac", c_dbl),
                ("phi0", c_dbl), ("c_grow", c_dbl), ("grow_checks", c_i64), ("snapshot_s", c_i64),
                ("block_rows", c_i64), ("independent_blocks", c_i32), ("reserved0", c_i32),
                ("delta", c_i64), ("warmup", c_i64), ("max_iter", c_i64), ("tau_E", c_dbl),
                ("tau_g_inf", c_dbl), ("n_ref", c_dbl), ("tau_stag", c_dbl), ("seed", c_u64), ("rho", c_dbl),
                ("beta1", c_dbl), ("beta2", c_dbl), ("beta3", c_dbl)]


class symnmf_stats(ctypes.Structure):
    _fields_ = [("t", c_i64), ("f", c_dbl), ("E", c_dbl), ("kkt", c_dbl), ("stag", c_dbl), ("phi", c_dbl),
                ("wall_ms", c_dbl), ("full", c_i32), ("reset_fired", c_i32), ("converged", c_i32),
                ("nonfinite", c_i32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class symnmf_control(ctypes.Structure):
    _fields_ = [("t", c_i64), ("phi", c_dbl), ("stag_run", c_i64), ("pw_resets", c_i64), ("pw_enabled", c_i32),
                ("pw_cooling", c_i32), ("pw_cool_target", c_dbl), ("pw_E_reset", c_dbl)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class symnmf_kmeans_stats(ctypes.Structure):
    _fields_ = [("iters", c_i64), ("J0", c_dbl), ("J", c_dbl), ("wall_ms", c_dbl), ("changed", c_i64),
                ("converged", c_i32), ("empty", c_i32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class symnmf_adamw(ctypes.Structure):
    _fields_ = [("lr", c_dbl), ("beta1", c_dbl), ("beta2", c_dbl), ("eps", c_dbl), ("weight_decay", c_dbl)]


class SymnmfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"symnmf error {code}: {msg}")
        self.code = code


_lib = None

# exported symbols and their signatures (restype, argtypes)
SIGNATURES = {
    "symnmf_abi_version": (c_i32, []),
    "symnmf_params_default": (None, [ctypes.POINTER(symnmf_params)]),
    "symnmf_create": (c_i32, [ctypes.POINTER(c_vp), c_i32, c_vp]),
    "symnmf_destroy": (None, [c_vp]),
    "symnmf_last_error": (ctypes.c_char_p, [c_vp]),
    "symnmf_S_bytes": (c_i64, [c_i64, c_i64, c_i32, c_i64]),
    "symnmf_S_offset": (c_i64, [c_i64, c_i64, c_i64, c_i64, c_i32]),
    "symnmf_build_S": (c_i32, [c_vp, c_vp, ctypes.POINTER(symnmf_sbuild_params), c_vp, c_i64,
                               ctypes.POINTER(symnmf_S)]),
    "symnmf_S_load": (c_i32, [c_vp, c_vp, c_i32, c_i64, c_i64, c_i64, c_i32, c_i64, c_vp, c_i64,
                              ctypes.POINTER(symnmf_S)]),
    "symnmf_init_H": (c_i32, [c_vp, ctypes.POINTER(symnmf_S), c_i64, c_u64, c_vp]),
    "symnmf_set_workspace": (c_i32, [c_vp, c_vp, c_i64]),
    "symnmf_workspace_info": (c_i32, [c_vp, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]),
    "symnmf_build_S_workspace": (c_i64, [ctypes.POINTER(symnmf_sbuild_params)]),
    "symnmf_objective_workspace": (c_i64, [c_vp, ctypes.POINTER(symnmf_S), c_i64, c_i32]),
    "symnmf_median_workspace": (c_i64, []),
    "symnmf_sketch_workspace": (c_i64, [c_vp, ctypes.POINTER(symnmf_S), c_i64]),
    "symnmf_canonical_workspace": (c_i64, [c_i64, c_i64, c_i64]),
    "symnmf_warm_start_workspace": (c_i64, [c_vp, ctypes.POINTER(symnmf_S), c_i64, c_i64]),
    "symnmf_subspace_error_workspace": (c_i64, [c_i64, c_i64]),
    "symnmf_mlp_reserve": (c_i32, [c_vp, c_vp, c_i64, c_i32]),
    "symnmf_mlp_set_output": (c_i32, [c_vp, c_vp, c_i32]),
    "symnmf_state_create": (c_i32, [c_vp, ctypes.POINTER(symnmf_S), c_i64, ctypes.POINTER(symnmf_params), c_vp,
                                    c_i32, ctypes.POINTER(c_vp)]),
    "symnmf_state_destroy": (None, [c_vp]),
    "symnmf_step": (c_i32, [c_vp, ctypes.POINTER(symnmf_S), c_vp, ctypes.POINTER(symnmf_stats)]),
    "symnmf_state_read": (c_i32, [c_vp, c_vp, c_i32, c_vp]),
    "symnmf_state_stats": (c_i32, [c_vp, c_vp, ctypes.POINTER(symnmf_stats)]),
    "symnmf_state_set_phi": (c_i32, [c_vp, c_dbl]),
    "symnmf_state_control": (c_i32, [c_vp, c_vp, ctypes.POINTER(symnmf_control)]),
    "symnmf_state_checks": (c_i32, [c_vp, c_vp, ctypes.POINTER(symnmf_stats), c_i64, ctypes.POINTER(c_i64)]),
    "symnmf_objective": (c_i32, [c_vp, ctypes.POINTER(symnmf_S), c_vp, c_i32, c_i64, ctypes.POINTER(c_dbl),
                                 ctypes.POINTER(c_dbl)]),
    "symnmf_solve_to_tol": (c_i32, [c_vp, ctypes.POINTER(symnmf_S), c_vp, c_dbl, c_dbl,
                                    ctypes.POINTER(symnmf_stats), c_vp]),
    "symnmf_solve_trace": (c_i32, [c_vp, ctypes.POINTER(symnmf_S), c_vp, c_i64, c_i64, c_vp, c_i64,
                                   ctypes.POINTER(c_dbl), ctypes.POINTER(c_i64)]),
    "symnmf_state_rebind": (c_i32, [c_vp, c_vp, ctypes.POINTER(symnmf_S)]),
    "symnmf_solve_trace_ladder": (c_i32, [c_vp, ctypes.POINTER(symnmf_S), ctypes.POINTER(symnmf_S), c_vp, c_i64,
                                          c_i64, c_vp, c_i64, ctypes.POINTER(c_dbl), c_dbl, ctypes.POINTER(c_i64),
                                          ctypes.POINTER(c_i64)]),
    "symnmf_subspace_error": (c_i32, [c_vp, c_vp, c_vp, c_i64, c_i64, ctypes.POINTER(c_dbl)]),
    "symnmf_median_sq": (c_i32, [c_vp, c_vp, c_i64, ctypes.POINTER(ctypes.c_float)]),
    "symnmf_median_sq_noalloc": (c_i32, [c_vp, c_vp, c_i64, c_vp]),
    "symnmf_piecewise_reset": (c_i32, [c_vp, c_vp, c_dbl, ctypes.POINTER(ctypes.c_float)]),
    "symnmf_sample_blocks": (None, [c_u64, c_i64, c_i32, c_i64, c_i64, ctypes.POINTER(c_i32)]),
    "symnmf_selfcheck_fp8": (c_i32, [c_vp]),
    "symnmf_profile": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_dbl), ctypes.POINTER(c_i64)]),
    "symnmf_probe_copy": (c_i32, [c_vp, c_vp, c_vp, c_i64]),
    "symnmf_probe_read": (c_i32, [c_vp, c_vp, c_vp, c_i64, c_i64]),
    "symnmf_mlp_param_count": (c_i64, [c_i64, c_i64, c_i64]),
    "symnmf_mlp_init": (c_i32, [c_vp, c_i64, c_i64, c_i64, c_u64, c_vp]),
    "symnmf_mlp_create": (c_i32, [c_vp, c_i64, c_i64, c_i64, c_vp, ctypes.POINTER(c_vp)]),
    "symnmf_mlp_destroy": (None, [c_vp]),
    "symnmf_mlp_read": (c_i32, [c_vp, c_vp, c_i32, c_vp]),
    "symnmf_mlp_write": (c_i32, [c_vp, c_vp, c_vp]),
    "symnmf_mlp_forward": (c_i32, [c_vp, c_vp, c_vp, c_i64, c_i32, c_vp]),
    "symnmf_mlp_train_step": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_i64, ctypes.POINTER(symnmf_adamw), c_i32,
                                      ctypes.POINTER(c_dbl)]),
    "symnmf_sketch": (c_i32, [c_vp, ctypes.POINTER(symnmf_S), c_u64, c_i64, c_vp]),
    "symnmf_canonical": (c_i32, [c_vp, c_vp, c_i64, c_i64, c_i64, c_vp, c_vp]),
    "symnmf_warm_start": (c_i32, [c_vp, ctypes.POINTER(symnmf_S), c_vp, c_i64, c_i64, c_u64, c_vp]),
    "symnmf_kmeans_seed_rows": (c_i32, [c_u64, c_i64, c_i64, ctypes.POINTER(c_i64)]),
    "symnmf_kmeans_seed_pp": (c_i32, [c_vp, ctypes.POINTER(symnmf_S), c_i64, c_u64, ctypes.POINTER(c_i64)]),
    "symnmf_row_norms": (c_i32, [c_vp, ctypes.POINTER(symnmf_S), c_vp]),
    "symnmf_kmeans_assign": (c_i32, [c_vp, ctypes.POINTER(symnmf_S), c_vp, c_i64, c_vp, c_vp,
                                     ctypes.POINTER(c_dbl)]),
    "symnmf_kmeans_centroids": (c_i32, [c_vp, ctypes.POINTER(symnmf_S), c_vp, c_i64, c_vp, c_vp]),
    "symnmf_kmeans": (c_i32, [c_vp, ctypes.POINTER(symnmf_S), c_i64, c_u64, c_vp, c_dbl, c_i64, c_vp, c_vp,
                              ctypes.POINTER(symnmf_kmeans_stats)]),
    "symnmf_spectral": (c_i32, [c_vp, ctypes.POINTER(symnmf_S), c_i64, c_dbl, ctypes.POINTER(c_dbl),
                                ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl), ctypes.POINTER(c_dbl),
                                ctypes.POINTER(c_dbl), ctypes.POINTER(c_i64), c_vp]),
    "symnmf_silhouette": (c_i32, [c_vp, ctypes.POINTER(symnmf_S), c_vp, c_i64, ctypes.POINTER(c_dbl)]),
}

PROFILE_KERNELS = ("stream", "update", "finalize", "plan", "image")


def lib():
    """The loaded shared library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2607_24518_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(ctx, code):
    if code != OK:
        msg = lib().symnmf_last_error(ctx)
        raise SymnmfError(code, msg.decode() if msg else "")


def _stream_handle(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Matrix:
    """A stored S: the descriptor plus the torch buffer that owns its memory."""

    def __init__(self, desc: symnmf_S, buf):
        self.desc = desc
        self.buf = buf

    @property
    def n(self):
        return self.desc.n

    def __getattr__(self, name):
        return getattr(self.desc, name)


def symnmf_abi_version():
    return lib().symnmf_abi_version()


def symnmf_params_default(**overrides) -> symnmf_params:
    p = symnmf_params()
    lib().symnmf_params_default(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def symnmf_create(device: int = 0, stream=None):
    ctx = c_vp()
    code = lib().symnmf_create(ctypes.byref(ctx), device, _stream_handle(stream))
    if code != OK:
        raise SymnmfError(code, "symnmf_create failed")
    return ctx


def symnmf_destroy(ctx):
    lib().symnmf_destroy(ctx)


def symnmf_last_error(ctx):
    return lib().symnmf_last_error(ctx).decode()


def symnmf_S_bytes(rows, n, dtype, fp8_panel_rows=256):
    return lib().symnmf_S_bytes(rows, n, dtype, fp8_panel_rows)


def symnmf_S_offset(r, c, rows_pad, ld, dtype):
    return lib().symnmf_S_offset(r, c, rows_pad, ld, dtype)


def _alloc_bytes(nbytes, device):
    import torch
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


def symnmf_build_S(ctx, X, kind=ABS_CORR, dtype=S_FP32, row0=0, rows=None, q=0.05, lower_tail=1,
                   fp8_panel_rows=256, raw_marginals=0) -> Matrix:
    """X: device float32 tensor T x n (contiguous)."""
    T, n = X.shape
    rows = n - row0 if rows is None else rows
    p = symnmf_sbuild_params(kind=kind, dtype=dtype, n=n, T=T, row0=row0, rows=rows, q=q,
                             lower_tail=lower_tail, raw_marginals=raw_marginals,
                             fp8_panel_rows=fp8_panel_rows)
    nbytes = symnmf_S_bytes(rows, n, dtype, fp8_panel_rows)
    if nbytes < 0:
        raise SymnmfError(EINVAL, "bad S shape")
    buf = _alloc_bytes(nbytes, X.device)
    desc = symnmf_S()
    _check(ctx, lib().symnmf_build_S(ctx, _ptr(X), ctypes.byref(p), _ptr(buf), nbytes, ctypes.byref(desc)))
    return Matrix(desc, buf)


def symnmf_S_load(ctx, S_dense, dtype=S_FP32, row0=0, fp8_panel_rows=256) -> Matrix:
    """S_dense: device float32/float64 tensor rows x n (a panel starting at global row row0)."""
    import torch
    rows, n = S_dense.shape
    nbytes = symnmf_S_bytes(rows, n, dtype, fp8_panel_rows)
    buf = _alloc_bytes(nbytes, S_dense.device)
    desc = symnmf_S()
    f64 = 1 if S_dense.dtype == torch.float64 else 0
    _check(ctx, lib().symnmf_S_load(ctx, _ptr(S_dense), f64, n, row0, rows, dtype, fp8_panel_rows, _ptr(buf),
                                    nbytes, ctypes.byref(desc)))
    return Matrix(desc, buf)


def symnmf_set_workspace(ctx, buf=None, nbytes=None):
    """buf: a device tensor whose memory the context's scratch pool uses (kept alive by the caller), or None to
    detach and let the library allocate its own pool."""
    if buf is None:
        _check(ctx, lib().symnmf_set_workspace(ctx, None, 0))
    else:
        nb = buf.numel() * buf.element_size() if nbytes is None else nbytes
        _check(ctx, lib().symnmf_set_workspace(ctx, _ptr(buf), nb))


def symnmf_workspace_info(ctx):
    """(bytes held by the scratch pool, blocks it has taken from hipMalloc)."""
    held, allocs = c_i64(), c_i64()
    _check(ctx, lib().symnmf_workspace_info(ctx, ctypes.byref(held), ctypes.byref(allocs)))
    return held.value, allocs.value


def symnmf_build_S_workspace(n, T, kind=ABS_CORR, dtype=S_FP32, row0=0, rows=None, q=0.05, lower_tail=1,
                             fp8_panel_rows=256, raw_marginals=0):
    rows = n - row0 if rows is None else rows
    p = symnmf_sbuild_params(kind=kind, dtype=dtype, n=n, T=T, row0=row0, rows=rows, q=q, lower_tail=lower_tail,
                             raw_marginals=raw_marginals, fp8_panel_rows=fp8_panel_rows)
    return lib().symnmf_build_S_workspace(ctypes.byref(p))


def symnmf_objective_workspace(ctx, S: Matrix, k: int, h_is_f64: int = 0):
    return lib().symnmf_objective_workspace(ctx, ctypes.byref(S.desc), k, h_is_f64)


def symnmf_median_workspace():
    return lib().symnmf_median_workspace()


def symnmf_sketch_workspace(ctx, S: Matrix, width: int):
    return lib().symnmf_sketch_workspace(ctx, ctypes.byref(S.desc), width)


def symnmf_canonical_workspace(n: int, width: int, k: int):
    return lib().symnmf_canonical_workspace(n, width, k)


def symnmf_warm_start_workspace(ctx, S: Matrix, width: int, k: int):
    return lib().symnmf_warm_start_workspace(ctx, ctypes.byref(S.desc), width, k)


def symnmf_subspace_error_workspace(n: int, k: int):
    return lib().symnmf_subspace_error_workspace(n, k)


def symnmf_init_H(ctx, S: Matrix, k: int, seed: int, H):
    _check(ctx, lib().symnmf_init_H(ctx, ctypes.byref(S.desc), k, seed, _ptr(H)))
    return H


class State:
    def __init__(self, ctx, handle, S, k, params):
        self.ctx, self.handle, self.S, self.k, self.params = ctx, handle, S, k, params

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.symnmf_state_destroy(self.handle)
            self.handle = None


def symnmf_state_create(ctx, S: Matrix, k: int, params: symnmf_params, H0) -> State:
    import torch
    h = c_vp()
    f64 = 1 if H0.dtype == torch.float64 else 0
    _check(ctx, lib().symnmf_state_create(ctx, ctypes.byref(S.desc), k, ctypes.byref(params), _ptr(H0), f64,
                                          ctypes.byref(h)))
    return State(ctx, h, S, k, params)


def symnmf_state_destroy(st: State):
    if st.handle is not None:
        lib().symnmf_state_destroy(st.handle)
        st.handle = None


def symnmf_step(ctx, S: Matrix, st: State, want_stats: bool = True):
    out = symnmf_stats() if want_stats else None
    _check(ctx, lib().symnmf_step(ctx, ctypes.byref(S.desc), st.handle, ctypes.byref(out) if out else None))
    return out


def symnmf_state_read(ctx, st: State, which: int, dst):
    _check(ctx, lib().symnmf_state_read(ctx, st.handle, which, _ptr(dst)))
    return dst


def symnmf_state_stats(ctx, st: State):
    out = symnmf_stats()
    _check(ctx, lib().symnmf_state_stats(ctx, st.handle, ctypes.byref(out)))
    return out


def symnmf_state_set_phi(st: State, phi: float):
    code = lib().symnmf_state_set_phi(st.handle, phi)
    if code != OK:
        raise SymnmfError(code, "bad phi")


def symnmf_state_control(ctx, st: State) -> symnmf_control:
    out = symnmf_control()
    _check(ctx, lib().symnmf_state_control(ctx, st.handle, ctypes.byref(out)))
    return out


def symnmf_state_checks(ctx, st: State):
    """List of the stats of every check iteration evaluated so far."""
    count = c_i64()
    _check(ctx, lib().symnmf_state_checks(ctx, st.handle, None, 0, ctypes.byref(count)))
    arr = (symnmf_stats * max(count.value, 1))()
    _check(ctx, lib().symnmf_state_checks(ctx, st.handle, arr, count.value, ctypes.byref(count)))
    return [arr[i] for i in range(count.value)]


def symnmf_objective(ctx, S: Matrix, H, k: int):
    import torch
    f, E = c_dbl(), c_dbl()
    f64 = 1 if H.dtype == torch.float64 else 0
    _check(ctx, lib().symnmf_objective(ctx, ctypes.byref(S.desc), _ptr(H), f64, k, ctypes.byref(f), ctypes.byref(E)))
    return f.value, E.value


def symnmf_solve_to_tol(ctx, S: Matrix, st: State, f_target: float = 0.0, rel_tol: float = 1e-4, H_out=None):
    """Returns (stats, converged: bool)."""
    out = symnmf_stats()
    code = lib().symnmf_solve_to_tol(ctx, ctypes.byref(S.desc), st.handle, f_target, rel_tol, ctypes.byref(out),
                                     _ptr(H_out) if H_out is not None else None)
    if code not in (OK, ENOTCONV):
        _check(ctx, code)
    return out, code == OK


def symnmf_solve_trace(ctx, S: Matrix, st: State, steps: int, save_every: int, H_save):
    """H_save: device tensor (slots, n, k).  Returns (ms per kept iterate, first
    certified t or -1)."""
    nsave = steps // save_every
    ms = (c_dbl * max(nsave, 1))()
    cert = c_i64()
    _check(ctx, lib().symnmf_solve_trace(ctx, ctypes.byref(S.desc), st.handle, steps, save_every, _ptr(H_save),
                                         H_save.shape[0], ms, ctypes.byref(cert)))
    return [ms[i] for i in range(nsave)], cert.value


def symnmf_state_rebind(ctx, st: State, S: Matrix):
    """Point the state at another storage S of its matrix (precision ladder)."""
    _check(ctx, lib().symnmf_state_rebind(ctx, st.handle, ctypes.byref(S.desc)))
    st.S = S


def symnmf_solve_trace_ladder(ctx, S_lo: Matrix, S_hi: Matrix, st: State, steps: int, save_every: int, H_save,
                              tau_switch: float):
    """symnmf_solve_trace starting on S_lo and moving to S_hi at the first check
    whose stagnation measure is below tau_switch.  Returns (ms per kept
    iterate, first certified t on S_hi or -1, switch t or -1)."""
    nsave = steps // save_every
    ms = (c_dbl * max(nsave, 1))()
    cert, sw = c_i64(), c_i64()
    _check(ctx, lib().symnmf_solve_trace_ladder(ctx, ctypes.byref(S_lo.desc), ctypes.byref(S_hi.desc), st.handle,
                                                steps, save_every, _ptr(H_save), H_save.shape[0], ms, tau_switch,
                                                ctypes.byref(cert), ctypes.byref(sw)))
    if sw.value >= 0:
        st.S = S_hi
    return [ms[i] for i in range(nsave)], cert.value, sw.value


def symnmf_subspace_error(ctx, A, B):
    out = c_dbl()
    n, k = A.shape
    _check(ctx, lib().symnmf_subspace_error(ctx, _ptr(A), _ptr(B), n, k, ctypes.byref(out)))
    return out.value


def symnmf_median_sq(ctx, g, m=None):
    out = ctypes.c_float()
    m = g.numel() if m is None else m
    _check(ctx, lib().symnmf_median_sq(ctx, _ptr(g), m, ctypes.byref(out)))
    return out.value


def symnmf_median_sq_noalloc(ctx, g, out_dev, m=None):
    """out_dev: device float64 tensor (first element receives the median); nothing waits."""
    m = g.numel() if m is None else m
    _check(ctx, lib().symnmf_median_sq_noalloc(ctx, _ptr(g), m, _ptr(out_dev)))
    return out_dev


def symnmf_piecewise_reset(ctx, st: State, c: float):
    med = ctypes.c_float()
    _check(ctx, lib().symnmf_piecewise_reset(ctx, st.handle, c, ctypes.byref(med)))
    return med.value


def symnmf_sample_blocks(seed: int, t: int, stream: int, nblocks: int, m: int):
    buf = (c_i32 * m)()
    lib().symnmf_sample_blocks(seed, t, stream, nblocks, m, buf)
    return list(buf)


def symnmf_selfcheck_fp8(ctx):
    return lib().symnmf_selfcheck_fp8(ctx)


def symnmf_profile(ctx, enable: bool, read: bool = True):
    """Returns {kernel: (ms, launches)} since the last call (when read) and
    switches HIP-event timing on or off."""
    if not read:
        _check(ctx, lib().symnmf_profile(ctx, int(enable), None, None))
        return None
    ms = (c_dbl * len(PROFILE_KERNELS))()
    cnt = (c_i64 * len(PROFILE_KERNELS))()
    _check(ctx, lib().symnmf_profile(ctx, int(enable), ms, cnt))
    return {name: (ms[i], cnt[i]) for i, name in enumerate(PROFILE_KERNELS)}


def symnmf_probe_read(ctx, src, sink, nbytes=None):
    """sink: device int32 tensor (>= 4 words)."""
    nbytes = src.numel() * src.element_size() if nbytes is None else nbytes
    _check(ctx, lib().symnmf_probe_read(ctx, _ptr(src), _ptr(sink), sink.numel(), nbytes))


def symnmf_probe_copy(ctx, src, dst, nbytes=None):
    nbytes = src.numel() * src.element_size() if nbytes is None else nbytes
    _check(ctx, lib().symnmf_probe_copy(ctx, _ptr(src), _ptr(dst), nbytes))


# ---------------------------------------------------------------------------
# learned warm start
# ---------------------------------------------------------------------------
MLP_BUFFERS = {"params": 0, "grad": 1, "m": 2, "v": 3}


class Mlp:
    """Handle of a device network (width -> hidden -> hidden -> k)."""

    def __init__(self, ctx, handle, width, hidden, k):
        self.ctx, self.handle, self.width, self.hidden, self.k = ctx, handle, width, hidden, k
        self.count = symnmf_mlp_param_count(width, hidden, k)

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.symnmf_mlp_destroy(self.handle)
            self.handle = None


def symnmf_mlp_param_count(width: int, hidden: int, k: int) -> int:
    return lib().symnmf_mlp_param_count(width, hidden, k)


def symnmf_mlp_init(ctx, width: int, hidden: int, k: int, seed: int, params):
    _check(ctx, lib().symnmf_mlp_init(ctx, width, hidden, k, seed, _ptr(params)))
    return params


def symnmf_mlp_create(ctx, width: int, hidden: int, k: int, params) -> Mlp:
    """params: device float32 tensor of symnmf_mlp_param_count floats."""
    h = c_vp()
    _check(ctx, lib().symnmf_mlp_create(ctx, width, hidden, k, _ptr(params), ctypes.byref(h)))
    return Mlp(ctx, h, width, hidden, k)


def symnmf_mlp_destroy(m: Mlp):
    if m.handle is not None:
        lib().symnmf_mlp_destroy(m.handle)
        m.handle = None


def symnmf_mlp_set_output(ctx, m: Mlp, residual: bool):
    _check(ctx, lib().symnmf_mlp_set_output(ctx, m.handle, 1 if residual else 0))


def symnmf_mlp_reserve(ctx, m: Mlp, rows: int, training: bool = False):
    _check(ctx, lib().symnmf_mlp_reserve(ctx, m.handle, rows, 1 if training else 0))


def symnmf_mlp_read(ctx, m: Mlp, which, dst):
    which = MLP_BUFFERS[which] if isinstance(which, str) else which
    _check(ctx, lib().symnmf_mlp_read(ctx, m.handle, which, _ptr(dst)))
    return dst


def symnmf_mlp_write(ctx, m: Mlp, params):
    _check(ctx, lib().symnmf_mlp_write(ctx, m.handle, _ptr(params)))


def symnmf_mlp_forward(ctx, m: Mlp, X, A, bf16_weights: bool = True):
    _check(ctx, lib().symnmf_mlp_forward(ctx, m.handle, _ptr(X), X.shape[0], int(bf16_weights), _ptr(A)))
    return A


def symnmf_mlp_train_step(ctx, m: Mlp, X, B, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=1e-4,
                          loss_kind=0):
    """One AdamW step on one instance; returns the loss before the update
    (loss_kind 0: Gram loss, 1: scale-free Gram loss)."""
    opt = symnmf_adamw(lr=lr, beta1=beta1, beta2=beta2, eps=eps, weight_decay=weight_decay)
    loss = c_dbl()
    _check(ctx, lib().symnmf_mlp_train_step(ctx, m.handle, _ptr(X), _ptr(B), X.shape[0], ctypes.byref(opt),
                                            int(loss_kind), ctypes.byref(loss)))
    return loss.value


def symnmf_sketch(ctx, S: Matrix, omega_seed: int, width: int, Y):
    _check(ctx, lib().symnmf_sketch(ctx, ctypes.byref(S.desc), omega_seed, width, _ptr(Y)))
    return Y


def symnmf_canonical(ctx, Y, k: int, X, anchors=None):
    n, width = Y.shape
    _check(ctx, lib().symnmf_canonical(ctx, _ptr(Y), n, width, k, _ptr(X),
                                       _ptr(anchors) if anchors is not None else None))
    return X


def symnmf_warm_start(ctx, S: Matrix, mlp, width: int, k: int, omega_seed: int, H0):
    """mlp: an Mlp, or None for the network-free coordinates clipped at zero."""
    _check(ctx, lib().symnmf_warm_start(ctx, ctypes.byref(S.desc), mlp.handle if mlp is not None else None,
                                        width, k, omega_seed, _ptr(H0)))
    return H0


def symnmf_kmeans_seed_rows(seed: int, n: int, K: int):
    out = (c_i64 * K)()
    code = lib().symnmf_kmeans_seed_rows(seed, n, K, out)
    if code != OK:
        raise SymnmfError(code, "kmeans_seed_rows: need 1 <= K <= n")
    return list(out)


def symnmf_kmeans_seed_pp(ctx, S: Matrix, K: int, seed: int = 0):
    """k-means++ seed rows (list of K ints, draw order)."""
    out = (c_i64 * K)()
    _check(ctx, lib().symnmf_kmeans_seed_pp(ctx, ctypes.byref(S.desc), K, seed, out))
    return list(out)


def symnmf_row_norms(ctx, S: Matrix, norms):
    """norms: device float64 tensor of n entries."""
    _check(ctx, lib().symnmf_row_norms(ctx, ctypes.byref(S.desc), _ptr(norms)))
    return norms


def symnmf_kmeans_assign(ctx, S: Matrix, C, labels, best=None):
    """C: device n x K (float64 for FP64 storage, else float32); labels: device
    int32 n.  Returns the objective J."""
    J = c_dbl()
    _check(ctx, lib().symnmf_kmeans_assign(ctx, ctypes.byref(S.desc), _ptr(C), C.shape[1], _ptr(labels),
                                           _ptr(best) if best is not None else None, ctypes.byref(J)))
    return J.value


def symnmf_kmeans_centroids(ctx, S: Matrix, labels, K: int, C, C_prev=None):
    _check(ctx, lib().symnmf_kmeans_centroids(ctx, ctypes.byref(S.desc), _ptr(labels), K,
                                              _ptr(C_prev) if C_prev is not None else None, _ptr(C)))
    return C


def symnmf_kmeans(ctx, S: Matrix, K: int, labels, seed: int = 0, init_rows=None, tol: float = 1e-4,
                  max_iter: int = 100, C=None, allow_notconv: bool = False):
    """Spherical K-means; returns the stats as a dict.  init_rows: host
    sequence of K distinct rows (None: Forgy draw of seed)."""
    st = symnmf_kmeans_stats()
    rows = None
    if init_rows is not None:
        rows = (ctypes.c_int64 * K)(*[int(r) for r in init_rows])
    code = lib().symnmf_kmeans(ctx, ctypes.byref(S.desc), K, seed, rows, tol, max_iter, _ptr(labels),
                               _ptr(C) if C is not None else None, ctypes.byref(st))
    if not (allow_notconv and code == ENOTCONV):
        _check(ctx, code)
    return st.as_dict()


def symnmf_silhouette(ctx, S: Matrix, labels, K: int):
    out = c_dbl()
    _check(ctx, lib().symnmf_silhouette(ctx, ctypes.byref(S.desc), _ptr(labels), K, ctypes.byref(out)))
    return out.value


def symnmf_spectral(ctx, S: Matrix, max_iter: int = 500, tol: float = 1e-10, u1=None):
    """Returns a dict: lambda1, trace, r_eff, collapse, collapse_rows, iters."""
    vals = [c_dbl() for _ in range(5)]
    it = c_i64()
    _check(ctx, lib().symnmf_spectral(ctx, ctypes.byref(S.desc), max_iter, tol, *[ctypes.byref(v) for v in vals],
                                      ctypes.byref(it), _ptr(u1) if u1 is not None else None))
    keys = ("lambda1", "trace", "r_eff", "collapse", "collapse_rows")
    out = {k: v.value for k, v in zip(keys, vals)}
    out["iters"] = it.value
    return out
