"""Helpers of the GPU tests: a session context and readers of stored S."""
import numpy as np
import torch

import paper_2607_24518_amd as sym

_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        if not torch.cuda.is_available():
            raise RuntimeError("GPU tests need a HIP device")
        sym.lib()
        _CTX = sym.symnmf_create(0)
    return _CTX


def dev():
    return torch.device("cuda:0")


def stored_numpy(S):
    """float64 rows x n matrix of what the solver multiplies with (decoded)."""
    d = S.desc
    rows, n, ld, rp = d.rows, d.n, d.ld, d.rows_pad
    buf = S.buf
    if d.dtype == sym.S_FP64:
        M = buf[: rp * ld * 8].view(torch.float64).view(rp, ld)[:rows, :n].double()
    elif d.dtype == sym.S_FP32:
        M = buf[: rp * ld * 4].view(torch.float32).view(rp, ld)[:rows, :n].double()
    elif d.dtype == sym.S_BF16:
        M = buf[: rp * ld * 2].view(torch.bfloat16).view(rp, ld)[:rows, :n].double()
    else:
        codes = buf[: rp * ld].view(torch.float8_e4m3fn).view(rp, ld)[:rows, :n].double()
        so = d.panel_scale - d.data
        do = d.diag - d.data
        panels = (rows + d.fp8_panel_rows - 1) // d.fp8_panel_rows
        scale = buf[so: so + 4 * panels].view(torch.float32).double()
        diag = buf[do: do + 4 * rows].view(torch.float32).double()
        rowscale = scale.repeat_interleave(d.fp8_panel_rows)[:rows]
        M = codes / rowscale[:, None]
        r = torch.arange(rows, device=M.device)
        M[r, r + d.row0] = diag
    return M.cpu().numpy()


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).to(dev()).contiguous()


def from_dev(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()
