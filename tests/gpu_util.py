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


def untile(flat, rows_pad, ld, E):
    """Row-major matrix from the tiled storage: 256 x 256 tiles in (row tile,
    column chunk) order; inside a tile [wave 4][sub-step 256/(4E)][row group 4]
    [lane 64][E], lane l holding row 64 wave + 16 group + l % 16 and columns
    (4E) sub-step + E (l // 16) + e."""
    R, C, NS = rows_pad // 256, ld // 256, 256 // (4 * E)
    t = flat.view(R, C, 4, NS, 4, 4, 16, E)            # R, C, wv, s, rg, lg, lr, e
    t = t.permute(0, 2, 4, 6, 1, 3, 5, 7)              # R, wv, rg, lr, C, s, lg, e
    return t.reshape(rows_pad, ld)


def stored_numpy(S):
    """float64 rows x n matrix of what the solver multiplies with (decoded)."""
    d = S.desc
    rows, n, ld, rp = d.rows, d.n, d.ld, d.rows_pad
    buf = S.buf
    if d.dtype == sym.S_FP64:
        M = buf[: rp * ld * 8].view(torch.float64).view(rp, ld)[:rows, :n].double()
    elif d.dtype == sym.S_FP32:
        M = untile(buf[: rp * ld * 4].view(torch.float32), rp, ld, 4)[:rows, :n].double()
    elif d.dtype == sym.S_BF16:
        M = untile(buf[: rp * ld * 2].view(torch.bfloat16), rp, ld, 8)[:rows, :n].double()
    else:
        codes = untile(buf[: rp * ld].view(torch.float8_e4m3fn), rp, ld, 16)[:rows, :n].double()
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


def stored_rows(S, rows):
    """float64 rows (global indices) of what the solver multiplies with,
    decoded from one 256-row tile row at a time (the tiles of a tile row are
    contiguous in the tiled layout), for matrices too large to decode whole."""
    d = S.desc
    rows = np.asarray(rows, dtype=np.int64)
    local = rows - d.row0
    out = torch.empty(rows.size, d.n, dtype=torch.float64, device=S.buf.device)
    if d.dtype == sym.S_FP64:
        M = S.buf[: d.rows_pad * d.ld * 8].view(torch.float64).view(d.rows_pad, d.ld)
        out[:] = M[torch.from_numpy(local).to(M.device), : d.n]
        return out.cpu().numpy()
    E, dt = {sym.S_FP32: (4, torch.float32), sym.S_BF16: (8, torch.bfloat16), sym.S_FP8: (16, torch.float8_e4m3fn)}[d.dtype]
    esz = torch.tensor([], dtype=dt).element_size()
    per = 256 * d.ld
    for R in np.unique(local // 256):
        sel = np.nonzero(local // 256 == R)[0]
        flat = S.buf[R * per * esz: (R + 1) * per * esz].view(dt)
        tile = untile(flat, 256, d.ld, E)[torch.from_numpy(local[sel] % 256).to(flat.device), : d.n].double()
        out[torch.from_numpy(sel).to(out.device)] = tile
    if d.dtype == sym.S_FP8:
        so = d.panel_scale - d.data
        do = d.diag - d.data
        panels = (d.rows + d.fp8_panel_rows - 1) // d.fp8_panel_rows
        scale = S.buf[so: so + 4 * panels].view(torch.float32).double()
        diag = S.buf[do: do + 4 * d.rows].view(torch.float32).double()
        li = torch.from_numpy(local).to(out.device)
        out /= scale[li // d.fp8_panel_rows][:, None]
        out[torch.arange(rows.size, device=out.device), torch.from_numpy(rows).to(out.device)] = diag[li]
    return out.cpu().numpy()


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).to(dev()).contiguous()


def from_dev(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()
