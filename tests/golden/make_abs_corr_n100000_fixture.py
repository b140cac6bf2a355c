"""Write abs_corr_n100000_k32_trajectory.json: the FP64 oracle's first
iterations on the 100000-instrument |corr| workload, for the full-size parity
test of the HIP path (tests/test_gpu_c3_trajectory.py).

Calls only ``oracle`` and ``synth`` (no GPU, no library).  Run from the
repository root:  python tests/golden/make_abs_corr_n100000_fixture.py
(about 15 minutes on 8 cores; S is held as float32 in host memory, 40 GB, and
every product with it is formed in FP64, see oracle.StoredRows).

Workload: returns T = 2500 x n = 100000 from synth.overlap_returns(seed 0,
32 overlapping groups, market loading 0.4, generated on the CPU), S = |corr|
with unit diagonal, k = 32, H0 = the counter-RNG initial factor (section
"Initialization and seeds", seed 0) rounded to float32 as a float32 solver
stores it.  Two FP64 trajectories of N steps from the same H0:
* projected AdaGrad, eta = sqrt(mean(S) / k), eps = 1e-10 (appendix family 3);
* ADMM, rho = 500 (appendix family 6).
Stored per step t = 0..N-1: f(H_t), E_t and the KKT measure; after the last
step: 64 sampled rows of H_N (ADMM: of W_N and U_N), row indices drawn by
numpy's generator with seed 12345.  Also stored: mean(S), ||S||_F^2 of the
float32-rounded S, and checksums of X (so a test can tell a different input
from a different result).
"""
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as o  # noqa: E402
import synth  # noqa: E402

N_STEPS = 30
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "abs_corr_n100000_k32_trajectory.json")


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def main():
    n, T, groups, k = 100000, 2500, 32, 32
    X = synth.overlap_returns(0, T=T, n=n, groups=groups, device="cpu").X.numpy()
    Xd = X.astype(np.float64)
    checks = {"sum": float(Xd.sum()), "sum_sq": float((Xd * Xd).sum()),
              "samples": [float(X[t, j]) for t, j in ((0, 0), (17, 4242), (2499, 99999), (1234, 56789))]}
    del Xd
    log("building S (float32 storage, FP64 panels)")
    S = o.StoredRows.abs_corr(X)
    del X
    mean = S.mean()
    log(f"S built: mean {mean:.12e} fro2 {S.fro2:.12e}")
    H0 = o.init_H(mean, n, k, 0, as_float32=True)
    rows = np.sort(np.random.default_rng(12345).choice(n, 64, replace=False))
    eta = math.sqrt(mean / k)
    out = {"n": n, "T": T, "groups": groups, "k": k, "seed": 0, "init_seed": 0, "mean": mean, "fro2": S.fro2,
           "eta": eta, "rho": 500.0, "steps": N_STEPS, "rows": rows.tolist(), "X_checksums": checks}
    for name, params in (("adagrad", o.Params(eta=eta)), ("admm", o.Params(method=o.ADMM, rho=500.0))):
        solver = o.Solver(S, k, params, H0)
        f, E, kkt = [], [], []
        for t in range(N_STEPS):
            st = solver.step()
            f.append(st.f)
            E.append(st.E)
            kkt.append(st.kkt)
            log(f"{name} t={t} f={st.f:.12e} kkt={st.kkt:.6e}")
        out[name] = {"f": f, "E": E, "kkt": kkt, "H_rows": solver.H[rows].tolist()}
        if name == "admm":
            out[name]["U_rows"] = solver.U[rows].tolist()
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    log(f"wrote {OUT}")


if __name__ == "__main__":
    main()
