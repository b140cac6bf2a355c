"""FP64 CPU oracle for the SymNMF hot path - test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path.
"""
from .symnmf_oracle import *  # noqa: F401,F403
from .symnmf_oracle import (  # noqa: F401
    ADAGRAD, RMSPROP, PIECEWISE_ADAGRAD, ROW_SVRG, BLOCK_SVRG, ADMM, ADAM, NADAM, ADAN, MU, Params, Stats, Solver,
    admm_update, adam_update, adan_update, mu_update,
)
