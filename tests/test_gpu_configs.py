"""GPU parity on the remaining benchmark configurations (synthetic seeded
inputs with the paper's shapes): the plain FP64 method at 16^3x32."""
import numpy as np
import pytest

from paper_1401_6749_amd import inputs
from tests import gpu_util as GU

pytestmark = pytest.mark.gpu


def test_c2_plain_f64_16c32(oracle):
    """Plain method on the GPU in FP64 at 16^3x32 (kappa 0.12, 2 kappa mu
    0.005, 64 Z4 sources solved to 1e-10, local and one-derivative loops):
    sampled sources' spin matrices equal the oracle's to 1e-10, and the
    estimate is the mean of the 64 per-source loops."""
    from paper_1401_6749_amd import tm

    ctx = GU.context()
    dims = (16, 16, 16, 32)
    U = inputs.gauge_field(dims, seed=2)
    g = GU.load(dims, U)
    P = tm.tsm_params(0.12, 0.005, 102, 0, 64, lp=tm.solver_params("f64", tol=1e-10), batch=12)
    r = tm.tm_loops_tsm(ctx, g, P, dims[3], want_raw=True)
    ids = [0, 37, 63]
    ref = oracle.loops_tsm(dims, -1, U, 0.12, 0.005, 102, 0, 64, lp_tol=1e-10, source_ids=ids, return_raw=True)
    for j in ids:
        assert GU.relerr(r["raw_lp"][j], ref["lp_raw"][j]) < 1e-10, j
    ops = tm.tm_project_loops(r["raw_lp"])
    assert GU.relerr(r["est"], ops.mean(axis=0)) < 1e-12
    assert r["stats"]["lp_solves"] == 64
    tm.tm_free_gauge(ctx, g)
