"""Error paths of the C ABI on the GPU: a solve that reaches max_iter before
its tolerance reports TM_ERR_NOCONV with its outputs written, and
tm_load_gauge rejects links that are not SU(3), NaN links and lattices too
large for the kernels' 32-bit buffer offsets."""
import ctypes

import numpy as np
import pytest

from paper_1401_6749_amd import inputs
from tests import gpu_util as GU

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["f64", "mixed"])
def test_cg_noconv_writes_outputs(oracle, mode):
    """max_iter = 4 with tol 1e-10: TM_ERR_NOCONV, four iterations in the
    stats, the iterated and true residuals written and above the tolerance,
    and x holding the fourth iterate (the oracle's four-iteration solve)."""
    torch = GU.torch_mod()
    from paper_1401_6749_amd import tm

    ctx = GU.context()
    dims = (4, 4, 4, 8)
    V = int(np.prod(dims))
    U = inputs.gauge_field(dims, seed=14)
    g = GU.load(dims, U)
    kappa, a = 0.13, 0.01
    eta = oracle.z4_source(dims, 9, 0)
    b = GU.to_dev(eta[None])
    x = torch.zeros_like(b)
    p = tm.solver_params(mode, tol=1e-10, max_iter=4)
    rc, st = tm.tm_cg_solve(ctx, g, kappa, a, p, 1, b, x, check=False)
    assert rc == tm.TM_ERR_NOCONV, tm.STATUS_NAMES.get(rc, rc)
    assert "max_iter" in tm.tm_last_error(ctx)
    assert st[0]["iters"] == 4
    assert 1e-10 < st[0]["cg_rel_resid"] < 1.0
    assert 1e-10 < st[0]["true_rel_resid"] < 1.0
    got = GU.from_dev(x[0]).reshape(V, 4, 3)
    s4, it4, _, _ = oracle.solve(dims, -1, U, kappa, a, eta, fixed_iters=4)
    assert it4 == 4
    assert GU.relerr(got, s4) < (1e-12 if mode == "f64" else 1e-5)
    # the true residual reported is that of the written x
    r = eta - oracle.apply_M(dims, -1, U, kappa, a, got)
    assert abs(np.linalg.norm(r) / np.linalg.norm(eta) - st[0]["true_rel_resid"]) < 1e-10


def _load_rc(ctx, dims, links, tbc=-1):
    from paper_1401_6749_amd import tm

    out = ctypes.c_void_p()
    links = np.ascontiguousarray(links, dtype=np.complex128)
    rc = tm._lib.tm_load_gauge(ctx, tm._dims(dims), links.ctypes.data, int(tbc), tm.PREC["f32"],
                               ctypes.byref(out))
    return rc, out.value


def test_load_gauge_rejects_bad_links():
    from paper_1401_6749_amd import tm

    ctx = GU.context()
    dims = (4, 4, 4, 4)
    U = inputs.gauge_field(dims, seed=15)
    rc, gh = _load_rc(ctx, dims, U)
    assert rc == tm.TM_OK and gh
    tm.tm_free_gauge(ctx, gh)
    cases = {}
    bad = U.copy()
    bad[37, 2] *= 1.001  # not unitary
    cases["non-unitary"] = bad
    bad = U.copy()
    bad[5, 3] *= np.exp(1j * np.pi / 7)  # unitary, det = exp(3 i pi / 7)
    cases["det != 1"] = bad
    bad = U.copy()
    bad[200, 0, 1, 2] = np.nan
    cases["NaN"] = bad
    bad = U.copy()
    bad[0, 1, 0, 0] = np.inf
    cases["inf"] = bad
    for name, links in cases.items():
        rc, gh = _load_rc(ctx, dims, links)
        assert rc == tm.TM_ERR_ARG, (name, rc)
        assert gh is None, name
        assert "SU(3)" in tm.tm_last_error(ctx), name
    rc, _ = _load_rc(ctx, dims, U, tbc=0)
    assert rc == tm.TM_ERR_ARG
    rc, _ = _load_rc(ctx, (4, 4, 3, 4), U)
    assert rc == tm.TM_ERR_ARG


def test_load_gauge_rejects_oversized_lattice():
    """64^4 sites need a 6 GiB FP64 link array, beyond 32-bit buffer offsets:
    rejected before any link is read (a one-site buffer is passed)."""
    from paper_1401_6749_amd import tm

    ctx = GU.context()
    one = inputs.gauge_field((2, 2, 2, 2), seed=1)
    rc, gh = _load_rc(ctx, (64, 64, 64, 64), one)
    assert rc == tm.TM_ERR_ARG and gh is None
    assert "too large" in tm.tm_last_error(ctx)
