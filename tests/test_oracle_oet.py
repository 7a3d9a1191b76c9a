"""Pins of the oracle's one-end trick estimators (Sec. 2.2, Eq. loopVv and
Eq. loopStD) against dense inverses of M_u = M(+mu) and M_d = M(-mu): with
full dilution (all 12V unit sources) the estimators give the exact
Tr(M_u^-1 X) -+ Tr(M_d^-1 X) for all 90 operators X, and with Z4 noise
``loops_oet`` is an unbiased estimate of the same traces."""
import numpy as np
import pytest

from paper_1401_6749_amd import inputs
from tests import helpers as H
from tests.test_oracle_loops import _exact_spin_matrices


def _dense(oracle, dims, tbc, U, kappa, a):
    V = int(np.prod(dims))
    return H.dense_from_apply(lambda e: oracle.apply_M(dims, tbc, U, kappa, a, e), 12 * V)


@pytest.mark.parametrize("tbc", [-1, 1])
def test_oet_full_dilution_equals_flavour_traces(oracle, tbc):
    """-2ia sum_e s_e^dag g5 X s_e = Tr(M_u^-1 X) - Tr(M_d^-1 X) and
    2 sum_e s_e^dag g5 X g5 D_W s_e = Tr(M_u^-1 X) + Tr(M_d^-1 X), s_e = M_u^-1 e,
    for the local, one-derivative and symmetrised operators."""
    dims = (2, 2, 2, 4)
    V = int(np.prod(dims))
    U = inputs.gauge_field(dims, seed=61)
    kappa, a = 0.13, 0.04
    Mu_inv = np.linalg.inv(_dense(oracle, dims, tbc, U, kappa, a))
    Md_inv = np.linalg.inv(_dense(oracle, dims, tbc, U, kappa, -a))
    DW = _dense(oracle, dims, tbc, U, kappa, 0.0)
    vv = np.zeros((9, dims[3], 4, 4), dtype=np.complex128)
    ws = np.zeros_like(vv)
    for j in range(12 * V):
        s = Mu_inv[:, j]
        vv += oracle.contract(dims, tbc, U, s, s)
        ws += oracle.contract(dims, tbc, U, s, DW @ s)
    gvv, gws = oracle.oet_gammas()
    lu = oracle.project(_exact_spin_matrices(dims, tbc, U, Mu_inv))
    ld = oracle.project(_exact_spin_matrices(dims, tbc, U, Md_inv))
    got_vv = oracle.project(-2j * a * vv, gvv)
    got_ws = oracle.project(2.0 * ws, gws)
    assert np.allclose(got_vv, lu - ld, atol=1e-12 * np.abs(lu).max())
    assert np.allclose(got_ws, lu + ld, atol=1e-12 * np.abs(lu).max())
    # the flavour difference is not trivially zero, and it is what the
    # isovector estimator measures (a sign error would double it)
    assert np.abs(lu - ld).max() > 1e-3


def test_oet_gammas_structure(oracle):
    """g5 G and g5 G g5: same sparsity as G, rows 2,3 (and columns 2,3) flipped."""
    G = oracle.gammas16()
    gvv, gws = oracle.oet_gammas()
    sgn = np.array([1, 1, -1, -1])
    assert np.allclose(gvv, sgn[None, :, None] * G)
    assert np.allclose(gws, sgn[None, :, None] * G * sgn[None, None, :])


def test_loops_oet_unbiased_with_noise(oracle):
    """Z4-noise estimates from ``loops_oet`` (N_HP = 0, converged solves) lie
    within 4 sigma of the exact flavour traces for every operator and t, and
    the TSM pieces reduce as for the standard estimator."""
    dims = (2, 2, 2, 2)
    U = inputs.gauge_field(dims, seed=62)
    kappa, a = 0.12, 0.05
    n = 300
    r = oracle.loops_oet(dims, -1, U, kappa, a, 77, 0, n, lp_tol=1e-12)
    Mu_inv = np.linalg.inv(_dense(oracle, dims, -1, U, kappa, a))
    Md_inv = np.linalg.inv(_dense(oracle, dims, -1, U, kappa, -a))
    lu = oracle.project(_exact_spin_matrices(dims, -1, U, Mu_inv))
    ld = oracle.project(_exact_spin_matrices(dims, -1, U, Md_inv))
    for f, exact in (("vv", lu - ld), ("ws", lu + ld)):
        est, vre, vim = r["est_" + f], r["var_re_" + f], r["var_im_" + f]
        dre = np.abs(est.real - exact.real) - 4 * np.sqrt(vre) - 1e-12
        dim = np.abs(est.imag - exact.imag) - 4 * np.sqrt(vim) - 1e-12
        assert (dre <= 0).mean() > 0.99 and (dim <= 0).mean() > 0.99, f
    # HP == LP (both converged): the correction vanishes and the estimate is the bulk mean
    r2 = oracle.loops_oet(dims, -1, U, kappa, a, 78, 3, 5, hp_tol=1e-12, lp_tol=1e-12)
    bulk = np.mean([r2["loops"]["lp_vv"][j] for j in range(3, 8)], axis=0)
    assert np.allclose(r2["est_vv"], bulk, atol=1e-10 * np.abs(bulk).max())
