"""Pins of the oracle's time dilution and coherent sources (Sec. 2.3):

  * the per-noise loops equal their definition written with the dense
    inverse: a source on a phase class of timeslices reaches the loop at t
    only through the blocks M^-1(x, y) with t(y) in the class of t(x), for the
    local and the forward time-derivative spin matrices (full dilution and
    coherent sources);
  * spacing 1 (one source covering all timeslices) is ``loops_tsm``;
  * the validity mask of the time-derivative operators;
  * with Z4 noise: unbiased against the dense traces for every covered entry
    (alone and with the hopping parameter expansion), and a smaller variance
    per noise vector than the undiluted estimator.
"""
import numpy as np
import pytest

from paper_1401_6749_amd import inputs
from tests import helpers as H
from tests.test_oracle_loops import _exact_spin_matrices


def _dense_inv(oracle, dims, tbc, U, kappa, a):
    V = int(np.prod(dims))
    return np.linalg.inv(H.dense_from_apply(lambda e: oracle.apply_M(dims, tbc, U, kappa, a, e), 12 * V))


@pytest.mark.parametrize("spacing", [8, 4, 2])
def test_tdil_loops_equal_block_definition(oracle, spacing):
    dims = (2, 2, 2, 8)
    tbc = -1
    U = inputs.gauge_field(dims, seed=81)
    kappa, a = 0.13, 0.03
    V, T = int(np.prod(dims)), dims[3]
    Minv = _dense_inv(oracle, dims, tbc, U, kappa, a)
    r = oracle.loops_tdil(dims, tbc, U, kappa, a, 17, 0, 3, spacing, lp_tol=1e-13, source_ids=[2],
                          return_raw=True)
    got = r["raw"]["lp_std"][2]
    eta = oracle.z4_source(dims, 17, 2).reshape(V, 12)
    tsite = np.array([H.coords(dims, x)[3] for x in range(V)])
    want_loc = np.zeros((T, 4, 4), dtype=complex)
    want_ft = np.zeros((T, 4, 4), dtype=complex)
    for t in range(T):
        cls = np.where(tsite % spacing == t % spacing)[0]  # sites in the phase class of t
        cols = (12 * cls[:, None] + np.arange(12)).reshape(-1)
        sol = (Minv[:, cols] @ eta[cls].reshape(-1)).reshape(V, 4, 3)  # M^-1 eta restricted to the class
        for x in np.where(tsite == t)[0]:
            e = eta[x].reshape(4, 3)
            want_loc[t] += np.einsum("ac,bc->ab", e.conj(), sol[x])
            f, sg = H.shifted(dims, x, 3, +1, tbc)
            us = sg * np.einsum("cd,bd->bc", U[x, 3], sol[f])
            want_ft[t] += np.einsum("ac,bc->ab", e.conj(), us)
    scale = np.abs(want_loc).max()
    assert np.allclose(got[0], want_loc, atol=1e-10 * scale)
    assert np.allclose(got[4], want_ft, atol=1e-10 * scale)
    if spacing < T:
        # coherent sources differ from full dilution (cross terms between their timeslices)
        r8 = oracle.loops_tdil(dims, tbc, U, kappa, a, 17, 0, 3, 8, lp_tol=1e-13, source_ids=[2], return_raw=True)
        assert np.abs(r8["raw"]["lp_std"][2][0] - got[0]).max() > 1e-6 * scale


def test_tdil_spacing_one_is_undiluted(oracle):
    dims = (2, 2, 2, 4)
    U = inputs.gauge_field(dims, seed=82)
    r = oracle.loops_tdil(dims, -1, U, 0.12, 0.02, 23, 2, 4, 1)
    ref = oracle.loops_tsm(dims, -1, U, 0.12, 0.02, 23, 2, 4)
    assert np.array_equal(r["est_std"], ref["est"])
    assert np.array_equal(r["var_re_std"], ref["var_re"])
    assert r["valid"].all()


def test_tdil_valid_mask(oracle):
    T = 8
    v = oracle.tdil_valid(T, 8, [3])
    assert v[:16, 3].all() and v[:16].sum() == 16
    tder = [16 + 4 * g + 3 for g in range(16)]
    sder = [16 + 4 * g + nu for g in range(16) for nu in range(3)]
    assert not v[tder].any()
    assert v[sder, 3].all() and v[sder].sum() == len(sder)
    v3 = oracle.tdil_valid(T, 8, [2, 3, 4])
    assert v3[tder, 3].all() and v3[tder].sum() == 16
    assert oracle.tdil_valid(T, 4, [0, 1, 2, 3]).all()
    # coherent: phase 1 of spacing 4 covers t = 1 and 5
    vc = oracle.tdil_valid(T, 4, [1])
    assert vc[0].tolist() == [False, True, False, False, False, True, False, False]
    with pytest.raises(ValueError):
        oracle.tdil_mask((2, 2, 2, 8), 3, 0)


def test_tdil_unbiased_and_smaller_variance(oracle):
    """Full time dilution (spacing T) with Z4 noise, converged solves: every
    covered entry within 4 sigma of the dense traces, also with the
    expansion; the local variance per noise vector below the undiluted one;
    with phases {t0-1, t0, t0+1} the time-derivative loops at t0 are
    covered and unbiased."""
    dims = (4, 4, 4, 4)
    U = inputs.gauge_field(dims, seed=83)
    kappa, a = 0.14, 0.05
    n = 40
    Minv = _dense_inv(oracle, dims, -1, U, kappa, a)
    exact = oracle.project(_exact_spin_matrices(dims, -1, U, Minv))
    r = oracle.loops_tdil(dims, -1, U, kappa, a, 29, 0, n, 4, hpe=True, lp_tol=1e-12)
    for f in ("std", "hpe"):
        est, vre, vim = r["est_" + f], r["var_re_" + f], r["var_im_" + f]
        ok = np.isfinite(est)
        assert ok.sum() == (r["valid"].sum() if f == "std" else 16 * dims[3])
        dre = np.abs(est.real - exact.real)[ok] <= 4 * np.sqrt(vre[ok]) + 1e-12
        dim = np.abs(est.imag - exact.imag)[ok] <= 4 * np.sqrt(vim[ok]) + 1e-12
        assert dre.mean() > 0.99 and dim.mean() > 0.99, f
    und = oracle.loops_tsm(dims, -1, U, kappa, a, 29, 0, n, lp_tol=1e-12)
    v_dil = (r["var_re_std"][:16] + r["var_im_std"][:16]).sum()
    v_und = (und["var_re"][:16] + und["var_im"][:16]).sum()
    assert v_dil < 0.9 * v_und, (v_dil, v_und)
    t0 = 2
    r3 = oracle.loops_tdil(dims, -1, U, kappa, a, 31, 0, n, 4, phases=[t0 - 1, t0, t0 + 1], lp_tol=1e-12)
    tder = [16 + 4 * g + 3 for g in range(16)]
    assert np.isfinite(r3["est_std"][tder, t0]).all() and np.isnan(r3["est_std"][tder, t0 + 1]).all()
    d = r3["est_std"][tder, t0] - exact[tder, t0]
    assert (np.abs(d.real) <= 4 * np.sqrt(r3["var_re_std"][tder, t0]) + 1e-12).all()
    assert (np.abs(d.imag) <= 4 * np.sqrt(r3["var_im_std"][tder, t0]) + 1e-12).all()
