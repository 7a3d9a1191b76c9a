"""Pins of the oracle's even-odd CG solve against LU, the free-field FFT
solution and pure-gauge covariance."""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_1401_6749_amd import inputs
from tests import helpers as H


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 4)])
def test_solve_matches_lu(oracle, dims):
    """I5/I7: the Schur + CG solution equals the dense LU solve of M s = eta
    within cond * tol."""
    V = int(np.prod(dims))
    U = inputs.gauge_field(dims, seed=41)
    kappa, a = 0.12, 0.01
    eta = oracle.z4_source(dims, 99, 0)
    M = H.dense_from_apply(lambda e: oracle.apply_M(dims, -1, U, kappa, a, e), 12 * V)
    lu = sla.lu_factor(M)
    s_lu = sla.lu_solve(lu, eta.reshape(-1))
    tol = 1e-12
    s, it, rel, true_rel = oracle.solve(dims, -1, U, kappa, a, eta, tol=tol)
    cond = np.linalg.cond(M)
    err = np.linalg.norm(s.reshape(-1) - s_lu) / np.linalg.norm(s_lu)
    assert rel <= tol
    assert err <= cond * cond * tol  # cond(M^dag M) = cond(M)^2
    assert err < 1e-9
    assert true_rel < 1e-10
    assert it > 3


def test_lp_truncation_residual(oracle):
    """A truncated (LP) solve stops at the first iteration with |r|/|r0| <= tol,
    and fixed_iters runs exactly that many iterations."""
    dims = (4, 4, 4, 4)
    U = inputs.gauge_field(dims, seed=1)
    eta = oracle.z4_source(dims, 101, 3)
    s1, it1, rel1, _ = oracle.solve(dims, -1, U, 0.12, 0.01, eta, tol=1e-2)
    assert rel1 <= 1e-2
    s0, it0, rel0, _ = oracle.solve(dims, -1, U, 0.12, 0.01, eta, fixed_iters=it1 - 1)
    assert it0 == it1 - 1 and rel0 > 1e-2
    s2, it2, rel2, _ = oracle.solve(dims, -1, U, 0.12, 0.01, eta, fixed_iters=it1)
    assert it2 == it1 and np.array_equal(s2, s1)


@pytest.mark.parametrize("tbc", [1, -1])
def test_free_field_fft_solve(oracle, tbc):
    """I8: on U = 1 the solution equals the momentum-space closed form."""
    dims = (8, 8, 8, 16)
    kappa, a = 0.12, 0.01
    U = inputs.unit_gauge(dims)
    eta = oracle.z4_source(dims, 7, 1)
    s, it, rel, true_rel = oracle.solve(dims, tbc, U, kappa, a, eta, tol=1e-12)
    want = H.free_solve_fft(dims, tbc, kappa, a, eta)
    err = np.linalg.norm(s - want) / np.linalg.norm(want)
    assert err < 1e-9, err


def test_pure_gauge_solve(oracle):
    """I9: on U_mu(x) = g(x) g(x+mu)^dag the solution is G M_free^-1 G^dag eta."""
    dims = (4, 4, 4, 8)
    V = int(np.prod(dims))
    kappa, a = 0.12, 0.005
    g = inputs.random_su3(V, seed=77)
    Ug = H.gauge_transform(dims, inputs.unit_gauge(dims), g)
    eta = oracle.z4_source(dims, 3, 2)
    s, it, rel, _ = oracle.solve(dims, -1, Ug, kappa, a, eta, tol=1e-12)
    gdag = np.conj(np.swapaxes(g, 1, 2))
    want = H.rotate_spinor(g, H.free_solve_fft(dims, -1, kappa, a, H.rotate_spinor(gdag, eta)))
    assert np.linalg.norm(s - want) / np.linalg.norm(want) < 1e-9
