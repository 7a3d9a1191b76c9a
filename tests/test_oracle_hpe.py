"""Pins of the oracle's hopping parameter expansion (Sec. 2.4, Eq. HPE and
Eq. loopHPE1) on 4^4 lattices with random SU(3) links:

  * ``apply_bh`` against B (M - B^-1) with M and B^-1 = M at kappa = 0 taken
    as dense matrices of the oracle's M (this fixes H = -kappa D_hop, sign and
    normalisation), and the expansion identity
    M^-1 = B - BHB + (BH)^2 B - (BH)^3 B + (BH)^4 M^-1 on vectors;
  * ``hpe_exact`` (a closed form) against the site-diagonal blocks of the
    four exact terms multiplied out as sparse matrices, for both time
    boundary conditions and two (kappa, a);
  * full dilution: exact part + stochastic term over all 12V unit sources
    gives the exact local traces of the dense inverse;
  * with Z4 noise: unbiased, and smaller variance than the standard
    estimator for the local operators.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1401_6749_amd import inputs
from tests import helpers as H
from tests.test_oracle_loops import _exact_spin_matrices

DIMS = (4, 4, 4, 4)


def _dense_M(oracle, dims, tbc, U, kappa, a):
    V = int(np.prod(dims))
    return H.dense_from_apply(lambda e: oracle.apply_M(dims, tbc, U, kappa, a, e), 12 * V)


def _sparse_BH(oracle, dims, tbc, U, kappa, a):
    """(B, H) as sparse matrices from dense M: B^-1 = M(kappa = 0), H = M - B^-1."""
    M = _dense_M(oracle, dims, tbc, U, kappa, a)
    A = _dense_M(oracle, dims, tbc, U, 0.0, a)
    assert np.count_nonzero(A - np.diag(np.diag(A))) == 0  # site- and spin-diagonal
    B = sp.diags(1.0 / np.diag(A)).tocsr()
    Hm = sp.csr_matrix(M - A)
    return M, B, Hm


@pytest.fixture(scope="module")
def field():
    return inputs.gauge_field(DIMS, seed=71)


def test_apply_bh_and_expansion_identity(oracle, field):
    kappa, a = 0.14, 0.07
    U = field
    V = int(np.prod(DIMS))
    M, B, Hm = _sparse_BH(oracle, DIMS, -1, U, kappa, a)
    rng = np.random.default_rng(5)
    for _ in range(3):
        v = rng.standard_normal(12 * V) + 1j * rng.standard_normal(12 * V)
        bh = oracle.apply_bh(DIMS, -1, U, kappa, a, v).reshape(-1)
        assert np.allclose(bh, B @ (Hm @ v), atol=1e-13 * np.abs(bh).max())
        # a flipped kappa sign is far off
        assert not np.allclose(bh, -(B @ (Hm @ v)), atol=1e-3 * np.abs(bh).max())
        y = np.linalg.solve(M, v)
        Bv = (v.reshape(V, 4, 3) / (1 + 1j * a * np.array([1, 1, -1, -1]))[None, :, None]).reshape(-1)
        terms, w = [], Bv
        for n in range(4):
            terms.append((-1) ** n * w)
            w = oracle.apply_bh(DIMS, -1, U, kappa, a, w).reshape(-1)
        y4 = y
        for _ in range(4):
            y4 = oracle.apply_bh(DIMS, -1, U, kappa, a, y4).reshape(-1)
        assert np.allclose(y, sum(terms) + y4, atol=1e-12 * np.abs(y).max())


@pytest.mark.parametrize("tbc,kappa,a", [(-1, 0.14, 0.07), (1, 0.16, 0.3)])
def test_hpe_exact_closed_form(oracle, field, tbc, kappa, a):
    """Site-diagonal blocks of B - BHB + (BH)^2 B - (BH)^3 B summed per
    timeslice equal ``hpe_exact``; the odd terms contribute nothing and the
    second-order term is not negligible."""
    U = field
    V = int(np.prod(DIMS))
    _, B, Hm = _sparse_BH(oracle, DIMS, tbc, U, kappa, a)
    BH = (B @ Hm).tocsr()
    terms = [B]
    for _ in range(3):
        terms.append((BH @ terms[-1]).tocsr())
    K = terms[0] - terms[1] + terms[2] - terms[3]
    T = DIMS[3]
    want = np.zeros((T, 4, 4), dtype=np.complex128)
    odd = 0.0
    for x in range(V):
        t = H.coords(DIMS, x)[3]
        blk = K[12 * x:12 * x + 12, 12 * x:12 * x + 12].toarray().reshape(4, 3, 4, 3)
        want[t] += np.einsum("bcac->ab", blk)
        for n in (1, 3):
            odd = max(odd, np.abs(terms[n][12 * x:12 * x + 12, 12 * x:12 * x + 12].toarray()).max())
    got = oracle.hpe_exact(DIMS, kappa, a)
    assert np.allclose(got, want, atol=1e-12 * np.abs(want).max())
    assert odd < 1e-14
    second = want - oracle.hpe_exact(DIMS, 0.0, a)
    assert np.abs(second).max() > 1e-3 * np.abs(want).max()


def test_hpe_exact_needs_even_extents(oracle):
    for dims in [(2, 4, 4, 4), (4, 4, 4, 6), (4, 4, 2, 4)]:
        if all(L >= 4 and L % 2 == 0 for L in dims):
            oracle.hpe_exact(dims, 0.1, 0.1)
        else:
            with pytest.raises(ValueError):
                oracle.hpe_exact(dims, 0.1, 0.1)


def test_hpe_full_dilution_equals_local_traces(oracle, field):
    """exact part + sum over all 12V unit sources of contract(e, (BH)^4 M^-1 e)
    equals the local traces of the dense inverse."""
    kappa, a = 0.15, 0.05
    U = field
    V = int(np.prod(DIMS))
    Minv = np.linalg.inv(_dense_M(oracle, DIMS, -1, U, kappa, a))
    stoch = np.zeros((DIMS[3], 4, 4), dtype=np.complex128)
    for j in range(12 * V):
        w = Minv[:, j]
        for _ in range(4):
            w = oracle.apply_bh(DIMS, -1, U, kappa, a, w)
        e = np.zeros(12 * V, dtype=np.complex128)
        e[j] = 1
        stoch += oracle.contract(DIMS, -1, U, e, w)[0]
    exact = _exact_spin_matrices(DIMS, -1, U, Minv)[0]
    got = oracle.hpe_exact(DIMS, kappa, a) + stoch
    assert np.allclose(got, exact, atol=1e-12 * np.abs(exact).max())
    # the stochastic term is a small remainder of the trace
    assert np.abs(stoch).max() < 0.2 * np.abs(exact).max()


def test_loops_hpe_unbiased_and_smaller_variance(oracle, field):
    """Z4 noise, converged solves: HPE estimates of the local loops within
    4 sigma of the exact traces; their variance below the standard
    estimator's; operators with a link are NaN; the standard half equals
    ``loops_tsm``."""
    kappa, a = 0.15, 0.05
    U = field
    n = 60
    r = oracle.loops_hpe(DIMS, -1, U, kappa, a, 91, 0, n, lp_tol=1e-12)
    Minv = np.linalg.inv(_dense_M(oracle, DIMS, -1, U, kappa, a))
    exact = oracle.project(_exact_spin_matrices(DIMS, -1, U, Minv))[:16]
    est, vre, vim = r["est_hpe"][:16], r["var_re_hpe"][:16], r["var_im_hpe"][:16]
    ok = (np.abs(est.real - exact.real) <= 4 * np.sqrt(vre) + 1e-12) & \
         (np.abs(est.imag - exact.imag) <= 4 * np.sqrt(vim) + 1e-12)
    assert ok.mean() > 0.99
    v_hpe = (r["var_re_hpe"][:16] + r["var_im_hpe"][:16]).sum()
    v_std = (r["var_re_std"][:16] + r["var_im_std"][:16]).sum()
    assert v_hpe < 0.5 * v_std, (v_hpe, v_std)
    assert np.isnan(r["est_hpe"][16:]).all() and np.isnan(r["var_re_hpe"][16:]).all()
    ref = oracle.loops_tsm(DIMS, -1, U, kappa, a, 91, 0, n, lp_tol=1e-12)
    assert np.allclose(r["est_std"], ref["est"], atol=1e-12 * np.abs(ref["est"]).max())
