"""Pin of the truncated solver method's error scaling (Sec. 2.1: with enough
correction sources the error of Eq. estiTSM falls as 1/sqrt(N_LP)), on the
oracle with crude LP solves (3 CG iterations) on 2^4:

  * for every N_LP the TSM error bars are calibrated: the deviations of the
    estimates from the dense traces, divided by their own sigma, have an RMS
    close to 1 over all operators and timeslices;
  * the error bars fall as N_LP^-1/2 (sigma * sqrt(N_LP) constant) while the
    correction term stays small.
"""
import numpy as np

from paper_1401_6749_amd import inputs
from tests import helpers as H
from tests.test_oracle_loops import _exact_spin_matrices


def test_tsm_error_scales_as_inverse_sqrt_n_lp(oracle):
    dims = (2, 2, 2, 2)
    V = int(np.prod(dims))
    U = inputs.gauge_field(dims, seed=91)
    kappa, a = 0.13, 0.05
    n_hp, n_lp = 16, 640
    r = oracle.loops_tsm(dims, -1, U, kappa, a, 55, n_hp, n_lp, lp_fixed_iters=3)
    Minv = np.linalg.inv(H.dense_from_apply(lambda e: oracle.apply_M(dims, -1, U, kappa, a, e), 12 * V))
    exact = oracle.project(_exact_spin_matrices(dims, -1, U, Minv))
    T = dims[3]
    hp = np.array([r["hp_loops"][j] for j in range(n_hp)])
    lp = np.array([r["lp_loops"][j] for j in range(n_hp + n_lp)])
    sig_sqrt_n = []
    for n in (80, 160, 320, 640):
        est, vre, vim = oracle.tsm_combine(hp, lp[:n_hp], lp[n_hp:n_hp + n])
        ok = vre > 0
        z = (est.real - exact.real)[ok] / np.sqrt(vre[ok])
        assert 0.7 < np.sqrt(np.mean(z ** 2)) < 1.4, n
        _, cre, _ = oracle.tsm_combine(hp, lp[:n_hp], lp[:0])
        assert np.median(cre[ok] / vre[ok]) < 0.25, n  # the correction term is small
        sig_sqrt_n.append(np.median(np.sqrt(vre[ok])) * np.sqrt(n))
    sig_sqrt_n = np.array(sig_sqrt_n)
    assert sig_sqrt_n.max() / sig_sqrt_n.min() < 1.25, sig_sqrt_n
    assert est.shape == (oracle.N_OPS, T)
