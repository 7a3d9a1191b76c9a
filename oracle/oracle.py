"""Plain FP64 CPU oracle for the twisted-mass disconnected-loop method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code with the HIP implementation in ``paper_1401_6749_amd`` and imports
nothing from it.

The heavy loops (hopping term, even-odd CG, Philox, contractions) are in
``tm_oracle.c`` (plain C99 complex arithmetic, built with gcc into
``libtm_oracle.so``); this file wraps them and adds the small host-side steps
in NumPy:

  * ``gamma`` / ``gammas16``    chiral basis and the 16 local insertions
  * ``project``                 spin matrices -> local, one-derivative and
                                symmetrised gamma_mu D_nu loops
  * ``tsm_combine``             the truncated-solver estimator (Sec. 2.1,
                                Eq. estiTSM) and its stochastic variance
  * ``loops_tsm``               the whole path: Z4 sources (Sec. 2), HP and LP
                                solves (Sec. 2.1), contractions at all
                                timeslices (Sec. 2.2), projection and TSM.
  * ``loops_oet``               the same with the one-end trick estimators
                                (Sec. 2.2, Eq. loopVv and Eq. loopStD).
  * ``apply_bh`` / ``hpe_exact`` / ``loops_hpe``
                                the hopping parameter expansion (Sec. 2.4,
                                Eq. HPE and Eq. loopHPE1).
  * ``tdil_mask`` / ``tdil_valid`` / ``loops_tdil``
                                time dilution and coherent sources (Sec. 2.3),
                                alone or with the expansion.

Array layouts (complex128): spinor (V, 4, 3), gauge (V, 4, 3, 3), with
lex = x + Lx*(y + Ly*(z + Lz*t)).  ``a`` always means 2*kappa*mu.

Pins for every function are in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libtm_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile tm_oracle.c with gcc (OpenMP) into libtm_oracle.so."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.orc_gamma.argtypes = [ctypes.c_int, dp]
        L.orc_dhop.argtypes = [ip, ctypes.c_int, dp, dp, dp]
        L.orc_apply_M.argtypes = [ip, ctypes.c_int, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp]
        L.orc_apply_mhat.argtypes = L.orc_apply_M.argtypes
        L.orc_cg_eo.argtypes = [ip, ctypes.c_int, dp, ctypes.c_double, ctypes.c_double, dp, dp,
                                ctypes.c_double, ctypes.c_int, ctypes.c_int, dp]
        L.orc_cg_eo.restype = ctypes.c_int
        L.orc_solve.argtypes = [ip, ctypes.c_int, dp, ctypes.c_double, ctypes.c_double, dp, dp,
                                ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, dp]
        L.orc_solve.restype = ctypes.c_int
        L.orc_philox4x64_10.argtypes = [u64p, u64p, u64p]
        L.orc_z4_source.argtypes = [ip, ctypes.c_uint64, ctypes.c_uint64, dp]
        L.orc_contract.argtypes = [ip, ctypes.c_int, dp, dp, dp, dp]
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dims(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    assert d.shape == (4,) and all(int(x) >= 2 and int(x) % 2 == 0 for x in d), dims
    return d


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if shape is not None:
        a = a.reshape(shape)
    return a


def volume(dims) -> int:
    return int(np.prod([int(x) for x in dims]))


def num_threads() -> int:
    return int(lib().orc_num_threads())


# ----------------------------------------------------------------------------
# Gamma matrices and the 16 local insertions
# ----------------------------------------------------------------------------
def gamma(mu: int) -> np.ndarray:
    """gamma_{mu+1} for mu = 0..3, gamma_5 for mu = 4 (oracle's own table)."""
    out = np.zeros((4, 4, 2))
    lib().orc_gamma(int(mu), _dp(out))
    return out[..., 0] + 1j * out[..., 1]


GAMMA_NAMES = [
    "1", "g1", "g2", "g3", "g4", "g5", "g1g5", "g2g5", "g3g5", "g4g5",
    "s12", "s13", "s14", "s23", "s24", "s34",
]


def gammas16() -> np.ndarray:
    """The 16 local insertions in the order 1, g1..g4, g5, g1g5..g4g5,
    s12, s13, s14, s23, s24, s34 with s_mn = (i/2)[g_m, g_n]."""
    g = [gamma(m) for m in range(5)]
    out = [np.eye(4, dtype=np.complex128)]
    out += [g[m] for m in range(4)]
    out.append(g[4])
    out += [g[m] @ g[4] for m in range(4)]
    for m in range(4):
        for n in range(m + 1, 4):
            out.append(0.5j * (g[m] @ g[n] - g[n] @ g[m]))
    return np.array(out)


# ----------------------------------------------------------------------------
# Operators (Sec. 2.2 twisted-mass operator; Sec. 2.4 hopping term)
# ----------------------------------------------------------------------------
def dhop(dims, tbc, U, psi):
    """D_hop psi (full lattice)."""
    d = _dims(dims)
    v = volume(d)
    U = _c(U, (v, 4, 3, 3))
    psi = _c(psi, (v, 4, 3))
    out = np.empty_like(psi)
    lib().orc_dhop(_ip(d), int(tbc), _dp(U), _dp(psi), _dp(out))
    return out


def apply_M(dims, tbc, U, kappa, a, psi, dag=False):
    """M psi = psi - kappa D_hop psi + i a g5 psi (or M^dag psi)."""
    d = _dims(dims)
    v = volume(d)
    U = _c(U, (v, 4, 3, 3))
    psi = _c(psi, (v, 4, 3))
    out = np.empty_like(psi)
    lib().orc_apply_M(_ip(d), int(tbc), _dp(U), float(kappa), float(a), int(bool(dag)), _dp(psi), _dp(out))
    return out


def apply_mhat(dims, tbc, U, kappa, a, psi, dag=False):
    """Even-odd Schur operator on the even sublattice (odd sites of the
    input are ignored, odd sites of the output are zero)."""
    d = _dims(dims)
    v = volume(d)
    U = _c(U, (v, 4, 3, 3))
    psi = _c(psi, (v, 4, 3))
    out = np.empty_like(psi)
    lib().orc_apply_mhat(_ip(d), int(tbc), _dp(U), float(kappa), float(a), int(bool(dag)), _dp(psi), _dp(out))
    return out


def cg_eo(dims, tbc, U, kappa, a, bhat, tol=1e-10, max_iter=100000, fixed_iters=0):
    """CG on Mhat^dag Mhat x = Mhat^dag bhat (zero start). Returns (x, iters, relres)."""
    d = _dims(dims)
    v = volume(d)
    U = _c(U, (v, 4, 3, 3))
    b = _c(bhat, (v, 4, 3))
    x = np.empty_like(b)
    rr = np.zeros(1)
    it = lib().orc_cg_eo(_ip(d), int(tbc), _dp(U), float(kappa), float(a), _dp(b), _dp(x),
                         float(tol), int(max_iter), int(fixed_iters), _dp(rr))
    return x, int(it), float(rr[0])


def solve(dims, tbc, U, kappa, a, eta, tol=1e-10, max_iter=100000, fixed_iters=0):
    """Solve M s = eta by even-odd CG. Returns (s, iters, cg_relres, true_relres)."""
    d = _dims(dims)
    v = volume(d)
    U = _c(U, (v, 4, 3, 3))
    e = _c(eta, (v, 4, 3))
    s = np.empty_like(e)
    rr = np.zeros(1)
    tr = np.zeros(1)
    it = lib().orc_solve(_ip(d), int(tbc), _dp(U), float(kappa), float(a), _dp(e), _dp(s),
                         float(tol), int(max_iter), int(fixed_iters), _dp(rr), _dp(tr))
    return s, int(it), float(rr[0]), float(tr[0])


# ----------------------------------------------------------------------------
# Z4 noise (Sec. 2: Z_N sources, Eq. 1-2; Z4 used in this work)
# ----------------------------------------------------------------------------
def philox4x64_10(counter, key):
    c = (ctypes.c_uint64 * 4)(*[int(x) & (2**64 - 1) for x in counter])
    k = (ctypes.c_uint64 * 2)(*[int(x) & (2**64 - 1) for x in key])
    o = (ctypes.c_uint64 * 4)()
    lib().orc_philox4x64_10(c, k, o)
    return [int(o[i]) for i in range(4)]


def z4_source(dims, seed, src):
    """Z4 noise vector eta (V, 4, 3): entries ((+-1) + i(+-1))/sqrt(2)."""
    d = _dims(dims)
    v = volume(d)
    out = np.empty((v, 4, 3), dtype=np.complex128)
    lib().orc_z4_source(_ip(d), ctypes.c_uint64(int(seed)), ctypes.c_uint64(int(src)), _dp(out))
    return out


# ----------------------------------------------------------------------------
# Contractions, projection, TSM
# ----------------------------------------------------------------------------
def contract(dims, tbc, U, eta, s):
    """Spin matrices per timeslice, shape (9, T, 4, 4): kind 0 local,
    1..4 forward F^nu, 5..8 backward B^nu (nu = x, y, z, t).

    ``eta`` is any left vector: the noise for the standard estimator, the
    solution itself for the one-end trick (``loops_oet``)."""
    d = _dims(dims)
    v = volume(d)
    U = _c(U, (v, 4, 3, 3))
    e = _c(eta, (v, 4, 3))
    s = _c(s, (v, 4, 3))
    out = np.empty((9, int(d[3]), 4, 4), dtype=np.complex128)
    lib().orc_contract(_ip(d), int(tbc), _dp(U), _dp(e), _dp(s), _dp(out))
    return out


N_LOCAL = 16
N_DERIV = 64
N_SYM = 10
N_OPS = N_LOCAL + N_DERIV + N_SYM
SYM_PAIRS = [(m, n) for m in range(4) for n in range(m, 4)]


def project(P, gam=None):
    """Spin matrices (9, T, 4, 4) -> operator loops (90, T) complex.

    ``gam`` replaces the 16 insertions G (e.g. g5 G for the one-end trick).

    ops 0..15         L_G(t)      = sum_ab G_ab P_ab(t)              (local, eta^dag G s)
    ops 16+4g+nu      L^D_{G,nu}  = 1/4 [F(t) + F(t-d) - B(t) - B(t-d)],
                      d = 1 for the time direction and 0 otherwise (t-1 mod T):
                      the symmetric covariant derivative attributed to x.
    ops 80..89        O_mn = (L^D_{g_m,n} + L^D_{g_n,m}) / 2 for m <= n.
    """
    P = np.asarray(P)
    G = gammas16() if gam is None else np.asarray(gam)
    T = P.shape[1]
    out = np.zeros((N_OPS, T), dtype=np.complex128)
    proj = np.einsum("gab,ktab->gkt", G, P)  # (16, 9, T)
    out[:N_LOCAL] = proj[:, 0]
    for g in range(16):
        for nu in range(4):
            F = proj[g, 1 + nu]
            B = proj[g, 5 + nu]
            if nu == 3:
                Fs, Bs = np.roll(F, 1), np.roll(B, 1)  # value at t-1
            else:
                Fs, Bs = F, B
            out[N_LOCAL + 4 * g + nu] = 0.25 * (F + Fs - B - Bs)
    for i, (m, n) in enumerate(SYM_PAIRS):
        out[N_LOCAL + N_DERIV + i] = 0.5 * (out[N_LOCAL + 4 * (1 + m) + n] + out[N_LOCAL + 4 * (1 + n) + m])
    return out


def _svar(x, axis=0):
    n = x.shape[axis]
    if n < 2:
        return np.full(np.delete(x.shape, axis), np.nan)
    return np.var(x, axis=axis, ddof=1)


def tsm_combine(hp, lp_corr, lp_bulk):
    """Truncated-solver estimator (Sec. 2.1, Eq. estiTSM) per operator and t.

    hp, lp_corr: (N_HP, ...) loops of the correction set (same sources, HP and
    LP solves); lp_bulk: (N_LP, ...) LP-only loops of the other sources.
      est = mean(hp - lp_corr) + mean(lp_bulk)
      var = s^2(hp - lp_corr)/N_HP + s^2(lp_bulk)/N_LP, real and imaginary
            parts separately, sample variances with n-1.
    A set with no members contributes 0 to both; a set with one member makes
    its variance NaN.
    Returns (est complex, var_re, var_im).
    """
    hp = np.asarray(hp)
    lp_corr = np.asarray(lp_corr)
    lp_bulk = np.asarray(lp_bulk)
    n_hp = hp.shape[0]
    n_lp = lp_bulk.shape[0]
    shape = (hp if n_hp else lp_bulk).shape[1:]
    est = np.zeros(shape, dtype=np.complex128)
    vre = np.zeros(shape)
    vim = np.zeros(shape)
    if n_hp:
        d = hp - lp_corr
        est = est + d.mean(axis=0)
        vre = vre + _svar(d.real) / n_hp
        vim = vim + _svar(d.imag) / n_hp
    if n_lp:
        est = est + lp_bulk.mean(axis=0)
        vre = vre + _svar(lp_bulk.real) / n_lp
        vim = vim + _svar(lp_bulk.imag) / n_lp
    return est, vre, vim


def loops_tsm(dims, tbc, U, kappa, a, noise_seed, n_hp, n_lp, hp_tol=1e-10, lp_tol=1e-2,
              max_iter=100000, lp_fixed_iters=0, source_ids=None, return_raw=False):
    """The whole path on the CPU in FP64.

    Source ids 0..n_hp-1 form the correction set (HP and LP solves of the same
    eta_j), ids n_hp..n_hp+n_lp-1 the bulk set (LP only), as in Eq. estiTSM.
    LP solves are FP64 solves truncated at lp_tol (or lp_fixed_iters
    iterations); HP solves run to hp_tol.  ``source_ids`` restricts the work to
    a subset (for timing samples); then the estimator is not formed.

    Returns dict with est (90, T), var_re, var_im, per-source loops
    hp (n_hp, 90, T), lp (n_hp+n_lp, 90, T), iteration counts and timings.
    """
    T = int(dims[3])
    ids = list(range(n_hp + n_lp)) if source_ids is None else list(source_ids)
    hp_loops, lp_loops, hp_raw, lp_raw = {}, {}, {}, {}
    hp_iters, lp_iters = {}, {}
    t0 = time.perf_counter()
    for j in ids:
        eta = z4_source(dims, noise_seed, j)
        if j < n_hp:
            s, it, _, _ = solve(dims, tbc, U, kappa, a, eta, tol=hp_tol, max_iter=max_iter)
            P = contract(dims, tbc, U, eta, s)
            hp_raw[j] = P
            hp_loops[j] = project(P)
            hp_iters[j] = it
        s, it, _, _ = solve(dims, tbc, U, kappa, a, eta, tol=lp_tol, max_iter=max_iter,
                            fixed_iters=lp_fixed_iters)
        P = contract(dims, tbc, U, eta, s)
        lp_raw[j] = P
        lp_loops[j] = project(P)
        lp_iters[j] = it
    wall = time.perf_counter() - t0
    res = {"hp_iters": hp_iters, "lp_iters": lp_iters, "seconds": wall,
           "hp_loops": hp_loops, "lp_loops": lp_loops}
    if return_raw:
        res["hp_raw"] = hp_raw
        res["lp_raw"] = lp_raw
    if source_ids is None:
        hp = np.array([hp_loops[j] for j in range(n_hp)]).reshape(n_hp, N_OPS, T)
        lpc = np.array([lp_loops[j] for j in range(n_hp)]).reshape(n_hp, N_OPS, T)
        lpb = np.array([lp_loops[j] for j in range(n_hp, n_hp + n_lp)]).reshape(n_lp, N_OPS, T)
        est, vre, vim = tsm_combine(hp, lpc, lpb)
        res.update(est=est, var_re=vre, var_im=vim)
    return res


def oet_gammas():
    """Insertions of the one-end trick estimators: g5 G (isovector) and
    g5 G g5 (isoscalar) for the 16 G of ``gammas16``."""
    G = gammas16()
    g5 = G[5]
    return np.einsum("ab,gbc->gac", g5, G), np.einsum("ab,gbc,cd->gad", g5, G, g5)


def loops_oet(dims, tbc, U, kappa, a, noise_seed, n_hp, n_lp, hp_tol=1e-10, lp_tol=1e-2,
              max_iter=100000, lp_fixed_iters=0, source_ids=None, return_raw=False):
    """The one-end trick (Sec. 2.2) with the truncated solver method.

    For each source s = M_u^-1 eta (M_u = D_W + i a g5, a = 2 kappa mu):
      isovector  L^vv_X = -2 i a  s^dag g5 X s          (Eq. loopVv)
                 estimates Tr(M_u^-1 X) - Tr(M_d^-1 X)
      isoscalar  L^ws_X =  2      s^dag g5 X g5 D_W s   (Eq. loopStD)
                 estimates Tr(M_u^-1 X) + Tr(M_d^-1 X)
    with D_W = M at a = 0, for the same 90 operators X as ``loops_tsm`` (the
    spin matrices are ``contract`` with left vector s and right vector s or
    D_W s).  The sign of the isovector factor follows from
    M_u^-1 - M_d^-1 = -2 i a M_u^-1 g5 M_d^-1 and M_d^-1 = g5 (M_u^-1)^dag g5
    in this normalisation.  Same source sets and TSM combination as
    ``loops_tsm``; returns est_vv / est_ws, their variances, per-source loops
    and (optionally) the raw spin matrices raw_vv / raw_ws.
    """
    T = int(dims[3])
    gvv, gws = oet_gammas()
    ids = list(range(n_hp + n_lp)) if source_ids is None else list(source_ids)
    loops = {"hp_vv": {}, "hp_ws": {}, "lp_vv": {}, "lp_ws": {}}
    raws = {"hp_vv": {}, "hp_ws": {}, "lp_vv": {}, "lp_ws": {}}

    def one(tag, j, s):
        R = apply_M(dims, tbc, U, kappa, 0.0, s)
        Pvv = -2j * a * contract(dims, tbc, U, s, s)
        Pws = 2.0 * contract(dims, tbc, U, s, R)
        raws[tag + "_vv"][j], raws[tag + "_ws"][j] = Pvv, Pws
        loops[tag + "_vv"][j] = project(Pvv, gvv)
        loops[tag + "_ws"][j] = project(Pws, gws)

    t0 = time.perf_counter()
    for j in ids:
        eta = z4_source(dims, noise_seed, j)
        if j < n_hp:
            s, _, _, _ = solve(dims, tbc, U, kappa, a, eta, tol=hp_tol, max_iter=max_iter)
            one("hp", j, s)
        s, _, _, _ = solve(dims, tbc, U, kappa, a, eta, tol=lp_tol, max_iter=max_iter, fixed_iters=lp_fixed_iters)
        one("lp", j, s)
    res = {"seconds": time.perf_counter() - t0, "loops": loops}
    if return_raw:
        res["raw"] = raws
    if source_ids is None:
        for f in ("vv", "ws"):
            hp = np.array([loops["hp_" + f][j] for j in range(n_hp)]).reshape(n_hp, N_OPS, T)
            lpc = np.array([loops["lp_" + f][j] for j in range(n_hp)]).reshape(n_hp, N_OPS, T)
            lpb = np.array([loops["lp_" + f][j] for j in range(n_hp, n_hp + n_lp)]).reshape(n_lp, N_OPS, T)
            est, vre, vim = tsm_combine(hp, lpc, lpb)
            res.update({"est_" + f: est, "var_re_" + f: vre, "var_im_" + f: vim})
    return res


# ----------------------------------------------------------------------------
# Hopping parameter expansion (Sec. 2.4, Eq. HPE and Eq. loopHPE1)
# ----------------------------------------------------------------------------
_G5_DIAG = np.array([1.0, 1.0, -1.0, -1.0])


def apply_bh(dims, tbc, U, kappa, a, psi):
    """B H psi with M = B^-1 + H: B = (1 + i a g5)^-1 (site-diagonal) and
    H = -kappa D_hop, the hopping term of M (Sec. 2.4, Eq. HPE)."""
    h = -kappa * dhop(dims, tbc, U, psi).reshape(-1, 4, 3)
    return h / (1.0 + 1j * a * _G5_DIAG)[None, :, None]


def hpe_exact(dims, kappa, a):
    """Spin matrices (T, 4, 4) of the exact part of Eq. HPE,
    K = B - BHB + (BH)^2 B - (BH)^3 B, in the convention of ``contract``:
    P_ab(t) = sum over x in t and colour of K(x b c; x a c).

    K's site-diagonal blocks follow from the hopping structure alone (Sec. 2.4:
    independent of the gauge field for local operators):
      * B is site-diagonal: B = b0 + b5 g5, b0 = 1/(1+a^2), b5 = -i a/(1+a^2);
      * H (and (BH)^3 B) only links sites an odd number of hops apart, so their
        diagonal blocks vanish on a lattice with even extents;
      * (BH)^2 B returns to x through x+mu or x-mu:
        H(x,x+mu) B H(x+mu,x) = kappa^2 (1 - g_mu) B (1 + g_mu) U U^dag
                              = 2 kappa^2 b5 g5 (1 + g_mu),
        the backward hop gives 2 kappa^2 b5 g5 (1 - g_mu); summed over mu,
        H B H(x,x) = 16 kappa^2 b5 g5, so (BH)^2 B(x,x) = 16 kappa^2 b5 g5 B^2
        (boundary signs cancel in U U^dag).
    Hence P(t) = 3 V3 diag_b(B_b + 16 kappa^2 b5 e_b B_b^2), B_b = 1/(1 + i a e_b),
    e_b = +1, +1, -1, -1.  Valid for even extents >= 4 in every direction
    (smaller or odd extents close hops around the torus)."""
    d = _dims(dims)
    if any(int(L) < 4 or int(L) % 2 for L in d):
        raise ValueError("hpe_exact needs even extents >= 4")
    v3 = int(d[0]) * int(d[1]) * int(d[2])
    b5 = -1j * a / (1.0 + a * a)
    Bb = 1.0 / (1.0 + 1j * a * _G5_DIAG)
    k = Bb + 16.0 * kappa * kappa * b5 * _G5_DIAG * Bb * Bb
    out = np.zeros((int(d[3]), 4, 4), dtype=np.complex128)
    out[:, np.arange(4), np.arange(4)] = 3 * v3 * k
    return out


def loops_hpe(dims, tbc, U, kappa, a, noise_seed, n_hp, n_lp, hp_tol=1e-10, lp_tol=1e-2,
              max_iter=100000, lp_fixed_iters=0, source_ids=None, return_raw=False):
    """Standard and HPE loops from the same solves, with the truncated solver
    method (Sec. 2.1 and Sec. 2.4).

    For each source s = M^-1 eta: the standard spin matrices contract(eta, s)
    (as ``loops_tsm``), and the stochastic term of Eq. loopHPE1, the local
    spin matrix of contract(eta, (BH)^4 s).  The HPE estimate of the 16 local
    loops is the projection of ``hpe_exact`` plus the TSM combination of the
    stochastic term; its variance is that of the stochastic term.  Operators
    with a link (ops 16..89) have a gauge-dependent exact part and are not
    estimated with the expansion: NaN in est_hpe and its variances.
    Raw HPE spin matrices are (9, T, 4, 4) with kinds 1..8 zero.
    """
    T = int(dims[3])
    exact_ops = project(np.concatenate([hpe_exact(dims, kappa, a)[None],
                                        np.zeros((8, T, 4, 4), dtype=np.complex128)]))
    ids = list(range(n_hp + n_lp)) if source_ids is None else list(source_ids)
    loops = {"hp_std": {}, "hp_hpe": {}, "lp_std": {}, "lp_hpe": {}}
    raws = {"hp_std": {}, "hp_hpe": {}, "lp_std": {}, "lp_hpe": {}}

    def one(tag, j, eta, s):
        w = s
        for _ in range(4):
            w = apply_bh(dims, tbc, U, kappa, a, w)
        P = contract(dims, tbc, U, eta, s)
        Ph = np.zeros_like(P)
        Ph[0] = contract(dims, tbc, U, eta, w)[0]
        raws[tag + "_std"][j], raws[tag + "_hpe"][j] = P, Ph
        loops[tag + "_std"][j] = project(P)
        loops[tag + "_hpe"][j] = project(Ph)

    t0 = time.perf_counter()
    for j in ids:
        eta = z4_source(dims, noise_seed, j)
        if j < n_hp:
            s, _, _, _ = solve(dims, tbc, U, kappa, a, eta, tol=hp_tol, max_iter=max_iter)
            one("hp", j, eta, s)
        s, _, _, _ = solve(dims, tbc, U, kappa, a, eta, tol=lp_tol, max_iter=max_iter, fixed_iters=lp_fixed_iters)
        one("lp", j, eta, s)
    res = {"seconds": time.perf_counter() - t0, "loops": loops, "exact_ops": exact_ops}
    if return_raw:
        res["raw"] = raws
    if source_ids is None:
        for f in ("std", "hpe"):
            hp = np.array([loops["hp_" + f][j] for j in range(n_hp)]).reshape(n_hp, N_OPS, T)
            lpc = np.array([loops["lp_" + f][j] for j in range(n_hp)]).reshape(n_hp, N_OPS, T)
            lpb = np.array([loops["lp_" + f][j] for j in range(n_hp, n_hp + n_lp)]).reshape(n_lp, N_OPS, T)
            est, vre, vim = tsm_combine(hp, lpc, lpb)
            if f == "hpe":
                est = est + exact_ops
                est[N_LOCAL:] = np.nan
                vre[N_LOCAL:] = np.nan
                vim[N_LOCAL:] = np.nan
            res.update({"est_" + f: est, "var_re_" + f: vre, "var_im_" + f: vim})
    return res


# ----------------------------------------------------------------------------
# Time dilution and coherent sources (Sec. 2.3)
# ----------------------------------------------------------------------------
def tdil_mask(dims, spacing, phase):
    """Sites (V,) bool of the diluted source: timeslices t with t mod spacing
    == phase.  spacing = T is full time dilution (one timeslice per source);
    a smaller spacing puts T/spacing coherent timeslices, spacing apart, in one
    source."""
    d = _dims(dims)
    T = int(d[3])
    if spacing < 1 or T % spacing or not 0 <= phase < spacing:
        raise ValueError("need 1 <= spacing, T % spacing == 0 and 0 <= phase < spacing")
    v3 = int(d[0]) * int(d[1]) * int(d[2])
    t = np.repeat(np.arange(T), v3)
    return t % spacing == phase


def tdil_valid(T, spacing, phases):
    """(90, T) bool: the (operator, t) entries the diluted estimator covers.
    The noise must cover the timeslices each contraction reads it on: t for
    local and spatial-derivative loops; t-1, t and t+1 for L^D_{G,t} (its F(t-1)
    and B(t) terms) and for the symmetrised operators that contain it."""
    cov = np.zeros(T, dtype=bool)
    for p in phases:
        cov[np.arange(T) % spacing == p] = True
    wide = cov & np.roll(cov, 1) & np.roll(cov, -1)
    ok = np.zeros((N_OPS, T), dtype=bool)
    ok[:N_LOCAL] = cov
    for g in range(16):
        for nu in range(4):
            ok[N_LOCAL + 4 * g + nu] = wide if nu == 3 else cov
    for i, (m, n) in enumerate(SYM_PAIRS):
        ok[N_LOCAL + N_DERIV + i] = wide if 3 in (m, n) else cov
    return ok


def loops_tdil(dims, tbc, U, kappa, a, noise_seed, n_hp, n_lp, spacing, phases=None, hpe=False, hp_tol=1e-10,
               lp_tol=1e-2, max_iter=100000, lp_fixed_iters=0, source_ids=None, return_raw=False):
    """Time-diluted loops (Sec. 2.3) with the truncated solver method.

    Noise vector r (``z4_source`` id r) is split into the sources
    eta_{r,p} = eta_r on the timeslices of ``tdil_mask(spacing, p)`` for p in
    ``phases`` (default: all spacing phases); each is solved (HP and LP for
    r < n_hp, LP only above), and the loops of noise vector r are the sums over
    its phases of contract(eta_{r,p}, s_{r,p}): a source contributes to the
    signal only on its own timeslices.  With ``hpe`` the same is done for the
    stochastic term of Eq. loopHPE1 (eta_{r,p}^dag G (BH)^4 s_{r,p}) and the
    exact part is added as in ``loops_hpe``.  TSM over noise vectors as in
    ``loops_tsm``; entries outside ``tdil_valid`` are NaN.
    """
    d = _dims(dims)
    T = int(d[3])
    phases = list(range(spacing)) if phases is None else [int(p) for p in phases]
    masks = {p: tdil_mask(dims, spacing, p) for p in phases}
    valid = tdil_valid(T, spacing, phases)
    ids = list(range(n_hp + n_lp)) if source_ids is None else list(source_ids)
    tags = ("std", "hpe") if hpe else ("std",)
    raws = {f"{h}_{f}": {} for h in ("hp", "lp") for f in tags}

    def add(tag, j, eta, s):
        P = contract(dims, tbc, U, eta, s)
        acc = raws[tag + "_std"]
        acc[j] = acc.get(j, 0) + P
        if hpe:
            w = s
            for _ in range(4):
                w = apply_bh(dims, tbc, U, kappa, a, w)
            Ph = np.zeros_like(P)
            Ph[0] = contract(dims, tbc, U, eta, w)[0]
            acch = raws[tag + "_hpe"]
            acch[j] = acch.get(j, 0) + Ph

    t0 = time.perf_counter()
    for j in ids:
        eta_full = z4_source(dims, noise_seed, j)
        for p in phases:
            eta = eta_full * masks[p][:, None, None]
            if j < n_hp:
                s, _, _, _ = solve(dims, tbc, U, kappa, a, eta, tol=hp_tol, max_iter=max_iter)
                add("hp", j, eta, s)
            s, _, _, _ = solve(dims, tbc, U, kappa, a, eta, tol=lp_tol, max_iter=max_iter,
                               fixed_iters=lp_fixed_iters)
            add("lp", j, eta, s)
    loops = {k: {j: project(v) for j, v in r.items()} for k, r in raws.items()}
    res = {"seconds": time.perf_counter() - t0, "loops": loops, "valid": valid}
    if return_raw:
        res["raw"] = raws
    if source_ids is None:
        exact_ops = None
        if hpe:
            exact_ops = project(np.concatenate([hpe_exact(dims, kappa, a)[None],
                                                np.zeros((8, T, 4, 4), dtype=np.complex128)]))
        for f in tags:
            hp = np.array([loops["hp_" + f][j] for j in range(n_hp)]).reshape(n_hp, N_OPS, T)
            lpc = np.array([loops["lp_" + f][j] for j in range(n_hp)]).reshape(n_hp, N_OPS, T)
            lpb = np.array([loops["lp_" + f][j] for j in range(n_hp, n_hp + n_lp)]).reshape(n_lp, N_OPS, T)
            est, vre, vim = tsm_combine(hp, lpc, lpb)
            ok = valid.copy()
            if f == "hpe":
                est = est + exact_ops
                ok[N_LOCAL:] = False
            est[~ok] = np.nan
            vre[~ok] = np.nan
            vim[~ok] = np.nan
            res.update({"est_" + f: est, "var_re_" + f: vre, "var_im_" + f: vim})
    return res
