"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds input generators only: random SU(3) gauge fields shaped
like the paper's lattices, random spinors and random gauge transformations.
It contains none of the method's arithmetic (no Dirac operator, no solver, no
noise, no contraction), so both the HIP path and the CPU oracle may use it.

The paper measures on a physical Nf=2+1+1 twisted-mass ensemble (32^3 x 64,
Sec. 3), which is not available; the synthetic links below stand in for it:
U = exp(i * eps * sum_a c_a lambda_a / 2) with c_a ~ N(0, 1), one independent
draw per link, projected to det U = 1.

Canonical host layouts (complex128, C order):
  gauge   [V][4][3][3]  with V = Lx*Ly*Lz*Lt, site lex = x + Lx*(y + Ly*(z + Lz*t)),
                         direction index 0..3 = x, y, z, t
  spinor  [V][4][3]     spin-major, colour-minor
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gell_mann",
    "gauge_field",
    "unit_gauge",
    "random_su3",
    "random_spinor",
    "volume",
]


def volume(dims) -> int:
    lx, ly, lz, lt = (int(d) for d in dims)
    return lx * ly * lz * lt


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3) complex128."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3)
    lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def _expi_hermitian(h: np.ndarray) -> np.ndarray:
    """exp(i h) for a stack of Hermitian 3x3 matrices, via eigh; det fixed to 1."""
    w, v = np.linalg.eigh(h)
    u = np.einsum("...ik,...k,...jk->...ij", v, np.exp(1j * w), v.conj())
    det = np.linalg.det(u)
    u /= (det ** (1.0 / 3.0))[..., None, None]
    return u


def gauge_field(dims, seed: int, eps: float = 0.4) -> np.ndarray:
    """Random near-unit SU(3) links, shape (V, 4, 3, 3) complex128.

    Draws c ~ N(0,1) with numpy's default_rng(seed) in the shape
    (Lt, Lz, Ly, Lx, 4, 8), i.e. in lexicographic site order, and builds
    U = exp(i eps sum_a c_a lambda_a / 2) per link.  Generated one timeslice
    at a time so that the 32^3 x 64 field stays within a few GB of host memory.
    """
    lx, ly, lz, lt = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    lam = gell_mann() / 2.0
    v3 = lx * ly * lz
    out = np.empty((lt * v3, 4, 3, 3), dtype=np.complex128)
    for t in range(lt):
        c = rng.standard_normal((v3, 4, 8))
        h = eps * np.einsum("sma,aij->smij", c, lam)
        out[t * v3 : (t + 1) * v3] = _expi_hermitian(h)
    return out


def unit_gauge(dims) -> np.ndarray:
    """Free field: every link the 3x3 identity."""
    v = volume(dims)
    u = np.zeros((v, 4, 3, 3), dtype=np.complex128)
    u[:, :, 0, 0] = u[:, :, 1, 1] = u[:, :, 2, 2] = 1.0
    return u


def random_su3(n: int, seed: int, eps: float = 3.0) -> np.ndarray:
    """n random SU(3) matrices (shape (n, 3, 3)); large eps spreads them widely."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((n, 8))
    h = eps * np.einsum("na,aij->nij", c, gell_mann() / 2.0)
    return _expi_hermitian(h)


def random_spinor(dims, seed: int) -> np.ndarray:
    """Gaussian complex spinor field, shape (V, 4, 3) complex128."""
    rng = np.random.default_rng(seed)
    v = volume(dims)
    return (rng.standard_normal((v, 4, 3)) + 1j * rng.standard_normal((v, 4, 3))) / np.sqrt(2.0)
