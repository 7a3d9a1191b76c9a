"""Pins of the oracle's counter-based Z4 noise (Sec. 2, Eq. 1-2)."""
import numpy as np
import pytest


def test_philox_matches_numpy_library(oracle):
    """I10: numpy's Philox bit generator is Philox4x64-10; it increments the
    counter before producing its first block, so counter c there yields the
    block at c + 1 here."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        key = [int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        ctr[0] += 1  # keep the pre-increment from carrying
        want = np.random.Philox(counter=[ctr[0] - 1] + ctr[1:], key=key).random_raw(4)
        assert oracle.philox4x64_10(ctr, key) == [int(x) for x in want]


def test_z4_entries_and_bit_mapping(oracle):
    dims = (4, 2, 2, 2)
    seed, src = 1234, 7
    eta = oracle.z4_source(dims, seed, src)
    h = np.sqrt(0.5)  # correctly rounded 2^-1/2
    assert np.all(np.isin(eta.real, [h, -h])) and np.all(np.isin(eta.imag, [h, -h]))
    # I11: |eta_i|^2 = 1 up to the rounding of 2^-1/2
    assert np.allclose(np.abs(eta) ** 2, 1.0, rtol=0, atol=4.5e-16)
    # mapping: component k of site lex uses bits 2k, 2k+1 of word 0 of
    # Philox(counter=(lex, src, 0, 0), key=(seed, 0))
    for lex in (0, 5, 31):
        w0 = oracle.philox4x64_10([lex, src, 0, 0], [seed, 0])[0]
        flat = eta[lex].reshape(12)
        for k in range(12):
            re = -h if (w0 >> (2 * k)) & 1 else h
            im = -h if (w0 >> (2 * k + 1)) & 1 else h
            assert flat[k] == re + 1j * im


def test_z4_noise_identities(oracle):
    """Eq. 1: the source mean is O(1/sqrt(N)); Eq. 2: (1/N) sum eta eta^dag
    = I + O(1/sqrt(N)), the diagonal being exactly 1."""
    dims = (2, 2, 2, 2)
    n = 12 * 16
    N = 400
    acc = np.zeros((n, n), dtype=np.complex128)
    mean = np.zeros(n, dtype=np.complex128)
    for j in range(N):
        e = oracle.z4_source(dims, 42, j).reshape(-1)
        acc += np.outer(e, e.conj())
        mean += e
    acc /= N
    mean /= N
    assert np.allclose(np.diag(acc), 1.0, atol=1e-14)
    off = acc[~np.eye(n, dtype=bool)]
    # each off-diagonal entry has mean 0 and variance 1/N
    z = np.abs(off) * np.sqrt(N)
    assert np.mean(z**2) == pytest.approx(1.0, rel=0.05)
    assert np.abs(off).max() < 6 / np.sqrt(N)
    assert np.mean(np.abs(mean) ** 2 * N) == pytest.approx(1.0, rel=0.2)


def test_z4_independent_of_volume_and_ids(oracle):
    """Counter-based: eta at a site depends only on (lex, src, seed), so two
    different lattices agree on their common lex range and sources differ."""
    a = oracle.z4_source((4, 4, 4, 4), 9, 3).reshape(-1, 12)
    b = oracle.z4_source((4, 4, 4, 8), 9, 3).reshape(-1, 12)
    assert np.array_equal(a, b[: a.shape[0]])
    c = oracle.z4_source((4, 4, 4, 4), 9, 4).reshape(-1, 12)
    assert not np.array_equal(a, c)
