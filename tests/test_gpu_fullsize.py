"""Parity at the benchmark's full size, 32^3 x 64 with its gauge seed, in the
launch configuration bench.py times: 12 right-hand sides per launch laid out
with the solver's slot pitch (the timeslice-walk kernels), the FP64 hopping
term, Z4 codes, and loop sources in matched-iteration mode.  The oracle
computes whole fields (its Dslash) or a few sampled sources (its solves)."""
import numpy as np
import pytest

from paper_1401_6749_amd import inputs
from tests import gpu_util as GU

pytestmark = pytest.mark.gpu

DIMS = (32, 32, 32, 64)
KAPPA, A = 0.1636, 0.0033


def slot_pitch(nbytes):
    return (nbytes + 255) // 256 * 256 + 17 * 256


@pytest.fixture(scope="module")
def big():
    from paper_1401_6749_amd import tm

    U = inputs.gauge_field(DIMS, 4)
    g = GU.load(DIMS, U)
    yield U, g
    tm.tm_free_gauge(GU.context(), g)


def _hop_12(g, prec, psis):
    """tm_dslash_ex hop on 12 right-hand sides at the solver's slot pitch;
    psis: two canonical spinors used alternately."""
    torch = GU.torch_mod()
    from paper_1401_6749_amd import tm

    ctx = GU.context()
    nrhs = 12
    fb = tm.tm_field_bytes(g, prec, True)
    pitch = slot_pitch(fb)
    fin = torch.zeros(nrhs * pitch, dtype=torch.uint8, device="cuda")
    dev = [GU.to_dev(p[None]) for p in psis]
    for r in range(nrhs):
        tm.tm_field_import(ctx, g, prec, 1, dev[r % 2], fin[r * pitch:r * pitch + fb])
    fout = torch.zeros_like(fin)
    tm.tm_dslash_ex(ctx, g, "hop", KAPPA, A, prec, nrhs, fin, pitch, fout, pitch)
    V = int(np.prod(DIMS))
    canon = torch.zeros(1, V, 4, 3, 2, dtype=torch.float64, device="cuda")

    def export(r):
        tm.tm_field_export(ctx, g, prec, 1, fout[r * pitch:r * pitch + fb], canon)
        torch.cuda.synchronize()
        return GU.from_dev(canon).reshape(V, 4, 3)

    return export


def test_fullsize_hop_12rhs(oracle, big):
    """FP64, FP32, FP16 and BF16 hop at 32^3x64, 12 RHS per launch: RHS against
    the oracle's FP64 hop of the same input (FP64 <= 1e-14; FP32 / FP16 / BF16
    within their storage rounding, as on the small lattices)."""
    U, g = big
    psis = [inputs.random_spinor(DIMS, 21), inputs.random_spinor(DIMS, 22)]
    want = [oracle.dhop(DIMS, -1, U, p) for p in psis]
    for prec, tol, rhs in (("f64", 1e-14, (0, 1, 11)), ("f32", 2e-6, (0, 11)), ("f16", 3e-3, range(12)),
                           ("bf16", 2e-2, (0, 5, 11))):
        export = _hop_12(g, prec, psis)
        first = {}
        for r in rhs:
            got = export(r)
            assert GU.relerr(got, want[r % 2]) < tol, (prec, r)
            # no right-hand side sees another's data: equal inputs give equal bits
            if r % 2 in first:
                assert np.array_equal(got, first[r % 2]), (prec, r)
            else:
                first[r % 2] = got


def test_fullsize_z4_codes(oracle):
    torch = GU.torch_mod()
    from paper_1401_6749_amd import tm

    ctx = GU.context()
    V = int(np.prod(DIMS))
    for seed, src in [(104, 0), (104, 1047)]:
        out = torch.empty(V, 4, 3, 2, dtype=torch.float64, device="cuda")
        tm.tm_z4_source(ctx, DIMS, seed, src, out)
        torch.cuda.synchronize()
        got = GU.from_dev(out).reshape(V, 4, 3)
        assert np.array_equal(got.view(np.float64), oracle.z4_source(DIMS, seed, src).view(np.float64))


def test_fullsize_loops_matched_iterations(oracle, big):
    """Loop spin matrices of sampled sources at 32^3x64, five CG iterations
    each: the FP64 path to 1e-10 of the oracle; the FP16 and BF16 LP paths
    (12 sources in one batch, the bench's launch shape) within their storage
    rounding, for every operator class (local, one-derivative, symmetrised)."""
    from paper_1401_6749_amd import tm

    U, g = big
    ctx = GU.context()
    lt = DIMS[3]
    ref = oracle.loops_tsm(DIMS, -1, U, KAPPA, A, 104, 0, 12, lp_fixed_iters=5, source_ids=[0, 11],
                           return_raw=True)
    P64 = tm.tsm_params(KAPPA, A, 104, 0, 12, lp=tm.solver_params("f64", fixed_iters=5), batch=12)
    r64 = tm.tm_loops_tsm(ctx, g, P64, lt, want_raw=True)
    for j in (0, 11):
        assert GU.relerr(r64["raw_lp"][j], ref["lp_raw"][j]) < 1e-10, j
    for half, tol in (("f16", 5e-3), ("bf16", 3e-2)):
        P = tm.tsm_params(KAPPA, A, 104, 0, 12, lp=tm.solver_params("lp", fixed_iters=5, half=half), batch=12)
        r = tm.tm_loops_tsm(ctx, g, P, lt, want_raw=True)
        for j in (0, 11):
            assert GU.relerr(r["raw_lp"][j], ref["lp_raw"][j]) < tol, (half, j)
            GU.assert_classes(r["raw_lp"][j], ref["lp_raw"][j], oracle, tol, (half, j))


def test_fullsize_loops_oet_f64(oracle, big):
    """One-end trick spin matrices of one source at 32^3x64 (FP64, five
    matched iterations) against the oracle, both flavours, to 1e-10."""
    from paper_1401_6749_amd import tm

    U, g = big
    ctx = GU.context()
    ref = oracle.loops_oet(DIMS, -1, U, KAPPA, A, 104, 0, 1, lp_fixed_iters=5, source_ids=[0], return_raw=True)
    P = tm.tsm_params(KAPPA, A, 104, 0, 1, lp=tm.solver_params("f64", fixed_iters=5), batch=1)
    r = tm.tm_loops_oet(ctx, g, P, DIMS[3], want_raw=True)
    for f in ("vv", "ws"):
        assert GU.relerr(r[f"raw_{f}_lp"][0], ref["raw"]["lp_" + f][0]) < 1e-10, f


def test_fullsize_loops_hpe(oracle, big):
    """Hopping parameter expansion at 32^3x64 (five matched iterations): the
    FP64 path's eta^dag (BH)^4 s local spin matrices to 1e-10 of the oracle,
    and the FP16 LP path (12 sources per batch, the bench's launch shape)
    within its storage rounding, on sampled sources."""
    from paper_1401_6749_amd import tm

    U, g = big
    ctx = GU.context()
    ref = oracle.loops_hpe(DIMS, -1, U, KAPPA, A, 104, 0, 12, lp_fixed_iters=5, source_ids=[0, 11],
                           return_raw=True)
    P64 = tm.tsm_params(KAPPA, A, 104, 0, 12, lp=tm.solver_params("f64", fixed_iters=5), batch=12)
    r64 = tm.tm_loops_hpe(ctx, g, P64, DIMS[3], want_raw=True)
    P16 = tm.tsm_params(KAPPA, A, 104, 0, 12, lp=tm.solver_params("lp", fixed_iters=5, half="f16"), batch=12)
    r16 = tm.tm_loops_hpe(ctx, g, P16, DIMS[3], want_raw=True)
    for j in (0, 11):
        assert GU.relerr(r64["raw_hpe_lp"][j], ref["raw"]["lp_hpe"][j]) < 1e-10, j
        assert GU.relerr(r16["raw_hpe_lp"][j], ref["raw"]["lp_hpe"][j]) < 5e-3, j


def test_fullsize_loops_tdil_one_timeslice(oracle, big):
    """Full time dilution at one insertion timeslice (t = 8 of 64, one solve
    per noise vector) at 32^3x64, FP16 LP in a batch of 12 with five
    iterations: sampled noise vectors against the oracle; only t = 8 is
    covered for the local loops."""
    from paper_1401_6749_amd import tm

    U, g = big
    ctx = GU.context()
    ref = oracle.loops_tdil(DIMS, -1, U, KAPPA, A, 105, 0, 12, 64, phases=[8], lp_fixed_iters=5,
                            source_ids=[0, 11], return_raw=True)
    P16 = tm.tsm_params(KAPPA, A, 105, 0, 12, lp=tm.solver_params("lp", fixed_iters=5, half="f16"), batch=12)
    r = tm.tm_loops_tdil(ctx, g, P16, DIMS[3], 64, phases=[8], want_raw=True)
    for j in (0, 11):
        assert GU.relerr(r["raw_std_lp"][j][0], ref["raw"]["lp_std"][j][0]) < 5e-3, j
    est = r["est_std"]
    assert np.isfinite(est[:16, 8]).all() and np.isnan(est[:16, 7]).all() and np.isnan(est[:16, 9]).all()


def test_fullsize_contract_12(oracle, big):
    """tm_contract at 32^3x64 with 12 FP32 solutions at the solver's slot
    pitch (the LP harvest's contraction shape the bench times) and one FP64
    solution: sampled sources against the oracle's contraction."""
    torch = GU.torch_mod()
    from paper_1401_6749_amd import tm

    U, g = big
    ctx = GU.context()
    lt = DIMS[3]
    psis = [inputs.random_spinor(DIMS, 31), inputs.random_spinor(DIMS, 32)]
    dev = [GU.to_dev(p[None]) for p in psis]
    ids = list(range(100, 112))
    for prec, n, tol in (("f32", 12, 2e-6), ("f64", 1, 1e-13)):
        fb = tm.tm_field_bytes(g, prec, True)
        pitch = slot_pitch(fb)
        fin = torch.zeros(n * pitch, dtype=torch.uint8, device="cuda")
        for r in range(n):
            tm.tm_field_import(ctx, g, prec, 1, dev[r % 2], fin[r * pitch:r * pitch + fb])
        raw = torch.zeros(n * 9 * lt * 32, dtype=torch.float64, device="cuda")
        tm.tm_contract(ctx, g, prec, n, fin, pitch, 104, ids[:n], raw)
        torch.cuda.synchronize()
        got = raw.cpu().numpy().reshape(n, 9, lt, 4, 4, 2)
        del fin, raw
        for r in sorted({0, n - 1}):
            want = oracle.contract(DIMS, -1, U, oracle.z4_source(DIMS, 104, ids[r]), psis[r % 2])
            gr = got[r][..., 0] + 1j * got[r][..., 1]
            assert GU.relerr(gr, want) < tol, (prec, r, GU.relerr(gr, want))
