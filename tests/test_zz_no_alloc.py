"""tm_dslash_noalloc (the entry point for callers that cannot allocate)
against tm_dslash_ex: the same bits on two calls in a row, the second with a
smaller input, no device memory taken from the context, and a request beyond
the fixed scratch rejected."""
import numpy as np
import pytest

from paper_1401_6749_amd import inputs
from tests import gpu_util as GU

pytestmark = pytest.mark.gpu


def _fields(torch, tm, ctx, g, dims, prec, nrhs, seed, full):
    fb = tm.tm_field_bytes(g, prec, True)
    hb = fb // 2
    psi = np.stack([inputs.random_spinor(dims, seed + r) for r in range(nrhs)])
    fin = torch.empty(nrhs * fb, dtype=torch.uint8, device="cuda")
    tm.tm_field_import(ctx, g, prec, nrhs, GU.to_dev(psi), fin)
    if full:
        return fin, fb
    ein = fin.view(nrhs, 2, hb)[:, 0].contiguous().view(-1)
    return ein, hb


def _both(torch, tm, ctx, g, dims, op, prec, nrhs, seed):
    full = op in ("hop", "m", "mdag", "bh")
    inp, stride = _fields(torch, tm, ctx, g, dims, prec, nrhs, seed, full)
    want = torch.zeros_like(inp)
    got = torch.full_like(inp, 0x5A)
    tm.tm_dslash_ex(ctx, g, op, 0.1636, 0.0033, prec, nrhs, inp, stride, want, stride)
    used0 = tm.tm_memory_usage(ctx)[0]
    tm.tm_dslash_noalloc(ctx, g, op, 0.1636, 0.0033, prec, nrhs, inp, stride, got, stride)
    torch.cuda.synchronize()
    assert tm.tm_memory_usage(ctx)[0] == used0
    return got, want


def test_noalloc_equals_dslash_ex():
    torch = GU.torch_mod()
    from paper_1401_6749_amd import tm

    ctx = tm.tm_create(0)
    try:
        dA, dB = (8, 6, 4, 10), (4, 4, 4, 4)
        gA = tm.tm_load_gauge(ctx, dA, inputs.gauge_field(dA, 3), -1, ("f32", "f16"))
        gB = tm.tm_load_gauge(ctx, dB, inputs.gauge_field(dB, 4), -1, ("f32",))
        # first call: the largest temporaries of the test (two half fields per RHS)
        got, want = _both(torch, tm, ctx, gA, dA, "mhat_dag_mhat", "f64", 3, 10)
        assert torch.equal(got, want)
        # second call, smaller input: another lattice, precision and operator
        got, want = _both(torch, tm, ctx, gB, dB, "mhat", "f32", 1, 20)
        assert torch.equal(got, want)
        # the other operators in a row
        for op, prec, n in (("mhat_dag", "f16", 2), ("hop", "f64", 2), ("m", "f32", 1)):
            got, want = _both(torch, tm, ctx, gA, dA, op, prec, n, 30)
            assert torch.equal(got, want), (op, prec)
        # temporaries beyond the fixed scratch: rejected, nothing launched
        dC = (16, 16, 16, 32)
        gC = tm.tm_load_gauge(ctx, dC, inputs.gauge_field(dC, 5), -1, ())
        hb = tm.tm_field_bytes(gC, "f64", False)
        assert 2 * 3 * hb > (64 << 20)
        fin = torch.zeros(3 * hb, dtype=torch.uint8, device="cuda")
        fout = torch.zeros_like(fin)
        rc = tm.tm_dslash_noalloc(ctx, gC, "mhat_dag_mhat", 0.12, 0.01, "f64", 3, fin, hb, fout, hb, check=False)
        assert rc == tm.TM_ERR_ARG
        assert "scratch" in tm.tm_last_error(ctx)
        torch.cuda.synchronize()
        assert int(fout.count_nonzero()) == 0
        for g in (gA, gB, gC):
            tm.tm_free_gauge(ctx, g)
    finally:
        tm.tm_destroy(ctx)
