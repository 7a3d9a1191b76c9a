"""tm_cg_update, the direction update that ends each CG iteration (x += alpha p,
then p = r + beta p, both from the old p), on caller fields through the C ABI.
The expected fields are the update written out in numpy (FP64) on the stored
inputs read back from the device, so only the kernel's arithmetic and the
rounding of its outputs to the storage format are measured: FP64 to rounding,
FP32/FP16/BF16 within their storage precision.  The odd half of each field,
and x when it is not passed, stay bit for bit as they were; bad arguments are
rejected before anything runs."""
import numpy as np
import pytest

from paper_1401_6749_amd import inputs
from tests import gpu_util as GU

pytestmark = pytest.mark.gpu

DIMS = (8, 6, 4, 10)  # V/2 = 960: not a multiple of the 256-site block
TOL = {"f64": 1e-15, "f32": 1e-6, "f16": 2e-3, "bf16": 1.5e-2}
ALPHA = [0.7, -1.3, 0.25]
BETA = [0.1, 0.9, -0.5]


def _even(dims):
    t, z, y, x = np.indices(dims[::-1]).reshape(4, -1)  # lexicographic, x fastest
    return (x + y + z + t) % 2 == 0


def _fields(torch, tm, ctx, g, prec, seeds):
    """Device fields (one allocation, field i at i * fb) and their stored values."""
    V = int(np.prod(DIMS))
    psi = np.stack([inputs.random_spinor(DIMS, s) for s in seeds])
    fb = tm.tm_field_bytes(g, prec, full=True)
    dev = torch.empty(len(seeds) * fb, dtype=torch.uint8, device="cuda")
    tm.tm_field_import(ctx, g, prec, len(seeds), GU.to_dev(psi), dev)
    return dev, _read(torch, tm, ctx, g, prec, dev, len(seeds)), fb, V


def _read(torch, tm, ctx, g, prec, dev, n):
    V = int(np.prod(DIMS))
    out = torch.empty(n, V, 4, 3, 2, dtype=torch.float64, device="cuda")
    tm.tm_field_export(ctx, g, prec, n, dev, out)
    torch.cuda.synchronize()
    return GU.from_dev(out).reshape(n, V, 4, 3)


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_cg_update_against_formula(prec):
    torch = GU.torch_mod()
    from paper_1401_6749_amd import tm

    ctx = GU.context()
    U = inputs.gauge_field(DIMS, seed=3)
    g = GU.load(DIMS, U)
    ev = _even(DIMS)
    p, p0, fb, _ = _fields(torch, tm, ctx, g, prec, [11, 12, 13])
    r, r0, _, _ = _fields(torch, tm, ctx, g, prec, [21, 22, 23])
    x, x0, _, _ = _fields(torch, tm, ctx, g, prec, [31, 32, 33])
    tm.tm_cg_update(ctx, g, prec, 3, p, r, x, fb, ALPHA, BETA)
    p1, r1, x1 = (_read(torch, tm, ctx, g, prec, f, 3) for f in (p, r, x))
    for i in range(3):
        want_x = x0[i][ev] + ALPHA[i] * p0[i][ev]
        want_p = r0[i][ev] + BETA[i] * p0[i][ev]
        assert GU.relerr(x1[i][ev], want_x) < TOL[prec], (prec, i, "x")
        assert GU.relerr(p1[i][ev], want_p) < TOL[prec], (prec, i, "p")
        # the odd halves and r are untouched
        for a, b in ((p1, p0), (x1, x0), (r1, r0)):
            assert np.array_equal(a[i][~ev], b[i][~ev]), (prec, i)
        assert np.array_equal(r1[i], r0[i]), (prec, i)

    # without x: only p = r + beta p; x keeps its bits
    tm.tm_cg_update(ctx, g, prec, 3, p, r, None, fb, ALPHA, BETA)
    p2, x2 = (_read(torch, tm, ctx, g, prec, f, 3) for f in (p, x))
    assert np.array_equal(x2, x1)
    for i in range(3):
        assert GU.relerr(p2[i][ev], r1[i][ev] + BETA[i] * p1[i][ev]) < TOL[prec], (prec, i)
    tm.tm_free_gauge(ctx, g)


def test_cg_update_one_rhs_equals_batch():
    """Slot i of a three-field call has the bits of a one-field call on it."""
    torch = GU.torch_mod()
    from paper_1401_6749_amd import tm

    ctx = GU.context()
    g = GU.load(DIMS, inputs.gauge_field(DIMS, seed=3))
    for prec in ("f32", "f16"):
        p, _, fb, _ = _fields(torch, tm, ctx, g, prec, [11, 12, 13])
        r, _, _, _ = _fields(torch, tm, ctx, g, prec, [21, 22, 23])
        x, _, _, _ = _fields(torch, tm, ctx, g, prec, [31, 32, 33])
        p_one, x_one = p[fb:2 * fb].clone(), x[fb:2 * fb].clone()
        tm.tm_cg_update(ctx, g, prec, 3, p, r, x, fb, ALPHA, BETA)
        tm.tm_cg_update(ctx, g, prec, 1, p_one, r[fb:2 * fb], x_one, fb, ALPHA[1:2], BETA[1:2])
        torch.cuda.synchronize()
        assert torch.equal(p[fb:2 * fb], p_one) and torch.equal(x[fb:2 * fb], x_one), prec
    tm.tm_free_gauge(ctx, g)


def test_cg_update_rejects_bad_arguments():
    torch = GU.torch_mod()
    from paper_1401_6749_amd import tm

    ctx = GU.context()
    g = GU.load(DIMS, inputs.gauge_field(DIMS, seed=3))
    p, p0, fb, _ = _fields(torch, tm, ctx, g, "f32", [11, 12])
    r, _, _, _ = _fields(torch, tm, ctx, g, "f32", [21, 22])
    x, x0, _, _ = _fields(torch, tm, ctx, g, "f32", [31, 32])
    hb = fb // 2
    bad = [
        dict(nrhs=0),
        dict(nrhs=17),
        dict(stride=hb - 16),                        # less than one even-half field
        dict(stride=fb + 8),                         # not a multiple of 16
        dict(r=p[hb:]),                              # r overlaps p
        dict(x=r),                                   # x is r
        dict(alpha=[np.nan, 0.1]),
        dict(beta=[0.1, np.inf]),
    ]
    for kw in bad:
        a = dict(nrhs=2, p=p, r=r, x=x, stride=fb, alpha=[0.5, 0.5], beta=[0.5, 0.5])
        a.update(kw)
        n = a["nrhs"]
        al = (list(a["alpha"]) + [0.0] * 17)[:n]
        be = (list(a["beta"]) + [0.0] * 17)[:n]
        rc = tm.tm_cg_update(ctx, g, "f32", n, a["p"], a["r"], a["x"], a["stride"], al, be, check=False)
        assert rc == tm.TM_ERR_ARG, kw
    torch.cuda.synchronize()
    assert np.array_equal(_read(torch, tm, ctx, g, "f32", p, 2), p0)
    assert np.array_equal(_read(torch, tm, ctx, g, "f32", x, 2), x0)
    tm.tm_free_gauge(ctx, g)
