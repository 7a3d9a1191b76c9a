"""Helpers for the GPU parity tests (import only inside gpu-marked tests)."""
from __future__ import annotations

import numpy as np


def torch_mod():
    import torch

    assert torch.cuda.is_available(), "GPU test needs a ROCm device"
    return torch


_CTX = {}


def context():
    from paper_1401_6749_amd import tm

    if "ctx" not in _CTX:
        _CTX["ctx"] = tm.tm_create(0)
    return _CTX["ctx"]


def load(dims, U, tbc=-1, precs=("f32", "f16", "bf16")):
    from paper_1401_6749_amd import tm

    return tm.tm_load_gauge(context(), dims, U, tbc, precs)


def to_dev(a):
    from paper_1401_6749_amd import tm

    return tm.canonical_to_torch(a)


def from_dev(t):
    from paper_1401_6749_amd import tm

    return tm.torch_to_canonical(t)


def apply_op(g, op, kappa, a, prec, psi, dims):
    """Run tm_dslash on nrhs canonical spinors psi (nrhs, V, 4, 3) -> (nrhs, V, 4, 3)."""
    torch = torch_mod()
    from paper_1401_6749_amd import tm

    ctx = context()
    psi = np.asarray(psi).reshape(-1, int(np.prod(dims)), 4, 3)
    nrhs = psi.shape[0]
    fb = tm.tm_field_bytes(g, prec, full=True)
    hb = fb // 2
    fin = torch.empty(nrhs * fb, dtype=torch.uint8, device="cuda")
    tm.tm_field_import(ctx, g, prec, nrhs, to_dev(psi), fin)
    full = op in ("hop", "m", "mdag", "bh")
    if full:
        fout = torch.zeros_like(fin)
        tm.tm_dslash(ctx, g, op, kappa, a, prec, nrhs, fin, fout)
    else:
        ein = fin.view(nrhs, 2, hb)[:, 0].contiguous()
        eout = torch.zeros_like(ein)
        tm.tm_dslash(ctx, g, op, kappa, a, prec, nrhs, ein, eout)
        fout = torch.zeros_like(fin)
        fout.view(nrhs, 2, hb)[:, 0] = eout
    canon = torch.zeros(nrhs, int(np.prod(dims)), 4, 3, 2, dtype=torch.float64, device="cuda")
    tm.tm_field_export(ctx, g, prec, nrhs, fout, canon)
    torch.cuda.synchronize()
    return from_dev(canon).reshape(nrhs, -1, 4, 3)


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


# operator classes of the 90 projected loops: 16 local, 64 one-derivative
# L^D_{G,nu}, 10 symmetrised g_mu D_nu
OP_CLASSES = {"local": slice(0, 16), "deriv": slice(16, 80), "sym": slice(80, 90)}


def op_class_errors(raw_test, raw_ref, oracle):
    """Relative error ||L_test - L_ref|| / ||L_ref|| per operator class, over
    the class's operators and all timeslices, of the loops projected (by the
    oracle) from spin matrices (9, T, 4, 4)."""
    a = oracle.project(np.asarray(raw_test))
    b = oracle.project(np.asarray(raw_ref))
    return {k: relerr(a[s], b[s]) for k, s in OP_CLASSES.items()}


def assert_classes(raw_test, raw_ref, oracle, tol, what=""):
    """Every operator class within tol (a whole small class cannot hide in
    the norm of the larger ones)."""
    e = op_class_errors(raw_test, raw_ref, oracle)
    for k, v in e.items():
        assert v < tol, (what, k, v, e)
    return e
