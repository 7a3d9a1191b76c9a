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
