"""Thin Python binding of libtm (ctypes).  Argument marshalling only: every
step of the computation runs in the library's HIP kernels.

Functions carry the C names (``tm_create``, ``tm_load_gauge``, ``tm_dslash``,
``tm_cg_solve``, ``tm_z4_source``, ``tm_loops_tsm`` ...).  Device buffers
are torch tensors on the context's GPU (or raw integer addresses); device
memory of the library itself comes from torch's caching allocator through
the allocator callbacks of ``tm_create``.  There is no fallback: importing
this module without the built library raises ImportError.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libtm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libtm.so is not built ({LIB_PATH}); run `python -c 'import __graft_entry__ as g; g.build()'`"
    )

# torch first: its HIP runtime (same soname as the one libtm links) must be
# the only one in the process, so device pointers, streams and the caching
# allocator are shared with the library.
import torch  # noqa: E402

_lib = ctypes.CDLL(LIB_PATH)


def _hip_runtimes():
    try:
        with open("/proc/self/maps") as f:
            return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln and "/" in ln})
    except OSError:
        return []


if len(_hip_runtimes()) > 1:
    raise ImportError(f"two HIP runtimes are loaded ({_hip_runtimes()}); import torch before loading libtm")

c_int, c_double, c_size_t, c_void_p, c_uint64 = (
    ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_uint64)
c_longlong = ctypes.c_longlong

TM_OK, TM_ERR_ARG, TM_ERR_NOMEM, TM_ERR_HIP, TM_ERR_NOCONV, TM_ERR_NUMERIC, TM_ERR_STATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "TM_OK", -1: "TM_ERR_ARG", -2: "TM_ERR_NOMEM", -3: "TM_ERR_HIP", -4: "TM_ERR_NOCONV",
                -5: "TM_ERR_NUMERIC", -6: "TM_ERR_STATE"}
PREC = {"f64": 1, "f32": 2, "f16": 4, "bf16": 8}
OPS = {"hop": 0, "m": 1, "mdag": 2, "mhat": 3, "mhat_dag": 4, "mhat_dag_mhat": 5, "bh": 6}
MODES = {"f64": 0, "mixed": 1, "lp": 2}
N_OPS = 90


class TMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class tm_solver_params(ctypes.Structure):
    _fields_ = [("mode", c_int), ("half_prec", c_int), ("tol", c_double), ("max_iter", c_int),
                ("fixed_iters", c_int), ("delta", c_double), ("chunk", c_int)]


class tm_solve_stats(ctypes.Structure):
    _fields_ = [("iters", c_int), ("reliable_updates", c_int), ("cg_rel_resid", c_double),
                ("true_rel_resid", c_double), ("seconds", c_double)]


class tm_tsm_params(ctypes.Structure):
    _fields_ = [("kappa", c_double), ("two_kappa_mu", c_double), ("noise_seed", c_uint64), ("n_hp", c_int),
                ("n_lp", c_int), ("hp", tm_solver_params), ("lp", tm_solver_params), ("batch", c_int),
                ("want_true_resid", c_int), ("ops", c_int)]


class tm_serve_status(ctypes.Structure):
    _fields_ = [("queued", c_int), ("active", c_int), ("finished", c_int), ("batches", c_int), ("in_flight", c_int),
                ("pending_jobs", c_int), ("running_slots", c_int), ("worker_error", c_int), ("arena_used", c_size_t),
                ("arena_size", c_size_t), ("arena_largest_free", c_size_t), ("t_snapshot", c_double),
                ("stall_s", c_double), ("busy_s", c_double), ("slot_s", c_double)]


class tm_tsm_stats(ctypes.Structure):
    _fields_ = [("hp_solves", c_int), ("lp_solves", c_int), ("hp_iters", c_longlong), ("lp_iters", c_longlong),
                ("hp_max_iters", c_int), ("lp_max_iters", c_int), ("reliable_updates", c_int),
                ("max_hp_true_resid", c_double), ("max_lp_true_resid", c_double), ("seconds", c_double),
                ("hp_seconds", c_double), ("lp_seconds", c_double)]


class tm_request(ctypes.Structure):
    _fields_ = [("gauge", c_void_p), ("params", tm_tsm_params), ("tag", c_uint64)]


class tm_result(ctypes.Structure):
    _fields_ = [("tag", c_uint64), ("status", c_int), ("lt", c_int), ("est", ctypes.POINTER(c_double)),
                ("var_re", ctypes.POINTER(c_double)), ("var_im", ctypes.POINTER(c_double)),
                ("stats", tm_tsm_stats), ("t_submit", c_double), ("t_admit", c_double), ("t_done", c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_size_t, c_int, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_int, c_void_p)

_sig = {
    "tm_create": (c_int, [c_int, c_size_t, ALLOC_FN, FREE_FN, c_void_p, ctypes.POINTER(c_void_p)]),
    "tm_destroy": (c_int, [c_void_p]),
    "tm_last_error": (ctypes.c_char_p, [c_void_p]),
    "tm_memory_usage": (c_int, [c_void_p, ctypes.POINTER(c_size_t), ctypes.POINTER(c_size_t)]),
    "tm_load_gauge": (c_int, [c_void_p, ctypes.POINTER(c_int), c_void_p, c_int, ctypes.c_uint, ctypes.POINTER(c_void_p)]),
    "tm_free_gauge": (c_int, [c_void_p, c_void_p]),
    "tm_field_bytes": (c_size_t, [c_void_p, c_int, c_int]),
    "tm_field_import": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p]),
    "tm_field_export": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p]),
    "tm_dslash": (c_int, [c_void_p, c_void_p, c_int, c_double, c_double, c_int, c_int, c_void_p, c_void_p, c_void_p]),
    "tm_dslash_ex": (c_int, [c_void_p, c_void_p, c_int, c_double, c_double, c_int, c_int, c_void_p, c_size_t,
                             c_void_p, c_size_t, c_void_p]),
    "tm_dslash_noalloc": (c_int, [c_void_p, c_void_p, c_int, c_double, c_double, c_int, c_int, c_void_p, c_size_t,
                                  c_void_p, c_size_t, c_void_p]),
    "tm_cg_solve": (c_int, [c_void_p, c_void_p, c_double, c_double, ctypes.POINTER(tm_solver_params), c_int,
                            c_void_p, c_void_p, ctypes.POINTER(tm_solve_stats), c_void_p]),
    "tm_cg_update": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p,
                             c_void_p, c_void_p]),
    "tm_z4_source": (c_int, [c_void_p, ctypes.POINTER(c_int), c_uint64, c_uint64, c_void_p, c_void_p]),
    "tm_loops_tsm": (c_int, [c_void_p, c_void_p, ctypes.POINTER(tm_tsm_params), c_void_p, c_void_p, c_void_p,
                             c_void_p, ctypes.POINTER(tm_tsm_stats)]),
    "tm_loops_oet": (c_int, [c_void_p, c_void_p, ctypes.POINTER(tm_tsm_params), c_void_p, c_void_p, c_void_p,
                             c_void_p, ctypes.POINTER(tm_tsm_stats)]),
    "tm_loops_hpe": (c_int, [c_void_p, c_void_p, ctypes.POINTER(tm_tsm_params), c_void_p, c_void_p, c_void_p,
                             c_void_p, ctypes.POINTER(tm_tsm_stats)]),
    "tm_loops_tdil": (c_int, [c_void_p, c_void_p, ctypes.POINTER(tm_tsm_params), c_int, c_void_p, c_int, c_int,
                              c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(tm_tsm_stats)]),
    "tm_project_loops": (c_int, [c_int, c_int, c_void_p, c_void_p]),
    "tm_contract": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p, c_size_t, c_uint64, c_void_p, c_void_p,
                            c_void_p]),
    "tm_serve_status_get": (c_int, [c_void_p, ctypes.POINTER(tm_serve_status)]),
    "tm_serve_create": (c_int, [c_void_p, c_int, c_size_t, ctypes.POINTER(c_void_p)]),
    "tm_serve_submit": (c_int, [c_void_p, ctypes.POINTER(tm_request)]),
    "tm_serve_footprint": (c_int, [c_void_p, ctypes.POINTER(tm_request), ctypes.POINTER(ctypes.c_size_t)]),
    "tm_serve_poll": (c_int, [c_void_p, ctypes.POINTER(tm_result), c_int]),
    "tm_serve_drain": (c_int, [c_void_p]),
    "tm_result_free": (None, [ctypes.POINTER(tm_result)]),
    "tm_serve_clock": (c_double, [c_void_p]),
    "tm_serve_destroy": (c_int, [c_void_p]),
    "tm_stream_copy": (c_int, [c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "tm_selftest": (c_int, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = sorted(_sig)


def _ptr(x):
    """Device or host address of a torch tensor / numpy array / int."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dims(dims):
    return (c_int * 4)(*[int(d) for d in dims])


def _check(ctx, rc, what):
    if rc != TM_OK:
        msg = _lib.tm_last_error(ctx).decode() if ctx else ""
        raise TMError(rc, f"{what}: {msg}")


# torch's caching allocator behind the library's allocation callbacks
def _torch_alloc(nbytes, device, user):
    import torch

    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), int(device))
    except Exception as e:  # out of memory -> NULL -> TM_ERR_NOMEM
        import sys

        print(f"libtm allocation of {int(nbytes)} bytes failed: {e}", file=sys.stderr)
        return None


def _torch_free(ptr, device, user):
    import torch

    torch.cuda.caching_allocator_delete(int(ptr))


_ALLOC_CB = ALLOC_FN(_torch_alloc)
_FREE_CB = FREE_FN(_torch_free)


# ----------------------------------------------------------------------------
# same-name wrappers
# ----------------------------------------------------------------------------
def tm_selftest() -> int:
    return int(_lib.tm_selftest())


def tm_create(device: int = 0, hbm_budget: int = 0, torch_allocator: bool = True):
    out = c_void_p()
    if torch_allocator:
        import torch

        torch.cuda.init()
        torch.cuda.set_device(int(device))
        rc = _lib.tm_create(device, hbm_budget, _ALLOC_CB, _FREE_CB, None, ctypes.byref(out))
    else:
        rc = _lib.tm_create(device, hbm_budget, ALLOC_FN(), FREE_FN(), None, ctypes.byref(out))
    if rc != TM_OK:
        raise TMError(rc, "tm_create failed")
    return out.value


def tm_destroy(ctx):
    _check(ctx, _lib.tm_destroy(ctx), "tm_destroy")


def tm_last_error(ctx) -> str:
    return _lib.tm_last_error(ctx).decode()


def tm_memory_usage(ctx):
    a, b = c_size_t(), c_size_t()
    _check(ctx, _lib.tm_memory_usage(ctx, ctypes.byref(a), ctypes.byref(b)), "tm_memory_usage")
    return a.value, b.value


def tm_load_gauge(ctx, dims, links: np.ndarray, t_bc: int = -1, precs=("f32", "f16", "bf16")):
    links = np.ascontiguousarray(links, dtype=np.complex128)
    mask = 0
    for p in precs:
        mask |= PREC[p]
    out = c_void_p()
    rc = _lib.tm_load_gauge(ctx, _dims(dims), links.ctypes.data, int(t_bc), mask, ctypes.byref(out))
    _check(ctx, rc, "tm_load_gauge")
    return out.value


def tm_free_gauge(ctx, gauge):
    _check(ctx, _lib.tm_free_gauge(ctx, gauge), "tm_free_gauge")


def tm_field_bytes(gauge, prec: str, full: bool = True) -> int:
    return int(_lib.tm_field_bytes(gauge, PREC[prec], 1 if full else 0))


def tm_field_import(ctx, gauge, prec, nrhs, canonical, field, stream=None):
    _check(ctx, _lib.tm_field_import(ctx, gauge, PREC[prec], nrhs, _ptr(canonical), _ptr(field), _stream(stream)),
           "tm_field_import")


def tm_field_export(ctx, gauge, prec, nrhs, field, canonical, stream=None):
    _check(ctx, _lib.tm_field_export(ctx, gauge, PREC[prec], nrhs, _ptr(field), _ptr(canonical), _stream(stream)),
           "tm_field_export")


def tm_dslash(ctx, gauge, op, kappa, two_kappa_mu, prec, nrhs, inp, out, stream=None):
    rc = _lib.tm_dslash(ctx, gauge, OPS[op] if isinstance(op, str) else int(op), float(kappa), float(two_kappa_mu),
                        PREC[prec], int(nrhs), _ptr(inp), _ptr(out), _stream(stream))
    _check(ctx, rc, "tm_dslash")


def tm_dslash_ex(ctx, gauge, op, kappa, two_kappa_mu, prec, nrhs, inp, in_stride, out, out_stride, stream=None):
    rc = _lib.tm_dslash_ex(ctx, gauge, OPS[op] if isinstance(op, str) else int(op), float(kappa),
                           float(two_kappa_mu), PREC[prec], int(nrhs), _ptr(inp), int(in_stride), _ptr(out),
                           int(out_stride), _stream(stream))
    _check(ctx, rc, "tm_dslash_ex")


def tm_dslash_noalloc(ctx, gauge, op, kappa, two_kappa_mu, prec, nrhs, inp, in_stride, out, out_stride, stream=None,
                      check=True):
    rc = _lib.tm_dslash_noalloc(ctx, gauge, OPS[op] if isinstance(op, str) else int(op), float(kappa),
                                float(two_kappa_mu), PREC[prec], int(nrhs), _ptr(inp), int(in_stride), _ptr(out),
                                int(out_stride), _stream(stream))
    if check:
        _check(ctx, rc, "tm_dslash_noalloc")
    return rc


def solver_params(mode="f64", tol=1e-10, max_iter=100000, fixed_iters=0, half="f16", delta=1e-3, chunk=0):
    return tm_solver_params(MODES[mode], PREC[half], float(tol), int(max_iter), int(fixed_iters), float(delta),
                            int(chunk))


def tm_cg_update(ctx, gauge, prec, nrhs, p, r, x, stride, alpha, beta, stream=None, check=True):
    """CG direction update on nrhs even-half fields (device, layout of prec):
    x += alpha p (x may be None), then p = r + beta p."""
    al = np.ascontiguousarray(np.asarray(alpha, dtype=np.float64).reshape(-1))
    be = np.ascontiguousarray(np.asarray(beta, dtype=np.float64).reshape(-1))
    assert al.size == nrhs and be.size == nrhs
    rc = _lib.tm_cg_update(ctx, gauge, PREC[prec], int(nrhs), _ptr(p), _ptr(r), _ptr(x), int(stride),
                           al.ctypes.data, be.ctypes.data, _stream(stream))
    if check:
        _check(ctx, rc, "tm_cg_update")
    return rc


def tm_cg_solve(ctx, gauge, kappa, two_kappa_mu, params, nrhs, b, x, stream=None, check=True):
    stats = (tm_solve_stats * nrhs)()
    rc = _lib.tm_cg_solve(ctx, gauge, float(kappa), float(two_kappa_mu), ctypes.byref(params), int(nrhs), _ptr(b),
                          _ptr(x), stats, _stream(stream))
    if check:
        _check(ctx, rc, "tm_cg_solve")
    return rc, [dict(iters=s.iters, reliable_updates=s.reliable_updates, cg_rel_resid=s.cg_rel_resid,
                     true_rel_resid=s.true_rel_resid, seconds=s.seconds) for s in stats]


def tm_z4_source(ctx, dims, seed, src, out, stream=None):
    _check(ctx, _lib.tm_z4_source(ctx, _dims(dims), c_uint64(int(seed)), c_uint64(int(src)), _ptr(out),
                                  _stream(stream)), "tm_z4_source")


def tsm_params(kappa, two_kappa_mu, noise_seed, n_hp, n_lp, hp=None, lp=None, batch=12, want_true_resid=0,
               local_only=False):
    hp = hp if hp is not None else solver_params("mixed", tol=1e-10)
    lp = lp if lp is not None else solver_params("lp", tol=1e-2, half="f16")
    return tm_tsm_params(float(kappa), float(two_kappa_mu), int(noise_seed), int(n_hp), int(n_lp), hp, lp,
                         int(batch), int(want_true_resid), 1 if local_only else 0)


def _stats_dict(st):
    return {k: getattr(st, k) for k, _ in tm_tsm_stats._fields_}


def tm_loops_tsm(ctx, gauge, params, lt, want_raw=False, check=True):
    """Returns dict(est (90, lt) complex, var_re, var_im (90, lt), raw or None, stats, status)."""
    est = np.zeros((N_OPS, lt, 2))
    vre = np.zeros((N_OPS, lt))
    vim = np.zeros((N_OPS, lt))
    n_raw = params.n_hp + params.n_hp + params.n_lp
    raw = np.zeros((n_raw, 9, lt, 4, 4, 2)) if want_raw else None
    st = tm_tsm_stats()
    rc = _lib.tm_loops_tsm(ctx, gauge, ctypes.byref(params), est.ctypes.data, vre.ctypes.data, vim.ctypes.data,
                           raw.ctypes.data if want_raw else None, ctypes.byref(st))
    if check:
        _check(ctx, rc, "tm_loops_tsm")
    out = dict(est=est[..., 0] + 1j * est[..., 1], var_re=vre, var_im=vim, stats=_stats_dict(st), status=rc)
    if want_raw:
        rawc = raw[..., 0] + 1j * raw[..., 1]
        out["raw_hp"] = rawc[: params.n_hp]
        out["raw_lp"] = rawc[params.n_hp:]
    return out


def _loops2(fn, names, ctx, gauge, params, lt, want_raw, check, extra=()):
    nf = len(names)
    est = np.zeros((nf, N_OPS, lt, 2))
    vre = np.zeros((nf, N_OPS, lt))
    vim = np.zeros((nf, N_OPS, lt))
    n_raw = params.n_hp + params.n_hp + params.n_lp
    raw = np.zeros((nf, n_raw, 9, lt, 4, 4, 2)) if want_raw else None
    st = tm_tsm_stats()
    rc = getattr(_lib, fn)(ctx, gauge, ctypes.byref(params), *extra, est.ctypes.data, vre.ctypes.data,
                           vim.ctypes.data, raw.ctypes.data if want_raw else None, ctypes.byref(st))
    if check:
        _check(ctx, rc, fn)
    out = dict(stats=_stats_dict(st), status=rc)
    for f, name in enumerate(names):
        out["est_" + name] = est[f, ..., 0] + 1j * est[f, ..., 1]
        out["var_re_" + name] = vre[f]
        out["var_im_" + name] = vim[f]
        if want_raw:
            rawc = raw[f, ..., 0] + 1j * raw[f, ..., 1]
            out[f"raw_{name}_hp"] = rawc[: params.n_hp]
            out[f"raw_{name}_lp"] = rawc[params.n_hp:]
    return out


def tm_loops_oet(ctx, gauge, params, lt, want_raw=False, check=True):
    """One-end trick loops: dict(est_vv, est_ws (90, lt) complex, var_re_vv, var_im_vv, var_re_ws,
    var_im_ws, optional raw_vv_hp, raw_vv_lp, raw_ws_hp, raw_ws_lp, stats, status)."""
    return _loops2("tm_loops_oet", ("vv", "ws"), ctx, gauge, params, lt, want_raw, check)


def tm_loops_hpe(ctx, gauge, params, lt, want_raw=False, check=True):
    """Standard and hopping-parameter-expansion loops from the same solves:
    dict(est_std, est_hpe (90, lt) complex (est_hpe NaN beyond the 16 local
    ops), var_re_std, var_im_std, var_re_hpe, var_im_hpe, optional raw_std_hp,
    raw_std_lp, raw_hpe_hp, raw_hpe_lp, stats, status)."""
    return _loops2("tm_loops_hpe", ("std", "hpe"), ctx, gauge, params, lt, want_raw, check)


def tm_loops_tdil(ctx, gauge, params, lt, spacing, phases=None, hpe=False, want_raw=False, check=True):
    """Time-diluted loops: one source per phase p (timeslices t = p mod spacing)
    of each noise vector, summed per noise vector, TSM over noise vectors.
    dict(est_std, var_re_std, var_im_std, and with hpe est_hpe, var_re_hpe,
    var_im_hpe (90, lt), NaN where not covered; optional raw_std_hp, raw_std_lp
    (, raw_hpe_hp, raw_hpe_lp) per noise vector; stats, status)."""
    ph = None if phases is None else np.ascontiguousarray(np.asarray(phases, dtype=np.int32))
    extra = (int(spacing), None if ph is None else ph.ctypes.data, 0 if ph is None else int(ph.size), int(bool(hpe)))
    names = ("std", "hpe") if hpe else ("std",)
    return _loops2("tm_loops_tdil", names, ctx, gauge, params, lt, want_raw, check, extra)


def tm_contract(ctx, gauge, prec, n, s, s_stride, noise_seed, src_ids, raw, stream=None):
    """Spin matrices of n solutions s (device, layout of prec) with their Z4
    sources into raw (device, n * 9 * lt * 32 doubles)."""
    ids = np.ascontiguousarray(np.asarray(src_ids, dtype=np.uint64))
    assert ids.size == n
    _check(ctx, _lib.tm_contract(ctx, gauge, PREC[prec], int(n), _ptr(s), int(s_stride), c_uint64(int(noise_seed)),
                                 ids.ctypes.data, _ptr(raw), _stream(stream)), "tm_contract")


def tm_project_loops(raw: np.ndarray) -> np.ndarray:
    """raw (n, 9, lt, 4, 4) complex -> (n, 90, lt) complex (host utility)."""
    raw = np.ascontiguousarray(raw, dtype=np.complex128)
    n, _, lt = raw.shape[:3]
    out = np.zeros((n, N_OPS, lt), dtype=np.complex128)
    rc = _lib.tm_project_loops(n, lt, raw.ctypes.data, out.ctypes.data)
    if rc != TM_OK:
        raise TMError(rc, "tm_project_loops")
    return out


def tm_stream_copy(ctx, src, dst, nbytes, stream=None):
    _check(ctx, _lib.tm_stream_copy(ctx, _ptr(src), _ptr(dst), int(nbytes), _stream(stream)), "tm_stream_copy")


# ----------------------------------------------------------------------------
# serving
# ----------------------------------------------------------------------------
def tm_serve_create(ctx, slots=12, workspace_budget=0):
    out = c_void_p()
    _check(ctx, _lib.tm_serve_create(ctx, int(slots), int(workspace_budget), ctypes.byref(out)), "tm_serve_create")
    return out.value


def tm_serve_submit(srv, gauge, params, tag):
    req = tm_request(gauge, params, int(tag))
    return int(_lib.tm_serve_submit(srv, ctypes.byref(req)))


def tm_serve_footprint(srv, gauge, params):
    """Workspace bytes a request needs from the budget with none of its batches resident."""
    req = tm_request(gauge, params, 0)
    n = ctypes.c_size_t(0)
    rc = _lib.tm_serve_footprint(srv, ctypes.byref(req), ctypes.byref(n))
    if rc != TM_OK:
        raise TMError(rc, "tm_serve_footprint")
    return int(n.value)


def tm_serve_poll(srv, max_results=64):
    buf = (tm_result * max_results)()
    n = _lib.tm_serve_poll(srv, buf, max_results)
    if n < 0:
        raise TMError(n, "tm_serve_poll")
    out = []
    for i in range(n):
        r = buf[i]
        lt = r.lt
        if r.status == TM_OK or r.est:
            est = np.ctypeslib.as_array(r.est, shape=(N_OPS * lt * 2,)).reshape(N_OPS, lt, 2).copy()
            vre = np.ctypeslib.as_array(r.var_re, shape=(N_OPS * lt,)).reshape(N_OPS, lt).copy()
            vim = np.ctypeslib.as_array(r.var_im, shape=(N_OPS * lt,)).reshape(N_OPS, lt).copy()
            est = est[..., 0] + 1j * est[..., 1]
        else:
            est = vre = vim = None
        out.append(dict(tag=r.tag, status=r.status, lt=lt, est=est, var_re=vre, var_im=vim,
                        stats=_stats_dict(r.stats), t_submit=r.t_submit, t_admit=r.t_admit, t_done=r.t_done))
        _lib.tm_result_free(ctypes.byref(buf[i]))
    return out


def tm_serve_drain(srv):
    return int(_lib.tm_serve_drain(srv))


def tm_serve_clock(srv):
    return float(_lib.tm_serve_clock(srv))


def tm_serve_status_get(srv):
    """Latest snapshot of the serving loop as a dict."""
    st = tm_serve_status()
    rc = _lib.tm_serve_status_get(srv, ctypes.byref(st))
    if rc != TM_OK:
        raise TMError(rc, "tm_serve_status_get")
    return {k: getattr(st, k) for k, _ in tm_serve_status._fields_}


def tm_serve_destroy(srv):
    return int(_lib.tm_serve_destroy(srv))


# ----------------------------------------------------------------------------
# convenience
# ----------------------------------------------------------------------------
def canonical_to_torch(a: np.ndarray, device="cuda"):
    """complex128 numpy spinor(s) -> float64 torch tensor [..., 2] on device."""
    import torch

    a = np.ascontiguousarray(a, dtype=np.complex128)
    return torch.from_numpy(a.view(np.float64).copy()).to(device)


def torch_to_canonical(t) -> np.ndarray:
    a = t.detach().cpu().numpy()
    return a.view(np.complex128)
