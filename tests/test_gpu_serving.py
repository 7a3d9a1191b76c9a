"""Serving loop on the GPU: continuous batching across requests gives every
request the same result as when it runs alone, and admission by footprint
queues requests under a small workspace budget."""
import time

import numpy as np
import pytest

from paper_1401_6749_amd import inputs
from tests import gpu_util as GU

pytestmark = pytest.mark.gpu


def _req_params(tm, kappa, a, seed, n_hp, n_lp, half="f16"):
    return tm.tsm_params(kappa, a, seed, n_hp, n_lp, hp=tm.solver_params("mixed", tol=1e-10),
                         lp=tm.solver_params("lp", tol=1e-2, half=half))


def _wait_all(tm, srv, n, timeout=120):
    out = {}
    t0 = time.time()
    while len(out) < n:
        for r in tm.tm_serve_poll(srv):
            out[r["tag"]] = r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"only {len(out)} of {n} results")
        time.sleep(0.002)
    return out


def test_serving_alone_equals_in_mix(oracle):
    from paper_1401_6749_amd import tm

    ctx = GU.context()
    dA, dB = (8, 8, 8, 16), (4, 4, 4, 8)
    gA = GU.load(dA, inputs.gauge_field(dA, 11))
    gA2 = GU.load(dA, inputs.gauge_field(dA, 12))
    UB = inputs.gauge_field(dB, 13)
    gB = GU.load(dB, UB)
    PA = _req_params(tm, 0.1636, 0.0033, 7, 3, 20)
    srv = tm.tm_serve_create(ctx, slots=12, workspace_budget=1 << 30)
    try:
        assert tm.tm_serve_submit(srv, gA, PA, 1) == 0
        alone = _wait_all(tm, srv, 1)[1]
        assert alone["status"] == 0
        # the same request inside a mix of other lattices, gauge fields, masses
        # and precisions, submitted together so their sources share launches
        # an FP64 request (HP to 1e-10, LP truncated at 1e-2, both in FP64):
        # its result has an oracle reference
        P64 = tm.tsm_params(0.12, 0.02, 31, 2, 5, hp=tm.solver_params("f64", tol=1e-10),
                            lp=tm.solver_params("f64", tol=1e-2))
        mix = [(gA2, _req_params(tm, 0.1636, 0.01, 8, 2, 15)),
               (gB, _req_params(tm, 0.12, 0.0033, 9, 4, 30, half="bf16")),
               (gA, _req_params(tm, 0.13, 0.01, 10, 1, 12)),
               (gA, PA),
               (gB, P64)]
        for k, (g, P) in enumerate(mix):
            assert tm.tm_serve_submit(srv, g, P, 100 + k) == 0
        res = _wait_all(tm, srv, len(mix))
        # the FP64 request against the oracle's whole path (Sec. 2.1, Eq. estiTSM)
        r64 = res[104]
        assert r64["status"] == 0
        ref = oracle.loops_tsm(dB, -1, UB, 0.12, 0.02, 31, 2, 5, hp_tol=1e-10, lp_tol=1e-2)
        assert GU.relerr(r64["est"], ref["est"]) < 1e-10
        for k, sl in GU.OP_CLASSES.items():
            assert GU.relerr(r64["est"][sl], ref["est"][sl]) < 1e-10, k
        for key in ("var_re", "var_im"):
            assert np.allclose(r64[key], ref[key], rtol=1e-8, atol=1e-14 * np.abs(ref[key]).max()), key
        assert r64["stats"]["hp_solves"] == 2 and r64["stats"]["lp_solves"] == 7
        inmix = res[103]
        assert inmix["status"] == 0
        assert np.array_equal(inmix["est"], alone["est"])
        assert np.array_equal(inmix["var_re"], alone["var_re"])
        assert inmix["stats"]["lp_iters"] == alone["stats"]["lp_iters"]
        assert inmix["stats"]["hp_iters"] == alone["stats"]["hp_iters"]
        # and the direct call gives the same bits
        direct = tm.tm_loops_tsm(ctx, gA, PA, dA[3])
        assert np.array_equal(direct["est"], alone["est"])
        for r in res.values():
            assert r["status"] == 0 and np.all(np.isfinite(r["est"]))
            assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
    finally:
        tm.tm_serve_destroy(srv)


def test_serving_admission_under_small_budget():
    from paper_1401_6749_amd import tm

    ctx = GU.context()
    d = (8, 8, 8, 16)
    gs = [GU.load(d, inputs.gauge_field(d, 20 + k)) for k in range(3)]
    P = _req_params(tm, 0.1636, 0.0033, 5, 2, 10)
    # room for one request's output buffers and pair of batches, not two
    probe = tm.tm_serve_create(ctx, slots=4, workspace_budget=1 << 20)
    try:
        need = tm.tm_serve_footprint(probe, gs[0], P)
    finally:
        tm.tm_serve_destroy(probe)
    srv = tm.tm_serve_create(ctx, slots=4, workspace_budget=need * 3 // 2)
    try:
        for k, g in enumerate(gs):
            assert tm.tm_serve_submit(srv, g, P, k) == 0
        # the worker's snapshot: the arena within its budget (a finishing request may overlap the next)
        import time as _time
        for _ in range(20):
            st = tm.tm_serve_status_get(srv)
            if st["t_snapshot"] > 0:  # published by the worker
                assert st["arena_size"] == need * 3 // 2
            assert st["active"] <= 2 and st["arena_used"] <= st["arena_size"]
            assert st["queued"] + st["active"] + st["finished"] <= 3 and st["worker_error"] == 0
            _time.sleep(0.005)
        res = _wait_all(tm, srv, 3)
        assert all(r["status"] == 0 for r in res.values())
        # utilisation integrals: the GPU was busy for part of the server's
        # time; at most two requests are active, each with an HP and an LP
        # batch of 4 slots
        _time.sleep(0.1)
        st = tm.tm_serve_status_get(srv)
        assert 0.0 < st["busy_s"] <= st["t_snapshot"]
        assert 0.0 < st["slot_s"] <= 16 * st["t_snapshot"]
        ordered = sorted(res.values(), key=lambda r: r["t_admit"])
        # later requests waited in the queue until earlier ones released their
        # workspace (only the final projection may overlap the next admission)
        for k in (1, 2):
            prev = ordered[k - 1]
            assert ordered[k]["t_admit"] - ordered[k]["t_submit"] > 0.5 * (prev["t_done"] - prev["t_admit"])
        # a request that can never fit is rejected at submission
        big = (16, 16, 16, 32)
        gbig = GU.load(big, inputs.gauge_field(big, 1))
        rc = tm.tm_serve_submit(srv, gbig, P, 99)
        assert rc == tm.TM_ERR_NOMEM
    finally:
        tm.tm_serve_destroy(srv)


def test_serving_rejects_bad_requests():
    from paper_1401_6749_amd import tm

    ctx = GU.context()
    d = (4, 4, 4, 4)
    g = GU.load(d, inputs.gauge_field(d, 1), precs=("f32",))  # no half-precision links
    srv = tm.tm_serve_create(ctx, slots=4, workspace_budget=64 << 20)
    try:
        P = _req_params(tm, 0.12, 0.01, 1, 1, 2)  # LP needs f16 links
        assert tm.tm_serve_submit(srv, g, P, 1) == tm.TM_ERR_ARG
        P2 = tm.tsm_params(0.12, 0.01, 1, 0, 0)
        assert tm.tm_serve_submit(srv, g, P2, 2) == tm.TM_ERR_ARG
    finally:
        tm.tm_serve_destroy(srv)
