#!/usr/bin/env python3
"""Benchmark of the TSM disconnected-loop path on one MI355X.

A step is one full pass of the hot path for one gauge field: Z4 sources,
mixed-precision HP solves, FP16-storage LP solves (12 right-hand sides per
multi-RHS launch), contractions at every timeslice, projection onto the 90
local and one-derivative insertions and the TSM combination - one
tm_loops_tsm call.  Default workload: the 32^3 x 64 lattice with the
batched TSM parameters (kappa = 0.1636, 2 kappa mu = 0.0033, N_HP = 48,
N_LP = 1000), synthetic seeded SU(3) links standing in for the paper's
ensemble.

Printed JSON line (one, rank 0):
  value         TSM loop sources/s, (N_HP + N_LP) * K / wall time of K steps
  plain_f64     the same loops by plain FP64 CG (no TSM, one RHS per launch)
                on the same GPU: sources/s and per-operator efficiency at
                equal statistical error
  roofline      the FP16 multi-RHS hopping kernel, timed with HIP events on
                the stream it is launched on, algorithmic bytes / duration
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: dims, kappa, 2 kappa mu, n_hp, n_lp, lp half precision, rhs per launch, gauge seed, noise seed
    "tsm-batched-32c64": dict(dims=(32, 32, 32, 64), kappa=0.1636, a=0.0033, n_hp=48, n_lp=1000, half="f16",
                              batch=12, gauge_seed=4, noise_seed=104),
    "tsm-24c48": dict(dims=(24, 24, 24, 48), kappa=0.1636, a=0.0033, n_hp=24, n_lp=500, half="f16", batch=12,
                      gauge_seed=3, noise_seed=103),
}
LINK_BYTES = {"f64": 96, "f32": 48, "f16": 36, "bf16": 36}
SPINOR_BYTES = {"f64": 192, "f32": 96, "f16": 52, "bf16": 52}
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dslash_f16_traffic.json")
KERNEL_SOURCES = ["paper_1401_6749_amd/csrc/k_dslash.hip", "paper_1401_6749_amd/csrc/tm_dev.h",
                  "paper_1401_6749_amd/csrc/tm_types.h"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def event_time(torch, fn, n, warm=3):
    s = torch.cuda.current_stream()
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(n):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / n


def slot_pitch(nbytes: int) -> int:
    """Pitch the solver uses between the fields of consecutive right-hand sides."""
    return (nbytes + 255) // 256 * 256 + 17 * 256


def measure_roofline(torch, tm, inputs, ctx, g, W, workload):
    """The dominant kernel: the FP16 hop over `batch` right-hand sides laid out
    with the solver's slot pitch (the LDS timeslice-walk kernel), timed with
    HIP events on the stream it is launched on, and the copy ceiling."""
    dims = W["dims"]
    vh = dims[0] * dims[1] * dims[2] * dims[3] // 2
    prec = W["half"]
    nrhs = W["batch"]
    fb = tm.tm_field_bytes(g, prec, True)
    pitch = slot_pitch(fb)
    fin = torch.zeros(nrhs * pitch, dtype=torch.uint8, device="cuda")
    psi = tm.canonical_to_torch(inputs.random_spinor(dims, 1)[None])
    for r in range(nrhs):
        tm.tm_field_import(ctx, g, prec, 1, psi, fin[r * pitch:r * pitch + fb])
    fout = torch.zeros_like(fin)
    n_calls = 20
    t_call = event_time(torch, lambda: tm.tm_dslash_ex(ctx, g, "hop", W["kappa"], W["a"], prec, nrhs, fin, pitch,
                                                        fout, pitch), n_calls)
    t_launch = t_call / 2  # one launch per output parity
    alg_bytes = vh * (8 * LINK_BYTES[prec] + nrhs * 2 * SPINOR_BYTES[prec])
    achieved = alg_bytes / t_launch / 1e9
    # copy ceiling with the library's streaming copy kernel (1 GiB)
    nb = 1 << 30
    ca = torch.empty(nb, dtype=torch.uint8, device="cuda")
    cb = torch.empty(nb, dtype=torch.uint8, device="cuda")
    t_copy = event_time(torch, lambda: tm.tm_stream_copy(ctx, ca, cb, nb), 20)
    copy_gbs = 2 * nb / t_copy / 1e9
    del ca, cb, fin, fout
    traffic = None
    khash = kernel_hash()
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_hash") == khash and tr.get("workload") == workload and tr.get("nrhs") == nrhs:
            traffic = tr.get("hbm_bytes_per_launch")
    log(f"dslash {prec} x{nrhs}: {t_launch * 1e6:.1f} us/launch, {achieved:.0f} GB/s; copy {copy_gbs:.0f} GB/s")
    return {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
        "kernel": f"k_dslash_walk {prec} hop, {nrhs} RHS per launch, {dims[0]}^3x{dims[3]}",
        "alg_bytes_per_launch": alg_bytes, "launch_us": round(t_launch * 1e6, 2),
        "copy_ceiling_GBs": round(copy_gbs, 1), "kernel_hash": khash,
    }


def write_traffic(fetch_db: str, write_db: str, workload: str) -> None:
    """Per-launch HBM bytes of the roofline kernel from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by what the same counter reads
    for the 1 GiB streaming copy (which reads and writes exactly 1 GiB)."""
    import sqlite3

    W = WORKLOADS[workload]

    def per_dispatch(db, counter):
        cur = sqlite3.connect(db).cursor()
        rows = cur.execute("select kernel_name, value from counters_collection where counter_name = ?",
                           (counter,)).fetchall()
        copy = [v for n, v in rows if "k_stream_copy" in n]
        kern = [v for n, v in rows if "k_dslash_walk<2, false, 0, false, false" in n]
        if not copy or not kern:
            raise SystemExit(f"{db}: no {counter} rows for the copy or the FP16 hop kernel")
        return sum(copy) / len(copy), sum(kern) / len(kern), len(kern)

    cf, kf, nf = per_dispatch(fetch_db, "FETCH_SIZE")
    cw, kw, nw = per_dispatch(write_db, "WRITE_SIZE")
    f_fetch = (1 << 30) / (cf * 1024.0)
    f_write = (1 << 30) / (cw * 1024.0)
    fetch = kf * 1024.0 * f_fetch
    write = kw * 1024.0 * f_write
    out = {
        "workload": workload, "nrhs": W["batch"], "kernel_hash": kernel_hash(),
        "kernel": "k_dslash_walk FP16 hop (uniform parameters), one launch per output parity",
        "fetch_scale": round(f_fetch, 4), "write_scale": round(f_write, 4),
        "fetch_bytes_per_launch": round(fetch), "write_bytes_per_launch": round(write),
        "hbm_bytes_per_launch": round(fetch + write), "dispatches": [nf, nw],
        "commands": ["rocprofv3 --pmc FETCH_SIZE -d gpurun_out/pmc_fetch -o fetch -- python3 bench.py --roofline-only",
                     "rocprofv3 --pmc WRITE_SIZE -d gpurun_out/pmc_write -o write -- python3 bench.py --roofline-only",
                     "python3 bench.py --traffic-from gpurun_out/pmc_fetch/fetch_results.db "
                     "gpurun_out/pmc_write/write_results.db"],
    }
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tsm-batched-32c64", choices=sorted(WORKLOADS))
    ap.add_argument("--plain-sources", type=int, default=48)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the copy calibration and the roofline kernel (for counter runs)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="write the roofline kernel's HBM traffic from two rocprofv3 --pmc databases "
                         "(FETCH_SIZE, WRITE_SIZE) of --roofline-only runs and exit")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic(args.traffic_from[0], args.traffic_from[1], args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the whole lattice is resident on a single MI355X and this build "
              f"has no multi-GPU path (requested --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1401_6749_amd import inputs, tm

    W = WORKLOADS[args.workload]
    dims = W["dims"]
    lt = dims[3]
    V = int(np.prod(dims))
    vh = V // 2
    ctx = tm.tm_create(0)
    t0 = time.time()
    U = inputs.gauge_field(dims, W["gauge_seed"])
    g = tm.tm_load_gauge(ctx, dims, U, -1, ("f32", "f16", "bf16"))
    log(f"gauge {dims} ready in {time.time() - t0:.1f}s")
    if args.roofline_only:
        print(json.dumps({"roofline": measure_roofline(torch, tm, inputs, ctx, g, W, args.workload)}), flush=True)
        tm.tm_free_gauge(ctx, g)
        tm.tm_destroy(ctx)
        return

    hp = tm.solver_params("mixed", tol=1e-10, delta=0.1)
    lp = tm.solver_params("lp", tol=1e-2, half=W["half"])
    P = tm.tsm_params(W["kappa"], W["a"], W["noise_seed"], W["n_hp"], W["n_lp"], hp=hp, lp=lp, batch=W["batch"])
    n_src = W["n_hp"] + W["n_lp"]

    for i in range(args.warmup):
        r = tm.tm_loops_tsm(ctx, g, P, lt)
        log(f"warmup step {i} {r['stats']['seconds']:.2f}s")
    torch.cuda.synchronize()
    ta = time.perf_counter()
    last = None
    for i in range(args.steps):
        last = tm.tm_loops_tsm(ctx, g, P, lt)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    wall = tb - ta
    value = n_src * args.steps / wall
    st = last["stats"]
    log(f"timed {args.steps} steps in {wall:.2f}s -> {value:.1f} sources/s")

    # ---- plain FP64 CG on the same GPU, and efficiency at equal error ----
    plain = None
    if not args.no_plain:
        Pp = tm.tsm_params(W["kappa"], W["a"], W["noise_seed"], 0, args.plain_sources,
                           lp=tm.solver_params("f64", tol=1e-10), batch=1)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        rp = tm.tm_loops_tsm(ctx, g, Pp, lt)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp0
        plain_rate = args.plain_sources / tp
        # single-source variance of the plain FP64 loops, per operator and t
        sig1 = (rp["var_re"] + rp["var_im"]) * args.plain_sources
        sig_tsm = last["var_re"] + last["var_im"]
        t_step = wall / args.steps
        ok = (sig1 > 0) & (sig_tsm > 0)
        eff = np.where(ok, sig1 / np.where(ok, sig_tsm, 1) / t_step, np.nan)  # plain-source equivalents per s
        ratio = eff / plain_rate
        loc, der = ratio[:16].reshape(-1), ratio[16:80].reshape(-1)
        plain = {
            "sources_per_s": round(plain_rate, 3),
            "n_sources": args.plain_sources,
            "rhs_per_launch": 1,
            "iters_mean": rp["stats"]["lp_iters"] / max(1, rp["stats"]["lp_solves"]),
            "tsm_effective_speedup_local_median": float(np.nanmedian(loc)),
            "tsm_effective_speedup_deriv_median": float(np.nanmedian(der)),
        }
        log(f"plain FP64: {plain_rate:.2f} sources/s; TSM equal-error speedup local "
            f"{plain['tsm_effective_speedup_local_median']:.1f}x deriv {plain['tsm_effective_speedup_deriv_median']:.1f}x")

    roofline = measure_roofline(torch, tm, inputs, ctx, g, W, args.workload)

    # ---- CPU oracle on a bounded sample (one LP source at the same lattice) ----
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O

        O.lib()
        threads = O.num_threads()
        tc0 = time.perf_counter()
        r1 = O.loops_tsm(dims, -1, U, W["kappa"], W["a"], W["noise_seed"], 0, 1, lp_tol=1e-2,
                         source_ids=[W["n_hp"]])
        t_lp_src = time.perf_counter() - tc0
        it_lp = r1["lp_iters"][W["n_hp"]]
        # the oracle's cost of a HP source, from its per-iteration cost and the GPU's HP iteration count
        hp_it = st["hp_iters"] / max(1, st["hp_solves"])
        t_it = t_lp_src / (it_lp + 4.0)  # prep, reconstruction and contraction ~ 4 iterations
        t_hp_src = t_it * (hp_it + 4.0)
        t_tsm = W["n_hp"] * t_hp_src + n_src * t_lp_src
        cpu = {"value": round(n_src / t_tsm, 6), "unit": "sources/s", "cores": threads, "kind": "oracle",
               "sample": f"1 LP source (FP64, tol 1e-2, {it_lp} iterations, contraction) at "
                         f"{dims[0]}^3x{lt}: {t_lp_src:.1f}s; HP sources extrapolated from it with the GPU's "
                         f"mean HP iteration count ({hp_it:.0f})"}
        log(f"cpu oracle: {t_lp_src:.1f}s per LP source with {threads} threads")

    line = {
        "metric": "TSM loop sources/s",
        "value": round(value, 3),
        "unit": "sources/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "lattice": list(dims),
            "kappa": W["kappa"],
            "two_kappa_mu": W["a"],
            "n_hp": W["n_hp"],
            "n_lp": W["n_lp"],
            "hp": "mixed FP32 CG with FP64 reliable updates, tol 1e-10",
            "lp": (f"{W['half']} storage; Dslash: " + ("f16 spin projection, f16 x f16 products summed in FP32"
                                                       if W["half"] == "f16" else "FP32 arithmetic")
                   + "; FP32 vector updates and preparation; truncated at |r|/|r0| = 1e-2"),
            "rhs_per_launch": W["batch"],
            "parallelism": "single GPU, whole lattice resident",
        },
        "iters": {"hp_mean": st["hp_iters"] / max(1, st["hp_solves"]),
                  "lp_mean": st["lp_iters"] / max(1, st["lp_solves"]),
                  "reliable_updates": st["reliable_updates"]},
        "plain_f64": plain,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    tm.tm_free_gauge(ctx, g)
    tm.tm_destroy(ctx)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
