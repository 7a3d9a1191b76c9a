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
    # the plain method in FP64 at 16^3x32 (64 sources to 1e-10): a segment of the default run
    "plain-16c32": dict(dims=(16, 16, 16, 32), kappa=0.12, a=0.005, n_hp=0, n_lp=64, half="f16", batch=12,
                        gauge_seed=2, noise_seed=102),
}
# Algorithmic bytes (what the method must move): every link as 12 reals
# (two rows; the third follows from unitarity), half-precision spinors with
# their FP32 per-site scale.  The library stores half-precision links with all
# nine entries (36 B); that storage figure is reported beside the algorithmic one.
LINK_BYTES = {"f64": 96, "f32": 48, "f16": 24, "bf16": 24}
LINK_STORAGE_BYTES = {"f64": 96, "f32": 48, "f16": 36, "bf16": 36}
SPINOR_BYTES = {"f64": 192, "f32": 96, "f16": 52, "bf16": 52}
# contraction (K6) per site and source: the solution and four links
CONTRACT_BYTES = {"f64": 192 + 4 * 96, "f32": 96 + 4 * 48}
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dslash_f16_traffic.json")
KERNEL_SOURCES = ["paper_1401_6749_amd/csrc/k_dslash.hip", "paper_1401_6749_amd/csrc/tm_dev.h",
                  "paper_1401_6749_amd/csrc/tm_types.h"]


def code_text(src: str) -> str:
    """C/C++ source without comments and with runs of whitespace collapsed:
    what the compiler sees of the kernel, so a comment edit does not retire
    counters taken on the same code."""
    out, i, n = [], 0, len(src)
    while i < n:
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif src[i] in "\"'":
            q, j = src[i], i + 1
            while j < n and src[j] != q:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(src[i])
            i += 1
    return " ".join("".join(out).split())


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            h.update(code_text(fh.read()).encode())
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
    storage_bytes = vh * (8 * LINK_STORAGE_BYTES[prec] + nrhs * 2 * SPINOR_BYTES[prec])
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
        "alg_bytes_per_launch": alg_bytes,
        "alg_bytes_per_site": 8 * LINK_BYTES[prec] + nrhs * 2 * SPINOR_BYTES[prec],
        "storage_bytes_per_launch": storage_bytes,
        "storage_GBs": round(storage_bytes / t_launch / 1e9, 1),
        "launch_us": round(t_launch * 1e6, 2),
        "copy_ceiling_GBs": round(copy_gbs, 1), "frac_of_copy_ceiling": round(achieved / copy_gbs, 4),
        "kernel_hash": khash,
    }


def kernel_rates(torch, tm, inputs, ctx, g, W):
    """Hop launches in each storage precision (single RHS and 12 RHS at the
    solver's slot pitch): microseconds per launch and algorithmic GB/s
    (8 links + 2 spinors per output site and RHS, links once per launch)."""
    dims = W["dims"]
    vh = dims[0] * dims[1] * dims[2] * dims[3] // 2
    psi = tm.canonical_to_torch(inputs.random_spinor(dims, 2)[None])
    out = []
    for prec, nrhs in (("f64", 1), ("f32", 1), ("f16", 1), ("f64", 12), ("f32", 12), ("f16", 12), ("bf16", 12)):
        fb = tm.tm_field_bytes(g, prec, True)
        pitch = slot_pitch(fb)
        fin = torch.zeros(nrhs * pitch, dtype=torch.uint8, device="cuda")
        for r in range(nrhs):
            tm.tm_field_import(ctx, g, prec, 1, psi, fin[r * pitch:r * pitch + fb])
        fout = torch.zeros_like(fin)
        t = event_time(torch, lambda: tm.tm_dslash_ex(ctx, g, "hop", W["kappa"], W["a"], prec, nrhs, fin, pitch,
                                                       fout, pitch), 10) / 2
        alg = vh * (8 * LINK_BYTES[prec] + nrhs * 2 * SPINOR_BYTES[prec])
        sto = vh * (8 * LINK_STORAGE_BYTES[prec] + nrhs * 2 * SPINOR_BYTES[prec])
        out.append({"prec": prec, "nrhs": nrhs, "launch_us": round(t * 1e6, 1), "alg_GBs": round(alg / t / 1e9, 1),
                    "frac_8TBs": round(alg / t / 1e9 / HBM_PEAK_GBS, 4), "storage_GBs": round(sto / t / 1e9, 1)})
        del fin, fout
    return out


def contract_rates(torch, tm, inputs, ctx, g, W):
    """The contraction (K6) alone through tm_contract: 12 FP32 solutions at
    the solver's slot pitch (the LP harvest's launch shape) and one FP64
    solution (the HP harvest's), timed with HIP events on the stream it runs
    on; algorithmic bytes = the solution and four links per site and source
    (the noise is regenerated from its counter, the neighbour reads are the
    stencil's own data)."""
    dims = W["dims"]
    V = dims[0] * dims[1] * dims[2] * dims[3]
    lt = dims[3]
    psi = tm.canonical_to_torch(inputs.random_spinor(dims, 3)[None])
    out = []
    for prec, n in (("f32", W["batch"]), ("f64", 1)):
        fb = tm.tm_field_bytes(g, prec, True)
        pitch = slot_pitch(fb)
        fin = torch.zeros(n * pitch, dtype=torch.uint8, device="cuda")
        for r in range(n):
            tm.tm_field_import(ctx, g, prec, 1, psi, fin[r * pitch:r * pitch + fb])
        raw = torch.zeros(n * 9 * lt * 32, dtype=torch.float64, device="cuda")
        ids = list(range(n))
        t = event_time(torch, lambda: tm.tm_contract(ctx, g, prec, n, fin, pitch, W["noise_seed"], ids, raw), 10)
        alg = V * n * CONTRACT_BYTES[prec]
        out.append({"prec": prec, "sources": n, "call_us": round(t * 1e6, 1), "us_per_source": round(t * 1e6 / n, 1),
                    "alg_bytes": alg, "alg_GBs": round(alg / t / 1e9, 1),
                    "frac_8TBs": round(alg / t / 1e9 / HBM_PEAK_GBS, 4)})
        del fin, raw
    return out


def update_rates(torch, tm, inputs, ctx, g, W):
    """The CG direction update (x += alpha p, then p = r + beta p) alone
    through tm_cg_update, on even-half fields at the solver's slot pitch, in
    the precisions the solves store them in (FP16 LP, FP32 HP inner, FP64
    plain), timed with HIP events on its stream; algorithmic bytes = p, r, x
    read and x, p written, 5 spinors per site and right-hand side."""
    dims = W["dims"]
    vh = dims[0] * dims[1] * dims[2] * dims[3] // 2
    out = []
    for prec, n in ((W["half"], W["batch"]), ("f32", W["batch"]), ("f64", W["batch"]), ("f64", 1)):
        fb = tm.tm_field_bytes(g, prec, True)
        hb = fb // 2
        pitch = slot_pitch(hb)
        tmp = torch.empty(fb, dtype=torch.uint8, device="cuda")
        fields = []
        for k in range(3):  # p, r, x: the even half of a random field in every slot
            tm.tm_field_import(ctx, g, prec, 1, tm.canonical_to_torch(inputs.random_spinor(dims, 40 + k)[None]), tmp)
            f = torch.empty(n * pitch, dtype=torch.uint8, device="cuda")
            for r in range(n):
                f[r * pitch:r * pitch + hb].copy_(tmp[:hb])
            fields.append(f)
        p, r, x = fields
        alpha, beta = [0.01] * n, [0.5] * n
        t = event_time(torch, lambda: tm.tm_cg_update(ctx, g, prec, n, p, r, x, pitch, alpha, beta), 20)
        alg = vh * n * 5 * SPINOR_BYTES[prec]
        out.append({"prec": prec, "nrhs": n, "launch_us": round(t * 1e6, 1), "alg_bytes": alg,
                    "alg_GBs": round(alg / t / 1e9, 1), "frac_8TBs": round(alg / t / 1e9 / HBM_PEAK_GBS, 4)})
        del p, r, x, fields, tmp
    return out


def plain_segment(tm, np, ctx, g, W, n_src, t_step, tsm_var, batches=(1, 12)):
    """Plain FP64 CG (Sec. 2, Eq. estiM: no TSM, FP64 to 1e-10) on the same
    GPU, one and 12 right-hand sides per launch: sources/s of each, and the
    TSM speed-up at equal statistical error against the faster of the two,
    per operator class.  The single-source variance sigma_1^2 comes from the
    n_src plain sources."""
    import torch

    lt = W["dims"][3]
    out = {"n_sources": n_src}
    best = None
    sig1 = None
    for b in batches:
        Pp = tm.tsm_params(W["kappa"], W["a"], W["noise_seed"], 0, n_src, lp=tm.solver_params("f64", tol=1e-10),
                           batch=b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rp = tm.tm_loops_tsm(ctx, g, Pp, lt)
        torch.cuda.synchronize()
        rate = n_src / (time.perf_counter() - t0)
        out[f"sources_per_s_batch{b}"] = round(rate, 3)
        if best is None or rate > best:
            best = rate
            out["rhs_per_launch"] = b
        sig1 = (rp["var_re"] + rp["var_im"]) * n_src
        out["iters_mean"] = rp["stats"]["lp_iters"] / max(1, rp["stats"]["lp_solves"])
    out["sources_per_s"] = round(best, 3)
    ok = (sig1 > 0) & (tsm_var > 0)
    eff = np.where(ok, sig1 / np.where(ok, tsm_var, 1) / t_step, np.nan)  # plain-source equivalents per s
    ratio = eff / best
    out["tsm_effective_speedup_local_median"] = float(np.nanmedian(ratio[:16]))
    out["tsm_effective_speedup_deriv_median"] = float(np.nanmedian(ratio[16:80]))
    out["tsm_effective_speedup_sym_median"] = float(np.nanmedian(ratio[80:90]))
    return out


def tsm_rate(tm, ctx, g, W, half=None, steps=2):
    """TSM loop sources/s of the workload (after one untimed step), LP in the
    given half precision; returns (sources/s, seconds per step, last result)."""
    import torch

    lt = W["dims"][3]
    P = tm.tsm_params(W["kappa"], W["a"], W["noise_seed"], W["n_hp"], W["n_lp"],
                      hp=tm.solver_params("mixed", tol=1e-10, delta=1e-3),
                      lp=tm.solver_params("lp", tol=1e-2, half=half or W["half"]), batch=W["batch"])
    tm.tm_loops_tsm(ctx, g, P, lt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = tm.tm_loops_tsm(ctx, g, P, lt)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    return (W["n_hp"] + W["n_lp"]) / t, t, r


def config_segment(tm, np, inputs, ctx, name, plain_sources=64):
    """Another benchmark configuration on its own seeded gauge field:
    tsm-24c48 (TSM sources/s with FP16 LP, per-operator loop error against
    the FP64 path, R_HP/LP, plain FP64 and the equal-error speed-up) or
    plain-16c32 (the plain FP64 method: sources/s)."""
    W = WORKLOADS[name]
    dims = W["dims"]
    t0 = time.perf_counter()
    g = tm.tm_load_gauge(ctx, dims, inputs.gauge_field(dims, W["gauge_seed"]), -1, ("f32", "f16", "bf16"))
    out = {"workload": name, "lattice": list(dims), "kappa": W["kappa"], "two_kappa_mu": W["a"]}
    try:
        if W["n_hp"] == 0:
            import torch

            Pp = tm.tsm_params(W["kappa"], W["a"], W["noise_seed"], 0, W["n_lp"],
                               lp=tm.solver_params("f64", tol=1e-10), batch=W["batch"])
            tm.tm_loops_tsm(ctx, g, Pp, dims[3])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rp = tm.tm_loops_tsm(ctx, g, Pp, dims[3])
            torch.cuda.synchronize()
            out.update(sources=W["n_lp"], rhs_per_launch=W["batch"],
                       plain_f64_sources_per_s=round(W["n_lp"] / (time.perf_counter() - t1), 2),
                       iters_mean=rp["stats"]["lp_iters"] / max(1, rp["stats"]["lp_solves"]))
        else:
            rate, t_step, r = tsm_rate(tm, ctx, g, W)
            out.update(n_hp=W["n_hp"], n_lp=W["n_lp"], tsm_sources_per_s=round(rate, 2),
                       ms_per_step=round(t_step * 1e3, 1))
            out["plain_f64"] = plain_segment(tm, np, ctx, g, W, plain_sources, t_step, r["var_re"] + r["var_im"])
            out["precision"] = precision_segment(tm, np, ctx, g, W)
            out["r_hp_lp"] = r_hp_lp(tm, ctx, g, W)
    finally:
        tm.tm_free_gauge(ctx, g)
    out["seconds"] = round(time.perf_counter() - t0, 1)
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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
        "commands": [f"rocprofv3 --pmc FETCH_SIZE -d {os.path.dirname(fetch_db)} -o fetch -- python3 bench.py "
                     f"--roofline-only",
                     f"rocprofv3 --pmc WRITE_SIZE -d {os.path.dirname(write_db)} -o write -- python3 bench.py "
                     f"--roofline-only",
                     f"python3 bench.py --traffic-from {fetch_db} {write_db}"],
    }
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


def counter_summary(out_json: str, kernel: str, bench_args: str, dbs, sites: int, sources: int) -> None:
    """Per-dispatch means of every counter that the rocprofv3 --pmc databases
    `dbs` hold for the kernels whose name contains `kernel`, with FETCH_SIZE
    and WRITE_SIZE turned into bytes by what the same counters read for the
    1 GiB streaming copy in the same run, and, where the counters are there,
    the VALU issue share (a wave64 VALU instruction takes four cycles of one
    of the 1024 SIMDs; GRBM_GUI_ACTIVE sums the cycles of the 8 XCDs), the
    time those instructions take to issue at 2.4 GHz, and the VALU lane
    instructions per site and source."""
    import sqlite3

    means, copy, commands, n = {}, {}, [], {}
    for db in dbs:
        cur = sqlite3.connect(db).cursor()
        rows = cur.execute("select kernel_name, counter_name, value from counters_collection").fetchall()
        names = sorted({c for _, c, _ in rows})
        for c in names:
            kv = [v for k, cn, v in rows if cn == c and kernel in k]
            cv = [v for k, cn, v in rows if cn == c and "k_stream_copy" in k]
            if kv:
                means[c] = sum(kv) / len(kv)
                n[c] = len(kv)
            if cv:
                copy[c] = sum(cv) / len(cv)
        commands.append(f"rocprofv3 --pmc {' '.join(names)} -d {os.path.dirname(db)} -o "
                        f"{os.path.basename(db).split('_results')[0]} -- python3 bench.py {bench_args}")
    if not means:
        raise SystemExit(f"no counter rows for kernels containing {kernel!r}")
    out = {"kernel": kernel, "bench_args": bench_args, "dispatches": n, "per_dispatch_means": means,
           "copy_kernel_per_dispatch_means": copy, "derived": {}}
    d = out["derived"]
    if "FETCH_SIZE" in means and "FETCH_SIZE" in copy:
        d["fetch_scale"] = round((1 << 30) / (copy["FETCH_SIZE"] * 1024.0), 4)
        d["fetch_bytes_per_dispatch"] = round(means["FETCH_SIZE"] * 1024.0 * d["fetch_scale"])
    if "WRITE_SIZE" in means and "WRITE_SIZE" in copy:
        d["write_scale"] = round((1 << 30) / (copy["WRITE_SIZE"] * 1024.0), 4)
        d["write_bytes_per_dispatch"] = round(means["WRITE_SIZE"] * 1024.0 * d["write_scale"])
    if "SQ_INSTS_VALU" in means:
        # the time the counted instructions take to issue at 2.4 GHz, to set
        # beside the kernel's traced duration (GRBM_GUI_ACTIVE can undercount
        # a kernel's span, so its share below may exceed 1)
        d["valu_issue_floor_us_at_2400MHz"] = round(means["SQ_INSTS_VALU"] * 4.0 / (1024.0 * 2400.0), 1)
        d["valu_lane_instructions_per_site_source"] = round(means["SQ_INSTS_VALU"] * 64.0 / (sites * sources), 1)
    if "SQ_INSTS_VALU" in means and "GRBM_GUI_ACTIVE" in means:
        cyc = means["GRBM_GUI_ACTIVE"] / 8.0
        d["gpu_cycles_per_xcd"] = round(cyc)
        d["valu_issue_busy"] = round(means["SQ_INSTS_VALU"] * 4.0 / (1024.0 * cyc), 3)
    if "TCC_HIT_sum" in means and "TCC_MISS_sum" in means:
        d["l2_hit_rate"] = round(means["TCC_HIT_sum"] / (means["TCC_HIT_sum"] + means["TCC_MISS_sum"]), 3)
    out["sites_per_dispatch"] = sites
    out["sources_per_dispatch"] = sources
    commands.append(f"python3 bench.py --counter-summary {out_json} '{kernel}' {bench_args.lstrip('-')} " +
                    " ".join(dbs))
    out["commands"] = commands
    with open(out_json, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


def trace_summary(trace_dir: str, command: str, top: int = 40) -> str:
    """Text summary of a rocprofv3 --kernel-trace --stats --output-format csv
    run: per kernel calls, total / average / min / max duration, share of the
    total kernel time, and the launch resources from the trace."""
    import csv
    import glob

    stats = glob.glob(os.path.join(trace_dir, "*_kernel_stats.csv"))
    trace = glob.glob(os.path.join(trace_dir, "*_kernel_trace.csv"))
    if not stats or not trace:
        raise SystemExit(f"{trace_dir}: no rocprofv3 kernel stats / trace csv")
    res = {}
    with open(trace[0]) as f:
        for row in csv.DictReader(f):
            res.setdefault(row["Kernel_Name"], (row["VGPR_Count"], row["Accum_VGPR_Count"], row["Scratch_Size"],
                                                int(row["Grid_Size_X"]) * int(row["Grid_Size_Y"]),
                                                row["Workgroup_Size_X"]))
    rows = []
    with open(stats[0]) as f:
        for row in csv.DictReader(f):
            rows.append(row)
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    out = ["# rocprofv3 kernel trace summary", f"# command: {command}",
           "# durations in microseconds; share of total kernel time; vgpr/agpr/scratch (bytes per lane), grid, block",
           f"{'kernel':80s} {'calls':>6s} {'total_us':>12s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} "
           f"{'share':>6s} vgpr agpr scratch grid block"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
        name = r["Name"]
        v = res.get(name, ("?", "?", "?", "?", "?"))
        out.append(f"{name[:80]:80s} {int(r['Calls']):6d} {float(r['TotalDurationNs']) / 1e3:12.1f} "
                   f"{float(r['AverageNs']) / 1e3:10.2f} {float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} "
                   f"{100 * float(r['TotalDurationNs']) / total:5.1f}% {v[0]} {v[1]} {v[2]} {v[3]} {v[4]}")
    out.append(f"# {len(rows)} kernels, {sum(int(r['Calls']) for r in rows)} dispatches, {total / 1e6:.1f} ms of kernel time")
    return "\n".join(out) + "\n"


def op_errors(tm, np, test, ref):
    """Per-operator relative error ||L_test - L_ref|| / ||L_ref|| over (t, source)
    of raw spin matrices (n, 9, T, 4, 4), summarised per operator class."""
    a = tm.tm_project_loops(test)
    b = tm.tm_project_loops(ref)
    num = np.sqrt((np.abs(a - b) ** 2).sum(axis=(0, 2)))
    den = np.sqrt((np.abs(b) ** 2).sum(axis=(0, 2)))
    e = np.where(den > 0, num / np.where(den > 0, den, 1), 0.0)
    out = {}
    for name, sl in (("local", slice(0, 16)), ("deriv", slice(16, 80)), ("sym", slice(80, 90))):
        out[name] = {"median": float(np.median(e[sl])), "max": float(e[sl].max())}
    return out


def precision_segment(tm, np, ctx, g, W, n_hp=4, n_lp=12):
    """Loop error of the precision paths against the FP64 path (itself pinned to
    the oracle at 1e-10) for the same source ids and stopping criteria:
    mixed HP vs FP64 HP at 1e-10; FP16 and BF16 LP vs FP64 LP at 1e-2."""
    lt = W["dims"][3]
    f64 = tm.solver_params("f64", tol=1e-10)
    ref = tm.tm_loops_tsm(ctx, g, tm.tsm_params(W["kappa"], W["a"], W["noise_seed"], n_hp, n_lp, hp=f64,
                                                lp=tm.solver_params("f64", tol=1e-2), batch=W["batch"]),
                          lt, want_raw=True)
    out = {"sources": {"hp": n_hp, "lp": n_hp + n_lp}, "reference": "GPU FP64 path (HP 1e-10, LP 1e-2)"}
    for half in ("f16", "bf16"):
        r = tm.tm_loops_tsm(ctx, g, tm.tsm_params(W["kappa"], W["a"], W["noise_seed"], n_hp, n_lp,
                                                  hp=tm.solver_params("mixed", tol=1e-10),
                                                  lp=tm.solver_params("lp", tol=1e-2, half=half),
                                                  batch=W["batch"]), lt, want_raw=True)
        if half == "f16":
            out["hp_mixed_vs_f64"] = op_errors(tm, np, r["raw_hp"], ref["raw_hp"])
        out[f"lp_{half}_vs_f64_lp"] = op_errors(tm, np, r["raw_lp"], ref["raw_lp"])
        d = np.abs(r["est"] - ref["est"]) / np.maximum(np.abs(ref["est"]), 1e-300)
        out[f"tsm_est_{half}_rel_median"] = float(np.median(d))
    return out


def oet_segment(tm, np, ctx, g, W, n_hp=12, n_lp=240):
    """One-end trick (isovector and isoscalar loops with TSM) against the
    standard eta^dag G s estimator on the same sources: sources/s of both, and
    for each operator class the median ratio of the TSM variance of the
    isovector one-end trick estimate (of Tr M_u^-1 X - Tr M_d^-1 X) to that of
    the standard single-flavour estimate (of Tr M_u^-1 X)."""
    lt = W["dims"][3]
    P = tm.tsm_params(W["kappa"], W["a"], W["noise_seed"] + 11, n_hp, n_lp, hp=tm.solver_params("mixed", tol=1e-10),
                      lp=tm.solver_params("lp", tol=1e-2, half=W["half"]), batch=W["batch"])
    t0 = time.perf_counter()
    ro = tm.tm_loops_oet(ctx, g, P, lt)
    t_oet = time.perf_counter() - t0
    t0 = time.perf_counter()
    rs = tm.tm_loops_tsm(ctx, g, P, lt)
    t_std = time.perf_counter() - t0
    var_o = ro["var_re_vv"] + ro["var_im_vv"]
    var_s = rs["var_re"] + rs["var_im"]
    ok = (var_s > 0) & np.isfinite(var_o)
    ratio = np.where(ok, var_o / np.where(ok, var_s, 1), np.nan)
    n = n_hp + n_lp
    return {"sources": n, "oet_sources_per_s": round(n / t_oet, 1), "standard_sources_per_s": round(n / t_std, 1),
            "isovector_variance_ratio_local_median": float(np.nanmedian(ratio[:16])),
            "isovector_variance_ratio_deriv_median": float(np.nanmedian(ratio[16:80]))}


def hpe_segment(tm, np, ctx, g, W, n_hp=12, n_lp=240):
    """Hopping parameter expansion of the local loops (with TSM) against the
    standard estimator: sources/s of tm_loops_hpe (both estimators from the
    same solves) and of tm_loops_tsm on the same sources, and the median over
    the 16 local operators and all t of the ratio of the HPE estimate's
    standard error to the standard one's."""
    lt = W["dims"][3]
    P = tm.tsm_params(W["kappa"], W["a"], W["noise_seed"] + 13, n_hp, n_lp, hp=tm.solver_params("mixed", tol=1e-10),
                      lp=tm.solver_params("lp", tol=1e-2, half=W["half"]), batch=W["batch"])
    t0 = time.perf_counter()
    rh = tm.tm_loops_hpe(ctx, g, P, lt)
    t_hpe = time.perf_counter() - t0
    t0 = time.perf_counter()
    rs = tm.tm_loops_tsm(ctx, g, P, lt)
    t_std = time.perf_counter() - t0
    var_h = (rh["var_re_hpe"] + rh["var_im_hpe"])[:16]
    var_s = (rh["var_re_std"] + rh["var_im_std"])[:16]
    ok = var_s > 0
    ratio = np.sqrt(np.where(ok, var_h / np.where(ok, var_s, 1), np.nan))
    n = n_hp + n_lp
    return {"sources": n, "hpe_sources_per_s": round(n / t_hpe, 1), "standard_sources_per_s": round(n / t_std, 1),
            "same_standard_estimate": bool(np.array_equal(rh["est_std"], rs["est"])),
            "error_ratio_local_median": float(np.nanmedian(ratio)),
            "error_ratio_local_range": [float(np.nanmin(ratio)), float(np.nanmax(ratio))]}


def tdil_segment(tm, np, ctx, g, W, t_ins=8, n_hp=12, n_lp=240):
    """Full time dilution at one insertion timeslice (one solve per noise
    vector on timeslice t_ins, with and without the expansion) against the
    undiluted estimator with the same number of solves: solves/s of both and,
    for the 16 local loops at t_ins, the median ratio of standard errors
    (time-diluted / undiluted, and time-diluted + HPE / undiluted)."""
    lt = W["dims"][3]
    P = tm.tsm_params(W["kappa"], W["a"], W["noise_seed"] + 17, n_hp, n_lp, hp=tm.solver_params("mixed", tol=1e-10),
                      lp=tm.solver_params("lp", tol=1e-2, half=W["half"]), batch=W["batch"])
    t0 = time.perf_counter()
    rd = tm.tm_loops_tdil(ctx, g, P, lt, lt, phases=[t_ins], hpe=True)
    t_dil = time.perf_counter() - t0
    t0 = time.perf_counter()
    ru = tm.tm_loops_tsm(ctx, g, P, lt)
    t_und = time.perf_counter() - t0
    vu = (ru["var_re"] + ru["var_im"])[:16, t_ins]
    vd = (rd["var_re_std"] + rd["var_im_std"])[:16, t_ins]
    vh = (rd["var_re_hpe"] + rd["var_im_hpe"])[:16, t_ins]
    n = 2 * n_hp + n_lp
    return {"t_ins": t_ins, "noise_vectors": n_hp + n_lp, "solves": n,
            "tdil_hpe_solves_per_s": round(n / t_dil, 1), "undiluted_solves_per_s": round(n / t_und, 1),
            "error_ratio_tdil_local_median": float(np.median(np.sqrt(vd / vu))),
            "error_ratio_tdil_hpe_local_median": float(np.median(np.sqrt(vh / vu))),
            "covered_local_timeslices": int(np.isfinite(rd["est_std"][0]).sum())}


def _tsm_var(np, hp, lpc, lpb):
    """TSM variance per (op, t) from per-source ops (Eq. estiTSM with sample
    variances, n - 1): s^2(hp - lpc)/N_HP + s^2(lpb)/N_LP, real + imaginary."""
    v = np.zeros(hp.shape[1:])
    if len(hp):
        d = hp - lpc
        v = v + (np.var(d.real, axis=0, ddof=1) + np.var(d.imag, axis=0, ddof=1)) / len(hp)
    if len(lpb):
        v = v + (np.var(lpb.real, axis=0, ddof=1) + np.var(lpb.imag, axis=0, ddof=1)) / len(lpb)
    return v


def tsm_scan(tm, np, ctx, g, W):
    """Tuning scan of the truncated solver method (Sec. 2.1, Fig. 1 and
    Table 1 analogues on the synthetic field):
      n_lp:        TSM error of the scalar loop and of i psibar g3 D3 psi
                   against N_LP at fixed N_HP (the error should fall as
                   N_LP^-1/2 while the correction term is small);
      truncation:  LP stopping residual against LP iterations and the
                   efficiency ratio R_C R_E^2 = (T_TSM s^2_TSM)/(T_plain s^2_plain)
                   (below 1: TSM is favourable), medians over local and
                   derivative operators and t;
      mass:        the same ratio against 2 kappa mu at the bench's kappa.
    The plain estimator is N HP solves (mixed precision to 1e-10)."""
    lt = W["dims"][3]
    hp = tm.solver_params("mixed", tol=1e-10)
    seed = W["noise_seed"] + 31
    out = {"workload": f"{W['dims'][0]}^3x{lt}", "kappa": W["kappa"]}

    # error against N_LP
    n_hp, n_lp = 24, 480
    P = tm.tsm_params(W["kappa"], W["a"], seed, n_hp, n_lp, hp=hp, lp=tm.solver_params("lp", tol=1e-2, half=W["half"]),
                      batch=W["batch"])
    r = tm.tm_loops_tsm(ctx, g, P, lt, want_raw=True)
    hp_ops, lp_ops = tm.tm_project_loops(r["raw_hp"]), tm.tm_project_loops(r["raw_lp"])
    d3 = 16 + 4 * 3 + 2  # i psibar gamma_3 D_3 psi: insertion gamma_3 (index 3), direction z
    rows = []
    for n in (30, 60, 120, 240, 480):
        v = _tsm_var(np, hp_ops, lp_ops[:n_hp], lp_ops[n_hp:n_hp + n])
        vc = _tsm_var(np, hp_ops, lp_ops[:n_hp], lp_ops[:0])
        rows.append({"n_lp": n, "sigma_scalar": float(np.median(np.sqrt(v[0]))),
                     "sigma_g3D3": float(np.median(np.sqrt(v[d3]))),
                     "correction_share_scalar": float(np.median(vc[0] / v[0]))})
    ln = np.log([x["n_lp"] for x in rows])
    out["n_lp"] = {"n_hp": n_hp, "rows": rows,
                   "slope_scalar": float(np.polyfit(ln, np.log([x["sigma_scalar"] for x in rows]), 1)[0]),
                   "slope_g3D3": float(np.polyfit(ln, np.log([x["sigma_g3D3"] for x in rows]), 1)[0])}

    def plain(a, n=24):
        Pp = tm.tsm_params(W["kappa"], a, seed + 1, 0, n, lp=hp, batch=W["batch"])
        t0 = time.perf_counter()
        rp = tm.tm_loops_tsm(ctx, g, Pp, lt)
        return time.perf_counter() - t0, rp["var_re"] + rp["var_im"], rp["stats"]["lp_iters"] / n

    def tsm(a, tol, n_hp=12, n_lp=120):
        Pt = tm.tsm_params(W["kappa"], a, seed + 2, n_hp, n_lp, hp=hp,
                           lp=tm.solver_params("lp", tol=tol, half=W["half"]), batch=W["batch"])
        t0 = time.perf_counter()
        rt = tm.tm_loops_tsm(ctx, g, Pt, lt)
        st = rt["stats"]
        return (time.perf_counter() - t0, rt["var_re"] + rt["var_im"], st["lp_iters"] / max(1, st["lp_solves"]),
                st["hp_iters"] / max(1, st["hp_solves"]))

    def ratio(tp, vp, tt, vt):
        q = (tt * vt) / (tp * vp)
        return float(np.median(q[:16])), float(np.median(q[16:80]))

    tp, vp, _ = plain(W["a"])
    rows = []
    for tol in (3e-1, 1e-1, 3e-2, 1e-2, 3e-3, 1e-3):
        tt, vt, it_lp, _ = tsm(W["a"], tol)
        loc, der = ratio(tp, vp, tt, vt)
        rows.append({"lp_tol": tol, "lp_iters": it_lp, "rc_re2_local": loc, "rc_re2_deriv": der})
    out["truncation"] = rows
    rows = []
    for a in (0.0033, 0.01, 0.03, 0.1):
        tp, vp, it_hp_plain = plain(a)
        tt, vt, it_lp, it_hp = tsm(a, 1e-2)
        loc, der = ratio(tp, vp, tt, vt)
        rows.append({"two_kappa_mu": a, "hp_iters": it_hp, "lp_iters": it_lp, "rc_re2_local": loc,
                     "rc_re2_deriv": der})
    out["mass"] = rows
    return out


def r_hp_lp(tm, ctx, g, W, n=12):
    """R_HP/LP (the paper's Table 2 analogue): GPU time of n HP sources (solve
    + contraction) over that of n LP sources, from one run with n LP-only
    sources and one with n HP sources (each with its LP partner, as the method
    requires); with the one-derivative contractions (value) and with the 16
    local loops only (local)."""
    lt = W["dims"][3]
    hp = tm.solver_params("mixed", tol=1e-10)
    lp = tm.solver_params("lp", tol=1e-2, half=W["half"])
    out = {}
    for key, local in (("value", False), ("local", True)):
        t = []
        for nh, nl in ((0, n), (n, 0)):
            P = tm.tsm_params(W["kappa"], W["a"], W["noise_seed"] + 7, nh, nl, hp=hp, lp=lp, batch=W["batch"],
                              local_only=local)
            t0 = time.perf_counter()
            tm.tm_loops_tsm(ctx, g, P, lt)
            t.append(time.perf_counter() - t0)
        out[key] = round((t[1] - t[0]) / t[0], 2)
        out["t_lp_s" if not local else "t_lp_local_s"] = round(t[0], 3)
        out["t_hp_plus_lp_s" if not local else "t_hp_plus_lp_local_s"] = round(t[1], 3)
    out["sources"] = n
    return out


def serving_segment(tm, np, inputs, ctx, g_big, W, rate_big, n_req, budget_gb=32, load=0.8, seed=5):
    """Continuous-batching serving run: Poisson arrivals of loop requests on
    four lattice sizes (the bench's 32^3x64 field and seeded fields of the
    smaller sizes), 2 kappa mu in {0.0033, 0.01}, N_HP ~ U{4..24},
    N_LP ~ U{50..500}; the arrival rate is `load` times the capacity estimated
    from the 32^3x64 throughput scaled by volume.  Latency = arrival (submit)
    to result on the server clock."""
    rng = np.random.default_rng(seed)
    sizes = [(8, 8, 8, 16), (16, 16, 16, 32), (24, 24, 24, 48), tuple(W["dims"])]
    pools = {}
    for d in sizes[:3]:
        pools[d] = [tm.tm_load_gauge(ctx, d, inputs.gauge_field(d, 40 + k), -1, ("f32", "f16", "bf16"))
                    for k in range(2 if d[0] < 24 else 1)]
    pools[sizes[3]] = [g_big]
    vbig = float(np.prod(sizes[3]))
    reqs = []
    for i in range(n_req):
        d = sizes[rng.integers(0, 4)]
        gp = pools[d][rng.integers(0, len(pools[d]))]
        a = float(rng.choice([0.0033, 0.01]))
        nh, nl = int(rng.integers(4, 25)), int(rng.integers(50, 501))
        P = tm.tsm_params(W["kappa"], a, 1000 + i, nh, nl, hp=tm.solver_params("mixed", tol=1e-10),
                          lp=tm.solver_params("lp", tol=1e-2, half=W["half"]), batch=W["batch"])
        service = (nh + nl) * float(np.prod(d)) / vbig / rate_big
        reqs.append((d, gp, P, nh + nl, service))
    mean_service = float(np.mean([r[4] for r in reqs]))
    lam = load / mean_service
    arrivals = np.cumsum(rng.exponential(1.0 / lam, n_req))
    srv = tm.tm_serve_create(ctx, slots=W["batch"], workspace_budget=int(budget_gb) << 30)
    res = {}
    stalled = False
    # a request still missing this long after the last arrival is reported, not
    # waited for; so is a server that has changed nothing for STALL_S seconds
    # while work is outstanding
    deadline = float(arrivals[-1]) + 2.0 * sum(r[4] for r in reqs) + 30.0
    STALL_S = 30.0
    try:
        t0 = time.perf_counter()
        k = 0
        next_log = 10.0
        while len(res) < n_req:
            now = time.perf_counter() - t0
            while k < n_req and arrivals[k] <= now:
                rc = tm.tm_serve_submit(srv, reqs[k][1], reqs[k][2], k)
                if rc != 0:
                    raise RuntimeError(f"serving request {k} rejected ({rc}): {tm.tm_last_error(ctx)}")
                k += 1
            for r in tm.tm_serve_poll(srv):
                res[r["tag"]] = r
            if now > next_log:
                st = tm.tm_serve_status_get(srv)
                log(f"serving: {len(res)}/{n_req} done, {k} submitted at {now:.0f}s; queued {st['queued']}, "
                    f"active {st['active']}, batches {st['batches']}, pending jobs {st['pending_jobs']}, "
                    f"slots {st['running_slots']}, arena {st['arena_used'] >> 20}/{st['arena_size'] >> 20} MiB, "
                    f"no progress for {st['stall_s']:.1f}s")
                next_log += 10.0
                if st["stall_s"] > STALL_S:
                    stalled = True
                    raise RuntimeError(f"serving: the server made no progress for {st['stall_s']:.0f}s: {st}")
            if now > deadline:
                stalled = True
                missing = sorted(set(range(k)) - set(res))
                raise RuntimeError(f"serving: requests {missing[:8]} (of {len(missing)}) not done after {now:.0f}s; "
                                   f"server {tm.tm_serve_status_get(srv)}; last error: {tm.tm_last_error(ctx)}")
            time.sleep(0.0005)
        wall = time.perf_counter() - t0
        st_end = tm.tm_serve_status_get(srv)
        # one request again alone: its result must have the same bits
        probe = min(range(n_req), key=lambda i: reqs[i][4])
        tm.tm_serve_submit(srv, reqs[probe][1], reqs[probe][2], 10 ** 6)
        alone = None
        t1 = time.perf_counter()
        while alone is None:
            for r in tm.tm_serve_poll(srv):
                alone = r
            if time.perf_counter() - t1 > 60.0:
                stalled = True
                raise RuntimeError(f"serving: the repeated request is not done after 60 s: {tm.tm_last_error(ctx)}")
            time.sleep(0.001)
    finally:
        # a stalled server still owns its requests and their gauge fields: left to the process exit
        if not stalled:
            tm.tm_serve_destroy(srv)
            for d in sizes[:3]:
                for gp in pools[d]:
                    tm.tm_free_gauge(ctx, gp)
    lat = np.array([res[i]["t_done"] - res[i]["t_submit"] for i in range(n_req)])
    wait = np.array([res[i]["t_admit"] - res[i]["t_submit"] for i in range(n_req)])
    n_src = sum(r[3] for r in reqs)
    bad = {}
    for i in range(n_req):
        if res[i]["status"] != 0:
            bad[str(res[i]["status"])] = bad.get(str(res[i]["status"]), 0) + 1
    ok = not bad
    same = bool(np.array_equal(alone["est"], res[probe]["est"]) and
                np.array_equal(alone["var_re"], res[probe]["var_re"]))
    return {
        "requests": n_req, "sources": int(n_src), "all_ok": ok, "failed_by_status": bad,
        "arrivals": f"Poisson at {load:.0%} of the volume-scaled capacity ({lam:.2f} requests/s)",
        "lattices": ["x".join(map(str, d)) for d in sizes], "slots": W["batch"], "workspace_budget_GB": budget_gb,
        "latency_p50_s": round(float(np.percentile(lat, 50)), 3), "latency_p99_s": round(float(np.percentile(lat, 99)), 3),
        "queue_wait_p50_s": round(float(np.percentile(wait, 50)), 3),
        "sources_per_s": round(n_src / wall, 1), "wall_s": round(wall, 2),
        "alone_equals_mix": same,
        # device utilisation over the mix: share of the time with a chunk on the
        # GPU, and occupied solver slots averaged over time
        "device_busy_frac": round(min(1.0, st_end["busy_s"] / wall), 3),
        "mean_occupied_slots": round(st_end["slot_s"] / wall, 2),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tsm-batched-32c64",
                    choices=sorted(k for k, w in WORKLOADS.items() if w["n_hp"] > 0))
    ap.add_argument("--plain-sources", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=200,
                    help="requests in the serving segment (0 skips it)")
    ap.add_argument("--serving-only", action="store_true", help="only the serving segment (after one warm-up step)")
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="serving arrival rate as a fraction of the volume-scaled capacity")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the hop-rate, precision, R_HP/LP, estimator-variant and serving segments")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the copy calibration and the roofline kernel (for counter runs)")
    ap.add_argument("--contract-only", action="store_true",
                    help="only the contraction rates (tm_contract; for kernel traces and counter runs)")
    ap.add_argument("--scan", metavar="OUT_JSON",
                    help="run the TSM tuning scan (after one warm-up step), write it to OUT_JSON and exit")
    ap.add_argument("--trace-summary", nargs=3, metavar=("TRACE_DIR", "OUT_TXT", "COMMAND"),
                    help="write a text summary of a rocprofv3 --kernel-trace --stats --output-format csv run "
                         "(the command that produced it as the third argument) and exit")
    ap.add_argument("--counter-summary", nargs="+", metavar="ARG",
                    help="OUT_JSON KERNEL MODE DB [DB ...]: per-dispatch counter means of the kernels whose "
                         "name contains KERNEL in rocprofv3 --pmc databases of `bench.py --MODE` runs (MODE "
                         "contract-only: 12 sources over the whole 32^3x64 lattice per dispatch; roofline-only: "
                         "12 right-hand sides over one parity), written to OUT_JSON, and exit")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="write the roofline kernel's HBM traffic from two rocprofv3 --pmc databases "
                         "(FETCH_SIZE, WRITE_SIZE) of --roofline-only runs and exit")
    args = ap.parse_args()
    if args.trace_summary:
        txt = trace_summary(args.trace_summary[0], args.trace_summary[2])
        with open(args.trace_summary[1], "w") as f:
            f.write(txt)
        print(txt, end="")
        return
    if args.traffic_from:
        write_traffic(args.traffic_from[0], args.traffic_from[1], args.workload)
        return
    if args.counter_summary:
        if len(args.counter_summary) < 4:
            ap.error("--counter-summary needs OUT_JSON KERNEL MODE DB [DB ...]")
        o, k, mode = args.counter_summary[:3]
        if mode not in ("contract-only", "roofline-only"):
            ap.error("--counter-summary: MODE is contract-only or roofline-only")
        b = "--" + mode
        Wc = WORKLOADS[args.workload]
        d0, d1, d2, d3 = Wc["dims"]
        # a contraction dispatch covers the whole lattice, a hop dispatch one parity
        sites = d0 * d1 * d2 * d3 // (2 if mode == "roofline-only" else 1)
        counter_summary(o, k, b, args.counter_summary[3:], sites=sites, sources=Wc["batch"])
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
    if args.roofline_only or args.contract_only:
        if args.roofline_only:
            out = {"roofline": measure_roofline(torch, tm, inputs, ctx, g, W, args.workload)}
        else:
            out = {"contraction_rates": contract_rates(torch, tm, inputs, ctx, g, W)}
            # the copy kernel calibrates FETCH_SIZE / WRITE_SIZE in counter runs of this mode
            nb = 1 << 30
            ca = torch.empty(nb, dtype=torch.uint8, device="cuda")
            cb = torch.empty(nb, dtype=torch.uint8, device="cuda")
            for _ in range(4):
                tm.tm_stream_copy(ctx, ca, cb, nb)
            torch.cuda.synchronize()
            del ca, cb
        print(json.dumps(out), flush=True)
        tm.tm_free_gauge(ctx, g)
        tm.tm_destroy(ctx)
        return

    hp = tm.solver_params("mixed", tol=1e-10, delta=1e-3)
    lp = tm.solver_params("lp", tol=1e-2, half=W["half"])
    P = tm.tsm_params(W["kappa"], W["a"], W["noise_seed"], W["n_hp"], W["n_lp"], hp=hp, lp=lp, batch=W["batch"])
    n_src = W["n_hp"] + W["n_lp"]

    for i in range(args.warmup):
        r = tm.tm_loops_tsm(ctx, g, P, lt)
        log(f"warmup step {i} {r['stats']['seconds']:.2f}s")
    if args.scan:
        t1 = time.perf_counter()
        scan = tsm_scan(tm, np, ctx, g, W)
        scan["command"] = f"python3 bench.py --scan {args.scan}"
        scan["seconds"] = round(time.perf_counter() - t1, 1)
        with open(args.scan, "w") as f:
            json.dump(scan, f, indent=1)
            f.write("\n")
        print(json.dumps(scan), flush=True)
        return
    if args.serving_only:
        rate = n_src / r["stats"]["seconds"]
        print(json.dumps({"serving": serving_segment(tm, np, inputs, ctx, g, W, rate, args.serve_requests,
                                                     load=args.serve_load)}), flush=True)
        return
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
        plain = plain_segment(tm, np, ctx, g, W, args.plain_sources, wall / args.steps,
                              last["var_re"] + last["var_im"])
        log(f"plain FP64: {plain['sources_per_s']:.2f} sources/s ({plain['rhs_per_launch']} RHS per launch); TSM "
            f"equal-error speedup local {plain['tsm_effective_speedup_local_median']:.1f}x deriv "
            f"{plain['tsm_effective_speedup_deriv_median']:.1f}x")

    roofline = measure_roofline(torch, tm, inputs, ctx, g, W, args.workload)
    rates = crates = urates = None
    if not args.no_extra:
        rates = kernel_rates(torch, tm, inputs, ctx, g, W)
        log("hop rates: " + ", ".join(f"{r['prec']}x{r['nrhs']} {r['launch_us']}us {r['alg_GBs']}GB/s" for r in rates))
        urates = update_rates(torch, tm, inputs, ctx, g, W)
        log("update rates: " + ", ".join(f"{r['prec']}x{r['nrhs']} {r['launch_us']}us {r['alg_GBs']}GB/s"
                                         for r in urates))
        crates = contract_rates(torch, tm, inputs, ctx, g, W)
        log("contraction: " + ", ".join(f"{r['prec']}x{r['sources']} {r['call_us']}us {r['alg_GBs']}GB/s"
                                        for r in crates))

    precision = rhl = serving = oet = hpe = tdil = bf16 = configs = None
    stalled_server = False
    if not args.no_extra:
        t0 = time.perf_counter()
        b_rate, b_step, b_last = tsm_rate(tm, ctx, g, W, half="bf16")
        bf16 = {"sources_per_s": round(b_rate, 2), "ms_per_step": round(b_step * 1e3, 1),
                "lp_iters_mean": b_last["stats"]["lp_iters"] / max(1, b_last["stats"]["lp_solves"]),
                "lp": "bf16 storage (per-site FP32 scale), FP32 arithmetic, truncated at 1e-2"}
        log(f"BF16 LP: {b_rate:.1f} sources/s")
        precision = precision_segment(tm, np, ctx, g, W)
        rhl = r_hp_lp(tm, ctx, g, W)
        oet = oet_segment(tm, np, ctx, g, W)
        log(f"one-end trick: {oet['oet_sources_per_s']} sources/s vs {oet['standard_sources_per_s']}; "
            f"isovector variance ratio local {oet['isovector_variance_ratio_local_median']:.2e}")
        hpe = hpe_segment(tm, np, ctx, g, W)
        log(f"HPE: {hpe['hpe_sources_per_s']} sources/s vs {hpe['standard_sources_per_s']}; "
            f"local error ratio {hpe['error_ratio_local_median']:.2f}")
        tdil = tdil_segment(tm, np, ctx, g, W)
        log(f"time dilution at t={tdil['t_ins']}: error ratio {tdil['error_ratio_tdil_local_median']:.2f}, "
            f"with HPE {tdil['error_ratio_tdil_hpe_local_median']:.2f} at equal solves")
        log(f"precision and R_HP/LP segments in {time.perf_counter() - t0:.1f}s; R_HP/LP {rhl['value']} "
            f"(local only {rhl['local']})")
        if args.workload == "tsm-batched-32c64":
            configs = {}
            for name in ("plain-16c32", "tsm-24c48"):
                configs[name] = config_segment(tm, np, inputs, ctx, name)
                log(f"{name}: {configs[name]}")
        if args.serve_requests > 0:
            try:
                serving = serving_segment(tm, np, inputs, ctx, g, W, value, args.serve_requests, load=args.serve_load)
            except RuntimeError as e:
                serving = {"error": str(e)}
                log(f"serving failed: {e}")
                # a stalled server still holds the device: the line is printed
                # without the CPU baseline and the process leaves without teardown
                stalled_server = "no progress" in str(e) or "not done" in str(e)
            else:
                log(f"serving: {serving['requests']} requests, p50 {serving['latency_p50_s']}s, "
                    f"p99 {serving['latency_p99_s']}s, {serving['sources_per_s']} sources/s")

    # ---- CPU oracle on a bounded sample (one LP source at the same lattice) ----
    cpu = None
    if not args.no_cpu_baseline and not stalled_server:
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
               "cpu_model": cpu_model(),
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
            "hp": "mixed FP32 CG with FP64 reliable updates (delta 0.001), tol 1e-10",
            "lp": (f"{W['half']} storage; Dslash: FP32 arithmetic ("
                   + ("FP32 FMAs with the f16 operands widened inside the instruction"
                      if W["half"] == "f16" else "bf16 widened to FP32")
                   + "); FP32 vector updates; right-hand side prepared in the same storage; FP32 "
                   + "reconstruction and contraction with FP64 sums; truncated at |r|/|r0| = 1e-2"),
            "rhs_per_launch": W["batch"],
            "parallelism": "single GPU, whole lattice resident",
        },
        "iters": {"hp_mean": st["hp_iters"] / max(1, st["hp_solves"]),
                  "lp_mean": st["lp_iters"] / max(1, st["lp_solves"]),
                  "reliable_updates": st["reliable_updates"]},
        "plain_f64": plain,
        "precision": precision,
        "r_hp_lp": rhl,
        "one_end_trick": oet,
        "hpe": hpe,
        "time_dilution": tdil,
        "serving": serving,
        "roofline": roofline,
        "kernel_rates": rates,
        "contraction_rates": crates,
        "update_rates": urates,
        "bf16_lp": bf16,
        "configs": configs,
        "cpu_baseline": cpu,
    }
    if stalled_server:
        print(json.dumps(line), flush=True)
        sys.stdout.flush()
        sys.stderr.flush()
        os._exit(0)
    tm.tm_free_gauge(ctx, g)
    tm.tm_destroy(ctx)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
