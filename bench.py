#!/usr/bin/env python3
"""Benchmark of the F-AMS pressure solve on one MI355X.

Headline workload: 3D 256x256x128 matrix grid (8.4M cells, 7-point TPFA, ln k
Gaussian random field std 4, correlation 8x8x4 cells) with 2000 random
vertical EDFM plates 20-60 cells long and 5-15 cells high (about 1M fracture
cells), fracture/matrix permeability contrast 1e6; Coupled-AMS with
coarsening 10x10x10 in the matrix and d_min = r_z = 10 in the fractures
(n_c = 17,810 coarse nodes, dense FP64 coarse inverse), truncation alpha =
1e-2; 64 right-hand sides (the Dirichlet boundary term plus 2-8 zero-sum
point sources each) reusing one setup, each solved by GMRES(30) with the
F-AMS two-stage preconditioner (multiscale stage + ILU(0)) to a relative
residual of 1e-6, in lock-step groups of 32.  The fine system is resident in
HBM before the clock starts.

One step = setup (basis functions, R, A_c and its inverse, ILU(0)) + the 64
solves.  `value` = solves per second of the precision form (FP32 basis,
ILU(0) and stage inside an FP64 outer iteration, FP64 coarse solve); the
plain FP64 form is timed beside it.  A right-hand side's latency is the time
from the start of its step to the end of the lock-step group that carries it.

Beside the headline: the error of both forms against the FP64 oracle's
pressure (cached by input hash under oracle/_pref/, written by
`python -m oracle.make_pref`), a conservative flux reconstruction with its
mass balance, per-kernel roofline figures, the oracle's CPU time on a bounded
sample, and three smaller legs (the 100x100x50 workload with all four
coupling strategies one request after another, the precision form against
FP64 across fracture contrasts, and a continuous-batching serving stream).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--legs ...]
"""
from __future__ import annotations

import argparse
import json
import os
import signal
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "solves/s + p50/p99 latency at rel. residual 1e-6, mixed-prec vs FP64 F-AMS"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6
RTOL = 1e-6
ALPHA = 1e-2
HEADLINE_NRHS = 64
GROUP = 32
RESTART = 30
VARIANT_NAMES = ["decoupled", "frac", "rock", "coupled"]
# coarse grid of each workload: (cx, cy, cz), d_min, r_z
GRIDS = {2: ((10, 10, 10), 8, 8), 3: ((10, 10, 10), 10, 10), 5: ((10, 10, 10), 10, 10)}


def say(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


# ---- algorithmic bytes per launch ---------------------------------------------
def block_bytes(name, z, K):
    """Algorithmic bytes of one launch of a lock-step kernel: every matrix
    entry and every vector entry once (gathered neighbours counted as cache
    hits).  z: sizes; K: right-hand sides per group; s: bytes per stage value
    (4 in the precision form).  The upper sweep also reads the prolongated
    coarse correction and writes the FP64 sum of the two stages (ILU(0)
    smoother without the per-medium stage, as in every lock-step leg here)."""
    n, nnz, zp, nc, s = z["n"], z["nnz"], z["nnz_P"], z["n_coarse"], z["s"]
    half = (nnz - n) / 2.0
    return {
        "bresid_outer": nnz * 12 + 4 * (n + 1) + 3 * K * n * 8,
        "bspmv": nnz * 12 + 4 * (n + 1) + 2 * K * n * 8,
        "bspmv_resid": nnz * (s + 4) + 4 * (n + 1) + 3 * K * n * s,
        "brestrict": zp * (s + 4) + 4 * (nc + 1) + K * n * s + K * nc * 8,
        "bcoarse": 8.0 * nc * nc + 2 * K * nc * 8,
        "bprolong": zp * (s + 4) + 4 * (n + 1) + K * nc * 8 + K * n * s,
        "bilu_lower": half * (s + 4) + 12 * n + 3 * K * n * s,
        "bilu_upper": (half + n) * (s + 4) + 12 * n + 2 * K * n * s + K * n * (s + 8),
        "bdot": K * n * 8,
        "bscale": 2 * K * n * 8,
        "bpack": 2 * K * n * 8,
        "bcast_d2f": K * n * 12,
        "badd": K * n * (2 * s + 8),
    }.get(name)


def arnoldi_steps(its, group, restart):
    """Basis sizes j + 1 of every Arnoldi step of the lock-step FGMRES: a
    group runs as many steps as its slowest right-hand side, restart cycles
    of `restart` steps."""
    jv = []
    for g0 in range(0, len(its), group):
        left = max(its[g0:g0 + group])
        while left > 0:
            c = min(restart, left)
            jv += list(range(1, c + 1))
            left -= c
    return jv


def krylov_bytes(name, z, K, jv):
    """Algorithmic bytes of all launches of one Gram-Schmidt kernel of the
    lock-step FGMRES, from the basis size j of every step (j = 1..30 in a
    restart cycle).  Two-pass form: the dots read the j - 1 finished vectors,
    the candidate and w; the update reads the same and writes the finished
    vector and the next candidate.  CGS2 form (restarts above 32): the
    multi-dot reads V_0..V_j and w; the fused correction + dots and the
    correction + norm read V_0..V_j and read and write w."""
    vec = z["n"] * K * 8.0
    extra = {"bgs_dots": 1, "bgs_update": 3, "bmdot": 1, "bmaxpy_mdot": 2,
             "bmaxpy_norm": 2}.get(name)
    return None if extra is None else sum((j + extra) * vec for j in jv)


def single_bytes(name, z):
    """The same for the one-right-hand-side kernels (the 100x100x50 leg)."""
    n, nnz, zp, nc, s = z["n"], z["nnz"], z["nnz_P"], z["n_coarse"], z["s"]
    half = (nnz - n) / 2.0
    return {
        "ilu_lower": half * (s + 4) + n * (s + 12) + n * s,
        "ilu_upper": (half + n) * (s + 4) + n * 12 + n * s,
        "spmv_resid": nnz * (s + 4) + 4 * (n + 1) + 3 * s * n,
        "spmv": nnz * 12 + 4 * (n + 1) + 2 * 8 * n,
        "prolong": zp * (s + 4) + 4 * (n + 1) + 8 * nc + s * n,
        "restrict": zp * (s + 4) + 4 * (nc + 1) + s * n + 8 * nc,
        "coarse_gemv": 8.0 * nc * nc,
    }.get(name)


TRAFFIC_DIR = os.path.join(ROOT, "profiles")


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed PMC summary of
    `workload`, or None when absent or taken on other sources."""
    try:
        with open(os.path.join(TRAFFIC_DIR, f"traffic_{workload}.json")) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    from paper_1705_05784_amd.profiling import source_digest
    if t.get("source_digest") != source_digest():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("traffic_bytes_per_launch")


def hbm_entry(name, stats, per_launch, workload):
    tot_ms, cnt = stats[name]
    avg_s = tot_ms / cnt * 1e-3
    ach = per_launch / avg_s / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic(workload, name),
            "algorithmic_bytes_per_launch": per_launch, "avg_launch_us": avg_s * 1e6,
            "launches": cnt}


# ---- inputs ---------------------------------------------------------------------
def load_system(config, dev, contrast=None):
    """A workload and its coarse grids, resident on `dev`."""
    import torch
    from paper_1705_05784_amd import fams
    from workloads import make_config
    sysm = make_config(config, contrast=contrast)
    coarse, d_min, r_z = GRIDS[config]
    wb, pr, vx, _ = fams.full_grid(sysm, coarse, d_min, r_z)
    A = dict(row_ptr=torch.from_numpy(sysm.row_ptr).to(dev),
             col=torch.from_numpy(sysm.col).to(dev), val=torch.from_numpy(sysm.val).to(dev),
             wb=torch.from_numpy(wb).to(dev), pr=torch.from_numpy(pr).to(dev),
             vx=torch.from_numpy(vx).to(dev))
    torch.cuda.synchronize()
    return sysm, A


def solver(sysm, A, variant, precision, profile=False):
    from paper_1705_05784_amd import fams
    return fams.Solver(A["row_ptr"], A["col"], A["val"], sysm.n_matrix, A["wb"], A["pr"], A["vx"],
                       variant=variant, precision=precision, alpha=ALPHA, profile=profile,
                       allocator="torch")


PREF_DIR = os.path.join(ROOT, "oracle", "_pref")


def pref_lookup(sysm, q):
    """The oracle's pressure for (A, q) when `python -m oracle.make_pref` has
    computed and stored it (a data file keyed by the input's hash; nothing
    of the oracle runs here)."""
    from workloads.edfm import system_key
    key = system_key(sysm.row_ptr, sysm.col, sysm.val, q)
    path = os.path.join(PREF_DIR, key + ".npy")
    if not os.path.exists(path):
        return None, key, None
    meta = None
    try:
        with open(path[:-4] + ".json") as f:
            meta = json.load(f)
    except (OSError, ValueError):
        pass
    return np.load(path).astype(np.float64), key, meta


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ---- the headline: 64 right-hand sides on one setup ---------------------------------
def headline(args, dev):
    import torch
    from paper_1705_05784_amd import fams
    from workloads.configs import config_rhs
    t0 = time.perf_counter()
    sysm, A = load_system(5, dev)
    Qh = config_rhs(sysm, 5, HEADLINE_NRHS)
    Q = torch.from_numpy(Qh).to(dev)
    torch.cuda.synchronize()
    say(f"config 5 ready: n={sysm.n} nnz={sysm.nnz} ({time.perf_counter() - t0:.1f} s)")

    def step(precision, profile=False, keep=False):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        S = solver(sysm, A, fams.COUPLED, precision, profile)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - ts
        lat, its, resid, P = [], [], [], []
        for g0 in range(0, HEADLINE_NRHS, GROUP):
            p, info = S.solve(Q[g0:g0 + GROUP], rtol=RTOL, max_iter=1000)
            torch.cuda.synchronize()
            t = time.perf_counter() - ts
            lat += [t] * len(info)
            its += [i["iterations"] for i in info]
            resid += [i["rel_residual"] for i in info]
            if not all(i["status"] == 0 for i in info):
                raise SystemExit(f"bench.py: a right-hand side did not converge: {info}")
            if keep:
                P.append(p)
            else:
                del p
        total = time.perf_counter() - ts
        out = dict(total=total, setup=t_setup, lat=lat, its=its, resid=resid,
                   setup_info=S.setup_info())
        if profile:
            out["stats"] = S.kernel_stats()
        if keep:
            out["P"] = torch.cat(P)
            out["S"] = S
        else:
            S.close()
        return out

    def leg(precision, k, warm):
        for _ in range(warm):
            step(precision)
        res = [step(precision) for _ in range(k)]
        tot = sum(r["total"] for r in res)
        lat = np.array([x for r in res for x in r["lat"]]) * 1e3
        its = [x for r in res for x in r["its"]]
        solve_s = sum(r["total"] - r["setup"] for r in res)
        return dict(solves_per_s=HEADLINE_NRHS * k / tot, ms_per_step=tot * 1e3 / k,
                    p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                    setup_ms_mean=float(np.mean([r["setup"] for r in res]) * 1e3),
                    solve_ms_per_rhs=solve_s * 1e3 / (HEADLINE_NRHS * k),
                    iterations_mean=float(np.mean(its)), iterations_max=int(max(its)),
                    cell_iterations_per_s=sysm.n * sum(its) / solve_s,
                    max_rel_residual=max(x for r in res for x in r["resid"]),
                    fp32_fallback_blocks=int(res[-1]["setup_info"]["fp32_fallback_blocks"]),
                    long_waits=int(sum(r["setup_info"]["long_waits"] for r in res)),
                    steps=k, setup_info=res[-1]["setup_info"])

    say(f"config 5: mixed, {args.warmup} warm-up + {args.steps} timed steps")
    m = leg(fams.MIXED, args.steps, args.warmup)
    m_si = m.pop("setup_info")
    k64 = max(1, min(args.steps, args.fp64_steps))
    say(f"config 5: fp64, {min(args.warmup, 1)} warm-up + {k64} timed steps")
    f = leg(fams.FP64, k64, min(args.warmup, 1))
    f.pop("setup_info")

    # accuracy: the timed tolerance against the oracle, and a tight solve
    acc = {}
    p_ref, key, meta = pref_lookup(sysm, Qh[0])
    acc["p_ref"] = (f"oracle GMRES (Decoupled-AMS) of right-hand side 0 to rel. residual "
                    f"{meta['rtol'] if meta else '?'}, key {key}" if p_ref is not None
                    else f"not cached (key {key}; python -m oracle.make_pref --config 5)")
    say("config 5: accuracy and flux")
    outs = {}
    for name, prec in (("mixed", fams.MIXED), ("fp64", fams.FP64)):
        S = solver(sysm, A, fams.COUPLED, prec)
        p6, i6 = S.solve(Q[0], rtol=RTOL, max_iter=1000)
        p10, i10 = S.solve(Q[0], rtol=1e-10, max_iter=2000)
        outs[name] = (p6.cpu().numpy(), p10.cpu().numpy(), i10[0])
        if name == "mixed":
            torch.cuda.synchronize()
            tf = time.perf_counter()
            _, _, imb = S.reconstruct_flux(Q[0], p6)
            torch.cuda.synchronize()
            acc["flux_ms_first"] = (time.perf_counter() - tf) * 1e3
            tf = time.perf_counter()
            _, _, imb2 = S.reconstruct_flux(Q[1], S.solve(Q[1], rtol=RTOL)[0])
            torch.cuda.synchronize()
            acc["flux_ms_next_incl_solve"] = (time.perf_counter() - tf) * 1e3
            acc["max_flux_imbalance"] = max(imb, imb2)
        S.close()
    acc["mixed_vs_fp64_at_rtol_1e-6"] = rel(outs["mixed"][0], outs["fp64"][0])
    acc["mixed_vs_fp64_at_rtol_1e-10"] = rel(outs["mixed"][1], outs["fp64"][1])
    acc["iterations_rtol_1e-10"] = {k: v[2]["iterations"] for k, v in outs.items()}
    acc["rel_residual_rtol_1e-10"] = {k: v[2]["rel_residual"] for k, v in outs.items()}
    if p_ref is not None:
        for k in ("mixed", "fp64"):
            acc[f"err_{k}_rtol_1e-6"] = rel(outs[k][0], p_ref)
            acc[f"err_{k}_rtol_1e-10"] = rel(outs[k][1], p_ref)
        acc["target_1e-6_met_at_rtol_1e-10"] = acc["err_mixed_rtol_1e-10"] <= 1e-6

    # profiled replica of one mixed step: HIP events around every launch on
    # the stream it runs on
    roof, kernels = None, {}
    if not args.no_profile:
        say("config 5: profiled step")
        r = step(fams.MIXED, profile=True)
        st = r["stats"]
        kernels = {k: v for k, v in st.items()}
        si = r["setup_info"]
        z = dict(n=si["n"], nnz=si["nnz"], nnz_P=si["nnz_P"], n_coarse=si["n_coarse"], s=4)
        entries = {}
        for name in st:
            b = block_bytes(name, z, GROUP)
            if b is not None:
                entries[name] = hbm_entry(name, st, b, "edfm3d_256x256x128")
        jv = arnoldi_steps(r["its"], GROUP, RESTART)
        for name in ("bgs_dots", "bgs_update", "bmdot", "bmaxpy_mdot", "bmaxpy_norm"):
            if name in st and st[name][1] == len(jv):
                entries[name] = hbm_entry(name, st, krylov_bytes(name, z, GROUP, jv) / len(jv),
                                          "edfm3d_256x256x128")
                entries[name]["note"] = ("average over the launches: basis sizes 1..30 per "
                                         "restart cycle, the group's slowest right-hand side")
        nc = si["n_coarse"]
        gje = [k for k in st if k.startswith("gje") or k == "gemm_mfma"]
        gje_ms = sum(st[k][0] for k in gje)
        gflop = 2.0 * nc ** 3
        entries["coarse_inverse"] = {
            "bound": "mfma", "kernel": "+".join(sorted(gje)),
            "achieved": gflop / (gje_ms * 1e-3) / 1e12, "peak": FP64_MFMA_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": gflop / (gje_ms * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS,
            "traffic": None, "algorithmic_flops": gflop, "total_ms": gje_ms,
            "note": "Gauss-Jordan inverse of A_c, 2 n_c^3 flops over all its launches"}
        gm = st.get("gemm_mfma")
        if gm:
            # the GEMMs alone: 2 n^2 1024 per block step plus the two panel products
            nb, steps_ = 1024, -(-nc // 1024)
            g_flop = sum(2.0 * nc * nc * min(nb, nc - k * nb) + 4.0 * nc * min(nb, nc - k * nb) ** 2
                         for k in range(steps_))
            entries["gemm_mfma"] = {
                "bound": "mfma", "kernel": "gemm_mfma", "achieved": g_flop / (gm[0] * 1e-3) / 1e12,
                "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": g_flop / (gm[0] * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS,
                "traffic": measured_traffic("edfm3d_256x256x128", "gemm_mfma"),
                "algorithmic_flops": g_flop, "avg_launch_us": gm[0] / gm[1] * 1e3,
                "launches": gm[1],
                "note": "block-step products of the inverse (the inner 32-wide steps' small "
                        "products are counted in the time, not in the flops)"}
        dom = max(st, key=lambda k: st[k][0])
        roof = entries.get(dom)
        if roof is None:
            roof = {"bound": "alu", "kernel": dom, "achieved": None, "peak": None, "unit": None,
                    "frac": None, "traffic": None, "avg_launch_us": st[dom][0] / st[dom][1] * 1e3}
        kernels = {"roofline_kernels": entries, "dominant": dom,
                   "kernels_ms": {k: round(v[0], 3) for k, v in
                                  sorted(st.items(), key=lambda kv: -kv[1][0])[:16]}}
    cfg = {"workload": ("EDFM 3D 256x256x128 + 2000 plates (contrast 1e6, ln k std 4), "
                        "Coupled-AMS, coarsening 10^3 / d_min=r_z=10, alpha 1e-2, 64 right-hand "
                        "sides per setup in lock-step groups of 32, FGMRES(30) to 1e-6; "
                        "step = setup + 64 solves"),
           "n": int(sysm.n), "n_matrix": int(sysm.n_matrix), "nnz": int(sysm.nnz),
           "n_coarse": int(m_si["n_coarse"]), "nnz_P": int(m_si["nnz_P"]),
           "device_bytes_peak_mixed": int(m_si["peak_device_bytes"]),
           "nrhs": HEADLINE_NRHS, "t_ratio": float(sysm.t_ratio)}
    return m, f, acc, roof, kernels, cfg


def pmc_step(dev):
    """One mixed step of the headline workload (setup + 64 solves), untimed."""
    import torch
    from paper_1705_05784_amd import fams
    from workloads.configs import config_rhs
    sysm, A = load_system(5, dev)
    Q = torch.from_numpy(config_rhs(sysm, 5, HEADLINE_NRHS)).to(dev)
    S = solver(sysm, A, fams.COUPLED, fams.MIXED)
    for g0 in range(0, HEADLINE_NRHS, GROUP):
        S.solve(Q[g0:g0 + GROUP], rtol=RTOL, max_iter=1000)
    torch.cuda.synchronize()
    S.close()


# ---- the 100x100x50 workload: four coupling strategies ------------------------------
def leg_config2(args, dev):
    import torch
    from paper_1705_05784_amd import fams
    sysm, A = load_system(2, dev)
    q = torch.from_numpy(sysm.q).to(dev)

    def request(variant, precision, profile=False):
        t0 = time.perf_counter()
        S = solver(sysm, A, variant, precision, profile)
        t1 = time.perf_counter()
        p, info = S.solve(q, outer="gmres", restart=30, rtol=RTOL, max_iter=1000)
        t2 = time.perf_counter()
        _, _, imb = S.reconstruct_flux(q, p)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        out = dict(total=t3 - t0, setup=t1 - t0, solve=t2 - t1, flux=t3 - t2, info=info[0],
                   imbalance=imb, p=p.cpu().numpy(), si=S.setup_info())
        if profile:
            out["stats"] = S.kernel_stats()
        S.close()
        return out

    k = max(1, min(args.steps, 3))
    res = {}
    for name, prec in (("mixed", fams.MIXED), ("fp64", fams.FP64)):
        for v in range(4):
            request(v, prec)
        t0 = time.perf_counter()
        rs = [request(v, prec) for _ in range(k) for v in range(4)]
        tot = time.perf_counter() - t0
        lat = np.array([r["total"] for r in rs]) * 1e3
        res[name] = dict(solves_per_s=len(rs) / tot, p50_ms=float(np.percentile(lat, 50)),
                         p99_ms=float(np.percentile(lat, 99)),
                         setup_ms_mean=float(np.mean([r["setup"] for r in rs]) * 1e3),
                         solve_ms_mean=float(np.mean([r["solve"] for r in rs]) * 1e3),
                         flux_ms_mean=float(np.mean([r["flux"] for r in rs]) * 1e3),
                         slowest_request_ms={
                             "setup": float(max(r["setup"] for r in rs) * 1e3),
                             "solve": float(max(r["solve"] for r in rs) * 1e3),
                             "flux": float(max(r["flux"] for r in rs) * 1e3),
                             "total": float(max(r["total"] for r in rs) * 1e3)},
                         long_waits=int(sum(r["si"]["long_waits"] for r in rs)),
                         iterations={VARIANT_NAMES[i]: rs[i]["info"]["iterations"]
                                     for i in range(4)},
                         max_flux_imbalance=max(r["imbalance"] for r in rs),
                         p=[r["p"] for r in rs[:4]])
    p_ref, key, _ = pref_lookup(sysm, sysm.q)
    for name in ("mixed", "fp64"):
        ps = res[name].pop("p")
        if p_ref is not None:
            res[name]["max_err_vs_oracle"] = max(rel(p, p_ref) for p in ps)
    res["speedup_mixed_vs_fp64"] = res["mixed"]["solves_per_s"] / res["fp64"]["solves_per_s"]
    if not args.no_profile:
        r = request(fams.COUPLED, fams.MIXED, profile=True)
        si = r["si"]
        z = dict(n=si["n"], nnz=si["nnz"], nnz_P=si["nnz_P"], n_coarse=si["n_coarse"], s=4)
        res["roofline_kernels"] = {
            nm: hbm_entry(nm, r["stats"], single_bytes(nm, z), "edfm3d_100x100x50")
            for nm in r["stats"] if single_bytes(nm, z) is not None}
    res["workload"] = ("EDFM 3D 100x100x50 + 100 plates (contrast 1e4), coarsening 10^3 / "
                       "d_min=r_z=8, alpha 1e-2, each request = setup + FGMRES(30) to 1e-6 + "
                       "flux, the four coupling strategies one after another")
    res["steps"] = k
    res["oracle_p_ref"] = key if p_ref is not None else None
    return res


# ---- the precision form across fracture contrasts (200x200x50 + 400 plates) ---------
def leg_contrast(args, dev):
    import torch
    from paper_1705_05784_amd import fams
    out = {"workload": ("EDFM 3D 200x200x50 + 400 plates, Coupled-AMS, coarsening 10^3 / "
                        "d_min=r_z=10, alpha 1e-2, both forms iterated to 1e-10")}
    for c in args.contrasts:
        sysm, A = load_system(3, dev, contrast=c)
        q = torch.from_numpy(sysm.q).to(dev)
        p_ref, key, meta = pref_lookup(sysm, sysm.q)
        row = {"t_ratio": float(sysm.t_ratio), "oracle_p_ref": key if p_ref is not None else None}
        ps = {}
        for name, prec in (("mixed", fams.MIXED), ("fp64", fams.FP64)):
            t0 = time.perf_counter()
            S = solver(sysm, A, fams.COUPLED, prec)
            p, info = S.solve(q, rtol=1e-10, max_iter=3000)
            _, _, imb = S.reconstruct_flux(q, p)
            torch.cuda.synchronize()
            ps[name] = p.cpu().numpy()
            row[name] = dict(status=info[0]["status"], iterations=info[0]["iterations"],
                             rel_residual=info[0]["rel_residual"], balance=imb,
                             ms=(time.perf_counter() - t0) * 1e3)
            if p_ref is not None:
                row[name]["err_vs_oracle"] = rel(ps[name], p_ref)
            S.close()
        row["mixed_vs_fp64"] = rel(ps["mixed"], ps["fp64"])
        if meta:
            row["oracle_rel_residual"] = meta.get("rel_residual")
            row["oracle_balance"] = meta.get("balance")
        out[f"{c:g}"] = row
        del A
        torch.cuda.empty_cache()
    return out


# ---- the serving stream ----------------------------------------------------------
def leg_serving(args):
    """Continuous batching of a Poisson stream of setup + solve requests
    (cubes of side 32-128 with 10-300 plates, 1-16 right-hand sides each),
    in worker processes of their own on the one GPU.  The dispatcher and its
    workers run in a session of their own; past the time limit the whole
    process group is killed and waited for, so that nothing of this leg is
    left on the GPU when the headline starts."""
    cmd = [sys.executable, "-m", "paper_1705_05784_amd.serving", "--requests",
           str(args.serving_requests), "--slots", "2", "--load", "0.7"]
    # its progress lines pass through on stderr
    proc = subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True, cwd=ROOT,
                            start_new_session=True)
    try:
        out, _ = proc.communicate(timeout=args.serving_timeout)
    except subprocess.TimeoutExpired:
        os.killpg(proc.pid, signal.SIGKILL)
        proc.communicate()
        _wait_group_gone(proc.pid)
        return {"error": f"timed out after {args.serving_timeout} s", "requests":
                args.serving_requests}
    _wait_group_gone(proc.pid)
    try:
        return json.loads(out.strip().splitlines()[-1])
    except Exception as e:  # reported, never required for the headline
        return {"error": f"{type(e).__name__}: {e}", "rc": proc.returncode}


def _wait_group_gone(pgid, limit_s=60.0):
    """Wait until no process of group `pgid` is left (the serving workers)."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < limit_s:
        try:
            os.killpg(pgid, 0)
        except ProcessLookupError:
            return
        time.sleep(0.2)


def cpu_baseline(timeout=600):
    """The FP64 oracle, single-threaded, on a bounded sample: one
    Decoupled-AMS request (setup + GMRES(30) to 1e-6) of the 100x100x50
    workload, in a child process."""
    code = r"""
import json, os, time, sys
sys.path.insert(0, os.getcwd())
from workloads import make_config
from oracle import grids, fams
s = make_config(2)
wb, pr, vx, ncm = grids.full_grid(s, (10, 10, 10), 8, 8)
t0 = time.perf_counter()
F = fams.FAMS(s.csr(), wb, vx, s.n_matrix, fams.DECOUPLED, alpha=1e-2)
t1 = time.perf_counter()
p, info = F.gmres(s.q, rtol=1e-6)
t2 = time.perf_counter()
print(json.dumps(dict(setup_s=t1 - t0, solve_s=t2 - t1, iterations=info["iterations"], n=s.n)))
"""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    env["HIP_VISIBLE_DEVICES"] = ""
    hi = host_info()
    try:
        out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                             env=env, timeout=timeout, cwd=ROOT)
        r = json.loads(out.stdout.strip().splitlines()[-1])
    except Exception as e:  # the baseline is reported, never required
        return {"value": None, "unit": "solves/s", "cores": 1, "kind": "oracle",
                "sample": f"failed: {e}", **hi}
    tot = r["setup_s"] + r["solve_s"]
    return {"value": 1.0 / tot, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"one Decoupled-AMS request of the 100x100x50 workload (n = {r['n']}; "
                       f"setup + GMRES(30) to 1e-6, {r['iterations']} iterations): setup "
                       f"{r['setup_s']:.1f} s, solve {r['solve_s']:.1f} s, FP64, 1 thread; "
                       f"the headline workload has 15x the cells"), **hi}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=3,
                    help="timed steps of the plain FP64 form (at most --steps)")
    ap.add_argument("--legs", nargs="*", default=["config2", "contrast", "serving"],
                    choices=["config2", "contrast", "serving"])
    ap.add_argument("--contrasts", type=float, nargs="*", default=[1e2, 1e4, 1e6, 1e8])
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--serving-timeout", type=int, default=600)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="a 1 GiB device copy, then one mixed step of the headline workload "
                         "(the program run under rocprofv3 --pmc for the traffic figures)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the F-AMS solve here runs on one GPU; run with --gpus 1 "
              "(sharding across GPUs is described, not implemented)", file=sys.stderr)
        sys.exit(2)

    if args.pmc_pass:
        import torch
        dev = torch.device("cuda", 0)
        torch.cuda.set_device(dev)
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)   # copy calibration: 1 GiB read, 1 GiB written
        torch.cuda.synchronize()
        del a, b
        args.steps, args.warmup, args.fp64_steps, args.no_profile = 1, 0, 0, True
        pmc_step(dev)
        print(json.dumps({"pmc_pass": True, "copy_bytes": 1 << 30}))
        return

    serving = leg_serving(args) if "serving" in args.legs else None   # before this process uses the GPU

    import torch
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    m, f, acc, roof, kern, cfg = headline(args, dev)
    legs = {}
    if "config2" in args.legs:
        say("leg: 100x100x50, four strategies")
        legs["edfm3d_100x100x50"] = leg_config2(args, dev)
    if "contrast" in args.legs:
        say("leg: contrast sweep")
        legs["contrast_200x200x50"] = leg_contrast(args, dev)
    if serving is not None:
        legs["serving"] = serving
    cpu = None if args.no_cpu_baseline else cpu_baseline()
    line = {
        "metric": METRIC,
        "value": m["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64",
        "data": "synthetic",
        "config": cfg,
        "p50_ms": m["p50_ms"],
        "p99_ms": m["p99_ms"],
        "mixed": m,
        "fp64": f,
        "speedup_mixed_vs_fp64": m["solves_per_s"] / f["solves_per_s"],
        "accuracy": acc,
        "roofline": roof,
        **kern,
        "cpu_baseline": cpu,
        "legs": legs,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
