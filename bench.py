#!/usr/bin/env python3
"""Benchmark of the F-AMS pressure solve on one MI355X.

Workload: 3D 100x100x50 matrix grid (7-point TPFA, ln k Gaussian random field
std 3, correlation 8x8x4 cells) with 100 random vertical EDFM plates 20-60
cells long and 10-40 cells high, fracture/matrix permeability contrast 1e4;
coarsening 10x10x10 in the matrix and d_min = r_z = 8 in the fractures;
truncation alpha = 1e-2; GMRES(30) preconditioned by the F-AMS two-stage
step (multiscale stage + ILU(0)) to ||r||/||r0|| <= 1e-6.

One step = one request per coupling strategy (Decoupled, Frac, Rock and
Coupled-AMS), each request = setup (basis functions, R, A_c and its LU,
ILU(0)) + solve + conservative flux reconstruction, with the fine system
already resident in HBM.  By default the four requests of a step run side by
side, one worker process per strategy on the one GPU (each worker loads the
system onto the device before the clock starts); `--concurrency 1` runs them
one after another, and those sequential figures are reported too.  `value` =
requests (solves) per second in the precision form; the plain FP64 form is
timed beside it.  Latency p50/p99 are per request.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

METRIC = "solves/s + p50/p99 latency at rel. residual 1e-6, mixed-prec vs FP64 F-AMS"
HBM_PEAK_GBS = 8000.0
COARSE = (10, 10, 10)
D_MIN, R_Z = 8, 8
ALPHA = 1e-2
RTOL = 1e-6
VARIANT_NAMES = ["decoupled", "frac", "rock", "coupled"]


def algorithmic_bytes(name, sizes, s):
    """Bytes a kernel must move per full application (not per launch).

    n cells, z = nnz(A), zp = nnz(P), nc coarse nodes, s bytes per value.
    Gathered vector entries (x[col]) are taken as cache hits: the
    algorithmic minimum streams the matrix once and each vector once."""
    n, z, zp, nc = sizes["n"], sizes["nnz"], sizes["nnz_P"], sizes["n_coarse"]
    half = (z - n) / 2.0
    if name == "ilu_lower":
        return half * (s + 4) + n * (s + 12) + n * s
    if name == "ilu_upper":
        return (half + n) * (s + 4) + n * 12 + n * s
    if name == "spmv_resid":
        return z * (s + 4) + 4 * (n + 1) + 3 * s * n
    if name == "spmv":
        return z * (8 + 4) + 4 * (n + 1) + 2 * 8 * n
    if name == "prolong":
        return zp * (s + 4) + 4 * (n + 1) + 8 * nc + s * n
    if name == "restrict":
        return zp * (s + 4) + 4 * (nc + 1) + s * n + 8 * nc
    if name == "coarse_gemv":
        return 8.0 * nc * nc
    return None


ITERATION_KERNELS = ("ilu_lower", "ilu_upper", "spmv_resid", "spmv", "prolong", "restrict",
                     "coarse_gemv")
FP32_VECTOR_PEAK_TFLOPS = 157.3
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "traffic_edfm3d_100x100x50.json")


def source_digest():
    """Hash of the HIP sources: measured traffic is only valid for the code
    it was measured on."""
    import hashlib
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1705_05784_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed PMC summary, or
    None if absent or taken on other sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_digest") != source_digest():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("traffic_bytes_per_launch")


def cpu_baseline(timeout=600):
    """The FP64 oracle, single-threaded, on one request of the same workload
    (Decoupled-AMS: setup + GMRES(30) to 1e-6), in a child process."""
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
print(json.dumps(dict(setup_s=t1 - t0, solve_s=t2 - t1, iterations=info["iterations"])))
"""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    env["HIP_VISIBLE_DEVICES"] = ""
    try:
        out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                             env=env, timeout=timeout, cwd=os.path.dirname(os.path.abspath(__file__)))
        r = json.loads(out.stdout.strip().splitlines()[-1])
    except Exception as e:  # the baseline is reported, never required
        return {"value": None, "unit": "solves/s", "cores": 1, "kind": "oracle",
                "sample": f"failed: {e}"}
    tot = r["setup_s"] + r["solve_s"]
    return {"value": 1.0 / tot, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": ("one Decoupled-AMS request of the same workload (setup + GMRES(30) "
                       f"to 1e-6, {r['iterations']} iterations): setup {r['setup_s']:.1f} s, "
                       f"solve {r['solve_s']:.1f} s, FP64, 1 thread")}


def _load_workload(dev):
    """The bench system and its coarse grids, resident on `dev`."""
    import torch
    from paper_1705_05784_amd import fams
    from workloads import make_config
    sysm = make_config(2)
    wb, pr, vx, _ = fams.full_grid(sysm, COARSE, D_MIN, R_Z)
    A = dict(row_ptr=torch.from_numpy(sysm.row_ptr).to(dev),
             col=torch.from_numpy(sysm.col).to(dev),
             val=torch.from_numpy(sysm.val).to(dev),
             wb=torch.from_numpy(wb).to(dev), pr=torch.from_numpy(pr).to(dev),
             vx=torch.from_numpy(vx).to(dev))
    q = torch.from_numpy(sysm.q).to(dev)
    torch.cuda.synchronize()
    return sysm, A, q


def _request(sysm, A, q, variant, precision, profile=False):
    """One request: setup + FGMRES(30) to RTOL + flux reconstruction."""
    import torch
    from paper_1705_05784_amd import fams
    t0 = time.perf_counter()
    S = fams.Solver(A["row_ptr"], A["col"], A["val"], sysm.n_matrix, A["wb"], A["pr"],
                    A["vx"], variant=variant, precision=precision, alpha=ALPHA,
                    profile=profile)
    t1 = time.perf_counter()
    p, info = S.solve(q, outer="gmres", restart=30, rtol=RTOL, max_iter=1000)
    t2 = time.perf_counter()
    flux, pfv, imb = S.reconstruct_flux(q, p)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    out = dict(total=t3 - t0, setup=t1 - t0, solve=t2 - t1, flux=t3 - t2, info=info[0],
               imbalance=imb, setup_info=S.setup_info(), p=p)
    if profile:
        out["stats"] = S.kernel_stats()
    S.close()
    return out


def _concurrent_worker(conn, variant):
    """One coupling strategy's requests, in a process of its own on GPU 0:
    loads the system once, then runs ("run", precision, k) batches."""
    try:
        import torch
        dev = torch.device("cuda", 0)
        torch.cuda.set_device(dev)
        sysm, A, q = _load_workload(dev)
        conn.send(("ready", None))
        while True:
            msg = conn.recv()
            if msg[0] == "stop":
                break
            _, precision, k = msg
            res = []
            for _ in range(k):
                r = _request(sysm, A, q, variant, precision)
                r["p"] = r["p"].cpu().numpy()
                res.append(r)
            conn.send(("done", res))
    except Exception as e:  # reported to the parent, which fails the run
        conn.send(("error", f"{type(e).__name__}: {e}"))
    conn.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="one mixed step plus a 1 GiB device copy (for rocprofv3 --pmc runs)")
    ap.add_argument("--concurrency", type=int, default=4, choices=(1, 4),
                    help="4: the four requests of a step run side by side, one worker "
                         "process per coupling strategy; 1: one after another")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the F-AMS solve here runs on one GPU; run with --gpus 1 "
              "(sharding across GPUs is described, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    # worker processes first, before this process touches the GPU
    workers = []
    if args.concurrency > 1 and not args.pmc_pass:
        import multiprocessing as mp
        ctx = mp.get_context("spawn")
        for v in range(4):
            parent, child = ctx.Pipe()
            proc = ctx.Process(target=_concurrent_worker, args=(child, v), daemon=True)
            proc.start()
            child.close()
            workers.append((proc, parent))

    from paper_1705_05784_amd import fams

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    sysm, A, q = _load_workload(dev)

    def request(variant, precision, profile=False):
        return _request(sysm, A, q, variant, precision, profile)

    def gather(tag_expected):
        out = []
        for _, conn in workers:
            tag, payload = conn.recv()
            if tag == "error":
                raise SystemExit(f"bench.py: a worker failed: {payload}")
            assert tag == tag_expected
            out.append(payload)
        return out

    def run_concurrent(precision, k):
        """The four strategies side by side; the clock runs from the start
        signal until every worker has finished (each synchronises its device
        after every request)."""
        t0 = time.perf_counter()
        for _, conn in workers:
            conn.send(("run", precision, k))
        per = gather("done")
        t = time.perf_counter() - t0
        res = []
        for step in range(k):  # step-major, strategy order within a step
            for v in range(4):
                r = per[v][step]
                r["p"] = torch.from_numpy(r["p"]).to(dev)
                res.append(r)
        return t, res

    def run_steps(precision, k, profile=False):
        res = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            for v in range(4):
                res.append(request(v, precision, profile))
        torch.cuda.synchronize()
        return time.perf_counter() - t0, res

    if args.pmc_pass:
        # copy calibration: one elementwise kernel reading 1 GiB and writing 1 GiB
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
        run_steps(fams.MIXED, 1)
        print(json.dumps({"pmc_pass": True, "copy_bytes": 1 << 30}))
        return

    conc = None
    if workers:
        gather("ready")
        run_concurrent(fams.MIXED, args.warmup)
        run_concurrent(fams.FP64, args.warmup)
        conc = (run_concurrent(fams.MIXED, args.steps), run_concurrent(fams.FP64, args.steps))
        for proc, conn in workers:
            conn.send(("stop",))
            proc.join(timeout=60)

    for _ in range(args.warmup):
        run_steps(fams.MIXED, 1)
        run_steps(fams.FP64, 1)
    t_mixed, r_mixed = run_steps(fams.MIXED, args.steps)
    t_fp64, r_fp64 = run_steps(fams.FP64, args.steps)

    # reference pressure for the error statement: FP64, tight tolerance
    S = fams.Solver(A["row_ptr"], A["col"], A["val"], sysm.n_matrix, A["wb"], A["pr"], A["vx"],
                    variant=0, precision=fams.FP64, alpha=ALPHA)
    p_ref, _ = S.solve(q, rtol=1e-12, max_iter=2000)
    S.close()
    nref = float(torch.linalg.norm(p_ref))

    def summarize(tot, res):
        lat = np.array([r["total"] * 1e3 for r in res])
        errs = [float(torch.linalg.norm(r["p"] - p_ref)) / nref for r in res]
        its = [r["info"]["iterations"] for r in res]
        solve_s = sum(r["solve"] for r in res)
        return dict(solves_per_s=len(res) / tot, ms_per_step=tot * 1e3 / args.steps,
                    p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                    setup_ms_mean=float(np.mean([r["setup"] for r in res]) * 1e3),
                    solve_ms_mean=float(np.mean([r["solve"] for r in res]) * 1e3),
                    flux_ms_mean=float(np.mean([r["flux"] for r in res]) * 1e3),
                    iterations={VARIANT_NAMES[i % 4]: its[i] for i in range(4)},
                    cell_iterations_per_s=sysm.n * sum(its) / solve_s,
                    max_rel_pressure_error=max(errs),
                    max_rel_residual=max(r["info"]["rel_residual"] for r in res),
                    max_flux_imbalance=max(r["imbalance"] for r in res),
                    fp32_fallback_blocks=int(sum(r["setup_info"]["fp32_fallback_blocks"]
                                                 for r in res)))

    m = summarize(t_mixed, r_mixed)
    f = summarize(t_fp64, r_fp64)
    sequential = None
    if conc is not None:  # the headline numbers are the side-by-side ones
        sequential = dict(mixed=m, fp64=f)
        m = summarize(*conc[0])
        f = summarize(*conc[1])
    si = r_mixed[-1]["setup_info"]
    sizes = dict(n=si["n"], nnz=si["nnz"], nnz_P=si["nnz_P"], n_coarse=si["n_coarse"],
                 ilu_levels_lower=si["ilu_levels_lower"], ilu_levels_upper=si["ilu_levels_upper"])

    roofline = None
    roofline_iter = None
    kernels = {}
    if not args.no_profile:
        # a profiled replica of the timed mixed steps: HIP events around every
        # launch, recorded on the stream the kernel runs on
        _, r_prof = run_steps(fams.MIXED, args.steps, profile=True)
        flops = {"local_solve": 0.0, "local_subst": 0.0}
        for r in r_prof:
            flops["local_solve"] += r["setup_info"]["local_flops"]
            flops["local_subst"] += r["setup_info"]["local_subst_flops"]
            for name, (ms, cnt) in r["stats"].items():
                a = kernels.setdefault(name, [0.0, 0])
                a[0] += ms
                a[1] += cnt

        def hbm_entry(name):
            per_launch = algorithmic_bytes(name, sizes, 4)   # FP32 preconditioner
            tot_ms, cnt = kernels[name]
            avg_s = tot_ms / cnt * 1e-3
            ach = per_launch / avg_s / 1e9
            tr = measured_traffic(name)
            return {"bound": "hbm", "kernel": name, "achieved": ach, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": tr,
                    "algorithmic_bytes_per_launch": per_launch, "avg_launch_us": avg_s * 1e6,
                    "launches": cnt}

        dom = max(kernels, key=lambda k: kernels[k][0])
        if dom in flops:
            tot_ms, cnt = kernels[dom]
            ach = flops[dom] / (tot_ms * 1e-3) / 1e12
            roofline = {"bound": "alu", "kernel": dom, "achieved": ach,
                        "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": ach / FP32_VECTOR_PEAK_TFLOPS, "traffic": measured_traffic(dom),
                        "algorithmic_flops_per_launch": flops[dom] / cnt,
                        "avg_launch_us": tot_ms / cnt * 1e3, "launches": cnt}
        elif algorithmic_bytes(dom, sizes, 4) is not None:
            roofline = hbm_entry(dom)
        else:
            roofline = {"bound": "alu", "kernel": dom, "achieved": None, "peak": None,
                        "unit": None, "frac": None, "traffic": None,
                        "avg_launch_us": kernels[dom][0] / kernels[dom][1] * 1e3}
        it = [k for k in ITERATION_KERNELS if k in kernels]
        if it:
            roofline_iter = hbm_entry(max(it, key=lambda k: kernels[k][0]))

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
        "config": {"workload": ("EDFM 3D 100x100x50 + 100 plates (contrast 1e4), coarsening "
                                "10^3 / d_min=r_z=8, alpha 1e-2, 4 coupling strategies, "
                                "FGMRES(30) to 1e-6, setup+solve+flux per request"),
                   "n": sizes["n"], "n_matrix": sysm.n_matrix, "nnz": sizes["nnz"],
                   "n_coarse": sizes["n_coarse"], "t_ratio": sysm.t_ratio,
                   "concurrency": ("4 requests side by side (one worker process per coupling "
                                   "strategy, inputs resident on the GPU)"
                                   if conc is not None else "1 (requests one after another)")},
        "p50_ms": m["p50_ms"],
        "p99_ms": m["p99_ms"],
        "mixed": m,
        "fp64": f,
        "speedup_mixed_vs_fp64": m["solves_per_s"] / f["solves_per_s"],
        "sequential": sequential,
        "roofline": roofline,
        "roofline_iteration": roofline_iter,
        "kernels_ms": {k: round(v[0], 3) for k, v in sorted(kernels.items(),
                                                            key=lambda kv: -kv[1][0])[:12]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
