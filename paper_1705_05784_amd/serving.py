"""Serving form: continuous batching of F-AMS setup + solve requests.

Requests arrive over time (each: a fine system with its coarse grids, a basis
variant and 1..16 right-hand sides).  A dispatcher admits them first come,
first served, as soon as a slot is free and the HBM reservation of the
requests in flight plus the new request's footprint (fams_footprint plus its
input and vector buffers) stays within the budget.  Each slot is a worker
process with its own HIP context on the same GPU (ProcessRunner): it runs
fams_setup, reuses that setup for every right-hand side (fams_solve,
optionally fams_reconstruct_flux), frees it and reports back, and the
dispatcher releases the reservation.  Kernels of different slots overlap on
the device; every kernel reduces in a fixed order, so a request's result
does not depend on what runs beside it.

Several host threads calling the library at once inside one process are not
used: such a run once ended in a host crash whose cause was not found, so
the in-process runner (GpuRunner) serves one slot only.

The execution of one request is a replaceable callable (`runner`), so the
admission logic is testable without a device.
"""
from __future__ import annotations

import sys
import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class ServedResult:
    rid: int
    status: int = 0
    error: str = ""
    iterations: list = field(default_factory=list)
    rel_residual: list = field(default_factory=list)
    pressures: np.ndarray | None = None   # [nrhs, n] when kept
    imbalance: list = field(default_factory=list)
    footprint: int = 0
    t_arrival: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0
    setup_ms: float = 0.0
    long_waits: int = 0     # dependency waits over ~1 ms in the request's sweeps/LU solves
    slot: int = -1

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


def prepare(requests, coarse=(10, 10, 10), d_min=8, r_z=8):
    """Build each distinct system's coarse grids once (host helpers) and keep
    them, with the coarse size, in the request's meta; grids are inputs of
    fams_setup, like the matrix."""
    from . import fams
    cache = {}
    for r in requests:
        key = id(r.system)
        if key not in cache:
            wb, pr, vx, _ = fams.full_grid(r.system, coarse, d_min, r_z)
            cache[key] = (wb, pr, vx)
        r.meta["grid"] = cache[key]
        r.meta["n_coarse"] = len(cache[key][2])
    return requests


def request_footprint(req, precision: int, restart: int = 30) -> int:
    """Device bytes a request may hold: the library's setup + workspace bound
    (lock-step work space for all of its right-hand sides), the borrowed
    inputs and the right-hand-side / pressure buffers."""
    from . import fams
    s = req.system
    nc = int(req.meta["n_coarse"])
    lib_bytes = fams.footprint(s.n, s.nnz, nc, precision, restart, int(req.rhs.shape[0]))
    inputs = 8 * (s.n + 1) + 12 * s.nnz + 13 * s.n + 8 * nc
    vectors = 2 * 8 * s.n * req.rhs.shape[0] + 2 * 8 * s.nnz
    return int(lib_bytes + inputs + vectors)


def _execute(system, grid, variant, rhs, precision, alpha, rtol, restart, flux, keep) -> dict:
    """Run one request on the current device and stream: one setup, reused
    for every right-hand side."""
    import torch

    from . import fams
    s = system
    out = dict(status=0, error="", iterations=[], rel_residual=[], imbalance=[], pressures=None,
               setup_ms=0.0)
    t0 = time.perf_counter()
    solver = fams.Solver(s["row_ptr"], s["col"], s["val"], s["n_matrix"], *grid, variant=variant,
                         precision=precision, alpha=alpha)
    try:
        out["setup_ms"] = (time.perf_counter() - t0) * 1e3
        q = torch.from_numpy(np.ascontiguousarray(rhs)).to("cuda")
        # every right-hand side of the request in one call: lock-step groups
        P, infos = solver.solve(q if q.shape[0] > 1 else q[0], outer=fams.GMRES,
                                restart=restart, rtol=rtol)
        P = P.reshape(q.shape)
        for k, info in enumerate(infos):
            out["iterations"].append(info["iterations"])
            out["rel_residual"].append(info["rel_residual"])
            out["status"] = max(out["status"], info["status"])
            if flux:
                _, _, imb = solver.reconstruct_flux(q[k], P[k])
                out["imbalance"].append(imb)
        if keep:
            out["pressures"] = P.cpu().numpy()
        torch.cuda.current_stream().synchronize()
        out["long_waits"] = int(solver.setup_info()["long_waits"])
    finally:
        solver.close()
    return out


def _system_arrays(req):
    s = req.system
    return dict(row_ptr=s.row_ptr, col=s.col, val=s.val, n_matrix=s.n_matrix)


def _fill(res: ServedResult, out: dict):
    res.status = out["status"]
    res.error = out["error"]
    res.iterations = out["iterations"]
    res.rel_residual = out["rel_residual"]
    res.imbalance = out["imbalance"]
    res.pressures = out["pressures"]
    res.setup_ms = out["setup_ms"]
    res.long_waits = out.get("long_waits", 0)


class GpuRunner:
    """Executes a request in this process on the current device and stream
    (one slot only)."""

    in_process = True

    def __init__(self, precision, alpha=1e-2, rtol=1e-6, restart=30, flux=False,
                 keep_pressures=False):
        self.args = (precision, alpha, rtol, restart, flux, keep_pressures)

    def __call__(self, req, res: ServedResult):
        _fill(res, _execute(_system_arrays(req), req.meta["grid"], req.variant, req.rhs, *self.args))


def _worker_main(conn, device, args):
    """Slot process: receives systems once, then runs requests on them."""
    import torch
    torch.cuda.set_device(device)
    from . import fams
    fams.lib()
    systems = {}
    conn.send(("ready", None))
    while True:
        msg = conn.recv()
        if msg[0] == "stop":
            break
        if msg[0] == "system":
            systems[msg[1]] = msg[2]
            continue
        _, key, variant, rhs = msg
        sysd, grid = systems[key]
        try:
            out = _execute(sysd, grid, variant, rhs, *args)
        except Exception as e:  # reported to the dispatcher; the slot goes on
            out = dict(status=-1, error=f"{type(e).__name__}: {e}", iterations=[],
                       rel_residual=[], imbalance=[], pressures=None, setup_ms=0.0)
        conn.send(("done", out))
    conn.close()


class ProcessRunner:
    """One worker process per slot, all on `device`.  Slot k of the server
    runs its requests in process k; each process receives a system's arrays
    the first time one of its requests uses it."""

    def __init__(self, slots, precision, alpha=1e-2, rtol=1e-6, restart=30, flux=False,
                 keep_pressures=False, device=0, timeout=600.0):
        import multiprocessing as mp
        ctx = mp.get_context("spawn")
        self.timeout = timeout
        self.conns, self.procs, self.sent = [], [], []
        args = (precision, alpha, rtol, restart, flux, keep_pressures)
        try:
            for _ in range(slots):
                a, b = ctx.Pipe()
                p = ctx.Process(target=_worker_main, args=(b, device, args), daemon=True)
                p.start()
                b.close()
                self.conns.append(a)
                self.procs.append(p)
                self.sent.append(set())
            for c in self.conns:
                if not c.poll(timeout):
                    raise TimeoutError("serving slot process did not start")
                c.recv()
        except BaseException:
            self.close()
            raise

    @property
    def slots(self):
        return len(self.conns)

    def __call__(self, req, res: ServedResult):
        c = self.conns[res.slot]
        key = id(req.system)
        if key not in self.sent[res.slot]:
            c.send(("system", key, (_system_arrays(req), req.meta["grid"])))
            self.sent[res.slot].add(key)
        c.send(("run", key, req.variant, req.rhs))
        if not c.poll(self.timeout):
            raise TimeoutError(f"request {req.rid} did not finish in {self.timeout} s")
        _, out = c.recv()
        _fill(res, out)

    def close(self):
        for c in self.conns:
            try:
                c.send(("stop",))
            except Exception:
                pass
        for p in self.procs:
            p.join(timeout=30)
            if p.is_alive():
                p.terminate()
                p.join(timeout=10)
        self.conns, self.procs = [], []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """Continuous-batching request loop.

    slots: requests in flight at most; hbm_budget: bytes the requests in
    flight may reserve together (default: 90% of the device's free memory
    when run() starts).
    """

    def __init__(self, runner, slots: int = 8, hbm_budget: int | None = None,
                 footprint=None, progress: int = 0):
        self.runner = runner
        self.slots = int(slots)
        self.hbm_budget = hbm_budget
        self.footprint = footprint
        self.progress = int(progress)  # a line on stderr every `progress` completions
        self.peak_inflight = 0
        self.peak_reserved = 0

    def run(self, requests, realtime: bool = True) -> list[ServedResult]:
        if getattr(self.runner, "in_process", False) and self.slots > 1:
            raise ValueError("the in-process runner serves one slot; use ProcessRunner")
        if hasattr(self.runner, "slots") and self.runner.slots < self.slots:
            raise ValueError("runner has fewer slot processes than the server has slots")
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        budget = self.hbm_budget
        if budget is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            budget = int(0.9 * free)
        fp = self.footprint or (lambda r: 0)
        results = {r.rid: ServedResult(r.rid, t_arrival=r.arrival) for r in reqs}
        cv = threading.Condition()
        jobs: deque = deque()
        state = dict(reserved=0, inflight=0, done=0, stop=False)
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        def worker(slot):
            while True:
                with cv:
                    while not jobs and not state["stop"]:
                        cv.wait()
                    if not jobs:
                        return
                    req, need = jobs.popleft()
                res = results[req.rid]
                res.slot = slot
                try:
                    self.runner(req, res)
                except Exception as e:  # a failed request reports, the server goes on
                    res.status = -1
                    res.error = f"{type(e).__name__}: {e}"
                with cv:
                    res.t_done = now()
                    state["reserved"] -= need
                    state["inflight"] -= 1
                    state["done"] += 1
                    if self.progress and state["done"] % self.progress == 0:
                        print(f"[serving] {state['done']}/{len(reqs)} requests done at "
                              f"{res.t_done:.1f} s", file=sys.stderr, flush=True)
                    cv.notify_all()

        threads = [threading.Thread(target=worker, args=(k,), daemon=True) for k in range(self.slots)]
        for t in threads:
            t.start()
        pending: deque = deque()
        nxt = 0
        arrive = (lambda r: r.arrival) if realtime else (lambda r: 0.0)
        try:
            with cv:
                while state["done"] < len(reqs):
                    t = now()
                    while nxt < len(reqs) and arrive(reqs[nxt]) <= t:
                        pending.append(reqs[nxt])
                        if not realtime:
                            results[reqs[nxt].rid].t_arrival = 0.0
                        nxt += 1
                    while pending and state["inflight"] < self.slots:
                        r = pending[0]
                        need = int(fp(r))
                        res = results[r.rid]
                        res.footprint = need
                        if need > budget:           # can never fit: reject
                            pending.popleft()
                            res.status, res.error = -6, f"footprint {need} B exceeds budget {budget} B"
                            res.t_admit = res.t_done = t
                            state["done"] += 1
                            continue
                        if state["reserved"] + need > budget:
                            break                    # first come, first served
                        pending.popleft()
                        res.t_admit = t
                        state["reserved"] += need
                        state["inflight"] += 1
                        self.peak_inflight = max(self.peak_inflight, state["inflight"])
                        self.peak_reserved = max(self.peak_reserved, state["reserved"])
                        jobs.append((r, need))
                        cv.notify_all()
                    if state["done"] >= len(reqs):
                        break
                    wait = None
                    if nxt < len(reqs):
                        wait = max(0.0, arrive(reqs[nxt]) - now())
                    cv.wait(wait if wait is None else max(wait, 1e-4))
        finally:
            with cv:
                state["stop"] = True
                cv.notify_all()
            for t in threads:
                t.join()
        return [results[r.rid] for r in sorted(reqs, key=lambda r: r.rid)]


def summarize(results, cells=None) -> dict:
    """p50/p99 latency (s), solves/s over the makespan, cell-iterations/s."""
    ok = [r for r in results if r.status >= 0]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    t_first = min(r.t_arrival for r in results) if results else 0.0
    t_last = max(r.t_done for r in results) if results else 0.0
    span = max(t_last - t_first, 1e-9)
    solves = sum(len(r.iterations) for r in ok)
    out = dict(requests=len(results), failed=len(results) - len(ok), solves=solves,
               makespan_s=span, solves_per_s=solves / span,
               p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)))
    if cells is not None:
        ci = sum(cells[r.rid] * sum(r.iterations) for r in ok)
        out["cell_iterations_per_s"] = ci / span
    return out


def _main(argv=None):
    """Run a seeded request stream and print one JSON line of serving figures."""
    import argparse
    import json
    import sys

    from . import fams
    from workloads.serving import make_stream

    ap = argparse.ArgumentParser(description="F-AMS serving run (continuous batching)")
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--rate", type=float, default=20.0, help="Poisson arrivals per second")
    ap.add_argument("--load", type=float, default=None,
                    help="arrival rate as a fraction of the measured closed-loop capacity "
                         "(overrides --rate): the first --probe requests are first run with "
                         "all arrivals at t = 0, and their completions per second set mu")
    ap.add_argument("--probe", type=int, default=48)
    # two slot processes: with four, the spin-waiting dataflow kernels of the
    # processes stalled one another (48 requests at once: 92 s and 4 requests
    # over the 2 s wait bound, against 12 s with one slot and 8.2 s with two)
    ap.add_argument("--slots", type=int, default=2)
    ap.add_argument("--pool", type=int, default=8, help="distinct systems in the stream")
    ap.add_argument("--side", type=int, nargs=2, default=(32, 128))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--fp64", action="store_true", help="plain FP64 form instead of mixed")
    a = ap.parse_args(argv)
    prec = fams.FP64 if a.fp64 else fams.MIXED
    reqs = prepare(make_stream(a.requests, 1.0, pool=a.pool, seed=a.seed, side=tuple(a.side)))
    gaps = np.diff([0.0] + [r.arrival for r in reqs])   # unit-rate Poisson gaps
    cells = {r.rid: r.system.n for r in reqs}
    print(f"[serving] {len(reqs)} requests ready", file=sys.stderr, flush=True)
    mu = None
    with ProcessRunner(a.slots, prec, alpha=1e-2, rtol=1e-6) as run:
        srv = Server(run, slots=a.slots, footprint=lambda r: request_footprint(r, prec),
                     progress=16)
        rate = a.rate
        if a.load is not None:
            probe = reqs[:max(1, min(a.probe, len(reqs)))]
            pres = srv.run(probe, realtime=False)
            span = max(r.t_done for r in pres)
            mu = len(probe) / span
            rate = a.load * mu
            print(f"[serving] closed-loop capacity {mu:.2f} requests/s -> rate {rate:.2f}",
                  file=sys.stderr, flush=True)
        t = 0.0
        for r, g in zip(reqs, gaps):
            t += g / rate
            r.arrival = t
        srv = Server(run, slots=a.slots, footprint=lambda r: request_footprint(r, prec),
                     progress=32)
        res = srv.run(reqs, realtime=True)
    a.rate = rate
    out = summarize(res, cells)
    errs = {}
    for r in res:
        if r.status < 0:
            key = r.error.split(":")[0] + ": " + r.error.split(":")[-1].strip()[:120]
            errs.setdefault(key, []).append((r.rid, cells[r.rid]))
    out["errors"] = {k: v for k, v in errs.items()}
    out.update(slots=a.slots, rate=a.rate, load=a.load, capacity_requests_per_s=mu,
               precision="fp64" if a.fp64 else "mixed",
               peak_inflight=srv.peak_inflight, peak_reserved_gb=srv.peak_reserved / 2**30,
               mean_setup_ms=float(np.mean([r.setup_ms for r in res if r.status >= 0])),
               max_setup_ms=float(max(r.setup_ms for r in res if r.status >= 0)),
               max_latency_s=float(max(r.latency for r in res if r.status >= 0)),
               long_waits=int(sum(r.long_waits for r in res)),
               mean_iterations=float(np.mean([np.mean(r.iterations) for r in res if r.iterations])),
               cells_range=[min(cells.values()), max(cells.values())])
    print(json.dumps(out))


if __name__ == "__main__":
    import sys
    sys.exit(_main())
