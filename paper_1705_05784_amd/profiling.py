"""Summaries of rocprofv3 output (rocpd SQLite databases).

    python -m paper_1705_05784_amd.profiling trace DB TITLE COMMAND [TOP]
        markdown table of per-kernel dispatch counts and durations
    python -m paper_1705_05784_amd.profiling traffic FETCH_DB WRITE_DB COPY_BYTES OUT.json
        HBM bytes per launch from FETCH_SIZE / WRITE_SIZE counter runs, each
        scaled by what the counter reads for the plain device copy of
        COPY_BYTES read + COPY_BYTES written that the run also performs

Kernel names are shortened to the function name with its template
arguments.  Host-only; nothing here touches the GPU.
"""
from __future__ import annotations

import json
import os
import sqlite3
import sys


def source_digest() -> str:
    """Hash of the library's HIP and C++ sources: a measured traffic figure is
    only valid for the code it was measured on."""
    import hashlib
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".cpp")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    n = name.replace("fams::(anonymous namespace)::", "").replace("void ", "")
    out = ""
    for ch in n:          # drop the argument list, keep template arguments
        if ch == "(":
            break
        out += ch
    return out.strip()


def _columns(cur, table):
    return [r[1] for r in cur.execute(f"pragma table_info({table})")]


def kernel_rows(db):
    cur = sqlite3.connect(db).cursor()
    return list(cur.execute(
        "select name, count(*), sum(duration), avg(duration) from kernels group by name "
        "order by sum(duration) desc"))


def trace_markdown(db, title, cmd, top=20) -> str:
    rows = kernel_rows(db)
    total = sum(r[2] for r in rows)
    lines = [f"# {title}", "", "Command (run from the repository root on one MI355X):", "",
             "```", cmd, "```", "",
             "Per-kernel durations from the rocprofv3 kernel trace (`kernels` view of the "
             "trace database; a duration is end - start of one dispatch).", "",
             "| kernel | calls | total ms | avg us | % of GPU time |", "|---|---:|---:|---:|---:|"]
    for n, c, tot, avg in rows[:top]:
        lines.append(f"| `{short(n)}` | {c} | {tot / 1e6:.2f} | {avg / 1e3:.2f} | "
                     f"{100 * tot / total:.1f} |")
    lines += ["", f"Total GPU kernel time: {total / 1e6:.1f} ms over "
              f"{sum(r[1] for r in rows)} dispatches."]
    return "\n".join(lines) + "\n"


def counter_per_kernel(db, counter):
    """{short kernel name: (dispatches, mean counter value per dispatch)}."""
    cur = sqlite3.connect(db).cursor()
    cols = _columns(cur, "counters_collection")
    kcol = next(c for c in ("kernel_name", "name") if c in cols)
    ncol = next(c for c in ("counter_name", "counter") if c in cols)
    vcol = next(c for c in ("value", "counter_value") if c in cols)
    dcol = next((c for c in ("dispatch_id", "id") if c in cols), None)
    q = (f"select {kcol}, {dcol}, sum({vcol}) from counters_collection where {ncol} = ? "
         f"group by {kcol}, {dcol}") if dcol else \
        (f"select {kcol}, rowid, {vcol} from counters_collection where {ncol} = ?")
    acc = {}
    for k, _, v in cur.execute(q, (counter,)):
        a = acc.setdefault(short(k), [0, 0.0])
        a[0] += 1
        a[1] += float(v)
    return {k: (c, s / c) for k, (c, s) in acc.items()}


def _copy_kernel(per):
    cands = [k for k in per if "copy" in k.lower() or "elementwise" in k.lower()]
    if not cands:
        raise SystemExit("no copy kernel in the counter run")
    return max(cands, key=lambda k: per[k][1])


def launch_name(symbol, launch_names=None):
    """The library's timer name of a kernel symbol: an exact entry of
    `launch_names`, else the longest key ending in '*' that prefixes it (the
    instantiations of one templated pass share one timer), else the symbol."""
    names = launch_names or {}
    if symbol in names:
        return names[symbol]
    best = None
    for k, v in names.items():
        if k.endswith("*") and symbol.startswith(k[:-1]) and (best is None or len(k) > len(best[0])):
            best = (k, v)
    return best[1] if best else symbol


def traffic(fetch_db, write_db, copy_bytes, out_json, source_digest, launch_names=None):
    fetch = counter_per_kernel(fetch_db, "FETCH_SIZE")
    write = counter_per_kernel(write_db, "WRITE_SIZE")
    ck_f, ck_w = _copy_kernel(fetch), _copy_kernel(write)
    # bytes per counter unit: the copy reads and writes copy_bytes each
    f_scale = copy_bytes / fetch[ck_f][1]
    w_scale = copy_bytes / write[ck_w][1]
    kernels = {}
    for k in fetch:
        if k not in write or k in (ck_f, ck_w):
            continue
        name = launch_name(k, launch_names)
        d = fetch[k][0]
        e = kernels.setdefault(name, {"symbols": [], "dispatches": 0, "fetch_kib": 0.0,
                                      "write_kib": 0.0, "bytes": 0.0})
        e["symbols"].append(k)
        e["dispatches"] += d
        e["fetch_kib"] += fetch[k][1] * d
        e["write_kib"] += write[k][1] * d
        e["bytes"] += (fetch[k][1] * f_scale + write[k][1] * w_scale) * d
    # per launch: averages over the dispatches of every symbol of one timer
    for name, e in list(kernels.items()):
        d = max(e["dispatches"], 1)
        kernels[name] = {"symbols": e["symbols"], "dispatches": e["dispatches"],
                         "fetch_kib_per_dispatch": e["fetch_kib"] / d,
                         "write_kib_per_dispatch": e["write_kib"] / d,
                         "traffic_bytes_per_launch": e["bytes"] / d}
    out = {"copy_kernel": ck_f, "copy_bytes": copy_bytes,
           "fetch_bytes_per_unit": f_scale, "write_bytes_per_unit": w_scale,
           "source_digest": source_digest, "kernels": kernels}
    with open(out_json, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    return out


# library kernel symbols -> the launch names used by the library's own timers
LAUNCH_NAMES = {
    "k_local_solve<float, float>": "local_solve",
    "k_sweep_ranges<float, false>": "ilu_lower", "k_sweep_ranges<float, true>": "ilu_upper",
    "k_sweep_lower<float>": "ilu_lower", "k_sweep_upper<float>": "ilu_upper",
    # lock-step kernels of the precision form with 32 right-hand sides
    "k_bsweep<float, false, 32>": "bilu_lower", "k_bsweep<float, true, 32>": "bilu_upper",
    "k_bspmv_ell<double, double, double, double, 32, true>": "bresid_outer",
    "k_bspmv_ell<double, double, double, double, 32, false>": "bspmv",
    "k_bspmv_ell<float, float, float, float, 32, true>": "bspmv_resid",
    "k_bspmv_ell<float, double, float, float, 32, false>": "bprolong",
    "k_brestrict<float, float, 32>": "brestrict", "k_bcoarse_mfma<32>": "bcoarse",
    "k_bcast<double, float>": "bcast_d2f",
    "k_gemm_mfma128": "gemm_mfma",
    # the Gram-Schmidt passes, one instantiation per basis size bucket
    "k_bmaxpy_mdot<32,*": "bmaxpy_mdot", "k_bmaxpy_norm<32,*": "bmaxpy_norm",
    "k_bmdot<32,*": "bmdot", "k_bmdot<32, 1>": "bdot",
    "k_dcgs_dots<32,*": "bgs_dots", "k_dcgs_update<32,*": "bgs_update",
}


def _main(argv):
    if len(argv) >= 4 and argv[0] == "trace":
        top = int(argv[4]) if len(argv) > 4 else 20
        sys.stdout.write(trace_markdown(argv[1], argv[2], argv[3], top))
        return 0
    if len(argv) == 5 and argv[0] == "traffic":
        out = traffic(argv[1], argv[2], int(argv[3]), argv[4], source_digest(), LAUNCH_NAMES)
        print(json.dumps({k: round(v["traffic_bytes_per_launch"]) for k, v in
                          out["kernels"].items()}, indent=1))
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(_main(sys.argv[1:]))
