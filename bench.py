"""Benchmark: partition-ordered FLUX5 forward + adjoint on one MI355X.

Workload (default): the 3D tetrahedral-mesh dual graph of a Kuhn 55^3 box,
n = 998,250 cells, m = 1,978,350 interior faces, 5 float32 states per cell,
face normal + area per edge, capacity 256, loss L = 1/2 sum r^2 (so the
adjoint's upstream gradient is r).  One step = forward (part kernel +
reduction) then adjoint (part kernel + reduction) over the whole mesh, inputs
resident in HBM.  The partitioned (EP) order gives `value`; the default
(cell-major input) order is timed the same way alongside, as the paper
compares its orders (Section 5.2, with memory transactions per order in
Figures 10 and 14; here the L2-miss bytes of rocprofv3's request counters).

Prints one JSON line.  Step time: the timed steps captured in one HIP graph
and replayed.  Kernel durations: each kernel's own dispatch timestamps
(epk_run_stage_timed), warm and after a read-only 1 GiB cache scrub.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
GRAPH_TIMING = True  # cleared by --eager
COLD_STEPS = 20  # set by --cold-steps
REPLAYS = 20  # timed replays of the K-step graph for the spread
WARM_REPLAYS = 3  # untimed replays of a captured graph before its timed one
SPMV_Y_WEIGHT = 4  # SpMV partition: a replicated y (partial, reduction) weighs 4 replicated x (one gather)
SPMV_HUB_DEGREE = 16  # SpMV partition: rows above 16 nonzeros go to the hub split
CSRC = os.path.join(ROOT, "paper_1605_02043_amd", "csrc")


def source_sha256() -> str:
    """Hash of the library sources: counter summaries are valid for one version only."""
    import hashlib

    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".cpp", ".h")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """Per-launch L2-miss traffic (request-size counters) from the committed counter summary,
    or None if it belongs to other sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    return t if t.get("source_sha256") == source_sha256() else None


def _short_name(name: str) -> str:
    """'void epk::flux_bwd_kernel<4, 1, true>(epk::DevPlan, ...)' -> 'flux_bwd_kernel<4, 1, true>'."""
    n = name.split("(")[0]
    for pre in ("void ", "epk::"):
        n = n.replace(pre, "")
    return n.strip()


def _is_scrub(name: str, grid: int) -> bool:
    """The cache scrub's dispatch (torch's row-sum kernel over the 1 GiB buffer; bench.py runs
    no other torch reduction)."""
    return "at::native::reduce_kernel" in name


def summarize_trace(path: str) -> str:
    """Markdown summary of a rocprofv3 kernel trace (CSV) of bench.py: per library kernel and grid
    size, the launches and their mean / median duration, all launches and those that directly
    follow the read-only cache scrub (the cold launches bench.py times for the roofline)."""
    import csv

    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"], int(r["Grid_Size_X"]),
                         int(r["Workgroup_Size_X"])))
    rows.sort()
    groups = {}
    prev_scrub = False
    for t0, t1, name, grid, wg in rows:
        if "epk::" in name:
            key = (_short_name(name), grid // max(wg, 1))
            g = groups.setdefault(key, {"all": [], "cold": []})
            g["all"].append((t1 - t0) / 1e3)
            if prev_scrub:
                g["cold"].append((t1 - t0) / 1e3)
        prev_scrub = _is_scrub(name, grid)
    out = ["| kernel | workgroups | launches | mean us | median us | cold launches | cold mean us | cold median us |",
           "|---|---|---|---|---|---|---|---|"]
    for (name, nwg), g in sorted(groups.items(), key=lambda kv: -sum(kv[1]["all"])):
        a, c = g["all"], g["cold"]
        out.append(f"| {name} | {nwg} | {len(a)} | {np.mean(a):.2f} | {np.median(a):.2f} | {len(c)} | "
                   + (f"{np.mean(c):.2f} | {np.median(c):.2f} |" if c else "- | - |"))
    return "\n".join(out)


def summarize_spmv_trace(path: str) -> str:
    """Markdown summary of a rocprofv3 kernel trace (CSV) of `bench.py --workload rmat20`, per task
    order: the orders run one after another, each after its own partition and plan build, and the
    plan of the transpose last, so the library's dispatches split at the len(SPMV_ORDERS) longest
    gaps between them."""
    import csv

    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if "epk::" in r["Kernel_Name"]:
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), _short_name(r["Kernel_Name"]),
                             int(r["Grid_Size_X"]) // max(int(r["Workgroup_Size_X"]), 1)))
    rows.sort()
    phases = SPMV_ORDERS + ("transpose plan (adjoint of " + SPMV_HEADLINE + ")",)
    gaps = sorted(range(len(rows) - 1), key=lambda i: rows[i][1] - rows[i + 1][0])[:len(phases) - 1]
    cuts = [0] + sorted(i + 1 for i in gaps) + [len(rows)]
    out = ["| order | kernel | workgroups | launches | mean us | median us |", "|---|---|---|---|---|---|"]
    for order, a, b in zip(phases, cuts[:-1], cuts[1:]):
        groups = {}
        for t0, t1, name, grid in rows[a:b]:
            groups.setdefault((name, grid), []).append((t1 - t0) / 1e3)
        for (name, grid), d in sorted(groups.items(), key=lambda kv: -len(kv[1])):
            out.append(f"| {order} | {name} | {grid} | {len(d)} | {np.mean(d):.2f} | {np.median(d):.2f} |")
    shortest = min(rows[i + 1][0] - rows[i][1] for i in gaps) / 1e9 if gaps else 0.0
    out.append("")
    out.append(f"(order boundaries: the {len(gaps)} longest gaps between library dispatches, the shortest of them "
               f"{shortest:.2f} s)")
    return "\n".join(out)


def summarize_counters(paths) -> str:
    """Markdown summary of rocprofv3 counter collections (CSV) of bench.py: per kernel and grid
    size, the mean value of every counter per dispatch (counters accumulate over the device's
    XCDs and channels as rocprofv3 reports them), and the bytes and L2 hit rate they give."""
    import csv

    acc = {}
    for path in paths:
        with open(path) as f:
            for r in csv.DictReader(f):
                wg = max(int(r["Workgroup_Size"]), 1)
                key = (_short_name(r["Kernel_Name"]), int(r["Grid_Size"]) // wg)
                d = acc.setdefault(key, {})
                d.setdefault(r["Counter_Name"], {})[r["Dispatch_Id"]] = float(r["Counter_Value"])
    names = sorted({c for d in acc.values() for c in d})
    derived = (("read_bytes", "read MB"), ("write_bytes", "write MB"), ("fetch_size_expression_bytes", "FETCH_SIZE expr MB"),
               ("l2_hit_rate", "L2 hit"))
    out = ["| kernel | workgroups | dispatches | " + " | ".join(names) + " | " + " | ".join(h for _, h in derived) + " |",
           "|---|---|---|" + "---|" * (len(names) + len(derived))]
    for (name, nwg), d in sorted(acc.items()):
        nd = max(len(v) for v in d.values())
        mean = {c: float(np.mean(list(v.values()))) for c, v in d.items()}
        vals = [f"{mean[c]:.6g}" if c in mean else "-" for c in names]
        b = _bytes_of(mean)
        vals += [("-" if key not in b else f"{b[key]:.3f}" if key == "l2_hit_rate" else f"{b[key] / 1e6:.1f}")
                 for key, _ in derived]
        out.append(f"| {name} | {nwg} | {nd} | " + " | ".join(vals) + " |")
    return "\n".join(out)


def _counter_table(paths):
    """{(short kernel name, workgroups): {counter: mean value per dispatch}} from rocprofv3 CSVs."""
    import csv

    acc = {}
    for path in paths:
        with open(path) as f:
            for r in csv.DictReader(f):
                wg = max(int(r["Workgroup_Size"]), 1)
                key = (_short_name(r["Kernel_Name"]), int(r["Grid_Size"]) // wg)
                acc.setdefault(key, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return {k: {c: float(np.mean(v)) for c, v in d.items()} for k, d in acc.items()}


def _bytes_of(c):
    """L2-miss traffic of one dispatch from the request counters (TCC_EA0_*, summed over the
    device): reads by request size, 32 / 64 / 128 bytes, writes as 32 or 64 bytes; also the
    rocprofv3 FETCH_SIZE expression (which takes TCC_BUBBLE as the count of 128-byte reads)."""
    out = {}
    if "TCC_EA0_RDREQ_sum" in c:
        r32, r64, r128 = (c.get(f"TCC_EA0_RDREQ_{b}B_sum", 0.0) for b in (32, 64, 128))
        other = max(c["TCC_EA0_RDREQ_sum"] - r32 - r64 - r128, 0.0)
        out["read_bytes"] = 32 * r32 + 64 * r64 + 128 * r128 + 64 * other
        out["read_requests"] = {"32B": r32, "64B": r64, "128B": r128, "other": other}
    if "TCC_EA0_WRREQ_sum" in c:
        w64 = c.get("TCC_EA0_WRREQ_64B_sum", 0.0)
        out["write_bytes"] = 32 * (c["TCC_EA0_WRREQ_sum"] - w64) + 64 * w64
    if "TCC_BUBBLE_sum" in c and "read_requests" in out:
        rq = out["read_requests"]
        tot = rq["32B"] + rq["64B"] + rq["128B"] + rq["other"]
        out["fetch_size_expression_bytes"] = (128 * c["TCC_BUBBLE_sum"] + 64 * (tot - c["TCC_BUBBLE_sum"] - rq["32B"])
                                              + 32 * rq["32B"])
    if "TCC_HIT_sum" in c and "TCC_MISS_sum" in c:
        out["l2_hit_rate"] = c["TCC_HIT_sum"] / max(c["TCC_HIT_sum"] + c["TCC_MISS_sum"], 1.0)
    return out


PMC_PASSES = (("R", "TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum"),
              ("W", "TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum TCC_BUBBLE_sum"),
              ("H", "TCC_HIT_sum TCC_MISS_sum"))


def pmc_commands(name: str, bench_args: str) -> list:
    """The three counter passes (one rocprofv3 run each) whose CSVs a traffic summary reads."""
    return [f"timeout -s KILL 400 rocprofv3 --pmc {ctr} --output-format csv -d <dir>/{name}_{p} -o {name} "
            f"-- python3 bench.py {bench_args}" for p, ctr in PMC_PASSES]


def traffic_json(workload: str, paths, cap: int = 256) -> dict:
    """Per-launch L2-miss traffic (reads to the fabric, MALL hits included, and writes) of the
    partitioned and default-order kernels of a mesh workload, from counter CSVs of
    `bench.py --eager ...` runs; dispatches are told apart by their grid (plans rebuilt here)."""
    import gen
    from paper_1605_02043_amd import Plan

    G = gen.workload(workload, seed=0)
    m = len(G["edges"])
    table = _counter_table(paths)
    out = {"source_sha256": source_sha256(), "workload": workload,
           "counters": "TCC_EA0_RDREQ{,_32B,_64B,_128B}_sum, TCC_EA0_WRREQ{,_64B}_sum, TCC_BUBBLE_sum, "
                       "TCC_HIT_sum, TCC_MISS_sum per dispatch (rocprofv3 --pmc, three passes); bytes = L2 misses to "
                       "the fabric by request size (MALL hits included) plus writes",
           "commands": pmc_commands(workload, ("" if workload == "tet55" else f"--workload {workload} ")
                                    + "--eager --steps 3 --warmup 1 --cold-steps 0 --no-cpu-baseline --no-baselines")}
    for order in ("ep", "input"):
        P = Plan(G["edges"], G["n"], cap, G["geom"].astype(np.float32), order=order)
        info, st = P.info(), P.stats
        k = info["n_parts"]
        grid_part = 8 * ((k + 7) // 8)
        grid_red = (st["replicated"] + (G["n"] - st["n_active"]) + 255) // 256
        algo = {"flux_fwd": info["bytes_fwd_kernel"], "flux_bwd": info["bytes_bwd_kernel"],
                "reduce_fwd": info["bytes_fwd"] - info["bytes_fwd_kernel"],
                "reduce_bwd": info["bytes_bwd"] - info["bytes_bwd_kernel"]}
        res = {}
        for (name, nwg), c in table.items():
            if name.startswith("flux_fwd_kernel") and nwg == grid_part:
                stage = "flux_fwd"
            elif name.startswith("flux_bwd_kernel") and nwg == grid_part:
                stage = "flux_bwd"
            elif name.startswith("reduce_kernel") and nwg == grid_red:
                stage = "reduce"
            else:
                continue
            b = _bytes_of(c)
            for st_name in ((stage,) if stage != "reduce" else ("reduce_fwd", "reduce_bwd")):
                e = res.setdefault(st_name, {"kernel": name, "workgroups": nwg, "launches_per_step": 1})
                e.update(b)
                e["bytes"] = e.get("read_bytes", 0.0) + e.get("write_bytes", 0.0)
                e["algorithmic_bytes"] = algo[st_name]
                e["measured_over_algorithmic"] = e["bytes"] / algo[st_name] if algo[st_name] else None
        out["ep" if order == "ep" else "default"] = res
        out[("ep" if order == "ep" else "default") + "_bytes_per_edge"] = sum(v["bytes"] for v in res.values()) / m
    return out


SPMV_ORDERS = ("ep_hub", "ep_weighted", "ep", "shuffled", "row_sorted")  # the order bench_spmv runs them in
SPMV_HEADLINE = "ep_hub"


def spmv_traffic_json(paths) -> dict:
    """Per-launch L2-miss traffic of the SpMV kernels of `bench.py --workload rmat20` counter runs,
    per task order.  The orders run one after another with the same number of launches each, so a
    kernel's dispatches, in dispatch order, split into equal consecutive runs, one per order."""
    import csv

    per = {}  # (kernel, file) -> {dispatch: {counter: value}}
    for path in paths:
        with open(path) as f:
            for r in csv.DictReader(f):
                name = _short_name(r["Kernel_Name"])
                if not name.startswith(("spmv_kernel", "spmv_adj_kernel", "reduce_kernel")):
                    continue
                per.setdefault((name, path), {}).setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = \
                    float(r["Counter_Value"])
    acc = {}
    for (name, path), disp in per.items():
        ids = sorted(disp)
        n_per = len(ids) // len(SPMV_ORDERS)
        for i, order in enumerate(SPMV_ORDERS):
            for d in ids[i * n_per:(i + 1) * n_per]:
                for c, v in disp[d].items():
                    acc.setdefault((order, name), {}).setdefault(c, []).append(v)
    out = {"source_sha256": source_sha256(), "workload": "rmat20",
           "counters": "request-size counters per dispatch as for tet55; dispatches split per order by dispatch order",
           "commands": pmc_commands("rmat20", "--workload rmat20 --steps 3 --warmup 1 --no-cpu-baseline "
                                              "--no-transpose-adjoint")}
    for (order, name), cs in sorted(acc.items()):
        b = _bytes_of({c: float(np.mean(v)) for c, v in cs.items()})
        b["bytes"] = b.get("read_bytes", 0.0) + b.get("write_bytes", 0.0)
        b["dispatches"] = max(len(v) for v in cs.values())
        out.setdefault(order, {})[name] = b
    return out


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="tet55", choices=["tet55", "tet32", "tet80", "rmat20", "batch256"])
    ap.add_argument("--cap", type=int, default=256)
    ap.add_argument("--wg", type=int, default=0, help="workgroup size (0: the plan's default)")
    ap.add_argument("--swizzle", type=int, default=1, help="XCD-aware part mapping (1) or identity (0)")
    ap.add_argument("--slot-layout", type=int, default=-1, choices=[-1, 0, 1],
                    help="FLUX5 workspace layout: -1 the plan's choice, 0 part-major, 1 vertex-major")
    ap.add_argument("--staging", type=int, default=1,
                    help="1: stage each part's states in LDS; 0: the cache-only variant (states read through L1/L2)")
    ap.add_argument("--fused", type=int, default=-1, choices=[-1, 0, 1],
                    help="FLUX5 replicated-vertex sums: -1 the plan's choice, 1 inside the part kernel, 0 a second launch")
    ap.add_argument("--pipe", type=int, default=0,
                    help="pipelined persistent launch, workgroups per CU (-1: as many as fit, 0: one per part)")
    ap.add_argument("--eager", action="store_true",
                    help="time K eagerly launched steps instead of one HIP graph holding the K steps")
    ap.add_argument("--cold-steps", type=int, default=20,
                    help="launches of each kernel, and steps, timed after a read-only 1 GiB cache scrub each (0: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-default-order", action="store_true")
    ap.add_argument("--no-baselines", action="store_true", help="skip the random and greedy vertex-cut orders")
    ap.add_argument("--no-transpose-adjoint", action="store_true",
                    help="rmat20: skip the adjoint through a plan of the transpose")
    ap.add_argument("--adaptive", type=int, default=0, metavar="STEPS",
                    help="run STEPS forward steps under adaptive overhead control (background partition) and exit")
    ap.add_argument("--cpu-budget-s", type=float, default=20.0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--summarize-trace", metavar="CSV",
                    help="print a markdown summary of a rocprofv3 kernel trace of this script and exit (no GPU)")
    ap.add_argument("--summarize-counters", nargs="+", metavar="CSV",
                    help="print a markdown summary of rocprofv3 counter collections of this script and exit (no GPU)")
    ap.add_argument("--summarize-spmv-trace", metavar="CSV",
                    help="print the per-order markdown summary of a rmat20 kernel trace and exit (no GPU)")
    ap.add_argument("--spmv-traffic-json", nargs="+", metavar="CSV",
                    help="print the per-order SpMV traffic JSON from rmat20 counter CSVs and exit (no GPU)")
    ap.add_argument("--traffic-json", nargs="+", metavar=("WORKLOAD", "CSV"),
                    help="print the per-launch traffic JSON of a mesh workload from counter CSVs and exit (no GPU)")
    return ap.parse_args()


def calibrate_copy(mib, torch):
    """A plain copy kernel of known size: reads and writes mib MiB each, 5 times."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes_read": n * 4, "calibrate_copy_bytes_written": n * 4, "launches": 5}))


def _step(P, torch, q, gr, r, gq, ev):
    """One fwd+bwd step through the C ABI; ev: 5 events or None."""
    from paper_1605_02043_amd._lib import check, lib
    from paper_1605_02043_amd.plan import _dptr

    s = torch.cuda.current_stream()
    h = C_void(s.cuda_stream)
    ws = _dptr(P.workspace)
    calls = [(0, 0, q, None, r), (0, 1, q, None, r), (1, 0, q, gr, gq), (1, 1, q, gr, gq)]
    for i, (op, stage, a, b, out) in enumerate(calls):
        if ev is not None:
            ev[i].record(s)
        check(lib.epk_run_stage(P._h, op, stage, _dptr(a), _dptr(b), _dptr(out), 0.0, None, ws, h))
    if ev is not None:
        ev[4].record(s)


def _stage(P, torch, i, q, gr, r, gq):
    """Stage i of a step alone: 0 forward part kernel, 1 its reduction, 2 adjoint part kernel, 3 its reduction."""
    from paper_1605_02043_amd._lib import check, lib
    from paper_1605_02043_amd.plan import _dptr

    op, stage, b, out = [(0, 0, None, r), (0, 1, None, r), (1, 0, gr, gq), (1, 1, gr, gq)][i]
    h = C_void(torch.cuda.current_stream().cuda_stream)
    check(lib.epk_run_stage(P._h, op, stage, _dptr(q), _dptr(b), _dptr(out), 0.0, None, _dptr(P.workspace), h))


def _ev(torch):
    """A timing event, created ahead of the timed regions: torch creates the HIP event at its
    first record, which costs about 0.1 ms of host time, so it is recorded once here."""
    e = torch.cuda.Event(enable_timing=True)
    e.record()
    return e


def _stage_timed(P, torch, i, q, gr, r, gq) -> float:
    """Stage i alone (as _stage), timed by the kernel's own dispatch timestamps: ms as the GPU ran it."""
    import ctypes

    from paper_1605_02043_amd._lib import check, lib
    from paper_1605_02043_amd.plan import _dptr

    op, stage, b, out = [(0, 0, None, r), (0, 1, None, r), (1, 0, gr, gq), (1, 1, gr, gq)][i]
    h = C_void(torch.cuda.current_stream().cuda_stream)
    ms = ctypes.c_float()
    check(lib.epk_run_stage_timed(P._h, op, stage, _dptr(q), _dptr(b), _dptr(out), 0.0, None, _dptr(P.workspace), h,
                                  ctypes.byref(ms)))
    return float(ms.value)


def C_void(x):
    import ctypes

    return ctypes.c_void_p(x)


def make_scrub(torch):
    """Read-only cache scrub: row sums of a 1 GiB buffer (4x the 256 MiB MALL, 256x an XCD's
    4 MiB L2), 65536 rows, so that every CU of every XCD streams its share (a full reduction to
    one value runs in a single workgroup and evicts one XCD's L2 only).  It writes 256 KiB of
    sums and leaves no other dirty lines, so the kernel timed after it pays only for its own
    misses."""
    buf = torch.ones(1 << 28, dtype=torch.float32, device="cuda").view(1 << 16, 1 << 12)
    out = torch.empty(1 << 16, dtype=torch.float32, device="cuda")

    def scrub():
        torch.sum(buf, dim=1, out=out)

    return scrub, buf


def _med(xs):
    return float(np.median(xs)) if len(xs) else None


def run_order(G, order, cap, steps, warmup, torch, wg=0, swizzle=1, pipe=-1, staging=1, layout=-1, scrub=None,
              fused=-1):
    """Time one task order: K steps (forward then adjoint of L = 1/2 sum r^2, so the adjoint's
    upstream gradient is r itself) captured in one HIP graph and replayed once (the timed
    region), the same graph replayed REPLAYS more times for the spread, per-kernel durations
    from HIP events in eager steps, each kernel alone in a graph of K launches (warm caches),
    and, with scrub, each kernel and the whole step after a read-only 1 GiB scrub (cold)."""
    from paper_1605_02043_amd import Plan

    import gen

    t0 = time.perf_counter()
    P = Plan(G["edges"], G["n"], cap, G["geom"].astype(np.float32), order=order)
    P.set_launch(wg, swizzle)
    if layout != -1:
        P.set_slot_layout(layout)
    if fused != -1:
        P.set_fused(fused)
    P.upload("cuda")
    if not staging:
        P.set_staging(0)
    elif pipe:
        P.set_pipeline(pipe)
    plan_s = time.perf_counter() - t0
    perm = P.perm()
    q = torch.from_numpy(gen.flux_state(G["n"], seed=0)[perm]).cuda()
    r = torch.empty_like(q)
    gq = torch.empty_like(q)
    gr = r  # L = 1/2 sum r^2: the adjoint's upstream gradient is r
    for _ in range(warmup):
        _step(P, torch, q, gr, r, gq, None)
    # per-kernel durations: HIP events around every launch of K eager steps
    evs = [[_ev(torch) for _ in range(5)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        _step(P, torch, q, gr, r, gq, evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    graph_ms = None
    replays = None
    if GRAPH_TIMING:
        # the K steps captured in one HIP graph (no events inside: ROCm refuses external events),
        # timed by events around its replay
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            _step(P, torch, q, gr, r, gq, None)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            for i in range(steps):
                _step(P, torch, q, gr, r, gq, None)
        for _ in range(WARM_REPLAYS):  # the first replays of a graph pay one-time launch costs
            graph.replay()
        g0, g1 = _ev(torch), _ev(torch)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g0.record()
        graph.replay()
        g1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        graph_ms = g0.elapsed_time(g1) / steps
        # the spread: the same graph replayed again, each replay timed by its own events
        rev = [(_ev(torch), _ev(torch)) for _ in range(REPLAYS)]
        for a, b in rev:
            a.record()
            graph.replay()
            b.record()
        torch.cuda.synchronize()
        per = [a.elapsed_time(b) / steps for a, b in rev]
        replays = {"n": REPLAYS, "steps_each": steps, "median_ms_per_step": _med(per), "min_ms_per_step": min(per),
                   "max_ms_per_step": max(per)}
        del graph
    names = ["flux_fwd", "reduce_fwd", "flux_bwd", "reduce_bwd"]
    dur = {nm: float(np.mean([e[i].elapsed_time(e[i + 1]) for e in evs])) for i, nm in enumerate(names)}
    step_gpu = float(np.mean([e[0].elapsed_time(e[4]) for e in evs]))
    # each stage alone, K back-to-back launches between two events: the launch gaps of a
    # step (kernel switches, event records) drop out, as in a kernel trace.  With graph
    # timing the K launches are one HIP graph, so host launch gaps drop out as well.
    loop = {}
    for i, nm in enumerate(names):
        e0, e1 = _ev(torch), _ev(torch)
        if GRAPH_TIMING:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                for _ in range(steps):
                    _stage(P, torch, i, q, gr, r, gq)
            g.replay()  # warm replay
            torch.cuda.synchronize()
            e0.record()
            g.replay()
            e1.record()
        else:
            e0.record()
            for _ in range(steps):
                _stage(P, torch, i, q, gr, r, gq)
            e1.record()
        torch.cuda.synchronize()
        loop[nm] = e0.elapsed_time(e1) / steps
    # each stage alone, K launches timed by their own dispatch timestamps (the kernel's duration as
    # a kernel trace reports it), each after a launch of the same stage: warm caches
    kernel_warm = {}
    for i, nm in enumerate(names):
        _stage(P, torch, i, q, gr, r, gq)
        kernel_warm[nm] = _med([_stage_timed(P, torch, i, q, gr, r, gq) for _ in range(steps)])
    cold = None
    if scrub is not None and COLD_STEPS > 0:
        # cold caches: the read-only scrub before every timed launch (each kernel alone, timed by its
        # dispatch timestamps, then whole steps with the per-kernel split by events)
        cold = {}
        for i, nm in enumerate(names):
            ts = []
            for _ in range(COLD_STEPS):
                scrub()
                ts.append(_stage_timed(P, torch, i, q, gr, r, gq))
            cold[nm] = _med(ts)
        cev = [[_ev(torch) for _ in range(5)] for _ in range(COLD_STEPS)]
        for i in range(COLD_STEPS):
            scrub()
            _step(P, torch, q, gr, r, gq, cev[i])
        torch.cuda.synchronize()
        cold["in_step"] = {nm: _med([e[i].elapsed_time(e[i + 1]) for e in cev]) for i, nm in enumerate(names)}
        cold["step"] = _med([e[0].elapsed_time(e[4]) for e in cev])
    # one clean step for the outputs the oracle checks (the stage loops above re-ran reductions)
    _step(P, torch, q, gr, r, gq, None)
    torch.cuda.synchronize()
    r_h = np.empty((G["n"], 5), np.float32)
    r_h[perm] = r.cpu().numpy()
    g_h = np.empty((G["n"], 5), np.float32)
    g_h[perm] = gq.cpu().numpy()
    info = P.info()
    st = P.stats
    m = len(G["edges"])
    return {
        "plan": P,
        "wall_ms_per_step": wall / steps * 1e3,
        "gpu_ms_per_step": step_gpu,
        "kernel_ms": dur,
        "kernel_loop_ms": loop,
        "kernel_warm_ms": kernel_warm,
        "info": info,
        "stats": st,
        "plan_seconds": plan_s,
        "bytes_per_edge_fwd_bwd": (info["bytes_fwd"] + info["bytes_bwd"]) / m,
        "edges_per_s": m / (wall / steps),
        "cold_ms": cold,
        "graph_gpu_ms_per_step": graph_ms,
        "replays": replays,
        "outputs": {"r": r_h, "g_q": g_h},
    }


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def oracle_error(G, q, gpu, n_sample=500, seed=0):
    """Error of the GPU's r and g_q (g_r = r) against the FP64 oracle on a seeded sample of
    vertices.  A vertex's r depends only on its incident edges, and its g_q on those edges and
    r at their endpoints, so the oracle runs on the two-hop edge set of the sample only."""
    from oracle import flux

    n = G["n"]
    E = np.asarray(G["edges"], dtype=np.int64)
    geom = G["geom"].astype(np.float32).astype(np.float64)
    S = np.random.default_rng(seed).choice(n, size=min(n_sample, n), replace=False)
    inS = np.zeros(n, bool)
    inS[S] = True
    e1 = np.flatnonzero(inS[E[:, 0]] | inS[E[:, 1]])
    N1 = np.zeros(n, bool)
    N1[E[e1].ravel()] = True
    e2 = np.flatnonzero(N1[E[:, 0]] | N1[E[:, 1]])
    q64 = q.astype(np.float64)
    r_ref = flux.forward(n, E[e2], geom[e2], q64)  # exact at every vertex of N1 (all its edges are in e2)
    r_abs = flux.forward_abs(n, E[e2], geom[e2], q64)
    g_ref = flux.backward(n, E[e1], geom[e1], q64, r_ref)  # exact on the sample
    g_abs = flux.backward_abs(n, E[e1], geom[e1], q64, np.abs(r_ref) + r_abs)
    out = {}
    for name, got, ref, A in (("r", gpu["r"], r_ref, r_abs), ("g_q", gpu["g_q"], g_ref, g_abs)):
        d = np.abs(got[S].astype(np.float64) - ref[S])
        den = np.abs(ref[S]) + A[S]
        out[name] = {"max_abs": float(d.max()), "max_rel_floored": float((d / np.where(den > 0, den, 1)).max()),
                     "normwise": float(np.linalg.norm(d) / max(np.linalg.norm(ref[S]), 1e-300))}
    out["sample"] = f"{len(S)} vertices (seed {seed}), oracle on their {len(e2)}-edge two-hop neighbourhood"
    out["bar"] = "elementwise |d| <= 1e-5 (|ref| + A), normwise <= 1e-5"
    return out


def cpu_baseline(G, budget_s, gpu_outputs=None):
    """The FP64 oracle (numpy, one thread) on the same workload: forward + adjoint, timed on a
    bounded sample; with gpu_outputs it also reports the GPU results' error against it."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    import gen
    from oracle import flux

    q = gen.flux_state(G["n"], seed=0).astype(np.float64)
    gr = gen.workloads.grad_seed(G["n"], seed=0).astype(np.float64)  # adjoint input of the timed sample
    geom = G["geom"].astype(np.float32).astype(np.float64)
    m_all = len(G["edges"])
    # bounded sample: a contiguous slice of the edge list sized to the budget
    ctx = threadpool_limits(1) if threadpool_limits else None
    try:
        if ctx:
            ctx.__enter__()
        m_s = min(m_all, 200_000)
        E = G["edges"][:m_s]
        t0 = time.perf_counter()
        flux.forward(G["n"], E, geom[:m_s], q)
        flux.backward(G["n"], E, geom[:m_s], q, gr)
        t_small = time.perf_counter() - t0
        per_edge = t_small / m_s
        m_s = int(min(m_all, max(m_s, budget_s / max(per_edge, 1e-12))))
        # the whole workload when it fits the budget, repeated to fill about half of it
        reps = max(1, int(0.5 * budget_s / (per_edge * m_s))) if m_s == m_all else 1
        E = G["edges"][:m_s]
        t0 = time.perf_counter()
        for _ in range(reps):
            flux.forward(G["n"], E, geom[:m_s], q)
            flux.backward(G["n"], E, geom[:m_s], q, gr)
        t = time.perf_counter() - t0
    finally:
        if ctx:
            ctx.__exit__(None, None, None)
    what = f"all {m_all} edges x {reps} passes" if m_s == m_all else f"first {m_s} of {m_all} edges"
    out = {"value": reps * m_s / t, "unit": "edges/s", "cores": 1, "kind": "oracle",
           "sample": f"{what} (all {G['n']} cells' states), FP64 forward + adjoint, "
                     f"{t:.1f} s on {cpu_model()} (host reports {os.cpu_count()} CPUs; 1 thread used)"}
    if gpu_outputs is not None:
        with threadpool_limits(1) if threadpool_limits else _nullctx():
            out["gpu_error_vs_oracle"] = oracle_error(G, gen.flux_state(G["n"], seed=0), gpu_outputs)
    return out


class _nullctx:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False


def _err(got, ref, A):
    d = np.abs(np.asarray(got, np.float64) - ref)
    den = np.abs(ref) + A
    return {"max_abs": float(d.max()) if d.size else 0.0,
            "max_rel_floored": float((d / np.where(den > 0, den, 1)).max()) if d.size else 0.0,
            "normwise": float(np.linalg.norm(d) / max(np.linalg.norm(ref), 1e-300)),
            "bar": "elementwise |d| <= 1e-5 (|ref| + A), normwise <= 1e-5"}


def cpu_baseline_spmv(R, budget_s, gpu_y=None):
    """The FP64 oracle SpMV (numpy bincount, one thread) over the whole R-MAT matrix, repeated;
    with gpu_y (original row order) the GPU result's error against it, over every row."""
    from threadpoolctl import threadpool_limits

    from gen.rmat import spmv_graph
    from oracle import spmv

    g = spmv_graph(R, R["shuffle"])
    m = len(g["edges"])
    with threadpool_limits(1):
        t0 = time.perf_counter()
        spmv.forward(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"])
        t1 = time.perf_counter() - t0
        reps = max(1, int(0.5 * budget_s / t1))
        t0 = time.perf_counter()
        for _ in range(reps):
            spmv.forward(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"])
        t = time.perf_counter() - t0
    out = {"value": reps * m / t, "unit": "edges/s", "cores": 1, "kind": "oracle",
           "sample": f"all {m} nonzeros x {reps} passes, FP64, {t:.1f} s on "
                     f"{cpu_model()} (host reports {os.cpu_count()} CPUs; 1 thread)"}
    if gpu_y is not None:
        ref = spmv.forward(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"])
        A = spmv.forward_abs(R["n_x"], R["n_y"], g["edges"], g["w"], R["x"])
        out["gpu_error_vs_oracle"] = dict(_err(gpu_y, ref, A), sample=f"all {R['n_y']} rows of y")
    return out


def main():
    args = _args()
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace))
        return
    if args.summarize_counters:
        print(summarize_counters(args.summarize_counters))
        return
    if args.summarize_spmv_trace:
        print(summarize_spmv_trace(args.summarize_spmv_trace))
        return
    if args.spmv_traffic_json:
        print(json.dumps(spmv_traffic_json(args.spmv_traffic_json), indent=1))
        return
    if args.traffic_json:
        print(json.dumps(traffic_json(args.traffic_json[0], args.traffic_json[1:], args.cap), indent=1))
        return
    global GRAPH_TIMING, COLD_STEPS
    GRAPH_TIMING = not args.eager
    COLD_STEPS = args.cold_steps
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for --gpus {args.gpus}): the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import gen

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy, torch)
        return
    if args.adaptive:
        return bench_adaptive(args, torch)
    if args.workload == "rmat20":
        return bench_spmv(args, torch)
    if args.workload == "batch256":
        return bench_batch(args, torch)
    G = gen.workload(args.workload, seed=0)
    m = len(G["edges"])
    print(f"# workload {args.workload}: n={G['n']} m={m}", file=sys.stderr, flush=True)
    scrub, scrub_buf = make_scrub(torch) if args.cold_steps > 0 else (None, None)
    ep = run_order(G, "ep", args.cap, args.steps, args.warmup, torch, args.wg, args.swizzle, args.pipe, args.staging,
                   args.slot_layout, scrub, args.fused)
    print(f"# ep: {ep['wall_ms_per_step']:.4f} ms/step kernels {ep['kernel_ms']}", file=sys.stderr, flush=True)
    default = None
    if not args.no_default_order:
        default = run_order(G, "input", args.cap, args.steps, args.warmup, torch, args.wg, args.swizzle, args.pipe,
                            args.staging, scrub=scrub, fused=args.fused)
        print(f"# default: {default['wall_ms_per_step']:.4f} ms/step kernels {default['kernel_ms']}", file=sys.stderr,
              flush=True)
    # dominant kernel of the partitioned step
    k_ms = ep["kernel_ms"]
    lp_ms = ep["kernel_loop_ms"]
    kw_ms = ep["kernel_warm_ms"]
    dom = max(kw_ms, key=kw_ms.get)
    info = ep["info"]
    algo = {"flux_fwd": info["bytes_fwd_kernel"], "flux_bwd": info["bytes_bwd_kernel"],
            "reduce_fwd": info["bytes_fwd"] - info["bytes_fwd_kernel"],
            "reduce_bwd": info["bytes_bwd"] - info["bytes_bwd_kernel"]}
    warm_achieved = algo[dom] / (kw_ms[dom] * 1e-3) / 1e9
    b2b_achieved = algo[dom] / (lp_ms[dom] * 1e-3) / 1e9
    cold = ep["cold_ms"]
    traffic = measured_traffic(args.workload)
    per_kernel = {nm: {"ms_in_step": k_ms[nm], "ms": kw_ms[nm], "ms_back_to_back": lp_ms[nm],
                       "algorithmic_bytes": algo[nm], "GB/s": algo[nm] / (kw_ms[nm] * 1e-3) / 1e9} for nm in k_ms}
    if cold:
        for nm in per_kernel:
            per_kernel[nm]["ms_cold"] = cold[nm]
            per_kernel[nm]["GB/s_cold"] = algo[nm] / (cold[nm] * 1e-3) / 1e9
    warm_timing = (f"median of {args.steps} launches of the kernel, each right after the previous one, timed by "
                   f"the dispatch's own timestamps")
    b2b_timing = (f"HIP events around a HIP-graph replay of {args.steps} back-to-back launches of the kernel "
                  f"(kernel plus the gap between launches)" if GRAPH_TIMING
                  else f"HIP events around {args.steps} back-to-back launches of the kernel")
    if cold:
        achieved = algo[dom] / (cold[dom] * 1e-3) / 1e9
        timing = (f"median of {COLD_STEPS} launches of the kernel, each after a read-only 1 GiB scrub, timed by "
                  f"the dispatch's own timestamps (hipExtLaunchKernel events)")
    else:
        achieved, timing = warm_achieved, warm_timing
    st = ep["stats"]
    out = {
        "metric": "edges/s + DRAM bytes/edge, partitioned vs default order, fwd+bwd, 1 MI355X",
        "value": ep["edges_per_s"],
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ep["wall_ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "wg": ep["info"]["wg"],
            "xcd_swizzle": args.swizzle,
            "workload": f"{args.workload}: 3D Kuhn-tetrahedral mesh dual, n={G['n']} cells, m={m} faces, "
                        f"5xFP32 state U[0.5,1.5], normal+area per face, capacity {args.cap}, forward then adjoint "
                        f"of L = 1/2 sum r^2 (upstream gradient r), partitioned (EP) task order",
            "capacity": args.cap,
            "order": "ep",
            "timing": "eager launches" if args.eager else "hip-graph replay of the timed steps",
            "launch": (f"pipelined persistent, grid {ep['info']['grid_pipe_fwd']} fwd / {ep['info']['grid_pipe_bwd']} bwd"
                       if ep["info"]["pipe"] else "one workgroup per part"),
            "staging": "LDS" if ep["info"]["staging"] else "caches only (no LDS staging of states)",
            "slot_layout": "vertex-major" if ep["info"]["vertex_major"] else "part-major",
            "reduction": ("single launch (the part kernel sums the replicated vertices)" if ep["info"]["fused"]
                          else "second launch"),
        },
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "timing": timing,
                     "traffic": traffic["ep"][dom]["bytes"] if traffic else None,
                     "warm": {"achieved": warm_achieved, "frac": warm_achieved / HBM_PEAK_GBS, "timing": warm_timing,
                              "note": "the step's working set fits the 256 MiB MALL, so back-to-back launches "
                                      "are served partly from it"},
                     "back_to_back": {"achieved": b2b_achieved, "frac": b2b_achieved / HBM_PEAK_GBS,
                                      "timing": b2b_timing}},
        "kernels": per_kernel,
        "gpu_ms_per_step": ep["gpu_ms_per_step"],
        "replays": ep["replays"],
        "cold_ms": {"ep": ep["cold_ms"], "default": default["cold_ms"] if default else None,
                    "protocol": f"median over {COLD_STEPS} launches (each kernel alone) and {COLD_STEPS} steps, "
                                f"each after a read-only sum over 1 GiB"},
        "algorithmic_bytes_per_edge": {"ep": ep["bytes_per_edge_fwd_bwd"]},
        "partition": {"loads_per_edge": st["loads"] / m, "cost": st["cost"], "replicated": st["replicated"],
                      "slots": st["slots"], "balance": st["balance"], "n_parts": st["n_parts"],
                      "partition_seconds": st["partition_seconds"], "plan_seconds": ep["plan_seconds"]},
    }
    if default is not None:
        dst = default["stats"]
        out["default_order"] = {"value": default["edges_per_s"], "ms_per_step": default["wall_ms_per_step"],
                                "kernels_ms": default["kernel_ms"], "loads_per_edge": dst["loads"] / m,
                                "algorithmic_bytes_per_edge": default["bytes_per_edge_fwd_bwd"]}
        out["algorithmic_bytes_per_edge"]["default"] = default["bytes_per_edge_fwd_bwd"]
        out["speedup_vs_default_order"] = default["wall_ms_per_step"] / ep["wall_ms_per_step"]
    if not args.no_baselines and args.staging:
        # the paper's cache-only alternative to LDS staging, same plan and order
        saved_cold, COLD_STEPS = COLD_STEPS, 0
        v = run_order(G, "ep", args.cap, min(args.steps, 20), args.warmup, torch, args.wg, args.swizzle, 0, 0)
        out["variants"] = {"cache_only": {"value": v["edges_per_s"], "ms_per_step": v["wall_ms_per_step"],
                                          "kernels": {nm: {"ms": v["kernel_loop_ms"][nm],
                                                           "GB/s": algo[nm] / (v["kernel_loop_ms"][nm] * 1e-3) / 1e9}
                                                      for nm in v["kernel_loop_ms"]}}}
        print(f"# cache-only: {out['variants']['cache_only']}", file=sys.stderr, flush=True)
        del v
        COLD_STEPS = saved_cold
    if not args.no_baselines:
        # the related work's vertex-cut placements (random, greedy) with the same capacity and kernels
        out["baseline_orders"] = {}
        saved_cold, COLD_STEPS = COLD_STEPS, 0
        for order in ("greedy", "random"):
            b = run_order(G, order, args.cap, min(args.steps, 20), args.warmup, torch, args.wg, args.swizzle, args.pipe,
                          args.staging)
            bst = b["stats"]
            out["baseline_orders"][order] = {"value": b["edges_per_s"], "ms_per_step": b["wall_ms_per_step"],
                                             "loads_per_edge": bst["loads"] / m, "cost": bst["cost"],
                                             "algorithmic_bytes_per_edge": b["bytes_per_edge_fwd_bwd"],
                                             "partition_seconds": bst["partition_seconds"]}
            print(f"# {order}: {out['baseline_orders'][order]}", file=sys.stderr, flush=True)
            del b
        COLD_STEPS = saved_cold
    if traffic:
        out["l2_miss_bytes_per_edge"] = {"ep": traffic["ep_bytes_per_edge"], "default": traffic["default_bytes_per_edge"],
                                         "note": "L2 misses to the fabric (MALL hits included) plus writes, "
                                                 "from request-size counters; see profiles/"}
        out["l2_miss_counters"] = traffic["counters"]
    out["source_sha256"] = source_sha256()
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline(G, args.cpu_budget_s, ep["outputs"])
    print(json.dumps(out), flush=True)


def bench_adaptive(args, torch):
    """Time to run a fixed number of forward steps when the partition is built in the
    background (the default order runs meanwhile), against waiting for it first."""
    import gen
    from paper_1605_02043_amd.adaptive import AdaptiveFlux

    G = gen.workload(args.workload, seed=0)
    m = len(G["edges"])
    q0 = gen.flux_state(G["n"], seed=0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ad = AdaptiveFlux(G["edges"], G["n"], args.cap, G["geom"].astype(np.float32))
    q = ad.pack(q0)
    switched_at = None
    for i in range(args.adaptive):
        if ad.decision is None and i % 64 == 0:
            q = ad.maybe_switch(q)
            if ad.decision is not None:
                switched_at = i
        ad.forward(q)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info = ad.bg.poll()
    t = ad.timings
    out = _common(args, "edges/s over a fixed run of forward steps, partition built in the background", 
                  args.adaptive * m / wall, wall * 1e3 / args.adaptive,
                  {"workload": f"{args.workload}: {args.adaptive} forward steps under adaptive overhead control",
                   "capacity": args.cap})
    est = {}
    if t:
        est = {"default_only_s": args.adaptive * t["input_ms"] * 1e-3,
               "partition_first_s": info["seconds"] + args.adaptive * t["ep_ms"] * 1e-3}
    out["adaptive"] = {"decision": ad.decision, "switched_at_step": switched_at, "wall_s": wall,
                       "partition_and_plan_s": info["seconds"], "saving_bound": info["saving_bound"],
                       "step_ms": t, "estimates": est}
    out["source_sha256"] = source_sha256()
    out["cpu_baseline"] = None
    ad.close()
    print(json.dumps(out), flush=True)


def _common(args, metric, value, ms, config):
    return {"metric": metric, "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": config}


def bench_spmv(args, torch):
    """R-MAT 2^20 x 2^20, 2^24 nonzeros: SpMV in partitioned vs shuffled vs row-sorted order."""
    import ctypes

    import gen
    from gen.rmat import spmv_graph
    from paper_1605_02043_amd import Plan
    from paper_1605_02043_amd._lib import check, lib
    from paper_1605_02043_amd.plan import _dptr

    R = gen.rmat(20, 1 << 24, seed=0)
    m = len(R["rows"])
    res = {}
    setups = {"ep_hub": (R["shuffle"], "ep", (1, SPMV_Y_WEIGHT), SPMV_HUB_DEGREE),
              "ep_weighted": (R["shuffle"], "ep", (1, SPMV_Y_WEIGHT), 0), "ep": (R["shuffle"], "ep", None, 0),
              "shuffled": (R["shuffle"], "input", None, 0),
              "row_sorted": (np.argsort(R["rows"], kind="stable"), "input", None, 0)}
    for name in SPMV_ORDERS:
        perm_e, order, cw, hub = setups[name]
        g = spmv_graph(R, perm_e)
        t0 = time.perf_counter()
        P = Plan(g["edges"], g["n"], args.cap, g["w"], order=order, kind="spmv", n_x=g["n_x"], class_weight=cw,
                 hub_degree=hub)
        P.set_launch(args.wg, args.swizzle)
        P.upload("cuda")
        plan_s = time.perf_counter() - t0
        auto_layout = P.info()["vertex_major"]
        perm = P.perm()
        x = torch.from_numpy(np.ascontiguousarray(R["x"][perm[:R["n_x"]]])).cuda()
        y = torch.empty(R["n_y"], dtype=torch.float32, device="cuda")
        s = torch.cuda.current_stream()
        h = C_void(s.cuda_stream)
        ws = _dptr(P.workspace)

        def step(ev):
            for i in range(2):
                if ev is not None:
                    ev[i].record(s)
                check(lib.epk_run_stage(P._h, 2, i, _dptr(x), None, _dptr(y), 0.0, None, ws, h))
            if ev is not None:
                ev[2].record(s)

        layouts = {}
        for layout in (auto_layout, 1 - auto_layout):  # the automatic choice first, then the other one
            P.set_slot_layout(layout)
            for _ in range(args.warmup):
                step(None)
            evs = [[_ev(torch) for _ in range(3)] for _ in range(args.steps)]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(args.steps):
                step(evs[i])
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / args.steps
            if GRAPH_TIMING:
                # the per-kernel split above comes from eager steps; the step time from the K
                # steps captured in one HIP graph and replayed once, as for the other workloads
                def graph_step():
                    hc = C_void(torch.cuda.current_stream().cuda_stream)
                    for i in range(2):
                        check(lib.epk_run_stage(P._h, 2, i, _dptr(x), None, _dptr(y), 0.0, None, ws, hc))

                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    for _ in range(args.steps):
                        graph_step()
                for _ in range(WARM_REPLAYS):
                    g.replay()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g.replay()
                torch.cuda.synchronize()
                wall = (time.perf_counter() - t0) / args.steps
                del g
            # each kernel by its own dispatch timestamps (the duration a kernel trace reports), median
            kt = [[], []]
            for _ in range(args.steps):
                for i in range(2):
                    ms = ctypes.c_float()
                    check(lib.epk_run_stage_timed(P._h, 2, i, _dptr(x), None, _dptr(y), 0.0, None, ws, h,
                                                  ctypes.byref(ms)))
                    kt[i].append(ms.value)
            info = P.info()
            layouts["vertex_major" if layout else "part_major"] = {
                "edges_per_s": m / wall, "ms_per_step": wall * 1e3,
                "kernels_ms": {"spmv": _med(kt[0]), "reduce": _med(kt[1])},
                "kernels_ms_in_step": {"spmv": float(np.mean([e[0].elapsed_time(e[1]) for e in evs])),
                                       "reduce": float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))},
                "algorithmic_bytes": {"spmv": info["bytes_fwd_kernel"],
                                      "reduce": info["bytes_fwd"] - info["bytes_fwd_kernel"]}}
        # the adjoint (g_x = A^T g_y) on the same plan
        gy = torch.ones(R["n_y"], dtype=torch.float32, device="cuda")
        for _ in range(args.warmup):
            P.spmv_adjoint(gy)
        a0, a1 = _ev(torch), _ev(torch)
        a0.record()
        for _ in range(args.steps):
            P.spmv_adjoint(gy)
        a1.record()
        torch.cuda.synchronize()
        adj_ms = a0.elapsed_time(a1) / args.steps
        st = P.stats
        auto = layouts["vertex_major" if auto_layout else "part_major"]
        best = min(layouts.values(), key=lambda v: v["ms_per_step"])
        # the partitioned order runs its automatic layout; the baselines are quoted at their best one
        use = auto if name.startswith("ep") else best
        res[name] = dict(use, layout="vertex_major" if use is layouts.get("vertex_major") else "part_major",
                         layouts=layouts, adjoint_ms=adj_ms, adjoint_edges_per_s=m / (adj_ms * 1e-3),
                         loads_per_edge=st["loads"] / m, slots_per_edge=st["slots"] / m,
                         plan_seconds=plan_s, partition_seconds=st["partition_seconds"])
        print(f"# {name}: {res[name]}", file=sys.stderr, flush=True)
        if name == SPMV_HEADLINE:  # the reported order's y, in original row order, for the oracle check
            P.set_slot_layout(auto_layout)
            yv = P.spmv(x).cpu().numpy()
            gpu_y = np.empty(R["n_y"], dtype=np.float32)
            gpu_y[perm[R["n_x"]:] - R["n_x"]] = yv
            # and its adjoint for a seeded g_y, in original column order (compared with the transpose plan)
            gy_orig = np.random.default_rng(3).standard_normal(R["n_y"]).astype(np.float32)
            gxv = P.spmv_adjoint(torch.from_numpy(np.ascontiguousarray(gy_orig[perm[R["n_x"]:] - R["n_x"]])).cuda())
            gx_same = np.empty(R["n_x"], dtype=np.float32)
            gx_same[perm[:R["n_x"]]] = gxv.cpu().numpy()
        del P
    if not args.no_transpose_adjoint:
        res[SPMV_HEADLINE]["adjoint_transpose_plan"] = spmv_adjoint_transpose_plan(args, torch, R, gy_orig, gx_same)
    ep = res[SPMV_HEADLINE]
    dom = max(ep["kernels_ms"], key=ep["kernels_ms"].get)
    ach = ep["algorithmic_bytes"][dom] / (ep["kernels_ms"][dom] * 1e-3) / 1e9
    out = _common(args, "edges/s, SpMV y += A x, partitioned vs shuffled order, 1 MI355X", ep["edges_per_s"],
                  ep["ms_per_step"], {"workload": f"rmat20: R-MAT 2^20 x 2^20, {m} nonzeros (a,b,c)=(0.57,0.19,0.19), "
                                                  f"w~U[0,1), x~N(0,1), capacity {args.cap}, partitioned order "
                                                  f"(the rows above {SPMV_HUB_DEGREE} nonzeros in runs of the "
                                                  f"capacity, the rest EP with y copies weighing {SPMV_Y_WEIGHT}; "
                                                  f"EP without the split under orders.ep_weighted, uniform weights "
                                                  f"under orders.ep)",
                                      "capacity": args.cap,
                                      "timing": ("step: the timed steps captured in one HIP graph, one replay"
                                                 if GRAPH_TIMING else "step: eager launches")
                                      + "; kernels: median of launches timed by their dispatch timestamps"})
    traffic = measured_traffic("rmat20")
    kern = [v["bytes"] for name, v in (traffic or {}).get(SPMV_HEADLINE, {}).items()
            if name.startswith({"spmv": "spmv_kernel", "reduce": "reduce_kernel"}[dom])]
    out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": ach / HBM_PEAK_GBS,
                       "timing": f"median of {args.steps} launches, timed by the dispatch's own timestamps",
                       "traffic": kern[0] if len(kern) == 1 else None}
    out["orders"] = res
    out["source_sha256"] = source_sha256()
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline_spmv(R, args.cpu_budget_s, gpu_y)
    print(json.dumps(out), flush=True)


def spmv_adjoint_transpose_plan(args, torch, R, gy_orig, gx_same):
    """g_x = A^T g_y as the forward SpMV of a plan of A^T (the headline order's partition rules
    applied to the transpose).  The same-plan adjoint scatters into the x class, which R-MAT
    replicates at almost every nonzero; the transpose plan reduces that class as the forward
    reduces y.  Returns its time per call (eager, events around K calls), its plan time and its
    normwise difference from the same-plan adjoint."""
    from gen.rmat import spmv_graph
    from paper_1605_02043_amd import Plan

    RT = {"rows": R["cols"], "cols": R["rows"], "w": R["w"], "n_x": R["n_y"], "n_y": R["n_x"]}
    g = spmv_graph(RT, R["shuffle"])
    t0 = time.perf_counter()
    P = Plan(g["edges"], g["n"], args.cap, g["w"], order="ep", kind="spmv", n_x=g["n_x"],
             class_weight=(1, SPMV_Y_WEIGHT), hub_degree=SPMV_HUB_DEGREE)
    P.upload("cuda")
    plan_s = time.perf_counter() - t0
    perm = P.perm()
    n_in = g["n_x"]
    gyp = torch.from_numpy(np.ascontiguousarray(gy_orig[perm[:n_in]])).cuda()
    for _ in range(args.warmup):
        gx = P.spmv(gyp)
    a0, a1 = _ev(torch), _ev(torch)
    torch.cuda.synchronize()
    a0.record()
    for _ in range(args.steps):
        gx = P.spmv(gyp, out=gx)
    a1.record()
    torch.cuda.synchronize()
    out = np.empty(R["n_x"], dtype=np.float32)
    out[perm[n_in:] - n_in] = gx.cpu().numpy()
    diff = float(np.linalg.norm(out.astype(np.float64) - gx_same) / max(np.linalg.norm(gx_same.astype(np.float64)), 1e-300))
    res = {"ms": a0.elapsed_time(a1) / args.steps, "plan_seconds": plan_s,
           "normwise_diff_vs_same_plan_adjoint": diff, "loads_per_edge": P.stats["loads"] / len(g["edges"])}
    print(f"# adjoint by the transpose plan: {res}", file=sys.stderr, flush=True)
    del P
    return res


def bench_batch(args, torch):
    """256 uneven mesh graphs, one persistent launch each way, the fwd+bwd step replayed from a HIP graph."""
    import gen
    from paper_1605_02043_amd import Plan
    from paper_1605_02043_amd.batch import Batch, autotune

    t0 = time.perf_counter()
    graphs = gen.batch_graphs(256, seed=0)
    gen_s = time.perf_counter() - t0
    m = sum(len(g["edges"]) for g in graphs)
    n = sum(g["n"] for g in graphs)
    t0 = time.perf_counter()
    caps, wgs, directs = autotune(graphs, caps=(64, 128, 256, 512))
    tune_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    plans = [Plan(g["edges"], g["n"], int(c), g["geom"].astype(np.float32)) for g, c in zip(graphs, caps)]
    B = Batch(plans).set_launch(int(wgs[0]), int(directs[0])).upload("cuda")
    plan_s = time.perf_counter() - t0
    q = torch.from_numpy(np.concatenate([gen.flux_state(g["n"], seed=i)[p.perm()] for i, (g, p) in
                                         enumerate(zip(graphs, plans))])).cuda()
    r = torch.empty_like(q)
    gq = torch.empty_like(q)
    gr = r  # L = 1/2 sum r^2 over every graph: the adjoint's upstream gradient is r
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(2):
            B.forward(q, out=r)
            B.backward(q, gr, out=gq)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    # as for the single-mesh workloads: the K timed steps are captured in one HIP graph and
    # replayed once (replaying a one-step graph K times adds a graph launch per step)
    warm = torch.cuda.CUDAGraph()
    with torch.cuda.graph(warm):
        B.forward(q, out=r)
        B.backward(q, gr, out=gq)
    for _ in range(args.warmup):
        warm.replay()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(args.steps):
            B.forward(q, out=r)
            B.backward(q, gr, out=gq)
    for _ in range(WARM_REPLAYS):
        graph.replay()
    e0, e1 = _ev(torch), _ev(torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    graph.replay()
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    gpu_ms = e0.elapsed_time(e1) / args.steps
    info = B.info()
    algo = info["bytes_fwd"] + info["bytes_bwd"]
    ach = algo / (gpu_ms * 1e-3) / 1e9
    # one clean step: the outputs the oracle checks (per graph, original vertex order)
    B.forward(q, out=r)
    B.backward(q, gr, out=gq)
    torch.cuda.synchronize()
    r_all, g_all = r.cpu().numpy(), gq.cpu().numpy()
    outs = []
    for i, p in enumerate(plans):
        sl = slice(int(B.offsets[i]), int(B.offsets[i + 1]))
        ri, gi = np.empty_like(r_all[sl]), np.empty_like(g_all[sl])
        ri[p.perm()] = r_all[sl]
        gi[p.perm()] = g_all[sl]
        outs.append((ri, gi))
    out = _common(args, "edges/s, batched FLUX5 fwd+bwd over 256 uneven meshes in one launch per pass, HIP-graph replay, 1 MI355X",
                  m / wall, wall * 1e3,
                  {"workload": f"batch256: 256 2D/3D mesh graphs, vertex counts log-uniform in [1024, 65536], "
                               f"total n={n}, m={m}, forward then adjoint of L = 1/2 sum r^2 (upstream gradient r), "
                               f"one capacity and launch shape autotuned over {{64, 128, 256, 512}} x {{64, 128, 256}} lanes x {{one workgroup per item, pipelined persistent}} by timing the batched launch",
                               "graphs": 256, "timing": "the timed steps captured in one HIP graph, one replay"})
    kind = "one workgroup per item" if info["direct"] else "pipelined persistent"
    out["roofline"] = {"bound": "hbm", "kernel": f"graph replay (fwd + reduce + bwd + reduce, {kind})",
                       "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                       "traffic": None}
    out["batch"] = {"items": info["items"], "launch": kind, "grid": info["items"] if info["direct"] else info["grid"],
                    "wg": info["wg"], "lds_fwd": info["lds_fwd"],
                    "caps": {int(c): int((caps == c).sum()) for c in np.unique(caps)}, "gpu_ms_per_step": gpu_ms,
                    "algorithmic_bytes_per_step": algo, "gen_s": gen_s, "autotune_s": tune_s, "plan_s": plan_s}
    out["source_sha256"] = source_sha256()
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline_batch(graphs, args.cpu_budget_s, outs)
    print(json.dumps(out), flush=True)


def cpu_baseline_batch(graphs, budget_s, gpu_outs=None):
    """The FP64 oracle forward + adjoint (numpy, one thread) over the leading graphs of the batch;
    with gpu_outs ((r, g_q) per graph, original order, upstream gradient r) the GPU results'
    error against it on those graphs."""
    from threadpoolctl import threadpool_limits

    import gen
    from oracle import flux

    done_m, t = 0, 0.0
    worst = {"r": [], "g_q": []}
    with threadpool_limits(1):
        for i, g in enumerate(graphs):
            q = gen.flux_state(g["n"], seed=i).astype(np.float64)
            geom = g["geom"].astype(np.float32).astype(np.float64)
            t0 = time.perf_counter()
            r = flux.forward(g["n"], g["edges"], geom, q)
            gq = flux.backward(g["n"], g["edges"], geom, q, r)
            t += time.perf_counter() - t0
            done_m += len(g["edges"])
            if gpu_outs is not None:
                rA = flux.forward_abs(g["n"], g["edges"], geom, q)
                worst["r"].append(_err(gpu_outs[i][0], r, rA))
                worst["g_q"].append(_err(gpu_outs[i][1], gq, flux.backward_abs(g["n"], g["edges"], geom, q,
                                                                              np.abs(r) + rA)))
            if t > 0.5 * budget_s:
                break
    out = {"value": done_m / t, "unit": "edges/s", "cores": 1, "kind": "oracle",
           "sample": f"graphs 0..{i} of {len(graphs)} ({done_m} edges), FP64 forward + adjoint, {t:.1f} s on "
                     f"{cpu_model()} (host reports {os.cpu_count()} CPUs; 1 thread)"}
    if gpu_outs is not None:
        out["gpu_error_vs_oracle"] = {
            k: {f: max(e[f] for e in v) for f in ("max_abs", "max_rel_floored", "normwise")} for k, v in worst.items()}
        out["gpu_error_vs_oracle"]["sample"] = f"graphs 0..{i}, every vertex (worst over the graphs)"
        out["gpu_error_vs_oracle"]["bar"] = "elementwise |d| <= 1e-5 (|ref| + A), normwise <= 1e-5"
    return out


if __name__ == "__main__":
    main()
