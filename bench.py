#!/usr/bin/env python3
"""Benchmark: FP64 time-centred steps of the moving-mesh Godunov scheme on
one MI355X.

Workload (default): advected wave on a 2048 x 2048 jittered lattice
(4,194,304 cells), periodic unit box, rho = 1 + 1e-3 sin(2 pi x), p = 0.6,
v = (1, 0.5), gamma = 5/3, Lagrangian mesh motion with cell rounding, HLLC.

A step is the whole hot path: stage 1 on mesh_n (half step), stage 2 on
mesh_{n+1/2} (full step from the start-of-step state).  The Voronoi meshes
come from the host tessellation stage, which is an input stage timed apart:
the benchmark first runs the real chain (GPU stages, host tessellation in
between) and keeps every mesh resident in HBM, then replays the same chain
from the same initial state with all inputs resident and times exactly K
steps (after W warm-up steps) with HIP events on the launch stream.  The
replayed final state must equal the live one bit for bit.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import glob
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per step (FP64) and HBM fraction; batched/served vs plain, p99"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the sources the stage kernels are built from."""
    h = hashlib.sha256()
    for f in (os.path.join(ROOT, "paper_1410_3219_amd", "csrc", g)
              for g in ("rich_device.hpp", "rich_kernels.hip")):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def totals_drift(Q0, Q1, t_end, steps):
    """Change of the domain totals of M, Px, Py, E between two states (host
    arrays), relative to the largest |total| of the quantity's cells times the
    cell count (so a total that starts at zero is measured against its cells);
    reported, not a bar: walls exert forces, so only M and E are conserved
    with walls, all four in a periodic box."""
    import numpy as np
    q0, q1 = np.asarray(Q0, dtype=np.float64), np.asarray(Q1, dtype=np.float64)
    t0, t1 = q0.sum(axis=1), q1.sum(axis=1)
    scale = np.abs(q0).max(axis=1) * q0.shape[1]
    rel = np.abs(t1 - t0) / np.where(scale > 0, scale, 1.0)
    return {"steps": steps, "t_end": t_end,
            "rel_change": {k: float(v) for k, v in zip(("M", "Px", "Py", "E"), rel)}}


def algorithmic_bytes(m, pass2):
    """Bytes one stage must move at least once (cells, state, edges, CSR,
    results): 40 B geometry + 32 B source state per cell, 32 B per edge,
    4 B per CSR offset and entry, 48 B of results per cell, and for the
    second stage 48 B more of start-of-step state and points."""
    n, ne, nc = m.n_cells, m.n_edges, m.n_csr
    b = 40 * n + 32 * n + 32 * ne + 4 * (n + 1) + 4 * nc + 48 * n
    if pass2:
        b += 48 * n
    return b


GATHER_PROBE_DOUBLES = (4, 8, 16)   # gather probe rows of 32, 64, 128 bytes


def _pmc_per_kernel(d):
    """Counters of one rocprofv3 --pmc run, by kernel: the mean per dispatch
    for k_cell and k_flux, the largest dispatch of the calibration copy, and
    each gather probe (torch's gather kernel behind index_select, in launch
    order: rows of 32, 64, 128 bytes).  Values are summed over a dispatch's instances."""
    import csv
    f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not f:
        raise SystemExit(f"no counter_collection.csv under {d}")
    disp = {}
    for row in csv.DictReader(open(f[0])):
        e = disp.setdefault(int(row["Dispatch_Id"]), {"name": row["Kernel_Name"], "c": {}})
        c = row["Counter_Name"]
        e["c"][c] = e["c"].get(c, 0.0) + float(row["Counter_Value"])
    out, acc = {}, {}
    for i in sorted(disp):
        name, c = disp[i]["name"], disp[i]["c"]
        key = "k_cell" if "k_cell" in name else "k_flux" if "k_flux" in name else None
        if key:
            for k, v in c.items():
                acc.setdefault((key, k), []).append(v)
    for k, v in acc.items():
        out[k] = sum(v) / len(v)
    copies = [disp[i]["c"] for i in disp if "copyBuffer" in disp[i]["name"]]
    if copies:
        first = sorted(copies[0])[0]
        big = max(copies, key=lambda c: c.get(first, 0.0))
        for k, v in big.items():
            out[("copy", k)] = v
    gathers = [disp[i]["c"] for i in sorted(disp) if "gather_kernel" in disp[i]["name"]]
    if len(gathers) == len(GATHER_PROBE_DOUBLES):
        for w, c in zip(GATHER_PROBE_DOUBLES, gathers):
            for k, v in c.items():
                out[(f"gather{8 * w}", k)] = v
    return out


def _probe_bytes(key, copy_bytes):
    """(read, write) bytes a calibration dispatch moves by construction."""
    if key == "copy":
        return copy_bytes, copy_bytes
    w = int(key[len("gather"):]) // 8
    nsel = (64 << 20) // (8 * w)
    return nsel * 8 * w + 8 * nsel, nsel * 8 * w


TRAFFIC_HEADER = """\
# HBM traffic per launch of k_cell and k_flux, workload '{w}', from rocprofv3 --pmc runs
# on one MI355X (program directly after --, from /tmp with TMPDIR=/tmp), one counter set
# per run:  FETCH_SIZE | WRITE_SIZE |
#   TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_32B_sum TCC_BUBBLE_sum TCC_EA0_RDREQ_DRAM_sum |
#   TCC_MISS_sum TCC_HIT_sum TCC_READ_sum TCC_WRITE_sum
#   timeout -s KILL 300 rocprofv3 --pmc <set> --output-format csv -d <repo>/<dir> -o p \\
#     -- python3 <repo>/bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-extras --copy-probe-mib {mib}
# summarised with:
#   python bench.py --summarize-pmc {dirs} --copy-probe-mib {mib}
# fetch/write_bytes_per_launch: FETCH_SIZE / WRITE_SIZE scaled by the factor that makes
# each read the size of a {mib} MiB device-to-device copy (copyBuffer) run after a 1 GiB
# flush.  Cross-check (read_requests): in the copy, k_cell and k_flux the EA read
# requests equal the L2 read-line misses (TCC_MISS less written bytes / 128) to 0.02%,
# so each request is one 128-byte line fill; FETCH_SIZE counts such a request as 64
# bytes, hence the copy's factor of 2, and the copy-scaled figure is 128 bytes per
# request for the two kernels.  The
# gather probes (torch's gather kernel over scattered 32-, 64- and 128-byte rows, 64 MiB
# of rows each) show what a fill can carry: 20-68 bytes of each 128 that the gather
# asked for.
# source_hash is a hash of the kernel sources the counters were taken on.
"""


def read_traffic(workload):
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    lines = [ln for ln in open(path) if ln.strip() and not ln.startswith("#")]
    return json.loads(lines[-1]) if lines else None


def summarize_pmc(args):
    """HBM bytes per launch of k_cell and k_flux from rocprofv3 --pmc runs of
    this script with --copy-probe-mib: FETCH_SIZE and WRITE_SIZE scaled by the
    calibration copy (the bench line's `traffic`), cross-checked, where the
    runs hold them, with the EA read-request and L2 miss counters."""
    pm = {}
    for d in args.summarize_pmc:
        pm.update(_pmc_per_kernel(d))
    nbytes = args.copy_probe_mib << 20
    cf = nbytes / (pm[("copy", "FETCH_SIZE")] * 1024.0)
    cw = nbytes / (pm[("copy", "WRITE_SIZE")] * 1024.0)
    out = {"source_hash": kernel_source_hash(), "copy_bytes": nbytes,
           "fetch_scale": cf, "write_scale": cw, "kernels": {}}
    keys = ["copy"] + [f"gather{8 * w}" for w in GATHER_PROBE_DOUBLES] + ["k_cell", "k_flux"]
    if all((k, c) in pm for k in keys for c in ("TCC_EA0_RDREQ_sum", "TCC_MISS_sum",
                                                "WRITE_SIZE")):
        xc = {}
        for k in keys:
            req = pm[(k, "TCC_EA0_RDREQ_sum")]
            rmiss = pm[(k, "TCC_MISS_sum")] - pm[(k, "WRITE_SIZE")] * 1024.0 / 128.0
            e = {"ea_read_requests": req, "l2_read_line_misses": rmiss,
                 "requests_per_miss": req / rmiss if rmiss > 0 else None}
            if not k.startswith("k_"):
                known = _probe_bytes(k, nbytes)[0]
                e["read_bytes_by_construction"] = known
                e["bytes_per_request"] = known / req
            else:
                e["read_bytes_at_128_per_request"] = 128.0 * req
            xc[k] = e
        out["read_requests"] = xc
    tot = 0.0
    for k in ("k_cell", "k_flux"):
        fb = pm[(k, "FETCH_SIZE")] * 1024.0 * cf
        wb = pm[(k, "WRITE_SIZE")] * 1024.0 * cw
        out["kernels"][k] = {"fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb}
        tot += fb + wb
    out["bytes_per_stage"] = tot
    out["bytes_per_step"] = 2 * tot
    P, _, make_state = make_problem(args.workload, args.k)
    out["n_cells"] = P.n
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    path = os.path.join(ROOT, "profiles", f"traffic_{args.workload}.txt")
    with open(path, "w") as f:
        f.write(TRAFFIC_HEADER.format(w=args.workload, mib=args.copy_probe_mib,
                                      dirs=" ".join(args.summarize_pmc)))
        f.write(json.dumps(out) + "\n")
    print(json.dumps(out, indent=1))


def summarize_trace(d, name, title, command):
    """Per-kernel durations of a rocprofv3 --kernel-trace --stats run (its
    *_kernel_stats.csv, nanoseconds) into profiles/NAME.txt."""
    import csv
    import re
    f = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    if not f:
        raise SystemExit(f"no kernel_stats.csv under {d}")
    rows = list(csv.DictReader(open(f[0])))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    path = os.path.join(ROOT, "profiles", f"{name}.txt")
    with open(path, "w") as out:
        out.write(f"# Kernel durations: {title}\n#\n# command (from the repository root, on one "
                  f"MI355X):\n#   {command}\n# summarised with:\n#   python bench.py "
                  f"--summarize-trace <dir> {name} '<title>' '<command>'\n#\n# source: "
                  f"*_kernel_stats.csv (durations in microseconds); copyBuffer entries are the\n"
                  f"# host<->device transfers of the host tessellation stage, outside the timed "
                  f"region.\n#\n")
        out.write(f"{'kernel':62s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s}\n")
        for r in rows:
            name = re.sub(r"\(.*$", "", r["Name"].replace("void ", ""))
            out.write(f"{name[:62]:62s} {int(r['Calls']):6d} "
                      f"{float(r['AverageNs']) / 1e3:10.1f} {float(r['MinNs']) / 1e3:10.1f} "
                      f"{float(r['MaxNs']) / 1e3:10.1f}\n")
    print(open(path).read())


def summarize_counters(d, name, command):
    """Per kernel of the HIP path, the mean per dispatch of every counter of a
    rocprofv3 --pmc run (counters summed over the dispatch's instances)."""
    import csv
    import re
    f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not f:
        raise SystemExit(f"no counter_collection.csv under {d}")
    acc = {}
    for row in csv.DictReader(open(f[0])):
        kname = re.sub(r"\(.*$", "", row["Kernel_Name"]).replace("void ", "")
        if not kname.startswith(("rich::", "retess::")):
            continue
        a = acc.setdefault(kname, {}).setdefault(row["Counter_Name"], {})
        a[row["Dispatch_Id"]] = a.get(row["Dispatch_Id"], 0.0) + float(row["Counter_Value"])
    counters = sorted({c for k in acc.values() for c in k})
    path = os.path.join(ROOT, "profiles", f"{name}.txt")
    with open(path, "w") as out:
        out.write(f"# rocprofv3 counters, mean per dispatch, per kernel\n#\n# command (on one "
                  f"MI355X, from /tmp with TMPDIR=/tmp):\n#   {command}\n# summarised with:\n"
                  f"#   python bench.py --summarize-counters <dir> {name} '<command>'\n#\n")
        out.write(f"{'kernel':40s} {'dispatches':>10s} " +
                  " ".join(f"{c:>22s}" for c in counters) + "\n")
        for k in sorted(acc):
            n = max(len(v) for v in acc[k].values())
            vals = [sum(acc[k][c].values()) / len(acc[k][c]) if c in acc[k] else float("nan")
                    for c in counters]
            out.write(f"{k[:40]:40s} {n:10d} " + " ".join(f"{v:22.4g}" for v in vals) + "\n")
    print(open(path).read())


def bench_batch(args, R, T, log):
    """Many independent shock-tube runs of uneven sizes (N log-uniform in
    [1024, 65536], interface angle, gamma and rounding strength drawn per
    run): one time-centred step of every run, either as batched launches
    (rich_stage_batch: one launch per kernel phase for all runs) or as
    separate per-run launches.  Meshes of step 0 come from the host stage
    (timed apart); the timed step is repeated from the same start."""
    import numpy as np
    import torch
    from paper_1410_3219_amd import inputs as I
    specs = I.batch_runs(args.batch_runs)
    runs = []
    t0 = time.time()
    for sp in specs:
        P = I.sod(k=sp["side"], seed=sp["seed"], angle=sp["angle"], gamma=sp["gamma"])
        hm = T.rich_tess_build(P.px, P.py, P.box, P.bc, args.threads)
        prm = R.Params(gamma=sp["gamma"], chi=sp["chi"])
        dm = R.DeviceMesh.from_host(hm)
        s0 = R.DeviceState.from_host(P.state(hm.area), np.stack([hm.px, hm.py]))
        runs.append(dict(hm=hm, dm=dm, s0=s0, half=R.DeviceState.empty_like(s0),
                         out=R.DeviceState.empty_like(s0), p=prm))
    total = sum(r["hm"].n_cells for r in runs)
    # stage 1 of every run once (per-run calls) to get the half-step points
    ws1 = R.workspace(max(r["hm"].n_cells for r in runs))
    for r in runs:
        r["dt"] = R.rich_cfl_dt(r["dm"], r["s0"], r["p"], ws1)
        R.rich_stage(r["dm"], r["s0"], r["s0"], r["half"], 0.5 * r["dt"], r["p"], ws1)
        xh = r["half"].X.cpu().numpy()
        r["dmh"] = R.DeviceMesh.from_host(T.rich_tess_build(xh[0], xh[1], r["hm"].box,
                                                            r["hm"].bc, args.threads))
    log(f"[bench] batch setup: {len(runs)} runs, {total} cells ({time.time() - t0:.1f}s)")
    wsb = R.batch_workspace([r["hm"].n_cells for r in runs])

    def batched():
        R.rich_stage_batch([r["dm"] for r in runs], [r["s0"] for r in runs],
                           [r["s0"] for r in runs], [r["half"] for r in runs],
                           [0.5 * r["dt"] for r in runs], [r["p"] for r in runs], wsb)
        R.rich_stage_batch([r["dmh"] for r in runs], [r["half"] for r in runs],
                           [r["s0"] for r in runs], [r["out"] for r in runs],
                           [r["dt"] for r in runs], [r["p"] for r in runs], wsb)

    def separate():
        for r in runs:
            R.rich_stage(r["dm"], r["s0"], r["s0"], r["half"], 0.5 * r["dt"], r["p"], ws1)
        for r in runs:
            R.rich_stage(r["dmh"], r["half"], r["s0"], r["out"], r["dt"], r["p"], ws1)

    res = {}
    for name, fn in (("batched", batched), ("per_run_launches", separate)):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = {"ms_per_step": ms, "cell_updates_per_s": total / (ms / 1e3)}
    # edge-tile shape autotuned on these runs (each stage of the step on its
    # own mesh), then the step as prepared plans with the tuned tiles whose
    # launches are captured once in a HIP graph and replayed (no host
    # marshalling, no descriptor upload)
    wsg = R.batch_workspace([r["hm"].n_cells for r in runs])
    a1 = ([r["dm"] for r in runs], [r["s0"] for r in runs], [r["s0"] for r in runs],
          [r["half"] for r in runs], [0.5 * r["dt"] for r in runs], [r["p"] for r in runs])
    a2 = ([r["dmh"] for r in runs], [r["half"] for r in runs], [r["s0"] for r in runs],
          [r["out"] for r in runs], [r["dt"] for r in runs], [r["p"] for r in runs])
    tile1, ms1 = R.rich_stage_batch_autotune(*a1, wsb, reps=3)
    tile2, ms2 = R.rich_stage_batch_autotune(*a2, wsg, reps=3)
    log(f"[bench] batch tile autotune: stage 1 {ms1} -> {tile1}, stage 2 {ms2} -> {tile2}")
    p1 = R.rich_stage_batch_prepare_tile(*a1, tile1, wsb)
    p2 = R.rich_stage_batch_prepare_tile(*a2, tile2, wsg)
    torch.cuda.synchronize()
    gs = torch.cuda.Stream()
    gs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(gs):
        R.rich_stage_batch_launch(p1, wsb, gs)
        R.rich_stage_batch_launch(p2, wsg, gs)
    torch.cuda.current_stream().wait_stream(gs)
    torch.cuda.synchronize()
    want = [r["out"].Q.clone() for r in runs]
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=gs):
        R.rich_stage_batch_launch(p1, wsb, gs)
        R.rich_stage_batch_launch(p2, wsg, gs)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    gms = e0.elapsed_time(e1) / reps
    res["graph_replay"] = {"ms_per_step": gms, "cell_updates_per_s": total / (gms / 1e3),
                           "bitwise_equal_to_eager": all(torch.equal(r["out"].Q, w)
                                                         for r, w in zip(runs, want)),
                           "flux_tiles": [tile1, tile2],
                           "autotune_ms_per_stage": {"stage1": ms1, "stage2": ms2}}
    del graph
    flags = R.rich_batch_flags(len(runs), wsb)
    res["device_dt"] = bench_batch_device_dt(runs, total, tile1, tile2, log)
    res["plain_sod"] = bench_plain_sod(args, R, T, total, log)
    return {"runs": len(runs), "cells": total, "flags_ok": not any(flags),
            "graph_replay": res["graph_replay"], "device_dt": res["device_dt"],
            "plain_sod": res["plain_sod"],

            "batched": res["batched"], "per_run_launches": res["per_run_launches"],
            "batched_over_per_run": res["batched"]["cell_updates_per_s"] /
            res["per_run_launches"]["cell_updates_per_s"]}


def bench_batch_device_dt(runs, total, tile1, tile2, log):
    """The batched step with every run's step taken on the device (a batched
    Courant stage, then the second stage reading its steps): eager (prepare
    and launch of both stages per step) and both launches replayed from one
    graph.  Each run's step equals its host step bitwise, so the half-step
    meshes built for the host-step legs serve here too."""
    import torch
    from paper_1410_3219_amd import rich as R
    n = len(runs)
    ns = [r["hm"].n_cells for r in runs]
    ws1, ws2 = R.batch_workspace(ns), R.batch_workspace(ns)
    m1 = [r["dm"] for r in runs]
    m2 = [r["dmh"] for r in runs]
    s0 = [r["s0"] for r in runs]
    half = [r["half"] for r in runs]
    out = [r["out"] for r in runs]
    prm = [r["p"] for r in runs]

    def prepare():
        q1 = R.rich_stage_batch_prepare_courant(m1, s0, s0, half, [0.5] * n, prm, ws1, tile=tile1)
        q2 = R.rich_stage_batch_prepare_courant(m2, half, s0, out, [1.0] * n, prm, ws2,
                                                dt_ws=ws1, tile=tile2)
        return q1, q2

    def eager():
        q1, q2 = prepare()
        R.rich_stage_batch_launch(q1, ws1)
        R.rich_stage_batch_launch(q2, ws2)

    eager()
    torch.cuda.synchronize()
    dts = R.rich_batch_dt(n, ws1)
    same_dt = all(d == r["dt"] for d, r in zip(dts, runs))
    want = [o.Q.clone() for o in out]
    res = {"steps_equal_host_steps": same_dt,
           "flags_ok": not any(R.rich_batch_flags(n, ws1) + R.rich_batch_flags(n, ws2))}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        eager()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    res["eager"] = {"ms_per_step": ms, "cell_updates_per_s": total / (ms / 1e3)}
    q1, q2 = prepare()
    gs = torch.cuda.Stream()
    gs.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    with torch.cuda.stream(gs):
        R.rich_stage_batch_launch(q1, ws1, gs)
        R.rich_stage_batch_launch(q2, ws2, gs)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=gs):
        R.rich_stage_batch_launch(q1, ws1, gs)
        R.rich_stage_batch_launch(q2, ws2, gs)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    gms = e0.elapsed_time(e1) / reps
    res["graph_replay"] = {"ms_per_step": gms, "cell_updates_per_s": total / (gms / 1e3),
                           "bitwise_equal_to_eager": all(torch.equal(o.Q, w)
                                                         for o, w in zip(out, want))}
    del graph
    log(f"[bench] batch with device steps: eager {ms:.3f} ms, graph {gms:.3f} ms per step")
    return res


def bench_plain_sod(args, R, T, cells, log):
    """One shock-tube run of about `cells` cells (the batch's total) as a
    plain single run with its step on the device, for a comparison of the
    batch with the same physics at the same size."""
    import numpy as np
    import torch
    from paper_1410_3219_amd import inputs as I
    k = int(round(cells ** 0.5))
    t0 = time.time()
    P = I.sod(k=k, seed=11)
    hm = T.rich_tess_build(P.px, P.py, P.box, P.bc, args.threads)
    prm = R.Params(gamma=P.gamma)
    dm = R.DeviceMesh.from_host(hm)
    cur = R.DeviceState.from_host(P.state(hm.area), np.stack([hm.px, hm.py]))
    half, nxt = R.DeviceState.empty_like(cur), R.DeviceState.empty_like(cur)
    ws, ws2 = R.workspace(hm.n_cells), R.workspace(hm.n_cells)
    R.rich_stage_courant(dm, cur, cur, half, 0.5, prm, ws)
    xh = half.X.cpu().numpy()
    dmh = R.DeviceMesh.from_host(T.rich_tess_build(xh[0], xh[1], P.box, P.bc, args.threads))
    log(f"[bench] plain shock tube: {hm.n_cells} cells ({time.time() - t0:.1f}s setup)")

    def step():
        R.rich_stage_courant(dm, cur, cur, half, 0.5, prm, ws)
        R.rich_stage_dt_of(dmh, half, cur, nxt, 1.0, ws, prm, ws2)

    step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"cells": hm.n_cells, "ms_per_step": ms,
            "cell_updates_per_s": hm.n_cells / (ms / 1e3),
            "flags_ok": R.rich_stage_flags(ws) == 0 and R.rich_stage_flags(ws2) == 0}


def bench_serve(args, R, log):
    """Continuous-batching serving loop (paper_1410_3219_amd.serve): Poisson
    step requests, sessions of 8 steps on meshes of 4k-1M cells (log-uniform,
    shock tube / point explosion), static mesh, HBM-budget admission."""
    import math
    from paper_1410_3219_amd import inputs as I
    from paper_1410_3219_amd import serve as S
    s = I.Stream(21)
    u = s.uniform(8)
    sizes = [int(round(math.exp(math.log(4096) + x * (math.log(1 << 20) - math.log(4096)))))
             for x in u]
    kinds = ["sod" if k % 2 == 0 else "sedov" for k in range(len(sizes))]
    t0 = time.time()
    tpl = S.build_templates(sizes, kinds, n_threads=args.threads)
    log(f"[bench] serving templates {[t.n for t in tpl]} ({time.time() - t0:.1f}s)")
    S.run(tpl, rate=args.serve_rate, duration=0.5, seed=8, log=log)   # warm-up, not reported
    res, _ = S.run(tpl, rate=args.serve_rate, duration=args.serve_seconds, log=log)
    # the same mix offered at ten times the rate for a short time: the loop
    # runs saturated, so its throughput is the most the served path delivers
    sat, _ = S.run(tpl, rate=10 * args.serve_rate, duration=0.25 * args.serve_seconds,
                   seed=10, log=log)
    res["saturated"] = {k: sat[k] for k in ("requests", "launches", "mean_batch", "max_batch",
                                            "mixed_launches", "p50_ms", "p99_ms",
                                            "cell_updates_per_s", "wall_s", "offered_rate",
                                            "offered_cell_updates_per_s")}
    return res


def bench_serve_moving(args, R, log, rate=500.0):
    """The serving loop with sessions on moving meshes: each step rebuilds
    both meshes of every session on the device (batched re-tessellation), so
    the loop never waits on the host stage.  Same size mix as the static leg
    (point-explosion templates Lloyd-relaxed), offered at a rate the device
    sustains, then at ten times that rate for a short time (saturated)."""
    import math
    from paper_1410_3219_amd import inputs as I
    from paper_1410_3219_amd import serve as S
    s = I.Stream(21)
    u = s.uniform(8)
    sizes = [int(round(math.exp(math.log(4096) + x * (math.log(1 << 20) - math.log(4096)))))
             for x in u]
    kinds = ["sod" if k % 2 == 0 else "sedov" for k in range(len(sizes))]
    t0 = time.time()
    tpl = S.build_templates(sizes, kinds, n_threads=args.threads, moving=True)
    log(f"[bench] moving serving templates {[t.n for t in tpl]} ({time.time() - t0:.1f}s)")
    S.run(tpl, rate=rate, duration=0.5, seed=8, log=log)   # warm-up, not reported
    res, _ = S.run(tpl, rate=rate, duration=args.serve_seconds, log=log)
    keys = ("requests", "failed_requests", "launches", "mean_batch", "p50_ms", "p99_ms",
            "cell_updates_per_s", "wall_s", "offered_rate", "offered_cell_updates_per_s")
    # the static leg's rate on moving meshes
    full, _ = S.run(tpl, rate=args.serve_rate, duration=args.serve_seconds, seed=11, log=log)
    res["at_static_rate"] = {k: full[k] for k in keys + ("host_fallback_steps",)}
    sat, _ = S.run(tpl, rate=10 * rate, duration=0.25 * args.serve_seconds, seed=10, log=log)
    res["saturated"] = {k: sat[k] for k in keys}
    return res


def bench_extrapolated(args, R, T, P, make_state, hm0, dm0, log, steps=3):
    """The same workload advanced with the extrapolated-fluxes integrator
    (section 2.3, AREPO's scheme: one stage and one tessellation per step).
    A live chain builds the meshes, then the steps are replayed with all
    inputs in HBM: Courant step, one stage."""
    import numpy as np
    import torch
    prm = R.Params(gamma=P.gamma, riemann=args.riemann, integrator=1)
    n = hm0.n_cells
    ws = R.workspace(n)
    cur = R.DeviceState.from_host(make_state(hm0.area), np.stack([hm0.px, hm0.py]))
    init = R.DeviceState(cur.Q.clone(), cur.X.clone())
    nxt = R.DeviceState.empty_like(cur)
    meshes, dts = [dm0], []
    for s in range(steps):
        dt = R.rich_cfl_dt(meshes[s], cur, prm, ws)
        dts.append(dt)
        R.rich_stage(meshes[s], cur, cur, nxt, dt, prm, ws)
        if R.rich_stage_flags(ws):
            raise SystemExit(f"extrapolated-fluxes step {s} flagged")
        if s + 1 < steps:
            xn = nxt.X.cpu().numpy()
            meshes.append(R.DeviceMesh.from_host(
                T.rich_tess_build(xn[0], xn[1], P.box, P.bc, args.threads)))
        cur, nxt = nxt, cur
    live = (cur.Q.clone(), cur.X.clone())
    cur.Q.copy_(init.Q)
    cur.X.copy_(init.X)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ok = True
    e0.record()
    for s in range(steps):
        dt = R.rich_cfl_dt(meshes[s], cur, prm, ws)
        ok = ok and dt == dts[s]
        R.rich_stage(meshes[s], cur, cur, nxt, dt, prm, ws)
        cur, nxt = nxt, cur
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ok = ok and bool(torch.equal(cur.Q, live[0]) and torch.equal(cur.X, live[1]))
    out = {"steps": steps, "ms_per_step": ms, "cell_updates_per_s": n / (ms / 1e3),
           "replay_bitwise_equal_to_live": ok}
    log(f"[bench] extrapolated fluxes {out}")
    return out


def bench_device_chain(args, R, P, make_state, hm0, dm0, live_final, n_steps, log, K=5):
    """The time-centred step with both meshes rebuilt on the device
    (rich_retess, candidates from the previous mesh) instead of by the host
    stage: stage 1 with the Courant step, re-tessellation of the half-step
    points, stage 2, re-tessellation of the new points; nothing leaves the
    device.  The chain runs n_steps steps from the initial state (the last K
    timed) and is compared with the live chain built on host meshes."""
    import numpy as np
    import torch
    K = max(1, min(K, n_steps))   # the chain ends at the live chain's step count
    n = hm0.n_cells
    prm = R.Params(gamma=P.gamma, riemann=args.riemann)
    ws = R.workspace(n)
    tws = R.retess_workspace(n)
    bufs = [R.DeviceMeshBufs(n, hm0.box, hm0.bc) for _ in range(3)]
    s = R.DeviceState.from_host(make_state(hm0.area), np.stack([hm0.px, hm0.py]))
    half = R.DeviceState.empty_like(s)
    nxt = R.DeviceState.empty_like(s)
    state = {"mesh": dm0, "b": 0, "s": s, "nxt": nxt}

    def step():
        mesh, b = state["mesh"], state["b"]
        mh, mn = bufs[b % 3], bufs[(b + 1) % 3]
        R.rich_stage_courant(mesh, state["s"], state["s"], half, 0.5, prm, ws)
        R.rich_retess(mesh, half.X, mh, tws)
        R.rich_stage_dt_of(mh.mesh(), half, state["s"], state["nxt"], 1.0, ws, prm, ws)
        R.rich_retess(mh.mesh(), state["nxt"].X, mn, tws)
        state["mesh"], state["b"] = mn.mesh(), b + 2
        state["s"], state["nxt"] = state["nxt"], state["s"]

    for _ in range(n_steps - K):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(K):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / K
    st, info = R.rich_retess_result(tws)
    flags = R.rich_stage_flags(ws)
    # re-tessellation alone, repeated on the last mesh pair
    mh = bufs[state["b"] % 3]
    e0.record()
    for _ in range(K):
        R.rich_retess(state["mesh"], state["s"].X, mh, tws)
    e1.record()
    torch.cuda.synchronize()
    ms_rt = e0.elapsed_time(e1) / K
    st2, info2 = R.rich_retess_result(tws)
    # re-tessellation after a real move: the half-step points of the next
    # step's first stage, from the last mesh (cells whose neighbours change
    # are clipped; the repeat above proves every cell by its previous ring)
    R.rich_stage_courant(state["mesh"], state["s"], state["s"], half, 0.5, prm, ws)
    R.rich_retess(state["mesh"], half.X, mh, tws)   # warm
    e0.record()
    for _ in range(K):
        R.rich_retess(state["mesh"], half.X, mh, tws)
    e1.record()
    torch.cuda.synchronize()
    ms_mv = e0.elapsed_time(e1) / K
    st3, info3 = R.rich_retess_result(tws)
    Q = state["s"].Q
    scale = Q.abs().amax(dim=1)
    diff = ((Q - live_final[0]).abs().amax(dim=1) / scale).max().item()
    # a re-tessellation's algorithmic bytes: the points in, the previous mesh's
    # CSR and edges (an entry's neighbour is named by its edge), the new mesh
    # out (cell records, edge records, CSR, first-edge offsets)
    ne, nc = info2["n_edges"], info2["n_csr"]
    rt_bytes = (16 * n + 4 * (n + 1) + 4 * hm0.n_csr + 32 * hm0.n_edges
                + 48 * n + 32 * ne + 4 * (n + 1) + 4 * nc + 4 * (n + 1))
    rt_gbs = rt_bytes / (ms_mv / 1e3) / 1e9
    out = {"steps": n_steps, "timed_steps": K, "ms_per_step": ms,
           "cell_updates_per_s": n / (ms / 1e3),
           "retess_ms": ms_rt, "retess_cells_per_s": n / (ms_rt / 1e3),
           "retess_clipped_cells": info2["n_clipped"],
           "retess_moved_ms": ms_mv, "retess_moved_cells_per_s": n / (ms_mv / 1e3),
           "retess_moved_clipped_cells": info3["n_clipped"],
           "retess_roofline": {"bound": "alu (FP64 VALU issue; see the counter profile)",
                               "on": "retess_moved_ms",
                               "algorithmic_bytes": rt_bytes, "achieved_GBps": rt_gbs,
                               "frac_of_hbm_peak": rt_gbs / HBM_PEAK_GBS},
           "all_certified": (st == 0 and st2 == 0 and st3 == 0 and info["sticky"] == 0
                             and flags == 0),
           "n_edges": info2["n_edges"],
           "max_rel_diff_vs_host_mesh_chain": diff}
    log(f"[bench] device chain {out}")
    return out


SOD_CHAINS = {}


def per_quantity_scale(Q, area, gamma):
    """Scale of each conserved quantity for the parity metric: max|M|,
    max M (c + |v|) for both momenta, max|E|."""
    import numpy as np
    M = Q[0]
    v2 = (Q[1] ** 2 + Q[2] ** 2) / (M * M)
    p = (gamma - 1.0) * (Q[3] / area - 0.5 * (M / area) * v2)
    mom = np.max(M * (np.sqrt(gamma * p / (M / area)) + np.sqrt(v2)))
    return np.array([np.abs(M).max(), mom, mom, np.abs(Q[3]).max()])


def l_shock(O, P, mesh, Q, t):
    """eq. (Lshock): sum |phi - phi_exact|^(1/4) / (|phi_exact|^(1/4) N) for
    density and pressure, the velocity difference normalised by the exact
    sound speed; the exact solution is the 1D Riemann problem of the tube
    sampled at (x - 1/2) / t."""
    import numpy as np
    g = P.gamma
    rho = Q[0] / mesh.area
    vx = Q[1] / Q[0]
    pr = (g - 1.0) * (Q[3] / mesh.area - 0.5 * rho * (vx * vx + (Q[2] / Q[0]) ** 2))
    WL, WR = np.array([1.0, 0.0, 0.0, 1.0]), np.array([0.125, 0.0, 0.0, 0.1])
    ex = np.array([O.exact_sample(g, WL, WR, (x - 0.5) / t)[0] for x in mesh.px])
    Lr = float(np.mean(np.abs(rho - ex[:, 0]) ** 0.25 / np.abs(ex[:, 0]) ** 0.25))
    Lp = float(np.mean(np.abs(pr - ex[:, 3]) ** 0.25 / np.abs(ex[:, 3]) ** 0.25))
    cs = np.sqrt(g * ex[:, 3] / ex[:, 0])
    Lv = float(np.mean(np.abs(vx - ex[:, 1]) ** 0.25 / cs ** 0.25))
    return {"density": Lr, "pressure": Lp, "velocity": Lv}


def sod_oracle_checks(O, T, log):
    """For each 100-step shock-tube chain the GPU ran: the oracle's own chain
    from the same initial state with the same time steps (its meshes built
    from its own points), the drift between the two end states per conserved
    quantity (largest difference over that quantity's scale, the parity
    metric), and both chains' error against the exact solution by eq.
    (Lshock)."""
    import numpy as np
    res = {}
    for key, c in SOD_CHAINS.items():
        P = c["P"]
        op = O.Params(gamma=P.gamma, riemann=c["riemann"])
        m = T.rich_tess_build(P.px, P.py, P.box, P.bc)
        Q = P.state(m.area)
        X = np.stack([m.px, m.py])
        t0 = time.perf_counter()
        for dt in c["dts"]:
            Q, X, m, _, st = O.step(m, Q, X, dt, op,
                                    lambda x, y, b, bc: T.rich_tess_build(x, y, b, bc))
            if st:
                raise SystemExit(f"{key}: oracle chain status {st}")
        sc = per_quantity_scale(Q, m.area, P.gamma)
        drift = (np.max(np.abs(c["Q"] - Q), axis=1) / sc).tolist()
        # the same chain on the oracle built with fused multiply-adds: how far
        # two correctly rounded runs of the method drift apart on this problem
        fma = None
        if os.path.exists(O.FMA_LIB_PATH):
            mf = T.rich_tess_build(P.px, P.py, P.box, P.bc)
            Qf, Xf = P.state(mf.area), np.stack([mf.px, mf.py])
            with O.use_library(O.FMA_LIB_PATH):
                for dt in c["dts"]:
                    Qf, Xf, mf, _, st = O.step(mf, Qf, Xf, dt, op,
                                               lambda x, y, b, bc: T.rich_tess_build(x, y, b, bc))
                    if st:
                        raise SystemExit(f"{key}: FMA oracle chain status {st}")
            fma = dict(zip(["M", "Px", "Py", "E"],
                           (np.max(np.abs(Qf - Q), axis=1) / sc).tolist()))
        t = float(sum(c["dts"]))
        res[key] = {"steps": len(c["dts"]), "t_end": t,
                    "drift_vs_oracle_per_quantity": dict(zip(["M", "Px", "Py", "E"], drift)),
                    "oracle_fma_build_vs_oracle_per_quantity": fma,
                    "points_drift": float(np.max(np.abs(c["X"] - X))),
                    "L_shock_gpu": l_shock(O, P, c["mesh"], c["Q"], t),
                    "L_shock_oracle": l_shock(O, P, m, Q, t),
                    "oracle_chain_s": time.perf_counter() - t0}
        log(f"[bench] {key} vs oracle: {res[key]}")
    return res


def bench_config(args, R, T, name, riemann, steps, log):
    """Another configuration of the same path (time-centred steps): a live
    chain builds the meshes, then the steps are replayed with all inputs in
    HBM (stage 1 with the Courant step fused, stage 2, no synchronisation
    inside a step), timed with events; kernel times and
    the HBM roofline fraction as for the main line."""
    import numpy as np
    import torch
    P, desc, make_state = make_problem(name, 0)
    prm = R.Params(gamma=P.gamma, riemann=riemann)
    hm0 = T.rich_tess_build(P.px, P.py, P.box, P.bc, args.threads)
    n = hm0.n_cells
    ws = R.workspace(n)
    cur = R.DeviceState.from_host(make_state(hm0.area), np.stack([hm0.px, hm0.py]))
    init = R.DeviceState(cur.Q.clone(), cur.X.clone())
    half = R.DeviceState.empty_like(cur)
    nxt = R.DeviceState.empty_like(cur)
    meshes, halves, dts, nbytes = [R.DeviceMesh.from_host(hm0)], [], [], 0
    hm = hm0
    for s in range(steps):
        dt = R.rich_cfl_dt(meshes[s], cur, prm, ws)
        dts.append(dt)
        R.rich_stage(meshes[s], cur, cur, half, 0.5 * dt, prm, ws)
        xh = half.X.cpu().numpy()
        hmh = T.rich_tess_build(xh[0], xh[1], P.box, P.bc, args.threads)
        nbytes += algorithmic_bytes(hm, False) + algorithmic_bytes(hmh, True)
        halves.append(R.DeviceMesh.from_host(hmh))
        R.rich_stage(halves[s], half, cur, nxt, dt, prm, ws)
        if R.rich_stage_flags(ws):
            raise SystemExit(f"{name}: step {s} flagged")
        xn = nxt.X.cpu().numpy()
        hm = T.rich_tess_build(xn[0], xn[1], P.box, P.bc, args.threads)
        meshes.append(R.DeviceMesh.from_host(hm))
        cur, nxt = nxt, cur
    live = (cur.Q.clone(), cur.X.clone())
    cur.Q.copy_(init.Q)
    cur.X.copy_(init.X)
    torch.cuda.synchronize()
    R.rich_profile_enable(True)
    for k in ("k_cell", "k_flux"):
        R.rich_profile_read(k)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ok = True
    e0.record()
    for s in range(steps):
        R.rich_stage_courant(meshes[s], cur, cur, half, 0.5, prm, ws)
        R.rich_stage_dt_of(halves[s], half, cur, nxt, 1.0, ws, prm, ws)
        cur, nxt = nxt, cur
    e1.record()
    torch.cuda.synchronize()
    ok = R.rich_stage_dt(ws) == dts[-1]
    kc, kf = R.rich_profile_read("k_cell"), R.rich_profile_read("k_flux")
    R.rich_profile_enable(False)
    ms = e0.elapsed_time(e1) / steps
    kern_ms = (kc[0] + kf[0]) / steps
    ok = ok and bool(torch.equal(cur.Q, live[0]) and torch.equal(cur.X, live[1]))
    if name == "sod":
        # the GPU chain's end state, for the oracle comparison of the CPU
        # baseline leg (the only leg that runs the oracle)
        SOD_CHAINS["sod_64sq_exact_100_steps" if riemann else "sod_64sq_hllc_100_steps"] = {
            "P": P, "riemann": riemann, "dts": list(dts), "mesh": hm,
            "Q": live[0].cpu().numpy(), "X": live[1].cpu().numpy()}
    out = {"workload": desc, "riemann": "exact" if riemann else "hllc", "n_cells": n,
           "steps": steps, "ms_per_step": ms, "cell_updates_per_s": n / (ms / 1e3),
           "kernel_ms_per_step": kern_ms,
           "roofline_frac": (nbytes / steps) / (kern_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
           "replay_bitwise_equal_to_live": ok,
           "conservation": totals_drift(init.Q.cpu().numpy(), live[0].cpu().numpy(),
                                        float(sum(dts)), steps)}
    log(f"[bench] {name} {out}")
    return out


def bench_sweep(args, log):
    """Section 6 cell-rounding sweep (Gresho vortex, 30x30 cells, a 6x6
    (chi, eta) grid) advanced by the batched time-centred step for a fixed
    number of steps: end-to-end rate, tessellation included, with the meshes
    built by the host stage and with them rebuilt on the device."""
    import numpy as np
    import torch
    from paper_1410_3219_amd import sweep as SW
    out = {}
    for mode, dev in (("host_meshes", False), ("device_meshes", True)):
        sw = SW.Sweep(SW.chi_eta_grid(6, 6), k=30, n_threads=args.threads or 0,
                      device_tess=dev)
        sw.step()            # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.sweep_steps):
            sw.step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        n = sw.mesh0.n_cells
        L = sw.density_L()
        out[mode] = {"runs": len(sw.grid), "cells_per_run": n, "steps": args.sweep_steps,
                     "s": dt,
                     "cell_updates_per_s_end_to_end": len(sw.grid) * n * args.sweep_steps / dt,
                     "all_ok": all(s == 0 for s in sw.status),
                     "meshes_device_host": sw.tess_counts(),
                     "density_L_min": float(np.nanmin(L)), "density_L_max": float(np.nanmax(L))}
        sw.close()
        log(f"[bench] sweep {mode} {out[mode]}")
    return out


def make_problem(name, k):
    from paper_1410_3219_amd import inputs as I
    if name == "wave":
        P = I.advected_wave(k=k or 2048, seed=3)
        desc = f"advected wave {P.extra.get('amp')} amp, {int(round(P.n ** 0.5))}^2 jittered lattice, periodic unit box, v=(1,0.5), p=0.6, gamma=5/3, moving mesh"
        state = P.state
    elif name == "sedov":
        P = I.sedov(k=k or 512, seed=2, lloyd_iters=5)
        desc = f"point explosion, {P.n} uniform-random points Lloyd-relaxed 5x, walls, rho=1, p=1e-6, E=1 in the centre cell, gamma=5/3, moving mesh"
        state = lambda area: I.sedov_state(P, area)   # noqa: E731
    elif name == "sod":
        P = I.sod(k=k or 64, seed=1)
        desc = f"shock tube, {P.n} jittered lattice points, walls, gamma=5/3, moving mesh"
        state = P.state
    else:
        raise SystemExit(f"unknown workload {name}")
    return P, desc, state


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="wave", choices=["wave", "sedov", "sod"])
    ap.add_argument("--k", type=int, default=0, help="lattice side (default per workload)")
    ap.add_argument("--riemann", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched and served measurements")
    ap.add_argument("--legs", default="",
                    help="comma-separated subset of the extra legs to run (default: all)")
    ap.add_argument("--batch-runs", type=int, default=256)
    ap.add_argument("--sweep-steps", type=int, default=20)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--threads", type=int, default=0, help="host tessellation threads")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a device-to-device copy of this size first (counter calibration)")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("PMC_DIR", "NAME", "COMMAND"),
                    help="average each counter per kernel over a rocprofv3 --pmc run into "
                         "profiles/NAME.txt, recording COMMAND as the run that made it")
    ap.add_argument("--summarize-trace", nargs=4, metavar=("TRACE_DIR", "NAME", "TITLE", "COMMAND"),
                    help="per-kernel durations of a rocprofv3 --kernel-trace --stats run into "
                         "profiles/NAME.txt, recording TITLE and COMMAND")
    ap.add_argument("--summarize-pmc", nargs="+", metavar="PMC_DIR",
                    help="turn rocprofv3 --pmc runs (FETCH_SIZE; WRITE_SIZE; optionally the "
                         "raw TCC read-request counters) of this script with --copy-probe-mib "
                         "into profiles/traffic_<workload>.txt")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        log("bench.py measures one GPU only: this build has no multi-GPU path "
            "(each run or batch runs on one MI355X); run with --gpus 1.")
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1410_3219_amd import rich as R
    from paper_1410_3219_amd import tess as T

    assert torch.cuda.is_available(), "needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    R.lib()  # fail loudly if the HIP library is missing

    t0 = time.time()
    P, desc, make_state = make_problem(args.workload, args.k)
    log(f"[bench] problem {args.workload}: {P.n} cells ({time.time() - t0:.1f}s)")
    params = R.Params(gamma=P.gamma, riemann=args.riemann)
    K, W = args.steps, args.warmup

    tess_times, h2d_times = [], []

    def tessellate(x, y):
        t = time.time()
        hm = T.rich_tess_build(x, y, P.box, P.bc, args.threads)
        tess_times.append(time.time() - t)
        return hm

    def upload(hm):
        torch.cuda.synchronize()
        t = time.time()
        dm = R.DeviceMesh.from_host(hm)
        torch.cuda.synchronize()
        h2d_times.append(time.time() - t)
        return dm

    if args.copy_probe_mib:
        # calibration copy of a known size; the source is evicted from the
        # last-level cache first by streaming through another buffer
        nbytes = args.copy_probe_mib << 20
        a = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        flush = torch.empty((1 << 30) // 8, dtype=torch.float64, device=dev).fill_(2.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        # gather probes of known size: rows of 32, 64 and 128 bytes at
        # distinct scattered rows (odd multiplicative hash, a bijection on a
        # power-of-two row count) of a 1 GiB table, 64 MiB of rows each,
        # each after a 1 GiB flush; read = rows + 8-byte indices, write = rows
        tab = torch.empty((1 << 30) // 8, dtype=torch.float64, device=dev).fill_(1.0)
        for w in GATHER_PROBE_DOUBLES:
            rows = tab.view(-1, w)
            nsel = (64 << 20) // (8 * w)
            idx = (torch.arange(nsel, dtype=torch.int64, device=dev) * 0x9E3779B1) & (rows.shape[0] - 1)
            flush.fill_(3.0)
            torch.cuda.synchronize()
            rows.index_select(0, idx)
            torch.cuda.synchronize()
        del tab, flush

    # ---------------- live chain: GPU stages + host tessellation -----------
    hm0 = tessellate(P.px, P.py)
    n = hm0.n_cells
    Q0 = make_state(hm0.area)
    X0 = np.stack([hm0.px, hm0.py])
    ws = R.workspace(n)
    meshes, halves, dts = [upload(hm0)], [], []
    cur = R.DeviceState.from_host(Q0, X0)
    init = R.DeviceState(cur.Q.clone(), cur.X.clone())
    half = R.DeviceState.empty_like(cur)
    nxt = R.DeviceState.empty_like(cur)
    host_half0 = None
    bytes_step = None
    for s in range(W + K):
        dt = R.rich_cfl_dt(meshes[s], cur, params, ws)
        dts.append(dt)
        R.rich_stage(meshes[s], cur, cur, half, 0.5 * dt, params, ws)
        f = R.rich_stage_flags(ws)
        if f:
            raise SystemExit(f"stage 1 of step {s} flagged {f}")
        xh = half.X.cpu().numpy()
        hmh = tessellate(xh[0], xh[1])
        if s == 0:
            host_half0 = (hmh, half.Q.cpu().numpy().copy())
            bytes_step = algorithmic_bytes(hm0, False) + algorithmic_bytes(hmh, True)
        halves.append(upload(hmh))
        R.rich_stage(halves[s], half, cur, nxt, dt, params, ws)
        f = R.rich_stage_flags(ws)
        if f:
            raise SystemExit(f"stage 2 of step {s} flagged {f}")
        xn = nxt.X.cpu().numpy()
        meshes.append(upload(tessellate(xn[0], xn[1])))
        cur, nxt = nxt, cur
        log(f"[bench] live step {s + 1}/{W + K}: dt={dt:.3e} tess {tess_times[-1]:.2f}s "
            f"(mesh {meshes[-1].nbytes() / 1e6:.0f} MB)")
    live_final = (cur.Q.clone(), cur.X.clone())

    # ---------------- timed replay, all inputs resident in HBM -------------
    stream = torch.cuda.current_stream()

    dt_mismatch = []

    def run_step(s, a, hbuf, b):
        # A0 fused into stage 1's cell pass: dt = cfl * min R/(c+|v-w|) is
        # reduced and kept on the device, stage 1 steps dt/2 and stage 2 dt
        # from it; nothing synchronises inside the step
        R.rich_stage_courant(meshes[s], a, a, hbuf, 0.5, params, ws)
        R.rich_stage_dt_of(halves[s], hbuf, a, b, 1.0, ws, params, ws)

    cur = R.DeviceState(init.Q.clone(), init.X.clone())
    nxt = R.DeviceState.empty_like(cur)
    for s in range(W):
        run_step(s, cur, half, nxt)
        cur, nxt = nxt, cur
    torch.cuda.synchronize()
    R.rich_profile_enable(True)
    for k_ in ("k_cell", "k_flux"):
        R.rich_profile_read(k_)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for s in range(W, W + K):
        run_step(s, cur, half, nxt)
        cur, nxt = nxt, cur
    ev1.record(stream)
    torch.cuda.synchronize()
    R.rich_profile_enable(False)
    ms_total = ev0.elapsed_time(ev1)
    kern = {k_: R.rich_profile_read(k_) for k_ in ("k_cell", "k_flux")}
    flags = R.rich_stage_flags(ws)
    dt_last = R.rich_stage_dt(ws)
    if dt_last != dts[W + K - 1]:
        dt_mismatch.append((W + K - 1, dt_last, dts[W + K - 1]))
    replay_ok = bool(torch.equal(cur.Q, live_final[0]) and torch.equal(cur.X, live_final[1])
                     and not dt_mismatch)
    log(f"[bench] timed {K} steps: {ms_total:.3f} ms, flags={flags}, replay bitwise={replay_ok}")

    # measured copy bandwidth: a 1 GiB device-to-device copy (read + write);
    # not in counter runs, whose calibration copy must stay the largest
    copy_gbs = None
    if not args.copy_probe_mib:
        ca = torch.empty((1 << 30) // 8, dtype=torch.float64, device=dev).fill_(1.0)
        cb = torch.empty_like(ca)
        cb.copy_(ca)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(5):
            cb.copy_(ca)
        ev1.record(stream)
        torch.cuda.synchronize()
        copy_gbs = 5 * 2 * (1 << 30) / (ev0.elapsed_time(ev1) / 1e3) / 1e9
        del ca, cb

    ms_per_step = ms_total / K
    value = n * K / (ms_total / 1e3)
    # one pass of the hot path = k_cell + k_flux; report the pair as the
    # dominant unit (two launches per stage, two stages per step)
    stage_ms = (kern["k_cell"][0] + kern["k_flux"][0]) / max(1, kern["k_cell"][1]) * 2
    achieved = bytes_step / (stage_ms / 1e3) / 1e9
    traffic = None
    traffic_kernels = None
    tj = read_traffic(args.workload)
    if tj and tj.get("source_hash") == kernel_source_hash() and tj.get("n_cells") == n:
        traffic = tj.get("bytes_per_step")
        # per kernel: counter bytes per launch, and the rate they move at in
        # this run's own launches
        traffic_kernels = {}
        for k_, e in tj["kernels"].items():
            b = e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]
            launch_ms = kern[k_][0] / max(1, kern[k_][1])
            traffic_kernels[k_] = {"bytes_per_launch": b, "bytes_per_cell": b / n,
                                   "GBps_at_measured_duration": b / (launch_ms / 1e3) / 1e9}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "n_cells": n,
            "n_edges": hm0.n_edges,
            "riemann": "exact" if args.riemann else "hllc",
            "scheme": "time-centred fluxes, two stages per step, switching limiter",
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_cell+k_flux (one stage; two stages per step)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_over_algorithmic": traffic / bytes_step if traffic else None,
            "traffic_per_kernel": traffic_kernels,
            "measured_copy_GBps": copy_gbs,
            "frac_of_measured_copy": achieved / copy_gbs if copy_gbs else None,
            "algorithmic_bytes_per_step": bytes_step,
            "kernel_ms_per_step": {k_: v[0] / K for k_, v in kern.items()},
            "launches": {k_: v[1] for k_, v in kern.items()},
        },
        "replay_bitwise_equal_to_live": replay_ok,
        "conservation": totals_drift(Q0, live_final[0].cpu().numpy(), float(sum(dts)), W + K),
        "host_input_stage": {
            "tessellation_s_mean": float(np.mean(tess_times)),
            "tessellations": len(tess_times),
            "h2d_s_mean": float(np.mean(h2d_times)),
            "end_to_end_ms_per_step_estimate": ms_per_step + 2e3 * (
                float(np.mean(tess_times)) + float(np.mean(h2d_times))),
        },
    }

    if not args.no_extras:
        legs = {
            "batched": lambda: bench_batch(args, R, T, log),
            "served": lambda: bench_serve(args, R, log),
            "served_moving": lambda: bench_serve_moving(args, R, log),
            "sweep_section6": lambda: bench_sweep(args, log),
            "extrapolated_fluxes": lambda: bench_extrapolated(args, R, T, P, make_state, hm0,
                                                              meshes[0], log),
            "device_retess_chain": lambda: bench_device_chain(args, R, P, make_state, hm0,
                                                              meshes[0], live_final, W + K, log),
            "sedov_512sq": lambda: bench_config(args, R, T, "sedov", 0, 5, log),
            "sod_64sq_hllc_100_steps": lambda: bench_config(args, R, T, "sod", 0, 100, log),
            "sod_64sq_exact_100_steps": lambda: bench_config(args, R, T, "sod", 1, 100, log),
        }
        want = [x for x in args.legs.split(",") if x] or list(legs)
        for name in want:
            out[name] = legs[name]()
        if "batched" in out:
            b = out["batched"]
            # the batch (shock tubes) against a plain single shock tube of the
            # same total size, its step taken on the device as in the timed
            # step above; and each batched form against this run's plain rate
            out["batched_over_plain"] = (b["device_dt"]["graph_replay"]["cell_updates_per_s"] /
                                         b["plain_sod"]["cell_updates_per_s"])
            out["batched_vs_plain_wave"] = {
                "eager_host_steps": b["batched"]["cell_updates_per_s"] / value,
                "graph_host_steps": b["graph_replay"]["cell_updates_per_s"] / value,
                "eager_device_steps": b["device_dt"]["eager"]["cell_updates_per_s"] / value,
                "graph_device_steps": b["device_dt"]["graph_replay"]["cell_updates_per_s"] / value}
        if "served" in out:
            out["served_saturated_over_plain"] = (
                out["served"]["saturated"]["cell_updates_per_s"] / value)

    # ---------------- CPU baseline: the oracle on one step -----------------
    if not args.no_cpu_baseline:
        sys.path.insert(0, os.path.join(ROOT, "oracle"))
        import oracle as O
        op = O.Params(gamma=params.gamma, cfl=params.cfl, theta=params.theta,
                      delta_v=params.delta_v, delta_p=params.delta_p, chi=params.chi,
                      eta=params.eta, riemann=params.riemann, motion=params.motion,
                      limiter=params.limiter)
        hmh, Qh_gpu = host_half0
        O.build()

        def oracle_step():
            t = time.perf_counter()
            r1 = O.stage(hm0, Q0, Q0, X0, 0.5 * dts[0], op)
            O.stage(hmh, Qh_gpu, Q0, X0, dts[0], op)
            return time.perf_counter() - t, r1

        # the reference (serial) build, then the same source with its
        # per-cell and per-edge loops on all host cores (OpenMP)
        t_cpu, r1 = oracle_step()
        with O.use_library(O.OMP_LIB_PATH):
            n_threads = O.threads()
            t_all, r1_all = oracle_step()
        same = bool(np.array_equal(r1.Q, r1_all.Q))
        err = float(np.max(np.abs(r1.Q - Qh_gpu), axis=1).max() / np.abs(Q0).max())
        log(f"[bench] oracle step {t_cpu:.1f}s on 1 core, {t_all:.2f}s on {n_threads} threads "
            f"(same bits: {same}; stage-1 max |diff| / max|Q| = {err:.2e})")
        out["cpu_baseline"] = {
            "value": n / t_all,
            "unit": "cell-updates/s",
            "cores": n_threads,
            "kind": "oracle",
            "sample": f"one full time-centred step (both stages) of the same {n}-cell workload, C oracle with its per-cell and per-edge loops on {n_threads} OpenMP threads, step 0 meshes",
            "single_core": {"value": n / t_cpu, "cores": 1,
                            "sample": "the same step, serial reference build"},
            "parallel_build_bitwise_equal": same,
            "host_cpus": os.cpu_count(),
        }
        out["full_size_stage1_max_rel_diff_vs_oracle"] = err
        if SOD_CHAINS:
            out["cpu_baseline"]["sod_64sq_oracle_checks"] = sod_oracle_checks(O, T, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
