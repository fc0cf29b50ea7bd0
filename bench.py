#!/usr/bin/env python3
"""Benchmark of the H-matrix hot path on one MI355X.

One step = the whole hot path on one synthetic mesh, for the FP32 and the
FP64 form: hm_build (Morton tree, Algorithm 1, near field, batched ACA),
H-matrix products (1 and 16 right-hand sides), the transposed product, a
GMRES solve, hm_free.

Printed: one JSON line.  `value` is the H-matvec throughput (algorithmic
bytes / time, single right-hand side) of the FP32 form; setup seconds, the
FP64 form, the sampled relative error against the oracle, the roofline of
the dominant kernel and the CPU oracle baseline are extra keys.

The CPU leg (oracle rows of the direct product on a process pool) runs first,
before the GPU is touched.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM traffic of the dominant kernel, from rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs; valid only while the sources it was taken on are unchanged.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_fwd2_f32_icosphere_L6_traffic.txt")
TRAFFIC_SOURCES = ("hm_matvec.hip", "hm_setup.hip", "hm_internal.h")
METRIC = "H-setup s + H-matvec GB/s (% HBM peak) at rel.err ≤1e-6, FP32 vs FP64"


# ---------------------------------------------------------------- CPU leg
_OP = None


def _rows_worker(args):
    rows, x = args
    return _OP.matvec_rows(x, rows)


def cpu_baseline(V, T, x, rows, workers):
    """Oracle: exact rows of the dense product A x, over a process pool."""
    global _OP
    import multiprocessing as mp
    from oracle import bem
    _OP = bem.Operator(V, T)
    chunks = [rows[i::workers] for i in range(workers)]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        parts = pool.map(_rows_worker, [(c, x) for c in chunks])
    t = time.perf_counter() - t0
    y = np.empty((rows.size,) + x.shape[1:])
    for i, c in enumerate(chunks):
        y[i::workers] = parts[i]
    return y, t


# ---------------------------------------------------------------- GPU leg
def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1806_11558_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(level, leaf, eps, form):
    """HBM bytes per launch of the dominant kernel from the stored counter
    summary, or None if it is missing, for another workload, or stale."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if (kv["sources_sha256"] != sources_sha256() or int(kv["level"]) != level
                or int(kv["leaf"]) != leaf or float(kv["eps"]) != eps or kv["form"] != form):
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_probe(mib):
    """A plain copy of known size (read mib MiB, write mib MiB) for scaling
    the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    x = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.add(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": mib << 20, "copy_probe_bytes_written": mib << 20,
                      "launches": 3}), flush=True)


def mv_bytes(st, s_store, s_vec, s_acc, nrhs=1):
    """Algorithmic bytes of one product: every stored value once, x and y
    once, the permutation, 16 B per block descriptor."""
    n = st["n"]
    return (s_store * (st["dense_entries"] + st["lr_entries"]) + n * nrhs * 2 * s_vec + 4 * n
            + 16 * (st["n_dense"] + st["n_lr"]))


def phase2_bytes(st, s_store, s_acc, s_vec, nrhs=1):
    """Algorithmic bytes of the dominant kernel (dense blocks and U slices
    applied per row leaf): stored values, gathered x and t once, y once,
    the permutation and one 4-byte column index per panel column."""
    n = st["n"]
    return (s_store * (st["dense_entries"] + st["lr_u_entries"]) + n * nrhs * s_acc
            + st["rank_sum"] * nrhs * s_acc + n * nrhs * s_vec + 4 * n + 4 * st["n_panel_cols"])


# Kernel evaluations of the setup: 7 nodes x (3 sub, 3 mul/fma, rsqrt, add)
# plus the centroid difference, weights and scale: about 66 operations per
# entry (the rsqrt counted as one).  ACA updates are not counted.
FLOPS_PER_ENTRY = 66
VALU_PEAK_TFLOPS = {"f32": 157.3, "f16": 157.3, "f64": 78.6}


def setup_roofline(o, form):
    """ALU roofline of the near field + ACA phases: entry evaluations (dense
    entries + ACA rows and columns) x FLOPS_PER_ENTRY over their time."""
    st = o["stats"]
    ms = o["setup_phases_ms"]["near_field"] + o["setup_phases_ms"]["aca"]
    ent = st["dense_entries"] + st["aca_entry_evals"]
    tf = ent * FLOPS_PER_ENTRY / (ms * 1e-3) / 1e12
    return {"bound": "alu", "entries": ent, "entries_per_s": round(ent / (ms * 1e-3), 1),
            "achieved": round(tf, 3), "peak": VALU_PEAK_TFLOPS[form], "unit": "TFLOP/s",
            "frac": round(tf / VALU_PEAK_TFLOPS[form], 5),
            "phases": "near_field + aca", "ms": round(ms, 3)}


def run_form(hm, torch, V, T, args, prec, xg, fg, keep):
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = hm.HMatrix(V, T, leaf_size=args.leaf, eta=1.0, eps=args.eps, max_rank=64,
                   precision=prec, profile=True)
    setup_s = time.perf_counter() - t0
    st = H.stats()
    n = st["n"]
    x1 = xg[:, 0].contiguous()
    y1 = torch.empty_like(x1)
    H.matvec(x1, out=y1)                     # untimed first call
    H.kernel_times()                          # reset kernel counters
    ms = []
    for _ in range(args.reps):
        a, b = ev(), ev()
        a.record()
        H.matvec(x1, out=y1)
        b.record()
        b.synchronize()
        ms.append(a.elapsed_time(b))
    kt = H.kernel_times()
    y16 = torch.empty_like(xg)
    ms16 = []
    for _ in range(3):
        a, b = ev(), ev()
        a.record()
        H.matvec(xg, out=y16)
        b.record()
        b.synchronize()
        ms16.append(a.elapsed_time(b))
    yT = H.matvec_T(x1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sig, info, status = H.solve(fg, tol=args.gmres_tol, restart=100, max_iter=2000)
    solve_s = time.perf_counter() - t0
    if keep is not None:
        keep[prec] = (y1.double().cpu().numpy(), yT.double().cpu().numpy(), st)
    tm = H.timings()
    H.free()
    return dict(setup_s=setup_s, st=st, ms=ms, ms16=ms16, kt=kt, solve_s=solve_s,
                gmres_iters=info.iters, gmres_status=int(status),
                gmres_rel_residual=info.rel_residual, timings=tm)


def run_batch48(args):
    """48 seeded perturbed spheres (seed g, level 4 + g mod 3) in one handle
    (hm_build_batch, autotuned product schedule), FP32 form; one step =
    build, 8-column products, GMRES with 8 right-hand sides per geometry
    (graph-replayed Arnoldi steps), free."""
    import torch
    import paper_1806_11558_amd as hm
    from synthetic import normal_columns, perturbed_sphere
    meshes = [perturbed_sphere(4 + g % 3, seed=g) for g in range(48)]
    sizes = [t.shape[0] for _, t in meshes]
    n = int(sum(sizes))
    X = np.concatenate([normal_columns(k, 8, seed=1000 + g) for g, k in enumerate(sizes)])
    torch.cuda.set_device(0)
    xg = torch.tensor(X, device="cuda")
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def step():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H = hm.HMatrix.batch(meshes, leaf_size=args.leaf, eta=1.0, eps=args.eps, max_rank=64,
                             precision="f32", autotune=True)
        setup = time.perf_counter() - t0
        y = torch.empty_like(xg)
        H.matvec(xg, out=y)
        ms = []
        for _ in range(max(3, args.reps // 4)):
            a, b = ev(), ev()
            a.record()
            H.matvec(xg, out=y)
            b.record()
            b.synchronize()
            ms.append(a.elapsed_time(b))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sig, info, status = H.solve(xg, tol=args.gmres_tol, restart=100, max_iter=2000, graph=True)
        solve = time.perf_counter() - t0
        st = H.stats()
        tune = H.tune_results().tolist()
        H.free()
        return setup, ms, solve, info, int(status), st, tune

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = [step() for _ in range(args.steps)]
    wall = time.perf_counter() - t0
    setup = float(np.median([r[0] for r in rs]))
    ms8 = float(np.median([m for r in rs for m in r[1]]))
    st = rs[-1][5]
    B = mv_bytes(st, 4, 8, 8, nrhs=8)
    print(f"# batch48: N={n}, setup {setup:.3f} s, 8-rhs product {ms8:.3f} ms, "
          f"gmres {rs[-1][3].iters} it {rs[-1][2]:.2f} s", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC,
        "value": round(B / ms8 / 1e6, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000 * wall / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"48 perturbed spheres (seed g, icosphere level 4 + g mod 3; "
                               f"N = {n} in one handle), leaf {args.leaf}, eta 1, ACA eps "
                               f"{args.eps:g}, FP32 form, autotuned product schedule; 8 "
                               f"right-hand sides N(0,1) seeds 1000 + g; graph GMRES to "
                               f"{args.gmres_tol:g}", "n": n, "nrhs": 8},
        "setup_s": round(setup, 4),
        "matvec8_ms": round(ms8, 4),
        "matvec8_bytes": B,
        "gmres_s": round(float(np.median([r[2] for r in rs])), 4),
        "gmres_iters": rs[-1][3].iters,
        "gmres_status": rs[-1][4],
        "gmres_rel_residual": rs[-1][3].rel_residual,
        "tune_unit_cols_ms": rs[-1][6],
        "stats": {k: st[k] for k in ("n_geom", "n_dense", "n_lr", "rank_max", "stored_bytes",
                                     "unit_cols", "aca_chunks")},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--level", type=int, default=6, help="icosphere refinements (N = 20*4^L)")
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--reps", type=int, default=20, help="timed 1-rhs products per form and step")
    ap.add_argument("--gmres-tol", type=float, default=1e-6)
    ap.add_argument("--cpu-rows", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="f32,f64",
                    help="comma list of f32, f64, f16 (FP32 dense + FP16 factors)")
    ap.add_argument("--rhs", default="ones", choices=["ones", "normal"],
                    help="GMRES right-hand side: f = 1 or a seeded N(0,1) column")
    ap.add_argument("--workload", default="single", choices=["single", "batch48"],
                    help="single: one icosphere (default); batch48: 48 perturbed spheres of "
                         "5,120 / 20,480 / 81,920 triangles in one handle, 8 right-hand sides")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain copy of MIB MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the path would shard by row clusters over GPUs; not built)", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.workload == "batch48":
        run_batch48(args)
        return

    from synthetic import icosphere, normal_columns, sample_rows
    V, T = icosphere(args.level)
    n = T.shape[0]
    X = normal_columns(n, 16, seed=0)
    rows = sample_rows(n, args.cpu_rows, seed=1)

    cpu = None
    if not args.no_cpu_baseline:
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
        y_ref, t_cpu = cpu_baseline(V, T, X[:, 0], rows, workers)
        cpu = dict(y_ref=y_ref, t=t_cpu, workers=workers)

    import torch
    import paper_1806_11558_amd as hm
    torch.cuda.set_device(0)
    forms = args.forms.split(",")
    xg = torch.tensor(X, device="cuda")
    if args.rhs == "ones":
        fg = torch.ones(n, dtype=torch.float64, device="cuda")
    else:
        fg = torch.tensor(normal_columns(n, 1, seed=2)[:, 0], device="cuda")

    for _ in range(args.warmup):
        for prec in forms:
            run_form(hm, torch, V, T, args, prec, xg, fg, None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = {p: [] for p in forms}
    keep = {}
    for k in range(args.steps):
        for prec in forms:
            r = run_form(hm, torch, V, T, args, prec, xg, fg, keep if k == args.steps - 1 else None)
            res[prec].append(r)
            print(f"# step {k} {prec}: setup {r['setup_s']:.3f} s, matvec "
                  f"{np.median(r['ms']):.3f} ms, gmres {r['gmres_iters']} it {r['solve_s']:.2f} s",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    out = {}
    for prec in forms:
        rs = res[prec]
        st = rs[-1]["st"]
        s_store = {"f32": 4, "f64": 8, "f16": 4}[prec]
        s_vec = 8                       # x is double (torch default)
        s_acc = 8
        B = mv_bytes(st, s_store, s_vec, s_acc)
        B16 = mv_bytes(st, s_store, s_vec, s_acc, 16)
        if prec == "f16":
            # dense blocks in FP32, factors in FP16: use the stored bytes
            extra = st["stored_bytes"] - s_store * (st["dense_entries"] + st["lr_entries"])
            B += extra
            B16 += extra
        ms = float(np.median([m for r in rs for m in r["ms"]]))
        ms16 = float(np.median([m for r in rs for m in r["ms16"]]))
        p2 = [r["kt"]["fwd_panels"] for r in rs]
        p2_ms = sum(q["ms"] for q in p2) / max(1, sum(q["launches"] for q in p2))
        p2_B = phase2_bytes(st, s_store, s_acc, s_vec)
        if prec == "f16":
            p2_B -= 2 * st["lr_u_entries"]
        o = dict(
            setup_s=float(np.median([r["setup_s"] for r in rs])),
            setup_phases_ms={k: round(v, 3) for k, v in rs[-1]["timings"].items()},
            matvec_ms=ms, matvec_gbs=B / ms / 1e6, matvec_bytes=B,
            matvec16_ms=ms16, matvec16_gbs=B16 / ms16 / 1e6,
            phase2_ms=p2_ms, phase2_bytes=p2_B, phase2_gbs=p2_B / p2_ms / 1e6,
            kernel_ms_per_launch={k: (v["ms"] / v["launches"] if v["launches"] else None)
                                  for k, v in rs[-1]["kt"].items() if v["launches"]},
            gmres_iters=rs[-1]["gmres_iters"], gmres_s=float(np.median([r["solve_s"] for r in rs])),
            gmres_status=rs[-1]["gmres_status"],
            gmres_rel_residual=rs[-1]["gmres_rel_residual"],
            stats={k: st[k] for k in ("n_dense", "n_lr", "dense_entries", "lr_entries",
                                      "rank_sum", "rank_max", "cap_hits", "stored_bytes",
                                      "aca_entry_evals", "device_bytes", "aca_chunks")},
        )
        if cpu is not None and prec in keep:
            y1 = keep[prec][0]
            o["rel_err_sampled"] = float(np.linalg.norm(y1[rows] - cpu["y_ref"]) /
                                         np.linalg.norm(cpu["y_ref"]))
        out[prec] = o

    main_form = "f32" if "f32" in out else forms[0]
    M = out[main_form]
    line = {
        "metric": METRIC,
        "value": round(M["matvec_gbs"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000 * wall / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_form,
        "data": "synthetic",
        "config": {"workload": f"unit icosphere L={args.level} (N={n}) Laplace single-layer "
                               f"collocation, leaf {args.leaf}, eta 1, ACA eps {args.eps:g}; "
                               f"product x: N(0,1) seed 0; GMRES f={args.rhs} to {args.gmres_tol:g}",
                   "n": n, "eps": args.eps, "forms": forms},
        "setup_s": {p: round(out[p]["setup_s"], 4) for p in out},
        "gmres_s": {p: round(out[p]["gmres_s"], 4) for p in out},
        "gmres_iters": {p: out[p]["gmres_iters"] for p in out},
        "matvec_gbs": {p: round(out[p]["matvec_gbs"], 1) for p in out},
        "matvec_pct_hbm_peak": {p: round(100 * out[p]["matvec_gbs"] / HBM_PEAK_GBS, 1) for p in out},
        "rel_err_sampled": {p: out[p].get("rel_err_sampled") for p in out},
        "roofline": {
            "kernel": "k_fwd2 + k_fwd2_sum (row-leaf panels: dense blocks + U slices), " + main_form,
            "bound": "hbm",
            "achieved": round(M["phase2_gbs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(M["phase2_gbs"] / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args.level, args.leaf, args.eps, main_form),
        },
        "setup_roofline": {p: setup_roofline(out[p], p) for p in out},
        "forms": out,
    }
    if cpu is not None:
        full_s = cpu["t"] * n / rows.size
        line["cpu_baseline"] = {
            "value": round(M["matvec_bytes"] / full_s / 1e9, 4),
            "unit": "GB/s",
            "cores": cpu["workers"],
            "kind": "oracle",
            "sample": f"{rows.size} exact rows of the dense product A x (7-point rule, FP64) at "
                      f"N={n} in {cpu['t']:.2f} s on {cpu['workers']} processes; full product "
                      f"extrapolated x{n / rows.size:.0f} to {full_s:.1f} s; reported as the "
                      "FP32 H-matvec's algorithmic bytes / that time",
        }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
