#!/usr/bin/env python3
"""Benchmark of the H-matrix hot path on one MI355X.

Workload (default): the unit icosphere refined 8 times, N = 1,310,720 flat
triangles, Laplace single-layer collocation, leaf 64, eta 1.

One timed step = the whole hot path for the FP32 form at ACA eps 1e-6:
hm_build (Morton tree, Algorithm 1, near field, batched ACA), H-matrix
products with 1 and 16 right-hand sides, the transposed product, and a solve
of H s = f (f a seeded N(0,1) column) to the relative residual 1e-8 by
iterative refinement around GMRES with float products, then hm_free.
After the timed steps the FP64 form (eps 1e-6, plain GMRES in double) and the
FP16-factor form (eps 1e-4, refinement) run the same pass once after one
warm-up, so that their setup + solve times at the same final residual stand
next to the FP32 form's.

Printed: one JSON line.  `value` is the FP32 form's H-matvec throughput
(algorithmic bytes / time, one right-hand side, inputs resident in HBM).
Setup seconds, the other forms, the relative error of every form's product
against 4,096 exact oracle rows, the roofline of the dominant product kernel
and the CPU oracle baseline are extra keys.

The CPU leg (the oracle's exact rows of the direct product, on a process
pool) runs first, before the GPU is touched.

--operator galerkin runs the same pass on the Galerkin matrix (piecewise
constants, HM_GALERKIN) and solves it by CG (HM_SOLVE_CG), the paper's own
discretisation and solver; its CPU leg and error reference are the Galerkin
oracle's exact rows.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM traffic of the dominant kernel, from rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs; valid only while the sources it was taken on are unchanged.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_fwd2_f32_icosphere_L8_traffic.txt")
TRAFFIC_SOURCES = ("hm_matvec.hip", "hm_setup.hip", "hm_internal.h")
# exact oracle rows of A X at 4,096 sampled indices for the icosphere L=8,
# written by tests/golden/make_fullsize_refs.py (oracle only)
GOLDEN_L8 = os.path.join(ROOT, "tests", "golden", "icosphere_L8_refs.npz")
METRIC = "H-setup s + H-matvec GB/s (% HBM peak) at rel.err ≤1e-6, FP32 vs FP64"
# the host's CPU share per GPU: worker pools never exceed it
CPU_SHARE = 16


# ---------------------------------------------------------------- CPU leg
_OP = None


def _rows_worker(args):
    rows, x = args
    return _OP.matvec_rows(x, rows)


def cpu_baseline(V, T, x, rows, workers, operator="collocation"):
    """Oracle: exact rows of the dense product A x, over a process pool."""
    global _OP
    import multiprocessing as mp
    from oracle import bem, galerkin
    _OP = galerkin.GalerkinOperator(V, T) if operator == "galerkin" else bem.Operator(V, T)
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


def measured_traffic(level, leaf, eps, form, vec, operator="collocation"):
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
                or int(kv["leaf"]) != leaf or float(kv["eps"]) != eps or kv["form"] != form
                or kv.get("vectors", "f64") != vec
                or kv.get("operator", "collocation") != operator):
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


FACTOR_BYTES = {"f64": 8, "f32": 4, "f16": 2}
DENSE_BYTES = {"f64": 8, "f32": 4, "f16": 4}


def stored_bytes(st, form):
    """Dense entries at the dense storage size, low-rank factor entries at the
    factor storage size, plus one FP32 scale per term of FP16 factors."""
    b = DENSE_BYTES[form] * st["dense_entries"] + FACTOR_BYTES[form] * st["lr_entries"]
    if form == "f16":
        b += 4 * st["rank_sum"]
    return b


def mv_bytes(st, form, s_vec, nrhs=1):
    """Algorithmic bytes of one product: every stored value once, x and y
    once, the permutation, 16 B per block descriptor."""
    n = st["n"]
    return (stored_bytes(st, form) + n * nrhs * 2 * s_vec + 4 * n
            + 16 * (st["n_dense"] + st["n_lr"]))


def phase2_bytes(st, form, s_vec, s_acc, nrhs=1):
    """Algorithmic bytes of the dominant kernel pair (dense blocks and U
    slices applied per row leaf, then the partial rows summed and scattered):
    the dense entries and U factor entries once, z = [x in Morton order ; t]
    read once, y written once, the permutation once."""
    n = st["n"]
    return (DENSE_BYTES[form] * st["dense_entries"] + FACTOR_BYTES[form] * st["lr_u_entries"]
            + (n + st["rank_sum"]) * nrhs * s_acc + n * nrhs * s_vec + 4 * n)


# Kernel evaluations of the setup: 7 nodes x (3 sub, 3 mul/fma, rsqrt, add)
# plus the centroid difference, weights and scale: about 66 operations per
# entry (the rsqrt counted as one).  ACA updates are not counted.  Packed FP32
# instructions are disabled in every build, so the FP32 peak is the
# non-packed vector rate, the same as FP64.
# A Galerkin entry is the same sum at each of the seven nodes of the row
# triangle: 7 x 66 (its singular entries, about 13 per row, are not counted).
FLOPS_PER_ENTRY = {"collocation": 66, "galerkin": 7 * 66}
VALU_PEAK_TFLOPS = {"f32": 78.6, "f16": 78.6, "f64": 78.6}


def setup_roofline(o, form, operator="collocation"):
    """ALU roofline of the near field + ACA phases: entry evaluations (dense
    entries + ACA rows and columns) x FLOPS_PER_ENTRY over their time.  The
    fraction of the ALU peak is a lower bound on how well the setup uses the
    chip: the counters show the ACA's workgroup classes bound by the bytes
    they stream and its wavefront classes by step latency (`note`)."""
    st = o["stats"]
    ms = o["setup_phases_ms"]["near_field"] + o["setup_phases_ms"]["aca"]
    ent = st["dense_entries"] + st["aca_entry_evals"]
    tf = ent * FLOPS_PER_ENTRY[operator] / (ms * 1e-3) / 1e12
    return {"bound": "alu", "entries": ent, "entries_per_s": round(ent / (ms * 1e-3), 1),
            "achieved": round(tf, 3), "peak": VALU_PEAK_TFLOPS[form], "unit": "TFLOP/s",
            "frac": round(tf / VALU_PEAK_TFLOPS[form], 5),
            "phases": "near_field + aca", "ms": round(ms, 3),
            "note": "ACA workgroup classes (blocks above 256) stream source records and "
                    "earlier terms at 6-7.5 TB/s by FETCH_SIZE; wavefront classes are bound "
                    "by step latency (profiles/setup_k_aca_k_near_f32_icosphere_L8_traffic.md)"}


def _timed(torch, fn, reps):
    """Median-ready list of HIP-event times (ms) of fn() on torch's current
    stream (the library's calls are issued on that stream)."""
    out = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        out.append(a.elapsed_time(b))
    return out


def run_form(hm, torch, V, T, args, spec, X, X1, f, keep):
    """One pass of the hot path for one form: build, products (1 and 16
    right-hand sides), transposed product, solve to args.gmres_tol, free."""
    prec, eps, vec, refine = spec["form"], spec["eps"], spec["vec"], spec["refine"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = hm.HMatrix(V, T, leaf_size=args.leaf, eta=1.0, eps=eps, max_rank=64, precision=prec,
                   profile=True, operator=args.operator)
    setup_s = time.perf_counter() - t0
    st = H.stats()
    xv = X[vec]
    x1 = X1[vec]
    y1 = torch.empty_like(x1)
    H.matvec(x1, out=y1)                      # untimed first call
    H.kernel_times()                          # reset kernel counters
    ms = _timed(torch, lambda: H.matvec(x1, out=y1), args.reps)
    kt = H.kernel_times()
    y16 = torch.empty_like(xv)
    ms16 = _timed(torch, lambda: H.matvec(xv, out=y16), 3)
    yT = torch.empty_like(x1)
    msT = _timed(torch, lambda: H.matvec_T(x1, out=yT), 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sig, info, status = H.solve(f, tol=args.gmres_tol, restart=100, max_iter=3000,
                                refine=refine, inner_tol=args.inner_tol, method=spec["method"])
    solve_s = time.perf_counter() - t0
    if keep is not None:
        keep["y1"] = y1.double().cpu().numpy()
    tm = H.timings()
    H.free()
    return dict(setup_s=setup_s, st=st, ms=ms, ms16=ms16, msT=msT, kt=kt, solve_s=solve_s,
                gmres_iters=info.iters, gmres_ir_steps=info.ir_steps, gmres_status=int(status),
                gmres_rel_residual=info.rel_residual, timings=tm)


def summarize(spec, rs, y_ref, rows):
    prec, vec = spec["form"], spec["vec"]
    st = rs[-1]["st"]
    s_vec = 4 if vec == "f32" else 8
    s_acc = 8 if (prec == "f64" or vec == "f64") else 4
    B = mv_bytes(st, prec, s_vec)
    B16 = mv_bytes(st, prec, s_vec, 16)
    ms = float(np.median([m for r in rs for m in r["ms"]]))
    ms16 = float(np.median([m for r in rs for m in r["ms16"]]))
    msT = float(np.median([m for r in rs for m in r["msT"]]))
    p2 = [r["kt"]["fwd_panels"] for r in rs]
    p2_ms = sum(q["ms"] for q in p2) / max(1, sum(q["launches"] for q in p2))
    p2_B = phase2_bytes(st, prec, s_vec, s_acc)
    o = dict(
        eps=spec["eps"], vectors=vec, refine=spec["refine"],
        setup_s=float(np.median([r["setup_s"] for r in rs])),
        setup_phases_ms={k: round(v, 3) for k, v in rs[-1]["timings"].items()},
        matvec_ms=ms, matvec_gbs=B / ms / 1e6, matvec_bytes=B,
        matvec16_ms=ms16, matvec16_gbs=B16 / ms16 / 1e6,
        matvecT_ms=msT, matvecT_gbs=B / msT / 1e6,
        phase2_ms=p2_ms, phase2_bytes=p2_B, phase2_gbs=p2_B / p2_ms / 1e6,
        phase2_index_bytes=4 * st["n_panel_cols"],
        kernel_ms_per_launch={k: (v["ms"] / v["launches"] if v["launches"] else None)
                              for k, v in rs[-1]["kt"].items() if v["launches"]},
        gmres_iters=rs[-1]["gmres_iters"], gmres_ir_steps=rs[-1]["gmres_ir_steps"],
        gmres_s=float(np.median([r["solve_s"] for r in rs])),
        gmres_status=rs[-1]["gmres_status"],
        gmres_rel_residual=rs[-1]["gmres_rel_residual"],
        stats={k: st[k] for k in ("n_dense", "n_lr", "dense_entries", "lr_entries",
                                  "lr_u_entries", "rank_sum", "rank_max", "cap_hits",
                                  "stored_bytes", "aca_entry_evals", "device_bytes",
                                  "aca_chunks", "n_panel_cols")},
    )
    o["setup_plus_solve_s"] = o["setup_s"] + o["gmres_s"]
    if y_ref is not None and "y1" in rs[-1]:
        y1 = rs[-1]["y1"]
        o["rel_err_sampled"] = float(np.linalg.norm(y1[rows] - y_ref) / np.linalg.norm(y_ref))
    return o


def run_batch48(args):
    """48 seeded perturbed spheres (seed g, level 4 + g mod 3) in one handle
    (hm_build_batch, autotuned ACA binning and product schedule), FP32 form;
    one step =
    build, 8-column products, GMRES with 8 right-hand sides per geometry
    (graph-replayed Arnoldi steps), free."""
    import torch
    import paper_1806_11558_amd as hm
    from synthetic import normal_columns, perturbed_sphere
    eps = args.eps if args.eps is not None else 1e-5
    tol = args.gmres_tol
    meshes = [perturbed_sphere(4 + g % 3, seed=g) for g in range(48)]
    sizes = [t.shape[0] for _, t in meshes]
    n = int(sum(sizes))
    X = np.concatenate([normal_columns(k, 8, seed=1000 + g) for g, k in enumerate(sizes)])
    torch.cuda.set_device(0)
    xg = torch.tensor(X, device="cuda")

    def step():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H = hm.HMatrix.batch(meshes, leaf_size=args.leaf, eta=1.0, eps=eps, max_rank=64,
                             precision="f32", autotune=True)
        setup = time.perf_counter() - t0
        y = torch.empty_like(xg)
        H.matvec(xg, out=y)
        ms = _timed(torch, lambda: H.matvec(xg, out=y), max(3, args.reps // 4))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sig, info, status = H.solve(xg, tol=tol, restart=100, max_iter=3000, graph=True)
        solve = time.perf_counter() - t0
        st = H.stats()
        tune = H.tune_results().tolist()
        aca = (H.aca_bins()[:, 1].tolist(), H.aca_tune().tolist())
        H.free()
        return setup, ms, solve, info, int(status), st, tune, aca

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = [step() for _ in range(args.steps)]
    wall = time.perf_counter() - t0
    setup = float(np.median([r[0] for r in rs]))
    ms8 = float(np.median([m for r in rs for m in r[1]]))
    st = rs[-1][5]
    B = mv_bytes(st, "f32", 8, nrhs=8)
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
                               f"{eps:g}, FP32 form, autotuned ACA binning and product "
                               f"schedule; 8 "
                               f"right-hand sides N(0,1) seeds 1000 + g; graph GMRES to "
                               f"{tol:g}", "n": n, "nrhs": 8},
        "setup_s": round(setup, 4),
        "matvec8_ms": round(ms8, 4),
        "matvec8_bytes": B,
        "gmres_s": round(float(np.median([r[2] for r in rs])), 4),
        "gmres_iters": rs[-1][3].iters,
        "gmres_status": rs[-1][4],
        "gmres_rel_residual": rs[-1][3].rel_residual,
        "tune_unit_cols_ms": rs[-1][6],
        "aca_bins": {"edges": [64, 128, 256, 512, 1024, 2048, 4096, "inf"],
                     "class": [hm.ACA_CLASSES[c] for c in rs[-1][7][0]],
                     "tuned_bin_class_blocks_ms": rs[-1][7][1]},
        "stats": {k: st[k] for k in ("n_geom", "n_dense", "n_lr", "rank_max", "stored_bytes",
                                     "unit_cols", "aca_chunks")},
    }
    print(json.dumps(line), flush=True)


DEFAULT_EPS = {"f32": 1e-6, "f64": 1e-6, "f16": 1e-4}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--level", type=int, default=8, help="icosphere refinements (N = 20*4^L)")
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--eps", type=float, default=None,
                    help="ACA eps of every form (default: 1e-6 for f32 and f64, 1e-4 for f16)")
    ap.add_argument("--reps", type=int, default=20, help="timed 1-rhs products per form and step")
    ap.add_argument("--gmres-tol", type=float, default=1e-8)
    ap.add_argument("--inner-tol", type=float, default=1e-4,
                    help="inner GMRES tolerance of the refined solves")
    ap.add_argument("--cpu-rows", type=int, default=1024,
                    help="oracle rows the CPU leg computes and times")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="f32,f64,f16",
                    help="comma list of f32, f64, f16 (FP32 dense + FP16 factors); the first "
                         "is the timed form, the others are measured once after the steps")
    ap.add_argument("--vec", default="auto", choices=["auto", "f32", "f64"],
                    help="vector dtype of the products (auto: f32 for the f32 and f16 forms, "
                         "f64 for the f64 form)")
    ap.add_argument("--workload", default="single", choices=["single", "batch48"],
                    help="single: one icosphere (default); batch48: 48 perturbed spheres of "
                         "5,120 / 20,480 / 81,920 triangles in one handle, 8 right-hand sides")
    ap.add_argument("--operator", default="collocation", choices=["collocation", "galerkin"],
                    help="galerkin: the Galerkin matrix (HM_GALERKIN), solved by CG")
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
        if args.gmres_tol == 1e-8 and "--gmres-tol" not in sys.argv:
            args.gmres_tol = 1e-6
        run_batch48(args)
        return

    from synthetic import icosphere, mesh_sha256, normal_columns, sample_rows
    forms = args.forms.split(",")
    gal = args.operator == "galerkin"
    if gal and "--cpu-rows" not in sys.argv:
        args.cpu_rows = 256            # a Galerkin row costs about seven collocation rows
    specs = []
    for p in forms:
        vec = args.vec if args.vec != "auto" else ("f64" if p == "f64" else "f32")
        specs.append(dict(form=p, eps=args.eps if args.eps is not None else DEFAULT_EPS[p],
                          vec=vec, refine=p != "f64" and not gal,
                          method="cg" if gal else "gmres"))
    V, T = icosphere(args.level)
    n = T.shape[0]
    X = normal_columns(n, 16, seed=0)
    # the one-column product takes x = first column of four N(0,1) columns
    # from seed 0 (the vector of the stored oracle rows)
    x1 = normal_columns(n, 4, seed=0)[:, 0]
    # reference rows of A x1: the stored oracle rows (4,096) when they are for
    # this mesh, else the rows computed by the CPU leg below
    ref_rows, ref_y = None, None
    if os.path.exists(GOLDEN_L8) and not gal:
        g = np.load(GOLDEN_L8, allow_pickle=False)
        if str(g["mesh_sha256"]) == mesh_sha256(V, T) and int(g["x_seed"]) == 0:
            ref_rows, ref_y = g["rows"], g["y"][:, 0]
    rows = ref_rows[: args.cpu_rows] if ref_rows is not None else sample_rows(n, args.cpu_rows,
                                                                                seed=1)
    cpu = None
    if not args.no_cpu_baseline:
        workers = max(1, min(CPU_SHARE, len(os.sched_getaffinity(0))))
        print(f"# cpu leg: {rows.size} oracle rows at N={n} on {workers} processes",
              file=sys.stderr, flush=True)
        y_cpu, t_cpu = cpu_baseline(V, T, x1, rows, workers, args.operator)
        cpu = dict(t=t_cpu, workers=workers, rows=rows.size)
        print(f"# cpu leg: {t_cpu:.1f} s", file=sys.stderr, flush=True)
        if ref_rows is None:
            ref_rows, ref_y = rows, y_cpu
        else:
            # the live oracle rows reproduce the stored ones
            dev = float(np.abs(y_cpu - ref_y[: rows.size]).max() / np.abs(ref_y).max())
            cpu["stored_rows_max_rel_dev"] = dev
            if dev > 1e-12:
                print(f"bench.py: stored oracle rows disagree with the oracle ({dev:.2e})",
                      file=sys.stderr)
                sys.exit(1)

    import torch
    import paper_1806_11558_amd as hm
    torch.cuda.set_device(0)
    xd = torch.tensor(X, device="cuda")
    Xd = {"f64": xd, "f32": xd.float().contiguous()}
    x1d = torch.tensor(x1, device="cuda")
    X1d = {"f64": x1d, "f32": x1d.float()}
    f = torch.tensor(normal_columns(n, 1, seed=2)[:, 0], device="cuda")

    main_spec = specs[0]
    for k in range(args.warmup):
        r = run_form(hm, torch, V, T, args, main_spec, Xd, X1d, f, None)
        print(f"# warmup {k} {main_spec['form']}: setup {r['setup_s']:.3f} s, gmres "
              f"{r['gmres_iters']} it {r['solve_s']:.2f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = {main_spec["form"]: []}
    for k in range(args.steps):
        keep = {} if k == args.steps - 1 else None
        r = run_form(hm, torch, V, T, args, main_spec, Xd, X1d, f, keep)
        if keep:
            r.update(keep)
        res[main_spec["form"]].append(r)
        print(f"# step {k} {main_spec['form']}: setup {r['setup_s']:.3f} s, matvec "
              f"{np.median(r['ms']):.3f} ms, gmres {r['gmres_iters']} it {r['solve_s']:.2f} s",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    # the other forms: one warm-up pass and one measured pass each
    for spec in specs[1:]:
        hm.release_memory()
        run_form(hm, torch, V, T, args, spec, Xd, X1d, f, None)
        keep = {}
        r = run_form(hm, torch, V, T, args, spec, Xd, X1d, f, keep)
        r.update(keep)
        res[spec["form"]] = [r]
        print(f"# {spec['form']} (eps {spec['eps']:g}): setup {r['setup_s']:.3f} s, matvec "
              f"{np.median(r['ms']):.3f} ms, gmres {r['gmres_iters']} it {r['solve_s']:.2f} s",
              file=sys.stderr, flush=True)
        hm.release_memory()

    out = {}
    for spec in specs:
        out[spec["form"]] = summarize(spec, res[spec["form"]], ref_y, ref_rows)
    M = out[main_spec["form"]]
    mf = main_spec["form"]
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
        "dtype": mf,
        "data": "synthetic",
        "config": {"workload": f"unit icosphere L={args.level} (N={n}) Laplace single-layer "
                               f"{'Galerkin (piecewise constants), CG' if gal else 'collocation'}"
                               f", leaf {args.leaf}, eta 1; timed form {mf} at ACA eps "
                               f"{main_spec['eps']:g} with {main_spec['vec']} vectors; product x: "
                               f"N(0,1) seed 0; solve f: N(0,1) seed 2 to relative residual "
                               f"{args.gmres_tol:g}; error on "
                               f"{0 if ref_rows is None else ref_rows.size} exact oracle rows",
                   "n": n, "forms": {s["form"]: {"eps": s["eps"], "vectors": s["vec"],
                                                  "refine": s["refine"]} for s in specs}},
        "setup_s": {p: round(out[p]["setup_s"], 4) for p in out},
        "gmres_s": {p: round(out[p]["gmres_s"], 4) for p in out},
        "setup_plus_solve_s": {p: round(out[p]["setup_plus_solve_s"], 4) for p in out},
        "gmres_iters": {p: out[p]["gmres_iters"] for p in out},
        "gmres_rel_residual": {p: out[p]["gmres_rel_residual"] for p in out},
        "matvec_gbs": {p: round(out[p]["matvec_gbs"], 1) for p in out},
        "matvec_pct_hbm_peak": {p: round(100 * out[p]["matvec_gbs"] / HBM_PEAK_GBS, 1) for p in out},
        "rel_err_sampled": {p: out[p].get("rel_err_sampled") for p in out},
        "roofline": {
            "kernel": f"k_fwd2 + k_fwd2_sum (row-leaf panels: dense blocks + U slices), {mf} form, "
                      f"{main_spec['vec']} vectors",
            "bound": "hbm",
            "achieved": round(M["phase2_gbs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(M["phase2_gbs"] / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args.level, args.leaf, main_spec["eps"], mf,
                                        main_spec["vec"], args.operator),
        },
        "setup_roofline": {p: setup_roofline(out[p], p, args.operator) for p in out},
        "forms": out,
    }
    if cpu is not None:
        full_s = cpu["t"] * n / rows.size
        if "stored_rows_max_rel_dev" in cpu:
            line["stored_oracle_rows_max_rel_dev"] = cpu["stored_rows_max_rel_dev"]
        line["cpu_baseline"] = {
            "value": round(M["matvec_bytes"] / full_s / 1e9, 4),
            "unit": "GB/s",
            "cores": cpu["workers"],
            "kind": "oracle",
            "sample": f"{rows.size} exact rows of the dense product A x "
                      f"({'Galerkin oracle' if gal else '7-point rule'}, FP64) at "
                      f"N={n} in {cpu['t']:.2f} s on {cpu['workers']} processes; full product "
                      f"extrapolated x{n / rows.size:.0f} to {full_s:.1f} s; reported as the "
                      f"{mf} H-matvec's algorithmic bytes / that time",
        }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
