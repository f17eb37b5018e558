"""Throughput of the finite-volume PonD step on one MI355X.

Workload: the Mach-10 double Mach reflection on 1920 x 480 cells (D2Q16), the 2D
configuration the metric is quoted on. A step is one pass of the whole hot path over the
grid (dt reduction, face predictor-corrector, cell update + reframe). W untimed steps from
t = 0 are followed by K timed steps (defaults 100 + 1900 = the configuration's 2000 steps).

Reported: converged Mcell-updates/s (cells advanced in steps where all of their faces met
the iteration tolerance) of the headline form, mixed precision (FP32 populations, FP64
conserved variables); the plain FP64 form timed beside it; the relative L1 distance of the
mixed form from the FP64 form (the FP64 form matches the FP64 oracle to 1e-12); the face
kernel's roofline position; and the FP64 CPU oracle timed on this host on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "converged Mcell-updates/s at fixed L1 err vs FP64 oracle; learned+FP32 vs plain"

# Algorithmic floating-point operations of the face kernel, per face iteration and per
# face (finalization), as counted in the kernel's arithmetic (FMA = 2): transform of the 8
# (2D) or 4 (1D) stencil cells into the face frame, population evaluation, limited MUSCL
# reconstruction, moments and frame update. 2D, per iteration: 8 stencil cells x (frame
# offsets 5 + f transform 49 + g transform 27, on factorial-scaled coefficients); populations
# of L and R in full (f 86, g 56) and of the 6 side cells in the 2 node columns each feeds
# (f 52, g 32); 32 limited populations x 16 + 60 shared; moments of f (108) and g (80);
# frame update 40.
FLOPS_FACE_ITER = {1: 330, 2: 2236}
# With the alternative regularization (--regularization eq) each iteration also sets the six
# fast f coefficients of the 8 stencil cells (43 flops each) and evaluates 16 f coefficients
# instead of 10 (L and R in full: 112 instead of 86; side cells, 2 columns: 76 instead of 52):
# 2,236 + 344 + 52 + 144 = 2,776.
FLOPS_FACE_ITER_EQ2 = 2776
FLOPS_FACE_FINAL = {1: 60, 2: 330}
# FP64 / FP32 vector peaks of MI355X (no packed FP32 instructions are used: FP32 issues at
# the FP64 rate, so both peaks are the 78.6 TFLOP/s non-packed figure)
PEAK_VALU_TFLOPS = 78.6
PEAK_HBM_GBPS = 8000.0
# Algorithmic bytes of one 2D cell update (read U, coefficients and the cell's share of its
# 4 face states, write U and coefficients), mixed / FP64
CELL_BYTES_2D = {"mixed": 312, "fp64": 560}


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "double_mach_1920x480_face_traffic.md")
KERNEL_SOURCES = ("pond_core.hpp", "pond_kernels.hpp", "pond_mlp.hpp", "pond.hip")


def measured_traffic(tiles):
    """HBM bytes per face-kernel launch at the given (BX, BY) tile from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a known-size copy; one record per tile the
    autotuner picks), or None without a record for that tile or once the kernel sources
    have changed since those counters were taken."""
    import hashlib

    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    recs = [json.loads(line.split(":", 1)[1]) for line in open(TRAFFIC_PROFILE)
            if line.startswith("traffic-json:")]
    rec = next((r for r in recs if list(r["tiles"]) == list(tiles)), None)
    if rec is None:
        return None
    csrc = os.path.join(ROOT, "paper_2203_05477_amd", "csrc")
    h = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read() for f in KERNEL_SOURCES))
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec


def cell_update_hbm(st, kt, steps, precision):
    fused = kt["tail"] > 0.01  # the tail launch (else only event overhead sits there)
    ms = kt["cell"] + (kt["tail"] if fused else 0.0)
    alg = CELL_BYTES_2D[precision] * st["cell_updates"] / steps
    gbps = alg / (ms * 1e-3) / 1e9 if ms > 0 else None
    return {"bound": "hbm", "kernels": "tail_cell_kernel_2d + cell_marked_kernel_2d"
            if fused else "cell_kernel<2>", "ms": ms, "algorithmic_bytes": alg,
            "achieved": gbps, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": gbps / PEAK_HBM_GBPS if gbps else None}


def run_form(cfg, fields, precision, warmup, steps, seed="prev", autotune=True, tiles=None, mlp=None,
             iter_split=None):
    from paper_2203_05477_amd import pond

    ctx = pond.Context(cfg, fields, precision=precision, seed=seed)
    if iter_split is not None:
        ctx.set_iter_split(iter_split)
    if mlp is not None:
        ctx.load_mlp(mlp, hard_iters=2)
    if warmup:
        ctx.step(warmup)
    if tiles:
        ctx.set_tiles(tiles[0], tiles[1], 256)
    elif autotune:
        ctx.autotune()
    ctx.enable_timing(True)
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = ctx.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = ctx.kernel_times()
    return ctx, st, t1 - t0, kt


def cpu_baseline(cfg, fields, budget_s=15.0, max_steps=20):
    """The FP64 oracle on this host's cores, first steps of the same workload."""
    import oracle

    sim = oracle.Sim(cfg, fields["rho"], fields["ux"], fields.get("uy"), fields["p"])
    n = cfg["nx"] * cfg["ny"]
    t0 = time.perf_counter()
    steps, conv = 0, 0
    while steps < max_steps:
        sim.step()
        steps += 1
        if sim.last["nonconverged"] == 0:
            conv += n
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": n * steps / el / 1e6, "unit": "Mcell-updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"first {steps} steps of the {cfg['nx']}x{cfg['ny']} double Mach reflection "
                      f"from t=0 (FP64, plain seed, tol {cfg['tol']:g}); {el:.1f} s"}


def other_workload(args):
    """The other workloads, mixed and FP64 forms (plain seed), same JSON line: the shocked
    interface (2048 x 512), the Mach-80 jet (2048 x 2048; it fails within tens of steps, so
    the default run is short and a failure is reported), or the batch of 4096 shock tubes."""
    import oracle
    from paper_2203_05477_amd import pond
    from paper_2203_05477_amd import workloads as W

    pond.load()
    name = args.workload
    if name == "shocked_interface":
        make = lambda tol: W.shocked_interface(tol=tol)
    elif name == "jet":
        make = lambda tol: W.jet(tol=tol)
    elif name == "explosion_box":
        make = lambda tol: W.explosion_box(tol=tol)
    else:
        make = lambda tol: W.tube_batch(tol=tol)
    out = {}
    for prec, tol in (("mixed", W.TOL_FP32), ("fp64", W.TOL_FP64)):
        cfg, fields = make(tol)
        cfg["scheme"] = args.scheme
        ctx = pond.Context(cfg, fields, precision=prec)
        if args.warmup:
            ctx.step(args.warmup, check=False)
        ctx.autotune()
        ctx.enable_timing(True)
        import torch

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.step(args.steps, check=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        kt = ctx.kernel_times()
        out[prec] = {"value": st["converged_cell_updates"] / el / 1e6, "ms_per_step": 1e3 * el / args.steps,
                     "cell_updates": st["cell_updates"], "mean_iters": st["iters_total"] / max(st["faces"], 1),
                     "failed_instances": st["failed_instances"], "status": st["status"],
                     "kernel_ms": {"dt": kt["dt"], "face": kt["face"], "tail_with_cells": kt["tail"],
                                   "cell": kt["cell"]}, "tiles": list(ctx.tiles())}
        ctx.close()
        if name == "tubes" and args.scheme == "fv":
            # the same steps with the resident kernel (one block per tube, every step in one
            # launch; the same bits), without per-kernel timing
            ctx = pond.Context(cfg, fields, precision=prec)
            if args.warmup:
                ctx.step(args.warmup, check=False)
            ctx.set_resident(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = ctx.step(args.steps, check=False)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            out[prec]["resident"] = {"value": st["converged_cell_updates"] / el / 1e6,
                                     "ms_per_step": 1e3 * el / args.steps}
            ctx.close()
    cpu = None
    if not args.no_cpu_baseline:
        if name == "tubes":
            cfg, fields = make(W.TOL_FP64)
            cfg["scheme"] = args.scheme
            t0 = time.perf_counter()
            cells, k = 0, 0
            while time.perf_counter() - t0 < 15.0 and k < len(cfg["lengths"]):
                c = dict(W.tube_config(cfg, k), scheme=args.scheme)
                ff = W.tube_fields(cfg, fields, k)
                sim = oracle.Sim(c, ff["rho"], ff["ux"], None, ff["p"])
                for _ in range(16):
                    sim.step()
                cells += 16 * c["nx"]
                k += 1
            el = time.perf_counter() - t0
            cpu = {"value": cells / el / 1e6, "unit": "Mcell-updates/s", "cores": oracle.num_threads(),
                   "kind": "oracle", "sample": f"tubes 0..{k - 1} of the batch, 16 steps each (FP64); {el:.1f} s"}
        else:
            cfg, fields = make(W.TOL_FP64)
            sim = oracle.Sim(cfg, fields["rho"], fields["ux"], fields["uy"], fields["p"])
            t0 = time.perf_counter()
            steps = 0
            while steps < 10 and time.perf_counter() - t0 < 15.0:
                sim.step()
                steps += 1
            el = time.perf_counter() - t0
            n = cfg["nx"] * cfg["ny"]
            cpu = {"value": n * steps / el / 1e6, "unit": "Mcell-updates/s", "cores": oracle.num_threads(),
                   "kind": "oracle", "sample": f"first {steps} steps from t=0 (FP64); {el:.1f} s"}
    m = out["mixed"]
    best = m
    if "resident" in m and m["resident"]["value"] > m["value"]:
        best = m["resident"]
    line = {
        "metric": METRIC, "value": best["value"], "unit": "Mcell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": best["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": {"shocked_interface": "shocked_interface_2048x512", "jet": "jet_2048x2048",
                                "tubes": "tube_batch_4096", "explosion_box": "explosion_box_256x256"}[name],
                   "scheme": args.scheme,
                   "precision": "mixed (f32 populations, f64 conserved)", "seed": "plain"},
        "roofline": None, "mixed": m, "fp64_plain": out["fp64"], "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def launch_mode(ctx, mode):
    """graph: autotuned tiles, launches replayed from a captured graph; resident: every
    step of a call in one launch, one block per tube (1D)."""
    if mode == "resident":
        ctx.set_resident(True)
    else:
        ctx.autotune()
        ctx.set_graph(True)


def riemann_workload(args):
    """The printed 1D Riemann problems (Lax, strong shock tube, double rarefaction, Le Blanc,
    1D jet) at the paper's resolutions, each run from t = 0 to its printed final time in
    the mixed and FP64 forms, with the relative L1 error of every conserved field against
    the exact Riemann solution. A first, untimed run counts the steps to the final time
    and times 200 steps in each of the two launch modes, which give the same bits:
    launches replayed from a captured graph, or the resident kernel (every step in one
    launch, one block per tube); the timed run then issues all the steps in one pond_step
    call on a fresh context in the faster mode. A case that fails (the double rarefaction
    opens a true vacuum) is reported with the step it failed in and left out of the
    totals. These grids hold 600-4,000 cells: a step is bound by the latency of the
    slowest face's iterations and of the launches, not by the GPU's throughput."""
    import oracle
    import torch

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import exact_riemann as ER
    from paper_2203_05477_amd import pond
    from paper_2203_05477_amd import workloads as W

    pond.load()
    cases, tot = {}, {"mixed": [0, 0.0], "fp64": [0, 0.0]}
    for name, case in W.RIEMANN_CASES.items():
        left, right, xi, (a, b), gamma, t_end, nx = case[:7]
        cases[name] = {"cells": nx, "t_end": t_end}
        for prec, tol in (("mixed", W.TOL_FP32), ("fp64", W.TOL_FP64)):
            cfg, fields = W.riemann_case(name, tol=tol)
            cfg["scheme"] = args.scheme
            ctx = pond.Context(cfg, fields, precision=prec)
            n, status = 0, pond.OK
            while ctx.time()[0] < t_end * (1 - 1e-12) and status == pond.OK:
                status = ctx.step(1, t_end, check=False)["status"]
                n += 1
            ctx.close()
            r = {"steps": n, "status": status}
            if status != pond.OK:
                r["failed_at_step"] = n
                cases[name][prec] = r
                continue
            trial = {}
            for mode in ("graph", "resident") if args.scheme == "fv" else ("graph",):
                ctx = pond.Context(cfg, fields, precision=prec)
                launch_mode(ctx, mode)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.step(min(n, 200), t_end, check=False)
                torch.cuda.synchronize()
                trial[mode] = time.perf_counter() - t0
                ctx.close()
            r["launch_mode"] = min(trial, key=trial.get)
            ctx = pond.Context(cfg, fields, precision=prec)
            launch_mode(ctx, r["launch_mode"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = ctx.step(n, t_end, check=False)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            ex = ER.cell_average(left, right, gamma, np.linspace(a, b, nx + 1), xi, ctx.time()[0])
            U = ctx.conserved()
            r.update({"status": st["status"], "ms": 1e3 * el, "ms_per_step": 1e3 * el / n,
                      "converged_cell_updates": st["converged_cell_updates"],
                      "fallback_faces": st["fallback"],
                      "rel_l1_vs_exact": {k: float(np.abs(U[q] - ex[q]).sum() / np.abs(ex[q]).sum())
                                          for q, k in enumerate(("rho", "rho_u", "rho_E"))}})
            ctx.close()
            cases[name][prec] = r
            tot[prec][0] += st["converged_cell_updates"]
            tot[prec][1] += el
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on the first 500 steps of each case (all of them would take minutes:
        # Le Blanc alone needs about 19,500 steps of 4,000 cells)
        cells, el = 0, 0.0
        for name in W.RIEMANN_CASES:
            cfg, fields = W.riemann_case(name, tol=W.TOL_FP64)
            cfg["scheme"] = args.scheme
            sim = oracle.Sim(cfg, fields["rho"], fields["ux"], None, fields["p"])
            t0 = time.perf_counter()
            k = 0
            while k < 500 and sim.t < cfg["t_end"] * (1 - 1e-12):
                sim.step(cfg["t_end"])
                k += 1
            el += time.perf_counter() - t0
            cells += k * cfg["nx"]
        cpu = {"value": cells / el / 1e6, "unit": "Mcell-updates/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"first 500 steps of each of the five cases from t=0 (FP64); {el:.1f} s"}
    m = tot["mixed"]
    line = {
        "metric": METRIC, "value": m[0] / m[1] / 1e6, "unit": "Mcell-updates/s", "n_gpus": 1,
        "steps": sum(c["mixed"]["steps"] for c in cases.values() if "ms" in c["mixed"]),
        "warmup": 0, "ms_per_step": 1e3 * m[1] / max(1, sum(c["mixed"]["steps"] for c in cases.values()
                                                           if "ms" in c["mixed"])),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "riemann_1d_printed_problems", "lattice": "D1Q4", "scheme": args.scheme,
                   "precision": "mixed (f32 populations, f64 conserved)", "seed": "plain",
                   "cfl": 0.2},
        "roofline": None, "fp64_plain": {"value": tot["fp64"][0] / tot["fp64"][1] / 1e6},
        "cases": cases, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1900)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--nx", type=int, default=1920)
    ap.add_argument("--ny", type=int, default=480)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-seed form")
    ap.add_argument("--tiles", type=str, default=None,
                    help="face tile BXxBY for both forms instead of the autotuner's choice")
    ap.add_argument("--workload", default="double_mach",
                    choices=["double_mach", "shocked_interface", "jet", "tubes", "riemann_1d",
                             "explosion_box"],
                    help="the benchmark's workload (default: the headline double Mach reflection)")
    ap.add_argument("--scheme", choices=["fv", "sl"], default="fv",
                    help="1D workloads (tubes, riemann_1d): the finite-volume scheme or the "
                         "semi-Lagrangian realization (Sec. III.A)")
    ap.add_argument("--regularization", choices=["grad", "eq"], default="grad",
                    help="transformation of the f populations between frames: third-order Grad "
                         "projection (the paper's choice) or the alternative with the fast moments "
                         "at equilibrium (Sec. II.C)")
    ap.add_argument("--iter-split", type=int, default=None,
                    help="face iterations per face in the face kernel before the tail kernel takes "
                         "over (0: no tail kernel, the cell update is one kernel)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (the known-size "
                         "kernel that scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the PonD step is built and timed on a single MI355X; "
              "multi-GPU runs are not supported by this implementation",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = 1 << 28  # 2^28 floats = 1 GiB read + 1 GiB written per copy
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 5}))
        return
    if args.scheme == "sl" and args.workload not in ("tubes", "riemann_1d"):
        print("the semi-Lagrangian scheme is built in 1D only (--workload tubes or riemann_1d)",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "riemann_1d":
        riemann_workload(args)
        return
    if args.workload != "double_mach":
        other_workload(args)
        return
    from paper_2203_05477_amd import pond
    from paper_2203_05477_amd import workloads as W

    pond.load()
    tol32, tol64 = W.TOL_FP32, W.TOL_FP64
    cfg32, fields = W.double_mach(args.nx, args.ny, tol=tol32)
    cfg64, _ = W.double_mach(args.nx, args.ny, tol=tol64)
    cfg32["regularization"] = cfg64["regularization"] = args.regularization
    ncell = args.nx * args.ny

    tiles = tuple(int(v) for v in args.tiles.split("x")) if args.tiles else None
    ctx32, st32, el32, kt32 = run_form(cfg32, fields, "mixed", args.warmup, args.steps,
                                       autotune=not args.no_autotune, tiles=tiles,
                                       iter_split=args.iter_split)
    # learned seed + FP32: a network trained on the GPU on face frames the solver itself
    # produced (first 300 steps of the same problem on a 4x coarser grid), then the same
    # timed run with the network seeding the faces that needed two or more iterations
    learned, Ul = None, None
    if not args.no_learned:
        from paper_2203_05477_amd import learned_seed as LS

        t0 = time.perf_counter()
        cfgh, fh = W.double_mach(args.nx // 4, args.ny // 4, tol=tol32)
        cfgh["regularization"] = args.regularization
        data = LS.harvest(cfgh, fh, steps=300, precision="mixed", hard_iters=2, every=2)
        net, losses, nsamp = LS.train([data], epochs=20, batch=4096, lr=2e-3)
        t_train = time.perf_counter() - t0
        ctxl, stl, ell, ktl = run_form(cfg32, fields, "mixed", args.warmup, args.steps,
                                       autotune=not args.no_autotune, tiles=tiles, seed="mlp", mlp=net)
        Ul = ctxl.conserved()
        learned = {
            "value": stl["converged_cell_updates"] / ell / 1e6,
            "ms_per_step": 1e3 * ell / args.steps,
            "mean_iters": stl["iters_total"] / max(stl["faces"], 1),
            "nonconverged_faces": stl["nonconverged"],
            "kernel_ms": {"seed": ktl["seed"], "face": ktl["face"], "tail_with_cells": ktl["tail"],
                          "cell": ktl["cell"]},
            "train": {"samples": nsamp, "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
                      "seconds": t_train},
        }
        ctxl.close()

    rec = {}
    if not args.no_fp64:
        ctx64, st64, el64, kt64 = run_form(cfg64, fields, "fp64", args.warmup, args.steps,
                                           autotune=not args.no_autotune, tiles=tiles,
                                           iter_split=args.iter_split)
        U32, U64 = ctx32.conserved(), ctx64.conserved()
        l1 = [float(np.abs(U32[k] - U64[k]).sum() / np.abs(U64[k]).sum()) for k in range(4)]
        if learned is not None:
            learned["rel_l1_vs_fp64"] = {q: float(np.abs(Ul[k] - U64[k]).sum() / np.abs(U64[k]).sum())
                                         for k, q in enumerate(("rho", "rho_u", "rho_v", "rho_E"))}
        rec["fp64_plain"] = {
            "value": st64["converged_cell_updates"] / el64 / 1e6,
            "ms_per_step": 1e3 * el64 / args.steps,
            "mean_iters": st64["iters_total"] / max(st64["faces"], 1),
            "kernel_ms": {"dt": kt64["dt"], "face": kt64["face"], "tail_with_cells": kt64["tail"],
                          "cell": kt64["cell"]},
            "cell_update_hbm": cell_update_hbm(st64, kt64, args.steps, "fp64"),
            "tiles": list(ctx64.tiles()),
        }
        rec["mixed_rel_l1_vs_fp64"] = {"rho": l1[0], "rho_u": l1[1], "rho_v": l1[2], "rho_E": l1[3]}
        ctx64.close()

    value = st32["converged_cell_updates"] / el32 / 1e6
    iters_per_face = st32["iters_total"] / max(st32["faces"], 1)
    # the face kernel proper (the tail kernel's share of faces and iterations taken out)
    main_iters = (st32["iters_total"] - st32["tail_iters"]) / args.steps
    main_finals = (st32["faces"] - st32["tail_faces"]) / args.steps
    it_flops = FLOPS_FACE_ITER_EQ2 if args.regularization == "eq" else FLOPS_FACE_ITER[2]
    face_flops = main_iters * it_flops + main_finals * FLOPS_FACE_FINAL[2]
    face_main_ms = kt32["face"]
    # the counter summary covers the Grad kernel only
    traffic = measured_traffic(list(ctx32.tiles())[:2]) if args.regularization == "grad" else None
    achieved = face_flops / (face_main_ms * 1e-3) / 1e12
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"double_mach_reflection_{args.nx}x{args.ny}", "lattice": "D2Q16",
                   "precision": "mixed (f32 populations, f64 conserved)", "seed": "plain",
                   "tol": tol32, "cfl": cfg32["cfl"], "mu": cfg32["mu"],
                   "regularization": args.regularization,
                   "steps_from_t0": args.warmup + args.steps},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_VALU_TFLOPS,
                     "traffic": traffic["bytes_per_launch"] if traffic else None,
                     "traffic_unit": "B per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE)",
                     "traffic_tiles": traffic["tiles"] if traffic else None,
                     "kernel": "face_kernel_2d<float, 0>" + (" (regularization eq)" if args.regularization == "eq" else ""), "kernel_ms": face_main_ms,
                     "flop_per_launch": face_flops},
        "cell_updates": st32["cell_updates"],
        "converged_fraction": st32["converged_cell_updates"] / max(st32["cell_updates"], 1),
        "mean_iters_per_face": iters_per_face,
        "fallback_faces": st32["fallback"],
        "nonconverged_faces": st32["nonconverged"],
        # face: the face kernel; tail_with_cells: the launch that finishes the deferred faces
        # and updates every cell; cell: a separate cell update (none in 2D with a tail)
        "kernel_ms": {"dt": kt32["dt"], "face": face_main_ms, "tail_with_cells": kt32["tail"],
                      "cell": kt32["cell"]},
        "tail_faces_per_step": st32["tail_faces"] / args.steps,
        # the cell update (reframe + flux + collision) against HBM: algorithmic bytes of the
        # cells updated per step over the launches that update them; with a tail kernel the
        # first of those launches also finishes the tail's faces (run --iter-split 0 for the
        # cell update kernel alone)
        "cell_update_hbm": cell_update_hbm(st32, kt32, args.steps, "mixed"),
        "tiles": list(ctx32.tiles()),
        "t_end": st32["t_max"],
    }
    line.update(rec)
    if learned is not None:
        line["learned_mixed"] = learned
    ctx32.close()
    if not args.no_cpu_baseline:
        cfgc, fc = W.double_mach(args.nx, args.ny, tol=tol64)
        cfgc["regularization"] = args.regularization
        line["cpu_baseline"] = cpu_baseline(cfgc, fc)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
