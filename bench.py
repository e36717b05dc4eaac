"""Benchmark of the corrector hot path on one MI355X.

A step is one pass of the hot path over the workload: GPU assembly of the
corrector matrices from the per-cell fields, then a Jacobi-PCG solve of each
to a true relative residual of 1e-10.  `value` is corrector solves per second
in float64 (whole job, one GPU); the same step in mixed precision, the
roofline of the dominant iteration kernel and the CPU oracle on a bounded
sample are reported beside it.  Inputs are seeded and synthetic (synth/) and
resident in HBM before timing starts.

Workloads (--workload)
  channel        4x1 channel with a porous block, ~1.0M triangles refined 4x
                 near the block, isotropic K; CP1x and CP2 per step (default)
  channel_aniso  the same recipe at ~4.0M triangles with anisotropic K (ratio
                 100 rotated 30 deg); CP2 per step; also reports the two-solve
                 CP2 sequence (cross terms of the first solution on the second
                 right-hand side) and its cross-term kernels, and the coupled
                 CP1 solved by the paper's loop over the x and y systems
  square         unit square 64x64 jittered grid (~8k triangles); CP2
  batch          64 unit squares of 50k-500k triangles with log-normal K;
                 one batched CP2 solve per step
  adjoint        channel forward CP2 solve + adjoint solve + gradient kernel

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "corrector PCG solves/s + SpMV HBM GB/s, mixed vs FP64 at 1e-10 residual"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def iter_summary(infos):
    its = [i["iters"] for i in infos]
    return its if len(its) <= 4 else {"min": min(its), "max": max(its), "sum": sum(its)}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def source_digest() -> str:
    """Digest of the kernel sources with comments and blank lines removed, to
    tell whether stored counter readings still describe the kernels in this
    tree (editing a comment does not change a kernel)."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in ("solver.hip", "kernels.h", "solver.h"):
        with open(os.path.join(ROOT, "paper_2309_03543_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        code = [ln.split("//", 1)[0].rstrip() for ln in text.splitlines()]
        h.update("\n".join(ln for ln in code if ln.strip()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, launch: dict, kernel: str):
    """HBM bytes per launch of the dominant kernel, for this launch shape, from
    the stored counter summary (FETCH_SIZE + WRITE_SIZE calibrated on a plain
    copy), or None when the summary lacks this shape or the kernels changed
    since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    digest, found = None, None
    with open(path) as fh:
        for line in fh:
            if line.startswith("source_digest:"):
                digest = line.split(":", 1)[1].strip()
            elif line.startswith("shape:"):
                f = line.split(":", 1)[1].split()
                # shape: <kernel> <iter_shape> <tile_rows> <block> <bytes per launch> ...
                if (f[0] == kernel and int(f[1]) == launch["iter_shape"]
                        and int(f[2]) == launch["tile_rows"] and int(f[3]) == launch["block"]):
                    found = float(f[4])
    if digest != source_digest():
        return None
    return found


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="channel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--solve-reps", type=int, default=10,
                    help="repeated float64 solves for the solve-only median (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, run a plain device copy of 256 MiB five times, whose "
                         "known traffic calibrates the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this corrector library is a single-GPU build and "
              "its multi-GPU sharding is a design note only; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2309_03543_amd import binding as B
    from synth import workloads

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    wl = args.workload
    t0 = time.time()
    if wl == "batch":
        ws = workloads.lognormal_batch(workers=min(16, len(os.sched_getaffinity(0))))
        wname = "lognormal_batch_64x50k-500k"
    elif wl == "channel_aniso":
        ws = [workloads.channel(552, 3, aniso=True)]
        wname = "channel_aniso_4M"
    elif wl == "square":
        ws = [workloads.square_inclusion()]
        wname = "square_inclusion_8k"
    elif wl in ("channel", "adjoint"):
        ws = [workloads.channel(276, 2)]
        wname = "channel_1M" if wl == "channel" else "channel_1M_adjoint"
    else:
        raise SystemExit(f"unknown workload {wl}")
    log(f"workload {wname}: {sum(w['mesh']['tri'].shape[0] for w in ws)} cells, "
        f"generated in {time.time() - t0:.1f}s")
    t0 = time.time()
    meshes = [B.Mesh(w["mesh"]["xy"], w["mesh"]["tri"], w["side_tag"]) for w in ws]
    prms = [{k: torch.tensor(v, device=dev) for k, v in w["params"].items()} for w in ws]
    n_cells = sum(m.n for m in meshes)
    nnz = sum(m.nnz for m in meshes)
    log(f"meshes ready in {time.time() - t0:.1f}s: n={n_cells} nnz={nnz} "
        f"maxT={max(m.stats['max_T'] for m in meshes):.3g} idx={meshes[0].stats['index_bits']}b")

    kinds = {"channel": [("cp1x", B.PM_CP1X), ("cp2", B.PM_CP2)]}.get(wl, [("cp2", B.PM_CP2)])
    rhs = [{k: torch.tensor(w["rhs"][k], device=dev) for k, _ in kinds} for w in ws]
    batch = B.Batch(meshes) if wl == "batch" else None
    w0, mesh0, prm0 = ws[0], meshes[0], prms[0]
    probes = torch.tensor(np.random.default_rng(5).choice(n_cells, 256, replace=False), device=dev)

    def step(precision):
        infos = []
        if wl == "batch":
            vals = [B.assemble_corrector(m, B.PM_CP2, p, w["nu"], w["dt"])["val64"]
                    for m, p, w in zip(meshes, prms, ws)]
            b = torch.cat([r["cp2"] for r in rhs])
            x, inf = B.pcg_solve_batched(batch, torch.cat(vals), b, precision=precision)
            bad = [i for i in inf if i["status"] != 0]
            if bad:
                raise RuntimeError(f"batched solve failed: {bad[0]}")
            return inf
        for key, kind in kinds:
            val = B.assemble_corrector(mesh0, kind, prm0, w0["nu"], w0["dt"])["val64"]
            x, info = B.pcg_solve(mesh0, val, rhs[0][key], precision=precision)
            if info["status"] != 0:
                raise RuntimeError(f"solve {key} failed: {info}")
            infos.append(info)
            if wl == "adjoint":
                g = torch.zeros_like(x)
                g[probes] = 2.0 * x[probes]
                lam, gs, ge, ia = B.pcg_adjoint(mesh0, kind, prm0, w0["nu"], w0["dt"], val, x, g,
                                                precision=precision)
                if ia["status"] != 0:
                    raise RuntimeError(f"adjoint solve failed: {ia}")
                infos.append(ia)
        return infos

    def timed(precision):
        for _ in range(args.warmup):
            step(precision)
        torch.cuda.synchronize()
        t = time.perf_counter()
        infos = []
        for k in range(args.steps):
            infos.append(step(precision))
            its = [i["iters"] for i in infos[-1]]
            log(f"  step {k + 1}/{args.steps} precision={precision} iters={its if len(its) < 8 else (min(its), max(its))} "
                f"max_res={max(i['rel_res_true'] for i in infos[-1]):.2e}")
        torch.cuda.synchronize()
        return time.perf_counter() - t, infos

    log("timing float64 steps")
    wall64, inf64 = timed(0)
    solves_per_step = len(inf64[-1])
    value = solves_per_step * args.steps / wall64
    # solve alone (assembly excluded): median of repeated float64 solves of
    # the step's last system, timed with HIP events on the current stream
    solve_only = None
    if batch is None and wl != "adjoint" and args.solve_reps > 0:
        key, kind = kinds[-1]
        val = B.assemble_corrector(mesh0, kind, prm0, w0["nu"], w0["dt"])["val64"]
        times = []
        for _ in range(args.solve_reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            _, info = B.pcg_solve(mesh0, val, rhs[0][key])
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        med = float(np.median(times))
        solve_only = {"system": key, "ms_median": med, "solves_per_s": 1e3 / med,
                      "iters": info["iters"], "reps": len(times)}
        # the same solve with the Chebyshev-polynomial preconditioner (degree
        # 6), float64 and mixed: fewer, costlier iterations
        cheb = {}
        for prec in (0, 1):
            B.pcg_solve(mesh0, val, rhs[0][key], precision=prec, precond=1, cheb_degree=6)
            times = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                _, ic = B.pcg_solve(mesh0, val, rhs[0][key], precision=prec, precond=1,
                                    cheb_degree=6)
                e1.record()
                e1.synchronize()
                times.append(e0.elapsed_time(e1))
            cheb["f64" if prec == 0 else "mixed"] = {
                "ms_median": float(np.median(times)), "iters": ic["iters"],
                "rel_res_true": ic["rel_res_true"], "status": ic["status"]}
        solve_only["chebyshev_degree6"] = cheb
        if wl == "channel":
            # both CP1 components: two scalar solves against one coupled CG
            # whose coupling is zero here (isotropic K): a two-right-hand-side
            # solve that reads the shared weights once
            vx = B.assemble_corrector(mesh0, B.PM_CP1X, prm0, w0["nu"], w0["dt"])["val64"]
            vy = B.assemble_corrector(mesh0, B.PM_CP1Y, prm0, w0["nu"], w0["dt"])["val64"]
            bx = rhs[0]["cp1x"]
            by = torch.tensor(w0["rhs"]["cp1y"], device=dev)
            B.pcg_solve(mesh0, vy, by)
            B.cp1_solve_coupled_pcg(mesh0, prm0, w0["nu"], w0["dt"], vx, vy, bx, by)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, i_x = B.pcg_solve(mesh0, vx, bx)
            _, i_y = B.pcg_solve(mesh0, vy, by)
            torch.cuda.synchronize()
            t_two = time.perf_counter() - t
            t = time.perf_counter()
            _, _, i_c = B.cp1_solve_coupled_pcg(mesh0, prm0, w0["nu"], w0["dt"], vx, vy, bx, by)
            torch.cuda.synchronize()
            t_pair = time.perf_counter() - t
            solve_only["cp1_pair"] = {"two_scalar_ms": t_two * 1e3,
                                      "two_scalar_iters": [i_x["iters"], i_y["iters"]],
                                      "one_coupled_cg_ms": t_pair * 1e3,
                                      "one_coupled_cg_iters": i_c["iters"],
                                      "coupled_rel_res_true": i_c["rel_res_true"]}
            log(f"  CP1 x and y: two scalar solves {t_two * 1e3:.1f} ms, one coupled CG "
                f"{t_pair * 1e3:.1f} ms ({i_c['iters']} it)")
        B.pcg_solve(mesh0, val, rhs[0][key])  # the kernel timing below uses the last solve's state
        log(f"  {key} solve: Jacobi {med:.1f} ms ({info['iters']} it); Chebyshev-6 "
            f"{cheb['f64']['ms_median']:.1f} ms ({cheb['f64']['iters']} it), mixed "
            f"{cheb['mixed']['ms_median']:.1f} ms")
    # per-kernel timing on the state of the last solve of the step
    tmesh = mesh0 if batch is None else None
    kern = {}
    if tmesh is not None:
        launch = B.pm_last_launch(tmesh)
        fused = launch["iter_shape"] > 0
        resident = launch["iter_shape"] in (4, 5)
        it_name = ({4: "k_chunk", 5: "k_chunk_win"}.get(launch["iter_shape"])
                   or ("k_iter" if fused else "k_update+k_spmv"))
        # the resident kernel runs a chunk's m - 1 = 49 iterations per launch
        per_launch = 49 if resident else 1
        for name, which, reps in (("k_spmv", 0, 200), (it_name, 1, 8 if resident else 200),
                                  ("k_resid", 2, 20)):
            ms, by = B.pm_time_kernel(tmesh, which, reps)
            k = per_launch if name == it_name else 1
            kern[name] = {"ms": ms * k, "bytes": by * k, "GBs": by / ms / 1e6,
                          "frac_hbm": by / ms / 1e6 / HBM_PEAK_GBS}
            if k > 1:
                kern[name]["iterations_per_launch"] = k
        kern["launch"] = launch
        it_last = inf64[-1][-1]["iters"]
        # fused: one k_iter launch per iteration (k_spmv opens each chunk of 50);
        # resident: one k_chunk launch per chunk; split: k_spmv is the larger of
        # the iteration's two kernels
        dom = it_name if fused else "k_spmv"
        achieved = kern[dom]["GBs"]
        roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic(wname, launch, dom),
                "ms_per_launch": kern[dom]["ms"], "bytes_per_launch": kern[dom]["bytes"],
                "launches_per_solve": -(-it_last // 50) if resident else it_last}
        if resident:
            roof["note"] = ("achieved = the iterations' algorithmic bytes (what a streaming "
                            "iteration moves) over the launch time; the resident kernel keeps "
                            "its tiles on chip, so traffic is the bytes it actually moves")
            # the streaming form of the same iteration (LDS-staged fused kernel,
            # same tiles), which is bound by HBM: its fraction of the roofline
            sl = {"tile_rows": launch["tile_rows"], "block": launch["block"], "iter_shape": 3}
            v2 = B.assemble_corrector(tmesh, B.PM_CP2, prm0, w0["nu"], w0["dt"])["val64"]
            B.pcg_solve(tmesh, v2, rhs[0]["cp2"], **sl)
            ms_s, by_s = B.pm_time_kernel(tmesh, 1, 200)
            roof["streaming_kernel"] = {
                "kernel": "k_iter_lds", "launch": sl, "ms_per_launch": ms_s,
                "bytes_per_launch": by_s, "achieved": by_s / ms_s / 1e6,
                "frac": by_s / ms_s / 1e6 / HBM_PEAK_GBS,
                "traffic": measured_traffic(wname, sl, "k_iter")}
            log(f"  streaming form (k_iter_lds): {ms_s * 1e3:.2f} us per iteration, "
                f"{by_s / ms_s / 1e6:.0f} GB/s ({by_s / ms_s / 1e6 / HBM_PEAK_GBS:.1%} of HBM peak)")
    else:
        roof = None

    two_step = None
    if wl == "channel_aniso":
        # the CP2 sequence of two solves with the cross terms of the first
        # solution on the second right-hand side, and the cross-term kernels
        log("timing the two-solve CP2 sequence")
        val = B.assemble_corrector(mesh0, B.PM_CP2, prm0, w0["nu"], w0["dt"])["val64"]
        b = rhs[0]["cp2"]
        torch.cuda.synchronize()
        t = time.perf_counter()
        eta, eta_t, infs = B.cp2_solve_two_step(mesh0, val, prm0, w0["nu"], w0["dt"], b)
        torch.cuda.synchronize()
        wall2 = time.perf_counter() - t
        ms3, by3 = B.pm_time_cross(mesh0, prm0, w0["nu"], w0["dt"], eta_t, b, 50)
        b2 = B.cp2_cross_rhs(mesh0, prm0, w0["nu"], w0["dt"], eta_t, b)
        ck = {name: {"ms": ms, "bytes": by, "GBs": by / ms / 1e6,
                     "frac_hbm": by / ms / 1e6 / HBM_PEAK_GBS}
              for name, ms, by in zip(("k_cross_prep", "k_cross_est", "k_cross_rhs"), ms3, by3)}
        two_step = {"ms": wall2 * 1e3, "iters": [i["iters"] for i in infs],
                    "status": [i["status"] for i in infs],
                    "rel_res_true": [i["rel_res_true"] for i in infs],
                    "cross_over_b": float(torch.linalg.norm(b2 - b) / torch.linalg.norm(b)),
                    "kernels": ck}
        log(f"  two-step: {two_step['iters']} iterations, {wall2 * 1e3:.1f} ms; cross kernels "
            + ", ".join(f"{k} {v['ms'] * 1e3:.1f}us {v['GBs']:.0f}GB/s" for k, v in ck.items()))

    cp1c = None
    if wl == "channel_aniso":
        # coupled CP1 by the paper's loop (App. B) at its toll 1e-3, at most
        # ten coupled passes (it converges slowly on this anisotropic block)
        log("timing the coupled CP1")
        vx = B.assemble_corrector(mesh0, B.PM_CP1X, prm0, w0["nu"], w0["dt"])["val64"]
        vy = B.assemble_corrector(mesh0, B.PM_CP1Y, prm0, w0["nu"], w0["dt"])["val64"]
        bx = torch.tensor(w0["rhs"]["cp1x"], device=dev)
        by = torch.tensor(w0["rhs"]["cp1y"], device=dev)
        B.cp1_solve_coupled(mesh0, prm0, w0["nu"], w0["dt"], vx, vy, bx, by, max_outer=0)  # tune
        torch.cuda.synchronize()
        t = time.perf_counter()
        u, v, ic = B.cp1_solve_coupled(mesh0, prm0, w0["nu"], w0["dt"], vx, vy, bx, by, toll=1e-3,
                                       max_outer=10)
        torch.cuda.synchronize()
        wallc = time.perf_counter() - t
        B.cp1_solve_coupled_pcg(mesh0, prm0, w0["nu"], w0["dt"], vx, vy, bx, by)  # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, ip = B.cp1_solve_coupled_pcg(mesh0, prm0, w0["nu"], w0["dt"], vx, vy, bx, by)
        torch.cuda.synchronize()
        wallp = time.perf_counter() - t
        log(f"  coupled CP1 by block-Jacobi CG: {ip['iters']} iterations, {wallp * 1e3:.1f} ms, "
            f"residual {ip['rel_res_true']:.2e}")
        B.cp1_solve_coupled_pcg(mesh0, prm0, w0["nu"], w0["dt"], vx, vy, bx, by, precision=1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, ipm = B.cp1_solve_coupled_pcg(mesh0, prm0, w0["nu"], w0["dt"], vx, vy, bx, by,
                                            precision=1)
        torch.cuda.synchronize()
        wallpm = time.perf_counter() - t
        log(f"  coupled CP1 by block-Jacobi CG, mixed: {ipm['iters']} iterations, "
            f"{wallpm * 1e3:.1f} ms, residual {ipm['rel_res_true']:.2e}")
        # the rest of the step around the CP2: averaged fluxes of the CP1
        # velocity, and the RT0 velocity from the two CP2 solutions above
        uc, vc, _ = B.cp1_solve_coupled_pcg(mesh0, prm0, w0["nu"], w0["dt"], vx, vy, bx, by)
        fb, _ = B.flux_average(mesh0, uc, vc)
        B.rt0_update(mesh0, prm0, w0["nu"], w0["dt"], eta_t, eta, fb)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(10):
            fb, b1v = B.flux_average(mesh0, uc, vc)
        torch.cuda.synchronize()
        ms_fa = (time.perf_counter() - t) / 10 * 1e3
        t = time.perf_counter()
        for _ in range(10):
            u2, v2, q2 = B.rt0_update(mesh0, prm0, w0["nu"], w0["dt"], eta_t, eta, fb)
        torch.cuda.synchronize()
        ms_rt = (time.perf_counter() - t) / 10 * 1e3
        tail = {"flux_average_ms": ms_fa, "rt0_update_ms": ms_rt}
        log(f"  flux_average {ms_fa:.3f} ms, rt0_update {ms_rt:.3f} ms (wall, with its sync)")
        cp1c = {"ms": wallc * 1e3, "toll": 1e-3, "max_passes": 10, "passes": ic["outer"],
                "err": ic["err"],
                "iters": [ic["x"]["iters"], ic["y"]["iters"]], "status": ic["status"],
                "coupled_cg": {"ms": wallp * 1e3, "iters": ip["iters"], "status": ip["status"],
                               "rel_res_true": ip["rel_res_true"]},
                "coupled_cg_mixed": {"ms": wallpm * 1e3, "iters": ipm["iters"],
                                     "status": ipm["status"],
                                     "rel_res_true": ipm["rel_res_true"]},
                "step_tail": tail}
        log(f"  coupled CP1: {ic['outer']} passes, iterations {cp1c['iters']}, {wallc * 1e3:.1f} ms")

    sequential = None
    if batch is not None:
        # the same systems solved one after another with pcg_solve
        log("timing the batch as sequential single solves")
        vals = [B.assemble_corrector(m, B.PM_CP2, p, w["nu"], w["dt"])["val64"]
                for m, p, w in zip(meshes, prms, ws)]
        for m, v, r in zip(meshes, vals, rhs):  # tune every shape first
            B.pcg_solve(m, v, r["cp2"])
        torch.cuda.synchronize()
        t = time.perf_counter()
        for m, v, r in zip(meshes, vals, rhs):
            _, info = B.pcg_solve(m, v, r["cp2"])
            if info["status"] != 0:
                raise RuntimeError(f"sequential solve failed: {info}")
        torch.cuda.synchronize()
        seq = time.perf_counter() - t
        sequential = {"ms": seq * 1e3, "solves_per_s": len(meshes) / seq,
                      "batched_speedup": value * seq / len(meshes)}

    mixed = None
    if not args.no_mixed:
        log("timing mixed steps")
        wallm, infm = timed(1)
        mixed = {
            "solves_per_s": solves_per_step * args.steps / wallm,
            "speedup_vs_fp64": (solves_per_step * args.steps / wallm) / value,
            "iters": iter_summary(infm[-1]),
            "max_rel_res_true": max(i["rel_res_true"] for i in infm[-1]),
        }
        if tmesh is not None:
            mk = {"launch": B.pm_last_launch(tmesh)}
            for name, which, reps in (("k_spmv", 0, 200), ("iteration", 1, 200)):
                ms, by = B.pm_time_kernel(tmesh, which, reps)
                mk[name] = {"ms": ms, "bytes": by, "GBs": by / ms / 1e6}
            mixed["kernels"] = mk

    cpu = None
    if not args.no_cpu_baseline and wl != "batch":
        log("timing the CPU oracle on a bounded sample")
        from oracle import assemble as oasm
        from oracle import geometry, ordering
        from oracle import pcg as opcg

        m = w0["mesh"]
        geo = geometry.build(m["xy"], m["tri"], w0["side_tag"])
        perm = ordering.rcm(geo["nbr"])
        A = oasm.assemble(geo, perm, oasm.CP2, w0["params"], w0["nu"], w0["dt"])["A"]
        b = w0["rhs"]["cp2"][perm]
        k = 50
        t = time.perf_counter()
        opcg.pcg(A, b, tol=1e-10, max_it=k)
        per_it = (time.perf_counter() - t) / k
        k = max(50, int(args.cpu_seconds / per_it) // 50 * 50)
        t = time.perf_counter()
        opcg.pcg(A, b, tol=1e-10, max_it=k)
        per_it = (time.perf_counter() - t) / k
        its = [i["iters"] for i in inf64[-1]]
        sec_per_step = per_it * sum(its)
        cpu = {
            "value": solves_per_step / sec_per_step,
            "unit": "solves/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"oracle Jacobi-PCG (NumPy/SciPy, single thread) on this workload's CP2 "
                      f"system: {k} iterations at {per_it * 1e3:.2f} ms each, scaled to the "
                      f"{sum(its)} iterations of one GPU step ({'+'.join(map(str, its))}); "
                      f"host {cpu_model()}, {len(os.sched_getaffinity(0))} cores available",
        }

    if args.copy_calibration:
        src = torch.empty(256 * 2**20 // 8, dtype=torch.float64, device=dev).normal_()
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall64 / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wname, "n_cells": n_cells, "nnz": nnz, "systems": len(ws),
                   "solves_per_step": solves_per_step, "tol": 1e-10,
                   "iters": iter_summary(inf64[-1])},
        "roofline": roof,
        "kernels": kern,
        "solve_only": solve_only,
        "mixed": mixed,
        "sequential": sequential,
        "cp2_two_step": two_step,
        "cp1_coupled": cp1c,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
