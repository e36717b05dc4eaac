"""Benchmark of the corrector hot path on one MI355X.

A step is one pass of the hot path over the workload: assembly of the CP1x
and CP2 matrices from the per-cell fields, then a PCG solve of each to a true
relative residual of 1e-10.  The reported value is corrector solves per
second (whole job), float64; the same step in mixed precision, the roofline of
the dominant iteration kernel and the CPU oracle on a bounded sample are
reported beside it.  Inputs are seeded and synthetic (synth/), resident in
HBM before timing starts.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload channel|square|channel_aniso]
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(name):
    from synth import workloads

    if name == "channel":
        return workloads.channel(276, 2), "channel_1M"
    if name == "channel_aniso":
        return workloads.channel(552, 3, aniso=True), "channel_aniso_4M"
    if name == "square":
        return workloads.square_inclusion(), "square_inclusion_8k"
    raise SystemExit(f"unknown workload {name}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="channel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the corrector library is a single-GPU build "
              "(the multi-GPU sharding is a design note only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2309_03543_amd import binding as B

    dev = torch.device("cuda:0")
    t0 = time.time()
    w, wname = build_workload(args.workload)
    m = w["mesh"]
    log(f"workload {wname}: {m['tri'].shape[0]} cells, generated in {time.time() - t0:.1f}s")
    t0 = time.time()
    mesh = B.Mesh(m["xy"], m["tri"], w["side_tag"])
    st = mesh.stats
    log(f"mesh: n={st['n_cells']} nnz={st['nnz']} bw={st['bandwidth']} idx={st['index_bits']}b "
        f"maxT={st['max_T']:.3g} ({time.time() - t0:.1f}s)")
    prm = {k: torch.tensor(v, device=dev) for k, v in w["params"].items()}
    rhs = {k: torch.tensor(w["rhs"][k], device=dev) for k in ("cp1x", "cp2")}
    nu, dt = w["nu"], w["dt"]
    stream = torch.cuda.current_stream()

    def step(precision):
        infos = []
        for kind, key in ((B.PM_CP1X, "cp1x"), (B.PM_CP2, "cp2")):
            val = B.assemble_corrector(mesh, kind, prm, nu, dt)["val64"]
            x, info = B.pcg_solve(mesh, val, rhs[key], precision=precision, tol=1e-10)
            if info["status"] != 0:
                raise RuntimeError(f"solve {key} failed: {info}")
            infos.append(info)
        return infos

    def timed(precision):
        for _ in range(args.warmup):
            step(precision)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        t = time.perf_counter()
        infos = []
        for k in range(args.steps):
            infos.append(step(precision))
            log(f"  step {k + 1}/{args.steps} precision={precision} iters="
                f"{[i['iters'] for i in infos[-1]]} res={['%.2e' % i['rel_res_true'] for i in infos[-1]]}")
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        gpu_ms = ev0.elapsed_time(ev1)
        return wall, gpu_ms, infos

    log("timing float64 steps")
    wall64, gms64, inf64 = timed(0)
    solves = 2 * args.steps
    value = solves / wall64
    # roofline of the dominant kernel, measured on the state of the last CP2 solve
    ms_spmv, by_spmv = B.pm_time_kernel(mesh, 0, 200)
    ms_upd, by_upd = B.pm_time_kernel(mesh, 1, 200)
    dom = ("k_spmv", ms_spmv, by_spmv) if ms_spmv >= ms_upd else ("k_update", ms_upd, by_upd)
    achieved = dom[2] / (dom[1] * 1e-3) / 1e9
    it64 = [i["iters"] for i in inf64[-1]]

    mixed = None
    if not args.no_mixed:
        log("timing mixed steps")
        wallm, gmsm, infm = timed(1)
        mixed = {
            "solves_per_s": solves / wallm,
            "speedup_vs_fp64": (solves / wallm) / value,
            "iters": [i["iters"] for i in infm[-1]],
            "rel_res_true": [i["rel_res_true"] for i in infm[-1]],
        }

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        from oracle import assemble as oasm
        from oracle import geometry, ordering
        from oracle import pcg as opcg

        perm, _, _ = mesh.export()
        geo = geometry.build(m["xy"], m["tri"], w["side_tag"])
        A = oasm.assemble(geo, perm, oasm.CP2, w["params"], nu, dt)["A"]
        b = w["rhs"]["cp2"][perm]
        k = 50
        t = time.perf_counter()
        opcg.pcg(A, b, tol=1e-10, max_it=k)
        per_it = (time.perf_counter() - t) / k
        k = max(50, int(args.cpu_seconds / per_it) // 50 * 50)
        t = time.perf_counter()
        opcg.pcg(A, b, tol=1e-10, max_it=k)
        per_it = (time.perf_counter() - t) / k
        sec_per_solve = per_it * (it64[1] + it64[0])
        cpu = {
            "value": 2.0 / sec_per_solve,
            "unit": "solves/s",
            "cores": 1,
            "kind": "oracle",
            "sample": f"oracle Jacobi-PCG on the CP2 system of this workload, {k} iterations "
                      f"({per_it * 1e3:.1f} ms/iteration, single-threaded NumPy/SciPy), scaled to the "
                      f"GPU step's {it64[0]}+{it64[1]} iterations",
        }

    out = {
        "metric": "corrector PCG solves/s (FP64, 1e-10 true residual)",
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
        "config": {"workload": wname, "n_cells": st["n_cells"], "nnz": st["nnz"],
                   "systems_per_step": ["CP1x", "CP2"], "iters": it64, "tol": 1e-10},
        "roofline": {"bound": "hbm", "kernel": dom[0], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "ms_per_launch": dom[1], "bytes_per_launch": dom[2]},
        "kernels": {"k_spmv": {"ms": ms_spmv, "GBs": by_spmv / ms_spmv / 1e6},
                    "k_update": {"ms": ms_upd, "GBs": by_upd / ms_upd / 1e6}},
        "mixed": mixed,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
