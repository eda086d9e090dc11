"""Benchmark of the VLBM hot path on one MI355X.

Workload: the 2-D isentropic vortex (periodic [0,10]^2, strength 5, background
flow (1,1), ideal gas gamma = 1.4, Sensor B, CFL 0.45) at its largest grid,
1024^2.  A step is one fused D2Q4 lattice update of the whole grid (moments,
EOS closure, retarget + reprojection, sensor, collision, streaming and the
reductions for the next step), launched through the C ABI.

Printed: one JSON line with MLUPS of the FP64 step (`value`), the FP32 form
beside it, the HBM roofline of the dominant kernel (algorithmic bytes
2 * 16 * sizeof(double) per lattice update, timed with HIP events on the
stream the kernel runs on), a larger 4096^2 grid for a working set well above
the 256 MB last-level cache, and the FP64 CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--grid", type=int, default=1024)
    ap.add_argument("--big-grid", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="headline measurement only")
    ap.add_argument("--cpu-steps", type=int, default=100)
    ap.add_argument("--only", default="", help="profiling aid: fp64 | fp32 | big64 | big32 | copy "
                                                "(headline otherwise)")
    return ap.parse_args()


def vortex_cfg(n):
    from paper_2609_10639_amd import problems as pr
    W0, dx = pr.vortex(n)
    cfg = dict(dim=2, nx=n, ny=n, dx=dx, bc=(0, 0, 0, 0), cfl=0.45, sensor=2, **pr.SENSOR_2D,
               **pr.IDEAL_AIR.config())
    return W0, cfg


def time_steps(n, precision, steps, warmup):
    """Run `warmup` untimed steps then time `steps` steps with HIP events on the
    library's stream.  Returns (ms per step, cells)."""
    import torch
    from paper_2609_10639_amd import Solver
    W0, cfg = vortex_cfg(n)
    s = Solver(precision=precision, **cfg)
    s.init(W0)
    if warmup:
        s.step(warmup)
    stream = s.stream
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    done = s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    assert done == steps
    ms = e0.elapsed_time(e1) / steps
    s.close()
    return ms, n * n


def bytes_per_lu(precision):
    return 2 * 16 * (8 if precision == "fp64" else 4)


def roofline(ms, cells, precision):
    gbs = bytes_per_lu(precision) * cells / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None}


def cpu_baseline(n, steps):
    import numpy as np
    from oracle import core
    W0, cfg = vortex_cfg(n)
    o = core.Oracle(**cfg)
    o.init(W0)
    o.step()
    t0 = time.perf_counter()
    for _ in range(steps):
        o.step()
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(n * n * steps / dt / 1e6, 2), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "%d FP64 steps of the %dx%d vortex (%.1f s)" % (steps, n, n, dt)}


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.only == "copy":
        # plain HBM copy of the FP64 D2Q4 population array at the big grid:
        # the reference for the hardware byte counters and attainable bandwidth
        nbytes = 16 * a.big_grid * a.big_grid * 8
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(a.warmup):
            dst.copy_(src)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.steps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / a.steps
        print(json.dumps({"only": "copy", "bytes_read": nbytes, "bytes_written": nbytes, "ms": ms,
                          "GBs": 2 * nbytes / (ms * 1e-3) / 1e9}))
        return
    if a.only:
        n = a.big_grid if a.only.startswith("big") else a.grid
        prec = "fp32" if a.only.endswith("32") else "fp64"
        ms, cells = time_steps(n, prec, a.steps, a.warmup)
        print(json.dumps({"only": a.only, "grid": n, "ms_per_step": ms, "MLUPS": cells / ms / 1e3,
                          "roofline": roofline(ms, cells, prec)}))
        return

    ms64, cells = time_steps(a.grid, "fp64", a.steps, a.warmup)
    out = {
        "metric": "MLUPS and % of HBM roofline (FP64 vs FP32), adjoint/forward step-cost ratio",
        "value": round(cells / ms64 / 1e3, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms64, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "isentropic vortex, periodic [0,10]^2, strength 5, background (1,1), "
                               "D2Q4, ideal gas 1.4, Sensor B, CFL 0.45", "grid": [a.grid, a.grid],
                   "cells": cells},
        "roofline": roofline(ms64, cells, "fp64"),
    }
    if not a.no_extra:
        ms32, _ = time_steps(a.grid, "fp32", a.steps, a.warmup)
        out["fp32"] = {"MLUPS": round(cells / ms32 / 1e3, 1), "ms_per_step": round(ms32, 5),
                       "roofline": roofline(ms32, cells, "fp32")}
        big = {}
        for prec in ("fp64", "fp32"):
            msb, cb = time_steps(a.big_grid, prec, max(20, a.steps // 4), 5)
            big[prec] = {"MLUPS": round(cb / msb / 1e3, 1), "ms_per_step": round(msb, 4),
                         "roofline": roofline(msb, cb, prec)}
        out["grid_%d" % a.big_grid] = big
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.grid, a.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
