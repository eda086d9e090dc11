"""Benchmark of the VLBM hot path on one MI355X.

Headline workload: the 2-D isentropic vortex (periodic [0,10]^2, strength 5,
background flow (1,1), ideal gas gamma = 1.4, Sensor B, CFL 0.45) on its
largest grid, 1024^2, FP64.  A step is one fused D2Q4 lattice update of the
whole grid (moments, EOS closure, retarget + reprojection, sensor, collision,
streaming and the reductions for the next step), launched through the C ABI;
`value` is lattice updates per second (MLUPS) of that step.

Beside it on the same JSON line:
  roofline      the fused step kernel against the 8 TB/s HBM peak, from the
                algorithmic bytes 2 * 16 * sizeof(double) per lattice update
                and the step time measured with HIP events on the stream the
                kernel runs on; `traffic` = measured HBM bytes per launch
                from the committed hardware-counter summary when it was
                taken on the current kernel source (else null);
  fp32          the FP32 forms (FP32 arithmetic; FP32 storage with FP64
                arithmetic) on the same grid;
  grid_4096     FP64 and FP32 at 4096^2, a working set far above the 256 MB
                last-level cache (the grid for roofline claims);
  riemann4096   four-quadrant Riemann configuration 3, 4096^2, outflow, Sensor A
                (the Ducros gate of Sensor B loses admissibility at this grid):
                per-step rates, and the whole FP32 run to t = 0.25;
  d1q2          the D1Q2 step (Sod shock tube data) at 2^26 cells;
  adjoint       adjoint/forward step-cost ratio on the adjoint workload
                (1024^2 perturbed vortex, frozen dt = 1/625, Sensor B), per
                step and end to end (checkpointed forward + backward);
  cpu_baseline  the FP64 CPU oracle (OpenMP) on a bounded sample of the
                headline workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "d2q4_fp64_vortex1024_traffic.txt")
KERNEL_SOURCES = ("paper_2609_10639_amd/csrc/vlbm_step2d.hip", "paper_2609_10639_amd/csrc/vlbm_common.hpp",
                  "paper_2609_10639_amd/csrc/vlbm_api.cpp")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--grid", type=int, default=1024)
    ap.add_argument("--big-grid", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="headline measurement only")
    ap.add_argument("--cpu-steps", type=int, default=500)   # about 10 s of host time on 16 threads
    ap.add_argument("--only", default="", help="profiling aid: fp64 | fp32 | fp32_mixed | big64 | big32 | "
                                                "riemann32 | d1q2_64 | d1q2_32 | adjoint32 | adjoint64 | copy")
    return ap.parse_args()


# ------------------------------------------------------------------ workloads

def vortex_cfg(n):
    from paper_2609_10639_amd import problems as pr
    W0, dx = pr.vortex(n)
    return W0, dict(dim=2, nx=n, ny=n, dx=dx, bc=(0, 0, 0, 0), cfl=0.45, sensor=2, **pr.SENSOR_2D,
                    **pr.IDEAL_AIR.config())


def riemann_cfg(n):
    """Configuration 3 with Sensor A (0.7, 1, 16): with the Ducros gate of
    Sensor B it loses admissibility on grids from 800^2 up."""
    from paper_2609_10639_amd import problems as pr
    W0, dx = pr.riemann2d(n, 3)
    return W0, dict(dim=2, nx=n, ny=n, dx=dx, bc=(1, 1, 1, 1), cfl=0.45, sensor=1, **pr.SENSOR_2D,
                    **pr.IDEAL_AIR.config())


def whole_run(W0, cfg, precision, t_end):
    """One run from W0 to t_end (every step retargeted, landing exactly), timed
    by the host clock around run_to_time: the whole-job rate, batches and their
    host read-backs included."""
    import torch
    from paper_2609_10639_amd import Solver
    s = Solver(precision=precision, **cfg)
    s.init(W0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = s.run_to_time(t_end)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert s.clock()[0] == t_end
    s.close()
    cells = cfg["nx"] * cfg["ny"]
    return {"t_end": t_end, "steps": n, "seconds": round(dt, 3), "MLUPS": round(n * cells / dt / 1e6, 1)}


def sod_cfg(n):
    from paper_2609_10639_amd import problems as pr
    W0, dx = pr.sod(n)
    return W0, dict(dim=1, nx=n, ny=1, dx=dx, bc=(1, 1, 1, 1), cfl=0.5, sensor=1, **pr.SENSOR_1D,
                    **pr.IDEAL_AIR.config())


def adjoint_cfg(n=1024, steps=625):
    from paper_2609_10639_amd import problems as pr
    W0, dx = pr.vortex_perturbed(n, amplitude=1e-3, seed=42)
    return W0, dict(dim=2, nx=n, ny=n, dx=dx, bc=(0, 0, 0, 0), retarget_every=0, c_fixed=dx * steps, sensor=2,
                    **pr.SENSOR_2D, **pr.IDEAL_AIR.config())


# ------------------------------------------------------------------ timing

def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_steps(W0, cfg, precision, steps, warmup):
    """`warmup` untimed steps, then `steps` steps timed with HIP events on the
    library's stream, synchronised on both sides.  Returns ms per step."""
    import torch
    from paper_2609_10639_amd import Solver
    s = Solver(precision=precision, **cfg)
    s.init(W0)
    if warmup:
        s.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record(s.stream)
    done = s.step(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    assert done == steps, (done, steps)
    s.close()
    return e0.elapsed_time(e1) / steps


def bytes_per_lu(dim, precision):
    nf = 16 if dim == 2 else 6
    return 2 * nf * (8 if precision == "fp64" else 4)


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(cells):
    """HBM bytes per launch of the FP64 step at `cells`, from the committed
    counter summary, if it was taken on the current kernel source."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha256") != kernel_source_hash() or int(kv.get("cells", -1)) != cells:
            return None
        return int(float(kv["hbm_bytes_per_launch"]))
    except (OSError, KeyError, ValueError):
        return None


def roofline(ms, cells, dim, precision, traffic=None):
    gbs = bytes_per_lu(dim, precision) * cells / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic}


def line(ms, cells, dim, precision):
    return {"MLUPS": round(cells / ms / 1e3, 1), "ms_per_step": round(ms, 5),
            "roofline": roofline(ms, cells, dim, precision)}


def adjoint_ratio(precision, n=1024, nsteps=625, reps=50):
    """Per-step cost of the adjoint step against the forward step on the same
    state (raw entry points, frozen link speed), and the end-to-end cost of
    the checkpointed backward pass against the forward pass."""
    import torch
    from paper_2609_10639_amd import Solver
    from paper_2609_10639_amd.adjoint import Rollout
    W0, cfg = adjoint_cfg(n, nsteps)
    s = Solver(precision=precision, **cfg)
    W = torch.tensor(W0, device="cuda")
    fa, fb = s.new_populations(), s.new_populations()
    na, nb = s.new_norms(), s.new_norms()
    s.raw_init(W, fa, na)
    for _ in range(5):
        s.raw_step(fa, na, fb, nb)
        s.raw_adjoint_step(fa, na, fb, fa.clone())
    lam0, lam1 = s.new_populations(), s.new_populations()
    lam0.fill_(1e-3)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record(s.stream)
    for i in range(reps):
        if i % 2 == 0:
            s.raw_step(fa, na, fb, nb)
        else:
            s.raw_step(fb, nb, fa, na)
    e1.record(s.stream)
    torch.cuda.synchronize()
    t_fwd = e0.elapsed_time(e1) / reps
    e0, e1 = _events()
    e0.record(s.stream)
    for i in range(reps):
        if i % 2 == 0:
            s.raw_adjoint_step(fa, na, lam0, lam1)
        else:
            s.raw_adjoint_step(fa, na, lam1, lam0)
    e1.record(s.stream)
    torch.cuda.synchronize()
    t_adj = e0.elapsed_time(e1) / reps
    # end to end: checkpointed forward, then backward (replay + adjoint), with
    # the replay overlapped on a second stream (default) and serial; the second
    # of two passes is reported (the first also fills torch's caching allocator
    # with the checkpoint and segment buffers)
    rho_t = torch.tensor(W0[0], device="cuda")
    e2e = {}
    for overlap in (True, False):
        run = Rollout(s, nsteps, overlap=overlap)
        for _ in range(2):
            ck = None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            WN, ck = run.forward(W)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            WNbar = torch.zeros_like(WN)
            WNbar[0] = (WN[0] - rho_t) * cfg["dx"] ** 2
            run.backward(W, ck, WNbar)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
        e2e["end_to_end" if overlap else "end_to_end_serial"] = {
            "steps": nsteps, "checkpoint_every": run.K, "forward_s": round(t1 - t0, 4),
            "backward_s": round(t2 - t1, 4), "ratio": round((t2 - t1) / (t1 - t0), 3)}
    s.close()
    return {"precision": precision, "grid": [n, n], "fwd_ms_per_step": round(t_fwd, 5),
            "adj_ms_per_step": round(t_adj, 5), "step_ratio": round(t_adj / t_fwd, 3), **e2e}


def cpu_baseline(n, steps):
    from oracle import core
    W0, cfg = vortex_cfg(n)
    o = core.Oracle(**cfg)
    o.init(W0)
    o.step()
    t0 = time.perf_counter()
    for _ in range(steps):
        o.step()
    dt = time.perf_counter() - t0
    return {"value": round(n * n * steps / dt / 1e6, 2), "unit": "MLUPS", "cores": core.threads(),
            "kind": "oracle", "sample": "%d FP64 steps of the %dx%d vortex (%.1f s, OpenMP)" % (steps, n, n, dt)}


def copy_bw(nbytes, steps, warmup):
    """Plain device copies of `nbytes`: torch's copy_ and the library's probe
    (16-byte non-temporal loads and stores): attainable bandwidth, and the
    reference for the hardware byte counters (torch's copy)."""
    import torch
    from paper_2609_10639_amd import _native
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream().cuda_stream

    def timed(fn):
        for _ in range(warmup):
            fn()
        e0, e1 = _events()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        return {"ms": round(ms, 5), "GBs": round(2 * nbytes / (ms * 1e-3) / 1e9, 1)}

    torch_copy = timed(lambda: dst.copy_(src))
    dst.zero_()
    probe = timed(lambda: _native.copy_probe(src.data_ptr(), dst.data_ptr(), nbytes, stream))
    ok = bool(torch.equal(src, dst))
    return {"bytes_read": nbytes, "bytes_written": nbytes, "torch_copy": torch_copy, "probe": probe,
            "probe_copied_exactly": ok}


# ------------------------------------------------------------------ main

def only(a):
    o = a.only
    if o == "copy":
        return dict(only=o, **copy_bw(16 * a.big_grid * a.big_grid * 8, a.steps, a.warmup))
    if o.startswith("adjoint"):
        return dict(only=o, **adjoint_ratio("fp32" if o.endswith("32") else "fp64"))
    prec = {"fp64": "fp64", "fp32": "fp32", "fp32_mixed": "fp32_mixed", "big64": "fp64", "big32": "fp32",
            "riemann32": "fp32", "d1q2_64": "fp64", "d1q2_32": "fp32"}[o]
    if o.startswith("d1q2"):
        W0, cfg = sod_cfg(1 << 26)
    elif o == "riemann32":
        W0, cfg = riemann_cfg(a.big_grid)
    else:
        W0, cfg = vortex_cfg(a.big_grid if o.startswith("big") else a.grid)
    ms = time_steps(W0, cfg, prec, a.steps, a.warmup)
    return dict(only=o, grid=[cfg["ny"], cfg["nx"]], **line(ms, cfg["nx"] * cfg["ny"], cfg["dim"], prec))


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.only:
        print(json.dumps(only(a)), flush=True)
        return

    W0, cfg = vortex_cfg(a.grid)
    cells = a.grid * a.grid
    ms64 = time_steps(W0, cfg, "fp64", a.steps, a.warmup)
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
        "config": {"workload": "isentropic vortex advection, periodic [0,10]^2, strength 5, background (1,1), "
                               "ideal gas 1.4, D2Q4, Sensor B, CFL 0.45", "grid": [a.grid, a.grid], "cells": cells},
        "roofline": roofline(ms64, cells, 2, "fp64", measured_traffic(cells)),
    }
    if not a.no_extra:
        out["fp32"] = {p: line(time_steps(W0, cfg, p, a.steps, a.warmup), cells, 2, p)
                       for p in ("fp32", "fp32_mixed")}
        nb = a.big_grid
        Wb, cb = vortex_cfg(nb)
        ksteps = max(20, a.steps // 4)
        out["grid_%d" % nb] = {p: line(time_steps(Wb, cb, p, ksteps, 5), nb * nb, 2, p)
                               for p in ("fp64", "fp32", "fp32_mixed")}
        del Wb
        Wr, cr = riemann_cfg(nb)
        out["riemann%d" % nb] = {p: line(time_steps(Wr, cr, p, ksteps, 5), nb * nb, 2, p) for p in ("fp32", "fp64")}
        out["riemann%d" % nb]["fp32_to_t_end"] = whole_run(Wr, cr, "fp32", 0.25)
        del Wr
        W1, c1 = sod_cfg(1 << 26)
        out["d1q2"] = {"cells": 1 << 26, **{p: line(time_steps(W1, c1, p, ksteps, 5), 1 << 26, 1, p)
                                            for p in ("fp64", "fp32")}}
        del W1
        out["adjoint"] = [adjoint_ratio("fp32"), adjoint_ratio("fp64")]
        # context for the roofline fractions: a plain device copy of one 4096^2 FP64 population array
        out["copy"] = copy_bw(16 * nb * nb * 8, 20, 3)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.grid, a.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
