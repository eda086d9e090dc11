"""Benchmark of the VLBM hot path on one MI355X.

Headline workload: the four-quadrant Riemann problem, configuration 3 of
Sec. IV.E (interacting shocks), on [0,1]^2 at 4096^2 cells, outflow edges,
ideal gas gamma = 1.4, D2Q4 with Sensor B (beta_min 0.7, beta_max 1, C 16),
CFL 0.45 with the link speed retargeted every 4 steps, FP32 populations and
FP32 arithmetic (clock, reductions and totals in FP64).  A step is one fused D2Q4 lattice update of the
whole grid (moments, EOS closure, retarget + reprojection, sensor, collision,
streaming and the reductions for the next step), launched through the C ABI;
`value` is lattice updates per second (MLUPS) over the K timed steps, the
populations resident in HBM when the timed region starts.

Beside it on the same JSON line:
  roofline      the fused step kernel against the 8 TB/s HBM peak: algorithmic
                bytes 2 * 16 * 4 per lattice update over the step time measured
                with HIP events on the library's stream; `traffic` = measured
                HBM bytes per launch from the committed hardware-counter summary
                when it was taken on the current kernel source (else null);
  c3            the Riemann configurations at 4096^2: configuration 3 in FP64
                and FP32 storage with FP64 arithmetic, configuration 12 in all
                three forms, and whole runs to t = 0.25 timed by the host clock
                (batches and their host read-backs included);
  c1_sod        the Sod tube, 1000 cells, whole runs to t = 0.2 in one resident
                workgroup (the library's path up to 4096 cells) and, for
                comparison, with one launch per step;
  c2_vortex     the isentropic vortex at 1024^2 (all forms) and 4096^2;
  c4_bzt        the dense-gas tube, 8192 cells, whole runs (one launch per
                step: launch-bound), and
                its 2-D extrusion at 2048^2 (all forms, shifted energy gauge in
                FP32), per step and whole run to t = 0.2;
  d1q2          the D1Q2 step (Sod data) at 2^26 cells;
  adjoint       adjoint/forward step-cost ratio on the adjoint workload
                (1024^2 perturbed vortex, frozen dt = 1/625, Sensor B), per
                step and end to end (checkpointed forward + backward);
  copy          plain device copies of one 4096^2 FP64 population array and a
                read-only stream: the attainable bandwidth; and the step's own
                access pattern without its arithmetic (march probe, FP32 and
                FP64 at the headline grid): the ceiling of that pattern;
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the headline
                workload, on all host threads and on one.
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "d2q4_fp32_riemann3_4096_traffic.txt")
# the step kernel, its launch configuration (configure_d2q4, in the same file) and the headers it includes
KERNEL_SOURCES = ("paper_2609_10639_amd/csrc/vlbm_step2d.hip", "paper_2609_10639_amd/csrc/vlbm_planes.hpp",
                  "paper_2609_10639_amd/csrc/vlbm_common.hpp")
WORKLOAD = ("four-quadrant Riemann problem, configuration 3 (interacting shocks), [0,1]^2, outflow, ideal gas "
            "gamma 1.4, D2Q4, Sensor B (0.7, 1, 16), CFL 0.45 retargeted every 4 steps, FP32 populations and arithmetic")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--grid", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="headline measurement only")
    ap.add_argument("--cpu-steps", type=int, default=20, help="oracle steps of the all-thread sample")
    ap.add_argument("--cpu-steps-1t", type=int, default=2, help="oracle steps of the one-thread sample")
    ap.add_argument("--only", default="", help="profiling aid: one measurement, e.g. headline | r12_fp64 | "
                                                "r3_fp32 | vortex1024_fp32 | bzt2048_fp32 | d1q2_fp32 | "
                                                "adjoint32 | copy | c1 | oracle_c2_1024")
    return ap.parse_args()


# ------------------------------------------------------------------ workloads

def riemann_cfg(n, config):
    """Configuration 3 or 12 under Sensor B, link speed retargeted every 4 steps."""
    from paper_2609_10639_amd import problems as pr
    W0, dx = pr.riemann2d(n, config)
    return W0, dict(dim=2, nx=n, ny=n, dx=dx, bc=(1, 1, 1, 1), cfl=0.45, retarget_every=pr.RETARGET_2D, sensor=2,
                    **pr.SENSOR_2D, **pr.IDEAL_AIR.config())


def vortex_cfg(n):
    from paper_2609_10639_amd import problems as pr
    W0, dx = pr.vortex(n)
    return W0, dict(dim=2, nx=n, ny=n, dx=dx, bc=(0, 0, 0, 0), cfl=0.45, retarget_every=pr.RETARGET_2D, sensor=2,
                    **pr.SENSOR_2D, **pr.IDEAL_AIR.config())


def sod_cfg(n):
    from paper_2609_10639_amd import problems as pr
    W0, dx = pr.sod(n)
    return W0, dict(dim=1, nx=n, ny=1, dx=dx, bc=(1, 1, 1, 1), cfl=0.5, sensor=1, **pr.SENSOR_1D,
                    **pr.IDEAL_AIR.config())


def energy_gauge(W0):
    """Mean specific internal energy of W0 (the e_offset of the FP32 dense-gas runs)."""
    D = W0.shape[0] - 2
    ke = 0.5 * sum(W0[1 + a] ** 2 for a in range(D)) / W0[0]
    return float(((W0[D + 1] - ke) / W0[0]).mean())


def bzt_cfg(n, dim):
    from paper_2609_10639_amd import problems as pr
    if dim == 1:
        W0, dx = pr.bzt_tube(n)
        cfg = dict(dim=1, nx=n, ny=1, dx=dx, bc=(1, 1, 1, 1), cfl=0.5, sensor=1, **pr.SENSOR_1D)
    else:
        W0, dx = pr.bzt_extrusion(n)
        cfg = dict(dim=2, nx=n, ny=n, dx=dx, bc=(1, 1, 0, 0), cfl=0.45, retarget_every=pr.RETARGET_2D, sensor=2,
                   **pr.SENSOR_2D)
    return W0, dict(cfg, **pr.VDW_REDUCED_CV50.config())


def adjoint_cfg(n=1024, steps=625):
    from paper_2609_10639_amd import problems as pr
    W0, dx = pr.vortex_perturbed(n, amplitude=1e-3, seed=42)
    return W0, dict(dim=2, nx=n, ny=n, dx=dx, bc=(0, 0, 0, 0), retarget_every=0, c_fixed=dx * steps, sensor=2,
                    **pr.SENSOR_2D, **pr.IDEAL_AIR.config())


def with_gauge(W0, cfg, precision):
    """FP32 dense-gas runs store the energy in the shifted gauge."""
    if cfg.get("eos", 0) == 1 and precision != "fp64":
        return dict(cfg, e_offset=energy_gauge(W0))
    return cfg


# ------------------------------------------------------------------ timing

def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_steps(W0, cfg, precision, steps, warmup):
    """`warmup` untimed steps, then `steps` steps timed with HIP events on the
    library's stream, synchronised on both sides.  Returns ms per step."""
    import torch
    from paper_2609_10639_amd import Solver
    s = Solver(precision=precision, **with_gauge(W0, cfg, precision))
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


def whole_run(W0, cfg, precision, t_end):
    """One run from W0 to t_end (retargeted as configured, landing exactly), timed
    by the host clock around run_to_time: the whole-job rate, batches and their
    host read-backs included."""
    import torch
    from paper_2609_10639_amd import Solver
    s = Solver(precision=precision, **with_gauge(W0, cfg, precision))
    s.init(W0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = s.run_to_time(t_end)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert s.clock()[0] == t_end
    s.close()
    cells = cfg["nx"] * cfg["ny"]
    return {"t_end": t_end, "steps": n, "seconds": round(dt, 4), "MLUPS": round(n * cells / dt / 1e6, 1)}


def small_1d_runs(W0, cfg, t_end, precisions):
    """Whole runs of a D1Q2 grid small enough for the library's resident path
    (batches of steps in one workgroup, populations on chip between steps: up
    to 4096 cells), and the same runs with one launch per step (the path of
    larger grids), each after one untimed run that loads the kernels."""
    out = {"path": "resident: batches of steps in one workgroup"}
    for p in precisions:
        whole_run(W0, cfg, p, t_end)
        out[p + "_to_t_end"] = whole_run(W0, cfg, p, t_end)
    os.environ["VLBM_D1_RESIDENT"] = "0"
    try:
        per = {}
        for p in precisions:
            whole_run(W0, cfg, p, t_end)
            per[p + "_to_t_end"] = whole_run(W0, cfg, p, t_end)
        out["one_launch_per_step"] = per
    finally:
        del os.environ["VLBM_D1_RESIDENT"]
    return out


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
    """HBM bytes per launch of the headline step, from the committed counter
    summary, if it was taken on the current kernel source and grid."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as fh:
            for ln in fh:
                if ":" in ln and not ln.startswith("#"):
                    k, v = ln.split(":", 1)
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


def per_step(W0, cfg, precisions, steps, warmup):
    cells = cfg["nx"] * cfg["ny"]
    return {p: line(time_steps(W0, cfg, p, steps, warmup), cells, cfg["dim"], p) for p in precisions}


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


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ORACLE_SAMPLE = """
import json, sys, time
sys.path.insert(0, %r)
from bench import riemann_cfg
from oracle import core
n, steps = %d, %d
W0, cfg = riemann_cfg(n, 3)
o = core.Oracle(**cfg)
o.init(W0)
o.step()
t0 = time.perf_counter()
for _ in range(steps):
    o.step()
dt = time.perf_counter() - t0
print(json.dumps({"seconds": dt, "steps": steps, "threads": core.threads()}))
"""


def oracle_sample(n, steps, threads=None):
    """The FP64 oracle on `steps` steps of the headline workload (after one
    untimed step), in a child process so that its OpenMP thread count can be
    set; returns the timing record."""
    env = dict(os.environ)
    if threads:
        env["OMP_NUM_THREADS"] = str(threads)
    out = subprocess.run([sys.executable, "-c", _ORACLE_SAMPLE % (ROOT, n, steps)], env=env, capture_output=True,
                         text=True, check=True)
    return json.loads(out.stdout.strip().splitlines()[-1])


_ORACLE_RUN = """
import json, sys, time
sys.path.insert(0, %r)
import bench
from oracle import core
name = %r
W0, cfg, t_end = {"c1_sod_1000": lambda: (*bench.sod_cfg(1000), 0.2),
                  "c4_bzt_tube_8192": lambda: (*bench.bzt_cfg(8192, 1), 0.2),
                  "c2_vortex_128": lambda: (*bench.vortex_cfg(128), 10.0),
                  "c2_vortex_256": lambda: (*bench.vortex_cfg(256), 10.0),
                  "c2_vortex_1024": lambda: (*bench.vortex_cfg(1024), 10.0)}[name]()
o = core.Oracle(**cfg)
o.init(W0)
t0 = time.perf_counter()
if %r:   # step by step, a progress line every 1000 steps on stderr
    steps = 0
    while o.clock()[0] < t_end:
        o.step(t_end)
        steps += 1
        if steps %% 1000 == 0:
            print("oracle %%s: %%d steps, t = %%.3f, %%.0f s" %% (name, steps, o.clock()[0], time.perf_counter() - t0),
                  file=sys.stderr, flush=True)
else:
    steps = o.run_to_time(t_end)
dt = time.perf_counter() - t0
print(json.dumps({"seconds": dt, "steps": steps, "cells": cfg["nx"] * cfg["ny"], "t_end": t_end,
                  "threads": core.threads()}))
"""


def oracle_run(name, threads=None, progress=False):
    """A whole oracle run of one configuration, in a child process (its OpenMP
    thread count set there); returns the timing record.  With `progress` the
    child reports every 1000 steps on this process's stderr."""
    env = dict(os.environ)
    if threads:
        env["OMP_NUM_THREADS"] = str(threads)
    out = subprocess.run([sys.executable, "-c", _ORACLE_RUN % (ROOT, name, progress)], env=env,
                         stdout=subprocess.PIPE, stderr=None if progress else subprocess.PIPE, text=True, check=True)
    return json.loads(out.stdout.strip().splitlines()[-1])


def oracle_whole_runs():
    """The FP64 oracle's whole runs of the Sod tube (1000 cells), the dense-gas
    tube (8192 cells) and the vortex (128^2; 256^2 on all threads only) to
    their end times, on all host threads and on one."""
    out = {}
    for name, one in (("c1_sod_1000", True), ("c4_bzt_tube_8192", True), ("c2_vortex_128", True),
                      ("c2_vortex_256", False)):
        rec = {}
        for label, threads in (("all_threads", None), ("one_thread", 1)) if one else (("all_threads", None),):
            r = oracle_run(name, threads)
            rec["steps"], rec["t_end"] = r["steps"], r["t_end"]
            rec[label] = {"seconds": round(r["seconds"], 3), "threads": r["threads"],
                          "MLUPS": round(r["cells"] * r["steps"] / r["seconds"] / 1e6, 2)}
        out[name] = rec
    return out


def cpu_baseline(n, steps_all, steps_one):
    allt = oracle_sample(n, steps_all)
    one = oracle_sample(n, steps_one, threads=1)
    cells = n * n
    rate = lambda r: round(cells * r["steps"] / r["seconds"] / 1e6, 2)
    return {"value": rate(allt), "unit": "MLUPS", "cores": allt["threads"], "kind": "oracle",
            "sample": "%d FP64 oracle steps of the headline workload at %dx%d (%.1f s, %d OpenMP threads)" % (
                steps_all, n, n, allt["seconds"], allt["threads"]),
            "one_thread": {"value": rate(one), "unit": "MLUPS", "cores": 1,
                           "sample": "%d steps (%.1f s)" % (steps_one, one["seconds"])},
            "whole_runs": oracle_whole_runs(),
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "build": "gcc -O3 -ffp-contract=off -fopenmp, FP64"}


def march_probe(W0, cfg, precision, steps, warmup):
    """The step's loads and stores without its arithmetic (vlbm_probe_march),
    timed like the step; returns the line of the step's algorithmic bytes."""
    import torch
    from paper_2609_10639_amd import Solver
    s = Solver(precision=precision, **cfg)
    s.init(W0)
    s.probe_march(warmup)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record(s.stream)
    s.probe_march(steps)
    e1.record(s.stream)
    torch.cuda.synchronize()
    s.close()
    return line(e0.elapsed_time(e1) / steps, cfg["nx"] * cfg["ny"], 2, precision)


def copy_bw(nbytes, steps, warmup):
    """Plain device copies of `nbytes` (torch's copy_, the library's copy probe)
    and the probe's read-only stream: attainable bandwidth, and the reference
    for the hardware byte counters."""
    import torch
    from paper_2609_10639_amd import _native
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream().cuda_stream

    def timed(fn, moved):
        for _ in range(warmup):
            fn()
        e0, e1 = _events()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        return {"ms": round(ms, 5), "GBs": round(moved / (ms * 1e-3) / 1e9, 1)}

    torch_copy = timed(lambda: dst.copy_(src), 2 * nbytes)
    dst.zero_()
    probe = timed(lambda: _native.copy_probe(src.data_ptr(), dst.data_ptr(), nbytes, stream, 0), 2 * nbytes)
    ok = bool(torch.equal(src, dst))
    read = timed(lambda: _native.copy_probe(src.data_ptr(), dst.data_ptr(), nbytes, stream, 1), nbytes)
    return {"bytes": nbytes, "torch_copy": torch_copy, "probe_copy": probe, "probe_copied_exactly": ok,
            "probe_read_only": read}


# ------------------------------------------------------------------ main

def only(a):
    o = a.only
    n = a.grid
    if o == "copy":
        return dict(only=o, **copy_bw(16 * n * n * 8, a.steps, a.warmup))
    if o.startswith("march"):
        W0, cfg = riemann_cfg(n, 3)
        return dict(only=o, **march_probe(W0, cfg, "fp32" if o.endswith("32") else "fp64", a.steps, a.warmup))
    if o == "oracle_c2_1024":   # the oracle's whole vortex run at 1024^2 (minutes of CPU)
        r = oracle_run("c2_vortex_1024", progress=True)
        return dict(only=o, **r, MLUPS=round(r["cells"] * r["steps"] / r["seconds"] / 1e6, 2), cpu_model=cpu_model())
    if o == "c1":
        W0, cfg = sod_cfg(1000)
        return dict(only=o, **small_1d_runs(W0, cfg, 0.2, ("fp64", "fp32")))
    if o.startswith("adjoint"):
        return dict(only=o, **adjoint_ratio("fp32" if o.endswith("32") else "fp64"))
    if o == "headline":
        W0, cfg, prec = *riemann_cfg(n, 3), "fp32"
    else:
        name, prec = o.rsplit("_", 1)
        prec = {"fp64": "fp64", "fp32": "fp32", "mixed": "fp32_mixed"}[prec]
        W0, cfg = {"r12": lambda: riemann_cfg(n, 12), "r3": lambda: riemann_cfg(n, 3),
                   "vortex1024": lambda: vortex_cfg(1024), "vortex4096": lambda: vortex_cfg(4096),
                   "bzt2048": lambda: bzt_cfg(2048, 2), "d1q2": lambda: sod_cfg(1 << 26)}[name]()
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

    n = a.grid
    cells = n * n
    W0, cfg = riemann_cfg(n, 3)
    ms = time_steps(W0, cfg, "fp32", a.steps, a.warmup)
    out = {
        "metric": "MLUPS and % of HBM roofline (FP64 vs FP32), adjoint/forward step-cost ratio",
        "value": round(cells / ms / 1e3, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "grid": [n, n], "cells": cells},
        "roofline": roofline(ms, cells, 2, "fp32", measured_traffic(cells)),
    }
    if not a.no_extra:
        k = max(20, a.steps // 4)
        c3 = {"config3": per_step(W0, cfg, ("fp64", "fp32_mixed"), k, 5)}
        c3["config3"]["fp32_to_t_end"] = whole_run(W0, cfg, "fp32", 0.25)
        c3["config3"]["fp64_to_t_end"] = whole_run(W0, cfg, "fp64", 0.25)
        del W0
        W12, cf12 = riemann_cfg(n, 12)
        c3["config12"] = per_step(W12, cf12, ("fp32", "fp64", "fp32_mixed"), k, 5)
        c3["config12"]["fp32_to_t_end"] = whole_run(W12, cf12, "fp32", 0.25)
        del W12
        out["c3"] = c3
        Ws, cs = sod_cfg(1000)
        out["c1_sod"] = small_1d_runs(Ws, cs, 0.2, ("fp64", "fp32"))
        Wv, cv = vortex_cfg(1024)
        out["c2_vortex"] = {"1024": per_step(Wv, cv, ("fp64", "fp32", "fp32_mixed"), a.steps, a.warmup)}
        Wv, cv = vortex_cfg(4096)
        out["c2_vortex"]["4096"] = per_step(Wv, cv, ("fp64", "fp32"), k, 5)
        del Wv
        Wt, ct = bzt_cfg(8192, 1)
        Wb, cb = bzt_cfg(2048, 2)
        out["c4_bzt"] = {"1d_8192": {"path": "one launch per step (launch-bound)",
                                     **{p + "_to_t_end": whole_run(Wt, ct, p, 0.2) for p in ("fp64", "fp32")}},
                         "2d_2048": per_step(Wb, cb, ("fp64", "fp32", "fp32_mixed"), a.steps, a.warmup)}
        out["c4_bzt"]["2d_2048"]["fp32_to_t_end"] = whole_run(Wb, cb, "fp32", 0.2)
        del Wb
        W1, c1 = sod_cfg(1 << 26)
        out["d1q2"] = {"cells": 1 << 26, **per_step(W1, c1, ("fp64", "fp32"), k, 5)}
        del W1
        out["adjoint"] = [adjoint_ratio("fp32"), adjoint_ratio("fp64")]
        out["copy"] = copy_bw(16 * n * n * 8, 20, 3)
        Wm, cm = riemann_cfg(n, 3)
        out["copy"]["march_probe"] = {p: march_probe(Wm, cm, p, k, 5) for p in ("fp32", "fp64")}
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, a.cpu_steps, a.cpu_steps_1t)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
