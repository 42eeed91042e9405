#!/usr/bin/env python3
"""Throughput benchmark of the composed split-operator time step on one MI355X.

Metric: grid-pt x surface substeps per second, where a substep is one kinetic
action (forward FFT, phase, inverse FFT of every surface) with the potential
action that precedes it, and a time step of a composition with M Strang
stages has M substeps (Table II: N_B = M).

Default workload: three-mode, three-surface linear vibronic coupling model
(seeded synthetic stand-in for the paper's pyrazine model), 128^3 grid on
[-7, 7)^3, triple-jump sixth-order composition of VTV (M = 9), dt = 10 a.u.,
complex128.  Inputs are generated on the host, copied to HBM and resident
before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One JSON line is printed.  Besides the contract fields it carries
  roofline     -- the dominant kernel's algorithmic bytes per launch over its
                  average launch duration (HIP events on the plan's stream,
                  inside this run), against the 8 TB/s HBM peak; `traffic` is
                  filled from a committed rocprofv3 counter summary when its
                  kernel source hash matches, else null;
  cpu_baseline -- the FP64 CPU oracle timed on this host on a bounded sample
                  of the same workload (its step loop only).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("grid-pt·surface substeps/s; time-to-error 1e-10 (FP64)/1e-5 (FP32) vs Strang")
UNIT = "grid-pt·surface substeps/s"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (ndim, n, comp, order, dt, dtype)
    "lvc3d_128cube_x3_tj6_vtv_c128": (3, 128, "triple_jump", 6, 10.0, "c128"),
    "lvc3d_256cube_x3_tj6_vtv_c128": (3, 256, "triple_jump", 6, 10.0, "c128"),
    "lvc3d_64cube_x3_tj8_vtv_c128": (3, 64, "triple_jump", 8, 10.0, "c128"),
    "lvc3d_64cube_x3_tj8_vtv_c64": (3, 64, "triple_jump", 8, 10.0, "c64"),
    "lvc3d_128cube_x3_tj6_vtv_c64": (3, 128, "triple_jump", 6, 10.0, "c64"),
    "twosurf1d_1024_strang_vtv_c128": (1, 1024, "strang", 2, 0.01, "c128"),
    "twosurf1d_1024_sf10_vtv_c128": (1, 1024, "suzuki", 10, 2.0**-6, "c128"),
}
DEFAULT = "lvc3d_128cube_x3_tj6_vtv_c128"
KERNEL_SOURCES = ["paper_1903_04946_amd/csrc/kernels_3d.hip",
                  "paper_1903_04946_amd/csrc/kernels_1d.hip",
                  "paper_1903_04946_amd/csrc/fft_core.hpp"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def make_model(ndim, n):
    from paper_1903_04946_amd import synth
    if ndim == 1:
        return synth.two_surface_1d(n=n)
    return synth.lvc_3d(n=n)


def traffic_from_profiles(workload: str, kernel_kind: str):
    """HBM bytes per launch of the dominant kernel from a committed rocprofv3
    counter summary (profiles/traffic_<workload>.json), if its kernel source
    hash matches the current sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            t = json.load(f)
        if t.get("kernel_source_hash") != kernel_source_hash():
            return None
        k = t["kernels"][kernel_kind]
        return float(k["hbm_bytes_per_launch"])
    except (KeyError, ValueError, OSError):
        return None


def cpu_baseline(model, comp, order, dt, substeps_per_step, budget_s=12.0):
    """Times the FP64 oracle's step loop on this host (all OpenMP threads)."""
    from oracle import oracle as O
    comp_id = {"strang": O.STRANG, "triple_jump": O.TRIPLE_JUMP, "suzuki": O.SUZUKI}[comp]
    P = O.Problem(model.n, model.lo, model.hi, model.nsurf, model.inv_mass, model.vtable,
                  model.hbar)
    _, sec1, threads = O.propagate_timed(P, model.psi0, O.VTV, comp_id, order, dt, 1)
    steps = 1
    if sec1 < budget_s / 2:
        steps = max(1, int(budget_s / max(sec1, 1e-3)))
        steps = min(steps, 1000)
        _, sec, threads = O.propagate_timed(P, model.psi0, O.VTV, comp_id, order, dt, steps)
    else:
        sec = sec1
    units = model.nsurf * model.npts * substeps_per_step * steps
    return {"value": units / sec, "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": f"{steps} step(s) x {substeps_per_step} substeps of the same workload, "
                      f"FP64 oracle step loop ({sec:.2f} s, plan-time eigendecomposition excluded)"}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain 1 GiB device copy (counter calibration)")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py runs on one GPU: this build has no multi-GPU path "
              f"(asked for --gpus {a.gpus}).", file=sys.stderr)
        return 2

    import torch
    from paper_1903_04946_amd import soprop

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    if a.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ndim, n, comp, order, dt, dts = WORKLOADS[a.workload]
    dtype = torch.complex128 if dts == "c128" else torch.complex64
    model = make_model(ndim, n)
    plan = soprop.Plan.from_model(model, comp=comp, order=order, dt=dt, dtype=dtype)
    info = plan.info
    M = info.M
    psi = torch.from_numpy(model.psi0).to(dtype).cuda()
    units_per_step = model.nsurf * model.npts * M

    # warm-up
    plan.propagate(psi, a.warmup)
    torch.cuda.synchronize()

    # timed region: exactly K steps
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    plan.propagate(psi, a.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / a.steps
    value = units_per_step * a.steps / (ms / 1e3)

    # per-kernel timing over a second run of the same K steps
    plan.set_timing(True)
    plan.propagate(psi, a.steps)
    kt = plan.timing_read()
    plan.set_timing(False)
    norm = plan.observables(psi)["norm"]

    dom = max(kt, key=lambda k: kt[k]["ms"])
    d = kt[dom]
    avg_ms = d["ms"] / d["count"]
    bytes_per_launch = d["bytes"] / d["count"]
    achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9
    traffic = traffic_from_profiles(a.workload, dom)
    kernels = {k: {"launches": v["count"], "avg_us": 1e3 * v["ms"] / v["count"],
                   "share": v["ms"] / sum(x["ms"] for x in kt.values()),
                   "alg_GBps": v["bytes"] / (v["ms"] / 1e3) / 1e9} for k, v in kt.items()}

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(model, comp, order, dt, M)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if dts == "c128" else "f32",
        "data": "synthetic",
        "config": {"workload": a.workload, "ndim": ndim, "grid": [n] * ndim,
                   "nsurf": model.nsurf, "split": "VTV", "composition": comp, "order": order,
                   "substeps_per_step": M, "dt": dt, "state_dtype": dts,
                   "v_tables": info.n_v_tables, "table_bytes": info.table_bytes},
        "roofline": {"bound": "hbm" if ndim == 3 else "alu", "kernel": dom,
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if traffic is None else traffic,
                     "avg_launch_us": avg_ms * 1e3, "alg_bytes_per_launch": bytes_per_launch},
        "kernels": kernels,
        "cpu_baseline": cpu,
        "checks": {"norm_after": norm, "wall_s_timed": wall},
        "kernel_source_hash": kernel_source_hash(),
    }
    if ndim == 1:
        # on-chip workload: report against the FP64 vector peak instead
        out["roofline"].update({"bound": "alu", "unit": "GB/s (on-chip, informational)"})
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
