"""Benchmark of the DG hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload slab96_q1] [--no-cpu-baseline]

Workload (default): the 96 x 96 x 192 voxel cathode slab (x = transport
axis, 1 um voxels), DG-Q1, 9 unknowns per node of which 7 are transported
(99,090,432 transported DoF), seeded Gaussian-threshold porosity 0.6, 1C.
All inputs are synthetic, seeded and resident in HBM before timing starts.

A step is one pass of the implemented hot path over the slab: the old-mass
kernel and the FP64 backward-Euler residual.  value = transported DoF per
residual application / its average time (GDoF/s).  The JSON line also holds
the HBM roofline of the residual kernel and the CPU oracle timed on a
bounded sub-block of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DG operator GDoF/s (% roofline) + s per full discharge, mixed vs FP64 at fixed error"
HBM_PEAK_GBS = 8000.0


def _state(ctx, mask, seed, dev, dtype):
    """Realistic random state (9 fields) generated on the device."""
    import torch
    g = torch.Generator(device=dev).manual_seed(seed)
    Ne, npn = ctx.n_elem, ctx.n_nodes
    typical = [1500.0, 6.0, 6.2e-3, 3.9e-3, 1.9e-3, 3.6e-12, 0.0, 0.2375, 6.9e-6]
    u = torch.empty((9, Ne, npn), dtype=dtype, device=dev)
    for f in range(9):
        z = torch.randn((Ne, npn), generator=g, dtype=dtype, device=dev)
        u[f] = 5e-3 * z if f == 6 else typical[f] * torch.exp(0.1 * z)
    pore = torch.tensor(mask.reshape(-1) == 0, device=dev)
    u[7:9, pore, :] = 0
    return u


def cpu_baseline(w, budget_s=12.0):
    """Oracle FP64 residual on a 24 x 24 x 48 sub-block of the workload."""
    import resource  # noqa: F401
    import synth
    from oracle import dg as odg
    from oracle import model as om
    mask = w.mask()[:48, :24, :24].copy()
    D0, i0 = synth.sample_transport_kinetics(w.param_seed)
    P = om.Problem(24, 24, 48, w.h, w.order, mask, D0=D0, kE=i0 / om.F, f_C=w.f_C)
    u = synth.random_state(P.n_elem, P.n_nodes, 1, phase=mask, phi_spread=5e-3)
    m = odg.old_mass(P, synth.random_state(P.n_elem, P.n_nodes, 2, phase=mask))
    odg.residual(P, u, m, 0.5, 0.05)
    n, t0, c0 = 0, time.perf_counter(), time.process_time()
    while time.perf_counter() - t0 < budget_s:
        odg.residual(P, u, m, 0.5, 0.05)
        n += 1
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    dof = P.n_elem * P.n_nodes * 7
    return {"value": dof * n / wall / 1e9, "unit": "GDoF/s", "cores": max(1, round(cpu / wall)),
            "kind": "oracle",
            "sample": f"FP64 residual of a 24x24x48-voxel sub-block (Q1, {dof} DoF) of the same "
                      f"workload, {n} evaluations in {wall:.1f} s"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="slab96_q1")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); run with --gpus 1.", file=sys.stderr)
        return 2

    import torch
    import synth
    from paper_2511_05233_amd import lsbdg

    w = synth.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    mask = w.mask()
    D0, i0 = synth.sample_transport_kinetics(w.param_seed)
    ctx = lsbdg.Context(w.nx, w.ny, w.nz, w.h, w.order, mask, D0=D0, kE=i0 / 96485.332, f_C=w.f_C)
    dtype = torch.float64
    u = _state(ctx, mask, 1, dev, dtype)
    uo = _state(ctx, mask, 2, dev, dtype)
    m = torch.empty((8, ctx.n_elem, ctx.n_nodes), dtype=dtype, device=dev)
    r = torch.empty((9, ctx.n_elem, ctx.n_nodes), dtype=dtype, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        ctx.mass(uo, out=m)
        ctx.residual(u, m, 0.5, 0.05, out=r)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # whole-step timing
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    # dominant kernel alone, same stream and launch configuration
    e0.record(stream)
    for _ in range(args.steps):
        ctx.residual(u, m, 0.5, 0.05, out=r)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_res = e0.elapsed_time(e1) / args.steps

    n_dof = ctx.n_elem * ctx.n_nodes * 7
    nodes = ctx.n_elem * ctx.n_nodes
    alg_bytes = nodes * 26 * 8 + ctx.n_elem       # u (9) + old mass (8) + R (9) doubles, phase byte
    achieved = alg_bytes / (ms_res * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(n_dof / (ms_res * 1e-3) / 1e9, 3),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.nx}x{w.ny}x{w.nz} voxels of {w.h * 1e6:g} um, "
                               f"DG-Q{w.order}, 7 transported + 2 node-local fields, porosity "
                               f"{w.porosity} (mask seed {w.mask_seed}), f_C = {w.f_C}/h",
                   "dof": n_dof, "step": "old mass + FP64 residual"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "resid_q1_kernel<double>", "ms": round(ms_res, 4),
                     "bytes_per_launch": alg_bytes},
    }
    if args.copy_probe:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = a.numel() * 8
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
