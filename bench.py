"""Benchmark of the DG hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--dt S] [--inner f32|f64]
                    [--workload slab96_q1] [--compare-f64] [--no-cpu-baseline]

Workload (default): the 96 x 96 x 192 voxel cathode slab (x = transport
axis, 1 um voxels), DG-Q1, 9 unknowns per node of which 7 are transported
(99,090,432 transported DoF), seeded Gaussian-threshold porosity 0.6,
synthetic transport and kinetic parameters, constant 1C discharge current.
All inputs are synthetic, seeded and resident in HBM before timing starts.

Set-up (untimed): the context, the initial state of the discharge on the
GPU (equilibrium concentrations and the steady potential).

A step is one accepted step of the discharge under the naive time
controller (every part of the hot path: FP64 residual and Newton update,
element block-Jacobi assembly and inversion, condensed JVP, block apply,
GMRES and coarse correction, halving dt after a failed solve), inner solve
in FP32 by default.  The K timed steps continue the discharge from the W
warm-up steps.  ms_per_step is their mean wall time.

value = DG operator GDoF/s: transported DoF / mean duration of one
application of the Krylov operator (the condensed tangent, in the inner
precision) at the state the timed steps reached, timed with HIP events on
the stream it runs on.  roofline = the kernel with the largest share of the
step (the block apply: one per GMRES iteration) against the HBM peak; the
other kernels are listed beside it.
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
FARADAY = 96485.332


def cpu_baseline(w, budget_s=12.0):
    """Oracle condensed JVP (the Krylov operator) on a 24 x 24 x 48 sub-block."""
    import synth
    from oracle import dg as odg
    from oracle import model as om
    mask = w.mask()[:48, :24, :24].copy()
    D0, i0 = synth.sample_transport_kinetics(w.param_seed)
    P = om.Problem(24, 24, 48, w.h, w.order, mask, D0=D0, kE=i0 / om.F, f_C=w.f_C)
    u = synth.random_state(P.n_elem, P.n_nodes, 1, phase=mask, phi_spread=5e-3)
    m = odg.old_mass(P, synth.random_state(P.n_elem, P.n_nodes, 2, phase=mask))
    v = synth.random_vector(7, P.n_elem, P.n_nodes, 3)
    odg.jvp_condensed(P, u, v, m, 0.5, 0.05)
    n, t0, c0 = 0, time.perf_counter(), time.process_time()
    while time.perf_counter() - t0 < budget_s:
        odg.jvp_condensed(P, u, v, m, 0.5, 0.05)
        n += 1
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    dof = P.n_elem * P.n_nodes * 7
    return {"value": dof * n / wall / 1e9, "unit": "GDoF/s", "cores": max(1, round(cpu / wall)),
            "kind": "oracle",
            "sample": f"FP64 condensed JVP (complex step) of a 24x24x48-voxel sub-block (Q1, {dof} DoF) "
                      f"of the same workload, {n} applications in {wall:.1f} s"}


def time_launches(fn, stream, reps):
    """Mean duration [ms] of fn() over reps launches, HIP events on `stream`."""
    import torch
    fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def run_steps(ctx, ctrl, u, t, n, inner, log, verbose=0):
    """n accepted steps of the naive controller (halving on failed solves)."""
    tot = {"newton_its": 0, "gmres_its": 0, "trials": 0, "halvings": 0}
    for _ in range(n):
        t, rep = ctx.advance(ctrl, t, u, inner=inner, verbose=verbose)
        for k in tot:
            tot[k] += rep[k]
        log(f"[bench] step of {rep['dt']:.4g} s to t = {t:.4f} s: {rep['trials']} trials, "
            f"{rep['newton_its']} Newton, {rep['gmres_its']} GMRES")
    return t, tot


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dt", type=float, default=0.1, help="first trial step [s]")
    ap.add_argument("--inner", default="f32", choices=["f32", "f64"])
    ap.add_argument("--workload", default="slab96_q1")
    ap.add_argument("--compare-f64", action="store_true",
                    help="repeat the timed steps with an FP64 inner solve from the same state")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", type=int, default=0, help="Newton progress lines on stderr")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path; "
              "run with --gpus 1.", file=sys.stderr)
        return 2

    import torch
    import synth
    from paper_2511_05233_amd import lsbdg

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    w = synth.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    mask = w.mask()
    D0, i0 = synth.sample_transport_kinetics(w.param_seed)
    ctx = lsbdg.Context(w.nx, w.ny, w.nz, w.h, w.order, mask, D0=D0, kE=i0 / FARADAY, f_C=w.f_C)
    stream = torch.cuda.current_stream()
    n_dof = ctx.n_elem * ctx.n_nodes * 7
    nodes = ctx.n_elem * ctx.n_nodes

    u, rep0 = ctx.initial_state(inner=args.inner, verbose=args.verbose)
    log(f"[bench] initial state: {rep0['newton_its']} Newton, {rep0['gmres_its']} GMRES")
    t = 0.0
    ctrl = lsbdg.controller("naive", dt0=args.dt)
    t, _ = run_steps(ctx, ctrl, u, t, args.warmup, args.inner, log, args.verbose)
    u_start = u.clone() if args.compare_f64 else None
    ctrl_start = lsbdg.DgController.from_buffer_copy(ctrl)
    t_start = t
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    t, tot = run_steps(ctx, ctrl, u, t, args.steps, args.inner, log, args.verbose)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = wall * 1e3 / args.steps

    # kernels of the step, each timed alone at the reached state
    S = torch.float32 if args.inner == "f32" else torch.float64
    sb = 4 if S == torch.float32 else 8
    uS = u.to(S)
    g = torch.Generator(device=dev).manual_seed(7)
    v7 = torch.randn((7, ctx.n_elem, ctx.n_nodes), generator=g, dtype=S, device=dev)
    y7 = torch.empty_like(v7)
    m8 = ctx.mass(u)
    r9 = torch.empty_like(u)
    reps = 20
    ms_jvp = time_launches(lambda: ctx.jvp(uS, v7, t, args.dt, out=y7, condensed=True), stream, reps)
    ms_res = time_launches(lambda: ctx.residual(u, m8, t, args.dt, out=r9), stream, reps)
    ctx.blockjacobi_setup(u, t, args.dt, dtype=S)
    ms_apply = time_launches(lambda: ctx.blockjacobi_apply(v7, out=y7), stream, reps)
    ms_setup = time_launches(lambda: ctx.blockjacobi_setup(u, t, args.dt, dtype=S), stream, 3)

    def gbs(nbytes, ms):
        return nbytes / (ms * 1e-3) / 1e9

    b_jvp = nodes * (9 + 7 + 7) * sb + ctx.n_elem           # u, v in; Jv out; phase
    b_res = nodes * (9 + 8 + 9) * 8 + ctx.n_elem            # u, old mass in; R out; phase
    b_apply = ctx.n_elem * (56 * 56 + 2 * 56) * sb          # blocks, x in, y out
    kernels = {
        "jvp_condensed": {"ms": ms_jvp, "GB/s": gbs(b_jvp, ms_jvp), "bytes": b_jvp},
        "residual_f64": {"ms": ms_res, "GB/s": gbs(b_res, ms_res), "bytes": b_res},
        "block_apply": {"ms": ms_apply, "GB/s": gbs(b_apply, ms_apply), "bytes": b_apply},
        "block_setup": {"ms": ms_setup},
    }
    for k in kernels.values():
        if "GB/s" in k:
            k["frac"] = round(k["GB/s"] / HBM_PEAK_GBS, 4)
            k["GB/s"] = round(k["GB/s"], 1)
        k["ms"] = round(k["ms"], 4)

    achieved = gbs(b_apply, ms_apply)
    out = {
        "metric": METRIC,
        "value": round(n_dof / (ms_jvp * 1e-3) / 1e9, 3),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{args.inner} inner / f64 outer" if args.inner == "f32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.nx}x{w.ny}x{w.nz} voxels of {w.h * 1e6:g} um, "
                               f"DG-Q{w.order}, 7 transported + 2 node-local fields, porosity "
                               f"{w.porosity} (mask seed {w.mask_seed}), {w.f_C}C discharge",
                   "dof": n_dof, "dt0_s": args.dt, "t_start_s": round(t_start, 6),
                   "t_end_s": round(t, 6),
                   "step": "accepted step of the naive time controller: backward-Euler solves "
                           "(Newton in FP64 + GMRES(30) with element block-Jacobi and coarse "
                           "correction), halving dt on failed solves",
                   "trials": tot["trials"], "halvings": tot["halvings"],
                   "newton_its": tot["newton_its"], "gmres_its": tot["gmres_its"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "apply_blocks_kernel", "ms": round(ms_apply, 4),
                     "bytes_per_launch": b_apply},
        "kernels": kernels,
    }
    if args.compare_f64 and args.inner == "f32":
        u64 = u_start.clone()
        torch.cuda.synchronize()
        w1 = time.perf_counter()
        ctrl64 = lsbdg.DgController.from_buffer_copy(ctrl_start)
        _, tot64 = run_steps(ctx, ctrl64, u64, t_start, args.steps, "f64", log, args.verbose)
        torch.cuda.synchronize()
        wall64 = time.perf_counter() - w1
        rel = [float(torch.linalg.norm(u[f] - u64[f]) / torch.clamp(torch.linalg.norm(u64[f]), min=1e-300))
               for f in range(9)]
        out["f64_inner"] = {"ms_per_step": round(wall64 * 1e3 / args.steps, 2),
                            "newton_its": tot64["newton_its"], "gmres_its": tot64["gmres_its"],
                            "mixed_speedup": round(wall64 / wall, 3),
                            "rel_l2_mixed_vs_f64": [float(f"{x:.3e}") for x in rel]}
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
