"""Benchmark of the DG hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--mode newton|controller] [--dt S]
                    [--inner f32|f64] [--workload slab96_q1] [--compare-f64]
                    [--no-cpu-baseline] [--no-mixed] [--no-batch] [--kernels-only] [--copy-probe]
                    [--step-only] [--batch] [--fp32-blocks]
                    [--coarse C] [--coarse-agg A] [--mg-levels L] [--mg-sweeps NU] [--block-reuse X]
                    [--discharge WORKLOAD [--discharge-rate C] [--limiter] [--t-stop T] [--max-wall S]]
                    [--controller-study NX F_C]

Workload (default): the 96 x 96 x 192 voxel cathode slab (x = transport
axis, 1 um voxels), DG-Q1, 9 unknowns per node of which 7 are transported
(99,090,432 transported DoF), seeded Gaussian-threshold porosity 0.6,
synthetic transport and kinetic parameters, constant 1C discharge current.
All inputs are synthetic, seeded and resident in HBM before timing starts.

Set-up (untimed): the context and the initial state of the discharge on the
GPU (equilibrium concentrations and the steady potential).

A step (--mode newton, the default) is one Newton iteration of the implicit
steps of the discharge from the initial state (dt = 0.1 s): FP64 residual,
linearisation, the element blocks (assembled and inverted where the solver
rebuilds them), the full GMRES solve (Krylov operator, block apply, coarse
correction -- the multigrid V-cycle on this slab --, Gram-Schmidt) and the
line-searched FP64 update: every part of the hot path but the time
controller.  Exactly K iterations are timed after W of warm-up on a copy of
the state; a step that converges hands over to the next implicit step.
--mode controller times K accepted steps of the naive controller instead
(an implicit step is 10-20 Newton iterations).  The solver runs with the
library's defaults unless the --coarse, --mg-*, --block-reuse or
--fp32-blocks flags change them.

value = DG operator GDoF/s: transported DoF / mean duration of one
application of the Krylov operator (the condensed tangent at a stored
linearisation, in the inner precision), timed with HIP events on the stream
it runs on.  roofline = that kernel against the HBM peak, with its
algorithmic bytes, the HBM bytes and vector-ALU counts of the committed
rocprofv3 summaries (while they were taken on the current kernel sources)
and the library's STREAM triad for the achievable bandwidth; the other
kernels of a GMRES iteration are listed beside it.

Beside the line (skipped with --no-mixed): five steps on the 16^3 cube and a
full 1C discharge of it to the 1.9 V cutoff, each with FP64 and with mixed
(FP32 inner) solves -- wall times, speedup and the difference of the results.
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
SOLVER_EXTRA = {}      # further dg_solver_opts fields of the timed solves (command line)
FARADAY = 96485.332
# coefficients per node that the Krylov operator reads from the stored
# linearisation (the solid-fraction condensation, both rows)
LIN_COEFFS = 14
# the kernel of the Krylov operator (condensed tangent at a stored
# linearisation), by inner precision, as rocprofv3 names it
JVP_KERNEL = {"f32": "q1_brick_jvp_kernel<float>", "f64": "q1_brick_jvp_kernel<double>"}


def _oracle_timing(workload, budget_s):
    """Worker of the CPU baseline (runs in a child process whose thread
    count is fixed by its environment): the oracle's FP64 residual and its
    condensed tangent (complex step) on a 12 x 12 x 24-voxel sub-block of
    the workload, each repeated for about budget_s / 2 seconds."""
    import synth
    from oracle import dg as odg
    from oracle import model as om
    w = synth.WORKLOADS[workload]
    mask = w.mask()[:24, :12, :12].copy()
    D0, i0 = synth.sample_transport_kinetics(w.param_seed)
    P = om.Problem(12, 12, 24, w.h, w.order, mask, D0=D0, kE=i0 / om.F, f_C=w.f_C)
    u = synth.random_state(P.n_elem, P.n_nodes, 1, phase=mask, phi_spread=5e-3)
    m = odg.old_mass(P, synth.random_state(P.n_elem, P.n_nodes, 2, phase=mask))
    v = synth.random_vector(7, P.n_elem, P.n_nodes, 3)
    dof = P.n_elem * P.n_nodes * 7
    out = {"dof": dof, "voxels": "12x12x24"}
    for name, fn in (("residual", lambda: odg.residual(P, u, m, 0.5, 0.05)),
                     ("jvp_condensed", lambda: odg.jvp_condensed(P, u, v, m, 0.5, 0.05))):
        fn()
        n, t0, c0 = 0, time.perf_counter(), time.process_time()
        while time.perf_counter() - t0 < budget_s / 2:
            fn()
            n += 1
        wall = time.perf_counter() - t0
        out[name] = {"gdofs": dof * n / wall / 1e9, "runs": n, "wall_s": wall,
                     "cpu_over_wall": (time.process_time() - c0) / wall}
    return out


def cpu_baseline(w, budget_s=24.0):
    """The oracle on the host: all host threads, then one thread (child
    processes with the BLAS/OpenMP thread counts set), about budget_s of
    CPU work in total."""
    import subprocess
    nproc = os.cpu_count() or 1
    legs = {}
    for label, threads in (("all", nproc), ("one", 1)):
        env = dict(os.environ)
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            env[k] = str(threads)
        env["CUDA_VISIBLE_DEVICES"] = ""
        env["HIP_VISIBLE_DEVICES"] = ""
        res = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-timing", w.name,
                              str(budget_s / 2)], capture_output=True, text=True, env=env, timeout=600)
        if res.returncode != 0:
            return {"error": res.stderr[-400:]}
        legs[label] = json.loads(res.stdout.strip().splitlines()[-1])
    a = legs["all"]
    dof = a["dof"]
    return {"value": round(a["jvp_condensed"]["gdofs"], 6), "unit": "GDoF/s", "cores": nproc,
            "kind": "oracle",
            "sample": f"FP64 condensed JVP (complex step, numpy) of a 12x12x24-voxel sub-block (Q1, {dof} DoF) "
                      f"of the same workload, {a['jvp_condensed']['runs']} applications in "
                      f"{a['jvp_condensed']['wall_s']:.1f} s with {nproc} host threads allowed",
            "host_nproc": nproc,
            "cpu_over_wall_all_threads": round(a["jvp_condensed"]["cpu_over_wall"], 2),
            "one_core": {"jvp_condensed_gdofs": round(legs["one"]["jvp_condensed"]["gdofs"], 6),
                         "residual_gdofs": round(legs["one"]["residual"]["gdofs"], 6)},
            "all_cores": {"jvp_condensed_gdofs": round(a["jvp_condensed"]["gdofs"], 6),
                          "residual_gdofs": round(a["residual"]["gdofs"], 6)}}


def source_hash():
    """Hash of the HIP sources (the recorded counters hold for this version only)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2511_05233_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy's readings),
    or None when absent or taken on other kernel sources."""
    import re
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    want = source_hash()
    with open(path) as fh:
        for line in fh:
            m = re.match(r"\s*traffic\s+(\S+)\s+bytes_per_launch=(\d+)\s+source=(\w+)", line)
            if m and m.group(1) == kernel and m.group(3) == want:
                return int(m.group(2))
    return None


def recorded_valu(workload, kernel):
    """Vector-ALU instructions per launch of `kernel` (rocprofv3 SQ_INSTS_VALU,
    summed over its wavefronts) from the committed counter summary, or None
    when absent or taken on other kernel sources."""
    import re
    path = os.path.join(ROOT, "profiles", f"valu_{workload}.txt")
    if not os.path.exists(path):
        return None
    want = source_hash()
    with open(path) as fh:
        for line in fh:
            m = re.match(r"\s*valu\s+(\S+)\s+insts_per_launch=(\d+)\s+waves_per_launch=(\d+)\s+source=(\w+)", line)
            if m and m.group(1) == kernel and m.group(4) == want:
                return int(m.group(2)), int(m.group(3))
    return None


# One wave64 vector-ALU instruction occupies a SIMD for 4 cycles; MI355X has
# 256 compute units of 4 SIMDs at 2.4 GHz.
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4


def copy_probe(dev):
    """Three STREAM triads (dg_triad) over 1 GiB arrays: 2 GiB read and
    1 GiB written per launch (reference for the HBM byte counters)."""
    import torch
    from paper_2511_05233_amd import lsbdg
    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    b = torch.ones_like(a)
    c = torch.empty_like(a)
    for _ in range(3):
        lsbdg.triad(c, a, b, 0.5)
    torch.cuda.synchronize()
    return a.numel() * 8


def triad_bandwidth(dev, stream, reps=10):
    """Achievable HBM bandwidth [GB/s]: the library's STREAM triad over three
    1 GiB arrays (24 bytes per element), HIP events on the launch stream."""
    import torch
    from paper_2511_05233_amd import lsbdg
    a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    b = torch.ones_like(a)
    c = torch.empty_like(a)
    ms = time_launches(lambda: lsbdg.triad(c, a, b, 0.5), stream, reps)
    ok = bool(torch.all(c == 1.5))
    del a, b, c
    return {"GB/s": round(24 * (1 << 27) / (ms * 1e-3) / 1e9, 1), "ms": round(ms, 4), "checked": ok}


def valu_view(workload, kernel, ms):
    """The kernel against the vector-ALU issue rate: recorded instructions
    per launch, the time they need at full issue, and that time over the
    measured one (None without a current counter summary)."""
    rec = recorded_valu(workload, kernel)
    if rec is None:
        return None
    insts, waves = rec
    t_issue = insts / VALU_ISSUE_PER_S * 1e3
    return {"insts_per_launch": insts, "waves_per_launch": waves, "insts_per_wave": round(insts / waves, 1),
            "ms_at_full_issue": round(t_issue, 4), "frac_of_issue": round(t_issue / ms, 4)}


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


def random_state(ctx, mask, seed, dev):
    """Seeded positive state around the equilibrium values (9 fields, FP64), on the device."""
    import torch
    g = torch.Generator(device=dev).manual_seed(seed)
    Ne, npn = ctx.n_elem, ctx.n_nodes
    typical = [1500.0, 6.0, 6.2e-3, 3.9e-3, 1.9e-3, 3.6e-12, 0.0, 0.2375, 6.9e-6]
    u = torch.empty((9, Ne, npn), dtype=torch.float64, device=dev)
    for f in range(9):
        z = torch.randn((Ne, npn), generator=g, dtype=torch.float64, device=dev)
        u[f] = 5e-3 * z if f == 6 else typical[f] * torch.exp(0.1 * z)
    pore = torch.tensor(mask.reshape(-1) == 0, device=dev)
    u[7:9, pore, :] = 0
    return u


def time_kernels(ctx, u, t, dt, inner, stream, dev, log):
    """The step's kernels, each timed alone (HIP events) at state u."""
    import torch
    S = torch.float32 if inner == "f32" else torch.float64
    sb = 4 if S == torch.float32 else 8
    nodes = ctx.n_elem * ctx.n_nodes
    uS = u.to(S)
    g = torch.Generator(device=dev).manual_seed(7)
    v7 = torch.randn((7, ctx.n_elem, ctx.n_nodes), generator=g, dtype=S, device=dev)
    y7 = torch.empty_like(v7)
    m8 = ctx.mass(u)
    r9 = torch.empty_like(u)
    reps = 20
    log("[bench] timing kernels")
    ms_lin = time_launches(lambda: ctx.linearize(uS, t, dt), stream, 5)
    ms_jvp = time_launches(lambda: ctx.jvp(uS, v7, t, dt, out=y7, linearized=True), stream, reps)
    ms_res = time_launches(lambda: ctx.residual(u, m8, t, dt, out=r9), stream, reps)
    q1 = ctx.n_nodes == 8
    blocks = ctx.n_nodes in (8, 64)                         # element blocks at k = 1 and 3
    ms_apply_h = None
    if blocks:
        ctx.blockjacobi_setup(uS, t, dt)
        ms_apply = time_launches(lambda: ctx.blockjacobi_apply(v7, out=y7), stream, reps)
        if q1 and S == torch.float32:
            ms_apply_h = time_launches(lambda: ctx.blockjacobi_apply(v7, out=y7, bf16=True), stream, reps)
        ms_setup = time_launches(lambda: ctx.blockjacobi_setup(uS, t, dt), stream, 3 if q1 else 1)

    def gbs(nbytes, ms):
        return nbytes / (ms * 1e-3) / 1e9

    # algorithmic bytes: every array of the operation's definition once per
    # launch -- the tangent reads u (9 fields) and v (7) and writes Jv (7);
    # the coefficients the linearisation stores are the implementation's
    # own traffic (listed apart, not counted)
    b_jvp = nodes * (9 + 7 + 7) * sb + ctx.n_elem           # u, v in; Jv out; phase
    b_lin = nodes * LIN_COEFFS * sb                         # stored linearisation read by the kernel
    b_res = nodes * (9 + 8 + 9) * 8 + ctx.n_elem            # u, old mass in; R out; phase
    nb = 7 * ctx.n_nodes
    b_apply = ctx.n_elem * (nb * nb + 2 * nb) * sb          # blocks, x in, y out
    b_apply_h = ctx.n_elem * (56 * 56 * 2 + 2 * 56 * 4)     # bfloat16 blocks, FP32 x in, y out
    kernels = {
        "jvp_condensed": {"ms": ms_jvp, "GB/s": gbs(b_jvp, ms_jvp), "bytes": b_jvp,
                          "linearisation_bytes_not_counted": b_lin},
        "residual_f64": {"ms": ms_res, "GB/s": gbs(b_res, ms_res), "bytes": b_res},
        "linearize": {"ms": ms_lin},
    }
    if blocks:
        kernels["block_apply"] = {"ms": ms_apply, "GB/s": gbs(b_apply, ms_apply), "bytes": b_apply}
        kernels["block_setup"] = {"ms": ms_setup}
        if not q1:
            # assembly: 2 colours x 448 probes of the Krylov operator; inversion:
            # 2 nb^3 flop per element on the matrix cores (see the kernel trace)
            kernels["block_setup"]["probes"] = 2 * nb
            kernels["block_setup"]["inversion_flop"] = 2 * nb ** 3 * ctx.n_elem
    if ms_apply_h is not None:
        kernels["block_apply_bf16"] = {"ms": ms_apply_h, "GB/s": gbs(b_apply_h, ms_apply_h), "bytes": b_apply_h}
    for k in kernels.values():
        if "GB/s" in k:
            k["frac"] = round(k["GB/s"] / HBM_PEAK_GBS, 4)
            k["GB/s"] = round(k["GB/s"], 1)
        k["ms"] = round(k["ms"], 4)
    return kernels, (JVP_KERNEL[inner], b_jvp, ms_jvp)


def newton_iterations(ctx, u, t, dt, n, inner, log, verbose=0, coarse=0, coarse_agg=0):
    """At most n Newton iterations of the implicit step from (t, u) (one
    dg_step call); fewer when the step converges first."""
    from paper_2511_05233_amd import lsbdg
    if n < 1:
        return {"newton_its": 0, "gmres_its": 0, "last_update": float("nan")}
    try:
        rep = ctx.step(u, t, dt, inner=inner, verbose=verbose, newton_maxit=n, coarse=coarse, **SOLVER_EXTRA,
                       coarse_agg=coarse_agg)
        rep["converged"] = True
    except lsbdg.DgError as e:
        if e.code != -4:                      # DG_ENOCONV: the iteration cap was reached
            raise
        rep = e.report
        rep["converged"] = False
    log(f"[bench] {rep['newton_its']} Newton iterations, {rep['gmres_its']} GMRES, "
        f"update {rep['last_update']:.2e}")
    return rep


GOLDEN_CUBE16 = os.path.join(ROOT, "tests", "golden", "cube16_q1_trajectory.npz")


def mixed_vs_f64(coarse, log, steps=5, dt=0.1):
    """Mixed precision against FP64 at fixed error: 5 backward-Euler steps
    on the 16^3 cube from the oracle's initial state, once with FP64 and
    once with mixed (FP32 inner) solves.  Each path's error against the
    oracle's own trajectory (stored by tests/golden/make_cube16_trajectory.py,
    read here as data) is reported per output: the nine fields (relative L2,
    largest over the steps), the cell voltage, the volume means and the
    conservation sums."""
    import torch
    import synth
    from paper_2511_05233_amd import lsbdg
    w = synth.WORKLOADS["cube16_q1"]
    D0, i0 = synth.sample_transport_kinetics(w.param_seed)
    ctx = lsbdg.Context(w.nx, w.ny, w.nz, w.h, w.order, w.mask(), D0=D0, kE=i0 / FARADAY, f_C=w.f_C)
    gold = None
    if os.path.exists(GOLDEN_CUBE16):
        with np.load(GOLDEN_CUBE16, allow_pickle=False) as z:
            gold = {k: z[k] for k in z.files}
    if gold is not None and abs(float(gold["dt"]) - dt) == 0.0 and gold["u"].shape[0] > steps:
        u0 = torch.tensor(gold["u"][0], device="cuda:0")
        start = "the oracle's initial state"
    else:
        gold = None
        u0, _ = ctx.initial_state(inner="f64", coarse=coarse)
        start = "the GPU initial state (no stored oracle trajectory)"
    area = w.ny * w.nz * w.h ** 2
    res = {}
    for inner in ("f64", "f32"):
        u = u0.clone()
        its = [0, 0]
        ctx.step(u.clone(), 0.0, dt, inner=inner, coarse=coarse)      # warm-up (allocations)
        keep = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            rep = ctx.step(u, k * dt, dt, inner=inner, coarse=coarse)
            its[0] += rep["newton_its"]
            its[1] += rep["gmres_its"]
            keep.append(u.clone())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        err = None
        if gold is not None:
            fe = np.zeros(9)
            ue = me = 0.0
            se = np.zeros(4)
            for k, uk in enumerate(keep, start=1):
                ref = gold["u"][k]
                got = uk.cpu().numpy()
                fe = np.maximum(fe, [np.linalg.norm(got[f] - ref[f]) / max(np.linalg.norm(ref[f]), 1e-300)
                                     for f in range(9)])
                out = ctx.outputs(uk, k * dt)
                ue = max(ue, abs(out["U_cell"] - gold["U_cell"][k]) / abs(gold["U_cell"][k]))
                scale = np.append(np.sqrt(np.mean(ref ** 2, axis=(1, 2))), abs(gold["means"][k][9]))
                me = max(me, float(np.max(np.abs(out["means"] - gold["means"][k]) / np.maximum(scale, 1e-300))))
                ds = np.abs(out["sums"] - gold["sums"][k])
                ds[:3] /= np.abs(gold["sums"][k][:3])
                ds[3] /= float(gold["j_el"]) * area
                se = np.maximum(se, ds)
            err = {"rel_l2_per_field": [float(f"{x:.2e}") for x in fe], "U_cell_rel": float(f"{ue:.2e}"),
                   "means_rel": float(f"{me:.2e}"), "sums_rel": [float(f"{x:.2e}") for x in se]}
        res[inner] = (wall, u, its, err)
    rel = [float(torch.linalg.norm(res["f32"][1][f] - res["f64"][1][f]) /
                 torch.clamp(torch.linalg.norm(res["f64"][1][f]), min=1e-300)) for f in range(9)]
    log(f"[bench] five 16^3 steps: f64 {res['f64'][0]:.3f} s, mixed {res['f32'][0]:.3f} s")
    ctx.close()
    return {"workload": f"cube16_q1: 16^3 voxels, 0.1C, 5 backward-Euler steps of 0.1 s from {start}",
            "s_f64": round(res["f64"][0], 4), "s_mixed": round(res["f32"][0], 4),
            "mixed_speedup": round(res["f64"][0] / res["f32"][0], 3),
            "newton_gmres_f64": res["f64"][2], "newton_gmres_mixed": res["f32"][2],
            "error_vs_oracle_f64": res["f64"][3], "error_vs_oracle_mixed": res["f32"][3],
            "rel_l2_mixed_vs_f64": [float(f"{x:.2e}") for x in rel]}


def discharge(workload, f_C, inner, coarse, coarse_agg, log, dt0=0.1, cutoff=1.9, max_steps=5000, limiter=0,
              max_wall=None, t_stop=None):
    """Full galvanostatic discharge under the naive controller (Sec. 2.8):
    from the initial state until U_cell <= cutoff or t >= 3600 / f_C
    (limiter = 1: every step's root limited, dg_limit; max_wall: stop after
    that many seconds, reported as ended_by "wall"; t_stop: stop once the
    simulated time reaches it, ended_by "t_stop")."""
    import torch
    import synth
    from paper_2511_05233_amd import lsbdg
    w = synth.WORKLOADS[workload]
    D0, i0 = synth.sample_transport_kinetics(w.param_seed)
    ctx = lsbdg.Context(w.nx, w.ny, w.nz, w.h, w.order, w.mask(), D0=D0, kE=i0 / FARADAY, f_C=f_C)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    u, _ = ctx.initial_state(inner=inner, coarse=coarse, coarse_agg=coarse_agg, **SOLVER_EXTRA)
    ctrl = lsbdg.controller("naive", dt0=dt0)
    t, t_end = 0.0, 3600.0 / f_C
    tot = {"steps": 0, "trials": 0, "halvings": 0, "newton_its": 0, "gmres_its": 0}
    U = ctx.outputs(u, t)["U_cell"]
    curve = [(0.0, U, time.perf_counter() - w0)]
    while t < t_end and U > cutoff and tot["steps"] < max_steps:
        if max_wall is not None and time.perf_counter() - w0 > max_wall:
            break
        if t_stop is not None and t >= t_stop:
            break
        t, rep = ctx.advance(ctrl, t, u, inner=inner, coarse=coarse, coarse_agg=coarse_agg, limiter=limiter,
                             **SOLVER_EXTRA)
        for k in ("trials", "halvings", "newton_its", "gmres_its"):
            tot[k] += rep[k]
        tot["steps"] += 1
        U = ctx.outputs(u, t)["U_cell"]
        curve.append((t, U, time.perf_counter() - w0))
        log(f"[discharge] step {tot['steps']}: t = {t:.4g} s, dt = {rep['dt']:.3g} s, U_cell = {U:.5f} V, "
            f"{rep['newton_its']} Newton, {rep['gmres_its']} GMRES, wall {curve[-1][2]:.1f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    soc = 1.0 - t / t_end
    return {"workload": f"{workload} at {f_C}C", "s_per_discharge": round(wall, 2), "t_end_s": round(t, 3),
            "U_end_V": round(U, 5), "soc_end": round(soc, 4), **tot,
            "limiter": limiter,
            "ended_by": "cutoff" if U <= cutoff else ("time" if t >= t_end else
                                                      ("t_stop" if t_stop is not None and t >= t_stop else
                                                       ("step limit" if tot["steps"] >= max_steps else "wall"))),
            "curve_tU": [(round(a, 3), round(b, 6)) for a, b, _ in curve[:: max(1, len(curve) // 40)]],
            "_curve": curve}


def discharge_mixed_vs_f64(workload, f_C, coarse, coarse_agg, log):
    """The same full discharge with FP64 and with mixed (FP32 inner) solves:
    wall time of each and the largest cell-voltage difference between the
    two discharge curves (at the accepted step times of the FP64 run)."""
    runs = {}
    for inner in ("f64", "f32"):
        runs[inner] = discharge(workload, f_C, inner, coarse, coarse_agg, log)
        log(f"[bench] discharge {workload} {inner}: {runs[inner]['s_per_discharge']} s")
    c64 = np.array(runs["f64"]["_curve"])[:, :2]
    c32 = np.array(runs["f32"]["_curve"])[:, :2]
    t_hi = min(c64[-1, 0], c32[-1, 0])
    sel = c64[:, 0] <= t_hi
    dU = np.abs(np.interp(c64[sel, 0], c32[:, 0], c32[:, 1]) - c64[sel, 1])
    strip = lambda r: {k: v for k, v in r.items() if k not in ("_curve", "curve_tU")}
    return {"workload": f"{workload} at {f_C}C, naive controller from the initial state to the 1.9 V cutoff",
            "s_f64": runs["f64"]["s_per_discharge"], "s_mixed": runs["f32"]["s_per_discharge"],
            "mixed_speedup": round(runs["f64"]["s_per_discharge"] / runs["f32"]["s_per_discharge"], 3),
            "max_abs_dU_cell_V": float(f"{dU.max():.3e}"),
            "f64": strip(runs["f64"]), "mixed": strip(runs["f32"])}


def batch_throughput(dev, log, n=64, reps=10, t=0.1, dt=0.1, full=True, solves=False):
    """Batching on the batch workload: n cubic structures with
    edges ~ U{24..64} voxels and porosities ~ U(0.4, 0.75) (seeded), each
    with its own kinetics draw.  Every operator runs as one launch over all
    structures; the same work as one launch per structure is timed beside
    it, eagerly and replayed from a captured graph."""
    import torch
    import synth
    from paper_2511_05233_amd import lsbdg
    specs = synth.batch_structures(n)
    structs, ctxs, parts = [], [], []
    for b, (edge, por, mseed) in enumerate(specs):
        mask = synth.porosity_mask((edge, edge, edge), por, mseed)
        D0, i0 = synth.sample_transport_kinetics(b)
        kw = dict(D0=D0, kE=i0 / FARADAY, f_C=0.1)
        structs.append(dict(nx=edge, ny=edge, nz=edge, h=1e-6, phase=mask, **kw))
        ctx = lsbdg.Context(edge, edge, edge, 1e-6, 1, mask, **kw)
        ctxs.append(ctx)
        parts.append(random_state(ctx, mask, 100 + b, dev))
    B = lsbdg.Batch(structs)
    E = B.n_elem
    log(f"[bench] batch: {n} structures, {E} voxels, {B.n_tiles} tiles")
    u64 = torch.cat(parts, dim=1)
    del parts
    u32 = u64.float()
    g = torch.Generator(device=dev).manual_seed(11)
    v7 = torch.randn((7, E, 8), generator=g, dtype=torch.float32, device=dev)
    y7 = torch.empty_like(v7)
    m8 = B.mass(u64)
    r9 = torch.empty_like(u64)
    tt = [t] * n
    dd = [dt] * n
    stream = torch.cuda.current_stream()
    # one launch over the whole batch
    B.linearize(u32, tt, dd)
    ms_jvp_b = time_launches(lambda: B.jvp(u32, v7, tt, dd, out=y7, linearized=True), stream, reps)
    ms_res_b = time_launches(lambda: B.residual(u64, m8, tt, dd, out=r9), stream, reps)
    # the same work, one launch per structure (contiguous per-structure copies)
    us32 = [B.part(u32, s).contiguous() for s in range(n)]
    us64 = [B.part(u64, s).contiguous() for s in range(n)]
    vs = [B.part(v7, s).contiguous() for s in range(n)]
    ys = [torch.empty_like(x) for x in vs]
    ms8 = [B.part(m8, s).contiguous() for s in range(n)]
    rs = [torch.empty_like(x) for x in us64]
    for s, c in enumerate(ctxs):
        c.linearize(us32[s], t, dt)

    def seq_jvp():
        for s, c in enumerate(ctxs):
            c.jvp(us32[s], vs[s], t, dt, out=ys[s], linearized=True)

    def seq_res():
        for s, c in enumerate(ctxs):
            c.residual(us64[s], ms8[s], t, dt, out=rs[s])

    ms_jvp_s = time_launches(seq_jvp, stream, reps)
    ms_res_s = time_launches(seq_res, stream, reps)
    def rel(a, b):
        return float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))

    diff_jvp = max(rel(B.part(y7, s), ys[s]) for s in range(n))
    diff_res = max(rel(B.part(r9, s), rs[s]) for s in range(n))
    # the per-structure launches replayed from a captured graph (the
    # product's outputs are compared with the eager ones after the replays)
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        seq_jvp()
    stream.wait_stream(side)
    with torch.cuda.graph(graph):
        seq_jvp()
    ref = [y.clone() for y in ys]
    ms_jvp_g = time_launches(graph.replay, stream, reps)
    graph_same = all(torch.equal(ys[s], ref[s]) for s in range(n))
    del graph
    # the autotuner: every launch shape of the residual and both tangents in
    # FP32 (the Krylov operator) and FP64 (the Newton residual), then the
    # batched calls again in the chosen shapes (same values as before)
    y_def, r_def = y7.clone(), r9.clone()
    v9 = torch.randn((9, E, 8), generator=g, dtype=torch.float32, device=dev)
    tune32, ncand = B.autotune(u32, v9, m8.float(), tt, dd, reps=reps)
    v9 = v9.double()
    tune64, _ = B.autotune(u64, v9, m8, tt, dd, reps=reps)
    del v9
    torch.cuda.empty_cache()
    B.linearize(u32, tt, dd)
    ms_jvp_t = time_launches(lambda: B.jvp(u32, v7, tt, dd, out=y7, linearized=True), stream, reps)
    ms_res_t = time_launches(lambda: B.residual(u64, m8, tt, dd, out=r9), stream, reps)
    tuned_same = bool(torch.equal(y7, y_def) and torch.equal(r9, r_def))
    del y_def, r_def

    def tuned(tune):
        return {op: {"shape": {"tile_voxels": sh[0], "persistent_per_cu": sh[1]}, "ms": round(ms, 3),
                     "ms_default": round(md, 3)} for op, (sh, ms, md) in tune.items()}

    autotune = {"shapes_per_operator": ncand, "f32": tuned(tune32), "f64": tuned(tune64),
                "jvp_f32_ms_tuned": round(ms_jvp_t, 3), "residual_f64_ms_tuned": round(ms_res_t, 3),
                "tuned_equals_default": tuned_same}
    log(f"[bench] batch autotune: JVP {ms_jvp_t:.3f} ms in {tune32['jvp_condensed'][0]}, residual "
        f"{ms_res_t:.3f} ms in {tune64['residual'][0]}")
    dof = E * 56
    b_apply = E * (56 * 56 + 2 * 56) * 4
    ms_setup_b = ms_apply_b = None
    if full:
        # batched block preconditioner (E blocks of 56 x 56 in FP32)
        ms_setup_b = time_launches(lambda: B.blockjacobi_setup(u32, tt, dd), stream, 1)
        ms_apply_b = time_launches(lambda: B.blockjacobi_apply(v7, out=y7), stream, reps)
    for c in ctxs:
        c.close()
    B.close()
    del u32, v7, y7, m8, r9, us32, us64, vs, ys, ms8, rs, ref
    torch.cuda.empty_cache()
    del u64
    torch.cuda.empty_cache()
    solve = batch_solves(structs, dof, log) if (full or solves) else None
    res = {
        "workload": f"{n} cubic structures, edges U{{24..64}} voxels, porosity U(0.4, 0.75), DG-Q1, "
                    f"{E} voxels, {dof} DoF; residual in {B.n_tiles} tiles of 32 voxels, "
                    f"Krylov operator on bricks of 4^3 voxels (its default shape)",
        "jvp_f32_ms": {"batched": round(ms_jvp_b, 3), "per_structure": round(ms_jvp_s, 3),
                       "per_structure_graph": round(ms_jvp_g, 3)},
        "jvp_f32_gdofs": {"batched": round(dof / ms_jvp_b / 1e6, 2),
                          "per_structure": round(dof / ms_jvp_s / 1e6, 2),
                          "per_structure_graph": round(dof / ms_jvp_g / 1e6, 2)},
        "residual_f64_ms": {"batched": round(ms_res_b, 3), "per_structure": round(ms_res_s, 3)},
        "batched_speedup_jvp": round(ms_jvp_s / ms_jvp_b, 3),
        "batched_speedup_residual": round(ms_res_s / ms_res_b, 3),
        "block_setup_f32_ms": round(ms_setup_b, 1) if full else None,
        "block_apply_f32": {"ms": round(ms_apply_b, 3), "GB/s": round(b_apply / ms_apply_b / 1e6, 1),
                            "frac": round(b_apply / ms_apply_b / 1e6 / HBM_PEAK_GBS, 4)} if full else None,
        "max_rel_diff_batched_vs_per_structure": {"jvp_f32": float(f"{diff_jvp:.3e}"),
                                                  "residual_f64": float(f"{diff_res:.3e}")},
        "graph_replay_equals_eager": bool(graph_same),
        "autotune": autotune,
        "implicit_step": solve,
    }
    if not full:
        for k in ("block_setup_f32_ms", "block_apply_f32") + (() if solves else ("implicit_step",)):
            res.pop(k)
    log(f"[bench] batch: JVP {ms_jvp_b:.3f} ms batched, {ms_jvp_s:.3f} ms per structure, "
        f"{ms_jvp_g:.3f} ms per structure from a graph")
    return res


def batch_solves(structs, dof, log, dt=0.1, iters=2):
    """The solver on the batch, FP32 inner solves: initial states of every
    structure, then `iters` Newton iterations of the first implicit step
    (dt) of every structure (the step definition of the main benchmark),
    with the structures' solves one after another (one worker: the
    sequential solves) and side by side (four workers, one HIP stream
    each), from the same initial states."""
    import torch
    from paper_2511_05233_amd import lsbdg
    B = lsbdg.Batch(structs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, reps0 = B.initial_state(inner="f32", workers=4)
    torch.cuda.synchronize()
    s_init = time.perf_counter() - t0
    log(f"[bench] batch: initial states in {s_init:.2f} s (four workers)")
    runs = {}
    for workers in (4, 1):
        uw = u.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            reps = B.step(uw, 0.0, dt, inner="f32", workers=workers, newton_maxit=iters)
        except lsbdg.DgError as e:      # capped at `iters` iterations: not converged, by design
            reps = e.reports
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        runs[workers] = (wall, uw, reps)
        log(f"[bench] batch: {iters} Newton iterations of every structure in {wall:.2f} s with {workers} worker(s)")
    same = torch.equal(runs[1][1], runs[4][1])
    reps = runs[4][2]
    B.close()
    its = sum(r["newton_its"] for r in reps)
    return {"dt_s": dt, "inner": "f32", "newton_iterations_per_structure": iters,
            "initial_states_s": round(s_init, 2),
            "initial_state_newton_its": sum(r["newton_its"] for r in reps0),
            "s_sequential": round(runs[1][0], 2), "s_side_by_side_4": round(runs[4][0], 2),
            "speedup": round(runs[1][0] / runs[4][0], 3),
            "gdof_newton_its_per_s": {"sequential": round(dof * iters / runs[1][0] / 1e9, 3),
                                      "side_by_side_4": round(dof * iters / runs[4][0] / 1e9, 3)},
            "newton_its": its, "gmres_its": sum(r["gmres_its"] for r in reps),
            "side_by_side_equals_sequential": bool(same)}


def controller_study(nx, f_C, log, max_wall=240.0, cutoff=1.9, inner="f64", limiter=0, only=None):
    """The time-stepping comparison of Sec. 3.3 on a one-dimensional
    homogenised cathode: nx voxels of 1 um, every voxel structure (the
    porous cathode of Tab. 5 through Eq. 57), the paper's parameters, the
    current on the separator face.  Strategies: backward Euler with a fixed
    dt = 0.1 s (halving only on a failed solve), the naive controller, and
    H211b at tol = 1e-8 and 1e-5; each from the initial state to the 1.9 V
    cutoff, the end of the nominal discharge or max_wall seconds.  Reports
    wall time, step, Newton and GMRES counts, the device workspace each
    strategy needs (dg_workspace_bytes: one or three saved states), and the
    largest cell-voltage difference to the naive run at common times."""
    import torch
    from paper_2511_05233_amd import lsbdg
    mask = np.ones((1, 1, nx), np.uint8)
    kinds = [("backward_euler_dt0.1", "naive", None), ("naive", "naive", None),
             ("h211b_tol1e-8", "h211b", 1e-8), ("h211b_tol1e-5", "h211b", 1e-5)]
    out = {"workload": f"{nx}x1x1 voxels of 1 um, all structure (homogenised), DG-Q1, paper parameters, "
                       f"{f_C}C, inner {inner}", "strategies": {}}
    curves = {}
    t_end = 3600.0 / f_C
    out["limiter"] = limiter
    for name, kind, tol in kinds:
        if only and name not in only:
            continue
        ctx = lsbdg.Context(nx, 1, 1, 1e-6, 1, mask, f_C=f_C)
        feats = lsbdg.DG_WS_STEP | (lsbdg.DG_WS_H211B if kind == "h211b" else lsbdg.DG_WS_NAIVE)
        ws = lsbdg.workspace_bytes(nx, 1, 1, 1e-6, 1, feats, inner=inner)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        u, _ = ctx.initial_state(inner=inner)
        c = lsbdg.controller(kind, dt0=0.1, tol=tol if tol else 1e-5)
        if name.startswith("backward_euler"):
            c.successes = 2 ** 30                 # dt never grows
        t, U = 0.0, ctx.outputs(u, 0.0)["U_cell"]
        tot = {"steps": 0, "trials": 0, "halvings": 0, "newton_its": 0, "gmres_its": 0}
        curve = [(0.0, U)]
        ended = "wall"
        last_log = time.perf_counter()
        while time.perf_counter() - w0 < max_wall:
            if time.perf_counter() - last_log > 30.0:
                log(f"[study] {name}: {tot['steps']} steps, t = {t:.4g} s, U_cell = {U:.4f} V")
                last_log = time.perf_counter()
            if U <= cutoff:
                ended = "cutoff"
                break
            if t >= t_end:
                ended = "time"
                break
            try:
                t, rep = ctx.advance(c, t, u, inner=inner, limiter=limiter)
            except lsbdg.DgError as e:
                ended = f"failed ({e.code})"
                break
            for k in ("trials", "halvings", "newton_its", "gmres_its"):
                tot[k] += rep[k]
            tot["steps"] += 1
            U = ctx.outputs(u, t)["U_cell"]
            curve.append((t, U))
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        ctx.close()
        curves[name] = np.array(curve)
        out["strategies"][name] = {"wall_s": round(wall, 2), "t_end_s": round(t, 3), "U_end_V": round(U, 5),
                                   "ended_by": ended, "workspace_bytes": ws, **tot}
        log(f"[study] {name}: {tot['steps']} steps to t = {t:.4g} s in {wall:.1f} s ({ended})")
    ref = curves.get("naive")
    for name, cv in curves.items():
        if ref is None:
            break
        hi = min(cv[-1, 0], ref[-1, 0])
        sel = (cv[:, 0] > 0) & (cv[:, 0] <= hi)
        if sel.any():
            dU = np.abs(cv[sel, 1] - np.interp(cv[sel, 0], ref[:, 0], ref[:, 1]))
            out["strategies"][name]["max_abs_dU_vs_naive_V"] = float(f"{dU.max():.3e}")
    return out


def run_steps(ctx, ctrl, u, t, n, inner, log, verbose=0, coarse=0, coarse_agg=0):
    """n accepted steps of the naive controller (halving on failed solves)."""
    tot = {"newton_its": 0, "gmres_its": 0, "trials": 0, "halvings": 0}
    for _ in range(n):
        t, rep = ctx.advance(ctrl, t, u, inner=inner, verbose=verbose, coarse=coarse, coarse_agg=coarse_agg,
                             **SOLVER_EXTRA)
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
    ap.add_argument("--mode", default="newton", choices=["newton", "controller"])
    ap.add_argument("--dt", type=float, default=0.1, help="first trial step [s]")
    ap.add_argument("--inner", default="f32", choices=["f32", "f64"])
    ap.add_argument("--coarse", type=int, default=0,
                    help="preconditioner coarse space (0: library default = 3, 1: global constants, "
                         "3: voxel aggregates, additive, 4: multiplicative)")
    ap.add_argument("--coarse-agg", type=int, default=0, help="aggregate edge in voxels (0: automatic)")
    ap.add_argument("--fp32-blocks", action="store_true",
                    help="stream the element-block inverses in FP32 in GMRES (default: a bfloat16 copy)")
    ap.add_argument("--workload", default="slab96_q1")
    ap.add_argument("--compare-f64", action="store_true",
                    help="repeat the timed steps with an FP64 inner solve from the same state")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-vs-FP64 comparisons on the 16^3 cube (5 steps and a full 1C discharge)")
    ap.add_argument("--verbose", type=int, default=0, help="Newton progress lines on stderr")
    ap.add_argument("--kernels-only", action="store_true",
                    help="profiling aid: skip the solves and time the kernels alone on a seeded "
                         "random state (prints the kernel table, not the benchmark line)")
    ap.add_argument("--discharge", default=None, metavar="WORKLOAD",
                    help="run one full discharge of WORKLOAD (naive controller, cutoff 1.9 V) and print "
                         "its wall time instead of the benchmark line")
    ap.add_argument("--discharge-rate", type=float, default=1.0, help="C-rate of --discharge")
    ap.add_argument("--limiter", action="store_true",
                    help="--discharge, --controller-study: limit every step's root (dg_limit)")
    ap.add_argument("--max-wall", type=float, default=None, help="--discharge: stop after this many seconds")
    ap.add_argument("--t-stop", type=float, default=None, help="--discharge: stop at this simulated time [s]")
    ap.add_argument("--strategies", default=None,
                    help="--controller-study: comma-separated subset of backward_euler_dt0.1, naive, "
                         "h211b_tol1e-8, h211b_tol1e-5")
    ap.add_argument("--controller-study", nargs=2, metavar=("NX", "F_C"), default=None,
                    help="the time-stepping comparison (backward Euler, naive, H211b at 1e-8 and 1e-5) on an "
                         "NX x 1 x 1 homogenised cathode at F_C (per hour); --max-wall caps each strategy")
    ap.add_argument("--batch", action="store_true",
                    help="the 64-structure batch workload in full (operators, block preconditioner, "
                         "side-by-side solves) and print that record only")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-operator record of the default line")
    ap.add_argument("--step-only", action="store_true",
                    help="time the steps only (no kernel timings, comparisons or baselines): "
                         "the run a kernel trace of the timed step is taken on")
    ap.add_argument("--mg-levels", type=int, default=None,
                    help="coarse solve by a V-cycle over this many aggregate levels (2..8; level-1 edge "
                         "--coarse-agg, 0: 4); 0: the exact two-level solve; default: the library's "
                         "automatic choice")
    ap.add_argument("--mg-sweeps", type=int, default=None,
                    help="block-Jacobi sweeps per level of the V-cycle (default: the library's)")
    ap.add_argument("--block-reuse", type=float, default=None,
                    help="keep the element blocks while Newton updates stay below this relative size")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--oracle-timing", nargs=2, metavar=("WORKLOAD", "SECONDS"), default=None,
                    help=argparse.SUPPRESS)
    args = ap.parse_args(argv)
    if args.oracle_timing:
        print(json.dumps(_oracle_timing(args.oracle_timing[0], float(args.oracle_timing[1]))), flush=True)
        return 0
    if args.fp32_blocks:
        SOLVER_EXTRA["block_bf16"] = 0
    if args.mg_levels is not None:
        SOLVER_EXTRA["mg_levels"] = args.mg_levels
    if args.mg_sweeps is not None:
        SOLVER_EXTRA["mg_sweeps"] = args.mg_sweeps
    if args.block_reuse is not None:
        SOLVER_EXTRA["block_reuse"] = args.block_reuse
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; "
              "run with --gpus 1.", file=sys.stderr)
        return 2

    import torch
    import synth
    from paper_2511_05233_amd import lsbdg

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.batch:
        print(json.dumps(batch_throughput(torch.device("cuda:0"), log)), flush=True)
        return 0
    if args.controller_study:
        nx, fc = args.controller_study
        print(json.dumps(controller_study(int(nx), float(fc), log, max_wall=args.max_wall or 240.0,
                                          limiter=int(args.limiter),
                                          only=args.strategies.split(",") if args.strategies else None)), flush=True)
        return 0
    if args.discharge:
        out = discharge(args.discharge, args.discharge_rate, args.inner, args.coarse, args.coarse_agg, log,
                        limiter=int(args.limiter), max_wall=args.max_wall, t_stop=args.t_stop)
        out["curve_tUw"] = [(round(a, 4), round(b, 7), round(c, 2)) for a, b, c in out.pop("_curve")]
        print(json.dumps(out), flush=True)
        return 0
    w = synth.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    mask = w.mask()
    D0, i0 = synth.sample_transport_kinetics(w.param_seed)
    ctx = lsbdg.Context(w.nx, w.ny, w.nz, w.h, w.order, mask, D0=D0, kE=i0 / FARADAY, f_C=w.f_C)
    stream = torch.cuda.current_stream()
    n_dof = ctx.n_elem * ctx.n_nodes * 7
    nodes = ctx.n_elem * ctx.n_nodes

    if args.kernels_only:
        u = random_state(ctx, mask, 1, dev)
        t = 0.5
        kernels, _ = time_kernels(ctx, u, t, args.dt, args.inner, stream, dev, log)
        out = {"workload": w.name, "inner": args.inner, "kernels": kernels}
        if args.copy_probe:
            out["copy_probe_bytes"] = copy_probe(dev)
        print(json.dumps(out), flush=True)
        return 0
    u, rep0 = ctx.initial_state(inner=args.inner, verbose=args.verbose, coarse=args.coarse,
                                coarse_agg=args.coarse_agg, **SOLVER_EXTRA)
    log(f"[bench] initial state: {rep0['newton_its']} Newton, {rep0['gmres_its']} GMRES")
    t = 0.0
    if args.mode == "newton":
        # warm-up on a copy: the timed iterations start from the step's own
        # initial iterate (the old mass of the step is that of u)
        newton_iterations(ctx, u.clone(), t, args.dt, args.warmup, args.inner, log, args.verbose, args.coarse,
                          args.coarse_agg)
        u_start = u.clone() if args.compare_f64 else None
        t_start = t
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        clocks0 = (time.monotonic_ns(), time.clock_gettime_ns(time.CLOCK_BOOTTIME))
        tot = {"newton_its": 0, "gmres_its": 0, "implicit_steps": 0}
        while tot["newton_its"] < args.steps:
            # a step that converges before the count is reached hands over
            # to the next implicit step (t + dt, old mass of the new root)
            rep = newton_iterations(ctx, u, t, args.dt, args.steps - tot["newton_its"], args.inner, log,
                                    args.verbose, args.coarse, args.coarse_agg)
            tot["newton_its"] += rep["newton_its"]
            tot["gmres_its"] += rep["gmres_its"]
            tot["implicit_steps"] += 1
            tot["mg_levels_used"] = rep.get("mg_levels", 0)
            if rep["newton_its"] < 1:
                break
            if rep.get("converged"):
                t += args.dt
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        clocks1 = (time.monotonic_ns(), time.clock_gettime_ns(time.CLOCK_BOOTTIME))
        done = max(tot["newton_its"], 1)
        ms_step = wall * 1e3 / done
    else:
        ctrl = lsbdg.controller("naive", dt0=args.dt)
        t, _ = run_steps(ctx, ctrl, u, t, args.warmup, args.inner, log, args.verbose, args.coarse, args.coarse_agg)
        u_start = u.clone() if args.compare_f64 else None
        ctrl_start = lsbdg.DgController.from_buffer_copy(ctrl)
        t_start = t
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        t, tot = run_steps(ctx, ctrl, u, t, args.steps, args.inner, log, args.verbose, args.coarse, args.coarse_agg)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        done = args.steps
        ms_step = wall * 1e3 / args.steps

    if args.step_only:
        # the timed region's clock readings let a kernel trace be cut to it
        extra = {"timed_ns": {"monotonic": [clocks0[0], clocks1[0]], "boottime": [clocks0[1], clocks1[1]]}} \
            if args.mode == "newton" else {}
        print(json.dumps({"workload": w.name, "inner": args.inner, "mode": args.mode, "steps": done,
                          "warmup": args.warmup, "ms_per_step": round(ms_step, 2), **tot, **extra}), flush=True)
        return 0
    kernels, (k_op, b_op, ms_op) = time_kernels(ctx, u, t, args.dt, args.inner, stream, dev, log)
    achieved = b_op / (ms_op * 1e-3) / 1e9
    triad = triad_bandwidth(dev, stream)
    out = {
        "metric": METRIC,
        "value": round(n_dof / (kernels["jvp_condensed"]["ms"] * 1e-3) / 1e9, 3),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": done,
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
                   "dof": n_dof, "dt_s": args.dt, "t_start_s": round(t_start, 6),
                   "step": ("Newton iteration of the implicit steps from the initial state (the next step "
                            "starts when one converges): FP64 residual, linearisation, "
                            "block-Jacobi setup, GMRES(30) with block-Jacobi and coarse correction, "
                            "FP64 update" if args.mode == "newton" else
                            "accepted step of the naive time controller (backward-Euler Newton-GMRES "
                            "solves, halving dt on failure)"),
                   "coarse": args.coarse, "coarse_agg": args.coarse_agg, "mg_levels": "auto" if args.mg_levels is None else args.mg_levels,
                   "mg_sweeps": "library default" if args.mg_sweeps is None else args.mg_sweeps, "timed_steps": done, **{k: v for k, v in tot.items()}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": recorded_traffic(w.name, k_op),
                     "kernel": k_op, "ms": round(ms_op, 4),
                     "bytes_per_launch": b_op,
                     "bytes_per_dof": round(b_op / n_dof, 2),
                     "achievable_triad": triad,
                     "frac_of_triad": round(achieved / triad["GB/s"], 4),
                     "residual_f64": {k: kernels["residual_f64"][k] for k in ("ms", "GB/s", "frac", "bytes")},
                     "valu": valu_view(w.name, k_op, ms_op)},
        "kernels": kernels,
    }
    if args.compare_f64 and args.inner == "f32":
        u64 = u_start.clone()
        torch.cuda.synchronize()
        w1 = time.perf_counter()
        if args.mode == "newton":
            rep64 = newton_iterations(ctx, u64, t_start, args.dt, args.steps, "f64", log, args.verbose, args.coarse, args.coarse_agg)
            tot64 = {"newton_its": rep64["newton_its"], "gmres_its": rep64["gmres_its"]}
        else:
            ctrl64 = lsbdg.DgController.from_buffer_copy(ctrl_start)
            _, tot64 = run_steps(ctx, ctrl64, u64, t_start, args.steps, "f64", log, args.verbose, args.coarse, args.coarse_agg)
        torch.cuda.synchronize()
        wall64 = time.perf_counter() - w1
        rel = [float(torch.linalg.norm(u[f] - u64[f]) / torch.clamp(torch.linalg.norm(u64[f]), min=1e-300))
               for f in range(9)]
        out["f64_inner"] = {"ms_per_step": round(wall64 * 1e3 / max(tot64["newton_its"] if args.mode == "newton"
                                                                   else args.steps, 1), 2),
                            "newton_its": tot64["newton_its"], "gmres_its": tot64["gmres_its"],
                            "mixed_speedup": round(wall64 / wall, 3),
                            "rel_l2_mixed_vs_f64": [float(f"{x:.3e}") for x in rel]}
    if not args.no_mixed:
        out["mixed_vs_f64"] = mixed_vs_f64(args.coarse, log)
        out["discharge_mixed_vs_f64"] = discharge_mixed_vs_f64("cube16_q1", 1.0, args.coarse, 0, log)
    if not args.no_batch:
        ctx.close()
        torch.cuda.empty_cache()
        out["batch_operators"] = batch_throughput(dev, log, full=False, solves=True)
    if args.copy_probe:
        out["copy_probe_bytes"] = copy_probe(dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
