"""Write the oracle's 16^3 trajectory: initial state plus five backward-Euler steps.

Workload: 16^3 voxels of 1 um, DG-Q1, porosity 0.6 (mask seed 0), transport
and kinetics of parameter seed 0, 0.1C current on the separator face; the
steady initial potential (Sec. 2.10, solved directly) and then five steps of
dt = 0.1 s (the paper's implicit-Euler step of the time-stepping study,
Sec. 3.3), each solved by the oracle's Newton iteration to a relative update
below 1e-12 (its linear systems by GMRES on the probed sparse Jacobian,
its multiplicative update capped at a factor 10 both ways).
Every value is computed by the CPU oracle alone (``oracle/``); nothing here
touches the HIP library.

Output: ``cube16_q1_trajectory.npz`` beside this script (float64 arrays,
no pickled objects): ``u`` of shape (6, 9, 4096, 8) -- the initial state and
the five step roots --, the times ``t`` and, per state, the oracle's cell
voltage, volume means and conservation sums.

Run from the repository root:  python tests/golden/make_cube16_trajectory.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import model as om  # noqa: E402
from oracle import outputs as oout  # noqa: E402
from oracle import solve as osolve  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cube16_q1_trajectory.npz")
DT = 0.1
STEPS = 5


def problem():
    w = synth.WORKLOADS["cube16_q1"]
    mask = w.mask()
    D0, i0 = synth.sample_transport_kinetics(w.param_seed)
    return om.Problem(w.nx, w.ny, w.nz, w.h, w.order, mask, D0=D0, kE=i0 / om.F, f_C=w.f_C)


def main():
    P = problem()
    t0 = time.time()
    u, info = osolve.initial_state(P, log=lambda s: print("[init]", s, flush=True))
    print(f"initial state: {info} ({time.time() - t0:.0f} s)", flush=True)
    states, times = [u], [0.0]
    t = 0.0
    for s in range(STEPS):
        t1 = time.time()
        u, info = osolve.be_step(P, u, t, DT, linear="sparse", gmres_rtol=1e-8, restart=60, two_sided=True, maxit=150,
                                 log=lambda m: print(f"[step {s + 1}]", m, flush=True))
        t += DT
        states.append(u)
        times.append(t)
        print(f"step {s + 1}: {info} ({time.time() - t1:.0f} s)", flush=True)
    U = np.array([oout.cell_voltage(P, x) for x in states])
    means = np.array([np.concatenate([oout.volume_means(P, x)[0], [oout.volume_means(P, x)[1]]])
                      for x in states])
    sums = np.array([oout.invariants(P, x, tt) for x, tt in zip(states, times)])
    np.savez_compressed(OUT, u=np.stack(states), t=np.array(times), U_cell=U, means=means, sums=sums,
                        j_el=np.array(P.j_el), dt=np.array(DT))
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
