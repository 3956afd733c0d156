"""Adaptive time controllers as plain algorithms (oracle side).

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

Naive feedback controller (Sec. 2.8, Fig. 4): a success counter sct is
raised after every converged step; when it reaches 3 the step grows by 1.2
and sct restarts.  A failed solve halves the step and retries; more than 30
consecutive halvings abort the run.  Reading (the flowchart is not
available): a failure also resets sct, and steps are capped at dt_max
(the snapshot interval, 100 s).

H211b controller (Sec. 2.8, Eq. 51-54): each trial solves one coarse step
(dt) and two fine steps (dt/2); err = ||z_F - z_C||_2/||z_F||_2 over all
unknowns (reading of Eq. 53 as a ratio of l2 norms);
rho = (tol/err)^(1/4) (tol/err_prev)^(1/4) (dt/dt_prev)^(-1/4),
lim = 1 + atan(rho - 1).  lim starts at 0 in every step; the trial is
repeated while err > 1.02 tol or lim < 0.9, with dt <- min(lim, 0.9) dt
(reading: the flowchart is missing; a rejected trial never grows the step,
which the plain dt <- lim dt would do whenever the history factor pushes
lim above 1 while err is still too large, and the loop would not end).  On
acceptance z = 2 z_F - z_C (Richardson), the history shifts and the next
step is min(lim dt, dt_max).  A solver failure inside a trial halves dt as
in the naive controller.  Reading: before the first accepted step
err_prev = tol and dt_prev = dt.
"""
from __future__ import annotations

import math

import numpy as np


class SolverFailure(RuntimeError):
    """Raised by a step function whose nonlinear solve did not converge."""


class ControllerAbort(RuntimeError):
    pass


class Naive:
    def __init__(self, dt0, dt_max=100.0, grow=1.2, successes=3, max_halvings=30):
        self.dt = dt0
        self.dt_max = dt_max
        self.grow = grow
        self.successes = successes
        self.max_halvings = max_halvings
        self.sct = 0

    def advance(self, step_fn, z, t):
        """One accepted step: returns (z_new, t_new, dt_used)."""
        halvings = 0
        while True:
            dt = self.dt
            try:
                z_new = step_fn(z, t, dt)
            except SolverFailure:
                halvings += 1
                self.sct = 0
                if halvings > self.max_halvings:
                    raise ControllerAbort("more than %d halvings" % self.max_halvings)
                self.dt = dt / 2.0
                continue
            self.sct += 1
            if self.sct == self.successes:
                self.dt = min(dt * self.grow, self.dt_max)
                self.sct = 0
            return z_new, t + dt, dt


def relative_error(zF, zC):
    """Eq. 53 read as ||z_F - z_C||_2 / ||z_F||_2."""
    return float(np.linalg.norm(np.ravel(zF - zC)) / np.linalg.norm(np.ravel(zF)))


def h211b_limiter(err, err_prev, dt, dt_prev, tol):
    rho = (tol / err) ** 0.25 * (tol / err_prev) ** 0.25 * (dt / dt_prev) ** (-0.25)
    return 1.0 + math.atan(rho - 1.0)


class H211b:
    def __init__(self, dt0, tol, dt_max=100.0, max_halvings=30, err_floor=1e-300, max_rejections=100):
        self.dt = dt0
        self.max_rejections = max_rejections
        self.tol = tol
        self.dt_max = dt_max
        self.max_halvings = max_halvings
        self.err_prev = tol
        self.dt_prev = dt0
        self.err_floor = err_floor
        self.trials = 0

    def advance(self, step_fn, z, t):
        """One accepted step: returns (z_new, t_new, dt_used, err)."""
        lim = 0.0
        err = math.inf
        halvings = 0
        rejections = 0
        while lim < 0.9 or err > 1.02 * self.tol:
            dt = self.dt
            self.trials += 1
            try:
                zC = step_fn(z, t, dt)
                zh = step_fn(z, t, dt / 2.0)
                zF = step_fn(zh, t + dt / 2.0, dt / 2.0)
            except SolverFailure:
                halvings += 1
                if halvings > self.max_halvings:
                    raise ControllerAbort("more than %d halvings" % self.max_halvings)
                self.dt = dt / 2.0
                lim, err = 0.0, math.inf
                continue
            err = max(relative_error(zF, zC), self.err_floor)
            lim = h211b_limiter(err, self.err_prev, dt, self.dt_prev, self.tol)
            if lim < 0.9 or err > 1.02 * self.tol:
                self.dt = min(lim, 0.9) * dt
                # an error estimate with a floor above tol (the solver's
                # attainable accuracy) would otherwise shrink dt forever
                rejections += 1
                if rejections > self.max_rejections:
                    raise ControllerAbort("more than %d trials rejected by their error" % self.max_rejections)
        z_new = 2.0 * zF - zC
        self.err_prev = err
        self.dt_prev = dt
        self.dt = min(lim * dt, self.dt_max)
        return z_new, t + dt, dt, err
