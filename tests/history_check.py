"""Comparison of the engine's per-step history with the FP64 oracle's.

Both histories have the rows [KE^n, W_E^n, P^{n+1/2}, K^{n+1/2}] (the
engine's layout in include/pic.h, the oracle's in ora_step).  The energies
are compared relative to the largest value of their column in the oracle's
history; the momentum, whose total is near zero for symmetric loads, relative
to the momentum scale m sum_p |v_p| of the initial velocities.

The bound of the FP32-state engine follows from the oracle itself: rounding
the state once to FP32 (as the engine stores it) changes the oracle's
history by some amount `sens` over a window of n steps; the engine rounds its
state once per step, and in the linear phase of an instability a rounding
made earlier is amplified at least as much as one made later, so its history
differs from the oracle's by at most (n + 1) sens.  Measured values sit at
about half of that (the rounding errors partly cancel).  The momentum total
is conserved by the scheme, so its roundings do not grow: they add up as a
random walk of the per-step rounding of the velocities,
6 sqrt((n + 1) np / 12) ulp(max|w|) (six standard deviations), plus twice the
oracle's own momentum drift over the window: the fixed-point deposit
truncates a weight that the gather uses unrounded (FP64 state), which breaks
the exact momentum balance of equal deposit and gather weights by up to 2^-32
per weight, on both sides alike.

Both sides also sum in FP64 in different orders (tile partials on the GPU,
particle order in the oracle): a sum of n terms differs by at most
n eps64 sum|terms| on each side, so every bound carries 2 np eps64 for the
particle sums (kinetic energies, momentum) and 2 ng eps64 for the field
energy.  This floor is what bounds the FP64-state engine's energies.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import oracle as O

COLS = ("KE", "W_E", "P", "K")


def momentum_scale(op, v) -> float:
    return O.particle_mass(op) * float(np.abs(np.asarray(v, dtype=np.float64)).sum())


def column_errors(h, ref, pscale):
    """Per-step errors of each history column, each relative to its scale."""
    h = np.asarray(h, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    out = {}
    for c, name in enumerate(COLS):
        scale = pscale if name == "P" else np.abs(ref[:, c]).max()
        out[name] = np.abs(h[:, c] - ref[:, c]) / scale
    return out


def stored_state(x, v, L, ng, dt, dtype):
    """The state the engine starts from, back in physical units: the stored
    position s = x/dx + 1/2 and velocity w = v dt/dx, each rounded once to the
    state precision `dtype` (a value that rounds up to ng + 1/2 is the point
    x = 0)."""
    dx = L / ng
    s = (np.asarray(x, dtype=np.float64) / dx + 0.5).astype(dtype)
    s = np.where(s < dtype(ng + 0.5), s, dtype(0.5))
    w = (np.asarray(v, dtype=np.float64) * (dt / dx)).astype(dtype)
    return (s.astype(np.float64) - 0.5) * dx, w.astype(np.float64) * (dx / dt)


def state_bounds(op, x, v, nsteps, windows, dtype=np.float32, mode=O.DEPOSIT_FIXED):
    """Bounds of the engine's history errors over each window (a number of
    leading steps), from the oracle's sensitivity to one rounding of the state
    to `dtype` (see the module docstring).  Returns {window: {column: bound}},
    the oracle's history from the FP64 inputs and the sensitivities."""
    ref = O.run(op, x, v, nsteps, mode=mode)["hist"]
    x1, v1 = stored_state(x, v, op.L, op.ng, op.dt, dtype)
    h1 = O.run(op, x1, v1, nsteps, mode=mode)["hist"]
    pscale = momentum_scale(op, v)
    sens = column_errors(h1, ref, pscale)
    dx = op.L / op.ng
    wmax = float(np.abs(v).max()) * op.dt / dx
    mant = 23 if dtype == np.float32 else 52
    ulp_w = 2.0 ** (math.floor(math.log2(wmax)) - mant) if wmax > 0 else 0.0
    sum_w = float(np.abs(v).sum()) * op.dt / dx
    eps64 = 2.0 ** -53
    floor = {"KE": 2 * op.np * eps64, "W_E": 2 * op.ng * eps64, "P": 2 * op.np * eps64, "K": 2 * op.np * eps64}
    out = {}
    for n in windows:
        b = {name: (n + 1) * float(sens[name][:n].max()) + floor[name] for name in COLS}
        drift = float(np.abs(ref[:n, 2] - ref[0, 2]).max()) / pscale
        b["P"] = 6 * math.sqrt((n + 1) * op.np / 12.0) * ulp_w / sum_w + 2 * drift + floor["P"]
        out[n] = b
    return out, ref, sens
