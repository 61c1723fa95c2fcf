"""Seeded synthetic inputs for the 1D electrostatic PIC runs.

This module only *draws* initial conditions (positions, velocities, run
parameters, arrival schedules).  It contains none of the PIC method's
arithmetic (no weighting, field solve or push), so both the GPU engine and the
CPU oracle may consume what it produces.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): element ``i`` of stream ``s`` is
the SplitMix64 output for the counter ``base(seed, s) + (i + 1) * GAMMA``, so a
draw depends only on ``(seed, stream, i)`` and any slice can be regenerated.
Uniforms take the top 53 bits; normals use the Box-Muller transform.

The physical set-ups follow the paper's normalisation (Sec. 2 and Sec. 4):
plasma frequency 1, epsilon_0 = 1, electron charge-to-mass ratio -1, immobile
uniform ion background of density 1, periodic domain of length L.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Tuple

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 22


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _stream_base(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        s = _mix(np.array([(seed * 0x100000001B3 + stream * 0x9E37 + 1) & ((1 << 64) - 1)],
                          dtype=np.uint64))
    return s[0]


def splitmix64(seed: int, stream: int, start: int, n: int) -> np.ndarray:
    """Raw 64-bit outputs ``start .. start+n-1`` of stream ``stream``."""
    base = _stream_base(seed, stream)
    idx = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(base + idx * _GAMMA)


_POOL = None


def _chunks(n: int, fill: Callable[[int, int], None]) -> None:
    """Run fill(a, b) over [0, n) in chunks, on a thread pool for large n
    (each element depends only on its index, so the result does not depend
    on the number of threads)."""
    global _POOL
    spans = [(a, min(n, a + _CHUNK)) for a in range(0, n, _CHUNK)]
    if len(spans) <= 1:
        for a, b in spans:
            fill(a, b)
        return
    if _POOL is None:
        from concurrent.futures import ThreadPoolExecutor
        _POOL = ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1))
    list(_POOL.map(lambda ab: fill(*ab), spans))


def uniform(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) (53-bit), generated in chunks to bound memory."""
    out = np.empty(n, dtype=np.float64)

    def fill(a, b):
        r = splitmix64(seed, stream, start + a, b - a)
        out[a:b] = (r >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    _chunks(n, fill)
    return out


def normal(seed: int, stream: int, n: int) -> np.ndarray:
    """Standard normal deviates by Box-Muller from two uniform streams."""
    out = np.empty(n, dtype=np.float64)

    def fill(a, b):
        u1 = uniform(seed, stream, b - a, start=a)
        u2 = uniform(seed, stream + 1, b - a, start=a)
        out[a:b] = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * math.pi * u2)
    _chunks(n, fill)
    return out


def wrap_positions(x: np.ndarray, L: float) -> np.ndarray:
    """Bring loader positions into [0, L) (input preparation only)."""
    x = x - L * np.floor(x / L)
    x[x >= L] = 0.0
    return x


def lattice(n: int, L: float) -> np.ndarray:
    """Quiet-start positions (i + 1/2) L / n: with n a multiple of the cell
    count, n/ng particles at the centres of equal sub-intervals of every
    cell, the appendix's initial load."""
    return (np.arange(n) + 0.5) * (L / n)


def loaded(L: float, np_: int, seed: int, pos_stream: int = 0, vel_stream: int = 1, amp: float = 0.0,
           k: float = 0.0, v0: float = 0.0, vth: float = 0.0, beams: int = 0,
           lattice_start: bool = False) -> Tuple[np.ndarray, np.ndarray]:
    """The initial state a device-loader description stands for (the
    pic_loader fields): x0 uniform from `pos_stream` or the lattice,
    displaced by amp sin(k x0) and wrapped; v = s_i v0 + vth n_i with the
    beam sign s_i = 1 (beams 0), alternating by index (1), or + when the
    uniform of stream vel_stream + 2 is below 1/2 (2, the appendix's sign
    draw); normals from streams vel_stream, vel_stream + 1."""
    x0 = lattice(np_, L) if lattice_start else L * uniform(seed, pos_stream, np_)
    x = wrap_positions(x0 + amp * np.sin(k * x0) if amp != 0.0 else x0, L)
    del x0
    v = np.full(np_, float(v0))
    if beams == 1:
        v[1::2] = -float(v0)
    elif beams == 2:
        v[~(uniform(seed, vel_stream + 2, np_) < 0.5)] = -float(v0)
    if vth != 0.0:
        v += vth * normal(seed, vel_stream, np_)
    return x, v


@dataclass
class RunSpec:
    """One simulation run: parameters plus a lazily generated initial state.

    ``v`` is the velocity at t = -dt/2 (leapfrog half step, Sec. 2.1).
    """
    L: float
    ng: int
    np_: int
    dt: float
    nsteps: int
    qm: float = -1.0
    rho0: float = 1.0
    name: str = ""
    make: Optional[Callable[[], Tuple[np.ndarray, np.ndarray]]] = field(default=None, repr=False)
    # the same initial state as a device-loader description (pic_loader
    # fields), for the set-ups that are a uniform or single-mode-displaced
    # plasma with beams and a Maxwellian spread
    loader: Optional[dict] = None

    def particles(self) -> Tuple[np.ndarray, np.ndarray]:
        x, v = self.make()
        assert x.shape == (self.np_,) and v.shape == (self.np_,)
        return x, v

    def params(self) -> dict:
        return dict(L=self.L, ng=self.ng, np=self.np_, dt=self.dt, qm=self.qm, rho0=self.rho0)


def _beam_signs(n: int) -> np.ndarray:
    s = np.ones(n, dtype=np.float64)
    s[1::2] = -1.0
    return s


def random_phase_displacement(x0: np.ndarray, L: float, amp: float, nmodes: int,
                              seed: int, stream: int) -> np.ndarray:
    """Displacement amp * sum_{m=1..M} sin(2 pi m x0 / L + phi_m), phi_m ~ U[0, 2 pi).

    The M-mode sum is evaluated exactly on a periodic table of K = 64 M
    points and linearly interpolated at x0 (relative interpolation error
    below (2 pi / 64)^2 / 8 = 1.2e-3 of the displacement), which keeps the
    cost O(Np) for 10^8-particle inputs."""
    phi = 2.0 * math.pi * uniform(seed, stream, nmodes)
    K = 64 * max(1, nmodes)
    xt = np.arange(K + 1) * (L / K)
    k0 = 2.0 * math.pi / L
    table = np.zeros(K + 1)
    for m in range(1, nmodes + 1):
        table += np.sin(k0 * m * xt + phi[m - 1])
    table[K] = table[0]
    return amp * np.interp(x0, xt, table)


# --------------------------------------------------------------------------
# Workloads.  Each mirrors a configuration of the paper's kind of experiment:
# two counter-streaming electron beams (Sec. 4) or a warm Maxwellian plasma
# (Sec. 5.2), with seeded synthetic particles.
# --------------------------------------------------------------------------

def two_stream_small(seed: int = 1, np_: int = 10_000, nsteps: int = 200) -> RunSpec:
    """Cold two-stream run: L=2.053, Ng=64, Np=10,000, beams +-0.2, dt=0.1.

    Positions uniform from the seed, displaced by 1e-3 sin(2 pi x0 / L);
    beams interleaved by particle index.
    """
    L = 2.053
    k = 2.0 * math.pi / L

    def make():
        x0 = L * uniform(seed, 0, np_)
        x = wrap_positions(x0 + 1e-3 * np.sin(k * x0), L)
        v = 0.2 * _beam_signs(np_)
        return x, v
    return RunSpec(L=L, ng=64, np_=np_, dt=0.1, nsteps=nsteps, name="two_stream_ng64_np1e4", make=make,
                   loader=dict(seed=seed, pos_stream=0, vel_stream=1, amp=1e-3, k=k, v0=0.2, vth=0.0,
                               beams=1))


def warm_two_stream_large(seed: int = 2, np_: int = 1 << 26, ng: int = 4096,
                          nsteps: int = 1000, L: Optional[float] = None) -> RunSpec:
    """Warm two-stream run: L=2.053*64, Ng=4096, Np=2^26, v=+-0.2 + 0.01 N(0,1),
    random-phase displacement 1e-4 over M=min(128, Ng/2) modes, dt=0.1.
    Other sizes (and L) may be given for smaller cases of the same kind."""
    L = 2.053 * 64 if L is None else float(L)

    def make():
        x0 = L * uniform(seed, 0, np_)
        dx = random_phase_displacement(x0, L, 1e-4, min(128, ng // 2), seed, 5)
        x = wrap_positions(x0 + dx, L)
        v = 0.2 * _beam_signs(np_) + 0.01 * normal(seed, 1, np_)
        return x, v
    return RunSpec(L=L, ng=ng, np_=np_, dt=0.1, nsteps=nsteps,
                   name=f"warm_two_stream_ng{ng}_np{np_}", make=make)


def ensemble(nruns: int = 256, seed: int = 3, nsteps: int = 500,
             np_scale: float = 1.0, steps_range: Optional[Tuple[int, int]] = None) -> List[RunSpec]:
    """Batched ensemble: Np log-uniform in [1e4, 4e6], Ng = 64 * 2^floor(6U),
    L = 0.032 Ng, v0 ~ U[0.1, 0.3], vth ~ U[0, 0.02], random-phase 1e-4, dt=0.1.

    ``np_scale`` shrinks every run (for tests); ``steps_range`` draws the step
    count uniformly from the inclusive integer range (serving load)."""
    u = uniform(seed, 100, 6 * nruns).reshape(nruns, 6)
    runs = []
    for r in range(nruns):
        npr = int(round(math.exp(u[r, 0] * math.log(4e6 / 1e4)) * 1e4 * np_scale))
        npr = max(1, npr)
        ng = 64 * (1 << min(5, int(math.floor(6.0 * u[r, 1]))))
        L = 0.032 * ng
        v0 = 0.1 + 0.2 * u[r, 2]
        vth = 0.02 * u[r, 3]
        ns = nsteps
        if steps_range is not None:
            lo, hi = steps_range
            ns = lo + min(hi - lo, int(math.floor(u[r, 4] * (hi - lo + 1))))
        rseed = seed * 100003 + r

        def make(npr=npr, L=L, ng=ng, v0=v0, vth=vth, rseed=rseed):
            x0 = L * uniform(rseed, 0, npr)
            dx = random_phase_displacement(x0, L, 1e-4, min(128, ng // 2), rseed, 5)
            x = wrap_positions(x0 + dx, L)
            v = v0 * _beam_signs(npr) + vth * normal(rseed, 1, npr)
            return x, v
        runs.append(RunSpec(L=L, ng=ng, np_=npr, dt=0.1, nsteps=ns,
                            name=f"ens{r}_ng{ng}_np{npr}", make=make))
    return runs


def arrival_times(nruns: int, rate: float = 50.0, seed: int = 4) -> np.ndarray:
    """Poisson arrivals: cumulative exponential gaps with mean 1/rate seconds."""
    gaps = -np.log1p(-uniform(seed, 200, nruns)) / rate
    return np.cumsum(gaps)


def warm_maxwellian_large(seed: int = 5, np_: int = 1 << 28, ng: int = 8192,
                          nsteps: int = 2000) -> RunSpec:
    """Warm Maxwellian plasma: vth=0.1, L=(2 pi/0.5)*16, Ng=8192, Np=2^28,
    density perturbation 1e-2 cos(kx) (k=0.5) loaded by displacement, dt=0.05."""
    k = 0.5
    L = 2.0 * math.pi / k * 16

    def make():
        x0 = L * uniform(seed, 0, np_)
        x = wrap_positions(x0 - (1e-2 / k) * np.sin(k * x0), L)
        v = 0.1 * normal(seed, 1, np_)
        return x, v
    return RunSpec(L=L, ng=ng, np_=np_, dt=0.05, nsteps=nsteps,
                   name=f"maxwellian_ng{ng}_np{np_}", make=make,
                   loader=dict(seed=seed, pos_stream=0, vel_stream=1, amp=-(1e-2 / k), k=k, v0=0.0, vth=0.1,
                               beams=0))


def quiet_two_stream(L: float = 2.053, ng: int = 64, ppc: int = 64, v0: float = 0.2,
                     amp: float = 1e-5, dt: float = 0.1, nsteps: int = 400) -> RunSpec:
    """Quiet start (regular lattice, both beams at the same sites), mode-1
    displacement ``amp`` * L * sin(2 pi x0 / L)."""
    npairs = ng * ppc // 2

    def make():
        x0 = (np.arange(npairs) + 0.5) * (L / npairs)
        x0 = wrap_positions(x0 + amp * L * np.sin(2.0 * math.pi * x0 / L), L)
        x = np.repeat(x0, 2)
        v = v0 * _beam_signs(2 * npairs)
        return x, v
    return RunSpec(L=L, ng=ng, np_=2 * npairs, dt=dt, nsteps=nsteps, name="quiet_two_stream", make=make)


def cold_plasma(L: float = 2.053, ng: int = 64, ppc: int = 64, amp: float = 1e-3,
                dt: float = 0.1, nsteps: int = 300) -> RunSpec:
    """Cold single-species plasma at rest, quiet start, mode-1 displacement."""
    n = ng * ppc

    def make():
        x0 = (np.arange(n) + 0.5) * (L / n)
        x = wrap_positions(x0 + amp * L * np.sin(2.0 * math.pi * x0 / L), L)
        return x, np.zeros(n)
    return RunSpec(L=L, ng=ng, np_=n, dt=dt, nsteps=nsteps, name="cold_plasma", make=make)


def paper_weak_scaling(cores: int = 128, seed: int = 6, nsteps: int = 1000) -> RunSpec:
    """The paper's weak-scaling workload (Sec. 5.2 and the appendix's
    parameters) at the size it reaches on `cores` UPC threads: 64 cells and
    64,000 particles per thread, L = 3.1415 per thread, Maxwellian vth = 0.2
    with no drift, dt = 0.1, 1000 cycles, from the appendix's lattice start
    (1000 particles per cell)."""
    L = 3.1415 * cores
    ng = 64 * cores
    np_ = 64000 * cores
    ld = dict(seed=seed, pos_stream=0, vel_stream=1, amp=0.0, k=0.0, v0=0.0, vth=0.2, beams=0, lattice=True)

    def make():
        return loaded(L, np_, **_host_loader(ld))
    return RunSpec(L=L, ng=ng, np_=np_, dt=0.1, nsteps=nsteps, name=f"paper_weak_scaling_{cores}", make=make,
                   loader=ld)


def paper_two_stream(cores: int = 4, seed: int = 8, nsteps: int = 200) -> RunSpec:
    """The two-stream verification run of Sec. 4 (its phase-space figure was
    made on four UPC threads) with the appendix's sizes per thread: 64 cells,
    64,000 particles and L = 3.1415 per thread, lattice start, each particle
    given +0.2 or -0.2 by a uniform draw, cold beams (the figure shows two
    lines), dt = 0.1, 200 cycles (t = 20, the figure's late snapshot)."""
    L = 3.1415 * cores
    ng = 64 * cores
    np_ = 64000 * cores
    ld = dict(seed=seed, pos_stream=0, vel_stream=1, amp=0.0, k=0.0, v0=0.2, vth=0.0, beams=2, lattice=True)

    def make():
        return loaded(L, np_, **_host_loader(ld))
    return RunSpec(L=L, ng=ng, np_=np_, dt=0.1, nsteps=nsteps, name=f"paper_two_stream_{cores}", make=make,
                   loader=ld)


def _host_loader(ld: dict) -> dict:
    d = dict(ld)
    d["lattice_start"] = bool(d.pop("lattice", False))
    return d


def warm_maxwellian_small(seed: int = 7, waves: int = 2, ng: int = 256, ppc: int = 800, vth: float = 0.1,
                          k: float = 0.5, alpha: float = 1e-2, dt: float = 0.05, nsteps: int = 400) -> RunSpec:
    """A small warm Maxwellian plasma for the Bohm-Gross frequency: `waves`
    wavelengths of k in the box, quiet start (lattice) displaced to a density
    perturbation alpha cos(k x), seeded Maxwellian velocities."""
    L = waves * 2.0 * math.pi / k
    n = ng * ppc
    ld = dict(seed=seed, pos_stream=0, vel_stream=1, amp=-(alpha / k), k=k, v0=0.0, vth=vth, beams=0, lattice=True)

    def make():
        return loaded(L, n, **_host_loader(ld))
    return RunSpec(L=L, ng=ng, np_=n, dt=dt, nsteps=nsteps, name="warm_maxwellian_small", make=make, loader=ld)
