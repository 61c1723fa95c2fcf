"""ctypes wrapper of the FP64 CPU oracle (``pic_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU engine never imports this
module.  The library is compiled with ``build()`` (plain gcc, no fast-math, no
FMA contraction) into ``oracle/libpic_oracle.so``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pic_oracle.c")
LIB = os.path.join(HERE, "libpic_oracle.so")

DEPOSIT_PLAIN = 0
DEPOSIT_FIXED = 1


class Params(C.Structure):
    _fields_ = [("L", C.c_double), ("ng", C.c_int32), ("solver", C.c_int32),
                ("np", C.c_int64), ("dt", C.c_double), ("qm", C.c_double),
                ("rho0", C.c_double), ("cg_iters", C.c_int32), ("pad_", C.c_int32)]


def build(src: str = SRC, out: str = LIB) -> str:
    """Compile the oracle (always; a few hundred milliseconds)."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_lib = None


def use_library(path: Optional[str]):
    """Point the wrapper at another build of the oracle source (the mutation
    tests load deliberately broken copies); ``None`` restores the default.
    Returns the previously loaded handle."""
    global _lib
    prev = _lib
    _lib = None if path is None else _bind(C.CDLL(path))
    return prev


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = _bind(C.CDLL(LIB))
    return _lib


def _bind(L):
    """Declare argument types of the oracle's C entry points."""
    dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
    ip = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
    P = C.POINTER(Params)
    L.ora_particle_charge.argtypes = [P]
    L.ora_particle_charge.restype = C.c_double
    L.ora_particle_mass.argtypes = [P]
    L.ora_particle_mass.restype = C.c_double
    L.ora_deposit_plain.argtypes = [P, dp, dp]
    L.ora_deposit_fixed.argtypes = [C.c_int32, C.c_int64, dp, ip]
    L.ora_density_fixed.argtypes = [P, ip, dp]
    L.ora_cell_order.argtypes = [C.c_int32, C.c_int64, dp, ip]
    L.ora_phase_space.argtypes = [P, C.c_int64, dp, dp, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                  C.c_void_p, C.POINTER(C.c_int64)]
    L.ora_solve.argtypes = [P, dp, dp, C.c_void_p]
    L.ora_cg_paper.argtypes = [P, dp, C.c_int32, dp, dp]
    L.ora_cg_paper.restype = C.c_int32
    L.ora_gather.argtypes = [P, dp, dp, dp]
    L.ora_push.argtypes = [P, dp, dp, dp, C.c_void_p]
    L.ora_field_energy.argtypes = [P, dp]
    L.ora_field_energy.restype = C.c_double
    L.ora_density.argtypes = [P, dp, C.c_int32, dp, C.c_void_p]
    L.ora_step.argtypes = [P, dp, dp, dp, C.c_int32, dp, dp, C.c_void_p]
    L.ora_run.argtypes = [P, dp, dp, C.c_int64, C.c_int32, dp, dp, C.c_void_p, C.c_void_p]
    L.ora_run_literal.argtypes = [P, dp, dp, C.c_int64, C.c_int32, dp, dp]
    return L


SOLVE_EXACT, SOLVE_CG_PAPER = 0, 1


def params(L: float, ng: int, np: int, dt: float = 0.1, qm: float = -1.0, rho0: float = 1.0,
           solver: int = SOLVE_EXACT, cg_iters: int = 0) -> Params:
    return Params(L=float(L), ng=int(ng), solver=int(solver), np=int(np), dt=float(dt), qm=float(qm),
                  rho0=float(rho0), cg_iters=int(cg_iters), pad_=0)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def particle_charge(p: Params) -> float:
    return lib().ora_particle_charge(C.byref(p))


def particle_mass(p: Params) -> float:
    return lib().ora_particle_mass(C.byref(p))


def deposit_plain(p: Params, x) -> np.ndarray:
    rho = np.empty(p.ng)
    lib().ora_deposit_plain(C.byref(p), _f64(x), rho)
    return rho


def deposit_fixed(ng: int, u) -> np.ndarray:
    u = _f64(u)
    S = np.empty(ng, dtype=np.int64)
    lib().ora_deposit_fixed(int(ng), int(u.size), u, S)
    return S


def cell_order(ng: int, u) -> np.ndarray:
    """Stable permutation of particles by cell key (u = x/dx)."""
    u = _f64(u)
    perm = np.empty(u.size, dtype=np.int64)
    lib().ora_cell_order(int(ng), int(u.size), u, perm)
    return perm


def phase_space(p: Params, u, w, nx: int, nv: int, vmin: float, vmax: float) -> Tuple[np.ndarray, int]:
    """(x, v) counts as an (nv, nx) image from state-form particles
    u = x/dx, w = v dt/dx, and the number with v outside [vmin, vmax)."""
    u, w = _f64(u), _f64(w)
    assert u.size == w.size
    counts = np.empty((int(nv), int(nx)), dtype=np.uint32)
    out = C.c_int64(0)
    lib().ora_phase_space(C.byref(p), int(u.size), u, w, int(nx), int(nv), float(vmin), float(vmax),
                          counts.ctypes.data, C.byref(out))
    return counts, out.value


def density_fixed(p: Params, S) -> np.ndarray:
    rho = np.empty(p.ng)
    lib().ora_density_fixed(C.byref(p), np.ascontiguousarray(S, dtype=np.int64), rho)
    return rho


def solve(p: Params, rho) -> Tuple[np.ndarray, np.ndarray]:
    E = np.empty(p.ng)
    phi = np.empty(p.ng)
    lib().ora_solve(C.byref(p), _f64(rho), E, _ptr(phi))
    return E, phi


def cg_paper(p: Params, rho, maxit: int = 150) -> Tuple[np.ndarray, np.ndarray, int]:
    phi = np.empty(p.ng)
    E = np.empty(p.ng)
    it = lib().ora_cg_paper(C.byref(p), _f64(rho), int(maxit), phi, E)
    return phi, E, it


def gather(p: Params, x, E) -> np.ndarray:
    Ep = np.empty(p.np)
    lib().ora_gather(C.byref(p), _f64(x), _f64(E), Ep)
    return Ep


def push(p: Params, x, v, Ep) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    x = _f64(x).copy()
    v = _f64(v).copy()
    acc = np.empty(3)
    lib().ora_push(C.byref(p), x, v, _f64(Ep), _ptr(acc))
    return x, v, acc


def field_energy(p: Params, E) -> float:
    return lib().ora_field_energy(C.byref(p), _f64(E))


def density(p: Params, x, mode: int = DEPOSIT_PLAIN) -> np.ndarray:
    rho = np.empty(p.ng)
    lib().ora_density(C.byref(p), _f64(x), int(mode), rho, None)
    return rho


def step(p: Params, x, v, E, mode: int = DEPOSIT_PLAIN):
    """One cycle; returns (x, v, E, rho, row) without touching the inputs."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    E = _f64(E).copy()
    rho = np.empty(p.ng)
    Ep = np.empty(max(1, p.np))
    row = np.empty(4)
    lib().ora_step(C.byref(p), x, v, E, int(mode), rho, Ep, _ptr(row))
    return x, v, E, rho, row


def run(p: Params, x, v, nsteps: int, mode: int = DEPOSIT_PLAIN, keep_E: bool = False):
    """Initial solve plus ``nsteps`` cycles.

    Returns dict with x, v (final), E, rho (final), hist (nsteps x 4:
    KE^n, W_E^n, P^{n+1/2}, K^{n+1/2}) and, if keep_E, E_hist (nsteps x ng)."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    E = np.empty(p.ng)
    rho = np.empty(p.ng)
    hist = np.empty((int(nsteps), 4))
    E_hist = np.empty((int(nsteps), p.ng)) if keep_E else None
    lib().ora_run(C.byref(p), x, v, int(nsteps), int(mode), E, rho, _ptr(hist), _ptr(E_hist))
    out = dict(x=x, v=v, E=E, rho=rho, hist=hist)
    if keep_E:
        out["E_hist"] = E_hist
    return out


def run_literal(p: Params, x, v, ncycles: int, mode: int = DEPOSIT_PLAIN):
    """``ncycles`` cycles in the appendix's order (drift, wrap, deposit,
    solve, gather, kick) from (x, v); returns final x, v, E."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    E = np.empty(p.ng)
    rho = np.empty(p.ng)
    lib().ora_run_literal(C.byref(p), x, v, int(ncycles), int(mode), E, rho)
    return dict(x=x, v=v, E=E)
