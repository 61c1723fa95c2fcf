"""Python binding of the engine's C ABI (``include/pic.h``).

Argument marshalling only: every step of the particle loop runs in the HIP
kernels of ``libpic1d.so``.  The functions keep the C names; status codes
below zero raise :class:`PicError` with the library's message.  PyTorch is
used for device memory (a ``torch.uint8`` buffer handed to the library) and
for the HIP stream.  If the extension is missing, loading fails loudly: there
is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpic1d.so")

PIC_OK, PIC_EINVAL, PIC_ENOMEM, PIC_EDEVICE, PIC_ESTATE, PIC_EBUDGET = 0, -1, -2, -3, -4, -5
PIC_FP32, PIC_FP64 = 0, 1
PIC_MAX_NG = 8192
PIC_HIST_COLS = 4
PIC_FLAG_NONFINITE, PIC_FLAG_MULTIWRAP, PIC_FLAG_SORT = 1, 2, 4
PIC_SOLVE_EXACT, PIC_SOLVE_CG_PAPER = 0, 1
PIC_BEAMS_ONE, PIC_BEAMS_ALTERNATE, PIC_BEAMS_RANDOM = 0, 1, 2
PIC_SORT_AUTO = -1

SYMBOLS = (
    "pic_last_error", "pic_version", "pic_footprint", "pic_create", "pic_create_loaded", "pic_sort",
    "pic_step", "pic_step_graph", "pic_batch_admit_loaded",
    "pic_step_profiled", "pic_batch_step_profiled", "pic_diagnostics", "pic_read_particles", "pic_read_raw", "pic_read_grid", "pic_read_history",
    "pic_phase_space", "pic_phase_space_noalloc", "pic_sort_period", "pic_destroy", "pic_batch_create", "pic_batch_admit", "pic_batch_step", "pic_batch_poll",
    "pic_bandwidth_probe", "pic_batch_run", "pic_batch_diagnostics", "pic_batch_release", "pic_batch_usage", "pic_batch_destroy",
)


class pic_params(C.Structure):
    _fields_ = [("L", C.c_double), ("ng", C.c_int32), ("precision", C.c_int32),
                ("np", C.c_int64), ("dt", C.c_double), ("qm", C.c_double),
                ("rho0", C.c_double), ("sort_every", C.c_int32), ("tile", C.c_int32),
                ("history_cap", C.c_int64), ("solver", C.c_int32), ("cg_iters", C.c_int32)]


class pic_diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("time", C.c_double), ("kinetic", C.c_double),
                ("field", C.c_double), ("momentum", C.c_double),
                ("charge_fixed_sum", C.c_int64), ("net_charge", C.c_double),
                ("flags", C.c_uint32), ("pad_", C.c_uint32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


class pic_loader(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("pos_stream", C.c_int32), ("vel_stream", C.c_int32),
                ("amp", C.c_double), ("k", C.c_double), ("v0", C.c_double), ("vth", C.c_double),
                ("beams", C.c_int32), ("lattice", C.c_int32)]


def make_loader(seed: int, pos_stream: int = 0, vel_stream: int = 1, amp: float = 0.0, k: float = 0.0,
                v0: float = 0.0, vth: float = 0.0, beams: int = 0, lattice: bool = False) -> pic_loader:
    return pic_loader(seed=int(seed), pos_stream=int(pos_stream), vel_stream=int(vel_stream), amp=float(amp),
                      k=float(k), v0=float(v0), vth=float(vth), beams=int(beams), lattice=int(bool(lattice)))


class pic_batch_config(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("arena", C.c_void_p), ("max_runs", C.c_int32),
                ("ng_max", C.c_int32), ("graph_steps", C.c_int32), ("grid_blocks", C.c_int32)]


class PicError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


class PicBudget(PicError):
    """PIC_EBUDGET: the run does not fit the batch's HBM budget right now."""


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (once).  torch is imported first so that the
    library binds to the HIP runtime torch already uses."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP extension not built: {path} is missing "
                           "(run `python -m paper_1108_1954_amd.build`)")
    try:
        import torch  # noqa: F401  (shares its HIP runtime with the library)
    except ImportError:
        pass
    L = C.CDLL(path)
    P = C.POINTER(pic_params)
    vp, i64, i32, sz = C.c_void_p, C.c_int64, C.c_int32, C.c_size_t
    dptr = C.POINTER(C.c_double)
    L.pic_last_error.restype = C.c_char_p
    L.pic_version.restype = C.c_char_p
    sig = {
        "pic_footprint": [P, C.POINTER(sz)],
        "pic_create": [P, dptr, dptr, vp, sz, vp, C.POINTER(vp)],
        "pic_create_loaded": [P, C.POINTER(pic_loader), vp, sz, vp, C.POINTER(vp)],
        "pic_batch_admit_loaded": [vp, P, C.POINTER(pic_loader), i64, C.POINTER(i64)],
        "pic_sort": [vp],
        "pic_sort_period": [vp, C.POINTER(i32)],
        "pic_step": [vp, i64],
        "pic_step_graph": [vp, i64, i32],
        "pic_step_profiled": [vp, i64, dptr, dptr],
        "pic_batch_step_profiled": [vp, i64, dptr, dptr],
        "pic_diagnostics": [vp, C.POINTER(pic_diag), vp, vp, i32],
        "pic_read_particles": [vp, vp, vp, i64],
        "pic_read_raw": [vp, vp, vp, i64],
        "pic_read_grid": [vp, vp, vp, vp, i32],
        "pic_read_history": [vp, i64, i64, vp],
        "pic_phase_space": [vp, i32, i32, C.c_double, C.c_double, vp, C.POINTER(i64)],
        "pic_phase_space_noalloc": [vp, i32, i32, C.c_double, C.c_double, vp, C.POINTER(i64)],
        "pic_destroy": [vp],
        "pic_bandwidth_probe": [vp, vp, i64, i32, i32, vp, dptr],
        "pic_batch_create": [C.POINTER(pic_batch_config), vp, C.POINTER(vp)],
        "pic_batch_admit": [vp, P, dptr, dptr, i64, C.POINTER(i64)],
        "pic_batch_step": [vp, i64],
        "pic_batch_poll": [vp, vp, i32, C.POINTER(i32)],
        "pic_batch_run": [vp, i64, C.POINTER(vp)],
        "pic_batch_diagnostics": [vp, i64, C.POINTER(pic_diag)],
        "pic_batch_release": [vp, i64],
        "pic_batch_usage": [vp, C.POINTER(sz), C.POINTER(sz), C.POINTER(i32)],
        "pic_batch_destroy": [vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    _lib = L
    return L


def _check(status: int) -> None:
    if status < 0:
        msg = load().pic_last_error().decode(errors="replace")
        cls = PicBudget if status == PIC_EBUDGET else PicError
        raise cls(status, msg)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(L: float, ng: int, np: int, dt: float, qm: float = -1.0, rho0: float = 1.0,
                precision: int = PIC_FP32, sort_every: int = 0, tile: int = 0,
                history_cap: int = 0, solver: int = 0, cg_iters: int = 0) -> pic_params:
    return pic_params(L=float(L), ng=int(ng), precision=int(precision), np=int(np), dt=float(dt),
                      qm=float(qm), rho0=float(rho0), sort_every=int(sort_every), tile=int(tile),
                      history_cap=int(history_cap), solver=int(solver), cg_iters=int(cg_iters))


def pic_version() -> str:
    return load().pic_version().decode()


def pic_footprint(params: pic_params) -> int:
    n = C.c_size_t(0)
    _check(load().pic_footprint(C.byref(params), C.byref(n)))
    return n.value


def pic_create(params: pic_params, x0, v_mhalf, dev_mem: Optional[int] = None, dev_bytes: int = 0,
               stream: Optional[int] = None) -> C.c_void_p:
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    v = np.ascontiguousarray(v_mhalf, dtype=np.float64)
    if x0.size != params.np or v.size != params.np:
        raise ValueError("x0 and v_mhalf must hold np values")
    out = C.c_void_p()
    _check(load().pic_create(C.byref(params), _dptr(x0), _dptr(v), dev_mem, dev_bytes, stream,
                             C.byref(out)))
    return out


def pic_create_loaded(params: pic_params, loader: pic_loader, dev_mem: Optional[int] = None, dev_bytes: int = 0,
                      stream: Optional[int] = None) -> C.c_void_p:
    out = C.c_void_p()
    _check(load().pic_create_loaded(C.byref(params), C.byref(loader), dev_mem, int(dev_bytes), stream,
                                    C.byref(out)))
    return out


def pic_batch_admit_loaded(batch, params: pic_params, loader: pic_loader, nsteps: int) -> int:
    rid = C.c_int64(0)
    _check(load().pic_batch_admit_loaded(batch, C.byref(params), C.byref(loader), int(nsteps), C.byref(rid)))
    return rid.value


def pic_sort(run) -> None:
    _check(load().pic_sort(run))


def pic_step(run, nsteps: int) -> None:
    _check(load().pic_step(run, int(nsteps)))


def pic_step_graph(run, nsteps: int, graph_steps: int) -> None:
    _check(load().pic_step_graph(run, int(nsteps), int(graph_steps)))


def pic_step_profiled(run, nsteps: int) -> Tuple[float, float]:
    """Mean (particle-pass, solve) launch durations in ms over `nsteps` steps."""
    a, b = C.c_double(0), C.c_double(0)
    _check(load().pic_step_profiled(run, int(nsteps), C.byref(a), C.byref(b)))
    return a.value, b.value


def pic_batch_step_profiled(batch, nsteps: int) -> Tuple[float, float]:
    a, b = C.c_double(0), C.c_double(0)
    _check(load().pic_batch_step_profiled(batch, int(nsteps), C.byref(a), C.byref(b)))
    return a.value, b.value


def pic_diagnostics(run, ng: int = 0) -> Tuple[dict, Optional[np.ndarray], Optional[np.ndarray]]:
    """Diagnostics; with ng > 0 also the density and field grids."""
    d = pic_diag()
    rho = np.empty(ng) if ng else None
    E = np.empty(ng) if ng else None
    _check(load().pic_diagnostics(run, C.byref(d), None if rho is None else rho.ctypes.data,
                                  None if E is None else E.ctypes.data, int(ng)))
    return d.as_dict(), rho, E


def pic_read_particles(run, np_: int) -> Tuple[np.ndarray, np.ndarray]:
    x = np.empty(np_)
    v = np.empty(np_)
    _check(load().pic_read_particles(run, x.ctypes.data, v.ctypes.data, int(np_)))
    return x, v


def pic_read_raw(run, np_: int, precision: int = PIC_FP32) -> Tuple[np.ndarray, np.ndarray]:
    dt = np.float32 if precision == PIC_FP32 else np.float64
    u = np.empty(np_, dtype=dt)
    w = np.empty(np_, dtype=dt)
    _check(load().pic_read_raw(run, u.ctypes.data, w.ctypes.data, int(np_)))
    return u, w


def pic_sort_period(run) -> int:
    """The run's cell-sort period K (0: never), as chosen at creation for
    sort_every = PIC_SORT_AUTO."""
    k = C.c_int32(0)
    _check(load().pic_sort_period(run, C.byref(k)))
    return k.value


def pic_phase_space(run, nx: int, nv: int, vmin: float, vmax: float) -> Tuple[np.ndarray, int]:
    """Device-binned (x, v) counts as an (nv, nx) uint32 image, and the
    number of particles with v outside [vmin, vmax)."""
    counts = np.zeros((int(nv), int(nx)), dtype=np.uint32)
    out = C.c_int64(0)
    _check(load().pic_phase_space(run, int(nx), int(nv), float(vmin), float(vmax), counts.ctypes.data,
                                  C.byref(out)))
    return counts, out.value


def pic_phase_space_noalloc(run, nx: int, nv: int, vmin: float, vmax: float) -> Tuple[np.ndarray, int]:
    """pic_phase_space binned in the library's fixed device scratch (no
    device allocation); nx nv <= 16384."""
    counts = np.zeros((int(nv), int(nx)), dtype=np.uint32)
    out = C.c_int64(0)
    _check(load().pic_phase_space_noalloc(run, int(nx), int(nv), float(vmin), float(vmax), counts.ctypes.data,
                                          C.byref(out)))
    return counts, out.value


def pic_read_grid(run, ng: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    S = np.empty(ng, dtype=np.int64)
    E = np.empty(ng)
    Eh = np.empty(ng, dtype=np.float32)
    _check(load().pic_read_grid(run, S.ctypes.data, E.ctypes.data, Eh.ctypes.data, int(ng)))
    return S, E, Eh


def pic_read_history(run, first: int, count: int) -> np.ndarray:
    rows = np.empty((int(count), PIC_HIST_COLS))
    _check(load().pic_read_history(run, int(first), int(count), rows.ctypes.data if count else None))
    return rows


def pic_destroy(run) -> None:
    _check(load().pic_destroy(run))


def pic_batch_create(hbm_budget: int, ng_max: int, max_runs: int = 1024, graph_steps: int = 16,
                     grid_blocks: int = 0, arena: Optional[int] = None,
                     stream: Optional[int] = None) -> C.c_void_p:
    cfg = pic_batch_config(hbm_budget=int(hbm_budget), arena=arena, max_runs=int(max_runs),
                           ng_max=int(ng_max), graph_steps=int(graph_steps),
                           grid_blocks=int(grid_blocks))
    out = C.c_void_p()
    _check(load().pic_batch_create(C.byref(cfg), stream, C.byref(out)))
    return out


def pic_batch_admit(batch, params: pic_params, x0, v_mhalf, nsteps: int) -> int:
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    v = np.ascontiguousarray(v_mhalf, dtype=np.float64)
    if x0.size != params.np or v.size != params.np:
        raise ValueError("x0 and v_mhalf must hold np values")
    rid = C.c_int64(0)
    _check(load().pic_batch_admit(batch, C.byref(params), _dptr(x0), _dptr(v), int(nsteps),
                                  C.byref(rid)))
    return rid.value


def pic_batch_step(batch, nsteps: int) -> None:
    _check(load().pic_batch_step(batch, int(nsteps)))


def pic_batch_poll(batch, cap: int = 4096) -> list:
    ids = np.empty(max(1, cap), dtype=np.int64)
    n = C.c_int32(0)
    _check(load().pic_batch_poll(batch, ids.ctypes.data, int(cap), C.byref(n)))
    return ids[:n.value].tolist()


def pic_batch_run(batch, run_id: int) -> C.c_void_p:
    out = C.c_void_p()
    _check(load().pic_batch_run(batch, int(run_id), C.byref(out)))
    return out


def pic_bandwidth_probe(a: int, b: int, n: int, reps: int = 10, stream: Optional[int] = None,
                        cached: bool = False) -> float:
    """Mean ms of one swap of two device FP32 arrays of n values (device
    pointers a, b): the particle pass's bytes without its work, with
    non-temporal or (cached=True) ordinary cached accesses."""
    ms = C.c_double(0)
    _check(load().pic_bandwidth_probe(a, b, int(n), int(reps), int(bool(cached)), stream, C.byref(ms)))
    return ms.value


def pic_batch_diagnostics(batch, run_id: int) -> dict:
    d = pic_diag()
    _check(load().pic_batch_diagnostics(batch, int(run_id), C.byref(d)))
    return d.as_dict()


def pic_batch_release(batch, run_id: int) -> None:
    _check(load().pic_batch_release(batch, int(run_id)))


def pic_batch_usage(batch) -> Tuple[int, int, int]:
    used, free, n = C.c_size_t(0), C.c_size_t(0), C.c_int32(0)
    _check(load().pic_batch_usage(batch, C.byref(used), C.byref(free), C.byref(n)))
    return used.value, free.value, n.value


def pic_batch_destroy(batch) -> None:
    _check(load().pic_batch_destroy(batch))


# ------------------------------------------------------ torch-owned memory --

def device_buffer(nbytes: int):
    """A torch uint8 device tensor of at least ``nbytes`` plus its 256-byte
    aligned address: (tensor, address).  Keep the tensor alive as long as the
    library uses the memory."""
    import torch
    t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device="cuda")
    addr = t.data_ptr()
    return t, (addr + 255) // 256 * 256


def current_stream() -> int:
    import torch
    return torch.cuda.current_stream().cuda_stream


class Run:
    """A run whose device memory is a torch tensor (kept alive here)."""

    def __init__(self, params: pic_params, x0=None, v_mhalf=None, use_torch_memory: bool = True,
                 loader: Optional[pic_loader] = None):
        """Host particles (x0, v_mhalf), or `loader` to draw them on the device."""
        self.params = params
        self._buf = None
        addr, nbytes = None, 0
        if use_torch_memory:
            nbytes = pic_footprint(params)
            self._buf, addr = device_buffer(nbytes)
        if loader is not None:
            self.handle = pic_create_loaded(params, loader, addr, nbytes, current_stream())
        else:
            self.handle = pic_create(params, x0, v_mhalf, addr, nbytes, current_stream())

    def step(self, n: int, graph_steps: int = 0) -> None:
        if graph_steps > 0:
            pic_step_graph(self.handle, n, graph_steps)
        else:
            pic_step(self.handle, n)

    def sort(self) -> None:
        pic_sort(self.handle)

    def sort_period(self) -> int:
        return pic_sort_period(self.handle)

    def diagnostics(self, grids: bool = False):
        return pic_diagnostics(self.handle, self.params.ng if grids else 0)

    def raw(self):
        return pic_read_raw(self.handle, self.params.np, self.params.precision)

    def particles(self):
        return pic_read_particles(self.handle, self.params.np)

    def grid(self):
        return pic_read_grid(self.handle, self.params.ng)

    def phase_space(self, nx: int, nv: int, vmin: float, vmax: float):
        return pic_phase_space(self.handle, nx, nv, vmin, vmax)

    def history(self, first: int = 0, count: Optional[int] = None):
        if count is None:
            d, _, _ = self.diagnostics()
            count = min(d["step"], self.params.history_cap) - first
        return pic_read_history(self.handle, first, count)

    def close(self) -> None:
        if self.handle:
            pic_destroy(self.handle)
            self.handle = None
        self._buf = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
