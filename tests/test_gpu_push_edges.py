"""The push's rare branches on the GPU (leapfrog and periodic wrap, Sec. 2.1).

Each case is a bounded input whose handling the kernel documents:
  * a field strong enough that a particle moves more than L in one step
    (PIC_FLAG_MULTIWRAP, positions wrapped as x - L floor(x/L));
  * drifts that land exactly on the domain's ends in FP32, including the
    rounding guard (a position just below 0 whose wrap rounds up to L is
    the point 0), which raise no flag;
  * a field whose change of velocity per step overflows FP32
    (PIC_FLAG_NONFINITE: the particle is put back at x = 0).
In every case positions stay in [0, L) and the deposit of the downloaded
state is bit-exact against the oracle's fixed-point rule.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1108_1954_amd import pic as P

import test_gpu_parity as G

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.load()
    yield


def one_step_against_oracle(p, x, v):
    """Create, read the state, take one step; returns (state before, field,
    state after, flags) with the oracle's step from the same state and field."""
    with P.Run(p, x, v) as r:
        u0, w0 = r.raw()
        S0, E0, Eh0 = r.grid()
        r.step(1)
        u1, w1 = r.raw()
        S1, _, _ = r.grid()
        d, _, _ = r.diagnostics()
    op = G.oracle_params(p)
    np.testing.assert_array_equal(S0, O.deposit_fixed(p.ng, u0.astype(np.float64)))
    np.testing.assert_array_equal(S1, O.deposit_fixed(p.ng, u1.astype(np.float64)))
    assert int(S1.sum()) == p.np << 32
    assert np.all((u1 >= 0) & (u1 < p.ng))
    dx = p.L / p.ng
    E_ora, _ = O.solve(op, O.density_fixed(op, S0))
    x0 = u0.astype(np.float64) * dx
    v0 = w0.astype(np.float64) * dx / p.dt
    x1, v1, _ = O.push(op, x0, v0, O.gather(op, x0, E_ora))
    return dict(u0=u0, w0=w0, Eh0=Eh0, u1=u1, w1=w1, u1o=x1 / dx, w1o=v1 * p.dt / dx, flags=d["flags"])


def test_particles_moving_more_than_the_domain_in_one_step():
    """ng = 8, 1000 particles at rest, qm = -1e5: the first kick moves many
    of them by more than ng cells.  Each is wrapped back into [0, ng) by
    x - L floor(x/L) and the run flags PIC_FLAG_MULTIWRAP."""
    ng, L, dt = 8, 8 * 0.032, 0.1
    x = np.random.default_rng(5).uniform(0, L, 1000)
    v = np.zeros_like(x)
    p = P.make_params(L, ng, x.size, dt, qm=-1e5)
    r = one_step_against_oracle(p, x, v)
    assert np.abs(r["w1o"]).max() > 2 * ng                 # the case really occurs
    assert r["flags"] == P.PIC_FLAG_MULTIWRAP
    # velocity: the rounding bound of one step; position: the drift and the
    # wrap round at the size of the unwrapped position |s + w| (four
    # roundings: add, shift, divide, subtract), plus the velocity's error
    _, dw = G.push_tolerance(r["u1o"], r["w1o"], np.abs(r["Eh0"]).max(), ng, EPS32)
    du = dw + 8 * EPS32 * (np.abs(r["w1o"]) + ng)
    err_w = np.abs(r["w1"].astype(np.float64) - r["w1o"])
    err_u = np.abs(G.periodic_diff(r["u1"], r["u1o"], ng))
    assert np.all(err_w <= dw), err_w.max()
    assert np.all(err_u <= du), (err_u.max(), du[np.argmax(err_u)])


def test_drifts_onto_the_domain_ends_and_the_rounding_guard():
    """A lattice of 4 particles per cell has an exactly uniform deposit, so
    E^0 = 0 and the first kick changes nothing.  Three particles then drift
    onto the ends in FP32: from x/dx = 1/8 by -1/8 - 2^-25 (just below 0: the
    wrap x + L rounds to L, which is the point 0), by exactly -1/8 (to 0),
    and from ng - 1/8 by +1/8 (exactly to L, i.e. 0).  None raises a flag;
    all three end at x = 0."""
    ng = 64
    L, dt = ng * 0.032, 0.1
    dx = L / ng
    u = (np.arange(4 * ng) + 0.5) / 4.0                    # 1/8, 3/8, ... exactly
    w = np.zeros_like(u)
    u_idx = {"guard": 0, "exact_zero": 8, "top": 4 * ng - 1}
    w[u_idx["guard"]] = -0.125 - 2.0 ** -25                 # 1/8 -> -2^-25
    w[u_idx["exact_zero"]] = -u[u_idx["exact_zero"]]         # 2 + 1/8 -> 0
    w[u_idx["top"]] = 0.125                                 # ng - 1/8 -> ng
    x = u * dx
    v = w * dx / dt
    p = P.make_params(L, ng, x.size, dt)
    r = one_step_against_oracle(p, x, v)
    assert np.all(r["Eh0"] == 0)                            # the uniform lattice has no field
    assert r["flags"] == 0
    for name, i in u_idx.items():
        assert r["u1"][i] == 0.0, (name, r["u1"][i])        # stored s = 1/2: the point x = 0
    _, dw = G.push_tolerance(r["u1o"], r["w1o"], 0.0, ng, EPS32)
    du = dw + 4 * EPS32 * (np.abs(r["w1o"]) + ng)
    np.testing.assert_array_equal(r["w1"], r["w0"])
    assert np.all(np.abs(G.periodic_diff(r["u1"], r["u1o"], ng)) <= du)


def test_velocity_change_overflowing_fp32_resets_the_particle():
    """qm = -1e43: the gather table E qm dt^2/dx overflows FP32 wherever
    E != 0, the kicked velocity is not finite, and the particle is put back at
    x = 0 with PIC_FLAG_NONFINITE set.  Positions stay in range and the
    deposit stays exact (no index is formed from a non-finite value)."""
    ng, L, dt = 16, 16 * 0.032, 0.1
    x = np.random.default_rng(9).uniform(0, L, 2000)
    v = np.zeros_like(x)
    p = P.make_params(L, ng, x.size, dt, qm=-1e43)
    with P.Run(p, x, v) as r:
        _, _, Eh = r.grid()
        assert np.any(np.isinf(Eh))
        r.step(2)
        u, w = r.raw()
        S, _, _ = r.grid()
        d, _, _ = r.diagnostics()
    assert d["flags"] & P.PIC_FLAG_NONFINITE
    assert np.all((u >= 0) & (u < ng))
    assert np.any(~np.isfinite(w)) and np.all(u[~np.isfinite(w)] == 0.0)
    np.testing.assert_array_equal(S, O.deposit_fixed(ng, u.astype(np.float64)))
    assert int(S.sum()) == x.size << 32
