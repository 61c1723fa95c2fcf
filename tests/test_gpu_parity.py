"""GPU parity of the HIP particle loop against the FP64 CPU oracle.

All inputs are seeded and synthetic (paper_1108_1954_amd.inputs).  Integer
work (the fixed-point charge deposit) must match bit for bit; floating-point
results are held to tolerances derived from the arithmetic (see
`push_tolerance`).  Every call goes through the C ABI.
"""
import dataclasses
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1108_1954_amd import inputs as I
from paper_1108_1954_amd import pic as P

import history_check as HC

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24
EPS64 = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.load()
    torch.cuda.init()
    yield


def make_run(spec, precision=P.PIC_FP32, history=0, tile=0, x=None, v=None):
    if x is None:
        x, v = spec.particles()
    p = P.make_params(spec.L, spec.ng, spec.np_, spec.dt, precision=precision,
                      history_cap=history, tile=tile)
    return P.Run(p, x, v), p


def oracle_params(p):
    return O.params(p.L, p.ng, p.np, dt=p.dt, qm=p.qm, rho0=p.rho0)


def periodic_diff(a, b, period):
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    return d - period * np.round(d / period)


def solve_tolerance(p, S):
    """Rounding bound of the FP64 solve: the face field is a sum of ng terms
    of size |rho - mean| dx in different orders on the two sides."""
    rho = O.density_fixed(oracle_params(p), S)
    dx = p.L / p.ng
    return 8 * p.ng * EPS64 * dx * np.abs(rho - rho.mean()).sum() + 1e-300


def push_tolerance(u_new, w_new, Ehat_max, ng, eps):
    """One GPU step in precision eps against the oracle's FP64 step from the
    same state and field.  GPU side: the gather weight f has at most one
    rounding, the stored table Ehat one, E_{j+1} - E_j and the FMA one each,
    so |dEp| <= 6 eps max|Ehat|; the kick adds eps |w_new|; the drift
    eps |u_new| and the wrap eps ng (factor 2 margin).  Oracle side: its FP64
    gather, kick, drift and wrap plus the unit conversions u <-> x, w <-> v
    add up to 8 roundings of the same magnitudes in FP64; in particular the
    oracle's position x/dx = (u dx)/dx is off by up to 2 ulp(ng), which moves
    its gather weight by that much and Ep by that times the field step
    |Ehat_{j+1} - Ehat_j| <= 2 max|Ehat|."""
    conv = 8 * EPS64 * ng * 2 * Ehat_max
    dw = (2 * eps + 8 * EPS64) * (np.abs(w_new) + 6 * Ehat_max) + conv
    du = dw + (2 * eps + 8 * EPS64) * (np.abs(u_new) + ng)
    return du, dw


def check_deposit_exact(run, p, u):
    S_gpu, _, _ = run.grid()
    S_ora = O.deposit_fixed(p.ng, u.astype(np.float64))
    np.testing.assert_array_equal(S_gpu, S_ora)
    assert int(S_gpu.sum()) == p.np * 2 ** 32


# ------------------------------------------------------------ single run ---

@pytest.mark.parametrize("precision", [P.PIC_FP32, P.PIC_FP64])
def test_initial_deposit_and_solve(precision):
    spec = I.two_stream_small()
    run, p = make_run(spec, precision)
    with run:
        u, _ = run.raw()
        check_deposit_exact(run, p, u)
        S, E, Eh = run.grid()
        E_ora, _ = O.solve(oracle_params(p), O.density_fixed(oracle_params(p), S))
        np.testing.assert_allclose(E, E_ora, rtol=0, atol=solve_tolerance(p, S))
        ecoef = p.qm * p.dt ** 2 / (p.L / p.ng)
        np.testing.assert_array_equal(Eh, (E * ecoef).astype(np.float32))
        d, rho, Eg = run.diagnostics(grids=True)
        assert d["step"] == 0 and d["charge_fixed_sum"] == p.np * 2 ** 32
        assert abs(d["net_charge"]) < 1e-12
        assert d["field"] == pytest.approx(O.field_energy(oracle_params(p), E_ora), rel=1e-12)
        np.testing.assert_array_equal(Eg, E)


@pytest.mark.parametrize("precision,np_,ng,tile", [
    (P.PIC_FP32, 10_000, 64, 0),
    (P.PIC_FP32, 300_001, 512, 0),        # many tiles, ragged tail (np mod 4 = 1)
    (P.PIC_FP32, 70_003, 100, 1024),      # non power-of-two grid, explicit tile
    (P.PIC_FP64, 300_001, 512, 0),
    (P.PIC_FP64, 70_003, 8192, 3072),     # largest grid, FP64 state (128 KiB LDS), 3-unit tiles
    (P.PIC_FP32, 1, 2, 0),                # one particle, smallest grid
    (P.PIC_FP32, 5, 3, 0),
    (P.PIC_FP32, 5000, 16, 1024),         # ntiles > 1 with the ragged unit in tile 0
])
def test_single_step_matches_oracle(precision, np_, ng, tile):
    """From the same (downloaded) state and field, one GPU step agrees with the
    FP64 oracle's step within the rounding bound, and the new deposit is bit
    exact."""
    spec = I.warm_two_stream_large(seed=11, np_=np_, ng=ng, nsteps=1, L=0.032 * ng)
    run, p = make_run(spec, precision, history=4, tile=tile)
    eps = EPS32 if precision == P.PIC_FP32 else EPS64
    with run:
        run.step(2)                                  # move away from the loader state
        u0, w0 = run.raw()
        S0, E0, Eh0 = run.grid()
        op = oracle_params(p)
        E_ora, _ = O.solve(op, O.density_fixed(op, S0))
        np.testing.assert_allclose(E0, E_ora, rtol=0, atol=solve_tolerance(p, S0))
        dx = p.L / p.ng
        x0 = u0.astype(np.float64) * dx
        v0 = w0.astype(np.float64) * dx / p.dt
        Ep = O.gather(op, x0, E_ora)
        x1, v1, _ = O.push(op, x0, v0, Ep)
        run.step(1)
        u1, w1 = run.raw()
        u1o, w1o = x1 / dx, v1 * p.dt / dx
        du, dw = push_tolerance(u1o, w1o, np.abs(Eh0).max(), p.ng, eps)
        err_w = np.abs(w1.astype(np.float64) - w1o)
        err_u = np.abs(periodic_diff(u1, u1o, p.ng))
        assert np.all(err_w <= dw), f"max w error {err_w.max():.3g} vs bound {dw.max():.3g}"
        assert np.all(err_u <= du), f"max u error {err_u.max():.3g} vs bound {du.max():.3g}"
        assert np.all((u1 >= 0) & (u1 < p.ng))
        check_deposit_exact(run, p, u1)
        d, _, _ = run.diagnostics()
        assert d["step"] == 3 and d["flags"] == 0


def test_deposit_stays_bit_exact_over_many_steps():
    spec = I.two_stream_small(np_=50_003)
    run, p = make_run(spec, history=64)
    with run:
        for n in (1, 4, 15, 40):
            run.step(n)
            u, _ = run.raw()
            check_deposit_exact(run, p, u)


def test_edge_positions_deposit_exactly():
    """Particles exactly on nodes, at 0, at cell edges and just below L."""
    ng, L = 16, 16 * 0.032
    dx = L / ng
    xs = [0.0, dx / 2, dx, 1.5 * dx, L - dx / 2, L - 1e-12, 0.25 * dx, 7 * dx + 1e-15]
    rng = np.random.default_rng(3)
    x = np.concatenate([xs, rng.uniform(0, L, 1000 - len(xs))])
    v = np.zeros_like(x)
    p = P.make_params(L, ng, x.size, 0.1)
    with P.Run(p, x, v) as run:
        u, _ = run.raw()
        check_deposit_exact(run, p, u)
        run.step(3)
        u, _ = run.raw()
        check_deposit_exact(run, p, u)


def test_graph_replay_is_bit_identical_to_plain_launches():
    spec = I.two_stream_small(np_=40_000)
    x, v = spec.particles()
    a, p = make_run(spec, history=64, x=x, v=v)
    b, _ = make_run(spec, history=64, x=x, v=v)
    with a, b:
        a.step(37)
        b.step(37, graph_steps=8)                    # 4 graph replays + 5 plain launches
        ua, wa = a.raw()
        ub, wb = b.raw()
        np.testing.assert_array_equal(ua, ub)
        np.testing.assert_array_equal(wa, wb)
        np.testing.assert_array_equal(a.history(), b.history())


# ----------------------------------------------------- runs vs the oracle ---

@pytest.mark.parametrize("precision", [P.PIC_FP32, P.PIC_FP64])
def test_two_stream_history_against_fp64_oracle(precision):
    """Two-stream run (Ng=64, Np=10,000, 200 steps): every column of the
    engine's history (KE^n, W_E^n, P^{n+1/2}, K^{n+1/2}) and the diagnostics
    after creation and after the last step against the FP64 oracle's steps
    from the same FP64 inputs with the same fixed-point deposit rule.  The
    bounds come from the oracle's own sensitivity to one rounding of the state
    to the engine's precision (tests/history_check.py): over the linear phase
    (100 steps, t < 10) and over the whole run."""
    spec = I.two_stream_small()
    x, v = spec.particles()
    run, p = make_run(spec, precision=precision, history=spec.nsteps, x=x, v=v)
    with run:
        d0, _, _ = run.diagnostics()
        run.step(spec.nsteps)
        h = run.history()
        d1, _, _ = run.diagnostics()
    op = oracle_params(p)
    lin, n = 100, spec.nsteps
    dtype = np.float32 if precision == P.PIC_FP32 else np.float64
    bounds, ref, sens = HC.state_bounds(op, x, v, n, (lin, n), dtype=dtype)
    pscale = HC.momentum_scale(op, v)
    err = HC.column_errors(h, ref, pscale)
    for window in (lin, n):
        for c in HC.COLS:
            e, bnd = float(err[c][:window].max()), bounds[window][c]
            print(f"two-stream {dtype.__name__} state, {c} over {window} steps: error {e:.3e}, "
                  f"bound {bnd:.3e} (one rounding moves it {float(sens[c][:window].max()):.3e})", flush=True)
            assert e <= bnd, (c, window, e, bnd)
    # diagnostics of the state after creation: (m/2) sum v^2 and m sum v of
    # the inputs, from the oracle's push with zero field (its sums of v_old);
    # each stored w rounds once to the state precision, the FP64 sums of np
    # terms in another order
    eps = EPS32 if precision == P.PIC_FP32 else EPS64
    m = O.particle_mass(op)
    _, _, acc = O.push(op, x, v, np.zeros(p.np))
    k0 = 0.5 * m * acc[0]
    assert abs(d0["kinetic"] - k0) <= (4 * eps + (p.np + 8) * EPS64) * k0
    assert abs(d0["momentum"] - m * float(np.sum(v))) <= (2 * eps + (p.np + 8) * EPS64) * pscale
    assert d0["step"] == 0 and d1["step"] == n
    # after the last step: K^{N-1/2} and P^{N-1/2}, the oracle's last row
    kscale = np.abs(ref[:, 3]).max()
    assert d1["kinetic"] == h[-1, 3] and d1["momentum"] == h[-1, 2]
    assert abs(d1["kinetic"] - ref[-1, 3]) <= bounds[n]["K"] * kscale
    assert abs(d1["momentum"] - ref[-1, 2]) <= bounds[n]["P"] * pscale


def test_cold_plasma_frequency_on_gpu():
    s = I.cold_plasma(nsteps=400)
    run, p = make_run(s, history=s.nsteps)
    with run:
        run.step(s.nsteps)
        we = run.history()[:, 1]
    # W_E oscillates at twice the plasma frequency; locate its minima to
    # sub-step accuracy with a parabola through the three nearest samples
    mins = []
    for i in range(1, len(we) - 1):
        if we[i] < we[i - 1] and we[i] <= we[i + 1]:
            den = we[i - 1] - 2 * we[i] + we[i + 1]
            mins.append((i + 0.5 * (we[i - 1] - we[i + 1]) / den) * s.dt)
    omega = math.pi * (len(mins) - 1) / (mins[-1] - mins[0])
    from test_oracle_pins import predicted_cold_plasma_frequency
    pred = predicted_cold_plasma_frequency(s.L, s.ng, s.dt, 2 * math.pi / s.L)
    assert len(mins) >= 10
    assert abs(omega - pred) < 1e-3, (omega, pred)


def test_two_stream_growth_rate_on_gpu():
    s = I.quiet_two_stream(nsteps=300)
    run, p = make_run(s, history=s.nsteps)
    with run:
        run.step(s.nsteps)
        we = run.history()[:, 1]
    from test_oracle_pins import two_stream_growth_rate, _mode1
    g_th = two_stream_growth_rate(2 * math.pi / s.L, 0.2)
    t = np.arange(s.nsteps) * s.dt
    # the fit window of the oracle's gate: 12..4 time units before the mode-1
    # amplitude reaches 1% of ng in the oracle's own run of the same set-up
    x, v = s.particles()
    ref = O.run(oracle_params(p), x, v, s.nsteps, keep_E=True)
    amp_o = np.abs(_mode1(ref["E_hist"])) * s.ng
    t01 = t[int(np.argmax(amp_o > 0.01 * s.ng))]
    m = (t >= t01 - 12) & (t <= t01 - 4)
    gamma = np.polyfit(t[m], 0.5 * np.log(we[m]), 1)[0]
    assert abs(gamma / g_th - 1) < 0.02, gamma


# ------------------------------------------------------------- batching ---

def small_ensemble(n, seed=3):
    runs = I.ensemble(nruns=n, seed=seed, nsteps=30, np_scale=0.02)
    return runs


@pytest.mark.parametrize("cached", [None, "1"])
def test_batched_runs_equal_the_same_runs_alone(monkeypatch, cached):
    """Six runs of different (np, ng <= 2048) in one batch: state, grids and
    history equal each run stepped alone, bit for bit (shapes as tuned, and
    with cached particle accesses forced on both sides)."""
    if cached is not None:
        monkeypatch.setenv("PIC1D_CACHED", cached)
    specs = small_ensemble(6)
    parts = [s.particles() for s in specs]
    alone = []
    for s, (x, v) in zip(specs, parts):
        r, p = make_run(s, history=s.nsteps, x=x, v=v)
        with r:
            r.step(s.nsteps)
            alone.append((r.raw(), r.grid(), r.history()))
    b = P.pic_batch_create(1 << 30, 2048, max_runs=16, graph_steps=4, stream=P.current_stream())
    try:
        ids = []
        for s, (x, v) in zip(specs, parts):
            p = P.make_params(s.L, s.ng, s.np_, s.dt, history_cap=s.nsteps)
            ids.append(P.pic_batch_admit(b, p, x, v, s.nsteps))
        P.pic_batch_step(b, 100)                       # more than needed: runs stop at their own count
        for rid, s, (raw, grid, hist) in zip(ids, specs, alone):
            view = P.pic_batch_run(b, rid)
            u, w = P.pic_read_raw(view, s.np_)
            np.testing.assert_array_equal(u, raw[0])
            np.testing.assert_array_equal(w, raw[1])
            S, E, _ = P.pic_read_grid(view, s.ng)
            np.testing.assert_array_equal(S, grid[0])
            np.testing.assert_array_equal(E, grid[1])
            np.testing.assert_array_equal(P.pic_read_history(view, 0, s.nsteps), hist)
            d, _, _ = P.pic_diagnostics(view)
            assert d["step"] == s.nsteps
        done = P.pic_batch_poll(b)
        assert sorted(done) == sorted(ids)
    finally:
        P.pic_batch_destroy(b)


def test_batch_with_runs_dealt_round_robin_equals_runs_alone(monkeypatch):
    """A batch large enough for the work list to deal runs to chunks round
    robin: 19.7M particles in seven runs (10M down to 100k, ng 64..2048) at
    1024 threads (256 workgroups, 16 wavefronts each), so the chunk target
    is about 38K particles and every run but the smallest gets K >= 8 chunks
    of at least one tile per wavefront, taking tiles c, c + K, ... (the
    100K-particle run keeps consecutive tiles).  State, grids and history
    equal each run stepped alone, bit for bit."""
    monkeypatch.setenv("PIC1D_BLOCK", "1024")
    monkeypatch.setenv("PIC1D_UNROLL", "1")
    sizes = [(10_000_000, 2048), (5_000_000, 1024), (2_500_000, 512), (1_200_000, 2048), (600_000, 256),
             (300_000, 128), (100_000, 64)]
    specs = [I.warm_two_stream_large(seed=40 + k, np_=n, ng=ng, nsteps=9, L=0.032 * ng)
             for k, (n, ng) in enumerate(sizes)]
    parts = [s.particles() for s in specs]
    alone = []
    for s, (x, v) in zip(specs, parts):
        r, p = make_run(s, history=s.nsteps, x=x, v=v)
        with r:
            r.step(s.nsteps)
            alone.append((r.raw(), r.grid(), r.history()))
    b = P.pic_batch_create(2 << 30, 2048, max_runs=8, graph_steps=4, stream=P.current_stream())
    try:
        ids = [P.pic_batch_admit(b, P.make_params(s.L, s.ng, s.np_, s.dt, history_cap=s.nsteps), x, v, s.nsteps)
               for s, (x, v) in zip(specs, parts)]
        P.pic_batch_step(b, 20)
        for rid, s, (raw, grid, hist) in zip(ids, specs, alone):
            view = P.pic_batch_run(b, rid)
            u, w = P.pic_read_raw(view, s.np_)
            np.testing.assert_array_equal(u, raw[0])
            np.testing.assert_array_equal(w, raw[1])
            S, E, _ = P.pic_read_grid(view, s.ng)
            np.testing.assert_array_equal(S, grid[0])
            np.testing.assert_array_equal(E, grid[1])
            np.testing.assert_array_equal(P.pic_read_history(view, 0, s.nsteps), hist)
    finally:
        P.pic_batch_destroy(b)


@pytest.mark.parametrize("forced", [True, False])
def test_batch_switching_between_queued_and_unqueued_launches(monkeypatch, forced):
    """Three persistent workgroups (the configured grid, also when the batch
    tunes its shape) and runs of 8K-15K particles, about one work item each:
    six runs make a work list longer than the grid (items 3.. come through
    the queue's tickets); when three of them have finished the list fits the
    grid (nothing is queued, no ticket is drawn); two admissions lengthen it
    again.  Both kinds of launch must leave the queue's counter at 0 for the
    next, and every run equals the same run alone, bit for bit."""
    import torch
    if forced:
        monkeypatch.setenv("PIC1D_BLOCK", "512")
        monkeypatch.setenv("PIC1D_UNROLL", "1")
    sizes = [(15_000, 1024), (9_000, 64), (12_000, 256), (8_000, 512), (14_000, 128), (10_000, 1024),
             (13_000, 64), (11_000, 512)]
    steps = [4, 6, 8, 14, 16, 18, 9, 11]
    specs = [I.warm_two_stream_large(seed=60 + k, np_=n, ng=ng, nsteps=st, L=0.032 * ng)
             for k, ((n, ng), st) in enumerate(zip(sizes, steps))]
    parts = [s.particles() for s in specs]
    alone = []
    for s, (x, v) in zip(specs, parts):
        r, p = make_run(s, history=s.nsteps, x=x, v=v)
        with r:
            r.step(s.nsteps)
            alone.append((r.raw(), r.grid(), r.history()))
    b = P.pic_batch_create(1 << 30, 2048, max_runs=16, graph_steps=2, grid_blocks=3, stream=P.current_stream())
    try:
        params = [P.make_params(s.L, s.ng, s.np_, s.dt, history_cap=s.nsteps) for s in specs]
        ids = [P.pic_batch_admit(b, params[k], *parts[k], specs[k].nsteps) for k in range(6)]
        P.pic_batch_step(b, 10)                        # runs of 4, 6 and 8 steps finish
        torch.cuda.synchronize()                       # the poll reports completed device work only
        assert sorted(P.pic_batch_poll(b)) == sorted(ids[:3])
        ids += [P.pic_batch_admit(b, params[k], *parts[k], specs[k].nsteps) for k in (6, 7)]
        P.pic_batch_step(b, 30)
        for rid, s, (raw, grid, hist) in zip(ids, specs, alone):
            view = P.pic_batch_run(b, rid)
            u, w = P.pic_read_raw(view, s.np_)
            np.testing.assert_array_equal(u, raw[0])
            np.testing.assert_array_equal(w, raw[1])
            S, E, _ = P.pic_read_grid(view, s.ng)
            np.testing.assert_array_equal(S, grid[0])
            np.testing.assert_array_equal(E, grid[1])
            np.testing.assert_array_equal(P.pic_read_history(view, 0, s.nsteps), hist)
    finally:
        P.pic_batch_destroy(b)


def test_batch_mixing_solvers_and_step_counts_equals_runs_alone():
    """A batch of a run with the paper's CG solver (5 steps) and runs with the
    exact solver (14 to 20 steps): the solve launch shrinks as runs finish
    (a different captured graph), and every run, both solvers, equals the
    same run alone, bit for bit."""
    specs = small_ensemble(4, seed=12)
    specs = [dataclasses.replace(s, nsteps=5 if k == 0 else 11 + 3 * k) for k, s in enumerate(specs)]
    parts = [s.particles() for s in specs]
    solvers = [P.PIC_SOLVE_CG_PAPER] + [P.PIC_SOLVE_EXACT] * (len(specs) - 1)
    params = [P.make_params(s.L, s.ng, s.np_, s.dt, history_cap=s.nsteps, solver=sv)
              for s, sv in zip(specs, solvers)]
    alone = []
    for s, p, (x, v) in zip(specs, params, parts):
        with P.Run(p, x, v) as r:
            r.step(s.nsteps)
            alone.append((r.raw(), r.grid()[1], r.history()))
    b = P.pic_batch_create(1 << 30, 2048, max_runs=8, graph_steps=4, stream=P.current_stream())
    try:
        ids = [P.pic_batch_admit(b, p, x, v, s.nsteps) for s, p, (x, v) in zip(specs, params, parts)]
        P.pic_batch_step(b, 3)
        P.pic_batch_step(b, 100)                       # runs stop at their own step counts
        for rid, s, (raw, E, hist) in zip(ids, specs, alone):
            view = P.pic_batch_run(b, rid)
            u, w = P.pic_read_raw(view, s.np_)
            np.testing.assert_array_equal(u, raw[0])
            np.testing.assert_array_equal(w, raw[1])
            np.testing.assert_array_equal(P.pic_read_grid(view, s.ng)[1], E)
            np.testing.assert_array_equal(P.pic_read_history(view, 0, s.nsteps), hist)
    finally:
        P.pic_batch_destroy(b)


def test_admission_under_a_small_budget_and_release():
    """A budget that holds only some runs: admission reports EBUDGET, runs are
    admitted as others release, and every result equals the run alone."""
    specs = small_ensemble(5, seed=8)
    parts = [s.particles() for s in specs]
    foot = [P.pic_footprint(P.make_params(s.L, s.ng, s.np_, s.dt, history_cap=s.nsteps)) for s in specs]
    budget = int(max(foot) * 1.5)
    b = P.pic_batch_create(budget, 2048, max_runs=8, graph_steps=2, stream=P.current_stream())
    results = {}
    try:
        pending = list(range(len(specs)))
        active = {}
        refused = 0
        while pending or active:
            still = []
            for k in pending:
                s = specs[k]
                p = P.make_params(s.L, s.ng, s.np_, s.dt, history_cap=s.nsteps)
                try:
                    active[P.pic_batch_admit(b, p, *parts[k], s.nsteps)] = k
                except P.PicBudget:
                    refused += 1
                    still.append(k)
            pending = still
            P.pic_batch_step(b, 7)
            import torch
            torch.cuda.synchronize()
            for rid in P.pic_batch_poll(b):
                k = active.pop(rid)
                view = P.pic_batch_run(b, rid)
                results[k] = P.pic_read_raw(view, specs[k].np_)
                P.pic_batch_release(b, rid)
        assert refused > 0
        assert P.pic_batch_usage(b)[0] == 0
    finally:
        P.pic_batch_destroy(b)
    for k, s in enumerate(specs):
        r, _ = make_run(s, x=parts[k][0], v=parts[k][1])
        with r:
            r.step(s.nsteps)
            u, w = r.raw()
        np.testing.assert_array_equal(results[k][0], u)
        np.testing.assert_array_equal(results[k][1], w)


def test_results_do_not_depend_on_the_launch_shape(monkeypatch):
    """Tiles and summation orders are fixed by the run, so every launch shape
    the autotuner may pick (threads, vectors per lane, the order in which
    workgroups take tiles, non-temporal or cached particle accesses) gives
    bit-identical state, grid and history."""
    spec = I.warm_two_stream_large(seed=21, np_=200_003, ng=256, nsteps=12, L=0.032 * 256)
    x, v = spec.particles()
    ref = None
    for block, unroll, order, cached in [(1024, 1, 0, 0), (512, 2, 1, 1), (256, 4, 0, 1), (1024, 4, 1, 0),
                                         (640, 1, 1, 1), (768, 2, 0, 0), (1024, 1, 1, 1), (1024, 1, 0, 1)]:
        monkeypatch.setenv("PIC1D_BLOCK", str(block))
        monkeypatch.setenv("PIC1D_UNROLL", str(unroll))
        monkeypatch.setenv("PIC1D_TILE_ORDER", str(order))
        monkeypatch.setenv("PIC1D_CACHED", str(cached))
        run, p = make_run(spec, history=spec.nsteps, x=x, v=v)
        with run:
            run.step(spec.nsteps)
            got = (*run.raw(), run.grid()[0], run.grid()[1], run.history())
        if ref is None:
            ref = got
        else:
            for a, b in zip(ref, got):
                np.testing.assert_array_equal(a, b)


def test_batch_diagnostics_of_a_live_member_against_the_oracle():
    """pic_batch_diagnostics on a batch member that is still running (the
    two-stream run, 60 of its 200 steps taken, beside another run): the step
    count and exact charge, the kinetic energy K^{N-1/2}, the momentum
    P^{N-1/2} and the field energy W_E^N against the FP64 oracle's run of
    the same inputs, within the history bounds of the FP32 state; the same
    values as pic_diagnostics on the member's view; EINVAL for an unknown id."""
    spec = I.two_stream_small()
    other = small_ensemble(1, seed=5)[0]
    x, v = spec.particles()
    n = 60
    b = P.pic_batch_create(1 << 28, 2048, max_runs=4, graph_steps=8, stream=P.current_stream())
    try:
        p = P.make_params(spec.L, spec.ng, spec.np_, spec.dt)
        rid = P.pic_batch_admit(b, p, x, v, spec.nsteps)
        P.pic_batch_admit(b, P.make_params(other.L, other.ng, other.np_, other.dt), *other.particles(),
                          other.nsteps)
        P.pic_batch_step(b, n)
        d = P.pic_batch_diagnostics(b, rid)
        dv, _, _ = P.pic_diagnostics(P.pic_batch_run(b, rid))
        assert d == dv
        with pytest.raises(P.PicError) as e:
            P.pic_batch_diagnostics(b, 10_000)
        assert e.value.status == P.PIC_EINVAL
    finally:
        P.pic_batch_destroy(b)
    op = oracle_params(p)
    bounds, _, _ = HC.state_bounds(op, x, v, n + 1, (n + 1,))      # rows 0..n: the field E^n too
    bounds = bounds[n + 1]
    out = O.run(op, x, v, n, mode=O.DEPOSIT_FIXED)
    ref = out["hist"]
    assert d["step"] == n and d["charge_fixed_sum"] == spec.np_ << 32 and d["flags"] == 0
    kscale, pscale = np.abs(ref[:, 3]).max(), HC.momentum_scale(op, v)
    assert abs(d["kinetic"] - ref[-1, 3]) <= bounds["K"] * kscale
    assert abs(d["momentum"] - ref[-1, 2]) <= bounds["P"] * pscale
    we = O.field_energy(op, out["E"])
    assert abs(d["field"] - we) <= bounds["W_E"] * ref[:, 1].max()
    print(f"batch member diagnostics after {n} steps: kinetic {abs(d['kinetic'] - ref[-1, 3]) / kscale:.2e}, "
          f"momentum {abs(d['momentum'] - ref[-1, 2]) / pscale:.2e}, field "
          f"{abs(d['field'] - we) / ref[:, 1].max():.2e} of scale", flush=True)
