"""Full-size runs on the GPU against the FP64 oracle and the physics.

  * Warm two-stream (np = 2^26, ng = 4096, 1000 steps): the engine's
    field-energy history W_E^n against the FP64 oracle's (stored by
    tests/golden/make_oracle_histories.py, oracle only).  The linear phase
    (until W_E first reaches 10% of its maximum) is deterministic growth from
    the same initial state; after saturation the dynamics are chaotic and the
    whole-run error is reported as a number, not held to a bound.
  * Warm Maxwellian (np = 2^28, ng = 8192, 2000 steps): the Langmuir
    oscillation of the loaded k = 0.5 mode must have the Bohm-Gross frequency
    with the leapfrog correction, and the FP32 and FP64-state histories are
    compared with the stored FP64 oracle history.
  * The batched ensemble (256 runs, ~1.45e8 particles) in the launch
    configuration the benchmark times: exact charge for every run, sampled
    runs' deposits bit-exact, fields and one step within the rounding bounds.

Inputs are the seeded generators of paper_1108_1954_amd.inputs.
"""
import math
import os

import numpy as np
import pytest

from paper_1108_1954_amd import inputs as I
from paper_1108_1954_amd import pic as P

import history_check as HC

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.load()
    yield


def golden(name):
    path = os.path.join(GOLDEN, f"oracle_history_{name}.txt")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written yet (tests/golden/make_oracle_histories.py {name})")
    return np.loadtxt(path)


def run_history(spec, x, v, precision=P.PIC_FP32, graph_steps=20):
    p = P.make_params(spec.L, spec.ng, spec.np_, spec.dt, precision=precision, history_cap=spec.nsteps)
    with P.Run(p, x, v) as r:
        r.step(spec.nsteps, graph_steps=graph_steps)
        d, _, _ = r.diagnostics()
        assert d["step"] == spec.nsteps and d["flags"] == 0
        assert d["charge_fixed_sum"] == spec.np_ << 32
        return r.history()


def history_errors(h, ref):
    """max_n |W_E^n - W_E,ref^n| / max_n W_E,ref^n over the linear phase and
    over the whole run."""
    we, wr = h[:, 1], ref[:, 1]
    scale = wr.max()
    err = np.abs(we - wr) / scale
    lin = int(np.argmax(wr >= 0.1 * scale))
    return float(err[:lin].max()), float(err.max()), lin


def column_report(name, h, ref, pscale, windows):
    """Errors of every history column (KE^n, W_E^n, P^{n+1/2}, K^{n+1/2})
    against the stored oracle history over each window of leading steps,
    printed and returned as {window: {column: error}}."""
    err = HC.column_errors(h, ref, pscale)
    out = {}
    for n in windows:
        out[n] = {c: float(err[c][:n].max()) for c in HC.COLS}
        print(f"{name}, first {n} steps: " + ", ".join(f"{c} {e:.3e}" for c, e in out[n].items()), flush=True)
    return out


def test_warm_two_stream_field_energy_history_vs_oracle():
    ref = golden("warm_two_stream")
    spec = I.warm_two_stream_large()
    print(f"warm two-stream np={spec.np_} ng={spec.ng} steps={spec.nsteps}", flush=True)
    x, v = spec.particles()
    h = run_history(spec, x, v)
    from oracle import oracle as O
    pscale = HC.momentum_scale(O.params(spec.L, spec.ng, spec.np_, dt=spec.dt), v)
    del x, v
    lin_err, all_err, lin = history_errors(h, ref)
    cols = column_report("warm two-stream FP32 state", h, ref, pscale, (lin, spec.nsteps))
    e0 = abs(h[0, 1] - ref[0, 1]) / ref[0, 1]
    print(f"W_E history vs FP64 oracle: step 0 rel. {e0:.3e}; linear phase (steps < {lin}) "
          f"{lin_err:.3e}; whole run {all_err:.3e}", flush=True)
    # Bounds at about 15x the measured errors (the oracle's own sensitivity
    # cannot be rerun at this size inside a test; the sizes are explained with
    # the tolerances of the design notes).  Measured: step 0 2.1e-8; linear
    # phase KE 7.0e-8, W_E 3.3e-7, P 6.0e-11, K 7.1e-8; P over the whole run
    # 5.5e-10 (momentum is conserved, so its error does not grow chaotically
    # as the energies' do after saturation, 9e-4 and 5e-3, which are reported).
    assert e0 < 3e-7
    lin_cols = cols[lin]
    assert lin_cols["KE"] < 1e-6 and lin_cols["K"] < 1e-6
    assert lin_cols["W_E"] < 5e-6 and lin_err == lin_cols["W_E"]
    assert lin_cols["P"] < 1e-9
    assert cols[spec.nsteps]["P"] < 1e-8
    # total energy (kinetic + field) is conserved alike: drift within 1e-3
    tot = h[:, 0] + h[:, 1]
    assert (tot.max() - tot.min()) / tot[0] < 1e-3


def oscillation_frequency(we, dt):
    """Angular frequency of the oscillating field energy, from the mean
    spacing of its successive maxima (parabolic refinement); W_E ~ cos^2 so
    the field oscillates at half the energy's frequency."""
    y = we - we.mean()
    peaks = [i for i in range(1, len(y) - 1) if y[i] > y[i - 1] and y[i] >= y[i + 1] and y[i] > 0]
    t = []
    for i in peaks:
        a, b, c = y[i - 1], y[i], y[i + 1]
        t.append((i + 0.5 * (a - c) / (a - 2 * b + c)) * dt)
    t = np.array(t)
    period_we = (t[-1] - t[0]) / (len(t) - 1)
    return math.pi / period_we


def test_warm_maxwellian_langmuir_frequency_and_precision():
    spec = I.warm_maxwellian_large()
    print(f"warm Maxwellian np={spec.np_} ng={spec.ng} steps={spec.nsteps}", flush=True)
    x, v = spec.particles()
    h32 = run_history(spec, x, v, P.PIC_FP32)
    h64 = run_history(spec, x, v, P.PIC_FP64)
    from oracle import oracle as O
    pscale = HC.momentum_scale(O.params(spec.L, spec.ng, spec.np_, dt=spec.dt), v)
    del x, v
    k, vth, dt = 0.5, 0.1, spec.dt
    w_bg = math.sqrt(1 + 3 * k * k * vth * vth)                  # Bohm-Gross
    w_lf = 2 / dt * math.asin(w_bg * dt / 2)                      # leapfrog dispersion
    for name, h in (("FP32", h32), ("FP64", h64)):
        w = oscillation_frequency(h[:, 1], dt)
        print(f"{name} state: Langmuir frequency {w:.5f} (Bohm-Gross with leapfrog {w_lf:.5f})", flush=True)
        assert abs(w / w_lf - 1) < 2e-3
    ref = golden("maxwellian")
    c32 = column_report("Maxwellian FP32 state", h32, ref, pscale, (spec.nsteps,))[spec.nsteps]
    c64 = column_report("Maxwellian FP64 state", h64, ref, pscale, (spec.nsteps,))[spec.nsteps]
    e32 = float(np.max(np.abs(h32[:, 1] - ref[:, 1])) / ref[:, 1].max())
    e64 = float(np.max(np.abs(h64[:, 1] - ref[:, 1])) / ref[:, 1].max())
    print(f"W_E history vs FP64 oracle over {spec.nsteps} steps: FP32 state {e32:.3e}, "
          f"FP64 state {e64:.3e}", flush=True)
    # A stable plasma: rounding differences do not grow exponentially as in
    # the two-stream run.  Bounds at 12-26x the measured errors (FP32 state:
    # KE 9.1e-9, W_E 4.2e-7, P 1.6e-10, K 9.1e-9; FP64 state: KE 1.2e-12,
    # W_E 3.1e-13, P 1.3e-13, K 1.5e-12).
    assert e64 <= e32
    assert e32 == c32["W_E"] and e64 == c64["W_E"]
    assert c32["KE"] < 2e-7 and c32["K"] < 2e-7 and c32["W_E"] < 5e-6 and c32["P"] < 3e-9
    assert c64["KE"] < 3e-11 and c64["K"] < 3e-11 and c64["W_E"] < 5e-12 and c64["P"] < 3e-12


def test_full_ensemble_in_the_bench_configuration():
    """The batched ensemble at full size (256 runs, ~1.45e8 particles), in
    the launch configuration bench.py times (persistent particle pass with
    the autotuned shape, graph replay of 20 steps): every run keeps its exact
    charge and raises no flag; on sampled runs the deposit of the downloaded
    state is bit-exact against the oracle, the field matches the oracle's
    solve of it, and one more step of sampled particles matches the oracle's
    gather and push within the rounding bound."""
    from concurrent.futures import ThreadPoolExecutor
    import test_gpu_parity as G
    from oracle import oracle as O
    specs = I.ensemble(nruns=256, seed=3, nsteps=500)
    with ThreadPoolExecutor(16) as ex:
        parts = list(ex.map(lambda s: s.particles(), specs))
    params = [P.make_params(s.L, s.ng, s.np_, s.dt) for s in specs]
    budget = int(sum(P.pic_footprint(p) for p in params) * 1.05) + (64 << 20)
    b = P.pic_batch_create(budget, max(s.ng for s in specs), max_runs=len(specs), graph_steps=20,
                           stream=P.current_stream())
    try:
        ids = [P.pic_batch_admit(b, p, x, v, 100) for p, (x, v) in zip(params, parts)]
        del parts
        P.pic_batch_step(b, 20)
        for rid, s in zip(ids, specs):
            d, _, _ = P.pic_diagnostics(P.pic_batch_run(b, rid))
            assert d["step"] == 20 and d["flags"] == 0
            assert d["charge_fixed_sum"] == s.np_ << 32
        order = np.argsort([s.np_ for s in specs])
        sample = sorted(set(int(order[k]) for k in np.linspace(0, len(specs) - 1, 8).astype(int)))
        rng = np.random.default_rng(0)
        state = {}
        for k in sample:
            s, p, view = specs[k], params[k], P.pic_batch_run(b, ids[k])
            u0, w0 = P.pic_read_raw(view, s.np_)
            S0, E0, Eh0 = P.pic_read_grid(view, s.ng)
            np.testing.assert_array_equal(S0, O.deposit_fixed(s.ng, u0.astype(np.float64)))
            op = G.oracle_params(p)
            E_ora, _ = O.solve(op, O.density_fixed(op, S0))
            np.testing.assert_allclose(E0, E_ora, rtol=0, atol=G.solve_tolerance(p, S0))
            pick = rng.choice(s.np_, size=min(s.np_, 200_000), replace=False)
            state[k] = (u0[pick], w0[pick], E_ora, np.abs(Eh0).max(), pick)
        P.pic_batch_step(b, 1)
        for k in sample:
            s, p, view = specs[k], params[k], P.pic_batch_run(b, ids[k])
            u0, w0, E_ora, eh_max, pick = state[k]
            u1, w1 = P.pic_read_raw(view, s.np_)
            dx = s.L / s.ng
            ops = O.params(s.L, s.ng, pick.size, dt=s.dt)
            x0 = u0.astype(np.float64) * dx
            v0 = w0.astype(np.float64) * dx / s.dt
            x1, v1, _ = O.push(ops, x0, v0, O.gather(ops, x0, E_ora))
            du, dw = G.push_tolerance(x1 / dx, v1 * s.dt / dx, eh_max, s.ng, G.EPS32)
            assert np.all(np.abs(w1[pick].astype(np.float64) - v1 * s.dt / dx) <= dw), k
            assert np.all(np.abs(G.periodic_diff(u1[pick], x1 / dx, s.ng)) <= du), k
            S1, _, _ = P.pic_read_grid(view, s.ng)
            np.testing.assert_array_equal(S1, O.deposit_fixed(s.ng, u1.astype(np.float64)))
        print(f"full ensemble: {len(specs)} runs, {sum(s.np_ for s in specs)} particles; "
              f"sampled runs {sample} checked", flush=True)
    finally:
        P.pic_batch_destroy(b)


def check_full_size_run(spec, p, r, sample=200_000, cg_iters=0):
    """After steps in the benchmark's configuration: the deposit of the
    downloaded state is bit-exact, the field equals the oracle's solve of it
    (exact solve, or the paper's CG with the same iteration count) within
    its bound, and one more step of a sample of particles matches the
    oracle's gather and push within the rounding bound."""
    import test_gpu_parity as G
    import test_gpu_cg as CG
    from oracle import oracle as O
    u0, w0 = r.raw()
    S0, E0, Eh0 = r.grid()
    np.testing.assert_array_equal(S0, O.deposit_fixed(spec.ng, u0.astype(np.float64)))
    assert int(S0.sum()) == spec.np_ << 32
    op = G.oracle_params(p)
    rho = O.density_fixed(op, S0)
    if cg_iters:
        _, E_ora, _ = O.cg_paper(op, rho, maxit=cg_iters)
        spread = np.abs(CG.cg_numpy(rho, spec.L / spec.ng, cg_iters) - E_ora).max()
        tol = 10 * spread + 16 * spec.ng * G.EPS64 * np.abs(E_ora).max()
    else:
        E_ora, _ = O.solve(op, rho)
        tol = G.solve_tolerance(p, S0)
    assert np.abs(E0 - E_ora).max() <= tol
    pick = np.random.default_rng(1).choice(spec.np_, size=min(spec.np_, sample), replace=False)
    r.step(1, graph_steps=0)
    u1, w1 = r.raw()
    dx = spec.L / spec.ng
    ops = O.params(spec.L, spec.ng, pick.size, dt=spec.dt)
    x0 = u0[pick].astype(np.float64) * dx
    v0 = w0[pick].astype(np.float64) * dx / spec.dt
    x1, v1, _ = O.push(ops, x0, v0, O.gather(ops, x0, E_ora))
    du, dw = G.push_tolerance(x1 / dx, v1 * spec.dt / dx, np.abs(Eh0).max(), spec.ng, G.EPS32)
    assert np.all(np.abs(w1[pick].astype(np.float64) - v1 * spec.dt / dx) <= dw)
    assert np.all(np.abs(G.periodic_diff(u1[pick], x1 / dx, spec.ng)) <= du)
    S1, _, _ = r.grid()
    np.testing.assert_array_equal(S1, O.deposit_fixed(spec.ng, u1.astype(np.float64)))


def test_single_large_run_in_the_bench_configuration():
    """The warm two-stream run at full size (2^26 particles, ng 4096) as the
    benchmark's single-run line times it: autotuned shape, graph replay."""
    spec = I.warm_two_stream_large()
    print(f"full-size single run np={spec.np_} ng={spec.ng}", flush=True)
    x, v = spec.particles()
    p = P.make_params(spec.L, spec.ng, spec.np_, spec.dt)
    with P.Run(p, x, v) as r:
        del x, v
        r.step(20, graph_steps=20)
        d, _, _ = r.diagnostics()
        assert d["step"] == 20 and d["flags"] == 0
        check_full_size_run(spec, p, r)


@pytest.mark.parametrize("solver", [P.PIC_SOLVE_EXACT, P.PIC_SOLVE_CG_PAPER])
def test_paper_workload_in_the_bench_configuration(solver):
    """The paper's weak-scaling workload at its 128-thread size (ng 8192,
    8.192M particles, lattice start drawn on the device), with the exact
    solve and with the paper's 150-iteration CG."""
    spec = I.paper_weak_scaling(cores=128)
    print(f"paper workload np={spec.np_} ng={spec.ng} solver={solver}", flush=True)
    p = P.make_params(spec.L, spec.ng, spec.np_, spec.dt, solver=solver, cg_iters=150)
    with P.Run(p, loader=P.make_loader(**spec.loader)) as r:
        r.step(20, graph_steps=20)
        d, _, _ = r.diagnostics()
        assert d["step"] == 20 and d["flags"] == 0
        check_full_size_run(spec, p, r, cg_iters=150 if solver == P.PIC_SOLVE_CG_PAPER else 0)
