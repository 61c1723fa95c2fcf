"""GPU cell sort against the oracle's stable cell order, and the sort's
effect on a run: none on the physics (positions, velocities and the
fixed-point grid are the same multiset / the same bits), and the same
order whether the steps are launched plainly, from graphs, alone or in a
batch.  Every call goes through the C ABI."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1108_1954_amd import inputs as I
from paper_1108_1954_amd import pic as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.load()
    yield


def uniform_state(np_, ng, seed, cold=False):
    L = 0.032 * ng
    x = L * I.uniform(seed, 0, np_)
    if cold:                                    # all particles in a few cells
        x = (x * 3.0 / ng) % L
    v = 0.1 * I.normal(seed, 1, np_)
    return L, x, v


@pytest.mark.parametrize("precision", [P.PIC_FP32, P.PIC_FP64])
@pytest.mark.parametrize("np_,ng,cold", [(1, 2, False), (1000, 3, False), (70000, 64, False),
                                         (300001, 2048, False), (200003, 512, True),
                                         (3000000, 8192, False)])
def test_sort_equals_the_oracle_cell_order(precision, np_, ng, cold):
    print(f"sort parity np={np_} ng={ng} cold={cold} precision={precision}", flush=True)
    L, x, v = uniform_state(np_, ng, seed=np_ % 1000 + ng, cold=cold)
    p = P.make_params(L, ng, np_, 0.1, precision=precision, sort_every=1000)
    with P.Run(p, x, v) as r:
        u0, w0 = r.raw()
        r.sort()
        u1, w1 = r.raw()
        perm = O.cell_order(ng, u0.astype(np.float64))
        np.testing.assert_array_equal(u1, u0[perm])
        np.testing.assert_array_equal(w1, w0[perm])
        r.sort()                                  # sorted input: unchanged
        u2, w2 = r.raw()
        np.testing.assert_array_equal(u2, u1)
        np.testing.assert_array_equal(w2, w1)
        d, _, _ = r.diagnostics()
        assert d["flags"] == 0


def by_particle(u, w):
    k = np.lexsort((w, u))
    return u[k], w[k]


@pytest.mark.parametrize("graph_steps", [0, 4])
def test_sorting_leaves_the_physics_unchanged(graph_steps):
    spec = I.two_stream_small(np_=50000, nsteps=30)
    x, v = spec.particles()
    hist = spec.nsteps
    plain = P.make_params(spec.L, spec.ng, spec.np_, spec.dt, history_cap=hist)
    sorted_ = P.make_params(spec.L, spec.ng, spec.np_, spec.dt, history_cap=hist, sort_every=7)
    with P.Run(plain, x, v) as a, P.Run(sorted_, x, v) as b:
        a.step(spec.nsteps)
        b.step(spec.nsteps, graph_steps=graph_steps)
        ua, wa = by_particle(*a.raw())
        ub, wb = by_particle(*b.raw())
        np.testing.assert_array_equal(ua, ub)
        np.testing.assert_array_equal(wa, wb)
        Sa, Ea, _ = a.grid()
        Sb, Eb, _ = b.grid()
        np.testing.assert_array_equal(Sa, Sb)
        np.testing.assert_array_equal(Ea, Eb)
        ha, hb = a.history(), b.history()
        np.testing.assert_array_equal(ha[:, 1], hb[:, 1])           # field energy: same bits
        # kinetic energy and momentum are FP64 sums of the same terms in
        # another order: each side's recursive-summation error is at most
        # np eps sum|term|, so they differ by at most twice that
        EPS64 = 2.0 ** -53
        n = spec.np_
        np.testing.assert_allclose(hb[:, [0, 3]], ha[:, [0, 3]], rtol=2 * n * EPS64, atol=0)
        m = spec.rho0 * spec.L / n
        _, vfin = a.particles()
        bound = 2 * n * EPS64 * m * np.abs(vfin).sum() * 1.5      # |v| over the run: within 1.5x the final
        assert np.max(np.abs(hb[:, 2] - ha[:, 2])) <= bound
        assert b.diagnostics()[0]["flags"] == 0


def test_graph_and_plain_sorting_runs_are_identical():
    spec = I.two_stream_small(np_=40000, nsteps=45)
    x, v = spec.particles()
    p = P.make_params(spec.L, spec.ng, spec.np_, spec.dt, history_cap=spec.nsteps, sort_every=5)
    with P.Run(p, x, v) as a, P.Run(p, x, v) as b:
        a.step(spec.nsteps)
        b.step(17, graph_steps=4)                 # graphs with and without a sort at the start
        b.step(spec.nsteps - 17, graph_steps=3)
        for ra, rb in zip(a.raw(), b.raw()):
            np.testing.assert_array_equal(ra, rb)
        np.testing.assert_array_equal(a.history(), b.history())


def test_batched_sorting_runs_equal_the_same_runs_alone():
    specs = I.ensemble(nruns=5, seed=12, nsteps=25, np_scale=0.02)
    parts = [s.particles() for s in specs]
    every = [3, 0, 7, 1, 10]
    alone = []
    for s, (x, v), k in zip(specs, parts, every):
        p = P.make_params(s.L, s.ng, s.np_, s.dt, history_cap=s.nsteps, sort_every=k)
        with P.Run(p, x, v) as r:
            r.step(s.nsteps)
            alone.append((r.raw(), r.history()))
    b = P.pic_batch_create(1 << 30, 2048, max_runs=8, graph_steps=4, stream=P.current_stream())
    try:
        ids = []
        for s, (x, v), k in zip(specs, parts, every):
            p = P.make_params(s.L, s.ng, s.np_, s.dt, history_cap=s.nsteps, sort_every=k)
            ids.append(P.pic_batch_admit(b, p, x, v, s.nsteps))
        P.pic_batch_step(b, 11)
        P.pic_batch_step(b, 100)
        for rid, s, (raw, hist) in zip(ids, specs, alone):
            view = P.pic_batch_run(b, rid)
            u, w = P.pic_read_raw(view, s.np_)
            np.testing.assert_array_equal(u, raw[0])
            np.testing.assert_array_equal(w, raw[1])
            np.testing.assert_array_equal(P.pic_read_history(view, 0, s.nsteps), hist)
    finally:
        P.pic_batch_destroy(b)


def test_auto_sort_period_leaves_no_trace_and_equals_its_fixed_period():
    """sort_every = PIC_SORT_AUTO: the creation-time trial (passes on the
    loaded state, a sort, passes on the sorted state) puts the state back,
    and the run then behaves exactly like one created with the period it
    chose."""
    spec = I.warm_two_stream_large(np_=2_000_003, ng=1024, nsteps=30, L=0.032 * 1024)
    x, v = spec.particles()

    def params(k):
        return P.make_params(spec.L, spec.ng, spec.np_, spec.dt, sort_every=k, history_cap=spec.nsteps)
    with P.Run(params(P.PIC_SORT_AUTO), x, v) as a, P.Run(params(0), x, v) as z:
        k = a.sort_period()
        print(f"auto sort period np={spec.np_} ng={spec.ng}: K = {k}", flush=True)
        assert k >= 0 and z.sort_period() == 0
        for ra, rz in zip(a.raw(), z.raw()):
            np.testing.assert_array_equal(ra, rz)
        for ga, gz in zip(a.grid(), z.grid()):
            np.testing.assert_array_equal(ga, gz)
        with P.Run(params(k), x, v) as b:
            a.step(spec.nsteps, graph_steps=10)
            b.step(spec.nsteps, graph_steps=10)
            for ra, rb in zip(a.raw(), b.raw()):
                np.testing.assert_array_equal(ra, rb)
            np.testing.assert_array_equal(a.history(), b.history())
            da, _, _ = a.diagnostics()
            assert da["step"] == spec.nsteps and da["flags"] == 0


def test_batches_reject_the_auto_sort_period():
    spec = I.two_stream_small(np_=3_000, nsteps=5)
    x, v = spec.particles()
    b = P.pic_batch_create(1 << 26, 64, max_runs=2, graph_steps=0, stream=P.current_stream())
    try:
        with pytest.raises(P.PicError) as e:
            P.pic_batch_admit(b, P.make_params(spec.L, spec.ng, spec.np_, spec.dt, sort_every=P.PIC_SORT_AUTO),
                              x, v, spec.nsteps)
        assert e.value.status == P.PIC_EINVAL
    finally:
        P.pic_batch_destroy(b)
