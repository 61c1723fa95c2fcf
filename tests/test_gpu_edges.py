"""Edge cases of the batch and the run API on the GPU: the largest grid in a
batch, releasing an unfinished run and reusing its slot and memory,
admission errors, a history shorter than the run, and the bandwidth probe's
swap with both cache policies."""
import ctypes

import numpy as np
import pytest

from paper_1108_1954_amd import inputs as I
from paper_1108_1954_amd import pic as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.load()
    yield


def alone(spec, x, v, nsteps):
    p = P.make_params(spec.L, spec.ng, spec.np_, spec.dt, history_cap=nsteps)
    with P.Run(p, x, v) as r:
        r.step(nsteps)
        return r.raw(), r.history()


def test_batch_at_the_largest_grid_mixes_ng_8192_and_64():
    big = I.warm_two_stream_large(np_=300_001, ng=8192, nsteps=12, L=0.032 * 8192)
    small = I.two_stream_small(np_=5_003, nsteps=12)
    parts = [big.particles(), small.particles()]
    ref = [alone(s, x, v, s.nsteps) for s, (x, v) in zip((big, small), parts)]
    b = P.pic_batch_create(1 << 30, P.PIC_MAX_NG, max_runs=4, graph_steps=4, stream=P.current_stream())
    try:
        ids = [P.pic_batch_admit(b, P.make_params(s.L, s.ng, s.np_, s.dt, history_cap=s.nsteps), x, v, s.nsteps)
               for s, (x, v) in zip((big, small), parts)]
        P.pic_batch_step(b, 50)
        for rid, s, (raw, hist) in zip(ids, (big, small), ref):
            view = P.pic_batch_run(b, rid)
            u, w = P.pic_read_raw(view, s.np_)
            np.testing.assert_array_equal(u, raw[0])
            np.testing.assert_array_equal(w, raw[1])
            np.testing.assert_array_equal(P.pic_read_history(view, 0, s.nsteps), hist)
    finally:
        P.pic_batch_destroy(b)


def test_release_of_an_unfinished_run_frees_its_slot_and_memory():
    """A run released before its last step stops; a new run admitted into
    the freed slot and arena span gives the same result as alone."""
    a = I.two_stream_small(np_=40_000, nsteps=500)
    c = I.warm_maxwellian_large(np_=50_003, ng=256, nsteps=17)
    xa, va = a.particles()
    xc, vc = c.particles()
    foot = P.pic_footprint(P.make_params(a.L, a.ng, a.np_, a.dt, history_cap=a.nsteps))
    b = P.pic_batch_create(foot + (1 << 20), 2048, max_runs=1, graph_steps=4, stream=P.current_stream())
    try:
        ra = P.pic_batch_admit(b, P.make_params(a.L, a.ng, a.np_, a.dt, history_cap=a.nsteps), xa, va, a.nsteps)
        P.pic_batch_step(b, 9)
        with pytest.raises(P.PicBudget):                 # table full (one slot) and arena full
            P.pic_batch_admit(b, P.make_params(c.L, c.ng, c.np_, c.dt, history_cap=c.nsteps), xc, vc, c.nsteps)
        d, _, _ = P.pic_diagnostics(P.pic_batch_run(b, ra))
        assert d["step"] == 9
        P.pic_batch_release(b, ra)
        assert P.pic_batch_usage(b) == (0, P.pic_batch_usage(b)[1], 0)
        rc = P.pic_batch_admit(b, P.make_params(c.L, c.ng, c.np_, c.dt, history_cap=c.nsteps), xc, vc, c.nsteps)
        P.pic_batch_step(b, 40)
        import torch
        torch.cuda.synchronize()
        assert P.pic_batch_poll(b) == [rc]
        view = P.pic_batch_run(b, rc)
        raw, hist = alone(c, xc, vc, c.nsteps)
        u, w = P.pic_read_raw(view, c.np_)
        np.testing.assert_array_equal(u, raw[0])
        np.testing.assert_array_equal(w, raw[1])
        np.testing.assert_array_equal(P.pic_read_history(view, 0, c.nsteps), hist)
    finally:
        P.pic_batch_destroy(b)


def test_admission_errors_leave_the_batch_usable():
    s = I.two_stream_small(np_=3_000, nsteps=5)
    x, v = s.particles()
    b = P.pic_batch_create(1 << 26, 32, max_runs=2, graph_steps=0, stream=P.current_stream())
    try:
        with pytest.raises(P.PicError) as e:                # ng 64 > ng_max 32
            P.pic_batch_admit(b, P.make_params(s.L, s.ng, s.np_, s.dt), x, v, s.nsteps)
        assert e.value.status == P.PIC_EINVAL
        with pytest.raises(P.PicError) as e:                # batches hold FP32 state
            P.pic_batch_admit(b, P.make_params(s.L, 32, s.np_, s.dt, precision=P.PIC_FP64), x, v, s.nsteps)
        assert e.value.status == P.PIC_EINVAL
        xb = x.copy()
        xb[7] = s.L                                          # outside [0, L)
        with pytest.raises(P.PicError) as e:
            P.pic_batch_admit(b, P.make_params(s.L, 32, s.np_, s.dt), xb, v, s.nsteps)
        assert e.value.status == P.PIC_EINVAL
        rid = P.pic_batch_admit(b, P.make_params(s.L, 32, s.np_, s.dt), x, v, s.nsteps)
        P.pic_batch_step(b, 10)
        d, _, _ = P.pic_diagnostics(P.pic_batch_run(b, rid))
        assert d["step"] == s.nsteps and d["charge_fixed_sum"] == s.np_ << 32
    finally:
        P.pic_batch_destroy(b)


def test_history_shorter_than_the_run():
    s = I.two_stream_small(np_=4_000, nsteps=30)
    x, v = s.particles()
    full = P.make_params(s.L, s.ng, s.np_, s.dt, history_cap=s.nsteps)
    short = P.make_params(s.L, s.ng, s.np_, s.dt, history_cap=10)
    with P.Run(full, x, v) as a, P.Run(short, x, v) as b:
        a.step(s.nsteps)
        b.step(s.nsteps)
        np.testing.assert_array_equal(b.history(0, 10), a.history(0, 10))
        with pytest.raises(P.PicError) as e:
            b.history(5, 10)                                 # rows 10..14 were never kept
        assert e.value.status == P.PIC_EINVAL
        for ra, rb in zip(a.raw(), b.raw()):
            np.testing.assert_array_equal(ra, rb)


def test_run_stays_inside_its_footprint():
    """A run created in caller memory of exactly pic_footprint() bytes (the
    particle state, grids, history and the device descriptor) writes nothing
    past it: a guard region after the span keeps its pattern through
    creation, graph-replayed steps, a sort and the diagnostics."""
    import torch
    spec = I.warm_two_stream_large(seed=31, np_=50_001, ng=512, nsteps=12, L=0.032 * 512)
    x, v = spec.particles()
    p = P.make_params(spec.L, spec.ng, spec.np_, spec.dt, history_cap=spec.nsteps, sort_every=5)
    need = P.pic_footprint(p)
    guard = 64 << 10
    buf = torch.empty(need + guard + 256, dtype=torch.uint8, device="cuda")
    off = (-buf.data_ptr()) % 256
    buf[off + need:off + need + guard].fill_(0xA5)
    torch.cuda.synchronize()
    h = P.pic_create(p, x, v, buf.data_ptr() + off, need, P.current_stream())
    try:
        P.pic_step_graph(h, spec.nsteps, 4)
        d, _, _ = P.pic_diagnostics(h, 0)
        assert d["step"] == spec.nsteps and d["flags"] == 0
    finally:
        P.pic_destroy(h)
    torch.cuda.synchronize()
    tail = buf[off + need:off + need + guard].cpu().numpy()
    assert (tail == 0xA5).all(), f"{int((tail != 0xA5).sum())} guard bytes overwritten"


@pytest.mark.parametrize("cached", [False, True])
def test_bandwidth_probe_swaps_the_arrays(cached):
    """pic_bandwidth_probe launches the swap reps + 1 times (one warm-up):
    the arrays end swapped for even reps and unchanged for odd reps, with
    either cache policy, over a ragged vector count; bad arguments are
    EINVAL."""
    import torch
    n = 4 * 300_001
    a0 = torch.arange(n, dtype=torch.float32, device="cuda")
    b0 = -a0 - 1.0
    for reps, swapped in ((2, True), (1, False)):
        a, b = a0.clone(), b0.clone()
        torch.cuda.synchronize()
        ms = P.pic_bandwidth_probe(a.data_ptr(), b.data_ptr(), n, reps=reps, stream=P.current_stream(),
                                   cached=cached)
        assert ms > 0
        assert torch.equal(a, b0 if swapped else a0) and torch.equal(b, a0 if swapped else b0)
    with pytest.raises(P.PicError) as e:
        P.pic_bandwidth_probe(a0.data_ptr(), b0.data_ptr(), n - 2, reps=1, stream=P.current_stream())
    assert e.value.status == P.PIC_EINVAL
    out = ctypes.c_double(0)
    st = P.load().pic_bandwidth_probe(a0.data_ptr(), b0.data_ptr(), n, 1, 2, P.current_stream(), ctypes.byref(out))
    assert st == P.PIC_EINVAL                                  # cached must be 0 or 1


@pytest.mark.slow
def test_largest_particle_count_and_grid():
    """np = 2^31 - 1 (the largest the ABI takes) on the largest grid
    (8192 nodes), drawn on the device: the charge total np 2^32 is held
    exactly in int64 (just below 2^63), no flag is raised, and the deposit
    of the downloaded state is bit-exact against the oracle."""
    from oracle import oracle as O
    np_ = (1 << 31) - 1
    spec = I.warm_maxwellian_large(np_=np_, ng=P.PIC_MAX_NG, nsteps=2)
    print(f"largest run: np={np_} ng={spec.ng}", flush=True)
    p = P.make_params(spec.L, spec.ng, np_, spec.dt)
    with P.Run(p, loader=P.make_loader(**spec.loader)) as r:
        r.step(2)
        d, _, _ = r.diagnostics()
        assert d["step"] == 2 and d["flags"] == 0
        assert d["charge_fixed_sum"] == np_ << 32
        u, _ = r.raw()
        S, _, _ = r.grid()
    np.testing.assert_array_equal(S, O.deposit_fixed(spec.ng, u))
