"""Device-side loader against the host generator.

The loader draws each particle from the same SplitMix64 counters and the
same formulas as paper_1108_1954_amd.inputs; only the device's sin, cos and
log1p may differ from the host library's in the last bit of an FP64 value.
So the FP32 state must equal the host-loaded state except where an FP64
value lies within an ulp of an FP32 rounding boundary (a few in 2^29), and
the FP64 state must agree to a few ulps."""
import numpy as np
import pytest

from paper_1108_1954_amd import inputs as I
from paper_1108_1954_amd import pic as P

pytestmark = pytest.mark.gpu

EPS64 = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    P.load()
    yield


CASES = {
    "two_stream": lambda: I.two_stream_small(np_=200_000),
    "maxwellian": lambda: I.warm_maxwellian_large(np_=1 << 21, ng=2048),
    "paper_weak_scaling": lambda: I.paper_weak_scaling(cores=4),
    "paper_two_stream": lambda: I.paper_two_stream(cores=4),
    "maxwellian_lattice": lambda: I.warm_maxwellian_small(),
}


@pytest.mark.parametrize("precision", [P.PIC_FP32, P.PIC_FP64])
@pytest.mark.parametrize("name", sorted(CASES))
def test_device_loader_equals_host_generator(name, precision):
    spec = CASES[name]()
    print(f"loader {name} np={spec.np_} precision={precision}", flush=True)
    x, v = spec.particles()
    p = P.make_params(spec.L, spec.ng, spec.np_, spec.dt, precision=precision)
    with P.Run(p, x, v) as host, P.Run(p, loader=P.make_loader(**spec.loader)) as dev:
        uh, wh = host.raw()
        ud, wd = dev.raw()
        Sh, Eh, _ = host.grid()
        Sd, Ed, _ = dev.grid()
    if precision == P.PIC_FP32:
        du = np.flatnonzero(uh != ud)
        dw = np.flatnonzero(wh != wd)
        assert du.size + dw.size <= 4, (du.size, dw.size)
        if du.size:
            assert np.all(np.abs(uh[du] - ud[du]) <= np.spacing(np.abs(uh[du]).astype(np.float32)))
        if dw.size:
            assert np.all(np.abs(wh[dw] - wd[dw]) <= np.spacing(np.abs(wh[dw]).astype(np.float32)))
        if du.size == 0:
            np.testing.assert_array_equal(Sh, Sd)          # same positions: same exact deposit
    else:
        assert np.max(np.abs(uh - ud)) <= 4 * EPS64 * spec.ng
        assert np.all(np.abs(wh - wd) <= 8 * EPS64 * np.abs(wh) + 1e-300)
    assert int(Sd.sum()) == spec.np_ << 32


def test_batch_admission_with_loader_equals_loaded_run_alone():
    specs = [I.two_stream_small(np_=30_000, nsteps=20), I.warm_maxwellian_large(np_=70_001, ng=512, nsteps=15)]
    alone = []
    for s in specs:
        p = P.make_params(s.L, s.ng, s.np_, s.dt, history_cap=s.nsteps)
        with P.Run(p, loader=P.make_loader(**s.loader)) as r:
            r.step(s.nsteps)
            alone.append((r.raw(), r.history()))
    b = P.pic_batch_create(1 << 28, 2048, max_runs=4, graph_steps=4, stream=P.current_stream())
    try:
        ids = [P.pic_batch_admit_loaded(b, P.make_params(s.L, s.ng, s.np_, s.dt, history_cap=s.nsteps),
                                        P.make_loader(**s.loader), s.nsteps) for s in specs]
        P.pic_batch_step(b, 50)
        for rid, s, (raw, hist) in zip(ids, specs, alone):
            view = P.pic_batch_run(b, rid)
            u, w = P.pic_read_raw(view, s.np_)
            np.testing.assert_array_equal(u, raw[0])
            np.testing.assert_array_equal(w, raw[1])
            np.testing.assert_array_equal(P.pic_read_history(view, 0, s.nsteps), hist)
    finally:
        P.pic_batch_destroy(b)
