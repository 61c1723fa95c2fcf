"""Device phase-space binning (pic_phase_space) against the oracle's counts
of the same downloaded state: integer images, so bit-exact, in both state
precisions, at the largest image, after a cell sort and for a batch member."""
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


def oracle_image(spec, u, w, nx, nv, vmin, vmax):
    return O.phase_space(O.params(spec.L, spec.ng, spec.np_, dt=spec.dt), u, w, nx, nv, vmin, vmax)


@pytest.mark.parametrize("precision", [P.PIC_FP32, P.PIC_FP64])
def test_two_stream_figure_run_phase_space(precision):
    spec = I.paper_two_stream(cores=1)
    print(f"phase space: paper two-stream np={spec.np_} precision={precision}", flush=True)
    p = P.make_params(spec.L, spec.ng, spec.np_, spec.dt, precision=precision)
    with P.Run(p, loader=P.make_loader(**spec.loader)) as r:
        img0, out0 = r.phase_space(64, 48, -0.6, 0.6)
        r.step(spec.nsteps)
        img, out = r.phase_space(64, 48, -0.6, 0.6)
        u, w = r.raw()
    assert out0 == 0 and len(np.flatnonzero(img0.sum(axis=1))) == 2     # two cold beams at t = 0
    ref, ref_out = oracle_image(spec, u, w, 64, 48, -0.6, 0.6)
    np.testing.assert_array_equal(img, ref)
    assert out == ref_out and int(img.sum()) + out == spec.np_
    assert len(np.flatnonzero(img.sum(axis=1))) > 2                      # mixed by t = 20


def test_large_run_largest_image_and_outside_counts():
    spec = I.warm_two_stream_large(np_=(1 << 24) + 777, ng=4096, nsteps=10)
    x, v = spec.particles()
    print(f"phase space: warm two-stream np={spec.np_}", flush=True)
    p = P.make_params(spec.L, spec.ng, spec.np_, spec.dt)
    with P.Run(p, x, v) as r:
        r.step(spec.nsteps)
        u, w = r.raw()
        outs = []
        for nx, nv, lo, hi in ((128, 128, -0.3, 0.3), (16384, 1, -0.1, 0.1), (1, 16384, -0.25, 0.25)):
            img, out = r.phase_space(nx, nv, lo, hi)
            ref, ref_out = oracle_image(spec, u, w, nx, nv, lo, hi)
            np.testing.assert_array_equal(img, ref)
            assert out == ref_out and int(img.sum()) + out == spec.np_
            outs.append(out)
        assert outs[1] > spec.np_ // 2                    # the beams at +-0.2 lie outside [-0.1, 0.1)


def test_sorted_run_has_the_same_image():
    spec = I.warm_two_stream_large(np_=300_001, ng=1024, nsteps=6)
    x, v = spec.particles()
    p = P.make_params(spec.L, spec.ng, spec.np_, spec.dt)
    ps = P.make_params(spec.L, spec.ng, spec.np_, spec.dt, sort_every=1 << 30)     # sorted on request only
    with P.Run(p, x, v) as a, P.Run(ps, x, v) as b:
        a.step(spec.nsteps)
        b.step(spec.nsteps)
        b.sort()
        ia = a.phase_space(100, 60, -0.35, 0.35)
        ib = b.phase_space(100, 60, -0.35, 0.35)
    np.testing.assert_array_equal(ia[0], ib[0])
    assert ia[1] == ib[1]


def test_batch_member_phase_space():
    spec = I.two_stream_small(np_=40_000, nsteps=30)
    x, v = spec.particles()
    b = P.pic_batch_create(1 << 27, 64, max_runs=2, graph_steps=4, stream=P.current_stream())
    try:
        rid = P.pic_batch_admit(b, P.make_params(spec.L, spec.ng, spec.np_, spec.dt), x, v, spec.nsteps)
        P.pic_batch_step(b, 12)
        view = P.pic_batch_run(b, rid)
        img, out = P.pic_phase_space(view, 32, 20, -0.5, 0.5)
        u, w = P.pic_read_raw(view, spec.np_)
        ref, ref_out = oracle_image(spec, u, w, 32, 20, -0.5, 0.5)
        np.testing.assert_array_equal(img, ref)
        assert out == ref_out
    finally:
        P.pic_batch_destroy(b)


@pytest.mark.parametrize("args", [(129, 128, -1.0, 1.0), (0, 4, -1.0, 1.0), (4, 4, 1.0, 1.0),
                                  (4, 4, float("nan"), 1.0), (4, 4, -1.0, float("inf"))])
def test_invalid_requests(args):
    spec = I.two_stream_small(np_=1000, nsteps=1)
    x, v = spec.particles()
    p = P.make_params(spec.L, spec.ng, spec.np_, spec.dt)
    with P.Run(p, x, v) as r:
        with pytest.raises(P.PicError) as e:
            r.phase_space(*args)
        assert e.value.status == P.PIC_EINVAL
        r.step(1)                                           # the run stays usable
        img, out = r.phase_space(8, 8, -1.0, 1.0)
        assert int(img.sum()) + out == spec.np_
