"""pic_phase_space_noalloc (the allocation-free variant, binned in the
library's fixed device scratch) against pic_phase_space (which allocates its
scratch per call), through the C ABI: two calls in a row on different runs,
the first at the largest image the scratch holds, the second with a smaller
image and fewer particles (the scratch keeps the first call's counts, so a
missing clear would show), then the first again.  Integer images: bit-exact,
and equal to the oracle's counts of the downloaded state."""
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


def both(run, spec, nx, nv, vmin, vmax):
    a, out_a = P.pic_phase_space_noalloc(run.handle, nx, nv, vmin, vmax)
    b, out_b = P.pic_phase_space(run.handle, nx, nv, vmin, vmax)
    np.testing.assert_array_equal(a, b)
    assert out_a == out_b and int(a.sum()) + out_a == spec.np_
    u, w = run.raw()
    ref, ref_out = O.phase_space(O.params(spec.L, spec.ng, spec.np_, dt=spec.dt), u, w, nx, nv, vmin, vmax)
    np.testing.assert_array_equal(a, ref)
    assert out_a == ref_out
    return a, out_a


def test_noalloc_phase_space_equals_the_allocating_call():
    big = I.paper_two_stream(cores=1)                     # 64,000 particles, ng 64
    small = I.two_stream_small(np_=5_003, nsteps=20)
    print(f"no-alloc phase space: np {big.np_} at 128 x 128 bins, then np {small.np_} at 16 x 8", flush=True)
    pb = P.make_params(big.L, big.ng, big.np_, big.dt)
    xs, vs = small.particles()
    ps = P.make_params(small.L, small.ng, small.np_, small.dt)
    with P.Run(pb, loader=P.make_loader(**big.loader)) as rb, P.Run(ps, xs, vs) as rs:
        rb.step(40)
        rs.step(small.nsteps)
        first, _ = both(rb, big, 128, 128, -0.6, 0.6)       # 16384 bins: the whole scratch
        assert int(first.sum()) > 0
        second, _ = both(rs, small, 16, 8, -0.25, 0.25)     # smaller image, fewer particles
        again, _ = both(rb, big, 128, 128, -0.6, 0.6)
        np.testing.assert_array_equal(again, first)
        with pytest.raises(P.PicError) as e:                # beyond the scratch's capacity
            P.pic_phase_space_noalloc(rb.handle, 129, 128, -0.6, 0.6)
        assert e.value.status == P.PIC_EINVAL and "scratch" in str(e.value)
