"""The seeded input generators (host side, no GPU): the quiet-start lattice
against the appendix's per-cell load, and the beam signs and Maxwellian
spread of the loader description."""
import math

import numpy as np

from paper_1108_1954_amd import inputs as I


def test_lattice_is_the_appendix_per_cell_load():
    # appendix: cell ig, particle ii of ppc: x = ig dx + (ii + 1/2) dx / ppc
    for ng, ppc, L in ((64, 1000, 3.1415), (256, 1000, 4 * 3.1415), (8, 3, 1.0)):
        dx = L / ng
        ig, ii = np.divmod(np.arange(ng * ppc), ppc)
        ref = ig * dx + (ii + 0.5) * (dx / ppc)
        x = I.lattice(ng * ppc, L)
        assert np.max(np.abs(x - ref)) <= 4 * np.spacing(L)
        assert np.all(np.diff(x) > 0) and 0 < x[0] and x[-1] < L


def test_beam_signs_and_spread():
    L, n = 2.0, 200_000
    x, v = I.loaded(L, n, seed=11, v0=0.3, beams=1)
    assert np.all(v[0::2] == 0.3) and np.all(v[1::2] == -0.3)
    x, v = I.loaded(L, n, seed=11, v0=0.3, beams=2)
    plus = np.mean(v > 0)
    assert set(np.unique(v)) == {-0.3, 0.3}
    assert abs(plus - 0.5) < 5 / math.sqrt(n)              # binomial, 10 sigma
    # neighbours independent: the sign pattern is not the alternating one
    assert 0.4 < np.mean(v[1:] != v[:-1]) < 0.6
    x, v = I.loaded(L, n, seed=12, vth=0.1, lattice_start=True)
    assert abs(v.mean()) < 5 * 0.1 / math.sqrt(n)
    assert abs(v.std() / 0.1 - 1) < 0.01
    np.testing.assert_array_equal(x, I.lattice(n, L))


def test_displaced_positions_stay_in_the_box():
    L, n = 1.0, 100_000
    x, _ = I.loaded(L, n, seed=3, amp=0.2, k=2 * math.pi / L, lattice_start=True)
    assert np.all((0 <= x) & (x < L))


def test_paper_workloads_have_the_appendix_sizes():
    s = I.paper_weak_scaling(cores=128, nsteps=1)
    assert (s.ng, s.np_, s.dt, s.nsteps) == (8192, 8_192_000, 0.1, 1)
    assert abs(s.L - 402.112) < 1e-9 and s.loader["lattice"] and s.loader["vth"] == 0.2
    t = I.paper_two_stream(cores=4)
    assert (t.ng, t.np_) == (256, 256_000) and t.loader["beams"] == 2 and t.loader["v0"] == 0.2
