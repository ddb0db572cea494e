"""qmc_integrate_noalloc (the allocation-free variant of qmc_integrate)
against qmc_integrate, through the C ABI: identical sums, means and errors
on two calls in a row (the second with a smaller input), and a call that
needs more than the fixed scratch array is refused without running."""

import numpy as np
import pytest

from gpu_util import gpu_plan
from paper_1508_02512_amd import frontend as fe
from paper_1508_02512_amd import qmc
from seeded_inputs.lattice import lattice
from seeded_inputs.rng import shift_table

pytestmark = pytest.mark.gpu


def _same(a, b):
    for key in ("mean", "err_re", "err_im", "sector_sums"):
        assert np.array_equal(a[key], b[key]), key
    for key in ("evals", "status", "violations"):
        assert a[key] == b[key], key


def test_noalloc_equals_integrate_on_two_calls():
    print("noalloc: double box n=100003 m=8, then box n=1009 m=3", flush=True)
    big, binfo = gpu_plan("doublebox")
    args = (fe.kin_vector(binfo, {"s": -3.0, "t": -1.0}), (100003, lattice(100003)),
            shift_table(0, 8, 8))
    want = big.integrate(*args, sector_sums=True)
    got = big.integrate(*args, sector_sums=True, noalloc=True)
    _same(want, got)
    small, sinfo = gpu_plan("box")
    args = (fe.kin_vector(sinfo, {"s": -3.0, "t": -2.0}), (1009, lattice(1009)),
            shift_table(4, 3, 8))
    want = small.integrate(*args, sector_sums=True)
    got = small.integrate(*args, sector_sums=True, noalloc=True)
    _same(want, got)
    big.close()
    small.close()


def test_noalloc_deformed_and_several_points():
    """The deformed kernel (s = 4.5, 5.5) and the real one (s = -2) in one
    multi-point bind through the scratch array; both entry points report
    the same sums and violation counts."""
    print("noalloc: np_vertex, 3 kinematic points", flush=True)
    plan, info = gpu_plan("np_vertex", lam=0.5)
    kin = np.stack([fe.kin_vector(info, {"s": s, "msq": 1.0}) for s in (4.5, 5.5, -2.0)])
    args = (kin, (4099, lattice(4099)), shift_table(2, 4, 8))
    want = plan.integrate(*args, sector_sums=True, allow_violations=True)
    got = plan.integrate(*args, sector_sums=True, allow_violations=True, noalloc=True)
    _same(want, got)
    plan.close()


def test_noalloc_with_poles_integrated_by_parts():
    """Plans expanded by Eq. 13 at the poles (pole-free sectors with up to 5
    orders, numerator factors, Laurent coefficient series): the double box
    (48798 sectors) then the dotted box, both entry points alike."""
    print("noalloc: double box and dotted box, poles by parts", flush=True)
    for name, kin, n, m in (("doublebox", {"s": -3.0, "t": -1.0}, 1009, 2),
                            ("box_dot", {"s": -3.0, "t": -2.0}, 4099, 3)):
        plan, info = gpu_plan(name, poles=True)
        args = (fe.kin_vector(info, kin), (n, lattice(n)), shift_table(1, m, 8))
        want = plan.integrate(*args, sector_sums=True)
        got = plan.integrate(*args, sector_sums=True, noalloc=True)
        _same(want, got)
        plan.close()


def test_noalloc_refuses_more_than_the_scratch_array():
    print("noalloc: oversized call refused", flush=True)
    plan, info = gpu_plan("box")
    one = fe.kin_vector(info, {"s": -3.0, "t": -2.0})
    kin = np.tile(one, (40000, 1))          # ~1e6 work items, > 64 MiB of scratch
    with pytest.raises(qmc.QMCError) as e:
        plan.integrate(kin, (1009, lattice(1009)), shift_table(0, 2, 8), noalloc=True)
    assert e.value.code == -5 and "scratch" in str(e.value)
    # the array is still usable afterwards
    args = (kin[:1], (1009, lattice(1009)), shift_table(0, 2, 8))
    _same(plan.integrate(*args, sector_sums=True),
          plan.integrate(*args, sector_sums=True, noalloc=True))
    plan.close()
