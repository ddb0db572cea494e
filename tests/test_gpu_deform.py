"""GPU contour deformation (Eq. 14) against the oracle and closed forms."""

import math

import numpy as np
import pytest

from gpu_util import compare_sectors, gpu_plan
from paper_1508_02512_amd import frontend as fe
from seeded_inputs.lattice import lattice
from seeded_inputs.rng import shift_table

pytestmark = pytest.mark.gpu


def test_massive_bubble_above_threshold():
    print("bubble_massive s=4.5 lambda=0.5", flush=True)
    res, _ = compare_sectors("bubble_massive", {"s": 4.5, "msq": 1.0}, 65521, 4, lam=0.5)
    want = 1.19173527491182 + 1.04719755119660j
    got = res["mean"][0, -1]
    assert abs(got.real - want.real) < 6 * res["err_re"][0, -1] + 1e-9
    assert abs(got.imag - want.imag) < 6 * res["err_im"][0, -1] + 1e-9
    assert res["violations"] == 0


def test_massless_bubble_negative_constant_f():
    # F = -s < 0 everywhere: log F = ln|F| - i pi
    print("bubble s=3 lambda=0.5", flush=True)
    res, _ = compare_sectors("bubble", {"s": 3.0}, 10007, 3, lam=0.5, eps_hi=1)
    assert abs(res["mean"][0, 1] - (0.324172046430357 + math.pi * 1j)) < 1e-9


def test_box_physical():
    print("box s=3 t=-2 lambda=0.5", flush=True)
    res, _ = compare_sectors("box", {"s": 3.0, "t": -2.0}, 10007, 4, lam=0.5)
    assert res["violations"] == 0


@pytest.mark.parametrize("lam", [0.25, 0.5])
def test_np_vertex_physical(lam):
    print(f"np_vertex s=4.5 lambda={lam}", flush=True)
    res, _ = compare_sectors("np_vertex", {"s": 4.5, "msq": 1.0}, 1009, 2, lam=lam)
    assert res["violations"] == 0


def test_np_vertex_lambda_independence():
    plan1, info = gpu_plan("np_vertex", lam=0.25)
    plan2, _ = gpu_plan("np_vertex", lam=0.5)
    args = (fe.kin_vector(info, {"s": 4.5, "msq": 1.0}), (262139, lattice(262139)),
            shift_table(0, 8, 8))
    a, b = plan1.integrate(*args), plan2.integrate(*args)
    err = np.hypot(a["err_re"], a["err_im"]) + np.hypot(b["err_re"], b["err_im"])
    assert np.all(np.abs(a["mean"] - b["mean"]) < 6 * err + 1e-10)
    plan1.close()
    plan2.close()


def test_np_vertex_lambda_too_large_is_reported():
    """lambda = 1 (in units of the largest |coefficient| of F) pushes Im F(z)
    above 0 at some points for this integral; the kernel counts them and the
    call returns QMC_EDEFORM (the oracle counts violations too)."""
    from oracle import qmc as oq
    from oracle.decompose import decompose as odec
    from seeded_inputs.problems import PROBLEMS
    plan, info = gpu_plan("np_vertex", lam=1.0)
    kin = {"s": 4.5, "msq": 1.0}
    res = plan.integrate(fe.kin_vector(info, kin), (1009, lattice(1009)), shift_table(0, 2, 8),
                         allow_violations=True)
    assert res["status"] == -6 and res["violations"] > 0
    osecs, oinfo = odec(PROBLEMS["np_vertex"])
    bad = 0
    for s in osecs:
        ns = oq.NumericSector(s, oinfo, kin)
        _, _, c = oq.sector_sums(ns, 1009, lattice(1009), shift_table(0, 2, 8), 2,
                                 oq.effective_lambda(ns, 1.0), 0, 1)
        bad += int(c[:, :2].sum())
    assert bad > 0
    plan.close()


@pytest.mark.parametrize("s", [-5.0, 6.0, 9.5])
def test_triangle2l(s):
    """Below threshold the sectors run undeformed (all F coefficients >= 0)."""
    print(f"triangle2l s={s}", flush=True)
    res, _ = compare_sectors("triangle2l", {"s": s, "msq": 1.0}, 1009, 2, lam=0.5)
    assert res["violations"] == 0


@pytest.mark.parametrize("name,lam", [("hh_planar", 1.0), ("hh_nonplanar", 0.5)])
def test_hh_double_boxes_sectors(name, lam):
    """The gg -> HH double boxes of Section IV.C-D at the Table 2-3 point:
    deformed six-dimensional sectors, sampled per pole count, against the
    oracle sector by sector."""
    from gpu_util import sample_sectors
    from seeded_inputs.problems import HH_POINT
    print(f"{name} sectors lambda={lam}", flush=True)
    res, _ = compare_sectors(name, HH_POINT, 1009, 2, lam=lam,
                             sectors=sample_sectors(name, per_class=6))
    assert res["violations"] == 0


def test_deformed_sectors_with_three_or_more_poles_refused():
    """The massless planar double box has sectors with three and four poles;
    with a deformation parameter the plan is refused (QMC_EUNSUPPORTED)
    before anything runs, since the deformed kernel's corner differences
    would not reach FP64 accuracy there.  The same sectors plan without
    deformation, and a deformed problem with at most two poles plans."""
    from paper_1508_02512_amd import qmc
    print("doublebox lambda=0.25 refused", flush=True)
    with pytest.raises(qmc.QMCError) as e:
        gpu_plan("doublebox", lam=0.25)
    assert e.value.code == -3
    plan, _ = gpu_plan("doublebox", lam=0.0)
    assert plan.info.max_poles == 4
    plan.close()
    plan, _ = gpu_plan("hh_planar", lam=1.0)
    assert plan.info.max_poles == 2 and plan.info.deform == 1
    plan.close()
