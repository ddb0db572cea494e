"""FP32 evaluation mode: FP32 integrand, FP64 lattice points and sums.

Per sector the FP32 sums stay within 1e-5 of sum|w g| of the FP64 oracle;
for the whole double box the FP32 result agrees with FP64 within the
stated statistical error at the 1e-3 relative level."""

import numpy as np
import pytest

from gpu_util import compare_sectors, gpu_plan, sample_sectors
from paper_1508_02512_amd import frontend as fe
from paper_1508_02512_amd import qmc
from seeded_inputs.lattice import lattice
from seeded_inputs.rng import shift_table

pytestmark = pytest.mark.gpu
FP32 = qmc.QMC_FP32_EVAL


def test_fp32_box_sectors():
    print("fp32 box n=10007 m=4", flush=True)
    compare_sectors("box", {"s": -3.0, "t": -2.0}, 10007, 4, tol=1e-5, precision=FP32,
                    quad_from=99)


def test_fp32_double_box_sectors():
    print("fp32 doublebox n=1009 m=2", flush=True)
    compare_sectors("doublebox", {"s": -3.0, "t": -1.0}, 1009, 2, tol=1e-5, precision=FP32,
                    sectors=sample_sectors("doublebox", per_class=4), quad_from=99)


def test_fp32_double_box_whole_result_within_error():
    print("fp32 vs fp64 doublebox n=65521 m=16", flush=True)
    p64, info = gpu_plan("doublebox")
    p32, _ = gpu_plan("doublebox", precision=FP32)
    args = (fe.kin_vector(info, {"s": -3.0, "t": -1.0}), (65521, lattice(65521)),
            shift_table(0, 16, 8))
    a, b = p64.integrate(*args), p32.integrate(*args)
    mean64, mean32 = a["mean"][0].real, b["mean"][0].real
    err32 = b["err_re"][0]
    rel = err32 / np.abs(mean64)
    assert np.all(rel[np.abs(mean64) > 1e-3] < 2e-3)        # at the 1e-3 level
    assert np.all(np.abs(mean32 - mean64) <= 3 * err32 + 1e-5 * np.abs(mean64))
    p64.close()
    p32.close()


def test_fp32_four_poles_next_to_the_corner():
    """Lattice index 0 placed at y_j = 1e-4 in every coordinate (first shift)
    and 2e-4 (second shift): the four pole variables of the double box's
    four-pole sectors are ~1e-11 there, where prod_j 1/t_j exceeds the float
    range.  FP32-eval sums stay finite, no point is rejected, and every
    sampled sector matches the FP64 oracle within 1e-5 of sum |w g|."""
    from gpu_util import oracle_sectors
    from oracle import qmc as oq
    print("fp32 doublebox four poles near the corner", flush=True)
    kin = {"s": -3.0, "t": -1.0}
    plan, info = gpu_plan("doublebox", precision=FP32)
    n = 1009
    z = lattice(n)
    sh = np.array([[1e-4] * 8, [2e-4] * 8])
    res = plan.integrate(fe.kin_vector(info, kin), (n, z), sh, sector_sums=True)
    assert res["status"] == 0 and res["violations"] == 0
    assert np.all(np.isfinite(res["sector_sums"]))
    osecs, oinfo = oracle_sectors("doublebox")
    four = [i for i, s in enumerate(osecs) if sum(1 for a in s["a"] if a == -1) == 4]
    for s in four[::19]:
        ns = oq.NumericSector(osecs[s], oinfo, kin)
        sums, abss, _ = oq.sector_sums(ns, n, z, sh, 2, 0.0, res["sec_lo"],
                                       plan.info.sec_orders)
        gpu = res["sector_sums"][0, s]
        scale = abss[..., 0] + abss[..., 1]
        assert np.all(np.abs(gpu - sums) <= 1e-5 * scale), s
    plan.close()


@pytest.mark.parametrize("name,kin,lam,strategy", [
    ("hh_planar", None, 1.0, "geometric"),
    ("np_vertex", {"s": 4.5, "msq": 1.0}, 0.5, "iterated"),
    ("box", {"s": 3.0, "t": -2.0}, 0.5, "iterated"),
])
def test_fp32_deformed_sectors(name, kin, lam, strategy):
    """Deformed sectors in the FP32-eval mode (FP32 power table, derivative
    terms, z and complex monomials; FP64 Jacobian determinant, logs and
    powers of U and F, series, corner differences and sums): every sampled
    sector within 1e-5 of sum |w g| of the FP64 oracle (measured: 4e-7 on
    the gg -> HH planar box, 7e-8 on the non-planar vertex)."""
    from seeded_inputs.problems import HH_POINT
    kin = HH_POINT if kin is None else kin
    print(f"fp32 deformed {name} lambda={lam}", flush=True)
    sectors = None if name == "box" else sample_sectors(name, per_class=6, strategy=strategy)
    res, _ = compare_sectors(name, kin, 1009, 2, lam=lam, tol=1e-5, precision=FP32,
                             quad_from=99, strategy=strategy, sectors=sectors)
    assert res["violations"] == 0


def test_fp32_deformed_whole_result_within_error():
    """I_C (Section IV.C) on its geometric sectors at n = 131071, 16 shifts:
    the FP32-eval result lies within three of its stated errors of the FP64
    result, order by order, and both meet the 1e-3 level."""
    from seeded_inputs.problems import HH_POINT
    print("fp32 vs fp64 I_C n=131071 m=16", flush=True)
    p64, info = gpu_plan("hh_planar", lam=1.0, strategy="geometric")
    p32, _ = gpu_plan("hh_planar", lam=1.0, strategy="geometric", precision=FP32)
    args = (fe.kin_vector(info, HH_POINT), (131071, lattice(131071)), shift_table(0, 16, 8))
    a, b = p64.integrate(*args), p32.integrate(*args)
    err32 = np.hypot(b["err_re"][0], b["err_im"][0])
    assert np.all(np.abs(b["mean"][0] - a["mean"][0]) <= 3 * err32)
    assert np.all(err32 / np.abs(a["mean"][0]) < 1e-3)
    p64.close()
    p32.close()


def test_fp32_serving_target_floor():
    """FP32-eval plans carry a rounding bias (measured up to 2.7e-6 relative
    on the double box); serving requests asking for less than 1e-5 on such
    a plan are refused."""
    from seeded_inputs.lattice import embedded_lattice
    plan, info = gpu_plan("box", precision=FP32)
    kin = fe.kin_vector(info, {"s": -3.0, "t": -2.0})
    with pytest.raises(qmc.QMCError) as e:
        qmc.submit(plan, kin, 1e-6, 1 << 10, 1 << 16, 4, 1, embedded_lattice())
    assert e.value.code == -1
    r = qmc.submit(plan, kin, 1e-5, 1 << 10, 1 << 16, 4, 1, embedded_lattice()).wait(60)
    assert r["rc"] in (0, -7)
    plan.close()
