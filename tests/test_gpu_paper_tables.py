"""End-to-end results of the GPU path against the values printed in
Section IV (tests/golden/paper_tables.json): the Euclidean off-shell double
box of Table 1 and the physical gg -> HH double boxes of Tables 2-3."""

import pytest

from gpu_util import gpu_plan
from paper_1508_02512_amd import frontend as fe
from paper_norm import GOLDEN, check_against, p_coefficients
from seeded_inputs.lattice import lattice
from seeded_inputs.problems import HH_POINT
from seeded_inputs.rng import shift_table

pytestmark = pytest.mark.gpu

N = 1000003


@pytest.mark.parametrize("legs", ["14", "24", "34"])
def test_table1_double_box_columns(legs):
    print(f"Table 1 column {legs}: n={N} m=16", flush=True)
    col = GOLDEN["table1"]["columns"][legs]
    kin = {"s": -2 / 3, "t": -2 / 3, **col["offshell"]}
    plan, info = gpu_plan(f"doublebox_off{legs}")
    res = plan.integrate(fe.kin_vector(info, kin), (N, lattice(N)), shift_table(0, 16, 8))
    P = p_coefficients(plan.orders, res["mean"][0], res["err_re"][0], res["err_im"][0], -2 / 3)
    check_against(P, col["qmc"], nsig=5.0, extra=1e-9)
    plan.close()


@pytest.mark.parametrize("table,lam", [("table2", 1.0), ("table3", 0.5)])
def test_tables2_3_physical_double_boxes(table, lam):
    print(f"{table}: n={N} m=16 lambda={lam}", flush=True)
    tab = GOLDEN[table]
    plan, info = gpu_plan(tab["problem"], lam=lam)
    res = plan.integrate(fe.kin_vector(info, HH_POINT), (N, lattice(N)), shift_table(0, 16, 8))
    assert res["violations"] == 0
    P = p_coefficients(plan.orders, res["mean"][0], res["err_re"][0], res["err_im"][0],
                       HH_POINT["s"])
    check_against(P, tab["qmc"], nsig=5.0)
    plan.close()


def test_hh_box_threshold_scan():
    """Section IV.A through the batched path: 48 kinematic points of the
    one-loop gg -> HH box from s = 70000 to 500000 at t = -6000 in one bind.
    Im J (= -16 pi^2 Re I_A) is zero within errors below s = 4 M_t^2 and
    clearly non-zero above; two points are checked sector by sector against
    the oracle."""
    import numpy as np
    from oracle import qmc as oq
    from oracle.decompose import decompose as odec
    from seeded_inputs.problems import PROBLEMS
    print("hh_box s-scan, 48 points", flush=True)
    plan, info = gpu_plan("hh_box", lam=0.5)
    svals = np.linspace(70000.0, 500000.0, 48)
    kin = np.stack([fe.kin_vector(info, {**HH_POINT, "s": float(v)}) for v in svals])
    n = 65521
    res = plan.integrate(kin, (n, lattice(n)), shift_table(0, 8, 8), sector_sums=True)
    assert res["violations"] == 0
    thr = 4 * HH_POINT["mtsq"]
    mean, ei = res["mean"][:, 0], res["err_im"][:, 0]
    below, above = svals < 0.97 * thr, svals > 1.1 * thr
    assert below.sum() == 5 and above.sum() >= 40
    assert np.all(np.abs(mean[below].imag) <= 5 * ei[below] + 1e-30)
    assert np.all(np.abs(mean[above].imag) > 20 * ei[above])
    osecs, oinfo = odec(PROBLEMS["hh_box"])
    z = lattice(1009)
    sh = shift_table(0, 2, 8)
    got = plan.integrate(kin[[3, 30]], (1009, z), sh, sector_sums=True)
    for row, p in enumerate((3, 30)):
        for s in range(len(osecs)):
            ns = oq.NumericSector(osecs[s], oinfo, {**HH_POINT, "s": float(svals[p])})
            sums, abss, _ = oq.sector_sums(ns, 1009, z, sh, 2, oq.effective_lambda(ns, 0.5),
                                           got["sec_lo"], plan.info.sec_orders)
            scale = abss[..., 0] + abss[..., 1]
            assert np.all(np.abs(got["sector_sums"][row, s] - sums) <= 1e-12 * scale)
    plan.close()
