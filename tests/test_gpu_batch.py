"""Batching: many kinematic points x all sectors with uneven lattice sizes,
persistent grids, graph replay and the autotuner."""

import numpy as np
import pytest

from gpu_util import ctx, gpu_plan
from oracle import qmc as oq
from oracle.decompose import decompose as odec
from paper_1508_02512_amd import frontend as fe
from paper_1508_02512_amd import qmc
from seeded_inputs.lattice import lattice
from seeded_inputs.problems import PROBLEMS
from seeded_inputs.rng import shift_table

pytestmark = pytest.mark.gpu

SIZES = [1009, 4099, 10007, 65521]


def _batch(n_points=24, seed=0):
    rng = np.random.default_rng(seed)
    s = rng.uniform(-10, 10, size=4 * n_points)
    s = s[np.abs(s - 4.0) >= 0.05][:n_points]
    return s


def _inputs(plan, info, svals):
    kin = np.stack([fe.kin_vector(info, {"s": float(v), "msq": 1.0}) for v in svals])
    lats = [(n, lattice(n)) for n in (SIZES[i % len(SIZES)] for i in range(plan.n_sectors))]
    return kin, lats


def test_batch_parity_graph_and_grid():
    print("batch: triangle2l 24 points, uneven lattices", flush=True)
    plan, info = gpu_plan("triangle2l", lam=0.25)
    svals = _batch()
    kin, lats = _inputs(plan, info, svals)
    sh = shift_table(5, 3, 8)
    eager = plan.integrate(kin, None, sh, lat_per_sector=lats, sector_sums=True)
    assert eager["violations"] == 0
    # persistent grids and graph replay give the same bits
    job = plan.bind(kin, None, sh, lat_per_sector=lats)
    job.use_graph(True)
    for rep in range(4):
        job.run()
        got = job.fetch(sector_sums=True)
        np.testing.assert_array_equal(got["sector_sums"], eager["sector_sums"])
        # eager work between replays
        plan.integrate(kin[:2], None, sh, lat_per_sector=lats)
    job.close()
    # oracle on sampled (point, sector) pairs
    osecs, oinfo = odec(PROBLEMS["triangle2l"])
    rng = np.random.default_rng(1)
    for p in rng.choice(len(svals), size=4, replace=False):
        for s in rng.choice(len(osecs), size=4, replace=False):
            ns = oq.NumericSector(osecs[s], oinfo, {"s": float(svals[p]), "msq": 1.0})
            n, z = lats[s]
            sums, abss, _ = oq.sector_sums(ns, n, z, sh, 2, oq.effective_lambda(ns, 0.25),
                                           eager["sec_lo"], plan.info.sec_orders)
            scale = abss[..., 0] + abss[..., 1]
            err = np.abs(eager["sector_sums"][p, s] - sums)
            assert np.all(err <= 1e-12 * np.maximum(scale, 1e-300)), (p, s)
    plan.close()


def test_autotune_then_same_result():
    print("batch: autotune", flush=True)
    plan, info = gpu_plan("triangle2l", lam=0.25)
    svals = _batch(8, seed=3)
    kin, lats = _inputs(plan, info, svals)
    sh = shift_table(6, 2, 8)
    before = plan.integrate(kin, None, sh, lat_per_sector=lats, sector_sums=True)
    choices = plan.autotune(kin, None, sh, lat_per_sector=lats)
    assert choices and all(c["points_per_lane"] > 0 for c in choices)
    assert all(c["occupancy_variant"] in (0, 1) for c in choices)
    after = plan.integrate(kin, None, sh, lat_per_sector=lats, sector_sums=True)
    b, a = before["sector_sums"], after["sector_sums"]
    assert np.allclose(a, b, rtol=1e-12, atol=1e-13 * np.max(np.abs(b)))
    plan.close()


def test_class_stats_account_for_the_whole_run():
    print("batch: per-class launch stats", flush=True)
    plan, info = gpu_plan("triangle2l", lam=0.25)
    svals = np.array([-5.0, -1.0, 2.0, 5.0, 7.0, -8.0, 9.0, 4.5])
    kin, lats = _inputs(plan, info, svals)
    sh = shift_table(2, 3, 8)
    job = plan.bind(kin, None, sh, lat_per_sector=lats)
    job.profile(True)
    job.run()
    res = job.fetch()
    st = job.class_stats()
    assert len(st) >= 2                      # real and deformed sectors both occur
    assert sum(c["evals"] for c in st) == res["evals"]
    assert np.isclose(sum(c["algo_flops"] for c in st), res["algo_flops"], rtol=1e-12)
    assert all(c["ms"] > 0 and c["grid"] >= 1 and c["items"] >= c["grid"] for c in st)
    assert sum(c["ms"] for c in st) <= res["kernel_ms"] * 1.01 + 0.05
    keys = [(c["poles"], c["width"]) for c in st]
    assert keys == sorted(keys) and len(set(keys)) == len(keys)
    # graph replay records no per-class events
    job.use_graph(True)
    job.run()
    job.fetch()
    assert all(c["ms"] == -1.0 for c in job.class_stats())
    job.close()


def test_more_items_than_one_launch_can_hold():
    """One work-group per item with more items than a launch may hold
    (2^32 work-items): the two-pole class of the double box with one
    lattice point per lane, n = 4194301, 4 shifts, has 272 x 4 x 16384
    items.  The grid is capped and the item loop covers the rest; the
    result equals the default tiling's up to summation order."""
    print("batch: > 2^24 items in one class", flush=True)
    n = 4194301
    sh = shift_table(9, 4, 8)
    kin = None
    out = []
    for ppl in (1, 0):
        plan, info = gpu_plan("doublebox", ppl=ppl)
        kin = fe.kin_vector(info, {"s": -3.0, "t": -1.0})
        job = plan.bind(kin, (n, lattice(n)), sh)
        st = job.class_stats()
        if ppl == 1:
            two = [c for c in st if c["poles"] == 2][0]
            assert two["items"] > 0xffffffff // 256 and two["grid"] == 0xffffffff // 256
        job.run()
        out.append(job.fetch())
        job.close()
        plan.close()
    a, b = out
    assert np.allclose(a["mean"], b["mean"], rtol=1e-12, atol=0)
    assert np.allclose(a["err_re"], b["err_re"], rtol=1e-9, atol=0)


def test_size_lattices_in_the_library():
    """qmc_size_lattices: every sector gets one of the offered sizes, their
    sum is the budget up to the log-scale rounding, and the sector with the
    largest pilot spread over the shifts gets at least the size of the one
    with the smallest."""
    print("batch: variance-weighted lattice sizes", flush=True)
    plan, info = gpu_plan("np_vertex", lam=0.5)
    kin = fe.kin_vector(info, {"s": 4.5, "msq": 1.0})
    avail = [10007, 65521, 100003, 262139, 1000003, 4194301, 10000019]
    total = 10 ** 6 * plan.n_sectors
    sizes = qmc.size_lattices(plan, kin, total, avail, 65521, lattice(65521),
                              shift_table(1, 8, 8))
    assert len(sizes) == plan.n_sectors and set(sizes) <= set(avail)
    assert total / 4 <= sum(sizes) <= total * 4
    pilot = plan.integrate(kin, (65521, lattice(65521)), shift_table(1, 8, 8),
                           sector_sums=True)
    ss = pilot["sector_sums"][0] / 65521.0
    spread = np.abs(ss - ss.mean(axis=1, keepdims=True)).max(axis=(1, 2))
    assert sizes[int(np.argmax(spread))] >= sizes[int(np.argmin(spread))]
    with pytest.raises(qmc.QMCError):
        qmc.size_lattices(plan, kin, total, [1], 65521, lattice(65521), shift_table(1, 8, 8))
    plan.close()
