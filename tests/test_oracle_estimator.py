"""Pins of the oracle's error estimate (Section III, Eqs. 19-20).

Eq. 20 estimates the mean-square error of the shift average Qbar by
sum_k (Q_k - Qbar)^2 / (m (m - 1)).  It is pinned here against facts that
do not restate that formula:

  - a per-shift table with a known spread: m equally spaced values
    0, 1, ..., m-1 have population variance (m^2 - 1)/12, so the standard
    error of their mean is sqrt((m + 1)/12);
  - sectors are summed shift by shift before the variance: two sectors with
    opposite per-shift sums give an exactly zero error;
  - calibration on the one-loop box, whose Laurent coefficients are known in
    closed form: over 40 independent shift seeds the error bars cover the
    exact value at 3 sigma in at least 95% of the seeds, and the mean squared
    deviation from the exact value matches the mean estimated variance
    (the estimator is unbiased for independent uniform shifts).
CPU only.
"""

import numpy as np
import pytest

from oracle import qmc
from oracle.decompose import decompose
from seeded_inputs.lattice import lattice
from seeded_inputs.problems import PROBLEMS
from seeded_inputs.rng import shift_table

# massless box at s = -3, t = -2 through eps^0 (textbook closed form, no
# e^{eps gamma} factor): the coefficients of eps^-2, eps^-1, eps^0
BOX_EXACT = {-2: 0.666666666666667, -1: -0.982063599677040, 0: -1.48360889993076}


@pytest.mark.parametrize("m", [2, 5, 16])
def test_error_of_equally_spaced_shift_values(m):
    """Per-shift values k and 2k i (k = 0..m-1): the error is sqrt((m+1)/12)
    for the real part and twice that for the imaginary part."""
    per = np.array([[k + 2j * k] for k in range(m)], dtype=complex)
    res = qmc.assemble([per], [1.0], {0: 1.0}, 0, 0, 1, 0, 0)
    assert res["mean"][0] == pytest.approx((m - 1) / 2 * (1 + 2j), rel=1e-15)
    assert res["err_re"][0] == pytest.approx(np.sqrt((m + 1) / 12.0), rel=1e-14)
    assert res["err_im"][0] == pytest.approx(2 * np.sqrt((m + 1) / 12.0), rel=1e-14)


def test_error_scales_with_lattice_size_and_constant():
    """Q_k = D * prefactor * S_k / n: the error scales linearly with D |pref| / n."""
    m = 7
    per = np.array([[float(k)] for k in range(m)], dtype=complex)
    base = qmc.assemble([per], [1.0], {0: 1.0}, 0, 0, 1, 0, 0)
    scaled = qmc.assemble([per], [3.0], {0: -2.0}, 0, 0, 10, 0, 0)
    assert scaled["err_re"][0] == pytest.approx(base["err_re"][0] * 3.0 * 2.0 / 10, rel=1e-14)
    assert scaled["mean"][0] == pytest.approx(base["mean"][0] * 3.0 * -2.0 / 10, rel=1e-14)


def test_sectors_summed_per_shift_before_the_variance():
    """Two sectors whose per-shift sums cancel shift by shift: the integral
    estimate is exactly 0 in every shift, so its error is exactly 0 (a
    variance taken per sector and added in quadrature would not be)."""
    m = 6
    s1 = np.array([[1.5 * k - 0.25j * k * k] for k in range(m)], dtype=complex)
    res = qmc.assemble([s1, -s1], [1.0, 1.0], {0: 1.0}, 0, 0, 1, 0, 0)
    assert res["err_re"][0] == 0.0 and res["err_im"][0] == 0.0
    one = qmc.assemble([s1], [1.0], {0: 1.0}, 0, 0, 1, 0, 0)
    assert one["err_re"][0] > 0.1


def test_prefactor_series_multiplies_per_shift():
    """Orders of the integral are the Cauchy product of the prefactor series
    with the sector sums, taken per shift: a sector series (a_k, b_k) in
    orders (-1, 0) times prefactor (1 + c eps) gives eps^0 = b_k + c a_k
    per shift, whose error follows from the spread of b_k + c a_k."""
    m = 4
    a = np.array([1.0, 2.0, 4.0, 3.0])
    b = np.array([0.5, -1.0, 0.0, 2.5])
    c = 0.75
    per = np.stack([a, b], axis=1).astype(complex)
    res = qmc.assemble([per], [1.0], {0: 1.0, 1: c}, 0, -1, 1, -1, 0)
    q0 = b + c * a
    assert res["mean"][1].real == pytest.approx(q0.mean(), rel=1e-15)
    want = np.sqrt(np.sum((q0 - q0.mean()) ** 2) / (m * (m - 1)))
    # by hand: q0 = (1.25, 0.5, 3, 4.75), mean 2.375, squared deviations
    # sum to 173/16, so the error is sqrt(173/16 / 12) = sqrt(173/192)
    assert want == pytest.approx(np.sqrt(173 / 192), rel=1e-14)
    assert res["err_re"][1] == pytest.approx(want, rel=1e-14)


def test_error_estimate_is_calibrated_on_the_box():
    """40 independent shift seeds, n = 1009, m = 10 shifts, one-loop box:
    |Qbar - exact| <= 3 err in at least 38 of 40 seeds for every order whose
    QMC error is above rounding, and the mean of (Qbar - exact)^2 over the
    seeds is within a factor 2.5 of the mean of err^2."""
    prob = PROBLEMS["box"]
    kin = {"s": -3.0, "t": -2.0}
    n, m = 1009, 10
    secs = decompose(prob)
    z = lattice(n)
    dev = {p: [] for p in BOX_EXACT}
    var = {p: [] for p in BOX_EXACT}
    for seed in range(100, 140):
        res = qmc.integrate(prob, kin, n, z, shift_table(seed, m, 8), sectors=secs)
        for p, want in BOX_EXACT.items():
            i = res["orders"].index(p)
            dev[p].append(res["mean"][i].real - want)
            var[p].append(res["err_re"][i] ** 2)
    checked = 0
    for p, want in BOX_EXACT.items():
        d, v = np.array(dev[p]), np.array(var[p])
        if np.sqrt(v.mean()) < 1e-10 * abs(want):
            continue                      # this order is integrated exactly
        checked += 1
        inside = np.sum(np.abs(d) <= 3 * np.sqrt(v))
        assert inside >= 38, (p, inside)
        ratio = np.mean(d ** 2) / np.mean(v)
        assert 0.4 <= ratio <= 2.5, (p, ratio)
    assert checked >= 2
