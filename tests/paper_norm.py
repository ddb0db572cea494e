"""The normalisation of the printed results of Section IV (Tables 1-3):
I = exp(-2 eps gamma_E) |s|^(-3-2 eps) sum_i P_i eps^-i, so
P(eps) = I(eps) |s|^3 exp(eps (2 gamma_E + 2 ln|s|)).  For the Euclidean
Table 1 point s < 0 and |s| = -s; for Tables 2-3 s > 0."""

import json
import math
import os

import numpy as np

GAMMA_E = 0.57721566490153286061
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def p_coefficients(orders, mean, err_re, err_im, s):
    """{i: (P_i, err_re(P_i), err_im(P_i))} from the Laurent coefficients
    I_o (o in orders) of one integral; errors propagated as independent."""
    a = abs(s)
    x = 2.0 * GAMMA_E + 2.0 * math.log(a)
    c = [x ** k / math.factorial(k) for k in range(12)]
    mean = np.asarray(mean).ravel()
    er, ei = np.asarray(err_re).ravel(), np.asarray(err_im).ravel()
    out = {}
    for i in range(0, -min(orders) + 1):
        p, vr, vi = 0j, 0.0, 0.0
        for k, ck in enumerate(c):
            o = -i - k
            if o in orders:
                j = orders.index(o)
                p += ck * mean[j]
                vr += (ck * er[j]) ** 2
                vi += (ck * ei[j]) ** 2
        out[i] = (p * a ** 3, math.sqrt(vr) * a ** 3, math.sqrt(vi) * a ** 3)
    return out


def check_against(P, printed, nsig=5.0, extra=0.0):
    """Every printed P_i (real [v, e] or complex [re, e, im, e]) agrees with
    ours within nsig combined standard errors; returns the worst pull."""
    worst = 0.0
    for key, val in printed.items():
        i = int(key[1:])
        ours, er, ei = P.get(i, (0j, 0.0, 0.0))
        if len(val) == 2:
            pairs = [(ours.real, er, val[0], val[1])]
        else:
            pairs = [(ours.real, er, val[0], val[1]), (ours.imag, ei, val[2], val[3])]
        for got, e1, want, e2 in pairs:
            tol = nsig * math.hypot(e1, e2) + extra
            pull = abs(got - want) / tol if tol > 0 else (0.0 if got == want else math.inf)
            assert abs(got - want) <= tol, f"P{i}: {got} vs printed {want} (tolerance {tol:.3g})"
            worst = max(worst, pull)
    return worst
