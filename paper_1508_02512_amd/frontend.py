"""Host front end: propagators -> U, F (Section II, Eq. 2) -> sectors (Eqs. 3-9).

Produces the input of ``qmc_plan_sectors``: a list of sectors, each a
monomial prod t_j^(a_j + b_j eps) times U^(u0 + u1 eps) F^(f0 + f1 eps) with
U and F given as exponent matrices and coefficient rows over the kinematic
invariants (column 0 is the constant invariant 1).

Conventions: propagators 1/(-q^2 + m^2 - i0)^nu, measure d^D k/(i pi^{D/2})
per loop, D = 4 - 2 eps, so that

    I = Gamma(N_nu - L D/2)/prod Gamma(nu_j) int dx delta(1 - sum x)
        prod x^(nu-1) U^(N_nu - (L+1) D/2) F^(-(N_nu - L D/2)),

with sum_j x_j (-q_j^2 + m_j^2) = -k^T M k + 2 k.Q + J, U = det M and
F = adj(M)[Q, Q] + U J.

Sector decomposition: primary sectors with x_l = 1 (Eqs. 3-6), then either
the geometric strategy the paper adopts (module ``geometric``: the normal
fan of the Newton polytope of U F, fewest sectors) or iterated splitting
until U and F are monomial x (constant + higher terms) (Eqs. 7-8).  The split rule (the paper leaves it open) takes the first
polynomial without a constant term (U before F), its exponent vectors that
no other exponent dominates componentwise, the closest pair (v, w) of them
in the 1-norm (ties: lexicographically smallest, v < w), and splits on
S = {i, j} with i the first index where v and w differ and j the first
index where v - w has the opposite sign; children t_x -> t_k t_x for x in
S minus k, k in S increasing.  Every child either loses a minimal vector or
brings the chosen pair strictly closer, so the recursion terminates.
"""

from __future__ import annotations

from fractions import Fraction
from math import factorial

import numpy as np

# ----------------------------------------------------------------- polynomials
# A polynomial is a dict {exponent tuple: coefficient vector}, the vector
# holding Fractions over (1, invariant_1, ..., invariant_r).


class _Poly:
    __slots__ = ("t", "nv", "ni")

    def __init__(self, nv, ni, terms=None):
        self.nv, self.ni = nv, ni
        self.t = {} if terms is None else terms

    @staticmethod
    def var(nv, ni, j, scale=1):
        e = [0] * nv
        e[j] = 1
        vec = [Fraction(0)] * ni
        vec[0] = Fraction(scale)
        return _Poly(nv, ni, {tuple(e): vec})

    def _acc(self, e, vec):
        cur = self.t.get(e)
        if cur is None:
            self.t[e] = list(vec)
        else:
            for i, v in enumerate(vec):
                cur[i] += v
        if all(v == 0 for v in self.t[e]):
            del self.t[e]

    def __add__(self, other):
        out = _Poly(self.nv, self.ni, {e: list(v) for e, v in self.t.items()})
        for e, v in other.t.items():
            out._acc(e, v)
        return out

    def scale(self, s):
        return _Poly(self.nv, self.ni, {e: [x * s for x in v] for e, v in self.t.items()})

    def __sub__(self, other):
        return self + other.scale(-1)

    def __mul__(self, other):
        """Product; at most one factor may carry invariants (linear forms)."""
        out = _Poly(self.nv, self.ni)
        for e1, v1 in self.t.items():
            s1 = all(x == 0 for x in v1[1:])
            for e2, v2 in other.t.items():
                s2 = all(x == 0 for x in v2[1:])
                if not (s1 or s2):
                    raise ValueError("product of two linear forms is not linear")
                if s1:
                    vec = [v1[0] * x for x in v2]
                else:
                    vec = [x * v2[0] for x in v1]
                out._acc(tuple(a + b for a, b in zip(e1, e2)), vec)
        return out

    def times_form(self, form):
        """Multiply a purely numerical polynomial by a constant linear form."""
        out = _Poly(self.nv, self.ni)
        for e, v in self.t.items():
            out._acc(e, [v[0] * f for f in form])
        return out


def _det_adj(M):
    """Determinant and adjugate of an L x L matrix of polynomials (L <= 3)."""
    L = len(M)
    if L == 1:
        one = _Poly(M[0][0].nv, M[0][0].ni)
        one._acc((0,) * M[0][0].nv, [Fraction(1)] + [Fraction(0)] * (M[0][0].ni - 1))
        return M[0][0], [[one]]

    def minor(r, c):
        return [[M[i][j] for j in range(L) if j != c] for i in range(L) if i != r]

    cof = [[None] * L for _ in range(L)]
    for r in range(L):
        for c in range(L):
            dm, _ = _det_adj(minor(r, c))
            cof[r][c] = dm if (r + c) % 2 == 0 else dm.scale(-1)
    det = _Poly(M[0][0].nv, M[0][0].ni)
    for c in range(L):
        det = det + M[0][c] * cof[0][c]
    adj = [[cof[c][r] for c in range(L)] for r in range(L)]
    return det, adj


def symanzik_polynomials(problem):
    """(U, F, invariant names) with U, F as dicts exps -> coefficient vector."""
    inv = ["1"] + list(problem.invariants)
    ni, N, L = len(inv), len(problem.props), problem.loops
    idx = {name: i for i, name in enumerate(inv)}

    def sp_vec(e1, e2):
        form = problem.sp.get((e1, e2), problem.sp.get((e2, e1)))
        vec = [Fraction(0)] * ni
        for k, v in form.items():
            vec[idx[k]] += Fraction(v)
        return vec

    zero = _Poly(N, ni)
    M = [[zero for _ in range(L)] for _ in range(L)]
    Q = [dict() for _ in range(L)]     # Q_a: external e -> polynomial coefficient
    J = zero
    for j, pr in enumerate(problem.props):
        xj = _Poly.var(N, ni, j)
        for a in range(L):
            for b in range(L):
                if pr.loop[a] * pr.loop[b]:
                    M[a][b] = M[a][b] + xj.scale(pr.loop[a] * pr.loop[b])
        for a in range(L):
            if pr.loop[a]:
                for e, c in pr.ext.items():
                    if c:
                        Q[a][e] = Q[a].get(e, zero) + xj.scale(-pr.loop[a] * c)
        # J += x_j (-P_j^2 + m_j^2)
        form = [Fraction(0)] * ni
        for e1, c1 in pr.ext.items():
            for e2, c2 in pr.ext.items():
                for i, v in enumerate(sp_vec(e1, e2)):
                    form[i] -= c1 * c2 * v
        if pr.mass:
            form[idx[pr.mass]] += 1
        J = J + xj.times_form(form)
    U, adj = _det_adj(M)
    F = U * J
    for a in range(L):
        for b in range(L):
            for e1, q1 in Q[a].items():
                for e2, q2 in Q[b].items():
                    F = F + (adj[a][b] * (q1 * q2)).times_form(sp_vec(e1, e2))
    return U.t, F.t, inv


# --------------------------------------------------------------- decomposition

class _Sec:
    """Exponent matrix + coefficient rows of U and F and the monomial."""
    __slots__ = ("a", "b", "EU", "CU", "EF", "CF", "D")

    def __init__(self, a, b, EU, CU, EF, CF):
        self.a, self.b = a, b
        self.D = 1
        self.EU, self.CU, self.EF, self.CF = EU, CU, EF, CF


def _to_mats(poly, drop):
    keys = sorted(poly)
    E = np.array([[e for i, e in enumerate(k) if i != drop] for k in keys], dtype=np.int64)
    C = [poly[k] for k in keys]
    # merge terms that coincide once x_drop = 1
    merged = {}
    for row, c in zip(map(tuple, E), C):
        if row in merged:
            merged[row] = [x + y for x, y in zip(merged[row], c)]
        else:
            merged[row] = list(c)
    merged = {k: v for k, v in merged.items() if any(x != 0 for x in v)}
    keys = sorted(merged)
    return np.array(keys, dtype=np.int64).reshape(len(keys), -1), [merged[k] for k in keys]


def _minimal_rows(E):
    le = np.all(E[:, None, :] <= E[None, :, :], axis=2)      # le[i, j]: E_i <= E_j
    np.fill_diagonal(le, False)
    dominated = np.any(le, axis=0)
    return E[~dominated]


def _split_set(E):
    mins = sorted(map(tuple, _minimal_rows(E)))
    best = None
    for x in range(len(mins)):
        for y in range(x + 1, len(mins)):
            dist = int(np.abs(np.subtract(mins[x], mins[y])).sum())
            key = (dist, mins[x], mins[y])
            if best is None or key < best:
                best = key
    _, v, w = best
    delta = np.subtract(v, w)
    i = int(np.flatnonzero(delta)[0])
    j = int(np.flatnonzero(delta * delta[i] < 0)[0])
    return (i, j) if i < j else (j, i)


def _decompose_primary(sec, ex, out, max_depth=64):
    u0, u1, f0, f1 = ex
    stack = [(sec, 0)]
    while stack:
        s, depth = stack.pop()
        if depth > max_depth:
            raise RuntimeError("sector decomposition too deep")
        mu = s.EU.min(axis=0)
        mf = s.EF.min(axis=0)
        EU, EF = s.EU - mu, s.EF - mf
        a = [x + int(p) * u0 + int(q) * f0 for x, p, q in zip(s.a, mu, mf)]
        b = [x + int(p) * u1 + int(q) * f1 for x, p, q in zip(s.b, mu, mf)]
        u_const = bool(np.any(np.all(EU == 0, axis=1)))
        f_const = bool(np.any(np.all(EF == 0, axis=1)))
        if u_const and f_const:
            out.append(_Sec(a, b, EU, s.CU, EF, s.CF))
            continue
        S = _split_set(EU if not u_const else EF)
        children = []
        for k in S:
            others = [x for x in S if x != k]
            na, nb = list(a), list(b)
            na[k] += sum(a[x] for x in others) + len(others)
            nb[k] += sum(b[x] for x in others)
            nEU, nEF = EU.copy(), EF.copy()
            nEU[:, k] += EU[:, others].sum(axis=1)
            nEF[:, k] += EF[:, others].sum(axis=1)
            children.append((_Sec(na, nb, nEU, s.CU, nEF, s.CF), depth + 1))
        stack.extend(reversed(children))      # first child is processed first


def _geometric_primary(sec, ex, out):
    """Sectors of one primary sector from the simplicial cones of the normal
    fan of Newt(U F) + R^d_{>=0} (module ``geometric``): t_j = prod_k
    s_k^{V_jk}, Jacobian |det V| prod_k s_k^{sum_j V_jk - 1}."""
    from . import geometric

    u0, u1, f0, f1 = ex
    for V, det in geometric.decompose_primary(sec.EU, sec.EF):
        EU, EF = sec.EU @ V, sec.EF @ V
        mu, mf = EU.min(axis=0), EF.min(axis=0)
        cols = V.sum(axis=0)
        a = [sum(int(V[j, k]) * sec.a[j] for j in range(V.shape[0])) + int(cols[k]) - 1
             + int(mu[k]) * u0 + int(mf[k]) * f0 for k in range(V.shape[1])]
        b = [sum(int(V[j, k]) * sec.b[j] for j in range(V.shape[0]))
             + int(mu[k]) * u1 + int(mf[k]) * f1 for k in range(V.shape[1])]
        s = _Sec(a, b, EU - mu, sec.CU, EF - mf, sec.CF)
        s.D = det
        out.append(s)


def decompose(problem, strategy="iterated"):
    """Sectors of a problem as a list of dicts plus global info.

    strategy "iterated" splits as described above; "geometric" takes the
    normal fan of each primary sector's Newton polytope (fewer sectors)."""
    if strategy not in ("iterated", "geometric"):
        raise ValueError(f"unknown decomposition strategy {strategy!r}")
    U, F, inv = symanzik_polynomials(problem)
    N, L = len(problem.props), problem.loops
    nus = [p.power for p in problem.props]
    Nnu = sum(nus)
    ex = (Fraction(Nnu - 2 * (L + 1)), Fraction(L + 1),
          Fraction(-(Nnu - 2 * L)), Fraction(-L))
    out = []
    for l in range(N):
        EU, CU = _to_mats(U, l)
        EF, CF = _to_mats(F, l)
        a = [Fraction(nus[j] - 1) for j in range(N) if j != l]
        b = [Fraction(0)] * (N - 1)
        if strategy == "geometric":
            _geometric_primary(_Sec(a, b, EU, CU, EF, CF), ex, out)
        else:
            _decompose_primary(_Sec(a, b, EU, CU, EF, CF), ex, out)
    sectors = [{"a": s.a, "b": s.b, "EU": s.EU, "CU": s.CU, "EF": s.EF, "CF": s.CF,
                "D": s.D} for s in out]
    info = {"invariants": inv, "u": ex[:2], "f": ex[2:], "gamma": (Nnu - 2 * L, L),
            "nus": nus, "dim": N - 1}
    return sectors, info


# ------------------------------------------------------------------ prefactor

def _series_mul(x, y, n):
    out = np.zeros(n)
    for i in range(n):
        out[i] = sum(x[k] * y[i - k] for k in range(i + 1))
    return out


def gamma_series(g0, g1, n):
    """Laurent coefficients of Gamma(g0 + g1 eps): (lowest order, coeffs[n]).

    Uses ln Gamma(1 + x) = -gamma x + sum_{k >= 2} (-1)^k zeta(k) x^k / k and
    the recurrence Gamma(x + 1) = x Gamma(x)."""
    from scipy.special import zeta
    g0 = int(g0)
    npole = 1 if g0 <= 0 else 0
    m = n + 2
    # ln Gamma(1 + g1 eps) as a series in eps
    lg = np.zeros(m)
    lg[1] = -np.euler_gamma * g1
    for k in range(2, m):
        lg[k] = (-1) ** k * zeta(k) * g1 ** k / k
    # exp of a series with zero constant term
    ex = np.zeros(m)
    ex[0] = 1.0
    for k in range(1, m):
        ex[k] = sum(j * lg[j] * ex[k - j] for j in range(1, k + 1)) / k
    series = ex        # Gamma(1 + g1 eps)
    if g0 >= 1:
        for c in range(1, g0):      # Gamma(g0 + x) = prod_{c=1}^{g0-1} (c + x) Gamma(1 + x)
            series = _series_mul(series, np.array([c, g1] + [0.0] * (m - 2)), m)
        return 0, series[:n]
    # g0 <= 0: Gamma(x) = Gamma(1 + x) / x with x = g0 + g1 eps, and for
    # g0 < 0 divide further by (x + 1)...(x - g0) ... written as
    # Gamma(g0 + y) = Gamma(1 + y) / prod_{c=g0}^{0} (c + y), y = g1 eps
    for c in range(g0, 1):
        if c == 0:
            # divide by g1 eps: shift down one order
            series = series / g1
        else:
            # divide by (c + g1 eps) = c (1 + (g1/c) eps)
            inv = np.array([(-g1 / c) ** k / c for k in range(m)])
            series = _series_mul(series, inv, m)
    return -npole, series[:n]


def prefactor_series(info, n):
    """Gamma(N_nu - L D/2)/prod Gamma(nu_j): (lowest order, complex coeffs)."""
    g0, g1 = info["gamma"]
    lo, c = gamma_series(g0, g1, n)
    norm = 1.0
    for nu in info["nus"]:
        norm *= factorial(nu - 1)
    return lo, c / norm


# ------------------------------------------------------- arrays for the C ABI

def sector_arrays(sectors, info):
    """Flat numpy arrays of each sector (float64 exponents, uint8 powers)."""
    ni = len(info["invariants"])
    out = []
    for s in sectors:
        out.append({
            "dim": len(s["a"]),
            "a": np.array([float(x) for x in s["a"]]),
            "b": np.array([float(x) for x in s["b"]]),
            "EU": np.ascontiguousarray(s["EU"], dtype=np.uint8),
            "CU": np.array([[float(x) for x in row] for row in s["CU"]]).reshape(-1, ni),
            "EF": np.ascontiguousarray(s["EF"], dtype=np.uint8),
            "CF": np.array([[float(x) for x in row] for row in s["CF"]]).reshape(-1, ni),
            "D": float(s.get("D", 1)),
            "u": tuple(float(x) for x in info["u"]),
            "f": tuple(float(x) for x in info["f"]),
        })
    return out


def kin_vector(info, values):
    """Kinematic vector (1, invariant values...) in the sectors' column order."""
    return np.array([1.0] + [float(values[k]) for k in info["invariants"][1:]])
