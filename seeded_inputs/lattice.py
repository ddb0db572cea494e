"""Generating vectors for the rank-1 lattice rule (Section III, Eq. 17).

The lattice points are x_i = {i z / n}; the rule needs an integer vector z
whose components are coprime to n.  The paper mentions the
component-by-component construction without parameters, so this module
builds Korobov vectors z = (1, a, a^2, ..., a^(d-1)) mod n and picks the
multiplier a among a fixed, seeded candidate set by the worst-case error
criterion P_2 of the weighted Korobov space with unit weights (Dick, Kuo
and Sloan, Acta Numerica 22 (2013), Section 5):

    P_2(z) = -1 + (1/n) sum_i prod_j (1 + 2 pi^2 B_2({i z_j / n})),
    B_2(x) = x^2 - x + 1/6.

For prime n up to CBC_MAX_N the file also holds a vector from the fast
component-by-component construction (cbc_vector), for the same criterion
over all DMAX components.  Neither rule dominates: on the integrals here
CBC lowers the error of the 3-variable box ~1000x and of the double box
2-4x at n = 65521, but raises it ~10x for the deformed gg -> HH double box
at n = 1000003; the Korobov vector stays the default.

The search is expensive for large n, so the vectors are generated once by
``python -m seeded_inputs.lattice`` and stored in ``lattices.json`` beside
this file; both the oracle and the GPU path read that file.  The vectors
are inputs of the method, not part of its arithmetic.
"""

from __future__ import annotations

import json
import math
import os
from functools import lru_cache

import numpy as np

from .rng import splitmix64

DMAX = 8               # every stored vector has this many components
SEARCH_DIM = 6         # P_2 is minimised for the largest sector dimension used
_DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lattices.json")

# Lattice sizes used by the tests and workloads.  Primes for the plain
# shifted rules; powers of two for the embedded (doubling) rules.
PRIME_SIZES = [1009, 4099, 10007, 65521, 100003, 131071, 262139, 524287,
               1000003, 1048573, 2097143, 4194301, 8388593, 10000019,
               16777213, 33554393, 67108859, 100000007]
POW2_SIZES = [1 << k for k in range(10, 27)]


def is_prime(n: int) -> bool:
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:          # deterministic for n < 3.3e24
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def korobov_vector(n: int, a: int, dim: int = DMAX) -> list[int]:
    z, p = [], 1
    for _ in range(dim):
        z.append(p % n)
        p = p * a % n
    return z


def p2_criterion(n: int, z, chunk: int = 1 << 21) -> float:
    """P_2 worst-case error of the unshifted rule (z, n); exact sum in chunks."""
    z = np.asarray(z, dtype=np.int64)
    total = 0.0
    two_pi2 = 2.0 * math.pi ** 2
    for lo in range(0, n, chunk):
        i = np.arange(lo, min(n, lo + chunk), dtype=np.int64)
        prod = np.ones(i.shape, dtype=np.float64)
        for zj in z:
            x = (i * int(zj) % n).astype(np.float64) / n
            prod *= 1.0 + two_pi2 * (x * x - x + 1.0 / 6.0)
        total += float(np.sum(prod))
    return total / n - 1.0


def korobov_candidates(n: int, count: int, seed: int = 0) -> list[int]:
    """Seeded candidate multipliers in [2, n-2] (odd when n is even)."""
    out = []
    for w in splitmix64(seed ^ n, 4 * count):
        a = 2 + w % (n - 3)
        if n % 2 == 0:
            a |= 1
        if math.gcd(a, n) == 1 and a not in out:
            out.append(a)
        if len(out) == count:
            break
    return out


def search_korobov(n: int, count: int = 64, seed: int = 0) -> tuple[int, float]:
    best = None
    for a in korobov_candidates(n, count, seed):
        crit = p2_criterion(n, korobov_vector(n, a, SEARCH_DIM))
        if best is None or crit < best[1]:
            best = (a, crit)
    return best


def primitive_root(n: int) -> int:
    """Smallest generator of the multiplicative group mod the prime n."""
    m, f, d = n - 1, [], 2
    while d * d <= m:
        if m % d == 0:
            f.append(d)
            while m % d == 0:
                m //= d
        d += 1
    if m > 1:
        f.append(m)
    for g in range(2, n):
        if all(pow(g, (n - 1) // q, n) != 1 for q in f):
            return g
    raise ValueError(n)


def cbc_vector(n: int, dim: int = DMAX, weights=None) -> tuple[list[int], float]:
    """Component-by-component construction (fast CBC: Nuyens and Cools,
    Math. Comp. 75 (2006)) of z for prime n, minimising the same P_2 as the
    Korobov search, with product weights (default 1).  Step s picks
    z_s = argmin_z sum_k P_{s-1}(k) omega({k z / n}), omega = 2 pi^2 B_2,
    P_{s-1}(k) = prod_{j<s} (1 + gamma_j omega({k z_j / n})).  With
    z = g^a and k = g^c (g a primitive root) the sum over k != 0 is the
    circular correlation of omega(g^x / n) with P(g^c), done by FFT; k = 0
    adds the same constant to every z.  Returns (z, P_2 for all dim
    components)."""
    assert is_prime(n)
    gam = np.ones(dim) if weights is None else np.asarray(weights, dtype=np.float64)
    g = primitive_root(n)
    m = n - 1
    # perm[a] = g^a mod n, in blocks: g^(kB + i) = g^(kB) g^i (int64 products
    # stay below 2^62 for n < 2^31)
    blk = min(m, 1 << 16)
    base = np.empty(blk, dtype=np.int64)
    x = 1
    for i in range(blk):
        base[i] = x
        x = x * g % n
    step = x                                    # g^blk
    perm = np.empty(m, dtype=np.int64)
    start = 1
    for lo in range(0, m, blk):
        hi = min(m, lo + blk)
        perm[lo:hi] = start * base[:hi - lo] % n
        start = start * step % n
    xs = perm.astype(np.float64) / n
    omega = 2.0 * math.pi ** 2 * (xs * xs - xs + 1.0 / 6.0)   # omega(g^a / n)
    fw = np.fft.rfft(omega)
    P = np.ones(m)                              # P_{s-1}(g^c), c = 0..m-1
    p0 = 1.0                                    # P_{s-1}(0)
    omega0 = 2.0 * math.pi ** 2 / 6.0
    z = [1]
    P *= 1.0 + gam[0] * omega
    p0 *= 1.0 + gam[0] * omega0
    for s in range(1, dim):
        # corr[a] = sum_c omega[(a + c) mod m] P[c]
        corr = np.fft.irfft(fw * np.conj(np.fft.rfft(P)), m)
        a = int(np.argmin(corr))
        zs = int(perm[a])
        z.append(zs)
        # P(g^c) *= 1 + gamma omega(g^(c + a) / n)
        P *= 1.0 + gam[s] * np.roll(omega, -a)
        p0 *= 1.0 + gam[s] * omega0
    p2 = (p0 + float(P.sum())) / n - 1.0
    return z, p2


@lru_cache(maxsize=1)
def _table() -> dict:
    if not os.path.exists(_DATA):
        raise FileNotFoundError(
            f"{_DATA} is missing; run `python -m seeded_inputs.lattice`")
    with open(_DATA) as fh:
        return json.load(fh)


CBC_MAX_N = 10000019    # CBC vectors are stored for the prime sizes up to this


def lattice(n: int, kind: str = "korobov") -> np.ndarray:
    """Stored generating vector z[DMAX] (uint32) for lattice size n: the
    Korobov vector (default) or, for prime n <= CBC_MAX_N, the CBC one."""
    rec = _table().get(str(n))
    if rec is None:
        raise KeyError(f"no stored generating vector for n={n}")
    if kind == "cbc":
        if "cbc" not in rec:
            raise KeyError(f"no stored CBC vector for n={n}")
        z = np.array(rec["cbc"]["z"], dtype=np.uint32)
    elif kind == "korobov":
        z = np.array(rec["z"], dtype=np.uint32)
    else:
        raise ValueError(kind)
    assert z.shape == (DMAX,)
    return z


def stored_sizes() -> list[int]:
    return sorted(int(k) for k in _table() if k.isdigit())


# The embedded (extensible) rank-1 rule of the serving path: one odd
# generating vector z, used at every n = 2^k as z mod 2^k, so that the
# points of size 2^k are the even-index points of size 2^(k+1) (Section
# III's lattice rule grown by doubling).  It is chosen among seeded Korobov
# candidates a (z = (1, a, a^2, ...) mod 2^24) by the P_2 criterion summed
# over the sizes the serving path uses, n = 2^14 .. 2^22, instead of at a
# single n.
EMBED_KMIN, EMBED_KMAX = 14, 22
EMBED_N = 1 << 24


def embedded_criterion(a: int, kmin: int = EMBED_KMIN, kmax: int = EMBED_KMAX,
                       dim: int = SEARCH_DIM) -> float:
    """Sum over n = 2^kmin .. 2^kmax of P_2 of the rule (z mod n, n) with
    z = (1, a, a^2, ...) mod 2^24."""
    z = korobov_vector(EMBED_N, a, dim)
    return sum(p2_criterion(1 << k, [v % (1 << k) for v in z]) for k in range(kmin, kmax + 1))


def _embedded_one(a: int) -> tuple[int, float]:
    return a, embedded_criterion(a)


def search_embedded(count: int = 64) -> dict:
    from multiprocessing import Pool
    cands = korobov_candidates(EMBED_N, count)
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        scores = dict(pool.map(_embedded_one, cands))
    a = min(cands, key=lambda c: scores[c])
    return {"a": a, "z": korobov_vector(EMBED_N, a, DMAX), "criterion": scores[a],
            "kmin": EMBED_KMIN, "kmax": EMBED_KMAX, "candidates": count,
            "search_dim": SEARCH_DIM}


def embedded_lattice() -> np.ndarray:
    """The stored odd generating vector z[DMAX] of the embedded rule for
    n = 2^k (serving); reduce it mod n for a rule of size n."""
    z = np.array(_table()["embedded"]["z"], dtype=np.uint32)
    assert z.shape == (DMAX,) and np.all(z % 2 == 1)
    return z


def _candidate_count(n: int) -> int:
    if n <= 1 << 20:
        return 64
    if n <= 1 << 24:
        return 16
    return 8


def _make_one(n: int) -> tuple[int, dict]:
    a, crit = search_korobov(n, _candidate_count(n))
    return n, {"a": a, "p2": crit, "z": korobov_vector(n, a, DMAX),
               "candidates": _candidate_count(n), "search_dim": SEARCH_DIM}


def _make_cbc(n: int) -> tuple[int, dict]:
    z, p2 = cbc_vector(n, DMAX)
    return n, {"z": z, "p2": p2, "weights": "unit"}


def main() -> None:
    from multiprocessing import Pool
    sizes = sorted(set(PRIME_SIZES + POW2_SIZES), reverse=True)
    for n in PRIME_SIZES:
        assert is_prime(n), n
    old = {}
    if os.path.exists(_DATA):
        with open(_DATA) as fh:
            old = json.load(fh)
    todo = [n for n in sizes if str(n) not in old]
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        for n, rec in pool.imap_unordered(_make_one, todo):
            old[str(n)] = rec
            print(n, rec["a"], rec["p2"], flush=True)
            _dump(old)
    todo = [n for n in PRIME_SIZES if n <= CBC_MAX_N and "cbc" not in old[str(n)]]
    with Pool(min(4, os.cpu_count() or 1)) as pool:
        for n, rec in pool.imap_unordered(_make_cbc, todo):
            old[str(n)]["cbc"] = rec
            print(n, "cbc", rec["p2"], flush=True)
            _dump(old)
    if "embedded" not in old:
        old["embedded"] = search_embedded()
        print("embedded", old["embedded"]["a"], old["embedded"]["criterion"], flush=True)
        _dump(old)


def _dump(table: dict) -> None:
    keys = sorted((k for k in table if k.isdigit()), key=int) + \
        sorted(k for k in table if not k.isdigit())
    with open(_DATA, "w") as fh:
        json.dump({k: table[k] for k in keys}, fh, indent=1)


if __name__ == "__main__":
    main()
