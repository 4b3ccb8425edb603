"""Closed forms and exact results that pin the oracle (test helpers).

None of these routines shares code with the oracle or the HIP path:
  * exact enumeration of all 2^(L*L) states of a small periodic lattice
    (energy from Eq. (1) with J = 1, no field), giving the exact density of
    states and thermal moments;
  * B. Kaufman's exact partition function of the finite periodic L x L
    lattice (Phys. Rev. 76, 1232 (1949)), in the form with the four
    products over gamma_k, evaluated with mpmath;
  * L. Onsager's infinite-lattice internal energy per site
    (Phys. Rev. 65, 117 (1944)) and C. N. Yang's spontaneous magnetisation
    (Phys. Rev. 85, 808 (1952));
  * the Binder cumulant U4 = 1 - <M^4> / (3 <M^2>^2), Eq. (2) of the paper.
"""
import math

import mpmath
import numpy as np
from scipy.special import ellipk

TC_EXACT = 2.0 / math.log(1.0 + math.sqrt(2.0))


def enumerate_states(L: int):
    """All 2^(L*L) configurations: returns (E, M) int64 arrays."""
    n = L * L
    assert n <= 20, "enumeration is for tiny lattices only"
    idx = np.arange(1 << n, dtype=np.int64)
    bits = ((idx[:, None] >> np.arange(n, dtype=np.int64)[None, :]) & 1).astype(np.int8)
    s = (2 * bits - 1).reshape(-1, L, L).astype(np.int64)
    E = -(s * np.roll(s, -1, axis=2) + s * np.roll(s, -1, axis=1)).sum(axis=(1, 2))
    M = s.sum(axis=(1, 2))
    return E, M


def density_of_states(L: int):
    """{E: number of states} from exact enumeration."""
    E, _ = enumerate_states(L)
    vals, counts = np.unique(E, return_counts=True)
    return {int(v): int(c) for v, c in zip(vals, counts)}


def exact_moments(L: int, T: float):
    """Exact thermal averages from enumeration: <E>/N, <M^2>/N^2, <M^4>/N^4, U4,
    and the exact probability of each energy level (dict)."""
    E, M = enumerate_states(L)
    beta = 1.0 / T
    e0 = E.min()
    w = np.exp(-beta * (E - e0).astype(np.float64))
    Z = w.sum()
    N = L * L
    m2 = (w * (M.astype(np.float64) ** 2)).sum() / Z
    m4 = (w * (M.astype(np.float64) ** 4)).sum() / Z
    eav = (w * E).sum() / Z
    levels = {}
    for e in np.unique(E):
        levels[int(e)] = float(w[E == e].sum() / Z)
    return {
        "e": eav / N,
        "m2": m2 / N ** 2,
        "m4": m4 / N ** 4,
        "u4": 1.0 - m4 / (3.0 * m2 * m2),
        "p_energy": levels,
    }


def kaufman_logZ(L: int, beta, dps: int = 60):
    """ln Z of the periodic L x L Ising model (J = 1, no field), Kaufman 1949.

    Z = 1/2 (2 sinh 2K)^(N/2) [P1 + P2 + P3 + P4], K = beta,
    P1 = prod_{r=0}^{L-1} 2 cosh(L g_{2r+1} / 2),  P2 = same with sinh,
    P3 = prod_{r=0}^{L-1} 2 cosh(L g_{2r} / 2),    P4 = same with sinh,
    cosh g_l = cosh 2K coth 2K - cos(pi l / L) for l >= 1, and
    g_0 = 2K + ln tanh K taken with its sign.
    """
    with mpmath.workdps(dps):
        K = mpmath.mpf(beta)
        c = mpmath.cosh(2 * K) * mpmath.coth(2 * K)

        def gamma(l):
            if l == 0:
                return 2 * K + mpmath.log(mpmath.tanh(K))
            return mpmath.acosh(c - mpmath.cos(mpmath.pi * l / L))

        P1 = P2 = P3 = P4 = mpmath.mpf(1)
        for r in range(L):
            go = gamma(2 * r + 1)
            ge = gamma(2 * r)
            P1 *= 2 * mpmath.cosh(L * go / 2)
            P2 *= 2 * mpmath.sinh(L * go / 2)
            P3 *= 2 * mpmath.cosh(L * ge / 2)
            P4 *= 2 * mpmath.sinh(L * ge / 2)
        N = L * L
        Z = mpmath.mpf(1) / 2 * (2 * mpmath.sinh(2 * K)) ** (mpmath.mpf(N) / 2) * (P1 + P2 + P3 + P4)
        return mpmath.log(Z)


def kaufman_energy_per_site(L: int, T: float, dps: int = 60) -> float:
    """Exact <E>/N of the finite periodic lattice: -d ln Z / d beta / N."""
    with mpmath.workdps(dps + 40):
        b = mpmath.mpf(1) / mpmath.mpf(T)
        h = mpmath.mpf(10) ** (-(dps // 2))
        d = (kaufman_logZ(L, b + h, dps + 40) - kaufman_logZ(L, b - h, dps + 40)) / (2 * h)
        return float(-d / (L * L))


def onsager_energy_per_site(T: float) -> float:
    """Onsager: u = -coth 2b [1 + (2/pi)(2 tanh^2 2b - 1) K(k)], k = 2 sinh 2b / cosh^2 2b."""
    b = 1.0 / T
    k = 2.0 * math.sinh(2 * b) / math.cosh(2 * b) ** 2
    Kk = float(ellipk(k * k))
    return -1.0 / math.tanh(2 * b) * (1.0 + (2.0 / math.pi) * (2.0 * math.tanh(2 * b) ** 2 - 1.0) * Kk)


def spontaneous_magnetisation(T: float) -> float:
    """Yang: m = (1 - sinh^-4 2b)^(1/8) below T_c, 0 above."""
    if T >= TC_EXACT:
        return 0.0
    b = 1.0 / T
    return (1.0 - math.sinh(2 * b) ** -4) ** 0.125


def binder(M) -> float:
    """U4 = 1 - <M^4> / (3 <M^2>^2) (Eq. (2)), from an integer series, summed exactly."""
    m = [int(v) for v in M]
    n = len(m)
    s2 = sum(v * v for v in m)
    s4 = sum(v ** 4 for v in m)
    from fractions import Fraction
    return float(1 - Fraction(s4, n) / (3 * Fraction(s2, n) ** 2))


def binned_mean_err(x, nbins: int = 50):
    """Mean and standard error from nbins consecutive bins (for correlated series)."""
    x = np.asarray(x, dtype=np.float64)
    n = (len(x) // nbins) * nbins
    b = x[:n].reshape(nbins, -1).mean(axis=1)
    return float(b.mean()), float(b.std(ddof=1) / math.sqrt(nbins))
