"""Equation of state of a relativistic perfect gas (Sec. II.B, eq. relativistic-eos):

    eps = 3 n T + n m K_1(m/T)/K_2(m/T),     P = n T.

Lattice units: T_R = 1 so m = mbar = zeta.  The inversion T(eps/n) uses plain
bisection on a bracket that follows from the heat capacity per particle lying
between the non-relativistic 3/2 and the ultra-relativistic 3 (the limits
discussed with eq. nonRel1): with h(T) = eps/n = 3T + m K_1/K_2 and h(0) = m,
    m + 1.5 T <= h(T) <= m + 3 T   and   3 T <= h(T),
so T lies in [(e - m)/3, min((e - m)/1.5, e/3)].  Bisection to the last bit
makes the root unambiguous (h is strictly increasing).
"""
import numpy as np
from .special import k_ratio_np


def energy_per_particle(T, zeta):
    T = np.asarray(T, dtype=np.float64)
    return 3.0 * T + zeta * k_ratio_np(1, 2, zeta / T)


def temperature(e, zeta, iters=200):
    """Invert e = eps/n = 3T + zeta K_1(zeta/T)/K_2(zeta/T) for T by bisection."""
    e = np.asarray(e, dtype=np.float64)
    lo = np.maximum((e - zeta) / 3.0, 0.0)
    hi = np.minimum((e - zeta) / 1.5, e / 3.0)
    lo = np.minimum(lo, hi)
    lo = np.where(lo <= 0.0, hi * 1e-6, lo)   # keep z = zeta/T finite
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        f = energy_per_particle(mid, zeta) - e
        lo = np.where(f < 0.0, mid, lo)
        hi = np.where(f < 0.0, hi, mid)
        if np.all((hi - lo) <= 4e-16 * np.abs(hi)):
            break
    return 0.5 * (lo + hi)
