"""Projection coefficients of the Maxwell-Juttner equilibrium on the
second-order polynomials (eq. mj-projection-coefficients, Appendix B).

a^(k)(U, T) = integral of f^eq J^(k) d^3p/p^0, written as a^(k) = b^(k)/T_R.
Lattice units set T_R = 1, so a = b.  f^eq is normalised to unit density,
N_E^mu = U^mu (eq. maxwell-juttner-normalization); the physical density n
multiplies it.  Each J^(k) is a polynomial of degree <= 2 in p^mu, so its
projection needs only the first three moments of the unit-density
Maxwell-Juttner distribution (Sec. II, eqs. quadri-flux, energy-tensor and the
integrals I, I^alpha of Sec. III.A):

    int f^eq d^3p/p^0                = K_1(z) / (mbar K_2(z)),      z = m/T
    int f^eq p^mu d^3p/p^0           = U^mu
    int f^eq p^mu p^nu d^3p/p^0      = mbar (K_3(z)/K_2(z)) U^mu U^nu - T eta^{mu nu}

(the last one is T_E/n with (eps + P)/n = 4T + m K_1/K_2 = m K_3/K_2).
This is the definition of a^(k) written out; the printed Appendix B forms are
checked against it (and against brute-force integration) in the tests.
"""
import numpy as np
from .special import k_ratio_np

ETA = np.diag([1.0, -1.0, -1.0, -1.0])


def mj_moments(U, T, mbar):
    """Zeroth, first and second moments of the unit-density MJ distribution.
    U: [..., 4] contravariant four-velocity, T: [...] temperature (T_R = 1)."""
    U = np.asarray(U, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    z = mbar / T
    m0 = k_ratio_np(1, 2, z) / mbar
    m2 = (mbar * k_ratio_np(3, 2, z))[..., None, None] * U[..., :, None] * U[..., None, :] \
        - T[..., None, None] * ETA
    return m0, U, m2


def projections(U, T, mbar, coeffs):
    """b^(k)(U, T) for the 14 polynomials given as (c, l, Q) coefficient sets
    (``polynomials.coefficients``).  Returns an array [14, ...]."""
    m0, m1, m2 = mj_moments(U, T, mbar)
    out = []
    for (c, l, Q) in coeffs:
        cf = float(c)
        lf = np.array([float(v) for v in l])
        Qf = np.array([[float(v) for v in row] for row in Q])
        out.append(cf * m0 + m1 @ lf + np.einsum("...ij,ij->...", m2, Qf))
    return np.array(out)
