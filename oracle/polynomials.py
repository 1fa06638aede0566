"""Second-order relativistic orthonormal polynomials (Sec. III.A, Appendix A).

The weight is the rest-frame Maxwell-Juettner distribution
omega(p0) = exp(-p0/T_R)/N_R with N_R = 4 pi mbar T_R^2 K_1(mbar)
(eq. mj-poly-weighting-factor, eq. cercignani-recurrence-relation), with the
measure d^3p/p^0.  Everything is written in the adimensional momenta
pbar = p/T_R, so T_R drops out and only mbar = m/T_R enters.

The 14 polynomials are kept in the order
    0, 1_0, 1_x, 1_y, 1_z, 2_00, 2_0x, 2_0y, 2_0z, 2_xx, 2_yy, 2_xz, 2_yz, 2_xy
with the labels of Appendix A (note: the appendix's "J_xx" is the
(p_y^2 - p_z^2) combination and its "J_yy" the (-2 p_x^2 + p_y^2 + p_z^2) one).
Momentum components are contravariant p^mu; a sign convention on the spatial
components flips J and its projection together and cancels in f^eq.

Two equivalent representations are provided:
  * ``evaluate_printed``: the expressions exactly as printed in Appendix A;
  * ``coefficients``: each J as c + l_mu p^mu + Q_{mu nu} p^mu p^nu, read off
    the printed expressions; used to integrate J against f^eq in closed form.
"""
import numpy as np
from mpmath import mp, mpf, sqrt as msqrt

LABELS = ["0", "1_0", "1_x", "1_y", "1_z", "2_00", "2_0x", "2_0y", "2_0z",
          "2_xx", "2_yy", "2_xz", "2_yz", "2_xy"]
NPOLY = len(LABELS)


def constants(mbar, dps=40):
    """Normalisation constants A..E and the mbar-dependent coefficients of
    Appendix A, evaluated with mpmath at ``dps`` digits.  Returns mpf values."""
    with mp.workdps(dps):
        m = mpf(mbar)
        k1, k2, k3 = mp.besselk(1, m), mp.besselk(2, m), mp.besselk(3, m)
        den = m * k1**2 + 3 * k2 * k1 - m * k2**2
        c = {
            "k1": k1, "k2": k2, "k3": k3,
            "A": msqrt(m * (m + k2 * (3 * k1 - m * k2) / k1**2)),
            "B": msqrt(m * k2 / k1),
            "C": msqrt(2 * m**2 + 5 * m * k2 / k1 - 3 * k1 * (m * k1 + 3 * k2) / den + 3),
            "D": msqrt(m**2 * (m * k2**2 + 5 * k3 * k2 - m * k3**2) / (k1 * k2)),
            "E": msqrt(m**2 * k3 / k1),
            # J_0^(1) offset, J_00^(2) linear and constant terms, J_0i^(2) offset
            "a1": m * k2 / k1,
            "c1": 3 / (-m * k1 / k2 + m * k2 / k1 - 3) - 3,
            "c0": 3 * k1 * (m * k1 + 3 * k2) / den - m**2 - 3,
            "d0": m * k3 / k2,
        }
        return c


def evaluate_printed(p, mbar, dps=40):
    """Evaluate the 14 polynomials of Appendix A, as printed, at momenta ``p``
    (array [..., 4] of contravariant pbar^mu, float or mpf objects).
    Returns a list of 14 arrays."""
    c = constants(mbar, dps)
    f = lambda v: v if isinstance(p, np.ndarray) and p.dtype == object else float(v)
    A, B, C, D, E = (f(c[k]) for k in "ABCDE")
    a1, c1, c0, d0 = f(c["a1"]), f(c["c1"]), f(c["c0"]), f(c["d0"])
    s3 = f(msqrt(3)) if not (isinstance(p, np.ndarray) and p.dtype == object) else msqrt(3)
    p0, px, py, pz = p[..., 0], p[..., 1], p[..., 2], p[..., 3]
    one = p0 * 0 + 1
    return [
        one,
        (p0 - a1) / A,
        px / B, py / B, pz / B,
        (p0**2 + p0 * c1 + c0) / (s3 * C),
        px * (p0 - d0) / D, py * (p0 - d0) / D, pz * (p0 - d0) / D,
        (py**2 / 2 - pz**2 / 2) / E,
        (-2 * px**2 + py**2 + pz**2) / (2 * s3 * E),
        px * pz / E, py * pz / E, px * py / E,
    ]


def coefficients(mbar, dps=40):
    """Each polynomial as (c, l[4], Q[4,4]) with J = c + l.p + p.Q.p, as mpf
    arrays (object dtype), read off the printed Appendix A expressions."""
    k = constants(mbar, dps)
    with mp.workdps(dps):
        z = mpf(0)
        s3 = msqrt(3)
        out = []

        def poly(c=z, l=None, q=None):
            L = np.array([z] * 4, dtype=object)
            Q = np.array([[z] * 4 for _ in range(4)], dtype=object)
            for (i, v) in (l or {}).items():
                L[i] = v
            for ((i, j), v) in (q or {}).items():
                Q[i, j] = v
            out.append((c, L, Q))

        poly(c=mpf(1))                                              # 0
        poly(c=-k["a1"] / k["A"], l={0: 1 / k["A"]})                # 1_0
        for i in (1, 2, 3):                                         # 1_x,y,z
            poly(l={i: 1 / k["B"]})
        n00 = s3 * k["C"]                                           # 2_00
        poly(c=k["c0"] / n00, l={0: k["c1"] / n00}, q={(0, 0): 1 / n00})
        for i in (1, 2, 3):                                         # 2_0x,0y,0z
            poly(l={i: -k["d0"] / k["D"]}, q={(0, i): 1 / k["D"]})
        E = k["E"]
        poly(q={(2, 2): 1 / (2 * E), (3, 3): -1 / (2 * E)})         # 2_xx (App. A label)
        poly(q={(1, 1): -2 / (2 * s3 * E), (2, 2): 1 / (2 * s3 * E),
                (3, 3): 1 / (2 * s3 * E)})                          # 2_yy (App. A label)
        poly(q={(1, 3): 1 / E})                                     # 2_xz
        poly(q={(2, 3): 1 / E})                                     # 2_yz
        poly(q={(1, 2): 1 / E})                                     # 2_xy
        return out


def evaluate_coefficients(coeffs, p):
    """Evaluate (c, l, Q) polynomials at float64 momenta p [..., 4]."""
    p = np.asarray(p, dtype=np.float64)
    res = []
    for (c, l, Q) in coeffs:
        cf = float(c)
        lf = np.array([float(v) for v in l])
        Qf = np.array([[float(v) for v in row] for row in Q])
        res.append(cf + p @ lf + np.einsum("...i,ij,...j->...", p, Qf, p))
    return np.array(res)
