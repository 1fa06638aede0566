"""Pins of the Appendix A polynomials and Appendix B projections used by the
oracle: orthonormality and projections by brute-force numerical integration
over momentum space, independent of the closed forms."""
import numpy as np
import pytest
from mpmath import mp
from scipy.special import kv

from oracle.polynomials import evaluate_printed, coefficients, evaluate_coefficients, NPOLY
from oracle.projections import projections
from oracle.lattice import four_velocity


def momentum_rule(mbar, h=0.01, tmax=None, n_theta=40, n_phi=40):
    """Nodes p [N, 4] and weights (for d^3p/p^0) of a product rule:
    |p| = mbar sinh t, p0 = mbar cosh t (so d^3p/p^0 = mbar^2 sinh^2 t dt dOmega),
    trapezoid in t, Gauss-Legendre in cos(theta), trapezoid in phi."""
    if tmax is None:
        tmax = np.arccosh(60.0 / mbar + 1.0) + 1.0
    t = np.arange(h / 2, tmax, h)
    wt = np.full_like(t, h) * mbar**2 * np.sinh(t) ** 2
    x, wx = np.polynomial.legendre.leggauss(n_theta)
    phi = np.arange(n_phi) * 2 * np.pi / n_phi
    wphi = np.full(n_phi, 2 * np.pi / n_phi)
    P = np.abs(mbar * np.sinh(t))[:, None, None]
    st = np.sqrt(1 - x**2)[None, :, None]
    p = np.stack(np.broadcast_arrays(mbar * np.cosh(t)[:, None, None],
                                     P * st * np.cos(phi)[None, None, :],
                                     P * st * np.sin(phi)[None, None, :],
                                     P * x[None, :, None]), axis=-1)
    w = wt[:, None, None] * wx[None, :, None] * wphi[None, None, :]
    return p.reshape(-1, 4), w.reshape(-1)


@pytest.mark.parametrize("mbar", [0.36, 1.0, 2.0, 5.0])
def test_orthonormality_numerical(mbar):
    p, w = momentum_rule(mbar, h=0.02, n_theta=10, n_phi=12)
    NR = 4 * np.pi * mbar * kv(1, mbar)                 # eq. cercignani-recurrence-relation
    omega = np.exp(-p[:, 0]) / NR
    J = np.array(evaluate_printed(p, mbar))             # [14, N]
    G = (J * (omega * w)) @ J.T
    assert np.abs(G - np.eye(NPOLY)).max() < 1e-11


def test_coefficient_form_equals_printed_form():
    rng = np.random.default_rng(1)
    p = rng.normal(size=(50, 4)) * 3
    for mbar in (0.36, 1.0, 5.0):
        a = np.array(evaluate_printed(p, mbar))
        b = evaluate_coefficients(coefficients(mbar), p)
        assert np.abs(a - b).max() < 1e-12 * max(1, np.abs(a).max())


def numeric_projection(mbar, U, T):
    """b^(k) = int f^eq J^(k) d^3p/p^0 with f^eq = exp(-p.U/T) normalised so that
    int f^eq p^0 d^3p/p^0 = U^0 (unit density), by brute-force quadrature."""
    p, w = momentum_rule(mbar, h=0.01 * min(1.0, T), n_theta=48, n_phi=48,
                         tmax=np.arccosh(80.0 * T / mbar + 1.0) + 1.0)
    pU = p[:, 0] * U[0] - p[:, 1:] @ U[1:]
    fe = np.exp(-(pU - mbar) / T) * w                   # constant factor cancels
    fe *= U[0] / np.sum(fe * p[:, 0])
    J = np.array(evaluate_printed(p, mbar))
    return J @ fe


@pytest.mark.parametrize("mbar,T,u", [(1.0, 1.0, (0.3, -0.2, 0.0)), (5.0, 0.7, (0.2, 0.1, 0.15)),
                                      (2.0, 0.7, (0.3, 0.0, 0.0)), (0.36, 1.3, (-0.1, 0.35, 0.0))])
def test_projections_bruteforce(mbar, T, u):
    g = 1 / np.sqrt(1 - sum(c * c for c in u))
    U = np.array([g, g * u[0], g * u[1], g * u[2]])
    b_num = numeric_projection(mbar, U, T)
    b = projections(U[None, :], np.array([T]), mbar, coefficients(mbar))[:, 0]
    assert np.abs(b - b_num).max() < 1e-9 * max(1.0, np.abs(b).max())


def test_rest_frame_at_reference_temperature():
    # f^eq(U = rest, T = T_R) = omega * K1(mbar)/(mbar K2(mbar)): only b^(0) survives
    for mbar in (0.36, 1.0, 5.0):
        b = projections(np.array([[1.0, 0, 0, 0]]), np.array([1.0]), mbar, coefficients(mbar))[:, 0]
        assert abs(b[0] - kv(1, mbar) / (mbar * kv(2, mbar))) < 1e-15
        assert np.abs(b[1:]).max() < 1e-13


def printed_appendix_b(mbar, U, T):
    """Appendix B as printed (T_R = 1), keyed by the printed label."""
    m = mbar
    k1, k2, k3 = (float(mp.besselk(i, m)) for i in (1, 2, 3))
    z = m / T
    r1 = kv(1, z) / kv(2, z)
    r3 = kv(3, z) / kv(2, z)
    A = np.sqrt(m * (m + k2 * (3 * k1 - m * k2) / k1**2))
    B = np.sqrt(m * k2 / k1)
    C = np.sqrt(2 * m**2 + 5 * m * k2 / k1 - 3 * k1 * (m * k1 + 3 * k2) / (m * k1**2 + 3 * k2 * k1 - m * k2**2) + 3)
    D = np.sqrt(m**2 * (m * k2**2 + 5 * k3 * k2 - m * k3**2) / (k1 * k2))
    E = np.sqrt(m**2 * k3 / k1)
    U0, Ux, Uy, Uz = U
    X = -m * k1 / k2 + m * k2 / k1 - 3
    Y = (-m**2 * k1**2 + (m**2 + 3) * k2**2 - 3 * m * k2 * k1) / (m * k1**2 + 3 * k2 * k1 - m * k2**2)
    return {
        "0": r1 / m,
        "1_0": (U0 - k2 / k1 * r1) / A,
        "1_x": Ux / B, "1_y": Uy / B, "1_z": Uz / B,
        "2_00_printed": (U0**2 * m * r3 + U0 * (1 / X - 1) + r1 * (Y + T / r1)) / (np.sqrt(3) * C),
        "2_00_reading": (U0**2 * m * r3 + 3 * U0 * (1 / X - 1) + r1 * Y - T) / (np.sqrt(3) * C),
        "2_0x": (m * r3 * U0 * Ux - m * k3 / k2 * Ux) / D,
        "2_0y": (m * r3 * U0 * Uy - m * k3 / k2 * Uy) / D,
        "2_0z": (m * r3 * U0 * Uz - m * k3 / k2 * Uz) / D,
        "2_xx_printed": m * r3 * (-2 * Ux**2 + Uy**2 + Uz**2) / (2 * np.sqrt(3) * E),
        "2_yy_printed": m * r3 * (Uy**2 - Uz**2) / (2 * E),
        "2_xz_printed": m * r3 * Ux * Uz / E,
        "2_yz_printed": m * r3 * Ux * Uy / E,
        "2_xy_printed": m * r3 * Uy * Uz / E,
    }


def test_appendix_b_against_definition():
    """The printed Appendix B entries agree with the projections by definition,
    pairing the spatial-quadratic coefficients with the Appendix A polynomial of
    the same tensor structure; the printed b_00 is garbled and the reading
    (factor 3 on the U_0 term, -T instead of +T) agrees instead."""
    rng = np.random.default_rng(3)
    for mbar in (0.36, 1.0, 2.0, 5.0):
        cf = coefficients(mbar)
        for _ in range(5):
            u = rng.uniform(-0.35, 0.35, 3)
            T = rng.uniform(0.5, 1.6)
            U = four_velocity(u[0], u[1]) * 0
            g = 1 / np.sqrt(1 - u @ u)
            U = np.array([g, g * u[0], g * u[1], g * u[2]])
            b = projections(U[None], np.array([T]), mbar, cf)[:, 0]
            pr = printed_appendix_b(mbar, U, T)
            ours = dict(zip(["0", "1_0", "1_x", "1_y", "1_z", "2_00", "2_0x", "2_0y", "2_0z",
                             "2_xx", "2_yy", "2_xz", "2_yz", "2_xy"], b))
            tol = 1e-12 * max(1.0, np.abs(b).max())
            for key in ("0", "1_0", "1_x", "1_y", "1_z", "2_0x", "2_0y", "2_0z"):
                assert abs(ours[key] - pr[key]) < tol, key
            assert abs(ours["2_00"] - pr["2_00_reading"]) < tol
            assert abs(ours["2_yy"] - pr["2_xx_printed"]) < tol   # (-2x^2+y^2+z^2) structure
            assert abs(ours["2_xx"] - pr["2_yy_printed"]) < tol   # (y^2-z^2) structure
            assert abs(ours["2_xz"] - pr["2_xz_printed"]) < tol
            assert abs(ours["2_xy"] - pr["2_yz_printed"]) < tol   # U_x U_y structure
            assert abs(ours["2_yz"] - pr["2_xy_printed"]) < tol   # U_y U_z structure
    # the printed b_00 does not vanish in the rest frame at T = T_R, where every
    # b except b^(0) must (f^eq is then proportional to the weight function)
    pr = printed_appendix_b(2.0, np.array([1.0, 0, 0, 0]), 1.0)
    assert abs(pr["2_00_printed"]) > 0.1 and abs(pr["2_00_reading"]) < 1e-13
