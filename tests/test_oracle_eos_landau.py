"""Pins of the oracle's equation of state (Sec. II.B) and Landau frame (Sec. II.A)."""
import json
import os

import numpy as np
import pytest
from mpmath import mp

from oracle import eos
from oracle.landau import landau_frame
from oracle.special import k_ratio_np

PINS = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_pins.json")))


def test_bessel_ratio_against_mpmath():
    z = np.geomspace(1e-3, 1e3, 61)
    with mp.workdps(30):
        ref = np.array([float(mp.besselk(1, x) / mp.besselk(2, x)) for x in z])
    assert np.abs(k_ratio_np(1, 2, z) / ref - 1).max() < 2e-14


def test_eos_limits():
    lim = PINS["eos_limits"]
    # eq. eos-difference: eps/(3nT) -> 1 for m/T -> 0
    T = 1.0
    for z in (1e-3, 1e-4):
        e = eos.energy_per_particle(T, z * T)
        assert abs(e / (3 * T) - lim["ultra_relativistic_ratio"]) < z
    # eq. nonRel1: (eps - n m)/(n T) -> 3/2 for m/T -> infinity
    for z in (1e3, 1e4):
        e = eos.energy_per_particle(T, z * T)
        assert abs((e - z * T) / T - lim["non_relativistic_kinetic_over_nT"]) < 2.0 / z


def test_heat_capacity_bounds():
    # d(eps/n)/dT between 3/2 and 3: the bracket used by the inversion
    T = np.geomspace(0.01, 100, 400)
    for zeta in (0.36, 1.0, 5.0, 10.0):
        h = 1e-6 * T
        cv = (eos.energy_per_particle(T + h, zeta) - eos.energy_per_particle(T - h, zeta)) / (2 * h)
        assert cv.min() > 1.5 - 1e-6 and cv.max() < 3 + 1e-6


@pytest.mark.parametrize("zeta", [0.36, 1.0, 5.0, 10.0])
def test_eos_inversion_round_trip(zeta):
    T = np.geomspace(0.05, 20, 200)
    e = eos.energy_per_particle(T, zeta)
    # conditioning: a rounding of e moves T by about ulp(e)/c_v with c_v >= 3/2
    err = np.abs(eos.temperature(e, zeta) - T)
    assert (err / (np.finfo(float).eps * (e / 1.5 + T))).max() < 4.0


def boost(u):
    u = np.asarray(u, dtype=float)
    g = 1 / np.sqrt(1 - u @ u)
    L = np.eye(4)
    L[0, 0] = g
    L[0, 1:] = L[1:, 0] = g * u
    if u @ u > 0:
        L[1:, 1:] += (g - 1) * np.outer(u, u) / (u @ u)
    return L


def test_landau_frame_recovers_boosted_rest_frame():
    """A tensor that is diag(eps, P1, P2, P3) + heat-flux-free in its rest frame,
    boosted by u: the Landau frame must return that u and eps exactly (P_i
    arbitrary, i.e. strongly non-equilibrium, shear and bulk stresses)."""
    rng = np.random.default_rng(7)
    for _ in range(50):
        eps = rng.uniform(1, 10)
        P = eps * rng.uniform(-0.2, 0.45, 3)
        n0 = rng.uniform(0.1, 3)
        q = rng.normal(size=3) * 0.3 * n0                    # particle diffusion (orthogonal to U)
        u = rng.normal(size=3)
        u *= rng.uniform(0, 0.8) / np.linalg.norm(u)
        L = boost(u)
        T = L @ np.diag([eps, *P]) @ L.T
        N = L @ np.array([n0, *q])
        e, U, n = landau_frame(T[None], N[None])
        assert abs(e[0] / eps - 1) < 1e-13
        assert np.abs(U[0] - L[:, 0]).max() < 1e-13
        assert abs(n[0] / n0 - 1) < 1e-13
        # 2D version: no z motion and no z stress coupling
        u2 = np.array([u[0], u[1], 0.0])
        L2 = boost(u2)
        T2 = (L2 @ np.diag([eps, *P]) @ L2.T)[:3, :3]
        N2 = (L2 @ np.array([n0, q[0], q[1], 0]))[:3]
        e, U, n = landau_frame(T2[None], N2[None])
        assert abs(e[0] / eps - 1) < 1e-13 and np.abs(U[0] - L2[:3, 0]).max() < 1e-13
