"""Pins of the oracle's streaming step, its outflow rule and the entropy
density inside the eta/s relaxation time.

Streaming (Sec. III.B, eq. discrete-relativistic-boltzmann): a population of
momentum p_i = p^0 (1, v0 n_i) (eq. four-momentum) moves by n_i sites per step
(eq. v0dt=dx).  The tests check what that implies without reading the
oracle's index arithmetic:
  * kinematics: the density centroid sum_x x N^0 moves in one step by
    sum_x N*^x / v0, the post-collision particle flux counted in sites, in
    both lattice directions;
  * dynamics: a Riemann problem started from rest (Sec. IV) drives the fluid
    toward the low-pressure side, and its momentum grows at the rate the
    pressure jump sets;
  * outflow (zero gradient): a box whose two ends differ gains and loses
    N^0 at the rate of the boundary fluxes, which a periodic box cannot do.
Each check is also run on an oracle with a planted mistake (streaming against
the velocity, outflow replaced by a periodic wrap) and must fail there.

Entropy density (Sec. IV): s = 4n - n ln(n/n_eq), n_eq = d_G T^3/pi^2 with
d_G = 16 is the entropy density of a massless Boltzmann gas.  It is pinned by
thermodynamics: s = dP/dT at fixed chemical potential, with P(T, mu) and
n(T, mu) integrated numerically over the Boltzmann distribution.
"""
import numpy as np
import pytest
from scipy import integrate, optimize

from oracle import groups, lattice as L

ZETA1 = ([1, 5, 11, 13, 17, 21], 1.0, 0.2403918860)
ZETA5 = ([1, 2, 3, 4, 5, 6], 5.0, 0.398)
_cache = {}


def stencil(which, mode="projected", dim=2):
    key = (which, mode, dim)
    if key not in _cache:
        gs, m, v0 = {"zeta1": ZETA1, "zeta5": ZETA5}[which]
        _cache[key] = L.build_stencil(groups.bases_of(gs), m, v0, mode=mode, dim=dim)
    return _cache[key]


class MirroredModel(L.Model):
    """A planted mistake: populations stream against their velocity."""

    def stream(self, fpost):
        saved = self.ps.disp
        self.ps.disp = -saved
        try:
            return super().stream(fpost)
        finally:
            self.ps.disp = saved


class WrappedModel(L.Model):
    """A planted mistake: outflow boundaries replaced by a periodic wrap."""

    def stream(self, fpost):
        saved = self.bc
        self.bc = ("periodic", "periodic")
        try:
            return super().stream(fpost)
        finally:
            self.bc = saved


def moving_bump(nx, ny):
    """A dense, moving blob of radius 7 sites (compact support) on a uniform
    gas at rest, so that nothing but the rest state comes near the edges."""
    x = np.arange(nx) - nx / 2 + 0.5
    y = np.arange(ny) - ny / 2 + 0.5
    X, Y = np.meshgrid(x, y)
    r = np.sqrt(X**2 + Y**2)
    g = np.where(r < 7.0, np.cos(np.pi * r / 14.0) ** 2, 0.0)
    return 1.0 + 0.4 * g, 1.0 + 0.2 * g, 0.3 * g, -0.2 * g


def centroid_shift(model_cls, which="zeta1", nx=32, ny=30):
    """(measured, predicted) one-step centroid shift of N^0 in x and y."""
    ps = stencil(which)
    m = model_cls(ps, nx, ny, tau=0.9)
    m.init_equilibrium(*moving_bump(nx, ny))
    xs, ys = np.meshgrid(np.arange(nx), np.arange(ny))
    N0 = lambda f: np.einsum("qyx,q->yx", f, ps.p[:, 0])
    before = N0(m.f)
    fpost = m.collide()
    # post-collision particle flux N*^i = sum_j f*_j p^i_j, in sites per step
    flux_x = np.einsum("qyx,q->", fpost, ps.p[:, 1]) / ps.v0
    flux_y = np.einsum("qyx,q->", fpost, ps.p[:, 2]) / ps.v0
    m.f = m.stream(fpost)
    after = N0(m.f)
    measured = np.array([(xs * (after - before)).sum(), (ys * (after - before)).sum()])
    return measured, np.array([flux_x, flux_y])


def test_centroid_moves_with_the_particle_flux():
    measured, predicted = centroid_shift(L.Model)
    assert np.abs(predicted).min() > 0.5          # the blob carries flux in both directions
    assert np.abs(measured - predicted).max() < 1e-11 * np.abs(predicted).max()


def test_centroid_check_rejects_mirrored_streaming():
    measured, predicted = centroid_shift(MirroredModel)
    assert np.abs(measured + predicted).max() < 1e-11 * np.abs(predicted).max()
    assert np.abs(measured - predicted).max() > 1.0


def riemann_run(model_cls, steps=40, nx=400):
    """Shock tube from rest: high pressure on the left (n = 1, T = 1.3),
    low pressure on the right (n = 0.3, T = 0.8); outflow ends."""
    ps = stencil("zeta1", "projected", dim=1)
    left = np.arange(nx) < nx // 2
    n = np.where(left, 1.0, 0.3)[None, :]
    T = np.where(left, 1.3, 0.8)[None, :]
    m = model_cls(ps, nx, 1, bc=("outflow", "periodic"), tau=1.0)
    m.init_equilibrium(n, T, 0 * n, 0 * n)
    P0 = (n * T)[0]
    m.step(steps)
    return m.fields(), P0, ps


def riemann_checks(fields, P0, ps, steps=40, nx=400):
    """Flow toward the low-pressure side, and the momentum budget: with both
    ends still at their initial states, sum_x T^0x grows by the pressure
    jump per unit time, (P_L - P_R) dt per step with dt = 1/v0 in units of
    dx (the net force on the fluid between the ends)."""
    ux = fields["ux"][0]
    mid = slice(nx // 2 - 5, nx // 2 + 5)
    toward_low = ux[mid].min() > 0.05
    T0x = fields["raw9"][4].sum()
    expected = steps * (P0[0] - P0[-1]) / ps.v0
    budget = abs(T0x - expected) < 1e-9 * expected
    return toward_low, budget


def test_riemann_flow_runs_toward_low_pressure():
    toward_low, budget = riemann_checks(*riemann_run(L.Model))
    assert toward_low
    assert budget


def test_riemann_check_rejects_mirrored_streaming():
    toward_low, budget = riemann_checks(*riemann_run(MirroredModel))
    assert not toward_low
    assert not budget


def outflow_balance(model_cls, axis):
    """One step on a box whose ends differ, outflow along ``axis`` (0: x, 1: y).
    Returns (change of sum N^0, predicted boundary balance)."""
    ps = stencil("zeta1")
    nx, ny = (20, 6) if axis == 0 else (6, 20)
    s = np.linspace(0.0, 1.0, 20)
    prof = lambda a, b: a + (b - a) * s
    shape = (ny, nx)
    tile = (lambda v: np.tile(v, (ny, 1))) if axis == 0 else (lambda v: np.tile(v[:, None], (1, nx)))
    n, T, u = tile(prof(1.0, 0.5)), tile(prof(1.2, 0.8)), tile(prof(0.3, 0.1))
    ux, uy = (u, np.zeros(shape)) if axis == 0 else (np.zeros(shape), u)
    bc = ("outflow", "periodic") if axis == 0 else ("periodic", "outflow")
    m = model_cls(ps, nx, ny, bc=bc, tau=0.9)
    m.init_equilibrium(n, T, ux, uy)
    p0 = ps.p[:, 0]
    total = lambda f: np.einsum("qyx,q->", f, p0)
    before = total(m.f)
    fpost = m.collide()
    m.f = m.stream(fpost)
    after = total(m.f)
    # Zero gradient: the populations a boundary site sends out of the box are
    # lost, and each end site stands for every site beyond it, so it feeds
    # |n| of its own post-collision values of each inward class back in.
    g = fpost if axis == 0 else np.swapaxes(fpost, 1, 2)  # [Q, transverse, along]
    d = ps.disp[:, axis]
    bal = 0.0
    for j in range(ps.Q):
        k = int(d[j])
        if k > 0:
            bal += p0[j] * (k * g[j, :, 0].sum() - g[j, :, -k:].sum())
        elif k < 0:
            bal += p0[j] * (-k * g[j, :, -1].sum() - g[j, :, :-k].sum())
    return after - before, bal


@pytest.mark.parametrize("axis", [0, 1])
def test_outflow_mass_follows_boundary_fluxes(axis):
    change, bal = outflow_balance(L.Model, axis)
    assert abs(bal) > 1e-3 * 20 * 6
    assert abs(change - bal) < 1e-12 * 20 * 6 * 10


@pytest.mark.parametrize("axis", [0, 1])
def test_outflow_check_rejects_periodic_wrap(axis):
    change, bal = outflow_balance(WrappedModel, axis)
    assert abs(change) < 1e-11 * 20 * 6 * 10       # a periodic box keeps its mass
    assert abs(change - bal) > 1e-3 * 20 * 6


# ---------------------------------------------------------------- entropy

HBARC = 0.1973269804   # GeV fm (CODATA)
D_G = 16.0             # degeneracy of the massless gas (gluons)


def boltzmann_n_P(T, mu):
    """Number density and pressure of a massless Boltzmann gas in natural
    units (GeV^3, GeV^4), by integrating d_G e^{-(p - mu)/T} over momentum."""
    fn = lambda p: p * p * np.exp(-(p - mu) / T)
    fP = lambda p: p**3 / 3.0 * np.exp(-(p - mu) / T)
    pref = D_G / (2.0 * np.pi**2)
    n = pref * integrate.quad(fn, 0, 60 * T, epsabs=0, epsrel=1e-13, limit=200)[0]
    P = pref * integrate.quad(fP, 0, 60 * T, epsabs=0, epsrel=1e-13, limit=200)[0]
    return n, P


def entropy_from_thermodynamics(n_fm3, T_GeV):
    """s = dP/dT at fixed mu, for the chemical potential that gives density
    n; returned in fm^-3."""
    n_nat = n_fm3 * HBARC**3
    mu = optimize.brentq(lambda m: boltzmann_n_P(T_GeV, m)[0] - n_nat, -50 * T_GeV, 20 * T_GeV, xtol=1e-15)
    h = 1e-4 * T_GeV
    s_nat = (boltzmann_n_P(T_GeV + h, mu)[1] - boltzmann_n_P(T_GeV - h, mu)[1]) / (2 * h)
    return s_nat / HBARC**3


@pytest.mark.parametrize("n_lat,T_lat", [(1.0, 1.0), (0.11, 0.5714), (2.5, 1.7)])
def test_entropy_density_in_tau_is_thermodynamic(n_lat, T_lat):
    """The relaxation time of the eta/s rule (Sec. IV) encodes s through
    tau - 1/2 = (3/2)(eta/s) s hbar_c v0 / (P dx); recover s from it and
    compare with dP/dT|_mu of the Boltzmann gas."""
    units = {"T_R_GeV": 0.35, "n_unit_fm3": 5.43 / 0.35, "dx_fm": 0.008}
    v0, es = 0.24, 0.1
    tau = L.tau_from_eta_over_s(np.array([n_lat]), np.array([T_lat]), es, v0, units)[0]
    n_phys = n_lat * units["n_unit_fm3"]
    T_phys = T_lat * units["T_R_GeV"]
    P_phys = n_phys * T_phys
    s_oracle = (tau - 0.5) * P_phys * units["dx_fm"] / (1.5 * es * HBARC * v0)
    s_thermo = entropy_from_thermodynamics(n_phys, T_phys)
    assert abs(s_oracle - s_thermo) < 1e-7 * abs(s_thermo)


def test_boltzmann_integrals_pinned_to_closed_forms():
    """The integrals above against n = d_G T^3 e^{mu/T}/pi^2, P = n T."""
    T, mu = 0.3, -0.2
    n, P = boltzmann_n_P(T, mu)
    assert abs(n - D_G * T**3 * np.exp(mu / T) / np.pi**2) < 1e-12 * n
    assert abs(P - n * T) < 1e-12 * P
