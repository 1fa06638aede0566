"""Pins of the oracle's lattice model: exact recovery of the Maxwell-Juttner
moments by the discrete equilibrium, conservation of N^0 and T^{0 nu} on
periodic boxes, the uniform fixed point, the equivalence of the projected
population classes with the paper's full 3D stencil, and 1D == 2D."""
import numpy as np
import pytest

from oracle import groups, lattice as L, eos

STENCILS = {
    "zeta5": ([1, 2, 3, 4, 5, 6], 5.0, 0.398),
    "zeta1": ([1, 5, 11, 13, 17, 21], 1.0, 0.2403918860),
    "zeta036": ([1, 14, 49, 51, 60, 70], 0.36, 0.1488231854),
}
_cache = {}


def stencil(name, mode="full", dim=2):
    key = (name, mode, dim)
    if key not in _cache:
        gs, m, v0 = STENCILS[name]
        _cache[key] = L.build_stencil(groups.bases_of(gs), m, v0, mode=mode, dim=dim)
    return _cache[key]


def random_fields(rng, ny, nx, umax=0.35):
    n = rng.uniform(0.5, 1.5, (ny, nx))
    T = rng.uniform(0.7, 1.3, (ny, nx))
    a = rng.uniform(0, 2 * np.pi, (ny, nx))
    r = rng.uniform(0, umax, (ny, nx))
    return n, T, r * np.cos(a), r * np.sin(a)


@pytest.mark.parametrize("name", list(STENCILS))
def test_equilibrium_moments_exact(name):
    """sum_i f_i^eq p_i = n U and sum_i f_i^eq p_i p_i = (eps + P) U U - P eta
    (eqs. quadri-flux, energy-tensor), eps and P from eq. relativistic-eos."""
    ps = stencil(name)
    rng = np.random.default_rng(11)
    n, T, ux, uy = (a.ravel() for a in random_fields(rng, 1, 40))
    U = L.four_velocity(ux, uy)
    f = L.equilibrium(ps, n, T, U)
    N, Tm = L.moments(ps, f)
    eps = n * eos.energy_per_particle(T, ps.mbar)
    P = n * T
    eta = np.diag([1.0, -1, -1, -1])
    TE = (eps + P)[:, None, None] * U[:, :, None] * U[:, None, :] - P[:, None, None] * eta
    assert np.abs(N - n[:, None] * U).max() < 1e-13 * np.abs(N).max()
    assert np.abs(Tm - TE).max() < 2e-13 * np.abs(TE).max()


@pytest.mark.parametrize("name", ["zeta5", "zeta1"])
def test_uniform_state_is_fixed_point(name):
    ps = stencil(name, "projected")
    m = L.Model(ps, 6, 5, tau=0.8)
    m.init_equilibrium(np.full((5, 6), 1.2), np.full((5, 6), 0.9), np.full((5, 6), 0.25), np.full((5, 6), -0.1))
    f0 = m.f.copy()
    m.step(10)
    assert np.abs(m.f - f0).max() < 5e-14 * np.abs(f0).max()


@pytest.mark.parametrize("name", ["zeta5", "zeta1"])
def test_conservation_periodic(name):
    ps = stencil(name, "projected")
    rng = np.random.default_rng(5)
    nx, ny = 12, 10
    m = L.Model(ps, nx, ny, tau=0.9)
    m.init_equilibrium(*random_fields(rng, ny, nx, 0.3))
    tot = lambda: m.fields()["raw9"].sum(axis=(1, 2))
    t0 = tot()
    m.step(30)
    t1 = tot()
    for k in (0, 3, 4, 5):      # N^0, T^00, T^0x, T^0y
        assert abs(t1[k] - t0[k]) < 1e-13 * abs(t0[3])


@pytest.mark.parametrize("name", ["zeta5", "zeta1", "zeta036"])
def test_projected_equals_full_2d(name):
    """The paper runs 2D problems on 1 x N x M slabs of the 3D stencil
    (Sec. IV); merging populations into in-plane classes is exact."""
    rng = np.random.default_rng(2)
    nx, ny = 9, 7
    fields = random_fields(rng, ny, nx, 0.3)
    out = []
    for mode in ("full", "projected"):
        m = L.Model(stencil(name, mode), nx, ny, tau=0.85)
        m.init_equilibrium(*fields)
        m.step(6)
        out.append(m.fields())
    for k in ("n", "eps", "T", "ux", "uy"):
        assert np.abs(out[0][k] - out[1][k]).max() < 1e-12, k


def test_projected_equals_full_1d_outflow():
    nx = 40
    n = np.where(np.arange(nx) < nx // 2, 1.0, 0.2)[None, :]
    T = np.where(np.arange(nx) < nx // 2, 1.0, 0.6)[None, :]
    out = []
    for mode, dim in (("full", 2), ("projected", 1)):
        m = L.Model(stencil("zeta1", mode, dim), nx, 1, bc=("outflow", "periodic"), tau=1.2)
        m.init_equilibrium(n, T, 0 * n, 0 * n)
        m.step(8)
        out.append(m.fields())
    for k in ("n", "eps", "T", "ux"):
        assert np.abs(out[0][k] - out[1][k]).max() < 1e-12, k
    assert np.abs(out[1]["uy"]).max() == 0.0


def test_1d_equals_2d():
    """A y-uniform 2D run equals the 1D run (Fig. 7: 1D and 2D agree to
    machine precision)."""
    nx, ny = 30, 4
    xs = np.arange(nx)
    n1 = np.where(xs < nx // 2, 1.0, 0.3)
    T1 = np.where(xs < nx // 2, 1.0, 0.7)
    ps = stencil("zeta5", "projected")
    m1 = L.Model(ps, nx, 1, bc=("outflow", "periodic"), tau=1.0)
    m1.init_equilibrium(n1[None], T1[None], 0 * n1[None], 0 * n1[None])
    m2 = L.Model(ps, nx, ny, bc=("outflow", "periodic"), tau=1.0)
    m2.init_equilibrium(np.tile(n1, (ny, 1)), np.tile(T1, (ny, 1)), np.zeros((ny, nx)), np.zeros((ny, nx)))
    m1.step(10)
    m2.step(10)
    a, b = m1.fields(), m2.fields()
    for k in ("n", "T", "ux"):
        assert np.abs(b[k] - a[k]).max() < 1e-14, k


def test_outflow_keeps_uniform_state():
    ps = stencil("zeta1", "projected", 1)
    m = L.Model(ps, 16, 1, bc=("outflow", "outflow"), tau=0.7)
    m.init_equilibrium(np.full((1, 16), 0.8), np.full((1, 16), 1.1), np.full((1, 16), 0.2), np.zeros((1, 16)))
    f0 = m.f.copy()
    m.step(5)
    assert np.abs(m.f - f0).max() < 1e-14 * np.abs(f0).max()
