"""Pins of the oracle's 3D lattice model (Sec. V: the method runs on
Nx x Ny x Nz lattices with every population of the 3D stencil).

* the discrete equilibrium recovers the Maxwell-Juttner moments N = nU and
  T = (eps + P) UU - P eta (eqs. quadri-flux, energy-tensor) for a
  four-velocity with all three spatial components;
* a z-uniform 3D run equals the 2D run of the same stencil (the paper's 2D
  lattices are 1-thick 3D slabs);
* the full-symmetric stencil maps onto itself under y <-> z, so a flow in
  the x-z plane is the x-y flow with the axes swapped;
* N^0 and T^{0 nu} are conserved on periodic boxes, a uniform state is a
  fixed point, and the z-centroid of N^0 moves by the post-collision
  z-flux (populations stream along their velocity in z too).
"""
import numpy as np
import pytest

from oracle import groups, lattice as L, eos

STENCILS = {"zeta5": ([1, 2, 3, 4, 5, 6], 5.0, 0.398), "zeta1": ([1, 5, 11, 13, 17, 21], 1.0, 0.2403918860)}
_cache = {}


def stencil(name):
    if name not in _cache:
        gs, m, v0 = STENCILS[name]
        _cache[name] = L.build_stencil(groups.bases_of(gs), m, v0, mode="full")
    return _cache[name]


def smooth3(rng, nz, ny, nx, umax=0.25, vary=(True, True, True)):
    """Random smooth periodic fields on a 3D box (a few Fourier modes)."""
    z, y, x = np.meshgrid(np.arange(nz) / nz, np.arange(ny) / ny, np.arange(nx) / nx, indexing="ij")

    def field(amp):
        f = np.zeros((nz, ny, nx))
        for _ in range(3):
            k = rng.integers(0, 3, 3) * np.array(vary)
            f += amp * rng.uniform(-1, 1) * np.cos(2 * np.pi * (k[0] * x + k[1] * y + k[2] * z) + rng.uniform(0, 6.3))
        return f

    return 1.0 + field(0.1), 1.0 + field(0.1), field(umax / 3), field(umax / 3), field(umax / 3)


@pytest.mark.parametrize("name", list(STENCILS))
def test_equilibrium_moments_exact_3d_velocity(name):
    ps = stencil(name)
    rng = np.random.default_rng(4)
    S = 30
    n, T = rng.uniform(0.5, 1.5, S), rng.uniform(0.7, 1.3, S)
    u = rng.normal(size=(S, 3))
    u *= (rng.uniform(0, 0.4, S) / np.linalg.norm(u, axis=1))[:, None]
    g = 1 / np.sqrt(1 - (u * u).sum(axis=1))
    U = np.concatenate([g[:, None], g[:, None] * u], axis=1)
    f = L.equilibrium(ps, n, T, U)
    N, Tm = L.moments(ps, f)
    epsv = n * eos.energy_per_particle(T, ps.mbar)
    P = n * T
    eta = np.diag([1.0, -1, -1, -1])
    TE = (epsv + P)[:, None, None] * U[:, :, None] * U[:, None, :] - P[:, None, None] * eta
    assert np.abs(N - n[:, None] * U).max() < 1e-13 * np.abs(N).max()
    assert np.abs(Tm - TE).max() < 2e-13 * np.abs(TE).max()


def test_z_uniform_run_equals_2d():
    ps = stencil("zeta5")
    rng = np.random.default_rng(6)
    nx, ny, nz = 9, 7, 3
    n, T, ux, uy, _ = smooth3(rng, 1, ny, nx, vary=(True, True, False))
    m2 = L.Model(ps, nx, ny, tau=0.85)
    m2.init_equilibrium(n[0], T[0], ux[0], uy[0])
    m3 = L.Model3D(ps, nx, ny, nz, tau=0.85)
    rep = lambda a: np.repeat(a, nz, axis=0)
    m3.init_equilibrium(rep(n), rep(T), rep(ux), rep(uy), np.zeros((nz, ny, nx)))
    m2.step(5)
    m3.step(5)
    a, b = m2.fields(), m3.fields()
    for k in ("n", "eps", "T", "ux", "uy"):
        for z in range(nz):
            assert np.abs(b[k][z] - a[k]).max() < 1e-13 * max(1.0, np.abs(a[k]).max()), k
    assert np.abs(b["uz"]).max() < 1e-15


@pytest.mark.parametrize("bc", ["periodic", "outflow"])
def test_yz_swap_symmetry(bc):
    """Fields on an (x, z) box with velocity (ux, 0, uz) evolve as the same
    fields on the (x, y) box with velocity (ux, uz, 0), axes swapped."""
    ps = stencil("zeta5")
    rng = np.random.default_rng(8)
    nx, nyz = 8, 6
    n, T, ux, uy, _ = smooth3(rng, 1, nyz, nx, vary=(True, True, False))
    # A: varies in (x, y), thin in z; B: varies in (x, z), thin in y
    mA = L.Model3D(ps, nx, nyz, 2, bc=("periodic", bc, "periodic"), tau=0.9)
    mA.init_equilibrium(*(np.repeat(a, 2, axis=0) for a in (n, T, ux, uy)), np.zeros((2, nyz, nx)))
    swap = lambda a: np.repeat(a[0][:, None, :], 2, axis=1)   # [nz = nyz, ny = 2, nx]
    mB = L.Model3D(ps, nx, 2, nyz, bc=("periodic", "periodic", bc), tau=0.9)
    mB.init_equilibrium(swap(n), swap(T), swap(ux), np.zeros((nyz, 2, nx)), swap(uy))
    mA.step(4)
    mB.step(4)
    a, b = mA.fields(), mB.fields()
    for ka, kb in (("n", "n"), ("eps", "eps"), ("T", "T"), ("ux", "ux"), ("uy", "uz")):
        assert np.abs(a[ka][0] - b[kb][:, 0, :]).max() < 1e-12 * max(1.0, np.abs(a[ka]).max()), ka
    assert np.abs(b["uy"]).max() < 1e-14


def test_conservation_and_fixed_point_3d():
    ps = stencil("zeta5")
    rng = np.random.default_rng(9)
    nx, ny, nz = 6, 5, 4
    m = L.Model3D(ps, nx, ny, nz, tau=0.9)
    m.init_equilibrium(*smooth3(rng, nz, ny, nx))
    tot = lambda: m.fields()["raw14"].sum(axis=(1, 2, 3))
    t0 = tot()
    m.step(12)
    t1 = tot()
    for k in (0, 4, 5, 6, 7):      # N^0, T^00, T^0x, T^0y, T^0z
        assert abs(t1[k] - t0[k]) < 1e-13 * abs(t0[4]), k
    u = np.full((nz, ny, nx), 1.0)
    m.init_equilibrium(1.2 * u, 0.9 * u, 0.2 * u, -0.1 * u, 0.15 * u)
    f0 = m.f.copy()
    m.step(5)
    assert np.abs(m.f - f0).max() < 5e-14 * np.abs(f0).max()


def test_z_centroid_moves_with_the_z_flux():
    ps = stencil("zeta5")
    nx, ny, nz = 6, 6, 24
    z = np.arange(nz) - nz / 2 + 0.5
    g = np.where(np.abs(z) < 6, np.cos(np.pi * z / 12) ** 2, 0.0)[:, None, None] * np.ones((nz, ny, nx))
    m = L.Model3D(ps, nx, ny, nz, tau=0.9)
    m.init_equilibrium(1 + 0.4 * g, 1 + 0.2 * g, 0.0 * g, 0.0 * g, 0.3 * g)
    N0 = lambda f: np.einsum("qzyx,q->zyx", f, ps.p[:, 0])
    before = N0(m.f)
    fpost = m.collide()
    flux = np.einsum("qzyx,q->", fpost, ps.p[:, 3]) / ps.v0
    m.f = m.stream(fpost)
    after = N0(m.f)
    zs = np.arange(nz)[:, None, None]
    shift = (zs * (after - before)).sum()
    assert flux > 1.0
    assert abs(shift - flux) < 1e-11 * flux
