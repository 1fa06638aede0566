"""Pins of the oracle's third-order model (Sec. III.A: 30 polynomials up to
third order; Sec. III.D: eleven groups; Fig. 2b: the third-order stencil
G1, G2, G3, G4, G5, G8, G9, G10, G12, G13, G15 with 161 populations).

Each pin comes from outside the oracle's own arithmetic:
* the Gram-Schmidt polynomials of degree <= 2 are the printed Appendix A
  polynomials (up to sign);
* all 30 are orthonormal under an independent integration (product Gauss
  rule over the sphere, scipy quadrature in |p|);
* the weights that solve the 465 polynomial-pair conditions equal those of
  the eleven invariant moment conditions (exact integration of p0^j,
  j <= 6, of p0^j p_x^4, j <= 2, and of p_x^2 p_y^2 p_z^2), written here
  from the sphere's moments;
* the projections equal a brute-force integral of the boosted
  Maxwell-Juttner distribution against the polynomials;
* the discrete equilibrium carries the exact third moment (which the
  second-order model does not).
"""
import numpy as np
import pytest
from scipy import integrate, special

from oracle import groups, lattice as L, polynomials, third_order as t3

MBAR, V0 = 7.5, 0.24827584
G3 = [1, 2, 3, 4, 5, 8, 9, 10, 12, 13, 15]


@pytest.fixture(scope="module")
def basis():
    return t3.basis(MBAR)


@pytest.fixture(scope="module")
def stencil():
    return L.build_stencil(groups.bases_of(G3), MBAR, V0, mode="full", order=3)


def sphere_rule(nt, nphi):
    """Product rule over the unit sphere: Gauss-Legendre in cos(theta) and
    the trapezoid rule in phi; exact for polynomials of degree < min(2 nt, nphi)."""
    x, wx = np.polynomial.legendre.leggauss(nt)
    phi = 2 * np.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    nhat = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=-1).reshape(-1, 3)
    w = (wx[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    return nhat, w


def radial_integral(fn, m, T=1.0):
    """int_0^inf fn(|p|, p0) |p|^2/p0 exp(-p0/T) d|p| with p0 = sqrt(m^2 + |p|^2)
    (fn may return an array: adaptive quadrature of the whole vector)."""
    def g(r):
        p0 = np.sqrt(m * m + r * r)
        return np.asarray(fn(r, p0)) * (r * r / p0 * np.exp(-(p0 - m) / T))
    val, err = integrate.quad_vec(g, 0, np.inf, epsabs=0, epsrel=1e-13, limit=400)
    return val * np.exp(-m / T)


def test_counts_and_dropped_monomials(basis):
    """30 polynomials, 14 of degree <= 2 (Sec. III.A); the monomials that
    the mass shell makes dependent are exactly those with a p_z^2 factor
    (after p0^2, p_x^2 and p_y^2 are in) and p_z^3."""
    assert basis.C.shape == (30, 35)
    dropped = [basis.mons[i] for i in range(35) if i not in basis.seeds]
    assert dropped == [(0, 0, 0, 2), (1, 0, 0, 2), (0, 1, 0, 2), (0, 0, 1, 2), (0, 0, 0, 3)]
    assert sum(1 for i in basis.seeds if sum(basis.mons[i]) <= 2) == 14


def test_low_orders_are_the_printed_polynomials(basis):
    """Degree <= 2: each Gram-Schmidt polynomial is one of Appendix A's, up
    to sign, at random on-shell momenta."""
    rng = np.random.default_rng(3)
    pv = rng.normal(size=(40, 3)) * 4
    p = np.concatenate([np.sqrt(MBAR ** 2 + (pv ** 2).sum(1))[:, None], pv], axis=1)
    mine = basis.evaluate(p)[:14]
    printed = np.array(polynomials.evaluate_printed(p, MBAR))
    used = set()
    for k in range(14):
        hits = [j for j in range(14) if np.allclose(np.abs(mine[k]), np.abs(printed[j]), rtol=1e-10, atol=1e-10)
                and (np.allclose(mine[k], printed[j], rtol=1e-10, atol=1e-10)
                     or np.allclose(mine[k], -printed[j], rtol=1e-10, atol=1e-10))]
        assert len(hits) == 1, k
        used.add(hits[0])
    assert used == set(range(14))


def test_orthonormal_by_independent_integration(basis):
    nhat, w = sphere_rule(8, 16)
    NR = 4 * np.pi * MBAR * special.kv(1, MBAR)

    def gram_at(r, p0):
        p = np.concatenate([np.full((len(w), 1), p0), r * nhat], axis=1)
        J = basis.evaluate(p)
        return (J * w[None, :]) @ J.T

    G = radial_integral(gram_at, MBAR) / NR
    assert np.abs(G - np.eye(30)).max() < 1e-9, np.abs(G - np.eye(30)).max()


def invariant_weights(bases, mbar, v0):
    """Weights from the eleven exact-integration conditions written from the
    sphere's moments, <n_x^4> = 1/5 and <n_x^2 n_y^2 n_z^2> = 1/105, with the
    radial integrals in |p| (mpmath, 30 digits): the system is far too
    ill-conditioned for float64."""
    from mpmath import mp, mpf
    with mp.workdps(30):
        m = mpf(mbar)
        NR = 4 * mp.pi * m * mp.besselk(1, m)
        conds = [(j, 0) for j in range(7)] + [(j, 4) for j in range(3)] + [(0, 6)]
        rhs = []
        for j, kind in conds:
            ang = {0: mpf(1), 4: mpf(1) / 5, 6: mpf(1) / 105}[kind]
            rad = mp.quad(lambda r: mp.sqrt(m * m + r * r) ** (j - 1) * r ** (2 + kind)
                          * mp.exp(-mp.sqrt(m * m + r * r)), [0, 1, 10, mp.inf])
            rhs.append(4 * mp.pi * ang * rad / NR)
        A = mp.matrix(11, len(bases))
        v = mpf(v0)
        for g, b in enumerate(bases):
            vecs = groups.fs_orbit(tuple(b))
            n2 = sum(c * c for c in b)
            gam = 1 / mp.sqrt(1 - v * v * n2)
            p0 = m * gam
            for r, (j, kind) in enumerate(conds):
                tot = mpf(0)
                for vec in vecs:
                    p = [m * gam * v * c for c in vec]
                    if kind == 0:
                        tot += p0 ** j
                    elif kind == 4:
                        tot += p0 ** j * p[0] ** 4
                    else:
                        tot += (p[0] * p[1] * p[2]) ** 2
                A[r, g] = tot
        w = mp.lu_solve(A, mp.matrix(rhs))
        return np.array([float(w[i]) for i in range(len(bases))])


def test_quadrature_equals_invariant_conditions():
    """The paper's third-order stencil at mbar = 7.5: the 465 pair
    conditions are consistent, their weights are all positive and equal the
    weights of the eleven invariant conditions."""
    bases = groups.bases_of(G3)
    w, res = t3.weights(bases, MBAR, V0, dps=40)
    w = np.array([float(x) for x in w])
    assert float(res) < 1e-30
    assert (w > 0).all()
    wi = invariant_weights(bases, MBAR, V0)
    assert np.abs(w - wi).max() < 1e-14 * np.abs(w).max(), (w, wi)
    assert sum(len(groups.fs_orbit(tuple(b))) for b in bases) == 161


def test_second_order_stencil_fails_third_order():
    """G1..G6 (57 populations) cannot satisfy the third-order conditions:
    the least-squares residual stays large."""
    _, res = t3.weights(groups.bases_of([1, 2, 3, 4, 5, 6]), 5.0, 0.398, dps=30)
    assert float(res) > 1e-3


def boost(U):
    g = U[0]
    u = U[1:] / g
    L4 = np.eye(4)
    L4[0, 0] = g
    L4[0, 1:] = L4[1:, 0] = g * u
    u2 = u @ u
    if u2 > 0:
        L4[1:, 1:] += (g - 1) * np.outer(u, u) / u2
    return L4


@pytest.mark.parametrize("u,T", [((0.3, -0.2, 0.1), 0.9), ((0.0, 0.5, 0.0), 1.2), ((0.1, 0.1, -0.45), 0.7)])
def test_projections_by_brute_force(basis, u, T):
    """a^(k) = int f^eq J^(k) d^3p/p^0 (unit density) by integration in the
    fluid's rest frame: f^eq = exp(-p'^0/T)/N, N = 4 pi m^2 T K_2(m/T), and
    p = Lambda(U) p' (the measure is invariant)."""
    u = np.array(u)
    g = 1 / np.sqrt(1 - u @ u)
    U = np.concatenate([[g], g * u])
    Lb = boost(U)
    nhat, w = sphere_rule(4, 8)
    Nn = 4 * np.pi * MBAR ** 2 * T * special.kv(2, MBAR / T)

    def ang(r, p0):
        pp = np.concatenate([np.full((len(w), 1), p0), r * nhat], axis=1)
        return basis.evaluate(pp @ Lb.T) @ w

    brute = radial_integral(ang, MBAR, T) / Nn
    mine = t3.projections(U[None, :], np.array([T]), MBAR)[:, 0]
    assert np.abs(mine - brute).max() < 1e-9 * max(1.0, np.abs(brute).max()), np.abs(mine - brute).max()


def test_rest_frame_at_reference_temperature(basis):
    """At U = (1, 0, 0, 0), T = T_R the equilibrium is the weight function
    times K_1/(mbar K_2): only the constant polynomial projects."""
    a = t3.projections(np.array([[1.0, 0, 0, 0]]), np.array([1.0]), MBAR)[:, 0]
    assert abs(a[0] - special.kv(1, MBAR) / (MBAR * special.kv(2, MBAR))) < 1e-14
    assert np.abs(a[1:]).max() < 1e-13


def test_equilibrium_carries_the_third_moment(stencil):
    """Sum_i f_i^eq p^mu p^nu p^la equals the Maxwell-Juttner third moment
    at third order; N and T are exact as at second order."""
    rng = np.random.default_rng(7)
    S = 12
    u = rng.normal(size=(S, 3))
    u *= (rng.uniform(0, 0.45, S) / np.linalg.norm(u, axis=1))[:, None]
    g = 1 / np.sqrt(1 - (u * u).sum(1))
    U = np.concatenate([g[:, None], g[:, None] * u], axis=1)
    T = rng.uniform(0.8, 1.25, S)
    n = rng.uniform(0.5, 1.5, S)
    f = L.equilibrium(stencil, n, T, U)
    p = stencil.p
    _, m1, m2, m3 = t3.mj_tensors(U, T, MBAR)
    N = np.einsum("qs,qa->sa", f, p)
    T2 = np.einsum("qs,qa,qb->sab", f, p, p)
    T3 = np.einsum("qs,qa,qb,qc->sabc", f, p, p, p)
    assert np.abs(N - n[:, None] * m1).max() < 1e-13 * np.abs(N).max()
    assert np.abs(T2 - n[:, None, None] * m2).max() < 1e-13 * np.abs(T2).max()
    assert np.abs(T3 - n[:, None, None, None] * m3).max() < 1e-13 * np.abs(T3).max()
    ps2 = L.build_stencil(groups.bases_of([1, 2, 3, 4, 5, 6]), MBAR, 0.38, mode="full")
    f2 = L.equilibrium(ps2, n, T, U)
    T3b = np.einsum("qs,qa,qb,qc->sabc", f2, ps2.p, ps2.p, ps2.p)
    assert np.abs(T3b - n[:, None, None, None] * m3).max() > 1e-4 * np.abs(T3b).max()


def test_rank3_tensor_trace_and_rest_component():
    """The rank-3 Maxwell-Juttner moment: its trace over one index pair is
    mbar^2 U (mass shell) and its rest-frame 000 component is <p0^2>,
    computed here by a radial integral."""
    T = 0.8
    U = np.array([[1.0, 0, 0, 0]])
    _, _, _, m3 = t3.mj_tensors(U, np.array([T]), MBAR)
    eta = np.diag([1.0, -1, -1, -1])
    tr = np.einsum("ab,sabc->sc", eta, m3)
    assert np.abs(tr[0] - MBAR ** 2 * U[0]).max() < 1e-12 * MBAR ** 2
    Nn = 4 * np.pi * MBAR ** 2 * T * special.kv(2, MBAR / T)
    p0sq = 4 * np.pi * radial_integral(lambda r, p0: p0 ** 3, MBAR, T) / Nn
    assert abs(m3[0, 0, 0, 0] - p0sq) < 1e-11 * p0sq


def test_lattice_third_order_runs(stencil):
    """Third-order lattices: a z-uniform 3D run equals the 2D run of merged
    classes; N^0 and T^{0 nu} are conserved; a uniform state is a fixed
    point."""
    bases = groups.bases_of(G3)
    w = stencil.group_weights
    ps2 = L.build_stencil(bases, MBAR, V0, mode="projected", dim=2, weights=w, order=3)
    rng = np.random.default_rng(2)
    nx, ny, nz = 7, 5, 2
    x, y = np.meshgrid(np.arange(nx) / nx, np.arange(ny) / ny)
    n = 1 + 0.1 * np.cos(2 * np.pi * x + rng.uniform(0, 6))
    T = 1 + 0.05 * np.sin(2 * np.pi * y)
    ux = 0.2 * np.sin(2 * np.pi * y)
    uy = 0.1 * np.cos(2 * np.pi * x)
    m2 = L.Model(ps2, nx, ny, tau=0.9)
    m2.init_equilibrium(n, T, ux, uy)
    m3 = L.Model3D(stencil, nx, ny, nz, tau=0.9)
    rep = lambda a: np.repeat(a[None], nz, axis=0)
    m3.init_equilibrium(rep(n), rep(T), rep(ux), rep(uy), np.zeros((nz, ny, nx)))
    t0 = m3.fields()["raw14"].sum(axis=(1, 2, 3))
    m2.step(3)
    m3.step(3)
    a, b = m2.fields(), m3.fields()
    for k in ("n", "eps", "T", "ux", "uy"):
        assert np.abs(b[k][1] - a[k]).max() < 1e-12 * max(1.0, np.abs(a[k]).max()), k
    t1 = b["raw14"].sum(axis=(1, 2, 3))
    for k in (0, 4, 5, 6, 7):
        assert abs(t1[k] - t0[k]) < 1e-12 * abs(t0[4]), k
    u = np.ones((ny, nx))
    m2.init_equilibrium(1.1 * u, 0.95 * u, 0.15 * u, -0.2 * u)
    f0 = m2.f.copy()
    m2.step(3)
    assert np.abs(m2.f - f0).max() < 1e-12 * np.abs(f0).max()
