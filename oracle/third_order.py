"""Third-order model (Sec. III.A, III.D): the 30 orthonormal polynomials of
degree <= 3, the quadrature conditions they impose on a stencil of eleven
velocity groups, the projections of the Maxwell-Juttner distribution on
them and the equilibrium they define (eq. mj-projected-distribution at
N = 3).

Test infrastructure (the oracle); nothing here is used by the GPU library.

The paper lists the third-order polynomials and projections only in its
supplemental material, which is not at hand, so they are rebuilt from their
definition:

* Polynomials (Sec. III.A, eq. ortho1).  The monomials of degree <= 3 in the
  adimensional momenta pbar^mu, taken by increasing degree and, within a
  degree, in decreasing order of the exponent tuple (a0, ax, ay, az), are
  orthonormalised by Gram-Schmidt with the inner product
      <f, g> = int omega(p0) f g d^3p/p^0,  omega = exp(-p0)/N_R,
      N_R = 4 pi mbar K_1(mbar)   (T_R = 1).
  On the mass shell p0^2 = mbar^2 + |p|^2 five of the 35 monomials depend on
  earlier ones; Gram-Schmidt drops them and keeps 30 polynomials (14 up to
  second order, matching the paper's counts).  The inner products of
  monomials are exact: an angular factor (moments of the unit sphere) times
  a one-dimensional radial integral in p0, evaluated with mpmath.
* Quadrature (Sec. III.D, eq. ortho2).  One weight per group; the
  conditions sum_i w_i J^(l)(p_i) J^(k)(p_i) = delta_lk for every pair of the
  30 polynomials form the linear system A(v0) w = b, solved in the
  least-squares sense (its residual certifies consistency), as at second
  order.
* Projections (eq. mj-projection-coefficients): a^(k) = int f^eq J^(k)
  d^3p/p^0 with f^eq of unit density (N_E = U).  J^(k) is a combination of
  monomials, so a^(k) combines the moment tensors of f^eq up to rank 3:
      rank 0:  K_1(z)/(mbar K_2(z))                      z = mbar/T
      rank 1:  U^mu
      rank 2:  mbar K_3(z)/K_2(z) U^mu U^nu - T eta^{mu nu}
      rank 3:  A3 U^mu U^nu U^la + B3 (eta^{mu nu} U^la + eta^{mu la} U^nu
               + eta^{nu la} U^mu)
  The rank-3 tensor is the only symmetric tensor built from U and eta; its
  two scalars follow from the mass shell (the trace over one index pair is
  mbar^2 U^la, so A3 + 6 B3 = mbar^2) and from its rest-frame 000 component
  <p0^2> = mbar^2 (1 + 3 K_3(z)/(z K_2(z))) (so A3 + 3 B3 = <p0^2>).
"""
import numpy as np
from mpmath import mp, mpf

from . import quadrature as quad
from .special import k_ratio_np

NPOLY3 = 30


def monomials():
    """Exponent tuples (a0, ax, ay, az) of degree <= 3 in Gram-Schmidt order."""
    out = []
    for deg in range(4):
        tup = [(a0, ax, ay, deg - a0 - ax - ay)
               for a0 in range(deg + 1) for ax in range(deg + 1 - a0) for ay in range(deg + 1 - a0 - ax)]
        out.extend(sorted(tup, reverse=True))
    return out


def _sphere_moment(ax, ay, az):
    """int over the unit sphere of nx^ax ny^ay nz^az dOmega."""
    if ax % 2 or ay % 2 or az % 2:
        return mpf(0)
    g = mp.gamma
    return 2 * g(mpf(ax + 1) / 2) * g(mpf(ay + 1) / 2) * g(mpf(az + 1) / 2) / g(mpf(ax + ay + az + 3) / 2)


def omega_moment(e, mbar):
    """int omega(p0) p0^a0 px^ax py^ay pz^az d^3p/p^0 (T_R = 1, exact up to
    the radial quadrature).  With d^3p/p^0 = |p| dp0 dOmega:
    (1/N_R) * sphere moment * int_mbar^inf |p|^(1+s) p0^a0 exp(-p0) dp0."""
    a0, ax, ay, az = e
    ang = _sphere_moment(ax, ay, az)
    if ang == 0:
        return mpf(0)
    m = mpf(mbar)
    s = ax + ay + az
    rad = mp.quad(lambda p0: (p0 * p0 - m * m) ** (mpf(1 + s) / 2) * p0 ** a0 * mp.exp(-p0), [m, m + 1, mp.inf])
    NR = 4 * mp.pi * m * mp.besselk(1, m)
    return ang * rad / NR


def gram_schmidt(mbar, dps=50):
    """Coefficients C [30, 35] (mpf) of the orthonormal polynomials over
    ``monomials()``, and the indices of the monomials that started each of
    them."""
    with mp.workdps(dps):
        mons = monomials()
        nm = len(mons)
        cache = {}

        def ip(i, j):
            e = tuple(a + b for a, b in zip(mons[i], mons[j]))
            if e not in cache:
                cache[e] = omega_moment(e, mbar)
            return cache[e]

        G = mp.matrix(nm, nm)
        for i in range(nm):
            for j in range(i, nm):
                G[i, j] = G[j, i] = ip(i, j)
        Gv = lambda c: [mp.fsum(G[a, b] * c[b] for b in range(nm) if c[b] != 0) for a in range(nm)]
        polys, gpolys, seeds = [], [], []
        for i in range(nm):
            c = [mpf(0)] * nm
            c[i] = mpf(1)
            for _ in range(2):   # modified Gram-Schmidt, repeated once for stability
                for q, gq in zip(polys, gpolys):
                    proj = mp.fsum(c[a] * gq[a] for a in range(nm) if c[a] != 0)
                    c = [c[a] - proj * q[a] for a in range(nm)]
            gc = Gv(c)
            nrm2 = mp.fsum(c[a] * gc[a] for a in range(nm))
            if nrm2 <= G[i, i] * mpf(10) ** (-(dps - 15)):
                continue         # dependent on earlier monomials on the mass shell
            r = mp.sqrt(nrm2)
            polys.append([x / r for x in c])
            gpolys.append([x / r for x in gc])
            seeds.append(i)
        assert len(polys) == NPOLY3, len(polys)
        return polys, seeds


class Basis3:
    """The 30 polynomials at one mbar: float64 coefficient matrix C [30, 35]
    plus an mpf copy for the quadrature solve."""

    def __init__(self, mbar, dps=50):
        self.mbar = float(mbar)
        self.mons = monomials()
        self.C_mp, self.seeds = gram_schmidt(mbar, dps)
        self.C = np.array([[float(x) for x in row] for row in self.C_mp])

    def monomial_values(self, p):
        """[35, ...] values of the monomials at momenta p [..., 4]."""
        return np.array([p[..., 0] ** a0 * p[..., 1] ** ax * p[..., 2] ** ay * p[..., 3] ** az
                         for (a0, ax, ay, az) in self.mons])

    def evaluate(self, p):
        """[30, ...] polynomial values at float64 momenta p [..., 4]."""
        p = np.asarray(p, dtype=np.float64)
        V = self.monomial_values(p)
        return np.tensordot(self.C, V, axes=(1, 0))

    def evaluate_mp(self, p):
        """Polynomial values at one mpf momentum p (length-4 sequence)."""
        v = [p[0] ** a0 * p[1] ** ax * p[2] ** ay * p[3] ** az for (a0, ax, ay, az) in self.mons]
        return [mp.fsum(c * x for c, x in zip(row, v)) for row in self.C_mp]


_basis_cache = {}


def basis(mbar):
    key = float(mbar)
    if key not in _basis_cache:
        _basis_cache[key] = Basis3(mbar)
    return _basis_cache[key]


def system(bases, mbar, v0, dps=50):
    """A(v0) (rows: pairs l <= k of the 30 polynomials, columns: groups) and b."""
    B = basis(mbar)
    with mp.workdps(dps):
        pops = quad.abscissae(bases, mbar, v0, dps)
        Jg = [[B.evaluate_mp(p[i]) for i in range(len(vecs))] for (vecs, p) in pops]
        rows, rhs = [], []
        for l in range(NPOLY3):
            for k in range(l, NPOLY3):
                rows.append([mp.fsum(J[l] * J[k] for J in Jg[g]) for g in range(len(bases))])
                rhs.append(mpf(1) if l == k else mpf(0))
        return mp.matrix(rows), mp.matrix(rhs)


def weights(bases, mbar, v0, dps=50):
    """Least-squares weights (mpf list) and the residual max |A w - b|."""
    with mp.workdps(dps):
        A, b = system(bases, mbar, v0, dps)
        At = A.T
        w = mp.lu_solve(At * A, At * b)
        r = A * w - b
        return [w[i] for i in range(len(bases))], max(abs(r[i]) for i in range(r.rows))


def min_weight(bases, mbar, v0, dps=40):
    try:
        w, _ = weights(bases, mbar, v0, dps)
    except ZeroDivisionError:
        return mpf("-inf")
    return min(w)


# ------------------------------------------------------------ projections

ETA = np.diag([1.0, -1.0, -1.0, -1.0])


def mj_tensors(U, T, mbar):
    """Moment tensors of rank 0..3 of the unit-density Maxwell-Juttner
    distribution: (m0 [...], m1 [..., 4], m2 [..., 4, 4], m3 [..., 4, 4, 4])."""
    U = np.asarray(U, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    z = mbar / T
    m0 = k_ratio_np(1, 2, z) / mbar
    m2 = (mbar * k_ratio_np(3, 2, z))[..., None, None] * U[..., :, None] * U[..., None, :] \
        - T[..., None, None] * ETA
    p0sq = mbar * mbar * (1.0 + 3.0 * k_ratio_np(3, 2, z) / z)
    B3 = (mbar * mbar - p0sq) / 3.0
    A3 = p0sq - 3.0 * B3
    UUU = U[..., :, None, None] * U[..., None, :, None] * U[..., None, None, :]
    EU = (ETA[:, :, None] * U[..., None, None, :] + ETA[:, None, :] * U[..., None, :, None]
          + ETA[None, :, :] * U[..., :, None, None])
    m3 = A3[..., None, None, None] * UUU + B3[..., None, None, None] * EU
    return m0, U, m2, m3


def monomial_moments(mons, U, T, mbar):
    """[35, ...] moments int f^eq (monomial) d^3p/p^0 of the unit-density
    Maxwell-Juttner distribution: the tensor component whose indices list
    the monomial's factors."""
    m0, m1, m2, m3 = mj_tensors(U, T, mbar)
    out = []
    for e in mons:
        idx = [0] * e[0] + [1] * e[1] + [2] * e[2] + [3] * e[3]
        if len(idx) == 0:
            out.append(m0)
        elif len(idx) == 1:
            out.append(m1[..., idx[0]])
        elif len(idx) == 2:
            out.append(m2[..., idx[0], idx[1]])
        else:
            out.append(m3[..., idx[0], idx[1], idx[2]])
    return np.array(out)


def projections(U, T, mbar):
    """a^(k)(U, T), k < 30, for the unit-density equilibrium: [30, ...]."""
    B = basis(mbar)
    M = monomial_moments(B.mons, U, T, mbar)
    return np.tensordot(B.C, M, axes=(1, 0))
