"""The discrete relativistic lattice Boltzmann model (Sec. II.A, Sec. III).

One time step (eq. discrete-relativistic-boltzmann), collide then stream:

    f_i(x + n_i, t + 1) = f_i(x, t) - (p_i^mu U_mu)/(p_i^0 tau) (f_i - f_i^eq)

with lattice units T_R = 1, dx = 1, dt = dx/v0 = 1 lattice step (eq. v0dt=dx).
Per site and step:
  1. N^alpha = sum_i f_i p_i^alpha, T^{alpha beta} = sum_i f_i p_i^alpha p_i^beta
     (eq. mj-discrete-second-moment);
  2. Landau frame eps, U from the eigenproblem, n = U_alpha N^alpha
     (eqs. landau-lifshitz-*);
  3. T from the equation of state (eq. relativistic-eos);
  4. f_i^eq = n w_i sum_k a^(k)(U, T) J^(k)(p_i) (eq. mj-discrete-feq), with f^eq
     normalised to N_E = n U (eq. maxwell-juttner-normalization);
  5. Anderson-Witting relaxation and exact streaming by the integer vector n_i.

Lattices are 2D (Nx x Ny) or 1D (Nx x 1), obtained as in the paper as
1-thick slabs of a 3D lattice (1 x N x M, 1 x 1 x N): the z axis has one
periodic cell, so z displacements do not move populations.

Two population sets are supported:
  * ``full``: every population of the 3D stencil (the paper's setup);
  * ``projected``: populations merged into classes of equal group and equal
    in-plane displacement (and, in 1D, equal x displacement).  Members of a
    class share p^0, the in-plane momentum and the relaxation frequency
    (U_z = 0, and U_y = 0 in 1D), so the class sums evolve in closed form.
    The tests check this mode against ``full``.
"""
import numpy as np

from .groups import fs_orbit
from .polynomials import coefficients, evaluate_printed
from . import quadrature as quad
from .projections import projections
from .eos import temperature
from .landau import landau_frame
from . import third_order

HBARC_GEV_FM = 0.1973269804


class PopulationSet:
    """disp [Q, 2] in-plane displacement, p [Q, d] momenta (d = 4 full,
    3 for 2D classes (p0, px, py), 2 for 1D classes (p0, px)), M [Q, 14]
    = sum over members of w_i J^(k)(p_i) (M [Q, 30] at third order);
    disp3 [Q, 3] the full 3D displacement (full stencils only)."""

    def __init__(self, disp, p, M, mbar, v0, coeffs, weights, group_index, disp3=None, order=2):
        self.order = int(order)
        self.disp3 = None if disp3 is None else np.asarray(disp3, dtype=np.int64)
        self.disp = np.asarray(disp, dtype=np.int64)
        self.p = np.asarray(p, dtype=np.float64)
        self.M = np.asarray(M, dtype=np.float64)
        self.mbar = float(mbar)
        self.v0 = float(v0)
        self.coeffs = coeffs
        self.group_weights = weights
        self.group_index = np.asarray(group_index, dtype=np.int64)

    @property
    def Q(self):
        return self.p.shape[0]

    @property
    def d(self):
        return self.p.shape[1]


def build_stencil(bases, mbar, v0, mode="full", dim=2, weights=None, dps=50, order=2):
    """Populations of a stencil.  ``weights``: per-group weights (floats);
    solved from the orthonormality conditions of the given order (2: the 14
    polynomials of Appendix A; 3: the 30 polynomials of ``third_order``)
    when None."""
    if order not in (2, 3):
        raise ValueError("order must be 2 or 3")
    if weights is None:
        w, _ = (quad.weights if order == 2 else third_order.weights)(bases, mbar, v0, dps)
        weights = [float(x) for x in w]
    pops = quad.abscissae(bases, mbar, v0, dps)
    vec, mom, wt, gid = [], [], [], []
    for g, (vecs, p) in enumerate(pops):
        for i in range(len(vecs)):
            vec.append(vecs[i])
            mom.append([float(x) for x in p[i]])
            wt.append(weights[g])
            gid.append(g)
    vec = np.array(vec, dtype=np.int64)
    mom = np.array(mom, dtype=np.float64)
    wt = np.array(wt, dtype=np.float64)
    gid = np.array(gid, dtype=np.int64)
    coeffs = coefficients(mbar)
    if order == 2:
        J = np.array(evaluate_printed(mom, mbar))        # [14, Q3]
    else:
        J = third_order.basis(mbar).evaluate(mom)        # [30, Q3]
    Mfull = (wt[None, :] * J).T                          # [Q3, 14 or 30]
    if mode == "full":
        return PopulationSet(vec[:, :2], mom, Mfull, mbar, v0, coeffs, weights, gid, disp3=vec, order=order)
    keyc = 2 if dim == 2 else 1
    keys = {}
    for i in range(len(vec)):
        key = (int(gid[i]),) + tuple(int(c) for c in vec[i, :keyc])
        keys.setdefault(key, []).append(i)
    disp, p, M, gi = [], [], [], []
    for key, members in keys.items():
        i0 = members[0]
        d = [int(vec[i0, 0]), int(vec[i0, 1]) if dim == 2 else 0]
        disp.append(d)
        p.append(mom[i0, :1 + keyc])
        M.append(Mfull[members].sum(axis=0))
        gi.append(key[0])
    return PopulationSet(disp, p, M, mbar, v0, coeffs, weights, gi, order=order)


# ---------------------------------------------------------------- per site

def moments(ps, f):
    """N [S, d] and T [S, d, d] of populations f [Q, S]."""
    N = np.einsum("qs,qa->sa", f, ps.p)
    T = np.einsum("qs,qa,qb->sab", f, ps.p, ps.p)
    return N, T


def macroscopic(ps, f):
    """Landau-frame fields of populations f [Q, S]: dict of n, eps, T, P, U
    (contravariant, d components), plus the raw moments."""
    N, Tm = moments(ps, f)
    eps, U, n = landau_frame(Tm, N)
    T = temperature(eps / n, ps.mbar)
    return {"n": n, "eps": eps, "T": T, "P": n * T, "U": U, "N": N, "Tmn": Tm}


def four_velocity(ux, uy):
    ux = np.asarray(ux, dtype=np.float64)
    uy = np.asarray(uy, dtype=np.float64)
    g = 1.0 / np.sqrt(1.0 - ux * ux - uy * uy)
    return np.stack([g, g * ux, g * uy, 0.0 * g], axis=-1)


def equilibrium(ps, n, T, U4):
    """f_i^eq = n sum_k b^(k)(U, T) M_{ik}; U4: [S, 4] contravariant."""
    if ps.order == 3:
        b = third_order.projections(U4, T, ps.mbar)     # [30, S]
    else:
        b = projections(U4, T, ps.mbar, ps.coeffs)      # [14, S]
    return np.asarray(n)[None, :] * (ps.M @ b)


def pad4(U):
    out = np.zeros(U.shape[:-1] + (4,))
    out[..., :U.shape[-1]] = U
    return out


def tau_from_eta_over_s(n, T, eta_s, v0, units):
    """Relaxation time in lattice units from eta/s (Sec. IV):
    eta = (2/3) P (tau_f - dt/2) and tau = tau_f v0/dx, with the entropy density
    s = 4 n - n ln(n / n_eq), n_eq = d_G T^3/pi^2, d_G = 16, in physical units
    (GeV, fm; hbar c converts).  ``units``: dict with T_R_GeV, n_unit_fm3, dx_fm."""
    n_phys = n * units["n_unit_fm3"]
    T_phys = T * units["T_R_GeV"]
    P_phys = n_phys * T_phys
    n_eq = 16.0 * T_phys**3 / (np.pi**2 * HBARC_GEV_FM**3)
    s = 4.0 * n_phys - n_phys * np.log(n_phys / n_eq)
    return 0.5 + 1.5 * eta_s * s * HBARC_GEV_FM * v0 / (P_phys * units["dx_fm"])


class Model:
    """A lattice of Nx x Ny sites with populations f [Q, Ny, Nx] (float64).

    bc: (bc_x, bc_y), each 'periodic' or 'outflow' (a population pulled from
    outside the domain takes the post-collision value of the nearest in-domain
    site).  tau: float (constant relaxation time) or dict(eta_s=..., units=...)."""

    def __init__(self, ps, nx, ny, bc=("periodic", "periodic"), tau=1.0):
        self.ps, self.nx, self.ny, self.bc, self.tau = ps, nx, ny, bc, tau
        self.f = None
        self.t = 0

    def init_equilibrium(self, n, T, ux, uy):
        S = self.nx * self.ny
        n = np.asarray(n, dtype=np.float64).reshape(S)
        T = np.asarray(T, dtype=np.float64).reshape(S)
        U4 = four_velocity(np.reshape(ux, S), np.reshape(uy, S))
        self.f = equilibrium(self.ps, n, T, U4).reshape(self.ps.Q, self.ny, self.nx)
        self.t = 0

    def fields(self, f=None):
        f = self.f if f is None else f
        mac = macroscopic(self.ps, f.reshape(self.ps.Q, -1))
        U = mac["U"]
        out = {k: mac[k].reshape(self.ny, self.nx) for k in ("n", "eps", "T", "P")}
        out["ux"] = (U[:, 1] / U[:, 0]).reshape(self.ny, self.nx)
        out["uy"] = ((U[:, 2] / U[:, 0]) if U.shape[1] > 2 else 0 * U[:, 0]).reshape(self.ny, self.nx)
        N, Tm = mac["N"], mac["Tmn"]
        d = N.shape[1]
        comp = lambda a, b: Tm[:, a, b] if max(a, b) < d else 0 * Tm[:, 0, 0]
        vec = lambda a: N[:, a] if a < d else 0 * N[:, 0]
        raw = [vec(0), vec(1), vec(2), comp(0, 0), comp(0, 1), comp(0, 2),
               comp(1, 1), comp(1, 2), comp(2, 2)]
        out["raw9"] = np.array(raw).reshape(9, self.ny, self.nx)
        out["_mac"] = mac
        return out

    def collide(self):
        return self._collide_flat().reshape(self.ps.Q, self.ny, self.nx)

    def _collide_flat(self):
        """Post-collision populations [Q, sites] (Anderson-Witting relaxation
        toward f^eq of the local Landau frame)."""
        ps = self.ps
        f = self.f.reshape(ps.Q, -1)
        mac = macroscopic(ps, f)
        U4 = pad4(mac["U"])
        feq = equilibrium(ps, mac["n"], mac["T"], U4)
        if isinstance(self.tau, dict):
            tau = tau_from_eta_over_s(mac["n"], mac["T"], self.tau["eta_s"], ps.v0, self.tau["units"])
        else:
            tau = np.full(f.shape[1], float(self.tau))
        eta = np.diag([1.0] + [-1.0] * (ps.d - 1))
        pU = ps.p @ eta @ mac["U"].T                      # [Q, S] p_i^mu U_mu
        omega = pU / (ps.p[:, :1] * tau[None, :])
        return f - omega * (f - feq)

    def stream(self, fpost):
        out = np.empty_like(fpost)
        xs, ys = np.arange(self.nx), np.arange(self.ny)
        for q in range(self.ps.Q):
            dx, dy = self.ps.disp[q]
            sx = xs - dx
            sy = ys - dy
            sx = np.mod(sx, self.nx) if self.bc[0] == "periodic" else np.clip(sx, 0, self.nx - 1)
            sy = np.mod(sy, self.ny) if self.bc[1] == "periodic" else np.clip(sy, 0, self.ny - 1)
            out[q] = fpost[q][np.ix_(sy, sx)]
        return out

    def step(self, nsteps=1):
        for _ in range(nsteps):
            self.f = self.stream(self.collide())
            self.t += 1


class Model3D(Model):
    """A lattice of Nx x Ny x Nz sites with every population of the 3D
    stencil, f [Q, Nz, Ny, Nx] (Sec. V: the method runs in three dimensions
    as in two).  bc: (bc_x, bc_y, bc_z), each 'periodic' or 'outflow'.  The
    collision is the parent's (it works on any population set with full
    four-momenta); streaming moves population i by its 3D vector n_i."""

    def __init__(self, ps, nx, ny, nz, bc=("periodic", "periodic", "periodic"), tau=1.0):
        if ps.disp3 is None:
            raise ValueError("3D lattices need the full stencil (mode='full')")
        super().__init__(ps, nx, ny, bc=bc[:2], tau=tau)
        self.nz, self.bc3 = nz, bc

    def init_equilibrium(self, n, T, ux, uy, uz):
        S = self.nx * self.ny * self.nz
        n = np.asarray(n, dtype=np.float64).reshape(S)
        T = np.asarray(T, dtype=np.float64).reshape(S)
        ux, uy, uz = (np.asarray(a, dtype=np.float64).reshape(S) for a in (ux, uy, uz))
        g = 1.0 / np.sqrt(1.0 - ux * ux - uy * uy - uz * uz)
        U4 = np.stack([g, g * ux, g * uy, g * uz], axis=-1)
        self.f = equilibrium(self.ps, n, T, U4).reshape(self.ps.Q, self.nz, self.ny, self.nx)
        self.t = 0

    def fields(self, f=None):
        f = self.f if f is None else f
        mac = macroscopic(self.ps, f.reshape(self.ps.Q, -1))
        U = mac["U"]
        shp = (self.nz, self.ny, self.nx)
        out = {k: mac[k].reshape(shp) for k in ("n", "eps", "T", "P")}
        for a, k in ((1, "ux"), (2, "uy"), (3, "uz")):
            out[k] = (U[:, a] / U[:, 0]).reshape(shp)
        N, Tm = mac["N"], mac["Tmn"]
        raw = [N[:, 0], N[:, 1], N[:, 2], N[:, 3], Tm[:, 0, 0], Tm[:, 0, 1], Tm[:, 0, 2], Tm[:, 0, 3],
               Tm[:, 1, 1], Tm[:, 1, 2], Tm[:, 1, 3], Tm[:, 2, 2], Tm[:, 2, 3], Tm[:, 3, 3]]
        out["raw14"] = np.array(raw).reshape((14,) + shp)
        out["_mac"] = mac
        return out

    def collide(self):
        return self._collide_flat().reshape(self.ps.Q, self.nz, self.ny, self.nx)

    def stream(self, fpost):
        out = np.empty_like(fpost)
        axes = [(self.nx, self.bc3[0]), (self.ny, self.bc3[1]), (self.nz, self.bc3[2])]
        for q in range(self.ps.Q):
            src = []
            for (n, bc), d in zip(axes, self.ps.disp3[q]):
                s = np.arange(n) - d
                src.append(np.mod(s, n) if bc == "periodic" else np.clip(s, 0, n - 1))
            out[q] = fpost[q][np.ix_(src[2], src[1], src[0])]
        return out

    def step(self, nsteps=1):
        for _ in range(nsteps):
            self.f = self.stream(self.collide())
            self.t += 1
