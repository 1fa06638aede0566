"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
runs: stencil choices (group base vectors, zeta = m/T_R, v0) and initial
fields.  This module holds no arithmetic of the method itself.

Stencils (group bases from Appendix C of arXiv:1703.04605):
  zeta5   G1..G6 at mbar = 5, v0 = 0.398: the paper's worked example (Sec. III.D)
  zeta1   G1,G5,G11,G13,G17,G21 at mbar = 1 (no stencil for mbar = 1 is printed;
          v0 at the midpoint of its positive-weight window)
  zeta036 G1,G14,G49,G51,G60,G70 at mbar = 0.36: the paper's 133-population
          stencil of its BAMPS comparison (Fig. 6), v0 at the window midpoint
  zeta10  G1..G6 at mbar = 10, v0 at the window midpoint
"""
import numpy as np

STENCILS = {
    "zeta5": {"groups": [1, 2, 3, 4, 5, 6],
              "bases": [(0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 1, 1), (2, 0, 0), (2, 1, 0)],
              "zeta": 5.0, "v0": 0.398},
    "zeta1": {"groups": [1, 5, 11, 13, 17, 21],
              "bases": [(0, 0, 0), (2, 0, 0), (3, 0, 0), (3, 2, 0), (3, 2, 2), (4, 0, 0)],
              "zeta": 1.0, "v0": 0.2403918860},
    "zeta036": {"groups": [1, 14, 49, 51, 60, 70],
                "bases": [(0, 0, 0), (3, 3, 0), (5, 4, 2), (5, 3, 3), (6, 3, 0), (6, 2, 2)],
                "zeta": 0.36, "v0": 0.1488231854},
    "zeta10": {"groups": [1, 2, 3, 4, 5, 6],
               "bases": [(0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 1, 1), (2, 0, 0), (2, 1, 0)],
               "zeta": 10.0, "v0": 0.3752119693},
}

# The quasi-1D Riemann workload: left P = 5.43 GeV/fm^3 at T = 0.35 GeV, right
# P = 0.339 GeV/fm^3 at T = 0.2 GeV, u = 0, eta/s = 0.1, on a 6.4 fm domain
# (pressures, eta/s and domain as in the paper's BAMPS benchmark, Sec. IV).
RIEMANN = {"P_left": 5.43, "T_left_GeV": 0.35, "P_right": 0.339, "T_right_GeV": 0.2, "eta_over_s": 0.1,
           "domain_fm": 6.4}


def riemann_1d(nx=800):
    """Quasi-1D shock tube: left/right constant states, u = 0, interface
    between cells nx/2 - 1 and nx/2.  The temperature unit T_R is the geometric
    mean of the two temperatures, so that the lattice temperatures (1.32 and
    0.76) straddle T_R, around which the polynomial expansion is built; n is in
    units of the left density."""
    TR = (RIEMANN["T_left_GeV"] * RIEMANN["T_right_GeV"]) ** 0.5
    nL = RIEMANN["P_left"] / RIEMANN["T_left_GeV"]           # fm^-3
    nR = RIEMANN["P_right"] / RIEMANN["T_right_GeV"]
    left = np.arange(nx) < nx // 2
    n = np.where(left, 1.0, nR / nL)[None, :]
    T = np.where(left, RIEMANN["T_left_GeV"] / TR, RIEMANN["T_right_GeV"] / TR)[None, :]
    z = np.zeros((1, nx))
    tau = {"eta_over_s": RIEMANN["eta_over_s"], "T_R_GeV": TR, "n_unit_fm3": nL,
           "dx_fm": RIEMANN["domain_fm"] / nx}
    return (n, T, z, z.copy()), tau


# Third-order model: the paper's third-order stencil (Fig. 2b; groups G1,
# G2, G3, G4, G5, G8, G9, G10, G12, G13, G15, 161 populations) at mbar = 7.5,
# inside the range where its eleven weights are all positive (about 6.5-8.2);
# v0 is the middle of the positive window the library finds.
THIRD_ORDER = {"bases": [(0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 1, 1), (2, 0, 0), (2, 1, 1), (2, 2, 1), (2, 2, 2),
                         (3, 1, 0), (3, 2, 0), (3, 1, 1)], "zeta": 7.5}


def taylor_green(nx, ny, seed=0, umax=0.3, noise=0.01):
    """Periodic Taylor-Green-type vortex with peak speed umax, plus 1%
    Gaussian noise on n and T around n = T = 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)
    ux = umax * np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
    uy = -umax * np.cos(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    n = 1.0 + noise * rng.standard_normal((ny, nx))
    T = 1.0 + noise * rng.standard_normal((ny, nx))
    return n, T, ux, uy


def taylor_green_3d(nx, ny, nz, seed=0, umax=0.3, noise=0.01):
    """Periodic 3D Taylor-Green vortex u = umax (sin x cos y cos z,
    -cos x sin y cos z, 0) (angles 2 pi x/L) with 1% Gaussian noise on n and
    T around n = T = 1; arrays [nz, ny, nx]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z, y, x = np.meshgrid(2 * np.pi * (np.arange(nz) + 0.5) / nz, 2 * np.pi * (np.arange(ny) + 0.5) / ny,
                          2 * np.pi * (np.arange(nx) + 0.5) / nx, indexing="ij")
    ux = umax * np.sin(x) * np.cos(y) * np.cos(z)
    uy = -umax * np.cos(x) * np.sin(y) * np.cos(z)
    n = 1.0 + noise * rng.standard_normal((nz, ny, nx))
    T = 1.0 + noise * rng.standard_normal((nz, ny, nx))
    return n, T, ux, uy, np.zeros((nz, ny, nx))


def kelvin_helmholtz(nx, ny, seed=0, beta=0.4, width=8.0, amp=0.01):
    """Doubly periodic shear layers at y = L/4, 3L/4 with tanh profile of the
    given width (cells), speed +-beta, and a seeded sinusoidal transverse
    perturbation of amplitude amp; n = T = 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = int(rng.integers(1, 5))
    phi = float(rng.uniform(0, 2 * np.pi))
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    X, Y = np.meshgrid(x, y)
    ux = beta * (np.tanh((Y - ny / 4) / width) - np.tanh((Y - 3 * ny / 4) / width) - 1.0)
    uy = amp * np.sin(2 * np.pi * k * X / nx + phi)
    return np.ones((ny, nx)), np.ones((ny, nx)), ux, uy


def random_smooth(nx, ny, seed=0, umax=0.3):
    """Random smooth periodic fields (a few Fourier modes) for parity tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.arange(nx) / nx
    y = np.arange(ny) / ny
    X, Y = np.meshgrid(x, y)

    def field(amp):
        f = np.zeros((ny, nx))
        for _ in range(3):
            kx, ky = rng.integers(0, 3, 2)
            f += amp * rng.uniform(-1, 1) * np.cos(2 * np.pi * (kx * X + ky * Y) + rng.uniform(0, 6.3))
        return f

    n = 1.0 + field(0.1)
    T = 1.0 + field(0.1)
    ux, uy = field(umax / 3), field(umax / 3)
    return n, T, ux, uy


# Stencils of the batched workload, by mbar band.  Each band lies inside the
# stencil's working range (positive weights for some v0), the bands cover
# [0.36, 10] without a gap, and within each band the stencil is the one whose
# smallest group weight is largest among the working ones (a stencil near the
# edge of its range has a nearly vanishing weight and runs strong shocks
# unstably):
#   s133: the paper's 133-population stencil (Fig. 6), works on [0.3585, 0.5823]
#   s46:  46 populations, works on [0.486, 1.185]
#   s67:  the 67-population mbar = 1 stencil, works on [0.975, 1.064], [1.665, 5.489]
#   s73:  73 populations, works on [1.025, > 8]
#   s57:  G1..G6 (57 populations), works on [4.01, > 40]
_S67 = [(0, 0, 0), (2, 0, 0), (3, 0, 0), (3, 2, 0), (3, 2, 2), (4, 0, 0)]
_S73 = [(0, 0, 0), (2, 0, 0), (2, 1, 1), (2, 2, 0), (2, 2, 1), (3, 0, 0)]
BATCH_BANDS = [
    (0.36, 0.52, "s133", [(0, 0, 0), (3, 3, 0), (5, 4, 2), (5, 3, 3), (6, 3, 0), (6, 2, 2)]),
    (0.52, 0.98, "s46", [(0, 0, 0), (3, 3, 0), (5, 0, 0), (5, 1, 0), (3, 3, 3), (5, 1, 1)]),
    (0.98, 1.06, "s67", _S67),
    (1.06, 1.70, "s73", _S73),
    (1.70, 4.20, "s67", _S67),
    (4.20, 10.0, "s57", [(0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 1, 1), (2, 0, 0), (2, 1, 0)]),
]
BATCH_ZETA_MIN = 0.36   # no second-order stencil has positive weights much below 0.3585


def batch_band(zeta):
    """(name, bases) of the stencil whose band holds mbar = zeta."""
    for lo, hi, name, bases in BATCH_BANDS:
        if lo <= zeta < hi or (hi == BATCH_BANDS[-1][1] and zeta == hi):
            return name, bases
    raise ValueError(f"mbar {zeta} outside [{BATCH_BANDS[0][0]}, {BATCH_BANDS[-1][1]}]")


def batched_riemann(nprob=64, seed=0, lmin=256, lmax=4096, zeta_range=(0.1, 10.0), eta_s_range=(0.05, 0.5),
                    ratio_range=(2.0, 50.0), dx_fm=0.002):
    """Independent quasi-1D shock tubes: length L ~ U{lmin..lmax}, mbar drawn
    log-uniform in zeta_range and clamped to [0.36, 10] (below 0.3585 no
    second-order stencil exists), each problem with the stencil of its band
    at its own mbar (v0 = 0: the middle of the stencil's positive-weight
    window), eta/s uniform, pressure ratio r log-uniform.  Left state
    T = 0.35 GeV, P = 5.43 GeV/fm^3; right state T r^(-1/4), n r^(-3/4) (P ~ T^4);
    T_R the geometric mean of the two temperatures; dx = 0.002 fm (the
    paper's lattice spacing); u = 0; interface at L/2.
    Returns (problems, fields) with fields = (n, T, ux) concatenated."""
    rng = np.random.Generator(np.random.PCG64(seed))
    probs, ns, Ts, us = [], [], [], []
    for _ in range(nprob):
        L = int(rng.integers(lmin, lmax + 1))
        zeta_drawn = float(np.exp(rng.uniform(np.log(zeta_range[0]), np.log(zeta_range[1]))))
        zeta = min(max(zeta_drawn, BATCH_ZETA_MIN), BATCH_BANDS[-1][1])
        band, bases = batch_band(zeta)
        eta_s = float(rng.uniform(*eta_s_range))
        r = float(np.exp(rng.uniform(np.log(ratio_range[0]), np.log(ratio_range[1]))))
        TL, TRt = 0.35, 0.35 * r ** -0.25
        TR = (TL * TRt) ** 0.5
        left = np.arange(L) < L // 2
        ns.append(np.where(left, 1.0, r ** -0.75))
        Ts.append(np.where(left, TL / TR, TRt / TR))
        us.append(np.zeros(L))
        probs.append({"nx": L, "band": band, "bases": bases, "zeta_drawn": zeta_drawn, "zeta": zeta, "v0": 0.0,
                      "eta_over_s": eta_s, "ratio": r, "T_R_GeV": TR, "n_unit_fm3": 5.43 / 0.35, "dx_fm": dx_fm})
    return probs, (np.concatenate(ns), np.concatenate(Ts), np.concatenate(us))
