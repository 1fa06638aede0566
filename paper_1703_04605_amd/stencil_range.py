"""Working range in mbar = m/T_R of second-order stencils.

A stencil (six velocity groups of App. C) gives a usable quadrature at mbar
only if the conditions of eq. ortho1 have a solution with all weights
positive for some v0 (Sec. III.C-D); the paper's Fig. 5 draws these ranges as
bars.  `working_ranges` scans mbar on a logarithmic grid with the library's
host-side stencil solver (which finds the positive-weight window of v0 or
reports that none exists) and bisects the edges of every run of working
points.
"""
import math


def works(bases, mbar):
    """True when the stencil has a positive-weight v0 window at mbar."""
    from paper_1703_04605_amd import rlbm
    try:
        rlbm.solve_stencil(bases, mbar)
        return True
    except rlbm.RlbmError as e:
        if e.code != rlbm.RLBM_ENOSTENCIL:
            raise
        return False


def _edge(bases, a, b, fa, tol):
    """Bisects [a, b] (works(a) == fa != works(b)) to relative width tol."""
    while b / a - 1.0 > tol:
        m = math.sqrt(a * b)
        if works(bases, m) == fa:
            a = m
        else:
            b = m
    return a if fa else b


def working_ranges(bases, lo=0.2, hi=40.0, points=121, tol=1e-3):
    """List of (mbar_min, mbar_max) intervals in [lo, hi] where the stencil
    works; interior edges are bisected to relative width tol.  Runs narrower
    than the grid spacing can be missed."""
    zs = [lo * (hi / lo) ** (i / (points - 1)) for i in range(points)]
    flags = [works(bases, z) for z in zs]
    out = []
    start = None
    for i, (z, f) in enumerate(zip(zs, flags)):
        if f and start is None:
            start = z if i == 0 else _edge(bases, zs[i - 1], z, False, tol)
        if start is not None and (not f or i == points - 1):
            end = z if f else _edge(bases, zs[i - 1], z, True, tol)
            out.append((start, end))
            start = None
    return out
