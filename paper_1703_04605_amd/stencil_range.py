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


def base_vectors(max_norm2):
    """Base vectors (a, b, c), a >= b >= c >= 0, 0 < a^2 + b^2 + c^2 <= max_norm2:
    one per velocity group of App. C (the group is the vector's orbit under
    the cube's symmetries)."""
    out = []
    a = 1
    while a * a <= max_norm2:
        for b in range(a + 1):
            for c in range(b + 1):
                if 0 < a * a + b * b + c * c <= max_norm2:
                    out.append((a, b, c))
        a += 1
    return sorted(out, key=lambda v: (v[0] ** 2 + v[1] ** 2 + v[2] ** 2, v))


def search(mbar, max_norm2=18):
    """Six-group stencils {(0,0,0)} + five groups with |n|^2 <= max_norm2 that
    work at mbar, each as a list of base vectors (about 10 ms per candidate;
    11,628 candidates for max_norm2 = 18)."""
    import itertools
    out = []
    for c in itertools.combinations(base_vectors(max_norm2), 5):
        cand = [(0, 0, 0)] + list(c)
        if works(cand, mbar):
            out.append(cand)
    return out
