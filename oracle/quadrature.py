"""Quadratures with prescribed abscissae (Sec. III.C-D).

Abscissae (eq. four-momentum): p_{i,k} = mbar gamma_k (1, v0 n_{i,k}) with
gamma_k = (1 - v0^2 |n_k|^2)^(-1/2), lattice units T_R = 1.  One weight per
group (every population of group k carries w_k).  The weights solve the
orthonormality conditions (eq. ortho1 / eq. orthonormal)

    sum_k w_k sum_{i in k} J^(l)(p_{i,k}) J^(k')(p_{i,k}) = delta_{l k'}

for every pair of second-order polynomials (l <= k').  This is the linear
system A(v0) w = b of the paper (b a binary vector); it is overdetermined but
consistent for a suitable group set, and is solved here in the least-squares
sense in mpmath so that its residual certifies consistency.
"""
import numpy as np
from mpmath import mp, mpf, sqrt as msqrt

from .groups import fs_orbit
from .polynomials import evaluate_printed, NPOLY


def abscissae(bases, mbar, v0, dps=50):
    """Populations of the stencil: list over groups of (vectors [N_k,3] int,
    momenta [N_k,4] mpf object array)."""
    with mp.workdps(dps):
        m, v = mpf(mbar), mpf(v0)
        out = []
        for b in bases:
            vecs = np.array(fs_orbit(tuple(b)), dtype=np.int64)
            n2 = int(sum(c * c for c in b))
            g = 1 / msqrt(1 - v * v * n2)
            p = np.empty((len(vecs), 4), dtype=object)
            for i, nv in enumerate(vecs):
                p[i, 0] = m * g
                for a in range(3):
                    p[i, a + 1] = m * g * v * int(nv[a])
            out.append((vecs, p))
        return out


def system(bases, mbar, v0, dps=50):
    """A(v0) (rows: pairs l <= k of polynomials, columns: groups) and b."""
    with mp.workdps(dps):
        pops = abscissae(bases, mbar, v0, dps)
        Jg = [evaluate_printed(p, mbar, dps) for (_, p) in pops]
        rows, rhs = [], []
        for l in range(NPOLY):
            for k in range(l, NPOLY):
                rows.append([mp.fsum(Jg[g][l][i] * Jg[g][k][i] for i in range(len(pops[g][0])))
                             for g in range(len(bases))])
                rhs.append(mpf(1) if l == k else mpf(0))
        return mp.matrix(rows), mp.matrix(rhs)


def weights(bases, mbar, v0, dps=50):
    """Least-squares weights (mpf list) and the residual max|A w - b|."""
    with mp.workdps(dps):
        A, b = system(bases, mbar, v0, dps)
        At = A.T
        w = mp.lu_solve(At * A, At * b)
        r = A * w - b
        return [w[i] for i in range(len(bases))], max(abs(r[i]) for i in range(r.rows))


def min_weight(bases, mbar, v0, dps=40):
    """Smallest weight at v0; -inf where A(v0) is singular (no unique
    weights exist there, so the point cannot carry a quadrature)."""
    try:
        w, _ = weights(bases, mbar, v0, dps)
    except ZeroDivisionError:
        return mpf("-inf")
    return min(w)


def positive_window(bases, mbar, lo, hi, grid=60, zoom=12, dps=40):
    """Interval of v0 in [lo, hi] on which every weight is positive.

    Grid search for the v0 maximising min_k w_k, repeated on a shrinking
    interval around the best point, then bisection of both edges.  Returns
    (v_lo, v_hi, v_best) as mpf, or None if no positive point was found."""
    with mp.workdps(dps):
        a, c = mpf(lo), mpf(hi)
        best, bestval = None, None
        for _ in range(zoom):
            pts = [a + (c - a) * i / grid for i in range(grid + 1)]
            vals = [min_weight(bases, mbar, v, dps) for v in pts]
            i = max(range(len(vals)), key=lambda j: vals[j])
            best, bestval = pts[i], vals[i]
            if bestval > 0:
                break
            h = (c - a) / grid
            a, c = max(pts[i] - 2 * h, mpf(lo)), min(pts[i] + 2 * h, mpf(hi))
        if bestval is None or bestval <= 0:
            return None

        def edge(inside, outside):
            for _ in range(80):
                mid = (inside + outside) / 2
                if min_weight(bases, mbar, mid, dps) > 0:
                    inside = mid
                else:
                    outside = mid
            return inside

        step = (c - a) / grid
        # (the bound is checked before the weights: beyond v_max the
        # abscissae are not real)
        left = best
        while left - step > lo and min_weight(bases, mbar, left - step, dps) > 0:
            left -= step
        right = best
        while right + step < hi and min_weight(bases, mbar, right + step, dps) > 0:
            right += step
        # (a window that reaches the search interval's end is cut there)
        return edge(left, max(left - step, mpf(lo))), edge(right, min(right + step, mpf(hi))), best
