"""Working range in mbar = m/T_R of second-order stencils, and the map of
Sec. III.D (Fig. 5) over all six-group stencils up to a group size.

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


def _probe(args):
    """Working points of one candidate on the mbar grid: for each grid point
    None, or (populations, v0, min weight, condition number)."""
    cand, grid = args
    from paper_1703_04605_amd import rlbm
    out = []
    for z in grid:
        try:
            i = rlbm.solve_stencil(cand, z)
            out.append((i["q3"], i["v0"], min(i["weights"][:6]), i["cond"]))
        except rlbm.RlbmError as e:
            if e.code != rlbm.RLBM_ENOSTENCIL:
                raise
            out.append(None)
    return cand, out


def stencil_map(lo=0.3, hi=40.0, points=36, max_norm2=18, processes=8):
    """The working-range map of Sec. III.D (Fig. 5) for every six-group
    stencil {(0,0,0)} + five groups with |n|^2 <= max_norm2, on a logarithmic
    mbar grid: each stencil that works somewhere, with its working grid
    points, and per grid point the stencil with the fewest populations (ties:
    the larger smallest weight) and the condition number of its system
    matrix at the window's middle."""
    import itertools
    from multiprocessing import get_context
    grid = [lo * (hi / lo) ** (i / (points - 1)) for i in range(points)]
    cands = [[(0, 0, 0)] + list(c) for c in itertools.combinations(base_vectors(max_norm2), 5)]
    with get_context("spawn").Pool(processes) as pool:
        res = pool.map(_probe, [(c, grid) for c in cands], chunksize=16)
    stencils = []
    for cand, pts in res:
        if any(p is not None for p in pts):
            stencils.append({"bases": cand, "populations": next(p[0] for p in pts if p is not None),
                             "works": [i for i, p in enumerate(pts) if p is not None],
                             "cond": [p[3] if p is not None else None for p in pts],
                             "min_weight": [p[2] if p is not None else None for p in pts]})
    best = []
    for i, z in enumerate(grid):
        ok = [s for s in stencils if i in s["works"]]
        if not ok:
            best.append(None)
            continue
        s = min(ok, key=lambda s: (s["populations"], -s["min_weight"][i]))
        best.append({"mbar": z, "bases": s["bases"], "populations": s["populations"], "cond": s["cond"][i],
                     "min_weight": s["min_weight"][i], "working_stencils": len(ok)})
    return {"grid": grid, "max_norm2": max_norm2, "candidates": len(cands), "stencils": stencils,
            "smallest_per_point": best}


def _probe3(args):
    cand, mbar = args
    from paper_1703_04605_amd import rlbm
    try:
        i = rlbm.solve_stencil(cand, mbar, 0.0, dim=3, order=3)
        return cand, (i["q3"], i["v0"], i["v0_lo"], i["v0_hi"], min(i["weights"]), i["cond"])
    except rlbm.RlbmError:
        # no positive window (RLBM_ENOSTENCIL), or more populations than the
        # library's tables hold (RLBM_EINVAL): not usable either way
        return cand, None


def search3(mbar, samples=4000, max_norm2=18, seed=0, processes=4):
    """Third order (Sec. III.D: eleven groups): a seeded random sample of
    eleven-group stencils {(0,0,0)} + ten groups with |n|^2 <= max_norm2,
    probed at mbar with the library's solver (about 30 ms per candidate).
    Returns the working ones as (base vectors, (populations, v0, v0_lo,
    v0_hi, smallest weight, condition number)), fewest populations first."""
    import random
    from multiprocessing import get_context
    rng = random.Random(seed)
    pool = base_vectors(max_norm2)
    cands = set()
    while len(cands) < samples:
        cands.add(tuple(sorted(rng.sample(range(len(pool)), 10))))
    args = [([(0, 0, 0)] + [pool[i] for i in c], mbar) for c in sorted(cands)]
    with get_context("spawn").Pool(processes) as p:
        res = p.map(_probe3, args, chunksize=32)
    ok = [(c, r) for c, r in res if r is not None]
    return sorted(ok, key=lambda t: (t[1][0], -t[1][4]))


def compact(m):
    """A compact form of ``stencil_map``'s result for storage: per grid point
    the number of working stencils, the smallest and the median condition
    number among them and the smallest stencil; per working stencil its base
    vectors (as digit strings), population count and working runs of grid
    indices [first, last]."""
    import statistics
    points = []
    for i, z in enumerate(m["grid"]):
        conds = sorted(s["cond"][i] for s in m["stencils"] if s["cond"][i] is not None)
        points.append({"mbar": z, "working": len(conds),
                       "cond_min": conds[0] if conds else None,
                       "cond_median": statistics.median(conds) if conds else None,
                       "smallest": m["smallest_per_point"][i]})
    stencils = []
    for s in m["stencils"]:
        runs, start, prev = [], None, None
        for i in s["works"]:
            if start is None:
                start = i
            elif i != prev + 1:
                runs.append([start, prev])
                start = i
            prev = i
        runs.append([start, prev])
        stencils.append(["".join(str(c) for c in b) for b in s["bases"]] + [s["populations"], runs])
    return {"grid": m["grid"], "max_norm2": m["max_norm2"], "candidates": m["candidates"],
            "points": points, "stencils": stencils}


if __name__ == "__main__":
    import json
    import os
    import sys
    n2 = int(sys.argv[1]) if len(sys.argv) > 1 else 18
    m = stencil_map(max_norm2=n2, processes=int(os.environ.get("RLBM_MAP_PROCESSES", "8")))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"stencil_map_n{n2}.json")
    with open(path, "w") as fh:
        json.dump(compact(m), fh, separators=(",", ":"))
    print(f"{len(m['stencils'])} of {m['candidates']} stencils work somewhere on the grid; written to {path}")
