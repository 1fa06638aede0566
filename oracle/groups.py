"""Velocity groups of Appendix C ("Stencils for three-dimensional lattices").

Each group is the full-symmetric (FS) orbit of a base vector (a, b, c) under
coordinate permutations and sign flips.  The table stores the base vector and
the cardinality printed in the paper's table, so a test can check the orbit
sizes against the printed column.  Group numbers follow the paper's table.
"""
import itertools

# group number -> (base vector, printed cardinality)
GROUPS = {
    1: ((0, 0, 0), 1), 2: ((1, 0, 0), 6), 3: ((1, 1, 0), 12), 4: ((1, 1, 1), 8),
    5: ((2, 0, 0), 6), 6: ((2, 1, 0), 24), 7: ((2, 2, 0), 12), 8: ((2, 1, 1), 24),
    9: ((2, 2, 1), 24), 10: ((2, 2, 2), 8),
    11: ((3, 0, 0), 6), 12: ((3, 1, 0), 24), 13: ((3, 2, 0), 24), 14: ((3, 3, 0), 12),
    15: ((3, 1, 1), 24), 16: ((3, 2, 1), 48), 17: ((3, 2, 2), 24), 18: ((3, 3, 1), 24),
    19: ((3, 3, 2), 24), 20: ((3, 3, 3), 8),
    21: ((4, 0, 0), 6), 22: ((4, 1, 0), 24), 23: ((4, 2, 0), 24), 24: ((4, 3, 0), 24),
    25: ((4, 4, 0), 12), 26: ((4, 1, 1), 24), 27: ((4, 2, 1), 48), 28: ((4, 3, 1), 48),
    29: ((4, 4, 1), 24), 30: ((4, 2, 2), 24), 31: ((4, 3, 2), 48), 32: ((4, 4, 2), 24),
    33: ((4, 3, 3), 24), 34: ((4, 4, 3), 24), 35: ((4, 4, 4), 8),
    36: ((5, 0, 0), 6), 37: ((5, 1, 0), 24), 38: ((5, 2, 0), 24), 39: ((5, 3, 0), 24),
    40: ((5, 4, 0), 24), 41: ((5, 5, 0), 12), 42: ((5, 1, 1), 24), 43: ((5, 2, 1), 48),
    44: ((5, 3, 1), 48), 45: ((5, 4, 1), 48), 46: ((5, 5, 1), 24), 47: ((5, 2, 2), 24),
    48: ((5, 3, 2), 48), 49: ((5, 4, 2), 48), 50: ((5, 5, 2), 24), 51: ((5, 3, 3), 24),
    52: ((5, 4, 3), 48), 53: ((5, 5, 3), 24), 54: ((5, 4, 4), 24), 55: ((5, 5, 4), 24),
    56: ((5, 5, 5), 8),
    57: ((6, 0, 0), 6), 58: ((6, 1, 0), 24), 59: ((6, 2, 0), 24), 60: ((6, 3, 0), 24),
    61: ((6, 4, 0), 24), 62: ((6, 5, 0), 24), 63: ((6, 6, 0), 12), 64: ((6, 1, 1), 24),
    65: ((6, 2, 1), 48), 66: ((6, 3, 1), 48), 67: ((6, 4, 1), 48), 68: ((6, 5, 1), 48),
    69: ((6, 6, 1), 24), 70: ((6, 2, 2), 24), 71: ((6, 3, 2), 48), 72: ((6, 4, 2), 48),
    73: ((6, 5, 2), 48), 74: ((6, 6, 2), 24), 75: ((6, 3, 3), 24), 76: ((6, 4, 3), 48),
    77: ((6, 5, 3), 48), 78: ((6, 6, 3), 24), 79: ((6, 4, 4), 24), 80: ((6, 5, 4), 48),
    81: ((6, 6, 4), 24), 82: ((6, 5, 5), 24), 83: ((6, 6, 5), 24), 84: ((6, 6, 6), 8),
}


def fs_orbit(base):
    """All distinct vectors obtained from ``base`` by permuting coordinates and
    flipping signs (the FS sets of Appendix C), in a fixed sorted order."""
    out = set()
    for perm in itertools.permutations(base):
        for signs in itertools.product((1, -1), repeat=3):
            out.add(tuple(s * c for s, c in zip(signs, perm)))
    return sorted(out)


def base_of(group_number):
    return GROUPS[group_number][0]


def bases_of(group_numbers):
    return [GROUPS[g][0] for g in group_numbers]
