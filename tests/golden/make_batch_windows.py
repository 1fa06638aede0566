"""Writes batch_windows.json: for the continuous-mbar parity subset of the
batched shock tubes (workloads.batched_riemann(nprob=8, seed=4, lmax=512)),
each problem's stencil, mbar and the positive-weight v0 window that the
oracle's own quadrature solver finds (oracle.quadrature.positive_window,
mpmath).  Only the oracle is called.  Run from the repository root:

    python tests/golden/make_batch_windows.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import quadrature as quad  # noqa: E402


def vmax(bases):
    return 1.0 / max(sum(c * c for c in b) for b in bases) ** 0.5


def main():
    problems, _ = workloads.batched_riemann(nprob=8, seed=4, lmax=512)
    out = []
    for i, p in enumerate(problems):
        # a grid fine enough to resolve windows 0.2% of the interval wide
        # (the window holding the largest min_k w_k is the one used)
        w = quad.positive_window(p["bases"], p["zeta"], 1e-4, vmax(p["bases"]) * (1 - 1e-9), grid=600)
        if w is None:
            raise SystemExit(f"no positive window for problem {i} (mbar {p['zeta']})")
        lo, hi, best = (float(x) for x in w)
        out.append({"index": i, "band": p["band"], "bases": p["bases"], "zeta": p["zeta"], "v0_lo": lo,
                    "v0_hi": hi, "v0": 0.5 * (lo + hi)})
        print(i, p["band"], p["zeta"], lo, hi, flush=True)
    path = os.path.join(ROOT, "tests", "golden", "batch_windows.json")
    json.dump({"source": "oracle.quadrature.positive_window on workloads.batched_riemann(nprob=8, seed=4, lmax=512)",
               "problems": out}, open(path, "w"), indent=1)


if __name__ == "__main__":
    main()
