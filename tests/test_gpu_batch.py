"""The batched persistent launch (many independent 1D shock tubes, each with
its own stencil at its own mass, eta/s and pressure ratio) against
per-problem oracle runs over the full 500-step horizon."""
import json
import os

import numpy as np
import pytest

import workloads
from tests.helpers import build_batch, oracle_run

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_batch_matches_oracle_full_horizon():
    """Eight problems with mbar drawn continuously over all five stencils of
    the bands (the mbar = 1 stencil in both of its ranges); v0 = the middle
    of the window that the oracle's
    own quadrature solver finds (tests/golden/batch_windows.json), the same
    for both sides.  Fields at steps 250 and 500 within 1e-5 of the oracle;
    no health flag raised."""
    problems, fields = workloads.batched_riemann(nprob=8, seed=4, lmax=512)
    win = json.load(open(os.path.join(ROOT, "tests", "golden", "batch_windows.json")))["problems"]
    assert [w["zeta"] for w in win] == [p["zeta"] for p in problems]
    v0s = [w["v0"] for w in win]
    b = build_batch(problems, fields, v0s)
    assert {p["band"] for p in problems} == {"s133", "s46", "s67", "s73", "s57"}
    samples = b.step(250, sample_every=50)
    mid = {k: v.cpu().numpy() for k, v in b.moments().items()}
    b.step(250)
    out = {k: v.cpu().numpy() for k, v in b.moments().items()}
    h = b.health()
    assert h["flags"] == 0, h
    off = 0
    n, T, ux = fields
    for p, v0 in zip(problems, v0s):
        L = p["nx"]
        sl = slice(off, off + L)
        tau = {k: p[k] for k in ("eta_over_s", "T_R_GeV", "n_unit_fm3", "dx_fm")}
        f1 = (n[sl][None], T[sl][None], ux[sl][None], np.zeros((1, L)))
        st = {"bases": p["bases"], "zeta": p["zeta"], "v0": v0}
        r = oracle_run(st, f1, 500, dim=1, bc=("outflow", "periodic"), tau=tau, checkpoints=[0, 250, 500])
        for step, got in ((250, mid), (500, out)):
            for k in ("n", "eps", "T", "P", "ux"):
                ref = r[step][k][0]
                scale = np.abs(ref).max() if k != "ux" else max(np.abs(ref).max(), 1e-3)
                err = np.abs(got[k][sl] - ref).max() / scale
                assert err < 1e-5, (p["band"], p["zeta"], step, k, err)
        # sample 0 is the initial state: moments and converged frame of f^eq
        s0 = samples[0].cpu().numpy()[sl]
        assert np.abs(s0[:, 9] - r[0]["eps"][0]).max() < 1e-5 * np.abs(r[0]["eps"]).max()
        assert np.abs(s0[:, 0] - r[0]["raw9"][0][0]).max() < 1e-5 * np.abs(r[0]["raw9"][0]).max()
        off += L


def test_batch_64_problems_full_horizon_healthy():
    """The full 64-problem, 500-step workload in one launch over the whole
    chip: no health flag of any kind (the neighbour hand-over included),
    finite fields, and a grid of at least one wave per 64-site tile within
    the device's resident limit."""
    problems, fields = workloads.batched_riemann(nprob=64, seed=0)
    b = build_batch(problems, fields)
    occ = b.occupancy()
    assert occ["tiles"] == sum((p["nx"] + 63) // 64 for p in problems)
    # at least one wave per tile (the grid is sized for the fullest XCD bin)
    assert min((occ["tiles"] + 3) // 4, occ["resident_limit"]) <= occ["workgroups"] <= occ["resident_limit"]
    b.step(500)
    h = b.health()
    out = b.moments()
    assert h["flags"] == 0, h
    assert np.isfinite(out["T"].cpu().numpy()).all()


def test_batch_short_problems_vs_oracle():
    """Problems of 1, 3, 5, 64, 65 and 129 sites (shorter than the stencil's
    reach, one exact tile, one site past a tile, a ragged third tile): the
    outflow ghosts at both ends come from the end sites' values; every
    problem against its own oracle run over 100 steps, <= 1e-5, each stencil
    at the v0 the library chose (the oracle is given the same v0)."""
    import torch
    from paper_1703_04605_amd import rlbm
    probs, parts = [], []
    for s, L in enumerate((1, 3, 5, 64, 65, 129)):
        p, f = workloads.batched_riemann(nprob=1, seed=40 + s, lmin=L, lmax=L)
        probs += p
        parts.append(f)
    fields = tuple(np.concatenate([f[i] for f in parts]) for i in range(3))
    stencils = [rlbm.Solver(p["bases"], p["zeta"], 0.0, dim=1, precision="fp32") for p in probs]
    v0s = [s.info["v0"] for s in stencils]
    b = rlbm.Batch(stencils, [dict(p, stencil=i) for i, p in enumerate(probs)])
    b.init(*[torch.tensor(a, dtype=torch.float64, device="cuda:0") for a in fields])
    b.step(100)
    out = {k: v.cpu().numpy() for k, v in b.moments().items()}
    assert b.health()["flags"] == 0
    off = 0
    n, T, ux = fields
    for p, v0 in zip(probs, v0s):
        L = p["nx"]
        sl = slice(off, off + L)
        tau = {k: p[k] for k in ("eta_over_s", "T_R_GeV", "n_unit_fm3", "dx_fm")}
        f1 = (n[sl][None], T[sl][None], ux[sl][None], np.zeros((1, L)))
        st = {"bases": p["bases"], "zeta": p["zeta"], "v0": v0}
        r = oracle_run(st, f1, 100, dim=1, bc=("outflow", "periodic"), tau=tau, checkpoints=[100])
        for k in ("n", "eps", "T", "P", "ux"):
            ref = r[100][k][0]
            scale = np.abs(ref).max() if k != "ux" else max(np.abs(ref).max(), 1e-3)
            err = np.abs(out[k][sl] - ref).max() / scale
            assert err < 1e-5, (L, p["band"], k, err)
        off += L
