"""The batched persistent launch (many independent 1D shock tubes with their
own stencils, eta/s and pressure ratios) against per-problem oracle runs."""
import numpy as np
import pytest

import workloads
from tests.helpers import oracle_run, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def build(problems, fields):
    import torch
    from paper_1703_04605_amd import rlbm
    names = sorted({p["stencil_name"] for p in problems})
    stencils = []
    for nm in names:
        st = workloads.STENCILS[nm]
        stencils.append(rlbm.Solver(st["bases"], st["zeta"], st["v0"], dim=1, precision="fp32"))
    probs = [dict(p, stencil=names.index(p["stencil_name"])) for p in problems]
    b = rlbm.Batch(stencils, probs)
    b.init(*[torch.tensor(a, dtype=torch.float64, device="cuda:0") for a in fields])
    return b


def test_batch_matches_oracle():
    problems, fields = workloads.batched_riemann(nprob=6, seed=3, lmin=256, lmax=420)
    b = build(problems, fields)
    steps = 60
    samples = b.step(steps, sample_every=20)
    out = {k: v.cpu().numpy() for k, v in b.moments().items()}
    assert b.health()["flags"] == 0
    off = 0
    n, T, ux = fields
    for p in problems:
        L = p["nx"]
        sl = slice(off, off + L)
        tau = {k: p[k] for k in ("eta_over_s", "T_R_GeV", "n_unit_fm3", "dx_fm")}
        f1 = (n[sl][None], T[sl][None], ux[sl][None], np.zeros((1, L)))
        r = oracle_run(workloads.STENCILS[p["stencil_name"]], f1, steps, dim=1, bc=("outflow", "periodic"),
                       tau=tau, checkpoints=[0, steps])
        for k in ("n", "eps", "T", "P", "ux"):
            ref = r[steps][k][0]
            scale = np.abs(ref).max() if k != "ux" else max(np.abs(ref).max(), 1e-3)
            assert np.abs(out[k][sl] - ref).max() < 1e-5 * scale, (p["stencil_name"], k)
        # sample 0 is the initial state: moments and converged frame of f^eq
        s0 = samples[0].cpu().numpy()[sl]
        assert np.abs(s0[:, 9] - r[0]["eps"][0]).max() < 1e-5 * np.abs(r[0]["eps"]).max()
        assert np.abs(s0[:, 0] - r[0]["raw9"][0][0]).max() < 1e-5 * np.abs(r[0]["raw9"][0]).max()
        off += L


def test_batch_64_problems_full_horizon_healthy():
    """The full 64-problem, 500-step workload in one launch stays healthy."""
    problems, fields = workloads.batched_riemann(nprob=64, seed=0)
    b = build(problems, fields)
    b.step(500)
    h = b.health()
    out = b.moments()
    assert h["flags"] & 0b1101 == 0, h
    assert np.isfinite(out["T"].cpu().numpy()).all()
