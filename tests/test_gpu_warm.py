"""Warm start of the Landau-frame solve (GPU): each site starts from the frame
it converged to in the previous step.  The solve itself is unchanged, so the
fields equal the plain run's to the Landau tolerance, with fewer iterations."""
import numpy as np
import pytest

import workloads
from tests.helpers import to_dev, field_errors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_04605_amd import rlbm
    rlbm.lib()


def _run(precision, landau, warm, variant="auto", steps=30):
    from paper_1703_04605_amd import rlbm
    st = workloads.STENCILS["zeta1"]
    fields = to_dev(workloads.taylor_green(130, 70, seed=5))   # ragged tiles in x
    s = rlbm.Solver(st["bases"], st["zeta"], st["v0"], precision=precision)
    s.init_fields(*fields, tau=0.9, landau=landau)
    s.set_step_variant(variant)
    if warm:
        s.set_warm_start(True)
    s.step(steps)
    h = s.health()
    out = {k: v.cpu().numpy() for k, v in s.moments().items()}
    return out, h["iter_sum"] / (130 * 70 * steps), h["flags"], s.step_kernel()


@pytest.mark.parametrize("precision,landau,variant,tol", [
    ("fp32", "newton", "auto", 1e-6), ("fp32", "fixed_point", "auto", 1e-6), ("fp32", "newton", "table", 1e-6),
    ("fp64", "newton", "auto", 1e-12), ("fp16", "newton", "auto", 1e-3)])
def test_warm_start_matches_plain_and_saves_iterations(precision, landau, variant, tol):
    """(float16 storage: a change of the solve's last bits can flip a stored
    value's rounding, so that path is held to its own tolerance.)"""
    a, ia, fa, ka = _run(precision, landau, True, variant)
    b, ib, fb, kb = _run(precision, landau, False, variant)
    assert ka == kb and fa == 0 and fb == 0
    errs = field_errors(a, b)
    print(precision, landau, variant, ka, "iterations plain %.2f warm %.2f" % (ib, ia), errs)
    assert max(errs.values()) < tol, errs
    assert ia < ib


def test_warm_start_rules():
    """Needs fields; exclusive with the learned guess; a new rlbm_init_fields
    turns it off (the run is then bit for bit the plain run)."""
    from paper_1703_04605_amd import rlbm, learned_guess
    st = workloads.STENCILS["zeta1"]
    s = rlbm.Solver(st["bases"], st["zeta"], st["v0"], precision="fp32")
    with pytest.raises(rlbm.RlbmError) as e:
        s.set_warm_start(True)
    assert e.value.code == rlbm.RLBM_ESTATE
    fields = to_dev(workloads.taylor_green(64, 16, seed=2))
    s.init_fields(*fields)
    s.set_warm_start(True)
    net = rlbm.MLP(learned_guess.init_params(seed=1), np.concatenate([np.zeros(9), np.ones(9), np.zeros(3),
                                                                       np.ones(3)]).astype(np.float32),
                   max_batch=64)
    with pytest.raises(rlbm.RlbmError) as e:
        s.set_landau_guess(net)
    assert e.value.code == rlbm.RLBM_EINVAL
    s.set_warm_start(False)
    s.set_landau_guess(net)
    with pytest.raises(rlbm.RlbmError) as e:
        s.set_warm_start(True)
    assert e.value.code == rlbm.RLBM_EINVAL
    s.set_landau_guess(None)
    s.set_warm_start(True)
    s.step(3)
    s.init_fields(*fields)          # turns the warm start off
    s.health(reset=True)
    s.step(6)
    p = rlbm.Solver(st["bases"], st["zeta"], st["v0"], precision="fp32")
    p.init_fields(*fields)
    p.step(6)
    assert s.health()["iter_sum"] == p.health()["iter_sum"]
    a = {k: v.cpu().numpy() for k, v in s.moments().items()}
    b = {k: v.cpu().numpy() for k, v in p.moments().items()}
    for k in a:
        assert np.array_equal(a[k], b[k]), k
