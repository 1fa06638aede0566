"""The generated fixed-stencil step kernels (GPU): selected for the configured
stencils in float32 / float16 storage, and equal to the table-driven kernel
(same arithmetic up to rounding order) and to the FP64 oracle."""
import numpy as np
import pytest

import workloads
from tests.helpers import oracle_run, field_errors, to_dev, FIELDS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_04605_amd import rlbm
    rlbm.lib()


def _run(st, fields, steps, precision, variant, tau=0.9):
    from paper_1703_04605_amd import rlbm
    s = rlbm.Solver(st["bases"], st["zeta"], st["v0"], dim=2, precision=precision)
    s.init_fields(*to_dev(fields), tau=tau)
    s.set_step_variant(variant)
    kernel = s.step_kernel()
    s.step(steps)
    out = {k: v.cpu().numpy() for k, v in s.moments(raw=True).items()}
    h = s.health()
    return out, kernel, h


@pytest.mark.parametrize("name,precision", [("zeta1", "fp32"), ("zeta5", "fp32"), ("zeta036", "fp32"),
                                            ("zeta1", "fp16"), ("zeta036", "fp16"), ("zeta10", "fp16")])
def test_fixed_matches_table_kernel(name, precision):
    """300 x 7 periodic box (five 64-site tiles per row with a ragged tail),
    8 steps: the fixed-stencil kernel against the table-driven kernel on the
    same input.  Both round differently (sums over symmetry orbits), so the
    fields agree to the storage precision's rounding, not bit for bit."""
    st = workloads.STENCILS[name]
    fields = workloads.random_smooth(300, 7, seed=21)
    a, ka, ha = _run(st, fields, 8, precision, "auto")
    b, kb, hb = _run(st, fields, 8, precision, "table")
    assert ka == "fixed" and kb == "table"
    assert ha["flags"] == 0 and hb["flags"] == 0
    tol = 2e-6 if precision == "fp32" else 2e-3
    errs = field_errors(a, b, ("n", "eps", "T", "P"))
    assert max(errs.values()) < tol, errs
    speed = max(np.abs(b["ux"]).max(), np.abs(b["uy"]).max())
    for k in ("ux", "uy"):
        assert np.abs(a[k] - b[k]).max() / speed < tol, k


@pytest.mark.parametrize("name", ["zeta1", "zeta5"])
def test_fixed_fp32_vs_oracle(name):
    """The fixed-stencil float32 kernel against the FP64 oracle (float32
    deviation tolerance 1e-5), 300 x 6 box, 5 steps."""
    st = workloads.STENCILS[name]
    fields = workloads.random_smooth(300, 6, seed=22)
    g, kern, h = _run(st, fields, 5, "fp32", "auto", tau=0.95)
    assert kern == "fixed" and h["flags"] == 0
    r = oracle_run(st, fields, 5, tau=0.95)
    errs = field_errors(g, r[5])
    assert max(errs.values()) < 1e-5, errs


def test_other_stencil_uses_table_kernel():
    """A stencil without generated code (the zeta = 1 groups at another v0 of
    their positive-weight window, 0.240391..0.240393) runs the table-driven
    kernel; float64 storage always does."""
    from paper_1703_04605_amd import rlbm
    st = dict(workloads.STENCILS["zeta1"])
    s = rlbm.Solver(st["bases"], st["zeta"], 0.2403915, dim=2, precision="fp32")
    s.init_fields(*to_dev(workloads.random_smooth(128, 4, seed=3)))
    assert s.step_kernel() == "table"
    s64 = rlbm.Solver(st["bases"], st["zeta"], st["v0"], dim=2, precision="fp64")
    s64.init_fields(*to_dev(workloads.random_smooth(128, 4, seed=3)))
    assert s64.step_kernel() == "table"
