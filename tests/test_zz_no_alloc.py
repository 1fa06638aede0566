"""The allocation-free field set-up (rlbm_init_fields_noalloc) against
rlbm_init_fields: the same fields and health after the same steps, on two
set-ups in a row (the second lattice smaller), plus its limits."""
import ctypes

import numpy as np
import pytest

import workloads
from tests.helpers import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def run(st, fields, precision, steps, noalloc, solver=None, variant="auto"):
    from paper_1703_04605_amd import rlbm
    s = solver or rlbm.Solver(st["bases"], st["zeta"], st["v0"], precision=precision)
    s.set_step_variant(variant)
    s.init_fields(*to_dev(fields), tau=0.9, noalloc=noalloc)
    s.step(steps)
    out = {k: v.cpu().numpy() for k, v in s.moments(raw=True).items()}
    return s, out, s.health()


@pytest.mark.parametrize("precision,variant", [("fp32", "auto"), ("fp64", "auto"), ("fp32", "table")])
def test_noalloc_matches_allocating_setup(precision, variant):
    from paper_1703_04605_amd import rlbm
    st = workloads.STENCILS["zeta1"]
    solver = rlbm.Solver(st["bases"], st["zeta"], st["v0"], precision=precision)
    for (nx, ny, seed, steps) in ((200, 70, 4, 9), (70, 33, 5, 6)):   # second call: a smaller lattice
        fields = workloads.random_smooth(nx, ny, seed=seed)
        _, ref, ref_h = run(st, fields, precision, steps, False, variant=variant)
        _, got, got_h = run(st, fields, precision, steps, True, solver=solver, variant=variant)
        for k in ("n", "eps", "T", "P", "ux", "uy", "raw9"):
            assert np.array_equal(got[k], ref[k]), (nx, ny, k)
        assert got_h == ref_h, (got_h, ref_h)
        assert got_h["iter_sum"] > 0


def test_noalloc_takes_over_and_limits():
    """A second context that takes the static slots drops the first one's
    fields (RLBM_ESTATE from its step); an allocating set-up gives them back;
    lattices beyond 262144 tiles are rejected before any device work."""
    import torch
    from paper_1703_04605_amd import rlbm
    L = rlbm.lib()
    st = workloads.STENCILS["zeta1"]
    fields = to_dev(workloads.random_smooth(64, 16, seed=6))
    a = rlbm.Solver(st["bases"], st["zeta"], st["v0"], precision="fp32")
    b = rlbm.Solver(st["bases"], st["zeta"], st["v0"], precision="fp32")
    a.init_fields(*fields, noalloc=True)
    a.step(2)
    b.init_fields(*fields, noalloc=True)
    assert L.rlbm_step(a.ctx, 1, None) == rlbm.RLBM_ESTATE
    b.step(2)
    a.init_fields(*fields)              # allocating set-up: a has its own slots again
    a.step(2)
    torch.cuda.synchronize()
    assert a.health()["flags"] == 0 and b.health()["flags"] == 0
    # 4097 x 4096 sites = 65 x 4096 tiles > 262144: real buffers of the claimed size
    c = rlbm.Solver(workloads.STENCILS["zeta5"]["bases"], 5.0, 0.398, precision="fp16")
    nx, ny = 4097, 4096
    nb = int(c.population_bytes(nx, ny))
    pa = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
    pb = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
    f = [torch.ones((ny, nx), dtype=torch.float64, device="cuda:0") for _ in range(2)] + \
        [torch.zeros((ny, nx), dtype=torch.float64, device="cuda:0") for _ in range(2)]
    lat = rlbm.lattice_desc(nx, ny)
    rc = L.rlbm_init_fields_noalloc(c.ctx, ctypes.byref(lat), *[t.data_ptr() for t in f], pa.data_ptr(),
                                    pb.data_ptr(), nb, None)
    assert rc == rlbm.RLBM_EINVAL
    assert b"262144" in L.rlbm_last_error(c.ctx)
    # the same lattice with the allocating set-up is fine
    rc = L.rlbm_init_fields(c.ctx, ctypes.byref(lat), *[t.data_ptr() for t in f], pa.data_ptr(), pb.data_ptr(), nb,
                            None)
    assert rc == rlbm.RLBM_OK
    torch.cuda.synchronize()
