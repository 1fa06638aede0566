"""3D lattices on the GPU (stencil dim 3: every population of the stencil,
14 moments, three velocity components) against the oracle's 3D model with
the full stencil, on boxes whose rows span two 64-site tiles and a ragged
tail, for periodic and outflow boundaries; plus the reductions that pin the
3D path to the 2D one."""
import ctypes

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

FIELDS3 = ("n", "eps", "T", "P", "ux", "uy", "uz")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def smooth3(nz, ny, nx, seed=0, umax=0.25):
    rng = np.random.Generator(np.random.PCG64(seed))
    z, y, x = np.meshgrid(np.arange(nz) / nz, np.arange(ny) / ny, np.arange(nx) / nx, indexing="ij")

    def field(amp):
        f = np.zeros((nz, ny, nx))
        for _ in range(3):
            k = rng.integers(0, 3, 3)
            f += amp * rng.uniform(-1, 1) * np.cos(2 * np.pi * (k[0] * x + k[1] * y + k[2] * z) + rng.uniform(0, 6.3))
        return f

    return 1.0 + field(0.1), 1.0 + field(0.1), field(umax / 3), field(umax / 3), field(umax / 3)


def gpu3(st, fields, steps, precision="fp64", bc=("periodic", "periodic", "periodic"), tau=0.9):
    from paper_1703_04605_amd import rlbm
    from tests.helpers import to_dev
    s = rlbm.Solver3D(st["bases"], st["zeta"], st["v0"], precision=precision)
    s.init_fields(*to_dev(fields), bc=bc, tau=tau)
    s.step(steps)
    out = {k: v.cpu().numpy() for k, v in s.moments(raw=True).items()}
    h = s.health()
    del s
    return out, h


def oracle3(st, fields, steps, bc=("periodic", "periodic", "periodic"), tau=0.9):
    from oracle import lattice as L
    nz, ny, nx = fields[0].shape
    ps = L.build_stencil(st["bases"], st["zeta"], st["v0"], mode="full")
    m = L.Model3D(ps, nx, ny, nz, bc=bc, tau=tau)
    m.init_equilibrium(*fields)
    m.step(steps)
    return m.fields()


def errs(a, b, keys=FIELDS3):
    return {k: float(np.abs(a[k] - b[k]).max() / max(np.abs(b[k]).max(), 1e-3 if k[0] == "u" else 0.0))
            for k in keys}


@pytest.mark.parametrize("name", ["zeta5", "zeta1"])
@pytest.mark.parametrize("bc", [("periodic", "periodic", "periodic"), ("periodic", "outflow", "outflow"),
                                ("outflow", "periodic", "periodic")])
def test_3d_fp64_vs_oracle(name, bc):
    """70 x 5 x 6 (two tiles per row, the second ragged), 4 steps, <= 1e-12."""
    st = workloads.STENCILS[name]
    fields = smooth3(6, 5, 70, seed=11)
    g, h = gpu3(st, fields, 4, "fp64", bc)
    r = oracle3(st, fields, 4, bc)
    e = errs(g, r)
    assert h["flags"] == 0, h
    assert max(e.values()) < 1e-12, e
    assert np.abs(g["raw14"] - r["raw14"]).max() < 1e-12 * np.abs(r["raw14"]).max()


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp16", 2e-3)])
def test_3d_reduced_precision_vs_oracle(precision, tol):
    st = workloads.STENCILS["zeta5"]
    fields = smooth3(6, 7, 70, seed=12)
    g, h = gpu3(st, fields, 8, precision)
    r = oracle3(st, fields, 8)
    e = errs(g, r)
    print(precision, e)
    assert h["flags"] == 0, h
    assert max(e.values()) < tol, e


def test_3d_lattice_smaller_than_reach():
    """3 x 2 x 1 periodic box of the zeta = 1 stencil (reach 4 on every
    axis): every ghost is an image several wraps away."""
    st = workloads.STENCILS["zeta1"]
    fields = smooth3(1, 2, 3, seed=13)
    for bc in (("periodic",) * 3, ("outflow",) * 3):
        g, _ = gpu3(st, fields, 5, "fp64", bc)
        r = oracle3(st, fields, 5, bc)
        e = errs(g, r)
        assert max(e.values()) < 1e-12, (bc, e)


def test_3d_z_uniform_equals_2d_path():
    """A z-uniform 3D run equals the 2D run (merged classes) of the same
    stencil on the GPU."""
    from tests.helpers import gpu_run
    st = workloads.STENCILS["zeta1"]
    n, T, ux, uy = workloads.random_smooth(80, 9, seed=14)
    g2, _ = gpu_run(st, (n, T, ux, uy), 6, precision="fp64", tau=0.9)
    rep = lambda a: np.repeat(a[None], 3, axis=0)
    g3, _ = gpu3(st, (rep(n), rep(T), rep(ux), rep(uy), np.zeros((3, 9, 80))), 6, "fp64")
    for k in ("n", "eps", "T", "ux", "uy"):
        for z in range(3):
            assert np.abs(g3[k][z] - g2[6][k]).max() < 1e-12 * max(1.0, np.abs(g2[6][k]).max()), k
    assert np.abs(g3["uz"]).max() < 1e-14


def test_3d_conservation():
    st = workloads.STENCILS["zeta5"]
    fields = smooth3(8, 8, 64, seed=15)
    g0, _ = gpu3(st, fields, 0, "fp64")
    g1, h = gpu3(st, fields, 30, "fp64")
    assert h["flags"] == 0
    t0, t1 = g0["raw14"].sum(axis=(1, 2, 3)), g1["raw14"].sum(axis=(1, 2, 3))
    for k in (0, 4, 5, 6, 7):
        assert abs(t1[k] - t0[k]) < 1e-12 * abs(t0[4]), k


def test_3d_entry_points_reject_mismatched_dimension():
    import torch
    from paper_1703_04605_amd import rlbm
    L = rlbm.lib()
    st = workloads.STENCILS["zeta5"]
    s2 = rlbm.Solver(st["bases"], st["zeta"], st["v0"], precision="fp64")
    s3 = rlbm.Solver3D(st["bases"], st["zeta"], st["v0"], precision="fp64")
    assert s2.population_bytes(8, 8) > 0 and L.rlbm_population_bytes3(s2.ctx, 8, 8, 8) == 0
    assert s3.population_bytes(8, 8) == 0 and s3.population_bytes3(8, 8, 8) > 0
    f = [torch.ones((2, 8, 8), dtype=torch.float64, device="cuda:0") for _ in range(5)]
    nb = s3.population_bytes3(8, 8, 2)
    pa = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
    pb = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
    lat = rlbm.lattice_desc(8, 8)
    lat.nz = 2
    assert L.rlbm_init_fields(s3.ctx, ctypes.byref(lat), *[t.data_ptr() for t in f[:4]], pa.data_ptr(),
                              pb.data_ptr(), nb, None) == rlbm.RLBM_EINVAL
    lat.landau_method = rlbm.LANDAU["fixed_point"]
    assert L.rlbm_init_fields3(s3.ctx, ctypes.byref(lat), *[t.data_ptr() for t in f], pa.data_ptr(), pb.data_ptr(),
                               nb, None) == rlbm.RLBM_EINVAL
    lat.landau_method = rlbm.LANDAU["newton"]
    assert L.rlbm_init_fields3(s3.ctx, ctypes.byref(lat), *[t.data_ptr() for t in f], pa.data_ptr(), pb.data_ptr(),
                               nb, None) == rlbm.RLBM_OK
    torch.cuda.synchronize()


@pytest.mark.parametrize("name,precision", [("zeta5", "fp32"), ("zeta5", "fp16"), ("zeta1", "fp32"),
                                            ("zeta1", "fp16")])
def test_3d_generated_kernel_matches_table_kernel(name, precision):
    """The generated sign-orbit kernel of a configured 3D stencil against the
    table-driven 3D kernel on the same input (70 x 5 x 6, periodic, 6
    steps): selected automatically, equal to the storage precision's
    rounding (the orbit sums round differently)."""
    from paper_1703_04605_amd import rlbm
    from tests.helpers import to_dev
    st = workloads.STENCILS[name]
    fields = smooth3(6, 5, 70, seed=16)
    out = {}
    for variant in ("auto", "table"):
        s = rlbm.Solver3D(st["bases"], st["zeta"], st["v0"], precision=precision)
        s.init_fields(*to_dev(fields), tau=0.9)
        s.set_step_variant(variant)
        kernel = s.step_kernel()
        s.step(6)
        out[variant] = ({k: v.cpu().numpy() for k, v in s.moments(raw=True).items()}, kernel, s.health())
        del s
    (a, ka, ha), (b, kb, hb) = out["auto"], out["table"]
    assert ka == "fixed" and kb == "table"
    assert ha["flags"] == 0 and hb["flags"] == 0
    tol = 2e-6 if precision == "fp32" else 2e-3
    e = errs(a, b, ("n", "eps", "T", "P"))
    assert max(e.values()) < tol, e
    # velocity components against the largest speed component (rounding moves
    # every component by the same absolute amount)
    speed = max(np.abs(b[k]).max() for k in ("ux", "uy", "uz"))
    for k in ("ux", "uy", "uz"):
        assert np.abs(a[k] - b[k]).max() / speed < tol, k


def test_3d_zeta1_fp32_vs_oracle():
    """The zeta = 1 stencil (67 populations) in float32 storage through the
    generated kernel against the oracle, 8 steps, <= 1e-5."""
    st = workloads.STENCILS["zeta1"]
    fields = smooth3(6, 7, 70, seed=17)
    g, h = gpu3(st, fields, 8, "fp32")
    r = oracle3(st, fields, 8)
    e = errs(g, r)
    assert h["flags"] == 0, h
    assert max(e.values()) < 1e-5, e
