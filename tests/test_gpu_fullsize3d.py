"""Parity at the full sizes of the 3D and third-order bench workloads, in
the kernels the benchmark runs (the generated code for float32/float16 and
for the third-order stencil): after k steps a site depends only on the
initial fields within k times the stencil's reach, so the oracle evaluates
sampled sites (corners, edges, interior) on periodic patches cut from the
same seeded initial fields."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

G3 = [1, 2, 3, 4, 5, 8, 9, 10, 12, 13, 15]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def sample_sites(nx, ny, nz, n, seed=0):
    rng = np.random.default_rng(seed)
    pts = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx // 2, 0, nz - 1), (64, 63, nz // 2)]
    pts += [(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))) for _ in range(n - len(pts))]
    return pts


def oracle_at(ps, fields, steps, pts, tau=1.0):
    from oracle import lattice as L
    S = int(np.abs(ps.disp).max())
    R = steps * S
    nz, ny, nx = fields[0].shape
    out = {k: [] for k in ("n", "eps", "T", "ux", "uy", "uz")}
    for (x, y, z) in pts:
        ix = np.arange(x - R, x + R + 1) % nx
        iy = np.arange(y - R, y + R + 1) % ny
        iz = np.arange(z - R, z + R + 1) % nz if nz > 1 else np.array([0])
        patch = [a[np.ix_(iz, iy, ix)] for a in fields]
        m = L.Model3D(ps, 2 * R + 1, 2 * R + 1, len(iz), tau=tau)
        m.init_equilibrium(*patch)
        m.step(steps)
        F = m.fields()
        c = 0 if nz == 1 else R
        for k in out:
            out[k].append(F[k][c, R, R])
    return {k: np.array(v) for k, v in out.items()}


def gpu_at(solver, fields, steps, pts):
    from tests.helpers import to_dev
    solver.init_fields(*to_dev(fields), tau=1.0)
    solver.step(steps)
    m = solver.moments()
    xs, ys, zs = (np.array([p[i] for p in pts]) for i in range(3))
    return {k: m[k].cpu().numpy()[zs, ys, xs] for k in ("n", "eps", "T", "ux", "uy", "uz")}


def check(vals, ref, tol):
    speed = max(np.sqrt(ref["ux"] ** 2 + ref["uy"] ** 2 + ref["uz"] ** 2).max(), 1e-300)
    for k in ref:
        scale = speed if k in ("ux", "uy", "uz") else np.abs(ref[k]).max()
        err = np.abs(vals[k] - ref[k]).max() / scale
        assert err < tol, (k, err)


@pytest.mark.parametrize("name,precision,tol", [("zeta5", "fp64", 1e-12), ("zeta5", "fp32", 1e-5),
                                                ("zeta5", "fp16", 2e-3), ("zeta1", "fp32", 1e-5)])
def test_taylor_green_3d_256x256x128(name, precision, tol):
    """The bench's 3D vortex (256 x 256 x 128), 2 steps, 8 sampled sites."""
    from oracle import lattice as L
    from paper_1703_04605_amd import rlbm
    st = workloads.STENCILS[name]
    fields = workloads.taylor_green_3d(256, 256, 128, seed=0)
    s = rlbm.Solver3D(st["bases"], st["zeta"], st["v0"], precision=precision)
    assert s.step_kernel() == ("table" if precision == "fp64" else "fixed")
    pts = sample_sites(256, 256, 128, 8)
    vals = gpu_at(s, fields, 2, pts)
    del s
    ps = L.build_stencil(st["bases"], st["zeta"], st["v0"], mode="full")
    check(vals, oracle_at(ps, fields, 2, pts), tol)


@pytest.mark.parametrize("dim,precision,tol", [(2, "fp64", 1e-12), (2, "fp32", 1e-5), (3, "fp64", 1e-12),
                                               (3, "fp32", 1e-5)])
def test_third_order_bench_sizes(dim, precision, tol):
    """The bench's third-order vortices (1024^2 in 2D, 128 x 128 x 64 in
    3D) with the library's own window and weights, i.e. the generated code;
    2 steps, 6 sampled sites, against the oracle's third-order model given
    the library's v0 and weights."""
    from oracle import groups, lattice as L
    from paper_1703_04605_amd import rlbm
    bases = groups.bases_of(G3)
    if dim == 2:
        n, T, ux, uy = workloads.taylor_green(1024, 1024, seed=0)
        fields = (n[None], T[None], ux[None], uy[None], np.zeros((1, 1024, 1024)))
        shape = (1024, 1024, 1)
    else:
        fields = workloads.taylor_green_3d(128, 128, 64, seed=0)
        shape = (128, 128, 64)
    s = rlbm.Solver3D(bases, 7.5, 0.0, order=3, dim=dim, precision=precision)
    assert s.step_kernel() == "fixed"
    v0, w = s.info["v0"], [float(x) for x in s.info["weights"]]
    pts = sample_sites(*shape, 6)
    vals = gpu_at(s, fields, 2, pts)
    del s
    ps = L.build_stencil(bases, 7.5, v0, mode="full", order=3, weights=w)
    check(vals, oracle_at(ps, fields, 2, pts), tol)
