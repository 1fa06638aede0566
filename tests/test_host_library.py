"""CPU tests of the C ABI library: it loads, exports every symbol the header
declares, and its host-side stencil construction (long double, reduced
six-condition system) agrees with the oracle (mpmath, all 105 pair conditions)."""
import json
import os
import re

import numpy as np
import pytest

import workloads
from paper_1703_04605_amd import rlbm
from oracle import quadrature as quad, lattice as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_pins.json")))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "rlbm.h")).read()
    return sorted(set(re.findall(r"\b(rlbm_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L_ = rlbm.lib()
    syms = declared_symbols()
    assert len(syms) >= 13
    for s in syms:
        assert hasattr(L_, s), s
    assert set(rlbm.EXPORTS) <= set(syms)


def test_printed_weights_from_library():
    q = PINS["quadrature_m5_G1_G6"]
    info = rlbm.solve_stencil(workloads.STENCILS["zeta5"]["bases"], 5.0, 0.398)
    for w, p in zip(info["weights"], q["weights_truncated"]):
        assert 0 <= w - p < 1e-10
    assert info["q3"] == q["n_populations"] and info["ortho_residual"] < 1e-13


def test_window_search_matches_paper():
    q = PINS["quadrature_m5_G1_G6"]
    info = rlbm.solve_stencil(workloads.STENCILS["zeta5"]["bases"], 5.0, 0.0, v0_lo=0.39, v0_hi=0.40)
    assert abs(info["v0_lo"] - q["prune_w2_v0"]) < 1e-9
    assert abs(info["v0_hi"] - q["prune_w3_v0"]) < 1e-9


@pytest.mark.parametrize("name", list(workloads.STENCILS))
def test_weights_match_oracle(name):
    st = workloads.STENCILS[name]
    info = rlbm.solve_stencil(st["bases"], st["zeta"], st["v0"])
    w, res = quad.weights(st["bases"], st["zeta"], st["v0"])
    for a, b in zip(info["weights"], w):
        assert abs(a - float(b)) < 1e-13 * max(1.0, abs(float(b))) + 1e-15
    assert info["ortho_residual"] < 1e-12 and min(info["weights"]) > 0


@pytest.mark.parametrize("name,dim", [("zeta5", 2), ("zeta1", 2), ("zeta036", 2), ("zeta1", 1)])
def test_class_table_matches_oracle_projection(name, dim):
    """The library's merged population classes equal the oracle's projected set
    (same displacement, momenta and aggregated w_i J_k(p_i))."""
    st = workloads.STENCILS[name]
    disp, mom, M = rlbm.class_table(st["bases"], st["zeta"], st["v0"], dim)
    ps = L.build_stencil(st["bases"], st["zeta"], st["v0"], mode="projected", dim=dim)
    assert ps.Q == disp.shape[0]
    # oracle column order: 0,1_0,1_x,1_y,1_z,2_00,2_0x,2_0y,2_0z,2_xx,2_yy,2_xz,2_yz,2_xy
    cols = [0, 1, 2, 3, 5, 6, 7, 9, 10, 13]
    key = lambda d, p0: (int(d[0]), int(d[1]), round(float(p0), 9))
    ours = {key(disp[j], mom[j, 0]): (mom[j], M[j]) for j in range(ps.Q)}
    for j in range(ps.Q):
        k = key(ps.disp[j], ps.p[j, 0])
        assert k in ours
        m_ours, M_ours = ours[k]
        p = np.zeros(3)
        p[:ps.d] = ps.p[j]
        assert np.abs(m_ours - p).max() < 1e-13 * max(1, np.abs(p).max())
        assert np.abs(M_ours - ps.M[j, cols]).max() < 1e-13 * max(1.0, np.abs(ps.M[j]).max())


def test_error_codes():
    b = workloads.STENCILS["zeta5"]["bases"]
    with pytest.raises(rlbm.RlbmError) as e:
        rlbm.solve_stencil(b[:5], 5.0, 0.398)          # five groups: not second order
    assert e.value.code == rlbm.RLBM_EINVAL
    with pytest.raises(rlbm.RlbmError) as e:
        rlbm.solve_stencil(b, 5.0, 0.30)               # weights not all positive
    assert e.value.code == rlbm.RLBM_ENOSTENCIL
    with pytest.raises(rlbm.RlbmError) as e:
        rlbm.solve_stencil(b, 5.0, 0.5)                # G6 faster than light
    assert e.value.code == rlbm.RLBM_EINVAL
    with pytest.raises(rlbm.RlbmError) as e:           # mbar = 0.1: no positive window for this set
        rlbm.solve_stencil(workloads.STENCILS["zeta036"]["bases"], 0.1, 0.0)
    assert e.value.code == rlbm.RLBM_ENOSTENCIL


@pytest.mark.parametrize("zeta", [0.36, 1.0, 5.0, 10.0])
def test_inverse_eos_table_against_oracle(zeta):
    """The GPU's inverse-EOS table (evaluated on the host) against the oracle's
    bisection, over T in [1e-3, 1e3]; and it builds in well under a second."""
    import time
    from oracle import eos
    T = np.geomspace(1e-3, 1e3, 2001)
    e = eos.energy_per_particle(T, zeta)
    t0 = time.perf_counter()
    Tl = rlbm.eos_temperature_host(zeta, e)
    assert time.perf_counter() - t0 < 2.0
    # bounded by the conditioning of the inversion: ulp(e)/c_v with c_v >= 3/2
    err = np.abs(Tl - T) / (np.finfo(float).eps * (e / 1.5 + T))
    assert err.max() < 8.0, err.max()


def test_lattice_checks_on_the_host():
    """rlbm_check_lattice (no GPU) rejects what rlbm_init_fields rejects
    before it touches the device: empty lattices, a 1D stencil on more than
    one row, more than 2^31 - 1 sites, 2^31 or more stored elements, tau <=
    1/2, unknown tau modes, boundary rules and Landau methods, an iteration
    cap above 10^6, and an eta/s rule without its physical units."""
    st = workloads.STENCILS["zeta1"]
    args = (st["bases"], st["zeta"], st["v0"])
    ok = [dict(nx=16, ny=8), dict(nx=4096, ny=4096), dict(nx=3, ny=2, bc=("outflow", "outflow")),
          dict(nx=1, ny=1), dict(nx=800, ny=1, tau={"eta_over_s": 0.1, "T_R_GeV": 0.26, "n_unit_fm3": 15.5,
                                                     "dx_fm": 0.008})]
    for kw in ok:
        rlbm.check_lattice(*args, precision="fp32", **kw)
    bad = [dict(nx=0, ny=4), dict(nx=4, ny=0), dict(nx=65536, ny=32769), dict(nx=32768, ny=32768),
           dict(nx=16, ny=16, tau=0.5), dict(nx=16, ny=16, landau_maxit=2000000),
           dict(nx=16, ny=16, landau="bogus"), dict(nx=16, ny=16, tau={"eta_over_s": 0.1, "T_R_GeV": 0.26,
                                                                      "n_unit_fm3": 0.0, "dx_fm": 0.008})]
    for kw in bad:
        if kw.get("landau") == "bogus":
            d = rlbm.make_desc(*args, precision="fp32")
            lat = rlbm.lattice_desc(16, 16)
            lat.landau_method = 7
            assert rlbm.lib().rlbm_check_lattice(d, lat) == rlbm.RLBM_EINVAL
            lat = rlbm.lattice_desc(16, 16)
            lat.bc_x = 2
            assert rlbm.lib().rlbm_check_lattice(d, lat) == rlbm.RLBM_EINVAL
            lat = rlbm.lattice_desc(16, 16)
            lat.tau_mode = 5
            assert rlbm.lib().rlbm_check_lattice(d, lat) == rlbm.RLBM_EINVAL
            continue
        with pytest.raises(rlbm.RlbmError) as e:
            rlbm.check_lattice(*args, precision="fp32", **kw)
        assert e.value.code == rlbm.RLBM_EINVAL, kw
    # a 1D stencil on two rows; the stored-element limit (44 class rows of
    # 4160 or 8256 elements per lattice row, plus 8 ghost rows)
    with pytest.raises(rlbm.RlbmError):
        rlbm.check_lattice(*args, dim=1, nx=8, ny=2)
    rlbm.check_lattice(*args, dim=1, nx=8, ny=1)
    rlbm.check_lattice(*args, precision="fp16", nx=4096, ny=8192)
    with pytest.raises(rlbm.RlbmError):
        rlbm.check_lattice(*args, precision="fp16", nx=8192, ny=8192)


def test_3d_stencil_and_lattice_checks_on_the_host():
    """A 3D stencil stores every population (q == q3); 3D lattice
    descriptions need nz >= 1 and the Newton Landau solve; 2D ones nz 0 or 1."""
    st = workloads.STENCILS["zeta5"]
    info = rlbm.solve_stencil(st["bases"], st["zeta"], st["v0"], dim=3)
    assert info["q"] == info["q3"] == 57
    d3 = rlbm.make_desc(st["bases"], st["zeta"], st["v0"], 3, "fp32")
    d2 = rlbm.make_desc(st["bases"], st["zeta"], st["v0"], 2, "fp32")
    L = rlbm.lib()
    lat = rlbm.lattice_desc(64, 32)
    for nz, want3, want2 in ((0, rlbm.RLBM_EINVAL, rlbm.RLBM_OK), (1, rlbm.RLBM_OK, rlbm.RLBM_OK),
                             (16, rlbm.RLBM_OK, rlbm.RLBM_EINVAL)):
        lat.nz = nz
        assert L.rlbm_check_lattice(d3, lat) == want3, nz
        assert L.rlbm_check_lattice(d2, lat) == want2, nz
    lat.nz = 16
    lat.landau_method = rlbm.LANDAU["fixed_point"]
    assert L.rlbm_check_lattice(d3, lat) == rlbm.RLBM_EINVAL
    lat.landau_method = rlbm.LANDAU["newton"]
    lat.bc_z = 3
    assert L.rlbm_check_lattice(d3, lat) == rlbm.RLBM_EINVAL
    lat = rlbm.lattice_desc(1024, 1024)
    lat.nz = 1024          # 2^30 sites but far more than 2^31 stored elements
    assert L.rlbm_check_lattice(d3, lat) == rlbm.RLBM_EINVAL


def test_third_order_quadrature_matches_oracle():
    """Third order (Sec. III.D, eleven conditions) on the paper's
    161-population stencil at mbar = 7.5: the library's window, weights and
    orthonormality against the oracle's 465 pair conditions.  The weights
    agree to the conditioning of the problem (cond ~3e5 times the moment
    integrals' ~1e-17), not to the last bit."""
    import numpy as np
    from oracle import groups, third_order as t3
    bases = groups.bases_of([1, 2, 3, 4, 5, 8, 9, 10, 12, 13, 15])
    infos = {dim: rlbm.solve_stencil(bases, 7.5, 0.0, dim=dim, order=3) for dim in (1, 2, 3)}
    assert [infos[d]["q"] for d in (1, 2, 3)] == [36, 95, 161]
    i = infos[3]
    assert i["q3"] == 161 and i["ortho_residual"] < 1e-12
    w, res = t3.weights(bases, 7.5, i["v0"], dps=40)
    w = np.array([float(x) for x in w])
    assert float(res) < 1e-30
    assert (np.abs(w - np.array(i["weights"])) < 1e-10 * w).all()
    # the window's edges: positive just inside, not just outside (oracle)
    for edge, sgn in ((i["v0_lo"], 1), (i["v0_hi"], -1)):
        assert t3.min_weight(bases, 7.5, edge + sgn * 1e-9, dps=30) > 0
        assert t3.min_weight(bases, 7.5, edge - sgn * 1e-9, dps=30) < 0
    # the paper's second-order example stencil cannot be a third-order one
    with pytest.raises(rlbm.RlbmError):
        rlbm.solve_stencil(groups.bases_of([1, 2, 3, 4, 5, 6]), 5.0, 0.0, order=3)


def test_given_weights_are_checked():
    """desc.weights replaces the solve; wrong weights fail the
    orthonormality check, and weights need a given v0."""
    from oracle import groups
    bases = groups.bases_of([1, 2, 3, 4, 5, 6])
    ref = rlbm.solve_stencil(bases, 5.0, 0.398)
    got = rlbm.solve_stencil(bases, 5.0, 0.398, weights=ref["weights"])
    assert got["weights"] == ref["weights"] and got["ortho_residual"] < 1e-12
    bad = list(ref["weights"])
    bad[2] *= 1.001
    with pytest.raises(rlbm.RlbmError):
        rlbm.solve_stencil(bases, 5.0, 0.398, weights=bad)
    with pytest.raises(rlbm.RlbmError):
        rlbm.solve_stencil(bases, 5.0, 0.0, weights=ref["weights"])
