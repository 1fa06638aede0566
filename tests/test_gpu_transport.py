"""Shear waves through the GPU library: the decay equals the oracle's, and
the float32 deviation path measures the same viscosity as float64."""
import numpy as np
import pytest

import workloads
from oracle import lattice as L
from paper_1703_04605_amd import transport

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1703_04605_amd import rlbm
    rlbm.lib()


def test_shear_wave_matches_oracle():
    """32-row wave on a 4-column GPU lattice (uniform in x) against the
    oracle's single column, 60 steps, amplitudes every 10 steps."""
    st = workloads.STENCILS["zeta1"]
    g = transport.measure(st, 0.9, L=32, nx=4, steps=60, every=10, fit_from=0)
    ps = L.build_stencil(st["bases"], st["zeta"], st["v0"], mode="projected")
    m = L.Model(ps, 1, 32, tau=0.9)
    m.init_equilibrium(*transport.shear_wave_fields(32, nx=1))
    for i, t in enumerate(g["times"]):
        if t:
            m.step(10)
        ref = transport.amplitude(m.fields()["ux"])
        assert abs(g["amplitudes"][i] - ref) <= 1e-10 * abs(ref), (t, g["amplitudes"][i], ref)


@pytest.mark.parametrize("name", ["zeta1", "zeta5"])
def test_fp32_measures_the_fp64_viscosity(name):
    st = workloads.STENCILS[name]
    a = transport.measure(st, 1.0, L=64, steps=200, U=1e-2, precision="fp64")
    b = transport.measure(st, 1.0, L=64, steps=200, U=1e-2, precision="fp32")
    print(name, "c_eta fp64 %.5f fp32 %.5f (Grad: 0.66667)" % (a["c_eta"], b["c_eta"]))
    assert abs(b["c_eta"] / a["c_eta"] - 1.0) < 1e-2
