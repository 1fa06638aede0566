"""Shared helpers of the GPU parity tests: run the HIP library and the oracle
on the same seeded inputs and compare fields element by element."""
import numpy as np

FIELDS = ("n", "eps", "T", "P", "ux", "uy")


def to_dev(arrs):
    import torch
    return [torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0") for a in arrs]


def gpu_run(st, fields, steps, precision="fp64", dim=2, bc=("periodic", "periodic"), tau=1.0, checkpoints=None,
            landau_tol=0.0, landau_maxit=0, landau="newton"):
    """Runs the library; returns {step: fields(numpy)} at the checkpoints."""
    from paper_1703_04605_amd import rlbm
    s = rlbm.Solver(st["bases"], st["zeta"], st["v0"], dim=dim, precision=precision)
    s.init_fields(*to_dev(fields), bc=bc, tau=tau, landau_tol=landau_tol, landau_maxit=landau_maxit, landau=landau)
    cps = sorted(set(checkpoints or [steps]))
    out, done = {}, 0
    for c in cps:
        s.step(c - done)
        done = c
        out[c] = {k: v.cpu().numpy() for k, v in s.moments(raw=True).items()}
    return out, s


def oracle_run(st, fields, steps, mode="projected", dim=2, bc=("periodic", "periodic"), tau=1.0,
               checkpoints=None):
    from oracle import lattice as L
    ny, nx = fields[0].shape
    ps = L.build_stencil(st["bases"], st["zeta"], st["v0"], mode=mode, dim=dim)
    if isinstance(tau, dict):
        tau = {"eta_s": tau["eta_over_s"],
               "units": {k: tau[k] for k in ("T_R_GeV", "n_unit_fm3", "dx_fm")}}
    m = L.Model(ps, nx, ny, bc=bc, tau=tau)
    m.init_equilibrium(*fields)
    cps = sorted(set(checkpoints or [steps]))
    out, done = {}, 0
    for c in cps:
        m.step(c - done)
        done = c
        out[c] = m.fields()
    return out


def rel_err(a, b):
    """max |a - b| / max |b| (per field, the error metric of the parity gates)."""
    scale = np.abs(b).max()
    return float(np.abs(a - b).max() / (scale if scale > 0 else 1.0))


def field_errors(gpu, ref, keys=FIELDS):
    return {k: rel_err(gpu[k], ref[k]) for k in keys}


def build_batch(problems, fields, v0s=None):
    """The batched launch of `problems` (workloads.batched_riemann), one
    float32 1D stencil context per problem at its own mbar; v0s overrides
    each problem's v0 (0: the library's own window midpoint)."""
    import torch
    from paper_1703_04605_amd import rlbm
    stencils = [rlbm.Solver(p["bases"], p["zeta"], p["v0"] if v0s is None else v0s[i], dim=1, precision="fp32")
                for i, p in enumerate(problems)]
    b = rlbm.Batch(stencils, [dict(p, stencil=i) for i, p in enumerate(problems)])
    b.init(*[torch.tensor(a, dtype=torch.float64, device="cuda:0") for a in fields])
    return b
