"""Benchmark of the relativistic lattice Boltzmann time step on one MI355X.

Workload (default): the 2D periodic Taylor-Green-type vortex, 1024 x 1024
sites, zeta = m/T_R = 1 (44 population classes), peak speed 0.3, 1% noise on
n and T, tau = 1, the full 2000-step horizon.  The headline path stores
populations as float32 deviations from a rest-frame equilibrium (float64
Landau frame, EOS and projections).  The plain float64 path and the scaled
float16 path are timed on the same workload for comparison.

Prints one JSON line: the headline MLUPS (value), its HBM-roofline fraction
and measured traffic (roofline), the oracle's CPU rate on a bounded sample
(cpu_baseline), and every other path of the method under paths.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ELEM = {"fp64": 8, "fp32": 4, "fp16": 2}
STEP_KERNEL_SOURCES = ["paper_1703_04605_amd/csrc/rlbm_lib.hip", "paper_1703_04605_amd/csrc/rlbm_device.h",
                       "paper_1703_04605_amd/csrc/rlbm_tables.h", "paper_1703_04605_amd/csrc/rlbm_mlp.h",
                       "paper_1703_04605_amd/csrc/bessel_ratio_coeffs.h", "paper_1703_04605_amd/csrc/gen_fixed_stencils.cpp"]


def kernel_source_hash():
    h = hashlib.sha256()
    for p in STEP_KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(precision, nx, ny):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    e = d.get("entries", {}).get(f"{precision}_{nx}x{ny}")
    return None if e is None else e.get("hbm_bytes_per_launch")


def time_path(st, fields, precision, steps, warmup, tau=1.0, landau="newton", guess=None, variant="auto",
              warm=False):
    import torch
    from paper_1703_04605_amd import rlbm
    s = rlbm.Solver(st["bases"], st["zeta"], st["v0"], dim=2, precision=precision)
    s.init_fields(*fields, tau=tau, landau=landau)
    s.set_step_variant(variant)
    if guess is not None:
        s.set_landau_guess(guess)
    if warm:
        s.set_warm_start(True)
    s.step(warmup)
    s.health(reset=True)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    h = s.health()
    return s, ms, wall, h


def train_guess(st, size=256, steps=400):
    """The learned Landau guess, trained by the library's kernels on moments of
    Taylor-Green and Kelvin-Helmholtz runs it produces itself."""
    import torch
    import workloads
    from paper_1703_04605_amd import rlbm, learned_guess
    from tests.helpers import to_dev
    X, Y = [], []
    for k, gen in enumerate((workloads.taylor_green(size, size, seed=11),
                             workloads.kelvin_helmholtz(size, size, seed=12))):
        s = rlbm.Solver(st["bases"], st["zeta"], st["v0"], dim=2, precision="fp32")
        s.init_fields(*to_dev(gen), tau=1.0)
        x, y = learned_guess.collect(s, steps=60, every=10, max_sites=32768, seed=k)
        X.append(x)
        Y.append(y)
    X, Y = torch.cat(X), torch.cat(Y)
    net = rlbm.MLP(learned_guess.init_params(seed=0), learned_guess.normalisation(X, Y), max_batch=4096)
    losses = learned_guess.train(net, X, Y, steps=steps, batch=4096, lr=2e-3)
    return net, losses[0], losses[-1]


def time_batched(steps=500):
    """64 independent quasi-1D shock tubes (lengths 256..4096, mbar snapped to
    0.36/1/5/10, eta/s 0.05..0.5, pressure ratios 2..50), 500 steps in one
    persistent launch, float32 deviation storage."""
    import torch
    import workloads
    from paper_1703_04605_amd import rlbm
    problems, fields = workloads.batched_riemann(nprob=64, seed=0)
    names = sorted({p["stencil_name"] for p in problems})
    stencils = [rlbm.Solver(workloads.STENCILS[nm]["bases"], workloads.STENCILS[nm]["zeta"],
                            workloads.STENCILS[nm]["v0"], dim=1, precision="fp32") for nm in names]
    b = rlbm.Batch(stencils, [dict(p, stencil=names.index(p["stencil_name"])) for p in problems])
    b.init(*[torch.tensor(a, dtype=torch.float64, device="cuda") for a in fields])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    b.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    h = b.health()
    return {"mlups": b.sites * steps / (ms * 1e-3) / 1e6, "ms": ms, "sites": int(b.sites), "steps": steps,
            "launches": 1, "landau_iter_mean": h["iter_sum"] / (b.sites * steps), "health_flags": h["flags"],
            "note": "one 1024-thread workgroup per problem; cache-resident (2 x 11.8 MB of populations), not HBM-bound"}


def calibration_copy(nbytes=1 << 28):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()


def cpu_baseline(st, nx, target_s=12.0):
    """The FP64 oracle (numpy, one thread) on a bounded sample of the same
    workload: a 64-row strip of the lattice, as many steps as fit ~target_s."""
    import numpy as np
    import workloads
    from threadpoolctl import threadpool_limits
    from oracle import lattice as L
    rows = 64
    n, T, ux, uy = workloads.taylor_green(nx, nx, seed=0)
    with threadpool_limits(limits=1):
        ps = L.build_stencil(st["bases"], st["zeta"], st["v0"], mode="projected", dim=2)
        m = L.Model(ps, nx, rows, tau=1.0)
        m.init_equilibrium(n[:rows], T[:rows], ux[:rows], uy[:rows])
        t0 = time.perf_counter()
        steps = 0
        while time.perf_counter() - t0 < target_s or steps == 0:
            m.step(1)
            steps += 1
        dt = time.perf_counter() - t0
    return {"value": nx * rows * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{nx}x{rows} strip of the {nx}x{nx} workload, {steps} steps, projected classes, "
                      f"numpy float64, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--stencil", default="zeta1")
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "fp16"])
    ap.add_argument("--no-compare", action="store_true", help="skip the other precision paths")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-guess", action="store_true", help="skip the learned-guess paths")
    ap.add_argument("--no-warm", action="store_true", help="skip the warm-start paths")
    ap.add_argument("--calibration-copy", action="store_true", help="also run a 256 MiB device copy")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 64-problem workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads
    from tests.helpers import to_dev

    st = workloads.STENCILS[args.stencil]
    nx = ny = args.size
    fields = to_dev(workloads.taylor_green(nx, ny, seed=0))
    if args.calibration_copy:
        calibration_copy()

    s, ms, wall, h = time_path(st, fields, args.precision, args.steps, args.warmup)
    q = s.info["q"]
    sites = nx * ny
    ms_step = ms / args.steps
    mlups = sites * args.steps / (ms * 1e-3) / 1e6
    alg_bytes = 2 * q * ELEM[args.precision] * sites
    achieved = alg_bytes / (ms_step * 1e-3) / 1e9
    traffic = measured_traffic(args.precision, nx, ny)
    out_hp = {k: v.cpu().numpy() for k, v in s.moments().items()}
    iters_mean = h["iter_sum"] / (sites * args.steps)
    kernel = s.step_kernel()
    del s

    paths = {args.precision: {"mlups": mlups, "ms_per_step": ms_step, "hbm_frac": achieved / HBM_PEAK_GBS,
                              "landau_iter_mean": iters_mean, "landau_iter_max": h["iter_max"],
                              "health_flags": h["flags"], "kernel": kernel}}
    if not args.no_compare:
        for key in ("fp64", "fp32", "fp16", "fp64_fixed_point", "fp32_fixed_point", "fp32_table", "fp16_table"):
            p = key.split("_")[0]
            landau = "fixed_point" if key.endswith("fixed_point") else "newton"
            variant = "table" if key.endswith("table") else "auto"
            if key == args.precision:
                continue
            s2, ms2, _, h2 = time_path(st, fields, p, args.steps, args.warmup, landau=landau, variant=variant)
            m2 = sites * args.steps / (ms2 * 1e-3) / 1e6
            ab = 2 * q * ELEM[p] * sites / (ms2 / args.steps * 1e-3) / 1e9
            o2 = {k: v.cpu().numpy() for k, v in s2.moments().items()}
            paths[key] = {"mlups": m2, "ms_per_step": ms2 / args.steps, "hbm_frac": ab / HBM_PEAK_GBS,
                        "landau_iter_mean": h2["iter_sum"] / (sites * args.steps),
                        "landau_iter_max": h2["iter_max"], "health_flags": h2["flags"], "kernel": s2.step_kernel()}
            if key == "fp64":
                # deviation of the headline path from the float64 GPU path (itself
                # parity-tested against the oracle) after the full horizon
                paths[args.precision]["max_rel_err_vs_fp64_path"] = {
                    k: float(np.abs(out_hp[k] - o2[k]).max() / np.abs(o2[k]).max())
                    for k in ("n", "eps", "T", "P", "ux", "uy")}
            del s2
        if "fp64" in paths:
            paths["speedup_vs_fp64"] = mlups / paths["fp64"]["mlups"]
    if not args.no_guess:
        net, l0, l1 = train_guess(st)
        for key, landau in (("fp32_guess", "newton"), ("fp32_guess_fixed_point", "fixed_point")):
            s2, ms2, _, h2 = time_path(st, fields, "fp32", args.steps, args.warmup, landau=landau, guess=net)
            m2 = sites * args.steps / (ms2 * 1e-3) / 1e6
            ab = 2 * q * 4 * sites / (ms2 / args.steps * 1e-3) / 1e9
            o2 = {k: v.cpu().numpy() for k, v in s2.moments().items()}
            paths[key] = {"mlups": m2, "ms_per_step": ms2 / args.steps, "hbm_frac": ab / HBM_PEAK_GBS,
                          "landau_iter_mean": h2["iter_sum"] / (sites * args.steps),
                          "landau_iter_max": h2["iter_max"], "health_flags": h2["flags"],
                          "kernel": s2.step_kernel()}
            # the same step kernel (fixed-stencil or table-driven, whichever the
            # guided run used) without the guess, and the fastest unguided path
            same = "auto" if paths[key]["kernel"] == "fixed" else "table"
            s3, ms3, _, h3 = time_path(st, fields, "fp32", args.steps, args.warmup, landau=landau, variant=same)
            m3 = sites * args.steps / (ms3 * 1e-3) / 1e6
            o3 = {k: v.cpu().numpy() for k, v in s3.moments().items()}
            del s3
            paths[key]["unguided_same_kernel_mlups"] = m3
            paths[key]["unguided_same_kernel_landau_iter_mean"] = h3["iter_sum"] / (sites * args.steps)
            paths[key]["speedup_vs_unguided_same_kernel"] = m2 / m3
            paths[key]["max_rel_err_vs_unguided_same_kernel"] = {
                k: float(np.abs(o2[k] - o3[k]).max() / np.abs(o3[k]).max()) for k in ("n", "eps", "T", "P", "ux", "uy")}
            ref_key = "fp32" if landau == "newton" else "fp32_fixed_point"
            if ref_key == args.precision or ref_key in paths:
                paths[key]["speedup_vs_fastest_unguided"] = m2 / paths[ref_key]["mlups"]
            if "fp64" in paths:
                paths[key]["speedup_vs_fp64"] = m2 / paths["fp64"]["mlups"]
            del s2
        paths["guess_training_loss"] = {"first": l0, "last": l1}
    if not args.no_warm and not args.no_compare:
        # Landau solve started from each site's frame of the previous step,
        # against the same kernel started plainly
        for key, landau in (("fp32_warm", "newton"), ("fp32_warm_fixed_point", "fixed_point")):
            s2, ms2, _, h2 = time_path(st, fields, "fp32", args.steps, args.warmup, landau=landau, warm=True)
            m2 = sites * args.steps / (ms2 * 1e-3) / 1e6
            ab = 2 * q * 4 * sites / (ms2 / args.steps * 1e-3) / 1e9
            o2 = {k: v.cpu().numpy() for k, v in s2.moments().items()}
            kern = s2.step_kernel()
            del s2
            s3, ms3, _, h3 = time_path(st, fields, "fp32", args.steps, args.warmup, landau=landau)
            m3 = sites * args.steps / (ms3 * 1e-3) / 1e6
            o3 = {k: v.cpu().numpy() for k, v in s3.moments().items()}
            del s3
            paths[key] = {"mlups": m2, "ms_per_step": ms2 / args.steps, "hbm_frac": ab / HBM_PEAK_GBS,
                          "landau_iter_mean": h2["iter_sum"] / (sites * args.steps),
                          "landau_iter_max": h2["iter_max"], "health_flags": h2["flags"], "kernel": kern,
                          "extra_bytes_per_site": 24,
                          "plain_same_kernel_mlups": m3,
                          "plain_landau_iter_mean": h3["iter_sum"] / (sites * args.steps),
                          "speedup_vs_plain": m2 / m3,
                          "max_rel_err_vs_plain": {k: float(np.abs(o2[k] - o3[k]).max() / np.abs(o3[k]).max())
                                                   for k in ("n", "eps", "T", "P", "ux", "uy")}}
            gkey = "fp32_guess" if landau == "newton" else "fp32_guess_fixed_point"
            if gkey in paths:
                paths[key]["speedup_vs_learned_guess"] = m2 / paths[gkey]["mlups"]

    if not args.no_batched and not args.no_compare:
        paths["batched_riemann_64x500"] = time_batched()
    cpu = None if args.no_cpu_baseline else cpu_baseline(st, nx)
    res = {
        "metric": "MLUPS (site updates per second / 1e6) of the RLBM time step",
        "value": mlups,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp16": "f16"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"taylor_green_{nx}x{ny}_{args.stencil}", "nx": nx, "ny": ny,
                   "zeta": st["zeta"], "v0": st["v0"], "population_classes": q,
                   "storage": {"fp64": "float64", "fp32": "float32 deviation",
                               "fp16": "scaled float16 deviation"}[args.precision],
                   "tau": 1.0, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": alg_bytes},
        "cpu_baseline": cpu,
        "paths": paths,
        "wall_s_timed_region": wall,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
