"""Benchmark of the relativistic lattice Boltzmann time step on one MI355X.

Headline: the learned Landau-frame guess inside a sheared flow
(Kelvin-Helmholtz), 2048 x 2048 periodic sites, zeta = m/T_R = 1 (44
population classes), shear +-0.4 across tanh layers 8 cells wide with a
seeded sinusoidal perturbation of amplitude 0.01, tau = 1.5, populations
stored as float32 deviations from a rest-frame equilibrium, the network's
guess followed by fixed-point Landau iterations to |d eps|/eps < 1e-10, 3000
steps.  value = site updates per second / 1e6 of that path, timed with HIP
events on the stream the kernels run on, populations resident in HBM.

Every other measured path sits under ``paths``, each with its rate, HBM
fraction and its per-field deviation from the float64 path on the same
workload:
  * sheared_flow_2048: the same flow without the guess (fixed point from
    u = 0, Newton), with the warm start, and in float64;
  * sheared_flow_4096_fp16: 4096 x 4096 sheared flows in scaled float16 for
    zeta = 0.36, 1, 5, 5000 steps, against float64 runs of the same flows;
  * taylor_green_1024: the 1024^2 vortex in float32, float16 and float64 over
    its 2000-step horizon (float32 accuracy gate 1e-5; the float32 buffers
    only partly exceed the 256 MB Infinity Cache, so this rate is cache
    assisted);
  * batched_riemann: 64 independent 1D shock tubes, 500 steps, one launch;
  * riemann_800: the 800 x 1 shock tube (float64, eta/s = 0.1, 500 steps;
    bound by one wave's per-step latency), launched step by step and replayed
    from a HIP graph;
  * taylor_green_3d: a 256 x 256 x 128 lattice with every population of the
    stencil (Sec. V), float64 / float32 / float16;
  * copy: the library's streaming device copy, the achievable HBM ceiling.
cpu_baseline times the float64 oracle on the host's cores on strips of the
headline workload.
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
FIELDS = ("n", "eps", "T", "P", "ux", "uy")
STEP_KERNEL_SOURCES = ["paper_1703_04605_amd/csrc/rlbm_lib.hip", "paper_1703_04605_amd/csrc/rlbm_device.h",
                       "paper_1703_04605_amd/csrc/rlbm_tables.h", "paper_1703_04605_amd/csrc/rlbm_mlp.h",
                       "paper_1703_04605_amd/csrc/bessel_ratio_coeffs.h",
                       "paper_1703_04605_amd/csrc/gen_fixed_stencils.cpp"]

# relaxation times at which the sheared flows stay healthy over their full
# horizons (at tau = 1 the roll-up loses positivity within ~200 steps, in the
# float64 oracle as on the GPU)
TAU_KH2048 = 1.5
TAU_KH4096 = {"zeta036": 3.0, "zeta1": 3.0, "zeta5": 6.0}


def kernel_source_hash():
    h = hashlib.sha256()
    for p in STEP_KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(key):
    """HBM bytes per launch of a step kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    e = d.get("entries", {}).get(key)
    return None if e is None else e.get("hbm_bytes_per_launch")


def run_path(st, fields, precision, steps, warmup, tau=1.0, landau="newton", guess=None, variant="auto",
             warm=False, keep=True):
    """Runs one path; returns (record, fields after warmup + steps as numpy)."""
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
    sites = s.nx * s.ny
    q = s.info["q"]
    ms_step = ms / steps
    rec = {"mlups": sites * steps / (ms * 1e-3) / 1e6, "ms_per_step": ms_step,
           "hbm_gbs": 2 * q * ELEM[precision] * sites / (ms_step * 1e-3) / 1e9,
           "landau_iter_mean": h["iter_sum"] / (sites * steps), "landau_iter_max": h["iter_max"],
           "health_flags": h["flags"], "kernel": s.step_kernel(), "wall_s": wall, "classes": q}
    rec["hbm_frac"] = rec["hbm_gbs"] / HBM_PEAK_GBS
    out = {k: v.cpu().numpy() for k, v in s.moments().items()} if keep else None
    del s
    torch.cuda.synchronize()
    return rec, out


def field_errors(a, b, vnorm=None, keys=FIELDS):
    """max |a - b| / max |b| per field; velocities optionally normalised by a
    given speed instead (fields whose own maximum is tiny)."""
    import numpy as np
    res = {}
    for k in keys:
        scale = float(np.abs(b[k]).max())
        if vnorm is not None and k in ("ux", "uy", "uz"):
            scale = vnorm
        res[k] = float(np.abs(a[k] - b[k]).max() / (scale if scale > 0 else 1.0))
    return res


def train_guess(st, size=256, steps=400):
    """The learned Landau guess, trained by the library's kernels on moment /
    frame pairs the library produces on the three training workloads: the
    Taylor-Green vortex, a sheared flow and the batched shock tubes."""
    import torch
    import workloads
    from paper_1703_04605_amd import rlbm, learned_guess
    from tests.helpers import to_dev
    X, Y, counts = [], [], {}
    for k, (name, gen, tau) in enumerate((("taylor_green", workloads.taylor_green(size, size, seed=11), 1.0),
                                          ("sheared_flow", workloads.kelvin_helmholtz(size, size, seed=12), 1.5))):
        s = rlbm.Solver(st["bases"], st["zeta"], st["v0"], dim=2, precision="fp32")
        s.init_fields(*to_dev(gen), tau=tau)
        x, y = learned_guess.collect(s, steps=60, every=10, max_sites=32768, seed=k)
        X.append(x)
        Y.append(y)
        counts[name] = int(x.shape[0])
    b, _ = batched(nprob=16, seed=7, lmax=1024)
    smp = b.step(100, sample_every=20).reshape(-1, 12)
    g = torch.Generator(device="cpu").manual_seed(5)
    idx = torch.randperm(smp.shape[0], generator=g)[:65536].to(smp.device)
    smp = smp[idx]
    X.append(smp[:, :9].contiguous())
    Y.append(smp[:, 9:12].contiguous())
    counts["batched_riemann"] = int(smp.shape[0])
    del b
    X, Y = torch.cat(X), torch.cat(Y)
    net = rlbm.MLP(learned_guess.init_params(seed=0), learned_guess.normalisation(X, Y), max_batch=4096)
    t0 = time.perf_counter()
    losses = learned_guess.train(net, X, Y, steps=steps, batch=4096, lr=2e-3)
    return net, {"first": losses[0], "last": losses[-1], "adam_steps": steps, "batch": 4096,
                 "samples": counts, "train_s": time.perf_counter() - t0}


def batched(nprob=64, seed=0, lmax=4096):
    import workloads
    from tests.helpers import build_batch
    problems, fields = workloads.batched_riemann(nprob=nprob, seed=seed, lmax=lmax)
    return build_batch(problems, fields), problems


def time_batched(steps=500):
    """64 independent quasi-1D shock tubes (mbar drawn continuously, each with
    its own stencil), 500 steps in one cooperative launch; tiles hand over
    to their neighbours without a grid-wide barrier."""
    import torch
    # one launch on a small batch first: the kernel's first launch in a
    # process also loads its code, which is not part of a step
    warm, _ = batched(nprob=2, seed=1, lmax=512)
    warm.step(2)
    torch.cuda.synchronize()
    del warm
    t0 = time.perf_counter()
    b, problems = batched()
    setup = time.perf_counter() - t0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    b.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    h = b.health()
    occ = b.occupancy()
    bands = {}
    for p in problems:
        bands[p["band"]] = bands.get(p["band"], 0) + 1
    return {"mlups": b.sites * steps / (ms * 1e-3) / 1e6, "ms": ms, "sites": int(b.sites), "steps": steps,
            "launches": 1, "landau_iter_mean": h["iter_sum"] / (b.sites * steps),
            "landau_iter_max": h["iter_max"], "health_flags": h["flags"], "occupancy": occ,
            "waves": occ["workgroups"] * 4, "waves_per_simd": occ["workgroups"] * 4 / 1024.0,
            "stencil_bands": bands, "zeta_range": [min(p["zeta"] for p in problems), max(p["zeta"] for p in problems)],
            "stencil_setup_s": setup,
            "note": "float32 deviations, one stencil per problem at its own mbar; the two population buffers "
                    f"(2 x {b.pop[0].numel() / 1e6:.1f} MB) stay in the caches, so the rate is not HBM bound"}


def time_riemann_800(steps=500):
    """The 800-site shock tube (FP64, zeta = 1, eta/s, outflow): one launch
    per step, and the same steps replayed from a HIP graph of 100 captured
    launches (torch.cuda.graph on the library's stream argument); the two
    runs end with identical fields."""
    import numpy as np
    import torch
    import workloads
    from paper_1703_04605_amd import rlbm
    from tests.helpers import to_dev
    st = workloads.STENCILS["zeta1"]
    fields, tau = workloads.riemann_1d(800)
    rec = {}
    out = {}
    for mode in ("eager", "graph"):
        s = rlbm.Solver(st["bases"], st["zeta"], st["v0"], dim=1, precision="fp64")
        s.init_fields(*to_dev(fields), bc=("outflow", "periodic"), tau=tau)
        s.step(10)
        chunk = 100
        g = None
        if mode == "graph":
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                s.step(chunk)       # recorded only: the replays below run them
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        if g is None:
            s.step(steps)
        else:
            for _ in range(steps // chunk):
                g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        rec[mode] = {"mlups": 800 * steps / (ms * 1e-3) / 1e6, "ms_per_step": ms / steps}
        out[mode] = {k: v.cpu().numpy() for k, v in s.moments().items()}
        rec[mode]["health_flags"] = s.health()["flags"]
        del s, g
    same = all(np.array_equal(out["eager"][k], out["graph"][k]) for k in out["eager"])
    return {"mlups": rec["eager"]["mlups"], "ms_per_step": rec["eager"]["ms_per_step"], "steps": steps,
            "health_flags": rec["eager"]["health_flags"], "graph": dict(rec["graph"], fields_equal_eager=same),
            "note": "800 sites (13 waves): a step takes one wave's chain of pulls, float64 Landau/EOS/tau and "
                    "stores; replaying 100-launch HIP graphs removes the launch gaps but not that chain"}


def time_3d(shape=(128, 256, 256), steps=200):
    """3D Taylor-Green vortex (Sec. V), every population of the stencil:
    float64, float32 and float16 for G1..G6 (zeta = 5, 57 populations), and
    float32 for the zeta = 1 stencil (67), each against its float64 run."""
    import torch
    import workloads
    from paper_1703_04605_amd import rlbm
    from tests.helpers import to_dev
    nz, ny, nx = shape
    sites = nx * ny * nz
    f = to_dev(workloads.taylor_green_3d(nx, ny, nz, seed=0))
    out = {"workload": f"3D Taylor-Green {nx} x {ny} x {nz}, tau 1, {steps} steps"}
    for name in ("zeta5", "zeta1"):
        st = workloads.STENCILS[name]
        runs, res = {}, {}
        for prec in (("fp64", "fp32", "fp16") if name == "zeta5" else ("fp64", "fp32")):
            s = rlbm.Solver3D(st["bases"], st["zeta"], st["v0"], precision=prec)
            s.init_fields(*f, tau=1.0)
            s.step(10)
            s.health(reset=True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            s.step(steps)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            h = s.health()
            q = s.info["q"]
            gbs = 2 * q * ELEM[prec] * sites / (ms * 1e-3) / 1e9
            res[prec] = {"mlups": sites / (ms * 1e-3) / 1e6, "ms_per_step": ms, "hbm_gbs": gbs,
                         "hbm_frac": gbs / HBM_PEAK_GBS, "landau_iter_mean": h["iter_sum"] / (sites * steps),
                         "health_flags": h["flags"], "populations": q}
            runs[prec] = {k: v.cpu().numpy() for k, v in s.moments().items()}
            del s
            torch.cuda.empty_cache()
        for prec in res:
            if prec != "fp64":
                res[prec]["max_rel_err_vs_fp64"] = field_errors(runs[prec], runs["fp64"], vnorm=0.3,
                                                                keys=FIELDS + ("uz",))
        out[name] = res
    return out


def time_third_order(steps=100):
    """Third-order model with the paper's 161-population stencil (Fig. 2b) at
    mbar = 7.5: a 2D Taylor-Green vortex on 1024^2 (95 merged classes) and a
    3D one on 128 x 128 x 64 (all 161 populations), in float64 and in float32
    deviations (error against the float64 run after the same steps).  The
    step reads every population twice (moments, then collision; the second
    read mostly misses the L2), so the HBM fraction uses the algorithmic
    2 Q S bytes per site."""
    import numpy as np
    import torch
    import workloads
    from paper_1703_04605_amd import rlbm
    from tests.helpers import to_dev
    st = workloads.THIRD_ORDER
    out = {"stencil": "G1 G2 G3 G4 G5 G8 G9 G10 G12 G13 G15 (161 populations)", "zeta": st["zeta"]}
    cases = (("tg2d_1024", 2, lambda: to_dev([a[None] for a in workloads.taylor_green(1024, 1024, seed=0)]
                                             + [np.zeros((1, 1024, 1024))])),
             ("tg3d_128x128x64", 3, lambda: to_dev(workloads.taylor_green_3d(128, 128, 64, seed=0))))
    for name, dim, make in cases:
        f = make()
        res, runs = {}, {}
        for prec in ("fp64", "fp32"):
            s = rlbm.Solver3D(st["bases"], st["zeta"], 0.0, order=3, dim=dim, precision=prec)
            s.init_fields(*f, tau=1.0)
            s.step(5)
            s.health(reset=True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            s.step(steps)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            h = s.health()
            q = s.info["q"]
            sites = f[0].numel()
            gbs = 2 * q * ELEM[prec] * sites / (ms * 1e-3) / 1e9
            res[prec] = {"mlups": sites / (ms * 1e-3) / 1e6, "ms_per_step": ms, "classes": q, "v0": s.info["v0"],
                         "hbm_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                         "landau_iter_mean": h["iter_sum"] / (sites * steps), "health_flags": h["flags"]}
            runs[prec] = {k: v.cpu().numpy() for k, v in s.moments().items()}
            del s
            torch.cuda.empty_cache()
        res["fp32"]["max_rel_err_vs_fp64"] = field_errors(runs["fp32"], runs["fp64"], vnorm=0.3,
                                                          keys=FIELDS + (("uz",) if dim == 3 else ()))
        out[name] = res
        del f
    return out


def copy_bandwidth(nbytes=4 << 30, reps=10):
    """The achievable HBM rate: the library's streaming copy of nbytes (bytes
    read plus written per second), best grid of a few; torch's copy beside it."""
    import torch
    from paper_1703_04605_amd import rlbm
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)

    def rate(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return 2 * nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9

    grids = {wg: rate(lambda: rlbm.device_copy(b, a, wg)) for wg in (16384, 65536, 262144)}
    best = max(grids, key=grids.get)
    res = {"gbs": grids[best], "bytes": nbytes, "workgroups": best, "by_grid": grids,
           "torch_copy_gbs": rate(lambda: b.copy_(a))}
    del a, b
    torch.cuda.empty_cache()
    return res


def _oracle_worker(args):
    """One host core: the float64 oracle (projected classes) on a strip of
    the headline workload for about target_s seconds."""
    nx, rows, row0, target_s = args
    from threadpoolctl import threadpool_limits
    import workloads
    from oracle import lattice as L
    st = workloads.STENCILS["zeta1"]
    n, T, ux, uy = workloads.kelvin_helmholtz(nx, nx, seed=0)
    sl = slice(row0, row0 + rows)
    with threadpool_limits(limits=1):
        ps = L.build_stencil(st["bases"], st["zeta"], st["v0"], mode="projected", dim=2)
        m = L.Model(ps, nx, rows, tau=TAU_KH2048)
        m.init_equilibrium(n[sl], T[sl], ux[sl], uy[sl])
        t0 = time.perf_counter()
        steps = 0
        while time.perf_counter() - t0 < target_s or steps == 0:
            m.step(1)
            steps += 1
        dt = time.perf_counter() - t0
    return nx * rows * steps, dt, steps


def cpu_baseline(nx=2048, rows=8, target_s=15.0):
    """The float64 oracle on every host core of this machine's share (at most
    16), one process per core, each stepping its own periodic strip of the
    headline workload; aggregate site updates per second."""
    import multiprocessing as mp
    cores = min(16, len(os.sched_getaffinity(0)))
    ctx = mp.get_context("spawn")
    jobs = [(nx, rows, (i * rows * 7) % (nx - rows), target_s) for i in range(cores)]
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    rate = sum(u / dt for u, dt, _ in res)
    steps = [s for _, _, s in res]
    return {"value": rate / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{cores} processes, each the float64 oracle (numpy, projected classes, one thread) on its "
                      f"own periodic {nx} x {rows} strip of the {nx}^2 sheared flow for {min(steps)}-{max(steps)} "
                      f"steps (~{target_s:.0f} s); rate summed over processes (pool wall {wall:.0f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3000, help="timed steps of the headline path")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--only", default=None,
                    help="run a single path of the headline workload (fp32_guess_fixed_point, fp32_fixed_point, "
                         "fp32, fp64, ...) or one of third_order, batched, taylor_green_3d, riemann_800 (--steps timed "
                         "steps) and print its record, e.g. for a profiler")
    ap.add_argument("--no-compare", action="store_true", help="headline only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp16-4096", action="store_true", help="skip the 4096^2 float16 flows")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="also run one 256 MiB device copy (scales the profiler's byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is not implemented)", file=sys.stderr)
        sys.exit(2)

    # the oracle's processes start before this process touches the GPU
    cpu = None if (args.no_cpu_baseline or args.only) else cpu_baseline()

    import numpy as np
    import torch
    import workloads
    from tests.helpers import to_dev

    if args.calibration_copy:
        from paper_1703_04605_amd import rlbm
        src = torch.ones(1 << 28, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        rlbm.device_copy(dst, src)
        torch.cuda.synchronize()
        del src, dst

    extra = {"third_order": lambda: time_third_order(args.steps), "batched": lambda: time_batched(args.steps),
             "taylor_green_3d": lambda: time_3d(steps=args.steps), "riemann_800": lambda: time_riemann_800(args.steps)}
    if args.only in extra:
        print(json.dumps({"path": args.only, **extra[args.only]()}))
        return
    st = workloads.STENCILS["zeta1"]
    N = 2048
    kh = to_dev(workloads.kelvin_helmholtz(N, N, seed=0))
    W, K = args.warmup, args.steps

    if args.only:
        p = args.only
        net = train_guess(st)[0] if "guess" in p else None
        rec, _ = run_path(st, kh, p.split("_")[0], K, W, tau=TAU_KH2048,
                          landau="fixed_point" if p.endswith("fixed_point") else "newton",
                          guess=net if "guess" in p else None, warm="warm" in p, keep=False)
        print(json.dumps({"path": p, **rec}))
        return

    net, training = train_guess(st)
    head, o_head = run_path(st, kh, "fp32", K, W, tau=TAU_KH2048, landau="fixed_point", guess=net)
    paths = {}
    if not args.no_compare:
        flow = {"fp32_guess_fixed_point": head}
        runs = {"fp32_guess_fixed_point": o_head}
        for key, prec, landau, g, warm in (("fp32_fixed_point", "fp32", "fixed_point", None, False),
                                           ("fp32_guess", "fp32", "newton", net, False),
                                           ("fp32", "fp32", "newton", None, False),
                                           ("fp32_warm_fixed_point", "fp32", "fixed_point", None, True),
                                           ("fp32_warm", "fp32", "newton", None, True),
                                           ("fp64_fixed_point", "fp64", "fixed_point", None, False),
                                           ("fp64", "fp64", "newton", None, False)):
            flow[key], runs[key] = run_path(st, kh, prec, K, W, tau=TAU_KH2048, landau=landau, guess=g, warm=warm)
        vmax = 0.4
        for key in flow:
            if key != "fp64":
                flow[key]["max_rel_err_vs_fp64"] = field_errors(runs[key], runs["fp64"], vnorm=vmax)
        for g, plain in (("fp32_guess_fixed_point", "fp32_fixed_point"), ("fp32_guess", "fp32"),
                         ("fp32_warm_fixed_point", "fp32_fixed_point"), ("fp32_warm", "fp32")):
            flow[g]["max_rel_err_vs_" + plain] = field_errors(runs[g], runs[plain], vnorm=vmax)
            flow[g]["speedup_vs_" + plain] = flow[g]["mlups"] / flow[plain]["mlups"]
            flow[g]["iteration_ratio_vs_" + plain] = flow[g]["landau_iter_mean"] / flow[plain]["landau_iter_mean"]
        flow["fp32_guess_fixed_point"]["speedup_vs_fp64"] = head["mlups"] / flow["fp64"]["mlups"]
        flow["fp32_fixed_point"]["speedup_vs_fp64_fixed_point"] = (flow["fp32_fixed_point"]["mlups"]
                                                                   / flow["fp64_fixed_point"]["mlups"])
        del runs
        paths["sheared_flow_2048"] = {"workload": f"Kelvin-Helmholtz {N}^2, zeta 1, tau {TAU_KH2048}, "
                                                  f"{K} steps after {W}", "velocity_error_scale": vmax, **flow}
        paths["guess_training"] = training

        # Taylor-Green 1024^2 over its 2000-step horizon
        tg = to_dev(workloads.taylor_green(1024, 1024, seed=0))
        tgp, tgo = {}, {}
        for key, prec, var in (("fp64", "fp64", "auto"), ("fp32", "fp32", "auto"), ("fp32_table", "fp32", "table"),
                               ("fp16", "fp16", "auto")):
            tgp[key], tgo[key] = run_path(st, tg, prec, 2000, 0, tau=1.0, variant=var)
        for key in ("fp32", "fp32_table", "fp16"):
            tgp[key]["max_rel_err_vs_fp64"] = field_errors(tgo[key], tgo["fp64"])
        del tgo, tg
        paths["taylor_green_1024"] = {"workload": "Taylor-Green 1024^2, zeta 1, tau 1, 2000 steps",
                                      "cache_assisted": True, **tgp}

        # 4096^2 sheared flows in scaled float16 for three masses
        if not args.no_fp16_4096:
            big = {}
            khb = to_dev(workloads.kelvin_helmholtz(4096, 4096, seed=0))
            for name in ("zeta036", "zeta1", "zeta5"):
                sb = workloads.STENCILS[name]
                tau = TAU_KH4096[name]
                r16, o16 = run_path(sb, khb, "fp16", 5000, 0, tau=tau)
                r64, o64 = run_path(sb, khb, "fp64", 5000, 0, tau=tau)
                r16["max_rel_err_vs_fp64"] = field_errors(o16, o64, vnorm=0.4)
                big[name] = {"zeta": sb["zeta"], "tau": tau, "fp16": r16, "fp64": r64,
                             "fp16_speedup_vs_fp64": r16["mlups"] / r64["mlups"]}
                del o16, o64
                torch.cuda.empty_cache()
            del khb
            paths["sheared_flow_4096_fp16"] = {"workload": "Kelvin-Helmholtz 4096^2, 5000 steps", **big}
        paths["taylor_green_3d"] = time_3d()
        paths["third_order"] = time_third_order()
        paths["batched_riemann"] = time_batched()
        paths["riemann_800"] = time_riemann_800()
    copy = copy_bandwidth()
    paths["copy"] = copy

    q = head["classes"]
    sites = N * N
    alg = 2 * q * 4 * sites
    res = {
        "metric": "MLUPS (site updates per second / 1e6) of the RLBM time step",
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"kelvin_helmholtz_{N}x{N}_zeta1_fp32_learned_guess", "nx": N, "ny": N,
                   "zeta": st["zeta"], "v0": st["v0"], "population_classes": q,
                   "storage": "float32 deviation", "landau": "learned guess, then fixed point to 1e-10",
                   "tau": TAU_KH2048, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": head["hbm_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["hbm_gbs"] / HBM_PEAK_GBS, "traffic": measured_traffic(f"fp32_guess_{N}x{N}"),
                     "algorithmic_bytes_per_launch": alg, "copy_gbs": copy["gbs"],
                     "copy_frac": head["hbm_gbs"] / copy["gbs"], "kernel": head["kernel"]},
        "cpu_baseline": cpu,
        "paths": paths,
        "landau_iter_mean": head["landau_iter_mean"],
        "health_flags": head["health_flags"],
        "wall_s_timed_region": head["wall_s"],
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
