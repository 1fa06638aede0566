"""Full-horizon runs of the Taylor-Green and Kelvin-Helmholtz workloads through the library.

Reports throughput, Landau iterations, health flags (with the step at which
any first appears) and the drift of the lattice totals of N^0, T^00, T^0x and
T^0y, which collide-then-stream conserves exactly up to rounding (the
collision keeps the moments of eq. mj-discrete-second-moment, streaming moves
populations without loss on a periodic lattice; Sec. III.B).
Usage: python -m paper_1703_04605_amd.horizon
"""
import json
import sys
import time


def totals(s):
    """Lattice sums of N^0, T^00, T^0x, T^0y of the solver's current state."""
    m = s.moments(raw=True)["raw9"]
    t = m.sum(dim=(1, 2)).cpu().numpy()
    return [float(t[0]), float(t[3]), float(t[4]), float(t[5])]


def run(st, size, steps, precision, guess=None, warm=False, chunk=250, seed=0, workload="kelvin_helmholtz",
        tau=1.0):
    """Steps in chunks, checking the health flags after each; stops at the
    first chunk that raises any (onset of an instability) and reports the
    drift of the totals over the healthy steps."""
    import torch
    import workloads
    from paper_1703_04605_amd import rlbm
    gen = getattr(workloads, workload)
    fields = [torch.tensor(a, dtype=torch.float64, device="cuda:0").contiguous() for a in gen(size, size, seed=seed)]
    s = rlbm.Solver(st["bases"], st["zeta"], st["v0"], dim=2, precision=precision)
    s.init_fields(*fields, tau=tau)
    if guess is not None:
        s.set_landau_guess(guess)
    if warm:
        s.set_warm_start(True)
    t0 = totals(s)
    t1 = t0
    s.health(reset=True)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms, done, flags, iters, iters_max = 0.0, 0, 0, 0, 0
    while done < steps:
        k = min(chunk, steps - done)
        torch.cuda.synchronize()
        e0.record(stream)
        s.step(k)
        e1.record(stream)
        torch.cuda.synchronize()
        ms += e0.elapsed_time(e1)
        h = s.health(reset=True)
        if h["flags"]:
            flags = h["flags"]
            break
        done += k
        iters += h["iter_sum"]
        iters_max = max(iters_max, h["iter_max"])
        t1 = totals(s)
    sites = size * size
    return {"workload": workload, "size": size, "steps": steps, "healthy_steps": done, "precision": precision,
            "zeta": st["zeta"], "tau": tau, "kernel": s.step_kernel(), "guess": guess is not None, "warm": warm,
            "mlups": sites * done / (ms * 1e-3) / 1e6 if done else None,
            "landau_iter_mean": iters / (sites * done) if done else None, "landau_iter_max": iters_max,
            "health_flags_at_stop": flags,
            "drift_N0": abs(t1[0] - t0[0]) / abs(t0[0]), "drift_T00": abs(t1[1] - t0[1]) / abs(t0[1]),
            "drift_T0x_over_T00": abs(t1[2] - t0[2]) / abs(t0[1]),
            "drift_T0y_over_T00": abs(t1[3] - t0[3]) / abs(t0[1])}


def trained_guess(st, size=256, steps=400):
    """The learned guess, trained on moments of a Kelvin-Helmholtz run."""
    import torch
    import workloads
    from paper_1703_04605_amd import rlbm, learned_guess
    s = rlbm.Solver(st["bases"], st["zeta"], st["v0"], dim=2, precision="fp32")
    s.init_fields(*[torch.tensor(a, dtype=torch.float64, device="cuda:0").contiguous()
                    for a in workloads.kelvin_helmholtz(size, size, seed=12)], tau=1.0)
    X, Y = learned_guess.collect(s, steps=60, every=10, max_sites=32768, seed=0)
    net = rlbm.MLP(learned_guess.init_params(seed=0), learned_guess.normalisation(X, Y), max_batch=4096)
    learned_guess.train(net, X, Y, steps=steps, batch=4096, lr=2e-3)
    return net


def main():
    import workloads
    S = workloads.STENCILS
    # the benchmark's Taylor-Green workload over its full horizon
    for prec in ("fp64", "fp32", "fp16"):
        print(json.dumps(run(S["zeta1"], 1024, 2000, prec, workload="taylor_green")), flush=True)
    # the sheared flows: float16 at 4096^2 (5000 steps) and float32 at 2048^2
    # (3000 steps, plain, warm start and learned guess), with tau = 1
    for name in ("zeta036", "zeta1", "zeta5"):
        print(json.dumps(run(S[name], 4096, 5000, "fp16")), flush=True)
    net = trained_guess(S["zeta1"])
    for kw in ({}, {"warm": True}, {"guess": net}):
        print(json.dumps(run(S["zeta1"], 2048, 3000, "fp32", **kw)), flush=True)


if __name__ == "__main__":
    sys.exit(main())
