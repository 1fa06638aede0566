"""Training driver of the learned Landau-frame guess.

Data: (N^a, T^ab) -> (eps, u_x, u_y) pairs that the library itself produces
(rlbm_moments of running lattices).  Training: the library's HIP kernels
(rlbm_mlp_train_step); this module only samples batches and moves arrays.
"""
import numpy as np


def init_params(seed=0):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases (seeded)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = [9, 64, 64, 64, 3]
    out = []
    for i in range(4):
        lim = 1.0 / np.sqrt(sizes[i])
        out.append(rng.uniform(-lim, lim, sizes[i + 1] * sizes[i]))
        out.append(np.zeros(sizes[i + 1]))
    return np.concatenate(out).astype(np.float32)


def collect(solver, steps, every, max_sites=None, seed=0):
    """Runs solver for `steps` steps and returns (raw9 [N, 9], target [N, 3])
    as CUDA float32 tensors sampled every `every` steps."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    X, Y = [], []
    done = 0
    while done < steps:
        solver.step(every)
        done += every
        m = solver.moments(raw=True)
        raw = m["raw9"].reshape(9, -1).T
        tgt = torch.stack([m["eps"].reshape(-1), m["ux"].reshape(-1), m["uy"].reshape(-1)], dim=1)
        if max_sites is not None and raw.shape[0] > max_sites:
            idx = torch.randperm(raw.shape[0], generator=g)[:max_sites].to(raw.device)
            raw, tgt = raw[idx], tgt[idx]
        X.append(raw.float())
        Y.append(tgt.float())
    return torch.cat(X), torch.cat(Y)


def normalisation(raw9, target):
    """mx, sx, my, sy of the inputs raw9/N^0 and outputs (eps/N^0, ux, uy)."""
    r = raw9.double().cpu().numpy()
    t = target.double().cpu().numpy()
    x = r / r[:, :1]
    y = np.stack([t[:, 0] / r[:, 0], t[:, 1], t[:, 2]], axis=1)
    sx = x.std(axis=0)
    sx[sx < 1e-12] = 1.0
    sy = y.std(axis=0)
    sy[sy < 1e-12] = 1.0
    return np.concatenate([x.mean(axis=0), sx, y.mean(axis=0), sy]).astype(np.float32)


def train(mlp, raw9, target, steps, batch=4096, lr=1e-3, seed=0, log_every=0):
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = raw9.shape[0]
    losses = []
    for it in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), generator=g).to(raw9.device)
        loss = mlp.train_step(raw9[idx].contiguous(), target[idx].contiguous(), lr)
        losses.append(loss)
        if log_every and it % log_every == 0:
            print(f"  mlp step {it}: loss {loss:.4e}", flush=True)
    return losses
