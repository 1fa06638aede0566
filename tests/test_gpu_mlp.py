"""The learned Landau-frame guess on the GPU against the float64 oracle:
training-step gradients and loss, array inference, the in-step matrix-core
inference, and the guided step against the unguided one."""
import numpy as np
import pytest

import workloads
from oracle import mlp as omlp
from tests.helpers import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def moment_batch(n=2048, seed=0):
    """Moments (raw9) and converged frames of the library's own states."""
    import torch
    from paper_1703_04605_amd import rlbm, learned_guess
    st = workloads.STENCILS["zeta1"]
    s = rlbm.Solver(st["bases"], st["zeta"], st["v0"], precision="fp32")
    s.init_fields(*to_dev(workloads.taylor_green(64, 64, seed=seed)), tau=0.9)
    X, Y = learned_guess.collect(s, steps=20, every=10)
    g = torch.Generator(device="cpu").manual_seed(seed)
    idx = torch.randperm(X.shape[0], generator=g)[:n].to(X.device)
    return X[idx].contiguous(), Y[idx].contiguous()


def oracle_batch(raw9, target, norm):
    r = raw9.cpu().numpy().astype(np.float64)
    t = target.cpu().numpy().astype(np.float64)
    stats = (norm[:9].astype(np.float64), norm[9:18].astype(np.float64), norm[18:21].astype(np.float64),
             norm[21:24].astype(np.float64))
    X = omlp.standardise(r, stats)
    y = np.stack([t[:, 0] / r[:, 0], t[:, 1], t[:, 2]], axis=1)
    return X, (y - stats[2]) / stats[3], stats


def test_train_step_matches_oracle():
    from paper_1703_04605_amd import rlbm, learned_guess
    raw9, target = moment_batch(1024)
    params = learned_guess.init_params(seed=4)
    norm = learned_guess.normalisation(raw9, target)
    net = rlbm.MLP(params, norm, max_batch=1024)
    loss = net.train_step(raw9, target, 1e-3)
    p1, g = net.params()
    X, Y, _ = oracle_batch(raw9, target, norm)
    lo, go = omlp.loss_and_grads(omlp.unpack(omlp.bf16(params)), X, Y)
    assert abs(loss - lo) <= 1e-5 * lo
    go = omlp.pack(go)
    for name, shape in omlp.SHAPES:      # per parameter block
        o = sum(int(np.prod(s)) for n, s in omlp.SHAPES[:[n for n, _ in omlp.SHAPES].index(name)])
        k = int(np.prod(shape))
        ref = go[o:o + k]
        assert np.abs(g[o:o + k] - ref).max() <= 1e-4 * np.abs(ref).max() + 1e-9, name
    # first Adam step from zero moments: p - lr g/(|g| + eps) with the GPU's gradient
    expect = params.astype(np.float64) - 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.abs(p1 - expect).max() < 1e-6


def test_predict_matches_oracle():
    import torch
    from paper_1703_04605_amd import rlbm, learned_guess
    raw9, target = moment_batch(2048, seed=1)
    params = learned_guess.init_params(seed=6)
    norm = learned_guess.normalisation(raw9, target)
    net = rlbm.MLP(params, norm, max_batch=2048)
    learned_guess.train(net, raw9, target, steps=20, batch=1024, lr=1e-3)
    p, _ = net.params()
    pred = net.predict(raw9).cpu().numpy().astype(np.float64)
    X, _, stats = oracle_batch(raw9, target, norm)
    out, _ = omlp.forward(omlp.unpack(omlp.bf16(p)), X)
    ref = out * stats[3] + stats[2]
    ref[:, 0] *= raw9[:, 0].cpu().numpy()
    for k in range(3):
        assert np.abs(pred[:, k] - ref[:, k]).max() <= 1e-4 * max(1.0, np.abs(ref[:, k]).max())


def test_in_step_inference_matches_oracle():
    """The matrix-core inference inside the step kernel (bfloat16 operands,
    float32 accumulation) against the oracle with bfloat16-rounded activations."""
    from paper_1703_04605_amd import rlbm, learned_guess
    raw9, target = moment_batch(2048, seed=2)
    params = learned_guess.init_params(seed=7)
    norm = learned_guess.normalisation(raw9, target)
    net = rlbm.MLP(params, norm, max_batch=2048)
    learned_guess.train(net, raw9, target, steps=50, batch=1024, lr=2e-3)
    p, _ = net.params()
    st = workloads.STENCILS["zeta1"]
    s = rlbm.Solver(st["bases"], st["zeta"], st["v0"], precision="fp32")
    s.init_fields(*to_dev(workloads.taylor_green(100, 30, seed=3)), tau=0.9)   # 3000 sites: ragged waves
    s.step(3)
    s.set_landau_guess(net)
    guess = s.landau_guess_fields().cpu().numpy().reshape(3, -1).T.astype(np.float64)
    m = s.moments(raw=True)
    r9 = m["raw9"].reshape(9, -1).T.cpu().numpy()
    X = omlp.standardise(r9.astype(np.float32).astype(np.float64), (norm[:9], norm[9:18], norm[18:21], norm[21:24]))
    out, _ = omlp.forward(omlp.unpack(omlp.bf16(p)), X, act_bf16=True)
    ref = out * norm[21:24] + norm[18:21]
    ref[:, 0] *= r9[:, 0]
    scale = np.abs(ref).max(axis=0)
    err = np.abs(guess - ref).max(axis=0) / np.maximum(scale, 1e-30)
    assert (err < 2e-2).all(), err


@pytest.mark.parametrize("landau,variant", [("newton", "table"), ("fixed_point", "table"), ("newton", "auto")])
def test_guided_step_matches_plain_and_saves_iterations(landau, variant):
    """With a trained network the fields equal the unguided run's to 1e-6 and
    the Landau solve takes fewer iterations.  Both runs use the same step
    kernel (table-driven, or both the generated fixed-stencil kernel), so the
    comparison sees the guess's effect only, not a change of rounding order."""
    from paper_1703_04605_amd import rlbm, learned_guess
    from tests.helpers import field_errors
    raw9, target = moment_batch(8192, seed=4)
    params = learned_guess.init_params(seed=8)
    norm = learned_guess.normalisation(raw9, target)
    net = rlbm.MLP(params, norm, max_batch=4096)
    learned_guess.train(net, raw9, target, steps=400, batch=4096, lr=2e-3)
    st = workloads.STENCILS["zeta1"]
    fields = to_dev(workloads.taylor_green(128, 128, seed=5))
    res = {}
    for guided in (False, True):
        s = rlbm.Solver(st["bases"], st["zeta"], st["v0"], precision="fp32")
        s.init_fields(*fields, tau=0.9, landau=landau)
        s.set_step_variant(variant)
        if guided:
            s.set_landau_guess(net)
        assert s.step_kernel() == ("table" if variant == "table" else "fixed")
        s.step(30)
        h = s.health()
        res[guided] = ({k: v.cpu().numpy() for k, v in s.moments().items()}, h["iter_sum"] / (128 * 128 * 30))
    errs = field_errors(res[True][0], res[False][0])
    print(landau, "iterations plain %.2f guided %.2f" % (res[False][1], res[True][1]), errs)
    assert max(errs.values()) < 1e-6, errs
    assert res[True][1] < res[False][1]
