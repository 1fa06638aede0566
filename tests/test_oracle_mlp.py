"""Pins of the float64 MLP reference (learned Landau-frame guess): gradients
against central finite differences, one Adam step against its closed form,
bfloat16 rounding against exactly representable cases."""
import numpy as np

from oracle import mlp


def small_net(seed=0):
    rng = np.random.default_rng(seed)
    flat = np.concatenate([rng.normal(0, 1 / np.sqrt(s[-1]), int(np.prod(s))) for _, s in mlp.SHAPES])
    return flat


def test_parameter_count():
    assert mlp.NPARAM == 9 * 64 + 64 + 2 * (64 * 64 + 64) + 64 * 3 + 3 == 9155


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    flat = small_net(1)
    X = rng.normal(size=(7, 9))
    Y = rng.normal(size=(7, 3))
    loss, g = mlp.loss_and_grads(mlp.unpack(flat), X, Y)
    gflat = mlp.pack(g)
    idx = rng.choice(mlp.NPARAM, 60, replace=False)
    h = 1e-6
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        num = (mlp.loss_and_grads(mlp.unpack(fp), X, Y)[0] - mlp.loss_and_grads(mlp.unpack(fm), X, Y)[0]) / (2 * h)
        assert abs(num - gflat[i]) <= 1e-7 * max(1.0, abs(gflat[i])) + 1e-9, (i, num, gflat[i])


def test_adam_first_step_closed_form():
    """After one step from zero moments, m_hat = g and v_hat = g^2, so the
    update is -lr g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    opt = mlp.Adam()
    new = opt.step(p, g, 1e-3)
    assert np.allclose(new, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_bf16_rounding():
    # exactly representable values are unchanged; halfway cases round to even
    assert mlp.bf16(np.float32(1.0)) == 1.0
    assert mlp.bf16(np.float32(1.0 + 2 ** -7)) == 1.0 + 2 ** -7
    assert mlp.bf16(np.float32(1.0 + 2 ** -8)) == 1.0          # tie -> even (1.0)
    assert mlp.bf16(np.float32(1.0 + 3 * 2 ** -8)) == 1.0 + 2 ** -6   # tie -> even (up)
    x = np.float32(1.0 + 2 ** -8 + 2 ** -12)
    assert mlp.bf16(x) == 1.0 + 2 ** -7


def test_silu_derivative():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    assert np.allclose((mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h), mlp.dsilu(z), atol=1e-9)


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    flat = small_net(3)
    X = rng.normal(size=(256, 9))
    Y = np.stack([np.tanh(X[:, 1]), X[:, 2] * 0.5, np.sin(X[:, 3])], axis=1)
    opt = mlp.Adam()
    l0 = mlp.loss_and_grads(mlp.unpack(flat), X, Y)[0]
    for _ in range(200):
        loss, g = mlp.loss_and_grads(mlp.unpack(flat), X, Y)
        flat = opt.step(flat, mlp.pack(g), 3e-3)
    assert loss < 0.2 * l0
