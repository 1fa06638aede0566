"""Float64 reference of the learned initial guess for the Landau-frame solve.

Not part of the paper's method: a small multilayer perceptron maps the nine
moments of a site, divided by N^0, to (eps/N^0, u_x, u_y).  Architecture
9 -> 64 -> 64 -> 64 -> 3 with SiLU activations, silu(z) = z / (1 + exp(-z)).
Inputs and outputs are standardised with per-component means and standard
deviations of the training set; the loss is the mean squared error of the
standardised outputs; training uses Adam (beta1 = 0.9, beta2 = 0.999,
epsilon = 1e-8, bias-corrected).

Parameters are one flat float vector in the order
    W1 [64 x 9], b1 [64], W2 [64 x 64], b2 [64], W3 [64 x 64], b3 [64], W4 [3 x 64], b4 [3]
(row-major, W_l maps layer l-1 to layer l: z = W a + b), 9155 values.

The GPU keeps float32 master weights and computes with their bfloat16
roundings (round to nearest, ties to even); ``bf16`` reproduces that rounding
so the oracle can be evaluated on the same weights.
"""
import numpy as np

SIZES = [9, 64, 64, 64, 3]
SHAPES = []
for _i in range(4):
    SHAPES.append(("W%d" % (_i + 1), (SIZES[_i + 1], SIZES[_i])))
    SHAPES.append(("b%d" % (_i + 1), (SIZES[_i + 1],)))
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat):
    flat = np.asarray(flat, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    return out


def pack(params):
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(a):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, X, act_bf16=False):
    """X [B, 9] standardised inputs -> standardised outputs [B, 3] and the
    pre-activations / activations of every layer.  act_bf16: round the inputs
    and every hidden activation to bfloat16 before it enters a product (the
    GPU's in-step inference)."""
    rnd = bf16 if act_bf16 else (lambda v: v)
    a = [rnd(np.asarray(X, dtype=np.float64))]
    zs = []
    for l in range(1, 5):
        z = a[-1] @ params["W%d" % l].T + params["b%d" % l]
        zs.append(z)
        a.append(rnd(silu(z)) if l < 4 else z)
    return a[-1], (zs, a)


def loss_and_grads(params, X, Y):
    """Mean squared error over the batch and the three standardised outputs,
    and its gradient with respect to every parameter (backpropagation)."""
    out, (zs, a) = forward(params, X)
    B = X.shape[0]
    diff = out - Y
    loss = float(np.mean(diff ** 2))
    g = {}
    d = 2.0 * diff / (B * out.shape[1])          # dL/dz4
    for l in range(4, 0, -1):
        g["W%d" % l] = d.T @ a[l - 1]
        g["b%d" % l] = d.sum(axis=0)
        if l > 1:
            d = (d @ params["W%d" % l]) * dsilu(zs[l - 2])
    return loss, g


class Adam:
    def __init__(self, beta1=0.9, beta2=0.999, eps=1e-8):
        self.b1, self.b2, self.eps = beta1, beta2, eps
        self.m, self.v, self.t = None, None, 0

    def step(self, flat, grad, lr):
        flat = np.asarray(flat, dtype=np.float64)
        grad = np.asarray(grad, dtype=np.float64)
        if self.m is None:
            self.m = np.zeros_like(flat)
            self.v = np.zeros_like(flat)
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * grad
        self.v = self.b2 * self.v + (1 - self.b2) * grad * grad
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return flat - lr * mh / (np.sqrt(vh) + self.eps)


def standardise(raw9, stats):
    """raw9 [B, 9] = (N^0, N^x, N^y, T^00, T^0x, T^0y, T^xx, T^xy, T^yy):
    divided by N^0, then standardised with stats = (mx[9], sx[9], my[3], sy[3])."""
    mx, sx = stats[0], stats[1]
    x = np.asarray(raw9, dtype=np.float64) / np.asarray(raw9, dtype=np.float64)[:, :1]
    return (x - mx) / sx


def predict(params, stats, raw9):
    """(eps/N^0, u_x, u_y) predicted for raw moments raw9 [B, 9]."""
    out, _ = forward(params, standardise(raw9, stats))
    return out * stats[3] + stats[2]
