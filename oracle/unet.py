"""FP64 reference of the warm-start 3D U-Net (test infrastructure only).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` alone; shares no code with
the GPU library and never imports it.

The paper has no learned component.  This network predicts a starting strain
field for the Lippmann-Schwinger iteration; the iteration itself still decides
convergence, so the network only changes eps^0 (the paper's schemes accept any
initial field).  Everything here is plain NumPy in float64, written out from
the definitions so that it can be read against them:

Fields are channel-last, shape (B, nz, ny, nx, C), periodic in the three grid
axes (the microstructures are periodic cells).

  conv3(x, w, b)[v, o] = b[o] + sum_t sum_c x[v + off(t), c] w[t, c, o]
      27 taps t = 9 (dz+1) + 3 (dy+1) + (dx+1), off(t) = (dz, dy, dx) in {-1,0,1}^3,
      indices taken modulo the grid (periodic padding).
  relu(y) = max(y, 0)
  pool(x)[Z, Y, X] = mean of the 2x2x2 children x[2Z+a, 2Y+b, 2X+c]
  up(x)[z, y, x] = x[z // 2, y // 2, x // 2]            (nearest, factor 2)

Architecture (4 levels, widths 16-32-64-128, two 3^3 convolutions per level,
each followed by relu):
  e1 = block(x0, 8 -> 16)          at N
  e2 = block(pool(e1), 16 -> 32)   at N/8
  e3 = block(pool(e2), 32 -> 64)   at N/64
  b  = block(pool(e3), 64 -> 128)  at N/512
  d3 = block([up(b), e3], 192 -> 64)
  d2 = block([up(d3), e2], 96 -> 32)
  d1 = block([up(d2), e1], 48 -> 16)
  p  = head(d1): p[v, o] = hb[o] + sum_c d1[v, c] hw[c, o]        (16 -> 6, linear)
  eps_pred = p - mean_v(p) + eps_bar                              (mean correction)
  loss = mean over samples, voxels and the 6 components of (eps_pred - eps)^2

Input features (8 channels): log10(E(x)) / 3, 10 (nu(x) - 0.3), and the six
components of eps_bar broadcast over the grid (tensor Voigt order 11, 22, 33,
23, 13, 12).  Output strain uses the same component order.

Parameters in canonical order (each weight followed by its bias):
  LAYERS below, then the head (16, 6) and (6,).

Storage precision: ``forward`` and ``loss_and_grad`` take an optional
``store`` function applied wherever the network keeps a tensor in memory
(input features, every convolution and pooling output, every activation
gradient handed from one layer to the next, up- and pool-gradients).  The
default keeps float64 throughout; ``bf16`` (round to nearest even to 8
significant bits) reproduces a network that stores those tensors in bfloat16
while accumulating at higher precision.

Pins (tests/test_oracle_unet.py): conv3 against a direct 7-loop sum and a
circular FFT convolution; pool/up adjointness; every gradient of the loss
against central finite differences on a small network and grid; Adam against
its closed-form first step and a hand-iterated scalar sequence; bf16 against
hand-rounded values.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "LAYERS", "TAPS", "param_shapes", "n_params", "init_params", "unflatten", "flatten",
    "conv3", "conv3_backward", "pool", "pool_backward", "up", "up_backward", "features",
    "forward", "loss_and_grad", "adam_step", "AdamState", "bf16",
]

# (name, c_in, c_out) of the fourteen 3^3 convolutions
LAYERS = [
    ("enc1a", 8, 16), ("enc1b", 16, 16),
    ("enc2a", 16, 32), ("enc2b", 32, 32),
    ("enc3a", 32, 64), ("enc3b", 64, 64),
    ("bota", 64, 128), ("botb", 128, 128),
    ("dec3a", 192, 64), ("dec3b", 64, 64),
    ("dec2a", 96, 32), ("dec2b", 32, 32),
    ("dec1a", 48, 16), ("dec1b", 16, 16),
]
HEAD = (16, 6)

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def param_shapes():
    shapes = []
    for name, ci, co in LAYERS:
        shapes.append((name + ".w", (27, ci, co)))
        shapes.append((name + ".b", (co,)))
    shapes.append(("head.w", HEAD))
    shapes.append(("head.b", (HEAD[1],)))
    return shapes


def n_params() -> int:
    return int(sum(np.prod(s) for _, s in param_shapes()))


def unflatten(flat):
    flat = np.asarray(flat, dtype=np.float64)
    out, o = {}, 0
    for name, shp in param_shapes():
        n = int(np.prod(shp))
        out[name] = flat[o:o + n].reshape(shp)
        o += n
    assert o == flat.size
    return out


def flatten(params) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], dtype=np.float64).reshape(-1) for name, _ in param_shapes()])


def init_params(rng: np.random.Generator):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases."""
    p = {}
    for name, shp in param_shapes():
        if name.endswith(".b"):
            p[name] = np.zeros(shp)
        else:
            fan_in = shp[0] * shp[1] if len(shp) == 3 else shp[0]
            p[name] = rng.standard_normal(shp) * np.sqrt(2.0 / fan_in)
    return p


# ---------------------------------------------------------------------------
# layers
# ---------------------------------------------------------------------------

def _ident(a):
    return a


def bf16(a):
    """Round to the nearest bfloat16 (8 significant bits, ties to even), returned
    as float64: x = m 2^e with |m| in [1, 2) is rounded to a multiple of 2^(e-7)."""
    a = np.asarray(a, dtype=np.float64)
    m, e = np.frexp(a)  # a = m 2^e, |m| in [0.5, 1)
    q = np.round(m * 256.0)  # numpy rounds halves to even
    return np.ldexp(q / 256.0, e)


def _shift(x, off):
    """x[v + off] on the periodic grid (axes 1, 2, 3 = z, y, x)."""
    dz, dy, dx = off
    return np.roll(x, shift=(-dz, -dy, -dx), axis=(1, 2, 3))


def conv3(x, w, b):
    y = np.zeros(x.shape[:4] + (w.shape[2],))
    for t, off in enumerate(TAPS):
        y += _shift(x, off) @ w[t]
    return y + b


def conv3_backward(x, w, gy):
    """Gradients of sum(gy * conv3(x, w, b)) with respect to x, w and b."""
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    for t, off in enumerate(TAPS):
        xs = _shift(x, off)
        gw[t] = xs.reshape(-1, x.shape[-1]).T @ gy.reshape(-1, gy.shape[-1])
        # y[v] gets x[v + off] w[t]  =>  x[u] receives gy[u - off] w[t]^T
        gx += _shift(gy @ w[t].T, tuple(-o for o in off))
    gb = gy.reshape(-1, gy.shape[-1]).sum(axis=0)
    return gx, gw, gb


def pool(x):
    B, nz, ny, nx, C = x.shape
    return x.reshape(B, nz // 2, 2, ny // 2, 2, nx // 2, 2, C).mean(axis=(2, 4, 6))


def pool_backward(g):
    return up(g) / 8.0


def up(x):
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def up_backward(g):
    B, nz, ny, nx, C = g.shape
    return g.reshape(B, nz // 2, 2, ny // 2, 2, nx // 2, 2, C).sum(axis=(2, 4, 6))


def features(phase, E, nu, macro):
    """(B, nz, ny, nx, 8) input of one batch: phase maps (B, nz, ny, nx) uint8,
    per-sample phase tables E[s], nu[s], and macro strains (B, 6)."""
    phase = np.asarray(phase)
    B = phase.shape[0]
    x = np.zeros(phase.shape + (8,))
    for s in range(B):
        Es = np.asarray(E[s], dtype=np.float64)
        ns = np.asarray(nu[s], dtype=np.float64)
        x[s, ..., 0] = np.log10(Es[phase[s]]) / 3.0
        x[s, ..., 1] = 10.0 * (ns[phase[s]] - 0.3)
        x[s, ..., 2:] = np.asarray(macro[s], dtype=np.float64)
    return x


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------

def _block(x, p, a, bname, cache, store):
    ya = store(np.maximum(conv3(x, p[a + ".w"], p[a + ".b"]), 0.0))
    yb = store(np.maximum(conv3(ya, p[bname + ".w"], p[bname + ".b"]), 0.0))
    cache[a] = (x, ya)
    cache[bname] = (ya, yb)
    return yb


def forward(params, x, macro, store=None):
    """Mean-corrected strain prediction (B, nz, ny, nx, 6) and the cache the
    backward pass needs."""
    s = store or _ident
    c = {"store": s}
    x = s(x)
    e1 = _block(x, params, "enc1a", "enc1b", c, s)
    e2 = _block(s(pool(e1)), params, "enc2a", "enc2b", c, s)
    e3 = _block(s(pool(e2)), params, "enc3a", "enc3b", c, s)
    bt = _block(s(pool(e3)), params, "bota", "botb", c, s)
    d3 = _block(np.concatenate([up(bt), e3], axis=-1), params, "dec3a", "dec3b", c, s)
    d2 = _block(np.concatenate([up(d3), e2], axis=-1), params, "dec2a", "dec2b", c, s)
    d1 = _block(np.concatenate([up(d2), e1], axis=-1), params, "dec1a", "dec1b", c, s)
    p = d1 @ params["head.w"] + params["head.b"]
    macro = np.asarray(macro, dtype=np.float64).reshape(-1, 1, 1, 1, 6)
    pred = p - p.mean(axis=(1, 2, 3), keepdims=True) + macro
    c["d1"] = d1
    return pred, c


def _block_backward(g, params, a, bname, cache, grads):
    s = cache["store"]
    ya_in, yb = cache[bname]
    g = g * (yb > 0)
    gx, gw, gb = conv3_backward(ya_in, params[bname + ".w"], g)
    grads[bname + ".w"], grads[bname + ".b"] = gw, gb
    x_in, ya = cache[a]
    g = s(gx) * (ya > 0)
    gx, gw, gb = conv3_backward(x_in, params[a + ".w"], g)
    grads[a + ".w"], grads[a + ".b"] = gw, gb
    return s(gx)


def loss_and_grad(params, x, macro, target, store=None):
    """Loss (mean squared error of the mean-corrected prediction) and its
    gradient with respect to every parameter."""
    pred, c = forward(params, x, macro, store)
    s = c["store"]
    diff = pred - target
    loss = float(np.mean(diff ** 2))
    g = 2.0 * diff / diff.size
    # through the mean correction: d p = g - mean_v(g)
    g = g - g.mean(axis=(1, 2, 3), keepdims=True)
    grads = {}
    d1 = c["d1"]
    grads["head.w"] = d1.reshape(-1, d1.shape[-1]).T @ g.reshape(-1, 6)
    grads["head.b"] = g.reshape(-1, 6).sum(axis=0)
    g = s(g @ params["head.w"].T)
    g = _block_backward(g, params, "dec1a", "dec1b", c, grads)
    g_up, g_e1 = g[..., :32], g[..., 32:]
    g = _block_backward(s(up_backward(g_up)), params, "dec2a", "dec2b", c, grads)
    g_up, g_e2 = g[..., :64], g[..., 64:]
    g = _block_backward(s(up_backward(g_up)), params, "dec3a", "dec3b", c, grads)
    g_up, g_e3 = g[..., :128], g[..., 128:]
    g = _block_backward(s(up_backward(g_up)), params, "bota", "botb", c, grads)
    g = _block_backward(s(pool_backward(g) + g_e3), params, "enc3a", "enc3b", c, grads)
    g = _block_backward(s(pool_backward(g) + g_e2), params, "enc2a", "enc2b", c, grads)
    _block_backward(s(pool_backward(g) + g_e1), params, "enc1a", "enc1b", c, grads)
    return loss, grads


# ---------------------------------------------------------------------------
# Adam (Kingma & Ba, 2015), bias-corrected moments
# ---------------------------------------------------------------------------

class AdamState:
    def __init__(self, n):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0


def adam_step(theta, grad, st: AdamState, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    st.t += 1
    st.m = beta1 * st.m + (1.0 - beta1) * grad
    st.v = beta2 * st.v + (1.0 - beta2) * grad * grad
    mhat = st.m / (1.0 - beta1 ** st.t)
    vhat = st.v / (1.0 - beta2 ** st.t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps)
