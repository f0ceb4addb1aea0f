"""Pins of the FP64 U-Net reference (oracle/unet.py) against definitions and
independent computations: direct loops, FFT circular correlation, adjoint
identities, central finite differences and closed-form Adam steps."""
import numpy as np
import pytest

from oracle import unet as U


def _rng(seed=0):
    return np.random.default_rng(seed)


def test_conv3_matches_a_direct_loop_sum():
    r = _rng(1)
    B, nz, ny, nx, ci, co = 2, 3, 4, 5, 2, 3
    x = r.standard_normal((B, nz, ny, nx, ci))
    w = r.standard_normal((27, ci, co))
    b = r.standard_normal(co)
    y = U.conv3(x, w, b)
    ref = np.zeros_like(y)
    for s in range(B):
        for z in range(nz):
            for yy in range(ny):
                for xx in range(nx):
                    for o in range(co):
                        acc = b[o]
                        for dz in (-1, 0, 1):
                            for dy in (-1, 0, 1):
                                for dx in (-1, 0, 1):
                                    t = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)
                                    for c in range(ci):
                                        acc += x[s, (z + dz) % nz, (yy + dy) % ny, (xx + dx) % nx, c] * w[t, c, o]
                        ref[s, z, yy, xx, o] = acc
    assert np.allclose(y, ref, rtol=1e-13, atol=1e-13)


def test_conv3_matches_fft_circular_correlation():
    r = _rng(2)
    nz, ny, nx, ci, co = 6, 5, 4, 3, 2
    x = r.standard_normal((1, nz, ny, nx, ci))
    w = r.standard_normal((27, ci, co))
    y = U.conv3(x, w, np.zeros(co))
    for o in range(co):
        acc = np.zeros((nz, ny, nx), dtype=complex)
        for c in range(ci):
            k = np.zeros((nz, ny, nx))
            for t, (dz, dy, dx) in enumerate(U.TAPS):
                k[dz % nz, dy % ny, dx % nx] += w[t, c, o]
            # y[v] = sum_u x[v + u] k[u]  <=>  Y = X conj(K) for real k
            acc += np.fft.fftn(x[0, ..., c]) * np.conj(np.fft.fftn(k))
        assert np.allclose(np.fft.ifftn(acc).real, y[0, ..., o], rtol=1e-12, atol=1e-12)


def test_conv3_backward_is_the_adjoint():
    r = _rng(3)
    x = r.standard_normal((2, 4, 6, 4, 3))
    w = r.standard_normal((27, 3, 5))
    gy = r.standard_normal((2, 4, 6, 4, 5))
    gx, gw, gb = U.conv3_backward(x, w, gy)
    # <conv3(x), gy> is linear in x, in w and in b
    dx = r.standard_normal(x.shape)
    assert np.isclose(np.sum(U.conv3(dx, w, np.zeros(5)) * gy), np.sum(dx * gx), rtol=1e-12)
    dw = r.standard_normal(w.shape)
    assert np.isclose(np.sum(U.conv3(x, dw, np.zeros(5)) * gy), np.sum(dw * gw), rtol=1e-12)
    db = r.standard_normal(5)
    assert np.isclose(np.sum((U.conv3(x, w, db) - U.conv3(x, w, np.zeros(5))) * gy), np.sum(db * gb), rtol=1e-12)


def test_pool_and_up_adjoints_and_values():
    r = _rng(4)
    a = r.standard_normal((2, 4, 6, 8, 3))
    b = r.standard_normal((2, 2, 3, 4, 3))
    assert np.isclose(np.sum(U.pool(a) * b), np.sum(a * U.pool_backward(b)), rtol=1e-12)
    assert np.isclose(np.sum(U.up(b) * a), np.sum(b * U.up_backward(a)), rtol=1e-12)
    assert np.isclose(U.pool(a)[1, 1, 2, 3, 2], a[1, 2:4, 4:6, 6:8, 2].mean())
    assert U.up(b)[0, 3, 5, 7, 1] == b[0, 1, 2, 3, 1]


def test_features_channels():
    phase = np.array([[[[0, 1], [1, 0]], [[1, 1], [0, 0]]]], dtype=np.uint8)
    x = U.features(phase, [[1.0, 1000.0]], [[0.25, 0.35]], [[0.1, 0.2, 0.3, 0.4, 0.5, 0.6]])
    assert x.shape == (1, 2, 2, 2, 8)
    assert x[0, 0, 0, 1, 0] == pytest.approx(1.0) and x[0, 0, 0, 0, 0] == 0.0
    assert x[0, 0, 0, 1, 1] == pytest.approx(0.5) and x[0, 0, 0, 0, 1] == pytest.approx(-0.5)
    assert np.all(x[0, 1, 1, 1, 2:] == np.array([0.1, 0.2, 0.3, 0.4, 0.5, 0.6]))


def test_prediction_mean_equals_the_applied_strain():
    r = _rng(5)
    p = U.init_params(r)
    x = r.standard_normal((2, 8, 8, 8, 8))
    macro = r.standard_normal((2, 6))
    pred, _ = U.forward(p, x, macro)
    assert np.allclose(pred.mean(axis=(1, 2, 3)), macro, atol=1e-14)


def test_every_gradient_matches_central_differences():
    """Central differences (h = 1e-6) of the loss for three entries of every
    parameter tensor, and along one random direction of all parameters."""
    r = _rng(6)
    p = U.init_params(r)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.1 * r.standard_normal(p[k].shape)
    x = r.standard_normal((2, 8, 8, 8, 8))
    macro = r.standard_normal((2, 6))
    target = r.standard_normal((2, 8, 8, 8, 6))
    loss, g = U.loss_and_grad(p, x, macro, target)
    h = 1e-6

    def L(pp):
        pred, _ = U.forward(pp, x, macro)
        return float(np.mean((pred - target) ** 2))

    for name, shp in U.param_shapes():
        flat = p[name].reshape(-1)
        for idx in r.choice(flat.size, size=min(3, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = L(p)
            flat[idx] = old - h
            lm = L(p)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3), (name, idx, fd, an)
    theta = U.flatten(p)
    d = r.standard_normal(theta.size)
    fd = (L(U.unflatten(theta + h * d)) - L(U.unflatten(theta - h * d))) / (2 * h)
    an = float(np.dot(U.flatten(g), d))
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_adam_first_step_and_a_scalar_sequence():
    st = U.AdamState(3)
    th = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    new = U.adam_step(th, g, st, lr=0.01, eps=0.0)
    assert np.allclose(new, th - 0.01 * np.sign(g), rtol=0, atol=1e-15)  # bias-corrected first step
    # three steps on a scalar, moments iterated by hand
    st = U.AdamState(1)
    t = np.array([0.0])
    m = v = 0.0
    ref = 0.0
    for k, gk in enumerate([1.0, -0.5, 2.0], start=1):
        t = U.adam_step(t, np.array([gk]), st, lr=0.1, beta1=0.9, beta2=0.999, eps=1e-8)
        m = 0.9 * m + 0.1 * gk
        v = 0.999 * v + 0.001 * gk * gk
        ref -= 0.1 * (m / (1 - 0.9 ** k)) / (np.sqrt(v / (1 - 0.999 ** k)) + 1e-8)
        assert t[0] == pytest.approx(ref, rel=1e-14)


def test_parameter_count():
    n = sum(27 * ci * co + co for _, ci, co in U.LAYERS) + 16 * 6 + 6
    assert U.n_params() == n == 1_462_694


def test_bf16_rounding_by_hand():
    one = 1.0
    assert U.bf16(one + 2.0 ** -8) == 1.0                      # tie -> even
    assert U.bf16(one + 3 * 2.0 ** -8) == one + 2.0 ** -6      # tie -> even (upward)
    assert U.bf16(one + 2.0 ** -8 + 2.0 ** -20) == one + 2.0 ** -7
    assert U.bf16(-(one + 2.0 ** -8 + 2.0 ** -20)) == -(one + 2.0 ** -7)
    assert U.bf16(2.0 - 2.0 ** -8) == 2.0                      # tie -> even, carries into the next binade
    assert U.bf16(0.0) == 0.0
    r = _rng(8).standard_normal(1000) * 10.0 ** _rng(9).uniform(-30, 30, 1000)
    q = U.bf16(r)
    assert np.all(np.abs(q - r) <= 2.0 ** -8 * np.abs(r))  # unit roundoff of 8 significant bits
    # 8 significant bits: q / 2^(floor(log2 |q|) - 7) is an integer
    e = np.floor(np.log2(np.abs(q)))
    assert np.all(np.ldexp(q, (7 - e).astype(int)) == np.round(np.ldexp(q, (7 - e).astype(int))))


def test_storage_rounding_hook_defaults_to_float64():
    r = _rng(10)
    p = U.init_params(r)
    x = r.standard_normal((1, 8, 8, 8, 8))
    macro = r.standard_normal((1, 6))
    a, _ = U.forward(p, x, macro)
    b, _ = U.forward(p, x, macro, store=lambda t: t)
    c, _ = U.forward(p, x, macro, store=U.bf16)
    assert np.array_equal(a, b)
    assert 0 < np.linalg.norm(c - a) <= 3e-2 * np.linalg.norm(a - macro.reshape(1, 1, 1, 1, 6))
