"""GPU parity of the warm-start U-Net (bf16 matrix-core kernels, fp32
accumulation) against the FP64 oracle (oracle/unet.py).

Tolerances, derived from the arithmetic:
* single convolution, bf16-exact inputs and weights: products of two bf16
  values are exact in fp32; each matrix-core step adds 32 of them to the fp32
  accumulator and there are at most 162 steps (192 channels), so
  |error| <= (162 + 32) 2^-24 sum|x w| < 2^-16 sum|x w| before the output is
  rounded to bf16 (unit roundoff 2^-8).  Tested: |y - y_ref| <= 2^-8 |y_ref|
  + 2^-16 sum|x w|, and at least 99.9% of the outputs equal bf16(y_ref) bit
  for bit (the rest sit within the accumulation error of a rounding
  boundary).
* weight gradients (fp32 outputs, sums over every voxel in fp32):
  |dw - dw_ref| <= 2^-14 sum_v |x| |g|.
* whole network (both sides use the same bf16-representable convolution
  weights): the network stores every activation and every activation
  gradient in bf16.  Against the oracle run with the same storage rounding
  (``store=bf16``) the sides differ only by fp32 vs fp64 accumulation, which
  moves a value across a bf16 rounding boundary rarely (single layers: more
  than 99.9% of outputs bit-identical) and then by one bf16 step.  A relu
  network at a random initialisation amplifies such one-step flips (relu
  states change and the mean-corrected output is a small difference of
  larger activations): the oracle itself moves by a few percent when its
  pre-rounding values are perturbed by 1e-6.  The bound is therefore three
  times that measured sensitivity (plus 0.2% of the output, 0.5% of a
  gradient): a wrong tap, transpose, mask, skip or pooling path moves the
  result by O(1).  Loss: <= 1e-3 relative.
"""
import numpy as np
import pytest

from microstructure import boolean_spheres
from oracle import unet as U

torch = pytest.importorskip("torch")
import paper_1412_8398_amd as fe  # noqa: E402

pytestmark = pytest.mark.gpu

FWD = [(8, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (64, 128), (128, 128), (192, 64), (96, 32), (48, 16)]


def bf16_bits(a):
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def from_bits(h):
    return (np.asarray(h).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16_round(a):
    return from_bits(bf16_bits(a))


def dev_bf16(a):
    return torch.from_numpy(bf16_bits(a).view(np.int16)).cuda().view(torch.bfloat16)


def host_bf16(t):
    return from_bits(t.contiguous().view(torch.int16).cpu().numpy().view(np.uint16))


def dev_f32(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32))).cuda()


def _conv_case(cin, cout, shape, seed):
    r = np.random.default_rng(seed)
    x = bf16_round(r.standard_normal(shape + (cin,)))
    w = bf16_round(r.standard_normal((27, cin, cout)) / np.sqrt(27 * cin))
    b = np.asarray(r.standard_normal(cout) * 0.1, dtype=np.float32).astype(np.float64)
    return x, w, b


# (1, 12, 12, 48) has a tile whose halo lies inside the grid (origin x 16,
# y 4, z 4): the staging path without periodic wrap; the others wrap
@pytest.mark.parametrize("cin,cout", FWD)
@pytest.mark.parametrize("shape", [(2, 5, 6, 20), (1, 8, 8, 32), (1, 12, 12, 48)])
def test_conv_forward(cin, cout, shape):
    x, w, b = _conv_case(cin, cout, shape, 100 * cin + cout)
    y = host_bf16(fe.conv3_forward(dev_bf16(x), dev_f32(w), dev_f32(b), relu=True))
    ref = np.maximum(U.conv3(x, w, b), 0.0)
    absum = U.conv3(np.abs(x), np.abs(w), np.zeros(cout))
    assert np.all(np.abs(y - ref) <= 2.0 ** -8 * np.abs(ref) + 2.0 ** -16 * absum)
    assert np.mean(y == U.bf16(ref)) >= 0.999


@pytest.mark.parametrize("cin,cout,ccoarse", [(48, 16, 32), (96, 32, 64), (192, 64, 128)])
@pytest.mark.parametrize("relu", [True, False])
@pytest.mark.parametrize("shape", [(2, 6, 8, 20), (1, 12, 12, 48)])
def test_decoder_layer_reads_its_concatenation_in_place(cin, cout, ccoarse, relu, shape):
    """The decoder layers of inference read [nearest upsampling of the coarse
    level, skip] in place; the result equals the layer on the materialised
    concatenation bit for bit (same staged values, same products), and the
    oracle on that concatenation within the layer bound.  Shapes (B, nz, ny,
    nx), even: tiles ragged in y and x, and one tile with its halo inside the
    grid."""
    r = np.random.default_rng(cin + cout)
    _, w, b = _conv_case(cin, cout, shape, 11 * cin + cout)
    coarse = bf16_round(r.standard_normal((shape[0], shape[1] // 2, shape[2] // 2, shape[3] // 2, ccoarse)))
    skip = bf16_round(r.standard_normal(shape + (cin - ccoarse,)))
    up = coarse.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)
    cat = np.concatenate([up, skip], axis=-1)
    y = fe.conv3_forward_cat(dev_bf16(coarse), dev_bf16(skip), dev_f32(w), dev_f32(b), relu=relu)
    y_cat = fe.conv3_forward(dev_bf16(cat), dev_f32(w), dev_f32(b), relu=relu)
    assert torch.equal(y.view(torch.int16), y_cat.view(torch.int16))
    ref = U.conv3(cat, w, b)
    if relu:
        ref = np.maximum(ref, 0.0)
    absum = U.conv3(np.abs(cat), np.abs(w), np.zeros(cout))
    assert np.all(np.abs(host_bf16(y) - ref) <= 2.0 ** -8 * np.abs(ref) + 2.0 ** -16 * absum)


@pytest.mark.parametrize("cin,cout", [s for s in FWD if s[0] % 16 == 0])
@pytest.mark.parametrize("shape", [(2, 5, 6, 20), (1, 12, 12, 48)])
def test_conv_backward_data(cin, cout, shape):
    r = np.random.default_rng(7 * cin + cout)
    _, w, _ = _conv_case(cin, cout, shape, cin + 3 * cout)
    dy = bf16_round(r.standard_normal(shape + (cout,)))
    ymask = bf16_round(r.standard_normal(shape + (cout,)))
    ymask[..., 0] = 0.0  # a relu output that is exactly zero blocks the gradient
    g = dy * (ymask > 0)
    dx = host_bf16(fe.conv3_backward_data(dev_bf16(dy), dev_f32(w), dev_bf16(ymask)))
    ref = U.conv3_backward(np.zeros(shape + (cin,)), w, g)[0]
    absum = U.conv3_backward(np.zeros(shape + (cin,)), np.abs(w), np.abs(g))[0]
    assert np.all(np.abs(dx - ref) <= 2.0 ** -8 * np.abs(ref) + 2.0 ** -16 * absum)
    assert np.mean(dx == U.bf16(ref)) >= 0.999


@pytest.mark.parametrize("cin,cout", FWD)
def test_conv_backward_weight(cin, cout):
    shape = (2, 8, 6, 20)
    r = np.random.default_rng(11 * cin + cout)
    x, _, _ = _conv_case(cin, cout, shape, 5 * cin + cout)
    dy = bf16_round(r.standard_normal(shape + (cout,)))
    ymask = bf16_round(r.standard_normal(shape + (cout,)))
    g = dy * (ymask > 0)
    dw, db = fe.conv3_backward_weight(dev_bf16(x), dev_bf16(dy), dev_bf16(ymask))
    dw, db = dw.cpu().numpy().astype(np.float64), db.cpu().numpy().astype(np.float64)
    _, rw, rb = U.conv3_backward(x, np.zeros((27, cin, cout)), g)
    _, aw, ab = U.conv3_backward(np.abs(x), np.zeros((27, cin, cout)), np.abs(g))
    assert np.all(np.abs(dw - rw) <= 2.0 ** -14 * aw + 1e-30)
    assert np.all(np.abs(db - rb) <= 2.0 ** -14 * ab + 1e-30)


def _net_case(shape=(16, 16, 16), B=2, seed=3, weight_scale=1.0, bias=None):
    """Parameters (convolution weights bf16-representable, as the network
    computes with them), a batch of two-phase microstructures and macro strains."""
    r = np.random.default_rng(seed)
    p = U.init_params(r)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.05 * r.standard_normal(p[k].shape) if bias is None else np.full(p[k].shape, float(bias))
        elif k != "head.w":
            p[k] = bf16_round(weight_scale * p[k])
    flat32 = U.flatten(p).astype(np.float32)
    p = U.unflatten(flat32.astype(np.float64))
    phases, E, nu, macro = [], [], [], []
    for s in range(B):
        ph, _ = boolean_spheres(shape, 2.5, 0.25, 40 + s)
        phases.append(ph)
        E.append([1.0, 10.0 ** (1 + s)])
        nu.append([0.3, 0.25 + 0.05 * s])
        macro.append(r.standard_normal(6) * 0.5)
    return p, flat32, np.stack(phases), E, nu, np.array(macro)


def _to_oracle(a):  # (B, 6, nz, ny, nx) -> (B, nz, ny, nx, 6)
    return np.moveaxis(a, 1, -1)


def _jitter_store(seed):
    """bf16 storage after a relative perturbation of 1e-6, the size of the
    float32-versus-float64 accumulation differences of one convolution (about
    (K-steps + 32) 2^-24 of the absolute sum, see the single-layer bounds)."""
    rng = np.random.default_rng(seed)
    return lambda a: U.bf16(a * (1.0 + 1e-6 * rng.standard_normal(np.shape(a))))


def test_network_prediction_matches_oracle():
    p, flat32, phase, E, nu, macro = _net_case(shape=(16, 24, 8))
    net = fe.UNet()
    net.set_params(flat32)
    assert np.array_equal(net.get_params(), flat32)
    out, sec = net.predict(torch.from_numpy(phase).cuda(), E, nu, macro)
    torch.cuda.synchronize()
    got = _to_oracle(out.cpu().numpy().astype(np.float64))
    x = U.features(phase, E, nu, macro)
    ref16, _ = U.forward(p, x, macro, store=U.bf16)
    ref64, _ = U.forward(p, x, macro)
    alt, _ = U.forward(p, x, macro, store=_jitter_store(1))
    fl = np.linalg.norm(ref64 - macro[:, None, None, None, :])
    sens = np.linalg.norm(alt - ref16)
    assert np.linalg.norm(got - ref16) <= 3.0 * sens + 2e-3 * fl, (np.linalg.norm(got - ref16) / fl, sens / fl)
    assert np.linalg.norm(got - ref64) <= 3.0 * sens + 3e-2 * fl
    assert np.allclose(got.mean(axis=(1, 2, 3)), macro, atol=1e-5)
    assert sec > 0
    net.close()


def test_network_loss_and_gradients_match_oracle():
    p, flat32, phase, E, nu, macro = _net_case()
    r = np.random.default_rng(9)
    target = macro[:, :, None, None, None] + 0.3 * r.standard_normal((2, 6) + phase.shape[1:])
    net = fe.UNet()
    net.set_params(flat32)
    loss = net.loss_grad(torch.from_numpy(phase).cuda(), E, nu, macro, dev_f32(target))
    grads = U.unflatten(net.get_grads().astype(np.float64))
    x = U.features(phase, E, nu, macro)
    tg = _to_oracle(target)
    ref_loss, ref_g = U.loss_and_grad(p, x, macro, tg, store=U.bf16)
    _, alt_g = U.loss_and_grad(p, x, macro, tg, store=_jitter_store(2))
    assert abs(loss - ref_loss) <= 1e-3 * ref_loss
    # the head bias cannot change the mean-corrected output: its exact gradient
    # is zero; in fp32 it is a sum of N terms of size 2 |diff| / (6 B N) whose
    # own mean was removed in fp32 (relative 2^-24 of |eps_bar|)
    assert np.linalg.norm(grads["head.b"]) <= 2.0 ** -18
    bad = {}
    for name, _ in U.param_shapes():
        if name == "head.b":
            continue
        ref = np.linalg.norm(ref_g[name])
        err = np.linalg.norm(grads[name] - ref_g[name])
        sens = np.linalg.norm(alt_g[name] - ref_g[name])
        if err > 3.0 * sens + 5e-3 * ref:
            bad[name] = (err / ref, sens / ref)
    assert not bad, bad
    loss2 = net.loss_grad(torch.from_numpy(phase).cuda(), E, nu, macro, dev_f32(target))
    assert loss2 == loss and np.array_equal(net.get_grads(), U.flatten(grads).astype(np.float32))  # bitwise
    net.close()


def test_training_steps_reduce_the_loss():
    _, flat32, phase, E, nu, macro = _net_case(seed=5)
    # a target correlated with the microstructure
    target = np.repeat(macro[:, :, None, None, None], 1, axis=0) * (1.0 + 0.5 * (phase[:, None] == 1))
    target = target - target.mean(axis=(2, 3, 4), keepdims=True) + macro[:, :, None, None, None]
    # lr 5e-4: the loss falls from the first step.  At 2e-3 it rose elevenfold
    # within two steps, and whether it then recovered or diverged depended on
    # the last-bit rounding of the weight-gradient sums (measured with two
    # summation orders: 0.0136 and 0.958 after 40 steps).
    net = fe.UNet(lr=5e-4)
    net.set_params(flat32)
    ph = torch.from_numpy(phase).cuda()
    tg = dev_f32(target)
    losses = [net.train_step(ph, E, nu, macro, tg) for _ in range(40)]
    assert losses[1] < losses[0], losses
    assert losses[-1] < 0.5 * losses[0], losses
    net.close()


# ---------------------------------------------------------------------------
# against the plain float64 oracle (no storage rounding), and Adam
# ---------------------------------------------------------------------------

WEIGHTS = __import__("os").path.join(__import__("os").path.dirname(__file__), "..", "paper_1412_8398_amd", "weights",
                                     "unet_warmstart.npy")


def _trained_case(shape=(32, 32, 32)):
    """The committed warm-start network with bf16-representable convolution
    weights (the head stays float32, as on the GPU), on two Boolean cells of
    contrast 10 and 1000 under unit normal loads."""
    flat = np.load(WEIGHTS).astype(np.float64)
    p = U.unflatten(flat)
    for name, _ in U.param_shapes():
        if name.endswith(".w") and name != "head.w":
            p[name] = bf16_round(p[name])
    flat32 = U.flatten(p).astype(np.float32)
    p = U.unflatten(flat32.astype(np.float64))
    phases, E, nu, macro = [], [], [], []
    for s in range(2):
        ph, _ = boolean_spheres(shape, 4.0, 0.25, 40 + s)
        phases.append(ph)
        E.append([1.0, 10.0 ** (1 + 2 * s)])
        nu.append([0.3, 0.25 + 0.05 * s])
        m = np.zeros(6)
        m[3 * s] = 1.0
        macro.append(m)
    return p, flat32, np.stack(phases), E, nu, np.array(macro)


def _storage_noise(seed):
    """The bf16 storage bound as noise: every stored tensor multiplied by
    1 + d with d uniform in [-2^-9, 2^-9] (round to nearest with 8
    significant bits changes a value by at most 2^-9 of itself)."""
    g = np.random.default_rng(seed)
    return lambda a: a * (1.0 + 2.0 ** -9 * g.uniform(-1.0, 1.0, np.shape(a)))


def test_network_prediction_matches_the_plain_oracle():
    """The GPU prediction against the float64 oracle without any storage
    rounding.  The GPU stores every activation in bf16 (relative error at
    most 2^-9 per stored value, plus fp32 accumulation, 2^-16 of the
    absolute sums, negligible beside it).  Propagated through the network
    to first order (relu is 1-Lipschitz, so a state that flips near zero
    moves its value by no more than the perturbation), these errors add up
    like independent noise; the oracle run with the storage bound injected
    as noise (three draws) measures their size sigma, and the bound is
    3 sigma.  A wrong tap, transpose, skip or pooling path moves the result
    by O(1) of the fluctuation."""
    p, flat32, phase, E, nu, macro = _trained_case()
    net = fe.UNet()
    net.set_params(flat32)
    out, _ = net.predict(torch.from_numpy(phase).cuda(), E, nu, macro)
    torch.cuda.synchronize()
    got = _to_oracle(out.cpu().numpy().astype(np.float64))
    x = U.features(phase, E, nu, macro)
    ref, _ = U.forward(p, x, macro)
    fl = np.linalg.norm(ref - macro[:, None, None, None, :])
    sigma = max(np.linalg.norm(U.forward(p, x, macro, store=_storage_noise(sd))[0] - ref) for sd in (1, 2, 3))
    err = np.linalg.norm(got - ref)
    print(f"prediction vs plain oracle: {err / fl:.3e} of the fluctuation, storage-noise sigma {sigma / fl:.3e}",
          flush=True)
    assert sigma <= 0.05 * fl  # the bound is tight enough to catch an O(1) slip
    assert err <= 3.0 * sigma
    net.close()


def test_network_gradients_match_the_plain_oracle():
    """Loss and every parameter gradient against the float64 oracle without
    storage rounding; the bound is 3 sigma per tensor, sigma from the
    storage-bound noise injected into the forward and backward stores of the
    oracle (as above, four draws).  The head bias has an exact gradient of zero (the mean
    correction removes it)."""
    p, flat32, phase, E, nu, macro = _trained_case(shape=(16, 16, 16))
    r = np.random.default_rng(9)
    target = macro[:, :, None, None, None] + 0.3 * r.standard_normal((2, 6) + phase.shape[1:])
    net = fe.UNet()
    net.set_params(flat32)
    loss = net.loss_grad(torch.from_numpy(phase).cuda(), E, nu, macro, dev_f32(target))
    grads = U.unflatten(net.get_grads().astype(np.float64))
    x = U.features(phase, E, nu, macro)
    tg = _to_oracle(target)
    ref_loss, ref_g = U.loss_and_grad(p, x, macro, tg)
    noisy = [U.loss_and_grad(p, x, macro, tg, store=_storage_noise(sd)) for sd in (3, 4, 5, 6)]
    sig_loss = max(abs(nl - ref_loss) for nl, _ in noisy)
    assert abs(loss - ref_loss) <= 3.0 * sig_loss + 1e-6 * ref_loss
    bad = {}
    for name, _ in U.param_shapes():
        if name == "head.b":
            continue
        ref = np.linalg.norm(ref_g[name])
        sig = max(np.linalg.norm(ng[name] - ref_g[name]) for _, ng in noisy)
        err = np.linalg.norm(grads[name] - ref_g[name])
        if not (err <= 3.0 * sig + 1e-6 * ref and sig <= 0.05 * ref):
            bad[name] = (err / ref, sig / ref)
    assert not bad, bad
    net.close()


@pytest.mark.parametrize("steps", [1, 10])
def test_adam_update_matches_oracle(steps):
    """fe_unet_train_step's parameter update against the oracle's Adam
    (bias-corrected moments) fed with the gradients the GPU computed (read
    back after each step), in float64.  The GPU keeps float32 master weights
    and moments: per step the update lr mhat/(sqrt(vhat) + eps) carries a
    relative rounding of a few float32 units (moments, bias corrections,
    square root, division: at most 16 u, u = 2^-24, with the moments' own
    error growing by 2 u per step), and the stored weight one rounding of
    u |theta|.  Bound after n steps, per element:
      |theta_gpu - theta_ref| <= n u |theta_ref|
                                 + (16 + 2 n) u sum_k lr mabs_k / (sqrt(vhat_k) + eps)
    with mabs the first moment of |g| (a missing bias correction, swapped
    betas or eps inside the square root are off by far more)."""
    _, flat32, phase, E, nu, macro = _net_case(seed=6)
    r = np.random.default_rng(12)
    target = macro[:, :, None, None, None] + 0.3 * r.standard_normal((2, 6) + phase.shape[1:])
    lr, b1, b2, eps = 2e-3, 0.9, 0.999, 1e-8
    net = fe.UNet(lr=lr, beta1=b1, beta2=b2, adam_eps=eps)
    net.set_params(flat32)
    ph, tg = torch.from_numpy(phase).cuda(), dev_f32(target)
    theta = flat32.astype(np.float64)
    st = U.AdamState(theta.size)
    mabs = np.zeros_like(theta)
    budget = np.zeros_like(theta)
    u = 2.0 ** -24
    for k in range(1, steps + 1):
        net.train_step(ph, E, nu, macro, tg)
        g = net.get_grads().astype(np.float64)
        theta = U.adam_step(theta, g, st, lr=lr, beta1=b1, beta2=b2, eps=eps)
        mabs = b1 * mabs + (1.0 - b1) * np.abs(g)
        vhat = st.v / (1.0 - b2 ** k)
        budget += lr * (mabs / (1.0 - b1 ** k)) / (np.sqrt(vhat) + eps)
    got = net.get_params().astype(np.float64)
    bound = steps * u * np.abs(theta) + (16 + 2 * steps) * u * budget
    moved = np.abs(theta - flat32)
    assert np.median(moved[moved > 0]) > 1e3 * np.median(bound[moved > 0])  # the update is far above the bound
    assert np.all(np.abs(got - theta) <= bound), float(np.max(np.abs(got - theta) / np.maximum(bound, 1e-300)))
    net.close()
