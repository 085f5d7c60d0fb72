"""Pins of the oracle's warm-start network primitives.

The convolution is checked against special cases with closed forms (a
delta input returns the flipped kernel, a constant input returns the tap
sum), against PyTorch's CPU convolution of a replicate-padded volume (the
operation reduces to that library routine), the backward passes against the
adjoint identities <conv(X), dY> = <X, dconv(dY)> = <W, wgrad(X, dY)>, and
the whole loss gradient against central finite differences.  Adam's first
step has the closed form theta - lr * g / (|g| + eps).
"""
import numpy as np
import pytest

import oracle
import synth


def tap_index(dx, dy, dz):
    return (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)


def test_delta_input_returns_flipped_kernel():
    n = 5
    cin, cout = 1, 2
    rng = np.random.default_rng(0)
    W = rng.standard_normal(27 * cin * cout)
    X = np.zeros(n**3)
    c = 2 + n * (2 + n * 2)
    X[c] = 1.0
    Y = oracle.conv3d_fwd(n, X, W, cin, cout).reshape(n, n, n, cout)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                # Y[v] = sum_t X[v + d_t] W[t]: nonzero where v + d_t = centre
                got = Y[2 - dz, 2 - dy, 2 - dx]
                np.testing.assert_array_equal(got, W.reshape(27, cin, cout)[tap_index(dx, dy, dz), 0])


def test_constant_input_returns_tap_sum():
    n = 4
    cin, cout = 3, 2
    rng = np.random.default_rng(1)
    W = rng.standard_normal(27 * cin * cout)
    X = np.full(n**3 * cin, 0.75)
    Y = oracle.conv3d_fwd(n, X, W, cin, cout).reshape(-1, cout)
    np.testing.assert_allclose(Y, np.broadcast_to(0.75 * W.reshape(27, cin, cout).sum((0, 1)), Y.shape),
                               rtol=1e-13)


def test_matches_torch_replicate_conv():
    torch = pytest.importorskip("torch")
    import torch.nn.functional as F
    dims = (6, 5, 4)
    cin, cout = 3, 4
    rng = np.random.default_rng(2)
    X = rng.standard_normal(np.prod(dims) * cin)
    W = rng.standard_normal(27 * cin * cout)
    Y = oracle.conv3d_fwd(dims, X, W, cin, cout)
    nx, ny, nz = dims
    xt = torch.from_numpy(X.reshape(nz, ny, nx, cin)).permute(3, 0, 1, 2)[None]
    wt = torch.from_numpy(W.reshape(3, 3, 3, cin, cout)).permute(4, 3, 0, 1, 2).contiguous()
    yt = F.conv3d(F.pad(xt, (1, 1, 1, 1, 1, 1), mode="replicate"), wt)
    ref = yt[0].permute(1, 2, 3, 0).reshape(-1).numpy()
    np.testing.assert_allclose(Y, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dims,cin,cout", [((5, 4, 3), 2, 3), ((3, 3, 3), 1, 4), ((4, 2, 5), 4, 1)])
def test_adjoint_identities(dims, cin, cout):
    rng = np.random.default_rng(3)
    nvox = int(np.prod(dims))
    X = rng.standard_normal(nvox * cin)
    W = rng.standard_normal(27 * cin * cout)
    dY = rng.standard_normal(nvox * cout)
    lhs = np.dot(oracle.conv3d_fwd(dims, X, W, cin, cout), dY)
    np.testing.assert_allclose(np.dot(X, oracle.conv3d_bwd_data(dims, dY, W, cin, cout)), lhs, rtol=1e-12)
    np.testing.assert_allclose(np.dot(W, oracle.conv3d_bwd_weight(dims, X, dY, cin, cout)), lhs, rtol=1e-12)


def test_loss_gradient_finite_differences():
    dims = (5, 4, 3)
    shapes = synth.net_layer_shapes(channels=3, layers=4)
    theta = synth.net_init(7, channels=3, layers=4).astype(np.float64)
    rng = np.random.default_rng(4)
    x = rng.standard_normal(int(np.prod(dims)))
    tgt = rng.standard_normal(int(np.prod(dims)))
    loss, grad = oracle.net_loss_grad(dims, x, tgt, theta, shapes)
    eps = 1e-6
    idx = rng.choice(len(theta), size=40, replace=False)
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (oracle.net_loss_grad(dims, x, tgt, tp, shapes)[0]
              - oracle.net_loss_grad(dims, x, tgt, tm, shapes)[0]) / (2 * eps)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(grad[i])), (i, fd, grad[i])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps = 1e-3, 1e-8
    th1, m, v = oracle.adam(th, np.zeros(50), np.zeros(50), g, lr, 1, eps=eps)
    np.testing.assert_allclose(th1, th - lr * g / (np.abs(g) + eps), rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-13)


def test_round_bf16_definition():
    """bfloat16 rounding (the network's activation storage): exact cases of
    round-to-nearest-even at 8 significant bits, sign symmetry, float32's
    subnormal spacing, and agreement with a bit-level version (keep the top
    16 bits of the float32 pattern after adding 0x7FFF plus the kept lsb)."""
    r = oracle.round_bf16
    u = 2.0**-7  # spacing just above 1
    cases = {1.0: 1.0, 1 + u / 2: 1.0, 1 + 3 * u / 2: 1 + 2 * u, 1 + u: 1 + u, 3.0: 3.0,
             -(1 + 3 * u / 2): -(1 + 2 * u), 2.0**-130: 2.0**-130, 1.5 * 2.0**-133: 2.0**-132,
             2.5 * 2.0**-133: 2.0**-132, 0.0: 0.0}
    got = r(np.array(list(cases.keys())))
    np.testing.assert_array_equal(got, np.array(list(cases.values())))
    rng = np.random.default_rng(5)
    a = (rng.standard_normal(20000) * np.exp(rng.uniform(-60, 60, 20000))).astype(np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    bits = ((bits + 0x7FFF + ((bits >> 16) & 1)) >> 16) << 16
    want = bits.astype(np.uint32).view(np.float32).astype(np.float64)
    np.testing.assert_array_equal(r(a), want)
    np.testing.assert_array_equal(r(r(a)), r(a))



def test_training_pair_definition():
    """input has unit RMS, target zero mean and unit RMS; both are invariant
    under positive scaling of b and p, and p + const gives the same target;
    zero b and constant p give zeros."""
    rng = np.random.default_rng(4)
    b = rng.standard_normal(1000) * 3.0 + 0.5
    p = rng.standard_normal(1000) * 40.0 + 7.0
    x, t = oracle.training_pair(b, p)
    assert x.dtype == np.float32 and t.dtype == np.float32
    assert abs(np.sqrt(np.mean(x.astype(np.float64) ** 2)) - 1.0) < 1e-6
    assert abs(np.mean(t.astype(np.float64))) < 1e-6
    assert abs(np.sqrt(np.mean(t.astype(np.float64) ** 2)) - 1.0) < 1e-6
    x2, t2 = oracle.training_pair(5.0 * b, 0.25 * p + 3.0)
    np.testing.assert_allclose(x2, x, rtol=1e-6)
    np.testing.assert_allclose(t2, t, rtol=1e-5, atol=1e-6)
    # ordering is preserved: the target is an increasing affine map of p
    assert np.all(np.argsort(t, kind="stable") == np.argsort(p, kind="stable"))
    z, c = oracle.training_pair(np.zeros(10), np.full(10, 2.0))
    assert not z.any() and not c.any()
