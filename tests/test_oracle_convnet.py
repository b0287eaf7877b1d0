"""Pins of the learned-guess network oracle (oracle/convnet.py).

* the convolution equals scipy.ndimage.correlate with zero padding (an
  independent implementation) and a brute-force loop on a tiny input;
* the data and weight backward passes are the adjoints of the forward map
  (inner-product identities), and pool / up are adjoint up to the factor 8;
* the gradient of the whole network's loss matches central finite
  differences in FP64 (skips, masks, pooling and up-sampling included);
* the first Adam step has the closed form -lr g / (|g| + eps);
* bf16 rounding agrees with torch's bfloat16 conversion;
* a zero network gives exactly the linear extrapolation.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import convnet as CN
from paper_2009_02171_amd import inputs


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_conv_matches_scipy_correlate():
    x = _rand((2, 5, 6, 7, 3), 0)
    w = _rand((4, 27, 3), 1)
    b = _rand(4, 2)
    y = CN.conv_fwd(x, w, b)
    for p in range(2):
        for co in range(4):
            ref = np.full(x.shape[1:4], b[co])
            for ci in range(3):
                ref += ndi.correlate(x[p, ..., ci], w[co, :, ci].reshape(3, 3, 3), mode="constant", cval=0.0)
            np.testing.assert_allclose(y[p, ..., co], ref, rtol=0, atol=1e-12)


def test_conv_brute_force_tiny():
    x = _rand((1, 3, 2, 4, 2), 3)
    w = _rand((2, 27, 2), 4)
    y = CN.conv_fwd(x, w)
    D, H, W = x.shape[1:4]
    for d in range(D):
        for h in range(H):
            for i in range(W):
                for co in range(2):
                    acc = 0.0
                    for t in range(27):
                        dz, dy, dx = t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1
                        if 0 <= d + dz < D and 0 <= h + dy < H and 0 <= i + dx < W:
                            acc += x[0, d + dz, h + dy, i + dx] @ w[co, t]
                    assert abs(y[0, d, h, i, co] - acc) < 1e-12


def test_backward_passes_are_adjoints():
    x = _rand((2, 4, 4, 6, 5), 5)
    w = _rand((3, 27, 5), 6)
    w2 = _rand((3, 27, 5), 7)
    g = _rand((2, 4, 4, 6, 3), 8)
    lhs = (CN.conv_fwd(x, w) * g).sum()
    assert abs(lhs - (x * CN.conv_bwd_data(g, w)).sum()) <= 1e-11 * abs(lhs)
    dw, db = CN.conv_bwd_weight(x, g)
    lhs2 = (CN.conv_fwd(x, w2) * g).sum()
    assert abs(lhs2 - (dw * w2).sum()) <= 1e-11 * abs(lhs2)
    np.testing.assert_allclose(db, g.sum(axis=(0, 1, 2, 3)), rtol=1e-13)
    xp = _rand((2, 4, 6, 8, 3), 9)
    yp = _rand((2, 2, 3, 4, 3), 10)
    assert abs((CN.pool(xp) * yp).sum() - (xp * CN.up(yp)).sum() / 8) < 1e-12
    np.testing.assert_allclose(CN.pool(CN.up(yp)), yp, rtol=0, atol=1e-15)


def test_network_gradient_finite_differences():
    widths = (4, 5, 6, 7)
    params = CN.unflatten(inputs.net_params(11, widths), widths)
    for li in range(8):  # non-zero biases so every branch is exercised
        params[li][1] = 0.1 * _rand(params[li][1].shape, 20 + li)
    x = _rand((6, 8, 8, 8, 8), 12)
    t = _rand((6, 8, 8, 8, 4), 13)

    def loss(p):
        return CN.loss_and_grad(CN.forward(p, x)[0], t)[0]

    y, a = CN.forward(params, x)
    _, dy = CN.loss_and_grad(y, t)
    grads = CN.backward(params, a, dy)
    rng = np.random.default_rng(14)
    h = 1e-6
    for li in range(8):
        for q in range(2):
            arr = params[li][q]
            for _ in range(3):
                idx = tuple(rng.integers(0, s) for s in arr.shape)
                old = arr[idx]
                arr[idx] = old + h
                lp = loss(params)
                arr[idx] = old - h
                lm = loss(params)
                arr[idx] = old
                fd = (lp - lm) / (2 * h)
                an = grads[li][q][idx]
                # 1e-6 relative, plus the central difference's round-off (~eps L / h)
                assert abs(fd - an) <= 1e-6 * abs(fd) + 2e-9 * abs(lp), (li, q, idx, fd, an)


def test_adam_first_step_closed_form():
    params = [[_rand((2, 27, 3), 15), _rand(2, 16)]]
    grads = [[_rand((2, 27, 3), 17), _rand(2, 18)]]
    before = [p.copy() for p in params[0]]
    opt = CN.Adam(params, lr=1e-2)
    opt.step(params, grads)
    for q in range(2):
        g = grads[0][q]
        np.testing.assert_allclose(params[0][q] - before[q], -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    v = np.concatenate([_rand(10000, 19) * 10.0 ** np.random.default_rng(20).integers(-8, 8, 10000),
                        [1.0 + 2.0**-8, 1.0 + 3 * 2.0**-8, -(1.0 + 2.0**-8), 0.0, 3.0e38]])
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(CN.bf16_round(v), ref)


def test_zero_network_is_linear_extrapolation():
    params = CN.unflatten(inputs.net_params(21, (4, 4, 4, 4)), (4, 4, 4, 4))
    for p in params:
        p[0][:] = 0
        p[1][:] = 0
    xm1, xm2 = _rand((6, 8, 8, 8, 4), 22), _rand((6, 8, 8, 8, 4), 23)
    np.testing.assert_array_equal(CN.guess(params, xm1, xm2), 2 * xm1 - xm2)


def test_parameter_count():
    assert CN.param_count() == 27 * (8 * 32 + 32 * 48 + 48 * 64 + 64 * 128 + 128 * 64 + 64 * 48 + 48 * 32
                                     + 32 * 4) + (32 + 48 + 64 + 128 + 64 + 48 + 32 + 4)
    assert CN.param_count() == 701988
    assert len(inputs.net_params(0)) == 701988
    np.testing.assert_array_equal(CN.flatten(CN.unflatten(inputs.net_params(0))), inputs.net_params(0))


def test_bf16_storage_emulation_stays_within_bf16_rounding():
    """The BF16-storage mode of the network oracle (the form the GPU computes) is
    the FP64 network up to BF16 rounding of the stored tensors: every stored value
    changes by at most half a BF16 unit (2^-9 relative), and the outputs and
    gradients move by a few such units, not more."""
    widths = (8, 8, 8, 8)
    params = CN.unflatten(inputs.net_params(24, widths), widths)
    x = CN.bf16_round(_rand((6, 8, 8, 8, 8), 25))
    y64, a64 = CN.forward(params, x)
    y16, a16 = CN.forward(params, x, bf16=True)
    for key in ("e0", "p0", "e1", "d0"):
        v = a16[key]
        assert np.array_equal(v, CN.bf16_round(v))            # stored in BF16
    rel = np.linalg.norm(y16 - y64) / np.linalg.norm(y64)
    assert 2.0**-12 < rel < 2.0**-5, rel
    dy = _rand(y64.shape, 26)
    g64 = CN.flatten(CN.backward(params, a64, dy))
    g16 = CN.flatten(CN.backward(params, a16, dy, bf16=True))
    relg = np.linalg.norm(g16 - g64) / np.linalg.norm(g64)
    assert 2.0**-12 < relg < 2.0**-5, relg
