"""GPU parity of the learned-guess kernels and network against the FP64
oracle (oracle/convnet.py) fed the same BF16-rounded inputs and weights.

Tolerances: a single convolution differs from the oracle by the final BF16
rounding of its output (relative 2^-9) plus FP32 accumulation (~1e-6); FP32
outputs and weight gradients by the accumulation only.  Through the network
every activation is rounded to BF16 (8 rounds forward, 15 more backward), so
whole-network outputs are compared norm-wise at a few 2^-9.
"""
import numpy as np
import pytest

import oracle.convnet as CN
from paper_2009_02171_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _csdyn():
    from paper_2009_02171_amd import csdyn
    return csdyn


def _bf16(a, c8=None):
    """numpy [.., c] -> device bf16 [.., c8] with zero padded channels."""
    a = np.asarray(a, dtype=np.float32)
    if c8 is not None and c8 != a.shape[-1]:
        a = np.concatenate([a, np.zeros(a.shape[:-1] + (c8 - a.shape[-1],), np.float32)], axis=-1)
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.bfloat16).cuda()


def _np(t, c=None):
    a = t.float().cpu().numpy().astype(np.float64)
    return a[..., :c] if c is not None else a


def _r8(c):
    return (c + 7) // 8 * 8


SHAPES = [  # (batch, d, h, w, cin, cout)
    (6, 4, 8, 8, 8, 32),
    (6, 3, 5, 7, 32, 48),
    (2, 4, 4, 8, 48, 64),
    (6, 2, 2, 2, 64, 128),
    (3, 4, 6, 4, 128, 64),
    (6, 4, 8, 8, 32, 4),
    (1, 3, 3, 9, 12, 20),
]


@pytest.mark.parametrize("shape", SHAPES)
def test_conv_fwd_matches_oracle(shape):
    cs = _csdyn()
    b, d, h, w, ci, co = shape
    rng = np.random.default_rng(sum(shape))
    x = CN.bf16_round(rng.standard_normal((b, d, h, w, ci)))
    W = (rng.standard_normal((co, 27, ci)) / np.sqrt(27 * ci)).astype(np.float32)
    bias = rng.standard_normal(co).astype(np.float32)
    res = CN.bf16_round(rng.standard_normal((b, d, h, w, co)))
    wf, _ = cs.conv_pack(shape, torch.from_numpy(W).cuda())
    xg = _bf16(x, _r8(ci))
    ref = CN.conv_fwd(x, CN.bf16_round(W), bias.astype(np.float64))
    # FP32 output, no activation
    y32 = cs.conv_fwd(shape, xg, wf, bias=torch.from_numpy(bias).cuda(), out32=True)
    assert np.abs(_np(y32) - ref).max() <= 1e-5 * np.abs(ref).max()
    # BF16 output with residual and relu; padded channels zero
    y = cs.conv_fwd(shape, xg, wf, bias=torch.from_numpy(bias).cuda(), residual=_bf16(res, _r8(co)), relu=True)
    refr = np.maximum(ref + res, 0)
    got = _np(y)
    assert np.abs(got[..., :co] - refr).max() <= 4e-3 * np.abs(refr).max()
    assert np.abs(got[..., :co] - refr).mean() <= 2e-3 * np.abs(refr).mean()
    assert (got[..., co:] == 0).all()


@pytest.mark.parametrize("shape", SHAPES)
def test_conv_bwd_data_matches_oracle(shape):
    cs = _csdyn()
    b, d, h, w, ci, co = shape
    rng = np.random.default_rng(100 + sum(shape))
    dy = CN.bf16_round(rng.standard_normal((b, d, h, w, co)))
    W = (rng.standard_normal((co, 27, ci)) / np.sqrt(27 * co)).astype(np.float32)
    mask = CN.bf16_round(rng.standard_normal((b, d, h, w, ci)))
    _, wb = cs.conv_pack(shape, torch.from_numpy(W).cuda())
    dx = cs.conv_bwd_data(shape, _bf16(dy, _r8(co)), wb, mask=_bf16(mask, _r8(ci)))
    ref = CN.conv_bwd_data(dy, CN.bf16_round(W)) * (mask > 0)
    got = _np(dx)
    assert np.abs(got[..., :ci] - ref).max() <= 4e-3 * np.abs(ref).max()
    assert (got[..., ci:] == 0).all()


@pytest.mark.parametrize("shape", SHAPES)
def test_conv_bwd_weight_matches_oracle(shape):
    cs = _csdyn()
    b, d, h, w, ci, co = shape
    rng = np.random.default_rng(200 + sum(shape))
    x = CN.bf16_round(rng.standard_normal((b, d, h, w, ci)))
    dy = CN.bf16_round(rng.standard_normal((b, d, h, w, co)))
    dw, db = cs.conv_bwd_weight(shape, _bf16(x, _r8(ci)), _bf16(dy, _r8(co)))
    rdw, rdb = CN.conv_bwd_weight(x, dy)
    assert np.abs(_np(dw) - rdw).max() <= 1e-5 * np.abs(rdw).max() * np.sqrt(b * d * h * w)
    assert np.abs(_np(db) - rdb).max() <= 1e-5 * np.abs(rdb).max() * np.sqrt(b * d * h * w)


def test_conv_full_resolution_sampled():
    """One full-resolution layer of the N=64 network (6 x 64^3 voxels, 48 -> 32)
    in the launch configuration the network uses; outputs sampled."""
    cs = _csdyn()
    shape = (6, 64, 64, 64, 48, 32)
    rng = np.random.default_rng(7)
    x = CN.bf16_round(rng.standard_normal((6, 64, 64, 64, 48)).astype(np.float32))
    W = (rng.standard_normal((32, 27, 48)) / np.sqrt(27 * 48)).astype(np.float32)
    wf, _ = cs.conv_pack(shape, torch.from_numpy(W).cuda())
    y = _np(cs.conv_fwd(shape, _bf16(x), wf, out32=True))
    Wr = CN.bf16_round(W)
    for idx in [(0, 0, 0, 0), (5, 63, 63, 63), (2, 31, 0, 17), (3, 5, 40, 63), (4, 63, 1, 0)]:
        p, k, j, i = idx
        ref = np.zeros(32)
        for t, (dz, dy, dx) in enumerate(CN.tap_offsets()):
            kk, jj, ii = k + dz, j + dy, i + dx
            if 0 <= kk < 64 and 0 <= jj < 64 and 0 <= ii < 64:
                ref += Wr[:, t, :] @ x[p, kk, jj, ii]
        assert np.abs(y[p, k, j, i] - ref).max() <= 1e-5 * np.abs(ref).max()


def test_adam_matches_closed_form():
    cs = _csdyn()
    rng = np.random.default_rng(9)
    n = 10007
    p, g = rng.standard_normal(n).astype(np.float32), rng.standard_normal(n).astype(np.float32)
    m, v = (0.1 * rng.standard_normal(n)).astype(np.float32), np.abs(rng.standard_normal(n)).astype(np.float32)
    tp, tg, tm, tv = (torch.from_numpy(a.copy()).cuda() for a in (p, g, m, v))
    cs.adam_step(tp, tg, tm, tv, step=3, lr=1e-2)
    b1, b2 = 0.9, 0.999
    m2 = b1 * m.astype(np.float64) + (1 - b1) * g
    v2 = b2 * v.astype(np.float64) + (1 - b2) * g.astype(np.float64) ** 2
    p2 = p - 1e-2 * (m2 / (1 - b1**3)) / (np.sqrt(v2 / (1 - b2**3)) + 1e-8)
    assert np.abs(tp.cpu().numpy() - p2).max() <= 1e-6 * np.abs(p2).max()
    assert np.abs(tm.cpu().numpy() - m2).max() <= 1e-6


N, NR = 16, 16


def _samples(n=N, nr=NR):
    x2 = inputs.rhs(n, nr, seed=31)
    x1 = x2 + 0.05 * inputs.rhs(n, nr, seed=32)
    xn = 2 * x1 - x2 + 0.01 * inputs.rhs(n, nr, seed=33)
    return x2, x1, xn


def _oracle_params(flat):
    return [[CN.bf16_round(w), b] for w, b in CN.unflatten(flat.astype(np.float64))]


def test_net_forward_matches_oracle():
    cs = _csdyn()
    flat = inputs.net_params(5)
    x2, x1, _ = _samples()
    net = cs.Net(N, NR, torch.from_numpy(flat).cuda())
    g = net.predict(torch.from_numpy(x1).cuda(), torch.from_numpy(x2).cuda()).cpu().numpy()
    feats, s, sd = CN.features(x1, x2)
    # the oracle stores its activations in BF16 at the same points as the GPU
    y_ref, _ = CN.forward(_oracle_params(flat), CN.bf16_round(feats), bf16=True)
    y_gpu = (g - (2 * x1 - x2)) / sd
    rel = np.linalg.norm(y_gpu - y_ref) / np.linalg.norm(y_ref)
    print(f"[net forward] rel {rel:.3e}", flush=True)
    assert rel <= 1e-2, rel


def test_net_zero_parameters_give_extrapolation():
    cs = _csdyn()
    flat = np.zeros_like(inputs.net_params(5))
    x2, x1, _ = _samples()
    net = cs.Net(N, NR, torch.from_numpy(flat).cuda())
    g = net.predict(torch.from_numpy(x1).cuda(), torch.from_numpy(x2).cuda()).cpu().numpy()
    np.testing.assert_array_equal(g, 2 * x1 - x2)


def test_net_gradient_matches_oracle():
    cs = _csdyn()
    flat = inputs.net_params(6)
    x2, x1, xn = _samples()
    net = cs.Net(N, NR, torch.from_numpy(flat).cuda())
    loss, gg = net.loss_grad(*(torch.from_numpy(a).cuda() for a in (x2, x1, xn)))
    feats, s, sd = CN.features(x1, x2)
    params = _oracle_params(flat)
    y, a = CN.forward(params, CN.bf16_round(feats), bf16=True)
    rloss, dy = CN.loss_and_grad(y, CN.target(xn, x1, x2, sd))
    grads = CN.flatten(CN.backward(params, a, dy, bf16=True))
    print(f"[net gradient] loss {loss:.6e} oracle {rloss:.6e}", flush=True)
    assert abs(loss - rloss) <= 1e-2 * rloss
    gg = gg.cpu().numpy().astype(np.float64)
    off = 0
    worst = 0.0
    for li, (co, ci) in enumerate(CN.layer_shapes()):
        nw = co * 27 * ci
        for part in (slice(off, off + nw), slice(off + nw, off + nw + co)):
            rel = np.linalg.norm(gg[part] - grads[part]) / np.linalg.norm(grads[part])
            worst = max(worst, rel)
            assert rel <= 1e-2, (li, rel)
        off += nw + co
    print(f"[net gradient] worst layer rel {worst:.3e}", flush=True)


def test_net_training_tracks_oracle_and_reduces_loss():
    cs = _csdyn()
    flat = inputs.net_params(7)
    x2, x1, xn = _samples()
    net = cs.Net(N, NR, torch.from_numpy(flat).cuda())
    t = [torch.from_numpy(a).cuda() for a in (x2, x1, xn)]
    gpu = [net.train_step(*t, lr=1e-4) for _ in range(12)]
    params = CN.unflatten(flat.astype(np.float64))
    opt = CN.Adam(params, lr=1e-4)
    ref = [CN.train_step(params, opt, x2, x1, xn) for _ in range(12)]
    assert gpu[-1] < 0.7 * gpu[0]
    # Adam normalises every update to about lr, so the parameters themselves
    # are not compared: BF16 noise flips the sign of near-zero gradients.
    for a, b in zip(gpu, ref):
        assert abs(a - b) <= 5e-2 * b, (gpu, ref)
