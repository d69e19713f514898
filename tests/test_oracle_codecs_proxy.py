"""Pins of the oracle's number codecs and proxy maths.

Codecs are checked exhaustively against PyTorch's CPU casts (a library routine written
independently of this repository).  Proxy gradients are checked against central finite
differences, Adam against its closed-form first step and against torch.optim.Adam, and
GELU against math.erf / torch's exact GELU.
"""
import math

import numpy as np
import pytest
import torch

from oracle import codecs, proxy


def test_e4m3_decode_all_codes_matches_torch():
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes.copy()).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = codecs.e4m3_decode(codes)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    assert set(codes[nan].tolist()) == {0x7F, 0xFF}
    np.testing.assert_array_equal(got[~nan], ref[~nan])
    assert np.nanmax(got) == 448.0


def test_e4m3_encode_matches_torch_in_range_including_ties():
    vals = codecs.e4m3_decode(np.arange(0, 0x7F, dtype=np.uint8))
    mids = (vals[:-1] + vals[1:]) / 2                         # exact ties between neighbours
    rng = np.random.default_rng(0)
    rnd = rng.uniform(-448, 448, 200000)
    small = rng.uniform(-0.02, 0.02, 50000)
    x = np.concatenate([vals, -vals, mids, -mids, rnd, small, [0.0, -0.0, 448.0, -448.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(codecs.e4m3_encode(x), ref)


def test_e4m3_encode_saturates_and_keeps_nan():
    x = np.array([448.0, 449.0, 464.0, 1e6, -500.0, np.inf, -np.inf, np.nan], np.float32)
    c = codecs.e4m3_encode(x)
    np.testing.assert_array_equal(c[:7], [0x7E, 0x7E, 0x7E, 0x7E, 0xFE, 0x7E, 0xFE])
    assert c[7] == 0x7F


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(200000) * 10.0 ** rng.integers(-8, 8, 200000),
                        [0.0, -0.0, 1.0, 3.0e38, -3.0e38, 1e-40]]).astype(np.float32)
    # exact ties at the bfloat16 rounding point
    u = (rng.integers(0, 2 ** 15, 1000).astype(np.uint32) << 16) | 0x8000
    x = np.concatenate([x, u.view(np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(codecs.bf16_round(x), ref)


def test_block_quantisation_roundtrip_error_bound():
    rng = np.random.default_rng(2)
    blk = rng.standard_normal((16, 128)).astype(np.float32)
    codes, sc = codecs.quantize_block(blk)
    assert sc == np.float32(np.max(np.abs(blk)) / np.float32(448.0))
    deq = codecs.e4m3_decode(codes) * sc
    # E4M3 has 3 mantissa bits: relative rounding error <= 2^-4 for normals; subnormal step 2^-9
    err = np.abs(deq - blk)
    assert np.all(err <= np.maximum(np.abs(blk) * 2.0 ** -4, sc * 2.0 ** -10) * (1 + 1e-6))
    z, s0 = codecs.quantize_block(np.zeros((16, 128), np.float32))
    assert s0 == 1.0 and np.all(z == 0)


def test_fp8_cache_roundtrip_blocks_by_brute_force():
    """Each 16-row block of each head (and the ragged last block) is scaled by its own amax
    and every element goes to the nearest of the 256 E4M3 values (exhaustive search)."""
    rng = np.random.default_rng(5)
    a = rng.standard_normal((3, 37, 8)) * np.array([0.1, 3.0, 40.0])[:, None, None]
    a[1, 20] *= 50.0                                   # one block with a large outlier
    got = codecs.fp8_cache_roundtrip(a)
    table = codecs.e4m3_decode_table()
    finite = table[np.isfinite(table)]
    for h in range(3):
        for r0 in (0, 16, 32):
            blk = a[h, r0:r0 + 16]
            sc = np.float64(np.float32(np.float32(np.abs(blk).max()) / np.float32(448.0)))
            q = (blk.astype(np.float32) / np.float32(sc)).astype(np.float64)
            near = finite[np.argmin(np.abs(q[..., None] - finite), axis=-1)]
            np.testing.assert_array_equal(got[h, r0:r0 + 16], near * sc)
    # blocks and heads are independent: changing block 2 of head 0 changes nothing else
    b = a.copy()
    b[0, 33] *= 7.0
    diff = codecs.fp8_cache_roundtrip(b) != got
    assert diff[0, 32:].any() and not diff[0, :32].any() and not diff[1:].any()


def test_fp8_cache_roundtrip_exact_on_representable_blocks():
    rng = np.random.default_rng(6)
    table = codecs.e4m3_decode_table()
    codes = rng.integers(0, 0x7E, (2, 32, 8))
    codes[:, ::16, 0] = 0x7E                            # 448 in every block: scale = 2^-5 exactly
    a = table[codes] * rng.choice([-1.0, 1.0], codes.shape) * 2.0 ** -5
    np.testing.assert_array_equal(codecs.fp8_cache_roundtrip(a), a)


# ----------------------------------------------------------------------------- proxy

def _params(rng, d_in=12, d_h=7, n_out=2, scale=0.5):
    return {"w1": rng.standard_normal((d_h, d_in)) * scale, "b1": rng.standard_normal(d_h) * 0.1,
            "w2": rng.standard_normal((n_out, d_h)) * scale, "b2": rng.standard_normal(n_out) * 0.1}


def test_gelu_matches_erf_definition_and_torch():
    x = np.linspace(-6, 6, 1001)
    ref = np.array([0.5 * v * (1 + math.erf(v / math.sqrt(2))) for v in x])
    np.testing.assert_allclose(proxy.gelu(x), ref, rtol=0, atol=1e-15)
    t = torch.nn.functional.gelu(torch.tensor(x), approximate="none").numpy()
    np.testing.assert_allclose(proxy.gelu(x), t, rtol=1e-14, atol=1e-15)
    h = 1e-6
    fd = (proxy.gelu(x + h) - proxy.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(proxy.gelu_grad(x), fd, rtol=1e-7, atol=1e-9)


def test_proxy_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    p = _params(rng)
    f = rng.standard_normal((9, 12))
    y = rng.integers(0, 2, 9)
    _, g = proxy.loss_and_grads(p, f, y)
    h = 1e-6
    for name in ("w1", "b1", "w2", "b2"):
        fd = np.zeros_like(p[name])
        for idx in np.ndindex(p[name].shape):
            pp = {k: v.copy() for k, v in p.items()}
            pm = {k: v.copy() for k, v in p.items()}
            pp[name][idx] += h
            pm[name][idx] -= h
            fd[idx] = (proxy.loss_and_grads(pp, f, y)[0] - proxy.loss_and_grads(pm, f, y)[0]) / (2 * h)
        np.testing.assert_allclose(g[name], fd, rtol=1e-6, atol=1e-10)


def test_proxy_forward_and_loss_match_torch():
    rng = np.random.default_rng(4)
    p = _params(rng)
    f = rng.standard_normal((6, 12))
    y = rng.integers(0, 2, 6)
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in p.items()}
    tf = torch.tensor(f)
    z = torch.nn.functional.linear(torch.nn.functional.gelu(torch.nn.functional.linear(tf, tp["w1"], tp["b1"])),
                                   tp["w2"], tp["b2"])
    loss = torch.nn.functional.cross_entropy(z, torch.tensor(y))
    loss.backward()
    l2, g = proxy.loss_and_grads(p, f, y)
    assert abs(l2 - loss.item()) < 1e-13
    for k in p:
        np.testing.assert_allclose(g[k], tp[k].grad.numpy(), rtol=1e-11, atol=1e-14)


def test_adam_first_step_closed_form_and_torch():
    rng = np.random.default_rng(5)
    w = rng.standard_normal(50)
    g = rng.standard_normal(50)
    g[3] = 0.0
    lr, eps = 1e-3, 1e-8
    w1, m, v = proxy.adam_step(w, g, np.zeros(50), np.zeros(50), 1, lr, eps=eps)
    np.testing.assert_allclose(w1, w - lr * g / (np.abs(g) + eps), rtol=1e-14, atol=1e-18)
    # three steps against torch.optim.Adam in float64
    tw = torch.tensor(w, requires_grad=True)
    opt = torch.optim.Adam([tw], lr=lr, betas=(0.9, 0.999), eps=eps)
    cur, m, v = w.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 4):
        gt = rng.standard_normal(50)
        opt.zero_grad()
        tw.grad = torch.tensor(gt)
        opt.step()
        cur, m, v = proxy.adam_step(cur, gt, m, v, t, lr, eps=eps)
    np.testing.assert_allclose(cur, tw.detach().numpy(), rtol=1e-13, atol=1e-16)


def test_predict_threshold_is_strict():
    p = {"w1": np.zeros((2, 3)), "b1": np.zeros(2), "w2": np.zeros((2, 2)), "b2": np.array([np.log(9.0), 0.0])}
    cls, conf, ans = proxy.predict(p, np.zeros((1, 3)), 0.5)
    assert cls[0] == 0 and conf[0] == pytest.approx(0.9) and ans[0]
    assert not proxy.predict(p, np.zeros((1, 3)), float(conf[0]))[2][0]        # equal is not above
    assert proxy.predict(p, np.zeros((1, 3)), float(conf[0]) - 1e-9)[2][0]
