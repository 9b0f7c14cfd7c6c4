"""Pins of the learned-proposal oracle (oracle/proposal.py) and of the tile generator
(synth/philox.py) against references other than themselves: torch CPU conv1d / autograd /
Adam in FP64 (independent libraries), finite differences, brute-force sums, closed forms and
the published Philox known-answer values."""
import math

import numpy as np
import pytest

from oracle import proposal as op
from synth import philox

torch = pytest.importorskip("torch")


# ------------------------------------------------------------------ bfloat16 rounding
def test_round_bf16_ties_and_torch():
    v = np.array([1.0, 1 + 2 ** -8, 1 + 2 ** -8 + 2 ** -20, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 3.0,
                  1e-30, -7.123456, 65504.3, 2 ** -130])
    want = [1.0, 1.0, 1 + 2 ** -7, 1 + 2 ** -6, -1.0, 3.0]
    got = op.round_bf16(v)
    assert list(got[:6]) == want
    rng = np.random.default_rng(0)
    r = np.concatenate([v, rng.standard_normal(10000) * 10.0 ** rng.integers(-5, 5, 10000)])
    ref = torch.tensor(r.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(op.round_bf16(r), ref)


# ------------------------------------------------------------------ features
def test_dit_features_brute_force():
    rng = np.random.default_rng(1)
    rows = 3
    x = rng.standard_normal((rows, op.TILE_LEN)).astype(np.float32) * 2 + 0.5
    mu = np.array([0.5, 0.4, 0.6])
    sg = np.array([2.0, 1.5, 2.5])
    F = op.dit_features(x, mu, sg)
    assert F.shape == (rows, op.P, op.C_IN)
    for r in range(rows):
        for c in range(op.C_IN):
            k = 4 + c
            for p in (0, 1, 77, 255):
                i = p >> c
                seg = [(float(x[r, t]) - mu[r]) / sg[r] for t in range(i << k, (i + 1) << k)]
                assert F[r, p, c] == pytest.approx(sum(seg) / 2 ** (k / 2), rel=1e-12, abs=1e-12)


def test_dit_features_constant_input():
    x = np.full((2, op.TILE_LEN), 3.0)
    F = op.dit_features(x, np.zeros(2), np.ones(2))
    for c in range(op.C_IN):
        assert np.allclose(F[:, :, c], 3.0 * 2 ** ((4 + c) / 2))


# ------------------------------------------------------------------ network vs torch (FP64)
def torch_net(net: op.Net):
    t = lambda a: torch.tensor(np.asarray(a, np.float64), requires_grad=True)
    return {"W1": t(net.W1), "b1": t(net.b1), "W2": t(net.W2), "b2": t(net.b2),
            "W3": t(net.W3), "b3": t(net.b3), "wh": t(net.wh), "bh": t(net.bh)}


def torch_forward(F, T):
    x = torch.tensor(F).permute(0, 2, 1)                         # [rows][ci][P]
    for l in (1, 2, 3):
        W = T[f"W{l}"].permute(0, 2, 1)                          # [co][ci][taps]
        x = torch.relu(torch.nn.functional.conv1d(x, W, T[f"b{l}"], padding=2))
    s = torch.einsum("rcp,c->rp", x, T["wh"]) + T["bh"]
    st = s.reshape(-1, op.TILE_ROWS * op.P)
    return torch.logsumexp(st, dim=1) - math.log(op.TILE_ROWS * op.P), s


def small_case(seed=2, tiles=2):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((tiles * op.TILE_ROWS, op.P, op.C_IN))
    net = op.init_net(seed)
    net.b1 = rng.standard_normal(op.C) * 0.1
    net.b2 = rng.standard_normal(op.C) * 0.1
    net.b3 = rng.standard_normal(op.C) * 0.1
    net.bh = 0.3
    y = np.array([1.0, 0.0] * (tiles // 2) + [1.0] * (tiles % 2))
    return F, net, y


def test_conv_matches_torch_conv1d():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((4, 50, 7))
    W = rng.standard_normal((6, op.TAPS, 7))
    b = rng.standard_normal(6)
    ref = torch.nn.functional.conv1d(torch.tensor(a).permute(0, 2, 1),
                                     torch.tensor(W).permute(0, 2, 1), torch.tensor(b), padding=2)
    assert np.allclose(op.conv(a, W, b), ref.permute(0, 2, 1).numpy(), rtol=1e-12, atol=1e-12)


def test_forward_matches_torch():
    F, net, _ = small_case()
    fw = op.forward(F, net)
    lg, s = torch_forward(F, torch_net(net))
    assert np.allclose(fw["s"], s.detach().numpy(), rtol=1e-11, atol=1e-11)
    assert np.allclose(fw["logits"], lg.detach().numpy(), rtol=1e-11, atol=1e-11)


def test_backward_matches_torch_autograd():
    F, net, y = small_case()
    loss, g = op.backward(F, y, net)
    T = torch_net(net)
    lg, _ = torch_forward(F, T)
    tl = torch.nn.functional.binary_cross_entropy_with_logits(lg, torch.tensor(y))
    tl.backward()
    assert loss == pytest.approx(tl.item(), rel=1e-12)
    for n in op.Net.NAMES:
        ref = T[n].grad.numpy()
        got = np.asarray(getattr(g, n))
        assert np.allclose(got, ref, rtol=1e-9, atol=1e-12 * max(1.0, np.abs(ref).max())), n


def test_backward_finite_differences():
    F, net, y = small_case(seed=4)
    _, g = op.backward(F, y, net)
    h = 1e-6
    rng = np.random.default_rng(5)
    for n in ("W1", "W2", "W3", "b1", "b3", "wh"):
        arr = getattr(net, n)
        for _ in range(3):
            idx = tuple(int(rng.integers(0, s)) for s in arr.shape)
            p, m = net.copy(), net.copy()
            getattr(p, n)[idx] += h
            getattr(m, n)[idx] -= h
            num = (op.loss_value(op.forward(F, p)["logits"], y) -
                   op.loss_value(op.forward(F, m)["logits"], y)) / (2 * h)
            assert getattr(g, n)[idx] == pytest.approx(num, rel=1e-5, abs=1e-9), (n, idx)
    p, m = net.copy(), net.copy()
    p.bh += h
    m.bh -= h
    num = (op.loss_value(op.forward(F, p)["logits"], y) -
           op.loss_value(op.forward(F, m)["logits"], y)) / (2 * h)
    assert g.bh == pytest.approx(num, rel=1e-6)


def test_conv_input_grad_is_adjoint_of_conv():
    rng = np.random.default_rng(6)
    a = rng.standard_normal((3, 40, 5))
    W = rng.standard_normal((4, op.TAPS, 5))
    dz = rng.standard_normal((3, 40, 4))
    # <conv(a), dz> == <a, conv_input_grad(dz)> and == <W, conv_weight_grad(dz, a)>
    lhs = float((op.conv(a, W) * dz).sum())
    assert lhs == pytest.approx(float((a * op.conv_input_grad(dz, W)).sum()), rel=1e-12)
    assert lhs == pytest.approx(float((W * op.conv_weight_grad(dz, a)).sum()), rel=1e-12)


def test_bf16_mode_rounds_stored_tensors():
    F, net, y = small_case(seed=7)
    fw = op.forward(F, net, bf16=True)
    for k in ("a0", "a1", "a2", "a3"):
        assert np.array_equal(fw[k], op.round_bf16(fw[k]))
    ref = op.forward(F, net)
    assert np.allclose(fw["logits"], ref["logits"], rtol=0.05, atol=0.05)
    loss_b, gb = op.backward(F, y, net, bf16=True)
    loss, g = op.backward(F, y, net)
    assert loss_b == pytest.approx(loss, rel=0.02)
    for n in ("W2", "W3", "wh"):
        a, b = getattr(gb, n), getattr(g, n)
        assert np.abs(a - b).max() <= 0.05 * np.abs(b).max(), n


def test_error_budget_bounds_bf16_rounding():
    """The stochastic bfloat16 error model bounds a real set of roundings: this module's bf16
    mode (round to nearest even at every store, an independent realisation) deviates from the
    FP64 network by less than the budget at every logit and gradient element; the budget is
    small against the values (so it is not vacuous), and a plausible mistake (a W2 gradient
    with its tap order reversed, one W3 element off by 5%) exceeds it."""
    F, net, y = small_case(seed=7)
    F = op.round_bf16(F)
    B = op.error_budget(F, y, net)
    fb, f = op.forward(F, net, bf16=True), op.forward(F, net)
    assert np.all(np.abs(fb["logits"] - f["logits"]) <= B["logits"])
    assert np.all(B["logits"] < 0.05)
    loss_b, gb = op.backward(F, y, net, bf16=True)
    loss, g = op.backward(F, y, net)
    assert abs(loss_b - loss) <= B["loss"]
    for n in op.Net.NAMES:
        a, b = np.asarray(getattr(gb, n)), np.asarray(getattr(g, n))
        assert np.all(np.abs(a - b) <= B[n]), n
        assert np.median(B[n] / np.maximum(np.abs(b), 1e-30)) < 0.5, n
        assert np.max(B[n]) < 0.2 * np.abs(b).max(), n
    bad = g.W2[:, ::-1, :]
    assert np.any(np.abs(bad - g.W2) > B["W2"])
    bad = g.W3.copy()
    i = np.unravel_index(np.argmax(np.abs(g.W3)), g.W3.shape)
    bad[i] *= 1.05
    assert np.any(np.abs(bad - g.W3) > B["W3"])


def test_adam_matches_torch():
    rng = np.random.default_rng(8)
    p0 = rng.standard_normal(20)
    grads = [rng.standard_normal(20) for _ in range(3)]
    tp = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(op.ADAM_B1, op.ADAM_B2), eps=op.ADAM_EPS)
    p, m, v = p0.copy(), np.zeros(20), np.zeros(20)
    for step, g in enumerate(grads, 1):
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = op.adam_update(p, g, m, v, step, 1e-2)
        assert np.allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_labels_and_tile_max():
    Y0 = np.array([[1.0, 7.0], [2.0, 3.0], [0.5, 0.1], [9.0, 4.0]])
    planes = [{"Y": Y0}, {"Y": np.array([[8.0], [1.0], [0.0], [2.0]])}]
    assert list(op.tile_max(planes, 2)) == [8.0, 9.0]
    assert list(op.tile_max(planes, 4)) == [8.0, 3.0, 0.5, 9.0]
    e = np.array([7.0, 7.0, 4.0, 10.0])
    l = np.array([6.0, 6.95, 3.0, 9.95])
    assert list(op.labels_from_max(e, l, 5.0, 0.01)) == [1.0, 0.0, 0.0, 0.0]


# ------------------------------------------------------------------ tile generator
def test_philox_known_answers():
    # published known-answer values of Philox4x32-10 (Random123 distribution)
    cases = [((0, 0, 0, 0, 0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
             ((0xffffffff,) * 6, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
             ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344, 0xa4093822, 0x299f31d0),
              (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1))]
    for args, want in cases:
        got = tuple(int(v) for v in philox.philox4x32_10(*args))
        assert got == want


def test_tile_noise_statistics_and_pulses():
    x = philox.tile(11, 5, pulses=False)
    assert x.shape == (philox.TILE_ROWS, philox.TILE_LEN) and x.dtype == np.float32
    assert abs(float(x.mean())) < 0.01 and abs(float(x.std()) - 1.0) < 0.01
    counts = [len(philox.tile_pulses(11, t)) for t in range(300)]
    assert set(counts) == {0, 1, 2} and 60 < counts.count(0) < 140
    for t in range(40):
        xp = philox.tile(11, t) - philox.tile(11, t, pulses=False)
        for row, start, S, snr in philox.tile_pulses(11, t):
            assert 0 <= row < philox.TILE_ROWS and 1 <= S <= philox.MAX_WIDTH
            assert 0 <= start and start + S <= philox.TILE_LEN
            assert philox.SNR_LO <= snr <= philox.SNR_HI
            # noise-free boxcar of width S on the pulse recovers its SNR (pulses may overlap)
            got = float(xp[row, start:start + S].astype(np.float64).sum()) / math.sqrt(S)
            assert got >= snr * (1 - 1e-5)
