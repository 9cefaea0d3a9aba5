"""Pins of the learned-preconditioner oracle (network, block loss, gradient)
against finite differences, torch autograd and closed-form losses."""
import numpy as np
import pytest

import synth
from oracle import learned as ol


def test_gradient_matches_central_differences():
    lay, B, T, F = synth.learned_blocks(1, [5, 9, 1, 17], [3, 0, 7, 40], equal_blocks=(2,))
    th = ol.random_theta(3)
    L, g = ol.loss_grad(th, F, lay, B, T)
    assert L == pytest.approx(ol.loss(th, F, lay, B, T), rel=1e-13)
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.choice(ol.NPAR, 60, replace=False), [0, ol.NPAR - 1, ol.NF * ol.NH]])
    h = 1e-6
    for i in idx:
        e = np.zeros(ol.NPAR)
        e[i] = h
        fd = (ol.loss(th + e, F, lay, B, T) - ol.loss(th - e, F, lay, B, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    lay, B, T, F = synth.learned_blocks(2, [7, 3, 12, 64], [10, 0, 64, 64])
    th = ol.random_theta(5)
    L, g = ol.loss_grad(th, F, lay, B, T)
    t = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    Ft = torch.tensor(F)
    W1 = t[:ol.NF * ol.NH].reshape(ol.NH, ol.NF)
    b1 = t[ol.NF * ol.NH:ol.NF * ol.NH + ol.NH]
    o2 = ol.NF * ol.NH + ol.NH
    W2 = t[o2:o2 + ol.NH * ol.NO].reshape(ol.NO, ol.NH)
    b2 = t[o2 + ol.NH * ol.NO:]
    O = torch.tanh(Ft @ W1.T + b1) @ W2.T + b2
    R = ol.RANK
    U = torch.stack([torch.complex(O[:, 2 * q], O[:, 2 * q + 1]) for q in range(R)], 1)
    W = torch.stack([torch.complex(O[:, 2 * R + 2 * q], O[:, 2 * R + 2 * q + 1]) for q in range(R)], 1)
    tot = 0
    for p, n, ne, io, to in zip(*lay):
        Bb = torch.zeros((n, ne), dtype=torch.complex128)
        Bb[:, :n] = torch.tensor(B[io:io + n * n].reshape(n, n, order="F"))
        Rb = torch.tensor(T[to:to + n * ne].reshape(n, ne, order="F"))
        D = Bb + U[p:p + n] @ W[p:p + ne].conj().T - Rb
        tot = tot + (D.abs() ** 2).sum() / ((Rb - Bb).abs() ** 2).sum()
    tot.backward()
    assert L == pytest.approx(tot.item(), rel=1e-13)
    np.testing.assert_allclose(g, t.grad.numpy(), rtol=1e-11, atol=1e-12 * np.abs(g).max())


def _constant_factor_theta(a: complex):
    """Network whose factor rows are U_j = (a, 0, 0, 0), W_j = (1, 0, 0, 0)."""
    b2 = np.zeros(ol.NO)
    b2[0], b2[1], b2[2 * ol.RANK] = a.real, a.imag, 1.0
    return ol.pack(np.zeros((ol.NH, ol.NF)), np.zeros(ol.NH), np.zeros((ol.NO, ol.NH)), b2)


def _shift_targets(lay, B, c):
    """Targets [B 0] + c J (J all ones)."""
    T = np.zeros(int(np.sum(lay[1] * lay[2])), dtype=np.complex128)
    for p, n, ne, io, to in zip(*lay):
        blk = np.full((n, ne), c, dtype=np.complex128)
        blk[:, :n] += B[io:io + n * n].reshape(n, n, order="F")
        T[to:to + n * ne] = blk.ravel(order="F")
    return T


def test_closed_form_losses():
    lay, B, _, F = synth.learned_blocks(4, [6, 11, 64], [5, 0, 64])
    a = 0.7 - 0.2j
    th = _constant_factor_theta(a)
    # targets [B 0] + a J: the correction U W^H = a J is exact, loss 0
    assert ol.loss(th, F, lay, B, _shift_targets(lay, B, a)) == pytest.approx(0.0, abs=1e-24)
    # targets [B 0] + 2a J: D = -a J, loss 1/4 per block
    assert ol.loss(th, F, lay, B, _shift_targets(lay, B, 2 * a)) == pytest.approx(0.75, rel=1e-13)
    # zero network output: loss 1 per block whose target differs from [B 0]
    lay, B, T, F = synth.learned_blocks(5, [6, 11, 64, 2], [6, 30, 0, 1], equal_blocks=(1,))
    assert ol.loss(np.zeros(ol.NPAR), F, lay, B, T) == pytest.approx(3.0, rel=1e-13)
    # U = 0, W_j = (1, 0, 0, 0): dL/d(Re + i Im) U_i0 = 2 w sum_l D_il with D = [B 0] - R
    L, g = ol.loss_grad(_constant_factor_theta(0j), F, lay, B, T)
    o2 = ol.NF * ol.NH + ol.NH + ol.NH * ol.NO
    exp = 0j
    for p, n, ne, io, to in zip(*lay):
        Bb = np.zeros((n, ne), dtype=np.complex128)
        Bb[:, :n] = B[io:io + n * n].reshape(n, n, order="F")
        Rb = T[to:to + n * ne].reshape(n, ne, order="F")
        r = np.sum(np.abs(Rb - Bb) ** 2)
        w = 1.0 / r if r > 1e-12 * np.sum(np.abs(Rb) ** 2) else 0.0
        exp += 2 * w * (Bb - Rb).sum()
    assert g[o2] == pytest.approx(exp.real, rel=1e-12)
    assert g[o2 + 1] == pytest.approx(exp.imag, rel=1e-12)


def test_block_weights_scale_each_block():
    """Extra block weights c_b scale each block's term: the weighted loss is
    the sum of single-block losses times c_b (each computed without weights
    on a layout holding that block alone), and the weighted gradient matches
    central differences of the weighted loss."""
    sizes, extras = [5, 9, 1, 17], [3, 0, 7, 40]
    lay, B, T, F = synth.learned_blocks(4, sizes, extras)
    th = ol.random_theta(8)
    c = np.array([0.5, 2.0, 0.0, 1.7])
    L, g = ol.loss_grad(th, F, lay, B, T, c)
    parts = []
    for b in range(len(sizes)):
        one = tuple(np.asarray(v)[b:b + 1] for v in lay)
        parts.append(ol.loss(th, F, one, B, T))
    assert L == pytest.approx(float(np.dot(c, parts)), rel=1e-12)
    h = 1e-6
    for i in (0, 17, ol.NPAR - 1, ol.NF * ol.NH + 3):
        e = np.zeros(ol.NPAR)
        e[i] = h
        fd = (ol.loss(th + e, F, lay, B, T, c) - ol.loss(th - e, F, lay, B, T, c)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i]))
