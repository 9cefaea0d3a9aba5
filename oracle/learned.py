"""Learned coupling correction of the block-Jacobi preconditioner: network,
block loss and gradient -- TEST INFRASTRUCTURE ONLY.

Not part of the paper's method: a preconditioner placed on top of its GMRES
solve of the Burton-Miller system (section 2.2, eq. Axb).  This module is the
plain definition of what the GPU kernels compute, written with dense numpy
arrays and the chain rule, for checking them on synthetic inputs:

* network, one row per (block b, point j of its overlapping set E_b):
  features f (12) -> h = tanh(W1 f + b1) (32) -> o = W2 h + b2 (16); the
  rank-4 factor rows are U_jq = o_2q + i o_2q+1 (read for the block's own
  points) and W_jq = o_8+2q + i o_9+2q;
* block loss: D_b = [B_b 0] + U_b W_b^H - R_b (n_b x ne_b, B_b the n_b x n_b
  block inverse, R_b the target rows), L = sum_b c_b w_b ||D_b||_F^2 (c_b an
  optional weight per block, 1 by default) with w_b =
  1 / ||R_b - [B_b 0]||_F^2, or 0 when that is <= 1e-12 ||R_b||_F^2;
* parameter vector: W1 (32 x 12, row-major), b1, W2 (16 x 32, row-major), b2.

Pins (tests/test_oracle_learned.py): central finite differences and torch
autograd of the loss, and closed-form losses for constant factors.  Blocks are
column-major complex arrays at the given offsets; block b owns feature rows
[poff_b, poff_b + ne_b), its own points first.
"""

from __future__ import annotations

import numpy as np

NF, NH, RANK = 12, 32, 4
NO = 4 * RANK
NPAR = NF * NH + NH + NH * NO + NO


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (NPAR,)
    i = 0
    W1 = theta[i:i + NF * NH].reshape(NH, NF)
    i += NF * NH
    b1 = theta[i:i + NH]
    i += NH
    W2 = theta[i:i + NH * NO].reshape(NO, NH)
    i += NH * NO
    b2 = theta[i:i + NO]
    return W1, b1, W2, b2


def pack(W1, b1, W2, b2):
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2)]).astype(np.float64)


def forward(theta, F):
    """Hidden activations, outputs and complex factor rows (U, W), rows x RANK."""
    W1, b1, W2, b2 = unpack(theta)
    Hh = np.tanh(F @ W1.T + b1)
    O = Hh @ W2.T + b2
    U = O[:, 0:2 * RANK:2] + 1j * O[:, 1:2 * RANK:2]
    W = O[:, 2 * RANK::2] + 1j * O[:, 2 * RANK + 1::2]
    return Hh, O, U, W


def _blocks(layout, Binv, T):
    for p, n, ne, bo, to in zip(*layout):
        B = np.zeros((n, ne), dtype=np.complex128)
        B[:, :n] = Binv[bo:bo + n * n].reshape(n, n, order="F")
        yield p, n, ne, B, T[to:to + n * ne].reshape(n, ne, order="F")


def block_weight(B, R):
    r = np.sum(np.abs(R - B) ** 2)
    t = np.sum(np.abs(R) ** 2)
    return 1.0 / r if r > 1e-12 * t else 0.0


def loss(theta, F, layout, Binv, T, c=None):
    """layout = (poff, n, ne, inv_off, target_off), one entry per block; c:
    optional extra weight per block (1 if None)."""
    _, _, U, W = forward(theta, F)
    total = 0.0
    for b, (p, n, ne, B, R) in enumerate(_blocks(layout, Binv, T)):
        D = B + U[p:p + n] @ W[p:p + ne].conj().T - R
        total += (1.0 if c is None else c[b]) * block_weight(B, R) * np.sum(np.abs(D) ** 2)
    return total


def loss_grad(theta, F, layout, Binv, T, c=None):
    """(loss, gradient) by the chain rule written out."""
    W1, b1, W2, b2 = unpack(theta)
    Hh, _, U, W = forward(theta, F)
    dO = np.zeros((F.shape[0], NO))
    total = 0.0
    for b, (p, n, ne, B, R) in enumerate(_blocks(layout, Binv, T)):
        Ub, Wb = U[p:p + n], W[p:p + ne]
        D = B + Ub @ Wb.conj().T - R
        wb = (1.0 if c is None else c[b]) * block_weight(B, R)
        total += wb * np.sum(np.abs(D) ** 2)
        # |D_il|^2 with D_il = sum_q U_iq conj(W_lq) + ...:
        # d/dRe U_iq + i d/dIm U_iq = 2 (D W)_iq, likewise 2 (D^H U)_lq for W
        gU = 2.0 * wb * (D @ Wb)
        gW = 2.0 * wb * (D.conj().T @ Ub)
        dO[p:p + n, 0:2 * RANK:2] += gU.real
        dO[p:p + n, 1:2 * RANK:2] += gU.imag
        dO[p:p + ne, 2 * RANK::2] += gW.real
        dO[p:p + ne, 2 * RANK + 1::2] += gW.imag
    dW2 = dO.T @ Hh
    db2 = dO.sum(axis=0)
    dA = (dO @ W2) * (1.0 - Hh ** 2)
    dW1 = dA.T @ F
    db1 = dA.sum(axis=0)
    return total, pack(dW1, db1, dW2, db2)


def random_theta(seed: int, out_scale: float = 0.3):
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (NH, NF)) * np.sqrt(3.0 / NF)
    b1 = rng.uniform(-0.5, 0.5, NH)
    W2 = rng.uniform(-1, 1, (NO, NH)) * out_scale
    b2 = rng.uniform(-0.5, 0.5, NO) * out_scale
    return pack(W1, b1, W2, b2)
