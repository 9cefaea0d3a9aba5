"""Seeded synthetic inputs for the learned preconditioner's loss: a ragged
block layout with random complex block inverses, targets and pair features.
Random numbers only; no arithmetic of the method."""

from __future__ import annotations

import numpy as np


def learned_blocks(seed: int, sizes, extras, n_features: int = 12, equal_blocks=()):
    """Blocks of sizes[b] own points and extras[b] added points.

    Returns (layout, Binv, T, F): layout = (pair_off, n, ne, inv_off,
    target_off) int64 arrays; Binv the n x n blocks and T the n x ne targets,
    column-major complex128 at their offsets; F the pair features (rows x
    n_features).  Targets equal [Binv 0] plus a random perturbation, except
    for the listed blocks, whose targets equal [Binv 0] exactly."""
    rng = np.random.default_rng(seed)
    n = np.asarray(sizes, dtype=np.int64)
    ne = n + np.asarray(extras, dtype=np.int64)
    poff = np.concatenate([[0], np.cumsum(ne)[:-1]]).astype(np.int64)
    ioff = np.concatenate([[0], np.cumsum(n * n)[:-1]]).astype(np.int64)
    toff = np.concatenate([[0], np.cumsum(n * ne)[:-1]]).astype(np.int64)
    Binv = rng.standard_normal(int(np.sum(n * n))) + 1j * rng.standard_normal(int(np.sum(n * n)))
    T = np.zeros(int(np.sum(n * ne)), dtype=np.complex128)
    for b in range(len(n)):
        blk = np.zeros((n[b], ne[b]), dtype=np.complex128)
        blk[:, :n[b]] = Binv[ioff[b]:ioff[b] + n[b] * n[b]].reshape(n[b], n[b], order="F")
        if b not in equal_blocks:
            blk += 0.3 * (rng.standard_normal(blk.shape) + 1j * rng.standard_normal(blk.shape))
        T[toff[b]:toff[b] + n[b] * ne[b]] = blk.ravel(order="F")
    F = rng.standard_normal((int(ne.sum()), n_features))
    return (poff, n, ne, ioff, toff), Binv, T, F
