"""Block-Jacobi and learned coupling preconditioners on the GPU: loss and
gradient kernels against the oracle, training, and GMRES iteration counts on a
held-out surface."""
import numpy as np
import pytest

import synth
from oracle import learned as ol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available()
    return t


def _dev(torch, a, dt):
    return torch.from_numpy(np.ascontiguousarray(a).astype(dt)).cuda()


def _raw(torch, net, lay, B, T, F, c=None):
    return net.loss_grad_raw(_dev(torch, lay[0], np.int64), _dev(torch, lay[1], np.int32),
                             _dev(torch, lay[2], np.int32), _dev(torch, lay[3], np.int64),
                             _dev(torch, lay[4], np.int64), _dev(torch, F, np.float64),
                             _dev(torch, B, np.complex128), _dev(torch, T, np.complex128),
                             None if c is None else _dev(torch, c, np.float64))


def _plan(el, k, **kw):
    import paper_1311_5202_amd as fdb

    pts, nrm, w = fdb.nystrom_nodes(el)
    print(f"[plan] N={len(w)} k={k}", flush=True)
    return fdb.build(pts, nrm, w, k, 1e-4, elements=el, corrections=1, **kw)


@pytest.mark.parametrize("seed", [0, 1])
def test_loss_and_gradient_match_oracle(torch, seed):
    import paper_1311_5202_amd as fdb

    # ragged layout: single-point block, full 64 + 64 block, a block whose
    # target equals its inverse, blocks with no added points
    sizes = [5, 64, 1, 33, 17, 64, 2, 40]
    extras = [7, 64, 0, 60, 3, 0, 126, 88]
    lay, B, T, F = synth.learned_blocks(seed, sizes, extras, equal_blocks=(2, 5))
    th = ol.random_theta(10 + seed)
    L_ref, g_ref = ol.loss_grad(th, F, lay, B, T)
    net = fdb.Net(seed)
    net.params = th
    np.testing.assert_array_equal(net.params, th)
    L, g = _raw(torch, net, lay, B, T, F)
    print(f"[learned] loss {L} vs {L_ref}", flush=True)
    assert L == pytest.approx(L_ref, rel=1e-12)
    assert np.abs(g - g_ref).max() <= 1e-11 * np.abs(g_ref).max()
    # deterministic reduction: a second evaluation is bitwise identical
    L2, g2 = _raw(torch, net, lay, B, T, F)
    assert L2 == L and np.array_equal(g2, g)
    # block weights (the GMRES-run weights of training)
    c = np.random.default_rng(seed).uniform(0.0, 3.0, len(sizes))
    Lc_ref, gc_ref = ol.loss_grad(th, F, lay, B, T, c)
    Lc, gc = _raw(torch, net, lay, B, T, F, c)
    assert Lc == pytest.approx(Lc_ref, rel=1e-12)
    assert np.abs(gc - gc_ref).max() <= 1e-11 * np.abs(gc_ref).max()


def test_raw_layout_is_checked(torch):
    import paper_1311_5202_amd as fdb

    net = fdb.Net(0)
    for sizes, extras in (([65], [0]), ([10], [119])):
        lay, B, T, F = synth.learned_blocks(3, sizes, extras)
        with pytest.raises(fdb.FdaError):
            _raw(torch, net, lay, B, T, F)


def test_block_jacobi_and_learned_solves(torch):
    import paper_1311_5202_amd as fdb
    from paper_1311_5202_amd import _abi

    k = 2.0
    test_plan = _plan(synth.star_surface(12, seed=99), k, precision="both")
    rhs = test_plan.rhs_plane_wave([0.0, 0.0, 1.0])
    x0, i0 = test_plan.solve(rhs, 1e-6, maxit=300, restart=300, precond=0)
    x1, i1 = test_plan.solve(rhs, 1e-6, maxit=300, restart=300, precond=1)
    x3, i3 = test_plan.solve(rhs, 1e-6, maxit=300, restart=300, precond=3)
    rel = lambda x: (torch.linalg.norm(x - x0) / torch.linalg.norm(x0)).item()  # noqa: E731
    print(f"[learned] iterations none {i0['iterations']} block-Jacobi {i1['iterations']} "
          f"overlapping rows {i3['iterations']}", flush=True)
    assert rel(x1) < 1e-5 and rel(x3) < 1e-5
    assert i1["iterations"] < 0.75 * i0["iterations"]
    assert i3["iterations"] < i1["iterations"]

    net = fdb.Net(7)
    # factors not loaded yet: precond 2 is refused
    _, info = test_plan.solve(rhs, 1e-6, maxit=10, restart=10, precond=2, raise_on_fail=False)
    assert info["status"] == _abi.FDA_ENOTSUP

    train = [_plan(synth.star_surface(8 + 2 * s, seed=s), kk) for s, kk in enumerate((1.5, 2.0, 2.5))]
    L_before = net.loss_grad(test_plan)[0]
    first = [net.loss_grad(p)[0] for p in train]
    for _ in range(300):
        last = [net.train_step(p, 3e-3) for p in train]
    L_after = net.loss_grad(test_plan)[0]
    print(f"[learned] training loss {first} -> {last}; held-out {L_before:.1f} -> {L_after:.1f}", flush=True)
    assert all(b < 0.6 * a for a, b in zip(first, last))
    assert L_after < 0.6 * L_before

    net.attach(test_plan)
    x2, i2 = test_plan.solve(rhs, 1e-6, maxit=300, restart=300, precond=2)
    x2f, i2f = test_plan.solve(rhs, 1e-6, maxit=300, restart=300, precond=2, fp32=True)
    print(f"[learned] block-Jacobi + learned coupling {i2['iterations']} (FP32 far field {i2f['iterations']})",
          flush=True)
    assert rel(x2) < 1e-5 and rel(x2f) < 1e-5
    assert i2["iterations"] <= 0.8 * i1["iterations"]
    fdb.Net.detach(test_plan)
    _, info = test_plan.solve(rhs, 1e-6, maxit=10, restart=10, precond=2, raise_on_fail=False)
    assert info["status"] == _abi.FDA_ENOTSUP

    # training data from the method's own GMRES runs: block weights from the
    # Krylov vectors of 20 block-Jacobi steps on each training surface
    L_plain = net.loss_grad(train[0])[0]
    for s_, p in enumerate(train):
        fdb.Net.weight_blocks(p, p.rhs_plane_wave(synth.random_directions(1, 50 + s_)[0]), 20)
    L_weighted = net.loss_grad(train[0])[0]
    fdb.Net.weight_blocks(train[0], None, 0)
    assert net.loss_grad(train[0])[0] == L_plain  # uniform weights restored exactly
    fdb.Net.weight_blocks(train[0], train[0].rhs_plane_wave(synth.random_directions(1, 50)[0]), 20)
    assert net.loss_grad(train[0])[0] == L_weighted  # the same run gives the same weights
    net_k = fdb.Net(7)
    for _ in range(300):
        for p in train:
            net_k.train_step(p, 3e-3)
    net_k.attach(test_plan)
    xk, ik = test_plan.solve(rhs, 1e-6, maxit=300, restart=300, precond=2)
    print(f"[learned] trained with GMRES-run block weights: {ik['iterations']} iterations "
          f"(uniform weights {i2['iterations']}, block-Jacobi {i1['iterations']})", flush=True)
    assert rel(xk) < 1e-5 and ik["iterations"] <= 0.8 * i1["iterations"]
    net_k.close()


def test_plan_gradient_matches_differences(torch):
    import paper_1311_5202_amd as fdb

    plan = _plan(synth.star_surface(8, seed=3), 3.0)
    net = fdb.Net(2)
    th = ol.random_theta(4, out_scale=0.05)
    net.params = th
    L, g = net.loss_grad(plan)
    idx = [0, 100, ol.NF * ol.NH + 3, ol.NF * ol.NH + ol.NH + 17, ol.NPAR - 1]
    h = 1e-5
    for i in idx:
        e = np.zeros(ol.NPAR)
        e[i] = h
        net.params = th + e
        lp = net.loss_grad(plan)[0]
        net.params = th - e
        lm = net.loss_grad(plan)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-5 * max(1.0, abs(g[i])), (i, fd, g[i])
