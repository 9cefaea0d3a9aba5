"""Captured mat-vecs and batches of uneven instances: graph replays and the
one-launch batched mat-vec reproduce the eager mat-vec bitwise; batched
GMRES reproduces the per-instance solves."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available()
    return t


def _plans(count, seed, n_range=(2000, 9000), kd_range=(5.0, 20.0), **opts):
    import paper_1311_5202_amd as fdb

    out = []
    for el, k, kind in synth.instance_batch(count, seed, n_range=n_range, kd_range=kd_range):
        pts, nrm, w = fdb.nystrom_nodes(el)
        print(f"[batch] {kind} N={len(w)} k={k:.2f}", flush=True)
        out.append(fdb.build(pts, nrm, w, k, 1e-4, elements=el, corrections=1, coupling=-1.0, **opts))
    return out


def test_graph_replay_matches_eager(torch):
    plan = _plans(1, 5)[0]
    u1 = torch.from_numpy(synth.random_densities(plan.n, 1)).cuda()
    ref1 = plan.matvec(u1, "BM_H")
    u = u1.clone()
    out = torch.empty_like(u)
    plan.set_graph(True)
    for rep in range(4):
        # new data in the same buffers between replays, eager work in between
        u.copy_(torch.from_numpy(synth.random_densities(plan.n, 10 + rep)).cuda())
        plan.matvec(u, "BM_H", out=out)
        plan.set_graph(False)
        ref = plan.matvec(u, "BM_H")
        plan.set_graph(True)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep
    u.copy_(u1)
    plan.matvec(u, "BM_H", out=out)
    assert torch.equal(out, ref1)
    # GMRES through the captured step: same iterates as without graphs
    b = plan.rhs_plane_wave((0.0, 0.0, 1.0))
    xg, ig = plan.solve(b, 1e-6, maxit=300, restart=300)
    plan.set_graph(False)
    xe, ie = plan.solve(b, 1e-6, maxit=300, restart=300)
    assert ig["iterations"] == ie["iterations"] and torch.equal(xg, xe)
    plan.close()


def test_batched_matvec_and_solve(torch):
    import paper_1311_5202_amd as fdb

    plans = _plans(6, 2, precision="both")
    batch = fdb.Batch(plans)
    us = [torch.from_numpy(synth.random_densities(p.n, i)).cuda() for i, p in enumerate(plans)]
    outs = [torch.empty_like(u) for u in us]
    for rep in range(3):
        for i, u in enumerate(us):
            u.copy_(torch.from_numpy(synth.random_densities(u.numel(), 100 * rep + i)).cuda())
        for fp32 in (False, True):
            batch.matvec(us, "BM_H", outs=outs, fp32=fp32)
            refs = [p.matvec(u, "BM_H", fp32=fp32) for p, u in zip(plans, us)]
            torch.cuda.synchronize()
            for i, (o, r) in enumerate(zip(outs, refs)):
                assert torch.equal(o, r), (rep, fp32, i)
    rhs = [p.rhs_plane_wave((0.0, 0.0, 1.0)) for p in plans]
    xs, info = batch.solve(rhs, 1e-6, maxit=300, restart=300, precond=1)
    print("[batch] iterations", info["iterations"], flush=True)
    for p, b, x, it in zip(plans, rhs, xs, info["iterations"]):
        xr, ir = p.solve(b, 1e-6, maxit=300, restart=300, precond=1)
        assert it == ir["iterations"]
        assert torch.equal(x, xr)
    with pytest.raises(fdb.FdaError):
        fdb.Batch([plans[0], plans[0]])
    batch.close()
    for p in plans:
        p.close()
