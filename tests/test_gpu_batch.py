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
    datas = [torch.from_numpy(synth.random_densities(plan.n, 10 + rep)).cuda() for rep in range(4)]
    u = torch.empty_like(datas[0])
    out = torch.empty_like(u)
    # eager references first (graphs off)
    refs = []
    for d in datas:
        u.copy_(d)
        refs.append(plan.matvec(u, "BM_H"))
    assert plan.stats()["graphs_captured"] == 0
    plan.set_graph(True)
    for rep, d in enumerate(datas):
        # new data in the same buffers between replays, eager work in between:
        # the first call captures fda_matvec into a graph, the others replay it
        u.copy_(d)
        plan.matvec(u, "BM_H", out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, refs[rep]), rep
        assert plan.stats()["graphs_captured"] == 1
    # GMRES through the captured step: same iterates as without graphs
    b = plan.rhs_plane_wave((0.0, 0.0, 1.0))
    xg, ig = plan.solve(b, 1e-6, maxit=300, restart=300)
    plan.set_graph(False)
    assert plan.stats()["graphs_captured"] == 0
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
    # operators are validated as by fda_matvec: BM_G needs the G table
    # (corrections & 2), unknown bits are refused
    from paper_1311_5202_amd import _abi
    with pytest.raises(fdb.FdaError) as e:
        batch.matvec(us, "BM_G", outs=outs)
    assert e.value.code == _abi.FDA_EINVAL
    with pytest.raises(fdb.FdaError) as e:
        batch.solve(rhs, 1e-6, maxit=10, restart=10, op="BM_G")
    assert e.value.code == _abi.FDA_EINVAL
    ptrs = batch._ptrs(us)
    optrs = batch._ptrs(outs)
    assert _abi.lib().fda_batch_matvec(batch._h, 0x1003, ptrs, optrs, None) == _abi.FDA_EINVAL
    assert _abi.lib().fda_batch_matvec(batch._h, 7, ptrs, optrs, None) == _abi.FDA_EINVAL
    batch.close()
    for p in plans:
        p.close()


def test_batched_instances_match_the_oracle(torch):
    """Uneven instances of the batch workload (sphere, prolate ellipsoid,
    star; different N and k) applied in one batched launch agree with the
    oracle: raw H sums with the dense FP64 sums (FP64 and FP32 far field) and
    the corrected Burton-Miller operator with the oracle's independently
    integrated rows (section 5.1 error measure over sampled rows)."""
    import oracle
    import paper_1311_5202_amd as fdb

    inst = synth.instance_batch(4, 2, n_range=(4000, 12000), kd_range=(5.0, 30.0))
    plans, els = [], []
    for el, k, kind in inst:
        pts, nrm, w = fdb.nystrom_nodes(el)
        print(f"[batch-oracle] {kind} N={len(w)} k={k:.2f}", flush=True)
        plans.append(fdb.build(pts, nrm, w, k, 1e-4, elements=el, corrections=1, precision="both"))
        els.append((el, pts, nrm, w, k))
    batch = fdb.Batch(plans)
    us = [torch.from_numpy(synth.random_densities(p.n, 40 + i)).cuda() for i, p in enumerate(plans)]
    raw64 = [o.cpu().numpy() for o in batch.matvec(us, "RAW_H")]
    raw32 = [o.cpu().numpy() for o in batch.matvec(us, "RAW_H", fp32=True)]
    bmh = [o.cpu().numpy() for o in batch.matvec(us, "BM_H")]
    for i, ((el, pts, nrm, w, k), u) in enumerate(zip(els, us)):
        un = u.cpu().numpy()
        rows = np.random.default_rng(i).choice(len(w), 300, replace=False)
        ref = oracle.dense_rows(pts, nrm, w, un, k, "H", rows=rows)
        e64 = oracle.rel_l2(raw64[i][rows], ref)
        e32 = oracle.rel_l2(raw32[i][rows], ref)
        rows_c = rows[:30]
        refc = oracle.near.corrected_rows(el, un, k, "H", rows=rows_c)
        ebm = oracle.rel_l2(bmh[i][rows_c], refc)
        print(f"[batch-oracle] instance {i}: raw H FP64 {e64:.2e} FP32 {e32:.2e}; BM_H {ebm:.2e}", flush=True)
        assert e64 <= 1e-4 and e32 <= 1e-4 and ebm <= 1e-4, (i, e64, e32, ebm)
    batch.close()
    for p in plans:
        p.close()
