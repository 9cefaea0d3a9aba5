"""Parity at the full benchmark size (unit sphere, N = 4,009,008, k = 500,
kD = 1000), in the configuration bench.py times: sampled rows of the raw H
sum (FP64 and FP32) and of the corrected BM_H operator against the oracle,
and the plane-wave solve against the Mie series.  The plan build takes
two to three minutes."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mie, near

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
def test_full_size_sampled_rows_and_mie():
    import torch

    import paper_1311_5202_amd as fdb

    k = 500.0
    el = synth.octa_sphere(289)
    pts, nrm, w = fdb.nystrom_nodes(el)
    n = len(w)
    print(f"[full] N={n} k={k}: building", flush=True)
    plan = fdb.build(pts, nrm, w, k, 1e-4, elements=el, corrections=1, precision="both", coupling=-1.0, verbose=1)
    u = synth.random_densities(n, 1)
    ud = torch.from_numpy(u).cuda()
    rows = np.sort(np.random.default_rng(7).choice(n, 200, replace=False))
    coefs = (0.0, 1.0, 1.0, -1j / k)  # alpha = -i/k, as the plan (coupling = -1)
    ref = oracle.dense_rows(pts, nrm, w, u, k, "H", rows=rows, coefs=coefs)
    for fp32 in (False, True):
        got = plan.matvec(ud, "RAW_H", fp32=fp32).cpu().numpy()[rows]
        err = oracle.rel_l2(got, ref)
        print(f"[full] raw H, FP32={fp32}: eps_a over 200 rows = {err:.3e}", flush=True)
        assert err <= 1e-4
    sub = rows[::5]
    refc = near.corrected_rows(el, u, k, "H", rows=sub, coefs=coefs)
    got = plan.matvec(ud, "BM_H").cpu().numpy()[sub]
    err = oracle.rel_l2(got, refc)
    print(f"[full] BM_H with corrections: rel L2 over {len(sub)} rows = {err:.3e}", flush=True)
    assert err <= 1e-4
    d = np.array([0.0, 0.0, 1.0])
    b = plan.rhs_plane_wave(d)
    x, info = plan.solve(b, 1e-4, maxit=100, restart=100)
    xs = x.cpu().numpy()[rows]
    r = np.linalg.norm(pts[rows], axis=1)
    u_mie = mie.mie_hard_total_surface(k, (pts[rows] @ d) / r)
    err = oracle.rel_l2(xs, u_mie)
    print(f"[full] GMRES {info['iterations']} iterations; total field vs Mie over 200 nodes: {err:.3e}", flush=True)
    # about 7 nodes per wavelength: the Nystrom discretisation, not the FDA, sets this error
    assert info["status"] == 0 and err <= 5e-2
    plan.close()
