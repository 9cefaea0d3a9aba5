"""GPU parity at the mid-size sphere workload and on the translation paths
the small tests do not reach: N = 196,608 (octahedral sphere n = 64), k = 50,
leaf <= 64, eps = 1e-4 in FP64 and FP32; scratch cut into many slabs; three
high-frequency levels with nested-wedge M2M between them.  Errors are the
relative L2 error over sampled target rows against the oracle (section 5.1
error measure)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mie, near

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available()
    return t


def _hf_levels_with_m2l(stats):
    return [L["w"] for L in stats["levels"] if L["hf"] and L["m2l_pairs"] > 0]


@pytest.mark.timeout(600)
def test_mid_size_sphere_fp64_fp32_and_solve(torch):
    import paper_1311_5202_amd as fdb

    k = 50.0
    el = synth.octa_sphere(64)
    pts, nrm, w = fdb.nystrom_nodes(el)
    n = len(w)
    assert n == 196_608
    print(f"[c2] N={n} k={k}: building", flush=True)
    plan = fdb.build(pts, nrm, w, k, 1e-4, elements=el, corrections=1, precision="both", coupling=-1.0)
    st = plan.stats()
    print("[c2] HF levels with M2L:", _hf_levels_with_m2l(st), flush=True)
    assert len(_hf_levels_with_m2l(st)) >= 2
    u = synth.random_densities(n, 1)
    ud = torch.from_numpy(u).cuda()
    rows = np.sort(np.random.default_rng(11).choice(n, 400, replace=False))
    for op, oop, coefs in (("RAW_H", "H", (0.0, 1.0, 1.0, -1j / k)), ("RAW_G", "G", (1.0, 0.0, 1.0, -1j / k)),
                           ("RAW_T1", "T1", (1.0, -1j / k, 1.0, 0.0))):
        ref = oracle.dense_rows(pts, nrm, w, u, k, oop, rows=rows, coefs=coefs)
        for fp32 in (False, True):
            got = plan.matvec(ud, op, fp32=fp32).cpu().numpy()[rows]
            err = oracle.rel_l2(got, ref)
            print(f"[c2] {op} FP32={fp32}: {err:.3e}", flush=True)
            assert err <= 1e-4, (op, fp32, err)
    sub = rows[::10]
    refc = near.corrected_rows(el, u, k, "H", rows=sub, coefs=(0.0, 1.0, 1.0, -1j / k))
    got = plan.matvec(ud, "BM_H").cpu().numpy()[sub]
    err = oracle.rel_l2(got, refc)
    print(f"[c2] BM_H over {len(sub)} rows: {err:.3e}", flush=True)
    assert err <= 1e-4
    d = np.array([0.0, 0.0, 1.0])
    b = plan.rhs_plane_wave(d)
    x, info = plan.solve(b, 1e-4, maxit=200, restart=200)
    xs = x.cpu().numpy()
    # the oracle's corrected operator applied to the GPU solution reproduces b
    Ax = near.corrected_rows(el, xs, k, "H", rows=sub, coefs=(0.0, 1.0, 1.0, -1j / k))
    res = oracle.rel_l2(Ax, b.cpu().numpy()[sub])
    r = np.linalg.norm(pts[rows], axis=1)
    mie_err = oracle.rel_l2(xs[rows], mie.mie_hard_total_surface(k, (pts[rows] @ d) / r))
    print(f"[c2] GMRES {info['iterations']} iterations, oracle residual {res:.2e}, Mie {mie_err:.2e}", flush=True)
    assert info["status"] == 0 and res <= 5e-4
    assert mie_err <= 2e-2
    plan.close()


@pytest.mark.timeout(600)
def test_many_slabs_and_three_hf_levels(torch):
    """Sphere n = 32 (N = 49,152) at k = 160 (kD = 320, about 3 nodes per
    wavelength: the raw sums do not care), every far pair translated
    (p2p_threshold < 0), has M2L on three high-frequency levels (w = lambda,
    2 lambda, 4 lambda) with nested-wedge M2M and L2L between them; with
    1 MiB slabs every translation runs over many slabs and the result is
    bitwise that of one slab, and both match the oracle.  Translating every
    far pair of such small leaves over three levels adds up truncation
    errors (at eps = 1e-4 the error is 1.9e-4, inside the 3.7 eps that
    Table 1 reports for the improved method), so the plan uses eps = 1e-5."""
    import paper_1311_5202_amd as fdb

    k = 160.0
    el = synth.octa_sphere(32)
    pts, nrm, w = fdb.nystrom_nodes(el)
    n = len(w)
    u = synth.random_densities(n, 3)
    ud = torch.from_numpy(u).cuda()
    rows = np.sort(np.random.default_rng(5).choice(n, 300, replace=False))
    outs = {}
    for slab in (0, 1):
        print(f"[slabs] N={n} k={k} slab_mb={slab}: building", flush=True)
        plan = fdb.build(pts, nrm, w, k, 1e-5, precision="both", slab_mb=slab, p2p_threshold=-1.0)
        hf = _hf_levels_with_m2l(plan.stats())
        print("[slabs] HF levels with M2L:", hf, flush=True)
        assert len(hf) >= 3
        outs[slab] = {(op, f): plan.matvec(ud, op, fp32=f).cpu().numpy()
                      for op in ("RAW_H", "RAW_G") for f in (False, True)}
        plan.close()
    for key in outs[0]:
        assert np.array_equal(outs[0][key], outs[1][key]), key
    for op, oop in (("RAW_H", "H"), ("RAW_G", "G")):
        ref = oracle.dense_rows(pts, nrm, w, u, k, oop, rows=rows)
        for f in (False, True):
            err = oracle.rel_l2(outs[1][(op, f)][rows], ref)
            print(f"[slabs] {op} FP32={f}: {err:.3e}", flush=True)
            assert err <= 1e-4


@pytest.mark.timeout(600)
def test_elongated_body_at_kd_1000(torch):
    """Stand-in for the large non-spherical body of section 5.3: a prolate
    ellipsoid with axes 1 : 1 : 8 (D = 16) at kD = 1000 (k = 62.5), N =
    442,368 nodes.  Its octree is anisotropic (many cubes along the axis,
    high-frequency levels from lambda up), and the raw H sum must match the
    oracle's dense sums to 1e-4 over 200 seeded rows in FP64 and FP32."""
    import paper_1311_5202_amd as fdb

    el = synth.ellipsoid(96, 8.0)
    pts, nrm, w = fdb.nystrom_nodes(el)
    n = len(w)
    k = 1000.0 / 16.0
    print(f"[ellipsoid] N={n} k={k}: building", flush=True)
    plan = fdb.build(pts, nrm, w, k, 1e-4, precision="both", verbose=1)
    st = plan.stats()
    hf = _hf_levels_with_m2l(st)
    print("[ellipsoid] HF levels with M2L:", hf, "s:", [L["s"] for L in st["levels"] if L["s"]], flush=True)
    assert len(hf) >= 3
    u = synth.random_densities(n, 8)
    ud = torch.from_numpy(u).cuda()
    rows = np.sort(np.random.default_rng(9).choice(n, 200, replace=False))
    ref = oracle.dense_rows(pts, nrm, w, u, k, "H", rows=rows)
    for fp32 in (False, True):
        err = oracle.rel_l2(plan.matvec(ud, "RAW_H", fp32=fp32).cpu().numpy()[rows], ref)
        print(f"[ellipsoid] raw H FP32={fp32}: {err:.3e}", flush=True)
        assert err <= 1e-4
    plan.close()


@pytest.mark.timeout(600)
def test_mie_error_falls_with_resolution(torch):
    """Where the remaining error of the sphere solve comes from: at a fixed
    k = 50 (kD = 100) the plane-wave solve (GMRES to 1e-6) is compared with
    the Mie series at 5 to 20 nodes per wavelength (octahedral n = 21 ... 83,
    the C5 sphere has about 7).  The FDA error against the dense oracle stays
    near 1e-5 at every resolution, while the error against Mie falls with the
    mesh size at about third order: the Nystrom discretisation sets it."""
    import paper_1311_5202_amd as fdb

    k = 50.0
    d = np.array([0.0, 0.0, 1.0])
    res = []
    for n_oct in (21, 29, 41, 58, 83):
        el = synth.octa_sphere(n_oct)
        pts, nrm, w = fdb.nystrom_nodes(el)
        ppw = np.sqrt(len(w) / (4 * np.pi)) * (2 * np.pi / k)   # nodes per wavelength
        plan = fdb.build(pts, nrm, w, k, 1e-4, elements=el, corrections=1, coupling=-1.0)
        x, info = plan.solve(plan.rhs_plane_wave(d), 1e-6, maxit=300, restart=300)
        rows = np.sort(np.random.default_rng(1).choice(len(w), 2000, replace=False))
        r = np.linalg.norm(pts[rows], axis=1)
        err = oracle.rel_l2(x.cpu().numpy()[rows], mie.mie_hard_total_surface(k, (pts[rows] @ d) / r))
        u = synth.random_densities(len(w), 2)
        rr = rows[:200]
        eps_a = oracle.rel_l2(plan.matvec(torch.from_numpy(u).cuda(), "RAW_H").cpu().numpy()[rr],
                              oracle.dense_rows(pts, nrm, w, u, k, "H", rows=rr, coefs=(0.0, 1.0, 1.0, -1j / k)))
        print(f"[mie] n={n_oct} N={len(w)} {ppw:.1f} nodes/wavelength: GMRES {info['iterations']}, "
              f"Mie error {err:.3e}, FDA eps_a {eps_a:.2e}", flush=True)
        res.append((ppw, err, eps_a))
        plan.close()
    ppw, err, ea = (np.array(v) for v in zip(*res))
    slope = -np.polyfit(np.log(ppw), np.log(err), 1)[0]
    print(f"[mie] fitted order {slope:.2f}; error at 7 nodes/wavelength "
          f"{np.exp(np.polyval(np.polyfit(np.log(ppw), np.log(err), 1), np.log(7.0))):.2e}", flush=True)
    assert np.all(np.diff(err) < 0) and slope >= 2.0
    assert np.all(ea <= 1e-4)
