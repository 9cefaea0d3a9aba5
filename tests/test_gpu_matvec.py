"""GPU parity of the fast directional mat-vec against the oracle's dense
FP64 sums (section 5.1 error measure: relative L2 over target rows)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

OPS = (("RAW_H", "H"), ("RAW_G", "G"), ("RAW_T1", "T1"))


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available()
    return t


def _geom(n):
    import paper_1311_5202_amd as fdb

    el = synth.octa_sphere(n)
    pts, nrm, w = fdb.nystrom_nodes(el)
    return el, pts, nrm, w


def _run(torch, plan, u, op):
    return plan.matvec(torch.from_numpy(u).cuda(), op).cpu().numpy()


@pytest.mark.parametrize("n", [3, 8])
def test_direct_sum_equals_oracle(torch, n):
    """far_field = 0: one leaf, every pair by the P2P kernel (ragged tiles at n = 3)."""
    import paper_1311_5202_amd as fdb

    _, pts, nrm, w = _geom(n)
    k = 5.0
    print(f"[direct] N={len(w)} k={k}", flush=True)
    plan = fdb.build(pts, nrm, w, k, 1e-4, far_field=0)
    u = synth.random_densities(len(w), 0)
    for op, oop in OPS:
        got = _run(torch, plan, u, op)
        ref = oracle.dense_rows(pts, nrm, w, u, k, oop)
        assert oracle.rel_l2(got, ref) < 1e-13, op
        assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref)), op
    plan.close()


def test_fda_small_sphere_all_rows(torch):
    """N = 3072, k = 5 (low-frequency levels only): every row within 1e-4."""
    import paper_1311_5202_amd as fdb

    _, pts, nrm, w = _geom(8)
    k = 5.0
    print(f"[fda-lf] N={len(w)} k={k}", flush=True)
    plan = fdb.build(pts, nrm, w, k, 1e-4)
    u = synth.random_densities(len(w), 0)
    for op, oop in OPS:
        got = _run(torch, plan, u, op)
        ref = oracle.dense_rows(pts, nrm, w, u, k, oop)
        err = oracle.rel_l2(got, ref)
        print(op, err)
        assert err <= 1e-4, op
    st = plan.stats()
    assert st["N"] == len(w)
    plan.close()


def test_fda_high_frequency_sampled_rows(torch):
    """N = 27,648, k = 25: one high-frequency (directional) level plus two
    low-frequency levels; 400 seeded rows against the oracle."""
    import paper_1311_5202_amd as fdb

    _, pts, nrm, w = _geom(24)
    k = 25.0
    print(f"[fda-hf] N={len(w)} k={k}", flush=True)
    plan = fdb.build(pts, nrm, w, k, 1e-4)
    st = plan.stats()
    assert any(L["hf"] and L["m2l_pairs"] > 0 for L in st["levels"])
    u = synth.random_densities(len(w), 1)
    rows = np.sort(np.random.default_rng(7).choice(len(w), 400, replace=False))
    for op, oop in OPS:
        got = _run(torch, plan, u, op)
        ref = oracle.dense_rows(pts, nrm, w, u, k, oop, rows=rows)
        err = oracle.rel_l2(got[rows], ref)
        print(op, err)
        assert err <= 1e-4, op
    plan.close()


def test_m2l_kernels_agree_and_tiles_are_deterministic(torch):
    """The translation schedules (operator chunks with per-pair results
    summed per output, on the wavefront or on the workgroup chunk kernel;
    operator chunks with atomic adds; per-target GEMV; workgroup target
    tiles) apply the same operators; the partial-sum and tiled ones are
    bitwise reproducible."""
    import paper_1311_5202_amd as fdb

    _, pts, nrm, w = _geom(12)
    k = 16.0
    u = torch.from_numpy(synth.random_densities(len(w), 3)).cuda()
    outs = {}
    modes = {"partial": 3, "partial_wg": 3, "chunks": 0, "gemv": 1, "tiles": 2}
    for name, tile, ck in (("partial", 0, 0), ("partial_wg", 0, 1), ("chunks", 1, 0), ("gemv", -1, 0),
                           ("tiles", 16, 0)):
        print(f"[m2l] schedule {name}", flush=True)
        plan = fdb.build(pts, nrm, w, k, 1e-4, m2l_tile=tile, chunk_kernel=ck)
        st = plan.stats()
        assert st["m2l_mode"] == modes[name]
        if name.startswith("partial"):
            kernels = {t["kernel"] for key in ("m2l_autotune", "m2m_autotune", "l2l_autotune") for t in st[key]}
            print(f"[m2l] {name}: chunk kernels {sorted(kernels)}", flush=True)
            assert ("wavefront" in kernels) == (ck == 0)
        a = plan.matvec(u, "RAW_H").cpu().numpy()
        b = plan.matvec(u, "RAW_H").cpu().numpy()
        if name in ("partial", "partial_wg", "tiles"):
            assert np.array_equal(a, b)
        else:
            assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))
        outs[name] = a
        plan.close()
    ref = outs["gemv"]
    for name in ("partial", "partial_wg", "chunks", "tiles"):
        assert np.max(np.abs(outs[name] - ref)) <= 1e-12 * np.max(np.abs(ref)), name


def test_fp32_far_and_near_field(torch):
    """FP32 point sums and far field (FDA_OP_FP32) on a plan holding both
    precisions: within 1e-4 of the FP64 oracle; the difference to the FP64
    path is reported."""
    import paper_1311_5202_amd as fdb

    _, pts, nrm, w = _geom(24)
    k = 25.0
    plan = fdb.build(pts, nrm, w, k, 1e-4, precision="both")
    u = synth.random_densities(len(w), 4)
    ud = torch.from_numpy(u).cuda()
    rows = np.sort(np.random.default_rng(8).choice(len(w), 300, replace=False))
    for op, oop in OPS:
        g64 = plan.matvec(ud, op).cpu().numpy()
        g32 = plan.matvec(ud, op, fp32=True).cpu().numpy()
        ref = oracle.dense_rows(pts, nrm, w, u, k, oop, rows=rows)
        e32 = oracle.rel_l2(g32[rows], ref)
        d = oracle.rel_l2(g32, g64)
        print(op, "fp32 vs oracle", e32, "fp32 vs fp64", d)
        assert e32 <= 1e-4 and d <= 5e-5, op
    plan.close()
    # an FP64-only plan refuses the FP32 flag
    from paper_1311_5202_amd import _abi

    plan = fdb.build(pts[:600], nrm[:600], w[:600], k, 1e-4)
    with pytest.raises(_abi.FdaError):
        plan.matvec(torch.from_numpy(u[:600]).cuda(), "RAW_H", fp32=True)
    plan.close()


@pytest.mark.parametrize("n_oct,k_over_pi,eps,original", [
    (39, 8, 1e-4, 0), (39, 8, 1e-6, 0), (39, 8, 1e-4, 1), (78, 16, 1e-4, 0)])
@pytest.mark.timeout(600)
def test_table1_accuracy_against_paper(torch, n_oct, k_over_pi, eps, original):
    """Table-1 summation (section 5.1, eq. eq_sum) at the table's two smaller
    sizes: N ~ 73,728 (k = 8 pi; eps = 1e-4, 1e-6) and ~294,912 (k = 16 pi;
    eps = 1e-4) nodes at about 20 per wavelength, 200 seeded targets (the
    other sizes and eps = 1e-8 run in the Table-1 benchmark); at the
    smaller size also the original method of the table (original = 1: no
    matrix reduction, no low-rank M2L).  The error must not exceed the
    paper's value for the same method (tests/golden/table1_eps_a.json) by
    more than 2x."""
    import json
    import os

    import paper_1311_5202_amd as fdb

    with open(os.path.join(os.path.dirname(__file__), "golden", "table1_eps_a.json")) as f:
        rows = json.load(f)["rows"]
    n_paper = {8: 73728, 16: 294912}[k_over_pi]
    ref_eps_a = next(r[3 + (0 if original else 1)] for r in rows if r[0] == n_paper and r[2] == eps)
    _, pts, nrm, w = _geom(n_oct)  # N = 73,008 / 292,032
    k = k_over_pi * np.pi
    print(f"[table1] N={len(w)} k={k:.3f} eps={eps} original={original}", flush=True)
    plan = fdb.build(pts, nrm, w, k, eps, original=original, verbose=1)
    st = plan.stats()
    print("[table1] s per level:", [L["s"] for L in st["levels"] if L["s"]], flush=True)
    u = synth.random_densities(len(w), 3)
    rows_t = np.sort(np.random.default_rng(7).choice(len(w), 200, replace=False))
    got = _run(torch, plan, u, "RAW_T1")[rows_t]
    ref = oracle.dense_rows(pts, nrm, w, u, k, "T1", rows=rows_t)
    err = oracle.rel_l2(got, ref)
    print(f"[table1] eps_a {err:.3e} (paper {'original' if original else 'improved'} {ref_eps_a:.2e})", flush=True)
    assert err <= 2 * ref_eps_a
    plan.close()


@pytest.mark.parametrize("chunk_kernel", [0, 1])
def test_autotuned_chunk_shapes_give_identical_results(torch, chunk_kernel):
    """The builder's autotuner picks 16 or 32 pairs per chunk per level for
    M2L, M2M and L2L (per wavefront or per workgroup); either shape gives
    bitwise the same mat-vec, and the choices are reported."""
    import paper_1311_5202_amd as fdb

    _, pts, nrm, w = _geom(16)
    k = 24.0
    u = torch.from_numpy(synth.random_densities(len(w), 5)).cuda()
    ref_plan = fdb.build(pts, nrm, w, k, 1e-4, autotune=0, chunk_kernel=chunk_kernel)
    ref = ref_plan.matvec(u, "RAW_H")
    st0 = ref_plan.stats()
    assert st0["m2l_autotune"] == [] and st0["m2m_autotune"] == [] and st0["l2l_autotune"] == []
    ref_plan.close()
    plan = fdb.build(pts, nrm, w, k, 1e-4, autotune=1, chunk_kernel=chunk_kernel)
    st = plan.stats()
    for key in ("m2l_autotune", "m2m_autotune", "l2l_autotune"):
        tuned = st[key]
        print("[autotune]", key, tuned, flush=True)
        assert tuned and all(t["pairs_per_chunk"] in (16, 32) for t in tuned), key
    assert torch.equal(plan.matvec(u, "RAW_H"), ref)
    plan.close()


@pytest.mark.parametrize("shape", ["ellipsoid", "star"])
def test_fda_adaptive_surfaces_sampled_rows(torch, shape):
    """Non-spherical surfaces (prolate ellipsoid 1:1:4, seeded star-shaped
    surface) give adaptive trees whose leaves sit on several levels, so the
    grouped S2M/L2T kernels see groups of different templates; 300 seeded
    rows of every raw operator against the oracle."""
    import paper_1311_5202_amd as fdb

    el = synth.ellipsoid(16, 4.0) if shape == "ellipsoid" else synth.star_surface(16, 3)
    pts, nrm, w = fdb.nystrom_nodes(el)
    k = 20.0
    print(f"[adaptive] {shape} N={len(w)} k={k}", flush=True)
    plan = fdb.build(pts, nrm, w, k, 1e-4, precision="both")
    u = synth.random_densities(len(w), 8)
    ud = torch.from_numpy(u).cuda()
    rows = np.sort(np.random.default_rng(9).choice(len(w), 300, replace=False))
    for op, oop in OPS:
        ref = oracle.dense_rows(pts, nrm, w, u, k, oop, rows=rows)
        for fp32 in (False, True):
            got = plan.matvec(ud, op, fp32=fp32).cpu().numpy()[rows]
            err = oracle.rel_l2(got, ref)
            print(shape, op, "fp32" if fp32 else "fp64", err, flush=True)
            assert err <= 1e-4, (op, fp32)
    plan.close()
