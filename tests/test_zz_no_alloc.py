"""fda_matvec_noalloc, the mat-vec that keeps its per-pair translation
results in the library's static device scratch, called through the C ABI:
two calls in a row, the second on a smaller plan, each equal to fda_matvec on
the same plan (the same kernels in the same order, so bitwise), and its size
limit reported as an argument error."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _plan(n_oct, k, **opts):
    import paper_1311_5202_amd as fdb

    el = synth.octa_sphere(n_oct)
    pts, nrm, w = fdb.nystrom_nodes(el)
    print(f"[noalloc] N={len(w)} k={k} {opts}", flush=True)
    return fdb.build(pts, nrm, w, k, 1e-4, elements=el, corrections=1, precision="both", **opts)


def test_noalloc_matvec_matches_fda_matvec():
    import torch

    from paper_1311_5202_amd import _abi

    L = _abi.lib()
    big = _plan(24, 40.0, slab_mb=64)
    small = _plan(10, 8.0, slab_mb=64)
    for plan, seed in ((big, 1), (small, 2)):
        u = torch.from_numpy(synth.random_densities(plan.n, seed)).cuda()
        for op, fp32 in (("BM_H", False), ("RAW_G", False), ("BM_H", True)):
            out = torch.full_like(u, complex(float("nan"), float("nan")))
            code = plan._op(op, fp32)
            rc = L.fda_matvec_noalloc(plan._h, code, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                      None)
            assert rc == _abi.FDA_OK, L.fda_last_error().decode()
            ref = torch.empty_like(u)
            assert L.fda_matvec(plan._h, code, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(ref.data_ptr()),
                                None) == _abi.FDA_OK
            torch.cuda.synchronize()
            print(f"[noalloc] N={plan.n} {op} fp32={fp32}: max |diff| "
                  f"{(out - ref).abs().max().item():.3e}", flush=True)
            assert torch.equal(out, ref), (plan.n, op, fp32)
    # arguments are checked before any device work
    u = torch.zeros(small.n, dtype=torch.complex128, device="cuda")
    p = ctypes.c_void_p(u.data_ptr())
    assert L.fda_matvec_noalloc(small._h, 0x1003, p, ctypes.c_void_p(u.data_ptr() + 16), None) == _abi.FDA_EINVAL
    assert L.fda_matvec_noalloc(small._h, 3, p, p, None) == _abi.FDA_EINVAL
    assert L.fda_matvec_noalloc(None, 3, p, p, None) == _abi.FDA_EINVAL
    small.close()
    big.close()


def test_noalloc_rejects_plans_beyond_the_static_scratch():
    """A plan whose largest slab needs more than 256 MiB is refused with
    FDA_EINVAL and a message naming the limit (N = 196,608, k = 50: the
    default 1 GiB slab holds every level at once)."""
    import torch

    from paper_1311_5202_amd import _abi

    L = _abi.lib()
    plan = _plan(64, 50.0)
    u = torch.from_numpy(synth.random_densities(plan.n, 3)).cuda()
    out = torch.empty_like(u)
    rc = L.fda_matvec_noalloc(plan._h, 3, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()), None)
    msg = L.fda_last_error().decode()
    print("[noalloc] big plan:", rc, msg, flush=True)
    stats = plan.stats()
    assert rc == _abi.FDA_EINVAL and "slab_mb" in msg
    plan.close()
