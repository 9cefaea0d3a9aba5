"""Thin Python binding over the C ABI: argument marshalling only.  Device
memory and streams come from PyTorch; every step of the mat-vec and solver
runs in the library's HIP kernels."""

from __future__ import annotations

import ctypes
import json

import numpy as np

from . import _abi


def nystrom_nodes(elements: np.ndarray):
    """Nodes, normals (into the body) and weights of the six-point rule on each
    curved quadratic element (bem_nystrom_nodes)."""
    el = np.ascontiguousarray(elements, dtype=np.float64).reshape(-1, 6, 3)
    ne = el.shape[0]
    pts = np.empty((6 * ne, 3))
    nrm = np.empty((6 * ne, 3))
    w = np.empty(6 * ne)
    _abi.check(_abi.lib().bem_nystrom_nodes(ne, el.ctypes.data, pts.ctypes.data, nrm.ctypes.data, w.ctypes.data))
    return pts, nrm, w


def near_correction(elements, pts, nrm, w, k: float, op: str = "BM_H", coupling: float = 1.0):
    """Host CSR table (row_ptr, col, val) of the locally corrected near field
    (bem_near_correction), caller node order; alpha = i coupling / k."""
    import scipy.sparse as sp

    el = np.ascontiguousarray(elements, dtype=np.float64).reshape(-1, 6, 3)
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    nrm = np.ascontiguousarray(nrm, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    L = _abi.lib()
    nnz = ctypes.c_int64(0)
    args = (el.shape[0], el.ctypes.data, pts.ctypes.data, nrm.ctypes.data, w.ctypes.data, float(k), _abi.OPS[op],
            float(coupling))
    _abi.check(L.bem_near_correction(*args, ctypes.byref(nnz), None, None, None))
    n = 6 * el.shape[0]
    rp = np.empty(n + 1, dtype=np.int64)
    col = np.empty(nnz.value, dtype=np.int64)
    val = np.empty(nnz.value, dtype=np.complex128)
    _abi.check(L.bem_near_correction(*args, ctypes.byref(nnz), rp.ctypes.data, col.ctypes.data, val.ctypes.data))
    return sp.csr_matrix((val, col, rp), shape=(n, n))


def _stream_ptr(stream):
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check_vec(t, n):
    import torch

    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()
            and t.numel() == n):
        raise ValueError(f"expected a contiguous complex128 CUDA tensor of length {n}")


class Plan:
    """A built fast directional Burton-Miller operator on the current GPU."""

    def __init__(self, pts, nrm, w, k: float, eps: float, elements=None, **opts):
        L = _abi.lib()
        self._pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        self._nrm = np.ascontiguousarray(nrm, dtype=np.float64).reshape(-1, 3)
        self._w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
        self.n = int(self._w.shape[0])
        self.k = float(k)
        self.eps = float(eps)
        el = None if elements is None else np.ascontiguousarray(elements, dtype=np.float64).reshape(-1, 6, 3)
        g = _abi.FdaGeometry(self.n, self._pts.ctypes.data, self._nrm.ctypes.data, self._w.ctypes.data,
                             0 if el is None else el.shape[0], None if el is None else el.ctypes.data)
        o = _abi.FdaOpts()
        _abi.check(L.fda_default_opts(ctypes.byref(o)))
        if isinstance(opts.get("precision"), str):
            opts["precision"] = _abi.PREC[opts["precision"]]
        for key, val in opts.items():
            if not hasattr(o, key):
                raise TypeError(f"unknown option {key}")
            setattr(o, key, val)
        h = ctypes.c_void_p()
        _abi.check(L.fda_build(ctypes.byref(g), self.k, self.eps, ctypes.byref(o), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _abi.lib().fda_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _op(op: str, fp32: bool) -> int:
        return _abi.OPS[op] | (_abi.FDA_OP_FP32 if fp32 else 0)

    def matvec(self, u, op: str = "RAW_H", out=None, stream=None, fp32: bool = False):
        import torch

        _check_vec(u, self.n)
        if out is None:
            out = torch.empty_like(u)
        _check_vec(out, self.n)
        _abi.check(_abi.lib().fda_matvec(self._h, self._op(op, fp32), ctypes.c_void_p(u.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def matvec_noalloc(self, u, op: str = "RAW_H", out=None, stream=None, fp32: bool = False):
        """fda_matvec_noalloc: the mat-vec with the library's static scratch
        (out must be supplied by callers that may not allocate)."""
        import torch

        _check_vec(u, self.n)
        if out is None:
            out = torch.empty_like(u)
        _check_vec(out, self.n)
        _abi.check(_abi.lib().fda_matvec_noalloc(self._h, self._op(op, fp32), ctypes.c_void_p(u.data_ptr()),
                                                 ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def rhs_plane_wave(self, d, stream=None):
        import torch

        out = torch.empty(self.n, dtype=torch.complex128, device="cuda")
        dd = (ctypes.c_double * 3)(*[float(v) for v in d])
        _abi.check(_abi.lib().fda_rhs_plane_wave(self._h, dd, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def rhs_neumann(self, q, stream=None):
        """(S + alpha M) q - alpha q / 2 with the corrected operators
        (fda_rhs_neumann): the right-hand side of a radiation problem."""
        import torch

        _check_vec(q, self.n)
        out = torch.empty_like(q)
        _abi.check(_abi.lib().fda_rhs_neumann(self._h, ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                              _stream_ptr(stream)))
        return out

    def solve(self, rhs, tol: float, maxit: int = 200, restart: int = 200, op: str = "BM_H", precond: int = 0,
              stream=None, raise_on_fail: bool = True, fp32: bool = False):
        import torch

        _check_vec(rhs, self.n)
        x = torch.empty_like(rhs)
        it = ctypes.c_int(0)
        rel = ctypes.c_double(0)
        hist = np.zeros(maxit + 1)
        rc = _abi.lib().bm_solve(self._h, self._op(op, fp32), ctypes.c_void_p(rhs.data_ptr()), float(tol), int(maxit),
                                 int(restart), int(precond), ctypes.c_void_p(x.data_ptr()), ctypes.byref(it),
                                 ctypes.byref(rel), hist.ctypes.data_as(ctypes.c_void_p), _stream_ptr(stream))
        info = {"status": rc, "iterations": it.value, "relres": rel.value, "history": hist[: it.value + 1].copy()}
        if rc != _abi.FDA_OK and raise_on_fail:
            _abi.check(rc)
        return x, info

    def set_graph(self, on: bool = True):
        """Replay mat-vecs (and bm_solve steps) from captured HIP graphs."""
        _abi.check(_abi.lib().fda_set_graph(self._h, 1 if on else 0))

    def set_timing(self, on: bool = True):
        _abi.check(_abi.lib().fda_set_timing(self._h, 1 if on else 0))

    def phase_times(self):
        buf = (ctypes.c_double * 8)()
        _abi.check(_abi.lib().fda_phase_times(self._h, buf, 8))
        names = ("p2p", "s2m", "m2m", "m2l", "l2l", "l2t", "near_corr", "permute")
        return dict(zip(names, list(buf)))

    def stats(self) -> dict:
        buf = ctypes.create_string_buffer(1 << 20)
        _abi.check(_abi.lib().fda_stats(self._h, buf, len(buf)))
        return json.loads(buf.value.decode())


def _opts(**opts):
    o = _abi.FdaOpts()
    _abi.check(_abi.lib().fda_default_opts(ctypes.byref(o)))
    if isinstance(opts.get("precision"), str):
        opts["precision"] = _abi.PREC[opts["precision"]]
    for key, val in opts.items():
        if not hasattr(o, key):
            raise TypeError(f"unknown option {key}")
        setattr(o, key, val)
    return o


def analyze(pts, nrm, w, k, eps, **opts) -> dict:
    """Host-side plan structure without a GPU (fda_analyze): levels, reduced
    dimensions, pair and operator counts."""
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    nrm = np.ascontiguousarray(nrm, dtype=np.float64).reshape(-1, 3)
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
    g = _abi.FdaGeometry(w.shape[0], pts.ctypes.data, nrm.ctypes.data, w.ctypes.data, 0, None)
    o = _opts(**opts)
    buf = ctypes.create_string_buffer(1 << 22)
    _abi.check(_abi.lib().fda_analyze(ctypes.byref(g), float(k), float(eps), ctypes.byref(o), buf, len(buf)))
    return json.loads(buf.value.decode())


def build(pts, nrm, w, k, eps, elements=None, **opts) -> Plan:
    return Plan(pts, nrm, w, k, eps, elements=elements, **opts)


class Batch:
    """Many plans applied in one graph launch (fda_batch_*); the plans must
    stay alive while the batch exists."""

    def __init__(self, plans):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        _abi.check(_abi.lib().fda_batch_create(arr, len(self.plans), ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _abi.lib().fda_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, vecs):
        if len(vecs) != len(self.plans):
            raise ValueError("one vector per plan")
        for v, p in zip(vecs, self.plans):
            _check_vec(v, p.n)
        return (ctypes.c_void_p * len(vecs))(*[v.data_ptr() for v in vecs])

    def matvec(self, us, op: str = "BM_H", outs=None, stream=None, fp32: bool = False):
        import torch

        if outs is None:
            outs = [torch.empty_like(u) for u in us]
        _abi.check(_abi.lib().fda_batch_matvec(self._h, Plan._op(op, fp32), self._ptrs(us), self._ptrs(outs),
                                               _stream_ptr(stream)))
        return outs

    def solve(self, rhs, tol: float, maxit: int = 200, restart: int = 200, op: str = "BM_H", precond: int = 0,
              fp32: bool = False, raise_on_fail: bool = True):
        import torch

        xs = [torch.empty_like(b) for b in rhs]
        n = len(self.plans)
        it = (ctypes.c_int * n)()
        rr = (ctypes.c_double * n)()
        stt = (ctypes.c_int * n)()
        torch.cuda.synchronize()
        rc = _abi.lib().fda_batch_solve(self._h, Plan._op(op, fp32), self._ptrs(rhs), float(tol), int(maxit),
                                        int(restart), int(precond), self._ptrs(xs), it, rr, stt)
        info = {"status": rc, "iterations": list(it), "relres": list(rr), "instance_status": list(stt)}
        if rc != _abi.FDA_OK and raise_on_fail:
            _abi.check(rc)
        return xs, info


class Net:
    """The learned low-rank correction of the block-Jacobi preconditioner
    (fda_net_*): parameters live on the current GPU; training, evaluation and
    the gradient run in the library's kernels."""

    def __init__(self, seed: int = 0):
        h = ctypes.c_void_p()
        _abi.check(_abi.lib().fda_net_create(int(seed), ctypes.byref(h)))
        self._h = h
        self.n_params = int(_abi.lib().fda_net_num_params())

    def close(self):
        if getattr(self, "_h", None):
            _abi.lib().fda_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def params(self) -> np.ndarray:
        th = np.empty(self.n_params)
        _abi.check(_abi.lib().fda_net_get_params(self._h, th.ctypes.data))
        return th

    @params.setter
    def params(self, th):
        th = np.ascontiguousarray(th, dtype=np.float64).reshape(-1)
        if th.shape[0] != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        _abi.check(_abi.lib().fda_net_set_params(self._h, th.ctypes.data))

    def loss_grad(self, plan: Plan):
        loss = ctypes.c_double(0)
        g = np.empty(self.n_params)
        _abi.check(_abi.lib().fda_net_loss_grad(self._h, plan._h, ctypes.byref(loss), g.ctypes.data))
        return loss.value, g

    def train_step(self, plan: Plan, lr: float) -> float:
        loss = ctypes.c_double(0)
        _abi.check(_abi.lib().fda_net_train_step(self._h, plan._h, float(lr), ctypes.byref(loss)))
        return loss.value

    def attach(self, plan: Plan):
        _abi.check(_abi.lib().fda_net_attach(self._h, plan._h))

    @staticmethod
    def detach(plan: Plan):
        _abi.check(_abi.lib().fda_net_attach(None, plan._h))

    @staticmethod
    def weight_blocks(plan: Plan, rhs, iters: int):
        """Block weights of the plan's training loss from `iters` steps of the
        method's block-Jacobi GMRES on rhs (fda_net_weight_blocks); iters = 0
        restores uniform weights."""
        import torch

        torch.cuda.synchronize()
        ptr = None if rhs is None else ctypes.c_void_p(rhs.data_ptr())
        _abi.check(_abi.lib().fda_net_weight_blocks(plan._h, ptr, int(iters)))

    def loss_grad_raw(self, pair_off, block_n, block_ne, inv_off, target_off, features, block_inv, targets,
                      block_weight=None):
        """Loss and gradient on caller data (fda_net_loss_grad_raw): CUDA
        tensors int64 pair_off, int32 block_n and block_ne, int64 inv_off and
        target_off, float64 features (rows x 12), complex128 block_inv and
        targets (column-major blocks at their offsets)."""
        import torch

        checks = [(pair_off, torch.int64), (block_n, torch.int32), (block_ne, torch.int32),
                  (inv_off, torch.int64), (target_off, torch.int64), (features, torch.float64),
                  (block_inv, torch.complex128), (targets, torch.complex128)]
        if block_weight is not None:
            checks.append((block_weight, torch.float64))
            if block_weight.numel() != pair_off.numel():
                raise ValueError("one weight per block")
        for t, dt in checks:
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt and t.is_contiguous()):
                raise ValueError(f"expected a contiguous {dt} CUDA tensor")
        nb = pair_off.numel()
        if any(t.numel() != nb for t in (block_n, block_ne, inv_off, target_off)) or nb == 0:
            raise ValueError("inconsistent block layout")
        if features.dim() != 2 or features.shape[1] != 12:
            raise ValueError("features must be rows x 12")
        n64 = block_n.to(torch.int64)
        if int((inv_off + n64 * n64).max().item()) > block_inv.numel() or \
                int((target_off + n64 * block_ne.to(torch.int64)).max().item()) > targets.numel():
            raise ValueError("block arrays too short for the layout")
        torch.cuda.synchronize()
        loss = ctypes.c_double(0)
        g = np.empty(self.n_params)
        ptr = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
        _abi.check(_abi.lib().fda_net_loss_grad_raw(
            self._h, nb, ptr(pair_off), ptr(block_n), ptr(block_ne), ptr(inv_off), ptr(target_off),
            features.shape[0], ptr(features), ptr(block_inv), ptr(targets),
            None if block_weight is None else ptr(block_weight), ctypes.byref(loss), g.ctypes.data))
        return loss.value, g
