"""Thin Python binding of libfmm.so (see include/fmm.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory (contiguous float64 tensors on
the context's device) and streams.  Importing this module loads the library
and fails loudly if it has not been built.

Stream ordering: the library queues its work on the context's stream (a
PyTorch stream, created by the context unless one is given).  Unless that
stream is PyTorch's current stream, every call here first makes it wait for
PyTorch's current stream, so inputs made by
earlier device work are complete before the library reads them, and
afterwards makes the current stream wait for the context's stream, so the
outputs are complete before later work on the current stream uses them and
before the caching allocator hands their memory (or the inputs') to anything
else.  The serving calls run on the library's own worker streams: submit()
synchronises the current stream before it queues a request, and a request's
outputs are complete once wait() returns.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# FMM_LIBRARY may point at another build of the same library (e.g. a variant
# with different code-shape options); the default is the in-tree build.
LIB_PATH = os.environ.get("FMM_LIBRARY") or os.path.join(_HERE, "libfmm.so")

FMM_OK, FMM_EINVAL, FMM_ENOMEM, FMM_EDEVICE, FMM_ESTATE, FMM_EBUSY, FMM_ETIMEOUT = range(7)
FMM_POT, FMM_FIELD, FMM_GRAD = 1, 2, 4   # output mask bits (FMM_GRAD: evaluate_grad only)
FMM_OVERLAP_OFF, FMM_OVERLAP_WHOLE, FMM_OVERLAP_SPLIT, FMM_OVERLAP_TAIL = 0, 1, 2, 3
FMM_METHOD_FMM, FMM_METHOD_BH = 0, 1
FMM_M2L_FULL, FMM_M2L_HARMONIC = 0, 1   # M2L contraction basis (fmm_ctx_set_m2l_basis)
FMM_M2L_ENGINE_VALU, FMM_M2L_ENGINE_MFMA, FMM_M2L_ENGINE_AUTO = 0, 1, 2   # units of the FP32 harmonic M2L
FMM_PREC_FP64, FMM_PREC_MIXED = 0, 1
FMM_SCHEDULE_HOST, FMM_SCHEDULE_DEVICE, FMM_SCHEDULE_AUTO = 0, 1, 2   # builder of the M2L schedule
FMM_P_MAX = 10
FMM_MIXED = 16          # order code FMM_MIXED | mask: several source orders (bit k: order k)
FMM_REQ_QUEUED, FMM_REQ_RUNNING, FMM_REQ_DONE, FMM_REQ_FAILED = range(4)

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                      "(there is no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64


class fmm_request(ctypes.Structure):
    _fields_ = [("pos", _vp), ("moments", _vp), ("phi", _vp), ("field", _vp), ("n", _i64),
                ("order", ctypes.c_int), ("p", ctypes.c_int), ("ncrit", ctypes.c_int), ("method", ctypes.c_int),
                ("precision", ctypes.c_int), ("outputs", ctypes.c_int), ("theta", ctypes.c_double)]


def _sig(name, args, res=ctypes.c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


fmm_ctx_create = _sig("fmm_ctx_create", [ctypes.c_int, _vp, ctypes.c_size_t, ctypes.POINTER(_vp)])
fmm_ctx_destroy = _sig("fmm_ctx_destroy", [_vp])
fmm_build_tree = _sig("fmm_build_tree", [_vp, _vp, _i64, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                         ctypes.POINTER(_vp)])
fmm_upward = _sig("fmm_upward", [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int])
fmm_evaluate = _sig("fmm_evaluate", [_vp, _vp, ctypes.c_int, _vp, _vp])
fmm_evaluate_grad = _sig("fmm_evaluate_grad", [_vp, _vp, ctypes.c_int, _vp, _vp, _vp])
fmm_evaluate_derivs = _sig("fmm_evaluate_derivs", [_vp, _vp, ctypes.c_int, _vp])
fmm_evaluate_grad_noalloc = _sig("fmm_evaluate_grad_noalloc", [_vp, _vp, ctypes.c_int, _vp, _vp, _vp])
fmm_run = _sig("fmm_run", [_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp])
fmm_tree_info = _sig("fmm_tree_info", [_vp, _vp])
fmm_tree_export = _sig("fmm_tree_export", [_vp] + [_vp] * 14)
fmm_tree_destroy = _sig("fmm_tree_destroy", [_vp])
fmm_last_error = _sig("fmm_last_error", [], ctypes.c_char_p)
fmm_ctx_set_overlap = _sig("fmm_ctx_set_overlap", [_vp, ctypes.c_int])
fmm_ctx_set_m2l_basis = _sig("fmm_ctx_set_m2l_basis", [_vp, ctypes.c_int])
fmm_ctx_set_graphs = _sig("fmm_ctx_set_graphs", [_vp, ctypes.c_int])
fmm_ctx_set_m2l_engine = _sig("fmm_ctx_set_m2l_engine", [_vp, ctypes.c_int])
fmm_ctx_set_tree_limit = _sig("fmm_ctx_set_tree_limit", [_vp, ctypes.c_size_t])
fmm_ctx_set_m2l_schedule = _sig("fmm_ctx_set_m2l_schedule", [_vp, ctypes.c_int])
fmm_tree_m2l_schedule = _sig("fmm_tree_m2l_schedule", [_vp] * 7)
fmm_profile_enable = _sig("fmm_profile_enable", [_vp, ctypes.c_int])
fmm_profile_reset = _sig("fmm_profile_reset", [_vp])
fmm_profile_read = _sig("fmm_profile_read", [_vp, _vp, _vp, _vp, ctypes.c_int])
fmm_work_counts = _sig("fmm_work_counts", [_vp, _vp])
fmm_serve_start = _sig("fmm_serve_start", [_vp, ctypes.c_int])
fmm_submit = _sig("fmm_submit", [_vp, ctypes.POINTER(fmm_request), ctypes.POINTER(ctypes.c_uint64)])
fmm_poll = _sig("fmm_poll", [_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)])
fmm_wait = _sig("fmm_wait", [_vp, ctypes.c_uint64, ctypes.c_double])
fmm_request_times = _sig("fmm_request_times", [_vp, ctypes.c_uint64, _vp, _vp])
fmm_request_phases = _sig("fmm_request_phases", [_vp, ctypes.c_uint64, _vp])
fmm_serve_stop = _sig("fmm_serve_stop", [_vp])
fmm_serve_stats = _sig("fmm_serve_stats", [_vp, _vp])
fmm_ctx_create_fake = _sig("fmm_ctx_create_fake", [ctypes.c_size_t, ctypes.c_double, ctypes.POINTER(_vp)])

EXPORTED = ["fmm_ctx_create", "fmm_ctx_destroy", "fmm_build_tree", "fmm_upward", "fmm_evaluate", "fmm_evaluate_grad", "fmm_evaluate_grad_noalloc", "fmm_evaluate_derivs", "fmm_run", "fmm_tree_info",
            "fmm_tree_export", "fmm_tree_destroy", "fmm_last_error", "fmm_ctx_set_overlap", "fmm_ctx_set_m2l_basis", "fmm_ctx_set_graphs", "fmm_ctx_set_m2l_engine", "fmm_ctx_set_tree_limit",
            "fmm_ctx_set_m2l_schedule", "fmm_tree_m2l_schedule", "fmm_profile_enable", "fmm_profile_reset",
            "fmm_profile_read", "fmm_work_counts", "fmm_serve_start", "fmm_submit", "fmm_poll", "fmm_wait",
            "fmm_request_times", "fmm_request_phases", "fmm_serve_stop", "fmm_serve_stats", "fmm_ctx_create_fake"]


class FMMError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what} failed with code {code}: {fmm_last_error().decode(errors='replace')}")
        self.code = code


def _check(rc, what):
    if rc != FMM_OK:
        raise FMMError(rc, what)


def _dev_f64(t: torch.Tensor, cols: Optional[int], name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous float64")
    if cols is not None and (t.dim() != 2 or t.shape[1] != cols) and not (cols == 1 and t.dim() == 1):
        raise ValueError(f"{name} must have shape (n, {cols})")
    return t


class Context:
    """A libfmm context bound to one device and one stream (a PyTorch stream of
    default priority; a new one unless `stream` is given)."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None, budget_bytes: int = 0,
                 _handle=None):
        self.device = device
        self.stream = stream
        if _handle is not None:
            self.h = _handle
            return
        if self.stream is None:
            self.stream = torch.cuda.Stream(device=device)
        elif self.stream.cuda_stream == 0:
            raise ValueError("the legacy default stream cannot be a context stream (its work cannot be captured "
                             "into graphs); pass a created stream or None")
        h = _vp()
        _check(fmm_ctx_create(device, self.stream.cuda_stream, budget_bytes, ctypes.byref(h)), "fmm_ctx_create")
        self.h = h

    def _enter(self):
        """the context's stream waits for the caller's current stream (nothing
        to do when the caller works on the context's stream itself)"""
        if self.stream is not None:
            cur = torch.cuda.current_stream(self.device)
            if cur != self.stream:
                self.stream.wait_stream(cur)

    def _leave(self):
        """the caller's current stream waits for the work just queued"""
        if self.stream is not None:
            cur = torch.cuda.current_stream(self.device)
            if cur != self.stream:
                cur.wait_stream(self.stream)

    def set_tree_limit(self, nbytes: int):
        """device bytes one tree may hold (0: no limit); beyond it calls fail with FMM_ENOMEM"""
        _check(fmm_ctx_set_tree_limit(self.h, int(nbytes)), "fmm_ctx_set_tree_limit")

    @classmethod
    def fake(cls, budget_bytes: int, ns_per_particle: float = 0.0):
        """device-less context whose server simulates execution (scheduler tests)"""
        h = _vp()
        _check(fmm_ctx_create_fake(int(budget_bytes), float(ns_per_particle), ctypes.byref(h)), "fmm_ctx_create_fake")
        return cls(-1, None, 0, _handle=h)

    # serving ---------------------------------------------------------
    def serve_start(self, max_concurrent: int):
        _check(fmm_serve_start(self.h, int(max_concurrent)), "fmm_serve_start")

    def serve_stop(self):
        _check(fmm_serve_stop(self.h), "fmm_serve_stop")

    def submit(self, n: int, order: int, p: int, theta: float, ncrit: int, pos=None, moments=None, phi=None,
               field=None, method: int = FMM_METHOD_FMM, precision: int = FMM_PREC_MIXED,
               outputs: int = FMM_POT | FMM_FIELD) -> int:
        def ptr(t):
            return None if t is None else t.data_ptr()
        if self.device >= 0:
            # the server's worker streams are not ordered after the caller's
            torch.cuda.current_stream(self.device).synchronize()
        r = fmm_request(ptr(pos), ptr(moments), ptr(phi), ptr(field), int(n), int(order), int(p), int(ncrit),
                        int(method), int(precision), int(outputs), float(theta))
        tk = ctypes.c_uint64()
        _check(fmm_submit(self.h, ctypes.byref(r), ctypes.byref(tk)), "fmm_submit")
        return tk.value

    def poll(self, ticket: int) -> int:
        st = ctypes.c_int()
        _check(fmm_poll(self.h, ticket, ctypes.byref(st)), "fmm_poll")
        return st.value

    def wait(self, ticket: int, timeout_s: float = -1.0):
        _check(fmm_wait(self.h, ticket, float(timeout_s)), "fmm_wait")

    def request_times(self, ticket: int):
        t = (ctypes.c_double * 3)()
        b = (ctypes.c_int64 * 2)()
        _check(fmm_request_times(self.h, ticket, ctypes.cast(t, _vp), ctypes.cast(b, _vp)), "fmm_request_times")
        return dict(submit=t[0], admit=t[1], done=t[2], footprint=int(b[0]), bytes_used=int(b[1]))

    def request_phases(self, ticket: int):
        t = (ctypes.c_double * 2)()
        _check(fmm_request_phases(self.h, ticket, ctypes.cast(t, _vp)), "fmm_request_phases")
        return dict(built=t[0], computed=t[1])

    def serve_stats(self) -> dict:
        a = (ctypes.c_int64 * 7)()
        _check(fmm_serve_stats(self.h, ctypes.cast(a, _vp)), "fmm_serve_stats")
        return dict(zip(["budget", "in_use", "peak_in_use", "running", "peak_running", "queued", "slots"],
                        [int(v) for v in a]))

    def close(self):
        if self.h:
            fmm_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_m2l_basis(self, basis: int):
        """FMM_M2L_FULL or FMM_M2L_HARMONIC (default); used from the next upward pass."""
        _check(fmm_ctx_set_m2l_basis(self.h, int(basis)), "fmm_ctx_set_m2l_basis")

    def set_m2l_engine(self, engine: int):
        """FMM_M2L_ENGINE_AUTO (default), _MFMA or _VALU; used from the next upward pass"""
        _check(fmm_ctx_set_m2l_engine(self.h, int(engine)), "fmm_ctx_set_m2l_engine")

    def set_m2l_schedule(self, where: int):
        """FMM_SCHEDULE_AUTO (default), _DEVICE or _HOST; used by trees built afterwards"""
        _check(fmm_ctx_set_m2l_schedule(self.h, int(where)), "fmm_ctx_set_m2l_schedule")

    def set_overlap(self, on=True):
        """False/0 off, True/1 the whole near field beside the far field, 2
        (FMM_OVERLAP_SPLIT) half beside M2M and half after the M2L, 3
        (FMM_OVERLAP_TAIL) the whole near field after the M2L"""
        _check(fmm_ctx_set_overlap(self.h, int(on)), "fmm_ctx_set_overlap")

    def set_graphs(self, on: bool = True):
        _check(fmm_ctx_set_graphs(self.h, int(on)), "fmm_ctx_set_graphs")

    # profiling -------------------------------------------------------
    def profile(self, on: bool = True):
        _check(fmm_profile_enable(self.h, int(on)), "fmm_profile_enable")

    def profile_reset(self):
        _check(fmm_profile_reset(self.h), "fmm_profile_reset")

    def profile_read(self) -> dict:
        cap = 64
        names = (ctypes.c_char_p * cap)()
        ms = (ctypes.c_double * cap)()
        cnt = (ctypes.c_int64 * cap)()
        k = fmm_profile_read(self.h, ctypes.cast(names, _vp), ctypes.cast(ms, _vp), ctypes.cast(cnt, _vp), cap)
        if k < 0:
            raise FMMError(k, "fmm_profile_read")
        return {names[i].decode(): (ms[i], int(cnt[i])) for i in range(min(k, cap))}


class Tree:
    """Octree + interaction lists resident on the device (fmm_build_tree)."""

    def __init__(self, ctx: Context, pos: torch.Tensor, ncrit: int, theta: float, method: int = FMM_METHOD_FMM):
        _dev_f64(pos, 3, "pos")
        self.ctx = ctx
        self.n = int(pos.shape[0])
        self.method = method
        h = _vp()
        ctx._enter()
        rc = fmm_build_tree(ctx.h, pos.data_ptr(), self.n, int(ncrit), float(theta), int(method), ctypes.byref(h))
        ctx._leave()
        _check(rc, "fmm_build_tree")
        self.h = h
        self._moments = None

    def close(self):
        if self.h:
            fmm_tree_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        a = (ctypes.c_int64 * 10)()
        _check(fmm_tree_info(self.h, ctypes.cast(a, _vp)), "fmm_tree_info")
        keys = ["n", "ncells", "nlevels", "nleaves", "n_m2l", "n_p2p", "n_classes", "n_tiles", "m2l_slots", "bytes"]
        return dict(zip(keys, [int(v) for v in a]))

    def upward(self, order: int, moments: torch.Tensor, p: int, precision: int = FMM_PREC_MIXED):
        _dev_f64(moments, None, "moments")
        self._moments = moments       # read by the queued upward work (and baked into its graph)
        self.ctx._enter()
        rc = fmm_upward(self.ctx.h, self.h, int(order), moments.data_ptr(), int(p), int(precision))
        self.ctx._leave()
        _check(rc, "fmm_upward")

    def evaluate(self, outputs: int = FMM_POT | FMM_FIELD, phi: Optional[torch.Tensor] = None,
                 field: Optional[torch.Tensor] = None):
        dev = torch.device("cuda", self.ctx.device)
        if (outputs & FMM_POT) and phi is None:
            phi = torch.empty(self.n, dtype=torch.float64, device=dev)
        if (outputs & FMM_FIELD) and field is None:
            field = torch.empty((self.n, 3), dtype=torch.float64, device=dev)
        self.ctx._enter()
        rc = fmm_evaluate(self.ctx.h, self.h, int(outputs), phi.data_ptr() if phi is not None else None,
                          field.data_ptr() if field is not None else None)
        self.ctx._leave()
        _check(rc, "fmm_evaluate")
        return phi, field

    def evaluate_grad(self, outputs: int = FMM_POT | FMM_FIELD | FMM_GRAD, phi: Optional[torch.Tensor] = None,
                      field: Optional[torch.Tensor] = None, grad: Optional[torch.Tensor] = None):
        """phi, field and the field gradient (n x 6: xx, xy, xz, yy, yz, zz)"""
        dev = torch.device("cuda", self.ctx.device)
        if (outputs & FMM_POT) and phi is None:
            phi = torch.empty(self.n, dtype=torch.float64, device=dev)
        if (outputs & FMM_FIELD) and field is None:
            field = torch.empty((self.n, 3), dtype=torch.float64, device=dev)
        if (outputs & FMM_GRAD) and grad is None:
            grad = torch.empty((self.n, 6), dtype=torch.float64, device=dev)
        ptr = lambda x: x.data_ptr() if x is not None else None  # noqa: E731
        self.ctx._enter()
        rc = fmm_evaluate_grad(self.ctx.h, self.h, int(outputs), ptr(phi), ptr(field), ptr(grad))
        self.ctx._leave()
        _check(rc, "fmm_evaluate_grad")
        return phi, field, grad

    def evaluate_derivs(self, K: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """derivatives of order K (1..3) of the potential, n x (K+1)(K+2)/2,
        multi-indices of order K in the index order"""
        if out is None:
            out = torch.empty((self.n, (K + 1) * (K + 2) // 2), dtype=torch.float64,
                              device=torch.device("cuda", self.ctx.device))
        self.ctx._enter()
        rc = fmm_evaluate_derivs(self.ctx.h, self.h, int(K), out.data_ptr())
        self.ctx._leave()
        _check(rc, "fmm_evaluate_derivs")
        return out

    def evaluate_grad_noalloc(self, outputs: int, phi: Optional[torch.Tensor], field: Optional[torch.Tensor],
                              grad: Optional[torch.Tensor]):
        """fmm_evaluate_grad_noalloc: caller-provided outputs, no device
        allocation inside the library"""
        ptr = lambda x: x.data_ptr() if x is not None else None  # noqa: E731
        self.ctx._enter()
        rc = fmm_evaluate_grad_noalloc(self.ctx.h, self.h, int(outputs), ptr(phi), ptr(field), ptr(grad))
        self.ctx._leave()
        _check(rc, "fmm_evaluate_grad_noalloc")
        return phi, field, grad

    def run(self, order: int, moments: torch.Tensor, p: int, precision: int = FMM_PREC_MIXED,
            outputs: int = FMM_POT | FMM_FIELD, phi: Optional[torch.Tensor] = None,
            field: Optional[torch.Tensor] = None):
        """upward + evaluate as one launch sequence (fmm_run)"""
        _dev_f64(moments, None, "moments")
        self._moments = moments
        dev = torch.device("cuda", self.ctx.device)
        if (outputs & FMM_POT) and phi is None:
            phi = torch.empty(self.n, dtype=torch.float64, device=dev)
        if (outputs & FMM_FIELD) and field is None:
            field = torch.empty((self.n, 3), dtype=torch.float64, device=dev)
        self.ctx._enter()
        rc = fmm_run(self.ctx.h, self.h, int(order), moments.data_ptr(), int(p), int(precision), int(outputs),
                     phi.data_ptr() if phi is not None else None, field.data_ptr() if field is not None else None)
        self.ctx._leave()
        _check(rc, "fmm_run")
        return phi, field

    def work_counts(self):
        a = (ctypes.c_double * 8)()
        _check(fmm_work_counts(self.h, ctypes.cast(a, _vp)), "fmm_work_counts")
        keys = ["m2l_pairs", "m2l_flops", "p2p_pairs", "p2p_flops", "m2p_pairs", "m2p_flops", "m2l_bytes",
                "p2p_bytes"]
        return dict(zip(keys, list(a)))

    def export(self):
        import numpy as np
        inf = self.info()
        n, nc = inf["n"], inf["ncells"]
        d = dict(geom=np.zeros(4), key=np.zeros(n, np.uint64), perm=np.zeros(n, np.int64),
                 level=np.zeros(nc, np.int32), ix=np.zeros((nc, 3), np.int32), first=np.zeros(nc, np.int64),
                 count=np.zeros(nc, np.int64), parent=np.zeros(nc, np.int64), child0=np.zeros(nc, np.int64),
                 nchild=np.zeros(nc, np.int32), m2l_ptr=np.zeros(nc + 1, np.int64),
                 m2l_src=np.zeros(max(1, inf["n_m2l"]), np.int64), p2p_ptr=np.zeros(nc + 1, np.int64),
                 p2p_src=np.zeros(max(1, inf["n_p2p"]), np.int64))
        order = ["geom", "key", "perm", "level", "ix", "first", "count", "parent", "child0", "nchild", "m2l_ptr",
                 "m2l_src", "p2p_ptr", "p2p_src"]
        _check(fmm_tree_export(self.h, *[d[k].ctypes.data for k in order]), "fmm_tree_export")
        d["m2l_src"] = d["m2l_src"][: inf["n_m2l"]]
        d["p2p_src"] = d["p2p_src"][: inf["n_p2p"]]
        return d


    def m2l_schedule(self):
        """the M2L schedule (fmm_tree_m2l_schedule) as numpy arrays, plus its builder"""
        import numpy as np
        inf = self.info()
        ncls, nt, slots = inf["n_classes"], inf["n_tiles"], inf["m2l_slots"]
        d = dict(tile_cell=np.zeros(max(1, 64 * nt), np.int32), tile_uoff=np.zeros(nt + 1, np.int32),
                 ucls=np.zeros(max(1, slots // 64), np.int32), usrc=np.zeros(max(1, slots), np.int32),
                 cls_geom=np.zeros(max(1, 4 * ncls), np.float64))
        where = ctypes.c_int(-1)
        _check(fmm_tree_m2l_schedule(self.h, *[d[k].ctypes.data for k in ("tile_cell", "tile_uoff", "ucls", "usrc",
                                                                          "cls_geom")], ctypes.byref(where)),
               "fmm_tree_m2l_schedule")
        d["tile_cell"] = d["tile_cell"][: 64 * nt]
        d["ucls"] = d["ucls"][: slots // 64]
        d["usrc"] = d["usrc"][:slots]
        d["cls_geom"] = d["cls_geom"][: 4 * ncls].reshape(-1, 4)
        d["where"] = where.value
        return d


def evaluate(pos: torch.Tensor, order: int, moments: torch.Tensor, p: int, theta: float, ncrit: int,
             outputs: int = FMM_POT | FMM_FIELD, precision: int = FMM_PREC_MIXED, method: int = FMM_METHOD_FMM,
             ctx: Optional[Context] = None):
    """One-shot convenience: build, upward, evaluate; returns (phi, field)."""
    own = ctx is None
    ctx = ctx or Context(pos.device.index or 0)
    try:
        t = Tree(ctx, pos, ncrit, theta, method)
        t.upward(order, moments, p, precision)
        out = t.evaluate(outputs)
        t.close()          # its memory is released in stream order after the evaluation
        return out
    finally:
        if own:
            ctx.close()
