"""Python access to the plain CPU oracle (``oracle/fmm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg, never by the GPU library or its binding.
The oracle computes in IEEE double, see the header of ``fmm_oracle.c`` for
the conventions it follows and the paper's passages it cites.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.orc_tree_build.restype = _vp
        L.orc_tree_build.argtypes = [ctypes.c_int64, _vp, ctypes.c_int]
        L.orc_tree_free.argtypes = [_vp]
        L.orc_tree_lists.argtypes = [_vp, ctypes.c_double]
        L.orc_tree_info.argtypes = [_vp, _vp]
        L.orc_tree_export.argtypes = [_vp] + [_vp] * 14
        L.orc_fmm_eval.argtypes = [_vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int64, _vp, _vp, _vp, _vp, _vp]
        L.orc_direct_grad.argtypes = [ctypes.c_int64, _vp, ctypes.c_int, _vp, ctypes.c_int64, _vp, _vp]
        L.orc_p2p_pair_grad.argtypes = [ctypes.c_int, _vp, _vp, _vp]
        L.orc_l2p_grad.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp]
        L.orc_bh_eval.argtypes = [_vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_double, ctypes.c_int64,
                                  _vp, _vp, _vp, _vp]
        L.orc_m2p_grad.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp]
        L.orc_upward.argtypes = [_vp, ctypes.c_int, _vp, ctypes.c_int, _vp]
        L.orc_direct.argtypes = [ctypes.c_int64, _vp, ctypes.c_int, _vp, ctypes.c_int64, _vp, _vp, _vp]
        L.orc_dtensor.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _vp]
        L.orc_index.argtypes = [ctypes.c_int] * 3
        L.orc_index.restype = ctypes.c_int
        L.orc_nterms.argtypes = [ctypes.c_int]
        L.orc_nterms.restype = ctypes.c_int
        L.orc_multi_index.argtypes = [ctypes.c_int, _vp]
        L.orc_p2m.argtypes = [ctypes.c_int, ctypes.c_int, _vp, ctypes.c_int64, _vp, _vp, _vp]
        L.orc_m2m.argtypes = [ctypes.c_int, _vp, _vp, _vp, _vp]
        L.orc_m2l.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp]
        L.orc_l2l.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp]
        L.orc_l2p.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp, _vp]
        L.orc_m2p.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp, _vp]
        L.orc_p2p_pair.argtypes = [ctypes.c_int, _vp, _vp, _vp, _vp]
        L.orc_cell_center.argtypes = [_vp, ctypes.c_int64, _vp, _vp]
        L.orc_pair_derivs.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]
        L.orc_direct_derivs.argtypes = [ctypes.c_int64, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int64, _vp, _vp]
        L.orc_l2p_derivs.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, ctypes.c_int, _vp]
        L.orc_fmm_derivs.argtypes = [_vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _vp, _vp]
        L.orc_m2p_derivs.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, ctypes.c_int, _vp]
        L.orc_bh_derivs.argtypes = [_vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int64,
                                    _vp, _vp]
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------- small ops
def nterms(p: int) -> int:
    return lib().orc_nterms(p)


def index(nx: int, ny: int, nz: int) -> int:
    return lib().orc_index(nx, ny, nz)


def multi_index(i: int):
    out = np.zeros(3, dtype=np.int32)
    lib().orc_multi_index(i, out.ctypes.data)
    return tuple(int(v) for v in out)


def dtensor(q: int, r) -> np.ndarray:
    D = np.zeros(nterms(q))
    lib().orc_dtensor(q, float(r[0]), float(r[1]), float(r[2]), D.ctypes.data)
    return D


# Source order codes: 0, 1, 2 for one order, or MIXED + a bit mask of the
# orders present (bit k: order k), with the moments of the present orders
# concatenated in ascending order in each row.
MIXED = 16


def mixed(mask: int) -> int:
    return MIXED + int(mask)


def min_order(code: int) -> int:
    return int(lib().orc_min_order(int(code)))


def p2p_pair(order: int, r, mom):
    r = _c(r)
    mom = _c(mom).ravel()
    phi = np.zeros(1)
    E = np.zeros(3)
    lib().orc_p2p_pair(order, _p(r), _p(mom), _p(phi), _p(E))
    return phi[0], E


def p2p_pair_grad(order: int, r, mom) -> np.ndarray:
    """Field gradient d_i E_j (xx, xy, xz, yy, yz, zz) of one source at r."""
    G = np.zeros(6)
    lib().orc_p2p_pair_grad(order, _p(_c(r)), _p(_c(mom).ravel()), _p(G))
    return G


def p2m(p: int, order: int, z, pos, mom) -> np.ndarray:
    pos = _c(pos).reshape(-1, 3)
    mom = _c(mom)
    M = np.zeros(nterms(p))
    lib().orc_p2m(p, order, _p(_c(z)), pos.shape[0], _p(pos), _p(mom), _p(M))
    return M


def m2m(p: int, zc, Mc, zp) -> np.ndarray:
    Mp = np.zeros(nterms(p))
    lib().orc_m2m(p, _p(_c(zc)), _p(_c(Mc)), _p(_c(zp)), _p(Mp))
    return Mp


def m2l(p: int, s: int, zA, MA, zB) -> np.ndarray:
    LB = np.zeros(nterms(p - s))
    lib().orc_m2l(p, s, _p(_c(zA)), _p(_c(MA)), _p(_c(zB)), _p(LB))
    return LB


def l2l(p: int, s: int, zP, LP, zC) -> np.ndarray:
    LC = np.zeros(nterms(p - s))
    lib().orc_l2l(p, s, _p(_c(zP)), _p(_c(LP)), _p(_c(zC)), _p(LC))
    return LC


def l2p(p: int, s: int, z, L, x):
    phi = np.zeros(1)
    E = np.zeros(3)
    lib().orc_l2p(p, s, _p(_c(z)), _p(_c(L)), _p(_c(x)), _p(phi), _p(E))
    return phi[0], E


def l2p_grad(p: int, s: int, z, L, x) -> np.ndarray:
    """Field gradient (xx, xy, xz, yy, yz, zz) of the local expansion L at x."""
    G = np.zeros(6)
    lib().orc_l2p_grad(p, s, _p(_c(z)), _p(_c(L)), _p(_c(x)), _p(G))
    return G


def m2p(p: int, s: int, zA, M, x):
    phi = np.zeros(1)
    E = np.zeros(3)
    lib().orc_m2p(p, s, _p(_c(zA)), _p(_c(M)), _p(_c(x)), _p(phi), _p(E))
    return phi[0], E


def m2p_grad(p: int, s: int, zA, M, x) -> np.ndarray:
    """Field gradient (xx, xy, xz, yy, yz, zz) of the multipole M about zA at x."""
    G = np.zeros(6)
    lib().orc_m2p_grad(p, s, _p(_c(zA)), _p(_c(M)), _p(_c(x)), _p(G))
    return G


def direct_grad(pos, order: int, mom, targets: Optional[np.ndarray] = None) -> np.ndarray:
    """O(N^2) field gradient (k x 6: xx, xy, xz, yy, yz, zz) at all (or the
    listed) targets."""
    pos = _c(pos).reshape(-1, 3)
    mom = _c(mom)
    n = pos.shape[0]
    tg = None if targets is None else _c(targets, np.int64)
    k = n if tg is None else tg.shape[0]
    G = np.zeros((k, 6))
    lib().orc_direct_grad(n, _p(pos), order, _p(mom), k, _p(tg), _p(G))
    return G


def nderivs(K: int) -> int:
    """number of derivatives of order K: the multi-indices k with |k| = K"""
    return (K + 1) * (K + 2) // 2


def pair_derivs(order: int, K: int, r, mom) -> np.ndarray:
    """d^k phi for every |k| = K of one source at displacement r"""
    out = np.zeros(nderivs(K))
    lib().orc_pair_derivs(order, K, _p(_c(r)), _p(_c(mom).ravel()), _p(out))
    return out


def direct_derivs(pos, order: int, mom, K: int, targets: Optional[np.ndarray] = None) -> np.ndarray:
    """O(N^2) derivatives of order K of the potential (k x nderivs(K)), in
    the index order within that order"""
    pos = _c(pos).reshape(-1, 3)
    mom = _c(mom)
    n = pos.shape[0]
    tg = None if targets is None else _c(targets, np.int64)
    k = n if tg is None else tg.shape[0]
    out = np.zeros((k, nderivs(K)))
    lib().orc_direct_derivs(n, _p(pos), order, _p(mom), K, k, _p(tg), _p(out))
    return out


def l2p_derivs(p: int, s: int, z, L, x, K: int) -> np.ndarray:
    """Eq. 10: derivatives of order K of the local expansion L about z at x"""
    out = np.zeros(nderivs(K))
    lib().orc_l2p_derivs(p, s, _p(_c(z)), _p(_c(L)), _p(_c(x)), K, _p(out))
    return out


def m2p_derivs(p: int, s: int, zA, M, x, K: int) -> np.ndarray:
    """Eq. 6 differentiated K times: derivatives of order K at x of the
    multipole M (physical units, nterms(p)) about zA"""
    out = np.zeros(nderivs(K))
    lib().orc_m2p_derivs(p, s, _p(_c(zA)), _p(_c(M)), _p(_c(x)), K, _p(out))
    return out


def direct(pos, order: int, mom, targets: Optional[np.ndarray] = None):
    """O(N^2) potential and field at all (or the listed) targets."""
    pos = _c(pos).reshape(-1, 3)
    mom = _c(mom)
    n = pos.shape[0]
    tg = None if targets is None else _c(targets, np.int64)
    k = n if tg is None else tg.shape[0]
    phi = np.zeros(k)
    E = np.zeros((k, 3))
    lib().orc_direct(n, _p(pos), order, _p(mom), k, _p(tg), _p(phi), _p(E))
    return phi, E


# ---------------------------------------------------------------- tree
@dataclass
class TreeDump:
    lo: np.ndarray
    W: float
    key: np.ndarray
    perm: np.ndarray
    level: np.ndarray
    ix: np.ndarray
    first: np.ndarray
    count: np.ndarray
    parent: np.ndarray
    child0: np.ndarray
    nchild: np.ndarray
    m2l_ptr: np.ndarray
    m2l_src: np.ndarray
    p2p_ptr: np.ndarray
    p2p_src: np.ndarray


class Tree:
    """Octree + dual-tree interaction lists built by the oracle."""

    def __init__(self, pos, ncrit: int, theta: Optional[float] = None):
        self.pos = _c(pos).reshape(-1, 3)
        self.n = self.pos.shape[0]
        h = lib().orc_tree_build(self.n, _p(self.pos), int(ncrit))
        if not h:
            raise ValueError("oracle tree build rejected its arguments")
        self._h = h
        self.ncrit = ncrit
        if theta is not None:
            self.lists(theta)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                lib().orc_tree_free(h)
            except TypeError:       # interpreter shutdown: module globals already cleared
                pass
            self._h = None

    def lists(self, theta: float):
        if lib().orc_tree_lists(self._h, float(theta)) != 0:
            raise ValueError("bad theta")
        self.theta = theta

    def info(self):
        out = np.zeros(6, dtype=np.int64)
        lib().orc_tree_info(self._h, _p(out))
        return dict(n=int(out[0]), ncells=int(out[1]), nlevels=int(out[2]), n_m2l=int(out[3]),
                    n_p2p=int(out[4]), nleaves=int(out[5]))

    def dump(self) -> TreeDump:
        inf = self.info()
        n, nc = inf["n"], inf["ncells"]
        geom = np.zeros(4)
        d = TreeDump(lo=None, W=0.0,
                     key=np.zeros(n, np.uint64), perm=np.zeros(n, np.int64),
                     level=np.zeros(nc, np.int32), ix=np.zeros((nc, 3), np.int32),
                     first=np.zeros(nc, np.int64), count=np.zeros(nc, np.int64),
                     parent=np.zeros(nc, np.int64), child0=np.zeros(nc, np.int64),
                     nchild=np.zeros(nc, np.int32),
                     m2l_ptr=np.zeros(nc + 1, np.int64), m2l_src=np.zeros(max(inf["n_m2l"], 1), np.int64),
                     p2p_ptr=np.zeros(nc + 1, np.int64), p2p_src=np.zeros(max(inf["n_p2p"], 1), np.int64))
        lib().orc_tree_export(self._h, _p(geom), _p(d.key), _p(d.perm), _p(d.level), _p(d.ix), _p(d.first),
                              _p(d.count), _p(d.parent), _p(d.child0), _p(d.nchild), _p(d.m2l_ptr),
                              _p(d.m2l_src), _p(d.p2p_ptr), _p(d.p2p_src))
        d.lo = geom[:3].copy()
        d.W = float(geom[3])
        d.m2l_src = d.m2l_src[: inf["n_m2l"]]
        d.p2p_src = d.p2p_src[: inf["n_p2p"]]
        return d

    def cell_center(self, c: int):
        z = np.zeros(3)
        r = np.zeros(1)
        lib().orc_cell_center(self._h, int(c), _p(z), _p(r))
        return z, float(r[0])

    def upward(self, order: int, mom, p: int) -> np.ndarray:
        mom = _c(mom)
        M = np.zeros((self.info()["ncells"], nterms(p)))
        lib().orc_upward(self._h, order, _p(mom), p, _p(M))
        return M

    def fmm(self, order: int, mom, p: int, targets: Optional[np.ndarray] = None, want_L: bool = False,
            want_grad: bool = False):
        """phi, E (and the local expansions L, the field gradient G (k x 6)
        when asked for, in that order)."""
        mom = _c(mom)
        tg = None if targets is None else _c(targets, np.int64)
        k = self.n if tg is None else tg.shape[0]
        phi = np.zeros(k)
        E = np.zeros((k, 3))
        L = np.zeros((self.info()["ncells"], nterms(p - min_order(order)))) if want_L else None
        G = np.zeros((k, 6)) if want_grad else None
        rc = lib().orc_fmm_eval(self._h, order, _p(mom), p, k, _p(tg), _p(phi), _p(E), _p(L), _p(G))
        if rc != 0:
            raise ValueError("oracle FMM rejected its arguments (lists missing or p < order+1)")
        out = (phi, E) + ((L,) if want_L else ()) + ((G,) if want_grad else ())
        return out

    def fmm_derivs(self, order: int, mom, p: int, K: int, targets: Optional[np.ndarray] = None) -> np.ndarray:
        """FMM derivatives of order K of the potential (k x nderivs(K))"""
        mom = _c(mom)
        tg = None if targets is None else _c(targets, np.int64)
        k = self.n if tg is None else tg.shape[0]
        out = np.zeros((k, nderivs(K)))
        if lib().orc_fmm_derivs(self._h, order, _p(mom), p, K, k, _p(tg), _p(out)) != 0:
            raise ValueError("oracle FMM derivatives rejected their arguments")
        return out

    def bh_derivs(self, order: int, mom, p: int, theta_bh: float, K: int,
                  targets: Optional[np.ndarray] = None) -> np.ndarray:
        """Barnes-Hut derivatives of order K of the potential (k x nderivs(K))"""
        mom = _c(mom)
        tg = None if targets is None else _c(targets, np.int64)
        k = self.n if tg is None else tg.shape[0]
        out = np.zeros((k, nderivs(K)))
        if lib().orc_bh_derivs(self._h, order, _p(mom), p, float(theta_bh), K, k, _p(tg), _p(out)) != 0:
            raise ValueError("oracle BH derivatives rejected their arguments")
        return out

    def bh(self, order: int, mom, p: int, theta_bh: float, targets: Optional[np.ndarray] = None,
           want_grad: bool = False):
        """phi, E (and the field gradient G, k x 6, when asked for)."""
        mom = _c(mom)
        tg = None if targets is None else _c(targets, np.int64)
        k = self.n if tg is None else tg.shape[0]
        phi = np.zeros(k)
        E = np.zeros((k, 3))
        G = np.zeros((k, 6)) if want_grad else None
        rc = lib().orc_bh_eval(self._h, order, _p(mom), p, float(theta_bh), k, _p(tg), _p(phi), _p(E), _p(G))
        if rc != 0:
            raise ValueError("oracle BH rejected its arguments")
        return (phi, E, G) if want_grad else (phi, E)


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """Relative L2 error of a against reference b (all components pooled)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt((b * b).sum())
    return float(np.sqrt(((a - b) ** 2).sum()) / (den if den > 0 else 1.0))
