"""ctypes binding of the plain C oracle (oracle/nfq_oracle.c).

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
baseline of the benchmark.  Builds the shared library on first use with gcc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

__all__ = ["build", "lib", "koornwinder", "gauss_jacobi", "conical_rule", "reference",
           "OracleRun", "METHOD", "TRUTH", "apply", "near_lists"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nfq_oracle.c")
_LIB = os.path.join(_HERE, "libnfq_oracle.so")
METHOD, TRUTH = 0, 1
MAXD = 12


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = C.CDLL(_LIB)
        _bind(_lib)
    return _lib


class _Problem(C.Structure):
    _fields_ = [
        ("P", C.c_int64), ("degree", C.c_void_p), ("node_ptr", C.c_void_p), ("xyz", C.c_void_p),
        ("NT", C.c_int64), ("txyz", C.c_void_p), ("node_of_target", C.c_void_p),
        ("near_row_ptr", C.c_void_p), ("near_patch", C.c_void_p),
        ("ref_uv", C.c_void_p * (MAXD + 1)),
        ("alpha_re", C.c_double), ("alpha_im", C.c_double), ("beta_re", C.c_double),
        ("beta_im", C.c_double), ("k_re", C.c_double), ("k_im", C.c_double),
        ("tol", C.c_double), ("loosen", C.c_double),
        ("max_depth", C.c_int), ("ng", C.c_int), ("mode", C.c_int), ("pad", C.c_int),
    ]


class Stats(C.Structure):
    _fields_ = [("visits", C.c_int64), ("checks", C.c_int64), ("nonconverged", C.c_int64),
                ("max_level", C.c_int64), ("near_pairs", C.c_int64),
                ("self_targets", C.c_int64), ("self_evals", C.c_int64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


def _bind(L):
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int, C.c_double
    L.orc_koornwinder.argtypes = [i32, dbl, dbl, vp, vp, vp]
    L.orc_koornwinder.restype = None
    L.orc_gauss_jacobi.argtypes = [i32, i32, i32, vp, vp]
    L.orc_conical_rule.argtypes = [i32, vp]
    L.orc_reference.argtypes = [i32, vp, vp, vp, vp]
    L.orc_pair_weights.argtypes = [vp, i64, i64, vp, vp]
    L.orc_row_ptr.argtypes = [vp, vp]
    L.orc_generate_rows.argtypes = [vp, i64, i64, vp, vp, vp, vp]
    L.orc_apply.argtypes = [i64, vp, vp, vp, vp, vp]
    L.orc_patch_info.argtypes = [vp, i64, vp, vp]
    L.orc_chart.argtypes = [vp, i64, dbl, dbl, vp]
    L.orc_patch_ball.argtypes = [vp, i64, i32, vp, vp]
    L.orc_set_trace.argtypes = [vp, i64]
    L.orc_set_trace.restype = None
    L.orc_trace_count.argtypes = []
    L.orc_trace_count.restype = i64


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def nd_of(d):
    return (d + 1) * (d + 2) // 2


def koornwinder(d, u, v):
    n = nd_of(d)
    K, Ku, Kv = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().orc_koornwinder(d, float(u), float(v), _p(K), _p(Ku), _p(Kv))
    return K, Ku, Kv


def gauss_jacobi(n, a=0, b=0):
    """Gauss rule on [0,1] for weight (1-y)^a y^b."""
    y, w = np.zeros(n), np.zeros(n)
    rc = lib().orc_gauss_jacobi(n, a, b, _p(y), _p(w))
    if rc:
        raise RuntimeError("gauss_jacobi failed %d" % rc)
    return y, w


def conical_rule(ng):
    r = np.zeros((ng * ng, 3))
    if lib().orc_conical_rule(ng, _p(r)):
        raise RuntimeError("rule failed")
    return r


def reference(d, uv):
    n = nd_of(d)
    uv = np.ascontiguousarray(uv, dtype=np.float64)
    V = np.zeros((n, n))
    nv = np.zeros(1)
    w = np.zeros(n)
    if lib().orc_reference(d, _p(uv), _p(V), _p(nv), _p(w)):
        raise RuntimeError("singular Vandermonde")
    return V, float(nv[0]), w


class OracleRun:
    """Oracle bound to one Problem (from paper_2006_02545_amd.surfaces)."""

    def __init__(self, prob, mode=METHOD, tol=None, loosen=1.0, max_depth=None, ng=0,
                 alpha=None, beta=None, k=None, target_xyz=None):
        self.prob = prob
        self._keep = []

        def keep(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a

        s = _Problem()
        s.P = prob.P
        s.degree = _p(keep(prob.degree, np.int32))
        s.node_ptr = _p(keep(prob.node_ptr, np.int64))
        s.xyz = _p(keep(prob.xyz, np.float64))
        txyz = prob.target_xyz if target_xyz is None else target_xyz
        s.NT = int(txyz.shape[0])
        s.txyz = _p(keep(txyz, np.float64))
        s.node_of_target = _p(keep(prob.node_of_target, np.int64))
        s.near_row_ptr = _p(keep(prob.near_row_ptr, np.int64))
        s.near_patch = _p(keep(prob.near_patch, np.int32))
        for d, uv in prob.ref_nodes.items():
            s.ref_uv[d] = _p(keep(uv, np.float64))
        al = prob.alpha if alpha is None else complex(alpha)
        be = prob.beta if beta is None else complex(beta)
        kk = prob.k if k is None else complex(k)
        s.alpha_re, s.alpha_im = al.real, al.imag
        s.beta_re, s.beta_im = be.real, be.imag
        s.k_re, s.k_im = kk.real, kk.imag
        s.tol = prob.tol if tol is None else tol
        s.loosen = loosen
        s.max_depth = (30 if mode == TRUTH else 16) if max_depth is None else max_depth
        s.ng = ng
        s.mode = mode
        self.s = s
        self.stats = Stats()

    def pair(self, t, j):
        """Weights a^j_l(x_t) (complex, length n_d)."""
        d = int(self.prob.degree[j])
        out = np.zeros(2 * nd_of(d))
        rc = lib().orc_pair_weights(C.byref(self.s), int(t), int(j), _p(out), C.byref(self.stats))
        if rc:
            raise RuntimeError("orc_pair_weights rc=%d" % rc)
        return out[0::2] + 1j * out[1::2]

    def row_ptr(self):
        rp = np.zeros(self.s.NT + 1, dtype=np.int64)
        lib().orc_row_ptr(C.byref(self.s), _p(rp))
        return rp

    def generate(self, t0=0, t1=None):
        """CSR rows (row_ptr, col, val complex) for targets [t0, t1)."""
        rp = self.row_ptr()
        t1 = self.s.NT if t1 is None else t1
        nnz = int(rp[-1])
        col = np.zeros(nnz, dtype=np.int32)
        val = np.zeros(2 * nnz)
        rc = lib().orc_generate_rows(C.byref(self.s), int(t0), int(t1), _p(rp), _p(col),
                                     _p(val), C.byref(self.stats))
        if rc:
            raise RuntimeError("orc_generate_rows rc=%d" % rc)
        return rp, col, val[0::2] + 1j * val[1::2]

    def pair_trace(self, t, j, cap=1 << 20):
        """Triangles checked by the adaptive scheme for pair (t, j):
        array of (depth << 56) | path code."""
        buf = np.zeros(cap, dtype=np.uint64)
        lib().orc_set_trace(_p(buf), cap)
        try:
            self.pair(t, j)
            n = lib().orc_trace_count()
        finally:
            lib().orc_set_trace(None, 0)
        return buf[:n].copy()

    def patch_info(self, j):
        dj, nv = np.zeros(1), np.zeros(1)
        lib().orc_patch_info(C.byref(self.s), int(j), _p(dj), _p(nv))
        return float(dj[0]), float(nv[0])

    def ball(self, j, lattice=64):
        """Centre (parametric mean of the chart) and radius (max over the
        lattice of T0) of patch j's bounding ball."""
        c, R = np.zeros(3), np.zeros(1)
        if lib().orc_patch_ball(C.byref(self.s), int(j), int(lattice), _p(c), _p(R)):
            raise RuntimeError("patch %d not set up" % j)
        return c, float(R[0])

    def chart(self, j, u, v):
        out = np.zeros(9)
        lib().orc_chart(C.byref(self.s), int(j), float(u), float(v), _p(out))
        return out[:3], out[3:6], out[6:]


def near_lists(prob, eta, centres, radii):
    """T_eta(x_t) by brute force (near-field definitions of Section 4): for
    every target, the patches j with |x_t - c_j| < eta R_j, own patch
    excluded, ascending; the balls (c_j, R_j) come from OracleRun.ball.
    Returns (row_ptr, patch, margin): margin[t] is the smallest
    | |x_t - c_j| - eta R_j | / R_j over all patches j, since a target that
    close to a ball's sphere can fall either way under rounding."""
    x = np.asarray(prob.target_xyz, dtype=np.float64)
    own = np.full(len(x), -1, dtype=np.int64)
    m = prob.node_of_target >= 0
    own[m] = np.searchsorted(prob.node_ptr, prob.node_of_target[m], side="right") - 1
    rows, margin = [], np.full(len(x), np.inf)
    for t0 in range(0, len(x), 512):
        xs = x[t0:t0 + 512]
        d = np.sqrt(((xs[:, None, :] - centres[None, :, :]) ** 2).sum(axis=2))
        r = eta * radii[None, :]
        margin[t0:t0 + 512] = (np.abs(d - r) / radii[None, :]).min(axis=1)
        hit = d < r
        for i in range(len(xs)):
            js = np.nonzero(hit[i])[0]
            rows.append(js[js != own[t0 + i]])
    rp = np.zeros(len(x) + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    pp = np.concatenate(rows).astype(np.int32) if rows else np.zeros(0, np.int32)
    return rp, pp, margin


def apply(row_ptr, col, val, sigma):
    nt = row_ptr.shape[0] - 1
    v = np.ascontiguousarray(np.stack([val.real, val.imag], 1).reshape(-1))
    s = np.asarray(sigma, dtype=np.complex128)
    sg = np.ascontiguousarray(np.stack([s.real, s.imag], 1).reshape(-1))
    y = np.zeros(2 * nt)
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    lib().orc_apply(nt, _p(rp), _p(cl), _p(v), _p(sg), _p(y))
    return y[0::2] + 1j * y[1::2]
