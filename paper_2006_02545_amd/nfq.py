"""Python binding of libnfq (include/nfq.h): argument marshalling only.

Every step of the generator runs in the HIP library; torch supplies device
memory and the stream.  Importing this module does not need a GPU; creating
a Context does, and fails loudly when the library or the device is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnfq.so")

NFQ_OK = 0
NFQ_WARN_NONCONVERGED = 1
NFQ_ERR_INVALID_ARG = -1
NFQ_ERR_NOT_REGISTERED = -2
STATUS = {0: "NFQ_OK", 1: "NFQ_WARN_NONCONVERGED", -1: "NFQ_ERR_INVALID_ARG",
          -2: "NFQ_ERR_NOT_REGISTERED", -3: "NFQ_ERR_DEGENERATE_PATCH",
          -4: "NFQ_ERR_SINGULAR_PAIR", -5: "NFQ_ERR_OUT_OF_MEMORY", -6: "NFQ_ERR_HIP",
          -7: "NFQ_ERR_UNSUPPORTED"}

EXPORTED = ["nfq_create", "nfq_destroy", "nfq_register_degree", "nfq_plan_create",
            "nfq_generate", "nfq_apply", "nfq_adjoint", "nfq_sync", "nfq_plan_destroy",
            "nfq_status_str", "nfq_last_error", "nfq_near_lists"]


class Surface(C.Structure):
    _fields_ = [("P", C.c_int64), ("degree", C.c_void_p), ("node_ptr", C.c_void_p),
                ("xyz", C.c_void_p)]


class Targets(C.Structure):
    _fields_ = [("NT", C.c_int64), ("xyz", C.c_void_p), ("node_of_target", C.c_void_p)]


class NearList(C.Structure):
    _fields_ = [("row_ptr", C.c_void_p), ("patch", C.c_void_p)]


class Kernel(C.Structure):
    _fields_ = [("alpha_re", C.c_double), ("alpha_im", C.c_double), ("beta_re", C.c_double),
                ("beta_im", C.c_double), ("k_re", C.c_double), ("k_im", C.c_double)]


class Params(C.Structure):
    _fields_ = [("tol", C.c_double), ("loosen", C.c_double), ("max_depth", C.c_int32),
                ("ng", C.c_int32), ("self_nr", C.c_int32), ("self_na", C.c_int32),
                ("flags", C.c_int32), ("min_depth", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("near_pairs", C.c_int64), ("self_pairs", C.c_int64), ("visits", C.c_int64),
                ("checks", C.c_int64), ("nonconverged", C.c_int64), ("max_level", C.c_int64),
                ("ms_builder", C.c_double), ("ms_prep", C.c_double), ("ms_self", C.c_double),
                ("ms_near", C.c_double), ("ms_weights", C.c_double)]

    def as_dict(self):
        return {f: (float(getattr(self, f)) if f.startswith("ms_") else int(getattr(self, f)))
                for f, _ in self._fields_}


NFQ_FLAG_TIMING = 1
NFQ_FLAG_PER_PAIR = 2


class NfqError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libnfq.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libnfq.so not built: run __graft_entry__.build() or "
                           "python -m paper_2006_02545_amd.build")
    L = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.nfq_create.argtypes = [C.c_int, vp, C.POINTER(vp)]
    L.nfq_create.restype = i32
    L.nfq_destroy.argtypes = [vp]
    L.nfq_destroy.restype = None
    L.nfq_register_degree.argtypes = [vp, C.c_int, vp, vp]
    L.nfq_register_degree.restype = i32
    L.nfq_plan_create.argtypes = [vp, C.POINTER(Surface), C.POINTER(Targets),
                                  C.POINTER(NearList), C.POINTER(vp), C.POINTER(i64), vp]
    L.nfq_plan_create.restype = i32
    L.nfq_generate.argtypes = [vp, C.POINTER(Kernel), C.POINTER(Params), vp, vp, vp]
    L.nfq_generate.restype = i32
    L.nfq_apply.argtypes = [vp, vp, vp, vp, vp]
    L.nfq_adjoint.argtypes = [vp, C.POINTER(Kernel), C.POINTER(Params), vp, vp, vp, vp, vp]
    L.nfq_adjoint.restype = i32
    L.nfq_apply.restype = i32
    L.nfq_sync.argtypes = [vp]
    L.nfq_sync.restype = i32
    L.nfq_near_lists.argtypes = [vp, C.POINTER(Surface), C.POINTER(Targets), C.c_double, vp, vp,
                                 i64, C.POINTER(i64), vp, vp]
    L.nfq_near_lists.restype = i32
    L.nfq_plan_destroy.argtypes = [vp]
    L.nfq_plan_destroy.restype = None
    L.nfq_status_str.argtypes = [i32]
    L.nfq_status_str.restype = C.c_char_p
    L.nfq_last_error.argtypes = [vp]
    L.nfq_last_error.restype = C.c_char_p
    _lib = L
    return L


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Context:
    """A library context on the current torch CUDA (HIP) device and stream."""

    def __init__(self, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the generator runs only on the GPU")
        self.torch = torch
        self.L = load()
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        h = C.c_void_p()
        self._check(self.L.nfq_create(self.device, C.c_void_p(self.stream.cuda_stream),
                                      C.byref(h)), None)
        self.h = h
        self.registered = {}
        # plans of this context, closed before it (whatever order the
        # garbage collector finalises them in)
        self._plans = weakref.WeakSet()

    def _check(self, st, h=None):
        if st < 0:
            raise NfqError(st, self.L.nfq_last_error(h).decode())
        return st

    def register_degree(self, d, uv, w=None):
        uv = np.ascontiguousarray(uv, dtype=np.float64)
        wp = None
        if w is not None:
            w = np.ascontiguousarray(w, dtype=np.float64)
            wp = w.ctypes.data_as(C.c_void_p)
        self._check(self.L.nfq_register_degree(self.h, int(d), uv.ctypes.data_as(C.c_void_p), wp),
                    self.h)
        self.registered[int(d)] = uv

    def near_lists(self, degree, node_ptr, xyz, target_xyz, node_of_target, eta):
        """Near lists on the device (nfq_near_lists): returns device tensors
        (row_ptr [NT+1] int64, patch [nnz] int32, centres [P,3], radii [P])."""
        torch = self.torch
        dev = torch.device("cuda", self.device)

        def dt(a, dtype):
            if isinstance(a, torch.Tensor):
                return a.to(device=dev, dtype=dtype).contiguous()
            return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=dev)

        deg, nptr, x = dt(degree, torch.int32), dt(node_ptr, torch.int64), dt(xyz, torch.float64)
        tx, nt = dt(target_xyz, torch.float64), dt(node_of_target, torch.int64)
        P, NT = int(deg.shape[0]), int(tx.shape[0])
        surf = Surface(P, deg.data_ptr(), nptr.data_ptr(), x.data_ptr())
        tg = Targets(NT, tx.data_ptr(), nt.data_ptr())
        row_ptr = torch.empty(NT + 1, dtype=torch.int64, device=dev)
        centres = torch.empty((P, 3), dtype=torch.float64, device=dev)
        radii = torch.empty(P, dtype=torch.float64, device=dev)
        nnz = C.c_int64()
        # first call sizes the output (capacity 0), the second fills it
        st = self.L.nfq_near_lists(self.h, C.byref(surf), C.byref(tg), float(eta), _ptr(row_ptr),
                                   None, 0, C.byref(nnz), _ptr(centres), _ptr(radii))
        if st < 0 and nnz.value == 0:
            self._check(st, self.h)
        patch = torch.empty(max(int(nnz.value), 1), dtype=torch.int32, device=dev)
        if nnz.value > 0:
            self._check(self.L.nfq_near_lists(self.h, C.byref(surf), C.byref(tg), float(eta),
                                              _ptr(row_ptr), _ptr(patch), int(nnz.value),
                                              C.byref(nnz), _ptr(centres), _ptr(radii)), self.h)
        return row_ptr, patch[:int(nnz.value)], centres, radii

    def close(self):
        if getattr(self, "h", None):
            for p in list(getattr(self, "_plans", ())):
                p.close()
            self.L.nfq_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Sizing and scratch for one (surface, targets, near list); owns the
    device copies of the inputs it was given (torch tensors)."""

    def __init__(self, ctx: Context, degree, node_ptr, xyz, target_xyz, node_of_target,
                 near_row_ptr, near_patch):
        torch = ctx.torch
        dev = torch.device("cuda", ctx.device)
        self.ctx = ctx

        def dt(a, dtype):
            if isinstance(a, torch.Tensor):
                return a.to(device=dev, dtype=dtype).contiguous()
            return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=dev)

        self.degree = dt(degree, torch.int32)
        self.node_ptr = dt(node_ptr, torch.int64)
        self.xyz = dt(xyz, torch.float64)
        self.target_xyz = dt(target_xyz, torch.float64)
        self.node_of_target = dt(node_of_target, torch.int64)
        self.near_row_ptr = dt(near_row_ptr, torch.int64)
        self.near_patch = dt(near_patch, torch.int32)
        self.P = int(self.degree.shape[0])
        self.NT = int(self.target_xyz.shape[0])
        self.N = int(self.xyz.shape[0])
        self.row_ptr = torch.empty(self.NT + 1, dtype=torch.int64, device=dev)
        self.surf = Surface(self.P, self.degree.data_ptr(), self.node_ptr.data_ptr(),
                            self.xyz.data_ptr())
        self.tg = Targets(self.NT, self.target_xyz.data_ptr(), self.node_of_target.data_ptr())
        self.near = NearList(self.near_row_ptr.data_ptr(), self.near_patch.data_ptr())
        h = C.c_void_p()
        nnz = C.c_int64()
        ctx._check(ctx.L.nfq_plan_create(ctx.h, C.byref(self.surf), C.byref(self.tg),
                                         C.byref(self.near), C.byref(h), C.byref(nnz),
                                         _ptr(self.row_ptr)), ctx.h)
        self.h = h
        self.nnz = int(nnz.value)
        ctx._plans.add(self)

    def generate(self, alpha, beta, k, tol, loosen=1.0, max_depth=16, self_nr=0, self_na=0,
                 col=None, val=None, stats=True, timing=False, per_pair=False, min_depth=0):
        """Run the generator; returns (col, val, stats dict or None).  val is
        complex128 (or float64 for a real kernel) of length nnz."""
        torch = self.ctx.torch
        dev = self.row_ptr.device
        alpha, beta, k = complex(alpha), complex(beta), complex(k)
        real = (k == 0 and alpha.imag == 0 and beta.imag == 0)
        if col is None:
            col = torch.empty(self.nnz, dtype=torch.int32, device=dev)
        if val is None:
            val = torch.empty(self.nnz, dtype=torch.float64 if real else torch.complex128,
                              device=dev)
        kern = Kernel(alpha.real, alpha.imag, beta.real, beta.imag, k.real, k.imag)
        flags = (NFQ_FLAG_TIMING if timing else 0) | (NFQ_FLAG_PER_PAIR if per_pair else 0)
        prm = Params(float(tol), float(loosen), int(max_depth), 0, int(self_nr), int(self_na),
                     flags, int(min_depth))
        st = Stats()
        rc = self.ctx.L.nfq_generate(self.h, C.byref(kern), C.byref(prm), _ptr(col), _ptr(val),
                                     C.byref(st) if stats else None)
        self.ctx._check(rc, self.ctx.h)
        self.last_status = rc
        return col, val, (st.as_dict() if stats else None)

    def adjoint(self, alpha, beta, k, tol, sigma, lam, loosen=1.0, max_depth=16, self_nr=0,
                self_na=0, min_depth=0):
        """Gradient of Phi = sum_t conj(lam_t) (A sigma)_t: returns
        (grad_xyz [N,3] complex, dPhi/dk, dPhi/dalpha, dPhi/dbeta)."""
        torch = self.ctx.torch
        dev = self.row_ptr.device
        alpha, beta, k = complex(alpha), complex(beta), complex(k)
        sig = torch.as_tensor(np.ascontiguousarray(sigma, dtype=np.complex128), device=dev)
        lmb = torch.as_tensor(np.ascontiguousarray(lam, dtype=np.complex128), device=dev)
        grad = torch.empty((self.N, 3), dtype=torch.complex128, device=dev)
        gk = torch.empty(1, dtype=torch.complex128, device=dev)
        dab = torch.empty(2, dtype=torch.complex128, device=dev)
        kern = Kernel(alpha.real, alpha.imag, beta.real, beta.imag, k.real, k.imag)
        prm = Params(float(tol), float(loosen), int(max_depth), 0, int(self_nr), int(self_na), 0,
                     int(min_depth))
        self.ctx._check(self.ctx.L.nfq_adjoint(self.h, C.byref(kern), C.byref(prm), _ptr(sig),
                                               _ptr(lmb), _ptr(grad), _ptr(gk), _ptr(dab)),
                        self.ctx.h)
        self.ctx.torch.cuda.synchronize()
        return grad.cpu().numpy(), complex(gk.cpu().numpy()[0]), *[complex(v) for v in dab.cpu().numpy()]

    def adjoint_into(self, alpha, beta, k, tol, sigma, lam, grad, gk, dab, loosen=1.0,
                     max_depth=16, min_depth=0):
        """Adjoint into caller-allocated device tensors (no host copies)."""
        alpha, beta, k = complex(alpha), complex(beta), complex(k)
        kern = Kernel(alpha.real, alpha.imag, beta.real, beta.imag, k.real, k.imag)
        prm = Params(float(tol), float(loosen), int(max_depth), 0, 0, 0, 0, int(min_depth))
        self.ctx._check(self.ctx.L.nfq_adjoint(self.h, C.byref(kern), C.byref(prm), _ptr(sigma),
                                               _ptr(lam), _ptr(grad), _ptr(gk), _ptr(dab)),
                        self.ctx.h)

    def apply(self, col, val, sigma):
        torch = self.ctx.torch
        y = torch.empty(self.NT, dtype=val.dtype, device=val.device)
        sigma = sigma.to(device=val.device, dtype=val.dtype).contiguous()
        self.ctx._check(self.ctx.L.nfq_apply(self.h, _ptr(col), _ptr(val), _ptr(sigma), _ptr(y)),
                        self.ctx.h)
        return y

    def close(self):
        if getattr(self, "h", None):
            self.ctx.L.nfq_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_for(ctx: Context, prob):
    """Register the problem's degrees and build a plan (surfaces.Problem)."""
    for d, uv in prob.ref_nodes.items():
        if int(d) not in ctx.registered:
            ctx.register_degree(int(d), uv)
    return Plan(ctx, prob.degree, prob.node_ptr, prob.xyz, prob.target_xyz, prob.node_of_target,
                prob.near_row_ptr, prob.near_patch)
