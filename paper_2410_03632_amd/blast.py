"""Python binding of ``libblast_hip.so`` (ctypes; argument marshalling only).

Every step of the C_ell evaluation runs in the HIP library; this module only
converts torch device tensors and numpy host arrays into the pointers and sizes
of the C ABI declared in ``include/blast_hip.h``.  If the library is missing the
import of any entry point raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libblast_hip.so")

OK, E_INVALID, E_OOM, E_HIP, E_UNSUPPORTED, E_BUSY, E_CANCELLED = range(7)
FP64, FP32, BF16, BF16X3, FP16X3 = range(5)
GG, GS, SS = 1, 2, 4
PRECISION = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "bf16x3": BF16X3, "fp16x3": FP16X3}
TYPE_BITS = {"gg": GG, "gs": GS, "ss": SS}


class BlastError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("blast status %d: %s" % (status, msg))
        self.status = status


class PlanDesc(C.Structure):
    _fields_ = [
        ("n_ell", C.c_int32), ("ell", C.POINTER(C.c_double)),
        ("n_chi", C.c_int32), ("chi", C.POINTER(C.c_double)), ("w_chi", C.POINTER(C.c_double)),
        ("n_R", C.c_int32), ("R", C.POINTER(C.c_double)), ("w_R", C.POINTER(C.c_double)),
        ("k_min", C.c_double), ("k_max", C.c_double),
        ("n_cheb", C.c_int32), ("types", C.c_uint32), ("precisions", C.c_uint32),
        ("kq_panels", C.c_int32), ("kq_phase", C.c_double),
    ]


class ClArgs(C.Structure):
    _fields_ = [
        ("batch", C.c_int32), ("precision", C.c_int32), ("p_dtype", C.c_int32), ("p_kind", C.c_int32),
        ("P", C.c_void_p), ("n_g", C.c_int32), ("n_s", C.c_int32),
        ("K_chi", C.c_void_p), ("K_chi2", C.c_void_p), ("types", C.c_uint32),
        ("n_ell_out", C.c_int32), ("ell_idx", C.POINTER(C.c_int32)),
        ("C", C.c_void_p), ("w_save", C.c_void_p),
        ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t), ("y_save", C.c_void_p),
    ]


class LimberArgs(C.Structure):
    _fields_ = [
        ("batch", C.c_int32), ("p_dtype", C.c_int32), ("P", C.c_void_p), ("P_sub", C.c_void_p),
        ("n_g", C.c_int32), ("n_s", C.c_int32), ("K_chi", C.c_void_p), ("types", C.c_uint32),
        ("n_ell_out", C.c_int32), ("ell_idx", C.POINTER(C.c_int32)), ("order", C.c_int32),
        ("accumulate", C.c_int32), ("C", C.c_void_p),
    ]


class ServerDesc(C.Structure):
    _fields_ = [("precision", C.c_int32), ("p_dtype", C.c_int32), ("batch", C.c_int32), ("n_sets", C.c_int32),
                ("max_g", C.c_int32), ("max_s", C.c_int32), ("hbm_budget", C.c_size_t), ("max_queue", C.c_int32),
                ("max_wait_ms", C.c_double), ("use_graphs", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("P", C.c_void_p), ("n_g", C.c_int32), ("n_s", C.c_int32), ("K_chi", C.c_void_p),
                ("K_chi2", C.c_void_p), ("n_ell", C.c_int32), ("ell_idx", C.POINTER(C.c_int32)),
                ("C_out", C.c_void_p)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64),
                ("launches", C.c_int64), ("queued", C.c_int64), ("in_flight", C.c_int64),
                ("mean_fill", C.c_double), ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("span_ms", C.c_double), ("cancelled", C.c_int64), ("max_sets_in_flight", C.c_int64),
                ("n_sets", C.c_int64), ("set_bytes", C.c_int64)]


EXPORTS = [
    "blast_last_error", "blast_version", "blast_grid_chi_simpson", "blast_grid_R_fejer", "blast_grid_k_cheb",
    "blast_plan_create", "blast_plan_destroy", "blast_plan_info", "blast_plan_k_nodes", "blast_plan_basis_point",
    "blast_cl_workspace_bytes", "blast_cl_forward", "blast_cl_forward_noalloc", "blast_cl_backward",
    "blast_plan_profile",
    "blast_plan_profile_read", "blast_plan_save", "blast_plan_load", "blast_plan_eval_points",
    "blast_plan_grids", "blast_plan_limber_k", "blast_cl_limber",
    "blast_server_create", "blast_server_footprint", "blast_server_submit", "blast_server_cancel",
    "blast_server_wait", "blast_server_poll", "blast_server_stats_get", "blast_server_destroy",
]
STAGES = ("projection", "contraction", "quad_R", "quad_chi")

_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libblast_hip.so is not built; run `python -m paper_2410_03632_amd.build_lib`")
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.blast_last_error.restype = C.c_char_p
        L.blast_version.restype = C.c_char_p
        L.blast_grid_chi_simpson.argtypes = [C.c_int32, C.c_double, C.c_double, dp, dp]
        L.blast_grid_R_fejer.argtypes = [C.c_int32, C.c_double, dp, dp]
        L.blast_grid_k_cheb.argtypes = [C.c_int32, C.c_double, C.c_double, dp]
        L.blast_plan_create.argtypes = [C.POINTER(PlanDesc), C.c_int32, C.POINTER(C.c_void_p)]
        L.blast_plan_destroy.argtypes = [C.c_void_p]
        L.blast_plan_info.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_size_t), C.POINTER(C.c_int64), dp]
        L.blast_plan_k_nodes.argtypes = [C.c_void_p, dp]
        L.blast_plan_basis_point.argtypes = [C.c_void_p, C.c_int32, C.c_int32, dp]
        L.blast_cl_workspace_bytes.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                               C.POINTER(C.c_size_t)]
        L.blast_cl_forward.argtypes = [C.c_void_p, C.POINTER(ClArgs), C.c_void_p]
        L.blast_cl_forward_noalloc.argtypes = [C.c_void_p, C.POINTER(ClArgs), C.c_void_p]
        L.blast_cl_backward.argtypes = [C.c_void_p, C.POINTER(ClArgs), C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p]
        L.blast_server_create.argtypes = [C.c_void_p, C.POINTER(ServerDesc), C.POINTER(C.c_void_p)]
        L.blast_server_submit.argtypes = [C.c_void_p, C.POINTER(Request), C.POINTER(C.c_uint64)]
        L.blast_server_wait.argtypes = [C.c_void_p, C.c_uint64, C.c_int32, C.POINTER(C.c_int),
                                        C.POINTER(C.c_double)]
        L.blast_server_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(C.c_int),
                                        C.POINTER(C.c_double)]
        L.blast_server_cancel.argtypes = [C.c_void_p, C.c_uint64]
        L.blast_server_footprint.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_size_t),
                                             C.POINTER(C.c_size_t)]
        L.blast_server_stats_get.argtypes = [C.c_void_p, C.POINTER(ServerStats)]
        L.blast_server_destroy.argtypes = [C.c_void_p]
        L.blast_plan_profile.argtypes = [C.c_void_p, C.c_int32]
        L.blast_plan_save.argtypes = [C.c_void_p, C.c_char_p]
        L.blast_plan_load.argtypes = [C.c_char_p, C.c_int32, C.c_uint32, C.POINTER(C.c_void_p)]
        L.blast_plan_eval_points.argtypes = [C.c_void_p, dp, dp]
        L.blast_plan_limber_k.argtypes = [C.c_void_p, dp]
        L.blast_cl_limber.argtypes = [C.c_void_p, C.POINTER(LimberArgs), C.c_void_p]
        i32p = C.POINTER(C.c_int32)
        L.blast_plan_grids.argtypes = [C.c_void_p, i32p, i32p, i32p, i32p, C.POINTER(C.c_uint32), dp, dp,
                                       dp, dp, dp, dp, dp]
        L.blast_plan_profile_read.argtypes = [C.c_void_p, dp, C.POINTER(C.c_int64)]
        for name in EXPORTS:
            if name not in ("blast_last_error", "blast_version"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(st):
    if st != OK:
        raise BlastError(st, lib().blast_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def version() -> str:
    return lib().blast_version().decode()


# ------------------------------------------------------------------------------- grids

def grid_chi_simpson(n, lo, hi):
    chi, w = np.empty(n), np.empty(n)
    _check(lib().blast_grid_chi_simpson(n, lo, hi, _dptr(chi), _dptr(w)))
    return chi, w


def grid_R_fejer(n, R_min):
    R, w = np.empty(n), np.empty(n)
    _check(lib().blast_grid_R_fejer(n, R_min, _dptr(R), _dptr(w)))
    return R, w


def grid_k_cheb(n, k_min, k_max):
    k = np.empty(n)
    _check(lib().blast_grid_k_cheb(n, k_min, k_max, _dptr(k)))
    return k


def types_mask(types) -> int:
    if isinstance(types, int):
        return types
    m = 0
    for t in types:
        m |= TYPE_BITS[t]
    return m


def n_pairs(n_g, n_s, types=7) -> int:
    t = types_mask(types)
    return ((n_g * (n_g + 1) // 2) if t & GG else 0) + ((n_g * n_s) if t & GS else 0) + \
        ((n_s * (n_s + 1) // 2) if t & SS else 0)


# ------------------------------------------------------------------------------- plan

def _pmask(precisions):
    m = 0
    for p in precisions or ():
        m |= 1 << (PRECISION[p] if isinstance(p, str) else int(p))
    return m


class Plan:
    """Grids plus the resident basis of Eq. t_tilde on one GPU.

    `precisions` lists the contraction arithmetics kept resident ("fp64" is always built):
    "fp64"; "fp32"; "fp16x3" (FP16 hi + lo parts with power-of-two row scales, the fastest path
    inside 1e-3; fused path only: at most 20 bins, no w_save, no adjoint); "bf16x3"; "bf16"."""

    def __init__(self, ell, chi, w_chi, R, w_R, k_min, k_max, n_cheb, *, types=7,
                 precisions=("fp64",), kq_panels=0, kq_phase=0.0, device=0):
        self.device = int(device)
        ell = np.ascontiguousarray(ell, dtype=np.float64)   # integer or not
        chi = np.ascontiguousarray(chi, dtype=np.float64)
        w_chi = np.ascontiguousarray(w_chi, dtype=np.float64)
        R = np.ascontiguousarray(R, dtype=np.float64)
        w_R = np.ascontiguousarray(w_R, dtype=np.float64)
        d = PlanDesc(len(ell), _dptr(ell),
                     len(chi), _dptr(chi), _dptr(w_chi), len(R), _dptr(R), _dptr(w_R),
                     float(k_min), float(k_max), int(n_cheb), types_mask(types), _pmask(precisions),
                     int(kq_panels), float(kq_phase))
        h = C.c_void_p()
        _check(lib().blast_plan_create(C.byref(d), self.device, C.byref(h)))
        self._attach(h)

    @classmethod
    def load(cls, path, device=0, precisions=()):
        """Rebuild a plan from a checkpoint written by save() (blast_plan_load); an empty
        `precisions` keeps the saved set."""
        h = C.c_void_p()
        _check(lib().blast_plan_load(os.fsencode(path), int(device), _pmask(precisions), C.byref(h)))
        self = cls.__new__(cls)
        self.device = int(device)
        self._attach(h)
        return self

    def save(self, path):
        """Checkpoint the grids and the FP64 basis (blast_plan_save)."""
        _check(lib().blast_plan_save(self._h, os.fsencode(path)))

    def _attach(self, h):
        self._h = h
        L = lib()
        ne, nc, nr, nch = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        ty = C.c_uint32()
        kmin, kmax = C.c_double(), C.c_double()
        _check(L.blast_plan_grids(h, C.byref(ne), C.byref(nc), C.byref(nr), C.byref(nch), C.byref(ty),
                                  C.byref(kmin), C.byref(kmax), None, None, None, None, None))
        self.ell = np.empty(ne.value)
        self.chi, self.w_chi = np.empty(nc.value), np.empty(nc.value)
        self.R, self.w_R = np.empty(nr.value), np.empty(nr.value)
        _check(L.blast_plan_grids(h, None, None, None, None, None, None, None,
                                  _dptr(self.ell), _dptr(self.chi),
                                  _dptr(self.w_chi), _dptr(self.R), _dptr(self.w_R)))
        self.k_min, self.k_max, self.n_cheb, self.types = kmin.value, kmax.value, nch.value, ty.value
        rows, ncp = C.c_int32(), C.c_int32()
        bb = (C.c_size_t * 5)()
        kq = C.c_int64()
        ms = C.c_double()
        _check(L.blast_plan_info(h, C.byref(rows), C.byref(ncp), bb, C.byref(kq), C.byref(ms)))
        self.rows, self.nc_pad = rows.value, ncp.value
        self.rows_pad = (self.rows + 15) // 16 * 16
        self.basis_bytes = list(bb)
        self.kq_nodes, self.build_ms = kq.value, ms.value
        self.k_nodes = np.empty(self.n_cheb)
        _check(L.blast_plan_k_nodes(h, _dptr(self.k_nodes)))

    @property
    def handle(self):
        return self._h

    @property
    def n_ell(self):
        return len(self.ell)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().blast_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def basis_point(self, a, b):
        out = np.empty((self.rows, self.n_cheb))
        _check(lib().blast_plan_basis_point(self._h, a, b, _dptr(out)))
        return out

    def profile(self, enable=True):
        """Record HIP events around the four stages of every forward call."""
        _check(lib().blast_plan_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """(dict stage -> summed ms, number of calls) since the last read."""
        ms = (C.c_double * 4)()
        n = C.c_int64()
        _check(lib().blast_plan_profile_read(self._h, ms, C.byref(n)))
        return dict(zip(STAGES, list(ms))), n.value

    def eval_points(self):
        """(chi_a, R_b chi_a): where to evaluate the kernels and P (blast_plan_eval_points)."""
        chi, chi2 = np.empty(len(self.chi)), np.empty((len(self.chi), len(self.R)))
        _check(lib().blast_plan_eval_points(self._h, _dptr(chi), _dptr(chi2)))
        return chi, chi2

    def workspace_bytes(self, batch, precision, n_bins):
        n = C.c_size_t()
        _check(lib().blast_cl_workspace_bytes(self._h, batch, PRECISION.get(precision, precision), n_bins,
                                              C.byref(n)))
        return n.value

    def _prepare(self, P, K_chi, K_chi2, n_g, n_s, precision, types, ell_idx, coef):
        import torch
        prec = PRECISION.get(precision, precision)
        if P.dim() == 3:
            P = P.unsqueeze(0)
        if K_chi.dim() == 2:
            K_chi = K_chi.unsqueeze(0)
        if K_chi2.dim() == 3:
            K_chi2 = K_chi2.unsqueeze(0)
        B = P.shape[0]
        for t, nm in ((P, "P"), (K_chi, "K_chi"), (K_chi2, "K_chi2")):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("%s must be a contiguous device tensor" % nm)
        if P.dtype not in (torch.float64, torch.float32):
            raise ValueError("P must be float64 or float32")
        if K_chi.dtype != torch.float64 or K_chi2.dtype != torch.float64:
            raise ValueError("kernels must be float64")
        nb = n_g + n_s
        if tuple(P.shape) != (B, len(self.chi), len(self.R), self.n_cheb):
            raise ValueError("P shape %s, expected %s" % (tuple(P.shape), (B, len(self.chi), len(self.R), self.n_cheb)))
        if tuple(K_chi.shape) != (B, nb, len(self.chi)) or tuple(K_chi2.shape) != (B, nb, len(self.chi), len(self.R)):
            raise ValueError("kernel shapes do not match (batch, bins, chi[, R])")
        tmask = self.types if types is None else types_mask(types)
        npair = n_pairs(n_g, n_s, tmask)
        if ell_idx is None:
            n_out, idx_arr, n_l = 0, None, self.n_ell
        else:
            idx_arr = np.ascontiguousarray(ell_idx, dtype=np.int32)
            n_out = n_l = len(idx_arr)
        args = ClArgs(B, prec, 0 if P.dtype == torch.float64 else 1, 1 if coef else 0, P.data_ptr(), n_g, n_s,
                      K_chi.data_ptr(), K_chi2.data_ptr(), tmask, n_out,
                      idx_arr.ctypes.data_as(C.POINTER(C.c_int32)) if idx_arr is not None else None,
                      None, None, None, 0, None)
        return args, (P, K_chi, K_chi2, idx_arr), (B, npair, n_l), prec

    def limber_k(self):
        """k[l][a] = (ell_l + 1/2) / chi_a: where the Limber approximation samples P."""
        k = np.empty((self.n_ell, len(self.chi)))
        _check(lib().blast_plan_limber_k(self._h, _dptr(k)))
        return k

    def limber(self, P, K_chi, n_g, n_s, *, P_sub=None, order=1, types=None, ell_idx=None, out=None,
               accumulate=False, stream=None):
        """Limber (order 1) or extended Limber (order 2) spectra C[batch][pair][ell] (blast_cl_limber)
        from P [B, n_ell, n_chi] at the Limber points (minus P_sub if given) and K_chi [B, bins, n_chi].
        With accumulate=True the result is added to `out` (e.g. the beyond-Limber C of the linear
        spectrum, for the non-linear correction)."""
        import torch
        if P.dim() == 2:
            P = P.unsqueeze(0)
        if K_chi.dim() == 2:
            K_chi = K_chi.unsqueeze(0)
        B = P.shape[0]
        if tuple(P.shape) != (B, self.n_ell, len(self.chi)) or not P.is_cuda or not P.is_contiguous():
            raise ValueError("P must be a contiguous device tensor of shape (batch, n_ell, n_chi)")
        if P.dtype not in (torch.float64, torch.float32):
            raise ValueError("P must be float64 or float32")
        if P_sub is not None and (P_sub.shape != P.shape or P_sub.dtype != P.dtype or not P_sub.is_contiguous()):
            raise ValueError("P_sub must match P")
        if K_chi.dtype != torch.float64 or tuple(K_chi.shape) != (B, n_g + n_s, len(self.chi)):
            raise ValueError("K_chi must be float64 of shape (batch, bins, n_chi)")
        tmask = self.types if types is None else types_mask(types)
        npair = n_pairs(n_g, n_s, tmask)
        if ell_idx is None:
            n_out, idx_arr, n_l = 0, None, self.n_ell
        else:
            idx_arr = np.ascontiguousarray(ell_idx, dtype=np.int32)
            n_out = n_l = len(idx_arr)
        shape = (B, npair, n_l)
        if out is None:
            if accumulate:
                raise ValueError("accumulate needs out")
            out = torch.empty(shape, dtype=torch.float64, device=P.device)
        elif tuple(out.shape) != shape or out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor of shape %s" % (shape,))
        args = LimberArgs(B, 0 if P.dtype == torch.float64 else 1, P.data_ptr(),
                          P_sub.data_ptr() if P_sub is not None else None, n_g, n_s, K_chi.data_ptr(), tmask, n_out,
                          idx_arr.ctypes.data_as(C.POINTER(C.c_int32)) if idx_arr is not None else None,
                          int(order), 1 if accumulate else 0, out.data_ptr())
        if stream is None:
            stream = torch.cuda.current_stream(P.device).cuda_stream
        _check(lib().blast_cl_limber(self._h, C.byref(args), C.c_void_p(stream)))
        return out

    def cl_hybrid(self, P, K_chi, K_chi2, P_limber, n_g, n_s, ell_cut, *, order=2, precision="fp64", types=None):
        """Beyond-Limber spectra below ell_cut and (extended) Limber spectra from ell_cut on: one
        forward call for the low multipoles, one Limber call for the high ones, assembled into
        C[batch][pair][ell] over all plan multipoles."""
        import torch
        lo = np.nonzero(self.ell < ell_cut)[0].astype(np.int32)
        hi = np.nonzero(self.ell >= ell_cut)[0].astype(np.int32)
        Pb = P if P.dim() == 4 else P.unsqueeze(0)
        tmask = self.types if types is None else types_mask(types)
        out = torch.empty((Pb.shape[0], n_pairs(n_g, n_s, tmask), self.n_ell), dtype=torch.float64, device=P.device)
        if len(lo):
            out[:, :, lo] = self.forward(P, K_chi, K_chi2, n_g, n_s, precision=precision, types=types, ell_idx=lo)
        if len(hi):
            out[:, :, hi] = self.limber(P_limber, K_chi, n_g, n_s, order=order, types=types, ell_idx=hi)
        return out

    def y_numel(self, batch, n_bins):
        """Values of a y_save buffer: batch * rows_pad * n_chi * (16 for at most 16 bins, else 32)."""
        return batch * self.rows_pad * len(self.chi) * (16 if n_bins <= 16 else 32)

    def _w_ws(self, args, B, prec, w_save, workspace, y_save=None, n_bins=0):
        import torch
        wdt = torch.float64 if prec == FP64 else torch.float32
        if w_save is not None:
            if w_save.dtype != wdt or w_save.numel() != B * len(self.chi) * len(self.R) * self.rows_pad \
                    or not w_save.is_contiguous():
                raise ValueError("w_save must hold batch*n_chi*n_R*rows_pad contiguous values of %s" % wdt)
            args.w_save = w_save.data_ptr()
        if y_save is not None:
            if y_save.dtype != wdt or y_save.numel() != self.y_numel(B, n_bins) or not y_save.is_contiguous():
                raise ValueError("y_save must hold %d contiguous values of %s" % (self.y_numel(B, n_bins), wdt))
            args.y_save = y_save.data_ptr()
        if workspace is not None:
            args.workspace = workspace.data_ptr()
            args.workspace_bytes = workspace.numel() * workspace.element_size()

    def forward(self, P, K_chi, K_chi2, n_g, n_s, *, precision="fp64", types=None, ell_idx=None,
                out=None, w_save=None, workspace=None, stream=None, coef=False, y_save=None):
        """C[batch][pair][ell] for device tensors P [B, n_chi, n_R, n_cheb] (float64/float32; nodal
        values, or Chebyshev coefficients with coef=True), K_chi [B, bins, n_chi] and
        K_chi2 [B, bins, n_chi, n_R] (float64)."""
        import torch
        args, keep, shape, prec = self._prepare(P, K_chi, K_chi2, n_g, n_s, precision, types, ell_idx, coef)
        P = keep[0]
        if out is None:
            out = torch.empty(shape, dtype=torch.float64, device=P.device)
        elif tuple(out.shape) != shape or out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor of shape %s" % (shape,))
        args.C = out.data_ptr()
        self._w_ws(args, shape[0], prec, w_save, workspace, y_save, n_g + n_s)
        if stream is None:
            stream = torch.cuda.current_stream(P.device).cuda_stream
        _check(lib().blast_cl_forward(self._h, C.byref(args), C.c_void_p(stream)))
        return out

    def forward_noalloc(self, P, K_chi, K_chi2, n_g, n_s, out, *, precision="fp64", types=None, ell_idx=None,
                        stream=None, coef=False):
        """forward() through blast_cl_forward_noalloc: the library allocates nothing (its scratch
        is a fixed 64 MiB device array per GPU) and `out` must be given."""
        import torch
        args, keep, shape, prec = self._prepare(P, K_chi, K_chi2, n_g, n_s, precision, types, ell_idx, coef)
        P = keep[0]
        if tuple(out.shape) != shape or out.dtype != torch.float64 or not out.is_contiguous() or not out.is_cuda:
            raise ValueError("out must be a contiguous float64 device tensor of shape %s" % (shape,))
        args.C = out.data_ptr()
        if stream is None:
            stream = torch.cuda.current_stream(P.device).cuda_stream
        _check(lib().blast_cl_forward_noalloc(self._h, C.byref(args), C.c_void_p(stream)))
        return out

    def backward(self, P, K_chi, K_chi2, n_g, n_s, dC, *, precision="fp64", types=None, ell_idx=None,
                 w_save=None, workspace=None, stream=None, coef=False, want=("P", "K_chi", "K_chi2"), y_save=None):
        """Gradients (dP, dK_chi, dK_chi2) of a scalar loss given dC = dL/dC (device float64,
        shaped like the forward output); entries not in `want` are None."""
        import torch
        args, keep, shape, prec = self._prepare(P, K_chi, K_chi2, n_g, n_s, precision, types, ell_idx, coef)
        P, K_chi, K_chi2 = keep[:3]
        if tuple(dC.shape) != shape or dC.dtype != torch.float64 or not dC.is_contiguous() or not dC.is_cuda:
            raise ValueError("dC must be a contiguous float64 device tensor of shape %s" % (shape,))
        self._w_ws(args, shape[0], prec, w_save, workspace, y_save, n_g + n_s)
        dP = torch.empty_like(P) if "P" in want else None
        dK = torch.empty_like(K_chi) if "K_chi" in want else None
        dK2 = torch.empty_like(K_chi2) if "K_chi2" in want else None
        if stream is None:
            stream = torch.cuda.current_stream(P.device).cuda_stream
        ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None else None
        _check(lib().blast_cl_backward(self._h, C.byref(args), C.c_void_p(dC.data_ptr()), ptr(dP), ptr(dK),
                                       ptr(dK2), C.c_void_p(stream)))
        return dP, dK, dK2


def _make_cl_function():
    import torch

    class ClFunction(torch.autograd.Function):
        """C = ClFunction.apply(plan, P, K_chi, K_chi2, n_g, n_s, precision, coef), differentiable in
        P (nodal values or Chebyshev coefficients) and the two kernel tables through the
        library's hand-written adjoint."""

        @staticmethod
        def forward(ctx, plan, P, K_chi, K_chi2, n_g, n_s, precision="fp64", coef=False):
            P, K_chi, K_chi2 = P.contiguous(), K_chi.contiguous(), K_chi2.contiguous()
            wdt = torch.float64 if PRECISION.get(precision, precision) == FP64 else torch.float32
            B = P.shape[0] if P.dim() == 4 else 1
            # the adjoint reads w only for dK_chi2 and Y only for dK_chi: keep what it will read
            keep_w, keep_y = ctx.needs_input_grad[3], ctx.needs_input_grad[2]
            w = torch.empty(B * len(plan.chi) * len(plan.R) * plan.rows_pad, dtype=wdt,
                            device=P.device) if keep_w else None
            y = torch.empty(plan.y_numel(B, n_g + n_s), dtype=wdt, device=P.device) if keep_y else None
            C = plan.forward(P, K_chi, K_chi2, n_g, n_s, precision=precision, w_save=w, coef=coef, y_save=y)
            ctx.plan, ctx.args = plan, (n_g, n_s, precision, coef)
            ctx.save_for_backward(P, K_chi, K_chi2, w, y)
            return C if P.dim() == 4 else C[0]

        @staticmethod
        def backward(ctx, gC):
            P, K_chi, K_chi2, w, y = ctx.saved_tensors
            n_g, n_s, precision, coef = ctx.args
            squeeze = P.dim() == 3
            g = gC.unsqueeze(0) if squeeze else gC
            want = tuple(nm for nm, need in zip(("P", "K_chi", "K_chi2"), ctx.needs_input_grad[1:4]) if need)
            dP, dK, dK2 = ctx.plan.backward(P, K_chi, K_chi2, n_g, n_s, g.contiguous().double(), precision=precision,
                                            w_save=w, coef=coef, want=want, y_save=y)
            if squeeze:
                dP = dP[0] if dP is not None else None
                dK = dK[0] if dK is not None else None
                dK2 = dK2[0] if dK2 is not None else None
            return None, dP, dK, dK2, None, None, None, None

    return ClFunction


_CLF = None


def cl_function():
    """The torch.autograd.Function wrapping forward and adjoint."""
    global _CLF
    if _CLF is None:
        _CLF = _make_cl_function()
    return _CLF


class Server:
    """Continuous-batching server over one plan (blast_server_*).  Request inputs are host
    arrays (numpy, or pinned torch CPU tensors for asynchronous copies) that must stay alive
    until the request completes; the wrapper keeps references until `wait` returns."""

    def __init__(self, plan, *, precision="fp32", p_dtype="fp32", batch=16, n_sets=0, max_g=15, max_s=5,
                 hbm_budget=0, max_queue=0, max_wait_ms=2.0, use_graphs=True):
        self.plan = plan
        self.p_dtype = p_dtype
        self.max_g, self.max_s = max_g, max_s
        d = ServerDesc(PRECISION.get(precision, precision), 0 if p_dtype == "fp64" else 1, batch, n_sets, max_g,
                       max_s, int(hbm_budget), max_queue, float(max_wait_ms), 1 if use_graphs else 0)
        h = C.c_void_p()
        _check(lib().blast_server_create(plan.handle, C.byref(d), C.byref(h)))
        self._h = h
        self._live = {}

    @staticmethod
    def _ptr(x):
        if hasattr(x, "data_ptr"):
            return x.data_ptr()
        return x.ctypes.data

    @staticmethod
    def _host_f64(x, shape, name):
        """A kernel table the server reads as host memory until completion: a float64,
        C-contiguous host array (numpy, or a torch CPU tensor, e.g. pinned) of exactly `shape`."""
        if hasattr(x, "data_ptr"):
            import torch
            ok = x.dtype == torch.float64 and x.is_contiguous() and not x.is_cuda
        else:
            x = np.ascontiguousarray(x, dtype=np.float64)
            ok = True
        if not ok or tuple(x.shape) != tuple(shape):
            raise ValueError("%s must be a contiguous float64 host array of shape %s" % (name, tuple(shape)))
        return x

    def submit(self, P, K_chi, K_chi2, n_g, n_s, ell_idx, out=None):
        plan = self.plan
        want = np.float64 if self.p_dtype == "fp64" else np.float32
        if hasattr(P, "data_ptr"):
            import torch
            ok = P.dtype == (torch.float64 if want is np.float64 else torch.float32) and P.is_contiguous() \
                and not P.is_cuda
        else:
            ok = P.dtype == want and P.flags.c_contiguous
        if not ok or tuple(P.shape) != (len(plan.chi), len(plan.R), plan.n_cheb):
            raise ValueError("P must be a contiguous host array [n_chi, n_R, n_cheb] of the server's dtype")
        nb = n_g + n_s
        K_chi = self._host_f64(K_chi, (nb, len(plan.chi)), "K_chi")
        K_chi2 = self._host_f64(K_chi2, (nb, len(plan.chi), len(plan.R)), "K_chi2")
        idx = np.ascontiguousarray(ell_idx, dtype=np.int32)
        shape = (n_pairs(n_g, n_s, plan.types), len(idx))
        if out is None:
            out = np.empty(shape)
        elif not (isinstance(out, np.ndarray) and out.dtype == np.float64 and out.flags.c_contiguous
                  and out.flags.writeable and tuple(out.shape) == shape):
            raise ValueError("out must be a writeable C-contiguous float64 numpy array of shape %s" % (shape,))
        r = Request(self._ptr(P), n_g, n_s, self._ptr(K_chi), self._ptr(K_chi2), len(idx),
                    idx.ctypes.data_as(C.POINTER(C.c_int32)), out.ctypes.data)
        t = C.c_uint64()
        _check(lib().blast_server_submit(self._h, C.byref(r), C.byref(t)))
        self._live[t.value] = (P, K_chi, K_chi2, idx, out)
        return t.value

    def wait(self, ticket, timeout_ms=-1):
        """(C [pairs, ell], latency in ms) of a ticket; raises BlastError with the request's status
        if it failed or was cancelled."""
        st, lat = C.c_int(), C.c_double()
        _check(lib().blast_server_wait(self._h, ticket, timeout_ms, C.byref(st), C.byref(lat)))
        keep = self._live.pop(ticket)
        if st.value != OK:
            raise BlastError(st.value, "request %d did not complete" % ticket)
        return keep[4], lat.value

    def poll(self, ticket):
        """None while the ticket is pending, else what wait() returns (or raises)."""
        done, st, lat = C.c_int32(), C.c_int(), C.c_double()
        _check(lib().blast_server_poll(self._h, ticket, C.byref(done), C.byref(st), C.byref(lat)))
        if not done.value:
            return None
        keep = self._live.pop(ticket)
        if st.value != OK:
            raise BlastError(st.value, "request %d did not complete" % ticket)
        return keep[4], lat.value

    def cancel(self, ticket):
        """Cancel a request that has not started (blast_server_cancel); wait() then raises
        BlastError with status E_CANCELLED."""
        _check(lib().blast_server_cancel(self._h, ticket))

    def footprint(self, n_g, n_s, count=1):
        """(arena bytes of a launch of `count` requests whose largest bins are (n_g, n_s), bytes of
        one set's arena)."""
        b, sb = C.c_size_t(), C.c_size_t()
        _check(lib().blast_server_footprint(self._h, n_g, n_s, count, C.byref(b), C.byref(sb)))
        return b.value, sb.value

    def stats(self):
        s = ServerStats()
        _check(lib().blast_server_stats_get(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().blast_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_for_config(cfg, precisions=("fp64",), device=0, ell=None, **kw):
    """Plan with the default grids of a workloads.Config (Simpson chi, Fejer R, Chebyshev k);
    `ell` replaces the configuration's multipole list (for instance by non-integer values)."""
    chi, wchi = grid_chi_simpson(cfg.n_chi, cfg.chi_min, cfg.chi_max)
    R, wR = grid_R_fejer(cfg.n_R, cfg.R_min)
    return Plan(cfg.ells() if ell is None else ell, chi, wchi, R, wR, cfg.k_min, cfg.k_max, cfg.n_cheb, precisions=precisions,
                device=device, **kw)
