"""Python binding of libmapmaker.so (the C ABI in include/mapmaker.h).

Argument marshalling only: every operation runs in the library's HIP kernels.
Device arrays are torch tensors on the context's GPU (torch provides memory and
streams); they are passed to the library as raw pointers.

The library must have been built (``python -m paper_1801_08937_amd.build``);
importing this module without it raises ImportError -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmapmaker.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "mapmaker.h")

MM_OK, MM_NOT_CONVERGED = 0, 1
STATUS = {0: "MM_OK", 1: "MM_NOT_CONVERGED", -1: "MM_E_INVALID", -2: "MM_E_OOM",
          -3: "MM_E_DEVICE", -4: "MM_E_SINGULAR_BLOCK", -5: "MM_E_COARSE_NOT_SPD",
          -6: "MM_E_BREAKDOWN", -7: "MM_E_NONFINITE", -8: "MM_E_BUSY"}
F64, F32 = 0, 1
NOISE_AUTO, NOISE_DIRECT, NOISE_FFT, NOISE_POLY = 0, 1, 2, 3
STOKES = {"IQU": 0, "I": 1, "QU": 2}


class MapmakerError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("breakdown", C.c_int32),
                ("pad", C.c_int32), ("rel_res_recursive", C.c_double),
                ("rel_res_true", C.c_double), ("solve_seconds", C.c_double),
                ("rel_res_precond", C.c_double)]


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("iters", C.c_int32), ("slot", C.c_int32),
                ("m2l_built", C.c_int32), ("precond", C.c_int32), ("waited", C.c_int32),
                ("rel_res", C.c_double),
                ("queue_seconds", C.c_double), ("latency_seconds", C.c_double)]


class RefineInfo(C.Structure):
    _fields_ = [("outer", C.c_int32), ("inner_iters", C.c_int32), ("converged", C.c_int32),
                ("pad", C.c_int32), ("rel_res_true", C.c_double), ("solve_seconds", C.c_double)]


class ArnoldiInfo(C.Structure):
    _fields_ = [("m", C.c_int32), ("k", C.c_int32), ("h_last", C.c_double),
                ("setup_seconds", C.c_double)]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1801_08937_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D, U32 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint32
        PP = C.POINTER(C.c_void_p)
        sig = {
            "mm_version": (C.c_char_p, []),
            "mm_ctx_create": (C.c_int, [C.c_int, P, PP]),
            "mm_ctx_destroy": (None, [P]),
            "mm_last_error": (C.c_char_p, [P]),
            "mm_pointing_build": (C.c_int, [P, I64, I32, P, P, I32, C.c_int, PP]),
            "mm_pointing_build_stokes": (C.c_int, [P, I64, I32, P, P, I32, C.c_int, C.c_int, PP]),
            "mm_pointing_stokes": (C.c_int, [P, C.POINTER(C.c_int), C.POINTER(C.c_int32)]),
            "mm_pair_sum_diff": (C.c_int, [P, I64, C.c_int, P, P, P, P]),
            "mm_pointing_counts": (C.c_int, [P, C.POINTER(I32), C.POINTER(I64)]),
            "mm_pointing_pt_layout": (C.c_int, [P, C.POINTER(I32), C.POINTER(I32)]),
            "mm_pointing_p_layout": (C.c_int, [P, C.POINTER(I32)]),
            "mm_pointing_set_grid": (C.c_int, [P, P, I32]),
            "mm_pointing_hits": (C.c_int, [P, P, P, P]),
            "mm_pointing_export": (C.c_int, [P, P, P, P, P]),
            "mm_pointing_destroy": (None, [P]),
            "mm_noise_build": (C.c_int, [P, I32, P, P, I32, I32, P, C.c_int, C.c_int, PP]),
            "mm_noise_method_used": (C.c_int, [P, C.POINTER(C.c_int)]),
            "mm_polyfilter_build": (C.c_int, [P, P, I32, P, P, I64, P, I32, P, I32, PP]),
            "mm_noise_fft_block": (C.c_int, [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
            "mm_noise_apply": (C.c_int, [P, P, I32, P, P]),
            "mm_noise_destroy": (None, [P]),
            "mm_apply_P": (C.c_int, [P, P, I32, P, P]),
            "mm_apply_PT": (C.c_int, [P, P, I32, P, P]),
            "mm_apply_A": (C.c_int, [P, P, P, I32, P, P]),
            "mm_rhs": (C.c_int, [P, P, P, I32, P, P]),
            "mm_mbd_build": (C.c_int, [P, P, P, PP]),
            "mm_mbd_rcond": (C.c_int, [P, C.POINTER(D)]),
            "mm_defl_build": (C.c_int, [P, P, P, P, P, I32, D, D, I32, P, P, PP]),
            "mm_defl_build_stop": (C.c_int, [P, P, P, P, P, I32, D, D, I32, I32, P, P, P, PP]),
            "mm_defl_build_pcg": (C.c_int, [P, P, P, P, P, I32, D, D, I32, P, P, P, PP]),
            "mm_defl_from_Z": (C.c_int, [P, P, P, P, I32, P, PP]),
            "mm_defl_transfer": (C.c_int, [P, P, P, P, P, P, PP]),
            "mm_noise_set_fft_block": (C.c_int, [P, P, I32]),
            "mm_solve_refined": (C.c_int, [P, P, P, P, P, P, I32, P, P, D, D, I32, I32,
                                           C.POINTER(RefineInfo)]),
            "mm_dense_gram": (C.c_int, [P, I64, I32, I32, P, I64, I64, P, I64, I64, P]),
            "mm_dense_tall": (C.c_int, [P, I64, I32, I32, P, P, P]),
            "mm_dense_rows": (C.c_int, [P, I64, I32, P, P, D, D, P]),
            "mm_apply_A_noalloc": (C.c_int, [P, P, P, I32, P, P, C.POINTER(C.c_size_t)]),
            "mm_apply_A_noalloc_max_bytes": (C.c_size_t, []),
            "mm_defl_export": (C.c_int, [P, P, C.POINTER(I32), P, P, P]),
            "mm_defl_arnoldi_export": (C.c_int, [P, P, C.POINTER(I32), P, P]),
            "mm_precond_apply": (C.c_int, [P, P, I32, P, P]),
            "mm_precond_destroy": (None, [P]),
            "mm_solve": (C.c_int, [P, P, P, P, I32, P, P, D, I32, U32, P, P]),
            "mm_profile_enable": (C.c_int, [P, C.c_int]),
            "mm_autotune": (C.c_int, [P, P, P, I32, I32, P, I32, C.POINTER(I32)]),
            "mm_server_create": (C.c_int, [C.c_int, I64, I32, I32, I32, PP]),
            "mm_server_set_prebuild": (C.c_int, [P, I32]),
            "mm_server_set_arnoldi": (C.c_int, [P, I32, D, I32]),
            "mm_server_add_strategy": (C.c_int, [P, I32, I64, I32, P, P, I32, I32, I32, P, P, I32,
                                                 I32, P, C.c_int]),
            "mm_server_submit": (C.c_int, [P, I32, P, D, I32, P, C.POINTER(I64)]),
            "mm_server_step": (C.c_int, [P, C.POINTER(I32), C.POINTER(I32)]),
            "mm_server_poll": (C.c_int, [P, I64, C.POINTER(RequestInfo)]),
            "mm_server_strategy_state": (C.c_int, [P, I32, C.POINTER(I32)]),
            "mm_server_last_error": (C.c_char_p, [P]),
            "mm_server_memory": (C.c_int, [P, I32] + [C.POINTER(I64)] * 4),
            "mm_server_destroy": (None, [P]),
            "mm_profile_read": (C.c_int, [P, I32, P, P, P, C.POINTER(I32)]),
            "mm_hessenberg_eig": (C.c_int, [I32, P, P, P, P, P]),
            "mm_pcg_create": (C.c_int, [P, P, P, P, I32, PP]),
            "mm_pcg_start": (C.c_int, [P, P, I32, P, D, I32]),
            "mm_pcg_iterate": (C.c_int, [P, P, I32]),
            "mm_pcg_use_graph": (C.c_int, [P, P, I32]),
            "mm_pcg_poll": (C.c_int, [P, P, P, P, P]),
            "mm_pcg_finish": (C.c_int, [P, P, I32, P]),
            "mm_pcg_destroy": (None, [P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_symbols() -> list[str]:
    """Names of the functions include/mapmaker.h declares."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[A-Za-z0-9_]+)\s*\(", src)) - {"mm_status"})


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _dev_check(t, dtype=None, numel=None, name="array"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a GPU torch tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")


def hessenberg_eig(H: np.ndarray):
    """Host-only Ritz eigensolver of the library (no GPU needed)."""
    H = np.asarray(H, dtype=np.float64)
    m = H.shape[0]
    Hc = np.asfortranarray(H)
    wr, wi = np.zeros(m), np.zeros(m)
    vr, vi = np.zeros((m, m), order="F"), np.zeros((m, m), order="F")
    st = lib().mm_hessenberg_eig(m, Hc.ctypes.data, wr.ctypes.data, wi.ctypes.data,
                                 vr.ctypes.data, vi.ctypes.data)
    if st != 0:
        raise MapmakerError(st, "hessenberg_eig failed")
    return wr + 1j * wi, vr + 1j * vi


class Context:
    """A library context on one GPU, enqueuing on a torch stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        self.torch_device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.torch_device)
        self.stream = stream
        h = C.c_void_p()
        st = lib().mm_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != 0:
            raise MapmakerError(st, "mm_ctx_create failed")
        self.h = h

    def _check(self, st, what):
        if st < 0 or (st > 1):
            msg = lib().mm_last_error(self.h)
            raise MapmakerError(st, f"{what}: {msg.decode() if msg else ''}")
        return st

    def close(self):
        if getattr(self, "h", None):
            lib().mm_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def synchronize(self):
        self.stream.synchronize()

    # ------------------------------------------------------------- builders
    def pointing(self, pix, psi, n_pix_total: int, min_hits: int = 3, prec: int = F64,
                 stokes: str = "IQU"):
        """P from per-sample pixels and angles; stokes "IQU", "I" (pair-sum
        stream, psi may be None) or "QU" (pair-difference stream)."""
        import torch
        _dev_check(pix, torch.int32, name="pix")
        if stokes not in STOKES:
            raise ValueError("stokes must be IQU, I or QU")
        if psi is not None:
            _dev_check(psi, torch.float64, pix.numel(), name="psi")
        h = C.c_void_p()
        self._check(lib().mm_pointing_build_stokes(self.h, pix.numel(), n_pix_total, _ptr(pix),
                                                   None if psi is None else _ptr(psi), min_hits,
                                                   prec, STOKES[stokes], C.byref(h)),
                    "mm_pointing_build_stokes")
        return Pointing(self, h, pix.numel(), n_pix_total, prec)

    def pair_sum_diff(self, a, b, plus=None, minus=None):
        """Sum and difference streams of a detector pair (Eqs. d+, d-):
        ((a + b) / 2, (a - b) / 2), on the device."""
        import torch
        if a.dtype not in (torch.float64, torch.float32):
            raise ValueError("a must be float64 or float32")
        _dev_check(a, a.dtype, name="a")
        _dev_check(b, a.dtype, a.numel(), name="b")
        plus = torch.empty_like(a) if plus is None else plus
        minus = torch.empty_like(a) if minus is None else minus
        _dev_check(plus, a.dtype, a.numel(), name="plus")
        _dev_check(minus, a.dtype, a.numel(), name="minus")
        prec = F32 if a.dtype == torch.float32 else F64
        self._check(lib().mm_pair_sum_diff(self.h, a.numel(), prec, _ptr(a), _ptr(b), _ptr(plus),
                                           _ptr(minus)), "mm_pair_sum_diff")
        return plus, minus

    def noise(self, interval_start, filter_id, band, half_bw: int, method: int = NOISE_AUTO,
              prec: int = F64):
        istart = np.ascontiguousarray(interval_start, dtype=np.int64)
        fid = np.ascontiguousarray(filter_id, dtype=np.int32)
        band = np.ascontiguousarray(band, dtype=np.float64).reshape(-1, half_bw + 1)
        h = C.c_void_p()
        self._check(lib().mm_noise_build(self.h, fid.shape[0], istart.ctypes.data,
                                         fid.ctypes.data, band.shape[0], half_bw,
                                         band.ctypes.data, method, prec, C.byref(h)),
                    "mm_noise_build")
        return Noise(self, h, int(istart[-1]), half_bw, prec)

    def polyfilter(self, p, interval_start, weight, subscan_start, order: int,
                   ground_bin=None, n_ground_bins: int = 0):
        """Template filter as the weight: F = W - W B (B^T W B)^-1 B^T W
        (piecewise Legendre polynomials of degree <= order per subscan), or
        with ground templates (ground_bin: int32 device tensor, one azimuth
        bin per sample, -1 = none) F = F_B W^+ F_G W^+ F_B."""
        import torch
        istart = np.ascontiguousarray(interval_start, dtype=np.int64)
        w = np.ascontiguousarray(weight, dtype=np.float64)
        sub = np.ascontiguousarray(subscan_start, dtype=np.int64)
        gb = None
        if ground_bin is not None:
            _dev_check(ground_bin, torch.int32, p.n_samp, "ground_bin")
            gb = _ptr(ground_bin)
        h = C.c_void_p()
        self._check(lib().mm_polyfilter_build(self.h, p.h, istart.shape[0] - 1, istart.ctypes.data,
                                              w.ctypes.data, sub.shape[0] - 1, sub.ctypes.data,
                                              order, gb, int(n_ground_bins), C.byref(h)),
                    "mm_polyfilter_build")
        return Noise(self, h, p.n_samp, 0, p.prec)

    # ------------------------------------------------------------ operators
    def _tod_dtype(self, prec):
        import torch
        return torch.float32 if prec == F32 else torch.float64

    def apply_P(self, p: "Pointing", x, y=None, nrhs: int = 1):
        import torch
        _dev_check(x, torch.float64, p.n * nrhs, "x")
        if y is None:
            y = torch.empty(p.n_samp * nrhs, dtype=self._tod_dtype(p.prec), device=x.device)
        self._check(lib().mm_apply_P(self.h, p.h, nrhs, _ptr(x), _ptr(y)), "mm_apply_P")
        return y

    def apply_PT(self, p: "Pointing", z, x=None, nrhs: int = 1):
        import torch
        _dev_check(z, self._tod_dtype(p.prec), p.n_samp * nrhs, "z")
        if x is None:
            x = torch.empty(p.n * nrhs, dtype=torch.float64, device=z.device)
        self._check(lib().mm_apply_PT(self.h, p.h, nrhs, _ptr(z), _ptr(x)), "mm_apply_PT")
        return x

    def noise_apply(self, nz: "Noise", y, z=None, nrhs: int = 1):
        import torch
        _dev_check(y, self._tod_dtype(nz.prec), nz.n_samp * nrhs, "y")
        if z is None:
            z = torch.empty_like(y)
        self._check(lib().mm_noise_apply(self.h, nz.h, nrhs, _ptr(y), _ptr(z)), "mm_noise_apply")
        return z

    def apply_A(self, p, nz, x, y=None, nrhs: int = 1):
        import torch
        _dev_check(x, torch.float64, p.n * nrhs, "x")
        if y is None:
            y = torch.empty_like(x)
        self._check(lib().mm_apply_A(self.h, p.h, nz.h, nrhs, _ptr(x), _ptr(y)), "mm_apply_A")
        return y

    def apply_A_noalloc(self, p, nz, x, y, nrhs: int = 1) -> int:
        """y = A x with no device allocation (the library's static scratch);
        y must be given.  Returns the scratch bytes the call needed."""
        import torch
        _dev_check(x, torch.float64, p.n * nrhs, "x")
        _dev_check(y, torch.float64, p.n * nrhs, "y")
        used = C.c_size_t(0)
        self._check(lib().mm_apply_A_noalloc(self.h, p.h, nz.h, nrhs, _ptr(x), _ptr(y),
                                             C.byref(used)), "mm_apply_A_noalloc")
        return used.value

    def rhs(self, p, nz, tod, b=None, nrhs: int = 1):
        import torch
        _dev_check(tod, self._tod_dtype(p.prec), p.n_samp * nrhs, "tod")
        if b is None:
            b = torch.empty(p.n * nrhs, dtype=torch.float64, device=tod.device)
        self._check(lib().mm_rhs(self.h, p.h, nz.h, nrhs, _ptr(tod), _ptr(b)), "mm_rhs")
        return b

    # ------------------------------------------------------ preconditioners
    def mbd(self, p, nz):
        h = C.c_void_p()
        self._check(lib().mm_mbd_build(self.h, p.h, nz.h, C.byref(h)), "mm_mbd_build")
        return Precond(self, h, p.n, 0)

    def defl_from_Z(self, p, nz, mbd, Z):
        import torch
        k = Z.shape[1] if Z.dim() == 2 else 1
        Zc = Z.t().contiguous() if Z.dim() == 2 else Z.contiguous()
        _dev_check(Zc, torch.float64, p.n * k, "Z")
        h = C.c_void_p()
        self._check(lib().mm_defl_from_Z(self.h, p.h, nz.h, mbd.h, k, _ptr(Zc), C.byref(h)),
                    "mm_defl_from_Z")
        return Precond(self, h, p.n, 1)

    def defl_transfer(self, p_src, src, p, nz, mbd):
        """M_2l on (p, nz) from the deflation vectors of src, an M_2l built on
        another subset (p_src): rows matched by global pixel id, A Z and E
        rebuilt here (the "simplified" two-level preconditioner)."""
        h = C.c_void_p()
        self._check(lib().mm_defl_transfer(self.h, p_src.h, src.h, p.h, nz.h, mbd.h, C.byref(h)),
                    "mm_defl_transfer")
        return Precond(self, h, p.n, 1)

    def defl_build(self, p, nz, mbd, b_seed, k: int = 32, eps_arn: float = 1e-8,
                   m_max: int = 256, eps_lambda: float = 0.0, stop: str = "h"):
        """M_2l by Arnoldi from r_0 = M_BD b_seed.  stop: "h" (h_{j+1,j} <=
        eps_arn) or "residual" (the Arnoldi solution's relative residual <=
        eps_arn).  The handle carries .h_history and .res_history per step."""
        import torch
        _dev_check(b_seed, torch.float64, p.n, "b_seed")
        rule = {"h": 0, "residual": 1}.get(stop)
        if rule is None:
            raise ValueError("stop is 'h' or 'residual'")
        hist = np.zeros(m_max)
        res = np.zeros(m_max)
        info = ArnoldiInfo()
        h = C.c_void_p()
        self._check(lib().mm_defl_build_stop(self.h, p.h, nz.h, mbd.h, _ptr(b_seed), k,
                                             eps_lambda, eps_arn, rule, m_max,
                                             hist.ctypes.data, res.ctypes.data, C.byref(info),
                                             C.byref(h)), "mm_defl_build_stop")
        M = Precond(self, h, p.n, 1)
        M.arnoldi_info = info
        M.h_history = hist[: info.m].copy()
        M.res_history = res[: info.m].copy()
        return M

    def defl_build_pcg(self, p, nz, mbd, b, k: int = 32, m_max: int = 256, tol: float = 0.0,
                       eps_lambda: float = 0.0, x_out=None):
        """M_2l from the Ritz vectors of a prior M_BD PCG run on A x = b (at
        most m_max iterations, stopped at ||r||/||b|| <= tol; Lanczos
        tridiagonal from the CG coefficients).  The returned handle carries
        .theta (Ritz values) and .arnoldi_info."""
        import torch
        _dev_check(b, torch.float64, p.n, "b")
        theta = np.zeros(m_max)
        info = ArnoldiInfo()
        h = C.c_void_p()
        if x_out is not None:
            _dev_check(x_out, torch.float64, p.n, "x_out")
        self._check(lib().mm_defl_build_pcg(self.h, p.h, nz.h, mbd.h, _ptr(b), k, eps_lambda,
                                            tol, m_max, theta.ctypes.data,
                                            None if x_out is None else _ptr(x_out), C.byref(info),
                                            C.byref(h)), "mm_defl_build_pcg")
        M = Precond(self, h, p.n, 1)
        M.arnoldi_info = info
        M.theta = theta[: info.m].copy()
        return M

    def precond_apply(self, M, v, out=None, nrhs: int = 1):
        import torch
        _dev_check(v, torch.float64, M.n * nrhs, "v")
        if out is None:
            out = torch.empty_like(v)
        self._check(lib().mm_precond_apply(self.h, M.h, nrhs, _ptr(v), _ptr(out)),
                    "mm_precond_apply")
        return out

    # ---------------------------------------------------------------- solve
    def solve(self, p, nz, M, b, x=None, tol: float = 1e-8, max_iter: int = 2000,
              nrhs: int = 1, check_every: int = 1, history: bool = True, graph: bool = False,
              block: bool = False, flexible: bool = False):
        """PCG (Eq. pcg).  block: O'Leary's block PCG over the columns;
        flexible: Polak-Ribiere beta (for the non-symmetric M_2l).  The info
        dict carries the plain residual ||b - Ax||/||b|| and the literal
        preconditioned one ||M (b - Ax)||/||M b||."""
        import torch
        _dev_check(b, torch.float64, p.n * nrhs, "b")
        if x is None:
            x = torch.zeros_like(b)
        hist = np.zeros((nrhs, max_iter + 1)) if history else None
        infos = (SolveInfo * nrhs)()
        st = lib().mm_solve(self.h, p.h, nz.h, M.h if M is not None else None, nrhs, _ptr(b),
                            _ptr(x), tol, max_iter,
                            (check_every & 0xFF) | (256 if graph else 0) | (512 if block else 0)
                            | (1024 if flexible else 0),
                            hist.ctypes.data if hist is not None else None, infos)
        self._check(st, "mm_solve")
        out = []
        for c in range(nrhs):
            i = infos[c]
            h = hist[c, : i.iters + 1].copy() if hist is not None else None
            out.append(dict(iters=i.iters, converged=bool(i.converged),
                            breakdown=bool(i.breakdown), rel_res_recursive=i.rel_res_recursive,
                            rel_res_true=i.rel_res_true, solve_seconds=i.solve_seconds,
                            rel_res_precond=i.rel_res_precond, history=h, status=st))
        return x, (out[0] if nrhs == 1 else out)

    def autotune(self, p, nz, nrhs: int = 1, fft_block: bool = False):
        """Per-stage autotuner; returns [(stage, candidate, ms)].  fft_block:
        also tune the FFT block length (changes results at rounding level)."""
        rep = np.zeros(3 * 32)
        n = C.c_int32()
        self._check(lib().mm_autotune(self.h, p.h, nz.h, nrhs, 1 if fft_block else 0,
                                      rep.ctypes.data, 32, C.byref(n)), "mm_autotune")
        if fft_block:
            nz._read_block()
        names = {0: "P", 1: "band_chunk", 2: "PT_order", 3: "fft_block"}
        return [(names[int(rep[3 * i])], int(rep[3 * i + 1]), float(rep[3 * i + 2]))
                for i in range(n.value)]

    def solve_refined(self, p_lo, nz_lo, p_hi, nz_hi, M, b, x=None, tol: float = 1e-8,
                      inner_tol: float = 1e-5, max_outer: int = 20, max_inner: int = 2000,
                      nrhs: int = 1):
        """Iterative refinement: FP64 residual (p_hi, nz_hi), corrections by PCG
        with (p_lo, nz_lo).  Returns (x, info dict)."""
        import torch
        _dev_check(b, torch.float64, p_hi.n * nrhs, "b")
        if x is None:
            x = torch.zeros_like(b)
        info = RefineInfo()
        st = lib().mm_solve_refined(self.h, p_lo.h, nz_lo.h, p_hi.h, nz_hi.h,
                                    M.h if M is not None else None, nrhs, _ptr(b), _ptr(x), tol,
                                    inner_tol, max_outer, max_inner, C.byref(info))
        self._check(st, "mm_solve_refined")
        return x, {f: getattr(info, f) for f, _ in RefineInfo._fields_ if f != "pad"}

    # ---------------------------------------------- small dense products
    def dense_gram(self, X, Y):
        """C = X^T Y for X (n, ka), Y (n, kb) torch float64 tensors (any
        strides), ka, kb <= 64."""
        import torch
        n, ka = X.shape
        kb = Y.shape[1]
        C_ = torch.empty(ka, kb, dtype=torch.float64, device=X.device)
        self._check(lib().mm_dense_gram(self.h, n, ka, kb, _ptr(X), X.stride(0), X.stride(1),
                                        _ptr(Y), Y.stride(0), Y.stride(1), _ptr(C_)),
                    "mm_dense_gram")
        return C_

    def dense_tall(self, V, Y):
        """Z = V Y for V (n, kin) and Y (kin, kout), column-major storage
        (V.t() and Y.t() contiguous); returns Z (n, kout) as a transposed view."""
        import torch
        n, kin = V.shape
        kout = Y.shape[1]
        Vc, Yc = V.t().contiguous(), Y.t().contiguous()
        Z = torch.empty(kout, n, dtype=torch.float64, device=V.device)
        self._check(lib().mm_dense_tall(self.h, n, kin, kout, _ptr(Vc), _ptr(Yc), _ptr(Z)),
                    "mm_dense_tall")
        return Z.t()

    def dense_rows(self, In, S, out=None, alpha: float = 1.0, beta: float = 0.0):
        """Out = beta Out + alpha In S for In (n, R) row-major, S (R, R)."""
        import torch
        n, R = In.shape
        Inc, Sc = In.contiguous(), S.contiguous()
        if out is None:
            out = torch.empty_like(Inc)
        self._check(lib().mm_dense_rows(self.h, n, R, _ptr(Inc), _ptr(Sc), alpha, beta, _ptr(out)),
                    "mm_dense_rows")
        return out

    def pcg_session(self, p, nz, M, nrhs: int):
        h = C.c_void_p()
        self._check(lib().mm_pcg_create(self.h, p.h, nz.h, M.h if M is not None else None, nrhs,
                                        C.byref(h)), "mm_pcg_create")
        return PcgSession(self, h, p.n, nrhs)

    # ------------------------------------------------------------ profiling
    def profile(self, on: bool):
        self._check(lib().mm_profile_enable(self.h, 1 if on else 0), "mm_profile_enable")

    def profile_read(self):
        mx = 64
        names = C.create_string_buffer(32 * mx)
        ms = np.zeros(mx)
        calls = np.zeros(mx, dtype=np.int64)
        n = C.c_int32()
        self._check(lib().mm_profile_read(self.h, mx, names, ms.ctypes.data, calls.ctypes.data,
                                          C.byref(n)), "mm_profile_read")
        res = {}
        for i in range(min(n.value, mx)):
            nm = names.raw[32 * i: 32 * i + 32].split(b"\0")[0].decode()
            res[nm] = (float(ms[i]), int(calls[i]))
        return res


class _Handle:
    _destroy = ""

    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h

    def close(self):
        if getattr(self, "h", None):
            getattr(lib(), self._destroy)(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pointing(_Handle):
    _destroy = "mm_pointing_destroy"

    def __init__(self, ctx, h, n_samp, n_pix_total, prec):
        super().__init__(ctx, h)
        self.n_samp, self.n_pix_total, self.prec = n_samp, n_pix_total, prec
        n_obs, n_valid = C.c_int32(), C.c_int64()
        lib().mm_pointing_counts(h, C.byref(n_obs), C.byref(n_valid))
        self.n_obs, self.n_valid = n_obs.value, n_valid.value
        st, nc = C.c_int(), C.c_int32()
        lib().mm_pointing_stokes(h, C.byref(st), C.byref(nc))
        self.stokes = {v: k for k, v in STOKES.items()}[st.value]
        self.nc = nc.value
        self.n = self.nc * self.n_obs

    def set_grid(self, width: int):
        """Locality hint: global ids are row-major with `width` columns."""
        self.ctx._check(lib().mm_pointing_set_grid(self.ctx.h, self.h, width),
                        "mm_pointing_set_grid")

    def p_copies(self) -> int:
        """Map copies the single-column IQU P gathers from (0 = no grid)."""
        g = C.c_int32(0)
        lib().mm_pointing_p_layout(self.h, C.byref(g))
        return g.value

    def pt_layout(self):
        """(slices, segments) of the sliced single-column P^T; (0, 0) when the
        one-wave-per-pixel form is used."""
        g, s = C.c_int32(0), C.c_int32(0)
        lib().mm_pointing_pt_layout(self.h, C.byref(g), C.byref(s))
        return g.value, s.value

    def hits(self):
        import torch
        dev = self.ctx.torch_device
        hits = torch.empty(self.n_pix_total, dtype=torch.int32, device=dev)
        obs = torch.empty(max(self.n_obs, 1), dtype=torch.int32, device=dev)
        self.ctx._check(lib().mm_pointing_hits(self.ctx.h, self.h, _ptr(hits), _ptr(obs)),
                        "mm_pointing_hits")
        return hits, obs[: self.n_obs]

    def export(self):
        import torch
        dev = self.ctx.torch_device
        j = torch.empty(self.n_samp, dtype=torch.int32, device=dev)
        perm = torch.empty(max(self.n_valid, 1), dtype=torch.int32, device=dev)
        off = torch.empty(self.n_obs + 1, dtype=torch.int32, device=dev)
        self.ctx._check(lib().mm_pointing_export(self.ctx.h, self.h, _ptr(j), _ptr(perm),
                                                 _ptr(off)), "mm_pointing_export")
        return j, perm[: self.n_valid], off


class Noise(_Handle):
    _destroy = "mm_noise_destroy"

    def __init__(self, ctx, h, n_samp, half_bw, prec):
        super().__init__(ctx, h)
        self.n_samp, self.half_bw, self.prec = n_samp, half_bw, prec
        m = C.c_int()
        lib().mm_noise_method_used(h, C.byref(m))
        self.method = m.value
        self._read_block()

    def _read_block(self):
        nf, nv = C.c_int32(0), C.c_int32(0)
        lib().mm_noise_fft_block(self.h, C.byref(nf), C.byref(nv))
        self.fft_n, self.fft_valid = nf.value, nv.value

    def set_fft_block(self, n_fft: int):
        """Overlap-save block length of the FFT method (16384, 32768, 0 = model)."""
        self.ctx._check(lib().mm_noise_set_fft_block(self.ctx.h, self.h, n_fft),
                        "mm_noise_set_fft_block")
        self._read_block()


class Precond(_Handle):
    _destroy = "mm_precond_destroy"

    def __init__(self, ctx, h, n, kind):
        super().__init__(ctx, h)
        self.n, self.kind = n, kind

    def rcond(self):
        r = C.c_double()
        lib().mm_mbd_rcond(self.h, C.byref(r))
        return r.value

    def export(self):
        import torch
        k = C.c_int32()
        self.ctx._check(lib().mm_defl_export(self.ctx.h, self.h, C.byref(k), None, None, None),
                        "mm_defl_export")
        k = k.value
        dev = self.ctx.torch_device
        Z = torch.empty(k, self.n, dtype=torch.float64, device=dev)
        AZ = torch.empty(k, self.n, dtype=torch.float64, device=dev)
        E = torch.empty(k, k, dtype=torch.float64, device=dev)
        self.ctx._check(lib().mm_defl_export(self.ctx.h, self.h, None, _ptr(Z), _ptr(AZ),
                                             _ptr(E)), "mm_defl_export")
        return Z.t(), AZ.t(), E

    def arnoldi(self):
        import torch
        m = C.c_int32()
        self.ctx._check(lib().mm_defl_arnoldi_export(self.ctx.h, self.h, C.byref(m), None, None),
                        "mm_defl_arnoldi_export")
        m = m.value
        W = torch.empty(m + 1, self.n, dtype=torch.float64, device=self.ctx.torch_device)
        H = np.zeros((m, m + 1))
        self.ctx._check(lib().mm_defl_arnoldi_export(self.ctx.h, self.h, None, _ptr(W),
                                                     H.ctypes.data), "mm_defl_arnoldi_export")
        return W.t(), H.T.copy()


class PcgSession(_Handle):
    """Step-wise lockstep PCG over nrhs column slots (continuous batching)."""
    _destroy = "mm_pcg_destroy"
    STATES = {0: "free", 1: "running", 2: "converged", 3: "budget", 4: "breakdown"}

    def __init__(self, ctx, h, n, nrhs):
        super().__init__(ctx, h)
        self.n, self.nrhs = n, nrhs

    def start(self, slot: int, b, tol: float, max_iter: int):
        import torch
        _dev_check(b, torch.float64, self.n, "b")
        self.ctx._check(lib().mm_pcg_start(self.ctx.h, self.h, slot, _ptr(b), tol, max_iter),
                        "mm_pcg_start")

    def use_graph(self, chunk: int):
        self.ctx._check(lib().mm_pcg_use_graph(self.ctx.h, self.h, chunk), "mm_pcg_use_graph")

    def iterate(self, n_iter: int):
        self.ctx._check(lib().mm_pcg_iterate(self.ctx.h, self.h, n_iter), "mm_pcg_iterate")

    def poll(self):
        st = np.zeros(self.nrhs, dtype=np.int32)
        it = np.zeros(self.nrhs, dtype=np.int32)
        rr = np.zeros(self.nrhs)
        self.ctx._check(lib().mm_pcg_poll(self.ctx.h, self.h, st.ctypes.data, it.ctypes.data,
                                          rr.ctypes.data), "mm_pcg_poll")
        return st, it, rr

    def finish(self, slot: int, x=None):
        import torch
        if x is None:
            x = torch.empty(self.n, dtype=torch.float64, device=self.ctx.torch_device)
        self.ctx._check(lib().mm_pcg_finish(self.ctx.h, self.h, slot, _ptr(x)), "mm_pcg_finish")
        return x


class Server:
    """Continuous-batching serving engine (mm_server_*): recurring strategies,
    cached M_BD/M_2l, per-strategy streams, column slots admitted mid-flight."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 200 << 30, slots: int = 8,
                 defl_k: int = 32, iters_per_step: int = 4, prebuild: bool = False,
                 arnoldi=None):
        """arnoldi: None (the library default) or (stop, eps_arn, m_max) for
        the background M_2l build, stop "h" or "residual"."""
        h = C.c_void_p()
        st = lib().mm_server_create(device, hbm_budget_bytes, slots, defl_k, iters_per_step,
                                    C.byref(h))
        if st != 0:
            raise MapmakerError(st, "mm_server_create failed")
        self.h = h
        if prebuild:
            lib().mm_server_set_prebuild(h, 1)
        if arnoldi is not None:
            stop, eps, m_max = arnoldi
            rule = {"h": 0, "residual": 1}[stop]
            st = lib().mm_server_set_arnoldi(h, rule, eps, m_max)
            if st != 0:
                lib().mm_server_destroy(h)
                self.h = None
                raise MapmakerError(st, "mm_server_set_arnoldi failed")
        self.device = device
        self.n = {}

    def _check(self, st, what):
        if st < 0:
            msg = lib().mm_server_last_error(self.h)
            raise MapmakerError(st, f"{what}: {msg.decode() if msg else ''}")
        return st

    def add_strategy(self, sid: int, pix, psi, n_pix_total: int, interval_start, filter_id, band,
                     half_bw: int, min_hits: int = 3, grid_width: int = 0, prec: int = F64):
        import torch
        _dev_check(pix, torch.int32, name="pix")
        _dev_check(psi, torch.float64, pix.numel(), name="psi")
        istart = np.ascontiguousarray(interval_start, dtype=np.int64)
        fid = np.ascontiguousarray(filter_id, dtype=np.int32)
        band = np.ascontiguousarray(band, dtype=np.float64).reshape(-1, half_bw + 1)
        self._check(lib().mm_server_add_strategy(
            self.h, sid, pix.numel(), n_pix_total, _ptr(pix), _ptr(psi), min_hits, grid_width,
            fid.shape[0], istart.ctypes.data, fid.ctypes.data, band.shape[0], half_bw,
            band.ctypes.data, prec), "mm_server_add_strategy")

    def submit(self, sid: int, tod, x_out, tol: float = 1e-8, max_iter: int = 1000) -> int:
        rid = C.c_int64()
        self._check(lib().mm_server_submit(self.h, sid, _ptr(tod), tol, max_iter, _ptr(x_out),
                                           C.byref(rid)), "mm_server_submit")
        return rid.value

    def step(self):
        nr, nq = C.c_int32(), C.c_int32()
        self._check(lib().mm_server_step(self.h, C.byref(nr), C.byref(nq)), "mm_server_step")
        return nr.value, nq.value

    def strategy_state(self, sid: int) -> int:
        """M_2l cache of a strategy: 0 not started, 1 building, 2 ready, 3 failed."""
        st = C.c_int32()
        self._check(lib().mm_server_strategy_state(self.h, sid, C.byref(st)),
                    "mm_server_strategy_state")
        return st.value

    def poll(self, rid: int) -> dict:
        info = RequestInfo()
        self._check(lib().mm_server_poll(self.h, rid, C.byref(info)), "mm_server_poll")
        return {f: getattr(info, f) for f, _ in RequestInfo._fields_}

    def memory(self, sid: int = -1) -> dict:
        """Budget, bytes in use, and (for a registered strategy sid) its
        resident bytes and the bytes of one lane session."""
        v = [C.c_int64() for _ in range(4)]
        self._check(lib().mm_server_memory(self.h, sid, C.byref(v[0]), C.byref(v[1]),
                                           C.byref(v[2]) if sid >= 0 else None,
                                           C.byref(v[3]) if sid >= 0 else None),
                    "mm_server_memory")
        out = {"budget": v[0].value, "used": v[1].value}
        if sid >= 0:
            out.update(resident=v[2].value, session=v[3].value)
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().mm_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
