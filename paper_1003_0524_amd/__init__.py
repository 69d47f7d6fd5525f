"""Python binding of the MI355X nonlocal-exchange library (``libexchange.so``).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI of ``include/exchange.h``. PyTorch provides device
memory and streams. There is no fallback: if the shared library is missing or
cannot be loaded, importing works but constructing :class:`Exchange` raises.

Typical use::

    ex = Exchange(n_bands, n_pw, ch_nrad, n_occ, E_list, D_list, C_list,
                  precision="bf16x6", form="herk", batched=True)
    V = ex.matrix_all([M_k0, M_k1, ...])      # list of n_b x n_b complex128 tensors
    e = ex.energy()
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

__all__ = ["Exchange", "ExchangeError", "load_library", "LIB_PATH", "PRECISIONS", "FORMS",
           "EXPORTED_SYMBOLS"]

# EXC_LIBRARY: another build of the same library (the host-sanitizer build of the ABI checks)
LIB_PATH = os.environ.get("EXC_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                         "libexchange.so")
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}
FORMS = {"gemm": 0, "herk": 1}
DTYPES = {"c128": 0, "c64": 1}
STATUS = {0: "EXC_OK", -1: "EXC_EINVAL", -2: "EXC_ENOMEM", -3: "EXC_ENOTPD", -4: "EXC_EHIP",
          -5: "EXC_ESTATE", -6: "EXC_EUNSUPPORTED"}
EXPORTED_SYMBOLS = ("exchange_init", "exchange_matrix", "exchange_matrix_noalloc", "exchange_matrix_all",
                    "exchange_energy",
                    "exchange_energy_device", "exchange_gamma_term", "exchange_back_transform",
                    "exchange_band_mask",
                    "exchange_last_error", "exchange_destroy", "exchange_query", "exchange_timing",
                    "exchange_nn_init", "exchange_nn_params", "exchange_nn_train", "exchange_nn_grad",
                    "exchange_nn_predict", "exchange_nn_features", "exchange_eigh", "exchange_nn_project",
                    "exchange_nn_expand")


class ExchangeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Desc(ctypes.Structure):
    _fields_ = [("n_k", ctypes.c_int32), ("n_q", ctypes.c_int32), ("n_occ", ctypes.c_int32),
                ("n_channels", ctypes.c_int32),
                ("n_bands", ctypes.POINTER(ctypes.c_int32)), ("n_pw", ctypes.POINTER(ctypes.c_int32)),
                ("ch_nrad", ctypes.POINTER(ctypes.c_int32)), ("w_q", ctypes.POINTER(ctypes.c_double)),
                ("precision", ctypes.c_int32), ("form", ctypes.c_int32), ("batched", ctypes.c_int32),
                ("device", ctypes.c_int32), ("inversion", ctypes.c_int32),
                ("w_kq", ctypes.POINTER(ctypes.c_double))]


class _Coulomb(ctypes.Structure):
    _fields_ = [("E", ctypes.POINTER(ctypes.c_void_p)), ("D", ctypes.POINTER(ctypes.c_void_p)),
                ("C", ctypes.POINTER(ctypes.c_void_p)), ("on_device", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load ``libexchange.so`` and declare the C signatures (no GPU needed)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ExchangeError(-6, f"{path} is not built; run `python -m paper_1003_0524_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.exchange_init.argtypes = [ctypes.POINTER(_Desc), ctypes.POINTER(_Coulomb), vp, ctypes.POINTER(vp)]
    lib.exchange_init.restype = i32
    lib.exchange_matrix.argtypes = [vp, i32, vp, i32, i32, vp, vp]
    lib.exchange_matrix.restype = i32
    lib.exchange_matrix_noalloc.argtypes = [vp, i32, vp, i32, vp, vp]
    lib.exchange_matrix_noalloc.restype = i32
    lib.exchange_matrix_all.argtypes = [vp, ctypes.POINTER(vp), i32, i32, ctypes.POINTER(vp), vp]
    lib.exchange_matrix_all.restype = i32
    lib.exchange_energy.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(vp),
                                    ctypes.POINTER(ctypes.c_double)]
    lib.exchange_energy.restype = i32
    lib.exchange_energy_device.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(vp), vp, vp]
    lib.exchange_gamma_term.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32),
                                        ctypes.c_double, i32, ctypes.POINTER(ctypes.c_double), vp]
    lib.exchange_gamma_term.restype = i32
    lib.exchange_back_transform.argtypes = [vp, i32, vp, i32, vp, vp]
    lib.exchange_back_transform.restype = i32
    lib.exchange_band_mask.argtypes = [vp, i32, vp]
    lib.exchange_band_mask.restype = i32
    lib.exchange_energy_device.restype = i32
    lib.exchange_last_error.argtypes = [vp]
    lib.exchange_last_error.restype = ctypes.c_char_p
    lib.exchange_destroy.argtypes = [vp]
    lib.exchange_destroy.restype = None
    lib.exchange_query.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double)]
    lib.exchange_query.restype = i32
    lib.exchange_timing.argtypes = [vp, i32]
    lib.exchange_timing.restype = i32
    f32p, f64p, u64, i64 = ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64
    vpp = ctypes.POINTER(vp)
    sigs = {
        "exchange_nn_init": [vp, i32, i32, i32, u64],
        "exchange_nn_params": [vp, vp, i64, i32, i32],
        "exchange_nn_train": [vp, vp, vp, i32, i32, ctypes.c_float, i32, f32p],
        "exchange_nn_grad": [vp, vp, vp, i32, i32, vp, f32p],
        "exchange_nn_predict": [vp, vp, i32, vp, i32, vp],
        "exchange_nn_features": [vp, vp, vp, i64, u64, i32, vp, vp, vp],
        "exchange_eigh": [vp, vpp, vp, vp, vp],
        "exchange_nn_project": [vp, vpp, vpp, vp, i32, ctypes.c_double, vp, vp],
        "exchange_nn_expand": [vp, vpp, vp, i32, vp, ctypes.c_double, vpp, vp],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = i32
    if path == LIB_PATH:
        _lib = lib
    return lib


def _i32(a):
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _stream_handle(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Exchange:
    """One prepared Coulomb matrix set + plans on one GPU (a ``exc_ctx``)."""

    def __init__(self, n_bands: Sequence[int], n_pw: Sequence[int], ch_nrad: Sequence[int],
                 n_occ: int, E: Sequence[np.ndarray], D: Sequence[np.ndarray], C: Sequence[np.ndarray],
                 w_q: Optional[Sequence[float]] = None, precision: str = "fp64", form: str = "herk",
                 batched: bool = True, device: int = 0, inversion: bool = False, w_kq=None,
                 D_q=None, C_q=None):
        """inversion=True: real v and real bands; M packs bands 2j, 2j+1 as the real and imaginary
        parts of column j (``synth.pack_real_pairs``) and V(k) comes back real (Im = 0).
        w_kq: [n_k][n_q] pair weights (0 leaves the pair out and its q block out of M(k)).
        D, C: the channel blocks of every q; D_q, C_q (lists over q of such lists) instead give
        each q its own (blocks of different q may be the same objects). E given as CUDA
        tensors: the blocks are taken from device memory (D and C copied there first)."""
        import torch
        if not torch.cuda.is_available():
            raise ExchangeError(-5, "no GPU visible: the exchange library runs only on a HIP device")
        self._torch = torch
        self.lib = load_library()
        self.device = device
        self.n_k, self.n_q = len(n_bands), len(n_pw)
        self.n_bands = [int(x) for x in n_bands]
        self.n_occ = int(n_occ)
        self.inversion = bool(inversion)
        self.n_cols = (self.n_occ + 1) // 2 if self.inversion else self.n_occ   # columns n'' of M
        self.precision, self.form, self.batched = precision, form, bool(batched)
        nb_arr, nb_p = _i32(n_bands)
        pw_arr, pw_p = _i32(n_pw)
        ch_arr, ch_p = _i32(ch_nrad if len(ch_nrad) else [0])
        wq_arr = None
        if w_q is not None:
            wq_arr = np.ascontiguousarray(np.asarray(w_q, dtype=np.float64))
        wkq_arr = None
        if w_kq is not None:
            wkq_arr = np.ascontiguousarray(np.asarray(w_kq, dtype=np.float64).reshape(self.n_k, self.n_q))
        self.pair_used = (np.ones((self.n_k, self.n_q), dtype=bool) if wkq_arr is None else wkq_arr != 0.0)
        n_s = int(sum(int(b) - 1 for b in ch_nrad))
        self.n_mb = [n_s + len(ch_nrad) + int(p) for p in n_pw]
        desc = _Desc(self.n_k, self.n_q, self.n_occ, len(ch_nrad), nb_p, pw_p,
                     ch_p if len(ch_nrad) else None,
                     wq_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if wq_arr is not None else None,
                     PRECISIONS[precision], FORMS[form], 1 if batched else 0, device,
                     1 if self.inversion else 0,
                     wkq_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if wkq_arr is not None else None)
        def cat(blocks, tr):
            return np.ascontiguousarray(np.concatenate(
                [(np.asarray(b, np.complex128).T if tr else np.asarray(b, np.complex128)).ravel() for b in blocks]
                + [np.zeros(0, np.complex128)]))
        if D_q is None:
            d_cats, c_cats = [cat(D, True)], [cat(C, False)]
            d_of, c_of = [0] * self.n_q, [0] * self.n_q
        else:
            # one copy per distinct set of blocks: q that share their blocks share a pointer
            d_cats, c_cats, d_of, c_of, seen = [], [], [], [], {}
            for q in range(self.n_q):
                key = (id(D_q[q]), id(C_q[q]))
                if key not in seen:
                    seen[key] = len(d_cats)
                    d_cats.append(cat(D_q[q], True))
                    c_cats.append(cat(C_q[q], False))
                d_of.append(seen[key])
                c_of.append(seen[key])
        on_dev = all(isinstance(e, torch.Tensor) and e.is_cuda for e in E)
        if on_dev:
            # blocks already in device memory: copied on the device (no host round trip)
            e_keep = [e.to(torch.complex128).T.contiguous() for e in E]         # column-major
            e_ptrs = (ctypes.c_void_p * self.n_q)(*[e.data_ptr() for e in e_keep])
            d_keep = [torch.from_numpy(x).to(E[0].device) for x in d_cats]
            c_keep = [torch.from_numpy(x).to(E[0].device) for x in c_cats]
            dp = [x.data_ptr() if x.numel() else None for x in d_keep]
            cp = [x.data_ptr() if x.numel() else None for x in c_keep]
            torch.cuda.synchronize()          # the copies above have landed before init reads them
        else:
            e_keep = [np.ascontiguousarray(np.asarray(e, dtype=np.complex128).T) for e in E]   # column-major
            e_ptrs = (ctypes.c_void_p * self.n_q)(*[e.ctypes.data for e in e_keep])
            dp = [x.ctypes.data if x.size else None for x in d_cats]
            cp = [x.ctypes.data if x.size else None for x in c_cats]
        d_ptrs = (ctypes.c_void_p * self.n_q)(*[dp[i] for i in d_of])
        c_ptrs = (ctypes.c_void_p * self.n_q)(*[cp[i] for i in c_of])
        coul = _Coulomb(e_ptrs, d_ptrs, c_ptrs, 1 if on_dev else 0)
        torch.cuda.set_device(device)
        ctx = ctypes.c_void_p()
        st = self.lib.exchange_init(ctypes.byref(desc), ctypes.byref(coul), _stream_handle(torch, device),
                                    ctypes.byref(ctx))
        if st != 0:
            raise ExchangeError(st, self.lib.exchange_last_error(None).decode())
        self.ctx = ctx
        self._keep = (nb_arr, pw_arr, ch_arr, wq_arr, wkq_arr)

    # -- helpers -----------------------------------------------------------
    def _check(self, st):
        if st != 0:
            raise ExchangeError(st, self.lib.exchange_last_error(self.ctx).decode())

    def _dtype_code(self, M):
        t = self._torch
        if M.dtype == t.complex128:
            return DTYPES["c128"]
        if M.dtype == t.complex64:
            return DTYPES["c64"]
        raise ExchangeError(-1, f"M must be complex64 or complex128, got {M.dtype}")

    def m_elems(self, k: int, n_mb: Optional[Sequence[int]] = None) -> int:
        """Complex elements of M(k): the q blocks of the pairs k computes, [n''][n][I] each."""
        n_mb = self.n_mb if n_mb is None else n_mb
        return int(sum(self.n_cols * self.n_bands[k] * int(n) for q, n in enumerate(n_mb) if self.pair_used[k, q]))

    def _check_m(self, k: int, M) -> None:
        """The kernels size their reads from the context's shapes, not from the buffer: a
        short M (or one that still holds the blocks of pairs left out by w_kq) is refused
        before anything is launched."""
        n = int(M.numel()) if hasattr(M, "numel") else int(np.asarray(M).size)
        want = self.m_elems(k)
        if n != want:
            raise ExchangeError(-1, f"M(k={k}) has {n} elements, the context needs {want} "
                                    f"(n_occ columns x n_b(k) x N_MB(q) over the computed q)")

    def _check_out(self, k: int, out) -> None:
        t = self._torch
        nb = self.n_bands[k]
        if out.dtype != t.complex128 or int(out.numel()) != nb * nb or not out.is_contiguous():
            raise ExchangeError(-1, f"out for k={k} must be a contiguous complex128 tensor of {nb * nb} elements")

    def accumulation_plan(self):
        """How the reduced-precision main kernel accumulates the band contraction in
        binary32 (exchange_query 14-19), as the error model of the tests takes it; None in
        FP64 and for the unbatched GEMM form."""
        kind = int(self.query(16))
        if kind < 0:
            return None
        return {"kind": kind, "nct": int(self.query(15)), "split": int(self.query(14)),
                "rs": int(self.query(17)), "rd": int(self.query(18)), "rbm": int(self.query(19))}

    # -- API ---------------------------------------------------------------
    def matrix(self, k: int, M, out=None):
        """V^x(k) (n_b x n_b complex128, column-major storage returned as its transpose view)."""
        t = self._torch
        nb = self.n_bands[k]
        self._dtype_code(M)
        self._check_m(k, M)
        if out is None:
            out = t.empty(nb * nb, dtype=t.complex128, device=M.device)
        self._check_out(k, out)
        if not (M.is_cuda and M.is_contiguous() and out.is_cuda):
            raise ExchangeError(-1, "M and out must be contiguous device tensors")
        st = self.lib.exchange_matrix(self.ctx, int(k), ctypes.c_void_p(M.data_ptr()), self._dtype_code(M), 1,
                                      ctypes.c_void_p(out.data_ptr()), _stream_handle(t, self.device))
        self._check(st)
        return out.view(nb, nb).T      # column-major -> [n][n'] view

    def matrix_noalloc(self, k: int, M, out):
        """V^x(k) through exchange_matrix_noalloc (no device allocation inside the call; out
        is the caller's contiguous complex128 device tensor of n_b(k)^2 elements)."""
        t = self._torch
        nb = self.n_bands[k]
        self._check_m(k, M)
        self._check_out(k, out)
        if not (M.is_cuda and M.is_contiguous() and out.is_cuda):
            raise ExchangeError(-1, "M and out must be contiguous device tensors")
        st = self.lib.exchange_matrix_noalloc(self.ctx, int(k), ctypes.c_void_p(M.data_ptr()),
                                              self._dtype_code(M), ctypes.c_void_p(out.data_ptr()),
                                              _stream_handle(t, self.device))
        self._check(st)
        return out.view(nb, nb).T

    def matrix_all(self, Ms: Sequence, outs=None):
        t = self._torch
        if len(Ms) != self.n_k:
            raise ExchangeError(-1, f"need {self.n_k} M tensors")
        code = self._dtype_code(Ms[0])
        for k, M in enumerate(Ms):
            if self._dtype_code(M) != code:
                raise ExchangeError(-1, "all M must have one dtype")
            self._check_m(k, M)
        if outs is None:
            outs = [t.empty(nb * nb, dtype=t.complex128, device=Ms[0].device) for nb in self.n_bands]
        if len(outs) != self.n_k:
            raise ExchangeError(-1, f"need {self.n_k} output tensors")
        for k, o in enumerate(outs):
            self._check_out(k, o)
        for M, o in zip(Ms, outs):
            if not (M.is_cuda and M.is_contiguous() and o.is_cuda):
                raise ExchangeError(-1, "all M and outputs must be contiguous device tensors")
        mp = (ctypes.c_void_p * self.n_k)(*[M.data_ptr() for M in Ms])
        vp = (ctypes.c_void_p * self.n_k)(*[o.data_ptr() for o in outs])
        st = self.lib.exchange_matrix_all(self.ctx, mp, code, 1, vp, _stream_handle(t, self.device))
        self._check(st)
        return [o.view(nb, nb).T for o, nb in zip(outs, self.n_bands)]

    def matrix_host(self, k: int, M: np.ndarray) -> np.ndarray:
        """Host-pointer variant (copies in and out; synchronous)."""
        nb = self.n_bands[k]
        M = np.ascontiguousarray(M)
        code = DTYPES["c64"] if M.dtype == np.complex64 else DTYPES["c128"]
        if M.dtype not in (np.complex64, np.complex128):
            raise ExchangeError(-1, "M must be complex64 or complex128")
        self._check_m(k, M)
        out = np.empty(nb * nb, dtype=np.complex128)
        st = self.lib.exchange_matrix(self.ctx, int(k), ctypes.c_void_p(M.ctypes.data), code, 0,
                                      ctypes.c_void_p(out.ctypes.data), _stream_handle(self._torch, self.device))
        self._check(st)
        return out.reshape(nb, nb).T.copy()

    def energy(self, w_k: Optional[Sequence[float]] = None, rho: Optional[Sequence] = None) -> float:
        wk = None
        if w_k is not None:
            wk_arr = np.ascontiguousarray(np.asarray(w_k, dtype=np.float64))
            wk = wk_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        rp = None
        if rho is not None:
            rp = (ctypes.c_void_p * self.n_k)(*[r.data_ptr() for r in rho])
        e = ctypes.c_double()
        self._check(self.lib.exchange_energy(self.ctx, wk, rp, ctypes.byref(e)))
        return e.value

    def energy_device(self, out, w_k: Optional[Sequence[float]] = None, rho: Optional[Sequence] = None,
                      stream=None) -> None:
        """E_x into out (a one-element float64 CUDA tensor) without synchronising."""
        if str(out.dtype) != "torch.float64" or not out.is_cuda or out.numel() < 1:
            raise ValueError("out must be a float64 CUDA tensor with at least one element")
        wk = None
        if w_k is not None:
            wk_arr = np.ascontiguousarray(np.asarray(w_k, dtype=np.float64))
            wk = wk_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        rp = None
        if rho is not None:
            rp = (ctypes.c_void_p * self.n_k)(*[r.data_ptr() for r in rho])
        st = ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)
        self._check(self.lib.exchange_energy_device(self.ctx, wk, rp, ctypes.c_void_p(out.data_ptr()), st))

    def gamma_term(self, recip, mesh: Sequence[int], beta: float = 0.005, apply: bool = True,
                   stream=None) -> float:
        """C of the q -> 0 term (exchange_gamma_term); with apply, later V(k) carry -C on the occupied diagonal."""
        b = np.ascontiguousarray(np.asarray(recip, dtype=np.float64).reshape(9))
        m = np.ascontiguousarray(np.asarray(mesh, dtype=np.int32).reshape(3))
        out = ctypes.c_double()
        st = (ctypes.c_void_p(stream.cuda_stream) if stream is not None
              else _stream_handle(self._torch, self.device))
        self._check(self.lib.exchange_gamma_term(self.ctx, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                 m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), float(beta),
                                                 int(bool(apply)), ctypes.byref(out), st))
        return out.value

    def back_transform(self, k: int, Z, out=None, stream=None):
        """V^x(k) in the LAPW basis, Z V(k) Z^H (Z = S c: an n_G x n_b(k) complex128 CUDA tensor,
        row-major [G][n] views are taken as given: pass Z laid out column-major, i.e. Z.T.contiguous().T)."""
        t = self._torch
        nG = int(Z.shape[0])
        if Z.dtype != t.complex128 or not Z.is_cuda or tuple(Z.shape) != (nG, self.n_bands[k]):
            raise ExchangeError(-1, "Z must be an n_G x n_b(k) complex128 CUDA tensor")
        nb = self.n_bands[k]
        if not ((nG == 1 or Z.stride(0) == 1) and (nb == 1 or Z.stride(1) == nG)):
            raise ExchangeError(-1, "Z must be column-major (strides (1, n_G))")
        if out is None:
            out = t.empty(nG * nG, dtype=t.complex128, device=Z.device)
        st = (ctypes.c_void_p(stream.cuda_stream) if stream is not None
              else _stream_handle(t, self.device))
        self._check(self.lib.exchange_back_transform(self.ctx, int(k), ctypes.c_void_p(Z.data_ptr()), nG,
                                                     ctypes.c_void_p(out.data_ptr()), st))
        return out.view(nG, nG).T      # column-major -> [G][G'] view

    def band_mask(self, k: int, keep=None) -> None:
        """Band pairs of V(k) to compute (n_b x n_b booleans; None: all). Tiles of 8 x 8 pairs
        whose elements (and mirror) are all False are skipped and come back as zeros."""
        if keep is None:
            self._check(self.lib.exchange_band_mask(self.ctx, int(k), None))
            return
        m = np.ascontiguousarray(np.asarray(keep, dtype=np.uint8).reshape(self.n_bands[k], self.n_bands[k]))
        self._check(self.lib.exchange_band_mask(self.ctx, int(k), ctypes.c_void_p(m.ctypes.data)))

    def gamma_kernel_ms(self):
        """(lattice-sum kernel ms, number of terms) of the last gamma_term call."""
        return self.query(11), int(self.query(12))

    def query(self, what: int) -> float:
        v = ctypes.c_double()
        self._check(self.lib.exchange_query(self.ctx, int(what), ctypes.byref(v)))
        return v.value

    def timing(self, n_slots: int) -> None:
        """Enable (n_slots > 0) or disable (0) live kernel timing of the batched path."""
        self._check(self.lib.exchange_timing(self.ctx, int(n_slots)))

    def kernel_ms(self):
        """(mean tile-kernel ms, mean sparse-kernel ms, replays timed)."""
        return self.query(5), self.query(7), int(self.query(6))

    # -- learned extrapolator ------------------------------------------------
    @staticmethod
    def _ptr(x):
        """(pointer, on_device) of a contiguous torch tensor or numpy array."""
        if hasattr(x, "data_ptr"):
            if not x.is_contiguous():
                raise ExchangeError(-1, "tensors must be contiguous")
            return ctypes.c_void_p(x.data_ptr()), int(x.is_cuda)
        if not x.flags["C_CONTIGUOUS"]:
            raise ExchangeError(-1, "arrays must be C-contiguous")
        return ctypes.c_void_p(x.ctypes.data), 0

    def _ptab(self, xs):
        if len(xs) != self.n_k:
            raise ExchangeError(-1, f"need {self.n_k} device tensors")
        for x in xs:
            if not (x.is_cuda and x.is_contiguous()):
                raise ExchangeError(-1, "per-k matrices must be contiguous device tensors")
        return (ctypes.c_void_p * self.n_k)(*[x.data_ptr() for x in xs])

    def nn_init(self, in_dim: int, hidden: int, out_dim: int, seed: int) -> None:
        self._check(self.lib.exchange_nn_init(self.ctx, int(in_dim), int(hidden), int(out_dim),
                                              ctypes.c_uint64(seed & (2 ** 64 - 1))))
        self._nn = (int(in_dim), int(hidden), int(out_dim))

    def nn_param_count(self) -> int:
        I, H, O = self._nn
        return H * I + H + H * H + H + O * H + O

    def nn_get_params(self) -> np.ndarray:
        out = np.empty(self.nn_param_count(), dtype=np.float32)
        self._check(self.lib.exchange_nn_params(self.ctx, ctypes.c_void_p(out.ctypes.data), out.size, 0, 0))
        return out

    def nn_set_params(self, theta) -> None:
        p, dev = self._ptr(theta)
        self._check(self.lib.exchange_nn_params(self.ctx, p, self.nn_param_count(), 1, dev))

    def nn_train(self, X, Y, epochs: int, lr: float) -> float:
        (px, dx), (py, dy) = self._ptr(X), self._ptr(Y)
        if dx != dy:
            raise ExchangeError(-1, "X and Y must both be host or both be device buffers")
        loss = ctypes.c_float()
        self._check(self.lib.exchange_nn_train(self.ctx, px, py, int(X.shape[0]), int(epochs), float(lr), dx,
                                               ctypes.byref(loss)))
        return loss.value

    def nn_grad(self, X, Y):
        (px, dx), (py, dy) = self._ptr(X), self._ptr(Y)
        if dx or dy:
            raise ExchangeError(-1, "nn_grad takes host arrays")
        g = np.empty(self.nn_param_count(), dtype=np.float32)
        loss = ctypes.c_float()
        self._check(self.lib.exchange_nn_grad(self.ctx, px, py, int(X.shape[0]), 0,
                                              ctypes.c_void_p(g.ctypes.data), ctypes.byref(loss)))
        return loss.value, g

    def nn_predict(self, X, out=None):
        t = self._torch
        px, dx = self._ptr(X)
        n = int(X.shape[0])
        if dx:
            if out is None:
                out = t.empty((n, self._nn[2]), dtype=t.float32, device=X.device)
            self._check(self.lib.exchange_nn_predict(self.ctx, px, n, ctypes.c_void_p(out.data_ptr()), 1,
                                                     _stream_handle(t, self.device)))
            return out
        out = np.empty((n, self._nn[2]), dtype=np.float32)
        self._check(self.lib.exchange_nn_predict(self.ctx, px, n, ctypes.c_void_p(out.ctypes.data), 0, None))
        return out

    def nn_features(self, P_new, P_old, m: int, seed: int):
        """(x (m floats, device), |P_new - P_old| (device double)) for float64/complex128 device tensors."""
        t = self._torch
        if not (P_new.is_cuda and P_old.is_cuda and P_new.is_contiguous() and P_old.is_contiguous()):
            raise ExchangeError(-1, "P_new and P_old must be contiguous device tensors")
        a = t.view_as_real(P_new) if P_new.is_complex() else P_new
        b = t.view_as_real(P_old) if P_old.is_complex() else P_old
        if a.dtype != t.float64 or b.dtype != t.float64 or a.numel() != b.numel():
            raise ExchangeError(-1, "P_new and P_old must be float64/complex128 of equal size")
        x = t.empty(m, dtype=t.float32, device=P_new.device)
        nrm = t.empty(1, dtype=t.float64, device=P_new.device)
        self._check(self.lib.exchange_nn_features(self.ctx, ctypes.c_void_p(a.data_ptr()),
                                                  ctypes.c_void_p(b.data_ptr()), a.numel(),
                                                  ctypes.c_uint64(seed & (2 ** 64 - 1)), int(m),
                                                  ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(nrm.data_ptr()),
                                                  _stream_handle(t, self.device)))
        return x, nrm

    def eigh(self, A_k):
        """(eigenvalues packed, eigenvectors packed) of the per-k Hermitian matrices (column-major storage)."""
        t = self._torch
        dev = A_k[0].device
        w = t.empty(sum(self.n_bands), dtype=t.float64, device=dev)
        Z = t.empty(sum(nb * nb for nb in self.n_bands), dtype=t.complex128, device=dev)
        self._check(self.lib.exchange_eigh(self.ctx, self._ptab(A_k), ctypes.c_void_p(w.data_ptr()),
                                           ctypes.c_void_p(Z.data_ptr()), _stream_handle(t, self.device)))
        return w, Z

    def nn_project(self, Va_k, Vb_k, Z, n_blk: int, scale: float):
        t = self._torch
        y = t.empty((self.n_k, n_blk * n_blk), dtype=t.float32, device=Z.device)
        self._check(self.lib.exchange_nn_project(self.ctx, self._ptab(Va_k), self._ptab(Vb_k),
                                                 ctypes.c_void_p(Z.data_ptr()), int(n_blk), float(scale),
                                                 ctypes.c_void_p(y.data_ptr()), _stream_handle(t, self.device)))
        return y

    def nn_expand(self, Vanc_k, Z, n_blk: int, y, scale: float, outs):
        t = self._torch
        if not (y.is_cuda and y.is_contiguous() and y.dtype == t.float32):
            raise ExchangeError(-1, "y must be a contiguous float32 device tensor")
        self._check(self.lib.exchange_nn_expand(self.ctx, self._ptab(Vanc_k), ctypes.c_void_p(Z.data_ptr()),
                                                int(n_blk), ctypes.c_void_p(y.data_ptr()), float(scale),
                                                self._ptab(outs), _stream_handle(t, self.device)))
        return outs

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.exchange_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
