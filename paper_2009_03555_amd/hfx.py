"""ctypes binding of libhfx.so (argument marshalling only).

Every step of the exchange build runs in the HIP library; this module turns
Python objects into the C structs and pointers of ``include/hfx.h``.  Device
arrays are torch tensors (float64, on the HIP device); torch supplies memory
and the stream, nothing else.  If the library is missing this module raises:
there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhfx.so")

HFX_OK, HFX_ERR_INVALID, HFX_ERR_OOM, HFX_ERR_DEVICE, HFX_ERR_STATE, HFX_ERR_UNSUPPORTED = range(6)
STATUS_NAMES = ["HFX_OK", "HFX_ERR_INVALID", "HFX_ERR_OOM", "HFX_ERR_DEVICE", "HFX_ERR_STATE",
                "HFX_ERR_UNSUPPORTED"]
HFX_SYNC = 1
HFX_TIMING = 2
HFX_GRAPH = 4
N_CLASSES = 21
OPS = {"coulomb": 0, "erfc": 1}
PRECISIONS = {"fp64": 0, "mixed": 1}


class HfxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 6 else status}: {msg}")
        self.status = status


class hfx_system(ctypes.Structure):
    _fields_ = [
        ("n_atoms", ctypes.c_int32), ("atom_xyz", ctypes.POINTER(ctypes.c_double)),
        ("n_shells", ctypes.c_int32), ("shell_atom", ctypes.POINTER(ctypes.c_int32)),
        ("shell_l", ctypes.POINTER(ctypes.c_int32)), ("shell_nprim", ctypes.POINTER(ctypes.c_int32)),
        ("prim_exp", ctypes.POINTER(ctypes.c_double)), ("prim_coef", ctypes.POINTER(ctypes.c_double)),
        ("lattice", ctypes.POINTER(ctypes.c_double)), ("pair_cutoff", ctypes.c_double),
        ("op", ctypes.c_int32), ("omega", ctypes.c_double), ("tau", ctypes.c_double),
        ("precision", ctypes.c_int32), ("fp32_cutoff", ctypes.c_double),
        ("spherical_d", ctypes.c_int32),
    ]


class hfx_block(ctypes.Structure):
    _fields_ = [("I", ctypes.c_int32), ("J", ctypes.c_int32), ("img", ctypes.c_int32 * 3),
                ("pad", ctypes.c_int32), ("offset", ctypes.c_int64)]


class hfx_build_info(ctypes.Structure):
    _fields_ = [("n_quartets", ctypes.c_int64), ("n_quartets_class", ctypes.c_int64 * N_CLASSES),
                ("n_prim_quartets", ctypes.c_int64), ("n_fp32_quartets", ctypes.c_int64),
                ("flops", ctypes.c_double), ("ms_density", ctypes.c_double),
                ("ms_screen", ctypes.c_double), ("ms_eri", ctypes.c_double),
                ("ms_finalize", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("ms_class", ctypes.c_double * N_CLASSES), ("flops_class", ctypes.c_double * N_CLASSES),
                ("n_chunks", ctypes.c_int64)]

    def as_dict(self):
        d = {}
        for k, _ in self._fields_:
            v = getattr(self, k)
            d[k] = list(v) if k in ("n_quartets_class", "ms_class", "flops_class") else v
        return d


TUNE_MAX_CAND = 12
VARIANT_NAMES = ["reg", "coop", "lane", "reg32", "lane32"]


class hfx_tune_candidate(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("fp32_list", ctypes.c_int32), ("max_blocks", ctypes.c_int64),
                ("ms", ctypes.c_double)]


class hfx_tune_report(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_int32 * N_CLASSES), ("sample_quartets", ctypes.c_int64 * N_CLASSES),
                ("sample_quartets32", ctypes.c_int64 * N_CLASSES), ("chosen", ctypes.c_int32 * N_CLASSES),
                ("chosen32", ctypes.c_int32 * N_CLASSES),
                ("cand", (hfx_tune_candidate * TUNE_MAX_CAND) * N_CLASSES)]

    def as_list(self):
        """per class: {"candidates": [(variant, fp32_list, max_blocks, ms)], "chosen", "chosen32", samples}"""
        out = []
        for r in range(N_CLASSES):
            c = [(VARIANT_NAMES[t.variant], bool(t.fp32_list), int(t.max_blocks), float(t.ms))
                 for t in list(self.cand[r])[: self.n_candidates[r]]]
            out.append({"candidates": c, "chosen": int(self.chosen[r]), "chosen32": int(self.chosen32[r]),
                        "sample_quartets": int(self.sample_quartets[r]),
                        "sample_quartets32": int(self.sample_quartets32[r])})
        return out


PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                               ctypes.c_int64)

_lib = None


def lib():
    """Load libhfx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_2009_03555_amd.build (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.hfx_last_error.restype = ctypes.c_char_p
        L.hfx_footprint.argtypes = [ctypes.POINTER(hfx_system), ctypes.POINTER(ctypes.c_size_t),
                                    ctypes.POINTER(ctypes.c_size_t)]
        L.hfx_plan.argtypes = [ctypes.POINTER(hfx_system), vp, ctypes.POINTER(vp)]
        L.hfx_pattern.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.POINTER(hfx_block))]
        L.hfx_schwarz.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.hfx_build_K.argtypes = [vp, vp, vp, ctypes.c_uint32, ctypes.POINTER(hfx_build_info)]
        L.hfx_build_K_multi.argtypes = [ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                        ctypes.POINTER(vp), ctypes.c_uint32, ctypes.POINTER(hfx_build_info)]
        L.hfx_export.argtypes = [vp, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_int64)]
        L.hfx_plan_destroy.argtypes = [vp]
        L.hfx_autotune.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.POINTER(hfx_tune_report)]
        L.hfx_screen_count.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.hfx_build_K_subset.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int64]
        L.hfx_set_list_limit.argtypes = [vp, ctypes.c_int64]
        L.hfx_set_progress.argtypes = [vp, PROGRESS_FN, vp]
        dpp = ctypes.POINTER(ctypes.c_double)
        L.hfx_nao2gto_fit.argtypes = [ctypes.c_int32, ctypes.c_int32, dpp, dpp, ctypes.c_int32, dpp, dpp, dpp]
        L.hfx_kspace.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_double, vp]
        L.hfx_build_K_spin.argtypes = [vp, vp, vp, vp, vp, ctypes.c_uint32, ctypes.POINTER(hfx_build_info)]
        L.hfx_build_K_noalloc.argtypes = [vp, vp, vp, ctypes.c_uint32, ctypes.POINTER(hfx_build_info)]
        for name in ("hfx_footprint", "hfx_plan", "hfx_pattern", "hfx_schwarz", "hfx_build_K",
                     "hfx_build_K_multi", "hfx_export", "hfx_plan_destroy", "hfx_autotune", "hfx_screen_count",
                     "hfx_build_K_subset", "hfx_set_list_limit", "hfx_build_K_noalloc", "hfx_build_K_spin", "hfx_kspace", "hfx_nao2gto_fit", "hfx_set_progress"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st: int):
    if st != HFX_OK:
        raise HfxError(st, lib().hfx_last_error().decode(errors="replace"))


def hfx_last_error() -> str:
    return lib().hfx_last_error().decode(errors="replace")


class _SystemArgs:
    """Keeps the numpy arrays behind an hfx_system alive."""

    def __init__(self, system):
        s = system
        self.xyz = np.ascontiguousarray(s.atom_xyz, dtype=np.float64).reshape(-1)
        self.sa = np.ascontiguousarray(s.shell_atom, dtype=np.int32)
        self.sl = np.ascontiguousarray(s.shell_l, dtype=np.int32)
        self.sn = np.ascontiguousarray(s.shell_nprim, dtype=np.int32)
        self.ex = np.ascontiguousarray(s.prim_exp, dtype=np.float64)
        self.co = np.ascontiguousarray(s.prim_coef, dtype=np.float64)
        self.lat = None if s.lattice is None else np.ascontiguousarray(s.lattice, dtype=np.float64).reshape(9)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        self.c = hfx_system(
            n_atoms=len(self.xyz) // 3, atom_xyz=self.xyz.ctypes.data_as(dp),
            n_shells=len(self.sl), shell_atom=self.sa.ctypes.data_as(ip), shell_l=self.sl.ctypes.data_as(ip),
            shell_nprim=self.sn.ctypes.data_as(ip), prim_exp=self.ex.ctypes.data_as(dp),
            prim_coef=self.co.ctypes.data_as(dp),
            lattice=self.lat.ctypes.data_as(dp) if self.lat is not None else dp(),
            pair_cutoff=float(s.pair_cutoff), op=OPS[s.op] if isinstance(s.op, str) else int(s.op),
            omega=float(s.omega), tau=float(s.tau),
            precision=PRECISIONS[s.precision] if isinstance(s.precision, str) else int(s.precision),
            fp32_cutoff=float(s.fp32_cutoff), spherical_d=int(bool(s.spherical_d)))


def hfx_footprint(system):
    a = _SystemArgs(system)
    dev = ctypes.c_size_t(0)
    per = ctypes.c_size_t(0)
    _check(lib().hfx_footprint(ctypes.byref(a.c), ctypes.byref(dev), ctypes.byref(per)))
    return int(dev.value), int(per.value)


def _ptr(t) -> int:
    """Device pointer of a torch tensor (float64, contiguous) or an int."""
    if isinstance(t, int):
        return t
    if not t.is_contiguous() or str(t.dtype) != "torch.float64":
        raise ValueError("D and K must be contiguous float64 device tensors")
    return t.data_ptr()


class Plan:
    """An exchange-build plan (``hfx_plan``) for one system."""

    def __init__(self, system, stream: Optional[int] = None):
        self._args = _SystemArgs(system)
        self.system = system
        self._h = ctypes.c_void_p(None)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        _check(lib().hfx_plan(ctypes.byref(self._args.c), ctypes.c_void_p(stream), ctypes.byref(self._h)))
        nb = ctypes.c_int64(0)
        nnz = ctypes.c_int64(0)
        bp = ctypes.POINTER(hfx_block)()
        _check(lib().hfx_pattern(self._h, ctypes.byref(nb), ctypes.byref(nnz), ctypes.byref(bp)))
        self.n_blocks = int(nb.value)
        self.nnz = int(nnz.value)
        raw = np.ctypeslib.as_array(ctypes.cast(bp, ctypes.POINTER(ctypes.c_int32)),
                                    shape=(self.n_blocks * 8,)).reshape(self.n_blocks, 8) if self.n_blocks else \
            np.zeros((0, 8), dtype=np.int32)
        self.blocks = raw[:, :5].astype(np.int32).copy()
        self.offsets = np.concatenate([raw[:, 6:8].copy().view(np.int64).reshape(-1), [self.nnz]]).astype(np.int64)

    @property
    def handle(self):
        return self._h

    def schwarz(self) -> np.ndarray:
        q = np.zeros(max(self.n_blocks, 1))
        n = ctypes.c_int64(0)
        _check(lib().hfx_schwarz(self._h, q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(n)))
        self.n_pairs = int(n.value)
        return q[: self.n_blocks]

    def build_K(self, D, K, flags: int = 0, info: bool = False):
        inf = hfx_build_info() if info else None
        _check(lib().hfx_build_K(self._h, ctypes.c_void_p(_ptr(D)), ctypes.c_void_p(_ptr(K)), ctypes.c_uint32(flags),
                                 ctypes.byref(inf) if inf is not None else None))
        return inf.as_dict() if inf is not None else None

    def build_K_spin(self, D_alpha, D_beta, K_alpha, K_beta, flags: int = 0, info: bool = False):
        """``hfx_build_K_spin``: K of both spin densities from one ERI
        evaluation (collinear spin)."""
        inf = hfx_build_info() if info else None
        _check(lib().hfx_build_K_spin(self._h, ctypes.c_void_p(_ptr(D_alpha)), ctypes.c_void_p(_ptr(D_beta)),
                                      ctypes.c_void_p(_ptr(K_alpha)), ctypes.c_void_p(_ptr(K_beta)),
                                      ctypes.c_uint32(flags), ctypes.byref(inf) if inf is not None else None))
        return inf.as_dict() if inf is not None else None

    def kspace(self, K, kpts, alpha: float, H):
        """``hfx_kspace``: H(k) = -(alpha/2) sum_G K^G exp(i k.(T_G + r_nu - r_mu))
        into H (complex128 device tensor [nk, nbf, nbf], or float64 with a
        trailing dimension of 2)."""
        k = np.ascontiguousarray(kpts, dtype=np.float64).reshape(-1, 3)
        if not H.is_contiguous():
            raise ValueError("H must be contiguous")
        _check(lib().hfx_kspace(self._h, ctypes.c_void_p(_ptr(K)), len(k),
                                k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.c_double(alpha),
                                ctypes.c_void_p(H.data_ptr())))

    def set_progress(self, fn):
        """``hfx_set_progress``: fn(list, chunk, quartets_done, quartets_total)
        after each finished chunk of a chunked build (None: off)."""
        if fn is None:
            self._progress = None
            _check(lib().hfx_set_progress(self._h, PROGRESS_FN(), None))
            return
        self._progress = PROGRESS_FN(lambda user, lst, chunk, done, total: fn(lst, chunk, done, total))
        _check(lib().hfx_set_progress(self._h, self._progress, None))

    def set_list_limit(self, max_quartets: int):
        """``hfx_set_list_limit``: longest quartet list a build holds at once
        (longer screened lists run in chunks); 0 restores the default."""
        _check(lib().hfx_set_list_limit(self._h, ctypes.c_int64(int(max_quartets))))

    def build_K_noalloc(self, D, K, flags: int = 0, info: bool = False):
        """``hfx_build_K_noalloc``: the build with its work arrays in the
        library's static scratch memory (no device allocation)."""
        inf = hfx_build_info() if info else None
        _check(lib().hfx_build_K_noalloc(self._h, ctypes.c_void_p(_ptr(D)), ctypes.c_void_p(_ptr(K)),
                                         ctypes.c_uint32(flags), ctypes.byref(inf) if inf is not None else None))
        return inf.as_dict() if inf is not None else None

    def build_K_subset(self, D, K, quartets: np.ndarray):
        """``hfx_build_K_subset``: K from the given unique quartets only
        (uint64 encoding of export(1))."""
        q = np.ascontiguousarray(quartets, dtype=np.uint64)
        _check(lib().hfx_build_K_subset(self._h, ctypes.c_void_p(_ptr(D)), ctypes.c_void_p(_ptr(K)),
                                        q.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), ctypes.c_int64(len(q))))

    def screen_count(self, D):
        """``hfx_screen_count``: (FP64-list, FP32-list) quartet counts for density D."""
        n64 = ctypes.c_int64(0)
        n32 = ctypes.c_int64(0)
        _check(lib().hfx_screen_count(self._h, ctypes.c_void_p(_ptr(D)), ctypes.byref(n64), ctypes.byref(n32)))
        return int(n64.value), int(n32.value)

    def autotune(self, D, K, max_quartets: int = 200_000):
        """``hfx_autotune``: choose the ERI kernel variant and grid per class
        by timing, then build K; returns the per-class report."""
        rep = hfx_tune_report()
        _check(lib().hfx_autotune(self._h, ctypes.c_void_p(_ptr(D)), ctypes.c_void_p(_ptr(K)),
                                  ctypes.c_int64(max_quartets), ctypes.byref(rep)))
        return rep.as_list()

    def export(self, what: int) -> np.ndarray:
        n = ctypes.c_int64(0)
        _check(lib().hfx_export(self._h, what, None, ctypes.byref(n)))
        if what == 0 or what == 3:
            out = np.zeros(max(n.value, 1), dtype=np.float64)
        elif what in (1, 5):
            out = np.zeros(max(n.value, 1), dtype=np.uint64)
        else:
            out = np.zeros((max(n.value, 1), 6), dtype=np.int32)
        _check(lib().hfx_export(self._h, what, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)))
        return out[: n.value]

    def destroy(self):
        if self._h is not None and self._h.value:
            _check(lib().hfx_plan_destroy(self._h))
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def build_K_multi(plans: Sequence[Plan], Ds, Ks, flags: int = 0, info: bool = False):
    """``hfx_build_K_multi``: every plan's K from its D in fused launches."""
    n = len(plans)
    hs = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    ds = (ctypes.c_void_p * n)(*[_ptr(d) for d in Ds])
    ks = (ctypes.c_void_p * n)(*[_ptr(k) for k in Ks])
    inf = hfx_build_info() if info else None
    _check(lib().hfx_build_K_multi(n, hs, ds, ks, ctypes.c_uint32(flags),
                                   ctypes.byref(inf) if inf is not None else None))
    return inf.as_dict() if inf is not None else None


def nao2gto_fit(l: int, r, radial, n_gto: int):
    """``hfx_nao2gto_fit``: (exponents, raw coefficients, relative rms) of
    the GTO contraction fitted to the radial function on grid r."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    R = np.ascontiguousarray(radial, dtype=np.float64)
    if r.shape != R.shape:
        raise ValueError("r and radial differ in length")
    ex = np.zeros(n_gto)
    co = np.zeros(n_gto)
    rms = ctypes.c_double(0.0)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().hfx_nao2gto_fit(int(l), len(r), r.ctypes.data_as(dp), R.ctypes.data_as(dp), int(n_gto),
                                 ex.ctypes.data_as(dp), co.ctypes.data_as(dp), ctypes.byref(rms)))
    return ex, co, float(rms.value)


def unpack_quartets(q: np.ndarray) -> np.ndarray:
    """uint64 list -> (n, 5) int64: bra pair, ket pair, G1, G2, G3."""
    q = q.astype(np.uint64)
    out = np.zeros((len(q), 5), dtype=np.int64)
    out[:, 0] = (q & np.uint64(0xFFFFFF)).astype(np.int64)
    out[:, 1] = ((q >> np.uint64(24)) & np.uint64(0xFFFFFF)).astype(np.int64)
    g = (q >> np.uint64(48)).astype(np.int64)
    out[:, 2] = (g & 31) - 16
    out[:, 3] = ((g >> 5) & 31) - 16
    out[:, 4] = ((g >> 10) & 31) - 16
    return out
