"""Python binding of libqdcb.so (the C ABI in include/qdcb.h).

Argument marshalling only: every step of the transformation runs in the
library's HIP kernels.  Host numpy arrays or torch CUDA tensors are accepted
for the MO coefficients and the output; torch is used only for device
memory and streams.  If the shared library has not been built, every entry
point raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqdcb.so")

HAM = {"LL": 0, "DC": 1, "DCG": 2, "DCB": 3}
PREC = {"fp64": 0, "mixed": 1}
PTR_DEVICE = 0x1
CLASS_COULOMB = 0x2
CLASS_GAUNT = 0x4
CLASS_GAUGE = 0x8
CLASSES = {None: 0, "all": 0, "coulomb": CLASS_COULOMB, "gaunt": CLASS_GAUNT,
           "gauge": CLASS_GAUGE, "breit": CLASS_GAUNT | CLASS_GAUGE}
FETCH_DMAX, FETCH_Q, FETCH_DMAX_GAUNT, FETCH_Q_GAUNT = 1, 2, 3, 4
PLAN_DIRECTED_TILES = 0x1
PLAN_TIER_BY_G = 0x2
PLAN_SPINOR = 0x4
PLAN_PRIM_BANDS = 0x8
PLAN_SCHWARZ_ROWS = 0x10

STATUS = {0: "OK", -1: "E_INVALID", -2: "E_NOMEM", -3: "E_DEVICE", -4: "E_UNSUPPORTED",
          -5: "E_BUSY", -6: "E_ABORTED"}


class QdcbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class PlanDesc(ctypes.Structure):
    _fields_ = [("ham", ctypes.c_int32), ("prec", ctypes.c_int32), ("n_mo", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("tau", ctypes.c_double),
                ("tier_fp32", ctypes.c_double), ("tier_bf16", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double), ("ms_density", ctypes.c_double),
                ("ms_screen", ctypes.c_double), ("ms_eri", ctypes.c_double),
                ("ms_first_half", ctypes.c_double), ("ms_second_half", ctypes.c_double),
                ("kept", ctypes.c_int64 * 4), ("total", ctypes.c_int64 * 4),
                ("kept_gaunt", ctypes.c_int64), ("total_gaunt", ctypes.c_int64),
                ("tiles_kept", ctypes.c_int64), ("tiles_total", ctypes.c_int64),
                ("flops_first_half", ctypes.c_double), ("flops_second_half", ctypes.c_double),
                ("flops_mfma", ctypes.c_double), ("n_batches", ctypes.c_int32),
                ("n_chunks", ctypes.c_int32), ("graph_replay", ctypes.c_int32),
                ("graph_fallback", ctypes.c_int32), ("tiles_made", ctypes.c_int64),
                ("tiles_tier", ctypes.c_int64 * 3), ("ms_tier", ctypes.c_double * 3),
                ("classes", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if isinstance(v, ctypes.Array) else v
        return d


class Tune(ctypes.Structure):
    _fields_ = [("eri_sched", ctypes.c_int32), ("fh_order", ctypes.c_int32),
                ("sq_tile", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {"eri_sched": self.eri_sched, "fh_order": self.fh_order, "sq_tile": self.sq_tile}


class TuneReport(ctypes.Structure):
    _fields_ = [("chosen", Tune), ("from_cache", ctypes.c_int32), ("trials", ctypes.c_int32),
                ("ms_eri", ctypes.c_double * 2), ("ms_first_half", ctypes.c_double * 2),
                ("ms_second_half", ctypes.c_double * 2)]

    def as_dict(self):
        return {"chosen": self.chosen.as_dict(), "from_cache": self.from_cache,
                "trials": self.trials, "ms_eri": list(self.ms_eri),
                "ms_first_half": list(self.ms_first_half),
                "ms_second_half": list(self.ms_second_half)}


BLOCK_CB = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                            ctypes.c_void_p, ctypes.c_int)

_lib = None
_P = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
        # torch ships its own HIP runtime (same soname); load it first so that the
        # library binds to that one and device pointers and streams are shared.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        L.qdcb_abi_version.restype = ctypes.c_int
        L.qdcb_last_error.restype = ctypes.c_char_p
        L.qdcb_ctx_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(_P)]
        L.qdcb_ctx_destroy.argtypes = [_P]
        L.qdcb_ctx_destroy.restype = None
        L.qdcb_basis_create.argtypes = [_P, ctypes.c_int32, _DP, _IP, _DP, _DP, ctypes.POINTER(_P)]
        L.qdcb_basis_create_cart.argtypes = [_P, ctypes.c_int32, _DP, _IP, _DP, _DP, _IP,
                                             ctypes.POINTER(_P)]
        L.qdcb_basis_create_rkb.argtypes = [_P, _P, _DP, ctypes.POINTER(_P)]
        L.qdcb_rkb_small_planes.argtypes = [ctypes.c_int32, ctypes.c_int32, _DP, _DP,
                                            ctypes.c_double, _DP]
        L.qdcb_rkb_small_quat.argtypes = [ctypes.c_int32, ctypes.c_int32, _DP, _DP,
                                          ctypes.c_double, _DP]
        L.qdcb_basis_destroy.argtypes = [_P]
        L.qdcb_basis_destroy.restype = None
        L.qdcb_basis_schwarz.argtypes = [_P, _DP]
        L.qdcb_eri_quartets.argtypes = [_P, _P, ctypes.c_int64, _IP, _DP]
        L.qdcb_eri_quartets_noalloc.argtypes = [_P, _P, ctypes.c_int64, _IP, _DP]
        L.qdcb_plan_create.argtypes = [_P, _P, _P, ctypes.POINTER(PlanDesc), ctypes.POINTER(_P)]
        L.qdcb_plan_destroy.argtypes = [_P]
        L.qdcb_plan_destroy.restype = None
        L.qdcb_plan_footprint.argtypes = [_P, ctypes.POINTER(ctypes.c_size_t)]
        L.qdcb_transform.argtypes = [_P, _P, _P, _P, ctypes.c_uint32, _P,
                                     ctypes.POINTER(Stats)]
        L.qdcb_plan_fetch.argtypes = [_P, ctypes.c_int32, _P, ctypes.c_size_t]
        L.qdcb_plan_estimate.argtypes = [_P, _P, ctypes.POINTER(PlanDesc),
                                         ctypes.POINTER(ctypes.c_size_t)]
        L.qdcb_plan_capture.argtypes = [_P, _P, _P, _P, _P]
        L.qdcb_plan_replay.argtypes = [_P, _P, ctypes.POINTER(Stats)]
        L.qdcb_plan_fetch_v.argtypes = [_P, _P, ctypes.c_int64, _P]
        L.qdcb_transform_blocks.argtypes = [_P, _P, _P, BLOCK_CB, _P, ctypes.c_uint32, _P,
                                            ctypes.POINTER(Stats)]
        L.qdcb_plan_set_mo_batch.argtypes = [_P, ctypes.c_int32]
        L.qdcb_plan_set_tune.argtypes = [_P, ctypes.POINTER(Tune)]
        L.qdcb_plan_get_tune.argtypes = [_P, ctypes.POINTER(Tune)]
        L.qdcb_plan_tune_key.argtypes = [_P, ctypes.c_char_p, ctypes.c_size_t]
        L.qdcb_tune_cache_lookup.argtypes = [ctypes.c_char_p, ctypes.c_char_p,
                                             ctypes.POINTER(Tune), _IP]
        L.qdcb_tune_cache_store.argtypes = [ctypes.c_char_p, ctypes.c_char_p,
                                            ctypes.POINTER(Tune)]
        L.qdcb_plan_autotune.argtypes = [_P, _P, _P, _P, ctypes.c_uint32, _P, ctypes.c_char_p,
                                         ctypes.POINTER(TuneReport)]
        for f in ("qdcb_ctx_create", "qdcb_basis_create", "qdcb_basis_create_cart",
                  "qdcb_basis_create_rkb", "qdcb_rkb_small_planes", "qdcb_rkb_small_quat",
                  "qdcb_basis_schwarz",
                  "qdcb_eri_quartets", "qdcb_eri_quartets_noalloc", "qdcb_plan_create", "qdcb_plan_footprint",
                  "qdcb_transform", "qdcb_plan_fetch", "qdcb_plan_estimate",
                  "qdcb_plan_capture", "qdcb_plan_replay", "qdcb_plan_fetch_v",
                  "qdcb_plan_set_tune", "qdcb_plan_get_tune", "qdcb_plan_tune_key",
                  "qdcb_tune_cache_lookup", "qdcb_tune_cache_store", "qdcb_plan_autotune",
                  "qdcb_transform_blocks", "qdcb_plan_set_mo_batch"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st: int):
    if st != 0:
        raise QdcbError(st, lib().qdcb_last_error().decode())


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _is_torch_cuda(x) -> bool:
    return hasattr(x, "is_cuda") and hasattr(x, "data_ptr") and bool(x.is_cuda)


class Context:
    def __init__(self, device: int = 0, budget_bytes: int = 0):
        h = _P()
        _check(lib().qdcb_ctx_create(int(device), int(budget_bytes), ctypes.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        if self.h:
            lib().qdcb_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Basis:
    """Device-resident basis: ``basis`` has centers, nprim, exps, coefs and
    optionally cart (0 = s, 1..3 = p_x, p_y, p_z, 4..9 = d_xx, d_yy, d_zz, d_xy, d_xz, d_yz,
    10..19 = f_xxx, f_yyy, f_zzz, f_xxy, f_xxz, f_xyy, f_yyz, f_xzz, f_yzz, f_xyz;
    qdcb_basis_create_cart)."""

    def __init__(self, ctx: Context, basis):
        self.ctx = ctx
        self.nfunc = int(np.asarray(basis.nprim).shape[0])
        c = _f64(basis.centers)
        k = np.ascontiguousarray(basis.nprim, dtype=np.int32)
        e = _f64(basis.exps)
        d = _f64(basis.coefs)
        cart = getattr(basis, "cart", None)
        h = _P()
        if cart is None:
            _check(lib().qdcb_basis_create(ctx.h, self.nfunc, c.ctypes.data_as(_DP),
                                           k.ctypes.data_as(_IP), e.ctypes.data_as(_DP),
                                           d.ctypes.data_as(_DP), ctypes.byref(h)))
        else:
            ct = np.ascontiguousarray(cart, dtype=np.int32)
            _check(lib().qdcb_basis_create_cart(ctx.h, self.nfunc, c.ctypes.data_as(_DP),
                                                k.ctypes.data_as(_IP), e.ctypes.data_as(_DP),
                                                d.ctypes.data_as(_DP), ct.ctypes.data_as(_IP),
                                                ctypes.byref(h)))
        self.h = h

    def schwarz(self) -> np.ndarray:
        Q = np.empty((self.nfunc, self.nfunc))
        _check(lib().qdcb_basis_schwarz(self.h, Q.ctypes.data_as(_DP)))
        return Q

    def close(self):
        if self.h:
            lib().qdcb_basis_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rkb_basis(ctx: Context, L: "Basis"):
    """(gradient basis of 3 nfunc p functions, norms) for RKB small components
    (qdcb_basis_create_rkb)."""
    b = Basis.__new__(Basis)
    b.ctx = ctx
    b.nfunc = 3 * L.nfunc
    norms = np.empty(3 * L.nfunc)
    h = _P()
    _check(lib().qdcb_basis_create_rkb(ctx.h, L.h, norms.ctypes.data_as(_DP), ctypes.byref(h)))
    b.h = h
    return b, norms


def rkb_small_planes(PS: np.ndarray, norms: np.ndarray, c: float) -> np.ndarray:
    """Small-component planes [4][3 N][m] over the gradient basis from RKB
    planes PS [4][N][m] (qdcb_rkb_small_planes)."""
    PS = _f64(PS)
    N, m = PS.shape[1], PS.shape[2]
    norms = _f64(norms)
    out = np.empty((4, 3 * N, m))
    _check(lib().qdcb_rkb_small_planes(N, m, PS.ctypes.data_as(_DP), norms.ctypes.data_as(_DP),
                                       float(c), out.ctypes.data_as(_DP)))
    return out


def rkb_small_quat(CS: np.ndarray, norms: np.ndarray, c: float) -> np.ndarray:
    """Quaternion RKB small-component coefficients [4][3 N][n] over the
    gradient basis of rkb_basis, from the RKB quaternion coefficients
    CS [4][N][n] of n Kramers pairs."""
    CS = _f64(CS)
    norms = _f64(norms)
    N, n = CS.shape[1], CS.shape[2]
    out = np.empty((4, 3 * N, n))
    _check(lib().qdcb_rkb_small_quat(N, n, CS.ctypes.data_as(_DP), norms.ctypes.data_as(_DP),
                                     float(c), out.ctypes.data_as(_DP)))
    return out


def tune_cache_lookup(path: str, key: str) -> Optional[dict]:
    t, found = Tune(), ctypes.c_int32(0)
    _check(lib().qdcb_tune_cache_lookup(path.encode(), key.encode(), ctypes.byref(t),
                                        ctypes.byref(found)))
    return t.as_dict() if found.value else None


def tune_cache_store(path: str, key: str, tune: dict):
    t = Tune(int(tune["eri_sched"]), int(tune["fh_order"]), int(tune["sq_tile"]), 0)
    _check(lib().qdcb_tune_cache_store(path.encode(), key.encode(), ctypes.byref(t)))


def eri_quartets(A: Basis, B: Basis, idx) -> np.ndarray:
    idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, 4)
    out = np.empty(idx.shape[0])
    _check(lib().qdcb_eri_quartets(A.h, B.h, idx.shape[0], idx.ctypes.data_as(_IP),
                                   out.ctypes.data_as(_DP)))
    return out


NOALLOC_MAX_QUARTETS = 262144  # QDCB_NOALLOC_MAX_QUARTETS


def eri_quartets_noalloc(A: Basis, B: Basis, idx) -> np.ndarray:
    """eri_quartets through the allocation-free entry point (at most
    NOALLOC_MAX_QUARTETS quartets per call)."""
    idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, 4)
    out = np.empty(idx.shape[0])
    _check(lib().qdcb_eri_quartets_noalloc(A.h, B.h, idx.shape[0], idx.ctypes.data_as(_IP),
                                           out.ctypes.data_as(_DP)))
    return out


class Plan:
    def __init__(self, ctx: Context, L: Basis, S: Optional[Basis], ham: str, n_mo: int,
                 tau: float, prec: str = "fp64", tier_fp32: float = 1e-4,
                 tier_bf16: float = 1e-7, flags: int = 0):
        self.ctx, self.L, self.S = ctx, L, S
        self.n = int(n_mo)
        self.ham = ham
        self.spinor = bool(flags & PLAN_SPINOR)  # n_mo spinors, complex G [n]^4 x 2
        desc = PlanDesc(HAM[ham], PREC[prec], self.n, int(flags), float(tau), float(tier_fp32),
                        float(tier_bf16))
        h = _P()
        _check(lib().qdcb_plan_create(ctx.h, L.h, S.h if S is not None else None,
                                      ctypes.byref(desc), ctypes.byref(h)))
        self.h = h

    def g_shape(self):
        n = self.n
        return (n, n, n, n, 2) if self.spinor else (n, n, n, n, 4, 4)

    def footprint(self) -> int:
        b = ctypes.c_size_t(0)
        _check(lib().qdcb_plan_footprint(self.h, ctypes.byref(b)))
        return int(b.value)

    @staticmethod
    def estimate(L: Basis, S: Optional[Basis], ham: str, n_mo: int, tau: float = 0.0,
                 prec: str = "fp64") -> int:
        desc = PlanDesc(HAM[ham], PREC[prec], int(n_mo), 0, float(tau), 1e-4, 1e-7)
        b = ctypes.c_size_t(0)
        _check(lib().qdcb_plan_estimate(L.h, S.h if S is not None else None, ctypes.byref(desc),
                                        ctypes.byref(b)))
        return int(b.value)

    def transform(self, CL, CS=None, G=None, stream=None, classes=None):
        """Returns (G, stats).  numpy inputs use the host path; torch CUDA
        tensors the device path (G must then be a CUDA float64 tensor or None).
        classes: None (all), "coulomb", "gaunt", "gauge" or "breit" (Gaunt + gauge)."""
        n = self.n
        st = Stats()
        cf = CLASSES[classes]
        if _is_torch_cuda(CL):
            import torch
            if G is None:
                G = torch.empty(self.g_shape(), dtype=torch.float64, device=CL.device)
            for t in (CL, CS, G):
                if t is not None and (t.dtype != torch.float64 or not t.is_contiguous()):
                    raise ValueError("device tensors must be contiguous float64")
            if stream is None:
                stream = torch.cuda.current_stream(CL.device).cuda_stream
            _check(lib().qdcb_transform(self.h, CL.data_ptr(),
                                        CS.data_ptr() if CS is not None else None,
                                        G.data_ptr(), PTR_DEVICE | cf, stream, ctypes.byref(st)))
            return G, st.as_dict()
        CLh = _f64(CL)
        CSh = _f64(CS) if CS is not None else None
        if G is None:
            G = np.empty(self.g_shape())
        _check(lib().qdcb_transform(self.h, CLh.ctypes.data,
                                    CSh.ctypes.data if CSh is not None else None,
                                    G.ctypes.data, cf, stream, ctypes.byref(st)))
        return G, st.as_dict()

    def transform_blocks(self, CL, CS, callback, stream=None, classes=None):
        """Blocked output: callback(i0, i1, B) for consecutive blocks of MO pairs
        (r <= s, r outer).  numpy inputs: B is a host array [i1 - i0][n][n][2][4][4]
        (a view valid during the call; [..., 0, :, :] = G_pqrs, [..., 1, :, :] =
        G_pqsr).  torch CUDA inputs: B is the integer device address of that
        array.  A truthy return value stops the transformation (QdcbError
        E_ABORTED).  Returns stats."""
        n = self.n
        st = Stats()
        cf = CLASSES[classes]
        dev = _is_torch_cuda(CL)
        err = []

        def cb(user, i0, i1, ptr, on_device):
            try:
                if on_device:
                    stop = callback(int(i0), int(i1), int(ptr))
                else:
                    cnt = (i1 - i0) * n * n * 32
                    arr = np.ctypeslib.as_array(ctypes.cast(ptr, _DP), shape=(cnt,))
                    stop = callback(int(i0), int(i1), arr.reshape(i1 - i0, n, n, 2, 4, 4))
                return 1 if stop else 0
            except BaseException as e:  # reported after the call
                err.append(e)
                return 1

        fn = BLOCK_CB(cb)
        if dev:
            import torch
            if stream is None:
                stream = torch.cuda.current_stream(CL.device).cuda_stream
            st_code = lib().qdcb_transform_blocks(self.h, CL.data_ptr(),
                                                  CS.data_ptr() if CS is not None else None,
                                                  fn, None, PTR_DEVICE | cf, stream,
                                                  ctypes.byref(st))
        else:
            CLh = _f64(CL)
            CSh = _f64(CS) if CS is not None else None
            st_code = lib().qdcb_transform_blocks(self.h, CLh.ctypes.data,
                                                  CSh.ctypes.data if CSh is not None else None,
                                                  fn, None, cf, stream, ctypes.byref(st))
        if err:
            raise err[0]
        _check(st_code)
        return st.as_dict()

    @property
    def tune(self) -> dict:
        t = Tune()
        _check(lib().qdcb_plan_get_tune(self.h, ctypes.byref(t)))
        return t.as_dict()

    @tune.setter
    def tune(self, d: dict):
        cur = self.tune
        cur.update(d)
        t = Tune(int(cur["eri_sched"]), int(cur["fh_order"]), int(cur["sq_tile"]), 0)
        _check(lib().qdcb_plan_set_tune(self.h, ctypes.byref(t)))

    def set_mo_batch(self, pairs: int):
        """MO-driven variant: batches of ``pairs`` MO pairs, each screened with
        its own density bound (0: the AO-driven transformation)."""
        _check(lib().qdcb_plan_set_mo_batch(self.h, int(pairs)))

    def tune_key(self) -> str:
        buf = ctypes.create_string_buffer(512)
        _check(lib().qdcb_plan_tune_key(self.h, buf, len(buf)))
        return buf.value.decode()

    def autotune(self, CL, CS=None, G=None, stream=None, cache: Optional[str] = None) -> dict:
        """Pick the plan's launch choices by timing them on these coefficients
        (or take them from the cache file); G is scratch.  Returns the report."""
        n = self.n
        rep = TuneReport()
        path = cache.encode() if cache else None
        if _is_torch_cuda(CL):
            import torch
            if G is None:
                G = torch.empty(self.g_shape(), dtype=torch.float64, device=CL.device)
            if stream is None:
                stream = torch.cuda.current_stream(CL.device).cuda_stream
            _check(lib().qdcb_plan_autotune(self.h, CL.data_ptr(),
                                            CS.data_ptr() if CS is not None else None,
                                            G.data_ptr(), PTR_DEVICE, stream, path,
                                            ctypes.byref(rep)))
            return rep.as_dict()
        CLh = _f64(CL)
        CSh = _f64(CS) if CS is not None else None
        if G is None:
            G = np.empty(self.g_shape())
        _check(lib().qdcb_plan_autotune(self.h, CLh.ctypes.data,
                                        CSh.ctypes.data if CSh is not None else None,
                                        G.ctypes.data, 0, stream, path, ctypes.byref(rep)))
        return rep.as_dict()

    def capture(self, CL, CS, G, stream):
        """Record the transformation of the device tensors CL, CS -> G into a
        HIP graph on ``stream`` (a torch.cuda.Stream, not the null stream)."""
        for t in (CL, CS, G):
            if t is not None and not _is_torch_cuda(t):
                raise ValueError("capture needs device tensors")
        self._graph_bufs = (CL, CS, G)  # keep the recorded buffers alive
        _check(lib().qdcb_plan_capture(self.h, CL.data_ptr(),
                                       CS.data_ptr() if CS is not None else None, G.data_ptr(),
                                       stream.cuda_stream))

    def replay(self, stream):
        st = Stats()
        _check(lib().qdcb_plan_replay(self.h, stream.cuda_stream, ctypes.byref(st)))
        return st.as_dict()

    def fetch(self, what: int, count: int) -> np.ndarray:
        out = np.empty(count)
        _check(lib().qdcb_plan_fetch(self.h, int(what), out.ctypes.data, out.nbytes))
        return out

    def fetch_v(self, pairs) -> np.ndarray:
        """First-half rows of the last transform for the given bra pairs
        (concatenated LL, SS, LS indexing), quaternion components."""
        idx = np.ascontiguousarray(pairs, dtype=np.int64)
        npair = self.n * (self.n + 1) // 2
        out = np.empty((idx.shape[0], (3 if self.ham in ("DCG", "DCB") else 1) * 4 * npair))
        _check(lib().qdcb_plan_fetch_v(self.h, idx.ctypes.data, int(idx.shape[0]),
                                       out.ctypes.data))
        return out

    def close(self):
        if self.h:
            lib().qdcb_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
