"""Python access to the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it as the correctness reference.  The GPU library never
imports, links or calls anything here, and nothing here imports the GPU
library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
HAMS = {"LL": 0, "DC": 1, "DCG": 2, "GAUNT": 3, "DCB": 4, "GAUGE": 5}
# hams with L-S (Gaunt-class) rows
LS_HAMS = ("DCG", "GAUNT", "DCB", "GAUGE")


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (no FMA contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wno-unused-variable",
           os.path.join(_HERE, "oracle.c"), "-o", _SO + ".tmp", "-lm"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def build_sanitized() -> str:
    """CPU check build: oracle.c with AddressSanitizer and
    UndefinedBehaviorSanitizer, linked into sanitize_check (a driver of every
    entry point on a tiny system).  Returns the executable's path."""
    out = os.path.join(_HERE, "_build_san")
    os.makedirs(out, exist_ok=True)
    exe = os.path.join(out, "sanitize_check")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-Wall",
           "-Wno-unused-variable", "-I", _HERE, os.path.join(_HERE, "sanitize_check.c"),
           os.path.join(_HERE, "oracle.c"), "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


class _Basis(ctypes.Structure):
    _fields_ = [("nfunc", ctypes.c_int32),
                ("centers", ctypes.POINTER(ctypes.c_double)),
                ("nprim", ctypes.POINTER(ctypes.c_int32)),
                ("exps", ctypes.POINTER(ctypes.c_double)),
                ("coefs", ctypes.POINTER(ctypes.c_double)),
                ("cart", ctypes.POINTER(ctypes.c_int32))]


class Stats(ctypes.Structure):
    _fields_ = [("kept", ctypes.c_int64 * 4), ("total", ctypes.c_int64 * 4),
                ("kept_gaunt", ctypes.c_int64), ("total_gaunt", ctypes.c_int64),
                ("tie_band", ctypes.c_int64),
                ("seconds_first_half", ctypes.c_double),
                ("seconds_second_half", ctypes.c_double),
                ("threads", ctypes.c_int32)]

    def as_dict(self):
        return {"kept": list(self.kept), "total": list(self.total),
                "kept_gaunt": self.kept_gaunt, "total_gaunt": self.total_gaunt,
                "tie_band": self.tie_band, "seconds_first_half": self.seconds_first_half,
                "seconds_second_half": self.seconds_second_half, "threads": self.threads}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        bp = ctypes.POINTER(_Basis)
        L.orc_boys0.restype = ctypes.c_double
        L.orc_boys0.argtypes = [ctypes.c_double]
        L.orc_boys.restype = ctypes.c_double
        L.orc_boys.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc_eri3.argtypes = [bp, ctypes.c_int, bp, ctypes.c_int, bp, ctypes.c_int, bp,
                               ctypes.c_int, dp]
        L.orc_norm_coefs.argtypes = [bp, dp]
        L.orc_prim_eri_cart.restype = ctypes.c_double
        L.orc_prim_eri_cart.argtypes = [ctypes.c_double, dp, ctypes.c_int] * 4
        L.orc_prim_eri3_cart.argtypes = [ctypes.c_double, dp, ctypes.c_int] * 4 + [dp]
        L.orc_eri.restype = ctypes.c_double
        L.orc_eri.argtypes = [bp, ctypes.c_int, ctypes.c_int, bp, ctypes.c_int, ctypes.c_int]
        L.orc_eri_tensor.argtypes = [bp, bp, bp, bp, dp]
        L.orc_schwarz.argtypes = [bp, bp, dp]
        L.orc_dmax_coulomb.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp]
        L.orc_dmax_gaunt.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int, dp]
        L.orc_transform_def.restype = ctypes.c_int
        L.orc_transform_def.argtypes = [bp, bp, dp, dp, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.orc_transform_direct.restype = ctypes.c_int
        L.orc_transform_direct.argtypes = [bp, bp, dp, dp, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_double, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_int, dp, ctypes.POINTER(Stats)]
        L.orc_first_half_rows.restype = ctypes.c_int
        L.orc_first_half_rows.argtypes = [bp, bp, dp, dp, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_void_p, ctypes.c_int64, dp]
        L.orc_first_half_rows_cols.restype = ctypes.c_int
        L.orc_first_half_rows_cols.argtypes = [bp, bp, dp, dp, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_double, ctypes.c_void_p, ctypes.c_int64,
                                               ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                               dp]
        L.orc_transform_spinor_def.restype = ctypes.c_int
        L.orc_transform_spinor_def.argtypes = [bp, bp, dp, dp, ctypes.c_int, ctypes.c_int, dp]
        L.orc_transform_spinor_direct.restype = ctypes.c_int
        L.orc_transform_spinor_direct.argtypes = [bp, bp, dp, dp, ctypes.c_int, ctypes.c_int,
                                                  ctypes.c_double, dp, ctypes.POINTER(Stats)]
        L.orc_transform_direct_dmax.restype = ctypes.c_int
        L.orc_transform_direct_dmax.argtypes = [bp, bp, dp, dp, ctypes.c_int, ctypes.c_int,
                                                ctypes.c_double, dp, dp, ctypes.POINTER(Stats)]
        L.orc_num_bra_pairs.restype = ctypes.c_int64
        L.orc_num_bra_pairs.argtypes = [bp, bp, ctypes.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class _B:
    """Keeps the numpy buffers of a basis alive next to its ctypes struct."""

    def __init__(self, b):
        self.centers = np.ascontiguousarray(b.centers, dtype=np.float64)
        self.nprim = np.ascontiguousarray(b.nprim, dtype=np.int32)
        self.exps = np.ascontiguousarray(b.exps, dtype=np.float64)
        self.coefs = np.ascontiguousarray(b.coefs, dtype=np.float64)
        cart = getattr(b, "cart", None)
        self.cart = None if cart is None else np.ascontiguousarray(cart, dtype=np.int32)
        ip = ctypes.POINTER(ctypes.c_int32)
        self.s = _Basis(int(self.nprim.shape[0]), _dp(self.centers),
                        self.nprim.ctypes.data_as(ip), _dp(self.exps), _dp(self.coefs),
                        self.cart.ctypes.data_as(ip) if self.cart is not None else ip())

    @property
    def ref(self):
        return ctypes.byref(self.s)


def boys0(T: float) -> float:
    return lib().orc_boys0(float(T))


def boys(m: int, T: float) -> float:
    return lib().orc_boys(int(m), float(T))


def prim_eri_cart(a, A, ca, b, B, cb, c, C, cc, d, D, cd) -> float:
    """[ab|cd] over unnormalized Cartesian primitives (centre, exponent,
    code 0 = s, 1..3 = p_x, p_y, p_z), by the Obara-Saika recursion."""
    args = []
    for e, X, k in ((a, A, ca), (b, B, cb), (c, C, cc), (d, D, cd)):
        X = np.ascontiguousarray(X, dtype=np.float64)
        args += [float(e), _dp(X), int(k)]
        args.append(X)  # keep alive
    keep = args[3::4]
    call = [x for i, x in enumerate(args) if i % 4 != 3]
    v = lib().orc_prim_eri_cart(*call)
    del keep
    return v


def prim_eri3_cart(a, A, ca, b, B, cb, c, C, cc, d, D, cd) -> np.ndarray:
    """[ab| r_K r_L / r^3 |cd] over unnormalized Cartesian primitives (codes as
    prim_eri_cart), as a 3 x 3 array [K][L], McMurchie-Davidson form."""
    keep, call = [], []
    for e, X, k in ((a, A, ca), (b, B, cb), (c, C, cc), (d, D, cd)):
        X = np.ascontiguousarray(X, dtype=np.float64)
        keep.append(X)
        call += [float(e), _dp(X), int(k)]
    out = np.zeros(9)
    lib().orc_prim_eri3_cart(*call, _dp(out))
    return out.reshape(3, 3)


def eri3(A, mu, B, nu, C, ka, D, la) -> np.ndarray:
    """(mu^A nu^B | r_K r_L / r^3 | ka^C la^D) as a 3 x 3 array [K][L]."""
    a, b, c, d = _B(A), _B(B), _B(C), _B(D)
    out = np.zeros(9)
    lib().orc_eri3(a.ref, int(mu), b.ref, int(nu), c.ref, int(ka), d.ref, int(la), _dp(out))
    return out.reshape(3, 3)


def norm_coefs(b) -> np.ndarray:
    B = _B(b)
    out = np.empty_like(B.coefs)
    lib().orc_norm_coefs(B.ref, _dp(out))
    return out


def eri(A, mu, nu, B, ka, la) -> float:
    a, b = _B(A), _B(B)
    return lib().orc_eri(a.ref, mu, nu, b.ref, ka, la)


def eri_tensor(A, B=None, C=None, D=None) -> np.ndarray:
    B = A if B is None else B
    C = A if C is None else C
    D = C if D is None else D
    bs = [_B(x) for x in (A, B, C, D)]
    out = np.empty((A.nfunc, B.nfunc, C.nfunc, D.nfunc))
    lib().orc_eri_tensor(bs[0].ref, bs[1].ref, bs[2].ref, bs[3].ref, _dp(out))
    return out


def schwarz(A, B=None) -> np.ndarray:
    B = A if B is None else B
    a, b = _B(A), _B(B)
    out = np.empty((A.nfunc, B.nfunc))
    lib().orc_schwarz(a.ref, b.ref, _dp(out))
    return out


def dmax_coulomb(C: np.ndarray) -> np.ndarray:
    C = np.ascontiguousarray(C, dtype=np.float64)
    N, n = C.shape[1], C.shape[2]
    out = np.empty((N, N))
    lib().orc_dmax_coulomb(N, _dp(C), n, _dp(out))
    return out


def dmax_gaunt(CL: np.ndarray, CS: np.ndarray) -> np.ndarray:
    CL = np.ascontiguousarray(CL, dtype=np.float64)
    CS = np.ascontiguousarray(CS, dtype=np.float64)
    NL, NS, n = CL.shape[1], CS.shape[1], CL.shape[2]
    out = np.empty((NL, NS))
    lib().orc_dmax_gaunt(NL, _dp(CL), NS, _dp(CS), n, _dp(out))
    return out


def _prep(L, S, CL, CS):
    bl = _B(L)
    bs = _B(S) if S is not None else None
    CL = np.ascontiguousarray(CL, dtype=np.float64)
    CS = np.ascontiguousarray(CS, dtype=np.float64) if CS is not None else None
    return bl, bs, CL, CS


def transform_def(L, S, CL, CS, ham: str = "LL", return_spinor: bool = False):
    """Unscreened definition route (literal four-spinor operators)."""
    bl, bs, CL, CS = _prep(L, S, CL, CS)
    n = CL.shape[2]
    G = np.zeros((n, n, n, n, 4, 4))
    sp = np.zeros((2 * n,) * 4 + (2,)) if return_spinor else None
    im = ctypes.c_double(0.0)
    rc = lib().orc_transform_def(bl.ref, bs.ref if bs else None, _dp(CL),
                                 _dp(CS) if CS is not None else None, n, HAMS[ham], _dp(G),
                                 _dp(sp) if sp is not None else None, ctypes.byref(im))
    if rc != 0:
        raise ValueError("orc_transform_def rejected the problem (too large or invalid)")
    if return_spinor:
        return G, sp[..., 0] + 1j * sp[..., 1], im.value
    return G, im.value


def transform_spinor_def(L, S, CL, CS, ham: str = "LL") -> np.ndarray:
    """General two-spinor input (planes [4][N][m]: alpha re, alpha im, beta re,
    beta im): unscreened definition route, complex (ab|cd) [m]^4."""
    bl, bs, CL, CS = _prep(L, S, CL, CS)
    m = CL.shape[2]
    sp = np.zeros((m,) * 4 + (2,))
    rc = lib().orc_transform_spinor_def(bl.ref, bs.ref if bs else None, _dp(CL),
                                        _dp(CS) if CS is not None else None, m, HAMS[ham],
                                        _dp(sp))
    if rc != 0:
        raise ValueError("orc_transform_spinor_def rejected the problem")
    return sp[..., 0] + 1j * sp[..., 1]


def transform_spinor(L, S, CL, CS, ham: str = "LL", tau: float = 0.0):
    """General two-spinor input: the paper's direct route with screening;
    returns (complex (ab|cd) [m]^4, stats)."""
    bl, bs, CL, CS = _prep(L, S, CL, CS)
    m = CL.shape[2]
    sp = np.zeros((m,) * 4 + (2,))
    st = Stats()
    rc = lib().orc_transform_spinor_direct(bl.ref, bs.ref if bs else None, _dp(CL),
                                           _dp(CS) if CS is not None else None, m, HAMS[ham],
                                           float(tau), _dp(sp), ctypes.byref(st))
    if rc != 0:
        raise ValueError("orc_transform_spinor_direct rejected the problem")
    return sp[..., 0] + 1j * sp[..., 1], st.as_dict()


def transform_direct(L, S, CL, CS, ham: str = "LL", tau: float = 0.0, rows=None,
                     second_half: bool = True):
    """The paper's screened direct route.  ``rows`` optionally restricts the
    bra pairs (indices into the concatenated LL, SS, LS pair list).
    Returns (G or None, stats dict)."""
    bl, bs, CL, CS = _prep(L, S, CL, CS)
    sel = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    n = CL.shape[2]
    G = np.zeros((n, n, n, n, 4, 4)) if second_half else None
    st = Stats()
    rc = lib().orc_transform_direct(bl.ref, bs.ref if bs else None, _dp(CL),
                                    _dp(CS) if CS is not None else None, n, HAMS[ham],
                                    float(tau), sel.ctypes.data if sel is not None else None,
                                    0 if sel is None else int(sel.shape[0]),
                                    1 if second_half else 0,
                                    _dp(G) if G is not None else None, ctypes.byref(st))
    if rc != 0:
        raise ValueError("orc_transform_direct rejected its arguments")
    return G, st.as_dict()


def first_half_rows(L, S, CL, CS, ham: str, tau: float, rows) -> np.ndarray:
    """First-half rows V of the selected bra pairs (indices into the
    concatenated LL, SS, LS pair list) in quaternion components, columns
    K * 4 * npair + 4 * idx(p <= q) + y (K blocks only with Gaunt)."""
    bl, bs, CL, CS = _prep(L, S, CL, CS)
    sel = np.ascontiguousarray(rows, dtype=np.int64)
    n = CL.shape[2]
    npair = n * (n + 1) // 2
    width = (3 if ham in LS_HAMS else 1) * 4 * npair
    Vq = np.zeros((sel.shape[0], width))
    rc = lib().orc_first_half_rows(bl.ref, bs.ref if bs else None, _dp(CL),
                                   _dp(CS) if CS is not None else None, n, HAMS[ham],
                                   float(tau), sel.ctypes.data, int(sel.shape[0]), _dp(Vq))
    if rc != 0:
        raise ValueError("orc_first_half_rows rejected its arguments")
    return Vq


def first_half_rows_cols(L, S, CL, CS, ham: str, tau: float, rows, cols,
                         dmax=None) -> np.ndarray:
    """first_half_rows for the MO pairs ``cols`` (indices of p <= q, p outer)
    only: columns K * 4 * len(cols) + 4 * j + y.  ``dmax`` (optional) is the
    density bound per pair of the concatenated LL, SS, LS list
    (pair_density_bounds); without it the bound is computed here."""
    bl, bs, CL, CS = _prep(L, S, CL, CS)
    sel = np.ascontiguousarray(rows, dtype=np.int64)
    cl = np.ascontiguousarray(cols, dtype=np.int64)
    width = (3 if ham in LS_HAMS else 1) * 4 * cl.shape[0]
    Vq = np.zeros((sel.shape[0], width))
    dm = None if dmax is None else np.ascontiguousarray(dmax, dtype=np.float64)
    rc = lib().orc_first_half_rows_cols(bl.ref, bs.ref if bs else None, _dp(CL),
                                        _dp(CS) if CS is not None else None, CL.shape[2],
                                        HAMS[ham], float(tau), sel.ctypes.data,
                                        int(sel.shape[0]), cl.ctypes.data, int(cl.shape[0]),
                                        dm.ctypes.data if dm is not None else None, _dp(Vq))
    if rc != 0:
        raise ValueError("orc_first_half_rows_cols rejected its arguments")
    return Vq


def pair_density_bounds(L, S, CL, CS, ham: str) -> np.ndarray:
    """Density bound Dmax of every pair of the concatenated bra pair list
    (LL pairs mu <= nu, nu-major, then SS pairs, then LS pairs mu-major) from
    the quaternion-route bounds dmax_coulomb and dmax_gaunt."""
    parts = []
    if ham not in ("GAUNT", "GAUGE"):
        for C in ((CL,) if ham == "LL" else (CL, CS)):
            D = dmax_coulomb(C)
            N = D.shape[0]
            iu = np.triu_indices(N)  # (mu, nu) with mu <= nu
            v = np.empty(N * (N + 1) // 2)
            v[iu[1] * (iu[1] + 1) // 2 + iu[0]] = D[iu[0], iu[1]]
            parts.append(v)
    if ham in LS_HAMS:
        parts.append(dmax_gaunt(CL, CS).reshape(-1))
    return np.concatenate(parts)


def num_bra_pairs(L, S, ham: str) -> int:
    bl = _B(L)
    bs = _B(S) if S is not None else None
    return int(lib().orc_num_bra_pairs(bl.ref, bs.ref if bs else None, HAMS[ham]))


# --------------------------------------------------------------------------
# MO-driven variant: per-batch density bound
# --------------------------------------------------------------------------

def _qconj_mul(a, b):
    """conj(a) b for quaternion arrays with the component on the first axis."""
    a0, a1, a2, a3 = a[0], -a[1], -a[2], -a[3]
    b0, b1, b2, b3 = b
    return np.array([a0 * b0 - a1 * b1 - a2 * b2 - a3 * b3,
                     a0 * b1 + a1 * b0 + a2 * b3 - a3 * b2,
                     a0 * b2 - a1 * b3 + a2 * b0 + a3 * b1,
                     a0 * b3 + a1 * b2 - a2 * b1 + a3 * b0])


_UNITS = {0: np.array([0.0, 0.0, 0.0, 1.0]),   # e_x = k
          1: np.array([0.0, 0.0, 1.0, 0.0]),   # e_y = j
          2: np.array([0.0, 1.0, 0.0, 0.0])}   # e_z = i


def _qmul(a, b):
    return _qconj_mul(a * np.array([1.0, -1.0, -1.0, -1.0]).reshape((4,) + (1,) * (a.ndim - 1)), b)


def dmax_batch(L, S, CL, CS, ham: str, mo_pairs) -> np.ndarray:
    """Density bound of one batch of quaternion MO pairs (r <= t), per pair of
    the concatenated bra list: for Coulomb pairs the largest |component| of
    conj(C_kr) C_lt and conj(C_lr) C_kt over the batch; for Gaunt (L-S) pairs
    of conj(C^L_mr) e_K C^S_nt + conj(C^S_nr) e_K C^L_mt over K and the batch
    (Eq. SchwarzDen restricted to the batch's MO pairs)."""
    out = []
    coul = ham in ("LL", "DC", "DCG", "DCB")
    gaunt = ham in LS_HAMS

    def coul_block(C):
        N = C.shape[1]
        M = np.zeros((N, N))
        for r, t in mo_pairs:
            d = _qconj_mul(C[:, :, r][:, :, None], C[:, :, t][:, None, :])  # [4][k][l]
            a = np.abs(d).max(axis=0)
            M = np.maximum(M, np.maximum(a, a.T))
        return np.array([M[mu, nu] for nu in range(N) for mu in range(nu + 1)])

    if coul:
        out.append(coul_block(CL))
        if ham != "LL":
            out.append(coul_block(CS))
    if gaunt:
        NL, NS = CL.shape[1], CS.shape[1]
        M = np.zeros((NL, NS))
        for r, t in mo_pairs:
            for K in range(3):
                e = _UNITS[K].reshape(4, 1, 1)
                lr = CL[:, :, r][:, :, None]
                st = CS[:, :, t][:, None, :]
                sr = CS[:, :, r][:, None, :]
                lt = CL[:, :, t][:, :, None]
                d = _qmul(_qconj_mul(lr, e), st) + _qmul(_qconj_mul(sr, e), lt)
                M = np.maximum(M, np.abs(d).max(axis=0))
        out.append(M.reshape(-1))
    return np.concatenate(out)


def transform_direct_mo(L, S, CL, CS, ham: str, tau: float, batch: int):
    """MO-driven variant of the direct route: the MO pairs (r <= t, r outer) in
    batches of ``batch``, each screened with its own density bound
    (dmax_batch); G of each batch's pairs (and their t, r mirrors) comes from
    that batch's screened transform.  Returns (G, stats with kept summed over
    the batches)."""
    bl, bs, CL, CS = _prep(L, S, CL, CS)
    n = CL.shape[2]
    pairs = [(r, t) for r in range(n) for t in range(r, n)]
    G = np.zeros((n, n, n, n, 4, 4))
    kept = np.zeros(4, dtype=np.int64)
    kept_g = 0
    for b0 in range(0, len(pairs), batch):
        bp = pairs[b0:b0 + batch]
        dm = np.ascontiguousarray(dmax_batch(L, S, CL, CS, ham, bp))
        Gb = np.zeros_like(G)
        st = Stats()
        rc = lib().orc_transform_direct_dmax(bl.ref, bs.ref if bs else None, _dp(CL),
                                             _dp(CS) if CS is not None else None, n, HAMS[ham],
                                             float(tau), _dp(dm), _dp(Gb), ctypes.byref(st))
        if rc != 0:
            raise ValueError("orc_transform_direct_dmax rejected the problem")
        for r, t in bp:
            G[:, :, r, t] = Gb[:, :, r, t]
            G[:, :, t, r] = Gb[:, :, t, r]
        kept += np.array(st.kept)
        kept_g += st.kept_gaunt
    return G, {"kept": [int(x) for x in kept], "kept_gaunt": int(kept_g)}
