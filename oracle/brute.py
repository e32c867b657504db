"""Brute-force O(N^8) spinor-integral sum in numpy (TEST INFRASTRUCTURE ONLY).

An independent second implementation for tiny bases: its own primitive
normalization, its own ERIs (scipy's erf rather than the C library's), and
the MO integrals as one unfactored sum over all AO and spinor indices of the
definitions in Eqs. (AOtoMO), (DCInt), (GauntInt), (gaugeInt) with the
four-spinor operators of Eq. (breit) and the alpha/Pauli matrices as printed
in Sec. 2.  The gauge term's r r^T / r^3 integrals take the Boys functions
F1, F2 from scipy's regularized incomplete gamma function.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf, gamma, gammainc

PAULI = [np.array([[0, 1], [1, 0]], dtype=complex),
         np.array([[0, -1j], [1j, 0]], dtype=complex),
         np.array([[1, 0], [0, -1]], dtype=complex)]


def alpha(K: int) -> np.ndarray:
    a = np.zeros((4, 4), dtype=complex)
    a[:2, 2:] = PAULI[K]
    a[2:, :2] = PAULI[K]
    return a


def qrep(q) -> np.ndarray:
    q0, q1, q2, q3 = q
    return np.array([[q0 + 1j * q1, q2 + 1j * q3], [-q2 + 1j * q3, q0 - 1j * q1]])


def _norm_prims(b):
    off = np.concatenate([[0], np.cumsum(b.nprim)])
    funcs = []
    for f in range(b.nfunc):
        a = b.exps[off[f]:off[f + 1]]
        d = b.coefs[off[f]:off[f + 1]] * (2 * a / math.pi) ** 0.75
        s = np.sum(d[:, None] * d[None, :] * (math.pi / (a[:, None] + a[None, :])) ** 1.5)
        funcs.append((b.centers[f], a, d / math.sqrt(s)))
    return funcs


def _boys0(T):
    T = np.asarray(T, dtype=float)
    out = np.ones_like(T)
    big = T > 1e-13
    out[big] = 0.5 * np.sqrt(math.pi / T[big]) * erf(np.sqrt(T[big]))
    out[~big] = 1 - T[~big] / 3
    return out


def _boys(m, T):
    """F_m(T) = Gamma(m + 1/2) P(m + 1/2, T) / (2 T^(m + 1/2)), 1 / (2m + 1) at 0."""
    T = np.asarray(T, dtype=float)
    out = np.full_like(T, 1.0 / (2 * m + 1))
    big = T > 1e-13
    a = m + 0.5
    out[big] = gamma(a) * gammainc(a, T[big]) / (2 * T[big] ** a)
    return out


def eri_tensor(funcs, kernel3: bool = False) -> np.ndarray:
    """Contracted (ij|kl); kernel3: the r_K r_L / r^3 integrals [K][L][i][j][k][l]
    = 2 pi^{5/2} / (p q sqrt(p+q)) K_ab K_cd (delta_KL F1 + 2 rho R_K R_L (F1 - F2))
    summed over primitives, R = P - Q."""
    n = len(funcs)
    out = np.zeros((3, 3, n, n, n, n) if kernel3 else (n, n, n, n))
    for i in range(n):
        A, a, ca = funcs[i]
        for j in range(n):
            B, b, cb = funcs[j]
            p = a[:, None] + b[None, :]
            P = (a[:, None, None] * A + b[None, :, None] * B) / p[..., None]
            Kab = np.exp(-a[:, None] * b[None, :] / p * np.sum((A - B) ** 2))
            cab = ca[:, None] * cb[None, :] * Kab
            for k in range(n):
                C, c, cc = funcs[k]
                for l in range(n):
                    D, d, cd = funcs[l]
                    q = c[:, None] + d[None, :]
                    Qc = (c[:, None, None] * C + d[None, :, None] * D) / q[..., None]
                    Kcd = np.exp(-c[:, None] * d[None, :] / q * np.sum((C - D) ** 2))
                    ccd = cc[:, None] * cd[None, :] * Kcd
                    pp = p[:, :, None, None]
                    qq = q[None, None, :, :]
                    Rv = P[:, :, None, None, :] - Qc[None, None, :, :, :]
                    R2 = np.sum(Rv ** 2, axis=-1)
                    rho = pp * qq / (pp + qq)
                    T = rho * R2
                    pref = 2 * math.pi ** 2.5 / (pp * qq * np.sqrt(pp + qq))
                    w = cab[:, :, None, None] * ccd[None, None]
                    if not kernel3:
                        out[i, j, k, l] = np.sum(w * pref * _boys0(T))
                        continue
                    F1, F2 = _boys(1, T), _boys(2, T)
                    for K in range(3):
                        for L in range(3):
                            v = (K == L) * F1 + 2 * rho * Rv[..., K] * Rv[..., L] * (F1 - F2)
                            out[K, L, i, j, k, l] = np.sum(w * pref * v)
    return out


def levi(i, j, k) -> int:
    return (i - j) * (j - k) * (k - i) // 2


def spinor4(CL, CS):
    """Four-spinor coefficients c4[f, w, a]: L functions on components 0,1,
    S functions on components 2,3; spinors 2p, 2p+1 are the columns of Q(C)."""
    n = CL.shape[2]
    NL = CL.shape[1]
    NS = CS.shape[1] if CS is not None else 0
    c4 = np.zeros((NL + NS, 4, 2 * n), dtype=complex)
    for mu in range(NL + NS):
        X, off, idx = (CL, 0, mu) if mu < NL else (CS, 2, mu - NL)
        for p in range(n):
            M = qrep(X[:, idx, p])
            c4[mu, off:off + 2, 2 * p:2 * p + 2] = M
    return c4


def spinor4_general(CL, CS):
    """Four-spinor coefficients c4[f, w, a] of general spinors given as planes
    [4][N][m] (alpha re, alpha im, beta re, beta im)."""
    m = CL.shape[2]
    NL = CL.shape[1]
    NS = CS.shape[1] if CS is not None else 0
    c4 = np.zeros((NL + NS, 4, m), dtype=complex)
    c4[:NL, 0] = CL[0] + 1j * CL[1]
    c4[:NL, 1] = CL[2] + 1j * CL[3]
    if NS:
        c4[NL:, 2] = CS[0] + 1j * CS[1]
        c4[NL:, 3] = CS[2] + 1j * CS[3]
    return c4


def spinor_integrals(L, S, CL, CS, ham: str, general: bool = False) -> np.ndarray:
    """(ab|cd) as one sum over all AO and spinor indices; general: CL, CS are
    general two-spinor planes instead of quaternion coefficients."""
    funcs = _norm_prims(L) + (_norm_prims(S) if ham != "LL" else [])
    eri = eri_tensor(funcs)
    make = spinor4_general if general else spinor4
    c4 = make(CL, CS if ham != "LL" else None)
    cc = c4.conj()
    out = 0
    if ham in ("LL", "DC", "DCG", "DCB"):
        out = out + np.einsum("iwa,jwb,ijkl,kvc,lvd->abcd", cc, c4, eri, cc, c4, optimize=False)
    if ham in ("DCB", "GAUGE"):
        # (alpha_1 x r) . (alpha_2 x r) / (2 r^3), the cross products by components
        e3 = eri_tensor(funcs, kernel3=True)
        for j in range(3):
            for l in range(3):
                N = 0
                for i in range(3):
                    for k in range(3):
                        for k2 in range(3):
                            if levi(i, j, k) and levi(i, l, k2):
                                N = N + 0.5 * levi(i, j, k) * levi(i, l, k2) * e3[k, k2]
                out = out + np.einsum("iwa,wu,jub,ijkl,kvc,vt,ltd->abcd", cc, alpha(j), c4, N,
                                      cc, alpha(l), c4, optimize=False)
    if ham in ("DCG", "GAUNT", "DCB"):
        for K in range(3):
            aK = alpha(K)
            out = out - np.einsum("iwa,wu,jub,ijkl,kvc,vt,ltd->abcd", cc, aK, c4, eri, cc, aK,
                                  c4, optimize=False)
    return out


def project(sp: np.ndarray) -> np.ndarray:
    """G^{xy}_{pqrs} = 1/4 sum conj(Q(e_x)_{a'b'}) conj(Q(e_y)_{c'd'}) (2p+a' 2q+b'|2r+c' 2s+d')."""
    m = sp.shape[0]
    n = m // 2
    E = [qrep(np.eye(4)[x]) for x in range(4)]
    blk = sp.reshape(n, 2, n, 2, n, 2, n, 2)
    G = np.zeros((n, n, n, n, 4, 4))
    for x in range(4):
        for y in range(4):
            G[..., x, y] = 0.25 * np.einsum("ab,cd,paqbrcsd->pqrs", E[x].conj(), E[y].conj(),
                                            blk).real
    return G


def transform(L, S, CL, CS, ham: str = "LL"):
    sp = spinor_integrals(L, S, CL, CS, ham)
    return project(sp), sp
