"""Elementwise a-priori error bound of the mixed-precision first half (test
infrastructure; independent of the GPU library).

A kept directed contribution c = (bra pair b <- ket pair k) runs in a reduced
tier only if its tile's bound is below that tier's threshold.  The tile bound
is at least the contribution's own bound,
    beta_c = Q_b * Q_k * Dmax_k                   (screening-bound rule)
    beta_c = Q_b * Dmax_b * Q_k * Dmax_k          (G-bound rule),
so a contribution with beta_c >= t32 is always FP64, one with beta_c >= t16 is
at worst FP32, and any other at worst BF16.  Its rounding error is then at most
eps(c) |I_bk| |D_k, col|, with eps the relative error of one product of
operands rounded to the tier's format (2 u_op + u_op^2; FP32 u = 2^-24, BF16
u = 2^-8, plus the FP64 -> FP32 step before BF16) and of its FP32 accumulation
(at most 64 ket rows of one task and one addition per task into the running
FP32 sum: gamma(64 + T) with T the number of ket tiles).  The power-of-2 block
scales are exact.  The first-half error of a column is therefore
    |dV_b,col| <= E_b,col = sum_k eps(c) |I_bk| |D_k,col|,
and the second half carries it into G through the bra-side pair densities,
    |dG^{xy}_{pqrs}| <= sum_b |D_b,pq,x| E_b,(rs,y)          (Coulomb)
                        + sum_K sum_b |D^K_b,pq,x| E^K_b,(rs,y)  (Gaunt),
which is what bound() returns (for r <= s; G_pqsr follows by the sign rule).

Densities: D_b,pq = conj(C_mu p) C_nu q + conj(C_nu p) C_mu q for mu < nu (one
term for mu = nu), the symmetrized quaternion pair density; Gaunt
D^K_b,pq = conj(C^L_mu p) e_K C^S_nu q + conj(C^S_nu p) e_K C^L_mu q with
e_x, e_y, e_z = k, j, i.  ERIs, Schwarz factors and density bounds come from
the oracle.
"""
import numpy as np

import oracle
from tests import qalg

U32 = 2.0 ** -24
U16 = 2.0 ** -8
E_UNITS = np.array([[0.0, 0.0, 0.0, 1.0], [0.0, 0.0, 1.0, 0.0], [0.0, 1.0, 0.0, 0.0]])


def _gamma(k):
    return k * U32 / (1.0 - k * U32)


def tier_eps(n_ket_tiles):
    acc = _gamma(64 + n_ket_tiles)
    d16 = U16 + U32 + U16 * U32  # FP64 -> FP32 -> BF16, round to nearest
    return 2 * U32 + U32 * U32 + acc, 2 * d16 + d16 * d16 + acc


def _pairs(N):
    return [(mu, nu) for nu in range(N) for mu in range(nu + 1)]


def coulomb_density(C, pairs):
    """D[b, p, q, x] for unordered pairs b = (mu <= nu)."""
    mu = np.array([p[0] for p in pairs])
    nu = np.array([p[1] for p in pairs])
    a = qalg.qconj(C[:, mu, :])[:, :, :, None]   # (4, P, n, 1)
    b = C[:, nu, :][:, :, None, :]               # (4, P, 1, n)
    D = qalg.qmul(a, b)
    a2 = qalg.qconj(C[:, nu, :])[:, :, :, None]
    b2 = C[:, mu, :][:, :, None, :]
    D2 = qalg.qmul(a2, b2)
    D = D + np.where((mu != nu)[None, :, None, None], D2, 0.0)
    return np.moveaxis(D, 0, -1)  # (P, n, n, 4)


def gaunt_density(CL, CS):
    """D^K[K, b, p, q, x] for ordered L-S pairs b = mu * N_S + nu."""
    NL, NS, n = CL.shape[1], CS.shape[1], CL.shape[2]
    out = np.empty((3, NL * NS, n, n, 4))
    for K in range(3):
        e = E_UNITS[K].reshape(4, 1, 1)
        lr = qalg.qmul(qalg.qconj(CL), e)  # conj(C^L_mu p) e_K: (4, NL, n)
        sr = qalg.qmul(qalg.qconj(CS), e)
        t1 = qalg.qmul(lr[:, :, None, :, None], CS[:, None, :, None, :])  # (4, NL, NS, n, n)
        t2 = qalg.qmul(sr[:, None, :, :, None], CL[:, :, None, None, :])
        out[K] = np.moveaxis((t1 + t2).reshape(4, NL * NS, n, n), 0, -1)
    return out


def _contribution_eps(Qb, Db, Qk, Dk, tau, rule, t32, t16, n_ket_tiles):
    e32, e16 = tier_eps(n_ket_tiles)
    kept = (Qb[:, None] * Qk[None, :]) * Dk[None, :] >= tau
    if rule == "g":
        beta = (Qb * Db)[:, None] * (Qk * Dk)[None, :]
    else:
        beta = Qb[:, None] * (Qk * Dk)[None, :]
    eps = np.where(beta < t16, e16, np.where(beta < t32, e32, 0.0))
    return np.where(kept, eps, 0.0)


def _coulomb_space(s, CL, CS):
    """Pair densities, Schwarz factors, density bounds and the ERI matrix of
    the Coulomb space (LL pairs, then SS pairs)."""
    spaces = [(s.L, CL)]
    if CS is not None and s.S is not None and s.ham != "LL":
        spaces.append((s.S, CS))
    idx, D, Q, Dm = [], [], [], []
    for B, C in spaces:
        pl = _pairs(B.nfunc)
        a = np.array([x for x, _ in pl])
        b = np.array([y for _, y in pl])
        idx.append((a, b))
        D.append(coulomb_density(C, pl))
        Q.append(oracle.schwarz(B)[a, b])
        Dm.append(oracle.dmax_coulomb(C)[a, b])
    rows = []
    for (ba, bb), (BA, _) in zip(idx, spaces):
        row = []
        for (ka, kb), (KB, _) in zip(idx, spaces):
            T = oracle.eri_tensor(BA, BA, KB, KB)
            row.append(T[ba[:, None], bb[:, None], ka[None, :], kb[None, :]])
        rows.append(row)
    return np.concatenate(D), np.concatenate(Q), np.concatenate(Dm), np.block(rows)


def _gaunt_space(s, CL, CS):
    NL, NS = s.L.nfunc, s.S.nfunc
    return (gaunt_density(CL, CS), oracle.schwarz(s.L, s.S).reshape(-1),
            oracle.dmax_gaunt(CL, CS).reshape(-1),
            oracle.eri_tensor(s.L, s.S, s.L, s.S).reshape(NL * NS, NL * NS))


def _spaces(s, CL, CS):
    out = [(_coulomb_space(s, CL, CS), False)]
    if s.ham in ("DCG", "DCB"):
        out.append((_gaunt_space(s, CL, CS), True))
    return out


def _rs(n):
    rs = [(r, t) for r in range(n) for t in range(r, n)]
    return np.array([a for a, _ in rs]), np.array([b for _, b in rs])


def _contract(bra_D, W, ket_D, n):
    """sum_b |bra| (W @ |ket|) or the signed product, as [n][n][npair][4][4]."""
    ri, ti = _rs(n)
    P = bra_D.shape[0]
    ket = ket_D[:, ri, ti, :].reshape(P, -1)
    bra = bra_D.reshape(P, n * n * 4)
    return (bra.T @ (W @ ket)).reshape(n, n, 4, len(ri), 4).transpose(0, 1, 3, 2, 4)


def bound(s, CL, CS, tau, rule, t32, t16):
    """Elementwise bound on |G_mixed - G_FP64| for r <= s, shape
    [n][n][npair][4][4] (p, q, pair index of r <= s with r outer, x, y)."""
    n = CL.shape[2]
    out = 0.0
    for (D, Q, Dm, I), gaunt in _spaces(s, CL, CS):
        eps = _contribution_eps(Q, Dm, Q, Dm, tau, rule, t32, t16, (Q.shape[0] + 63) // 64)
        W = eps * np.abs(I)
        for Dk in (D if gaunt else [D]):
            out = out + _contract(np.abs(Dk), W, np.abs(Dk), n)
    return out


def model(s, CL, CS, tau, rule="g", t32=0.0, t16=0.0, rounding=None):
    """G (r <= s) from the same pieces, G = sum D^T (I o keep) D per space; with
    rounding = (f32, f16), the integral and density operands of contributions
    with beta_c below the tier thresholds are passed through those rounding
    functions (a model of the reduced tiers; products and sums in FP64)."""
    n = CL.shape[2]
    out = 0.0
    for (D, Q, Dm, I), gaunt in _spaces(s, CL, CS):
        keep = (Q[:, None] * Q[None, :]) * Dm[None, :] >= tau
        Ik = np.where(keep, I, 0.0)
        for Dk in (D if gaunt else [D]):
            if rounding is None:
                out = out + _contract(Dk, Ik, Dk, n)
                continue
            if rule == "g":
                beta = (Q * Dm)[:, None] * (Q * Dm)[None, :]
            else:
                beta = Q[:, None] * (Q * Dm)[None, :]
            ri, ti = _rs(n)
            ket = Dk[:, ri, ti, :].reshape(Dk.shape[0], -1)
            V = np.zeros((Dk.shape[0], ket.shape[1]))
            for tier, f in ((1, rounding[0]), (2, rounding[1])):
                sel = (beta < t16) if tier == 2 else ((beta >= t16) & (beta < t32))
                Ir = f(np.where(sel, Ik, 0.0))
                V += Ir @ f(ket)
            V += np.where(beta >= t32, Ik, 0.0) @ ket
            bra = Dk.reshape(Dk.shape[0], n * n * 4)
            out = out + (bra.T @ V).reshape(n, n, 4, len(ri), 4).transpose(0, 1, 3, 2, 4)
    return out


def upper_part(G):
    """G[p][q][r][s][x][y] restricted to r <= s: [n][n][npair][4][4]."""
    n = G.shape[0]
    rs = [(r, t) for r in range(n) for t in range(r, n)]
    return np.stack([G[:, :, r, t] for r, t in rs], axis=2)
