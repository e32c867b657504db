"""Seeded synthetic inputs for the quaternion AO->MO transformation.

This module only *constructs inputs*: atom positions, s-type contracted
Gaussian basis sets, and quaternion MO coefficient matrices.  It holds none of
the transformation's arithmetic (no two-electron integrals, densities,
screening or contractions) and imports neither the GPU binding nor the
oracle, so both sides can take their inputs from it.

Basis convention shared by every consumer (the C-ABI and the oracle):
``coefs`` multiply *normalized* primitives (2a/pi)^{3/4} exp(-a r^2), and the
contracted function is then rescaled to unit self-overlap.  The generator
needs that normalization itself only to build the overlap matrix S used for
Loewdin orthonormalization of the coefficients.

Quaternion coefficients are stored planar, ``C[z, mu, p]`` with
C = C0 + i C1 + j C2 + k C3 (shape ``(4, N, n)``, float64).

The synthetic systems mirror the paper's workloads (Sec. 3): linear atomic
chains (Hg and Pu chains, Sec. 3.1 and 3.3.1) and a compact cluster (the Au6
cluster, Sec. 3.3.2).  The paper's Dyall basis sets and geometries are not
available, so seeded s-type Gaussians stand in for them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SPEED_OF_LIGHT = 137.035999074  # a.u., the value quoted in Sec. 3


@dataclasses.dataclass
class Basis:
    """Contracted Cartesian Gaussian basis (all arrays float64/int32,
    C-contiguous).  ``cart`` gives each function's type: 0 = s, 1, 2, 3 =
    p_x, p_y, p_z (None: every function is s).  A p shell is three functions
    with the same centre, exponents and coefficients."""

    centers: np.ndarray  # (nfunc, 3) bohr
    nprim: np.ndarray  # (nfunc,) int32
    exps: np.ndarray  # (sum nprim,)
    coefs: np.ndarray  # (sum nprim,)
    cart: Optional[np.ndarray] = None  # (nfunc,) int32

    @property
    def nfunc(self) -> int:
        return int(self.nprim.shape[0])

    def offsets(self) -> np.ndarray:
        off = np.zeros(self.nfunc + 1, dtype=np.int64)
        np.cumsum(self.nprim, out=off[1:])
        return off

    def subset(self, idx) -> "Basis":
        idx = np.asarray(idx, dtype=np.int64)
        off = self.offsets()
        e, c = [], []
        for f in idx:
            e.append(self.exps[off[f]:off[f + 1]])
            c.append(self.coefs[off[f]:off[f + 1]])
        return Basis(np.ascontiguousarray(self.centers[idx]),
                     np.ascontiguousarray(self.nprim[idx]).astype(np.int32),
                     np.ascontiguousarray(np.concatenate(e)) if e else np.zeros(0),
                     np.ascontiguousarray(np.concatenate(c)) if c else np.zeros(0),
                     None if self.cart is None
                     else np.ascontiguousarray(self.cart[idx]).astype(np.int32))


@dataclasses.dataclass
class System:
    name: str
    ham: str  # "LL", "DC" or "DCG"
    L: Basis
    S: Optional[Basis]
    CL: np.ndarray  # (4, N_L, n)
    CS: Optional[np.ndarray]  # (4, N_S, n)
    tau: float
    atoms: np.ndarray

    @property
    def n_mo(self) -> int:
        return int(self.CL.shape[2])


# ----------------------------------------------------------------------------
# quaternion helpers used only for building inputs
# ----------------------------------------------------------------------------

def quat_left_matrix(q: np.ndarray) -> np.ndarray:
    """Real 4x4 matrix of left multiplication y -> q*y (q = q0 + q1 i + q2 j + q3 k)."""
    q0, q1, q2, q3 = q
    return np.array([[q0, -q1, -q2, -q3],
                     [q1, q0, -q3, q2],
                     [q2, q3, q0, -q1],
                     [q3, -q2, q1, q0]])


def quat_to_real(A: np.ndarray) -> np.ndarray:
    """Planar quaternion matrix (4, N, n) -> real (4N, 4n) block matrix of L(A_mu,p)."""
    _, N, n = A.shape
    R = np.zeros((4 * N, 4 * n))
    for mu in range(N):
        for p in range(n):
            R[4 * mu:4 * mu + 4, 4 * p:4 * p + 4] = quat_left_matrix(A[:, mu, p])
    return R


def real_to_quat(R: np.ndarray) -> np.ndarray:
    """Inverse of quat_to_real: column 0 of block (mu,p) is the quaternion A_mu,p."""
    N, n = R.shape[0] // 4, R.shape[1] // 4
    A = np.empty((4, N, n))
    for z in range(4):
        A[z] = R[z::4, 0::4]
    return A


def quat_qr_plus(A: np.ndarray) -> np.ndarray:
    """Quaternion-orthonormalize the columns of A (QR of the 4x4 real
    representation with R's diagonal forced positive, which is Gram-Schmidt
    in the quaternion sense and keeps the L(q) block structure)."""
    R = quat_to_real(A)
    Qm, Rm = np.linalg.qr(R)
    s = np.sign(np.diag(Rm))
    s[s == 0] = 1.0
    Qm = Qm * s[None, :]
    return real_to_quat(Qm)


def gaussian_quat(rng: np.random.Generator, N: int, n: int) -> np.ndarray:
    return rng.standard_normal((4, N, n))


# ----------------------------------------------------------------------------
# basis construction
# ----------------------------------------------------------------------------

def make_basis(rng: np.random.Generator, atoms: np.ndarray, nfunc: int,
               nprim, exp_lo: float, exp_hi: float, exp_scale: float = 1.0) -> Basis:
    """``nfunc`` s functions placed round-robin on the atoms (function f sits on
    atom f mod n_atoms).  ``nprim`` is an int or a (lo, hi) range drawn
    uniformly per function.  Exponents are exp_scale * 10^U(log10 lo, log10 hi),
    coefficients U(0.1, 1)."""
    nat = atoms.shape[0]
    centers = np.ascontiguousarray(atoms[np.arange(nfunc) % nat])
    if isinstance(nprim, (tuple, list)):
        k = rng.integers(nprim[0], nprim[1] + 1, size=nfunc).astype(np.int32)
    else:
        k = np.full(nfunc, int(nprim), dtype=np.int32)
    tot = int(k.sum())
    exps = exp_scale * 10.0 ** rng.uniform(math.log10(exp_lo), math.log10(exp_hi), size=tot)
    coefs = rng.uniform(0.1, 1.0, size=tot)
    return Basis(centers, k, np.ascontiguousarray(exps), np.ascontiguousarray(coefs))


def _normalized_coefs(b: Basis) -> np.ndarray:
    """Contraction coefficients of normalized primitives (2a/pi)^{3/4} e^{-a r^2}
    rescaled so that each contracted s function has unit self-overlap."""
    off = b.offsets()
    out = np.empty_like(b.coefs)
    for f in range(b.nfunc):
        a = b.exps[off[f]:off[f + 1]]
        d = b.coefs[off[f]:off[f + 1]] * (2.0 * a / math.pi) ** 0.75
        s = (d[:, None] * d[None, :] * (math.pi / (a[:, None] + a[None, :])) ** 1.5).sum()
        out[off[f]:off[f + 1]] = d / math.sqrt(s)
    return out


def overlap_matrix(A: Basis, B: Basis, block: int = 2048) -> np.ndarray:
    """Overlap of the normalized contracted s functions of A and B (input
    construction only: Loewdin orthonormalization of the MO coefficients):
    primitive overlaps d_i d_j (pi/p)^{3/2} exp(-a_i b_j R^2 / p), summed over
    each function's primitives (blocks of A's primitives at a time)."""
    ca, cb = _normalized_coefs(A), _normalized_coefs(B)
    oa, ob = A.offsets(), B.offsets()
    fa = np.repeat(np.arange(A.nfunc), np.diff(oa))  # function of each primitive
    fb = np.repeat(np.arange(B.nfunc), np.diff(ob))
    PA, PB = A.centers[fa], B.centers[fb]
    S = np.zeros((A.nfunc, B.nfunc))
    for i0 in range(0, fa.shape[0], block):
        i1 = min(fa.shape[0], i0 + block)
        a = A.exps[i0:i1, None]
        p = a + B.exps[None, :]
        r2 = ((PA[i0:i1, None, :] - PB[None, :, :]) ** 2).sum(-1)
        prim = (ca[i0:i1, None] * cb[None, :] * (math.pi / p) ** 1.5
                * np.exp(-a * B.exps[None, :] / p * r2))
        byfunc = np.add.reduceat(prim, ob[:-1], axis=1) if B.nfunc else prim[:, :0]
        np.add.at(S, fa[i0:i1], byfunc)
    return S


LINDEP_CUT = 1e-6  # overlap eigenvalues below this are treated as linear dependencies


def orthonormalizer(S: np.ndarray, cut: float = LINDEP_CUT):
    """Symmetric (Loewdin) orthonormalizer restricted to the numerically
    non-redundant subspace: X = U_k w_k^{-1/2} U_k^T and the projector
    P = U_k U_k^T over eigenvalues w >= cut.  With no eigenvalue below the
    cut this is exactly S^{-1/2} and P = I."""
    w, U = np.linalg.eigh(S)
    keep = w >= cut
    Uk = U[:, keep]
    X = (Uk * (1.0 / np.sqrt(w[keep]))[None, :]) @ Uk.T
    P = Uk @ Uk.T if not keep.all() else np.eye(S.shape[0])
    return X, P, int((~keep).sum())


def inv_sqrt_sym(S: np.ndarray) -> np.ndarray:
    return orthonormalizer(S)[0]


def _apply_planes(M: np.ndarray, A: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.einsum("mn,znp->zmp", M, A))


def loewdin_coefficients(rng: np.random.Generator, L: Basis, S: Optional[Basis], n: int,
                         G: Optional[np.ndarray] = None):
    """C^X = X_X Q_X, with X_X the Loewdin orthonormalizer of basis X and Q a
    random quaternion-orthonormal (N_L + N_S) x n matrix (block-diagonal
    metric over L and S).  Q is the positive-diagonal quaternion QR of a
    Gaussian quaternion matrix whose blocks are first projected onto the
    non-redundant subspace of each basis, so C^dagger S C = I holds exactly
    even when a basis is numerically linearly dependent."""
    NL = L.nfunc
    NS = S.nfunc if S is not None else 0
    if G is None:
        G = gaussian_quat(rng, NL + NS, n)
    XL, PL, _ = orthonormalizer(overlap_matrix(L, L))
    parts = [_apply_planes(PL, G[:, :NL])]
    if S is not None:
        XS, PS, _ = orthonormalizer(overlap_matrix(S, S))
        parts.append(_apply_planes(PS, G[:, NL:]))
    Q = quat_qr_plus(np.concatenate(parts, axis=1))
    CL = _apply_planes(XL, Q[:, :NL])
    CS = _apply_planes(XS, Q[:, NL:]) if S is not None else None
    return CL, CS


# ----------------------------------------------------------------------------
# geometries
# ----------------------------------------------------------------------------

def chain(n_atoms: int, spacing: float) -> np.ndarray:
    a = np.zeros((n_atoms, 3))
    a[:, 0] = spacing * np.arange(n_atoms)
    return a


def cube(rng, n_atoms: int, edge: float) -> np.ndarray:
    return rng.uniform(0.0, edge, size=(n_atoms, 3))


def ball(rng, n_atoms: int, radius: float, min_sep: float) -> np.ndarray:
    pts = []
    while len(pts) < n_atoms:
        x = rng.uniform(-radius, radius, size=3)
        if (x ** 2).sum() > radius ** 2:
            continue
        if any(((x - y) ** 2).sum() < min_sep ** 2 for y in pts):
            continue
        pts.append(x)
    return np.array(pts)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def qr_coefficients(rng: np.random.Generator, L: Basis, S: Optional[Basis], n: int):
    """C = QR+(G): a random quaternion-orthonormal (N_L + N_S) x n matrix (the
    positive-diagonal quaternion QR of a Gaussian quaternion matrix), split
    into its L and S rows; not orthonormal in the AO metric, which the
    transformation does not need.  |C_mu p| <= 1, so the MO integrals are
    not small differences of large terms (well-conditioned inputs)."""
    NL = L.nfunc
    NS = S.nfunc if S is not None else 0
    Q = quat_qr_plus(gaussian_quat(rng, NL + NS, n))
    CL = np.ascontiguousarray(Q[:, :NL])
    CS = np.ascontiguousarray(Q[:, NL:]) if S is not None else None
    return CL, CS


def _coefficients(kind: str, rng, L, S, n):
    if kind == "loewdin":
        return loewdin_coefficients(rng, L, S, n)
    if kind == "qr":
        return qr_coefficients(rng, L, S, n)
    raise ValueError(f"coefficient kind {kind!r} (loewdin or qr)")


def _streams(seed: int):
    ss = np.random.SeedSequence(seed).spawn(4)
    return [np.random.default_rng(s) for s in ss]  # atoms, basis, C, perturbations


def small_ll(seed: int = 1, n_atoms: int = 8, nfunc: int = 24, n: int = 12,
             nprim: int = 3, edge: float = 6.0, tau: float = 0.0,
             coefs: str = "loewdin") -> System:
    """Large-component-only system: ``nfunc`` s functions (3 per atom by
    default) on atoms uniform in a cube.  coefs: "loewdin" (orthonormal in
    the AO metric) or "qr" (quaternion-orthonormal, see qr_coefficients)."""
    ra, rb, rc, _ = _streams(seed)
    atoms = cube(ra, n_atoms, edge)
    L = make_basis(rb, atoms, nfunc, nprim, 0.1, 10.0)
    CL, _ = _coefficients(coefs, rc, L, None, n)
    return System(f"ll_{nfunc}_{n}", "LL", L, None, CL, None, tau, atoms)


def linear_chain(seed: int = 2, n_atoms: int = 40, spacing: float = 2.5,
                 nl_per_atom: int = 10, ns_per_atom: int = 20, n: int = 64,
                 nprim=3, tau: float = 1e-10, ham: str = "DC",
                 coefs: str = "loewdin") -> System:
    """Linear chain with a large-component basis and a tighter (exponents x4)
    stand-in small-component basis of twice the size (coefs as in small_ll)."""
    ra, rb, rc, _ = _streams(seed)
    atoms = chain(n_atoms, spacing)
    L = make_basis(rb, atoms, nl_per_atom * n_atoms, nprim, 0.1, 10.0)
    S = make_basis(rb, atoms, ns_per_atom * n_atoms, nprim, 0.1, 10.0, exp_scale=4.0)
    CL, CS = _coefficients(coefs, rc, L, S, n)
    return System(f"chain{n_atoms}_{ham}_{n}", ham, L, S, CL, CS, tau, atoms)


def cluster(seed: int = 3, n_atoms: int = 60, radius: float = 20.0, min_sep: float = 2.0,
            nl_per_atom: int = 10, ns_per_atom: int = 20, n: int = 128,
            nprim=(1, 6), tau: float = 1e-10, ham: str = "DCG",
            coefs: str = "loewdin") -> System:
    """Compact 3-D cluster with mixed contraction depth 1..6 (coefs as in
    small_ll)."""
    ra, rb, rc, _ = _streams(seed)
    atoms = ball(ra, n_atoms, radius, min_sep)
    L = make_basis(rb, atoms, nl_per_atom * n_atoms, nprim, 0.1, 10.0)
    S = make_basis(rb, atoms, ns_per_atom * n_atoms, nprim, 0.1, 10.0, exp_scale=4.0)
    CL, CS = _coefficients(coefs, rc, L, S, n)
    return System(f"cluster{n_atoms}_{ham}_{n}", ham, L, S, CL, CS, tau, atoms)


def make_sp_basis(rng: np.random.Generator, atoms: np.ndarray, s_per_atom: int,
                  p_shells_per_atom: int, nprim, exp_lo: float, exp_hi: float,
                  exp_scale: float = 1.0, d_shells_per_atom: int = 0,
                  f_shells_per_atom: int = 0) -> Basis:
    """Per atom ``s_per_atom`` s functions, ``p_shells_per_atom`` p shells
    (p_x, p_y, p_z with one shared set of exponents and coefficients) and
    ``d_shells_per_atom`` Cartesian d shells (codes 4..9: d_xx, d_yy, d_zz,
    d_xy, d_xz, d_yz, shared exponents and coefficients) and
    ``f_shells_per_atom`` Cartesian f shells (codes 10..19), drawn as in
    make_basis; functions are listed atom by atom."""
    centers, nprim_l, exps, coefs, cart = [], [], [], [], []

    def draw():
        return int(rng.integers(nprim[0], nprim[1] + 1)) if isinstance(nprim, (tuple, list)) \
            else int(nprim)

    for a in atoms:
        for _ in range(s_per_atom):
            k = draw()
            e = exp_scale * 10.0 ** rng.uniform(math.log10(exp_lo), math.log10(exp_hi), size=k)
            c = rng.uniform(0.1, 1.0, size=k)
            centers.append(a); nprim_l.append(k); exps.append(e); coefs.append(c); cart.append(0)
        for _ in range(p_shells_per_atom):
            k = draw()
            e = exp_scale * 10.0 ** rng.uniform(math.log10(exp_lo), math.log10(exp_hi), size=k)
            c = rng.uniform(0.1, 1.0, size=k)
            for comp in (1, 2, 3):
                centers.append(a); nprim_l.append(k); exps.append(e); coefs.append(c)
                cart.append(comp)
        for _ in range(d_shells_per_atom):
            k = draw()
            e = exp_scale * 10.0 ** rng.uniform(math.log10(exp_lo), math.log10(exp_hi), size=k)
            c = rng.uniform(0.1, 1.0, size=k)
            for comp in range(4, 10):
                centers.append(a); nprim_l.append(k); exps.append(e); coefs.append(c)
                cart.append(comp)
        for _ in range(f_shells_per_atom):
            k = draw()
            e = exp_scale * 10.0 ** rng.uniform(math.log10(exp_lo), math.log10(exp_hi), size=k)
            c = rng.uniform(0.1, 1.0, size=k)
            for comp in range(10, 20):
                centers.append(a); nprim_l.append(k); exps.append(e); coefs.append(c)
                cart.append(comp)
    return Basis(np.ascontiguousarray(np.array(centers, dtype=np.float64)),
                 np.array(nprim_l, dtype=np.int32),
                 np.ascontiguousarray(np.concatenate(exps)),
                 np.ascontiguousarray(np.concatenate(coefs)),
                 np.array(cart, dtype=np.int32))


def sp_cluster(seed: int = 5, n_atoms: int = 8, edge: float = 6.0, s_per_atom: int = 1,
               p_shells_per_atom: int = 1, ns_per_atom: int = 1, nsp_per_atom: int = 1,
               nprim=(1, 3), n: int = 8, tau: float = 0.0, ham: str = "DC") -> System:
    """Atoms uniform in a cube with s and p shells on every atom (L: exponents
    10^U(-1, 1); S: the same recipe with exponents x4).  The MO coefficients
    are a quaternion-orthonormal n-column matrix (positive-diagonal QR of a
    Gaussian quaternion matrix) over the L and S functions together, not
    orthonormalized in the AO metric: the transformation does not need it."""
    ra, rb, rc, _ = _streams(seed)
    atoms = cube(ra, n_atoms, edge)
    L = make_sp_basis(rb, atoms, s_per_atom, p_shells_per_atom, nprim, 0.1, 10.0)
    S = None
    if ham != "LL":
        S = make_sp_basis(rb, atoms, ns_per_atom, nsp_per_atom, nprim, 0.1, 10.0,
                          exp_scale=4.0)
    NL, NS = L.nfunc, (S.nfunc if S is not None else 0)
    Q = quat_qr_plus(gaussian_quat(rc, NL + NS, n))
    CL = np.ascontiguousarray(Q[:, :NL])
    CS = np.ascontiguousarray(Q[:, NL:]) if S is not None else None
    return System(f"sp{n_atoms}_{ham}_{n}", ham, L, S, CL, CS, tau, atoms)


def spd_cluster(seed: int = 7, n_atoms: int = 4, edge: float = 4.0, nprim=(1, 2), n: int = 4,
                tau: float = 0.0, ham: str = "DC", d_l: int = 1, d_s: int = 0, f_l: int = 0,
                p_s: int = 1) -> System:
    """Atoms uniform in a cube with one s function, one p shell, ``d_l``
    Cartesian d shells and ``f_l`` Cartesian f shells per atom in L (10
    functions per atom by default) and one s function, ``p_s`` p shells and
    ``d_s`` d shells in S (exponents x4).  MO coefficients as in sp_cluster
    (quaternion QR, |C| <= 1)."""
    ra, rb, rc, _ = _streams(seed)
    atoms = cube(ra, n_atoms, edge)
    L = make_sp_basis(rb, atoms, 1, 1, nprim, 0.1, 10.0, d_shells_per_atom=d_l,
                      f_shells_per_atom=f_l)
    S = None
    if ham != "LL":
        S = make_sp_basis(rb, atoms, 1, p_s, nprim, 0.1, 10.0, exp_scale=4.0,
                          d_shells_per_atom=d_s)
    NL, NS = L.nfunc, (S.nfunc if S is not None else 0)
    Q = quat_qr_plus(gaussian_quat(rc, NL + NS, n))
    CL = np.ascontiguousarray(Q[:, :NL])
    CS = np.ascontiguousarray(Q[:, NL:]) if S is not None else None
    return System(f"spd{n_atoms}_{ham}_{n}", ham, L, S, CL, CS, tau, atoms)


def sp_chain(seed: int = 6, n_atoms: int = 40, spacing: float = 2.5, l_s: int = 4,
             l_p: int = 2, s_s: int = 8, s_p: int = 4, nprim=3, n: int = 64,
             tau: float = 1e-10, ham: str = "DC", l_d: int = 0) -> System:
    """The linear-chain recipe with p shells: per atom l_s s functions, l_p
    p shells and l_d Cartesian d shells in L (10 functions by default, N_L =
    400 for 40 atoms) and s_s + 3 s_p in S (20, exponents x4).  MO
    coefficients as in sp_cluster."""
    ra, rb, rc, _ = _streams(seed)
    atoms = chain(n_atoms, spacing)
    L = make_sp_basis(rb, atoms, l_s, l_p, nprim, 0.1, 10.0, d_shells_per_atom=l_d)
    S = make_sp_basis(rb, atoms, s_s, s_p, nprim, 0.1, 10.0, exp_scale=4.0)
    Q = quat_qr_plus(gaussian_quat(rc, L.nfunc + S.nfunc, n))
    return System(f"chain{n_atoms}_sp{'d' if l_d else ''}_{ham}_{n}", ham, L, S,
                  np.ascontiguousarray(Q[:, :L.nfunc]), np.ascontiguousarray(Q[:, L.nfunc:]),
                  tau, atoms)


def perturbed_coefficients(system: System, k: int, eps: float = 1e-2):
    """Re-transform input k: the system's quaternion-orthonormal Q0
    (C = X Q0) is perturbed by eps * G_k (G_k Gaussian, seed 3000 + k) and
    re-orthonormalized the same way as the original coefficients."""
    L, S = system.L, system.S
    NL = L.nfunc
    SL = overlap_matrix(L, L)
    w, U = np.linalg.eigh(SL)
    half = lambda w, U: (U * np.sqrt(np.clip(w, 0, None))[None, :]) @ U.T
    parts = [_apply_planes(half(w, U), system.CL)]
    if S is not None:
        SS = overlap_matrix(S, S)
        w2, U2 = np.linalg.eigh(SS)
        parts.append(_apply_planes(half(w2, U2), system.CS))
    Q0 = np.concatenate(parts, axis=1)
    g = np.random.default_rng(3000 + k).standard_normal(Q0.shape)
    return loewdin_coefficients(None, L, S, system.n_mo, G=Q0 + eps * g)


def config(name: str) -> System:
    """Named workloads.

    ``ll24``   24 functions / 8 atoms in a 6 bohr cube, n = 12, LL only.
    ``chain40`` 40-atom chain (2.5 bohr), N_L = 400, N_S = 800, n = 64, DC, tau 1e-10.
    ``cluster60`` 60-atom cluster (20 bohr ball), N_L = 600, N_S = 1200,
               K in 1..6, n = 128, DC + Gaunt, tau 1e-10.
    ``chain40_dcg``, ``chain40_dcb``, ``cluster60_dcb``  the same systems with
               the Gaunt term, or the whole Breit term (Gaunt + gauge).
    ``chain40_sp`` the chain40 shape with p shells: per atom 4 s + 2 p shells in
               L (N_L = 400) and 8 s + 4 p shells in S (N_S = 800), K = 3, n = 64,
               DC, tau 1e-10.
    ``chain40_sp_dcb`` ``chain40_sp`` with the whole Breit term (Gaunt + gauge).
    ``chain40_spd`` the chain40 shape with p and d shells: per atom 4 s + 1 p +
               1 Cartesian d shell in L (N_L = 520) and 8 s + 4 p shells in S
               (N_S = 800), K = 3, n = 64, DC, tau 1e-10.
    ``sp8``    8 atoms in a 6 bohr cube with one s function and one p shell per
               atom in L and in S (N_L = N_S = 32), K in 1..3, n = 8, DC.
    """
    if name == "ll24":
        return small_ll(seed=1)
    if name == "chain40":
        return linear_chain(seed=2)
    if name == "chain40_dcg":
        return linear_chain(seed=2, ham="DCG")
    if name == "chain40_dcb":
        return linear_chain(seed=2, ham="DCB")
    if name == "cluster60":
        return cluster(seed=3)
    if name == "cluster60_dcb":
        return cluster(seed=3, ham="DCB")
    if name == "sp8":
        return sp_cluster(seed=5)
    if name == "chain40_sp":
        return sp_chain(seed=6)
    if name == "chain40_spd":
        return sp_chain(seed=6, l_p=1, l_d=1)
    if name == "chain40_sp_dcb":
        return sp_chain(seed=6, ham="DCB")
    if name == "cluster24":
        # the cluster recipe at 24 atoms (radius scaled by (24/60)^(1/3)), n = 64
        return cluster(seed=3, n_atoms=24, radius=20.0 * (24 / 60) ** (1 / 3), n=64)
    raise KeyError(name)


# ----------------------------------------------------------------------------
# general (Kramers-unrestricted) two-spinor inputs
# ----------------------------------------------------------------------------

def quat_to_spinor_planes(C: np.ndarray) -> np.ndarray:
    """Two-spinor planes [4][N][2n] (alpha re, alpha im, beta re, beta im) of the
    Kramers pairs that quaternion coefficients C[4][N][n] stand for: spinors
    2p and 2p + 1 are the columns of Q(C_mu p) = [[c0 + i c1, c2 + i c3],
    [-c2 + i c3, c0 - i c1]] (rows alpha, beta)."""
    c0, c1, c2, c3 = C
    N, n = C.shape[1], C.shape[2]
    P = np.empty((4, N, 2 * n))
    P[0, :, 0::2], P[1, :, 0::2] = c0, c1      # alpha of spinor 2p
    P[0, :, 1::2], P[1, :, 1::2] = c2, c3      # alpha of spinor 2p + 1
    P[2, :, 0::2], P[3, :, 0::2] = -c2, c3     # beta of spinor 2p
    P[2, :, 1::2], P[3, :, 1::2] = c0, -c1     # beta of spinor 2p + 1
    return P


def mix_spinors(P: np.ndarray, U: np.ndarray) -> np.ndarray:
    """Planes of the spinors c' = c U (U complex [m][m'])."""
    ca = (P[0] + 1j * P[1]) @ U
    cb = (P[2] + 1j * P[3]) @ U
    return np.stack([ca.real, ca.imag, cb.real, cb.imag])


def random_unitary(rng: np.random.Generator, m: int, k: int) -> np.ndarray:
    """First k columns of a random m x m unitary (QR of a complex Gaussian)."""
    Z = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    Q, R = np.linalg.qr(Z)
    Q = Q * (np.diag(R) / np.abs(np.diag(R)))[None, :]
    return Q[:, :k]


def general_spinors(system: System, m: int, seed: int = 0):
    """m orthonormal general two-spinor MOs for a system: its 2n Kramers-paired
    spinors mixed by a random unitary (seeded), which breaks every Kramers
    pair.  Returns (planes for L, planes for S or None, U)."""
    n = system.n_mo
    if m > 2 * n:
        raise ValueError("at most 2 n_mo spinors")
    U = random_unitary(np.random.default_rng(7000 + seed), 2 * n, m)
    PL = mix_spinors(quat_to_spinor_planes(system.CL), U)
    PS = mix_spinors(quat_to_spinor_planes(system.CS), U) if system.CS is not None else None
    return PL, PS, U
