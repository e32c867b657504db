"""Restricted-kinetic-balance (RKB) small components for the oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper's small-component basis follows from the large one by the RKB
condition (Eq. RKB): chi^S_{mu tau} = (1/2c) (sigma . p) chi^L_{mu tau}, with
p = -i nabla, so N_S = N_L.  For a contracted s function
chi_mu = sum_i n_i exp(-a_i |r - A|^2) the gradient components are p functions,
d/dr_K chi_mu = sum_i (-2 a_i n_i) (r_K - A_K) exp(-a_i |r - A|^2).
Written over the scalar gradient functions g_{mu K} = d_K chi_mu, the small
component of a two-spinor with RKB coefficients C^S_{mu tau} is

    phi^S = sum_{mu K} [ (-i / 2c) sum_tau sigma_K[:, tau] C^S_{mu tau} ] g_{mu K},

a two-spinor expansion over 3 N_L scalar functions.  The four-component
Dirac-Coulomb integrals (Eq. DCInt) of such spinors are therefore the oracle's
general two-spinor transformation with the gradient functions as the small
basis; this module builds that basis and those coefficients.  Nothing here
evaluates an integral itself.
"""
from __future__ import annotations

import dataclasses

import numpy as np

import oracle

SPEED_OF_LIGHT = 137.035999074  # a.u., the value the paper's Sec. 3 quotes


@dataclasses.dataclass
class _Basis:
    """Basis record in the layout the oracle's ctypes wrapper reads."""
    centers: np.ndarray
    nprim: np.ndarray
    exps: np.ndarray
    coefs: np.ndarray
    cart: np.ndarray

    @property
    def nfunc(self) -> int:
        return int(self.nprim.shape[0])

    def offsets(self) -> np.ndarray:
        off = np.zeros(self.nfunc + 1, dtype=np.int64)
        np.cumsum(self.nprim, out=off[1:])
        return off

# Pauli matrices as printed in the paper's notation section
PAULI = (np.array([[0, 1], [1, 0]], dtype=complex),
         np.array([[0, -1j], [1j, 0]], dtype=complex),
         np.array([[1, 0], [0, -1]], dtype=complex))


def gradient_basis(L):
    """(G, norms): G holds the 3 N_L functions g_{mu K} (index 3 mu + K) as
    normalized Cartesian p functions, norms[3 mu + K] = ||d_K chi_mu||, so
    that d_K chi_mu = norms * (the normalized function).  L must be s-only."""
    if getattr(L, "cart", None) is not None and np.any(np.asarray(L.cart) != 0):
        raise ValueError("RKB gradients are built for s functions")
    nc = oracle.norm_coefs(L)  # chi_mu = sum_i nc_i exp(-a_i r^2)
    off = np.zeros(L.nfunc + 1, dtype=np.int64)
    np.cumsum(np.asarray(L.nprim), out=off[1:])
    cen, npr, ex, co, cart = [], [], [], [], []
    for mu in range(L.nfunc):
        a = L.exps[off[mu]:off[mu + 1]]
        w = -2.0 * a * nc[off[mu]:off[mu + 1]]  # weights of (r_K - A_K) exp(-a r^2)
        pnorm = (2 * a / np.pi) ** 0.75 * 2 * np.sqrt(a)  # normalized p primitive
        for K in range(3):
            cen.append(L.centers[mu])
            npr.append(len(a))
            ex.append(a)
            co.append(w / pnorm)
            cart.append(K + 1)
    G = _Basis(np.ascontiguousarray(np.array(cen)), np.array(npr, np.int32),
               np.ascontiguousarray(np.concatenate(ex)),
               np.ascontiguousarray(np.concatenate(co)), np.array(cart, np.int32))
    ncg = oracle.norm_coefs(G)
    offg = G.offsets()
    norms = np.array([G.coefs[offg[f]] * (2 * G.exps[offg[f]] / np.pi) ** 0.75 *
                      2 * np.sqrt(G.exps[offg[f]]) / ncg[offg[f]] for f in range(G.nfunc)])
    return G, norms


def small_component_planes(PS: np.ndarray, norms: np.ndarray, c: float) -> np.ndarray:
    """Planes [4][3 N][m] (alpha re, alpha im, beta re, beta im) of the small
    components over the normalized gradient functions, from the RKB
    two-spinor planes PS [4][N][m] of the same spinors."""
    N, m = PS.shape[1], PS.shape[2]
    cs = np.stack([PS[0] + 1j * PS[1], PS[2] + 1j * PS[3]])  # [tau][mu][a]
    out = np.zeros((2, 3 * N, m), dtype=complex)
    for K in range(3):
        # component upsilon: (-i / 2c) sum_tau sigma_K[upsilon, tau] C^S_{mu tau}
        comp = np.einsum("ut,tma->uma", PAULI[K], cs) * (-1j / (2.0 * c))
        out[:, K::3, :] = comp * norms[K::3][None, :, None]
    return np.ascontiguousarray(np.stack([out[0].real, out[0].imag, out[1].real, out[1].imag]))


def transform_rkb(L, PL: np.ndarray, PS: np.ndarray, c: float = SPEED_OF_LIGHT,
                  tau: float = 0.0, ham: str = "DC"):
    """Four-component MO integrals (ab|cd) [m]^4 (complex) of general
    two-spinors with large-component planes PL [4][N][m] over L and RKB
    small-component planes PS [4][N][m] (N_S = N_L): Dirac-Coulomb (ham "DC")
    or with the Gaunt term ("DCG")."""
    G, norms = gradient_basis(L)
    PG = small_component_planes(PS, norms, c)
    return oracle.transform_spinor(L, G, PL, PG, ham, tau)[0]
