"""Quaternion helpers for the tests (planar arrays, C = C0 + i C1 + j C2 + k C3).

Independent of both the oracle and the GPU library; used to build test
inputs (unitary rotations, identity coefficients) and to evaluate
invariants and symmetry relations of the outputs.
"""
import math

import numpy as np

SIGNS = np.array([1.0, -1.0, -1.0, -1.0])  # quaternion conjugation signs s_x


def qmul(a, b):
    """Componentwise-broadcast quaternion product a*b (leading axis = component)."""
    a0, a1, a2, a3 = a
    b0, b1, b2, b3 = b
    return np.array([a0 * b0 - a1 * b1 - a2 * b2 - a3 * b3,
                     a0 * b1 + a1 * b0 + a2 * b3 - a3 * b2,
                     a0 * b2 - a1 * b3 + a2 * b0 + a3 * b1,
                     a0 * b3 + a1 * b2 - a2 * b1 + a3 * b0])


def qconj(a):
    return a * SIGNS.reshape((4,) + (1,) * (a.ndim - 1))


def qmatmul(A, B):
    """Quaternion matrix product (4,N,k) x (4,k,n) -> (4,N,n)."""
    out = np.zeros((4, A.shape[1], B.shape[2]))
    for k in range(A.shape[2]):
        out += qmul(A[:, :, k][:, :, None], B[:, k, :][:, None, :])
    return out


def qrep(q):
    q0, q1, q2, q3 = q
    return np.array([[q0 + 1j * q1, q2 + 1j * q3], [-q2 + 1j * q3, q0 - 1j * q1]])


def pair_density(C, mu, nu):
    """[conj(C_mu r) C_nu t] for all r, t: shape (4, n, n)."""
    a = qconj(C[:, mu, :])[:, :, None]
    b = C[:, nu, :][:, None, :]
    return qmul(a, b)


def identity_coefficients(N):
    C = np.zeros((4, N, N))
    C[0] = np.eye(N)
    return C


def schwarz_scale(Qs, Cs):
    """Magnitude scale of the MO-integral sums: Gabs <= (max_pq a_pq)^2 with
    a_pq = sum_X sum_{mu nu} |C^X_mu p| Q^X_{mu nu} |C^X_nu q| (quaternion
    norms, Schwarz matrices Q^X).  Floating-point error of any summation
    order is a small multiple of eps times this scale."""
    a = 0
    for Q, C in zip(Qs, Cs):
        nrm = np.sqrt((C ** 2).sum(axis=0))  # (N, n)
        a = a + nrm.T @ Q @ nrm
    return float(np.max(a)) ** 2
