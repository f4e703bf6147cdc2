"""Exact references used to pin the oracle (test infrastructure only).

Everything here is independent of lrh_oracle.py: Hamiltonians are applied to state
vectors by tensor contraction on the full Hilbert space, never through the
relaxation's lift / partial-trace code.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def apply_H(desc, psi: np.ndarray) -> np.ndarray:
    """H |psi> for H = sum of the problem's terms; psi has shape (prod d,)."""
    dims = [int(d) for d in desc.site_dim]
    n = len(dims)
    t = psi.reshape(dims)
    out = np.zeros_like(t, dtype=np.complex128)
    for sites, m in desc.terms():
        k = len(sites)
        op = m.reshape([dims[s] for s in sites] * 2)
        # contract the operator's input legs with psi's legs `sites`
        r = np.tensordot(op, t, axes=(list(range(k, 2 * k)), list(sites)))
        # r has the operator's output legs first, then psi's remaining legs in order
        rest = [i for i in range(n) if i not in sites]
        src = list(range(k)) + [k + j for j in range(len(rest))]
        dst = list(sites) + rest
        out += np.moveaxis(r, src, dst)
    return out.reshape(-1)


def dense_H(desc) -> np.ndarray:
    N = int(np.prod(desc.site_dim))
    H = np.zeros((N, N), dtype=np.complex128)
    e = np.zeros(N, dtype=np.complex128)
    for j in range(N):
        e[:] = 0
        e[j] = 1
        H[:, j] = apply_H(desc, e)
    return H


def ground_energy(desc, dense_max: int = 4096) -> float:
    """Exact E0 = lambda_min(H): dense diagonalisation or Lanczos (scipy eigsh)."""
    N = int(np.prod(desc.site_dim))
    if N <= dense_max:
        return float(np.linalg.eigvalsh(dense_H(desc))[0])
    from scipy.sparse.linalg import LinearOperator, eigsh
    op = LinearOperator((N, N), matvec=lambda v: apply_H(desc, v.astype(np.complex128)),
                        dtype=np.complex128)
    w = eigsh(op, k=1, which='SA', tol=1e-12, return_eigenvectors=False)
    return float(w[0].real)


def tfim_open_chain_E0(n: int, J: float, h: float) -> float:
    """Free-fermion ground energy of H = -J sum_{i<n-1} Z_i Z_{i+1} - h sum_i X_i (open chain).

    After the basis change X <-> Z and a Jordan-Wigner map to Majoranas
    g_{2i} = P_i X_i, g_{2i+1} = P_i Y_i (P_i = prod_{k<i} Z_k):  Z_i = -i g_{2i} g_{2i+1},
    X_i X_{i+1} = -i g_{2i+1} g_{2i+2}, so H = (i/4) g^T M g with M antisymmetric,
    M_{2i,2i+1} = 2h, M_{2i+1,2i+2} = 2J, and E0 = -(1/4) * sum of singular values of M.
    """
    M = np.zeros((2 * n, 2 * n))
    for i in range(n):
        M[2 * i, 2 * i + 1] = 2 * h
        M[2 * i + 1, 2 * i] = -2 * h
    for i in range(n - 1):
        M[2 * i + 1, 2 * i + 2] = 2 * J
        M[2 * i + 2, 2 * i + 1] = -2 * J
    return float(-0.25 * np.sum(np.linalg.svd(M, compute_uv=False)))


def classical_min(desc) -> float:
    """Brute-force minimum over product basis states, for problems whose terms are all
    diagonal in the computational basis."""
    dims = [int(d) for d in desc.site_dim]
    terms = list(desc.terms())
    for _, m in terms:
        if np.max(np.abs(m - np.diag(np.diag(m)))) > 0:
            raise ValueError("classical_min needs diagonal terms")
    best = math.inf
    for conf in itertools.product(*[range(d) for d in dims]):
        E = 0.0
        for sites, m in terms:
            idx = 0
            for s in sites:
                idx = idx * dims[s] + conf[s]
            E += m[idx, idx].real
        best = min(best, E)
    return best
