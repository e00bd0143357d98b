"""Seeded input recipes.

The paper's test systems (diamond, C60 clusters, Cu256, Si216, Al4000) are
DFT Hamiltonians that are not available; these synthetic matrices stand in
for them.  They have the properties the method relies on (Section
"Methodology"): a real symmetric matrix whose previous-step eigenvectors are
close to the current ones, so the rotated matrix is diagonally dominant.

Recipe (all FP64, numpy PCG64 streams, one seed per ingredient):
  * spectrum: n_occ "occupied" values  -0.8 + u**(2/3)   (density ~ sqrt(E+0.8))
              n-n_occ "unoccupied" values 0.2 + 1.3 u, sorted ascending,
              optional 3-fold exact clusters at every 32nd level;
  * Q = H_1 H_2 ... H_n, H_k = I - 2 u u^T / u^T u, u ~ N(0, I);
  * A = Q diag(lam) Q^T (symmetrised);
  * V_prev = Q exp(K), K antisymmetric Gaussian scaled to ||K||_F = kappa.

Random numbers come from numpy; the dense products use torch so that large
instances can be assembled on a GPU.  The generator never calls the method
under test.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch


@dataclasses.dataclass(frozen=True)
class WorkloadConfig:
    name: str
    n: int
    n_occ: int
    clusters: bool
    kappa: float
    slice_size: int
    halo: int
    iterations: int
    seed_base: int


# Five workloads: plain FP64 small case, FP64 SCF sequence, mixed N=8192,
# batched uneven instances, differentiation.
CONFIGS = {
    "c1_n256": WorkloadConfig("c1_n256", 256, 128, False, 1e-2, 64, 32, 3, 1000),
    "c2_n2048_seq": WorkloadConfig("c2_n2048_seq", 2048, 1024, True, 1e-2, 256, 128, 3, 2000),
    "c3_n8192": WorkloadConfig("c3_n8192", 8192, 2048, True, 5e-3, 256, 128, 3, 3000),
    "c4_batched": WorkloadConfig("c4_batched", 0, 0, False, 1e-2, 128, 64, 3, 4000),
    "c5_grad_n4096": WorkloadConfig("c5_grad_n4096", 4096, 2048, False, 1e-2, 256, 128, 3, 5000),
}

BATCH_SIZES = (384, 512, 768, 1024, 1536, 2048)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def spectrum(n: int, n_occ: int, seed: int, clusters: bool = False) -> np.ndarray:
    """Ascending prescribed eigenvalues (occupied sqrt-DOS band + flat unoccupied band)."""
    g = _rng(seed)
    u_occ = g.random(n_occ)
    u_un = g.random(n - n_occ)
    lam = np.concatenate([-0.8 + u_occ ** (2.0 / 3.0), 0.2 + 1.3 * u_un])
    lam.sort()
    if clusters:
        for j in range(n // 32):
            b = 32 * j
            if b + 2 < n:
                lam[b + 1] = lam[b]
                lam[b + 2] = lam[b]
    return lam


def householder_q(n: int, seed: int, device="cpu", block: int = 64) -> torch.Tensor:
    """Q = H_1 H_2 ... H_n as an explicit n x n FP64 matrix (compact-WY accumulation)."""
    g = _rng(seed)
    Q = torch.eye(n, dtype=torch.float64, device=device)
    for b0 in range(0, n, block):
        nb = min(block, n - b0)
        U = torch.from_numpy(g.standard_normal((nb, n))).to(device).T.contiguous()  # n x nb
        U = U / torch.linalg.vector_norm(U, dim=0, keepdim=True)
        # product H_{b0} ... H_{b0+nb-1} = I - U T U^T, T upper triangular (tau = 2)
        T = torch.zeros(nb, nb, dtype=torch.float64, device=device)
        for j in range(nb):
            T[j, j] = 2.0
            if j:
                T[:j, j] = -2.0 * (T[:j, :j] @ (U[:, :j].T @ U[:, j]))
        Q = Q - (Q @ U) @ (T @ U.T)
    return Q


def antisym_k(n: int, kappa: float, seed: int, device="cpu") -> torch.Tensor:
    g = _rng(seed)
    G = torch.from_numpy(g.standard_normal((n, n))).to(device)
    K = G - G.T
    return K * (kappa / torch.linalg.matrix_norm(K))


def expm_small(K: torch.Tensor, terms: Optional[int] = None) -> torch.Tensor:
    """exp(K) by a Taylor series in Horner form, for ||K||_F <= 0.1.

    With terms=None the series is cut after the first t whose remainder bound
    ||K||_F^(t+1) / (t+1)! falls below 1e-18."""
    n = K.shape[0]
    if terms is None:
        r = float(torch.linalg.matrix_norm(K))
        assert r <= 0.1, "expm_small is meant for small perturbations"
        terms, bound = 1, r * r / 2.0
        while bound > 1e-18:
            terms += 1
            bound *= r / (terms + 1)
    I = torch.eye(n, dtype=K.dtype, device=K.device)
    E = I.clone()
    for j in range(terms, 0, -1):
        E = I + (K @ E) / j
    return E


def prescribed_problem(n: int, n_occ: int, kappa: float, seed_base: int, clusters: bool = False,
                       device="cpu", seeds: Optional[Tuple[int, int, int]] = None):
    """Return (A, V_prev, lam_exact, Q) as FP64 torch tensors on `device` (row-major storage).

    A is exactly symmetric.  Columns of V_prev are the previous eigenvectors,
    ordered by ascending eigenvalue.
    """
    s_lam, s_q, s_k = seeds if seeds is not None else (seed_base + 1, seed_base + 2, seed_base + 3)
    lam = spectrum(n, n_occ, s_lam, clusters)
    Q = householder_q(n, s_q, device)
    lam_t = torch.from_numpy(lam).to(device)
    A = (Q * lam_t[None, :]) @ Q.T
    A = 0.5 * (A + A.T)
    if kappa > 0:
        V = Q @ expm_small(antisym_k(n, kappa, s_k, device))
    else:
        V = Q.clone()
    return A, V, lam, Q


def random_symmetric_unit(n: int, seed: int) -> np.ndarray:
    """Symmetric Gaussian direction with unit Frobenius norm."""
    g = _rng(seed)
    G = g.standard_normal((n, n))
    E = 0.5 * (G + G.T)
    return E / np.linalg.norm(E)


def scf_sequence(A0: torch.Tensor, steps: int, seed_base: int, scale0: float = 1e-2) -> List[torch.Tensor]:
    """A_k = A_{k-1} + E_k, E_k symmetric Gaussian with ||E_k||_F = scale0 * 2^-k, k = 1..steps."""
    out = []
    A = A0
    n = A0.shape[0]
    for k in range(1, steps + 1):
        E = torch.from_numpy(random_symmetric_unit(n, seed_base + 10 + k)).to(A0.device)
        A = A + (scale0 * 2.0 ** (-k)) * E
        out.append(A)
    return out


def batch_sizes(count: int = 64, seed: int = 4004) -> List[int]:
    g = _rng(seed)
    idx = g.integers(0, len(BATCH_SIZES), size=count)
    return [int(BATCH_SIZES[i]) for i in idx]


def batch_instance(b: int, n_b: int, kappa: float = 1e-2, seed_base: int = 4000, device="cpu"):
    s = seed_base + 100 + 10 * b
    return prescribed_problem(n_b, n_b // 2, kappa, seed_base, clusters=False, device=device,
                              seeds=(s + 1, s + 2, s + 3))


def loss_weights(n_occ: int, n: int, seed_base: int = 5000) -> Tuple[np.ndarray, np.ndarray]:
    """w_i ~ U[0,1) for the occupied eigenvalues and the diagonal d ~ N(0,1) of D."""
    w = _rng(seed_base + 5).random(n_occ)
    d = _rng(seed_base + 6).standard_normal(n)
    return w, d


def uniform_layout(n: int, slice_size: int) -> List[int]:
    """Partition offsets 0, m, 2m, ..., n (last slice may be shorter)."""
    offs = list(range(0, n, slice_size)) + [n]
    return offs


def overlap_matrix(n: int, delta: float, seed: int, device="cpu") -> torch.Tensor:
    """Synthetic overlap matrix B = I + delta G G^T / n (G Gaussian, PCG64 seed):
    symmetric positive definite with eigenvalues in about [1, 1 + 4 delta] and
    diagonal near 1 + delta, so I - D^{-1} B has spectral radius about
    3 delta / (1 + delta).  Stands in for the ultrasoft-pseudopotential overlap
    of the paper's Implementation section (B close to, but not, the identity)."""
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    G = torch.randn(n, n, dtype=torch.float64, generator=g).to(device)
    B = (G @ G.T) * (delta / n)
    B = 0.5 * (B + B.T)
    B.diagonal().add_(1.0)
    return B

