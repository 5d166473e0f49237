"""Seeded synthetic inputs shared by the CPU oracle tests and the GPU path.

This module only draws random numbers and evaluates smooth periodic fields;
it contains none of the solver's arithmetic (no operator, energy, transform
or line search).  The paper publishes no datasets: its experiments (Sec. 6)
use smooth periodic data on square boxes, so every workload here is a random
superposition of low Fourier modes sampled at cell centres, following the
cell-centred grid of Sec. 5.1 (cell i has centre (i + 1/2) h, 0-based).

Field recipe (one instance):
  * integer mode vectors k with 0 < |k|_2 <= K, taken over a half space
    (first non-zero component positive) so each real mode appears once;
  * amplitudes a_k, b_k ~ N(0, 1) * A(|k|), with A = 1/(1+|k|^2)^q;
  * value a_k cos(2 pi k.x / L) + b_k sin(2 pi k.x / L) summed at cell centres;
  * the mean is zero by construction (k = 0 excluded);
  * scaled so max|field| = amp, then optional white noise added.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

SEED_BASE = 1607_000


def seed_for(config: int, instance: int = 0) -> int:
    return SEED_BASE + 100 * config + instance


def _half_space_modes(dim: int, K: int) -> np.ndarray:
    rng = np.arange(-K, K + 1)
    grids = np.meshgrid(*([rng] * dim), indexing="ij")
    ks = np.stack([g.ravel() for g in grids], axis=1)
    norm2 = (ks.astype(np.int64) ** 2).sum(axis=1)
    keep = (norm2 > 0) & (norm2 <= K * K)
    ks = ks[keep]
    # half space: first non-zero component positive
    first = np.zeros(len(ks), dtype=np.int64)
    for row, k in enumerate(ks):
        nz = np.nonzero(k)[0][0]
        first[row] = k[nz]
    return ks[first > 0]


def fourier_field(dim: int, n: int, L: float, K: int, q: int, amp: float,
                  seed: int, noise: float = 0.0) -> np.ndarray:
    """Random smooth periodic field on an n^dim cell-centred grid (float64).

    Array layout is x fastest: for dim=2 the numpy shape is (n_y, n_x), for
    dim=3 it is (n_z, n_y, n_x); element [.., j, i] is cell (i, j, ..).
    """
    if K >= n // 2:
        raise ValueError("mode cut-off must stay below the Nyquist index")
    gen = np.random.default_rng(seed)
    ks = _half_space_modes(dim, K)
    knorm2 = (ks.astype(np.float64) ** 2).sum(axis=1)
    A = 1.0 / (1.0 + knorm2) ** q
    a = gen.standard_normal(len(ks)) * A
    b = gen.standard_normal(len(ks)) * A
    h = L / n
    x = (np.arange(n) + 0.5) * h
    # complex coefficient c_k with Re(c_k e^{i theta}) = a cos + b sin
    c = a - 1j * b
    # separable evaluation: E_axis[i, k_axis] = exp(2 pi i k_axis x_i / L)
    kr = np.arange(-K, K + 1)
    E = np.exp(2j * np.pi * np.outer(x, kr) / L)  # (n, 2K+1)
    C = np.zeros((2 * K + 1,) * dim, dtype=np.complex128)
    idx = tuple((ks[:, ax] + K) for ax in range(dim))
    C[idx] = c
    if dim == 2:
        # field[j, i] = sum_{kx,ky} C[kx,ky] E[i,kx] E[j,ky]
        tmp = E @ C  # (i, ky)
        field = (tmp @ E.T).T.real  # (j, i)
    elif dim == 3:
        # contract x, then y, then z
        t1 = np.tensordot(E, C, axes=([1], [0]))      # (i, ky, kz)
        t2 = np.tensordot(E, t1, axes=([1], [1]))     # (j, i, kz)
        t3 = np.tensordot(E, t2, axes=([1], [2]))     # (k, j, i)
        field = t3.real
    else:
        raise ValueError("dim must be 2 or 3")
    field = np.ascontiguousarray(field, dtype=np.float64)
    field *= amp / np.abs(field).max()
    if noise:
        field += noise * gen.standard_normal(field.shape)
    return field


@dataclasses.dataclass
class Workload:
    """One solver instance: problem parameters plus seeded inputs."""
    name: str
    dim: int
    n: int
    L: float
    order: int
    p: float
    s: float
    eps: float
    lam: float
    f: np.ndarray
    g: Optional[np.ndarray] = None
    u_target: Optional[np.ndarray] = None


def config1(n: int = 64) -> Workload:
    """2D fourth order, p=4, [0,12.8]^2, s=0.01, eps=0.1, K=8, A=1/(1+|k|^2)."""
    f = fourier_field(2, n, 12.8, 8, 1, 1.0, seed_for(1))
    return Workload("c1_2d_o4", 2, n, 12.8, 4, 4.0, 0.01, 0.1, 0.0, f)


def config2(p: float = 4.0, n: int = 1024) -> Workload:
    """2D fourth order, [0,25.6]^2, s=0.005, eps=0.05, smooth f + 1e-3 noise."""
    f = fourier_field(2, n, 25.6, 8, 1, 1.0, seed_for(2), noise=1e-3)
    return Workload(f"c2_2d_o4_p{p:g}", 2, n, 25.6, 4, p, 0.005, 0.05, 0.0, f)


def config3(n: int = 256) -> Workload:
    """3D fourth order, p=4, [0,12.8]^3, s=0.01, eps=0.1, K=12, A=1/(1+|k|^2)^2."""
    f = fourier_field(3, n, 12.8, 12, 2, 0.5, seed_for(3))
    return Workload("c3_3d_o4", 3, n, 12.8, 4, 4.0, 0.01, 0.1, 0.0, f)


C4_SIZES = (128, 192, 256, 384, 512)


def config4_sizes(batch: int = 64) -> List[int]:
    gen = np.random.default_rng(seed_for(4, 99))
    return [int(v) for v in gen.choice(C4_SIZES, batch)]


def config4(batch: int = 64, sizes: Optional[List[int]] = None) -> List[Workload]:
    """Batch of 2D sixth-order (u,w) instances, p=4, lambda=1, s=0.02, eps=0.1."""
    if sizes is None:
        sizes = config4_sizes(batch)
    out = []
    for i, n in enumerate(sizes):
        f = fourier_field(2, n, 12.8, 10, 1, 1.0, seed_for(4, 2 * i))
        g = fourier_field(2, n, 12.8, 10, 1, 1.0, seed_for(4, 2 * i + 1))
        out.append(Workload(f"c4_2d_o6_{i}_n{n}", 2, n, 12.8, 6, 4.0, 0.02, 0.1, 1.0,
                            f, g=g))
    return out


def config5(batch: int = 8, n: int = 128) -> List[Workload]:
    """Batch of 3D fourth-order solves with a target field for the adjoint."""
    out = []
    for i in range(batch):
        f = fourier_field(3, n, 12.8, 12, 2, 0.5, seed_for(5, 2 * i))
        ut = fourier_field(3, n, 12.8, 12, 2, 0.5, seed_for(5, 2 * i + 1))
        out.append(Workload(f"c5_3d_o4_{i}", 3, n, 12.8, 4, 4.0, 0.01, 0.1, 0.0, f,
                            u_target=ut))
    return out


def small_field(dim: int, n: int, L: float, seed: int, K: int = 3, amp: float = 1.0,
                noise: float = 0.0) -> np.ndarray:
    """Small-case helper used by tests (same recipe, reduced cut-off)."""
    K = min(K, n // 2 - 1)
    return fourier_field(dim, n, L, K, 1, amp, seed, noise=noise)


def white_noise(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    return scale * np.random.default_rng(seed).standard_normal(shape)
