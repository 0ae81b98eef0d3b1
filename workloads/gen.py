"""Seeded synthetic inputs for Block CUR workloads.

This module holds no part of the method's arithmetic: it only draws the
matrices, block partitions and random numbers that both the FP64 oracle and
the GPU path consume.  Everything is generated on the host with
``numpy.random.default_rng(seed)`` so a (recipe, seed) pair names one exact
input.

Random numbers that the method itself draws are produced here and passed in:
  * ``omega``: the n x l Rademacher (+1/-1) test matrix of the randomized
    range finder;
  * ``draws``: one uniform 64-bit word per sampled block (the sampler maps a
    word r to the fraction r / 2**64).

Recipes (sizes and value distributions of the paper's workloads):
  * ``lowrank_haar``: A = U diag(sigma) V^T + nu * N(0, 1), U and V Haar
    random (QR of a Gaussian with the sign of R's diagonal folded in).
  * ``biometric``: m users x n time samples; each row is a Gaussian mix of
    ``n_latent`` AR(1) series (coefficient phi, unit stationary variance) plus
    white noise.  Stands in for the paper's proprietary EDA matrix (Sec. 4.1),
    which is not available.
  * ``gaussian_product``: A = U V with i.i.d. Gaussian factors, the paper's
    synthetic generator for the distributed experiments (Sec. 4.2).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


# --------------------------------------------------------------------------
# block partitions
# --------------------------------------------------------------------------

def contiguous_blocks(n: int, b: int) -> np.ndarray:
    """Offsets of ceil(n/b) contiguous blocks of width b (last one may be short).

    Returns int64 offsets of length G+1 with offsets[0]=0 and offsets[G]=n
    (Sec. 3: G = ceil(n/s) predefined blocks of s columns)."""
    if n <= 0 or b <= 0:
        raise ValueError("n and b must be positive")
    g = -(-n // b)
    off = np.minimum(np.arange(g + 1, dtype=np.int64) * b, n)
    return off.astype(np.int64)


def ragged_blocks(n: int, g: int, seed: int) -> np.ndarray:
    """Offsets of g contiguous blocks of random, unequal widths (each >= 1)."""
    if not (1 <= g <= n):
        raise ValueError("need 1 <= g <= n")
    rng = np.random.default_rng(seed)
    cuts = np.sort(rng.choice(np.arange(1, n), size=g - 1, replace=False)) if g > 1 else np.array([], dtype=np.int64)
    return np.concatenate([[0], cuts, [n]]).astype(np.int64)


# --------------------------------------------------------------------------
# random factors
# --------------------------------------------------------------------------

def haar_orthonormal(rng: np.random.Generator, rows: int, cols: int) -> np.ndarray:
    """rows x cols matrix with orthonormal columns, Haar distributed."""
    g = rng.standard_normal((rows, cols))
    q, r = np.linalg.qr(g)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


def rademacher(n: int, l: int, seed: int) -> np.ndarray:
    """n x l test matrix with i.i.d. +1/-1 entries (float32, row-major)."""
    rng = np.random.default_rng([seed, 0x0A3E6A])
    bits = rng.integers(0, 2, size=(n, l), dtype=np.int8)
    return (1.0 - 2.0 * bits).astype(np.float32)


def draws_u64(count: int, seed: int) -> np.ndarray:
    """``count`` uniform 64-bit words (the sampler's random numbers)."""
    rng = np.random.default_rng([seed, 0x5A3F1E])
    return rng.integers(0, np.iinfo(np.uint64).max, size=count, dtype=np.uint64, endpoint=True)


# --------------------------------------------------------------------------
# matrices
# --------------------------------------------------------------------------

def lowrank_haar(m: int, n: int, sigma: np.ndarray, noise: float, seed: int,
                 dtype=np.float32, chunk_rows: int = 8192) -> np.ndarray:
    """A = U diag(sigma) V^T + noise * N(0,1), built in row chunks.

    The signal is formed in float64 and the sum is rounded once to ``dtype``.
    """
    rng = np.random.default_rng(seed)
    rank = len(sigma)
    u = haar_orthonormal(rng, m, rank)
    v = haar_orthonormal(rng, n, rank)
    sv = (v * np.asarray(sigma, dtype=np.float64)).T          # rank x n
    out = np.empty((m, n), dtype=dtype)
    nrng = np.random.default_rng([seed, 0x401CE])
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        blk = u[r0:r1] @ sv
        if noise:
            blk += noise * nrng.standard_normal((r1 - r0, n))
        out[r0:r1] = blk
    return out


def biometric(m: int, n: int, n_latent: int, phi: float, noise: float, seed: int,
              dtype=np.float32) -> np.ndarray:
    """Rows are Gaussian mixes of AR(1) latent series plus white noise.

    x_t = phi * x_{t-1} + sqrt(1 - phi^2) * eps_t with x_0 ~ N(0,1), so every
    latent series has unit stationary variance."""
    rng = np.random.default_rng(seed)
    eps = rng.standard_normal((n_latent, n))
    x = np.empty((n_latent, n))
    x[:, 0] = eps[:, 0]
    a = np.sqrt(1.0 - phi * phi)
    for t in range(1, n):
        x[:, t] = phi * x[:, t - 1] + a * eps[:, t]
    load = rng.standard_normal((m, n_latent))
    out = load @ x + noise * rng.standard_normal((m, n))
    return out.astype(dtype)


def gaussian_product(m: int, n: int, rank: int, seed: int, dtype=np.float64) -> np.ndarray:
    """A = U V with i.i.d. N(0,1) factors: exactly rank ``rank`` (Sec. 4.2)."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((m, rank)) @ rng.standard_normal((rank, n))).astype(dtype)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    A: np.ndarray                 # m x n, the matrix handed to the GPU (float32)
    offsets: np.ndarray           # G+1 column-block offsets (int64)
    k: int
    s: int
    p: int
    q: int
    omega: np.ndarray             # n x (k+p) Rademacher, float32
    draws: np.ndarray             # uint64 words: s column draws, then s_r row draws
    row_offsets: Optional[np.ndarray] = None
    s_r: int = 0
    A64: Optional[np.ndarray] = None   # pre-rounding float64 data, when the recipe has it
    precision: str = "fp32"

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]

    @property
    def l(self) -> int:
        return self.omega.shape[1]

    @property
    def G(self) -> int:
        return len(self.offsets) - 1


def _finish(name, A, offsets, k, s, p, q, seed, row_offsets=None, s_r=0, A64=None,
            precision="fp32") -> Workload:
    m, n = A.shape
    l = min(k + p, m, n)
    return Workload(name=name, A=np.ascontiguousarray(A, dtype=np.float32), offsets=offsets,
                    k=k, s=s, p=l - k, q=q, omega=rademacher(n, l, seed),
                    draws=draws_u64(s + s_r, seed), row_offsets=row_offsets, s_r=s_r,
                    A64=A64, precision=precision)


def tiny(seed: int = 0) -> Workload:
    """512 x 256, rank-10 signal sigma_i = 1/i with Haar factors, 0.01 noise;
    32 blocks of 8; k=10, s=4.  The float64 data is rounded to float32 for the
    GPU; the oracle consumes that float32 array widened to float64."""
    sig = 1.0 / np.arange(1, 11)
    A64 = lowrank_haar(512, 256, sig, 0.01, seed, dtype=np.float64)
    return _finish("tiny-512x256", A64.astype(np.float32), contiguous_blocks(256, 8),
                   k=10, s=4, p=10, q=2, seed=seed, A64=A64)


def plain_fp32(seed: int = 0, m: int = 8192, n: int = 4096, b: int = 16, k: int = 50,
               s: int = 16) -> Workload:
    """8192 x 4096 float32, rank-50 signal sigma_i = 1/i, 1e-3 Gaussian noise;
    256 blocks of 16; k=50, s=16, two power iterations."""
    sig = 1.0 / np.arange(1, 51)
    A = lowrank_haar(m, n, sig, 1e-3, seed)
    return _finish(f"plain-fp32-{m}x{n}", A, contiguous_blocks(n, b), k=k, s=s, p=10, q=2,
                   seed=seed)


def biometric_cfg(seed: int = 0) -> Workload:
    """1000 users x 20000 samples, 20 AR(1) (phi=0.98) latent series with
    Gaussian loadings + 0.05 noise; 200 blocks of 100 columns; k=20, s=10;
    row-block variant with 50 row blocks of 20 rows, 10 of them sampled."""
    A = biometric(1000, 20000, 20, 0.98, 0.05, seed)
    return _finish("biometric-1000x20000", A, contiguous_blocks(20000, 100), k=20, s=10,
                   p=10, q=2, seed=seed, row_offsets=contiguous_blocks(1000, 20), s_r=10,
                   precision="bf16")


def large_share(seed: int = 0, m: int = 65536, n: int = 16384) -> Workload:
    """65536 x 16384 float32 (4 GiB), rank-100 signal sigma_i = exp(-i/20),
    1e-4 noise; 256 blocks of 64; k=100, s=32."""
    sig = np.exp(-np.arange(1, 101) / 20.0)
    A = lowrank_haar(m, n, sig, 1e-4, seed)
    return _finish(f"large-{m}x{n}", A, contiguous_blocks(n, 64), k=100, s=32, p=10, q=2,
                   seed=seed, precision="bf16")


@dataclasses.dataclass
class ServingSpec:
    """Shape and parameters of one serving request (the matrix is drawn separately)."""
    req_id: int
    m: int
    n: int
    rank: int
    b: int
    s: int
    offsets: np.ndarray

    @property
    def k(self) -> int:
        return self.rank

    @property
    def l(self) -> int:
        return min(self.rank + 10, self.m, self.n)


def serving_spec(req_id: int, m_range=(256, 8192), n_range=(256, 4096)) -> ServingSpec:
    """The request recipe of ``serving_request`` without its matrix: m in
    [256, 8192], n in [256, 4096], rank uniform in [5, 50] (k = rank), block
    width in {8, 16, 32, 64}, s in [4, 32] clamped to min(s, G, m // b)."""
    rng = np.random.default_rng([req_id, 0x5E7E])
    m = int(rng.integers(m_range[0], m_range[1] + 1))
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    rank = int(rng.integers(5, 51))
    b = int(rng.choice([8, 16, 32, 64]))
    s = int(rng.integers(4, 33))
    off = contiguous_blocks(n, b)
    G = len(off) - 1
    rank = min(rank, m, n)
    s = max(1, min(s, G, m // b))
    return ServingSpec(req_id, m, n, rank, b, s, off)


def serving_matrix_device(spec: ServingSpec, device="cuda", noise: float = 1e-3):
    """A = U diag(1/i) V^T + noise N(0, 1) for one serving request, drawn on the
    GPU with a torch generator seeded by the request id (U, V: QR of Gaussian
    matrices with R's diagonal signs folded in, the Haar recipe above), as a
    float32 tensor whose leading dimension is a multiple of 4.  Used where
    thousands of distinct request matrices are needed at once."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(1_000_003 * (spec.req_id + 1))
    r = spec.rank

    def haar(rows):
        q, rr = torch.linalg.qr(torch.randn((rows, r), generator=g, device=device, dtype=torch.float64))
        d = torch.sign(torch.diagonal(rr))
        d[d == 0] = 1.0
        return q * d

    u, v = haar(spec.m), haar(spec.n)
    sig = 1.0 / torch.arange(1, r + 1, device=device, dtype=torch.float64)
    ld = (spec.n + 3) // 4 * 4
    out = torch.empty((spec.m, ld), dtype=torch.float32, device=device)[:, :spec.n]
    a = (u * sig) @ v.T + noise * torch.randn((spec.m, spec.n), generator=g, device=device, dtype=torch.float64)
    out.copy_(a)
    return out


def serving_request(req_id: int, m_range=(256, 8192), n_range=(256, 4096)) -> Workload:
    """One request of the serving mix: m in [256, 8192], n in [256, 4096],
    rank uniform in [5, 50] (sigma_i = 1/i, 1e-3 noise), block width in
    {8,16,32,64}, k = rank, s in [4, 32]; s is clamped to min(s, G, m // b)."""
    rng = np.random.default_rng([req_id, 0x5E7E])
    m = int(rng.integers(m_range[0], m_range[1] + 1))
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    rank = int(rng.integers(5, 51))
    b = int(rng.choice([8, 16, 32, 64]))
    s = int(rng.integers(4, 33))
    off = contiguous_blocks(n, b)
    G = len(off) - 1
    rank = min(rank, m, n)
    s = max(1, min(s, G, m // b))
    sig = 1.0 / np.arange(1, rank + 1)
    A = lowrank_haar(m, n, sig, 1e-3, req_id)
    return _finish(f"req{req_id}-{m}x{n}", A, off, k=rank, s=s, p=10, q=2, seed=req_id)


def small_case(m: int, n: int, b: int, k: int, s: int, seed: int, p: int = 10, q: int = 2,
               rank: Optional[int] = None, noise: float = 1e-3, ragged: bool = False,
               decay: str = "harmonic", sigma: Optional[np.ndarray] = None) -> Workload:
    """Parametric small workload used by the parity tests."""
    r = rank if rank is not None else k
    if sigma is None:
        if decay == "harmonic":
            sigma = 1.0 / np.arange(1, r + 1)
        elif decay == "geometric":
            sigma = 0.8 ** np.arange(r)
        else:
            raise ValueError(decay)
    A = lowrank_haar(m, n, sigma, noise, seed)
    off = ragged_blocks(n, -(-n // b), seed) if ragged else contiguous_blocks(n, b)
    return _finish(f"small-{m}x{n}", A, off, k=k, s=s, p=p, q=q, seed=seed)
