"""Tolerances of the GPU parity tests, each derived from the arithmetic.

Scores (Def. 2) of the sketched top-k subspace.
    The GPU runs the range finder's products in FP32 (or, for the first q
    power iterations of the BF16 path, on BF16-rounded operands).  A
    floating-point inner product of length K is the exact product of operands
    perturbed elementwise by at most gamma_K = K u relatively, and for
    rounding errors that behave like independent random variables by about
    sqrt(K) u (the probabilistic bound of Higham and Mary, SIAM J. Sci.
    Comput. 41 (2019)).  So the GPU's scores are the exact scores of a matrix
    within that perturbation of A.  How far such a perturbation moves the
    scores depends on the spectrum (the gap after k, the convergence of the
    sketch), so it is measured rather than bounded: the FP64 twin is re-run on
    A o (1 + eps R), R a random +-1 matrix, and d = max_g |l_g(perturbed) -
    l_g| / (k/G) over a few draws of R.  The gate is
        |l_g(GPU) - l_g(twin)| <= tau max(l_g, k/G),  tau = max(16 u32, 4 d)
    (the factor 4 covers the unknown constant of the probabilistic bound and
    the FP32 roundings the model leaves out: the stored bases Q and V_k, each
    a relative u32 per entry; 16 u32 is the change of a score from rounding
    V_k alone).  eps = sqrt(K) u32 with K = max(m, n) for an FP32 pass; on the
    BF16 path the first q iterations use eps = 2 u_bf16 = 2^-7 (A, Q and A Q
    each rounded to BF16, about 2 u_bf16 for their combined RMS) and the last
    iteration and the Rayleigh-Ritz step the FP32 eps.

Least-squares solution U = C^+ A (Sec. 2.1).
    Normal equations in FP32 with one refinement step whose right-hand side
    H - G U is formed in FP32 leave U at the accuracy of a backward-stable
    solve of a perturbed problem.  The perturbation is that of the FP32
    products H = C^T A and C^T C, inner products of length m: by the same
    probabilistic bound about sqrt(m) u32 relatively, and at least 10 u32 for
    the factorization and the solve, so eps = max(10, sqrt(m)) u32.  The
    sensitivity of least squares to such a perturbation (Golub and Van Loan,
    Matrix Computations, Sec. 5.3.8; Wedin) is
        ||dU|| / ||U|| <= eps (2 cond(C) / cos th + cond(C)^2 tan th),
    sin th = ||A - C U|| / ||A||.  Gate: that bound, at least 1e-5.

Row-block variant U = C^+ A R^+.
    Computed in FP64 from the FP32 data (exact widening): C^+ by Cholesky QR2
    (error about u64 cond(C)), R^+ by the normal equations of R R^T (about
    u64 cond(R)^2), then rounded to FP32.  Gate: 8 u32 + 256 u64 (cond(C) +
    cond(R)^2).
"""
from __future__ import annotations

import math

import numpy as np

from oracle import bcur_oracle as O

U32 = 2.0 ** -24
U64 = 2.0 ** -53
UBF16 = 2.0 ** -8


def perturbed(A64: np.ndarray, eps: float, seed: int, chunk: int = 4096) -> np.ndarray:
    """A o (1 + eps R) with R a seeded random +-1 matrix (built in row chunks)."""
    rng = np.random.default_rng(seed)
    out = np.empty_like(A64)
    for i in range(0, A64.shape[0], chunk):
        blk = A64[i:i + chunk]
        sgn = rng.integers(0, 2, size=blk.shape, dtype=np.int8)
        out[i:i + chunk] = blk + eps * blk * (1.0 - 2.0 * sgn)
    return out


def score_gate(A, offsets, k, q, omega, scores_ref, precision="fp32", draws=3, row_offsets=None,
               row_scores_ref=None):
    """Tolerances of the score gate above: a dict with ``tol`` (per block),
    ``tau`` and ``d``, and for the row blocks (scored by U_k; Def. 2 on A^T)
    ``tol_r``, ``tau_r``, ``d_r`` when ``row_offsets`` is given.  The
    reference scores are the twin's from the same test matrix ``omega``."""
    A64 = np.asarray(A, dtype=np.float64)
    G = len(offsets) - 1
    eps32 = math.sqrt(max(A64.shape)) * U32
    d = d_r = 0.0
    for r in range(draws):
        if precision == "bf16" and q > 0:
            Abf = perturbed(A64, 2.0 * UBF16, 9100 + r)
            Q = O.range_finder(Abf, omega, q - 1, k)["Q"]
            del Abf
            Ap = perturbed(A64, eps32, 9000 + r)
            rf = O.range_finder(Ap, Q, 0, k)
        else:
            Ap = perturbed(A64, eps32, 9000 + r)
            rf = O.range_finder(Ap, omega, q, k)
        del Ap
        d = max(d, float(np.abs(O.block_scores(rf["Vk"], offsets) - scores_ref).max()) / (k / G))
        if row_offsets is not None:
            Gr = len(row_offsets) - 1
            d_r = max(d_r, float(np.abs(O.block_scores(rf["Uk"], row_offsets) - row_scores_ref).max()) / (k / Gr))
    tau = max(16.0 * U32, 4.0 * d)
    out = {"tol": tau * np.maximum(scores_ref, k / G), "tau": tau, "d": d}
    if row_offsets is not None:
        tau_r = max(16.0 * U32, 4.0 * d_r)
        out.update(tol_r=tau_r * np.maximum(row_scores_ref, k / (len(row_offsets) - 1)), tau_r=tau_r, d_r=d_r)
    return out


def index_margin_needed(tol: np.ndarray) -> float:
    """Indices must agree when the oracle's smallest sampling margin exceeds
    the largest shift any partial sum of the scores can see: 2 G max tol."""
    return 2.0 * len(tol) * float(np.max(tol))


def u_gate(cond: float, err: float, frob: float, m: int) -> float:
    """Relative Frobenius gate for U = C^+ A with C of m rows (see the module
    docstring)."""
    sin = min(err / frob, 1.0 - 1e-12) if frob > 0 else 0.0
    cos = math.sqrt(1.0 - sin * sin)
    eps = max(10.0, math.sqrt(m)) * U32
    return max(1e-5, eps * (2.0 * cond / cos + cond * cond * sin / cos))


def u_gate_rows(cond_c: float, cond_r: float) -> float:
    """Relative Frobenius gate for the row variant's U = C^+ A R^+."""
    return 8.0 * U32 + 256.0 * U64 * (cond_c + cond_r * cond_r)
