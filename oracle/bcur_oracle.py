"""FP64 CPU oracle for Block CUR (Oswal, Jain, Xu, Eriksson, arXiv 1703.06065).

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
reference that the GPU path is checked against.  Only the tests, the smoke
check of the package entry script and the CPU-baseline leg of the benchmark
may import it.  It shares no code with the HIP path and imports nothing from
the product package.

Everything is float64 NumPy.  Inputs are the float32 arrays handed to the GPU,
widened to float64.  Random numbers that the method draws (the Rademacher test
matrix and the sampler's 64-bit words) are inputs, never drawn here.

Two references are provided:
  * exact  - top-k singular subspaces from a full LAPACK SVD (Sec. 2.1);
  * twin   - the randomized range finder (the sketching replacement for the
             score step that Sec. 3.1 allows) carried out in float64 with the
             same test matrix, so that the GPU's sketch can be compared step
             for step.

Readings taken where the paper is silent or ambiguous (each is listed in the
design notes of the repository):
  R1  sampling probabilities are p_g = l_g / k from the top-k right singular
      vectors of A itself (the block column-subset-selection special case
      R = A of the Remark in Sec. 3.3, with the p_i = l_i/k form of the
      generalized-regression lemma of App. A.1.1);
  R2  sampling is without replacement by default (the footnote of Sec. 4.1
      says the experiments were run that way); with replacement (Alg. 1,
      step 2) is a flag;
  R3  scores are quantized to integers before sampling so that selection is
      exact and independent of summation order (see ``quantize_scores``);
  R4  C is returned unscaled; the weights 1/sqrt(s p) of the sampling matrix S
      (Sec. 3.1) are returned beside the indices.  The residual does not
      depend on them because C C^+ A is a projection (Sec. 2.1);
  R5  duplicated blocks (with replacement) are removed before the fit.

  R11 (Alg. 1) step 1 draws r distinct rows uniformly: the sampler below
      with unit weights on m one-row blocks; R is scaled by 1/sqrt(r p_i) =
      sqrt(m / r) (the sampling matrix S_R of Sec. 3.1);
  R12 (Alg. 1) the scores use the top-kr right singular vectors of R; the
      listing says r, the text says k, so kr is a parameter (r by default);
  R13 (Alg. 1) U = W^+ treats singular values of W at or below
      max(r, c) 2^-24 sigma_1 as zero (W holds FP32 data);
  R14 (Sec. 4.1) U_k is read as (W_k)^+, the pseudoinverse of the best
      rank-k approximation of W: it keeps the k largest singular values of W
      (the best rank-k approximation of W^+ itself would keep the smallest);
  R15 (Alg. 1) a block drawn with zero weight (only when every remaining
      score is zero) enters S with scale 1, since 1/sqrt(s p) is undefined.

Parity unpinned: the (1+eps) relative-error guarantees (Thm. 2, the Remark
of Sec. 3.3, Lemma 3 of App. A.1.1) carry unspecified constants; they are
reported as context only.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


# ---------------------------------------------------------------------------
# Sec. 2.1: norms and singular subspaces
# ---------------------------------------------------------------------------

def frob2(A: np.ndarray) -> float:
    """||A||_F^2 = sum_ij A_ij^2 (Sec. 2.1, Frobenius norm)."""
    A = np.asarray(A, dtype=np.float64)
    return float(np.sum(A * A))


def all_finite(A: np.ndarray) -> bool:
    return bool(np.all(np.isfinite(A)))


def exact_svd(A: np.ndarray):
    """Thin SVD A = U diag(sigma) V^T with sigma descending (Sec. 2.1)."""
    U, s, Vt = np.linalg.svd(np.asarray(A, dtype=np.float64), full_matrices=False)
    return U, s, Vt.T


def exact_right_subspace(A: np.ndarray, k: int) -> np.ndarray:
    """V_{A,k}: the top-k right singular vectors of A as an n x k matrix."""
    _, _, V = exact_svd(A)
    return V[:, :k]


def exact_left_subspace(A: np.ndarray, k: int) -> np.ndarray:
    """U_{A,k}: the top-k left singular vectors of A as an m x k matrix."""
    U, _, _ = exact_svd(A)
    return U[:, :k]


# ---------------------------------------------------------------------------
# Def. 1, Def. 2, Def. 3, Def. 4
# ---------------------------------------------------------------------------

def column_leverage(V: np.ndarray) -> np.ndarray:
    """l_j = ||V_k^T e_j||_2^2 for every column j (Def. 1)."""
    V = np.asarray(V, dtype=np.float64)
    return np.array([float(V[j, :] @ V[j, :]) for j in range(V.shape[0])])


def block_scores(V: np.ndarray, offsets: Sequence[int]) -> np.ndarray:
    """l_g(A, k) = ||V_k^T E_g||_F^2 for every block g (Def. 2).

    ``V`` is n x k; block g holds the columns offsets[g] .. offsets[g+1]-1.
    E_g selects those rows of V, so the score is the sum of squares of that
    slice of V."""
    V = np.asarray(V, dtype=np.float64)
    off = np.asarray(offsets, dtype=np.int64)
    out = np.empty(len(off) - 1)
    for g in range(len(off) - 1):
        blk = V[off[g]:off[g + 1], :]
        out[g] = float(np.sum(blk * blk))
    return out


def block_stable_rank(V: np.ndarray, offsets: Sequence[int]) -> Tuple[float, np.ndarray]:
    """alpha = min_g ||V_k^T E_g||_F^2 / ||V_k^T E_g||_2^2 (Def. 3).

    Returns (alpha, per-block ratios); a block whose slice is zero has no
    defined ratio and is skipped (NaN in the per-block array)."""
    V = np.asarray(V, dtype=np.float64)
    off = np.asarray(offsets, dtype=np.int64)
    ratios = np.full(len(off) - 1, np.nan)
    for g in range(len(off) - 1):
        blk = V[off[g]:off[g + 1], :]
        fro2 = float(np.sum(blk * blk))
        if fro2 > 0.0:
            spec = float(np.linalg.norm(blk, 2))
            ratios[g] = fro2 / (spec * spec)
    return float(np.nanmin(ratios)), ratios


def incoherence(U: np.ndarray) -> float:
    """mu = (m/k) max_i ||U_k^T e_i||_2^2 (Def. 4), U is m x k."""
    U = np.asarray(U, dtype=np.float64)
    m, k = U.shape
    return float(m / k * np.max(np.sum(U * U, axis=1)))


# ---------------------------------------------------------------------------
# The test matrix of the range finder, drawn from a seed
# ---------------------------------------------------------------------------
#
# The sketch needs random numbers of its own (the test matrix Omega).  They
# come from a counter-based generator so that the host and the device draw
# the same matrix from the same seed without exchanging it: Philox4x64-10 of
# Salmon, Moraes, Dror and Shaw ("Parallel random numbers: as easy as 1, 2,
# 3", SC 2011), written here from that definition.

_PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)   # round multipliers
_PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)   # key increments (Weyl)
_MASK64 = (1 << 64) - 1


def philox4x64_10(counter: Sequence[int], key: Sequence[int]) -> List[int]:
    """Philox4x64 with 10 rounds: four 64-bit counter words, two key words.

    A round multiplies words 0 and 2 by the two multipliers (full 128-bit
    products), and forms the new words (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2),
    hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key is bumped by the Weyl constants
    after each round."""
    c = [int(x) & _MASK64 for x in counter]
    k0, k1 = int(key[0]) & _MASK64, int(key[1]) & _MASK64
    for _ in range(10):
        p0 = _PHILOX_M[0] * c[0]
        p1 = _PHILOX_M[1] * c[2]
        c = [((p1 >> 64) ^ c[1] ^ k0) & _MASK64, p1 & _MASK64,
             ((p0 >> 64) ^ c[3] ^ k1) & _MASK64, p0 & _MASK64]
        k0 = (k0 + _PHILOX_W[0]) & _MASK64
        k1 = (k1 + _PHILOX_W[1]) & _MASK64
    return c


def rademacher_omega(n: int, l: int, seed: int) -> np.ndarray:
    """The n x l Rademacher test matrix of seed ``seed`` (l <= 256).

    Row i is one Philox4x64-10 block with counter (i, 0, 0, 0) and key
    (seed, 0); its 256 output bits, word 0 first and the least significant
    bit of a word first, give Omega[i, j] = +1 for a 0 bit j and -1 for a 1
    bit.  A narrower sketch therefore uses the leading columns of a wider one."""
    if not (0 <= l <= 256):
        raise ValueError("the test matrix has at most 256 columns")
    out = np.empty((n, l))
    for i in range(n):
        words = philox4x64_10((i, 0, 0, 0), (seed, 0))
        for j in range(l):
            bit = (words[j >> 6] >> (j & 63)) & 1
            out[i, j] = -1.0 if bit else 1.0
    return out


# ---------------------------------------------------------------------------
# Randomized range finder (sketched scores; Sec. 3.1 allows sketching)
# ---------------------------------------------------------------------------

def range_finder(A: np.ndarray, omega: np.ndarray, q: int, k: int) -> Dict[str, np.ndarray]:
    """Top-k right singular subspace of A from a sketch, in float64.

    Q starts as the test matrix; q+1 times, Q <- orth(A^T (A Q)).  Then a
    Rayleigh-Ritz step: Z = A Q, T = Z^T Z, T = W diag(lam) W^T with lam
    descending, V_k = Q W[:, :k], Ritz singular values sqrt(lam), and the
    matching left vectors U_k = Z W[:, :k] diag(1/sqrt(lam_k)).

    Only span(Q) matters in exact arithmetic; orth is a Householder QR here
    (the GPU uses Cholesky QR, which spans the same space)."""
    A = np.asarray(A, dtype=np.float64)
    Q = np.asarray(omega, dtype=np.float64)
    for _ in range(q + 1):
        Z = A @ Q
        Y = A.T @ Z
        Q, _ = np.linalg.qr(Y)
    Z = A @ Q
    T = Z.T @ Z
    lam, W = np.linalg.eigh(T)
    order = np.argsort(lam)[::-1]
    lam = lam[order]
    W = W[:, order]
    ritz = np.sqrt(np.maximum(lam, 0.0))
    Vk = Q @ W[:, :k]
    with np.errstate(divide="ignore", invalid="ignore"):
        Uk = (Z @ W[:, :k]) / ritz[:k]
    return {"Q": Q, "Vk": Vk, "Uk": Uk, "lam": lam, "ritz": ritz, "W": W}


def score_condition(lam: np.ndarray, k: int) -> float:
    """kappa = lam_1 / (lam_k - lam_{k+1}) of the Ritz values (inf without gap)."""
    if k >= len(lam):
        return 1.0
    gap = lam[k - 1] - lam[k]
    return float(lam[0] / gap) if gap > 0 else math.inf


# ---------------------------------------------------------------------------
# Block sampling (Alg. 1 step 2; the sampling matrix S of Sec. 3.1)
# ---------------------------------------------------------------------------

SCORE_BITS = 62


def _ceil_log2(x: int) -> int:
    return (x - 1).bit_length() if x > 1 else 0


def quantize_scores(scores: Sequence[float]) -> Tuple[List[int], int]:
    """Integer weights q_g = floor(l_g * 2^sh) with one power-of-two scale.

    sh is chosen from the largest score M = f 2^E (f in [0.5, 1)) as
    sh = 62 - ceil(log2 G) - E, so every q_g < 2^(62 - ceil(log2 G)) and the
    total stays below 2^62.  Scaling by a power of two and taking the floor
    are exact in float64, so q is a function of the scores alone.  Returns
    (q, sh); all-zero scores give q = 0 and sh = 0."""
    G = len(scores)
    if G == 0:
        return [], 0
    vals = [float(x) for x in scores]
    for x in vals:
        if not math.isfinite(x) or x < 0.0:
            raise ValueError("scores must be finite and non-negative")
    M = max(vals)
    if M == 0.0:
        return [0] * G, 0
    _, E = math.frexp(M)
    sh = SCORE_BITS - _ceil_log2(G) - E
    return [int(math.floor(math.ldexp(x, sh))) for x in vals], sh


def draw_point(r: int, W: int) -> int:
    """floor(r * W / 2^64): the draw r / 2^64 scaled to [0, W)."""
    return (int(r) * int(W)) >> 64


def sample_blocks(scores: Sequence[float], draws: Sequence[int], s: int,
                  replace: bool = False) -> Dict[str, object]:
    """Pick s blocks with probability proportional to their scores.

    For draw t the remaining blocks (all blocks with replacement, the
    not-yet-chosen ones without) are laid out in index order on [0, W), each
    taking a length equal to its integer weight.  The point x = floor(r_t W /
    2^64) falls in exactly one of them, and that block is chosen (the smallest
    j whose running total exceeds x).  A zero-weight block is never chosen
    while any remaining block has positive weight; when none has, the smallest
    remaining index is taken.

    The weight of a chosen block is 1/sqrt(s p_j) with p_j = q_j / sum(q)
    (the scaling of the sampling matrix S in Sec. 3.1); +inf for q_j = 0.
    The margin of draw t is the distance from x to the nearer edge of the
    chosen interval, converted back to score units (2^-sh)."""
    G = len(scores)
    if s < 0 or (not replace and s > G):
        raise ValueError("need 0 <= s <= G without replacement")
    if len(draws) < s:
        raise ValueError("need s draws")
    q, sh = quantize_scores(scores)
    total = sum(q)
    chosen: List[int] = []
    taken = [False] * G
    margins: List[float] = []
    for t in range(s):
        W = sum(q[g] for g in range(G) if replace or not taken[g])
        if W == 0:
            j = next(g for g in range(G) if replace or not taken[g])
            margins.append(0.0)
        else:
            x = draw_point(int(draws[t]), W)
            acc = 0
            j = -1
            for g in range(G):
                if not replace and taken[g]:
                    continue
                lo = acc
                acc += q[g]
                if acc > x:
                    j = g
                    margins.append(math.ldexp(float(min(x - lo, acc - 1 - x)), -sh))
                    break
            assert j >= 0
        chosen.append(j)
        taken[j] = True
    weights = []
    for j in chosen:
        if q[j] == 0:
            weights.append(math.inf)
        else:
            weights.append(math.sqrt(float(total) / (s * float(q[j]))))
    return {"idx": np.array(chosen, dtype=np.int64), "weights": np.array(weights),
            "margins": np.array(margins), "q": q, "shift": sh}


def sampling_matrix(offsets: Sequence[int], idx: Sequence[int], weights: Sequence[float]) -> np.ndarray:
    """Dense S of Sec. 3.1: n x c, the t-th slot of columns holds
    I / sqrt(s p_{j_t}) in the rows of block j_t (blocks may have unequal widths)."""
    off = np.asarray(offsets, dtype=np.int64)
    n = int(off[-1])
    widths = [int(off[j + 1] - off[j]) for j in idx]
    S = np.zeros((n, int(sum(widths))))
    c0 = 0
    for j, w, bw in zip(idx, weights, widths):
        for i in range(bw):
            S[off[j] + i, c0 + i] = w
        c0 += bw
    return S


def selected_columns(offsets: Sequence[int], idx: Sequence[int], dedupe: bool = True) -> np.ndarray:
    """Column indices of the chosen blocks, in selection order (duplicates of a
    block dropped when ``dedupe``)."""
    off = np.asarray(offsets, dtype=np.int64)
    seen = set()
    cols: List[int] = []
    for j in idx:
        j = int(j)
        if dedupe and j in seen:
            continue
        seen.add(j)
        cols.extend(range(int(off[j]), int(off[j + 1])))
    return np.array(cols, dtype=np.int64)


def gather_columns(A: np.ndarray, offsets: Sequence[int], idx: Sequence[int], dedupe: bool = True) -> np.ndarray:
    """C = A S without the scaling: the chosen column blocks side by side."""
    return np.asarray(A)[:, selected_columns(offsets, idx, dedupe)]


def gather_rows(A: np.ndarray, row_offsets: Sequence[int], idx: Sequence[int], dedupe: bool = True) -> np.ndarray:
    """R = S_R^T A without the scaling: the chosen row blocks stacked."""
    return np.asarray(A)[selected_columns(row_offsets, idx, dedupe), :]


# ---------------------------------------------------------------------------
# Fits and residuals (Sec. 2.1 pseudoinverse; Remark of Sec. 3.3)
# ---------------------------------------------------------------------------

def fit_columns(A: np.ndarray, C: np.ndarray) -> Tuple[np.ndarray, float]:
    """U = C^+ A (minimum-norm least squares) and err = ||A - C U||_F,
    the block column-subset-selection error C C^+ A of the Remark, Sec. 3.3."""
    A = np.asarray(A, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    U = np.linalg.lstsq(C, A, rcond=None)[0]
    E = A - C @ U
    return U, float(math.sqrt(float(np.sum(E * E))))


def fit_columns_qr(A: np.ndarray, C: np.ndarray, cols: Optional[Sequence[int]] = None,
                   panel: int = 1024) -> Tuple[float, Optional[np.ndarray]]:
    """err = ||A - C C^+ A||_F for a C of full column rank, by the thin
    Householder QR C = Q R: C C^+ = Q Q^T (Sec. 2.1 projection), so the
    residual of each column panel A_J is A_J - Q (Q^T A_J); panels of
    ``panel`` columns keep the memory at a few m x panel arrays.  With
    ``cols``, also U[:, cols] = R^-1 Q^T A[:, cols] (C^+ A on those columns).
    For a rank-deficient C use ``fit_columns``."""
    A = np.asarray(A)
    C = np.asarray(C, dtype=np.float64)
    Q, R = np.linalg.qr(C)
    n = A.shape[1]
    e2 = 0.0
    for j0 in range(0, n, panel):
        AJ = np.asarray(A[:, j0:j0 + panel], dtype=np.float64)
        E = AJ - Q @ (Q.T @ AJ)
        e2 += float(np.sum(E * E))
    U = None
    if cols is not None:
        AJ = np.asarray(A[:, np.asarray(cols, dtype=np.int64)], dtype=np.float64)
        U = np.linalg.solve(R, Q.T @ AJ)
    return float(math.sqrt(e2)), U


def fit_cur(A: np.ndarray, C: np.ndarray, R: np.ndarray) -> Tuple[np.ndarray, float]:
    """U = C^+ A R^+ and err = ||A - C U R||_F (the CUR fit with both
    projections, Sec. 2.1)."""
    A = np.asarray(A, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    U = np.linalg.pinv(C) @ A @ np.linalg.pinv(R)
    E = A - C @ U @ R
    return U, float(math.sqrt(float(np.sum(E * E))))


def fit_intersection(A: np.ndarray, C: np.ndarray, R: np.ndarray, Wmat: np.ndarray) -> Tuple[np.ndarray, float]:
    """Alg. 1 step 3: U = W^+ with W = R S the scaled intersection, and
    err = ||A - C U R||_F."""
    U = np.linalg.pinv(np.asarray(Wmat, dtype=np.float64))
    E = np.asarray(A, dtype=np.float64) - np.asarray(C, dtype=np.float64) @ U @ np.asarray(R, dtype=np.float64)
    return U, float(math.sqrt(float(np.sum(E * E))))


def pinv_cut(Wmat: np.ndarray, rank_k: int = 0) -> Tuple[np.ndarray, int]:
    """W^+ from the SVD with the cutoff of R13; rank_k > 0 keeps at most the
    rank_k largest singular values, giving (W_k)^+ (R14).  Returns the
    pseudoinverse and the number of singular values kept."""
    W = np.asarray(Wmat, dtype=np.float64)
    Uw, sw, Vtw = np.linalg.svd(W, full_matrices=False)
    if sw.size == 0 or sw[0] == 0.0:
        return np.zeros((W.shape[1], W.shape[0])), 0
    keep = int(np.sum(sw > max(W.shape) * 2.0 ** -24 * sw[0]))
    if rank_k > 0:
        keep = min(keep, rank_k)
    inv = np.zeros_like(sw)
    inv[:keep] = 1.0 / sw[:keep]
    return (Vtw.T * inv) @ Uw.T, keep


def cond2(C: np.ndarray) -> float:
    s = np.linalg.svd(np.asarray(C, dtype=np.float64), compute_uv=False)
    return float(s[0] / s[-1]) if s[-1] > 0 else math.inf


# ---------------------------------------------------------------------------
# The whole path
# ---------------------------------------------------------------------------

def decompose(A: np.ndarray, offsets: Sequence[int], k: int, s: int, omega: Optional[np.ndarray],
              draws: Sequence[int], q: int = 2, replace: bool = False, mode: str = "twin",
              row_offsets: Optional[Sequence[int]] = None, s_r: int = 0,
              with_fit: bool = True) -> Dict[str, object]:
    """Block CUR selection and fit.

    mode "twin": scores from the float64 randomized range finder with the
    given test matrix; mode "exact": scores from a full SVD.  Then s blocks
    are sampled from the first s draws, C is gathered and U = C^+ A fitted
    with its residual.  With ``row_offsets`` and s_r > 0 the row-block variant
    also samples s_r row blocks from draws s .. s+s_r-1 by the row scores
    ||U_k[rows_h, :]||_F^2 (Def. 2 applied to A^T; Corollary 1 uses the same
    left-vector leverage), gathers R and fits U = C^+ A R^+."""
    A64 = np.asarray(A, dtype=np.float64)
    out: Dict[str, object] = {"frob2": frob2(A64), "finite": all_finite(A64)}
    if mode == "twin":
        rf = range_finder(A64, omega, q, k)
        Vk, Uk = rf["Vk"], rf["Uk"]
        out.update(ritz=rf["ritz"], lam=rf["lam"], kappa=score_condition(rf["lam"], k))
    elif mode == "exact":
        U_, sv, V_ = exact_svd(A64)
        Vk, Uk = V_[:, :k], U_[:, :k]
        lam = sv ** 2
        out.update(ritz=sv, lam=lam, kappa=score_condition(lam, k))
    else:
        raise ValueError(mode)
    out["Vk"] = Vk
    scores = block_scores(Vk, offsets)
    out["scores"] = scores
    samp = sample_blocks(scores, draws[:s], s, replace)
    out.update(idx=samp["idx"], weights=samp["weights"], margins=samp["margins"])
    C = gather_columns(A64, offsets, samp["idx"])
    out["cols"] = selected_columns(offsets, samp["idx"])
    if row_offsets is not None and s_r > 0:
        rscores = block_scores(Uk, row_offsets)
        out["row_scores"] = rscores
        rs = sample_blocks(rscores, draws[s:s + s_r], s_r, replace)
        out.update(idx_r=rs["idx"], weights_r=rs["weights"], margins_r=rs["margins"])
        out["rows"] = selected_columns(row_offsets, rs["idx"])
        if with_fit:
            R = gather_rows(A64, row_offsets, rs["idx"])
            U, err = fit_cur(A64, C, R)
            out.update(U=U, err=err)
    elif with_fit:
        U, err = fit_columns(A64, C)
        out.update(U=U, err=err)
    if with_fit:
        out["rel_err"] = out["err"] / math.sqrt(out["frob2"]) if out["frob2"] > 0 else 0.0
    return out


def alg1_rows(m: int, r: int, draws: Sequence[int]) -> np.ndarray:
    """Alg. 1 step 1: r distinct rows, each remaining row equally likely
    (p_i = 1/m; R11): the sampler with unit weights on m one-row blocks."""
    return sample_blocks(np.ones(m), draws, r, replace=False)["idx"]


def alg1_fit(A: np.ndarray, offsets: Sequence[int], rows: Sequence[int], idx: Sequence[int],
             weights: Sequence[float], rank_k: int = 0) -> Dict[str, object]:
    """Alg. 1 step 3 for given row and column draws: R = sqrt(m/r) A[rows],
    C = A S with the first weight of each distinct block (R5, R15), W = R S,
    U = W^+ (R13) or U_k = (W_k)^+ (R14), err = ||A - C U R||_F."""
    A64 = np.asarray(A, dtype=np.float64)
    m = A64.shape[0]
    r = len(rows)
    R = math.sqrt(m / r) * A64[np.asarray(rows, dtype=np.int64), :]
    seen, keep_idx, keep_w = set(), [], []
    for j, wgt in zip(idx, weights):
        if int(j) not in seen:
            seen.add(int(j))
            keep_idx.append(int(j))
            keep_w.append(float(wgt) if math.isfinite(wgt) else 1.0)
    S = sampling_matrix(offsets, keep_idx, keep_w)
    C = A64 @ S
    Wmat = R @ S
    U, rank_w = pinv_cut(Wmat, rank_k)
    E = A64 - C @ U @ R
    return dict(R=R, kept=keep_idx, kept_weights=keep_w, cols=selected_columns(offsets, keep_idx), C=C, W=Wmat,
                U=U, rank_w=rank_w, err=float(math.sqrt(float(np.sum(E * E)))))


def alg1(A: np.ndarray, offsets: Sequence[int], r: int, s: int, omega: Optional[np.ndarray],
         draws: Sequence[int], kr: Optional[int] = None, q: int = 1, replace: bool = False,
         rank_k: int = 0, mode: str = "exact") -> Dict[str, object]:
    """Algorithm 1 of Sec. 3.1 (Block CUR with uniform rows), steps in order.

    1. r rows drawn uniformly (draws[:r]; R11): R = S_R^T A = sqrt(m/r) A[rows].
    2. scores l_g(R, kr) = ||V_{R,kr}^T E_g||_F^2 (Def. 2 on R; R12) from the
       SVD of the small matrix R ("exact", the step as the algorithm states it)
       or from the float64 range finder on R with the test matrix omega
       ("twin"); s blocks drawn from draws[r:r+s] with p_g = l_g / kr.
    3. C = A S with S scaled by 1/sqrt(s p) (Sec. 3.1), W = R S, U = W^+ or
       U_k = (W_k)^+, err = ||A - C U R||_F (alg1_fit)."""
    A64 = np.asarray(A, dtype=np.float64)
    m, n = A64.shape
    kr = r if kr is None else kr
    out: Dict[str, object] = {"frob2": frob2(A64), "finite": all_finite(A64)}
    rows = alg1_rows(m, r, draws[:r])
    R = math.sqrt(m / r) * A64[rows, :]
    if mode == "twin":
        Vr = range_finder(R, omega, q, kr)["Vk"]
    elif mode == "exact":
        Vr = exact_right_subspace(R, kr)
    else:
        raise ValueError(mode)
    scores = block_scores(Vr, offsets)
    samp = sample_blocks(scores, draws[r:r + s], s, replace)
    fit = alg1_fit(A64, offsets, rows, samp["idx"], samp["weights"], rank_k)
    out.update(fit)
    out.update(rows=rows, scores=scores, idx=samp["idx"], weights=samp["weights"], margins=samp["margins"],
               sv_r=np.linalg.svd(A64[rows, :], compute_uv=False),
               rel_err=fit["err"] / math.sqrt(out["frob2"]) if out["frob2"] > 0 else 0.0)
    return out


# ---------------------------------------------------------------------------
# Boosting (Sec. 3.3: Thm. 2 from Lemma 3 by keeping the best of t runs)
# ---------------------------------------------------------------------------

def trial_draws(draws: Sequence[int], i: int, s: int) -> Sequence[int]:
    """The s draws of trial i: words i*s .. i*s+s-1 (independent across trials)."""
    return draws[i * s:(i + 1) * s]


def boost_pick(errs: Sequence[float]) -> int:
    """The kept trial: the smallest error, the first one on ties."""
    best = 0
    for i, e in enumerate(errs):
        if e < errs[best]:
            best = i
    return best


def boost(A: np.ndarray, offsets: Sequence[int], k: int, s: int, omega: Optional[np.ndarray],
          draws: Sequence[int], t: int, q: int = 2, replace: bool = False,
          mode: str = "twin") -> Dict[str, object]:
    """Boosting over t independent samplings (Sec. 3.3): the scores come from
    one top-k subspace V_k (shared by the trials); trial i samples s blocks
    with its own draws, fits U_i = C_i^+ A and err_i = ||A - C_i C_i^+ A||_F;
    the trial with the smallest error is returned (t = ln(1/delta) turns a
    per-run failure probability below 1/e into delta)."""
    base = decompose(A, offsets, k, s, omega, draws[:s], q=q, replace=replace, mode=mode, with_fit=False)
    trials = []
    for i in range(t):
        samp = sample_blocks(base["scores"], trial_draws(draws, i, s), s, replace)
        C = gather_columns(A, offsets, samp["idx"])
        U, err = fit_columns(A, C)
        trials.append({"idx": samp["idx"], "weights": samp["weights"], "margins": samp["margins"], "U": U,
                       "err": err, "cols": selected_columns(offsets, samp["idx"])})
    errs = [tr["err"] for tr in trials]
    b = boost_pick(errs)
    out = {key: base[key] for key in ("frob2", "finite", "scores", "Vk") if key in base}
    for key in ("kappa", "ritz", "lam"):
        if key in base:
            out[key] = base[key]
    out.update(trials=trials, errs=np.array(errs), best=b, idx=trials[b]["idx"], weights=trials[b]["weights"],
               U=trials[b]["U"], err=trials[b]["err"], cols=trials[b]["cols"],
               rel_err=trials[b]["err"] / math.sqrt(out["frob2"]) if out["frob2"] > 0 else 0.0)
    return out


# ---------------------------------------------------------------------------
# Blocks of arbitrary column (row) sets
# ---------------------------------------------------------------------------

def decompose_mapped(A: np.ndarray, offsets: Sequence[int], k: int, s: int, omega: Optional[np.ndarray],
                     draws: Sequence[int], col_map: Optional[Sequence[int]] = None,
                     row_map: Optional[Sequence[int]] = None, **kw) -> Dict[str, object]:
    """Block g holds the columns col_map[offsets[g] .. offsets[g+1]-1] (the E_g
    of Def. 2 may pick any set of columns; the blocks partition the columns),
    and likewise row block h the rows row_map[...].  This is the contiguous
    case on A with its columns (rows) listed in map order: the test matrix
    rows follow the columns, the chosen positions map back through the maps,
    U = C^+ A gets its columns back in A's order; errors are unchanged by the
    reordering (Frobenius norms)."""
    A64 = np.asarray(A, dtype=np.float64)
    m, n = A64.shape
    cm = np.arange(n) if col_map is None else np.asarray(col_map, dtype=np.int64)
    rm = np.arange(m) if row_map is None else np.asarray(row_map, dtype=np.int64)
    if sorted(cm.tolist()) != list(range(n)) or sorted(rm.tolist()) != list(range(m)):
        raise ValueError("the maps must be permutations")
    Ap = A64[np.ix_(rm, cm)]
    om = None if omega is None else np.asarray(omega)[cm]
    out = decompose(Ap, offsets, k, s, om, draws, **kw)
    out["cols"] = cm[np.asarray(out["cols"], dtype=np.int64)]
    if "rows" in out:
        out["rows"] = rm[np.asarray(out["rows"], dtype=np.int64)]
    inv = np.argsort(cm)
    out["Vk"] = np.asarray(out["Vk"])[inv]
    if "U" in out and "rows" not in out:
        out["U"] = np.asarray(out["U"])[:, inv]
    return out


def alg1_boost(A: np.ndarray, offsets: Sequence[int], r: int, s: int, draws: Sequence[int], t: int,
               kr: Optional[int] = None, rank_k: int = 0, replace: bool = False) -> Dict[str, object]:
    """Boosting as Thm. 2 states it (Sec. 3.3): Algorithm 1 run t times with
    independent draws (trial i takes words i(r+s) .. i(r+s)+r+s-1: its r row
    draws, then its s column draws), the run of smallest error kept (the first
    on ties)."""
    runs = [alg1(A, offsets, r, s, None, trial_draws(draws, i, r + s), kr=kr, rank_k=rank_k, replace=replace)
            for i in range(t)]
    errs = [run["err"] for run in runs]
    b = boost_pick(errs)
    out = dict(runs[b])
    out.update(trials=runs, errs=np.array(errs), best=b)
    return out
