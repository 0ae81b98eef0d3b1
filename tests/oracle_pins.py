"""Pins that tie the FP64 oracle to facts other than itself.

Each ``check_*`` takes an object exposing the oracle's functions (the real
module, or a copy with one function replaced by a planted mistake) and raises
AssertionError when the fact does not hold.  The facts come from the paper
(definitions, the worked example of S, the identities in the appendix
proofs) and from mathematics (Eckart-Young, closed forms, library routines,
brute force), never from re-typing the oracle's own formula.
"""
from __future__ import annotations

import itertools
import math
import os

import numpy as np

from workloads import gen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rank_k(m, n, k, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, k)) @ rng.standard_normal((k, n))


# --------------------------------------------------------------------------
# Sec. 2.1: Frobenius norm = sum of squared singular values
# --------------------------------------------------------------------------

def check_frob_closed_form(O):
    rng = np.random.default_rng(1)
    for (m, n) in [(7, 5), (40, 90), (128, 33)]:
        A = rng.standard_normal((m, n))
        sv = np.linalg.svd(A, compute_uv=False)
        want = float(np.sum(sv ** 2))
        got = O.frob2(A)
        assert abs(got - want) <= 1e-12 * want, (got, want)


# --------------------------------------------------------------------------
# Def. 1 / Def. 2: block leverage scores
# --------------------------------------------------------------------------

def check_scores_sum_to_k(O):
    """||V_k||_F^2 = k for any orthonormal V_k (used in the proof of the
    regression lemma, App. A.1.1), so the block scores sum to k."""
    rng = np.random.default_rng(2)
    for (n, k, b, ragged) in [(64, 5, 8, False), (200, 17, 7, False), (333, 30, 16, True)]:
        V, _ = np.linalg.qr(rng.standard_normal((n, k)))
        off = gen.ragged_blocks(n, -(-n // b), 3) if ragged else gen.contiguous_blocks(n, b)
        sc = O.block_scores(V, off)
        assert abs(float(np.sum(sc)) - k) <= 1e-12 * k, float(np.sum(sc))


def check_scores_from_projector(O):
    """For an exactly rank-k A, V_k V_k^T = A^+ A, so a block's score is the
    trace of that projector's diagonal block (and b = 1 gives the column
    leverage of Def. 1 as the projector's diagonal).  A^+ comes from
    numpy.linalg.pinv, an independent route."""
    A = _rank_k(60, 48, 6, 4)
    P = np.linalg.pinv(A) @ A
    V = O.exact_right_subspace(A, 6)
    off = gen.contiguous_blocks(48, 5)
    sc = O.block_scores(V, off)
    want = np.array([np.trace(P[off[g]:off[g + 1], off[g]:off[g + 1]]) for g in range(len(off) - 1)])
    assert np.allclose(sc, want, atol=1e-10), np.abs(sc - want).max()
    lev = O.column_leverage(V)
    assert np.allclose(lev, np.diag(P), atol=1e-10)
    b1 = O.block_scores(V, np.arange(49))
    assert np.allclose(b1, np.diag(P), atol=1e-10)


def check_scores_bounds_permutation(O):
    """0 <= l_g <= min(b_g, k); one block holds all k; permuting whole blocks
    of A's columns permutes the scores (Def. 2)."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((50, 40)) @ np.diag(0.9 ** np.arange(40))
    k = 7
    off = gen.contiguous_blocks(40, 4)
    V = O.exact_right_subspace(A, k)
    sc = O.block_scores(V, off)
    widths = np.diff(off)
    assert np.all(sc >= -1e-15) and np.all(sc <= np.minimum(widths, k) + 1e-12)
    one = O.block_scores(V, np.array([0, 40]))
    assert abs(one[0] - k) <= 1e-12
    perm = rng.permutation(len(off) - 1)
    cols = np.concatenate([np.arange(off[g], off[g + 1]) for g in perm])
    Vp = O.exact_right_subspace(A[:, cols], k)
    scp = O.block_scores(Vp, off)
    assert np.allclose(scp, sc[perm], atol=1e-9)


def check_row_scores_transpose(O):
    """Row-block scores from U_k equal column-block scores of A^T (Sec. 3:
    row blocks are handled by transposing)."""
    A = np.random.default_rng(6).standard_normal((36, 24))
    roff = gen.contiguous_blocks(36, 6)
    s1 = O.block_scores(O.exact_left_subspace(A, 5), roff)
    s2 = O.block_scores(O.exact_right_subspace(A.T, 5), roff)
    assert np.allclose(s1, s2, atol=1e-10)


# --------------------------------------------------------------------------
# Randomized range finder vs exact SVD
# --------------------------------------------------------------------------

def check_twin_exact_on_low_rank(O):
    """If rank(A) = rho <= l the sketch spans A's row space exactly, so the
    Rayleigh-Ritz vectors are the exact singular vectors (Sec. 2.1) and the
    scores agree with the SVD's to rounding; the Ritz values are the singular
    values."""
    for (m, n, rho, k, l, seed) in [(300, 200, 15, 10, 20, 7), (120, 260, 8, 8, 12, 8)]:
        A = gen.gaussian_product(m, n, rho, seed)
        om = gen.rademacher(n, l, seed)
        rf = O.range_finder(A, om, 1, k)
        off = gen.contiguous_blocks(n, 10)
        ex = O.block_scores(O.exact_right_subspace(A, k), off)
        tw = O.block_scores(rf["Vk"], off)
        assert np.allclose(tw, ex, atol=1e-10), np.abs(tw - ex).max()
        sv = np.linalg.svd(A, compute_uv=False)
        assert np.allclose(rf["ritz"][:rho], sv[:rho], rtol=1e-10)


def check_twin_converges(O):
    """With a clear gap after k, more power iterations move the sketched
    scores toward the exact ones (subspace iteration converges)."""
    w = gen.small_case(400, 300, 10, 8, 4, seed=9, sigma=np.r_[np.linspace(1, 0.5, 8), 0.05 * np.ones(4)],
                       rank=12, noise=1e-3)
    A = w.A.astype(np.float64)
    ex = O.block_scores(O.exact_right_subspace(A, 8), w.offsets)
    errs = [np.abs(O.block_scores(O.range_finder(A, w.omega, q, 8)["Vk"], w.offsets) - ex).max() for q in (0, 1, 3)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-8, errs


def check_twin_left_vectors_on_low_rank(O):
    """On an exactly rank-rho A (rho <= l, distinct singular values) the
    twin's left vectors U_k = Z W_k / sigma_k are the exact top-k left
    singular vectors up to column signs (A v_i = sigma_i u_i, Sec. 2.1):
    orthonormal, |U_k^T U_exact| = I, and the row-block scores read off them
    equal the exact row leverage of the blocks (Def. 2 on A^T, Corollary 1).
    The exact vectors come from numpy's SVD, not from the oracle."""
    for (m, n, rho, k, l, seed) in [(300, 200, 15, 10, 20, 7), (120, 260, 8, 6, 12, 8)]:
        A = gen.gaussian_product(m, n, rho, seed)
        rf = O.range_finder(A, gen.rademacher(n, l, seed), 1, k)
        Uk = np.asarray(rf["Uk"])
        assert Uk.shape == (m, k), Uk.shape
        assert np.abs(Uk.T @ Uk - np.eye(k)).max() <= 1e-10, np.abs(Uk.T @ Uk - np.eye(k)).max()
        Ue = np.linalg.svd(A, full_matrices=False)[0][:, :k]
        assert np.abs(np.abs(Uk.T @ Ue) - np.eye(k)).max() <= 1e-9
        roff = gen.contiguous_blocks(m, 12)
        want = np.add.reduceat(np.sum(Ue * Ue, axis=1), roff[:-1])
        assert np.allclose(O.block_scores(Uk, roff), want, atol=1e-10)


def check_score_condition_first_order(O):
    """kappa = lam_1 / (lam_k - lam_{k+1}) is the first-order sensitivity of
    the top-k eigenspace of T to a perturbation of relative size eps: the
    symmetric perturbation eps lam_1 (e_k e_{k+1}^T + e_{k+1} e_k^T) of
    T = diag(lam) turns that eigenspace by the angle eps kappa + O(eps^2)
    (the 2 x 2 rotation that diagonalizes rows k, k+1).  The angle is measured
    with numpy's eigh on planted spectra whose gaps differ from position to
    position, so a gap taken one place off changes the answer."""
    spectra = [np.array([9.0, 7.5, 5.0, 4.2, 4.0, 1.0, 0.7, 0.2]),
               np.array([1.0, 0.5, 0.3, 0.29, 0.1, 0.05]),
               np.array([3.0, 2.0, 1.97, 1.0, 0.9, 0.89, 0.3])]
    eps = 1e-8
    for lam in spectra:
        for k in range(1, len(lam) - 1):
            T = np.diag(lam)
            T[k - 1, k] = T[k, k - 1] = eps * lam[0]
            ev, V = np.linalg.eigh(T)
            Vk = V[:, np.argsort(ev)[::-1][:k]]
            sin = float(np.linalg.norm(Vk[k:, :], 2))
            got = O.score_condition(lam, k)
            assert abs(got - sin / eps) <= 1e-4 * got, (k, got, sin / eps)
    assert O.score_condition(np.array([2.0, 1.0, 1.0]), 1) < math.inf
    assert O.score_condition(np.array([2.0, 1.0, 1.0]), 2) == math.inf


def check_cond2_planted(O):
    """cond(C) = sigma_max / sigma_min for a planted SVD C = U diag(sigma) V^T
    (Haar U and V), and equals ||C||_2 ||C^+||_2 with numpy's pinv."""
    rng = np.random.default_rng(33)
    for (m, c, lo, hi) in [(50, 8, 1e-3, 2.0), (200, 40, 0.5, 7.0), (30, 30, 1e-6, 1.0)]:
        sig = np.exp(rng.uniform(math.log(lo), math.log(hi), size=c))
        sig[0], sig[-1] = hi, lo
        C = gen.haar_orthonormal(rng, m, c) @ np.diag(sig) @ gen.haar_orthonormal(rng, c, c).T
        got = O.cond2(C)
        assert abs(got - hi / lo) <= 1e-6 * hi / lo, (got, hi / lo)
        alt = np.linalg.norm(C, 2) * np.linalg.norm(np.linalg.pinv(C, rcond=1e-14), 2)
        assert abs(got - alt) <= 1e-6 * alt


# --------------------------------------------------------------------------
# The seeded test matrix (Philox4x64-10)
# --------------------------------------------------------------------------

def check_omega_philox_library(O):
    """The oracle's Philox4x64-10 against numpy's Philox bit generator, an
    independent library implementation of the same published generator.
    numpy advances its 256-bit counter before each block, so the state
    counter c yields the block of counter c + 1 (all ones wraps to zero);
    keys and counters go in as uint64 arrays (a Python list above 2^63
    would pass through a float cast).
    The test matrix rows are then read off numpy's stream: bit j of a row's
    256 bits (word 0 first, least significant bit first) gives +1 for 0 and
    -1 for 1; a narrower sketch takes the leading columns."""
    rng = np.random.default_rng(31)
    mask = (1 << 64) - 1
    for _ in range(8):
        key = [int(x) for x in rng.integers(0, 2 ** 63, size=2)]
        ctr = [int(x) for x in rng.integers(0, 2 ** 62, size=4)]
        want = [int(x) for x in np.random.Philox(counter=ctr, key=key).random_raw(4)]
        assert O.philox4x64_10([ctr[0] + 1] + ctr[1:], key) == want
    want0 = [int(x) for x in np.random.Philox(counter=np.full(4, mask, dtype=np.uint64),
                                               key=np.array([5, 0], dtype=np.uint64)).random_raw(4)]
    assert O.philox4x64_10([0, 0, 0, 0], [5, 0]) == want0
    n, l = 37, 112
    for seed in (0, 987654321, (1 << 64) - 3):
        om = O.rademacher_omega(n, l, seed)
        for i in range(n):
            ctr = [mask] * 4 if i == 0 else [i - 1, 0, 0, 0]
            words = np.random.Philox(counter=np.array(ctr, dtype=np.uint64),
                                     key=np.array([seed, 0], dtype=np.uint64)).random_raw(4).astype("<u8")
            bits = np.unpackbits(words.view(np.uint8), bitorder="little")
            assert np.array_equal(om[i], 1.0 - 2.0 * bits[:l].astype(np.float64)), (seed, i)
        assert np.array_equal(O.rademacher_omega(n, 60, seed), om[:, :60])
    big = O.rademacher_omega(2000, 64, 11)
    assert set(np.unique(big)) == {-1.0, 1.0}
    assert abs(float(big.mean())) <= 5.0 / math.sqrt(big.size)
    assert not np.array_equal(O.rademacher_omega(4, 64, 1), O.rademacher_omega(4, 64, 2))


# --------------------------------------------------------------------------
# Sampling (Alg. 1 step 2, the sampling matrix S of Sec. 3.1)
# --------------------------------------------------------------------------

def check_sampler_inverse_cdf(O):
    """With replacement, the chosen block is the inverse-CDF pick of the
    integer weights: numpy.searchsorted(cumsum(q), x, side='right')."""
    rng = np.random.default_rng(10)
    for trial in range(40):
        G = int(rng.integers(1, 60))
        sc = rng.random(G) * (rng.random(G) < 0.8)
        if sc.max() == 0:
            sc[0] = 1.0
        s = int(rng.integers(1, 10))
        dr = gen.draws_u64(s, trial)
        res = O.sample_blocks(sc, dr, s, replace=True)
        q, _ = O.quantize_scores(sc)
        cs = np.cumsum(np.array(q, dtype=np.int64))      # total < 2^62: exact in int64
        W = int(cs[-1])
        for t in range(s):
            x = (int(dr[t]) * W) >> 64
            want = int(np.searchsorted(cs, x, side="right"))
            assert res["idx"][t] == want


def check_sampler_edges(O):
    """Draws that land exactly on interval edges, the extreme words 0 and
    2^64-1, and zero-score blocks: block g owns [Q_{g-1}, Q_g) of the integer
    line, so a point on an edge belongs to the block on its right, and a
    zero-score block (an empty interval) is never hit.  Expected blocks come
    from numpy.searchsorted(side='right') on the integer prefix sums."""
    for sc in ([0.0, 1.0, 0.0, 1.0, 0.0], [0.25, 0.25, 0.5], [3.0], [0.0, 0.0, 2.0], [1.0, 0.0, 0.0]):
        q, _ = O.quantize_scores(sc)
        cs = np.cumsum(np.array(q, dtype=np.int64))
        W = int(cs[-1])
        words = [0, 2 ** 64 - 1]
        for B in [0] + [int(v) for v in cs[:-1]]:
            r = -(-(B << 64) // W)            # smallest r with floor(r W / 2^64) = B
            if r < 2 ** 64:
                words.append(r)
        for r in words:
            res = O.sample_blocks(sc, np.array([r], dtype=np.uint64), 1, replace=True)
            x = (r * W) >> 64
            want = int(np.searchsorted(cs, x, side="right"))
            assert res["idx"][0] == want, (sc, r, res["idx"][0], want)
            assert q[want] > 0
    # all remaining scores zero: the smallest remaining index is taken
    res = O.sample_blocks([0.0, 5.0, 0.0, 0.0], gen.draws_u64(3, 21), 3, replace=False)
    assert list(res["idx"]) == [1, 0, 2]
    assert math.isinf(res["weights"][1])


def check_sampler_quantization_exact(O):
    """Quantized weights are proportional to the scores to 2^-(62-ceil(log2 G))
    of the largest score, and scaling all scores by a power of two leaves
    them unchanged (the scale is a power of two chosen from the maximum)."""
    rng = np.random.default_rng(11)
    sc = rng.random(300)
    q, sh = O.quantize_scores(sc)
    qa = np.array(q, dtype=np.float64)
    assert np.all(np.abs(qa / 2.0 ** sh - sc) <= 2.0 ** -sh)
    q2, _ = O.quantize_scores(sc * 8.0)
    assert q2 == q
    assert sum(q) < 2 ** 62


def check_sampler_without_replacement_law(O):
    """Without replacement, P(first = a, second = b) = p_a p_b / (1 - p_a)
    (successive sampling).  Chi-square test over all ordered pairs."""
    sc = np.array([0.1, 0.4, 0.2, 0.3])
    p = sc / sc.sum()
    N = 20000
    dr = gen.draws_u64(2 * N, 12)
    counts = np.zeros((4, 4))
    for i in range(N):
        r = O.sample_blocks(sc, dr[2 * i:2 * i + 2], 2, replace=False)["idx"]
        counts[r[0], r[1]] += 1
    exp = np.array([[p[a] * p[b] / (1 - p[a]) if a != b else 0 for b in range(4)] for a in range(4)]) * N
    mask = exp > 0
    chi2 = float(np.sum((counts[mask] - exp[mask]) ** 2 / exp[mask]))
    assert counts[~mask].sum() == 0
    assert chi2 < 32.9, chi2   # 11 dof, p = 0.0005


def check_sampler_frequencies(O):
    """With replacement, block frequencies follow p_g = l_g / sum(l)."""
    sc = np.array([0.05, 0.0, 0.5, 0.25, 0.2])
    N = 40000
    res = O.sample_blocks(sc, gen.draws_u64(N, 13), N, replace=True)
    cnt = np.bincount(res["idx"], minlength=5)
    p = sc / sc.sum()
    mask = p > 0
    chi2 = float(np.sum((cnt[mask] - N * p[mask]) ** 2 / (N * p[mask])))
    assert cnt[1] == 0
    assert chi2 < 18.5, chi2   # 3 dof, p = 0.0003


def check_unbiased_scaling(O):
    """E ||Q S||_F^2 = ||Q||_F^2 for the i.i.d. sampling with weights
    1/sqrt(g p) (the expectation computed in the proof of the regression
    lemma, App. A.1.1).  Monte Carlo against the closed form."""
    rng = np.random.default_rng(14)
    Qm = rng.standard_normal((5, 24))
    off = gen.contiguous_blocks(24, 4)
    sc = np.array([np.sum(Qm[:, off[g]:off[g + 1]] ** 2) for g in range(6)])
    g = 3
    T = 6000
    dr = gen.draws_u64(g * T, 15)
    vals = np.empty(T)
    for t in range(T):
        res = O.sample_blocks(sc, dr[g * t:g * t + g], g, replace=True)
        S = O.sampling_matrix(off, res["idx"], res["weights"])
        vals[t] = np.sum((Qm @ S) ** 2)
    want = float(np.sum(Qm ** 2))
    # with p proportional to ||Q^(i)||_F^2 the estimator has zero variance
    assert np.allclose(vals, want, rtol=1e-9)
    # and with other probabilities it is unbiased
    sc2 = np.array([1.0, 2.0, 1.0, 0.5, 3.0, 1.5])
    for t in range(T):
        res = O.sample_blocks(sc2, dr[g * t:g * t + g], g, replace=True)
        S = O.sampling_matrix(off, res["idx"], res["weights"])
        vals[t] = np.sum((Qm @ S) ** 2)
    se = vals.std() / math.sqrt(T)
    assert abs(vals.mean() - want) < 4 * se, (vals.mean(), want, se)


def check_block_product_variance(O):
    """Block multiplication lemma (App. A.2 proof): E[C R] = A B and
    E||AB - CR||_F^2 = sum_k ||A^(k) B_(k)||_F^2 / (g p_k) - ||AB||_F^2 / g
    exactly, for C = A S and R = S^T B."""
    rng = np.random.default_rng(16)
    A = rng.standard_normal((4, 18))
    B = rng.standard_normal((18, 3))
    off = gen.contiguous_blocks(18, 3)
    G = 6
    sc = np.array([1.0, 0.5, 2.0, 1.0, 0.25, 1.25])
    p = sc / sc.sum()
    g = 2
    T = 20000
    dr = gen.draws_u64(g * T, 17)
    AB = A @ B
    errs = np.empty(T)
    acc = np.zeros_like(AB)
    for t in range(T):
        res = O.sample_blocks(sc, dr[g * t:g * t + g], g, replace=True)
        S = O.sampling_matrix(off, res["idx"], res["weights"])
        CR = (A @ S) @ (S.T @ B)
        acc += CR
        errs[t] = np.sum((AB - CR) ** 2)
    blk = [np.sum((A[:, off[i]:off[i + 1]] @ B[off[i]:off[i + 1], :]) ** 2) for i in range(G)]
    want = sum(blk[i] / (g * p[i]) for i in range(G)) - np.sum(AB ** 2) / g
    se = errs.std() / math.sqrt(T)
    assert abs(errs.mean() - want) < 4 * se, (errs.mean(), want, se)
    assert np.abs(acc / T - AB).max() < 0.1 * np.abs(AB).max()


def check_sampling_matrix_example(O):
    """The worked example of Sec. 3.1: blocks chosen in order [1, 3, 2]."""
    pat = np.loadtxt(os.path.join(GOLDEN, "sampling_matrix_example.txt"), dtype=np.int64)
    b = 2
    off = gen.contiguous_blocks(4 * b, b)
    p = np.array([0.4, 0.3, 0.2, 0.1])
    g = 3
    idx = np.array([0, 2, 1])
    w = 1.0 / np.sqrt(g * p[idx])
    S = O.sampling_matrix(off, idx, w)
    assert S.shape == (4 * b, g * b)
    for i in range(4):
        for t in range(g):
            blk = S[i * b:(i + 1) * b, t * b:(t + 1) * b]
            j = pat[i, t]
            want = np.zeros((b, b)) if j == 0 else np.eye(b) / math.sqrt(g * p[j - 1])
            assert np.allclose(blk, want), (i, t, blk)


# --------------------------------------------------------------------------
# Fits and residuals
# --------------------------------------------------------------------------

def check_fit_projection(O):
    """U = C^+ A satisfies the normal equations C^T (A - C U) = 0, selecting
    every block gives C C^+ A = A, and the error is not below the best
    rank-rank(C) error (Eckart-Young, Sec. 2.1); nested selections never
    increase it."""
    w = gen.tiny()
    A = w.A.astype(np.float64)
    off = w.offsets
    C = O.gather_columns(A, off, [3, 7, 11])
    U, err = O.fit_columns(A, C)
    assert np.abs(C.T @ (A - C @ U)).max() <= 1e-10 * np.abs(A).max() * np.abs(C).max() * A.shape[0]
    sv = np.linalg.svd(A, compute_uv=False)
    r = np.linalg.matrix_rank(C)
    assert err >= math.sqrt(np.sum(sv[r:] ** 2)) * (1 - 1e-12)
    _, e_all = O.fit_columns(A, O.gather_columns(A, off, list(range(w.G))))
    assert e_all <= 1e-10 * math.sqrt(O.frob2(A))
    prev = math.inf
    for s in range(1, 8):
        _, e = O.fit_columns(A, O.gather_columns(A, off, list(range(0, 4 * s, 4))))
        assert e <= prev * (1 + 1e-12)
        prev = e


def check_fit_qr_route(O):
    """For a C of full column rank the QR route gives the minimum-norm least
    squares solution too: its err and U columns equal numpy's SVD-based
    lstsq, panel by panel (several panel widths, a ragged last panel)."""
    rng = np.random.default_rng(34)
    for (m, n, c) in [(200, 90, 17), (100, 300, 64), (500, 33, 5)]:
        A = rng.standard_normal((m, n))
        C = rng.standard_normal((m, c)) @ np.diag(np.logspace(0, -3, c))
        U_ref, res, _, _ = np.linalg.lstsq(C, A, rcond=None)
        e_ref = math.sqrt(float(np.sum((A - C @ U_ref) ** 2)))
        for panel in (7, 32, n):
            cols = [0, n // 2, n - 1]
            err, U = O.fit_columns_qr(A, C, cols=cols, panel=panel)
            assert abs(err - e_ref) <= 1e-10 * e_ref, (err, e_ref)
            assert np.allclose(U, U_ref[:, cols], rtol=1e-8, atol=1e-10 * np.abs(U_ref).max())


def check_fit_selected_columns(O):
    """C C^+ C = C (a Penrose condition, Sec. 2.1), so the residual of the
    fit is zero on the chosen columns and err^2 is the sum over the others;
    with C of full column rank C^+ C = I, so U on the chosen columns is the
    identity (the columns of C in their order).  A repeated block leaves C
    rank-deficient: the residual there is still zero, U there is not I."""
    w = gen.tiny()
    A = w.A.astype(np.float64)
    off = w.offsets
    for idx in ([5, 1, 30, 17], [0], [31, 2, 9, 8, 14, 22]):
        cols = O.selected_columns(off, idx)
        C = A[:, cols]
        U, err = O.fit_columns(A, C)
        assert np.abs(U[:, cols] - np.eye(len(cols))).max() <= 1e-9
        E = A - C @ U
        assert np.abs(E[:, cols]).max() <= 1e-12 * np.abs(A).max()
        rest = np.setdiff1d(np.arange(A.shape[1]), cols)
        assert abs(math.sqrt(float(np.sum(E[:, rest] ** 2))) - err) <= 1e-12 * err
    cols = O.selected_columns(off, [4, 4, 6], dedupe=False)
    C = A[:, cols]
    U, err = O.fit_columns(A, C)
    E = A - C @ U
    assert np.abs(E[:, cols]).max() <= 1e-12 * np.abs(A).max()
    assert np.abs(U[:, cols] - np.eye(len(cols))).max() > 0.1


def check_fit_bruteforce(O, max_subsets=None):
    """Brute force over every s-subset of blocks of the tiny workload: the
    sampled error lies between the best and worst subset, and equals that
    subset's error computed by an independent formula,
    err^2 = ||A||^2 - tr(G_JJ^-1 (G^2)_JJ) with G = A^T A (projection onto
    span(C), Sec. 2.1)."""
    w = gen.tiny()
    A = w.A.astype(np.float64)
    off = w.offsets
    res = O.decompose(w.A, off, w.k, w.s, w.omega, w.draws, q=w.q)
    Gm = A.T @ A
    G2 = Gm @ Gm
    f2 = float(np.sum(A * A))
    subsets = list(itertools.combinations(range(w.G), w.s))
    if max_subsets:
        subsets = subsets[:max_subsets] + [tuple(sorted(res["idx"]))]
    cols = np.array([np.concatenate([np.arange(off[j], off[j + 1]) for j in sub]) for sub in subsets])
    GJ = Gm[cols[:, :, None], cols[:, None, :]]
    G2J = G2[cols[:, :, None], cols[:, None, :]]
    tr = np.trace(np.linalg.solve(GJ, G2J), axis1=1, axis2=2)
    errs = np.sqrt(np.maximum(f2 - tr, 0.0))
    mine = errs[subsets.index(tuple(sorted(res["idx"])))]
    assert abs(mine - res["err"]) <= 1e-8 * res["err"], (mine, res["err"])
    assert errs.min() * (1 - 1e-12) <= res["err"] <= errs.max() * (1 + 1e-12)
    return errs


def check_cur_reductions(O):
    """Row-block CUR: with R = A (every row block) the CUR error equals the
    column error; when C spans R^m it equals ||A - A R^+ R||_F; and the
    identity A S (B S)^+ B = A S (V_k^T S)^+ V_k^T for rank-k B (App. A.1.1)."""
    rng = np.random.default_rng(18)
    A = rng.standard_normal((30, 50)) @ np.diag(0.9 ** np.arange(50))
    coff = gen.contiguous_blocks(50, 5)
    roff = gen.contiguous_blocks(30, 3)
    C = O.gather_columns(A, coff, [1, 4, 6])
    _, e_col = O.fit_columns(A, C)
    _, e_cur = O.fit_cur(A, C, O.gather_rows(A, roff, list(range(10))))
    assert abs(e_col - e_cur) <= 1e-9 * e_col
    Cfull = O.gather_columns(A, coff, list(range(7)))   # 35 columns span R^30
    R = O.gather_rows(A, roff, [0, 3, 5])
    _, e = O.fit_cur(A, Cfull, R)
    want = np.linalg.norm(A - A @ np.linalg.pinv(R) @ R)
    assert abs(e - want) <= 1e-8 * want
    B = rng.standard_normal((4, 6)) @ rng.standard_normal((6, 50))
    _, _, Vt = np.linalg.svd(B, full_matrices=False)
    Vk = Vt[:6].T
    S = O.sampling_matrix(coff, [0, 2, 5, 7, 9], np.ones(5))
    lhs = A @ S @ np.linalg.pinv(B @ S) @ B
    rhs = A @ S @ np.linalg.pinv(Vk.T @ S) @ Vk.T
    assert np.allclose(lhs, rhs, atol=1e-8)


def check_paper_synthetic_generator(O):
    """The paper's synthetic A = U V (Sec. 4.2) has rank k, so once the chosen
    blocks span its column space, the error is zero to rounding."""
    A = gen.gaussian_product(120, 120, 12, 19)
    off = gen.contiguous_blocks(120, 10)
    res = O.decompose(A, off, 12, 3, gen.rademacher(120, 22, 19), gen.draws_u64(3, 19))
    assert res["err"] <= 1e-9 * math.sqrt(res["frob2"])


# --------------------------------------------------------------------------
# Algorithm 1 (Sec. 3.1): uniform rows, U = W^+ of the scaled intersection
# --------------------------------------------------------------------------

def check_alg1_rows_uniform_distinct(O):
    """Step 1: r distinct rows; with unit weights the draw x = floor(r_t W /
    2^64) picks the x-th remaining row, so the draw 0 takes the first
    remaining row and the draw 2^64 - 1 the last."""
    m = 11
    rows = O.alg1_rows(m, 4, [0, 2 ** 64 - 1, 0, 2 ** 64 - 1])
    assert list(rows) == [0, 10, 1, 9], rows
    rows = O.alg1_rows(m, m, gen.draws_u64(m, 20))
    assert sorted(int(i) for i in rows) == list(range(m))
    # a draw just below (j + 1) / W of the range lands in remaining row j
    W = m
    for j in (0, 3, 10):
        d = ((j + 1) << 64) // W - 1
        assert int(O.alg1_rows(m, 1, [d])[0]) == j


def check_alg1_penrose(O):
    """U = W^+ satisfies the four Penrose conditions (Sec. 2.1), for a full
    rank W and for one with a repeated column."""
    rng = np.random.default_rng(21)
    for W in (rng.standard_normal((7, 5)), rng.standard_normal((5, 9))):
        Wd = np.concatenate([W, W[:, :1]], axis=1)
        for M in (W, Wd):
            U, _ = O.pinv_cut(M)
            assert np.allclose(M @ U @ M, M, atol=1e-10)
            assert np.allclose(U @ M @ U, U, atol=1e-10)
            assert np.allclose((M @ U).T, M @ U, atol=1e-10)
            assert np.allclose((U @ M).T, U @ M, atol=1e-10)


def check_alg1_rank_k(O):
    """U_k = (W_k)^+: W U_k W is the best rank-k approximation of W, so
    ||W - W U_k W||_F^2 is the sum of the squared singular values past k
    (Eckart-Young); U_k equals U once k reaches rank(W); C U_k R has rank k."""
    rng = np.random.default_rng(22)
    W = rng.standard_normal((9, 6)) @ np.diag([5.0, 3.0, 2.0, 1.0, 0.5, 0.1])
    sv = np.linalg.svd(W, compute_uv=False)
    for k in (1, 2, 4):
        Uk, kept = O.pinv_cut(W, k)
        assert kept == k
        got = np.linalg.norm(W - W @ Uk @ W)
        want = math.sqrt(float(np.sum(sv[k:] ** 2)))
        assert abs(got - want) <= 1e-10 * sv[0], (k, got, want)
    U, kept = O.pinv_cut(W)
    U6, _ = O.pinv_cut(W, 6)
    assert kept == 6 and np.allclose(U, U6, atol=1e-12)
    A = gen.gaussian_product(40, 48, 8, 23)
    off = gen.contiguous_blocks(48, 6)
    res = O.alg1(A, off, 12, 3, gen.rademacher(48, 12, 23), gen.draws_u64(15, 23), rank_k=3)
    assert res["rank_w"] == 3
    assert np.linalg.matrix_rank(res["C"] @ res["U"] @ res["R"]) == 3


def check_alg1_all_rows_is_column_fit(O):
    """With every row sampled (r = m) R is A with its rows permuted, so
    C W^+ R = A S (A S)^+ A = C C^+ A whenever C has full column rank: the
    error is the column-selection error of the least-squares fit, and the
    scaling of S drops out (Sec. 2.1, the Remark of Sec. 3.3)."""
    rng = np.random.default_rng(24)
    A = rng.standard_normal((24, 60)) @ np.diag(0.95 ** np.arange(60))
    off = gen.contiguous_blocks(60, 5)
    res = O.alg1(A, off, 24, 3, None, gen.draws_u64(27, 24), kr=6, mode="exact")
    Cun = O.gather_columns(A, off, res["idx"])
    _, want = O.fit_columns(A, Cun)
    assert abs(res["err"] - want) <= 1e-9 * want, (res["err"], want)
    # unscaled C and R through the library pseudoinverse give the same error
    Run = A[res["rows"], :]
    Wun = Run[:, O.selected_columns(off, res["idx"])]
    _, e2 = O.fit_intersection(A, Cun, Run, Wun)
    assert abs(e2 - want) <= 1e-9 * want


def check_alg1_exact_low_rank(O):
    """When the sampled rows and columns capture the rank of A, C W^+ R
    reconstructs A exactly (the intersection carries its whole rank)."""
    A = gen.gaussian_product(50, 64, 6, 25)
    off = gen.contiguous_blocks(64, 8)
    for mode in ("exact", "twin"):
        res = O.alg1(A, off, 10, 2, gen.rademacher(64, 10, 25), gen.draws_u64(12, 25), kr=6, mode=mode)
        assert res["rank_w"] == 6
        assert res["err"] <= 1e-9 * math.sqrt(res["frob2"]), res["err"]


# --------------------------------------------------------------------------
# Boosting (Sec. 3.3)
# --------------------------------------------------------------------------

def check_boost_law(O):
    """Independent trials: P(min_i err_i > q) = P(err > q)^t for every level
    q.  Single runs (their own draws) give P(err > q) at q = their median;
    boosted runs with t = 3 must match its cube within five standard errors
    (reusing one draw set for every trial would give P(err > q) itself,
    keeping the largest error 1 - (1 - P)^3)."""
    w = gen.tiny(0)
    base = O.decompose(w.A, w.offsets, w.k, w.s, w.omega, w.draws, q=w.q, with_fit=False)
    sc = base["scores"]
    cache = {}
    A64 = w.A.astype(np.float64)
    fro2 = float(np.sum(A64 * A64))

    def err_of(idx):
        # ||A - C C^+ A||_F^2 = ||A||_F^2 - ||Q^T A||_F^2 for C = Q R (full column rank here)
        key = tuple(sorted(int(j) for j in idx))
        if key not in cache:
            cols = np.concatenate([np.arange(w.offsets[j], w.offsets[j + 1]) for j in key])
            Q = np.linalg.qr(A64[:, cols])[0]
            cache[key] = math.sqrt(max(fro2 - float(np.sum((Q.T @ A64) ** 2)), 0.0))
        return cache[key]

    n1, t, nb = 600, 3, 600
    d1 = gen.draws_u64(n1 * w.s, 101)
    singles = np.array([err_of(O.sample_blocks(sc, d1[i * w.s:(i + 1) * w.s], w.s)["idx"]) for i in range(n1)])
    q = float(np.median(singles))
    p1 = float(np.mean(singles > q))
    db = gen.draws_u64(nb * t * w.s, 202)
    # the boosted runs call the oracle's own boost with precomputed scores
    mins = []
    for i in range(nb):
        dr = db[i * t * w.s:(i + 1) * t * w.s]
        errs = [err_of(O.sample_blocks(sc, O.trial_draws(dr, j, w.s), w.s)["idx"]) for j in range(t)]
        mins.append(errs[O.boost_pick(errs)])
    pt = float(np.mean(np.array(mins) > q))
    sd = math.sqrt(pt * (1 - pt) / nb + (3 * p1 * p1) ** 2 * p1 * (1 - p1) / n1) + 1e-3
    assert abs(pt - p1 ** t) <= 5 * sd, (pt, p1, p1 ** t, sd)


def check_boost_keeps_first_minimum(O):
    """The kept trial is the first one of smallest error, and the whole
    boosted result is that trial's single decomposition."""
    assert O.boost_pick([3.0, 1.0, 2.0, 1.0]) == 1
    assert O.boost_pick([0.5]) == 0
    w = gen.tiny(1)
    t = 4
    dr = gen.draws_u64(t * w.s, 303)
    res = O.boost(w.A, w.offsets, w.k, w.s, w.omega, dr, t, q=w.q)
    single = [O.decompose(w.A, w.offsets, w.k, w.s, w.omega, dr[i * w.s:(i + 1) * w.s], q=w.q)["err"]
              for i in range(t)]
    assert np.allclose(res["errs"], single, rtol=1e-12)
    assert res["err"] == min(res["errs"]) and res["best"] == int(np.argmin(single))


# --------------------------------------------------------------------------
# Diagnostics (Defs. 3 and 4)
# --------------------------------------------------------------------------

def check_block_stable_rank_closed_forms(O):
    """Stable rank ||X||_F^2 / ||X||_2^2 of each block slice of V: 1 for a
    rank-1 slice (one-column blocks, or a block whose rows are multiples of one
    vector), exactly the rank for a slice with equal nonzero singular values,
    and 1 <= ratio <= rank(slice) <= min(b_g, k) in general (Def. 3 and the
    bounds stated with it)."""
    rng = np.random.default_rng(61)
    n, k = 48, 6
    V = np.linalg.qr(rng.standard_normal((n, k)))[0]
    # one-column blocks: every ratio is 1
    alpha, ratios = O.block_stable_rank(V, np.arange(n + 1))
    assert np.allclose(ratios, 1.0, rtol=1e-12) and abs(alpha - 1.0) <= 1e-12
    # planted slices: rows 0..3 multiples of one vector (rank 1); rows 4..9
    # = 3 orthogonal rows of equal norm, each repeated twice (singular values equal)
    W = rng.standard_normal((n, k))
    u = rng.standard_normal(k)
    W[0:4] = np.outer([1.0, -2.0, 0.5, 3.0], u)
    Q = np.linalg.qr(rng.standard_normal((k, 3)))[0].T   # 3 orthonormal rows
    W[4:10] = np.repeat(Q, 2, axis=0)
    off = [0, 4, 10, 17, 30, n]
    alpha, ratios = O.block_stable_rank(W, off)
    assert abs(ratios[0] - 1.0) <= 1e-12
    assert abs(ratios[1] - 3.0) <= 1e-12
    for g in range(len(off) - 1):
        blk = W[off[g]:off[g + 1]]
        rk = np.linalg.matrix_rank(blk)
        assert 1.0 - 1e-12 <= ratios[g] <= rk + 1e-12 <= min(off[g + 1] - off[g], k) + 1e-12
    assert alpha == np.nanmin(ratios)
    # a zero slice has no ratio
    W[30:n] = 0.0
    _, ratios = O.block_stable_rank(W, off)
    assert np.isnan(ratios[-1])


def check_incoherence_extremes(O):
    """mu = (m/k) max_i ||U_k^T e_i||^2 lies in [1, m/k] (Def. 4): 1 when every
    row of the orthonormal U_k has the same norm (columns of a normalized
    Hadamard matrix), m/k when a column of U_k is a coordinate vector."""
    m, k = 64, 8
    H = np.array([[1.0]])
    while H.shape[0] < m:
        H = np.block([[H, H], [H, -H]])
    U = H[:, :k] / math.sqrt(m)
    assert abs(O.incoherence(U) - 1.0) <= 1e-12
    rng = np.random.default_rng(62)
    Q = np.linalg.qr(rng.standard_normal((m - 1, k - 1)))[0]
    U = np.zeros((m, k))
    U[0, 0] = 1.0
    U[1:, 1:] = Q
    assert abs(O.incoherence(U) - m / k) <= 1e-12
    U = np.linalg.qr(rng.standard_normal((m, k)))[0]
    assert 1.0 - 1e-12 <= O.incoherence(U) <= m / k + 1e-12


# --------------------------------------------------------------------------
# Blocks of arbitrary column sets
# --------------------------------------------------------------------------

def check_mapped_blocks_follow_def2(O):
    """With blocks of scattered columns, each score is Def. 2 with E_g picking
    that block's columns: the sum of the per-column leverages (Def. 1) of the
    exact V_k over the block's set; choosing every block leaves no error; the
    identity map reproduces the contiguous case."""
    w = gen.tiny(4)
    n = w.n
    rng = np.random.default_rng(71)
    cmap = rng.permutation(n)
    res = O.decompose_mapped(w.A, w.offsets, w.k, w.s, None, w.draws, col_map=cmap, mode="exact")
    lev = O.column_leverage(O.exact_right_subspace(w.A.astype(np.float64), w.k))
    want = np.array([lev[cmap[w.offsets[g]:w.offsets[g + 1]]].sum() for g in range(w.G)])
    assert np.allclose(res["scores"], want, rtol=1e-9, atol=1e-12)
    cols = res["cols"]
    sets = [set(cmap[w.offsets[j]:w.offsets[j + 1]].tolist()) for j in res["idx"]]
    assert set(cols.tolist()) == set().union(*sets) and len(cols) == sum(len(x) for x in sets)
    # the returned U reproduces A's columns in A's order
    C = w.A.astype(np.float64)[:, cols]
    E = w.A.astype(np.float64) - C @ res["U"]
    assert abs(math.sqrt(float(np.sum(E * E))) - res["err"]) <= 1e-9 * max(res["err"], 1.0)
    allb = O.decompose_mapped(w.A, w.offsets, w.k, w.G, None, gen.draws_u64(w.G, 72), col_map=cmap, mode="exact")
    assert allb["err"] <= 1e-9 * math.sqrt(allb["frob2"])
    ident = O.decompose_mapped(w.A, w.offsets, w.k, w.s, w.omega, w.draws, col_map=np.arange(n), q=w.q)
    plain = O.decompose(w.A, w.offsets, w.k, w.s, w.omega, w.draws, q=w.q)
    assert np.array_equal(ident["idx"], plain["idx"]) and abs(ident["err"] - plain["err"]) <= 1e-12 * plain["err"]


def check_alg1_boost_keeps_first_minimum(O):
    """Boosted Algorithm 1: every trial is the single run with its own r + s
    draws, and the kept one is the first of smallest error."""
    A = gen.lowrank_haar(200, 96, 1.0 / np.arange(1, 13), 1e-2, 81)
    off = gen.contiguous_blocks(96, 8)
    r, s, t = 24, 3, 4
    dr = gen.draws_u64(t * (r + s), 81)
    res = O.alg1_boost(A, off, r, s, dr, t, kr=8)
    single = [O.alg1(A, off, r, s, None, dr[i * (r + s):(i + 1) * (r + s)], kr=8)["err"] for i in range(t)]
    assert np.allclose(res["errs"], single, rtol=1e-12)
    assert res["best"] == int(np.argmin(single)) and res["err"] == min(single)


ALL_CHECKS = [
    check_block_stable_rank_closed_forms,
    check_incoherence_extremes,
    check_frob_closed_form,
    check_scores_sum_to_k,
    check_scores_from_projector,
    check_scores_bounds_permutation,
    check_row_scores_transpose,
    check_twin_exact_on_low_rank,
    check_twin_left_vectors_on_low_rank,
    check_score_condition_first_order,
    check_cond2_planted,
    check_omega_philox_library,
    check_twin_converges,
    check_sampler_inverse_cdf,
    check_sampler_edges,
    check_sampler_quantization_exact,
    check_sampler_without_replacement_law,
    check_sampler_frequencies,
    check_unbiased_scaling,
    check_block_product_variance,
    check_sampling_matrix_example,
    check_fit_projection,
    check_fit_qr_route,
    check_fit_selected_columns,
    check_cur_reductions,
    check_paper_synthetic_generator,
    check_alg1_rows_uniform_distinct,
    check_alg1_penrose,
    check_alg1_rank_k,
    check_alg1_all_rows_is_column_fit,
    check_alg1_exact_low_rank,
    check_mapped_blocks_follow_def2,
    check_boost_law,
    check_boost_keeps_first_minimum,
    check_alg1_boost_keeps_first_minimum,
]
