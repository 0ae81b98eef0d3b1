"""Planted mistakes in the oracle (on the CPU) must trip at least one pin.

Each mutant copies the oracle module's functions and replaces one of them
with a plausible bug: a dropped square, a shifted block edge, a wrong sort
order, a >= for a >, a missing factor, a transposed operand.  The test
passes only if some pin raises for it."""
import math
import types

import numpy as np
import pytest

from oracle import bcur_oracle as O

from . import oracle_pins as P


def _clone(**over):
    ns = types.SimpleNamespace(**{k: getattr(O, k) for k in dir(O) if not k.startswith("__")})
    for k, v in over.items():
        setattr(ns, k, v)
    # decompose calls module globals; rebind it to the clone's functions
    return ns


def _scores_norm_not_squared(V, offsets):
    V = np.asarray(V, dtype=np.float64)
    return np.array([np.sqrt(np.sum(V[offsets[g]:offsets[g + 1]] ** 2)) for g in range(len(offsets) - 1)])


def _scores_edge_shift(V, offsets):
    V = np.asarray(V, dtype=np.float64)
    return np.array([np.sum(V[offsets[g]:offsets[g + 1] - 1] ** 2) for g in range(len(offsets) - 1)])


def _frob_drops_row(A):
    A = np.asarray(A, dtype=np.float64)
    return float(np.sum(A[:-1] ** 2))


def _range_finder_ascending(A, omega, q, k):
    out = O.range_finder(A, omega, q, k)
    W = out["W"][:, ::-1]
    out = dict(out)
    out["Vk"] = out["Q"] @ W[:, :k]
    out["ritz"] = out["ritz"][::-1]
    return out


def _range_finder_no_transpose(A, omega, q, k):
    # forgets A^T: iterates Q <- orth(A Q) on the row side (only valid when m == n)
    A = np.asarray(A, dtype=np.float64)
    Q = np.asarray(omega, dtype=np.float64)
    for _ in range(q + 1):
        Q, _ = np.linalg.qr(A[: Q.shape[0], : Q.shape[0]] @ Q)
    T = Q.T @ (A.T @ A) @ Q
    lam, W = np.linalg.eigh(T)
    o = np.argsort(lam)[::-1]
    return {"Q": Q, "Vk": Q @ W[:, o[:k]], "Uk": None, "lam": lam[o], "ritz": np.sqrt(np.abs(lam[o])), "W": W[:, o]}


def _sample_ge(scores, draws, s, replace=False):
    q, sh = O.quantize_scores(scores)
    idx = []
    taken = set()
    for t in range(s):
        W = sum(q[g] for g in range(len(q)) if replace or g not in taken)
        x = O.draw_point(int(draws[t]), W)
        acc = 0
        for g in range(len(q)):
            if not replace and g in taken:
                continue
            acc += q[g]
            if acc >= x:
                break
        idx.append(g)
        taken.add(g)
    total = sum(q)
    w = [math.sqrt(total / (s * q[j])) if q[j] else math.inf for j in idx]
    return {"idx": np.array(idx), "weights": np.array(w), "margins": np.zeros(s), "q": q, "shift": sh}


def _sample_weight_without_s(scores, draws, s, replace=False):
    out = dict(O.sample_blocks(scores, draws, s, replace))
    out["weights"] = out["weights"] * math.sqrt(s)
    return out


def _fit_transpose(A, C):
    A = np.asarray(A, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    U = C.T @ A / max(1.0, float(np.sum(C * C)) / C.shape[1])
    E = A - C @ U
    return U, float(np.sqrt(np.sum(E * E)))


def _gather_wrong_block(A, offsets, idx, dedupe=True):
    return O.gather_columns(A, offsets, [min(int(j) + 1, len(offsets) - 2) for j in idx], dedupe)


def _pinv_smallest(Wmat, rank_k=0):
    # the literal best rank-k approximation of W^+: keeps the smallest singular values of W
    W = np.asarray(Wmat, dtype=np.float64)
    Uw, sw, Vtw = np.linalg.svd(W, full_matrices=False)
    keep = int(np.sum(sw > max(W.shape) * 2.0 ** -24 * sw[0]))
    inv = np.zeros_like(sw)
    lo = keep - rank_k if 0 < rank_k < keep else 0
    inv[lo:keep] = 1.0 / sw[lo:keep]
    return (Vtw.T * inv) @ Uw.T, keep - lo


def _pinv_transpose(Wmat, rank_k=0):
    W = np.asarray(Wmat, dtype=np.float64)
    return W.T / max(1.0, float(np.sum(W * W))), min(W.shape)


def _rows_with_replacement(m, r, draws):
    return O.sample_blocks(np.ones(m), draws, r, replace=True)["idx"]


def _pick_largest(errs):
    return int(np.argmax(errs))


def _stable_rank_spectral_unsquared(V, offsets):
    V = np.asarray(V, dtype=np.float64)
    off = np.asarray(offsets, dtype=np.int64)
    ratios = np.full(len(off) - 1, np.nan)
    for g in range(len(off) - 1):
        blk = V[off[g]:off[g + 1], :]
        fro2 = float(np.sum(blk * blk))
        if fro2 > 0.0:
            ratios[g] = fro2 / float(np.linalg.norm(blk, 2))
    return float(np.nanmin(ratios)), ratios


def _incoherence_without_m_over_k(U):
    U = np.asarray(U, dtype=np.float64)
    return float(np.max(np.sum(U * U, axis=1)))


def _uk_divides_by_lam(A, omega, q, k):
    out = dict(O.range_finder(A, omega, q, k))
    out["Uk"] = (np.asarray(A, dtype=np.float64) @ out["Q"] @ out["W"][:, :k]) / out["lam"][:k]
    return out


def _uk_from_q(A, omega, q, k):
    out = dict(O.range_finder(A, omega, q, k))
    out["Uk"] = (out["Q"] @ out["W"][:, :k]) / out["ritz"][:k]
    return out


def _kappa_gap_shifted(lam, k):
    if k + 1 >= len(lam):
        return 1.0
    gap = lam[k] - lam[k + 1]
    return float(lam[0] / gap) if gap > 0 else math.inf


def _kappa_without_lam1(lam, k):
    if k >= len(lam):
        return 1.0
    gap = lam[k - 1] - lam[k]
    return float(1.0 / gap) if gap > 0 else math.inf


def _cond_without_ratio(C):
    return float(np.linalg.svd(np.asarray(C, dtype=np.float64), compute_uv=False)[0])


def _philox_weyl_swapped(counter, key):
    c = [int(x) & O._MASK64 for x in counter]
    k0, k1 = int(key[0]), int(key[1])
    for _ in range(10):
        p0 = O._PHILOX_M[0] * c[0]
        p1 = O._PHILOX_M[1] * c[2]
        c = [((p1 >> 64) ^ c[1] ^ k0) & O._MASK64, p1 & O._MASK64,
             ((p0 >> 64) ^ c[3] ^ k1) & O._MASK64, p0 & O._MASK64]
        k0 = (k0 + O._PHILOX_W[1]) & O._MASK64
        k1 = (k1 + O._PHILOX_W[0]) & O._MASK64
    return c


def _omega_msb_first(n, l, seed):
    out = np.empty((n, l))
    for i in range(n):
        words = O.philox4x64_10((i, 0, 0, 0), (seed, 0))
        for j in range(l):
            out[i, j] = -1.0 if (words[j >> 6] >> (63 - (j & 63))) & 1 else 1.0
    return out


def _omega_counter_from_one(n, l, seed):
    out = np.empty((n, l))
    for i in range(n):
        words = O.philox4x64_10((i + 1, 0, 0, 0), (seed, 0))
        for j in range(l):
            out[i, j] = -1.0 if (words[j >> 6] >> (j & 63)) & 1 else 1.0
    return out


def _fit_qr_drops_last_panel(A, C, cols=None, panel=1024):
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[1]
    last = ((n - 1) // panel) * panel
    return O.fit_columns_qr(A[:, :last] if last > 0 else A, C, cols=cols, panel=panel)[0], \
        O.fit_columns_qr(A, C, cols=cols, panel=panel)[1]


def _fit_qr_without_rinv(A, C, cols=None, panel=1024):
    err, _ = O.fit_columns_qr(A, C, panel=panel)
    if cols is None:
        return err, None
    Q, R = np.linalg.qr(np.asarray(C, dtype=np.float64))
    return err, Q.T @ np.asarray(A, dtype=np.float64)[:, cols]


MUTANTS = {
    "uk-divides-by-lam": dict(range_finder=_uk_divides_by_lam),
    "fit-qr-drops-last-panel": dict(fit_columns_qr=_fit_qr_drops_last_panel),
    "fit-qr-without-rinv": dict(fit_columns_qr=_fit_qr_without_rinv),
    "uk-from-q": dict(range_finder=_uk_from_q),
    "kappa-gap-off-by-one": dict(score_condition=_kappa_gap_shifted),
    "kappa-without-lam1": dict(score_condition=_kappa_without_lam1),
    "cond-without-ratio": dict(cond2=_cond_without_ratio),
    "philox-weyl-swapped": dict(philox4x64_10=_philox_weyl_swapped),
    "omega-msb-first": dict(rademacher_omega=_omega_msb_first),
    "omega-counter-from-one": dict(rademacher_omega=_omega_counter_from_one),
    "stable-rank-spectral-unsquared": dict(block_stable_rank=_stable_rank_spectral_unsquared),
    "incoherence-without-m-over-k": dict(incoherence=_incoherence_without_m_over_k),
    "boost-reuses-draws": dict(trial_draws=lambda draws, i, s: draws[:s]),
    "boost-keeps-largest": dict(boost_pick=_pick_largest),
    "pinv-keeps-smallest": dict(pinv_cut=_pinv_smallest),
    "pinv-transpose": dict(pinv_cut=_pinv_transpose),
    "rows-with-replacement": dict(alg1_rows=_rows_with_replacement),
    "scores-not-squared": dict(block_scores=_scores_norm_not_squared),
    "scores-edge-shift": dict(block_scores=_scores_edge_shift),
    "frob-drops-row": dict(frob2=_frob_drops_row),
    "ritz-ascending": dict(range_finder=_range_finder_ascending),
    "range-finder-no-transpose": dict(range_finder=_range_finder_no_transpose),
    "sampler-ge": dict(sample_blocks=_sample_ge),
    "weights-without-s": dict(sample_blocks=_sample_weight_without_s),
    "fit-transpose": dict(fit_columns=_fit_transpose),
}


def _pins_for(ns):
    """The first pin that fails on the clone (the pins run cheapest first)."""
    fails = []
    for chk in P.ALL_CHECKS:
        try:
            chk(ns)
        except Exception as e:  # AssertionError, shape errors, ...
            fails.append((chk.__name__, type(e).__name__))
            break
    return fails


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    ns = _clone(**MUTANTS[name])
    # decompose inside the clone must use the mutated pieces
    def decompose(A, offsets, k, s, omega, draws, q=2, replace=False, mode="twin", row_offsets=None,
                  s_r=0, with_fit=True):
        A64 = np.asarray(A, dtype=np.float64)
        rf = ns.range_finder(A64, omega, q, k)
        sc = ns.block_scores(rf["Vk"], offsets)
        smp = ns.sample_blocks(sc, draws[:s], s, replace)
        C = ns.gather_columns(A64, offsets, smp["idx"])
        U, err = ns.fit_columns(A64, C)
        return {"idx": smp["idx"], "err": err, "frob2": ns.frob2(A64), "scores": sc}
    ns.decompose = decompose
    fails = _pins_for(ns)
    assert fails, f"mutant {name} passed every pin"


def test_gather_mutant_caught_by_bruteforce():
    ns = _clone(gather_columns=_gather_wrong_block)

    def decompose(A, offsets, k, s, omega, draws, q=2, **kw):
        A64 = np.asarray(A, dtype=np.float64)
        rf = ns.range_finder(A64, omega, q, k)
        smp = ns.sample_blocks(ns.block_scores(rf["Vk"], offsets), draws[:s], s)
        U, err = ns.fit_columns(A64, ns.gather_columns(A64, offsets, smp["idx"]))
        return {"idx": smp["idx"], "err": err}
    ns.decompose = decompose
    with pytest.raises(AssertionError):
        P.check_fit_bruteforce(ns, max_subsets=2000)
