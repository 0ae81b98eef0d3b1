"""Parity of the BF16 sketch passes and of the row-block CUR variant.

BF16: the oracle rounds A and Q to BF16 itself (round to nearest even on the
bit pattern, written here, independent of the HIP code) and forms
A_bf^T bf16(A_bf Q_bf) in FP64; the GPU differs only by FP32 accumulation
order (and, rarely, by a one-ulp BF16 flip of an intermediate), so the
normwise relative gap is bounded by 1e-3.  The whole BF16 range finder ends
with an FP32 power pass and an FP32 Rayleigh-Ritz step; its scores are
compared with the FP64 twin at the BF16 gate of tests/gates.py (the scores'
response to a BF16-sized perturbation in the first q iterations and an
FP32-sized one after).

Row variant: U = C^+ A R^+ and ||A - C U R||_F against the oracle (pinv),
residual within 1e-5 relative (plus the 16 u32 ||A|| floor) and U within the
gate of tests/gates.py (from cond(C) and cond(R)) given identical column and
row blocks; a different selection (allowed only where the margins are within
the score gate) is checked against the oracle's fit of the GPU's own blocks.
"""
import math

import numpy as np
import pytest
import torch

from oracle import bcur_oracle as O
from workloads import gen

from .gates import index_margin_needed, score_gate, u_gate_rows

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def ctx():
    from paper_1703_06065_amd import Context
    return Context(0)


def dev(a):
    from paper_1703_06065_amd.binding import to_device
    return to_device(a)


def dense(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def note(*a):
    print(*a, flush=True)


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), as float64."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# the last three take the split-BF16 sketch tiles (m l n >= 1e9): 128 x 64
# on whole tiles, then 128 x 64 and 128 x 128 on ragged ones
@pytest.mark.parametrize("m,n,l", [(300, 200, 20), (517, 1030, 60), (2048, 1024, 110), (8192, 4096, 60),
                                   (8200, 4100, 60), (8200, 4100, 100)])
def test_sketch_pass_fp32(ctx, m, n, l):
    from paper_1703_06065_amd.binding import PREC_FP32
    note(f"sketch fp32 m={m} n={n} l={l}")
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n)).astype(np.float32)
    Q = rng.standard_normal((n, l)).astype(np.float32)
    Y = ctx.sketch_pass(dev(A), dev(Q), PREC_FP32).cpu().numpy().astype(np.float64)
    A64, Q64 = A.astype(np.float64), Q.astype(np.float64)
    ref = A64.T @ (A64 @ Q64)
    absb = np.abs(A64).T @ (np.abs(A64) @ np.abs(Q64))
    rel = np.linalg.norm(Y - ref) / np.linalg.norm(absb)
    note(f"  normwise rel gap {rel:.2e}")
    assert rel < 1e-5


@pytest.mark.parametrize("m,n,l", [(300, 200, 20), (517, 1030, 60), (2048, 1024, 110)])
def test_sketch_pass_bf16(ctx, m, n, l):
    from paper_1703_06065_amd.binding import PREC_BF16
    note(f"sketch bf16 m={m} n={n} l={l}")
    rng = np.random.default_rng(m * n)
    A = rng.standard_normal((m, n)).astype(np.float32)
    Q = rng.standard_normal((n, l)).astype(np.float32)
    Y = ctx.sketch_pass(dev(A), dev(Q), PREC_BF16).cpu().numpy().astype(np.float64)
    Ab, Qb = bf16_round(A), bf16_round(Q)
    Z = Ab @ Qb
    ref = Ab.T @ bf16_round(Z.astype(np.float32))
    absb = np.abs(Ab).T @ (np.abs(Ab) @ np.abs(Qb))
    rel = np.linalg.norm(Y - ref) / np.linalg.norm(absb)
    exact = A.astype(np.float64).T @ (A.astype(np.float64) @ Q.astype(np.float64))
    rel_exact = np.linalg.norm(Y - exact) / np.linalg.norm(absb)
    note(f"  normwise gap to the BF16-rounded FP64 product {rel:.2e}, to the unrounded one {rel_exact:.2e}")
    assert rel < 1e-3
    assert rel_exact < 2e-2


@pytest.mark.parametrize("m,n,b,k,s,seed", [(600, 400, 10, 10, 5, 21), (1000, 2000, 50, 20, 6, 22)])
def test_decompose_bf16(ctx, m, n, b, k, s, seed):
    from paper_1703_06065_amd.binding import PREC_BF16
    w = gen.small_case(m, n, b, k, s, seed=seed, decay="geometric", noise=1e-3)
    note(f"decompose bf16 m={m} n={n} k={k} l={w.l}")
    res = ctx.decompose(dev(w.A), w.offsets, w.k, w.s, dense(w.omega), w.draws, q=w.q, precision=PREC_BF16)
    ref = O.decompose(w.A, w.offsets, w.k, w.s, w.omega, w.draws, q=w.q)
    gt = score_gate(w.A, w.offsets, w.k, w.q, w.omega, ref["scores"], precision="bf16")
    tol = gt["tol"]
    dl = np.abs(res["scores"] - ref["scores"])
    note(f"  kappa={ref['kappa']:.3g} d={gt['d']:.2e} tau={gt['tau']:.2e} max|dl|/tol={np.max(dl / tol):.3f} "
         f"max|dl|/(k/G)={dl.max() / (w.k / w.G):.2e} idx={list(res['idx'])} oracle={list(ref['idx'])}")
    assert np.all(dl <= tol)
    need = index_margin_needed(tol)
    if ref["margins"].min() > need:
        assert np.array_equal(res["idx"], ref["idx"])
    if np.array_equal(res["idx"], ref["idx"]):
        assert abs(res["err"] - ref["err"]) <= 1e-5 * ref["err"] + 16 * U32 * math.sqrt(ref["frob2"])
    else:
        # a different but valid selection: its residual is the oracle's fit of the GPU's own blocks
        idx = res["idx"]
        assert len(set(idx.tolist())) == len(idx) and idx.min() >= 0 and idx.max() < w.G
        _, e2 = O.fit_columns(w.A, O.gather_columns(w.A, w.offsets, idx))
        assert abs(res["err"] - e2) <= 1e-5 * e2 + 16 * U32 * math.sqrt(ref["frob2"])


def _check_rows(ctx, w, label, precision="fp32"):
    from paper_1703_06065_amd.binding import PREC_BF16, PREC_FP32
    note(f"rows {label} m={w.m} n={w.n} G={w.G} Gr={len(w.row_offsets) - 1} k={w.k} s={w.s} s_r={w.s_r} "
         f"precision={precision}")
    res = ctx.decompose(dev(w.A), w.offsets, w.k, w.s, dense(w.omega), w.draws, q=w.q,
                        row_offsets=w.row_offsets, s_r=w.s_r, refine=1,
                        precision=PREC_BF16 if precision == "bf16" else PREC_FP32)
    ref = O.decompose(w.A, w.offsets, w.k, w.s, w.omega, w.draws, q=w.q, row_offsets=w.row_offsets, s_r=w.s_r)
    gt = score_gate(w.A, w.offsets, w.k, w.q, w.omega, ref["scores"], precision=precision,
                    row_offsets=w.row_offsets, row_scores_ref=ref["row_scores"])
    dl = np.abs(res["scores"] - ref["scores"])
    dr = np.abs(res["row_scores"] - ref["row_scores"])
    Gr = len(w.row_offsets) - 1
    note(f"  kappa={ref['kappa']:.3g} tau={gt['tau']:.2e} tau_r={gt['tau_r']:.2e} "
         f"max|dl|/(k/G)={dl.max() / (w.k / w.G):.2e} max|dr|/(k/Gr)={dr.max() / (w.k / Gr):.2e}")
    assert np.all(dl <= gt["tol"])
    assert np.all(dr <= gt["tol_r"])
    note(f"  idx={list(res['idx'])} oracle={list(ref['idx'])} idx_r={list(res['idx_r'])} "
         f"oracle={list(ref['idx_r'])}")
    if ref["margins"].min() > index_margin_needed(gt["tol"]):
        assert np.array_equal(res["idx"], ref["idx"])
    if ref["margins_r"].min() > index_margin_needed(gt["tol_r"]):
        assert np.array_equal(res["idx_r"], ref["idx_r"])
    if np.array_equal(res["idx"], ref["idx"]) and np.array_equal(res["idx_r"], ref["idx_r"]):
        gap = abs(res["err"] - ref["err"])
        note(f"  err={res['err']:.9g} oracle={ref['err']:.9g} rel={gap / ref['err']:.2e} flags={res['flags']}")
        assert gap <= 1e-5 * ref["err"] + 16 * U32 * math.sqrt(ref["frob2"])
        assert res["c"] == len(ref["cols"]) and res["r"] == len(ref["rows"])
        U = res["U"].cpu().numpy().astype(np.float64)
        C = O.gather_columns(w.A, w.offsets, ref["idx"])
        R = O.gather_rows(w.A, w.row_offsets, ref["idx_r"])
        cond_c, cond_r = O.cond2(C), O.cond2(R)
        rel_u = np.linalg.norm(U - ref["U"]) / np.linalg.norm(ref["U"])
        gate = u_gate_rows(cond_c, cond_r)
        note(f"  rel U gap {rel_u:.2e} gate {gate:.2e} cond(C)={cond_c:.3g} cond(R)={cond_r:.3g}")
        assert rel_u <= gate
    else:
        # a different but valid selection: the oracle's fit of the GPU's own blocks
        assert len(set(res["idx"].tolist())) == w.s and len(set(res["idx_r"].tolist())) == w.s_r
        C = O.gather_columns(w.A, w.offsets, res["idx"])
        R = O.gather_rows(w.A, w.row_offsets, res["idx_r"])
        _, e2 = O.fit_cur(w.A, C, R)
        note(f"  different selection: err={res['err']:.9g} oracle fit of the same blocks={e2:.9g}")
        assert abs(res["err"] - e2) <= 1e-5 * e2 + 16 * U32 * math.sqrt(ref["frob2"])
    return res, ref


def test_rows_small(ctx):
    w = gen.small_case(400, 300, 10, 8, 4, seed=31)
    w.row_offsets = gen.contiguous_blocks(400, 20)
    w.s_r = 5
    w.draws = gen.draws_u64(w.s + w.s_r, 31)
    _check_rows(ctx, w, "small")


def test_rows_biometric(ctx):
    w = gen.biometric_cfg(0)
    _check_rows(ctx, w, "biometric")


def test_rows_biometric_bf16(ctx):
    # the biometric-shaped workload at its stated precision: BF16 range finder
    # (the first q power iterations), final FP32 pass, the row variant's fit
    w = gen.biometric_cfg(0)
    _check_rows(ctx, w, "biometric", precision="bf16")
