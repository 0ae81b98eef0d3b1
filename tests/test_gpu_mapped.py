"""Blocks of arbitrary column (row) sets on the GPU: block g is the set
col_map[off[g] .. off[g+1]-1] (Def. 2 with a scattered E_g).  Parity with the
FP64 oracle's decompose_mapped under the tolerances of tests/test_gpu_parity.py
(scores within the derived gate of tests/gates.py, blocks identical when the margin allows, err 1e-5
relative plus 16 u32 ||A||_F); the identity map reproduces the contiguous
path bit for bit, and the server returns the same result as the direct call.
"""
import math

import numpy as np
import pytest
import torch

from oracle import bcur_oracle as O
from workloads import gen

from .gates import index_margin_needed, score_gate

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def ctx():
    from paper_1703_06065_amd import Context
    return Context(0)


def dev(a):
    from paper_1703_06065_amd.binding import to_device
    return to_device(a)


def dev_dense(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def note(*a):
    print(*a, flush=True)


def err_tol(err_ref, frob2):
    return 1e-5 * err_ref + 16 * U32 * math.sqrt(frob2)


def check_mapped(ctx, w, col_map=None, row_map=None, row_offsets=None, s_r=0, label=""):
    note(f"mapped {label} {w.name} G={w.G} k={w.k} s={w.s} col_map={col_map is not None} "
         f"row_map={row_map is not None} s_r={s_r}")
    draws = w.draws if s_r == 0 else gen.draws_u64(w.s + s_r, 99)
    res = ctx.decompose(dev(w.A), w.offsets, w.k, w.s, dev_dense(w.omega), draws, q=w.q, col_map=col_map,
                        row_map=row_map, row_offsets=row_offsets, s_r=s_r)
    ref = O.decompose_mapped(w.A, w.offsets, w.k, w.s, w.omega, draws, col_map=col_map, row_map=row_map, q=w.q,
                             row_offsets=row_offsets, s_r=s_r)
    # the gate of the contiguous problem on A with its rows and columns in map order
    cm = np.arange(w.n) if col_map is None else np.asarray(col_map)
    rm = np.arange(w.m) if row_map is None else np.asarray(row_map)
    gt = score_gate(w.A[np.ix_(rm, cm)], w.offsets, w.k, w.q, w.omega[cm], ref["scores"])
    tol = gt["tol"]
    assert np.all(np.abs(res["scores"] - ref["scores"]) <= tol)
    need = index_margin_needed(tol)
    note(f"  idx gpu={list(res['idx'])} oracle={list(ref['idx'])} margin={ref['margins'].min():.2e} need {need:.2e}")
    if ref["margins"].min() > need:
        assert np.array_equal(res["idx"], ref["idx"])
    if s_r:
        if "margins_r" in ref and ref["margins_r"].min() > need:
            assert np.array_equal(res["idx_r"], ref["idx_r"])
    if np.array_equal(res["idx"], ref["idx"]) and (not s_r or np.array_equal(res["idx_r"], ref["idx_r"])):
        note(f"  err={res['err']:.9g} oracle={ref['err']:.9g}")
        assert abs(res["err"] - ref["err"]) <= err_tol(ref["err"], ref["frob2"])
        assert res["c"] == len(ref["cols"])
    if not s_r:
        # the returned U is for C = A[:, cols] with the map applied: its own residual is err
        cols = np.concatenate([np.asarray(col_map if col_map is not None else np.arange(w.n))[
            w.offsets[j]:w.offsets[j + 1]] for j in dict.fromkeys(res["idx"].tolist())])
        C = w.A.astype(np.float64)[:, cols]
        E = w.A.astype(np.float64) - C @ res["U"][: res["c"]].cpu().numpy().astype(np.float64)
        assert abs(math.sqrt(float(np.sum(E * E))) - res["err"]) <= err_tol(res["err"], ref["frob2"])
    return res, ref


@pytest.mark.parametrize("seed", [0, 1])
def test_mapped_columns_tiny(ctx, seed):
    w = gen.tiny(seed)
    cmap = np.random.default_rng(100 + seed).permutation(w.n)
    check_mapped(ctx, w, col_map=cmap, label="tiny")


def test_mapped_columns_ragged(ctx):
    w = gen.small_case(257, 515, 16, 12, 5, seed=2, ragged=True)
    cmap = np.random.default_rng(102).permutation(w.n)
    check_mapped(ctx, w, col_map=cmap, label="ragged")


def test_mapped_rows_and_columns_row_variant(ctx):
    w = gen.small_case(400, 300, 10, 8, 4, seed=3)
    roff = gen.contiguous_blocks(400, 20)
    rng = np.random.default_rng(103)
    check_mapped(ctx, w, col_map=rng.permutation(w.n), row_map=rng.permutation(w.m), row_offsets=roff, s_r=5,
                 label="row variant")


def test_identity_map_is_the_contiguous_path(ctx):
    w = gen.tiny(5)
    a = ctx.decompose(dev(w.A), w.offsets, w.k, w.s, dev_dense(w.omega), w.draws, q=w.q, col_map=np.arange(w.n))
    b = ctx.decompose(dev(w.A), w.offsets, w.k, w.s, dev_dense(w.omega), w.draws, q=w.q)
    assert np.array_equal(a["idx"], b["idx"]) and a["err"] == b["err"]
    assert np.array_equal(a["scores"], b["scores"])
    assert torch.equal(a["U"], b["U"])


def test_boost_with_map_matches_permuted_matrix(ctx):
    # boosting with a column map equals boosting the column-permuted matrix
    w = gen.tiny(6)
    cmap = np.random.default_rng(106).permutation(w.n)
    dr = gen.draws_u64(3 * w.s, 106)
    a = ctx.decompose_boost(dev(w.A), w.offsets, w.k, w.s, dev_dense(w.omega), dr, 3, q=w.q, col_map=cmap)
    b = ctx.decompose_boost(dev(w.A[:, cmap]), w.offsets, w.k, w.s, dev_dense(w.omega[cmap]), dr, 3, q=w.q)
    note(f"boost errs mapped={a['errs']} permuted={b['errs']}")
    assert np.array_equal(a["idx"], b["idx"]) and a["best"] == b["best"]
    frob2 = float(np.sum(w.A.astype(np.float64) ** 2))
    assert np.all(np.abs(a["errs"] - b["errs"]) <= err_tol(np.max(b["errs"]), frob2))


def test_server_copies_the_map(ctx):
    from paper_1703_06065_amd.binding import Server
    w = gen.tiny(7)
    cmap = np.random.default_rng(107).permutation(w.n)
    direct = ctx.decompose(dev(w.A), w.offsets, w.k, w.s, dev_dense(w.omega), w.draws, q=w.q, col_map=cmap)
    srv = Server(0, hbm_budget=1 << 30, max_slots=2)
    try:
        A, om = dev(w.A), dev_dense(w.omega)
        tk = srv.submit(A, w.offsets, w.k, w.s, om, w.draws, q=w.q, col_map=cmap.copy())
        out = srv.wait(tk)
    finally:
        srv.close()
    assert np.array_equal(out["idx"], direct["idx"]) and out["err"] == direct["err"]


def test_invalid_maps_rejected(ctx):
    from paper_1703_06065_amd import binding
    w = gen.tiny(8)
    bad = np.arange(w.n)
    bad[3] = bad[4]
    for kw in (dict(col_map=bad), dict(col_map=np.arange(1, w.n + 1))):
        with pytest.raises(binding.BcurError) as e:
            ctx.decompose(dev(w.A), w.offsets, w.k, w.s, dev_dense(w.omega), w.draws, q=w.q, **kw)
        assert e.value.status == binding.E_ARG
