"""Parity of boosting (Sec. 3.3) on the GPU, through the C ABI, with the FP64
oracle: t samplings from one set of scores, each fitted, the trial of
smallest error kept.

Tolerances are those of the single decomposition (tests/test_gpu_parity.py):
scores within the derived gate of tests/gates.py; each trial's
blocks identical when its smallest margin exceeds 2 G max_g tol_g; each
trial's err within 1e-5 relative plus 16 u32 ||A||_F.  The kept trial must be
the oracle's whenever the oracle's best error is ahead of every other trial's
by more than two such tolerances; otherwise it must be within one tolerance of
the smallest error.  The returned U is checked through its own residual.
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


def check_boost(ctx, w, t, seed, replace=False, label=""):
    draws = gen.draws_u64(t * w.s, seed)
    note(f"boost {label} {w.name} m={w.m} n={w.n} G={w.G} k={w.k} s={w.s} t={t} replace={replace}")
    res = ctx.decompose_boost(dev(w.A), w.offsets, w.k, w.s, dev_dense(w.omega), draws, t, q=w.q, replace=replace)
    ref = O.boost(w.A, w.offsets, w.k, w.s, w.omega, draws, t, q=w.q, replace=replace)
    tol = score_gate(w.A, w.offsets, w.k, w.q, w.omega, ref["scores"])["tol"]
    assert np.all(np.abs(res["scores"] - ref["scores"]) <= tol)
    assert abs(res["frob2"] - ref["frob2"]) <= 1e-12 * ref["frob2"]
    need = index_margin_needed(tol)
    etol = err_tol(max(ref["errs"]), ref["frob2"])
    # every trial: the oracle's errors where the selections agree
    for i, tr in enumerate(ref["trials"]):
        ok = tr["margins"].min() > need
        note(f"  trial {i}: err gpu={res['errs'][i]:.9g} oracle={tr['err']:.9g} margin={tr['margins'].min():.2e}")
        if ok:
            assert abs(res["errs"][i] - tr["err"]) <= etol
    # the kept trial
    errs = np.asarray(ref["errs"])
    b = ref["best"]
    others = np.delete(errs, b)
    clear = others.size == 0 or np.min(others) - errs[b] > 2 * etol
    note(f"  best gpu={res['best']} oracle={b} clear={clear} err={res['err']:.9g}")
    if clear and all(tr["margins"].min() > need for tr in ref["trials"]):
        assert res["best"] == b
        assert np.array_equal(res["idx"], ref["idx"])
    assert res["err"] == res["errs"][res["best"]] == np.min(res["errs"])
    assert res["err"] <= errs.min() + etol
    # the returned U is the kept trial's: its own residual is the reported err
    C = O.gather_columns(w.A, w.offsets, res["idx"])
    U = res["U"][: res["c"]].cpu().numpy().astype(np.float64)
    E = w.A.astype(np.float64) - C @ U
    own = math.sqrt(float(np.sum(E * E)))
    assert abs(own - res["err"]) <= err_tol(res["err"], ref["frob2"])
    return res, ref


@pytest.mark.parametrize("t", [1, 3, 5])
def test_boost_tiny(ctx, t):
    check_boost(ctx, gen.tiny(0), t, seed=40 + t, label="tiny")


@pytest.mark.parametrize("m,n,b,k,s,ragged,seed,t", [
    (300, 200, 10, 8, 4, False, 1, 3),
    (257, 515, 16, 12, 5, True, 2, 2),
    (1000, 129, 3, 5, 7, False, 3, 4),
    (640, 384, 32, 30, 3, False, 5, 3),
])
def test_boost_shapes(ctx, m, n, b, k, s, ragged, seed, t):
    w = gen.small_case(m, n, b, k, s, seed=seed, ragged=ragged)
    check_boost(ctx, w, t, seed=seed, label="shape")


def test_boost_with_replacement(ctx):
    w = gen.small_case(400, 300, 10, 8, 12, seed=11, noise=1e-2)
    check_boost(ctx, w, 3, seed=11, replace=True, label="replace")


def test_boost_one_trial_is_decompose(ctx):
    w = gen.tiny(2)
    draws = gen.draws_u64(w.s, 77)
    a = ctx.decompose_boost(dev(w.A), w.offsets, w.k, w.s, dev_dense(w.omega), draws, 1, q=w.q)
    b = ctx.decompose(dev(w.A), w.offsets, w.k, w.s, dev_dense(w.omega), draws, q=w.q)
    assert np.array_equal(a["idx"], b["idx"]) and a["best"] == 0
    assert abs(a["err"] - b["err"]) <= err_tol(b["err"], b["frob2"])


def test_boost_errors(ctx):
    from paper_1703_06065_amd import binding
    w = gen.tiny(3)
    dA, dO = dev(w.A), dev_dense(w.omega)
    for t in (0, 65):
        with pytest.raises(binding.BcurError) as e:
            ctx.decompose_boost(dA, w.offsets, w.k, w.s, dO, gen.draws_u64(max(t, 1) * w.s, 1), t, q=w.q)
        assert e.value.status == binding.E_ARG


def test_boost_plain_fp32_full_size(ctx):
    """The 8192 x 4096 workload with t = 3 (delta = 0.05)."""
    w = gen.plain_fp32(0)
    check_boost(ctx, w, 3, seed=5, label="plain-fp32 full size")
