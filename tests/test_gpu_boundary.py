"""The C ABI's seeded test matrix, asynchronous decomposition and scratch
budget, through the library.

  * bcur_test_matrix: the Philox4x64-10 Rademacher matrix drawn on the device
    equals the oracle's own implementation of the same generator bit for bit
    (integer-valued output: exact);
  * a decomposition whose test matrix comes from a seed equals, bit for bit,
    the decomposition handed the oracle's matrix of that seed, and matches the
    oracle twin run from that matrix (the single-decomposition bars);
  * bcur_decompose_async + bcur_wait give the same bits as bcur_decompose;
  * a context's scratch budget refuses a call that needs more workspace,
    before anything is allocated.
"""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import bcur_oracle as O
from workloads import gen

from .test_gpu_parity import _check_decompose, dev, dev_dense, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1703_06065_amd import Context
    return Context(0)


@pytest.mark.parametrize("n,l,seed", [(1, 1, 0), (37, 60, 5), (300, 112, 2 ** 64 - 3), (130, 128, 7),
                                      (65, 256, 11), (4097, 64, 123456789)])
def test_test_matrix_bits(ctx, n, l, seed):
    note(f"test matrix n={n} l={l} seed={seed}")
    got = ctx.test_matrix(n, l, seed).cpu().numpy()
    want = O.rademacher_omega(n, l, seed)
    assert np.array_equal(got.astype(np.float64), want)


def test_test_matrix_leaves_padding(ctx):
    from paper_1703_06065_amd import binding
    note("test matrix padding untouched")
    n, l, ld = 70, 30, 36
    buf = torch.full((n, ld), 7.0, dtype=torch.float32, device="cuda")
    st = ctx.lib.bcur_test_matrix(ctx.h, n, l, 9, buf.data_ptr(), ld)
    assert st == binding.OK
    h = buf.cpu().numpy()
    assert np.array_equal(h[:, :l].astype(np.float64), O.rademacher_omega(n, l, 9))
    assert np.all(h[:, l:] == 7.0)
    for bad in ((n, 0, ld), (n, 257, 300), (n, l, l - 1), (0, l, ld)):
        assert ctx.lib.bcur_test_matrix(ctx.h, bad[0], bad[1], 9, buf.data_ptr(), bad[2]) == binding.E_ARG


def _seeded(w, seed):
    """The workload with the oracle's Philox test matrix of `seed`."""
    return dataclasses.replace(w, omega=O.rademacher_omega(w.n, w.l, seed).astype(np.float32))


@pytest.mark.parametrize("case", ["tiny", "shape", "ragged"])
def test_decompose_from_seed(ctx, case):
    w = {"tiny": lambda: gen.tiny(0),
         "shape": lambda: gen.small_case(640, 384, 32, 30, 3, seed=5),
         "ragged": lambda: gen.small_case(257, 515, 16, 12, 5, seed=2, ragged=True)}[case]()
    seed = 1000 + len(case)
    sw = _seeded(w, seed)
    note(f"decompose from seed {seed} ({case})")
    A = dev(w.A)
    a = ctx.decompose(A, w.offsets, w.k, w.s, seed, w.draws, q=w.q, l=w.l)
    b = ctx.decompose(A, w.offsets, w.k, w.s, dev_dense(sw.omega), w.draws, q=w.q)
    assert np.array_equal(a["idx"], b["idx"])
    assert np.array_equal(a["scores"], b["scores"])
    assert a["err"] == b["err"] and a["frob2"] == b["frob2"]
    assert torch.equal(a["U"], b["U"])
    _check_decompose(ctx, sw, label=f"seeded {case}")


def _same(a, b):
    assert np.array_equal(a["idx"], b["idx"])
    assert np.array_equal(a["weights"], b["weights"])
    assert np.array_equal(a["scores"], b["scores"])
    assert np.array_equal(a["ritz"], b["ritz"])
    assert a["err"] == b["err"] and a["c"] == b["c"] and a["flags"] == b["flags"]
    assert torch.equal(a["U"], b["U"])
    if "idx_r" in a:
        assert np.array_equal(a["idx_r"], b["idx_r"])


@pytest.mark.parametrize("case", ["uniform", "ragged", "rows"])
def test_async_equals_sync(ctx, case):
    from paper_1703_06065_amd import BcurError, binding
    note(f"async vs sync ({case})")
    if case == "rows":
        w = gen.small_case(400, 300, 10, 8, 4, seed=21)
        roff = gen.contiguous_blocks(w.m, 20)
        draws = gen.draws_u64(w.s + 3, 21)
        kw = dict(row_offsets=roff, s_r=3)
    else:
        w = gen.small_case(500, 300, 10, 10, 5, seed=13, ragged=(case == "ragged"))
        draws = w.draws
        kw = {}
    A = dev(w.A)
    om = dev_dense(w.omega)
    ref = ctx.decompose(A, w.offsets, w.k, w.s, om, draws, q=w.q, **kw)
    pend = ctx.decompose_async(A, w.offsets, w.k, w.s, om, draws, q=w.q, **kw)
    assert pend is not None
    # the context refuses other calls while the decomposition is in flight
    st = ctx.lib.bcur_synchronize(ctx.h)
    assert st in (binding.E_STATE,)
    got = ctx.wait()
    _same(got, ref)
    assert ctx.wait() is None
    # seeded and asynchronous
    a = ctx.decompose(A, w.offsets, w.k, w.s, 77, draws, q=w.q, **kw)
    ctx.decompose_async(A, w.offsets, w.k, w.s, 77, draws, q=w.q, **kw)
    _same(ctx.wait(), a)
    # an argument error found on the context's thread is reported by wait
    ctx.decompose_async(A, w.offsets, w.m + w.n, w.s, om, draws, q=w.q, **kw)
    with pytest.raises(BcurError) as e:
        ctx.wait()
    assert e.value.status == binding.E_ARG


def test_async_ordered_after_caller_stream(ctx):
    # A is written on the caller's stream right before the asynchronous call:
    # the decomposition must see the new values
    note("async ordering after the caller's stream")
    w = gen.small_case(300, 200, 10, 8, 4, seed=1)
    A = dev(w.A)
    om = dev_dense(w.omega)
    ref = ctx.decompose(A, w.offsets, w.k, w.s, om, w.draws, q=w.q)
    B = torch.zeros_like(A)
    torch.cuda.synchronize()
    B.copy_(A)   # queued on the current stream, which is the context's
    ctx.decompose_async(B, w.offsets, w.k, w.s, om, w.draws, q=w.q)
    _same(ctx.wait(), ref)


def test_scratch_budget(ctx):
    from paper_1703_06065_amd import BcurError, Context, binding
    note("scratch budget")
    w = gen.small_case(300, 200, 10, 8, 4, seed=1)
    A = dev(w.A)
    om = dev_dense(w.omega)
    need = ctx.footprint(w.m, w.n, w.offsets, w.k, w.s, w.l, q=w.q)
    small = Context(0, scratch_budget=need // 2)
    with pytest.raises(BcurError) as e:
        small.decompose(A, w.offsets, w.k, w.s, om, w.draws, q=w.q)
    assert e.value.status == binding.E_NOMEM
    assert small.workspace_bytes == 0
    fits = Context(0, scratch_budget=need)
    res = fits.decompose(A, w.offsets, w.k, w.s, om, w.draws, q=w.q)
    ref = ctx.decompose(A, w.offsets, w.k, w.s, om, w.draws, q=w.q)
    _same(res, ref)
    assert 0 < fits.workspace_bytes <= need
    small.close()
    fits.close()
