"""bcur_decompose_noalloc through the C ABI: the same results as
bcur_decompose, bit for bit (the same kernels on the same data; only the
workspace and host staging differ), on two calls in a row with the second on a
smaller input; no device memory is allocated by the calls; a workspace above
the scratch array's 128 MiB and block maps are refused before any work."""
import numpy as np
import pytest
import torch

from workloads import gen

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)


def _dev(a):
    from paper_1703_06065_amd.binding import to_device
    return to_device(a)


def _dense(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _same(a, b):
    assert np.array_equal(a["idx"], b["idx"])
    assert np.array_equal(a["weights"], b["weights"])
    assert np.array_equal(a["scores"], b["scores"])
    assert np.array_equal(a["ritz"], b["ritz"])
    assert a["err"] == b["err"] and a["frob2"] == b["frob2"]
    assert a["c"] == b["c"] and a["r"] == b["r"] and a["flags"] == b["flags"]
    assert a["rr_sweeps"] == b["rr_sweeps"]
    assert torch.equal(a["U"], b["U"])
    if "idx_r" in a:
        assert np.array_equal(a["idx_r"], b["idx_r"])


def test_noalloc_equals_decompose():
    from paper_1703_06065_amd import Context
    from paper_1703_06065_amd.binding import padded_empty
    ref_ctx = Context(0)
    ctx = Context(0)
    # one call first, so that runtime set-up outside the library (staging of
    # pageable copies) is not counted against the calls below
    w0 = gen.tiny(0)
    ctx.decompose_noalloc(_dev(w0.A), w0.offsets, w0.k, w0.s, _dense(w0.omega), w0.draws,
                          padded_empty(w0.s * 8, w0.n), q=w0.q)
    torch.cuda.synchronize()
    cases = [
        ("plain-fp32 8192x4096", gen.plain_fp32(0), {}),
        ("small 640x384", gen.small_case(640, 384, 32, 30, 3, seed=5), {}),
    ]
    for label, w, kw in cases:
        note(f"noalloc vs decompose: {label}")
        A = _dev(w.A)
        om = _dense(w.omega)
        U1 = padded_empty(w.s * int(np.max(np.diff(w.offsets))), w.n)
        U2 = padded_empty(w.s * int(np.max(np.diff(w.offsets))), w.n)
        ref = ref_ctx.decompose(A, w.offsets, w.k, w.s, om, w.draws, q=w.q, U_out=U1, **kw)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        got = ctx.decompose_noalloc(A, w.offsets, w.k, w.s, om, w.draws, U2, q=w.q, **kw)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        note(f"  err={got['err']:.9g} ref={ref['err']:.9g} device memory free before/after: {free0} / {free1}")
        _same(got, ref)
        assert ctx.workspace_bytes == 0
        assert free1 == free0
    # the row variant and a seeded test matrix
    w = gen.small_case(400, 300, 10, 8, 4, seed=21)
    roff = gen.contiguous_blocks(w.m, 20)
    draws = gen.draws_u64(w.s + 3, 21)
    A = _dev(w.A)
    U1 = padded_empty(40, 60)
    U2 = padded_empty(40, 60)
    note("noalloc vs decompose: row variant, seeded")
    ref = ref_ctx.decompose(A, w.offsets, w.k, w.s, 5, draws, q=w.q, l=w.l, row_offsets=roff, s_r=3, U_out=U1)
    got = ctx.decompose_noalloc(A, w.offsets, w.k, w.s, 5, draws, U2, q=w.q, l=w.l, row_offsets=roff, s_r=3)
    _same(got, ref)
    assert ctx.workspace_bytes == 0


def test_noalloc_refusals():
    from paper_1703_06065_amd import BcurError, Context, binding
    from paper_1703_06065_amd.binding import PREC_BF16, padded_empty
    ctx = Context(0)
    w = gen.plain_fp32(0)
    A = _dev(w.A)
    U = padded_empty(w.s * 16, w.n)
    note("noalloc refusals: BF16 workspace above the scratch array")
    with pytest.raises(BcurError) as e:
        ctx.decompose_noalloc(A, w.offsets, w.k, w.s, 3, w.draws, U, q=w.q, l=w.l, precision=PREC_BF16)
    assert e.value.status == binding.E_NOMEM
    assert ctx.workspace_bytes == 0
    note("noalloc refusals: block maps")
    prm = binding.Params(k=w.k, s=w.s, l=w.l, q=w.q, seed=3)
    cmap = np.arange(w.n, dtype=np.int64)
    prm.col_map = cmap.ctypes.data_as(binding.ctypes.POINTER(binding.ctypes.c_int64))
    idx = np.empty(w.s, dtype=np.int64)
    res = binding.Result()
    res.idx = idx.ctypes.data_as(binding.ctypes.POINTER(binding.ctypes.c_int64))
    res.U, res.ldu, res.u_rows_cap = U.data_ptr(), U.stride(0), U.shape[0]
    off = np.ascontiguousarray(w.offsets, dtype=np.int64)
    dr = np.ascontiguousarray(w.draws, dtype=np.uint64)
    st = ctx.lib.bcur_decompose_noalloc(ctx.h, A.data_ptr(), w.m, w.n, A.stride(0),
                                        off.ctypes.data_as(binding.ctypes.POINTER(binding.ctypes.c_int64)),
                                        len(off) - 1, None, 0, binding.ctypes.byref(prm), None,
                                        dr.ctypes.data_as(binding.ctypes.POINTER(binding.ctypes.c_uint64)),
                                        binding.ctypes.byref(res))
    assert st == binding.E_ARG
