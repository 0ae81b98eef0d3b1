"""Continuous batching: requests of uneven shapes, block widths and ranks,
submitted together and run concurrently in several slots, give results that
are bitwise identical to the same decompositions run alone; admission
honours the device-memory budget; an oversized request is refused."""
import time

import numpy as np
import pytest
import torch

from workloads import gen

pytestmark = pytest.mark.gpu


def dev(a):
    from paper_1703_06065_amd.binding import to_device
    return to_device(a)


def dense(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def note(*a):
    print(*a, flush=True)


def _requests(count, m_range=(256, 1536), n_range=(256, 1024)):
    return [gen.serving_request(i, m_range, n_range) for i in range(count)]


def test_mix_equals_alone():
    from paper_1703_06065_amd import Context, Server
    from paper_1703_06065_amd.binding import padded_empty
    ws = _requests(12)
    inputs = [(dev(w.A), dense(w.omega)) for w in ws]
    ctx = Context(0)
    alone = []
    for w, (A, om) in zip(ws, inputs):
        note(f"alone {w.name} G={w.G} k={w.k} s={w.s}")
        alone.append(ctx.decompose(A, w.offsets, w.k, w.s, om, w.draws, q=w.q))
    torch.cuda.synchronize()
    srv = Server(0, hbm_budget=4 << 30, max_slots=4)
    tickets = []
    for w, (A, om) in zip(ws, inputs):
        cap = min(w.s * int(np.max(np.diff(w.offsets))), w.n)
        tickets.append(srv.submit(A, w.offsets, w.k, w.s, om, w.draws, q=w.q, U_out=padded_empty(cap, w.n)))
    mixed = [srv.wait(t) for t in tickets]
    st = srv.stats()
    note(f"stats {st}")
    assert st["completed"] == len(ws) and st["failed"] == 0
    assert st["peak_running"] >= 2
    for w, a, b in zip(ws, alone, mixed):
        assert np.array_equal(a["idx"], b["idx"]), w.name
        assert a["err"] == b["err"], (w.name, a["err"], b["err"])
        assert np.array_equal(a["scores"], b["scores"])
        assert torch.equal(a["U"], b["U"])
    srv.close()


def test_budget_and_refusal():
    from paper_1703_06065_amd import BcurError, Server, binding
    ws = _requests(6, (512, 1024), (512, 1024))
    inputs = [(dev(w.A), dense(w.omega)) for w in ws]
    # a budget that holds about one request at a time
    lib = binding.load_library()
    import ctypes
    fps = []
    for w in ws:
        prm = binding.Params(k=w.k, s=w.s, l=w.l, q=w.q, replace=0, precision=0, refine=1, reserved=0, s_r=0)
        b = ctypes.c_size_t()
        off = np.ascontiguousarray(w.offsets, dtype=np.int64)
        assert lib.bcur_footprint(w.m, w.n, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), w.G, None, 0,
                                  ctypes.byref(prm), 1, ctypes.byref(b)) == 0
        fps.append(b.value)
    budget = int(max(fps) * 1.2)
    note(f"footprints {fps} budget {budget}")
    # a request whose own footprint exceeds the budget must be refused
    big = gen.serving_request(99, (8192, 8192), (4096, 4096))
    prm = binding.Params(k=big.k, s=big.s, l=big.l, q=big.q, replace=0, precision=0, refine=1, reserved=0, s_r=0)
    b = ctypes.c_size_t()
    off = np.ascontiguousarray(big.offsets, dtype=np.int64)
    assert lib.bcur_footprint(big.m, big.n, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), big.G, None, 0,
                              ctypes.byref(prm), 1, ctypes.byref(b)) == 0
    assert b.value > budget
    srv = Server(0, hbm_budget=budget, max_slots=3)
    tickets = [srv.submit(A, w.offsets, w.k, w.s, om, w.draws, q=w.q) for w, (A, om) in zip(ws, inputs)]
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    note(f"stats {st}")
    assert st["completed"] == len(ws)
    assert st["hbm_peak"] <= budget
    assert all(np.isfinite(r["err"]) for r in res)
    with pytest.raises(BcurError) as e:
        srv.submit(dev(big.A), big.offsets, big.k, big.s, dense(big.omega), big.draws)
    assert e.value.status == binding.E_ADMIT
    srv.close()


def test_poll_pending_then_done():
    from paper_1703_06065_amd import Server
    w = gen.serving_request(7, (2048, 2048), (1024, 1024))
    srv = Server(0, hbm_budget=4 << 30, max_slots=1)
    t = srv.submit(dev(w.A), w.offsets, w.k, w.s, dense(w.omega), w.draws)
    r = None
    for _ in range(20000):
        r = srv.poll(t)
        if r is not None:
            break
        time.sleep(0.001)
    assert r is not None and np.isfinite(r["err"])
    srv.close()
