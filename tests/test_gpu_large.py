"""The large-share workload (65536 x 16384 FP32, 256 blocks of 64, k = 100,
s = 32, BF16 range finder) at its real size, checked on sampled outputs and on
properties that hold at any size (the FP64 oracle cannot run the whole path
here in reasonable time):

  * ||A||_F^2 against an exact FP64 sum (relative 1e-12);
  * block scores: non-negative, at most min(b_g, k), summing to k (the scores
    of an orthonormal k-column basis; relative 1e-4);
  * the s sampled blocks are distinct and in range; C has 2048 columns;
  * err against ||A - C U||_F recomputed on the host from the returned U
    (relative 1e-5: the same U, FP32 products summed in another order);
  * 16 sampled columns j: ||a_j - C u_j|| against the least-squares optimum
    min_u ||a_j - C u|| from an FP64 QR of C (relative 1e-5).
"""
import math
import time

import numpy as np
import pytest

from oracle import bcur_oracle as O
from workloads import gen

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def note(*a):
    print(*a, flush=True)


def test_large_share_sampled():
    import torch

    from paper_1703_06065_amd import Context
    from paper_1703_06065_amd.binding import PREC_BF16, to_device
    t0 = time.time()
    w = gen.large_share(0)
    note(f"large share {w.m}x{w.n} generated in {time.time() - t0:.1f} s")
    ctx = Context(0)
    A = to_device(w.A)
    om = torch.from_numpy(w.omega).cuda()
    res = ctx.decompose(A, w.offsets, w.k, w.s, om, w.draws, q=w.q, precision=PREC_BF16)
    torch.cuda.synchronize()
    note(f"  decompose done: c={res['c']} err={res['err']:.6g} rel={res['rel_err']:.4g} flags={res['flags']}")
    del A
    fro = 0.0
    for i in range(0, w.m, 4096):
        blk = w.A[i:i + 4096].astype(np.float64)
        fro += float(np.einsum("ij,ij->", blk, blk))
    assert abs(res["frob2"] - fro) <= 1e-12 * fro
    sc = res["scores"]
    widths = np.diff(w.offsets)
    assert np.all(sc >= -1e-6) and np.all(sc <= np.minimum(widths, w.k) * (1 + 1e-4))
    assert abs(sc.sum() - w.k) <= 1e-4 * w.k
    idx = res["idx"]
    assert len(set(idx.tolist())) == w.s and idx.min() >= 0 and idx.max() < w.G
    cols = O.selected_columns(w.offsets, idx)
    assert res["c"] == len(cols) == 2048
    C = np.ascontiguousarray(w.A[:, cols])
    U = res["U"][: res["c"]].cpu().numpy()
    t1 = time.time()
    e2 = 0.0
    for i in range(0, w.m, 4096):
        R = w.A[i:i + 4096] - C[i:i + 4096] @ U
        e2 += float(np.einsum("ij,ij->", R.astype(np.float64), R.astype(np.float64)))
    note(f"  host residual {math.sqrt(e2):.6g} vs gpu {res['err']:.6g} ({time.time() - t1:.1f} s)")
    assert abs(res["err"] - math.sqrt(e2)) <= 1e-5 * math.sqrt(e2)
    t1 = time.time()
    Q, _ = np.linalg.qr(C.astype(np.float64))
    J = np.random.default_rng(7).choice(w.n, 16, replace=False)
    AJ = w.A[:, J].astype(np.float64)
    r_opt = np.linalg.norm(AJ - Q @ (Q.T @ AJ), axis=0)
    r_gpu = np.linalg.norm(AJ - C.astype(np.float64) @ U[:, J].astype(np.float64), axis=0)
    note(f"  sampled columns: max rel excess {np.max((r_gpu - r_opt) / r_opt):.2e} ({time.time() - t1:.1f} s)")
    assert np.all(np.abs(r_gpu - r_opt) <= 1e-5 * r_opt)
