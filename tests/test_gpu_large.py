"""The large-share workload (65536 x 16384 FP32, 256 blocks of 64, k = 100,
s = 32) at its real size and in the configuration the benchmark times: test
matrix drawn on the device from seed 0, BF16 range finder (two BF16 power
iterations, a final FP32 pass and the FP32 Rayleigh-Ritz step), FP32 fit with
one refinement step.

Against the FP64 oracle twin run from the same test matrix (the oracle's own
Philox implementation) and the same draws:
  * ||A||_F^2 (relative 1e-12);
  * block scores within the BF16 score gate of tests/gates.py (two perturbed
    twins at this size), and the sampled blocks identical wherever the
    twin's margins exceed the gate's shift;
  * err against the oracle's least-squares fit of the same blocks (QR route,
    column panels; relative 1e-5 plus 16 u32 ||A||_F);
  * U on 16 sampled columns against R^-1 Q^T a_j within the U gate.
"""
import math
import time

import numpy as np
import pytest

from oracle import bcur_oracle as O
from workloads import gen

from .gates import index_margin_needed, score_gate, u_gate

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

U32 = 2.0 ** -24


def note(*a):
    print(*a, flush=True)


@pytest.mark.timeout(900)
def test_large_share_against_twin():
    import torch

    from paper_1703_06065_amd import Context
    from paper_1703_06065_amd.binding import PREC_BF16, to_device
    t0 = time.time()
    w = gen.large_share(0)
    seed = 0
    note(f"large share {w.m}x{w.n} generated in {time.time() - t0:.1f} s")
    ctx = Context(0)
    A = to_device(w.A)
    res = ctx.decompose(A, w.offsets, w.k, w.s, seed, w.draws, q=w.q, l=w.l, precision=PREC_BF16)
    torch.cuda.synchronize()
    Ug = res["U"][: res["c"]].cpu().numpy()
    note(f"  decompose done: c={res['c']} err={res['err']:.9g} rel={res['rel_err']:.6g} flags={res['flags']}")
    del A
    torch.cuda.empty_cache()

    t1 = time.time()
    A64 = w.A.astype(np.float64)
    om = O.rademacher_omega(w.n, w.l, seed)
    ref = O.decompose(A64, w.offsets, w.k, w.s, om, w.draws, q=w.q, with_fit=False)
    note(f"  oracle twin in {time.time() - t1:.1f} s: kappa={ref['kappa']:.3g} margin={ref['margins'].min():.3e}")
    assert abs(res["frob2"] - ref["frob2"]) <= 1e-12 * ref["frob2"]
    t1 = time.time()
    gt = score_gate(A64, w.offsets, w.k, w.q, om, ref["scores"], precision="bf16", draws=2)
    dl = np.abs(res["scores"] - ref["scores"])
    note(f"  score gate in {time.time() - t1:.1f} s: d={gt['d']:.2e} tau={gt['tau']:.2e} "
         f"max|dl|/(k/G)={dl.max() / (w.k / w.G):.2e} max|dl|/tol={np.max(dl / gt['tol']):.3f}")
    assert np.all(dl <= gt["tol"])
    need = index_margin_needed(gt["tol"])
    same = np.array_equal(res["idx"], ref["idx"])
    note(f"  idx gpu={list(res['idx'])}\n      oracle={list(ref['idx'])} need margin>{need:.2e}")
    if ref["margins"].min() > need:
        assert same
    note(f"  blocks {'identical to' if same else 'differ from'} the twin's")
    idx = res["idx"]
    assert len(set(idx.tolist())) == w.s and idx.min() >= 0 and idx.max() < w.G
    cols = O.selected_columns(w.offsets, idx)
    assert res["c"] == len(cols) == 2048
    C = A64[:, cols]
    t1 = time.time()
    J = np.random.default_rng(7).choice(w.n, 16, replace=False)
    err_o, UJ = O.fit_columns_qr(A64, C, cols=J)
    note(f"  oracle fit of the GPU's blocks in {time.time() - t1:.1f} s: err={err_o:.9g} "
         f"rel gap {abs(res['err'] - err_o) / err_o:.2e}")
    assert abs(res["err"] - err_o) <= 1e-5 * err_o + 16 * U32 * math.sqrt(ref["frob2"])
    R = np.linalg.qr(C, mode="r")
    cond = O.cond2(R)
    rel_u = np.linalg.norm(Ug[:, J].astype(np.float64) - UJ) / np.linalg.norm(UJ)
    gate = u_gate(cond, err_o, math.sqrt(ref["frob2"]), w.m)
    note(f"  U on 16 sampled columns: rel gap {rel_u:.2e} gate {gate:.2e} cond(C)={cond:.3g}")
    assert rel_u <= gate
