"""The parity gates of tests/gates.py are tight enough to matter: on the
workloads the GPU tests use, a score error of 1e-4 (k/G) on one block fails
the score gate, and the U gate stays within the FP32 accuracy it is derived
from (CPU only: the FP64 twin and the oracle's fits)."""
import math

import numpy as np
import pytest

from oracle import bcur_oracle as O
from workloads import gen

from .gates import score_gate, u_gate


def _cases():
    return [("tiny", gen.tiny(0)),
            ("300x200", gen.small_case(300, 200, 10, 8, 4, seed=1)),
            ("257x515 ragged", gen.small_case(257, 515, 16, 12, 5, seed=2, ragged=True)),
            ("1000x129", gen.small_case(1000, 129, 3, 5, 7, seed=3)),
            ("129x1000", gen.small_case(129, 1000, 25, 20, 6, seed=4)),
            ("640x384", gen.small_case(640, 384, 32, 30, 3, seed=5))]


@pytest.mark.parametrize("case", range(6))
def test_score_gate_rejects_1e4_error(case):
    name, w = _cases()[case]
    ref = O.decompose(w.A, w.offsets, w.k, w.s, w.omega, w.draws, q=w.q, with_fit=False)
    gt = score_gate(w.A, w.offsets, w.k, w.q, w.omega, ref["scores"])
    bad = ref["scores"].copy()
    g = int(np.argmax(ref["scores"]))
    bad[g] += 1e-4 * w.k / w.G
    ok = np.all(np.abs(bad - ref["scores"]) <= gt["tol"])
    print(f"{name}: kappa={ref['kappa']:.3g} tau={gt['tau']:.2e} tol at the largest score "
          f"{gt['tol'][g] / (w.k / w.G):.2e} (k/G)")
    assert not ok


def test_score_gate_bf16_rejects_1e2_error():
    w = gen.small_case(600, 400, 10, 10, 5, seed=21, decay="geometric", noise=1e-3)
    ref = O.decompose(w.A, w.offsets, w.k, w.s, w.omega, w.draws, q=w.q, with_fit=False)
    gt = score_gate(w.A, w.offsets, w.k, w.q, w.omega, ref["scores"], precision="bf16")
    assert gt["tau"] < 1e-2
    bad = ref["scores"] + 1e-2 * w.k / w.G
    assert not np.all(np.abs(bad - ref["scores"]) <= gt["tol"])


def test_u_gate_floor_and_growth():
    # at least 1e-5; grows with cond(C) squared and with the residual angle
    assert u_gate(1.0, 0.0, 1.0, 100) == 1e-5
    lo = u_gate(10.0, 0.1, 1.0, 10000)
    hi = u_gate(100.0, 0.1, 1.0, 10000)
    assert hi > 30 * lo
    assert u_gate(10.0, 0.9, 1.0, 10000) > u_gate(10.0, 0.1, 1.0, 10000)
    # the FP32 backward error: max(10, sqrt(m)) u32
    assert math.isclose(u_gate(30.0, 0.5, 1.0, 65536) / u_gate(30.0, 0.5, 1.0, 100), 25.6, rel_tol=1e-12)
