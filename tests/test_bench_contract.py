"""Host-side checks of bench.py (no GPU): the one-GPU refusal, the HBM
traffic figure derived from the committed counter readings, and the FLOP
model of a decomposition."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_is_the_scaled_counter_readings():
    b = _bench()
    src = b._source_hash()
    fake = {"fit_E": {"src": src, "fetch_kib": 1000.0, "fetch_scale": 2.0, "write_kib": 10.0, "write_scale": 1.0}}
    assert b.traffic_for(fake, "fit_E") == round(1024.0 * (1000.0 * 2.0 + 10.0 * 1.0))
    assert b.traffic_for(fake, "fit_H") is None
    # readings taken on another kernel source are not reported
    stale = {"fit_E": dict(fake["fit_E"], src="0" * 16)}
    assert b.traffic_for(stale, "fit_E") is None
    # committed readings: at least the algorithmic bytes of one launch, 4 (mn + mc + cn)
    # for H and 4 (m ne + mc + c ne) for the residual over its ne columns
    for table, (m, n, c) in ((b.TRAFFIC_LARGE, (65536, 16384, 2048)), (b.TRAFFIC_PLAIN, (8192, 4096, 256))):
        for st in table:
            got = b.traffic_for(table, st)
            w = b.resid_columns(m, n, c) if st == "fit_E" else n
            if got is not None:
                assert got >= 4 * (m * w + m * c + c * w), (st, got)


def test_flop_model():
    b = _bench()
    m, n, k, l, q, c = 8192, 4096, 50, 60, 2, 256
    rf, fit = b.algorithmic_flops(m, n, k, l, q, c)
    rfL, fitL = b.algorithmic_flops(65536, 16384, 100, 110, 2, 2048)
    # 2q + 3 passes over A in the range finder (q + 1 times A Q and A^T Z, then the Rayleigh-Ritz A Q)
    assert rf == (2 * q + 3) * 2.0 * m * n * l
    # H = C^T A and the residual, then G^-1 H, H - G U, G^-1 F and G^-1 = X^T X;
    # at 8192 x 4096 x 256 the residual over the 3840 columns outside C would
    # take as many rounds of workgroups as over all 4096: it covers them all
    assert b.resid_columns(m, n, c) == n
    assert fit == 4.0 * m * c * n + 6.0 * c * c * n + 2.0 * c ** 3
    # at 65536 x 16384 x 2048 it covers the n - c columns outside C
    mL, nL, cL = 65536, 16384, 2048
    assert b.resid_columns(mL, nL, cL) == nL - cL
    assert fitL == 2.0 * mL * cL * nL + 2.0 * mL * cL * (nL - cL) + 6.0 * cL * cL * nL + 2.0 * cL ** 3
    # below the split tile's size the pass covers every column
    assert b.resid_columns(4096, 4096, 256) == 4096
    assert b.resid_columns(8192, 4096, 4000) == 4096
