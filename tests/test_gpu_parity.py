"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (derived in tests/gates.py):
  * ||A||_F^2, block scores of a given V: FP64 accumulation of exact squares
    of FP32 values on both sides, so only the summation order differs:
    relative 1e-12.
  * sampling, gather: integer / copy results, bit-exact.
  * sketched scores: the GPU runs the range finder in FP32, the oracle twin
    in FP64 from the same test matrix; the gate is four times the scores'
    measured response to an FP32-sized backward perturbation of A
    (gates.score_gate), at least 16 u32.
  * indices: identical whenever the oracle's smallest sampling margin exceeds
    2 G max_g tol_g (the largest shift any interval edge can see).
  * residual err = ||A - C C^+ A||_F: relative 1e-5 given identical indices
    (first order insensitive to errors in U at the least-squares optimum).
  * U = C^+ A: the least-squares perturbation bound for the FP32 backward
    error of the normal equations, max(10, sqrt(m)) u32; at least 1e-5
    (gates.u_gate).
"""
import math

import numpy as np
import pytest
import torch

from oracle import bcur_oracle as O
from workloads import gen

from .gates import index_margin_needed, score_gate, u_gate

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
SCORE_C = 64.0   # exactly low-rank inputs against the exact SVD (range-finder stage tests)


@pytest.fixture(scope="module")
def ctx():
    from paper_1703_06065_amd import Context
    return Context(0)


def dev(a):
    from paper_1703_06065_amd.binding import to_device
    return to_device(a)


def dev_dense(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def dev_ld(a, ld):
    t = torch.zeros((a.shape[0], ld), dtype=torch.float32)
    t[:, :a.shape[1]] = torch.from_numpy(np.asarray(a, dtype=np.float32))
    return t.cuda()[:, :a.shape[1]]


def note(*a):
    print(*a, flush=True)


def err_tol(err_ref, frob2):
    """1e-5 relative, with a floor of 16 u32 ||A||_F for residuals that are
    zero in exact arithmetic (the FP32 residual cannot resolve below it)."""
    return 1e-5 * err_ref + 16 * U32 * math.sqrt(frob2)


def out_quant_tol(C, U):
    """Residual added by storing an exact least-squares U in FP32: at most
    ||C (U - fl32(U))||_F <= u32 ||C||_F ||U||_F.  Used where the fit is
    flagged rank-deficient or ill-conditioned (a basic solution can have a
    large norm)."""
    return 4 * U32 * math.sqrt(O.frob2(C)) * math.sqrt(O.frob2(U))


# ---------------------------------------------------------------------------
# stage parity
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,pad", [(1, 1, 0), (7, 5, 3), (300, 200, 0), (513, 257, 7), (1024, 4096, 0)])
def test_frob2(ctx, m, n, pad):
    note(f"frob2 m={m} n={n} pad={pad}")
    A = np.random.default_rng(m * 7 + n).standard_normal((m, n)).astype(np.float32)
    ld = (n + pad + 3) // 4 * 4
    got, fin = ctx.frob2(dev_ld(A, ld))
    want = O.frob2(A.astype(np.float64))
    assert fin
    assert abs(got - want) <= 1e-12 * want


def test_frob2_nonfinite(ctx):
    note("frob2 nonfinite")
    A = np.ones((64, 32), dtype=np.float32)
    A[5, 7] = np.nan
    assert ctx.frob2(dev(A))[1] is False
    A[5, 7] = np.inf
    assert ctx.frob2(dev(A))[1] is False


@pytest.mark.parametrize("n,k,b,ragged", [(64, 5, 8, False), (1000, 17, 1, False), (333, 30, 16, True),
                                          (4096, 50, 16, False), (77, 3, 77, False)])
def test_block_scores(ctx, n, k, b, ragged):
    note(f"block_scores n={n} k={k} b={b} ragged={ragged}")
    V = np.random.default_rng(n + k).standard_normal((n, k)).astype(np.float32)
    off = gen.ragged_blocks(n, -(-n // b), 5) if ragged else gen.contiguous_blocks(n, b)
    got = ctx.block_scores(dev(V), off)
    want = O.block_scores(V.astype(np.float64), off)
    assert np.all(np.abs(got - want) <= 1e-12 * np.maximum(want, 1e-30))


def _sampler_cases():
    rng = np.random.default_rng(31)
    cases = []
    for t in range(30):
        G = int(rng.integers(1, 3000)) if t % 3 else int(rng.integers(1, 40))
        sc = rng.random(G) * (rng.random(G) < 0.7) * 10.0 ** rng.integers(-5, 5)
        if t % 5 == 0:
            sc[:] = 0.0
            sc[rng.integers(0, G)] = 1.0
        replace = bool(t % 2)
        s = int(rng.integers(1, min(G, 40) + 1)) if not replace else int(rng.integers(1, 60))
        dr = gen.draws_u64(s, 100 + t)
        if t % 4 == 0:
            dr[0] = 0
            dr[-1] = np.uint64(2 ** 64 - 1)
        cases.append((sc, dr, s, replace))
    return cases


@pytest.mark.parametrize("case", range(30))
def test_sampler_bit_exact(ctx, case):
    sc, dr, s, replace = _sampler_cases()[case]
    note(f"sample case={case} G={len(sc)} s={s} replace={replace}")
    idx, w, mg = ctx.sample_blocks(sc, dr, s, replace)
    ref = O.sample_blocks(sc, dr, s, replace)
    assert np.array_equal(idx, ref["idx"])
    fin = np.isfinite(ref["weights"])
    assert np.array_equal(np.isfinite(w), fin)
    assert np.allclose(w[fin], ref["weights"][fin], rtol=1e-15, atol=0)
    assert np.allclose(mg, ref["margins"], rtol=1e-15, atol=0)


def _large_sampler_cases():
    """G above the sampler's LDS capacity (4096 weights): the kernel's global
    memory path, with and without replacement, all-zero and sparse scores, and
    the edge draws 0 and 2^64 - 1."""
    rng = np.random.default_rng(77)
    cases = []
    for t, G in enumerate([4097, 5000, 8192, 12345, 20000, 20000]):
        sc = rng.random(G) * 10.0 ** rng.integers(-3, 3)
        if t == 2:
            sc[:] = 0.0
        if t == 3:
            sc *= rng.random(G) < 0.05
        replace = bool(t % 2)
        s = 40 if not replace else 64
        dr = gen.draws_u64(s, 500 + t)
        dr[0] = 0
        dr[-1] = np.uint64(2 ** 64 - 1)
        cases.append((sc, dr, s, replace))
    return cases


@pytest.mark.parametrize("case", range(6))
def test_sampler_bit_exact_large_g(ctx, case):
    sc, dr, s, replace = _large_sampler_cases()[case]
    note(f"sample large-G case={case} G={len(sc)} s={s} replace={replace}")
    idx, w, mg = ctx.sample_blocks(sc, dr, s, replace)
    ref = O.sample_blocks(sc, dr, s, replace)
    assert np.array_equal(idx, ref["idx"])
    fin = np.isfinite(ref["weights"])
    assert np.array_equal(np.isfinite(w), fin)
    assert np.allclose(w[fin], ref["weights"][fin], rtol=1e-15, atol=0)
    assert np.allclose(mg, ref["margins"], rtol=1e-15, atol=0)


def test_sampler_rejects_bad_scores(ctx):
    from paper_1703_06065_amd import BcurError
    note("sample bad scores")
    for bad in (np.array([1.0, -1.0]), np.array([1.0, np.nan]), np.array([np.inf, 1.0])):
        with pytest.raises(BcurError):
            ctx.sample_blocks(bad, gen.draws_u64(1, 0), 1, False)


@pytest.mark.parametrize("m,n,b,idx", [(50, 40, 4, [3, 0, 9]), (33, 100, 7, [14, 2, 2, 5]), (8, 8, 8, [0])])
def test_gather_bit_exact(ctx, m, n, b, idx):
    note(f"gather m={m} n={n} b={b} idx={idx}")
    A = np.random.default_rng(m).standard_normal((m, n)).astype(np.float32)
    off = gen.contiguous_blocks(n, b)
    C = ctx.gather_columns(dev(A), off, idx).cpu().numpy()
    want = A[:, O.selected_columns(off, idx)]
    assert np.array_equal(C, want)


@pytest.mark.parametrize("m,n,b,blocks", [(300, 200, 10, [1, 5, 7]), (257, 515, 16, [0, 31, 12, 4]),
                                          (1000, 129, 3, [40, 2, 11, 30, 7])])
def test_fit_columns(ctx, m, n, b, blocks):
    note(f"fit m={m} n={n} b={b} blocks={blocks}")
    w = gen.small_case(m, n, b, 8, 4, seed=m + n)
    C = w.A[:, O.selected_columns(w.offsets, blocks)]
    U, err, flags = ctx.fit_columns(dev(w.A), dev(C), refine=1)
    Uo, erro = O.fit_columns(w.A, C)
    U = U.cpu().numpy().astype(np.float64)
    cond = O.cond2(C)
    rel_u = np.linalg.norm(U - Uo) / np.linalg.norm(Uo)
    gate = u_gate(cond, erro, math.sqrt(O.frob2(w.A)), w.m)
    note(f"  err={err:.9g} oracle={erro:.9g} rel_u={rel_u:.2e} gate={gate:.2e} cond={cond:.3g} flags={flags}")
    assert abs(err - erro) <= err_tol(erro, O.frob2(w.A))
    assert rel_u <= gate


# ---------------------------------------------------------------------------
# the range finder
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,rho,k,l", [(300, 200, 12, 10, 20), (120, 260, 8, 8, 12), (1000, 640, 30, 25, 40)])
def test_range_finder_exact_low_rank(ctx, m, n, rho, k, l):
    note(f"range_finder low-rank m={m} n={n} rho={rho} k={k} l={l}")
    A = gen.gaussian_product(m, n, rho, m + n).astype(np.float32)
    om = gen.rademacher(n, l, m)
    V, _, ritz = ctx.range_finder(dev(A), dev_dense(om), k, q=1)
    off = gen.contiguous_blocks(n, 10)
    got = ctx.block_scores(V, off)
    ex = O.block_scores(O.exact_right_subspace(A.astype(np.float64), k), off)
    sv = np.linalg.svd(A.astype(np.float64), compute_uv=False)
    kappa = sv[0] ** 2 / (sv[k - 1] ** 2 - sv[k] ** 2)
    dev_ = np.abs(got - ex).max() / (k / len(ex))
    note(f"  max |dl|/(k/G) = {dev_:.2e} kappa={kappa:.3g}  ritz rel err={np.abs(ritz[:rho] - sv[:rho]).max() / sv[0]:.2e}")
    assert dev_ <= max(1e-5, SCORE_C * U32 * kappa)
    assert np.allclose(ritz[:rho], sv[:rho], rtol=1e-4, atol=1e-5 * sv[0])
    Vh = V.cpu().numpy().astype(np.float64)
    assert np.abs(Vh.T @ Vh - np.eye(k)).max() < 1e-5


# ---------------------------------------------------------------------------
# the whole path
# ---------------------------------------------------------------------------

def _check_decompose(ctx, w, replace=False, refine=1, label="", omega=None, precision="fp32", gate_draws=3):
    """One decomposition against the oracle twin.  omega: what the GPU is
    handed (default: w.omega uploaded; an int seed draws the same matrix on the
    device when w.omega is the oracle's Philox matrix of that seed)."""
    from paper_1703_06065_amd import binding
    note(f"decompose {label} {w.name} m={w.m} n={w.n} G={w.G} k={w.k} s={w.s} l={w.l} replace={replace} "
         f"precision={precision}")
    prec = binding.PREC_BF16 if precision == "bf16" else binding.PREC_FP32
    om = dev_dense(w.omega) if omega is None else omega
    res = ctx.decompose(dev(w.A), w.offsets, w.k, w.s, om, w.draws, q=w.q, replace=replace, refine=refine,
                        precision=prec, l=w.l)
    ref = O.decompose(w.A, w.offsets, w.k, w.s, w.omega, w.draws, q=w.q, replace=replace)
    gt = score_gate(w.A, w.offsets, w.k, w.q, w.omega, ref["scores"], precision=precision, draws=gate_draws)
    tol = gt["tol"]
    dl = np.abs(res["scores"] - ref["scores"])
    note(f"  kappa={ref['kappa']:.3g} d={gt['d']:.2e} tau={gt['tau']:.2e} max|dl|/tol={np.max(dl / tol):.3f} "
         f"max|dl|/(k/G)={dl.max() / (w.k / w.G):.2e} margin={ref['margins'].min():.3e}")
    assert np.all(dl <= tol)
    assert abs(res["frob2"] - ref["frob2"]) <= 1e-12 * ref["frob2"]
    need = index_margin_needed(tol)
    same = np.array_equal(res["idx"], ref["idx"])
    note(f"  idx gpu={list(res['idx'])} oracle={list(ref['idx'])} need margin>{need:.2e}")
    if ref["margins"].min() > need:
        assert same
    if same:
        tol = err_tol(ref["err"], ref["frob2"])
        C = O.gather_columns(w.A, w.offsets, res["idx"])
        Ug = res["U"][: res["c"]].cpu().numpy().astype(np.float64)
        if res["flags"] & (binding.FLAG_RANKDEF_C | binding.FLAG_ILLCOND_C):
            tol += out_quant_tol(C, Ug)
        note(f"  err={res['err']:.9g} oracle={ref['err']:.9g} rel={abs(res['err'] - ref['err']) / ref['err']:.2e} "
             f"tol={tol:.3g} flags={res['flags']}")
        assert abs(res["err"] - ref["err"]) <= tol
        assert res["c"] == len(ref["cols"])
        if not res["flags"] & (binding.FLAG_RANKDEF_C | binding.FLAG_ILLCOND_C):
            # U itself: a rank-deficient or ill-conditioned C gets a basic solution instead
            cond = O.cond2(C)
            rel_u = np.linalg.norm(Ug - ref["U"]) / np.linalg.norm(ref["U"])
            gate = u_gate(cond, ref["err"], math.sqrt(ref["frob2"]), w.m)
            note(f"  rel U gap {rel_u:.2e} gate {gate:.2e} cond(C)={cond:.3g} reported estimate {res['cond_c']:.3g}")
            assert rel_u <= gate
            # the reported estimate is a lower bound on cond(C): the diagonal of a triangular factor
            assert 1.0 - 1e-6 <= res["cond_c"] <= cond * (1 + 1e-4)
    # the precision report: kappa from the returned Ritz values, near the twin's
    lam = np.asarray(res["ritz"], dtype=np.float64) ** 2
    if w.k < w.l:
        k_own = lam[0] / (lam[w.k - 1] - lam[w.k])
        assert abs(res["kappa"] - k_own) <= 1e-6 * k_own
        note(f"  kappa reported {res['kappa']:.4g} twin {ref['kappa']:.4g}")
        assert abs(res["kappa"] - ref["kappa"]) <= 0.1 * ref["kappa"]
    else:
        # a different but valid selection: distinct blocks, in range, and a
        # residual that matches the oracle's fit of the GPU's own blocks
        idx = res["idx"]
        assert len(set(idx.tolist())) == len(idx) or replace
        assert idx.min() >= 0 and idx.max() < w.G
        _, e2 = O.fit_columns(w.A, O.gather_columns(w.A, w.offsets, idx))
        assert abs(res["err"] - e2) <= err_tol(e2, ref["frob2"])
    return res, ref


def test_decompose_tiny(ctx):
    _check_decompose(ctx, gen.tiny(0), label="tiny")


@pytest.mark.parametrize("m,n,b,k,s,ragged,seed", [
    (300, 200, 10, 8, 4, False, 1),
    (257, 515, 16, 12, 5, True, 2),
    (1000, 129, 3, 5, 7, False, 3),
    (129, 1000, 25, 20, 6, False, 4),
    (640, 384, 32, 30, 3, False, 5),
])
def test_decompose_shapes(ctx, m, n, b, k, s, ragged, seed):
    w = gen.small_case(m, n, b, k, s, seed=seed, ragged=ragged)
    _check_decompose(ctx, w, label="shape")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_frob2_fused_in_split_bf16_sketch(ctx, precision):
    # ||A||_F^2 is summed by the first FP32 pass over A (A Q), which at
    # m l n >= 8e9 runs on the 256 x 128 split-BF16 tile: every element of A
    # counted exactly once (the kernel's last step repeats a load that must
    # not count twice)
    from paper_1703_06065_amd import binding
    m, n, l, k, s = 8192, 8192, 120, 100, 8
    note(f"fused ||A||^2 through the split-BF16 sketch tile m={m} n={n} l={l} precision={precision}")
    rng = np.random.default_rng(4242)
    A = rng.standard_normal((m, n), dtype=np.float32)
    offsets = np.arange(0, n + 1, 64, dtype=np.int64)
    draws = rng.integers(0, 2 ** 63, size=s, dtype=np.int64).astype(np.uint64)
    prec = binding.PREC_BF16 if precision == "bf16" else binding.PREC_FP32
    res = ctx.decompose(dev(A), offsets, k, s, 5, draws, q=1, l=l, precision=prec)
    want = float(np.sum(A.astype(np.float64) ** 2))
    note(f"  frob2 gpu={res['frob2']:.17g} exact={want:.17g} rel={abs(res['frob2'] - want) / want:.2e}")
    assert abs(res["frob2"] - want) <= 1e-12 * want


def test_decompose_with_replacement(ctx):
    w = gen.small_case(400, 300, 10, 8, 12, seed=11, noise=1e-2)
    _check_decompose(ctx, w, replace=True, label="replace")


@pytest.mark.parametrize("word", [0x9E3779B97F4A7C15, 2 ** 64 - 1])
def test_decompose_fewer_columns_than_laid_out(ctx, word):
    """Draws with replacement that all pick one block: the workspace is laid
    out for s blocks (432 columns, for which the residual product is large
    enough for the 256 x 256 tile) but the fit runs with one block's columns,
    whose residual takes the 128 x 128 tile and writes more partial sums
    than the larger product would.  err and U against the oracle's fit of
    the same columns."""
    from paper_1703_06065_amd import binding
    m, n, b, s = 5181, 3590, 16, 27
    w = gen.small_case(m, n, b, k=22, s=s, seed=1531)
    draws = np.full(s, word, dtype=np.uint64)
    res = ctx.decompose(dev(w.A), w.offsets, w.k, w.s, dev_dense(w.omega), draws, q=w.q, replace=True, l=w.l)
    idx = res["idx"]
    assert len(set(idx.tolist())) == 1
    cols = O.selected_columns(w.offsets, idx)
    c = len(cols)
    assert res["c"] == c and c in (6, 16)
    assert not res["flags"] & (binding.FLAG_RANKDEF_C | binding.FLAG_ILLCOND_C)
    A64 = w.A.astype(np.float64)
    U_ref, e_ref = O.fit_columns(A64, A64[:, cols])
    frob2 = O.frob2(A64)
    note(f"one block of {c} columns: err={res['err']:.9g} oracle={e_ref:.9g}")
    assert abs(res["err"] - e_ref) <= err_tol(e_ref, frob2)
    Ug = res["U"][:c].cpu().numpy().astype(np.float64)
    rel_u = np.linalg.norm(Ug - U_ref) / np.linalg.norm(U_ref)
    assert rel_u <= u_gate(O.cond2(A64[:, cols]), e_ref, math.sqrt(frob2), m)


def test_decompose_all_blocks_zero_error(ctx):
    w = gen.small_case(300, 96, 8, 6, 12, seed=12, noise=1e-2)
    note("decompose all blocks")
    res = ctx.decompose(dev(w.A), w.offsets, w.k, w.G, dev_dense(w.omega), w.draws[:w.G] if len(w.draws) >= w.G
                        else gen.draws_u64(w.G, 12), q=w.q)
    note(f"  rel_err={res['rel_err']:.3e} flags={res['flags']}")
    assert sorted(res["idx"].tolist()) == list(range(w.G))
    assert res["rel_err"] <= 1e-5


def test_decompose_deterministic(ctx):
    w = gen.small_case(500, 300, 10, 10, 5, seed=13)
    note("decompose determinism")
    a = ctx.decompose(dev(w.A), w.offsets, w.k, w.s, dev_dense(w.omega), w.draws)
    b = ctx.decompose(dev(w.A), w.offsets, w.k, w.s, dev_dense(w.omega), w.draws)
    assert a["err"] == b["err"]
    assert np.array_equal(a["scores"], b["scores"])
    assert torch.equal(a["U"], b["U"])


def test_decompose_errors(ctx):
    from paper_1703_06065_amd import BcurError, binding
    w = gen.small_case(100, 80, 8, 5, 3, seed=14)
    A = dev(w.A)
    om = dev_dense(w.omega)
    note("decompose errors")
    bad = w.A.copy()
    bad[3, 4] = np.nan
    with pytest.raises(BcurError) as e:
        ctx.decompose(dev(bad), w.offsets, w.k, w.s, om, w.draws)
    assert e.value.status == binding.E_NONFINITE
    with pytest.raises(BcurError) as e:
        ctx.decompose(A, w.offsets, w.k, w.G + 1, om, gen.draws_u64(w.G + 1, 0))
    assert e.value.status == binding.E_ARG
    off = w.offsets.copy()
    off[2] = off[1]
    with pytest.raises(BcurError) as e:
        ctx.decompose(A, off, w.k, w.s, om, w.draws)
    assert e.value.status == binding.E_ARG
    with pytest.raises(BcurError) as e:
        ctx.decompose(A, w.offsets, w.l + 1, w.s, om, w.draws)
    assert e.value.status == binding.E_ARG
    # sketch width above the eigensolver's limit of 128
    Aw = dev(gen.gaussian_product(200, 200, 8, 15).astype(np.float32))
    with pytest.raises(BcurError) as e:
        ctx.range_finder(Aw, dev_dense(gen.rademacher(200, 129, 16)), 8, q=1)
    assert e.value.status == binding.E_ARG


# ---------------------------------------------------------------------------
# kernel-selection boundaries: sketch widths around the two Jacobi variants
# (L <= 64 and L <= 128), the limit 128 and the smallest widths, C widths around the single-kernel
# Cholesky limit (c <= 256) and the 64-wide panels of the blocked path
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("l", [1, 2, 3, 4, 5, 6, 7, 63, 64, 65, 66, 100, 127, 128])
def test_range_finder_sketch_widths(ctx, l):
    k = max(1, l - 3)
    m, n = 400, 300
    note(f"range_finder width l={l} k={k}")
    A = gen.gaussian_product(m, n, k, 1000 + l).astype(np.float32)
    om = gen.rademacher(n, l, 2000 + l)
    V, _, ritz = ctx.range_finder(dev(A), dev_dense(om), k, q=1)
    off = gen.contiguous_blocks(n, 10)
    got = ctx.block_scores(V, off)
    ex = O.block_scores(O.exact_right_subspace(A.astype(np.float64), k), off)
    sv = np.linalg.svd(A.astype(np.float64), compute_uv=False)
    kappa = sv[0] ** 2 / max(sv[k - 1] ** 2 - sv[k] ** 2, 1e-300)
    d = np.abs(got - ex).max() / (k / len(ex))
    note(f"  max |dl|/(k/G) = {d:.2e} kappa={kappa:.3g}")
    assert d <= max(1e-5, SCORE_C * U32 * kappa)
    assert np.allclose(ritz[:k], sv[:k], rtol=1e-4, atol=1e-5 * sv[0])
    Vh = V.cpu().numpy().astype(np.float64)
    assert np.abs(Vh.T @ Vh - np.eye(k)).max() < 1e-5


@pytest.mark.parametrize("c", [1, 63, 64, 65, 255, 256, 257, 320])
def test_fit_columns_widths(ctx, c):
    m, n = 700, 150
    note(f"fit width c={c}")
    rng = np.random.default_rng(3000 + c)
    C = rng.standard_normal((m, c))
    A = C[:, : min(c, 40)] @ rng.standard_normal((min(c, 40), n)) + 0.1 * rng.standard_normal((m, n))
    A = A.astype(np.float32)
    C = C.astype(np.float32)
    U, err, flags = ctx.fit_columns(dev(A), dev(C), refine=1)
    Uo, erro = O.fit_columns(A, C)
    U = U.cpu().numpy().astype(np.float64)
    cond = O.cond2(C)
    rel_u = np.linalg.norm(U - Uo) / np.linalg.norm(Uo)
    gate = u_gate(cond, erro, math.sqrt(O.frob2(A)), m)
    note(f"  err={err:.9g} oracle={erro:.9g} rel_u={rel_u:.2e} gate={gate:.2e} cond={cond:.3g} flags={flags}")
    assert abs(err - erro) <= err_tol(erro, O.frob2(A))
    assert rel_u <= gate


@pytest.mark.parametrize("m,n,c", [(4096, 4096, 512), (4100, 3900, 520)])
def test_fit_columns_split_bf16_products(ctx, m, n, c):
    # products of at least 8e9 multiply-adds (H = C^T A, ||A - C U||) run as
    # six BF16 products of the exact three-term splits of their operands;
    # whole 256 x 256 tiles take the path without bounds checks, a ragged
    # shape the checked one.  Same gates as the FP32 products.
    note(f"fit through the split-BF16 products m={m} n={n} c={c}")
    rng = np.random.default_rng(m + n + c)
    C = rng.standard_normal((m, c))
    A = C[:, :60] @ rng.standard_normal((60, n)) + 0.05 * rng.standard_normal((m, n))
    A = A.astype(np.float32)
    C = C.astype(np.float32)
    U, err, flags = ctx.fit_columns(dev(A), dev(C), refine=1)
    Uo, erro = O.fit_columns(A, C)
    U = U.cpu().numpy().astype(np.float64)
    cond = O.cond2(C)
    rel_u = np.linalg.norm(U - Uo) / np.linalg.norm(Uo)
    gate = u_gate(cond, erro, math.sqrt(O.frob2(A)), m)
    note(f"  err={err:.9g} oracle={erro:.9g} rel_u={rel_u:.2e} gate={gate:.2e} cond={cond:.3g} flags={flags}")
    assert abs(err - erro) <= err_tol(erro, O.frob2(A))
    assert rel_u <= gate


def test_fit_columns_rank_deficient_wide(ctx):
    # c > m and a repeated column: the Gram matrix C^T C is singular.  The
    # fit must flag the dropped pivots, redo the solve in FP64 (Cholesky QR2)
    # and return a least-squares solution: its residual is the optimum (zero
    # here) up to the FP32 storage of U, and the reported err is its own.
    from paper_1703_06065_amd import binding
    m, n, c = 200, 90, 300
    rng = np.random.default_rng(31)
    C = rng.standard_normal((m, c)).astype(np.float32)
    C[:, 5] = C[:, 2]
    A = rng.standard_normal((m, n)).astype(np.float32)
    note("fit rank-deficient c > m")
    U, err, flags = ctx.fit_columns(dev(A), dev(C), refine=1)
    Uh = U.cpu().numpy().astype(np.float64)[:c]
    own = math.sqrt(O.frob2(A.astype(np.float64) - C.astype(np.float64) @ Uh))
    note(f"  err={err:.6g} own residual={own:.6g} flags={flags}")
    assert flags & binding.FLAG_RANKDEF_C
    assert np.all(np.isfinite(Uh)) and math.isfinite(err)
    _, erro = O.fit_columns(A, C)
    tol = err_tol(erro, O.frob2(A)) + out_quant_tol(C.astype(np.float64), Uh)
    note(f"  oracle={erro:.3e} tol={tol:.3e}")
    assert err <= erro + tol and own <= erro + tol
    assert abs(err - own) <= tol


def test_fit_columns_rank_deficient_many_panels(ctx):
    # The FP64 fallback solves n > 1024 columns of A in panels of 1024; each
    # panel of U is written where it belongs and nothing else of the output
    # buffer is touched (U is a c x n view inside a wider, taller buffer whose
    # other elements hold a sentinel).
    import torch
    from paper_1703_06065_amd import binding
    m, n, c = 400, 2600, 120
    rng = np.random.default_rng(32)
    C = rng.standard_normal((m, c)).astype(np.float32)
    C[:, 7] = C[:, 3]
    A = rng.standard_normal((m, n)).astype(np.float32)
    sentinel = 7.25
    big = torch.full((c + 3, n + 12), sentinel, dtype=torch.float32, device="cuda")
    note("fit rank-deficient, three fallback panels, guarded output")
    U, err, flags = ctx.fit_columns(dev(A), dev(C), refine=1, U_out=big[:c, :n])
    torch.cuda.synchronize()
    hb = big.cpu().numpy()
    assert flags & binding.FLAG_RANKDEF_C
    assert np.all(hb[:c, n:] == sentinel) and np.all(hb[c:] == sentinel)
    Uh = hb[:c, :n].astype(np.float64)
    own = math.sqrt(O.frob2(A.astype(np.float64) - C.astype(np.float64) @ Uh))
    _, erro = O.fit_columns(A, C)
    tol = err_tol(erro, O.frob2(A)) + out_quant_tol(C.astype(np.float64), Uh)
    note(f"  err={err:.9g} own residual={own:.9g} oracle={erro:.9g} tol={tol:.3e} flags={flags}")
    assert np.all(np.isfinite(Uh))
    assert abs(err - erro) <= tol and abs(own - erro) <= tol


# ---------------------------------------------------------------------------
# full size, in the configuration the benchmark times
# ---------------------------------------------------------------------------

def test_decompose_plain_fp32_full_size(ctx):
    w = gen.plain_fp32(0)
    res, ref = _check_decompose(ctx, w, label="full-size")
    assert np.array_equal(res["idx"], ref["idx"])


def _residual_skips_chosen(m, n, c):
    """The documented rule: the residual pass covers only the n - c columns
    outside C when that product runs on the split-BF16 tile and its 256 x 256
    tiles take fewer rounds of 256 workgroups than over all n columns."""
    ne = n - c
    if not (ne >= 256 and m >= 256 and c >= 256 and n <= 262144 and m * ne * c >= 8e9):
        return False
    rounds = lambda cols: -(-(-(-m // 256) * -(-cols // 256)) // 256)
    return rounds(ne) < rounds(n)


@pytest.mark.parametrize("s,replace,refine,ragged", [
    (48, False, 1, False),   # n - c = 2040 columns: the tile-checked form of the column list
    (48, False, 0, False),   # no refinement: U[:, cols] = I set before the residual pass
    (70, True, 1, False),    # draws with replacement: repeated blocks dropped on the host
    (70, False, 1, True),    # ragged blocks: the columns expanded on the host
])
def test_decompose_residual_over_unchosen_columns(ctx, s, replace, refine, ragged):
    """A residual product that runs fewer rounds of workgroups over the
    n - c columns outside C: U on C's own columns is set to the identity (C
    e_k is that column of A, so their residual is exactly zero) and the pass
    covers the other columns through their list.  err against the oracle's
    fit of the GPU's own blocks, U on C's columns bit-exactly I, and U on 16
    other columns against R^-1 Q^T a_j within the U gate."""
    from paper_1703_06065_amd import binding
    m, n, b = 16384, 3000, 20
    w = gen.small_case(m, n, b, k=20, s=s, seed=11, ragged=ragged)
    note(f"residual over unchosen columns: {m}x{n} s={s} replace={replace} refine={refine} ragged={ragged}")
    res = ctx.decompose(dev(w.A), w.offsets, w.k, w.s, dev_dense(w.omega), w.draws, q=w.q, replace=replace,
                        refine=refine, l=w.l)
    assert not res["flags"] & (binding.FLAG_RANKDEF_C | binding.FLAG_ILLCOND_C)
    cols = O.selected_columns(w.offsets, res["idx"])
    c = len(cols)
    assert res["c"] == c and _residual_skips_chosen(m, n, c), c
    Ug = res["U"][:c].cpu().numpy()
    assert np.array_equal(Ug[:, cols], np.eye(c, dtype=np.float32))
    A64 = w.A.astype(np.float64)
    C = A64[:, cols]
    rest = np.setdiff1d(np.arange(n), cols)
    J = np.sort(np.random.default_rng(5).choice(rest, 16, replace=False))
    e_ref, U_J = O.fit_columns_qr(A64, C, cols=J)
    frob2 = O.frob2(A64)
    tol = err_tol(e_ref, frob2)
    note(f"  c={c} err={res['err']:.9g} oracle={e_ref:.9g} rel={abs(res['err'] - e_ref) / e_ref:.2e}")
    assert abs(res["err"] - e_ref) <= tol
    cond = O.cond2(C)
    rel_u = np.linalg.norm(Ug[:, J].astype(np.float64) - U_J) / np.linalg.norm(U_J)
    gate = u_gate(cond, e_ref, math.sqrt(frob2), m)
    note(f"  rel U gap on 16 other columns {rel_u:.2e} gate {gate:.2e} cond(C)={cond:.3g}")
    assert rel_u <= gate


def test_residual_rule_at_the_benchmarked_sizes():
    """The column list is taken at 65536 x 16384 with c = 2048 (64 rounds of
    workgroups over all columns, 56 over the others), not at 8192 x 4096 with
    c = 256 (two rounds either way)."""
    assert _residual_skips_chosen(65536, 16384, 2048)
    assert not _residual_skips_chosen(8192, 4096, 256)
