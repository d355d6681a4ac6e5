"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (on the paper's normalised scale g = f / B_eff):
  * reweighting: bit-exact (integer counts, correctly rounded 1/m, index-order B_eff);
  * objective: |f_gpu - f_oracle| / |f_oracle| <= 1e-5 per site;
  * gradient: max |g_gpu - g_oracle| / B_eff <= 2e-6.  The energies are FP32 sums
    of up to N - 1 couplings (|J| ~ 0.1-1 here), so each softmax probability
    carries a relative error of order sqrt(N) * 2^-24 * max|E| (~1e-6); the
    data gradient is a B_eff-normalised sum of w_b (P - I) and inherits it;
  * scores: relative 1e-9 (FP64 on identical FP32 couplings).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.helpers import clustered_msa, fixed_point_bounds, hilo_bounds, load_reweight_golden, random_params

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def plm():
    import paper_1401_4832_amd as plm
    return plm


def _note(msg):
    print(f"[case] {msg}", flush=True)


def _to(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


# ---------------------------------------------------------------- reweighting
@pytest.mark.parametrize("theta", [0.0, 0.6, 0.8, 1.0])
def test_reweight_golden(plm, theta):
    import os
    rows, cases = load_reweight_golden(os.path.join(os.path.dirname(__file__), "golden", "reweight_tiny.txt"))
    _note(f"reweight golden theta={theta}")
    m, w, beff = plm.reweight(_to(rows), theta=theta)
    plm.sync(DEV)
    m_o, w_o, beff_o = oracle.reweight(rows, theta=theta)
    assert np.array_equal(m.cpu().numpy(), m_o)
    assert np.array_equal(w.cpu().numpy(), w_o)
    assert beff.item() == beff_o


@pytest.mark.parametrize("B,N,p_mut,theta", [(1, 7, 0.1, 0.8), (65, 13, 0.1, 0.8), (700, 37, 0.12, 0.8),
                                             (1300, 120, 0.2, 0.8), (999, 64, 0.15, 0.7),
                                             (513, 5, 0.3, 0.6)])
def test_reweight_clustered_bit_exact(plm, B, N, p_mut, theta):
    _note(f"reweight clustered B={B} N={N} theta={theta}")
    msa = clustered_msa(seed=B + N, B=B, N=N, n_anc=max(1, B // 40), p_mut=p_mut)
    m, w, beff = plm.reweight(_to(msa), theta=theta)
    plm.sync(DEV)
    m_o, w_o, beff_o = oracle.reweight(msa, theta=theta)
    assert np.array_equal(m.cpu().numpy(), m_o)
    assert np.array_equal(w.cpu().numpy(), w_o)
    assert beff.item() == beff_o


def test_reweight_workload_gapped(plm):
    s = synth.workload("potts_n120_b5000_gaps")
    _note("reweight potts_n120_b5000_gaps")
    m, w, beff = plm.reweight(_to(s.msa), theta=0.8)
    plm.sync(DEV)
    m_o, w_o, beff_o = oracle.reweight(s.msa, theta=0.8)
    assert np.array_equal(m.cpu().numpy(), m_o) and beff.item() == beff_o


def test_reweight_uniform(plm):
    msa = clustered_msa(seed=1, B=300, N=20, n_anc=3, p_mut=0.05)
    m, w, beff = plm.reweight(_to(msa), uniform=True)
    plm.sync(DEV)
    assert torch.all(w == 1.0) and beff.item() == 300.0


# ----------------------------------------------------------- objective/grad
# paths held to the FP32 tolerance: gather/scatter; gather + three-piece BF16 MFMA gradient;
# three-piece MFMA both ways; gather + FP16 hi/lo MFMA gradient (22 significant bits of R, error
# <= 2^-22 |R| per residual, i.e. <= 2.4e-7 on the normalised gradient, inside the FP32 bound)
PATHS = [0, 2, 3, 4, 5, 6, 7]


def _objgrad_case(plm, msa, w_o, beff_o, h, J, lh=0.01, lJ=0.01, sites=None, path=0, fabs=False):
    B, N = msa.shape
    q = h.shape[1]
    w = _to(w_o)
    beff = _to(np.array([beff_o]))
    f, gh, gJ = plm.objgrad(_to(msa), w, beff, _to(h.astype(np.float32)), _to(J.astype(np.float32)),
                            lh, lJ, sites=sites, path=path)
    plm.sync(DEV)
    Jz = J.astype(np.float32).astype(np.float64)
    for r in range(N):
        Jz[r, r] = 0
    hz = h.astype(np.float32).astype(np.float64)
    idx = np.arange(N) if sites is None else np.asarray(sites)
    fo, gho, gJo = oracle.objgrad(msa, w_o, beff_o, hz, Jz, lh, lJ, sites=idx)
    f = f.cpu().numpy()[idx]
    gh = gh.cpu().numpy()[idx]
    gJ = gJ.cpu().numpy()[idx]
    frel = np.max(np.abs(f - fo) / np.abs(fo))
    gerr = max(np.max(np.abs(gJ - gJo)), np.max(np.abs(gh - gho))) / beff_o
    if fabs:
        return np.max(np.abs(f - fo)) / beff_o, gerr, gJ
    return frel, gerr, gJ


@pytest.mark.parametrize("B,N,q", [(500, 40, 21), (7, 17, 21), (3001, 33, 21), (1537, 49, 11), (700, 97, 21)])
def test_objgrad_hilo_path_within_derived_bound(plm, B, N, q):
    _note(f"objgrad hi/lo B={B} N={N} q={q}")
    rng = np.random.default_rng(B * 7 + N)
    msa = rng.integers(0, q, size=(B, N), dtype=np.uint8)
    w_o = rng.uniform(0.2, 1.0, size=B)
    beff_o = float(np.sum(w_o))
    h, J = random_params(B + q, N, q, 0.3, 0.2)
    fb, gb = hilo_bounds(msa, h, J, range(N))
    ferr, gerr, gJ = _objgrad_case(plm, msa, w_o, beff_o, h, J, path=1, fabs=True)
    print(f"  hi/lo errors: f {ferr:.2e} (bound {fb:.2e}), grad {gerr:.2e} (bound {gb:.2e})")
    assert gerr <= gb + 2e-6, (gerr, gb)
    assert ferr <= fb + 1e-5 * np.log(q) * 10, (ferr, fb)
    for r in range(N):
        assert np.all(gJ[r, r] == 0)


@pytest.mark.parametrize("B,N,q,sd", [(700, 97, 21, 1.0), (3001, 33, 21, 2.0), (1537, 49, 11, 0.5), (400, 200, 21, 0.8)])
def test_objgrad_fixed_point_path_within_derived_bound(plm, B, N, q, sd):
    _note(f"objgrad int8 fixed point B={B} N={N} q={q} sd={sd}")
    rng = np.random.default_rng(B * 3 + N)
    msa = rng.integers(0, q, size=(B, N), dtype=np.uint8)
    w_o = rng.uniform(0.2, 1.0, size=B)
    beff_o = float(np.sum(w_o))
    h, J = random_params(B + 2 * q, N, q, 0.3, sd)
    fb, gb = fixed_point_bounds(msa, w_o, beff_o, J, range(N))
    ferr, gerr, gJ = _objgrad_case(plm, msa, w_o, beff_o, h, J, path=6, fabs=True)
    print(f"  int8 errors: f {ferr:.2e} (bound {fb:.2e}), grad {gerr:.2e} (bound {gb:.2e})")
    # the FP32 parts (softmax, residuals before rounding) add at most the FP32 tolerance
    assert ferr <= fb + 1e-5 * np.log(q) * 10, (ferr, fb)
    assert gerr <= gb + 2e-6, (gerr, gb)
    for r in range(N):
        assert np.all(gJ[r, r] == 0)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("B,N,q", [(500, 40, 21), (1, 2, 21), (7, 17, 21), (3001, 33, 21), (800, 25, 3),
                                   (1537, 49, 11), (4000, 70, 21), (700, 97, 21)])
def test_objgrad_random_point(plm, B, N, q, path):
    _note(f"objgrad random B={B} N={N} q={q} path={path}")
    rng = np.random.default_rng(B * 7 + N)
    msa = rng.integers(0, q, size=(B, N), dtype=np.uint8)
    w_o = rng.uniform(0.2, 1.0, size=B)
    beff_o = float(np.sum(w_o))
    h, J = random_params(B + q, N, q, 0.3, 0.2)
    frel, gerr, gJ = _objgrad_case(plm, msa, w_o, beff_o, h, J, path=path)
    assert frel <= 1e-5, frel
    assert gerr <= 2e-6, gerr
    for r in range(N):
        assert np.all(gJ[r, r] == 0)


@pytest.mark.parametrize("B,N,q", [(500, 40, 21), (1, 2, 21), (3001, 33, 21), (800, 25, 3), (1537, 49, 11),
                                   (4000, 70, 21)])
def test_objgrad_precise_path_is_fp64_class(plm, B, N, q):
    """Path 7 (FP64 energies, log-softmax and residuals; residuals carried to
    2^-45 in two exact integer passes) agrees with the FP64 oracle to FP64
    rounding: relative objective within 1e-11, and every gradient entry
    within the FP32 rounding of the call's FP32 output (2^-24 relative) plus
    1e-11 on the normalised scale."""
    _note(f"objgrad precise path B={B} N={N} q={q}")
    rng = np.random.default_rng(B * 13 + N)
    msa = rng.integers(0, q, size=(B, N), dtype=np.uint8)
    w_o = rng.uniform(0.2, 1.0, size=B)
    beff_o = float(np.sum(w_o))
    h, J = random_params(B + 5 * q, N, q, 0.3, 0.3)
    f, gh, gJ = plm.objgrad(_to(msa), _to(w_o), _to(np.array([beff_o])), _to(h.astype(np.float32)),
                            _to(J.astype(np.float32)), 0.01, 0.01, path=7)
    plm.sync(DEV)
    Jz = J.astype(np.float32).astype(np.float64)
    for r in range(N):
        Jz[r, r] = 0
    fo, gho, gJo = oracle.objgrad(msa, w_o, beff_o, h.astype(np.float32).astype(np.float64), Jz, 0.01, 0.01)
    f, gh, gJ = f.cpu().numpy(), gh.cpu().numpy().astype(np.float64), gJ.cpu().numpy().astype(np.float64)
    frel = float(np.max(np.abs(f - fo) / np.abs(fo)))
    excess = max(float(np.max(np.abs(gJ - gJo) - 2.0 ** -24 * np.abs(gJo))),
                 float(np.max(np.abs(gh - gho) - 2.0 ** -24 * np.abs(gho)))) / beff_o
    print(f"  precise path: f rel {frel:.2e}, gradient beyond FP32 output rounding {excess:.2e}")
    assert frel <= 1e-11, frel
    assert excess <= 1e-11, excess
    for r in range(N):
        assert np.all(gJ[r, r] == 0)


@pytest.mark.parametrize("path", [5, 6, 7])
def test_objgrad_int8_gradient_either_side_of_2e17_sequences(plm, path):
    """The int8 gradient builds its one-hot operand with -128 for a one while an
    alignment has fewer than 2^17 padded sequences (the int32 sums then hold
    -128 times the digit sums exactly) and with +1 beyond.  One more sequence
    of weight zero moves an alignment of 42 * 3072 = 129 024 sequences (the
    largest multiple of the 3072-sequence padding below 2^17) across that
    limit: the
    coupling gradient stays the same bit for bit (its digit sums are exact
    either way), the objective and field gradient agree to FP64 rounding, and
    the larger call matches the oracle (FP32 tolerance on paths 5 and 6,
    FP64 class on path 7)."""
    B, N, q = 42 * 3072, 5, 21
    _note(f"objgrad int8 gradient B={B}/{B + 1} N={N} path={path}")
    rng = np.random.default_rng(131)
    msa = rng.integers(0, q, size=(B + 1, N), dtype=np.uint8)
    w_o = rng.uniform(0.2, 1.0, size=B + 1)
    w_o[B] = 0.0
    beff_o = float(np.sum(w_o))
    h, J = random_params(131, N, q, 0.3, 0.2)
    h32, J32 = h.astype(np.float32), J.astype(np.float32)
    outs = []
    for n in (B, B + 1):
        f, gh, gJ = plm.objgrad(_to(msa[:n]), _to(w_o[:n]), _to(np.array([beff_o])), _to(h32), _to(J32),
                                0.01, 0.01, path=path)
        plm.sync(DEV)
        outs.append((f.cpu().numpy(), gh.cpu().numpy(), gJ.cpu().numpy()))
    (fa, gha, gJa), (fb, ghb, gJb) = outs
    assert np.array_equal(gJa, gJb)
    assert np.all(np.abs(fa - fb) <= 1e-12 * np.abs(fb)), np.max(np.abs(fa - fb) / np.abs(fb))
    gha64, ghb64 = gha.astype(np.float64), ghb.astype(np.float64)
    assert np.all(np.abs(gha64 - ghb64) <= 2.0 ** -22 * np.abs(ghb64) + 1e-12 * beff_o)
    Jz = J32.astype(np.float64)
    for r in range(N):
        Jz[r, r] = 0
    fo, gho, gJo = oracle.objgrad(msa, w_o, beff_o, h32.astype(np.float64), Jz, 0.01, 0.01)
    frel = float(np.max(np.abs(fb - fo) / np.abs(fo)))
    if path == 7:
        excess = max(float(np.max(np.abs(gJb - gJo) - 2.0 ** -24 * np.abs(gJo))),
                     float(np.max(np.abs(ghb - gho) - 2.0 ** -24 * np.abs(gho)))) / beff_o
        assert frel <= 1e-11 and excess <= 1e-11, (frel, excess)
    else:
        gerr = max(float(np.max(np.abs(gJb - gJo))), float(np.max(np.abs(ghb - gho)))) / beff_o
        assert frel <= 1e-5 and gerr <= 2e-6, (frel, gerr)
    for r in range(N):
        assert np.all(gJb[r, r] == 0)


@pytest.mark.parametrize("path", PATHS)
def test_objgrad_workload_gapped(plm, path):
    s = synth.workload("potts_n120_b5000_gaps")
    _note(f"objgrad potts_n120_b5000_gaps path={path}")
    m_o, w_o, beff_o = oracle.reweight(s.msa, theta=0.8)
    h, J = random_params(3, s.N, 21, 0.1, 0.1)
    frel, gerr, _ = _objgrad_case(plm, s.msa, w_o, beff_o, h, J, sites=[0, 5, 60, 119], path=path)
    assert frel <= 1e-5 and gerr <= 2e-6, (frel, gerr)


@pytest.mark.parametrize("path", PATHS + [1])
def test_objgrad_ignores_self_blocks(plm, path):
    """The self blocks J[r][r] take no part in any result (eq. condpfinal sums
    over i != r): large finite values there give exactly the results of zero
    self blocks, and the gradient's self blocks are zero."""
    _note(f"objgrad with garbage self blocks path={path}")
    B, N, q = 1300, 27, 21
    rng = np.random.default_rng(77)
    msa = rng.integers(0, q, size=(B, N), dtype=np.uint8)
    w = _to(rng.uniform(0.2, 1.0, size=B))
    beff = _to(np.array([float(w.sum().item())]))
    h, J = random_params(78, N, q, 0.3, 0.2)
    Jg = J.astype(np.float32).copy()
    for r in range(N):
        Jg[r, r] = (1e4 * rng.standard_normal((q, q))).astype(np.float32)
    ht = _to(h.astype(np.float32))
    a = plm.objgrad(_to(msa), w, beff, ht, _to(J.astype(np.float32)), path=path)
    b = plm.objgrad(_to(msa), w, beff, ht, _to(Jg), path=path)
    plm.sync(DEV)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
    for r in range(N):
        assert torch.all(b[2][r, r] == 0)


def test_fit_ignores_start_point_self_blocks(plm):
    """A start point with garbage self blocks gives the fit of zero self
    blocks, bit for bit, with zero self blocks returned."""
    _note("fit with garbage self blocks in the start point")
    s = synth.make_msa("sb", N=14, B=700, npairs=8, seed=34, cache=False, burnin=100, thin=2)
    msa = _to(s.msa)
    m, w, beff = plm.reweight(msa, theta=0.8)
    N, q = 14, 21
    J0 = torch.zeros(N, N, q, q, dtype=torch.float32, device=DEV)
    Jg = J0.clone()
    for r in range(N):
        Jg[r, r] = 1e4 * torch.randn(q, q, device=DEV, generator=None)
    h0 = torch.zeros(N, q, dtype=torch.float32, device=DEV)
    a = plm.fit(msa, w, beff, plm.FitOptions(tol=1e-6), h0=h0, J0=J0)
    b = plm.fit(msa, w, beff, plm.FitOptions(tol=1e-6), h0=h0, J0=Jg)
    assert torch.equal(a.J, b.J) and torch.equal(a.h, b.h)
    for r in range(N):
        assert torch.all(b.J[r, r] == 0)


@pytest.mark.parametrize("path", PATHS + [1])
def test_objgrad_without_gradient_gives_the_same_objective(plm, path):
    """With the gradient outputs absent only the forward runs; its objective is
    the one of the full evaluation, bit for bit (the forward's own set-up, such
    as the int8 path's packed symbols, runs either way)."""
    _note(f"objgrad without gradient path={path}")
    B, N, q = 2100, 31, 21
    rng = np.random.default_rng(91)
    msa = rng.integers(0, q, size=(B, N), dtype=np.uint8)
    w = _to(rng.uniform(0.2, 1.0, size=B))
    beff = _to(np.array([float(w.sum().item())]))
    h, J = random_params(92, N, q, 0.3, 0.2)
    ht, Jt = _to(h.astype(np.float32)), _to(J.astype(np.float32))
    full = plm.objgrad(_to(msa), w, beff, ht, Jt, path=path)
    fonly, gh, gJ = plm.objgrad(_to(msa), w, beff, ht, Jt, path=path, grad=False)
    plm.sync(DEV)
    assert gh is None and gJ is None
    assert torch.equal(full[0], fonly)


def test_objgrad_at_origin_is_beff_log_q(plm):
    s = synth.workload("potts_n40_b500")
    msa = _to(s.msa)
    m, w, beff = plm.reweight(msa, uniform=True)
    f, gh, gJ = plm.objgrad(msa, w, beff, torch.zeros(40, 21, device=DEV),
                            torch.zeros(40, 40, 21, 21, device=DEV))
    plm.sync(DEV)
    np.testing.assert_allclose(f.cpu().numpy(), 500 * np.log(21.0), rtol=1e-7)


@pytest.mark.parametrize("path", PATHS)
def test_objgrad_deterministic(plm, path):
    rng = np.random.default_rng(9)
    msa = rng.integers(0, 21, size=(2000, 30), dtype=np.uint8)
    w = _to(np.ones(2000))
    beff = _to(np.array([2000.0]))
    h, J = random_params(10, 30, 21)
    ht, Jt = _to(h.astype(np.float32)), _to(J.astype(np.float32))
    a = plm.objgrad(_to(msa), w, beff, ht, Jt, path=path)
    b = plm.objgrad(_to(msa), w, beff, ht, Jt, path=path)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])


# ---------------------------------------------------------------- scoring
@pytest.mark.parametrize("N,q", [(2, 21), (40, 21), (9, 4), (130, 21)])
def test_score_matches_oracle(plm, N, q):
    _note(f"score N={N} q={q}")
    rng = np.random.default_rng(N)
    J = rng.standard_normal((N, N, q, q)).astype(np.float32)
    fn, cfn = plm.score(_to(J))
    plm.sync(DEV)
    fn_o, cfn_o = oracle.score(J)
    np.testing.assert_allclose(fn.cpu().numpy(), fn_o, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(cfn.cpu().numpy(), cfn_o, rtol=1e-9, atol=1e-12)


# ---------------------------------------------------------------- errors
def test_symbol_out_of_range_is_reported(plm):
    msa = np.zeros((10, 5), dtype=np.uint8)
    msa[3, 2] = 21
    plm.reweight(_to(msa), theta=0.8)
    with pytest.raises(plm.PlmError) as e:
        plm.sync(DEV)
    assert e.value.code == -2


def test_nonfinite_input_is_reported(plm):
    msa = np.zeros((10, 5), dtype=np.uint8)
    w = _to(np.ones(10))
    beff = _to(np.array([10.0]))
    J = torch.zeros(5, 5, 21, 21, device=DEV)
    J[1, 2, 3, 4] = float("nan")
    plm.objgrad(_to(msa), w, beff, torch.zeros(5, 21, device=DEV), J)
    with pytest.raises(plm.PlmError) as e:
        plm.sync(DEV)
    assert e.value.code == -3


def test_invalid_arguments_are_rejected(plm):
    msa = _to(np.zeros((10, 5), dtype=np.uint8))
    with pytest.raises(plm.PlmError) as e:
        plm.reweight(msa, theta=1.5)
    assert e.value.code == -1
    with pytest.raises(plm.PlmError):
        plm.reweight(msa, q=22)
