"""Symmetric pseudolikelihood maximisation on the GPU (plm_fit_symmetric)
against the FP64 oracle's minimiser.

F is strongly convex with modulus mu = 2 min(lambda_h, lambda_J) (0.02 at
the default strengths), so ||theta - theta*|| <= ||grad F(theta)|| / mu.
The GPU stops at ||grad F|| <= 1e-6 (its FP32 evaluation, over all sites)
and the oracle below 1e-7, so every field and coupling must agree to about
1e-4; the certificate is re-checked with the oracle's FP64 gradient at the
GPU's final point.  The result must also be exactly consistent (J[i][r] is
J[r][i] transposed, bit for bit; self blocks zero) and satisfy the gauge the
l2 penalty fixes at the optimum (eq. symmetricgauge) to the accuracy the
certificate allows."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import symmetric as sym
from tests.helpers import split_words_ok

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def plm():
    import paper_1401_4832_amd as plm
    return plm


@pytest.fixture(scope="module")
def small():
    # B = 700: several forward tiles and a ragged tail at every tile size
    s = synth.make_msa("sym10", N=10, B=700, npairs=6, seed=41, cache=False, burnin=100, thin=2)
    m, w, beff = oracle.reweight(s.msa, theta=0.8)
    h_o, J_o, gn_o = sym.fit(s.msa, w, beff, 0.01, 0.01, q=21)
    assert gn_o <= 1e-7, gn_o
    return s, h_o, J_o


def _gpu_problem(plm, s):
    msa = torch.from_numpy(s.msa).to(DEV)
    m, w, beff = plm.reweight(msa, theta=0.8)
    return msa, w, beff


def _check_consistent(J):
    N = J.shape[0]
    for r in range(N):
        assert np.all(J[r, r] == 0.0), r
        for i in range(r + 1, N):
            assert np.array_equal(J[i, r], J[r, i].T), (r, i)


def _certificate(s, h, J, lh, lJ):
    m, w, beff = oracle.reweight(s.msa, theta=0.8)
    F, gh, gJ = sym.objective(s.msa, w, beff, h, J, lh, lJ)
    return F, float(np.sqrt(np.sum(gh ** 2) + np.sum(gJ ** 2)))


@pytest.mark.parametrize("path", [0, 2, 3, 4, 5, 6])
def test_symmetric_fit_matches_oracle(plm, small, path):
    s, h_o, J_o = small
    print(f"[case] symmetric fit N=10 B=700 path={path}", flush=True)
    msa, w, beff = _gpu_problem(plm, s)
    opts = plm.FitOptions(tol=1e-6, path=path)
    res = plm.fit_symmetric(msa, w, beff, opts)
    (st,) = res.stats
    assert st["status"] == "converged", st
    assert st["gnorm"] <= 1e-6
    h = res.h.cpu().numpy().astype(np.float64)
    J = res.J.cpu().numpy().astype(np.float64)
    _check_consistent(J)
    err = max(np.max(np.abs(J - J_o)), np.max(np.abs(h - h_o)))
    assert err <= 1e-4, err
    F, gn = _certificate(s, h, J, 0.01, 0.01)
    mu = 2 * 0.01
    assert gn / mu <= 2e-4, gn
    assert abs(st["f"] - F) <= 1e-6 * abs(F), (st["f"], F)
    # gauge at the optimum: lambda_J sum_k J_ri(k, s) = lambda_h h_r(s), sum_s h_r(s) = 0
    # (both hold exactly at the optimum and move by at most sqrt(q) resp.
    # lambda_J sqrt(q) + lambda_h times the distance to it)
    dist = gn / mu
    for r in range(10):
        assert abs(h[r].sum()) <= np.sqrt(21) * dist + 1e-7
        for i in range(10):
            if i != r:
                res_ri = np.max(np.abs(0.01 * J[r, i].sum(axis=0) - 0.01 * h[r]))
                assert res_ri <= (0.01 * np.sqrt(21) + 0.01) * dist + 1e-8, (r, i, res_ri)


def test_symmetric_refinement_continues_the_first_fit(plm, small):
    """After a fixed-point path the symmetric fit is refined (automatically, on
    the precise path 7) from the first fit's point: the first fit is the refine = -1 fit
    bit for bit, the statistics and timing add both, the final gradient norm
    is that of the refinement path's evaluation, and the result stays within
    1e-4 of the oracle's minimiser."""
    s, h_o, J_o = small
    print("[case] symmetric refinement after path 5", flush=True)
    msa, w, beff = _gpu_problem(plm, s)
    N = 10
    base = plm.fit_symmetric(msa, w, beff, plm.FitOptions(tol=1e-6, path=5, refine=-1, timing=True))
    tb = plm.last_fit_timing(DEV)
    assert tb["refine_site_evals"] == 0 and tb["refine_iterations"] == 0
    ref = plm.fit_symmetric(msa, w, beff, plm.FitOptions(tol=1e-6, path=5, timing=True))
    tr = plm.last_fit_timing(DEV)
    (sb,), (sr,) = base.stats, ref.stats
    assert sr["status"] == "converged" and sr["gnorm"] <= 1e-6
    assert tr["refine_iterations"] >= 1
    assert tr["refine_site_evals"] == (sr["evaluations"] - sb["evaluations"]) * N > 0
    assert tr["site_evals"] == tb["site_evals"] + tr["refine_site_evals"]
    assert tr["iterations"] == tb["iterations"] + tr["refine_iterations"]
    assert sr["iterations"] >= sb["iterations"]
    h = ref.h.cpu().numpy().astype(np.float64)
    J = ref.J.cpu().numpy().astype(np.float64)
    _check_consistent(J)
    assert max(np.max(np.abs(J - J_o)), np.max(np.abs(h - h_o))) <= 1e-4
    # the refinement's own evaluation at the returned point: a further fit on
    # the precise path from it stops at once
    again = plm.fit_symmetric(msa, w, beff, plm.FitOptions(tol=1e-6, path=7),
                              h0=ref.h, J0=ref.J)
    assert again.stats[0]["iterations"] == 0
    # an explicit refinement path, none after an FP32-class path, an unknown one rejected
    exp = plm.fit_symmetric(msa, w, beff, plm.FitOptions(tol=1e-6, path=5, refine=1 + 2))
    assert exp.stats[0]["status"] == "converged"
    plain = plm.fit_symmetric(msa, w, beff, plm.FitOptions(tol=1e-6, path=4, timing=True))
    assert plm.last_fit_timing(DEV)["refine_iterations"] == 0 and plain.stats[0]["status"] == "converged"
    with pytest.raises(plm.PlmError):
        plm.fit_symmetric(msa, w, beff, plm.FitOptions(tol=1e-6, path=5, refine=1 + 9))


def test_symmetric_start_point_is_made_consistent(plm, small):
    # an inconsistent start (random blocks everywhere, self blocks included)
    # reaches the same unique minimiser; only the blocks r < i are read
    s, h_o, J_o = small
    print("[case] symmetric fit from an inconsistent start", flush=True)
    msa, w, beff = _gpu_problem(plm, s)
    g = torch.Generator().manual_seed(5)
    h0 = (0.2 * torch.randn(10, 21, generator=g)).to(DEV)
    J0 = (0.2 * torch.randn(10, 10, 21, 21, generator=g)).to(DEV)
    res = plm.fit_symmetric(msa, w, beff, plm.FitOptions(tol=1e-6, path=4), h0=h0, J0=J0)
    assert res.stats[0]["status"] == "converged", res.stats
    J = res.J.cpu().numpy().astype(np.float64)
    _check_consistent(J)
    err = max(np.max(np.abs(J - J_o)), np.max(np.abs(res.h.cpu().numpy() - h_o)))
    assert err <= 1e-4, err
    # the caller's tensors are not modified
    assert not torch.equal(J0, res.J)


def test_symmetric_graph_and_eager_are_identical(plm, small):
    s, _, _ = small
    print("[case] symmetric graph vs eager", flush=True)
    msa, w, beff = _gpu_problem(plm, s)
    a = plm.fit_symmetric(msa, w, beff, plm.FitOptions(tol=1e-6, use_graph=True))
    b = plm.fit_symmetric(msa, w, beff, plm.FitOptions(tol=1e-6, use_graph=False, sync_every=3))
    assert torch.equal(a.J, b.J) and torch.equal(a.h, b.h)
    assert a.stats == b.stats


def test_symmetric_fit_larger_gapped(plm):
    # N = 24 with 10% forced gaps, on the path the autotuner prefers
    s = synth.make_msa("sym24", N=24, B=1500, npairs=12, seed=43, gap_p=0.1, cache=False, burnin=100,
                        thin=2)
    print("[case] symmetric fit N=24 B=1500 path=4", flush=True)
    m, w_o, beff_o = oracle.reweight(s.msa, theta=0.8)
    h_o, J_o, gn_o = sym.fit(s.msa, w_o, beff_o, 0.01, 0.01, q=21)
    msa, w, beff = _gpu_problem(plm, s)
    res = plm.fit_symmetric(msa, w, beff, plm.FitOptions(tol=1e-6, path=4))
    assert res.stats[0]["status"] == "converged", res.stats
    J = res.J.cpu().numpy().astype(np.float64)
    _check_consistent(J)
    err = max(np.max(np.abs(J - J_o)), np.max(np.abs(res.h.cpu().numpy() - h_o)))
    assert err <= 1e-4, err


@pytest.mark.timeout(400)
def test_symmetric_fit_gapped_n120_precise_refinement(plm):
    """N = 120, B = 5000 with gaps (the paper-sized single-alignment workload):
    the symmetric fit on the int8-gradient path to 1e-5, refined automatically
    on the precise path to 1e-6, converges at ||grad F|| <= 1e-6 over all
    3.1 M parameters;
    the oracle's FP64 gradient at the returned point is within 1e-9 of the
    device's norm and at most 1e-6, so by strong convexity (mu = 0.02) every
    parameter is within 5e-5 of the exact minimiser."""
    print("[case] symmetric fit potts_n120_b5000_gaps path 5 + precise refinement", flush=True)
    s = synth.workload("potts_n120_b5000_gaps")
    msa, w, beff = _gpu_problem(plm, s)
    # the int8-gradient path to 1e-5 (above its rounding floor, about 2e-6 here),
    # then the precise path to 1e-6
    res = plm.fit_symmetric(msa, w, beff, plm.FitOptions(tol=1e-5, refine_tol=1e-6, path=5, timing=True))
    tm = plm.last_fit_timing(DEV)
    st = res.stats[0]
    assert st["status"] == "converged" and st["gnorm"] <= 1e-6, st
    assert tm["refine_iterations"] >= 1
    h = res.h.cpu().numpy().astype(np.float64)
    J = res.J.cpu().numpy().astype(np.float64)
    _check_consistent(J)
    F, gn = _certificate(s, h, J, 0.01, 0.01)
    print(f"  device ||grad F|| {st['gnorm']:.3e}, oracle {gn:.3e}, iterations {st['iterations']} "
          f"(refinement {tm['refine_iterations']})", flush=True)
    assert abs(gn - st["gnorm"]) <= 1e-9, (gn, st["gnorm"])
    assert gn <= 1e-6 and gn / 0.02 <= 5e-5


def test_symmetric_split_fit_n120(plm):
    """The symmetric fit with the parameters carried as FP32 pairs (high and
    low word, plm_fit_symmetric_split), N = 120, B = 5000 with gaps: the
    int8-gradient path to 1e-5, then the precise path, which evaluates at the
    FP64 sums, to 3e-7.  The oracle's FP64 gradient at h + h_lo, J + J_lo is
    within 1e-9 of the device's norm and at most 3e-7; every low word is within
    half the FP32 spacing of its high word and the low-word blocks are
    consistent like J; the high words alone are further from stationarity (at this size only
    slightly: FP32 storage matters at N = 500, where an FP32-stored fit stalls
    near 2.9e-6 -- the full-size test)."""
    print("[case] split symmetric fit potts_n120_b5000_gaps to 3e-7", flush=True)
    s = synth.workload("potts_n120_b5000_gaps")
    msa, w, beff = _gpu_problem(plm, s)
    res = plm.fit_symmetric(msa, w, beff, plm.FitOptions(tol=1e-5, refine_tol=3e-7, path=5), split=True)
    st = res.stats[0]
    assert st["status"] == "converged" and st["gnorm"] <= 3e-7, st
    h64 = res.h.double() + res.h_lo.double()
    J64 = res.J.double() + res.J_lo.double()
    assert split_words_ok(res.h, res.h_lo) and split_words_ok(res.J, res.J_lo)
    h = h64.cpu().numpy()
    J = J64.cpu().numpy()
    _check_consistent(res.J_lo.cpu().numpy())
    _check_consistent(J)
    F, gn = _certificate(s, h, J, 0.01, 0.01)
    print(f"  device ||grad F|| {st['gnorm']:.3e}, oracle at the FP64 sums {gn:.3e}, "
          f"iterations {st['iterations']}", flush=True)
    assert abs(gn - st["gnorm"]) <= 1e-9, (gn, st["gnorm"])
    assert gn <= 3e-7
    # the high words alone: FP32 storage moves the gradient well above the pairs'
    _, gn32 = _certificate(s, res.h.cpu().numpy().astype(np.float64), res.J.cpu().numpy().astype(np.float64),
                           0.01, 0.01)
    print(f"  oracle at the high words alone {gn32:.3e}", flush=True)
    assert gn32 > gn


def test_symmetric_split_start_words_and_errors(plm, small):
    """A split fit from a split start point: the low words given on entry are
    part of the point (a start that is already the result of a split fit stays
    converged at once); both low-order arrays or neither."""
    s, _, _ = small
    msa, w, beff = _gpu_problem(plm, s)
    opts = plm.FitOptions(tol=1e-6, refine_tol=1e-8, path=5)
    a = plm.fit_symmetric(msa, w, beff, opts, split=True)
    assert a.stats[0]["status"] == "converged" and a.stats[0]["gnorm"] <= 1e-8, a.stats
    b = plm.fit_symmetric(msa, w, beff, plm.FitOptions(tol=1e-8, path=7), h0=a.h, J0=a.J, split=True,
                          h0_lo=a.h_lo, J0_lo=a.J_lo)
    assert b.stats[0]["status"] == "converged" and b.stats[0]["iterations"] == 0, b.stats
    assert torch.equal(a.h, b.h) and torch.equal(a.J, b.J)
    assert torch.equal(a.h_lo, b.h_lo) and torch.equal(a.J_lo, b.J_lo)
    with pytest.raises(ValueError):
        plm.fit_symmetric(msa, w, beff, opts, h0_lo=a.h_lo, J0_lo=a.J_lo)
    import ctypes
    from paper_1401_4832_amd import _lib as L
    from paper_1401_4832_amd.api import _ptr, context, workspace
    B, N = msa.shape
    co = opts.to_c()
    nbytes = L.lib().plm_fit_symmetric_workspace_bytes(B, N, 21, ctypes.byref(co))
    ws = workspace(nbytes, DEV)
    h = torch.zeros(N, 21, device=DEV)
    J = torch.zeros(N, N, 21, 21, device=DEV)
    hl = torch.zeros_like(h)
    stats = (L.SiteStats * 1)()
    rc = L.lib().plm_fit_symmetric_split(context(DEV), _ptr(msa), B, N, 21, _ptr(w), _ptr(beff), ctypes.byref(co),
                                         _ptr(ws), ws.numel(), _ptr(h), _ptr(J), _ptr(hl), None, stats)
    assert rc == L.PLM_E_INVALID


def test_symmetric_errors(plm, small):
    s, _, _ = small
    msa, w, beff = _gpu_problem(plm, s)
    with pytest.raises(plm.PlmError):
        plm.fit_symmetric(msa, w, beff, plm.FitOptions(single_site=True))
    with pytest.raises(plm.PlmError):
        plm.fit_symmetric(msa, w, beff, plm.FitOptions(path=17))
    bad = msa.clone()
    bad[3, 2] = 30  # a symbol >= q
    with pytest.raises(plm.PlmError):
        plm.fit_symmetric(bad, w, beff, plm.FitOptions())
