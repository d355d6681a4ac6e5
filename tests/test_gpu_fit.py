"""GPU fit parity: every site's minimiser against the FP64 oracle's.

Each per-site objective is strongly convex with modulus mu = 2 min(lambda_h,
lambda'_J) (= 0.01 at the default strengths), so ||theta - theta*|| <=
||grad g_r^reg(theta)|| / mu.  The GPU stops at ||grad|| <= 0.9e-6 on an
FP32-class evaluation (which differs from FP64 by a few 1e-8) and the oracle
at 1e-8, so every coupling must agree to 1e-4; the certificate is re-checked
with the oracle's FP64 gradient at the GPU's final point (at most 1e-6, i.e.
a distance of at most 1e-4)."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def plm():
    import paper_1401_4832_amd as plm
    return plm


def _fit_case(plm, s, uniform, opts, sites_check):
    msa = torch.from_numpy(s.msa).to(DEV)
    m, w, beff = plm.reweight(msa, theta=0.8, uniform=uniform)
    res = plm.fit(msa, w, beff, opts)
    m_o, w_o, beff_o = oracle.reweight(s.msa, theta=0.8, uniform=uniform)
    h_o, J_o, st_o = oracle.fit(s.msa, w_o, beff_o, opts.lambda_h, opts.lambda_J, sites=sites_check,
                                tol=1e-8)
    h = res.h.cpu().numpy().astype(np.float64)
    J = res.J.cpu().numpy().astype(np.float64)
    err = 0.0
    cert = 0.0
    mu = 2 * min(opts.lambda_h, 0.5 * opts.lambda_J)
    for t, r in enumerate(sites_check):
        err = max(err, np.max(np.abs(J[r] - J_o[t])), np.max(np.abs(h[r] - h_o[t])))
        f, gh, gJ = oracle.site_objgrad(s.msa, r, w_o, beff_o, h[r], J[r], opts.lambda_h, opts.lambda_J)
        gn = np.sqrt(np.sum(gh ** 2) + np.sum(gJ ** 2)) / beff_o
        cert = max(cert, gn / mu)
    return res, err, cert, (h_o, J_o)


def _certificates(s, w_o, beff_o, h, J, sites, opts):
    """Per-site distance bounds ||theta_r - theta_r*||_2 <= ||grad g_r^reg||_2 / mu
    from the oracle's FP64 gradient at the given point (h, J: the sites' slices)."""
    mu = 2 * min(opts.lambda_h, 0.5 * opts.lambda_J)
    out = {}
    for t, r in enumerate(sites):
        _, gh, gJ = oracle.site_objgrad(s.msa, r, w_o, beff_o, h[t], J[t], opts.lambda_h, opts.lambda_J)
        out[r] = np.sqrt(np.sum(gh ** 2) + np.sum(gJ ** 2)) / beff_o / mu
    return out


def _score_bounds(fn_o, eps):
    """Bounds on |FN_gpu - FN_oracle| and |CFN_gpu - CFN_oracle| per pair when
    every site's parameter vector differs by at most eps[r] (Euclidean) between
    the two fits.  The Ising gauge (eq. gauge_change2) is an orthogonal
    projection and the transpose keeps the Frobenius norm, so the averaged
    block (eq. average2) moves by at most (eps_i + eps_j) / 2 in Frobenius norm
    and FN_ij (eq. frob_normtrans2) by at most that.  The APC term (eq.
    corr_norm2) FN_i: FN_:j / FN_:: is bounded over the box of its three means
    moved by the averaged FN bounds."""
    e = 0.5 * (eps[:, None] + eps[None, :])
    np.fill_diagonal(e, 0.0)
    a = fn_o.mean(axis=1)
    c = fn_o.mean()
    A = e.mean(axis=1)
    C = e.mean()
    assert np.all(a > A) and c > C
    ab = np.outer(a, a) / c
    hi = np.outer(a + A, a + A) / (c - C) - ab
    lo = ab - np.outer(a - A, a - A) / (c + C)
    s = e + np.maximum(hi, lo)
    np.fill_diagonal(s, 0.0)
    return e, s


def test_fit_small_all_sites(plm):
    """All 40 sites against the oracle's fit, and the whole pipeline: the GPU's
    scores of its own fit against the oracle's scores of the oracle's fit
    (sec. 3.4 steps 4-6), to the bound the two fits' certificates give."""
    print("[case] fit potts_n40_b500 all sites", flush=True)
    s = synth.workload("potts_n40_b500")
    opts = plm.FitOptions(tol=0.9e-6)
    sites = list(range(40))
    res, err, cert, (h_o, J_o) = _fit_case(plm, s, True, opts, sites)
    bad = [k for k, st in enumerate(res.stats) if st["status"] != "converged"]
    assert not bad, [res.stats[k] for k in bad]
    assert err <= 1e-4, err
    assert cert <= 1e-4, cert  # distance bound from the FP64 gradient at the GPU point
    fn, cfn = plm.score(res.J)
    fn, cfn = fn.cpu().numpy(), cfn.cpu().numpy()
    # the scorer on identical couplings
    fn_same, cfn_same = oracle.score(res.J.cpu().numpy())
    np.testing.assert_allclose(cfn, cfn_same, rtol=1e-9, atol=1e-12)
    # the pipelines: GPU fit -> GPU score against oracle fit -> oracle score
    m_o, w_o, beff_o = oracle.reweight(s.msa, theta=0.8, uniform=True)
    h = res.h.cpu().numpy().astype(np.float64)
    J = res.J.cpu().numpy().astype(np.float64)
    cg = _certificates(s, w_o, beff_o, h, J, sites, opts)
    co = _certificates(s, w_o, beff_o, h_o, J_o, sites, opts)
    eps = np.array([cg[r] + co[r] for r in sites])
    fn_o, cfn_o = oracle.score(J_o)
    efn, ecfn = _score_bounds(fn_o, eps)
    print(f"  FN max diff {np.max(np.abs(fn - fn_o)):.2e} (bound {efn.max():.2e}), "
          f"CFN max diff {np.max(np.abs(cfn - cfn_o)):.2e} (bound {ecfn.max():.2e})", flush=True)
    assert np.all(np.abs(fn - fn_o) <= efn + 1e-12)
    assert np.all(np.abs(cfn - cfn_o) <= ecfn + 1e-12)
    # the strongest predicted contacts agree up to pairs the bound cannot order
    iu = np.triu_indices(40, 1)
    k = 80
    top_g = set(np.argsort(-cfn[iu], kind="stable")[:k].tolist())
    top_o = np.argsort(-cfn_o[iu], kind="stable")
    kth = cfn_o[iu][top_o[k - 1]]
    for p in top_g - set(top_o[:k].tolist()):
        assert cfn_o[iu][p] >= kth - 2 * ecfn[iu][p] - 1e-12, p


def test_fit_gapped_sampled_pairs_score(plm):
    """N = 120 with gaps: FN of pairs of sampled sites from the GPU pipeline
    against FN from the oracle's fits of those sites, each pair through both
    of its estimates (the APC needs every site and is covered at N = 40)."""
    print("[case] fit potts_n120_b5000_gaps sampled pairs FN", flush=True)
    s = synth.workload("potts_n120_b5000_gaps")
    opts = plm.FitOptions(tol=1e-6, refine_tol=0.9e-6, path=6)
    sites = [3, 9, 40, 41, 77, 118]
    res, err, cert, (h_o, J_o) = _fit_case(plm, s, False, opts, sites)
    assert err <= 1e-4 and cert <= 1e-4, (err, cert)
    m_o, w_o, beff_o = oracle.reweight(s.msa, theta=0.8)
    h = res.h.cpu().numpy().astype(np.float64)
    J = res.J.cpu().numpy().astype(np.float64)
    cg = _certificates(s, w_o, beff_o, h[sites], J[sites], sites, opts)
    co = _certificates(s, w_o, beff_o, h_o, J_o, sites, opts)
    fn, _ = plm.score(res.J)
    fn = fn.cpu().numpy()
    Jfull = np.zeros_like(J)
    for t, r in enumerate(sites):
        Jfull[r] = J_o[t]
    fn_o, _ = oracle.score(Jfull)  # FN_ij uses only the rows of i and j
    worst = 0.0
    for a in range(len(sites)):
        for b in range(a + 1, len(sites)):
            i, j = sites[a], sites[b]
            bound = 0.5 * (cg[i] + co[i] + cg[j] + co[j])
            d = abs(fn[i, j] - fn_o[i, j])
            worst = max(worst, d / bound)
            assert d <= bound + 1e-12, (i, j, d, bound)
    print(f"  FN differences at most {worst:.2f} of their bounds", flush=True)


@pytest.mark.parametrize("path", [0, 1, 2, 3, 4, 5, 6, 7])
def test_fit_gapped_sampled_sites(plm, path):
    """Every evaluation path reaches the oracle's minimiser: each fit ends on
    an FP32-class evaluation at 0.9e-6, so the FP64 gradient at the returned
    point certifies 1e-4.  The two-piece BF16 path (1) stops at 2e-5 (its
    16-bit operands leave a gradient error of that order) and the library
    refines it on the three-piece path (3); the int8 path (6) is refined on
    path 5."""
    print(f"[case] fit potts_n120_b5000_gaps sampled sites path={path}", flush=True)
    s = synth.workload("potts_n120_b5000_gaps")
    opts = plm.FitOptions(tol=2e-5 if path == 1 else (1e-6 if path == 6 else 0.9e-6), refine_tol=0.9e-6,
                          path=path)
    sites = [0, 1, 37, 60, 88, 119]
    res, err, cert, _ = _fit_case(plm, s, False, opts, sites)
    assert all(st["status"] == "converged" for st in res.stats), res.stats[:3]
    assert max(st["gnorm"] for st in res.stats) <= 0.9e-6
    assert err <= 1e-4, err
    assert cert <= 1e-4, cert
    if path == 7:
        # the precise path's gradient norm is the FP64 one
        m_o, w_o, beff_o = oracle.reweight(s.msa, theta=0.8)
        h = res.h.cpu().numpy().astype(np.float64)
        J = res.J.cpu().numpy().astype(np.float64)
        for r in sites:
            _, gh, gJ = oracle.site_objgrad(s.msa, r, w_o, beff_o, h[r], J[r], opts.lambda_h, opts.lambda_J)
            gn = np.sqrt(np.sum(gh ** 2) + np.sum(gJ ** 2)) / beff_o
            assert abs(gn - res.stats[r]["gnorm"]) <= 1e-10, (r, gn, res.stats[r]["gnorm"])


@pytest.mark.parametrize("lbfgs_m", [3, 10, 20])
def test_fit_history_fp64_matches_fp32_history(plm, lbfgs_m):
    """Curvature pairs and gradient copy stored in FP64 (history_fp64) against
    the default FP32 storage: both fits converge, their couplings agree within
    1e-4, and the FP64-history fit meets the oracle's bar on sampled sites."""
    print(f"[case] fit potts_n120_b5000_gaps FP64 history m={lbfgs_m}", flush=True)
    s = synth.workload("potts_n120_b5000_gaps")
    msa = torch.from_numpy(s.msa).to(DEV)
    m, w, beff = plm.reweight(msa, theta=0.8)
    a = plm.fit(msa, w, beff, plm.FitOptions(tol=0.9e-6, path=2, lbfgs_m=lbfgs_m))
    opts = plm.FitOptions(tol=0.9e-6, path=2, lbfgs_m=lbfgs_m, history_fp64=True)
    b = plm.fit(msa, w, beff, opts)
    assert all(st["status"] == "converged" for st in a.stats + b.stats)
    d = max(float((a.J - b.J).abs().max()), float((a.h - b.h).abs().max()))
    print(f"  FP32 vs FP64 history: max-abs difference {d:.2e}; evaluations {a.evaluations} vs "
          f"{b.evaluations}", flush=True)
    assert d <= 1e-4
    m_o, w_o, beff_o = oracle.reweight(s.msa, theta=0.8)
    sites = [0, 60, 119]
    h = b.h.cpu().numpy().astype(np.float64)
    J = b.J.cpu().numpy().astype(np.float64)
    cert = _certificates(s, w_o, beff_o, h[sites], J[sites], sites, opts)
    assert max(cert.values()) <= 1e-4, cert


def test_graph_and_eager_are_identical(plm):
    print("[case] graph vs eager", flush=True)
    s = synth.make_msa("ge", N=18, B=900, npairs=12, seed=31, cache=False, burnin=100, thin=2)
    msa = torch.from_numpy(s.msa).to(DEV)
    m, w, beff = plm.reweight(msa, theta=0.8)
    a = plm.fit(msa, w, beff, plm.FitOptions(tol=1e-6, use_graph=True))
    b = plm.fit(msa, w, beff, plm.FitOptions(tol=1e-6, use_graph=False, sync_every=3))
    assert torch.equal(a.J, b.J) and torch.equal(a.h, b.h)
    assert [x["evaluations"] for x in a.stats] == [x["evaluations"] for x in b.stats]


def test_single_site_plain_path_matches_batched(plm):
    print("[case] single-site plain path", flush=True)
    s = synth.make_msa("ss", N=12, B=600, npairs=8, seed=32, cache=False, burnin=100, thin=2)
    msa = torch.from_numpy(s.msa).to(DEV)
    m, w, beff = plm.reweight(msa, theta=0.8)
    a = plm.fit(msa, w, beff, plm.FitOptions(tol=1e-6))
    b = plm.fit(msa, w, beff, plm.FitOptions(tol=1e-6, single_site=True))
    # the same kernels and per-site decisions: identical trajectories
    assert torch.equal(a.J, b.J) and torch.equal(a.h, b.h)


def test_maxiter_status(plm):
    s = synth.make_msa("mi", N=10, B=300, npairs=5, seed=33, cache=False, burnin=50, thin=2)
    msa = torch.from_numpy(s.msa).to(DEV)
    m, w, beff = plm.reweight(msa, theta=0.8)
    res = plm.fit(msa, w, beff, plm.FitOptions(tol=1e-12, max_iter=3))
    assert res.status == 1
    assert all(st["status"] == "maxiter" and st["iterations"] == 3 for st in res.stats)


def test_refinement_fit_continues_the_first_one(plm):
    """refine = 0 (automatic) after path 6 runs a second fit on path 5 from the
    first fit's point: the first fit is the refine = -1 fit bit for bit, the
    statistics and the timing add both, and the result meets the tolerance on
    the refinement path's evaluation and within 1e-4 of the oracle's minimiser."""
    print("[case] refinement fit after path 6", flush=True)
    s = synth.workload("potts_n120_b5000_gaps")
    msa = torch.from_numpy(s.msa).to(DEV)
    m, w, beff = plm.reweight(msa, theta=0.8)
    base = plm.fit(msa, w, beff, plm.FitOptions(tol=1e-6, path=6, refine=-1, timing=True))
    tb = plm.last_fit_timing(DEV)
    assert tb["refine_site_evals"] == 0 and tb["refine_iterations"] == 0
    ref = plm.fit(msa, w, beff, plm.FitOptions(tol=1e-6, path=6, timing=True))
    tr = plm.last_fit_timing(DEV)
    ev_b = sum(x["evaluations"] for x in base.stats)
    ev_r = sum(x["evaluations"] for x in ref.stats)
    assert tr["refine_site_evals"] == ev_r - ev_b > 0
    assert tr["site_evals"] == tb["site_evals"] + tr["refine_site_evals"]
    assert tr["iterations"] == tb["iterations"] + tr["refine_iterations"]
    assert all(a["iterations"] <= b["iterations"] for a, b in zip(base.stats, ref.stats))
    assert all(st["status"] == "converged" for st in ref.stats)
    # the refined point, evaluated on the refinement path, meets the tolerance
    _, gh, gJ = plm.objgrad(msa, w, beff, ref.h, ref.J, 0.01, 0.01, path=5)
    beff_h = float(beff.item())
    gn = torch.sqrt(gh.double().pow(2).sum(1) + gJ.double().pow(2).sum((1, 2, 3))) / beff_h
    assert float(gn.max()) <= 1.05e-6, float(gn.max())
    # and against the oracle's minimiser
    sites = [0, 60, 119]
    m_o, w_o, beff_o = oracle.reweight(s.msa, theta=0.8)
    h_o, J_o, _ = oracle.fit(s.msa, w_o, beff_o, 0.01, 0.01, sites=sites, tol=1e-8)
    J = ref.J.cpu().numpy().astype(np.float64)
    for t, r in enumerate(sites):
        assert np.max(np.abs(J[r] - J_o[t])) <= 1e-4
    # an explicit refinement path, and an unknown one rejected
    exp = plm.fit(msa, w, beff, plm.FitOptions(tol=1e-6, path=6, refine=1 + 2))
    assert all(st["status"] == "converged" for st in exp.stats)
    with pytest.raises(plm.PlmError):
        plm.fit(msa, w, beff, plm.FitOptions(tol=1e-6, path=6, refine=1 + 9))


@pytest.fixture(scope="module")
def small_oracle():
    s = synth.workload("potts_n40_b500")
    sites = [0, 13, 39]
    m_o, w_o, beff_o = oracle.reweight(s.msa, theta=0.8, uniform=True)
    h_o, J_o, _ = oracle.fit(s.msa, w_o, beff_o, 0.01, 0.01, sites=sites, tol=1e-8)
    return s, sites, h_o, J_o


@pytest.mark.parametrize("lbfgs_m", [1, 3, 4, 5, 11, 20, 32])
def test_fit_history_sizes(plm, small_oracle, lbfgs_m):
    """Every history size reaches the same minimiser: the dot-product passes
    read 1..4 pairs on the acceptance pass and up to six per further pass, so
    m = 1 .. 32 covers every pair count of both (and m = 32, the largest,
    five further passes)."""
    print(f"[case] fit potts_n40_b500 lbfgs_m={lbfgs_m}", flush=True)
    s, sites, h_o, J_o = small_oracle
    msa = torch.from_numpy(s.msa).to(DEV)
    m, w, beff = plm.reweight(msa, theta=0.8, uniform=True)
    res = plm.fit(msa, w, beff, plm.FitOptions(tol=1e-6, lbfgs_m=lbfgs_m))
    assert all(st["status"] == "converged" for st in res.stats), res.stats[:3]
    J = res.J.cpu().numpy().astype(np.float64)
    h = res.h.cpu().numpy().astype(np.float64)
    for t, r in enumerate(sites):
        assert np.max(np.abs(J[r] - J_o[t])) <= 1e-4
        assert np.max(np.abs(h[r] - h_o[t])) <= 1e-4


@pytest.mark.parametrize("q,path", [(5, 2), (5, 6), (11, 4)])
def test_fit_small_alphabet(plm, q, path):
    """Alphabets below 21 states (the alphabet size is taken from the start
    point): every site converges to the oracle's minimiser."""
    print(f"[case] fit q={q} path={path}", flush=True)
    N, B = 15, 800
    s = synth.make_msa(f"fq{q}", N=N, B=B, npairs=6, seed=70 + q, min_sep=1, q=q, cache=False,
                       burnin=100, thin=2)
    msa = torch.from_numpy(s.msa).to(DEV)
    m, w, beff = plm.reweight(msa, theta=0.8, q=q)
    h0 = torch.zeros(N, q, dtype=torch.float32, device=DEV)
    J0 = torch.zeros(N, N, q, q, dtype=torch.float32, device=DEV)
    res = plm.fit(msa, w, beff, plm.FitOptions(tol=1e-6, path=path), h0=h0, J0=J0)
    assert all(st["status"] == "converged" for st in res.stats), res.stats[:3]
    sites = [0, 7, 14]
    m_o, w_o, beff_o = oracle.reweight(s.msa, theta=0.8)
    h_o, J_o, _ = oracle.fit(s.msa, w_o, beff_o, 0.01, 0.01, sites=sites, q=q, tol=1e-8)
    J = res.J.cpu().numpy().astype(np.float64)
    h = res.h.cpu().numpy().astype(np.float64)
    for t, r in enumerate(sites):
        assert np.max(np.abs(J[r] - J_o[t])) <= 1e-4, (r, np.max(np.abs(J[r] - J_o[t])))
        assert np.max(np.abs(h[r] - h_o[t])) <= 1e-4
        assert np.all(J[r, r] == 0)
