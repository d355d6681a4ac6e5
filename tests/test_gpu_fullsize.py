"""The benchmark alignment at its full size (N = 500, B = 50 000, q = 21), in
the launch configuration the benchmark times, against the FP64 oracle's
stored results (``tests/golden/make_fullsize.py``, which calls only the
oracle):

* reweighting (sec. 3.1, eq. inverse_weights; sec. 3.4 step 2): every m_b,
  w_b and B_eff bit for bit, on the planted-Potts alignment and on a
  clustered alignment of the same size whose counts are far from 1;
* one all-sites objective/gradient evaluation (sec. 3.4 step 3, eqs.
  g_regdef2, g_gradh2, g_gradJ2) at a seeded point on every evaluation path,
  compared on the eight sampled sites (``synth.sample_sites(55, 500, 8)``)
  with the oracle fed its own weights: FP32-class paths to the FP32
  tolerance, the two-piece BF16 path and the int8 fixed-point path to their
  derived bounds;
* fits: the autotuned schedule (int8 path refined on path 5), and one fit per
  evaluation path for the per-path error table -- the FP32 gather path, the
  int8 paths, the three-piece and the two-piece (hi/lo, refined on the
  three-piece path) BF16 contractions.  Every site converges; on the sampled
  sites the oracle's FP64 gradient at the returned point is at most 1e-6, so
  by strong convexity (modulus mu = 2 min(lambda_h, lambda'_J) = 0.01) the
  returned parameters are within 1e-4 of the exact minimiser, and they are
  within 1e-4 max-abs of the oracle's stored minimisers.

With PLM_REPORT_DIR set, the per-path errors are written there as a table."""
import math
import os

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.helpers import clustered_msa, fixed_point_bounds, hilo_bounds, split_words_ok

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
NAME = "potts_n500_b50000"
# the clustered alignment of the stored reweighting values
CLUSTERED = dict(seed=5005, B=50000, N=500, n_anc=1250, p_mut=0.1)
LH, LJ = 0.01, 0.01
MU = 2 * min(LH, 0.5 * LJ)
# every fit ends on an FP32-class evaluation at this tolerance, so that the FP64
# gradient is below 1e-6: at this size the FP32 evaluations' gradient norms
# near the optimum differ from the FP64 ones by up to about 3e-7 (measured)
FIT_TOL = 0.65e-6
ROWS = []  # the error table


def _golden(name):
    return np.load(os.path.join(GOLD, name), allow_pickle=False)


def _report(row):
    ROWS.append(row)
    d = os.environ.get("PLM_REPORT_DIR")
    if not d:
        return
    os.makedirs(d, exist_ok=True)
    keys = ["case", "path", "f_rel", "grad_maxabs", "gnorm_fp64_max", "coupling_bound", "J_maxabs_vs_oracle",
            "site_evals", "seconds"]
    with open(os.path.join(d, "c5_error_table.md"), "w") as fh:
        fh.write("| " + " | ".join(keys) + " |\n|" + "---|" * len(keys) + "\n")
        for r in ROWS:
            fh.write("| " + " | ".join(_fmt(r.get(k)) for k in keys) + " |\n")


def _fmt(v):
    if v is None:
        return "-"
    if isinstance(v, float):
        return f"{v:.3g}"
    return str(v)


@pytest.fixture(scope="module")
def plm():
    import paper_1401_4832_amd as plm
    return plm


@pytest.fixture(scope="module")
def full(plm):
    print(f"[case] generating {NAME}", flush=True)
    s = synth.workload(NAME)
    g = _golden(f"{NAME}_reweight.npz")
    assert str(g["digest"]) == synth.msa_digest(s.msa), "the generator no longer gives the stored alignment"
    msa = torch.from_numpy(s.msa).to(DEV)
    m, w, beff = plm.reweight(msa, theta=0.8)
    plm.sync(DEV)
    return s, msa, m, w, beff, g


@pytest.fixture(scope="module")
def sites_gold():
    g = _golden(f"{NAME}_sites.npz")
    sites = synth.sample_sites(55, 500, 8)
    assert g["sites"].tolist() == sites
    assert float(np.max(g["gnorm"])) <= 1e-8
    return sites, g


def test_reweight_full_size_every_row(plm, full):
    s, msa, m, w, beff, g = full
    print("[case] reweight N=500 B=50000 every row vs the oracle", flush=True)
    assert np.array_equal(m.cpu().numpy(), g["m"])
    assert np.array_equal(w.cpu().numpy(), g["w"])
    assert float(beff.item()) == float(g["beff"][0])


def test_reweight_clustered_full_size_every_row(plm):
    print("[case] reweight clustered N=500 B=50000 every row vs the oracle", flush=True)
    cm = clustered_msa(**CLUSTERED)
    g = _golden("clustered_n500_b50000_reweight.npz")
    assert str(g["digest"]) == synth.msa_digest(cm)
    assert int(g["m"].max()) > 10  # the counts are far from 1 here
    m, w, beff = plm.reweight(torch.from_numpy(cm).to(DEV), theta=0.8)
    plm.sync(DEV)
    assert np.array_equal(m.cpu().numpy(), g["m"])
    assert np.array_equal(w.cpu().numpy(), g["w"])
    assert float(beff.item()) == float(g["beff"][0])


@pytest.fixture(scope="module")
def random_point(full, sites_gold):
    """A seeded point (h ~ N(0, 0.3^2), J ~ N(0, 0.05^2), zero self blocks) and
    the oracle's objective and gradient there on the sampled sites, with the
    oracle's own weights."""
    s, msa, m, w, beff, g = full
    sites, _ = sites_gold
    N, q = 500, 21
    rng = np.random.default_rng(2024)
    h = (0.3 * rng.standard_normal((N, q))).astype(np.float32)
    J = (0.05 * rng.standard_normal((N, N, q, q))).astype(np.float32)
    for r in range(N):
        J[r, r] = 0.0
    beff_o = float(g["beff"][0])
    fo, gho, gJo = oracle.objgrad_slices(s.msa, g["w"], beff_o, h[sites].astype(np.float64),
                                         J[sites].astype(np.float64), sites, LH, LJ)
    return h, J, fo, gho, gJo


@pytest.mark.parametrize("path", [0, 1, 2, 3, 4, 5, 6, 7])
def test_objgrad_full_size_sampled_sites(plm, full, sites_gold, random_point, path):
    s, msa, m, w, beff, g = full
    sites, _ = sites_gold
    h, J, fo, gho, gJo = random_point
    print(f"[case] objgrad N=500 B=50000 all sites, path {path}", flush=True)
    N, q, B = 500, 21, s.msa.shape[0]
    f, gh, gJ = plm.objgrad(msa, w, beff, torch.from_numpy(h).to(DEV), torch.from_numpy(J).to(DEV), LH, LJ,
                            path=path)
    plm.sync(DEV)
    beff_o = float(g["beff"][0])
    f = f.cpu().numpy()[sites]
    gh = gh.cpu().numpy()[sites]
    gJs = np.stack([gJ[r].cpu().numpy() for r in sites])
    del gJ
    frel = float(np.max(np.abs(f - fo) / np.abs(fo)))
    fabs = float(np.max(np.abs(f - fo))) / beff_o
    gerr = max(float(np.max(np.abs(gJs - gJo))), float(np.max(np.abs(gh - gho)))) / beff_o
    print(f"  errors: f rel {frel:.2e} (abs {fabs:.2e}), grad {gerr:.2e}", flush=True)
    _report(dict(case="objgrad at a random point", path=path, f_rel=frel, grad_maxabs=gerr))
    if path == 6:
        fb, gb = fixed_point_bounds(s.msa, g["w"], beff_o, J, sites)
        assert fabs <= fb + 1e-5 * math.log(q) * 10, (fabs, fb)
        assert gerr <= gb + 2e-6, (gerr, gb)
    elif path == 1:
        fb, gb = hilo_bounds(s.msa, h, J, sites)
        assert fabs <= fb + 1e-5 * math.log(q) * 10, (fabs, fb)
        assert gerr <= gb + 2e-6, (gerr, gb)
    elif path == 7:  # the precise path: FP64-class up to the FP32 rounding of the returned gradient
        assert frel <= 1e-11, frel
        excess = max(float(np.max(np.abs(gJs - gJo) - 2.0 ** -24 * np.abs(gJo))),
                     float(np.max(np.abs(gh - gho) - 2.0 ** -24 * np.abs(gho)))) / beff_o
        assert excess <= 1e-11, excess
    else:
        assert frel <= 1e-5, frel
        assert gerr <= 2e-6, gerr
    for t, r in enumerate(sites):
        assert np.all(gJs[t][r] == 0)


def _check_fit(plm, full, sites_gold, res, label, path, seconds):
    """Every site converged; on the sampled sites the FP64 gradient certifies
    the 1e-4 bar and the parameters match the oracle's minimisers to 1e-4."""
    s, msa, m, w, beff, g = full
    sites, go = sites_gold
    bad = [k for k, st in enumerate(res.stats) if st["status"] != "converged"]
    assert not bad, [res.stats[k] for k in bad[:5]]
    h = res.h.cpu().numpy()
    J = res.J.cpu().numpy()
    beff_o = float(g["beff"][0])
    fo, gho, gJo = oracle.objgrad_slices(s.msa, g["w"], beff_o, h[sites].astype(np.float64),
                                         J[sites].astype(np.float64), sites, LH, LJ)
    gn = [math.sqrt(float(np.sum(gho[t] ** 2) + np.sum(gJo[t] ** 2))) / beff_o for t in range(len(sites))]
    jerr = max(max(float(np.max(np.abs(J[r] - go["J"][t]))), float(np.max(np.abs(h[r] - go["h"][t]))))
               for t, r in enumerate(sites))
    frel = max(abs(res.stats[r]["f"] - fo[t] / beff_o) / abs(fo[t] / beff_o) for t, r in enumerate(sites))
    for t, r in enumerate(sites):
        print(f"  site {r}: oracle gradient norm {gn[t]:.2e} (device {res.stats[r]['gnorm']:.2e})", flush=True)
    print(f"  {label}: max-abs vs oracle minimiser {jerr:.2e}, evaluations {res.evaluations}, {seconds:.1f} s",
          flush=True)
    _report(dict(case=label, path=path, f_rel=frel, gnorm_fp64_max=max(gn), coupling_bound=max(gn) / MU,
                 J_maxabs_vs_oracle=jerr, site_evals=res.evaluations, seconds=seconds))
    assert max(gn) <= 1e-6, gn
    assert max(gn) / MU <= 1e-4
    assert jerr <= 1e-4, jerr


def _timed_fit(plm, msa, w, beff, opts):
    torch.cuda.synchronize()
    import time
    t = time.perf_counter()
    res = plm.fit(msa, w, beff, opts)
    torch.cuda.synchronize()
    return res, time.perf_counter() - t


@pytest.mark.timeout(300)
def test_fit_full_size_autotuned_schedule(plm, full, sites_gold):
    s, msa, m, w, beff, g = full
    print("[case] fit N=500 B=50000 autotuned schedule", flush=True)
    ch = plm.autotune.choose([(msa, w, beff)], plm.FitOptions())
    opts = plm.FitOptions(tol=1e-6, refine_tol=FIT_TOL, path=int(ch["path"]), tile_seqs=int(ch["tile_seqs"]))
    res, dt = _timed_fit(plm, msa, w, beff, opts)
    _check_fit(plm, full, sites_gold, res, f"fit, autotuned path {ch['path']} (+ refinement)", int(ch["path"]), dt)


# (path, first-fit tolerance, refinement path or -1): the int8 path and the
# two-piece BF16 path leave gradient errors near or above 1e-6 and are refined
# by the library (on path 5 and on the three-piece path 3)
FITS = [(0, FIT_TOL, -1), (5, FIT_TOL, -1), (6, 1e-6, 5), (3, FIT_TOL, -1), (1, 2e-5, 3)]


@pytest.mark.timeout(420)
@pytest.mark.parametrize("path,tol,refine", FITS)
def test_fit_full_size_per_path(plm, full, sites_gold, path, tol, refine):
    s, msa, m, w, beff, g = full
    print(f"[case] fit N=500 B=50000 path {path} tol {tol} refinement {refine}", flush=True)
    opts = plm.FitOptions(tol=tol, refine_tol=FIT_TOL, path=path, refine=0 if refine >= 0 else -1)
    res, dt = _timed_fit(plm, msa, w, beff, opts)
    label = f"fit, path {path}" + (f" to {tol:g}, refined on path {refine}" if refine >= 0 else "")
    _check_fit(plm, full, sites_gold, res, label, path, dt)


@pytest.mark.timeout(900)
def test_symmetric_split_fit_full_size(plm, full):
    """The symmetric fit (sec. 3.2, eqs. npll_1, l2reg) at the full size with
    every parameter carried as a pair of FP32 words (plm_fit_symmetric_split):
    the int8-gradient path to five times its rounding-floor estimate, then the
    precise path, evaluating at the FP64 sums, to ||grad F|| <= 1e-6 over all
    55 M parameters.  The oracle's FP64 gradient (its own weights) at
    h + h_lo, J + J_lo agrees with the device's norm and is at most 1e-6, so
    every parameter is within ||grad F|| / mu <= 5e-5 of the exact minimiser
    (mu = 2 min(lambda_h, lambda_J) = 0.02).  The high words alone (the FP32
    arrays plm_fit_symmetric returns) are a little further from stationarity
    and meet the same bar too (measured 8.9e-7; the run is deterministic): an
    FP32-stored fit stalls near 2.9e-6 because its steps below half an FP32
    spacing vanish, not for want of a good FP32 point."""
    import oracle.symmetric as sym
    s, msa, m, w, beff, g = full
    print("[case] symmetric split fit N=500 B=50000 to 1e-6", flush=True)
    floor = plm.autotune.symmetric_floor((msa, w, beff), 21)
    res = plm.fit_symmetric(msa, w, beff, plm.FitOptions(tol=5 * floor, refine_tol=1e-6, path=5), split=True)
    st = res.stats[0]
    print(f"  device ||grad F|| {st['gnorm']:.3e} after {st['iterations']} iterations", flush=True)
    assert st["status"] == "converged" and st["gnorm"] <= 1e-6, st
    assert split_words_ok(res.h, res.h_lo) and split_words_ok(res.J, res.J_lo)
    beff_o = float(g["beff"][0])

    def certificate(h, J):
        _, gh, gJ = sym.objective(s.msa, g["w"], beff_o, h, J, LH, LJ)
        return float(np.sqrt(np.sum(gh ** 2) + np.sum(gJ ** 2)))

    gn = certificate((res.h.double() + res.h_lo.double()).cpu().numpy(),
                     (res.J.double() + res.J_lo.double()).cpu().numpy())
    print(f"  oracle ||grad F|| at the FP64 sums {gn:.3e}", flush=True)
    assert abs(gn - st["gnorm"]) <= 2e-9, (gn, st["gnorm"])
    assert gn <= 1e-6 and gn / (2 * min(LH, LJ)) <= 5e-5
    gn32 = certificate(res.h.cpu().numpy().astype(np.float64), res.J.cpu().numpy().astype(np.float64))
    print(f"  oracle ||grad F|| at the high words alone {gn32:.3e}", flush=True)
    assert gn < gn32 <= 1e-6
