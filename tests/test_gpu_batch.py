"""Ragged batches of alignments (plm_fit_batch): one set of launches per
iteration for all sites of all alignments.

Each alignment's result must be bit-identical to plm_fit on that alignment
alone (same kernels and per-item arithmetic; the forward tile size is fixed
so that both use the same tiles), and sampled sites must meet the fit bar of
the single-alignment tests against the FP64 oracle (couplings within 1e-4,
strong-convexity certificate)."""
import os

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


@pytest.fixture(scope="module")
def ragged():
    # 5 alignments, N in [10, 60], B in [200, 2500]: several tiles, ragged tails
    return synth.ragged_set(count=5, seed=11, n_range=(10, 60), b_range=(200, 2500), burnin=200,
                            thin=2, cache=False)


def _prep(plm, s):
    msa = torch.from_numpy(s.msa).to(DEV)
    m, w, beff = plm.reweight(msa, theta=0.8)
    return msa, w, beff


@pytest.mark.parametrize("path", [0, 2, 3, 4, 5, 6])
def test_batch_equals_single_alignment_fits(plm, ragged, path):
    print(f"[case] batch vs single fits path={path} sizes={[s.msa.shape for s in ragged]}", flush=True)
    items = [_prep(plm, s) for s in ragged]
    opts = plm.FitOptions(tol=1e-6, path=path, tile_seqs=16)
    res = plm.fit_batch(items, opts)
    assert len(res) == len(items)
    for k, ((msa, w, beff), r) in enumerate(zip(items, res)):
        one = plm.fit(msa, w, beff, opts)
        assert torch.equal(one.h, r.h) and torch.equal(one.J, r.J), k
        assert [x["evaluations"] for x in one.stats] == [x["evaluations"] for x in r.stats], k
        assert all(x["status"] == "converged" for x in r.stats), k


def test_batch_sampled_sites_match_oracle(plm, ragged):
    print("[case] batch vs oracle on sampled sites", flush=True)
    items = [_prep(plm, s) for s in ragged]
    opts = plm.FitOptions(tol=0.9e-6, path=2)
    res = plm.fit_batch(items, opts)
    mu = 2 * min(opts.lambda_h, 0.5 * opts.lambda_J)
    for k in (0, 3):
        s = ragged[k]
        N = s.msa.shape[1]
        sites = [0, N // 2, N - 1]
        m_o, w_o, beff_o = oracle.reweight(s.msa, theta=0.8)
        h_o, J_o, _ = oracle.fit(s.msa, w_o, beff_o, opts.lambda_h, opts.lambda_J, sites=sites, tol=1e-8)
        h = res[k].h.cpu().numpy().astype(np.float64)
        J = res[k].J.cpu().numpy().astype(np.float64)
        for t, r in enumerate(sites):
            err = max(np.max(np.abs(J[r] - J_o[t])), np.max(np.abs(h[r] - h_o[t])))
            assert err <= 1e-4, (k, r, err)
            f, gh, gJ = oracle.site_objgrad(s.msa, r, w_o, beff_o, h[r], J[r], opts.lambda_h, opts.lambda_J)
            gn = np.sqrt(np.sum(gh ** 2) + np.sum(gJ ** 2)) / beff_o
            assert gn / mu <= 1e-4, (k, r, gn)


def test_batch_of_one_and_errors(plm, ragged):
    msa, w, beff = _prep(plm, ragged[1])
    opts = plm.FitOptions(tol=1e-6, tile_seqs=16)
    a = plm.fit(msa, w, beff, opts)
    (b,) = plm.fit_batch([(msa, w, beff)], opts)
    assert torch.equal(a.J, b.J) and torch.equal(a.h, b.h)
    with pytest.raises(plm.PlmError):
        plm.fit_batch([(msa, w, beff)], plm.FitOptions(single_site=True))
    with pytest.raises(ValueError):
        plm.fit_batch([], opts)


def test_tuner_times_every_candidate_and_autotuned_fit_converges(plm, ragged, tmp_path, monkeypatch):
    print("[case] autotune on the ragged batch", flush=True)
    monkeypatch.setenv("PLM_TUNE_CACHE", str(tmp_path / "tune.json"))
    items = [_prep(plm, s) for s in ragged]
    res = plm.tune(items, plm.FitOptions(), fp32_only=True)
    # paths 5, 4, 2 and 0 with three forward tiles each, paths 6 and 3 with their MFMA forwards
    assert len(res) == 14
    assert sorted((r["path"], r["tile_seqs"]) for r in res) == sorted(
        [(5, 16), (5, 32), (5, 64), (4, 16), (4, 32), (4, 64), (2, 16), (2, 32), (2, 64), (0, 16), (0, 32),
         (0, 64), (3, 0), (6, 0)])
    assert all(r["eval_ms"] > 0 for r in res)
    assert [r["eval_ms"] for r in res] == sorted(r["eval_ms"] for r in res)
    out = plm.fit_batch(items, plm.FitOptions(tol=1e-6, autotune=True))
    assert all(x["status"] == "converged" for r in out for x in r.stats)
    ch = plm.autotune.choose(items)  # now cached
    assert (ch["path"], ch["tile_seqs"]) in [(r["path"], r["tile_seqs"]) for r in res]


@pytest.mark.timeout(420)
def test_ragged16_configured_sizes(plm):
    """The 16-alignment ragged batch at its configured sizes (N in [60, 300],
    B in [2000, 30000], seeds 400 + k) on the autotuned schedule, as the
    benchmark runs it: every alignment's weights bit for bit against the
    oracle's stored ones; every site converges; on two sampled sites per
    alignment the oracle's FP64 gradient at the returned point is at most
    1e-6 (so, by strong convexity, within 1e-4 of the minimiser); and the
    main fit of the batch equals each alignment's own fit, bit for bit, for
    the smallest, the middle and the largest alignment."""
    print("[case] ragged16 at configured sizes", flush=True)
    sets = synth.ragged_set(16)
    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ragged16_reweight.npz"),
                allow_pickle=False)
    assert [str(x) for x in g["digest"]] == [synth.msa_digest(a.msa) for a in sets]
    items, gold = [], []
    off = 0
    for k, a in enumerate(sets):
        msa = torch.from_numpy(a.msa).to(DEV)
        m, w, beff = plm.reweight(msa, theta=0.8)
        plm.sync(DEV)
        m_o, w_o = g["m"][off:off + a.B], g["w"][off:off + a.B]
        off += a.B
        assert np.array_equal(m.cpu().numpy(), m_o), k
        assert np.array_equal(w.cpu().numpy(), w_o), k
        assert float(beff.item()) == float(g["beff"][k]), k
        items.append((msa, w, beff))
        gold.append((w_o, float(g["beff"][k])))
    ch = plm.autotune.choose(items, plm.FitOptions())
    print(f"  schedule: path {ch['path']} tile {ch['tile_seqs']}", flush=True)
    opts = plm.FitOptions(tol=1e-6, refine_tol=0.9e-6, path=int(ch["path"]), tile_seqs=int(ch["tile_seqs"]))
    res = plm.fit_batch(items, opts)
    mu = 2 * min(opts.lambda_h, 0.5 * opts.lambda_J)
    worst = 0.0
    for k, (a, r) in enumerate(zip(sets, res)):
        assert all(x["status"] == "converged" for x in r.stats), k
        sites = synth.sample_sites(400 + k, a.N, 2)
        h = r.h.cpu().numpy().astype(np.float64)
        J = r.J.cpu().numpy().astype(np.float64)
        w_o, beff_o = gold[k]
        _, gh, gJ = oracle.objgrad_slices(a.msa, w_o, beff_o, h[sites], J[sites], sites)
        for t, site in enumerate(sites):
            gn = np.sqrt(np.sum(gh[t] ** 2) + np.sum(gJ[t] ** 2)) / beff_o
            worst = max(worst, gn)
            assert gn <= 1e-6 and gn / mu <= 1e-4, (k, site, gn)
    print(f"  largest FP64 gradient norm on the sampled sites {worst:.2e}", flush=True)
    # batch = single alignment, main fit (its forward tile does not depend on the batch)
    o1 = plm.FitOptions(tol=1e-6, path=int(ch["path"]), tile_seqs=int(ch["tile_seqs"]), refine=-1)
    one_batch = plm.fit_batch(items, o1)
    cost = [a.B * a.N * a.N for a in sets]
    order = np.argsort(cost)
    for k in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        msa, w, beff = items[k]
        one = plm.fit(msa, w, beff, o1)
        assert torch.equal(one.h, one_batch[k].h) and torch.equal(one.J, one_batch[k].J), k
        assert [x["evaluations"] for x in one.stats] == [x["evaluations"] for x in one_batch[k].stats], k
