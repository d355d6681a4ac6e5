"""GPU score variants (sec. 7) and contact TPR (sec. 6) against the FP64 oracle.

FP64 on identical FP32 couplings: relative agreement 1e-9 (exp/log/pow
differ from numpy's by a few ulp).  The TPR uses the GPU's own scores on
both sides and the same tie rule, so it must agree exactly."""
import numpy as np
import pytest
import torch

import synth
from oracle import score_variants as sv

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def plm():
    import paper_1401_4832_amd as plm
    return plm


def _J(seed, N, q, scale=0.5):
    rng = np.random.default_rng(seed)
    J = (scale * rng.standard_normal((N, N, q, q))).astype(np.float32)
    for r in range(N):
        J[r, r] = 0
    return J


CASES = [("avg", "frob", 2.0, False, "none"), ("min", "frob", 2.0, False, "apc"),
         ("max", "lp", 1.5, False, "asc"), ("avg", "lp", 1.0, True, "apc"),
         ("avg", "burkoff", 2.0, False, "apc"), ("max", "burkoff", 2.0, True, "asc"),
         ("min", "lp", 3.0, True, "none"), ("avg", "frob", 2.0, True, "asc")]


@pytest.mark.parametrize("combine,norm,p,gap,corr", CASES)
@pytest.mark.parametrize("N,q", [(23, 21), (9, 5)])
def test_score_variants_match_oracle(plm, combine, norm, p, gap, corr, N, q):
    print(f"[case] score {combine} {norm} p={p} gap={gap} {corr} N={N} q={q}", flush=True)
    J = _J(N * 100 + q, N, q)
    rng = np.random.default_rng(N + q)
    msa = rng.integers(0, q, size=(400, N), dtype=np.uint8)
    w = rng.uniform(0.2, 1.0, size=400)
    beff = float(w.sum())
    f_o = sv.frequencies(msa, w, beff, q)
    f = plm.frequencies(torch.from_numpy(msa).to(DEV), torch.from_numpy(w).to(DEV),
                        torch.tensor([beff], dtype=torch.float64, device=DEV), q)
    np.testing.assert_allclose(f.cpu().numpy(), f_o, rtol=1e-12, atol=1e-15)
    raw, cor = plm.score(torch.from_numpy(J).to(DEV), combine=combine, norm=norm, p=p, exclude_gap=gap,
                         correction=corr, freq=f if norm == "burkoff" else None)
    raw_o = sv.raw_scores(J.astype(np.float64), combine, norm, p, gap, f_o)
    cor_o = sv.correct(raw_o, corr)
    np.testing.assert_allclose(raw.cpu().numpy(), raw_o, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(cor.cpu().numpy(), cor_o, rtol=1e-9, atol=1e-11)


def test_planted_contacts_tpr(plm):
    print("[case] planted-contact TPR potts_n120_b5000_gaps", flush=True)
    s = synth.workload("potts_n120_b5000_gaps")
    msa = torch.from_numpy(s.msa).to(DEV)
    m, w, beff = plm.reweight(msa, theta=0.8)
    res = plm.fit(msa, w, beff, plm.FitOptions(tol=1e-6, path=2))
    raw, cfn = plm.score(res.J)
    N = s.N
    C = np.zeros((N, N), dtype=np.uint8)
    for i, j in s.pairs:
        C[i, j] = C[j, i] = 1
    t = plm.contact_tpr(cfn, torch.from_numpy(C), min_sep=5, kmax=len(s.pairs))
    t_o = sv.tpr_curve(cfn.cpu().numpy(), C.astype(bool), min_sep=5, kmax=len(s.pairs))
    np.testing.assert_array_equal(t, t_o)
    # the planted pairs are recovered: the strongest predictions are planted contacts
    print("  TPR at 1, 10, P/4, P/2, P:", t[0], t[9], t[len(t) // 4 - 1], t[len(t) // 2 - 1], t[-1])
    assert t[9] >= 0.8 and t[len(t) // 2 - 1] >= 0.9, t[:20]
