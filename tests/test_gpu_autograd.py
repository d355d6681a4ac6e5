"""Autograd path: PLMObjective over (h, J) on the N=150, B=8000 workload.

The backward (library gradient with the upstream gradient applied as a per-site
multiplier inside the library) is checked against FP64 central finite
differences of the oracle's objective on 200 seeded coordinates, and against
the oracle's full gradient rows.  Tolerance on the B_eff-normalised scale:
2e-6 (the FP32 evaluation bound of the gradient parity tests) plus the
finite-difference error (step 1e-4: truncation ~1e-9, round-off ~1e-11)."""
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


def test_autograd_backward_matches_fd_and_oracle(plm):
    print("[case] autograd potts_n150_b8000", flush=True)
    s = synth.workload("potts_n150_b8000")
    N, q = s.N, 21
    msa = torch.from_numpy(s.msa).to(DEV)
    m, w, beff = plm.reweight(msa, theta=0.8)
    w_np, beff_f = w.cpu().numpy(), float(beff.item())
    rng = np.random.default_rng(33)
    h0 = (0.1 * rng.standard_normal((N, q))).astype(np.float32)
    J0 = (0.1 * rng.standard_normal((N, N, q, q))).astype(np.float32)
    for r in range(N):
        J0[r, r] = 0
    h = torch.tensor(h0, device=DEV, requires_grad=True)
    J = torch.tensor(J0, device=DEV, requires_grad=True)
    f = plm.plm_objective(h, J, msa, w, beff)
    wts = torch.tensor(rng.uniform(0.5, 1.5, size=N), dtype=torch.float64, device=DEV)
    (f * wts).sum().backward()
    gh, gJ = h.grad.cpu().numpy(), J.grad.cpu().numpy()
    wt = wts.cpu().numpy()

    # forward values against the oracle at the same FP32 point
    sites = np.arange(N, dtype=np.int32)
    fo, _, _ = oracle.objgrad_slices(s.msa, w_np, beff_f, h0.astype(np.float64), J0.astype(np.float64),
                                     sites, grad=False)
    assert np.max(np.abs(f.detach().cpu().numpy() - fo) / np.abs(fo)) <= 1e-5

    # 200 seeded coordinates, central differences of the FP64 objective
    crng = np.random.default_rng(33)
    eps = 1e-4
    coords = []
    for _ in range(200):
        r = int(crng.integers(N))
        if crng.random() < 0.1:
            coords.append((r, "h", int(crng.integers(q)), 0, 0))
        else:
            i = int(crng.integers(N - 1))
            i = i + 1 if i >= r else i
            coords.append((r, "J", i, int(crng.integers(q)), int(crng.integers(q))))
    hs = np.zeros((400, q))
    Js = np.zeros((400, N, q, q))
    rs = np.zeros(400, dtype=np.int32)
    for t, (r, kind, a, k, ss) in enumerate(coords):
        for sgn, row in ((1, 2 * t), (-1, 2 * t + 1)):
            hs[row] = h0[r]
            Js[row] = J0[r]
            if kind == "h":
                hs[row, a] += sgn * eps
            else:
                Js[row, a, k, ss] += sgn * eps
            rs[row] = r
    fp, _, _ = oracle.objgrad_slices(s.msa, w_np, beff_f, hs, Js, rs, grad=False)
    worst = 0.0
    for t, (r, kind, a, k, ss) in enumerate(coords):
        fd = wt[r] * (fp[2 * t] - fp[2 * t + 1]) / (2 * eps)
        g = gh[r, a] if kind == "h" else gJ[r, a, k, ss]
        worst = max(worst, abs(g - fd) / beff_f)
    assert worst <= 2e-6 + 1e-8, worst

    # full gradient rows of three sites against the oracle
    chk = np.array([0, 77, 149], dtype=np.int32)
    _, gho, gJo = oracle.objgrad_slices(s.msa, w_np, beff_f, h0[chk].astype(np.float64),
                                        J0[chk].astype(np.float64), chk)
    for t, r in enumerate(chk):
        assert np.max(np.abs(gJ[r] - wt[r] * gJo[t])) / beff_f <= 2e-6
        assert np.max(np.abs(gh[r] - wt[r] * gho[t])) / beff_f <= 2e-6


def test_autograd_forward_needs_no_scatter_and_grad_flows_to_sum(plm):
    rng = np.random.default_rng(4)
    B, N, q = 700, 12, 21
    msa = torch.from_numpy(rng.integers(0, q, size=(B, N), dtype=np.uint8)).to(DEV)
    m, w, beff = plm.reweight(msa, theta=0.8)
    h = torch.zeros(N, q, device=DEV, requires_grad=True)
    J = torch.zeros(N, N, q, q, device=DEV, requires_grad=True)
    f = plm.plm_objective(h, J, msa, w, beff)
    f.sum().backward()
    # at the origin the h-gradient is B_eff (1/q - f_r(s)) (sec. 3.1 frequencies)
    counts = np.zeros((N, q))
    msa_np = msa.cpu().numpy()
    for r in range(N):
        counts[r] = np.bincount(msa_np[:, r], minlength=q)
    expect = B / q - counts
    np.testing.assert_allclose(h.grad.cpu().numpy(), expect, atol=2e-3)
