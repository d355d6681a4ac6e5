"""Shared test helpers: seeded input construction, fixture loading, and the
error bounds the reduced-precision paths are held to (derived from their
arithmetic).  Nothing here computes any part of the method itself."""
from __future__ import annotations

import numpy as np

import synth


def load_reweight_golden(path):
    """(rows uint8 [B,N], [(theta, m list), ...]) from the hand-worked fixture."""
    rows, cases, theta, mode = [], [], None, "rows"
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line:
                continue
            if line.startswith("#"):
                if line.startswith("# rows"):
                    mode = "rows"
                elif line.startswith("# theta"):
                    theta = float(line.split()[2].rstrip(":"))
                    mode = "m"
                continue
            vals = [int(v) for v in line.split()]
            if mode == "rows":
                rows.append(vals)
            else:
                cases.append((theta, vals))
    return np.array(rows, dtype=np.uint8), cases


def clustered_msa(seed, B, N, n_anc, p_mut, q=21):
    """Rows are mutated copies of n_anc random ancestors (each column replaced
    by a random symbol with probability p_mut), so that pairwise identities
    straddle the 0.8 threshold and reweighting is non-trivial."""
    u = synth.uniform(seed, 901, n_anc * N + 3 * B * N + B)
    pos = 0
    anc = np.minimum((u[pos:pos + n_anc * N] * q).astype(np.int64), q - 1).reshape(n_anc, N)
    pos += n_anc * N
    pick = np.minimum((u[pos:pos + B] * n_anc).astype(np.int64), n_anc - 1)
    pos += B
    mut = u[pos:pos + B * N].reshape(B, N) < p_mut
    pos += B * N
    sym = np.minimum((u[pos:pos + B * N] * q).astype(np.int64), q - 1).reshape(B, N)
    msa = anc[pick].copy()
    msa[mut] = sym[mut]
    return msa.astype(np.uint8)


def random_params(seed, N, q, sd_h=0.1, sd_J=0.1):
    """Seeded h [N,q], J [N,N,q,q] with zero self blocks."""
    rng = np.random.default_rng(seed)
    h = sd_h * rng.standard_normal((N, q))
    J = sd_J * rng.standard_normal((N, N, q, q))
    for r in range(N):
        J[r, r] = 0.0
    return h, J


def weighted_frequencies(msa, w, q):
    """Reweighted one- and two-point frequencies of sec. 3.1 (fi [N,q],
    fij [N,N,q,q] with fij[i,j,k,l] = freq of (sigma_i=k, sigma_j=l))."""
    B, N = msa.shape
    beff = float(np.sum(w))
    oh = np.zeros((B, N, q))
    oh[np.arange(B)[:, None], np.arange(N)[None, :], msa] = 1.0
    fi = np.einsum("b,bik->ik", w, oh) / beff
    fij = np.einsum("b,bik,bjl->ijkl", w, oh, oh) / beff
    return fi, fij


def hilo_bounds(msa, h, J, sites):
    """Error bounds of the two-piece (hi/lo BF16) path, from its arithmetic.

    hi + lo represents each coupling and residual to 16 significant bits, so
    |dJ| <= 2^-16 |J| and |dR| <= 2^-16 |R| <= 2^-16 w_b.  An energy then moves
    by at most eps_E = 2^-16 max_b sum_i max_s |J_ri(s, sigma_i^b)|; the
    log-partition function by at most eps_E, each probability by a factor
    exp(+-2 eps_E).  Hence, on the B_eff-normalised scale,
    |dg| <= 2 eps_E + 2^-16 per gradient entry and |df| <= 2 eps_E.  The FP32
    accumulation bounds of the other paths are added on top."""
    u = 2.0 ** -16
    Jf = np.abs(J.astype(np.float32).astype(np.float64))
    epsE = 0.0
    for r in sites:
        # max over s of |J_ri(s, k)|, indexed by (i, k): layout [i][k][s]
        mx = Jf[r].max(axis=2)
        mx[r] = 0
        per_b = mx[np.arange(msa.shape[1])[None, :], msa.astype(np.int64)].sum(axis=1)
        epsE = max(epsE, u * float(per_b.max()))
    return 2 * epsE, 2 * epsE + u


def fixed_point_bounds(msa, w, beff, J, sites):
    """Error bounds of the int8 fixed-point path (6), from its arithmetic.

    Each site's couplings are scaled by 2^k_r with max|J_r| 2^k_r in
    [2^21, 2^22) and rounded, so |dJ| <= 2^-22 max_{i != r} |J_r|; an energy
    moves by at most eps_E = (N - 1) 2^-22 max|J_r|, log Z by at most eps_E and
    each probability by a factor exp(+-2 eps_E): |df| <= 2 eps_E per weighted
    sequence.  The residuals are rounded to 2^-23 absolute (|R| <= w_b <= 1) and
    accumulated exactly, so a normalised gradient entry moves by at most
    2 eps_E + 2^-23 B / B_eff.  FP32 rounding of the softmax comes on top."""
    N = msa.shape[1]
    eps = 0.0
    for r in sites:
        Jr = np.abs(J[r].astype(np.float32).astype(np.float64))
        Jr[r] = 0
        eps = max(eps, (N - 1) * 2.0 ** -22 * float(Jr.max()))
    return 2 * eps, 2 * eps + 2.0 ** -23 * msa.shape[0] / beff


def split_words_ok(hi, lo):
    """The low word of an FP32 pair is within half the FP32 spacing above the
    high word's magnitude (hi = fl32(v), lo = fl32(v - hi))."""
    import torch
    a = hi.abs()
    spacing = torch.nextafter(a, torch.full_like(a, float("inf"))) - a
    return bool(torch.all(lo.abs() <= 0.5 * spacing))
