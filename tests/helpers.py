"""Shared test helpers: seeded input construction and fixture loading.

Nothing here computes any part of the method; inputs only."""
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
