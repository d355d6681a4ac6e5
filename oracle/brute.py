"""Brute-force Potts enumeration for tiny systems (TEST INFRASTRUCTURE ONLY).

For N <= 4 and q = 3 (at most 81 configurations) every quantity of the Potts
model of sec. 2 (eq. potts_model) can be computed exactly: the partition
function Z, the joint probabilities, the single-site conditionals
P(sigma_r = s | sigma_rest) that the pseudolikelihood of sec. 3 (eq. condpfinal)
is built from, and exact samples.  Used to pin the oracle, independently of it.

Model parameters here are in the symmetric form of eq. potts_model: fields
h[i, k] and one block Jsym[i, j, k, l] per pair i < j (state k at i, l at j).
"""
from __future__ import annotations

import itertools

import numpy as np


def energy(sigma, h, Jsym):
    """Exponent of eq. potts_model for one configuration."""
    N = len(sigma)
    e = 0.0
    for i in range(N):
        e += h[i, sigma[i]]
    for i in range(N):
        for j in range(i + 1, N):
            e += Jsym[i, j, sigma[i], sigma[j]]
    return e


def all_states(N, q):
    return [tuple(s) for s in itertools.product(range(q), repeat=N)]


def joint(h, Jsym):
    """(states, probabilities) by full enumeration."""
    N, q = h.shape
    states = all_states(N, q)
    e = np.array([energy(s, h, Jsym) for s in states])
    p = np.exp(e - e.max())
    return states, p / p.sum()


def conditional(sigma, r, h, Jsym):
    """P(sigma_r = s | rest of sigma) for s = 0..q-1, from ratios of joint
    probabilities (the partition function cancels)."""
    N, q = h.shape
    e = np.empty(q)
    for s in range(q):
        x = list(sigma)
        x[r] = s
        e[s] = energy(x, h, Jsym)
    p = np.exp(e - e.max())
    return p / p.sum()


def sample(h, Jsym, B, rng):
    """B exact independent samples (uint8 [B, N])."""
    states, p = joint(h, Jsym)
    idx = rng.choice(len(states), size=B, p=p)
    return np.array([states[i] for i in idx], dtype=np.uint8)


def site_params(h, Jsym, r):
    """The site-r parameters (h_r, J_r) in the per-site layout J_r[i, k, s] =
    coupling between state s of r and state k of i, built from the symmetric
    model (J_ri(s,k) = Jsym[r,i,s,k] for r < i, Jsym[i,r,k,s] for i < r)."""
    N, q = h.shape
    Jr = np.zeros((N, q, q))
    for i in range(N):
        if i == r:
            continue
        for s in range(q):
            for k in range(q):
                Jr[i, k, s] = Jsym[r, i, s, k] if r < i else Jsym[i, r, k, s]
    return h[r].copy(), Jr


def random_model(N, q, rng, h_sd=1.0, j_sd=0.5):
    h = h_sd * rng.standard_normal((N, q))
    Jsym = np.zeros((N, N, q, q))
    for i in range(N):
        for j in range(i + 1, N):
            Jsym[i, j] = j_sd * rng.standard_normal((q, q))
    return h, Jsym


def ising_gauge_couplings(Jsym):
    """Exact Ising-gauge blocks of a symmetric model (double centring)."""
    out = np.zeros_like(Jsym)
    N = Jsym.shape[0]
    for i in range(N):
        for j in range(i + 1, N):
            A = Jsym[i, j]
            out[i, j] = A - A.mean(axis=0, keepdims=True) - A.mean(axis=1, keepdims=True) + A.mean()
    return out
