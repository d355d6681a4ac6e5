"""Writes the stored expected values of the full-size tests (N = 500, B = 50 000).

Every value here comes from the FP64 CPU oracle (``oracle/``) run on seeded
synthetic inputs (``synth``, ``tests.helpers``); nothing is taken from the GPU
library.  Run from the repository root:

    python tests/golden/make_fullsize.py [--threads T] [--only ragged]

Files (numpy .npz, loaded with allow_pickle=False):

* ``potts_n500_b50000_reweight.npz`` -- m_b for every row of the planted-Potts
  alignment at theta = 0.8 (sec. 3.1, eq. inverse_weights), w_b = 1/m_b and
  B_eff (sec. 3.4 step 2), with the alignment's digest.
* ``clustered_n500_b50000_reweight.npz`` -- the same for a clustered alignment
  of the same size (mutated copies of 1250 ancestors, mutation rate 0.1, so
  that pair identities straddle the 0.8 threshold and m_b is far from 1).
* ``ragged16_reweight.npz`` -- m_b and w_b of every row of each of the 16
  alignments of ``synth.ragged_set(16)`` (N in [60, 300], B in [2000, 30000]),
  concatenated in set order, B_eff of each, and their digests.
* ``potts_n500_b50000_sites.npz`` -- the oracle's minimisers of the site
  problems (sec. 3.4 step 3, eq. g_regdef2) for the eight sites drawn by
  ``synth.sample_sites(55, 500, 8)``, from zero to ||grad g_r^reg||_2 <= 1e-8,
  with the oracle's own weights; couplings stored in FP32 (rounding <= 6e-8
  relative, far below the 1e-4 comparisons they serve), the oracle's final
  gradient norms, iteration and evaluation counts, and the wall time of the
  oracle fit per site on the machine that wrote the file.
"""
from __future__ import annotations

import argparse
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from tests.helpers import clustered_msa  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
THETA = 0.8
CLUSTERED = dict(seed=5005, B=50000, N=500, n_anc=1250, p_mut=0.1)
SITE_SEED = 55


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def write_reweight(path, msa, threads):
    t = time.perf_counter()
    m, w, beff = oracle.reweight(msa, theta=THETA, nthreads=threads)
    dt = time.perf_counter() - t
    np.savez_compressed(path, m=m, w=w, beff=np.array([beff]), digest=np.array(synth.msa_digest(msa)),
                        theta=np.array([THETA]))
    print(f"{os.path.basename(path)}: B_eff {beff!r}, m in [{m.min()}, {m.max()}], {dt:.0f} s", flush=True)
    return m, w, beff


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=None)
    ap.add_argument("--skip-sites", action="store_true")
    ap.add_argument("--only", choices=("all", "ragged"), default="all")
    args = ap.parse_args()
    threads = oracle._threads(args.threads)

    if args.only in ("all", "ragged"):
        sets = synth.ragged_set(16)
        ms, ws, beffs, digests = [], [], [], []
        t = time.perf_counter()
        for a in sets:
            m, w, beff = oracle.reweight(a.msa, theta=THETA, nthreads=threads)
            ms.append(m)
            ws.append(w)
            beffs.append(beff)
            digests.append(synth.msa_digest(a.msa))
        np.savez_compressed(os.path.join(HERE, "ragged16_reweight.npz"), m=np.concatenate(ms),
                            w=np.concatenate(ws), beff=np.array(beffs),
                            B=np.array([a.B for a in sets], dtype=np.int32),
                            N=np.array([a.N for a in sets], dtype=np.int32), digest=np.array(digests),
                            theta=np.array([THETA]))
        print(f"ragged16_reweight.npz: {time.perf_counter() - t:.0f} s", flush=True)
        if args.only == "ragged":
            return

    s = synth.workload("potts_n500_b50000")
    m, w, beff = write_reweight(os.path.join(HERE, "potts_n500_b50000_reweight.npz"), s.msa, threads)
    cm = clustered_msa(**CLUSTERED)
    write_reweight(os.path.join(HERE, "clustered_n500_b50000_reweight.npz"), cm, threads)
    if args.skip_sites:
        return

    sites = synth.sample_sites(SITE_SEED, s.N, 8)
    t = time.perf_counter()
    h, J, stats = oracle.fit(s.msa, w, beff, s.lambda_h, s.lambda_J, sites=sites, tol=1e-8,
                             nthreads=threads)
    dt = time.perf_counter() - t
    gn = np.array([st["gnorm"] for st in stats])
    ev = np.array([st["evaluations"] for st in stats], dtype=np.int32)
    it = np.array([st["iterations"] for st in stats], dtype=np.int32)
    status = np.array([st["status"] for st in stats], dtype=np.int32)
    assert np.all(status == 0), stats
    # wall time per site fit: the sites ran one per thread, so each took about
    # dt * (threads used) / (sites) of one core
    used = min(threads, len(sites))
    np.savez_compressed(os.path.join(HERE, "potts_n500_b50000_sites.npz"),
                        sites=np.array(sites, dtype=np.int32), h=h, J=J.astype(np.float32), gnorm=gn,
                        evaluations=ev, iterations=it, digest=np.array(synth.msa_digest(s.msa)),
                        beff=np.array([beff]), fit_seconds_all=np.array([dt]),
                        fit_threads=np.array([used]), cpu_model=np.array(cpu_model()))
    print(f"sites {sites}: gnorm max {gn.max():.2e}, evaluations {ev.tolist()}, {dt:.0f} s on {used} threads",
          flush=True)


if __name__ == "__main__":
    main()
