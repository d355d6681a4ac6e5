"""plm_objgrad_static, the objective/gradient entry point that allocates
nothing (its scratch is the library's fixed per-GPU array), against
plm_objgrad with a caller workspace: the same kernels, so the results agree
bit for bit.  Two calls in a row, the second on a smaller problem (the array
keeps the first call's contents), on every evaluation path; a problem larger
than the array is rejected; the call leaves torch's allocator untouched when
its outputs are preallocated."""
import ctypes

import numpy as np
import pytest
import torch

from tests.helpers import random_params

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def plm():
    import paper_1401_4832_amd as plm
    return plm


def _problem(seed, B, N, q=21):
    rng = np.random.default_rng(seed)
    msa = torch.from_numpy(rng.integers(0, q, size=(B, N), dtype=np.uint8)).to(DEV)
    w = torch.from_numpy(rng.uniform(0.2, 1.0, size=B)).to(DEV)
    beff = w.sum().reshape(1).clone()
    h, J = random_params(seed + 1, N, q, 0.3, 0.2)
    return msa, w, beff, torch.from_numpy(h.astype(np.float32)).to(DEV), torch.from_numpy(J.astype(np.float32)).to(DEV)


@pytest.mark.parametrize("path", [0, 1, 2, 3, 4, 5, 6, 7])
def test_static_scratch_matches_workspace_call(plm, path):
    print(f"[case] plm_objgrad_static path={path}", flush=True)
    for seed, B, N in ((5, 3100, 37), (6, 700, 19)):  # the second call is smaller
        msa, w, beff, h, J = _problem(seed + 10 * path, B, N)
        a = plm.objgrad(msa, w, beff, h, J, path=path)
        b = plm.objgrad_static(msa, w, beff, h, J, path=path)
        plm.sync(DEV)
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2]), (seed, B, N)


def test_static_scratch_site_list_and_no_gradient(plm):
    print("[case] plm_objgrad_static site list, objective only", flush=True)
    msa, w, beff, h, J = _problem(41, 1500, 25)
    sites = torch.tensor([3, 0, 24, 11], dtype=torch.int32, device=DEV)
    a = plm.objgrad(msa, w, beff, h, J, sites=sites, path=6)
    b = plm.objgrad_static(msa, w, beff, h, J, sites=sites, path=6)
    f_only, gh, gJ = plm.objgrad_static(msa, w, beff, h, J, path=6, grad=False)
    plm.sync(DEV)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
    assert gh is None and gJ is None
    full = plm.objgrad(msa, w, beff, h, J, path=6)
    plm.sync(DEV)
    assert torch.equal(full[0], f_only)


def test_static_scratch_rejects_oversized_problems(plm):
    from paper_1401_4832_amd import _lib
    L = _lib.lib()
    B, N = 5000, 120
    assert L.plm_objgrad_workspace_bytes(B, N, 21, 0) > _lib.STATIC_SCRATCH_BYTES
    msa, w, beff, h, J = _problem(7, B, N)
    with pytest.raises(plm.PlmError) as e:
        plm.objgrad_static(msa, w, beff, h, J)
    assert e.value.code == _lib.PLM_E_WORKSPACE


def test_static_scratch_call_allocates_nothing(plm):
    """With preallocated outputs the call goes through torch's allocator not at
    all: its statistics do not move."""
    msa, w, beff, h, J = _problem(8, 900, 21)
    N, q = 21, 21
    out = (torch.zeros(N, dtype=torch.float64, device=DEV), torch.zeros(N, q, dtype=torch.float32, device=DEV),
           torch.zeros(N, N, q, q, dtype=torch.float32, device=DEV))
    plm.objgrad_static(msa, w, beff, h, J, path=6, out=out)
    torch.cuda.synchronize()
    before = torch.cuda.memory_stats(DEV)["allocation.all.allocated"]
    for _ in range(3):
        plm.objgrad_static(msa, w, beff, h, J, path=6, out=out)
    torch.cuda.synchronize()
    assert torch.cuda.memory_stats(DEV)["allocation.all.allocated"] == before
    ref = plm.objgrad(msa, w, beff, h, J, path=6)
    plm.sync(DEV)
    assert torch.equal(ref[0], out[0]) and torch.equal(ref[2], out[2])
