"""Autotuner cache logic on the CPU: buckets, keys, the JSON store, and that a
cached choice is used without timing again."""
import dataclasses

import pytest
import torch

from paper_1401_4832_amd import api, autotune


def test_bucket_edges():
    assert autotune.bucket(40, 500) == (6, 9)
    assert autotune.bucket(64, 512) == (6, 9)
    assert autotune.bucket(65, 513) == (7, 10)
    assert autotune.bucket(2, 1) == (1, 1)


def test_key_is_order_free_and_separates_classes(monkeypatch):
    monkeypatch.setattr(autotune, "_arch", lambda dev: "gfx950")
    a = torch.zeros(500, 40, dtype=torch.uint8)
    b = torch.zeros(5000, 120, dtype=torch.uint8)
    k1 = autotune.key([(a,), (b,)], 21, True)
    k2 = autotune.key([(b,), (a,)], 21, True)
    assert k1 == k2 == "gfx950|q21|fp32|6x9,7x13"
    assert autotune.key([(a,)], 21, False) != autotune.key([(a,)], 21, True)


def test_store_load_roundtrip_and_cached_choice(monkeypatch, tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    monkeypatch.setattr(autotune, "_arch", lambda dev: "gfx950")
    a = torch.zeros(500, 40, dtype=torch.uint8)
    k = autotune.key([(a,)], 21, True)
    autotune.store({k: dict(path=2, tile_seqs=32, eval_ms=1.5, candidates=[])}, path)
    assert autotune.load(path)[k]["tile_seqs"] == 32

    def no_timing(*args, **kw):
        raise AssertionError("a cached bucket must not be timed again")
    monkeypatch.setattr(api, "tune", no_timing)
    ch = autotune.choose([(a,)], api.FitOptions(), 21, True, path=path)
    assert (ch["path"], ch["tile_seqs"]) == (2, 32)
    monkeypatch.setenv("PLM_TUNE_CACHE", path)
    o = autotune.tuned_options([(a,)], api.FitOptions(autotune=True, path=0), 21)
    assert (o.path, o.tile_seqs, o.autotune) == (2, 32, False)
    assert dataclasses.replace(o, path=0).path == 0


def test_fixed_point_paths_left_out_where_their_rounding_floor_reaches_tol(monkeypatch, tmp_path):
    path = str(tmp_path / "tune.json")
    monkeypatch.setattr(autotune, "_arch", lambda dev: "gfx950")
    cands = [dict(path=6, tile_seqs=0, eval_ms=1.0), dict(path=5, tile_seqs=32, eval_ms=1.5),
             dict(path=4, tile_seqs=32, eval_ms=2.0), dict(path=0, tile_seqs=16, eval_ms=3.0)]
    monkeypatch.setattr(api, "tune", lambda *a, **k: [dict(c) for c in cands])
    # 2^-23 sqrt(N q^2 B / 3) / B_eff: 1.4e-7 at N = 500, B = B_eff = 50000 (allowed at tol 1e-6),
    # 1.4e-6 at N = B = B_eff = 100 (left out)
    big = (torch.zeros(50000, 500, dtype=torch.uint8), None, torch.tensor([50000.0], dtype=torch.float64))
    small = (torch.zeros(100, 100, dtype=torch.uint8), None, torch.tensor([100.0], dtype=torch.float64))
    assert autotune.fixed_point_floor(big, 21) == pytest.approx(2.0 ** -23 * (500 * 441 * 50000 / 3) ** 0.5 / 50000)
    assert autotune.choose([big], api.FitOptions(), 21, path=path)["path"] == 6
    assert autotune.choose([small], api.FitOptions(), 21, path=path)["path"] == 4
    assert autotune.choose([big], api.FitOptions(), 21, path=path, fixed_point=False)["path"] == 4
    # a looser tolerance admits them again
    assert autotune.choose([small], api.FitOptions(tol=1e-5), 21, path=path)["path"] == 6


def test_symmetric_fit_takes_only_the_fp32_energy_fixed_point_path(monkeypatch, tmp_path):
    path = str(tmp_path / "tune.json")
    monkeypatch.setattr(autotune, "_arch", lambda dev: "gfx950")
    cands = [dict(path=6, tile_seqs=0, eval_ms=1.0), dict(path=5, tile_seqs=32, eval_ms=1.5),
             dict(path=4, tile_seqs=32, eval_ms=2.0), dict(path=0, tile_seqs=16, eval_ms=3.0)]
    monkeypatch.setattr(api, "tune", lambda *a, **k: [dict(c) for c in cands])
    big = (torch.zeros(50000, 500, dtype=torch.uint8), None, torch.tensor([50000.0], dtype=torch.float64))
    # over all N q + N (N - 1) / 2 q^2 parameters: 2.28e-6 at N = 500, B = B_eff = 50000
    P = 500 * 21 + 500 * 499 // 2 * 441
    fl = autotune.symmetric_floor(big, 21)
    assert fl == pytest.approx(2.0 ** -23 * (P * 50000 / 3) ** 0.5 / 50000)
    assert 2.2e-6 < fl < 2.4e-6
    # twice the floor below the tolerance: path 5 (never 6); else the FP32-class paths
    assert autotune.choose([big], api.FitOptions(tol=5e-6), 21, path=path, symmetric=True)["path"] == 5
    assert autotune.choose([big], api.FitOptions(tol=1e-6), 21, path=path, symmetric=True)["path"] == 4
    assert autotune.choose([big], api.FitOptions(tol=5e-6), 21, path=path, symmetric=True,
                           fixed_point=False)["path"] == 4
    # separate cache entries from the per-site fit's
    assert autotune.choose([big], api.FitOptions(tol=5e-6), 21, path=path)["path"] == 6
    assert autotune.key([big], 21, True, True, True) != autotune.key([big], 21, True, True, False)


def test_load_tolerates_missing_and_corrupt_files(tmp_path):
    assert autotune.load(str(tmp_path / "none.json")) == {}
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    assert autotune.load(str(bad)) == {}
