"""Host logic of the batch autotuner (no GPU): choice rules, sampling, signature, cache."""
import torch

from paper_1805_01844_amd import tune


def test_block_length_choice_trades_ratio_for_speed():
    # (L, compress ms, decompress ms, ratio)
    res = [(256, 1.0, 1.0, 3.00), (512, 0.9, 0.9, 3.10), (1024, 0.5, 0.5, 3.08), (4096, 0.2, 0.2, 2.50)]
    assert tune.choose_block_length(res, 0.01) == 1024   # 3.08 is within 1% of 3.10; fastest of those
    assert tune.choose_block_length(res, 0.0) == 512     # no slack: best ratio only
    assert tune.choose_block_length(res, 0.5) == 4096    # everything allowed: fastest


def test_block_length_ties_prefer_ratio_then_smaller_L():
    res = [(256, 1.0, 1.0, 3.0), (512, 1.0, 1.0, 3.02), (1024, 1.0, 1.0, 3.02)]
    assert tune.choose_block_length(res, 0.1) == 512


def test_grid_choice():
    assert tune.choose_grid([(0, 1.0, 1.0), (1024, 0.9, 1.0), (2048, 0.9, 1.0)]) == 1024
    assert tune.choose_grid([(0, 1.0, 1.0)]) == 0


def test_sample_is_spread_and_bounded():
    segs = [torch.zeros(1000 + i, dtype=torch.uint16) for i in range(500)]
    s = tune.sample_segments(segs, max_segments=50)
    assert 45 <= len(s) <= 50 and s[0] is segs[0] and s[-1] is not segs[49]
    s = tune.sample_segments(segs, max_segments=500, max_bytes=10000)
    assert sum(x.numel() * 2 for x in s) <= 10000 + 2 * 1500
    assert tune.sample_segments([], 10) == []


def test_signature_depends_on_mix_and_variant():
    a = [torch.zeros(74200, dtype=torch.uint16), torch.zeros(100, dtype=torch.uint32)]
    b = [torch.zeros(74200, dtype=torch.uint16), torch.zeros(100, dtype=torch.uint16)]
    assert tune.signature(a, 0) != tune.signature(b, 0)
    assert tune.signature(a, 0) != tune.signature(a, 0x100)
    assert tune.signature(a, 0) == tune.signature(list(reversed(a)), 0)


def test_cache_round_trip(tmp_path, monkeypatch):
    p = tmp_path / "t.json"
    monkeypatch.setenv("PCOMP_TUNE_CACHE", str(p))
    assert tune.cache_path() == str(p)
    tune._store_cache(str(p), {"k": {"block_len": [256, 512, 1024], "grid": 0}})
    assert tune._load_cache(str(p))["k"]["grid"] == 0
    assert tune._load_cache(str(tmp_path / "missing.json")) == {}
