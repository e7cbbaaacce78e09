"""Host logic of the block-size autotuner (cache keys, candidates, reuse)."""
import json

from paper_2510_26574_amd import autotune as at


def test_candidates_divide_rank():
    assert at.candidates(64) == [16, 32]
    assert at.candidates(512) == [16, 32, 64, 128]
    assert at.candidates(96) == [16, 32]
    assert all(96 % b == 0 for b in at.candidates(96))


def test_classes_and_cache(tmp_path):
    calls = []

    def fake_tuner(job, cands, reps):
        calls.append((job, tuple(cands)))
        return cands[-1], {b: 1.0 / b for b in cands}

    probs = [(5000, 32, 64), (5100, 32, 64), (90000, 512, 512), (5000, 128, 64)]
    path = str(tmp_path / "tune.json")
    bs, cache = at.tune(probs, lambda i, b: ("job", i, b), cache_path=path, tuner=fake_tuner)
    assert bs == [32, 32, 128, 32]
    assert len(calls) == 3  # the first two problems share a class
    assert at.job_class(5000, 32, 64) == at.job_class(5100, 32, 64)
    assert json.load(open(path)) == cache
    calls.clear()
    bs2, _ = at.tune(probs, lambda i, b: None, cache_path=path, tuner=fake_tuner)
    assert bs2 == bs and not calls  # everything from the cache
