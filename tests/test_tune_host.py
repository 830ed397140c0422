"""Host logic of the access-pattern chooser (paper_1510_03560_amd/tune.py),
with the GPU timing replaced by fixed figures."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1510_03560_amd import lbm as L  # noqa: E402
from paper_1510_03560_amd import tune  # noqa: E402


def fake(timings):
    def time_pattern(case, pattern, store=L.STORE_F32, steps=40, warmup=8):
        ms, nbytes = timings[pattern]
        return {"pattern": pattern, "ms_per_step": ms, "bytes_reserved": nbytes, "steps": steps}
    return time_pattern


def test_fastest_pattern_wins(monkeypatch):
    monkeypatch.setattr(tune, "time_pattern", fake({L.PATTERN_AB: (0.70, 2200), L.PATTERN_AA: (0.82, 1200)}))
    assert tune.choose_pattern(None)["pattern"] == L.PATTERN_AB
    monkeypatch.setattr(tune, "time_pattern", fake({L.PATTERN_AB: (6.56, 9800), L.PATTERN_AA: (5.51, 5950)}))
    r = tune.choose_pattern(None)
    assert r["pattern"] == L.PATTERN_AA and len(r["timings"]) == 2


def test_memory_budget(monkeypatch):
    monkeypatch.setattr(tune, "time_pattern", fake({L.PATTERN_AB: (0.70, 2200), L.PATTERN_AA: (0.82, 1200)}))
    assert tune.choose_pattern(None, max_bytes=2200)["pattern"] == L.PATTERN_AB
    assert tune.choose_pattern(None, max_bytes=2199)["pattern"] == L.PATTERN_AA
    with pytest.raises(ValueError):
        tune.choose_pattern(None, max_bytes=1199)
