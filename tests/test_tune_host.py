"""Host logic of the access-pattern chooser (paper_1510_03560_amd/tune.py):
the device bytes of each pattern come from the library's lbm_plan_bytes
(no GPU needed), the GPU timing is replaced by fixed figures."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1510_03560_amd import lbm as L  # noqa: E402
from paper_1510_03560_amd import tune  # noqa: E402
from paper_1510_03560_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module")
def case():
    return W.porous_injection(64, seed=0)


def fake(ms, calls=None, enomem=()):
    def time_pattern(case, pattern, store=L.STORE_F32, steps=40, warmup=8):
        if calls is not None:
            calls.append(pattern)
        if pattern in enomem:
            raise L.LbmError(-3, "device allocation failed")
        return {"pattern": pattern, "ms_per_step": ms[pattern], "bytes_reserved": 0, "steps": steps}
    return time_pattern


def test_planned_bytes_order(case):
    ab = tune.planned_bytes(case, L.PATTERN_AB)
    aa = tune.planned_bytes(case, L.PATTERN_AA)
    ab16 = tune.planned_bytes(case, L.PATTERN_AB, L.STORE_F16DEV)
    # 64 blocks hold fluid: two FP32 buffers of 38 planes hold 2 * 38 * 4 B per cell,
    # one buffer plus psi 38 * 4 + 8 B
    n = 64 * 4096
    assert ab - aa == (38 * 4 - 8) * (n + 4096)
    assert ab - ab16 == (2 * 38 * 2 - 16) * (n + 4096)


def test_fastest_pattern_wins(monkeypatch, case):
    monkeypatch.setattr(tune, "time_pattern", fake({L.PATTERN_AB: 0.70, L.PATTERN_AA: 0.82}))
    assert tune.choose_pattern(case)["pattern"] == L.PATTERN_AB
    monkeypatch.setattr(tune, "time_pattern", fake({L.PATTERN_AB: 6.56, L.PATTERN_AA: 5.51}))
    r = tune.choose_pattern(case)
    assert r["pattern"] == L.PATTERN_AA and len(r["timings"]) == 2


def test_memory_budget_skips_before_allocating(monkeypatch, case):
    ab = tune.planned_bytes(case, L.PATTERN_AB)
    aa = tune.planned_bytes(case, L.PATTERN_AA)
    calls = []
    monkeypatch.setattr(tune, "time_pattern", fake({L.PATTERN_AB: 0.70, L.PATTERN_AA: 0.82}, calls))
    assert tune.choose_pattern(case, max_bytes=ab)["pattern"] == L.PATTERN_AB
    calls.clear()
    r = tune.choose_pattern(case, max_bytes=ab - 1)
    assert r["pattern"] == L.PATTERN_AA
    assert calls == [L.PATTERN_AA]  # the two-buffer pattern was never created
    assert r["skipped"][0]["pattern"] == L.PATTERN_AB
    with pytest.raises(ValueError):
        tune.choose_pattern(case, max_bytes=aa - 1)


def test_out_of_memory_falls_back(monkeypatch, case):
    """A pattern the device cannot hold (LBM_ENOMEM from its creation) is
    dropped and the other one returned."""
    monkeypatch.setattr(tune, "time_pattern",
                        fake({L.PATTERN_AB: 0.70, L.PATTERN_AA: 0.82}, enomem=(L.PATTERN_AB,)))
    r = tune.choose_pattern(case)
    assert r["pattern"] == L.PATTERN_AA
    assert r["skipped"][0]["reason"] == "out of device memory"
