"""Host-side logic that needs no GPU: the W-cycle stage structure of the
multi-level driver and the bench's lookup of committed counter profiles."""

import json
import os

import pytest

torch = pytest.importorskip("torch")

from paper_1712_07070_amd import hydro  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _driver(n_levels):
    ml = object.__new__(hydro.MultiLevel)   # the stage logic only reads the level count
    ml.L = n_levels
    return ml


@pytest.mark.parametrize("n_levels", [1, 2, 3, 4])
def test_wcycle_stage_membership(n_levels):
    """Over the 2^(L-1) stages of a coarse step level l advances 2^l times
    (dt_l = dt_0 / 2^l), every stage advances the finest level, and a level
    that advances in a stage also advances every finer level there."""
    ml = _driver(n_levels)
    stages = [ml.stage_levels(s) for s in range(2 ** (n_levels - 1))]
    for l in range(n_levels):
        assert sum(l in st for st in stages) == 2 ** l
    for st in stages:
        assert n_levels - 1 in st
        assert st == list(range(st[0], n_levels))
    assert stages[0] == list(range(n_levels))


def test_wcycle_three_levels_exact():
    assert [_driver(3).stage_levels(s) for s in range(4)] == [[0, 1, 2], [2], [1, 2], [2]]


def test_measured_profile_guards(monkeypatch):
    import bench
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        rec = json.load(fh)
    key = next(iter(rec))
    variants = rec[key]["by_variant"]
    v = next(iter(variants))
    # a record is used only for the sources it was measured on
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: rec[key]["source_sha256"])
    assert bench.measured_traffic(key, v) == variants[v]["bytes_per_launch"]
    assert bench.measured_profile(key, 99, "bytes_per_launch") is None
    assert bench.measured_profile("no such kernel", v, "bytes_per_launch") is None
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "0" * 64)
    assert bench.measured_traffic(key, v) is None
