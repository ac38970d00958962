"""ROCTx ranges of the serving loop: they nest, pass exceptions through and
are no-ops when switched off (no GPU needed)."""
import importlib

import pytest

from paper_2511_04261_amd import markers


def _fresh(monkeypatch, value):
    monkeypatch.setenv("DPPIX_ROCTX", value)
    m = importlib.reload(markers)
    return m


def test_ranges_nest_and_pass_exceptions(monkeypatch):
    m = _fresh(monkeypatch, "1")
    with m.marker_range("outer"):
        with m.marker_range("inner"):
            m.mark("point")
    with pytest.raises(ValueError):
        with m.marker_range("raises"):
            raise ValueError("inside a range")
    # the loop still runs ranges afterwards
    with m.marker_range("after"):
        pass


def test_switched_off_opens_nothing(monkeypatch):
    m = _fresh(monkeypatch, "0")
    assert m.library() is None
    with m.marker_range("off"):
        m.mark("off")


def test_scheduler_runs_with_markers(monkeypatch):
    """The scheduler with ranges on around its phases (the oracle as a CPU
    backend), including a launch that fails inside its range: every request
    still ends with its own result or its own error."""
    _fresh(monkeypatch, "1")
    from paper_2511_04261_amd.serving import MemoryLedger, Scheduler
    from tests.test_serving_cpu import CpuBackend, FakeClock, make_requests, run
    be = CpuBackend(explode_on={4})
    sch = Scheduler(be, MemoryLedger(10**9), max_batch=4, max_inflight=2, clock=FakeClock())
    reqs = make_requests(10)
    run(sch, reqs, per_pump=2)
    assert len(sch.finished) == 9 and [r.rid for r in sch.rejected] == [4]
