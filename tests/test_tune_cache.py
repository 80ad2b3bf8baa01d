"""Host logic of the tune cache and of the history-mode choice (no GPU).

The velocity-history mode (full history or checkpoints) decides how much
device memory a survey takes, so it follows the memory budget and never a
cached tune; a cached kernel choice must not switch it on."""
import json
import os

from paper_2005_00281_amd._lib import NOT_CACHED, Survey, cached_kernel_tune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


class _Stub:
    """The parts of a Survey that use_full_history_if_fits touches: bytes per
    history mode stand in for bhfwi_sizes."""

    def __init__(self, full, nbytes):
        self.t = {"full_history": full}
        self.nbytes = nbytes

    def set_tune(self, **kw):
        self.t.update(kw)

    def get_tune(self):
        return dict(self.t)

    def device_bytes(self):
        return self.nbytes[self.t["full_history"]]


def test_full_history_switched_off_over_budget_even_when_already_on():
    s = _Stub(1, {0: 10, 1: 100})
    assert Survey.use_full_history_if_fits(s, 50) is False
    assert s.t["full_history"] == 0


def test_full_history_switched_on_within_budget():
    s = _Stub(0, {0: 10, 1: 100})
    assert Survey.use_full_history_if_fits(s, 100) is True
    assert s.t["full_history"] == 1


def test_cached_tune_never_carries_the_history_mode():
    tune = {"tb_steps": 8, "adj_tb_rows": 64, "full_history": 1, "time_kernels": 1}
    kept = cached_kernel_tune(tune)
    assert "full_history" not in kept and "time_kernels" not in kept
    assert kept == {"tb_steps": 8, "adj_tb_rows": 64}


def test_committed_tune_cache_holds_kernel_choices_only():
    with open(os.path.join(ROOT, "paper_2005_00281_amd", "tune_cache.json")) as f:
        table = json.load(f)
    assert table
    for key, entry in table.items():
        assert not set(NOT_CACHED) & set(entry["tune"]), key
