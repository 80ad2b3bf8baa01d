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


def test_committed_tune_cache_names_known_fields_with_valid_values():
    # every cached field is a bhfwi_tune field the binding knows, switches are
    # 0 or 1, and the shapes are ones the library compiles (by the header's list)
    from paper_2005_00281_amd._lib import Tune
    names = {n for n, _ in Tune._fields_}
    compiled = {(2, 16, 4), (3, 16, 4), (4, 16, 4), (2, 16, 8), (3, 16, 8), (4, 16, 8),
                (2, 24, 8), (3, 24, 8), (4, 24, 8), (6, 24, 8), (4, 32, 8), (6, 32, 8),
                (8, 32, 8), (2, 16, 16), (3, 16, 16), (4, 16, 16), (4, 32, 16), (6, 32, 16),
                (8, 32, 16), (4, 48, 16), (6, 48, 16), (8, 48, 16), (4, 64, 16), (8, 64, 16)}
    with open(os.path.join(ROOT, "paper_2005_00281_amd", "tune_cache.json")) as f:
        table = json.load(f)
    for key, entry in table.items():
        t = entry["tune"]
        assert set(t) <= names, (key, set(t) - names)
        for flag in ("use_graph", "tile_map", "pml_overlap", "rec_overlap", "fwd_tile_overlap"):
            assert t.get(flag, 0) in (0, 1), (key, flag)
        assert not (t.get("pml_overlap") and t.get("rec_overlap")), key
        if t.get("tb_steps", 0) >= 2:
            assert (t["tb_steps"], t["tb_rows"], t["tb_waves"]) in compiled, key
        if t.get("adj_tb_steps", 0) >= 2:
            shape = (t["adj_tb_steps"], t["adj_tb_rows"], t["adj_tb_waves"])
            assert shape in compiled and shape != (4, 64, 16), key
