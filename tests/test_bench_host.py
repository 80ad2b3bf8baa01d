"""Host-side logic of bench.py, on the CPU: the adjoint launch count that the
blocked roofline is priced on, the launch-gap summary of a kernel trace, the
counter tables' keys, and the refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_adjoint_blocks_full_record():
    # 8000 steps in 250-step segments, six steps per block: 41 blocks of six
    # and one of four per segment, 32 segments
    assert bench.adjoint_blocks([8000], 8000, 250, 6) == [32 * 42]
    # one segment holding the whole record, eight steps per block
    assert bench.adjoint_blocks([8000], 8000, 8000, 8) == [1000]
    # one step per launch
    assert bench.adjoint_blocks([37], 37, 10, 1) == [37]


def test_adjoint_blocks_ragged_shots():
    # record of 300 steps in one segment, blocks of 8 from step 299 down:
    # lowest steps 292, 284, ..., 4 (37 blocks) and a last block 3..0.  A shot
    # of 100 steps takes part in the blocks whose lowest step is below 100:
    # 92, 84, ..., 4 (12 blocks) and the last one.
    assert bench.adjoint_blocks([300, 100, 1], 300, 300, 8) == [38, 13, 1]
    # segments of 128: [256, 300) has 44 steps (blocks lo 292..260 and 256),
    # [128, 256) and [0, 128) 16 blocks each
    assert bench.adjoint_blocks([300, 200], 300, 128, 8) == [6 + 16 + 16, 0 + 16 + 16 - 7]


def test_adjoint_blocks_brute_force():
    # the count equals a step-by-step replay of the launch sequence
    import random
    rng = random.Random(7)
    for _ in range(50):
        nt_max = rng.randint(1, 400)
        nts = [rng.randint(1, nt_max) for _ in range(rng.randint(1, 4))] + [nt_max]
        seg = rng.randint(1, nt_max)
        T = rng.randint(1, 9)
        want = [0] * len(nts)
        for j0 in range(0, nt_max, seg):
            steps = list(range(min(j0 + seg, nt_max) - 1, j0 - 1, -1))
            for b in range(0, len(steps), T):
                lo = steps[min(b + T, len(steps)) - 1]
                for s, nt in enumerate(nts):
                    want[s] += lo < nt
        assert bench.adjoint_blocks(nts, nt_max, seg, T) == want


def test_adj_shape():
    tune = {"adj_tb_steps": 6, "adj_tb_rows": 32, "adj_tb_waves": 16,
            "tb_steps": 8, "tb_rows": 48, "tb_waves": 16}
    assert bench.adj_shape(tune) == (6, 32, 16)
    assert bench.adj_shape(dict(tune, adj_tb_steps=1)) == (0, 0, 0)
    assert bench.adj_shape(dict(tune, adj_tb_steps=0)) == (8, 48, 16)


def _trace(tmp_path, rows):
    p = tmp_path / "k_kernel_trace.csv"
    with open(p, "w") as f:
        f.write("Kernel_Name,Start_Timestamp,End_Timestamp\n")
        for name, t0, t1 in rows:
            f.write('"%s",%d,%d\n' % (name, t0, t1))
    return str(p)


def test_trace_gaps(tmp_path, capsys):
    us = 1000  # timestamps in ns
    rows = [("k_fwd_tb<8, 48, 16, 0>", 0, 100 * us),
            ("k_fwd_tb<8, 48, 16, 1>", 102 * us, 150 * us),    # 2 us step gap
            ("k_fill", 151 * us, 152 * us),                    # not a step kernel
            ("k_adj_tb<6, 32, 16, 0, 0>", 152 * us, 400 * us),
            ("k_adj_tb<6, 32, 16, 1, 0>", 390 * us, 500 * us),  # overlaps: no gap
            ("k_adj_tb<6, 32, 16, 0, 0>", 2500 * us, 2600 * us)]  # 2 ms host pause
    bench.trace_gaps(_trace(tmp_path, rows))
    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert out["dispatches"] == 6 and out["step_dispatches"] == 5
    assert out["span_ms"] == pytest.approx(2.6)
    # busy: 100 + 48 + 1 + 348 (152..500) + 100 us
    assert out["busy_ms"] == pytest.approx(0.597)
    assert out["idle_ms"] == pytest.approx(0.002 + 0.001 + 2.0)
    # step pairs: fwd -> fwd and the pause; k_fill breaks one, the overlap another
    assert out["step_pairs"] == 2 and out["host_pauses"] == 1
    assert out["step_gap_ms"] == pytest.approx(0.002)
    assert out["host_pause_ms"] == pytest.approx(2.0)


def test_counter_tables_are_keyed_alike():
    # every vector-instruction entry was taken on sources that also have a
    # traffic entry, for the same kernel, tile order and workload
    for key in bench.PMC_VALU:
        assert key in bench.PMC_TRAFFIC, key
    for (kname, tile_map, workload, sha), (rd, wr) in bench.PMC_TRAFFIC.items():
        assert "k_adj" in kname and tile_map in (0, 1) and len(sha) == 16
        assert rd > 0 and wr > 0
    assert len(bench.kernel_sources_sha()) == 16


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
