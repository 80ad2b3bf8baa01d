"""HBM planner: every shot lands in exactly one group, groups fit the budget,
and the chosen checkpoint interval minimises checkpoint + history memory."""
import pytest

import workloads
from paper_2005_00281_amd import plan


@pytest.mark.parametrize("name,budget", [("c3", 240e9), ("c4", 240e9), ("c4", 120e9)])
def test_groups_partition_and_fit(name, budget):
    w = workloads.make(name)
    p = plan.plan(w.shots, budget)
    flat = sorted(s for g in p.groups for s in g)
    assert flat == list(range(len(w.shots)))
    assert p.bytes_workspace + p.bytes_traces <= budget
    assert len(p.groups) == len(p.ckpt_every)


def test_interval_minimises_memory():
    w = workloads.make("c3")
    K = plan.best_interval(w.shots)
    mem = lambda k: sum(plan.workspace_bytes(w.shots, k).values())
    for other in (K // 2, K - 8, K + 8, 2 * K):
        assert mem(K) <= mem(other)


def test_single_shot_keeps_requested_interval():
    w = workloads.make("c2")
    p = plan.plan(w.shots, 1e12, ckpt_every=250)
    assert p.groups == [[0]] and p.ckpt_every == [250]


def test_impossible_budget_raises():
    w = workloads.make("c2")
    with pytest.raises(MemoryError):
        plan.plan(w.shots, 1e6)


@pytest.mark.gpu
def test_plan_bytes_are_the_context_sizes():
    """The planner's figures are the workspace sizes a context of the same
    shots asks for."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_00281_amd as P
    w = workloads.make("c4")
    p = plan.plan(w.shots, 120e9)
    for grp, K in zip(p.groups, p.ckpt_every):
        shots = [w.shots[s] for s in grp]
        z = P.Survey(shots, (w.NRg, w.NZg), ckpt_every=K).sizes
        b = plan.workspace_bytes(shots, K)
        assert (z.fwd_ws_bytes, z.ckpt_bytes, z.adj_ws_bytes, 4 * z.acc_elems) == \
            (b["fwd"], b["ckpt"], b["adj"], b["acc"])


@pytest.mark.gpu
def test_full_history_is_taken_when_it_fits():
    """The single-shot benchmark survey keeps its whole velocity history
    (8 nt cells bytes in place of checkpoints) under an 80 % budget of the
    device, and falls back to checkpoints when the budget is smaller than that
    history."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2005_00281_amd as P
    w = workloads.make("c2")
    sv = P.Survey(w.shots, (w.NRg, w.NZg), ckpt_every=250)
    ckpt_bytes = sv.sizes.ckpt_bytes
    hist = 8 * sv.sizes.nt_max * sv.sizes.cells
    assert sv.use_full_history_if_fits(0.8 * torch.cuda.get_device_properties(0).total_memory)
    assert sv.get_tune()["full_history"] == 1 and sv.sizes.ckpt_bytes == hist
    sv.set_tune(full_history=0)
    assert sv.sizes.ckpt_bytes == ckpt_bytes
    assert not sv.use_full_history_if_fits(hist / 2)
    assert sv.get_tune()["full_history"] == 0 and sv.sizes.ckpt_bytes == ckpt_bytes
