"""HBM planner: groups of shots whose checkpointed gradient evaluations fit
the device memory, evaluated one after the other with shared workspaces and
their gradients summed into one global model.

The computation is the library's (bhfwi_plan, bhfwi_plan_bytes: the same
packing as bhfwi_create); this module only gives it a Python shape.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

from . import _lib


def workspace_bytes(shots, K):
    """Bytes of the fwd, ckpt and adj workspaces and the accumulators of shots
    evaluated as one group with checkpoint interval K."""
    b = _lib.plan_bytes(shots, K)
    return {"fwd": b.fwd_ws_bytes, "ckpt": b.ckpt_bytes, "adj": b.adj_ws_bytes,
            "acc": b.acc_bytes}


def best_interval(shots):
    """Memory-optimal checkpoint interval (a multiple of 8) for one group."""
    return _lib.plan_bytes(shots, 0).ckpt_every


@dataclass
class Plan:
    groups: List[List[int]]
    ckpt_every: List[int]
    bytes_workspace: int      # shared workspaces (max over groups)
    bytes_traces: int         # traces, residuals and observed data of every group


def plan(shots, budget_bytes, ckpt_every=None, max_groups=None):
    """Split shots into the fewest groups whose shared workspaces plus all
    traces fit budget_bytes (MemoryError if none does)."""
    gof, Ks, info = _lib.plan(shots, budget_bytes, ckpt_every or 0, max_groups or 0)
    groups = [[] for _ in range(info.ngroups)]
    for s, g in enumerate(gof):
        groups[g].append(s)
    return Plan(groups, Ks, int(info.workspace_bytes), int(info.trace_bytes))
