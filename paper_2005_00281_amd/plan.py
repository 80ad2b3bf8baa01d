"""HBM planner for the checkpointed gradient evaluation.

One-level checkpointing keeps ceil(nt/K) - 1 forward states and the velocity
history of one K-step segment.  For a set of shots with F floats of state and
C cells per step of history, the memory (ceil(nt/K) - 1) F + 2 K C is smallest
near K = sqrt(nt F / (2 C)).  When all shots do not fit the budget at that K,
the shots are split into groups (longest-processing-time first on cells x nt)
that are evaluated one after the other with shared workspaces, their
gradients summed into one global model.

Sizes follow the library's packing (64-float alignment per shot).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List

ALIGN = 64


def _al(x: int) -> int:
    return (x + ALIGN - 1) // ALIGN * ALIGN


def shot_floats(sh):
    NR, NZ = sh.nr + sh.pr, sh.nz + 2 * sh.pz
    cells = _al(NR * NZ)
    fst = _al(6 * NR * NZ + 4 * sh.pr * NZ + 4 * NR * 2 * sh.pz)
    ast = _al(6 * NR * NZ + 5 * sh.pr * NZ + 5 * NR * 2 * sh.pz)
    return cells, fst, ast


def workspace_bytes(shots, K):
    """Bytes of the fwd, ckpt and adj workspaces and the accumulators."""
    C = F = A = 0
    for sh in shots:
        c, f, a = shot_floats(sh)
        C, F, A = C + c, F + f, A + a
    ntmax = max(sh.nt for sh in shots)
    nseg = -(-ntmax // K)
    return {"fwd": 8 * F, "ckpt": 4 * max(0, nseg - 1) * F, "adj": 4 * (2 * A + 2 * K * C),
            "acc": 16 * C}


def trace_bytes(shots):
    return 4 * sum(len(sh.rec_k) * sh.nt for sh in shots)


def best_interval(shots, multiple=8):
    C = F = 0
    for sh in shots:
        c, f, _ = shot_floats(sh)
        C, F = C + c, F + f
    ntmax = max(sh.nt for sh in shots)
    k = math.sqrt(ntmax * F / (2.0 * C))
    cands = {max(multiple, int(k) // multiple * multiple),
             max(multiple, -(-int(k) // multiple) * multiple)}
    cands = {min(c, ntmax) for c in cands}
    return min(cands, key=lambda K: sum(workspace_bytes(shots, K).values()))


@dataclass
class Plan:
    groups: List[List[int]]
    ckpt_every: List[int]
    bytes_workspace: int      # shared workspaces (max over groups)
    bytes_traces: int         # traces, residuals and observed data of every group


def plan(shots, budget_bytes, ckpt_every=None, max_groups=None):
    """Split shots into the fewest groups whose shared workspaces plus all
    traces fit budget_bytes."""
    n = len(shots)
    load = [sh.cells * sh.nt for sh in shots]
    order = sorted(range(n), key=lambda s: -load[s])
    for G in range(1, (max_groups or n) + 1):
        groups = [[] for _ in range(G)]
        tot = [0] * G
        for s in order:
            g = min(range(G), key=lambda q: tot[q])
            groups[g].append(s)
            tot[g] += load[s]
        groups = [sorted(g) for g in groups if g]
        Ks = [ckpt_every or best_interval([shots[s] for s in g]) for g in groups]
        ws = {}
        for g, K in zip(groups, Ks):
            for name, b in workspace_bytes([shots[s] for s in g], K).items():
                ws[name] = max(ws.get(name, 0), b)
        wsb = sum(ws.values())
        trb = 3 * trace_bytes(shots)
        if wsb + trb <= budget_bytes:
            return Plan(groups, Ks, wsb, trb)
    raise MemoryError("no grouping of %d shots fits %.1f GB" % (n, budget_bytes / 1e9))
