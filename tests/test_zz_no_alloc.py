"""The allocation-free misfit (bhfwi_misfit_noalloc) against bhfwi_misfit,
called through the C-ABI: the same residual and the same misfit, bit for bit
(both run the same two-level reduction over the same number of blocks), on
two calls in a row, the second on a smaller input, and with accumulation."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU")]


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _case(nt, seed):
    import paper_2005_00281_amd as P
    w = workloads.tiny(nt=nt)
    sv = P.Survey(w.shots, (w.NRg, w.NZg), ckpt_every=50)
    n = sv.sizes.trace_elems
    g = torch.Generator().manual_seed(seed)
    dev = torch.device("cuda", 0)
    tr = torch.randn(n, generator=g).to(dev)
    obs = torch.randn(n, generator=g).to(dev)
    return sv, n, tr, obs


def test_noalloc_misfit_matches_context_misfit_twice_second_smaller():
    from paper_2005_00281_amd import _lib
    L = _lib.load()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    dev = torch.device("cuda", 0)
    sizes = []
    for nt, seed in ((240, 1), (97, 2)):  # second call: a smaller input
        sv, n, tr, obs = _case(nt, seed)
        sizes.append(n)
        r_ref = torch.empty(n, device=dev)
        J_ref = torch.zeros((), dtype=torch.float64, device=dev)
        r_new = torch.full((n,), float("nan"), device=dev)
        J_new = torch.full((), float("nan"), dtype=torch.float64, device=dev)
        assert L.bhfwi_misfit(sv._h, stream, _ptr(tr), _ptr(obs), _ptr(r_ref), _ptr(J_ref),
                              0) == 0
        assert L.bhfwi_misfit_noalloc(stream, n, _ptr(tr), _ptr(obs), _ptr(r_new),
                                      _ptr(J_new), 0) == 0
        torch.cuda.synchronize()
        assert torch.equal(r_new, r_ref)
        assert J_new.item() == J_ref.item()
        # the definition, in float64 on the host
        r64 = tr.double().cpu() - obs.double().cpu()
        assert abs(J_new.item() - 0.5 * float((r64 * r64).sum())) <= 1e-6 * J_new.item()
        # accumulation adds to the given value
        J_acc = torch.full((), 1.5, dtype=torch.float64, device=dev)
        assert L.bhfwi_misfit_noalloc(stream, n, _ptr(tr), _ptr(obs), _ptr(r_new),
                                      _ptr(J_acc), 1) == 0
        torch.cuda.synchronize()
        assert J_acc.item() == 1.5 + J_ref.item()
    assert sizes[1] < sizes[0]


def test_noalloc_misfit_rejects_bad_arguments_and_handles_empty():
    from paper_2005_00281_amd import _lib
    L = _lib.load()
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    dev = torch.device("cuda", 0)
    J = torch.full((), 7.0, dtype=torch.float64, device=dev)
    assert L.bhfwi_misfit_noalloc(stream, -1, None, None, None, _ptr(J), 0) == -1
    assert b"negative" in L.bhfwi_last_error(None)
    assert L.bhfwi_misfit_noalloc(stream, 4, None, None, None, _ptr(J), 0) == -1
    assert L.bhfwi_misfit_noalloc(stream, 0, None, None, None, _ptr(J), 0) == 0
    torch.cuda.synchronize()
    assert J.item() == 0.0
