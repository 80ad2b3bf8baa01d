"""Full acquisition (near, far and ultra-far monopoles below a 13-receiver
array, logging every 0.5 ft) realigned to one source with 39 receivers, as
the Numerical Examples section describes its data.

CPU: the realignment is pure re-indexing, checked on data that encode their
own source and receiver positions; the workload's receiver rows form one
contiguous array.  GPU: a realigned 39-receiver shot records exactly the
traces of the three 13-receiver arrays modelled as separate shots.
"""
import numpy as np
import pytest

import workloads


def test_realigned_receivers_form_one_contiguous_array():
    z = workloads.realigned_receivers(0.3)
    sp = workloads.REC_SPACING_HALF_FOOT
    assert len(z) == 39
    assert np.allclose(np.diff(z), sp)
    assert z[0] == pytest.approx(0.3 + workloads.SOURCE_OFFSETS_STEPS[0] * sp)


def test_realign_gathers_each_source_with_its_receivers():
    offs = workloads.SOURCE_OFFSETS_STEPS
    D, Q, M = 60, 3, 13
    raw = np.empty((D, Q, M), np.int64)
    for d in range(D):
        for q in range(Q):
            for j in range(M):
                # receiver at position d + j, source q at position d - offs[q]
                raw[d, q, j] = 1000 * (d + j) + (d - offs[q])
    out = workloads.realign(raw)
    assert out.shape == (D - max(offs), Q * M)
    for s in range(out.shape[0]):
        src = out[s] % 1000
        rec = out[s] // 1000
        assert np.all(src == s)
        assert np.array_equal(rec - s, np.arange(offs[0], offs[0] + Q * M))


def test_workload_rows_match_the_realigned_geometry():
    w = workloads.full_acquisition(nsrc=3)
    sh = w.shots[0]
    z = workloads.realigned_receivers(0.3)
    rows = [workloads.row_of(zz, sh.dz, sh.pz) for zz in z]
    assert list(sh.rec_k) == rows and len(set(rows)) == 39
    assert (sh.nt - 1) * sh.dt >= 7.0 / 2000.0  # S at the farthest receiver


@pytest.mark.gpu
def test_realigned_shot_records_the_three_arrays():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import copy
    import paper_2005_00281_amd as P
    dev = torch.device("cuda", 0)
    w = workloads.full_acquisition(nsrc=2, nr=32, h=5e-3, p=8, dt=0.5e-6, nt=1200)
    print("[case] realigned acquisition", w.shots[0].NR, w.shots[0].NZ, flush=True)
    f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=dev)
    rho = f32(w.rho)
    lam, mu = P.moduli(f32(w.vp_true), f32(w.vs_true), rho)
    sv = P.Survey(w.shots, (w.NRg, w.NZg), ckpt_every=100)
    wav = sv.pack_wavelets([sh.wavelet for sh in w.shots])
    full = sv.unpack_traces(sv.fwd_model(lam, mu, rho, wav))
    for q in range(3):
        parts = []
        for sh in w.shots:
            s2 = copy.copy(sh)
            s2.rec_k = sh.rec_k[13 * q: 13 * (q + 1)]
            parts.append(s2)
        sv2 = P.Survey(parts, (w.NRg, w.NZg), ckpt_every=100)
        tr = sv2.unpack_traces(sv2.fwd_model(lam, mu, rho, sv2.pack_wavelets(
            [sh.wavelet for sh in parts])))
        for s in range(len(w.shots)):
            assert np.array_equal(tr[s], full[s][13 * q: 13 * (q + 1)])
