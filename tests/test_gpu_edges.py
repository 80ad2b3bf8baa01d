"""Edge cases of the HIP path against the oracle: a grid without PML, a grid
smaller than one tile with a record shorter than one time block, a zero
residual, a shot without receivers inside a batch, and the largest per-shot
grid the benchmark workloads define (532 x 16424 padded cells), also 48 of
them in one batch (state buffers beyond 2^31 floats).

Tolerances as in the main parity tests: traces relative L2 <= 1e-4,
gradients <= 1e-3, exact where the same arithmetic repeats.
"""
import copy

import numpy as np
import pytest

import oracle
import workloads
from util import geom, oracle_models, rel_l2
from test_gpu_parity import T, _dev, _say, f32, gpu_models, survey

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EDGE_TUNES = [T(2, 4, 1), T(tb=4, graph=0), T(tb=8, tbr=64, tbw=16, atb=6, atbr=48, atbw=16),
              T(tb=8, tbr=64, tbw=16, atb=8, atbr=48, atbw=16, rov=1)]


def _forward_and_gradient(w, tune, ckpt):
    sh = w.shots[0]
    g = geom(sh)
    lam_o, mu_o, rho_o = oracle_models(w, 0, "start")
    lt, mt, _ = oracle_models(w, 0, "true")
    d_obs = oracle.forward(g, lt, mt, rho_o, sh.wavelet)
    d_o = oracle.forward(g, lam_o, mu_o, rho_o, sh.wavelet)
    _, r = oracle.misfit(d_o, d_obs)
    gl_o, gm_o, il_o = oracle.gradient(g, lam_o, mu_o, rho_o, sh.wavelet, r, seg=ckpt)
    sv = survey(w, ckpt=ckpt, tune=tune)
    lam, mu, rho = gpu_models(w)
    wav = sv.pack_wavelets([sh.wavelet])
    tr = sv.fwd_model(lam, mu, rho, wav, store_ckpt=True)
    d_g = sv.unpack_traces(tr)[0]
    acc = sv.adjoint_model(lam, mu, rho, wav, f32(r.ravel()))
    gl, gm, il = (t.cpu().numpy() for t in sv.gradient(mu, acc))
    torch.cuda.synchronize()
    return (d_g, gl, gm, il), (d_o, gl_o, gm_o, il_o)


@pytest.mark.parametrize("tune", EDGE_TUNES)
def test_grid_without_pml(tune):
    w = workloads.tiny(nr=30, nz=120, p=0, nt=200)
    _say("no PML", tune)
    (d, gl, gm, il), (d_o, gl_o, gm_o, il_o) = _forward_and_gradient(w, tune, ckpt=45)
    assert rel_l2(d, d_o) <= 1e-4, rel_l2(d, d_o)
    assert rel_l2(gl, gl_o) <= 1e-3 and rel_l2(gm, gm_o) <= 1e-3
    assert rel_l2(il, il_o) <= 1e-4


@pytest.mark.parametrize("tune", EDGE_TUNES)
@pytest.mark.parametrize("nt", [1, 3, 11])
def test_grid_smaller_than_a_tile_and_short_records(tune, nt):
    """5 x 18 padded cells (one formation row outside a 4-cell hole, one PML
    row): every tile overhangs the grid on all sides; 1, 3 and 11 steps are
    shorter than, or not a multiple of, the time blocks."""
    w = workloads.tiny(nr=4, nz=16, p=1, nt=nt)
    _say("tiny grid", w.shots[0].NR, w.shots[0].NZ, "nt", nt, tune)
    (d, gl, gm, il), (d_o, gl_o, gm_o, il_o) = _forward_and_gradient(w, tune, ckpt=5)
    assert rel_l2(d, d_o) <= 1e-4, rel_l2(d, d_o)
    if np.abs(gl_o).max() > 0:
        assert rel_l2(gl, gl_o) <= 1e-3 and rel_l2(gm, gm_o) <= 1e-3
    assert rel_l2(il, il_o) <= 1e-4


@pytest.mark.parametrize("tune", [T(2, 4, 1), T(tb=8, tbr=64, tbw=16, atb=8, atbr=48,
                                                atbw=16, rov=1)])
def test_zero_residual_gives_zero_gradient(tune):
    w = workloads.tiny(nr=30, nz=120, p=6, nt=150)
    _say("zero residual", tune)
    sv = survey(w, ckpt=40, tune=tune)
    lam, mu, rho = gpu_models(w)
    wav = sv.pack_wavelets([w.shots[0].wavelet])
    sv.fwd_model(lam, mu, rho, wav, store_ckpt=True)
    r = torch.zeros(sv.sizes.trace_elems, device=_dev())
    gl, gm, il = sv.gradient(mu, sv.adjoint_model(lam, mu, rho, wav, r))
    assert not gl.any() and not gm.any()
    assert il.abs().max().item() > 0


def test_shot_without_receivers_in_a_batch():
    """A batch of a shot with no receivers and a shot with three: the second
    shot's traces and the batch gradient equal the single-shot run bit for
    bit (the receiverless shot adds exact zeros)."""
    base = workloads.batched_layered(nshot=2, nr=24, nz=90, h=5e-3, p=6, dt=0.5e-6, nt=180,
                                     f0=40e3, nrec=3, step_m=0.05, cfg_id=78)
    for sh in base.shots:
        sh.src_k = sh.pz + 10
        sh.rec_k = np.array([sh.pz + 40 + 12 * j for j in range(3)], np.int32)
    base.shots[0].rec_k = np.zeros(0, np.int32)
    _say("receiverless shot", [len(s.rec_k) for s in base.shots])
    lam, mu, rho = gpu_models(base)
    tune = T(tb=4, tbw=8)
    sv = survey(base, ckpt=50, tune=tune)
    assert sv.sizes.trace_elems == 3 * 180
    wav = sv.pack_wavelets([s.wavelet for s in base.shots])
    tr = sv.fwd_model(lam, mu, rho, wav, store_ckpt=True)
    torch.manual_seed(2)
    r = torch.randn(sv.sizes.trace_elems, device=_dev())
    g_b = [t.cpu().numpy() for t in sv.gradient(mu, sv.adjoint_model(lam, mu, rho, wav, r))]
    w1 = copy.copy(base)
    w1.shots = [base.shots[1]]
    sv1 = survey(w1, ckpt=50, tune=tune)
    wav1 = sv1.pack_wavelets([base.shots[1].wavelet])
    tr1 = sv1.fwd_model(lam, mu, rho, wav1, store_ckpt=True)
    assert np.array_equal(sv1.unpack_traces(tr1)[0], sv.unpack_traces(tr)[1])
    g1 = [t.cpu().numpy() for t in sv1.gradient(mu, sv1.adjoint_model(lam, mu, rho, wav1, r))]
    for a, b in zip(g_b[:2], g1[:2]):
        assert np.array_equal(a, b)


def test_largest_grid_forward():
    """The per-shot grid of the 128-shot workload, 532 x 16424 padded cells,
    in the launch shapes tuned for the batched workloads: 150 steps with the
    Ricker wavelet started near its peak and the source 20 rows from the first
    receiver."""
    import paper_2005_00281_amd as P
    w = workloads.make("c5", nshot=1)
    sh = copy.copy(w.shots[0])
    nt = 150
    peak = int(round(1.5 / sh.f0 / sh.dt))
    sh.wavelet = np.ascontiguousarray(sh.wavelet[peak - 60: peak - 60 + nt])
    sh.nt = nt
    sh.src_k = int(sh.rec_k[0]) - 20
    w.shots = [sh]
    _say("largest grid", sh.NR, sh.NZ, nt)
    lam_o, mu_o, rho_o = oracle_models(w, 0, "start")
    d_o = oracle.forward(geom(sh), lam_o, mu_o, rho_o, sh.wavelet)
    assert np.abs(d_o[0]).max() > 1e-3 * np.abs(d_o).max() > 0
    sv = P.Survey(w.shots, (w.NRg, w.NZg), ckpt_every=250)
    sv.set_tune(tb_steps=8, tb_rows=48, tb_waves=16, adj_tb_steps=6, adj_tb_rows=32,
                adj_tb_waves=16, tile_map=0)
    lam, mu, rho = gpu_models(w)
    tr = sv.fwd_model(lam, mu, rho, sv.pack_wavelets([sh.wavelet]))
    d_g = sv.unpack_traces(tr)[0]
    assert rel_l2(d_g, d_o) <= 1e-4, rel_l2(d_g, d_o)


def test_batched_offsets_beyond_int32():
    """48 shots of the 128-shot workload's grid (532 x 16424 padded cells) in
    one batch: each state buffer then holds more than 2^31 floats, so the
    last shots sit at offsets an int32 cannot address.  Their traces must
    equal those of the same shots run alone, bit for bit (150 steps, the
    wavelet started near its peak, the source 20 rows from the first
    receiver), and the last shot's traces equal the oracle's (<= 1e-4)."""
    from concurrent.futures import ThreadPoolExecutor
    import paper_2005_00281_amd as P
    w = workloads.make("c5", nshot=48)
    nt = 150
    shots = []
    for s in w.shots:
        sh = copy.copy(s)
        peak = int(round(1.5 / sh.f0 / sh.dt))
        sh.wavelet = np.ascontiguousarray(sh.wavelet[peak - 60: peak - 60 + nt])
        sh.nt = nt
        sh.src_k = int(sh.rec_k[0]) - 20
        shots.append(sh)
    w.shots = shots
    _say("batched offsets beyond int32", len(shots), shots[0].NR, shots[0].NZ, nt)
    ex = ThreadPoolExecutor(1)
    lo, mo, ro = oracle_models(w, 47, "start")
    f_o = ex.submit(oracle.forward, geom(shots[47]), lo, mo, ro, shots[47].wavelet)
    tune = dict(tb_steps=8, tb_rows=48, tb_waves=16, adj_tb_steps=6, adj_tb_rows=32,
                adj_tb_waves=16, tile_map=0)
    sv = P.Survey(shots, (w.NRg, w.NZg), ckpt_every=250)
    sv.set_tune(**tune)
    assert sv.sizes.fwd_ws_bytes // 8 > 2 ** 31  # floats per state buffer
    lam, mu, rho = gpu_models(w)
    wav = sv.pack_wavelets([sh.wavelet for sh in shots])
    tr = sv.unpack_traces(sv.fwd_model(lam, mu, rho, wav))
    del sv
    torch.cuda.empty_cache()
    for s in (0, 46, 47):
        sv1 = P.Survey([shots[s]], (w.NRg, w.NZg), ckpt_every=250)
        sv1.set_tune(**tune)
        tr1 = sv1.unpack_traces(sv1.fwd_model(lam, mu, rho, sv1.pack_wavelets([shots[s].wavelet])))
        torch.cuda.synchronize()
        assert np.abs(tr1[0]).max() > 0
        assert np.array_equal(tr1[0], tr[s]), s
        del sv1
    d_o = f_o.result()
    ex.shutdown()
    assert rel_l2(tr[47], d_o) <= 1e-4, rel_l2(tr[47], d_o)
