"""Parity at the single-shot workload's full grid (340 x 2088 padded cells) in
the launch shapes its tune-cache entry names (forward 8x64x16 with 8x32x16
PML sub-tiles, adjoint 8x64x16, HIP graphs), in the three history modes the
benchmark can run it in: checkpoints every 250 steps with sequential
recompute (the workload's configuration), the same with the recompute
overlapped on a second stream, and the velocity history of every step kept
instead of checkpoints.

The record is cut to 900 steps (four checkpoint segments, the last one
ragged, so the overlap is exercised) and the source is moved 30 rows above the
third receiver so that the waves reach four receivers inside it (the Ricker
wavelet alone is delayed by 1.5/f0 = 500 steps); the oracle then finishes in
under two minutes.  Tolerances as everywhere: traces relative L2 <= 1e-4, gradients
<= 1e-3, illumination <= 1e-4.

The 64-shot workload and a planner group of the ragged 96-shot workload are
checked the same way at their full sizes and launch shapes, on sampled shots.
"""
import copy
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from util import geom, oracle_models, rel_l2
from test_gpu_parity import _say, f32, gpu_models

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NT = 900


def _bench_tune():
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2005_00281_amd", "tune_cache.json")
    with open(path) as f:
        table = json.load(f)
    key = [k for k in table if k.endswith("|K250|340x2088x8000*1")]
    assert len(key) == 1, key
    return table[key[0]]["tune"]


@pytest.fixture(scope="module")
def full_grid():
    w = copy.copy(workloads.make("c2"))
    sh = copy.copy(w.shots[0])
    sh.nt = NT
    sh.wavelet = sh.wavelet[:NT]
    sh.src_k = int(sh.rec_k[2]) + 30
    w.shots = [sh]
    g = geom(sh)
    lam_o, mu_o, rho_o = oracle_models(w, 0, "start")
    lt, mt, _ = oracle_models(w, 0, "true")
    d_obs = oracle.forward(g, lt, mt, rho_o, sh.wavelet)
    d_o = oracle.forward(g, lam_o, mu_o, rho_o, sh.wavelet)
    _, r = oracle.misfit(d_o, d_obs)
    assert np.abs(r).max() > 1e-3 * np.abs(d_o).max()  # the arrivals are inside the record
    gl_o, gm_o, il_o = oracle.gradient(g, lam_o, mu_o, rho_o, sh.wavelet, r, seg=250)
    return w, r, (d_o, gl_o, gm_o, il_o)


@pytest.mark.parametrize("form", ["checkpoints", "overlapped recompute", "full history"])
def test_full_grid_in_the_benchmark_launch_configuration(full_grid, form):
    import paper_2005_00281_amd as P
    w, r, (d_o, gl_o, gm_o, il_o) = full_grid
    sh = w.shots[0]
    tune = dict(_bench_tune())
    # a cached tune holds kernel choices only; the history mode is set here
    assert "full_history" not in tune and tune["adj_tb_rows"] == 64
    tune.update(full_history=1 if form == "full history" else 0,
                rec_overlap=1 if form == "overlapped recompute" else 0)
    _say("full grid", form, sh.NR, sh.NZ, NT, tune)
    sv = P.Survey(w.shots, (w.NRg, w.NZg), ckpt_every=250)
    sv.set_tune(**tune)
    assert sv.kernel_shapes()["adj"] == (8, 64, 16)
    lam, mu, rho = gpu_models(w)
    wav = sv.pack_wavelets([sh.wavelet])
    tr = sv.fwd_model(lam, mu, rho, wav, store_ckpt=True)
    d_g = sv.unpack_traces(tr)[0]
    assert rel_l2(d_g, d_o) <= 1e-4, rel_l2(d_g, d_o)
    strong = [j for j in range(d_o.shape[0]) if np.abs(d_o[j]).max() > 1e-2 * np.abs(d_o).max()]
    assert len(strong) >= 4
    for j in strong:
        assert rel_l2(d_g[j], d_o[j]) <= 1e-4, (j, rel_l2(d_g[j], d_o[j]))
    acc = sv.adjoint_model(lam, mu, rho, wav, f32(r.ravel()))
    gl, gm, il = (t.cpu().numpy() for t in sv.gradient(mu, acc))
    torch.cuda.synchronize()
    form = w.mask.astype(bool)
    errs = (rel_l2(gl, gl_o), rel_l2(gm, gm_o), rel_l2(gl[form], gl_o[form]),
            rel_l2(gm[form], gm_o[form]), rel_l2(il, il_o))
    print("[case] full grid rel-L2 g_lam %.3g g_mu %.3g (formation %.3g %.3g) illum %.3g" % errs)
    assert max(errs[:4]) <= 1e-3 and errs[4] <= 1e-4


@pytest.mark.parametrize("full", [1, 0])
def test_full_grid_order4_blocks_against_one_step(full_grid, full):
    """The fourth-order single-shot benchmark's configuration (two-step blocks;
    full velocity history, and checkpoints every 250 steps) on the full grid
    against the one-step kernels, whose parity with the fourth-order oracle is
    checked on the smaller grids (the assembled oracle is too slow at this
    size): traces and illumination within 1e-5, the modulus gradients within
    1e-4.  The gradients are zero-lag correlations summed in FP32 over 900
    steps in two groupings (per launch in registers against per step in
    memory); with the full history they differ by 3.0e-5 (g_mu) and 2.6e-6
    (g_lambda) of their norms here, against about 1e-6 on the small grids, so
    the bar is set at 1e-4, ten times inside the 1e-3 oracle bar."""
    import paper_2005_00281_amd as P
    w, r, _ = full_grid
    sh = w.shots[0]
    _say("full grid order 4", sh.NR, sh.NZ, NT, "full history", full)
    lam, mu, rho = gpu_models(w)
    out = {}
    for steps in (2, 0):
        sv = P.Survey(w.shots, (w.NRg, w.NZg), ckpt_every=250, order=4)
        sv.set_tune(full_history=full)
        sv.set_order4_blocks(steps)
        wav = sv.pack_wavelets([sh.wavelet])
        tr = sv.fwd_model(lam, mu, rho, wav, store_ckpt=True)
        acc = sv.adjoint_model(lam, mu, rho, wav, f32(r.ravel()))
        out[steps] = [sv.unpack_traces(tr)[0]] + [t.cpu().numpy() for t in sv.gradient(mu, acc)]
        del sv
    torch.cuda.synchronize()
    errs = [rel_l2(a, b) for a, b in zip(out[2], out[0])]
    print("[case] full grid order 4 blocked/one-step: traces %.3g g_lam %.3g g_mu %.3g "
          "illum %.3g" % tuple(errs), flush=True)
    assert np.abs(out[0][0]).max() > 0
    assert errs[0] <= 1e-5 and errs[3] <= 1e-5, errs
    assert errs[1] <= 1e-4 and errs[2] <= 1e-4, errs


def _c3_tune():
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2005_00281_amd", "tune_cache.json")
    with open(path) as f:
        table = json.load(f)
    key = [k for k in table if k.endswith("|K250|276x4136x8000*64")]
    assert len(key) == 1, key
    return table[key[0]]["tune"]


def test_64_shot_grids_sampled_shots_against_oracle():
    """The 64-shot workload at its full size (64 windows of 276 x 4136 padded
    cells over one global model) batched in the launch shapes of its
    tune-cache entry (forward 8x48x16, adjoint 6x32x16, XCD-chunked tile
    order, HIP graphs).  The record is cut to 200 steps with the wavelet
    started 60 samples before its peak and the source 20 rows from the first
    receiver, so that the oracle can follow sampled shots one by one: traces
    of shots 0, 31 and 63 against it (<= 1e-4), and, with a residual on shot
    63 only, the gradient: zero outside that shot's window and, inside it,
    the oracle's gradient of that shot (<= 1e-3)."""
    from concurrent.futures import ThreadPoolExecutor
    import paper_2005_00281_amd as P
    w = copy.copy(workloads.make("c3"))
    nt, sampled, gshot = 200, (0, 31, 63), 63
    shots = []
    for s in w.shots:
        sh = copy.copy(s)
        peak = int(round(1.5 / sh.f0 / sh.dt))
        sh.wavelet = np.ascontiguousarray(sh.wavelet[peak - 60: peak - 60 + nt])
        sh.nt = nt
        sh.src_k = int(sh.rec_k[0]) - 20
        shots.append(sh)
    w.shots = shots
    _say("64-shot grids, sampled shots", len(shots), shots[0].NR, shots[0].NZ, nt)
    r_g = np.random.default_rng(64).standard_normal((len(shots[gshot].rec_k), nt))

    def fwd(s):
        lo, mo, ro = oracle_models(w, s, "start")
        return oracle.forward(geom(shots[s]), lo, mo, ro, shots[s].wavelet)

    def grad():
        lo, mo, ro = oracle_models(w, gshot, "start")
        return oracle.gradient(geom(shots[gshot]), lo, mo, ro, shots[gshot].wavelet, r_g,
                               seg=100)

    with ThreadPoolExecutor(4) as ex:
        fs = {s: ex.submit(fwd, s) for s in sampled}
        fg = ex.submit(grad)
        d_o = {s: f.result() for s, f in fs.items()}
        gl_o, gm_o, _ = fg.result()

    sv = P.Survey(shots, (w.NRg, w.NZg), ckpt_every=100)
    sv.set_tune(**_c3_tune())
    ks = sv.kernel_shapes()
    assert tuple(ks["fwd"]) == (8, 48, 16) and tuple(ks["adj"]) == (6, 32, 16)
    lam, mu, rho = gpu_models(w)
    wav = sv.pack_wavelets([sh.wavelet for sh in shots])
    tr = sv.unpack_traces(sv.fwd_model(lam, mu, rho, wav, store_ckpt=True))
    errs = {s: rel_l2(tr[s], d_o[s]) for s in sampled}
    print("[case] traces rel-L2 %s" % errs, flush=True)
    for s in sampled:
        assert np.abs(d_o[s]).max() > 0 and errs[s] <= 1e-4
    res = np.zeros(sv.sizes.trace_elems, np.float32)
    off, nrec, ntt = sv.trace_slices()[gshot]
    res[off: off + nrec * ntt] = r_g.ravel()
    acc = sv.adjoint_model(lam, mu, rho, wav, f32(res))
    gl, gm, _ = (t.cpu().numpy() for t in sv.gradient(mu, acc))
    sh = shots[gshot]
    inside = np.zeros(gl.shape, bool)
    inside[: sh.NR, sh.win_k0: sh.win_k0 + sh.NZ] = True
    assert not gl[~inside].any() and not gm[~inside].any()
    e = (rel_l2(w.window(gl, gshot), gl_o), rel_l2(w.window(gm, gshot), gm_o))
    print("[case] shot %d gradient rel-L2 g_lam %.2e g_mu %.2e" % ((gshot,) + e), flush=True)
    assert e[0] <= 1e-3 and e[1] <= 1e-3


def test_ragged_96_shot_group_sampled_shots_against_oracle():
    """The ragged 96-shot workload at full size: the first group the HBM
    planner makes of it (48 shots of mixed grids, frequencies, time steps and
    records over one global model) in the launch shapes of its tune-cache
    entry.  Records cut to 300 steps (wavelet started 60 samples before its
    peak, source 20 rows from the first receiver): traces of the group's
    smallest and largest shot against the oracle (<= 1e-4), and with a
    residual on the smallest shot only, its gradient in its window (<= 1e-3)
    and zero outside."""
    from concurrent.futures import ThreadPoolExecutor
    import paper_2005_00281_amd as P
    from paper_2005_00281_amd import plan as planner
    w = copy.copy(workloads.make("c4"))
    budget = 0.8 * torch.cuda.get_device_properties(0).total_memory
    pl = planner.plan(w.shots, budget, ckpt_every=w.meta.get("ckpt"))
    group = pl.groups[0]
    sv0 = P.Survey([w.shots[s] for s in group], (w.NRg, w.NZg), ckpt_every=pl.ckpt_every[0])
    key = sv0.shape_key()
    del sv0
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2005_00281_amd", "tune_cache.json")
    with open(path) as f:
        tune = json.load(f)[key]["tune"]
    nt = 300
    shots = []
    for s in group:
        sh = copy.copy(w.shots[s])
        peak = int(round(1.5 / sh.f0 / sh.dt))
        sh.wavelet = np.ascontiguousarray(sh.wavelet[peak - 60: peak - 60 + nt])
        sh.nt = nt
        sh.src_k = int(sh.rec_k[0]) - 20
        shots.append(sh)
    w.shots = shots
    cells = [sh.NR * sh.NZ for sh in shots]
    small, large = int(np.argmin(cells)), int(np.argmax(cells))
    _say("ragged group, sampled shots", len(shots), (shots[small].NR, shots[small].NZ),
         (shots[large].NR, shots[large].NZ), nt, tune)
    r_g = np.random.default_rng(96).standard_normal((len(shots[small].rec_k), nt))

    def fwd(s):
        lo, mo, ro = oracle_models(w, s, "start")
        return oracle.forward(geom(shots[s]), lo, mo, ro, shots[s].wavelet)

    def grad():
        lo, mo, ro = oracle_models(w, small, "start")
        return oracle.gradient(geom(shots[small]), lo, mo, ro, shots[small].wavelet, r_g,
                               seg=100)

    with ThreadPoolExecutor(3) as ex:
        fs = {s: ex.submit(fwd, s) for s in (small, large)}
        fg = ex.submit(grad)
        d_o = {s: f.result() for s, f in fs.items()}
        gl_o, gm_o, _ = fg.result()

    sv = P.Survey(shots, (w.NRg, w.NZg), ckpt_every=100)
    sv.set_tune(**tune)
    lam, mu, rho = gpu_models(w)
    wav = sv.pack_wavelets([sh.wavelet for sh in shots])
    tr = sv.unpack_traces(sv.fwd_model(lam, mu, rho, wav, store_ckpt=True))
    errs = {s: rel_l2(tr[s], d_o[s]) for s in (small, large)}
    print("[case] traces rel-L2 %s" % errs, flush=True)
    for s in (small, large):
        assert np.abs(d_o[s]).max() > 0 and errs[s] <= 1e-4
    res = np.zeros(sv.sizes.trace_elems, np.float32)
    off, nrec, ntt = sv.trace_slices()[small]
    res[off: off + nrec * ntt] = r_g.ravel()
    acc = sv.adjoint_model(lam, mu, rho, wav, f32(res))
    gl, gm, _ = (t.cpu().numpy() for t in sv.gradient(mu, acc))
    sh = shots[small]
    inside = np.zeros(gl.shape, bool)
    inside[: sh.NR, sh.win_k0: sh.win_k0 + sh.NZ] = True
    assert not gl[~inside].any() and not gm[~inside].any()
    e = (rel_l2(w.window(gl, small), gl_o), rel_l2(w.window(gm, small), gm_o))
    print("[case] smallest shot gradient rel-L2 g_lam %.2e g_mu %.2e" % e, flush=True)
    assert e[0] <= 1e-3 and e[1] <= 1e-3
