"""Parity of the fourth-order HIP kernels (bhfwi_set_order(4)) with the
oracle's assembled fourth-order operators.

Tolerances as for the second-order path: traces relative L2 <= 1e-4,
gradients <= 1e-3 (all cells and the interior; PML cells alone <= 1e-2),
illumination <= 1e-4; exact equality where the same FP32 arithmetic is
repeated (batched vs single shot).
"""
import copy

import numpy as np
import pytest

import oracle
import workloads
from util import geom, oracle_models, rel_l2
from test_gpu_parity import T, _dev, _multi_shot_workload, _regions, _say, f32, gpu_models

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def survey4(w, ckpt=250, graph=1, full=0, rov=0):
    import paper_2005_00281_amd as P
    sv = P.Survey(w.shots, (w.NRg, w.NZg), ckpt_every=ckpt, order=4)
    sv.set_tune(use_graph=graph, full_history=full, rec_overlap=rov)
    return sv


@pytest.mark.parametrize("graph", [0, 1])
def test_order4_forward_parity_tiny_ragged(graph):
    w = workloads.tiny(nr=40, nz=150, p=6, nt=300)
    sh = w.shots[0]
    _say("order 4 fwd tiny", sh.NR, sh.NZ, "graph", graph)
    lam_o, mu_o, rho_o = oracle_models(w, 0, "start")
    d_o = oracle.forward(geom(sh), lam_o, mu_o, rho_o, sh.wavelet, order=4)
    sv = survey4(w, graph=graph)
    lam, mu, rho = gpu_models(w)
    tr = sv.fwd_model(lam, mu, rho, sv.pack_wavelets([sh.wavelet]))
    torch.cuda.synchronize()
    d_g = sv.unpack_traces(tr)[0]
    assert rel_l2(d_g, d_o) <= 1e-4, rel_l2(d_g, d_o)
    # and it is not the second-order result
    d2 = oracle.forward(geom(sh), lam_o, mu_o, rho_o, sh.wavelet)
    assert rel_l2(d_g, d2) > 1e-2


@pytest.mark.parametrize("ckpt,graph,full,rov", [(37, 1, 0, 0), (300, 0, 0, 0), (37, 1, 1, 0),
                                                (37, 1, 0, 1)])
def test_order4_gradient_parity_tiny(ckpt, graph, full, rov):
    w = workloads.tiny(nr=40, nz=150, p=6, nt=300)
    sh = w.shots[0]
    _say("order 4 grad tiny", ckpt, graph, "full history", full, "overlapped recompute", rov)
    lam_o, mu_o, rho_o = oracle_models(w, 0, "start")
    lt, mt, _ = oracle_models(w, 0, "true")
    d_obs = oracle.forward(geom(sh), lt, mt, rho_o, sh.wavelet, order=4)
    d_o = oracle.forward(geom(sh), lam_o, mu_o, rho_o, sh.wavelet, order=4)
    _, r = oracle.misfit(d_o, d_obs)
    gl_o, gm_o, il_o = oracle.gradient(geom(sh), lam_o, mu_o, rho_o, sh.wavelet, r, seg=50,
                                       order=4)
    sv = survey4(w, ckpt=ckpt, graph=graph, full=full, rov=rov)
    lam, mu, rho = gpu_models(w)
    wav = sv.pack_wavelets([sh.wavelet])
    sv.fwd_model(lam, mu, rho, wav, store_ckpt=True)
    acc = sv.adjoint_model(lam, mu, rho, wav, f32(r.ravel()))
    gl, gm, il = (t.cpu().numpy() for t in sv.gradient(mu, acc))
    reg = _regions(sh, gl.shape)
    errs = {k: (rel_l2(gl[m], gl_o[m]), rel_l2(gm[m], gm_o[m])) for k, m in reg.items()}
    print("[case] rel-L2 (g_lam, g_mu) by region:", errs, "illum", rel_l2(il, il_o))
    assert errs["all"][0] <= 1e-3 and errs["all"][1] <= 1e-3
    assert errs["interior"][0] <= 1e-3 and errs["interior"][1] <= 1e-3
    for k in ("pml_r", "pml_z"):
        assert errs[k][0] <= 1e-2 and errs[k][1] <= 1e-2, (k, errs[k])
    assert rel_l2(il, il_o) <= 1e-4


def test_order4_single_shot_128x512():
    """The 128 x 512 workload (4000 steps, 10 kHz, water-filled hole): every
    trace and the formation gradient."""
    w = workloads.make("c1")
    sh = w.shots[0]
    _say("order 4 c1", sh.NR, sh.NZ, sh.nt)
    lam_o, mu_o, rho_o = oracle_models(w, 0, "start")
    lt, mt, _ = oracle_models(w, 0, "true")
    d_obs = oracle.forward(geom(sh), lt, mt, rho_o, sh.wavelet, order=4)
    d_o = oracle.forward(geom(sh), lam_o, mu_o, rho_o, sh.wavelet, order=4)
    _, r = oracle.misfit(d_o, d_obs)
    gl_o, gm_o, _ = oracle.gradient(geom(sh), lam_o, mu_o, rho_o, sh.wavelet, r, seg=200,
                                    order=4)
    sv = survey4(w)
    lam, mu, rho = gpu_models(w)
    wav = sv.pack_wavelets([sh.wavelet])
    tr = sv.fwd_model(lam, mu, rho, wav, store_ckpt=True)
    d_g = sv.unpack_traces(tr)[0]
    for j in range(d_o.shape[0]):
        assert rel_l2(d_g[j], d_o[j]) <= 1e-4, (j, rel_l2(d_g[j], d_o[j]))
    acc = sv.adjoint_model(lam, mu, rho, wav, f32(r.ravel()))
    gl, gm, _ = (t.cpu().numpy() for t in sv.gradient(mu, acc))
    form = w.mask.astype(bool)
    assert rel_l2(gl[form], gl_o[form]) <= 1e-3 and rel_l2(gm[form], gm_o[form]) <= 1e-3


def test_order4_batched_equals_single_shots():
    """Three shots over one global model with ragged nt and receiver counts:
    the batched fourth-order traces and gradient are the single-shot ones bit
    for bit (gradient: their shot-order sum)."""
    w = _multi_shot_workload()
    _say("order 4 batched", [(s.NR, s.NZ, s.nt) for s in w.shots])
    lam, mu, rho = gpu_models(w)
    sv = survey4(w, ckpt=50)
    wav = sv.pack_wavelets([s.wavelet for s in w.shots])
    tr = sv.fwd_model(lam, mu, rho, wav, store_ckpt=True)
    torch.manual_seed(0)
    r = torch.randn(sv.sizes.trace_elems, device=_dev())
    g_b = [t.cpu().numpy() for t in sv.gradient(mu, sv.adjoint_model(lam, mu, rho, wav, r))]
    tr_b = sv.unpack_traces(tr)
    r_np = r.cpu().numpy()
    sums = [np.zeros((w.NRg, w.NZg), np.float32) for _ in range(3)]
    for s, (off, nrec, nt) in enumerate(sv.trace_slices()):
        w1 = copy.copy(w)
        w1.shots = [w.shots[s]]
        sv1 = survey4(w1, ckpt=50)
        wav1 = sv1.pack_wavelets([w.shots[s].wavelet])
        tr1 = sv1.fwd_model(lam, mu, rho, wav1, store_ckpt=True)
        assert np.array_equal(sv1.unpack_traces(tr1)[0], tr_b[s])
        acc1 = sv1.adjoint_model(lam, mu, rho, wav1, f32(r_np[off: off + nrec * nt]))
        for q, t in enumerate(sv1.gradient(mu, acc1)):
            sums[q] += t.cpu().numpy()
        lo, mo, ro = oracle_models(w, s, "start")
        d_o = oracle.forward(geom(w.shots[s]), lo, mo, ro, w.shots[s].wavelet, order=4)
        assert rel_l2(tr_b[s], d_o) <= 1e-4
    for q in range(3):
        assert np.array_equal(sums[q], g_b[q]), q


def test_order4_rules():
    """Order 3 is rejected, a time step within the second-order bound but not
    the fourth-order one is rejected, and the workspaces are those of order 2."""
    import paper_2005_00281_amd as P
    from paper_2005_00281_amd._lib import BhfwiError
    w = workloads.tiny(nr=20, nz=60, p=4, nt=50)
    _say("order 4 rules")
    sv = P.Survey(w.shots, (w.NRg, w.NZg), ckpt_every=25)
    a2 = sv.sizes.adj_ws_bytes
    with pytest.raises(BhfwiError):
        sv.set_order(3)
    sv.set_order(4)
    assert sv.sizes.adj_ws_bytes == a2
    lam, mu, rho = gpu_models(w)
    wav = sv.pack_wavelets([w.shots[0].wavelet])
    sv.fwd_model(lam, mu, rho, wav, store_ckpt=True)
    sv.set_order(2)
    assert sv.sizes.adj_ws_bytes == a2
    w2 = copy.deepcopy(w)
    sh = w2.shots[0]
    # Courant 0.9 of the second-order limit: fine for order 2, not for order 4
    sh.dt = 0.9 / (sh.vmax * np.sqrt(1 / sh.dr ** 2 + 1 / sh.dz ** 2))
    sv2 = P.Survey(w2.shots, (w2.NRg, w2.NZg), ckpt_every=25)
    with pytest.raises(BhfwiError):
        sv2.set_order(4)


@pytest.mark.parametrize("ckpt,full", [(37, 0), (37, 1)])
def test_order4_density_and_pseudo_hessian_parity(ckpt, full):
    """The density correlation and the pseudo-Hessian of the fourth-order
    adjoint against the assembled oracle: dJ/drho <= 1e-3, H <= 1e-4 relative
    L2; the modulus gradients with the extra outputs within 1e-6 of those
    without."""
    w = workloads.tiny(nr=40, nz=150, p=6, nt=300)
    sh = w.shots[0]
    _say("order 4 density + pseudo-Hessian", ckpt, "full history", full)
    lam_o, mu_o, rho_o = oracle_models(w, 0, "start")
    r = np.random.default_rng(3).standard_normal((len(sh.rec_k), sh.nt))
    gl_o, gm_o, il_o, gr_o, hl_o, hm_o = oracle.gradient(
        geom(sh), lam_o, mu_o, rho_o, sh.wavelet, r, seg=50, density=True, hessian=True,
        order=4)
    sv = survey4(w, ckpt=ckpt, full=full)
    lam, mu, rho = gpu_models(w)
    wav = sv.pack_wavelets([sh.wavelet])
    sv.fwd_model(lam, mu, rho, wav, store_ckpt=True)
    res = f32(r.ravel())
    acc, acc_rho, acc_h = sv.adjoint_model_ex(lam, mu, rho, wav, res, density=True,
                                              hessian=True)
    gl, gm, il = (t.cpu().numpy() for t in sv.gradient(mu, acc))
    gr = sv.gradient_density(rho, acc_rho).cpu().numpy()
    hl, hm = (t.cpu().numpy() for t in sv.gradient_hessian(acc_h))
    acc0 = sv.adjoint_model(lam, mu, rho, wav, res)
    g0 = [t.cpu().numpy() for t in sv.gradient(mu, acc0)]
    torch.cuda.synchronize()
    errs = (rel_l2(gl, gl_o), rel_l2(gm, gm_o), rel_l2(il, il_o), rel_l2(gr, gr_o),
            rel_l2(hl, hl_o), rel_l2(hm, hm_o))
    print("[case] rel-L2 g_lam %.3g g_mu %.3g illum %.3g g_rho %.3g H_lam %.3g H_mu %.3g" % errs,
          flush=True)
    assert errs[0] <= 1e-3 and errs[1] <= 1e-3 and errs[2] <= 1e-4
    assert errs[3] <= 1e-3
    assert errs[4] <= 1e-4 and errs[5] <= 1e-4
    for a, b in zip((gl, gm, il), g0):
        assert rel_l2(a, b) <= 1e-6
    # and it is not the second-order density gradient
    gr2 = oracle.gradient(geom(sh), lam_o, mu_o, rho_o, sh.wavelet, r, seg=50,
                          density=True)[3]
    assert rel_l2(gr, gr2) > 1e-2


def test_order4_joint_iteration_parity():
    """One joint (lambda, mu, rho) iteration at order 4 with the
    pseudo-Hessian diagonal and a radial taper, against the same steps in the
    oracle (step lengths within 1e-2, model changes within 2e-2)."""
    import paper_2005_00281_amd as P
    from paper_2005_00281_amd.fwi import Inversion
    w = workloads.tiny(nr=30, nz=100, p=6, nt=300)
    sh = w.shots[0]
    _say("order 4 joint iteration", sh.NR, sh.NZ, sh.nt)
    g = geom(sh)
    bounds = (1000.0, 7000.0, 300.0, 4500.0)
    rb = (1500.0, 3000.0)
    lam_o, mu_o, rho_o = oracle_models(w, 0, "start")
    lt, mt, rt = oracle_models(w, 0, "true")
    rt = rt * (1.0 + 0.05 * np.random.default_rng(13).standard_normal(rt.shape))
    d_obs = oracle.forward(g, lt, mt, rt, sh.wavelet, order=4)
    _, r_o = oracle.misfit(oracle.forward(g, lam_o, mu_o, rho_o, sh.wavelet, order=4), d_obs)
    gl, gm, il, gr, hl, hm = oracle.gradient(g, lam_o, mu_o, rho_o, sh.wavelet, r_o, seg=50,
                                             density=True, hessian=True, order=4)
    dr = sh.dr
    wt_o = oracle.radial_taper(g.NR, dr, 6 * dr, 12 * dr)
    pr = oracle.precondition_diag(gr, w.mask, 1e-3, diag=il, row_weight=wt_o)
    rho1, ar_o = oracle.update_density(rho_o, pr, w.mask, 0.02, *rb)
    pl = oracle.precondition_diag(gl, w.mask, 1e-3, diag=hl, row_weight=wt_o)
    pm = oracle.precondition_diag(gm, w.mask, 1e-3, diag=hm, row_weight=wt_o)
    l1, m1, a_o = oracle.update(lam_o, mu_o, rho1, pl, pm, w.mask, 0.02,
                                vp_bounds=bounds[:2], vs_bounds=bounds[2:])
    vp_o, vs_o = oracle.velocities(l1, m1, rho1)

    sv = survey4(w, ckpt=50)
    wav = sv.pack_wavelets([sh.wavelet])
    mask = torch.as_tensor(w.mask, device=_dev())
    wt = P.radial_taper(g.NR, dr, 6 * dr, 12 * dr)
    inv = Inversion(sv, f32(w.vp_start), f32(w.vs_start), f32(w.rho), wav, f32(d_obs.ravel()),
                    mask, eta=0.02, bounds=bounds, density=True, rho_bounds=rb,
                    precond="pseudo_hessian", row_weight=wt)
    J0, a = inv.iterate()
    a, ar = a.item(), inv.alpha_rho.item()
    print("[case] alpha %.6g/%.6g alpha_rho %.6g/%.6g" % (a, a_o, ar, ar_o), flush=True)
    assert abs(a - a_o) <= 1e-2 * a_o and abs(ar - ar_o) <= 1e-2 * ar_o
    drho = inv.rho.cpu().numpy() - w.rho.astype(np.float32)
    dvp = inv.vp.cpu().numpy() - w.vp_start.astype(np.float32)
    dvs = inv.vs.cpu().numpy() - w.vs_start.astype(np.float32)
    assert rel_l2(drho, rho1 - w.rho) <= 2e-2
    assert rel_l2(dvp, vp_o - w.vp_start) <= 2e-2 and rel_l2(dvs, vs_o - w.vs_start) <= 2e-2
    Js = [J0.item()] + [inv.iterate()[0].item() for _ in range(3)]
    assert Js[-1] < Js[0], Js


@pytest.mark.parametrize("nr,nz,p,nt", [(40, 150, 6, 301), (5, 18, 3, 7), (24, 70, 0, 41)])
def test_order4_blocks_against_one_step_and_oracle(nr, nz, p, nt):
    """The fourth-order forward and adjoint in two-step blocks (the default)
    against the one-step kernels and the oracle: traces, gradients,
    illumination, the density correlation and the pseudo-Hessian (each extra
    output alone and both together), on a ragged grid with PML, a grid
    smaller than one tile with an odd step count, and a grid without PML."""
    w = workloads.tiny(nr=nr, nz=nz, p=p, nt=nt)
    sh = w.shots[0]
    _say("order 4 blocks", sh.NR, sh.NZ, sh.nt)
    lam_o, mu_o, rho_o = oracle_models(w, 0, "start")
    d_o = oracle.forward(geom(sh), lam_o, mu_o, rho_o, sh.wavelet, order=4)
    r = np.random.default_rng(5).standard_normal(d_o.shape)
    lam, mu, rho = gpu_models(w)
    out = {}
    for steps in (2, 0):
        sv = survey4(w, ckpt=25)
        sv.set_order4_blocks(steps)
        wav = sv.pack_wavelets([sh.wavelet])
        tr = sv.fwd_model(lam, mu, rho, wav, store_ckpt=True)
        res = f32(r.ravel())
        acc = sv.adjoint_model(lam, mu, rho, wav, res)
        x = []
        for dens, hess in ((True, False), (False, True), (True, True)):
            acc_x, acc_rho, acc_h = sv.adjoint_model_ex(lam, mu, rho, wav, res, density=dens,
                                                        hessian=hess)
            x += [t.cpu().numpy() for t in sv.gradient(mu, acc_x)]
            if dens:
                x.append(sv.gradient_density(rho, acc_rho).cpu().numpy())
            if hess:
                x += [t.cpu().numpy() for t in sv.gradient_hessian(acc_h)]
        out[steps] = (sv.unpack_traces(tr)[0], [t.cpu().numpy() for t in sv.gradient(mu, acc)],
                      x)
    torch.cuda.synchronize()
    (d2, g2, x2), (d1, g1, x1) = out[2], out[0]
    gl_o, gm_o, il_o, gr_o, hl_o, hm_o = oracle.gradient(
        geom(sh), lam_o, mu_o, rho_o, sh.wavelet, r, seg=25, density=True, hessian=True,
        order=4)
    print("[case] traces blocked/one-step %.3g, vs oracle %.3g; gradient blocked/one-step %s, "
          "vs oracle %s" % (rel_l2(d2, d1), rel_l2(d2, d_o),
                            [float("%.3g" % rel_l2(a, b)) for a, b in zip(g2, g1)],
                            [float("%.3g" % rel_l2(a, b)) for a, b in zip(g2, (gl_o, gm_o, il_o))]),
          flush=True)
    assert rel_l2(d2, d_o) <= 1e-4
    assert rel_l2(d2, d1) <= 1e-5
    for a, b in zip(g2, g1):
        assert rel_l2(a, b) <= 1e-5
    assert rel_l2(g2[0], gl_o) <= 1e-3 and rel_l2(g2[1], gm_o) <= 1e-3
    assert rel_l2(g2[2], il_o) <= 1e-4
    # extra outputs: blocked against one step, field by field, then the last
    # pass (density and pseudo-Hessian together) against the oracle
    ex = [rel_l2(a, b) for a, b in zip(x2, x1)]
    print("[case] extra outputs blocked/one-step %s" % [float("%.3g" % e) for e in ex],
          flush=True)
    assert len(x2) == len(x1) == 15 and max(ex) <= 1e-5
    gr2, hl2, hm2 = x2[-3:]
    for a, b in zip(x2[-6:-3], g2):  # the modulus gradients do not change
        assert rel_l2(a, b) <= 1e-6
    assert rel_l2(gr2, gr_o) <= 1e-3
    assert rel_l2(hl2, hl_o) <= 1e-4 and rel_l2(hm2, hm_o) <= 1e-4


def test_order4_block_shape_rules():
    """Uncompiled fourth-order block shapes are refused; one step per launch
    and the default two-step blocks are accepted."""
    import paper_2005_00281_amd as P
    from paper_2005_00281_amd._lib import BhfwiError
    w = workloads.tiny(nr=20, nz=60, p=4, nt=50)
    _say("order 4 block shape rules")
    sv = P.Survey(w.shots, (w.NRg, w.NZg), ckpt_every=25, order=4)
    with pytest.raises(BhfwiError):
        sv.set_order4_blocks(3, 32, 16)
    with pytest.raises(BhfwiError):
        sv.set_order4_blocks(2, 48, 16)
    sv.set_order4_blocks(0)
    sv.set_order4_blocks(2, 32, 16)
