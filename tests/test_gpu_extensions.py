"""Parity of the preconditioner and joint-inversion extensions on the HIP
path with the FP64 oracle: the virtual-source pseudo-Hessian diagonal of the
adjoint pass, the general diagonal preconditioner with a radial taper, the
density step, and a whole joint iteration through Inversion.

Tolerances: pseudo-Hessian relative L2 <= 1e-4 (a sum of squares of the
forward wavefield, like the illumination); elementwise steps on identical
FP32 inputs <= 1e-6; one joint iteration: the model change within 2e-2 of
the oracle's (the step-length tolerance of the line-search iteration test).
"""
import numpy as np
import pytest

import oracle
import workloads
from util import geom, oracle_models, rel_l2
from test_gpu_parity import T, _dev, _say, f32, gpu_models, survey

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HESSIAN_TUNES = [T(1, 1, 1), T(4, 4, 0), T(tb=4), T(tb=6, tbr=24, tbw=8, graph=0),
                 T(tb=8, tbr=64, tbw=16, atb=6, atbr=48, atbw=16),
                 T(tb=6, tbr=32, tbw=16, atb=1, rows=2)]


@pytest.mark.parametrize("tune", HESSIAN_TUNES)
@pytest.mark.parametrize("density", [False, True])
def test_pseudo_hessian_parity(tune, density):
    w = workloads.tiny(nr=40, nz=150, p=6, nt=300)
    sh = w.shots[0]
    _say("pseudo-Hessian", tune, "density", density)
    lam_o, mu_o, rho_o = oracle_models(w, 0, "start")
    r = np.random.default_rng(3).standard_normal((len(sh.rec_k), sh.nt))
    out = oracle.gradient(geom(sh), lam_o, mu_o, rho_o, sh.wavelet, r, seg=50, density=True,
                          hessian=True)
    hl_o, hm_o, gr_o = out[4], out[5], out[3]
    sv = survey(w, ckpt=37, tune=tune)
    lam, mu, rho = gpu_models(w)
    wav = sv.pack_wavelets([sh.wavelet])
    sv.fwd_model(lam, mu, rho, wav, store_ckpt=True)
    res = f32(r.ravel())
    acc, acc_rho, acc_h = sv.adjoint_model_ex(lam, mu, rho, wav, res, density=density,
                                              hessian=True)
    hl, hm = (t.cpu().numpy() for t in sv.gradient_hessian(acc_h))
    g = [t.cpu().numpy() for t in sv.gradient(mu, acc)]
    if density:
        gr = sv.gradient_density(rho, acc_rho).cpu().numpy()
    acc0 = sv.adjoint_model(lam, mu, rho, wav, res)
    g0 = [t.cpu().numpy() for t in sv.gradient(mu, acc0)]
    torch.cuda.synchronize()
    print("[case] rel-L2 H_lambda %.3g H_mu %.3g" % (rel_l2(hl, hl_o), rel_l2(hm, hm_o)))
    assert rel_l2(hl, hl_o) <= 1e-4 and rel_l2(hm, hm_o) <= 1e-4
    for a, b in zip(g, g0):
        assert rel_l2(a, b) <= 1e-6
    if density:
        assert rel_l2(gr, gr_o) <= 1e-3


def test_precondition_diag_taper_and_density_step_parity():
    import paper_2005_00281_amd as P
    _say("precondition_diag, radial taper, density step")
    w = workloads.tiny()
    sv = survey(w)
    rng = np.random.default_rng(7)
    shp = (w.NRg, w.NZg)
    d = rng.uniform(0, 5, shp).astype(np.float32)
    g = rng.standard_normal(shp).astype(np.float32)
    mask = w.mask
    dr = w.shots[0].dr
    wt = P.radial_taper(shp[0], dr, 3 * dr, 9 * dr)
    wt_o = oracle.radial_taper(shp[0], dr, 3 * dr, 9 * dr)
    assert np.abs(wt.cpu().numpy() - wt_o).max() <= 1e-6
    mk = torch.as_tensor(mask, device=_dev())
    for diag, roww in ((d, None), (None, wt_o), (d, wt_o)):
        tg = f32(g)
        gpg = torch.zeros((), dtype=torch.float64, device=_dev())
        sv.precondition_diag(tg, mk, 1e-3, f32(diag) if diag is not None else None,
                             f32(roww) if roww is not None else None, gpg=gpg)
        want, gpg_o = oracle.precondition_diag(
            g, mask, 1e-3, diag=diag,
            row_weight=roww.astype(np.float32) if roww is not None else None, return_gpg=True)
        assert rel_l2(tg.cpu().numpy(), want) <= 1e-6
        assert abs(gpg.item() - gpg_o) <= 1e-6 * abs(gpg_o)
    rho = rng.uniform(1800, 2800, shp).astype(np.float32)
    gr = rng.standard_normal(shp).astype(np.float32)
    trho = f32(rho)
    a = sv.update_density(trho, f32(gr), mk, 0.02, 1900.0, 2700.0)
    r_o, a_o = oracle.update_density(rho, gr, mask, 0.02, 1900.0, 2700.0)
    assert abs(a.item() - a_o) <= 1e-6 * a_o
    assert rel_l2(trho.cpu().numpy(), r_o) <= 1e-6


@pytest.mark.parametrize("precond", ["illum", "pseudo_hessian"])
def test_joint_iteration_parity(precond):
    """One joint (lambda, mu, rho) iteration with the chosen diagonal and a
    radial taper, against the same steps in the FP64 oracle."""
    import paper_2005_00281_amd as P
    from paper_2005_00281_amd.fwi import Inversion
    w = workloads.tiny(nr=30, nz=100, p=6, nt=300)
    sh = w.shots[0]
    _say("joint iteration", precond, sh.NR, sh.NZ, sh.nt)
    g = geom(sh)
    bounds = (1000.0, 7000.0, 300.0, 4500.0)
    rb = (1500.0, 3000.0)
    lam_o, mu_o, rho_o = oracle_models(w, 0, "start")
    lt, mt, rt = oracle_models(w, 0, "true")
    rt = rt * (1.0 + 0.05 * np.random.default_rng(13).standard_normal(rt.shape))
    d_obs = oracle.forward(g, lt, mt, rt, sh.wavelet)
    _, r_o = oracle.misfit(oracle.forward(g, lam_o, mu_o, rho_o, sh.wavelet), d_obs)
    gl, gm, il, gr, hl, hm = oracle.gradient(g, lam_o, mu_o, rho_o, sh.wavelet, r_o, seg=50,
                                             density=True, hessian=True)
    dr = sh.dr
    wt_o = oracle.radial_taper(g.NR, dr, 6 * dr, 12 * dr)
    dl, dm = (hl, hm) if precond == "pseudo_hessian" else (il, il)
    pr = oracle.precondition_diag(gr, w.mask, 1e-3, diag=il, row_weight=wt_o)
    rho1, ar_o = oracle.update_density(rho_o, pr, w.mask, 0.02, *rb)
    pl = oracle.precondition_diag(gl, w.mask, 1e-3, diag=dl, row_weight=wt_o)
    pm = oracle.precondition_diag(gm, w.mask, 1e-3, diag=dm, row_weight=wt_o)
    l1, m1, a_o = oracle.update(lam_o, mu_o, rho1, pl, pm, w.mask, 0.02,
                                vp_bounds=bounds[:2], vs_bounds=bounds[2:])
    vp_o, vs_o = oracle.velocities(l1, m1, rho1)

    sv = survey(w, ckpt=50, tune=T(tb=4, tbw=8))
    wav = sv.pack_wavelets([sh.wavelet])
    rho = f32(w.rho)
    mask = torch.as_tensor(w.mask, device=_dev())
    wt = P.radial_taper(g.NR, dr, 6 * dr, 12 * dr)
    inv = Inversion(sv, f32(w.vp_start), f32(w.vs_start), rho, wav, f32(d_obs.ravel()), mask,
                    eta=0.02, bounds=bounds, density=True, rho_bounds=rb, precond=precond,
                    row_weight=wt)
    J0, a = inv.iterate()
    a, ar = a.item(), inv.alpha_rho.item()
    print("[case] alpha %.6g/%.6g alpha_rho %.6g/%.6g" % (a, a_o, ar, ar_o), flush=True)
    assert abs(a - a_o) <= 1e-2 * a_o and abs(ar - ar_o) <= 1e-2 * ar_o
    drho_o = rho1 - w.rho
    drho = inv.rho.cpu().numpy() - w.rho.astype(np.float32)
    dvp_o, dvs_o = vp_o - w.vp_start, vs_o - w.vs_start
    dvp = inv.vp.cpu().numpy() - w.vp_start.astype(np.float32)
    dvs = inv.vs.cpu().numpy() - w.vs_start.astype(np.float32)
    assert rel_l2(drho, drho_o) <= 2e-2, rel_l2(drho, drho_o)
    assert rel_l2(dvp, dvp_o) <= 2e-2 and rel_l2(dvs, dvs_o) <= 2e-2
    # next to the wall (the hole is 4 cells wide) the taper leaves the model
    # untouched: rows 4 and 5 lie inside r0 = 6 dr
    near = np.zeros_like(w.mask, bool)
    near[:6, :] = True
    near &= w.mask.astype(bool)
    assert near.any()
    assert not drho[near].any()
    # (the velocities pass through the moduli and back: FP32 rounding only)
    assert np.abs(dvp[near]).max() <= 1e-2 and np.abs(dvs[near]).max() <= 1e-2
    # and the joint iterations keep lowering the misfit
    Js = [J0.item()] + [inv.iterate()[0].item() for _ in range(3)]
    assert Js[-1] < Js[0], Js
