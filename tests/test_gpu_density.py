"""Parity of the density gradient (joint inversion, an extension of the
paper's fixed density) on the HIP path with the FP64 oracle.

The adjoint kernels accumulate the density correlation in a summed-by-parts
form (increment of the adjoint velocity times the stored velocity), the
oracle in the direct form (adjoint velocity times the velocity increment);
they agree to FP32 rounding.  Tolerances as for the modulus gradients:
relative L2 <= 1e-3 overall and on the interior, <= 1e-2 on PML cells alone.
"""
import copy

import numpy as np
import pytest

import oracle
import workloads
from util import geom, oracle_models, rel_l2
from test_gpu_parity import T, _dev, _regions, _say, f32, gpu_models, survey

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DENSITY_TUNES = [T(1, 1, 1), T(4, 4, 0), T(64, 8, 0), T(tb=4), T(tb=3, graph=0),
                 T(tb=6, tbr=24, tbw=8), T(tb=8, tbr=32, tbw=16),
                 T(tb=6, tbr=48, tbw=16, atb=6, atbr=32, atbw=16),
                 T(tb=6, tbr=32, tbw=16, atb=1, rows=2),
                 T(tb=8, tbr=64, tbw=16, atb=6, atbr=48, atbw=16),
                 T(tb=8, tbr=48, tbw=16, atb=8, atbr=48, atbw=16, graph=0)]


def _observed_with_density_contrast(w, s=0, seed=11):
    """Data of the true moduli over a density 5% off the starting one."""
    sh = w.shots[s]
    lt, mt, rt = oracle_models(w, s, "true")
    rt = rt * (1.0 + 0.05 * np.random.default_rng(seed).standard_normal(rt.shape))
    return oracle.forward(geom(sh), lt, mt, rt, sh.wavelet)


def _density_case(w, ckpt, seg_oracle, tune=None):
    sh = w.shots[0]
    lam_o, mu_o, rho_o = oracle_models(w, 0, "start")
    d_obs = _observed_with_density_contrast(w)
    _, r = oracle.misfit(oracle.forward(geom(sh), lam_o, mu_o, rho_o, sh.wavelet), d_obs)
    gl_o, gm_o, il_o, gr_o = oracle.gradient(geom(sh), lam_o, mu_o, rho_o, sh.wavelet, r,
                                             seg=seg_oracle, density=True)
    sv = survey(w, ckpt=ckpt, tune=tune)
    lam, mu, rho = gpu_models(w)
    wav = sv.pack_wavelets([sh.wavelet])
    sv.fwd_model(lam, mu, rho, wav, store_ckpt=True)
    res = f32(r.ravel())
    acc, acc_rho = sv.adjoint_model_density(lam, mu, rho, wav, res)
    g_rho = sv.gradient_density(rho, acc_rho)
    g = [t.cpu().numpy() for t in sv.gradient(mu, acc)]
    acc0 = sv.adjoint_model(lam, mu, rho, wav, res)
    g0 = [t.cpu().numpy() for t in sv.gradient(mu, acc0)]
    torch.cuda.synchronize()
    return g_rho.cpu().numpy(), g, g0, (gl_o, gm_o, il_o, gr_o)


@pytest.mark.parametrize("tune", DENSITY_TUNES)
def test_density_gradient_parity_tiny(tune):
    w = workloads.tiny(nr=40, nz=150, p=6, nt=300)
    _say("density grad tiny", tune)
    gr, g, g0, (gl_o, gm_o, il_o, gr_o) = _density_case(w, ckpt=37, seg_oracle=50, tune=tune)
    reg = _regions(w.shots[0], gr.shape)
    errs = {k: rel_l2(gr[m], gr_o[m]) for k, m in reg.items()}
    print("rel-L2 g_rho by region:", errs)
    assert errs["all"] <= 1e-3 and errs["interior"] <= 1e-3, errs
    assert errs["pml_r"] <= 1e-2 and errs["pml_z"] <= 1e-2, errs
    # the modulus gradients of the same pass are those of the plain adjoint
    for a, b in zip(g, g0):
        assert rel_l2(a, b) <= 1e-6, rel_l2(a, b)
    assert rel_l2(g[0], gl_o) <= 1e-3 and rel_l2(g[1], gm_o) <= 1e-3


def test_density_gradient_parity_single_shot_128x512():
    """The 128 x 512 workload (4000 steps, 10 kHz, water-filled hole)."""
    w = workloads.make("c1")
    _say("density grad c1")
    gr, g, g0, (gl_o, gm_o, il_o, gr_o) = _density_case(w, ckpt=250, seg_oracle=200)
    form = w.mask.astype(bool)
    assert rel_l2(gr[form], gr_o[form]) <= 1e-3, rel_l2(gr[form], gr_o[form])
    assert rel_l2(gr, gr_o) <= 1e-3, rel_l2(gr, gr_o)


def test_density_gradient_batched_equals_single_shots():
    """Three shots over one global model (ragged nt and receiver counts):
    the batched density gradient is the shot-order sum of the single-shot
    ones, bit for bit, and each shot matches the oracle."""
    from test_gpu_parity import _multi_shot_workload
    w = _multi_shot_workload()
    tune = T(tb=4, tbr=32, tbw=8)
    _say("density batched 3 shots", [(s.NR, s.NZ, s.nt) for s in w.shots])
    lam, mu, rho = gpu_models(w)
    sv = survey(w, ckpt=50, tune=tune)
    wav = sv.pack_wavelets([s.wavelet for s in w.shots])
    sv.fwd_model(lam, mu, rho, wav, store_ckpt=True)
    torch.manual_seed(0)
    r = torch.randn(sv.sizes.trace_elems, device=_dev())
    _, acc_rho = sv.adjoint_model_density(lam, mu, rho, wav, r)
    g_b = sv.gradient_density(rho, acc_rho).cpu().numpy()
    r_np = r.cpu().numpy()
    total = np.zeros((w.NRg, w.NZg), np.float32)
    for s, (off, nrec, nt) in enumerate(sv.trace_slices()):
        w1 = copy.copy(w)
        w1.shots = [w.shots[s]]
        sv1 = survey(w1, ckpt=50, tune=tune)
        wav1 = sv1.pack_wavelets([w.shots[s].wavelet])
        sv1.fwd_model(lam, mu, rho, wav1, store_ckpt=True)
        rs = r_np[off: off + nrec * nt]
        _, a1 = sv1.adjoint_model_density(lam, mu, rho, wav1, f32(rs))
        g1 = sv1.gradient_density(rho, a1).cpu().numpy()
        total += g1
        lo, mo, ro = oracle_models(w, s, "start")
        _, _, _, gro = oracle.gradient(geom(w.shots[s]), lo, mo, ro, w.shots[s].wavelet,
                                       rs.astype(np.float64), seg=50, density=True)
        win = w.window(g1, s)
        assert rel_l2(win, gro) <= 1e-3, (s, rel_l2(win, gro))
    assert np.array_equal(total, g_b)


def test_joint_velocity_density_autograd():
    """Moduli and BoreholeFWI with vp, vs and rho all requiring grad: dJ/drho
    collects the moduli's share (chain-rule kernel) and the buoyancy part
    (density correlation) and matches the oracle's sum (<= 1e-3); dJ/dvp and
    dJ/dvs are unchanged by asking for it."""
    import paper_2005_00281_amd as P
    w = workloads.tiny(nr=30, nz=100, p=6, nt=300)
    sh = w.shots[0]
    _say("joint vp vs rho autograd", sh.NR, sh.NZ)
    lam_o, mu_o, rho_o = oracle_models(w, 0, "start")
    d_obs = _observed_with_density_contrast(w, seed=12)
    _, r_o = oracle.misfit(oracle.forward(geom(sh), lam_o, mu_o, rho_o, sh.wavelet), d_obs)
    gl_o, gm_o, _, grb_o = oracle.gradient(geom(sh), lam_o, mu_o, rho_o, sh.wavelet, r_o,
                                           seg=64, density=True)
    gvp_o, gvs_o, grm_o = oracle.moduli_grad(w.vp_start, w.vs_start, w.rho, gl_o, gm_o,
                                             density=True)

    sv = survey(w, ckpt=64)
    wav = sv.pack_wavelets([sh.wavelet])
    obs = f32(d_obs.ravel())
    vp = f32(w.vp_start).requires_grad_(True)
    vs = f32(w.vs_start).requires_grad_(True)
    rho = f32(w.rho).requires_grad_(True)
    lam, mu = P.Moduli.apply(vp, vs, rho)
    tr = P.BoreholeFWI.apply(lam, mu, sv, rho, wav)
    loss = 0.5 * ((tr - obs).double() ** 2).sum()
    loss.backward()
    assert rel_l2(vp.grad.cpu().numpy(), gvp_o) <= 1e-3
    assert rel_l2(vs.grad.cpu().numpy(), gvs_o) <= 1e-3
    assert rel_l2(rho.grad.cpu().numpy(), grm_o + grb_o) <= 1e-3, \
        rel_l2(rho.grad.cpu().numpy(), grm_o + grb_o)
    # the chain-rule kernel's density share on its own, same FP32 inputs
    rng = np.random.default_rng(5)
    gl, gm = rng.standard_normal(w.vp_start.shape), rng.standard_normal(w.vp_start.shape)
    _, _, c = P.moduli_grad(f32(w.vp_start), f32(w.vs_start), f32(w.rho), f32(gl), f32(gm),
                            density=True)
    _, _, co = oracle.moduli_grad(w.vp_start.astype(np.float32), w.vs_start.astype(np.float32),
                                  w.rho.astype(np.float32), gl.astype(np.float32),
                                  gm.astype(np.float32), density=True)
    assert rel_l2(c.cpu().numpy(), co) <= 1e-6
