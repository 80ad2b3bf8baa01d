"""Invariants of the discrete forward model and closed-form checks of the
elementwise steps (Eq. 3-4, 9-12, preconditioner)."""
import numpy as np

import oracle
import workloads
from util import geom, golden, oracle_models


def test_moduli_and_velocities_closed_form():
    gd = golden("closed_forms.json")["moduli_eq3_eq4"]
    lam, mu = oracle.moduli(np.array([gd["vp"]]), np.array([gd["vs"]]), np.array([gd["rho"]]))
    assert lam[0] == gd["lambda"] and mu[0] == gd["mu"]
    vp, vs = oracle.velocities(lam, mu, np.array([gd["rho"]]))
    assert abs(vp[0] - gd["vp"]) < 1e-9 and abs(vs[0] - gd["vs"]) < 1e-9
    # fluid: mu = 0, lambda = rho c^2
    lam, mu = oracle.moduli(np.array([1500.0]), np.array([0.0]), np.array([1000.0]))
    assert lam[0] == 2.25e9 and mu[0] == 0.0


def test_fluid_normal_stresses_equal_and_wall_shear_zero():
    w = workloads.tiny(nt=200)
    sh = w.shots[0]
    lam, mu, rho = oracle_models(w, 0, "true")
    _, st = oracle.forward(geom(sh), lam, mu, rho, sh.wavelet, return_state=True)
    trr, ttt, tzz, trz = st[2], st[3], st[4], st[5]
    fl = mu == 0
    scale = np.abs(trr).max()
    assert np.abs(trr[fl] - ttt[fl]).max() < 1e-12 * scale
    assert np.abs(trr[fl] - tzz[fl]).max() < 1e-12 * scale
    # tau_rz nodes touching a fluid cell carry zero rigidity: tau_rz stays 0 on the wall
    wall_i = int(np.argmax(~fl[:, 0]))
    assert wall_i > 0 and np.all(trz[wall_i, :] == 0.0)
    assert np.all(trz[0, :] == 0.0) and np.all(st[0][0, :] == 0.0)  # axis


def test_traces_linear_in_source_and_causal():
    w = workloads.tiny(nt=200)
    sh = w.shots[0]
    g = geom(sh)
    lam, mu, rho = oracle_models(w, 0, "true")
    d1 = oracle.forward(g, lam, mu, rho, sh.wavelet)
    d2 = oracle.forward(g, lam, mu, rho, 2.0 * sh.wavelet)
    assert np.array_equal(d2, 2.0 * d1)
    # the staggered stencil moves information by at most one row per step
    for j, kr in enumerate(sh.rec_k):
        dist = abs(int(kr) - sh.src_k)
        assert not d1[j, : dist - 1].any()
        assert d1[j].any()


def test_long_run_bounded_without_pml():
    """Rigid box, no PML, Courant 0.6: 1e5 source-free steps after a Ricker
    excitation; the field amplitude stays of the order of its initial value
    (an unstable scheme grows by many orders of magnitude)."""
    w = workloads.tiny(p=0, nr=20, nz=40)
    sh = w.shots[0]
    vmax = w.vp_true.max()
    dt = 0.6 * sh.dr / vmax
    g = oracle.Geom(sh.nr, sh.nz, 0, 0, sh.dr, sh.dz, dt, 200, sh.f0, vmax, sh.src_k, sh.rec_k)
    lam, mu, rho = oracle_models(w, 0, "true")
    _, st = oracle.forward(g, lam, mu, rho, workloads.ricker(sh.f0, dt, 200), return_state=True)
    a0 = np.abs(st[:6]).max()
    st = oracle.propagate(g, lam, mu, rho, st.ravel(), 100000)
    assert np.isfinite(st).all()
    assert np.abs(st.reshape(14, g.NR, g.NZ)[:6]).max() < 3.0 * a0


def test_precondition_hand_case():
    illum = np.array([4.0, 1.0, 0.0, 100.0])
    mask = np.array([1, 1, 1, 0], np.uint8)
    gl, gm = oracle.precondition(illum, mask, 0.25, np.array([8.0, 2.0, 1.0, 5.0]),
                                 np.array([-4.0, 1.0, 3.0, 5.0]))
    # max over mask cells is 4 -> P = 1/(E + 1)
    assert np.allclose(gl, [8 / 5, 2 / 2, 1 / 1, 0.0]) and np.allclose(gm, [-4 / 5, 1 / 2, 3, 0])


def test_update_hand_case():
    lam = np.array([10.0, 20.0, 5.0])
    mu = np.array([4.0, 8.0, 2.0])
    rho = np.ones(3)
    gl = np.array([1.0, -2.0, 50.0])
    gm = np.array([0.5, 1.0, 50.0])
    mask = np.array([1, 1, 0], np.uint8)
    l2, m2, a = oracle.update(lam, mu, rho, gl, gm, mask, eta=0.1)
    # masked maxima: |gl| 2 / max lam 20 = 0.1; |gm| 1 / max mu 8 = 0.125 -> alpha = 0.1/0.125
    assert abs(a - 0.8) < 1e-15
    assert np.allclose(l2, [10 - 0.8, 20 + 1.6, 5.0]) and np.allclose(m2, [4 - 0.4, 8 - 0.8, 2.0])
    # the velocity box clip: Vs <= 2 caps mu at 4; Vp >= 5 lifts cell 0 to lam + 2 mu = 25,
    # cell 1 keeps lam + 2 mu = 21.6 + 8 = 29.6 inside the box
    l3, m3, _ = oracle.update(lam, mu, rho, gl, gm, mask, eta=0.1, alpha_override=0.8,
                              vp_bounds=(5.0, 100.0), vs_bounds=(0.0, 2.0))
    assert np.allclose(m3, [3.6, 4.0, 2.0]) and np.allclose(l3 + 2 * m3, [25.0, 29.6, 9.0])
