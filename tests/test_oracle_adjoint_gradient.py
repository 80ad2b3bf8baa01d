"""Pins of the oracle's adjoint (Eq. 6, read as the exact discrete transpose)
and of its gradient (Eq. 7-8) against brute force.

A sign error, a dropped PML or 1/r term in the transpose, a wrong time
alignment of the correlation or a wrong harmonic-mean chain rule each break
one of these checks.
"""
import numpy as np
import pytest

import oracle
import workloads
from util import geom, oracle_models


def _tiny(**kw):
    w = workloads.tiny(**kw)
    return w, w.shots[0], geom(w.shots[0])


@pytest.mark.parametrize("pml,fluid", [(6, True), (0, True), (5, False)])
def test_state_dot_product(pml, fluid):
    """<F x, y> == <x, F^T y> for 25 source-free steps on the full state
    (fields and PML memory variables)."""
    w, sh, g = _tiny(p=pml, fluid=fluid, nr=18, nz=30)
    lam, mu, rho = oracle_models(w, 0, "start")
    rng = np.random.default_rng(3)
    n = 14 * g.NR * g.NZ
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    Fx = oracle.propagate(g, lam, mu, rho, x, 25)
    Fty = oracle.propagate(g, lam, mu, rho, y, 25, adjoint=True)
    a, b = float(Fx @ y), float(x @ Fty)
    assert abs(a - b) <= 1e-12 * max(abs(a), np.linalg.norm(Fx) * np.linalg.norm(y) * 1e-3)


def test_source_to_trace_dot_product():
    """<F w, r> == <w, F^T r> for the wavelet -> traces map (source injection,
    recording and every propagation term)."""
    w, sh, g = _tiny()
    lam, mu, rho = oracle_models(w, 0, "true")
    rng = np.random.default_rng(4)
    wv = rng.standard_normal(g.nt)
    r = rng.standard_normal((len(sh.rec_k), g.nt))
    d = oracle.forward(g, lam, mu, rho, wv)
    wa = oracle.source_adjoint(g, lam, mu, rho, r)
    a, b = float((d * r).sum()), float(wv @ wa)
    assert abs(a - b) <= 1e-12 * abs(a)


def _fd_setup(nr=12, nz=24, p=4, nt=150):
    w, sh, g = _tiny(nr=nr, nz=nz, p=p, nt=nt)
    lam, mu, rho = oracle_models(w, 0, "start")
    lt, mt, _ = oracle_models(w, 0, "true")
    dobs = oracle.forward(g, lt, mt, rho, sh.wavelet)

    def J(l, m):
        return oracle.misfit(oracle.forward(g, l, m, rho, sh.wavelet), dobs)[0]

    J0, res = oracle.misfit(oracle.forward(g, lam, mu, rho, sh.wavelet), dobs)
    gl, gm, il = oracle.gradient(g, lam, mu, rho, sh.wavelet, res, seg=37)
    return w, g, lam, mu, rho, J, gl, gm, il


@pytest.mark.slow
def test_gradient_matches_central_differences_every_cell():
    """dJ/dlambda and dJ/dmu of the discrete misfit, by central differences at
    h = 1e-6 of the modulus, for every cell of a 16 x 32 padded grid (fluid,
    formation and PML).  mu is checked on solid cells (mu > 0)."""
    w, g, lam, mu, rho, J, gl, gm, il = _fd_setup()
    scale_l, scale_m = np.abs(gl).max(), np.abs(gm).max()
    bad = []
    for i in range(g.NR):
        for k in range(g.NZ):
            h = 1e-6 * lam[i, k]
            p, q = lam.copy(), lam.copy()
            p[i, k] += h
            q[i, k] -= h
            fd = (J(p, mu) - J(q, mu)) / (2 * h)
            if abs(fd - gl[i, k]) > 1e-6 * scale_l + 1e-5 * abs(fd):
                bad.append(("lam", i, k, fd, gl[i, k]))
            if mu[i, k] > 0:
                h = 1e-6 * mu[i, k]
                p, q = mu.copy(), mu.copy()
                p[i, k] += h
                q[i, k] -= h
                fd = (J(lam, p) - J(lam, q)) / (2 * h)
                if abs(fd - gm[i, k]) > 1e-6 * scale_m + 1e-5 * abs(fd):
                    bad.append(("mu", i, k, fd, gm[i, k]))
    assert not bad, bad[:10]


@pytest.mark.parametrize("region", ["formation", "fluid", "pml"])
def test_gradient_directional_derivative(region):
    """Directional derivative along random perturbations confined to one region;
    this reaches PML cells whose single-cell gradients are too small for
    single-cell differences."""
    w, g, lam, mu, rho, J, gl, gm, il = _fd_setup()
    NR, NZ = g.NR, g.NZ
    ii, kk = np.meshgrid(np.arange(NR), np.arange(NZ), indexing="ij")
    fluid = (mu == 0)
    pml = (ii >= g.nr) | (kk < g.pz) | (kk >= g.pz + g.nz)
    sel = {"formation": ~fluid & ~pml, "fluid": fluid & ~pml, "pml": pml}[region]
    rng = np.random.default_rng(5)
    dl = rng.standard_normal((NR, NZ)) * sel * lam
    dm = rng.standard_normal((NR, NZ)) * (sel & ~fluid) * mu
    eps = 1e-6
    fd = (J(lam + eps * dl, mu + eps * dm) - J(lam - eps * dl, mu - eps * dm)) / (2 * eps)
    an = float((gl * dl).sum() + (gm * dm).sum())
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


def test_checkpoint_segment_length_does_not_change_gradient():
    """The recompute from checkpoints is exact: any segment length gives the
    same FP64 gradient."""
    w, sh, g = _tiny(nt=120)
    lam, mu, rho = oracle_models(w, 0, "start")
    r = np.random.default_rng(6).standard_normal((len(sh.rec_k), g.nt))
    a = oracle.gradient(g, lam, mu, rho, sh.wavelet, r, seg=120)
    b = oracle.gradient(g, lam, mu, rho, sh.wavelet, r, seg=7)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_gradient_vanishes_at_true_model():
    w, sh, g = _tiny(nt=100)
    lt, mt, rho = oracle_models(w, 0, "true")
    dobs = oracle.forward(g, lt, mt, rho, sh.wavelet)
    J, r = oracle.misfit(oracle.forward(g, lt, mt, rho, sh.wavelet), dobs)
    assert J == 0.0
    gl, gm, _ = oracle.gradient(g, lt, mt, rho, sh.wavelet, r, seg=30)
    assert not gl.any() and not gm.any()


def test_velocity_gradient_chain_rule_matches_differences():
    """dJ/dVp, dJ/dVs from the oracle's chain rule of Eq. 3-4 against central
    differences of the misfit in velocity space (directional, formation)."""
    w, sh, g = _tiny(nr=12, nz=24, p=4, nt=150)
    rho = np.ascontiguousarray(w.rho)
    lt, mt, _ = oracle_models(w, 0, "true")
    dobs = oracle.forward(g, lt, mt, rho, sh.wavelet)

    def J(vp, vs):
        lam, mu = oracle.moduli(vp, vs, rho)
        return oracle.misfit(oracle.forward(g, lam, mu, rho, sh.wavelet), dobs)[0]

    vp, vs = w.vp_start.copy(), w.vs_start.copy()
    lam, mu = oracle.moduli(vp, vs, rho)
    _, r = oracle.misfit(oracle.forward(g, lam, mu, rho, sh.wavelet), dobs)
    gl, gm, _ = oracle.gradient(g, lam, mu, rho, sh.wavelet, r, seg=40)
    gvp, gvs = oracle.moduli_grad(vp, vs, rho, gl, gm)
    rng = np.random.default_rng(8)
    form = w.mask.astype(bool)
    dvp = rng.standard_normal(vp.shape) * form * vp
    dvs = rng.standard_normal(vs.shape) * form * vs
    eps = 1e-6
    fd = (J(vp + eps * dvp, vs + eps * dvs) - J(vp - eps * dvp, vs - eps * dvs)) / (2 * eps)
    an = float((gvp * dvp).sum() + (gvs * dvs).sum())
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


def _rho_setup(nr=12, nz=24, p=4, nt=150):
    """Misfit against data from a model whose density differs from the
    starting one, so dJ/drho is far from zero."""
    w, sh, g = _tiny(nr=nr, nz=nz, p=p, nt=nt)
    lam, mu, rho = oracle_models(w, 0, "start")
    lt, mt, rt = oracle_models(w, 0, "true")
    rng = np.random.default_rng(11)
    rt = rt * (1.0 + 0.05 * rng.standard_normal(rt.shape))
    dobs = oracle.forward(g, lt, mt, rt, sh.wavelet)

    def J(r):
        return oracle.misfit(oracle.forward(g, lam, mu, r, sh.wavelet), dobs)[0]

    J0, res = oracle.misfit(oracle.forward(g, lam, mu, rho, sh.wavelet), dobs)
    out = oracle.gradient(g, lam, mu, rho, sh.wavelet, res, seg=37, density=True)
    base = oracle.gradient(g, lam, mu, rho, sh.wavelet, res, seg=37)
    return g, lam, mu, rho, J, out, base


@pytest.mark.slow
def test_density_gradient_matches_central_differences_every_cell():
    """dJ/drho by central differences at h = 1e-6 rho for every cell of the
    padded grid: both buoyancy stencils (radial pair and axial pair), the
    axis row, the clamped top row and the PML are each reached."""
    g, lam, mu, rho, J, (gl, gm, il, gr), _ = _rho_setup()
    scale = np.abs(gr).max()
    assert scale > 0
    bad = []
    for i in range(g.NR):
        for k in range(g.NZ):
            h = 1e-6 * rho[i, k]
            p, q = rho.copy(), rho.copy()
            p[i, k] += h
            q[i, k] -= h
            fd = (J(p) - J(q)) / (2 * h)
            if abs(fd - gr[i, k]) > 1e-6 * scale + 1e-5 * abs(fd):
                bad.append((i, k, fd, gr[i, k]))
    assert not bad, bad[:10]


@pytest.mark.parametrize("region", ["formation", "fluid", "pml"])
def test_density_gradient_directional_derivative(region):
    g, lam, mu, rho, J, (gl, gm, il, gr), _ = _rho_setup()
    NR, NZ = g.NR, g.NZ
    ii, kk = np.meshgrid(np.arange(NR), np.arange(NZ), indexing="ij")
    fluid = (mu == 0)
    pml = (ii >= g.nr) | (kk < g.pz) | (kk >= g.pz + g.nz)
    sel = {"formation": ~fluid & ~pml, "fluid": fluid & ~pml, "pml": pml}[region]
    rng = np.random.default_rng(6)
    d = rng.standard_normal((NR, NZ)) * sel * rho
    eps = 1e-6
    fd = (J(rho + eps * d) - J(rho - eps * d)) / (2 * eps)
    an = float((gr * d).sum())
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


def test_density_output_leaves_modulus_gradients_unchanged():
    """Asking for dJ/drho changes nothing else the gradient routine returns."""
    g, lam, mu, rho, J, (gl, gm, il, gr), (bl, bm, bi) = _rho_setup()
    assert np.array_equal(gl, bl) and np.array_equal(gm, bm) and np.array_equal(il, bi)


def test_density_gradient_vanishes_for_zero_residual():
    """With data generated from the same model the residual is zero and so is
    every gradient, dJ/drho included."""
    w, sh, g = _tiny(nr=10, nz=20, p=3, nt=80)
    lam, mu, rho = oracle_models(w, 0, "start")
    d = oracle.forward(g, lam, mu, rho, sh.wavelet)
    J0, res = oracle.misfit(d, d)
    assert J0 == 0.0
    gl, gm, il, gr = oracle.gradient(g, lam, mu, rho, sh.wavelet, res, seg=20, density=True)
    assert not gr.any()


def test_velocity_density_parameterisation_matches_central_differences():
    """Joint (Vp, Vs, rho): the density enters both through the moduli of
    Eq. 3-4 and through the buoyancies; dJ/drho at fixed velocities is the
    moduli's share plus the buoyancy part.  Directional central differences
    along a perturbation of all three on formation cells."""
    w, sh, g = _tiny(nr=12, nz=24, p=4, nt=150)
    lt, mt, rt = oracle_models(w, 0, "true")
    rt = rt * (1.0 + 0.05 * np.random.default_rng(12).standard_normal(rt.shape))
    dobs = oracle.forward(g, lt, mt, rt, sh.wavelet)

    def J(vp, vs, r):
        lam, mu = oracle.moduli(vp, vs, r)
        return oracle.misfit(oracle.forward(g, lam, mu, r, sh.wavelet), dobs)[0]

    vp, vs, rho = w.vp_start.copy(), w.vs_start.copy(), np.ascontiguousarray(w.rho)
    lam, mu = oracle.moduli(vp, vs, rho)
    _, r = oracle.misfit(oracle.forward(g, lam, mu, rho, sh.wavelet), dobs)
    gl, gm, _, grb = oracle.gradient(g, lam, mu, rho, sh.wavelet, r, seg=40, density=True)
    gvp, gvs, grm = oracle.moduli_grad(vp, vs, rho, gl, gm, density=True)
    grho = grm + grb
    rng = np.random.default_rng(9)
    form = w.mask.astype(bool)
    dvp = rng.standard_normal(vp.shape) * form * vp
    dvs = rng.standard_normal(vs.shape) * form * vs
    drh = rng.standard_normal(rho.shape) * form * rho
    eps = 1e-6
    fd = (J(vp + eps * dvp, vs + eps * dvs, rho + eps * drh)
          - J(vp - eps * dvp, vs - eps * dvs, rho - eps * drh)) / (2 * eps)
    an = float((gvp * dvp).sum() + (gvs * dvs).sum() + (grho * drh).sum())
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
    # the density direction alone, so that its share is not hidden by the others
    fd = (J(vp, vs, rho + eps * drh) - J(vp, vs, rho - eps * drh)) / (2 * eps)
    an = float((grho * drh).sum())
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
