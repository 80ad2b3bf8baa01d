"""Pins of the oracle's extensions beyond the paper's fixed density and
illumination preconditioner: the virtual-source pseudo-Hessian diagonal, the
general diagonal preconditioner with a radial taper, and the density step.

The pseudo-Hessian is pinned by brute force on the oracle's own time step:
its terms are, step by step, the squared change of the stress update under a
unit change of a modulus, which the test measures by differencing one step of
the state with and without that change.
"""
import numpy as np
import pytest

import oracle
import workloads
from util import geom

H = 1e8  # Pa: the stress update is linear in the moduli, so a large step is exact


def _uniform_solid(nr=10, nz=22, p=3, nt=40):
    w = workloads.tiny(nr=nr, nz=nz, p=p, nt=nt, fluid=False)
    sh = w.shots[0]
    g = geom(sh)
    shp = (g.NR, g.NZ)
    lam = np.full(shp, 9.0e9)
    mu = np.full(shp, 6.0e9)
    rho = np.full(shp, 2400.0)
    return sh, g, lam, mu, rho


def _states(g, lam, mu, rho, wavelet, nt):
    """The full state after n = 0 .. nt-1 source-driven steps."""
    out = [np.zeros((14, g.NR, g.NZ))]
    for n in range(1, nt):
        gn = geom_with_nt(g, n)
        out.append(oracle.forward(gn, lam, mu, rho, wavelet, return_state=True)[1])
    return out


def geom_with_nt(g, nt):
    return oracle.Geom(g.nr, g.nz, g.pr, g.pz, g.dr, g.dz, g.dt, nt, g.f0, g.vmax, g.src_k,
                       g.rec_k)


@pytest.mark.slow
def test_pseudo_hessian_is_the_squared_stress_update_derivative():
    """For interior cells (clear of the PML), H_lambda(c) is the sum over steps
    of the squared change of (tau_rr, tau_tt, tau_zz)(c) per unit lambda(c),
    and H_mu(c) that per unit mu(c) plus the squared change of tau_rz at the
    node (i, k) per unit change of its harmonic-mean rigidity (in a uniform
    solid, raising the four cells around the node by h raises it by h)."""
    sh, g, lam, mu, rho = _uniform_solid()
    nt = g.nt
    r = np.zeros((len(sh.rec_k), nt))
    _, _, _, hl, hm = oracle.gradient(g, lam, mu, rho, sh.wavelet, r, seg=nt, hessian=True)
    states = _states(g, lam, mu, rho, sh.wavelet, nt)
    cells = [(0, g.pz + 3), (1, g.pz + 7), (4, g.pz + 10), (g.nr - 2, g.pz + g.nz - 2)]
    TRR, TTT, TZZ, TRZ = 2, 3, 4, 5
    for (i, k) in cells:
        el = np.zeros_like(lam)
        el[i, k] = H
        em = np.zeros_like(mu)
        em[i, k] = H
        es = np.zeros_like(mu)
        if i >= 1:
            es[i - 1:i + 1, k:k + 2] = H
        hl_fd = hm_fd = 0.0
        for n in range(nt):
            x = states[n].ravel()
            base = oracle.propagate(g, lam, mu, rho, x, 1).reshape(-1, g.NR, g.NZ)
            pl = oracle.propagate(g, lam + el, mu, rho, x, 1).reshape(-1, g.NR, g.NZ)
            pm = oracle.propagate(g, lam, mu + em, rho, x, 1).reshape(-1, g.NR, g.NZ)
            d = (pl - base) / H
            hl_fd += sum(d[f, i, k] ** 2 for f in (TRR, TTT, TZZ))
            d = (pm - base) / H
            hm_fd += sum(d[f, i, k] ** 2 for f in (TRR, TTT, TZZ))
            if i >= 1:
                ps = oracle.propagate(g, lam, mu + es, rho, x, 1).reshape(-1, g.NR, g.NZ)
                hm_fd += ((ps - base)[TRZ, i, k] / H) ** 2
        assert hl[i, k] > 0 and hm[i, k] > 0
        assert abs(hl[i, k] - hl_fd) <= 1e-6 * hl_fd, ((i, k), hl[i, k], hl_fd)
        assert abs(hm[i, k] - hm_fd) <= 1e-6 * hm_fd, ((i, k), hm[i, k], hm_fd)


def test_pseudo_hessian_leaves_the_gradient_unchanged_and_vanishes_without_source():
    w = workloads.tiny(nr=10, nz=20, p=3, nt=60)
    sh = w.shots[0]
    g = geom(sh)
    from util import oracle_models
    lam, mu, rho = oracle_models(w, 0, "start")
    r = np.random.default_rng(2).standard_normal((len(sh.rec_k), g.nt))
    a = oracle.gradient(g, lam, mu, rho, sh.wavelet, r, seg=25)
    b = oracle.gradient(g, lam, mu, rho, sh.wavelet, r, seg=25, hessian=True)
    for x, y in zip(a, b[:3]):
        assert np.array_equal(x, y)
    assert (b[3] >= 0).all() and (b[4] >= 0).all()
    z = oracle.gradient(g, lam, mu, rho, np.zeros(g.nt), r, seg=25, hessian=True)
    assert not z[3].any() and not z[4].any()


def test_precondition_diag_by_hand():
    """P = w[i] / (d + eps max d) on mask cells, 0 elsewhere; the max runs
    over mask cells only; sum g P g before the scaling."""
    g = np.array([[8.0, 2.0, 1.0], [5.0, -4.0, 3.0]])
    d = np.array([[4.0, 1.0, 0.0], [100.0, 3.0, 1e6]])
    mask = np.array([[1, 1, 1], [1, 1, 0]], np.uint8)
    w = np.array([0.5, 2.0])
    out, gpg = oracle.precondition_diag(g, mask, 0.25, diag=d, row_weight=w, return_gpg=True)
    # max over mask of d is 100: eps max d = 25
    want = np.array([[0.5 * 8 / 29, 0.5 * 2 / 26, 0.5 * 1 / 25],
                     [2 * 5 / 125, 2 * -4 / 28, 0.0]])
    assert np.allclose(out, want, rtol=1e-15, atol=0)
    assert gpg == pytest.approx(0.5 * 64 / 29 + 0.5 * 4 / 26 + 0.5 / 25 + 2 * 25 / 125
                                + 2 * 16 / 28, rel=1e-15)
    # without a diagonal the weights alone; without either, the mask alone
    assert np.allclose(oracle.precondition_diag(g, mask, 0.25, row_weight=w),
                       np.where(mask, g * w[:, None], 0.0))
    assert np.array_equal(oracle.precondition_diag(g, mask, 0.25), np.where(mask, g, 0.0))


def test_precondition_diag_with_the_illumination_is_the_paper_preconditioner():
    rng = np.random.default_rng(4)
    il = rng.uniform(0, 5, (6, 9))
    gl, gm = rng.standard_normal((6, 9)), rng.standard_normal((6, 9))
    mask = (rng.uniform(size=(6, 9)) > 0.3).astype(np.uint8)
    a, b, gpg = oracle.precondition(il, mask, 1e-3, gl, gm, return_gpg=True)
    x, p = oracle.precondition_diag(gl, mask, 1e-3, diag=il, return_gpg=True)
    y, q = oracle.precondition_diag(gm, mask, 1e-3, diag=il, return_gpg=True)
    assert np.allclose(a, x, rtol=1e-14, atol=0) and np.allclose(b, y, rtol=1e-14, atol=0)
    assert p + q == pytest.approx(gpg, rel=1e-13)


def test_radial_taper_closed_form():
    dr = 0.01
    w = oracle.radial_taper(40, dr, 0.1, 0.2)
    r = (np.arange(40) + 0.5) * dr
    assert (w[r <= 0.1] == 0).all() and (w[r >= 0.2] == 1).all()
    # the middle of the ramp, r = 0.15, is row 14.5: rows 14 and 15 straddle 1/2
    assert w[14] < 0.5 < w[15]
    assert w[14] + w[15] == pytest.approx(1.0, abs=1e-12)  # sin^2 + cos^2 by symmetry
    assert np.all(np.diff(w) >= 0)
    step = oracle.radial_taper(10, dr, 0.05, 0.05)
    assert list(step) == [0.0] * 5 + [1.0] * 5


def test_update_density_by_hand():
    rho = np.array([[2000.0, 2500.0], [1000.0, 3000.0]])
    g = np.array([[10.0, -20.0], [5.0, 40.0]])
    mask = np.array([[1, 1], [1, 0]], np.uint8)
    r, a = oracle.update_density(rho, g, mask, 0.02, 1500.0, 2600.0)
    # alpha = 0.02 * 2500 / 20 over mask cells
    assert a == pytest.approx(2.5, rel=1e-15)
    assert np.array_equal(r, np.array([[1975.0, 2550.0], [1500.0, 3000.0]]))
