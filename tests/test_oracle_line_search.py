"""Pins of the oracle's line search (reading of the step rule of Eq. 9-10)
and of the slope it uses.

* On an exact quadratic J(a) = J0 - g a + c a^2 the parabola through J0, the
  slope -g and J(alpha1) is the quadratic itself: the step is g / (2c)
  whenever that lies in [alpha1/10, 3 alpha1], and the clamp otherwise.
* Without curvature (c <= 0) the trial step is kept when it lowered the
  misfit and halved when it did not.
* The slope -sum(g . P g) returned by the preconditioner is the derivative of
  the oracle's own misfit along the preconditioned step, checked by central
  differences of forward runs on a small borehole model.
"""
import numpy as np
import pytest

import oracle
import workloads
from util import geom, oracle_models


@pytest.mark.parametrize("seed", range(6))
def test_exact_quadratic_gives_its_minimiser(seed):
    rng = np.random.default_rng(seed)
    J0, g, c = rng.uniform(1, 10), rng.uniform(0.1, 5), rng.uniform(0.1, 5)
    amin = g / (2 * c)
    a1 = amin * rng.uniform(0.4, 5.0)  # minimiser inside [a1/10, 3 a1]
    J1 = J0 - g * a1 + c * a1 * a1
    a = oracle.line_search(J0, J1, g, a1)
    want = min(max(amin, 0.1 * a1), 3 * a1)
    assert a == pytest.approx(want, rel=1e-12)


def test_clamps():
    J0, g, c = 5.0, 2.0, 1.0  # minimiser at 1
    a1 = 0.2                  # minimiser 5 trial steps away -> 3 a1
    assert oracle.line_search(J0, J0 - g * a1 + c * a1 * a1, g, a1) == pytest.approx(0.6)
    a1 = 20.0                 # minimiser at a1/20 -> a1/10
    assert oracle.line_search(J0, J0 - g * a1 + c * a1 * a1, g, a1) == pytest.approx(2.0)


def test_no_curvature_branches():
    # linear or concave along the step: keep the trial step if it helped
    assert oracle.line_search(1.0, 0.5, 1.0, 0.5) == 0.5      # J1 = J0 - g a1 exactly (c = 0)
    assert oracle.line_search(1.0, 0.2, 1.0, 0.5) == 0.5      # concave, lower
    # a wrong-signed slope with a higher trial misfit: halve
    assert oracle.line_search(1.0, 1.5, -1.0, 0.5) == 0.25
    assert oracle.line_search(1.0, 0.9, 1.0, 0.0) == 0.0


def test_slope_is_the_directional_derivative_of_the_misfit():
    w = workloads.tiny(seed=3)
    sh = w.shots[0]
    g = geom(sh)
    lam, mu, rho = oracle_models(w, 0, "start")
    lt, mt, _ = oracle_models(w, 0, "true")
    dobs = oracle.forward(g, lt, mt, rho, sh.wavelet)
    J0, r = oracle.misfit(oracle.forward(g, lam, mu, rho, sh.wavelet), dobs)
    gl, gm, il = oracle.gradient(g, lam, mu, rho, sh.wavelet, r, seg=60)
    pl, pm, gpg = oracle.precondition(il, w.mask, 1e-3, gl, gm, return_gpg=True)
    assert gpg > 0
    # the same sum written out
    assert gpg == pytest.approx(float(np.sum(gl * pl + gm * pm)), rel=1e-12)

    def J(a):
        d = oracle.forward(g, lam - a * pl, mu - a * pm, rho, sh.wavelet)
        return oracle.misfit(d, dobs)[0]

    h = 1e-4 * max(np.abs(lam).max() / np.abs(pl).max(), np.abs(mu).max() / np.abs(pm).max())
    fd = (J(h) - J(-h)) / (2 * h)
    assert fd == pytest.approx(-gpg, rel=1e-5)
    # one line-search step from the greatest-change trial lowers the misfit
    l1, m1, a1 = oracle.update(lam, mu, rho, pl, pm, w.mask, 0.02)
    J1 = oracle.misfit(oracle.forward(g, l1, m1, rho, sh.wavelet), dobs)[0]
    a = oracle.line_search(J0, J1, gpg, a1)
    l2, m2, _ = oracle.update(lam, mu, rho, pl, pm, w.mask, 0.02, alpha_override=a)
    J2 = oracle.misfit(oracle.forward(g, l2, m2, rho, sh.wavelet), dobs)[0]
    assert J2 < J0
