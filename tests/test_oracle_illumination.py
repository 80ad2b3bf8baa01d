"""Pin of the oracle's illumination (the preconditioner's diagonal, the
Numerical Examples section's Fig. 6 discussion) against a closed form.

In a fluid full space (mu = 0, no borehole) an on-axis point source gives the
normal stress tau(R, t) = s'(t - R/c) / (4 pi c^2 R), the form the forward
pin of test_oracle_closed_forms checks.  Momentum balance rho dv/dt = grad tau
integrated in time gives the radial particle velocity

    v_R(R, t) = -[ s'(t - R/c) / (c R) + s(t - R/c) / R^2 ] / (4 pi rho c^2),

so the illumination of a cell, sum_n dt |v(t_{n+1/2})|^2 with v averaged to
the cell centre, approximates the integral of v_R^2 over the record at the
cell centre's distance R from the source.  The integral is taken here by
adaptive quadrature of the closed form, independently of the oracle.

Plausible mistakes and the check that catches each:
  * a missing or doubled dt, a wrong component or a missing square: the
    full-record values (within 0.6 % at 2.5 mm);
  * velocities not averaged to the cell centre (a half-cell offset in r or
    z): first-order error, caught by the convergence ratio per halving of h;
  * the velocity of the wrong half step (v^{n-1/2}): invisible on a full
    record (the sum is shift-invariant), caught on a record that ends at the
    arrival's peak, where one step of misalignment costs 1.3e-3 at 2.5 mm
    against the 1e-4 the scheme reaches.
The same closed form pins the fourth-order variant's illumination.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

import oracle
import workloads

pytestmark = pytest.mark.filterwarnings("ignore")

C, RHO, F0, ZS = 1500.0, 1000.0, 10e3, 0.3
# cells (r, z - zs) in metres around the source
CELLS = [(0.1, 0.1), (0.05, 0.2), (0.2, 0.0), (0.15, -0.1)]


def _s(t):
    a = (math.pi * F0 * (t - 1.5 / F0)) ** 2
    return (1 - 2 * a) * math.exp(-a)


def _ds(t):
    tt = t - 1.5 / F0
    a = (math.pi * F0 * tt) ** 2
    return 2 * math.pi ** 2 * F0 ** 2 * tt * (2 * a - 3) * math.exp(-a)


def _v_radial(R, t):
    return -(_ds(t - R / C) / (C * R) + _s(t - R / C) / R ** 2) / (4 * math.pi * RHO * C * C)


def _energy(R, T):
    """Integral over [0, T] of v_R(R, t)^2 (quadrature of the closed form)."""
    return quad(lambda t: _v_radial(R, t) ** 2, 0.0, T, limit=400, epsabs=0, epsrel=1e-12)[0]


def _illumination(h, nt=None, courant=0.3, Lr=0.4, Lz=0.8, p=20, order=2):
    """Oracle illumination of a homogeneous fluid with an on-axis source at
    z = ZS (zero residual: the gradient pass runs only for its forward
    illumination), with the second- or fourth-order stencil."""
    nr, nz = int(round(Lr / h)), int(round(Lz / h))
    dt = courant * h / C
    if nt is None:  # the pulse has passed every test cell
        nt = int(math.ceil((1.5 / F0 + 0.35 / C + 2.5 / F0) / dt))
    NR, NZ = nr + p, nz + 2 * p
    lam, mu = oracle.moduli(np.full((NR, NZ), C), np.zeros((NR, NZ)), np.full((NR, NZ), RHO))
    ks = workloads.row_of(ZS, h, p)
    g = oracle.Geom(nr, nz, p, p, h, h, dt, nt, F0, C, ks, np.array([ks + 5], np.int32))
    _, _, illum = oracle.gradient(g, lam, mu, np.full((NR, NZ), RHO),
                                  workloads.ricker(F0, dt, nt), np.zeros((1, nt)), seg=nt,
                                  order=order)
    return illum, dt, nt, ks


def _cell(h, ks, r, dz):
    i, k = int(round(r / h - 0.5)), ks + int(round(dz / h))
    return i, k, math.hypot((i + 0.5) * h, (k - ks) * h)


def test_illumination_full_record_closed_form_second_order():
    errs = {}
    for h in (5e-3, 2.5e-3):
        illum, dt, nt, ks = _illumination(h)
        errs[h] = []
        for r, dz in CELLS:
            i, k, R = _cell(h, ks, r, dz)
            errs[h].append(illum[i, k] / _energy(R, nt * dt) - 1.0)
    assert max(abs(e) for e in errs[2.5e-3]) < 6e-3, errs
    for j in range(len(CELLS)):
        ratio = abs(errs[5e-3][j] / errs[2.5e-3][j])
        assert 3.3 < ratio < 5.0, (j, errs, ratio)


def test_illumination_time_alignment_on_a_record_ending_at_the_arrival():
    r, dz = CELLS[0]
    for h, tol in ((5e-3, 3e-3), (2.5e-3, 5e-4)):
        dt = 0.3 * h / C
        nt = int(round((1.5 / F0 + math.hypot(r, dz) / C) / dt))
        illum, dt, nt, ks = _illumination(h, nt=nt)
        i, k, R = _cell(h, ks, r, dz)
        err = illum[i, k] / _energy(R, nt * dt) - 1.0
        assert abs(err) < tol, (h, err)


def test_illumination_fourth_order_closed_form():
    # The fourth-order wavefield with the same two-point means to the cell
    # centre: the means keep the illumination second order in h (error ratio
    # near 4 per halving), within 0.8 % of the closed form at 2.5 mm.
    errs = {}
    for h in (5e-3, 2.5e-3):
        illum, dt, nt, ks = _illumination(h, order=4)
        errs[h] = []
        for r, dz in CELLS:
            i, k, R = _cell(h, ks, r, dz)
            errs[h].append(illum[i, k] / _energy(R, nt * dt) - 1.0)
    assert max(abs(e) for e in errs[2.5e-3]) < 8e-3, errs
    for j in range(len(CELLS)):
        ratio = abs(errs[5e-3][j] / errs[2.5e-3][j])
        assert 3.3 < ratio < 5.0, (j, errs, ratio)
