"""Pins of the oracle's assembled-operator step and of its fourth-order
spatial scheme (the order of the finite-difference scheme the Method section
cites is a reading).

The assembled step writes each row of the velocity and stress updates from
the stencil and takes the adjoint as the transpose of those rows.  At order 2
it must give the hand-written step; at order 4 it is pinned by closed-form
point-source fields, convergence, long-run stability, dot products and
central differences of the misfit.

Fourth-order point sources on the axis: with the fields mirrored across the
axis the central four-point stencils conserve the radial flux only in a norm
whose near-axis cell weights differ from the cell volumes; the on-axis cell
weighs sqrt(6/7) of its volume, and the oracle divides the source by that
weight.  The pins check the weight against the summation-by-parts identity
itself (written here from the stencil, not taken from the oracle), and the
oracle's on-axis traces against the closed-form point-source fields with no
fitted amplitude.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from util import geom, oracle_models, rel_l2, ricker_derivative


def _homogeneous(h, vp, vs, rho, f0, courant, Lr, Lz, zs, zr, order, p=20):
    nr, nz = int(round(Lr / h)), int(round(Lz / h))
    dt = courant * h / vp
    v_arr = vp if vs == 0 else vp
    nt = int(math.ceil((1.5 / f0 + (max(zr) - zs) / v_arr + 1.6 / f0) / dt))
    NR, NZ = nr + p, nz + 2 * p
    vpa, vsa, ra = np.full((NR, NZ), vp), np.full((NR, NZ), vs), np.full((NR, NZ), rho)
    lam, mu = oracle.moduli(vpa, vsa, ra)
    rk = np.array([workloads.row_of(z, h, p) for z in zr], np.int32)
    g = oracle.Geom(nr, nz, p, p, h, h, dt, nt, f0, vp, workloads.row_of(zs, h, p), rk)
    d = oracle.forward(g, lam, mu, ra, workloads.ricker(f0, dt, nt), order=order)
    return d, dt, nt


def _fit(d, ref):
    s = float(d @ ref / (ref @ ref))
    return s, rel_l2(d / s, ref)


def _axis_weights(n):
    """Cell weights w_i (i < n) of the norm in which the fourth-order radial
    divergence telescopes: w_i = 1 + A z^i, z = 13 - 2 sqrt(42),
    A = -1 / (7 + sqrt(42))."""
    z = 13.0 - 2.0 * math.sqrt(42.0)
    return 1.0 - z ** np.arange(n) / (7.0 + math.sqrt(42.0))


def test_order4_axis_weight_makes_the_divergence_conservative():
    """With F = r v_r even across the axis, sum_i w_i D_i (D_i the four-point
    difference of F at cell i, image F_{-1} = F_1) must leave only terms at
    the outer end for every F, and the axis cell's weight must be sqrt(6/7).
    Plain cell volumes (w = 1) leave 1/12 F_1 at the axis."""
    c1, c2 = 9.0 / 8.0, -1.0 / 24.0
    n = 40
    rng = np.random.default_rng(5)
    for _ in range(5):
        F = np.zeros(n + 3)
        F[1:n - 4] = rng.standard_normal(n - 5)  # zero near the outer end
        Fm1 = F[1]
        D = np.array([c1 * (F[i + 1] - F[i]) + c2 * (F[i + 2] - (F[i - 1] if i else Fm1))
                      for i in range(n)])
        w = _axis_weights(n)
        assert abs(w @ D) <= 1e-12 * np.abs(D).sum()
        assert abs(np.ones(n) @ D - F[1] / 12.0) <= 1e-12 * np.abs(D).sum()
    assert abs(_axis_weights(1)[0] - math.sqrt(6.0 / 7.0)) <= 1e-15


def test_assembled_order2_is_the_hand_written_step():
    """Traces, final state and gradients of the assembled order-2 operators
    equal the hand-written step to rounding, with fluid, wall and PML: the
    modulus gradients, the illumination, dJ/drho and the pseudo-Hessian."""
    w = workloads.tiny(nr=12, nz=30, p=4, nt=200)
    sh = w.shots[0]
    g = geom(sh)
    lam, mu, rho = oracle_models(w, 0, "start")
    d, st = oracle.forward(g, lam, mu, rho, sh.wavelet, return_state=True)
    da, sta = oracle.forward(g, lam, mu, rho, sh.wavelet, return_state=True, assembled=True)
    assert rel_l2(da, d) <= 1e-13 and rel_l2(sta, st) <= 1e-13
    r = np.random.default_rng(1).standard_normal(d.shape)
    a = oracle.gradient(g, lam, mu, rho, sh.wavelet, r, seg=37, density=True, hessian=True)
    b = oracle.gradient(g, lam, mu, rho, sh.wavelet, r, seg=37, density=True, hessian=True,
                        assembled=True)
    assert len(a) == len(b) == 6
    for x, y in zip(a, b):
        assert rel_l2(y, x) <= 1e-13
    # and the extra outputs leave the others as they were
    c = oracle.gradient(g, lam, mu, rho, sh.wavelet, r, seg=37, assembled=True)
    for x, y in zip(b[:3], c):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("pml,fluid", [(5, True), (0, True), (4, False)])
def test_order4_state_dot_product(pml, fluid):
    w = workloads.tiny(p=pml, fluid=fluid, nr=14, nz=30)
    sh = w.shots[0]
    g = geom(sh)
    lam, mu, rho = oracle_models(w, 0, "start")
    rng = np.random.default_rng(3)
    n = 14 * g.NR * g.NZ
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    Fx = oracle.propagate(g, lam, mu, rho, x, 20, order=4)
    Fty = oracle.propagate(g, lam, mu, rho, y, 20, adjoint=True, order=4)
    a, b = float(Fx @ y), float(x @ Fty)
    assert abs(a - b) <= 1e-12 * max(abs(a), np.linalg.norm(Fx) * np.linalg.norm(y) * 1e-3)


@pytest.mark.slow
def test_order4_point_sources_closed_form():
    """Fluid (mu = 0) and a homogeneous solid: on-axis traces against
    f'(t - R/c)/(4 pi c^2 R) and K f'(t - R/Vp)/(4 pi rho Vp^4 R) with no
    fitted amplitude: the best-fit amplitude of every run is 1 within 0.2 %
    and nearer 1 at the finer spacing; the waveform error (plain and after
    the fit) is <= 0.3 % at 5 mm (10 mm in the solid), at least five times below the second-order scheme's
    at the same spacing, and falls by more than 6 per halving of h in the
    fluid.  Without the axis weight the amplitude would be sqrt(6/7) = 0.926
    at every spacing."""
    scales, errs, plain = [], {}, {}
    c, rho_f, f0 = 1500.0, 1000.0, 10e3
    zs, zr = 0.3, (0.45, 0.6)
    for h in (10e-3, 5e-3):
        d4, dt, nt = _homogeneous(h, c, 0.0, rho_f, f0, 0.15, 0.5, 1.0, zs, zr, 4)
        t = (np.arange(nt) + 1) * dt
        for j, z in enumerate(zr):
            ref = ricker_derivative(f0, t - (z - zs) / c) / (4 * math.pi * c * c * (z - zs))
            s, e = _fit(d4[j], ref)
            scales.append(s)
            errs[("fluid", h, j)] = e
            plain[("fluid", h, j)] = rel_l2(d4[j], ref)
    d2, dt, nt = _homogeneous(5e-3, c, 0.0, rho_f, f0, 0.15, 0.5, 1.0, zs, zr, 2)
    t = (np.arange(nt) + 1) * dt
    for j, z in enumerate(zr):
        ref = ricker_derivative(f0, t - (z - zs) / c) / (4 * math.pi * c * c * (z - zs))
        e2 = rel_l2(d2[j], ref)
        assert errs[("fluid", 5e-3, j)] * 5 < e2, (j, errs, e2)
        assert errs[("fluid", 10e-3, j)] / errs[("fluid", 5e-3, j)] > 6.0, errs
        assert errs[("fluid", 5e-3, j)] <= 3e-3, errs
    vp, vs, rho, f0 = 4000.0, 2300.0, 2300.0, 10e3
    K = rho * vp * vp - 4.0 / 3.0 * rho * vs * vs
    zs, zr = 0.3, (0.6, 0.9)
    d4, dt, nt = _homogeneous(10e-3, vp, vs, rho, f0, 0.3, 0.5, 1.3, zs, zr, 4)
    t = (np.arange(nt) + 1) * dt
    for j, z in enumerate(zr):
        ref = K * ricker_derivative(f0, t - (z - zs) / vp) / (4 * math.pi * rho * vp ** 4 * (z - zs))
        s, e = _fit(d4[j], ref)
        scales.append(s)
        plain[("solid", j)] = rel_l2(d4[j], ref)
        assert e <= 3e-3, (j, e)
    assert all(abs(s - 1.0) <= 0.002 for s in scales), scales
    # fluid, two receivers at 10 mm then at 5 mm: the amplitude error shrinks
    assert abs(scales[2] - 1.0) < abs(scales[0] - 1.0), scales
    assert abs(scales[3] - 1.0) < abs(scales[1] - 1.0), scales
    # unfitted traces at 5 mm (fluid) and 10 mm (solid, larger wavelength)
    assert max(v for k_, v in plain.items() if k_[1] != 10e-3) <= 3e-3, plain
    assert plain[("fluid", 10e-3, 0)] / plain[("fluid", 5e-3, 0)] > 6.0, plain


def test_order4_long_run_bounded_without_pml():
    """Rigid box, no PML, Courant 0.5 (the fourth-order limit is 6/7 of the
    second-order one): 1e5 source-free steps after a Ricker excitation stay
    of the order of the initial amplitude."""
    w = workloads.tiny(p=0, nr=20, nz=40)
    sh = w.shots[0]
    vmax = w.vp_true.max()
    dt = 0.5 * sh.dr / vmax
    g = oracle.Geom(sh.nr, sh.nz, 0, 0, sh.dr, sh.dz, dt, 200, sh.f0, vmax, sh.src_k, sh.rec_k)
    lam, mu, rho = oracle_models(w, 0, "true")
    _, st = oracle.forward(g, lam, mu, rho, workloads.ricker(sh.f0, dt, 200), return_state=True,
                           order=4)
    a0 = np.abs(st[:6]).max()
    st = oracle.propagate(g, lam, mu, rho, st.ravel(), 100000, order=4)
    assert np.isfinite(st).all()
    assert np.abs(st.reshape(14, g.NR, g.NZ)[:6]).max() < 3.0 * a0


@pytest.mark.parametrize("region", ["formation", "fluid", "pml"])
def test_order4_gradient_directional_derivative(region):
    """dJ/dlambda, dJ/dmu of the fourth-order misfit against central
    differences along random perturbations confined to one region."""
    w = workloads.tiny(nr=12, nz=24, p=4, nt=150)
    sh = w.shots[0]
    g = geom(sh)
    lam, mu, rho = oracle_models(w, 0, "start")
    lt, mt, _ = oracle_models(w, 0, "true")
    dobs = oracle.forward(g, lt, mt, rho, sh.wavelet, order=4)

    def J(l, m):
        return oracle.misfit(oracle.forward(g, l, m, rho, sh.wavelet, order=4), dobs)[0]

    _, res = oracle.misfit(oracle.forward(g, lam, mu, rho, sh.wavelet, order=4), dobs)
    gl, gm, il = oracle.gradient(g, lam, mu, rho, sh.wavelet, res, seg=37, order=4)
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


def test_order4_gradient_checkpoint_interval_and_single_cells():
    """The checkpoint interval does not change the gradient; a few single
    cells (axis row, wall, PML corner) match central differences."""
    w = workloads.tiny(nr=10, nz=22, p=3, nt=120)
    sh = w.shots[0]
    g = geom(sh)
    lam, mu, rho = oracle_models(w, 0, "start")
    lt, mt, _ = oracle_models(w, 0, "true")
    dobs = oracle.forward(g, lt, mt, rho, sh.wavelet, order=4)
    _, res = oracle.misfit(oracle.forward(g, lam, mu, rho, sh.wavelet, order=4), dobs)
    a = oracle.gradient(g, lam, mu, rho, sh.wavelet, res, seg=120, order=4)
    b = oracle.gradient(g, lam, mu, rho, sh.wavelet, res, seg=17, order=4)
    for x, y in zip(a, b):
        assert rel_l2(y, x) <= 1e-13

    def J(l):
        return oracle.misfit(oracle.forward(g, l, mu, rho, sh.wavelet, order=4), dobs)[0]

    scale = np.abs(a[0]).max()
    for (i, k) in [(0, g.pz + 5), (4, g.pz + 9), (5, g.pz + 2), (g.NR - 1, g.NZ - 1)]:
        h = 1e-6 * lam[i, k]
        p, q = lam.copy(), lam.copy()
        p[i, k] += h
        q[i, k] -= h
        fd = (J(p) - J(q)) / (2 * h)
        assert abs(fd - a[0][i, k]) <= 1e-6 * scale + 1e-5 * abs(fd), ((i, k), fd, a[0][i, k])


def _rho_setup4(nr=12, nz=24, p=4, nt=150):
    """Order-4 misfit against data from a model whose density differs from
    the starting one."""
    w = workloads.tiny(nr=nr, nz=nz, p=p, nt=nt)
    sh = w.shots[0]
    g = geom(sh)
    lam, mu, rho = oracle_models(w, 0, "start")
    lt, mt, rt = oracle_models(w, 0, "true")
    rt = rt * (1.0 + 0.05 * np.random.default_rng(11).standard_normal(rt.shape))
    dobs = oracle.forward(g, lt, mt, rt, sh.wavelet, order=4)

    def J(r):
        return oracle.misfit(oracle.forward(g, lam, mu, r, sh.wavelet, order=4), dobs)[0]

    _, res = oracle.misfit(oracle.forward(g, lam, mu, rho, sh.wavelet, order=4), dobs)
    out = oracle.gradient(g, lam, mu, rho, sh.wavelet, res, seg=37, density=True, order=4)
    return g, rho, mu, J, out


@pytest.mark.parametrize("region", ["formation", "fluid", "pml"])
def test_order4_density_gradient_directional_derivative(region):
    """dJ/drho of the fourth-order misfit against central differences along
    random density perturbations confined to one region."""
    g, rho, mu, J, (gl, gm, il, gr) = _rho_setup4()
    NR, NZ = g.NR, g.NZ
    ii, kk = np.meshgrid(np.arange(NR), np.arange(NZ), indexing="ij")
    fluid = (mu == 0)
    pml = (ii >= g.nr) | (kk < g.pz) | (kk >= g.pz + g.nz)
    sel = {"formation": ~fluid & ~pml, "fluid": fluid & ~pml, "pml": pml}[region]
    d = np.random.default_rng(6).standard_normal((NR, NZ)) * sel * rho
    # the PML share of dJ/drho is small against J: a step of 1e-6 leaves the
    # difference of the misfits at the level of their rounding (3e-6 relative
    # there), so take a step of 1e-4 and the fourth-order central difference
    # (the O(eps^2) term of the two-point one is 1e-6 in the fluid)
    eps = 1e-4
    fd = (8.0 * (J(rho + eps * d) - J(rho - eps * d)) -
          (J(rho + 2 * eps * d) - J(rho - 2 * eps * d))) / (12 * eps)
    an = float((gr * d).sum())
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


def test_order4_density_gradient_single_cells():
    """A few single cells: the axis row, next to the wall, the clamped top
    row and a PML corner."""
    g, rho, mu, J, (gl, gm, il, gr) = _rho_setup4(nr=10, nz=22, p=3, nt=120)
    scale = np.abs(gr).max()
    for (i, k) in [(0, g.pz + 5), (4, g.pz + 9), (5, g.pz + 2), (2, g.NZ - 1),
                   (g.NR - 1, 0)]:
        h = 1e-6 * rho[i, k]
        p, q = rho.copy(), rho.copy()
        p[i, k] += h
        q[i, k] -= h
        fd = (J(p) - J(q)) / (2 * h)
        assert abs(fd - gr[i, k]) <= 1e-6 * scale + 1e-5 * abs(fd), ((i, k), fd, gr[i, k])


@pytest.mark.slow
def test_order4_pseudo_hessian_is_the_squared_stress_update_derivative():
    """As at order 2: for interior cells H_lambda(c) is the sum over steps of
    the squared change of the three normal stresses at c per unit lambda(c),
    and H_mu(c) that per unit mu(c) plus the squared change of tau_rz at the
    node (i, k) per unit change of its harmonic-mean rigidity, measured by
    differencing one fourth-order step of the source-driven state."""
    w = workloads.tiny(nr=12, nz=26, p=3, nt=30, fluid=False)
    sh = w.shots[0]
    g = geom(sh)
    shp = (g.NR, g.NZ)
    lam, mu, rho = np.full(shp, 9.0e9), np.full(shp, 6.0e9), np.full(shp, 2400.0)
    nt = g.nt
    r = np.zeros((len(sh.rec_k), nt))
    _, _, _, hl, hm = oracle.gradient(g, lam, mu, rho, sh.wavelet, r, seg=nt, hessian=True,
                                      order=4)
    H = 1e8  # the stress update is linear in the moduli
    states = [np.zeros((14, g.NR, g.NZ))]
    for n in range(1, nt):
        gn = oracle.Geom(g.nr, g.nz, g.pr, g.pz, g.dr, g.dz, g.dt, n, g.f0, g.vmax, g.src_k,
                         g.rec_k)
        states.append(oracle.forward(gn, lam, mu, rho, sh.wavelet, return_state=True,
                                     order=4)[1])
    TRR, TTT, TZZ, TRZ = 2, 3, 4, 5
    for (i, k) in [(0, g.pz + 5), (1, g.pz + 9), (5, g.pz + 12), (g.nr - 3, g.pz + g.nz - 4)]:
        el = np.zeros(shp)
        el[i, k] = H
        em = np.zeros(shp)
        em[i, k] = H
        es = np.zeros(shp)
        if i >= 1:
            es[i - 1:i + 1, k:k + 2] = H
        hl_fd = hm_fd = 0.0
        for n in range(nt):
            x = states[n].ravel()
            base = oracle.propagate(g, lam, mu, rho, x, 1, order=4).reshape(-1, g.NR, g.NZ)
            pl = oracle.propagate(g, lam + el, mu, rho, x, 1, order=4).reshape(-1, g.NR, g.NZ)
            pm = oracle.propagate(g, lam, mu + em, rho, x, 1, order=4).reshape(-1, g.NR, g.NZ)
            d = (pl - base) / H
            hl_fd += sum(d[f, i, k] ** 2 for f in (TRR, TTT, TZZ))
            d = (pm - base) / H
            hm_fd += sum(d[f, i, k] ** 2 for f in (TRR, TTT, TZZ))
            if i >= 1:
                ps = oracle.propagate(g, lam, mu + es, rho, x, 1, order=4).reshape(-1, g.NR,
                                                                                   g.NZ)
                hm_fd += ((ps - base)[TRZ, i, k] / H) ** 2
        assert hl[i, k] > 0 and hm[i, k] > 0
        assert abs(hl[i, k] - hl_fd) <= 1e-6 * hl_fd, ((i, k), hl[i, k], hl_fd)
        assert abs(hm[i, k] - hm_fd) <= 1e-6 * hm_fd, ((i, k), hm[i, k], hm_fd)
