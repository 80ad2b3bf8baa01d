"""Pins of the FP64 oracle's forward scheme (Eq. 2) against closed forms.

Each test would fail for a plausible mistake in the scheme: a wrong source
scale or sign, a wrong 1/r term, a wrong modulus combination, a wrong axis
treatment or fluid-solid wall condition, or first-order accuracy.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from util import golden, rel_l2, ricker_derivative

pytestmark = pytest.mark.filterwarnings("ignore")


def _homogeneous_run(h, vp, vs, rho, f0, courant, Lr, Lz, zs, zr, p=20, borehole=False,
                     t_tail=1.6):
    nr, nz = int(round(Lr / h)), int(round(Lz / h))
    dt = courant * h / vp
    vslow = min(v for v in (vp, vs, 1378.0 if borehole else vp) if v > 0)
    nt = int(math.ceil((1.5 / f0 + (max(zr) - zs) / vslow + t_tail / f0) / dt))
    NR, NZ = nr + p, nz + 2 * p
    vpa, vsa, ra = np.full((NR, NZ), vp), np.full((NR, NZ), vs), np.full((NR, NZ), rho)
    if borehole:
        workloads._fill_borehole(vpa, vsa, ra, h)
    lam, mu = oracle.moduli(vpa, vsa, ra)
    rk = np.array([workloads.row_of(z, h, p) for z in zr], np.int32)
    g = oracle.Geom(nr, nz, p, p, h, h, dt, nt, f0, vp, workloads.row_of(zs, h, p), rk)
    d = oracle.forward(g, lam, mu, ra, workloads.ricker(f0, dt, nt))
    return d, dt, nt


def test_fluid_point_source_green_function_second_order():
    """mu = 0 everywhere: on-axis traces equal f'(t - R/c)/(4 pi c^2 R); the
    error falls by ~4 per halving of h at a fixed Courant number."""
    c, rho, f0 = 1500.0, 1000.0, 10e3
    zs, zr = 0.3, (0.45, 0.6)
    errs = {}
    for h in (10e-3, 5e-3):
        d, dt, nt = _homogeneous_run(h, c, 0.0, rho, f0, 0.15, 0.5, 1.0, zs, zr)
        t = (np.arange(nt) + 1) * dt  # receivers sample tau^{n+1}
        errs[h] = [rel_l2(d[j], ricker_derivative(f0, t - (z - zs) / c) /
                          (4 * math.pi * c * c * (z - zs))) for j, z in enumerate(zr)]
    for j in range(len(zr)):
        ratio = errs[10e-3][j] / errs[5e-3][j]
        assert 3.5 < ratio < 4.7, (j, errs, ratio)
    assert errs[5e-3][0] < 0.045 and errs[5e-3][1] < 0.085, errs


def test_solid_explosion_mean_stress_closed_form():
    """Homogeneous solid 4000/2300/2300, no borehole: mean normal stress equals
    K f'(t - R/Vp)/(4 pi rho Vp^4 R); second order in h."""
    vp, vs, rho, f0 = 4000.0, 2300.0, 2300.0, 10e3
    K = rho * vp * vp - 4.0 / 3.0 * rho * vs * vs
    zs, zr = 0.3, (0.6, 0.9)
    errs = {}
    for h in (10e-3, 5e-3):
        d, dt, nt = _homogeneous_run(h, vp, vs, rho, f0, 0.3, 0.5, 1.3, zs, zr)
        t = (np.arange(nt) + 1) * dt
        errs[h] = [rel_l2(d[j], K * ricker_derivative(f0, t - (z - zs) / vp) /
                          (4 * math.pi * rho * vp ** 4 * (z - zs))) for j, z in enumerate(zr)]
    for j in range(len(zr)):
        ratio = errs[10e-3][j] / errs[5e-3][j]
        assert 3.0 < ratio < 4.7, (j, errs, ratio)
    assert max(errs[5e-3]) < 0.01, errs


def test_tube_wave_low_frequency_speed():
    """Fluid-filled hole (a = 0.1 m, water) in 4000/2300/2300: the phase speed
    between two on-axis receivers at 300-600 Hz equals White's low-frequency
    tube-wave speed (1/Vf^2 + rho_f/mu)^(-1/2) = 1378.0 m/s."""
    gd = golden("closed_forms.json")["tube_wave_low_frequency"]
    vt = (1 / gd["vf"] ** 2 + gd["rho_f"] / (gd["rho"] * gd["vs"] ** 2)) ** -0.5
    assert abs(vt - gd["v_t"]) / gd["v_t"] < gd["rel_tol_vs_formula"]
    zr = (2.5, 4.5)
    d, dt, nt = _homogeneous_run(0.01, 4000.0, 2300.0, 2300.0, 1e3, 0.5, 1.2, 5.0, 0.5, zr,
                                 borehole=True, t_tail=2.0)
    n = 1 << int(math.ceil(math.log2(nt * 4)))
    F1, F2 = np.fft.rfft(d[0], n), np.fft.rfft(d[1], n)
    f = np.fft.rfftfreq(n, dt)
    ph = np.unwrap(np.angle(F2 * np.conj(F1)))
    for fq in (300.0, 400.0, 500.0, 600.0):
        i = int(np.argmin(abs(f - fq)))
        V = -2 * math.pi * f[i] * (zr[1] - zr[0]) / ph[i]
        assert abs(V - vt) / vt < 0.005, (fq, V, vt)


@pytest.mark.slow
def test_p_head_wave_moveout_single_shot_geometry():
    """The 128 x 512 single-shot workload, start model: the first arrival is
    the refracted P wave; it arrives at t0 + z/Vp + 2a sqrt(1/Vf^2 - 1/Vp^2)
    and its moveout across the array is 1/Vp."""
    gd = golden("closed_forms.json")["p_head_wave"]
    w = workloads.make("c1")
    sh = w.shots[0]
    from util import geom, oracle_models
    lam, mu, rho = oracle_models(w, 0, "start")
    d = oracle.forward(geom(sh), lam, mu, rho, sh.wavelet)
    t = (np.arange(sh.nt) + 1) * sh.dt
    zsrc = (sh.src_k - sh.pz) * sh.dz
    intercept = 2 * gd["a"] * math.sqrt(1 / gd["vf"] ** 2 - 1 / gd["vp"] ** 2)
    assert abs(intercept * 1e3 - gd["intercept_ms"]) < 1e-4

    def window(j, half=0.1e-3):
        z = (sh.rec_k[j] - sh.pz) * sh.dz - zsrc
        tp = 1.5 / sh.f0 + z / gd["vp"] + intercept
        return np.where((t > tp - half) & (t < tp + half), d[j], 0.0), z, tp

    for j in range(len(sh.rec_k)):
        x, z, tp = window(j)
        onset = t[np.argmax(np.abs(d[j]) > 0.01 * np.abs(d[j]).max())]
        assert abs(onset - tp) < 0.15 / sh.f0, (j, onset, tp)
    x, z1, _ = window(3)
    y, z2, _ = window(7)
    c = np.correlate(y, x, mode="full")
    i = int(np.argmax(c))
    frac = 0.5 * (c[i - 1] - c[i + 1]) / (c[i - 1] - 2 * c[i] + c[i + 1])
    lag = (i - (len(x) - 1) + frac) * sh.dt
    v = (z2 - z1) / lag
    assert abs(v - gd["vp"]) / gd["vp"] < 0.015, v
