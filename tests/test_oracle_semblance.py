"""Pins of the oracle's semblance analysis and starting-model builder (the
starting models of the Introduction and the Numerical Examples section).

* A plane wave whose moveout is a whole number of samples per receiver has
  coherence 1 at its slowness and less elsewhere; with fractional moveout the
  peak is at the slowness grid point nearest the true one.
* Coherence does not depend on a common scale of the traces, and uncorrelated
  noise has coherence near 1/M.
* Two plane arrivals of different slowness are each recovered in their band.
* Waveforms modelled by the oracle's own solver in a fluid-filled borehole in
  a homogeneous formation give the formation P and S velocities (the S head
  wave interferes with the pseudo-Rayleigh mode, hence its wider tolerance).
* The starting model takes the wall values at r = a, the far values at and
  beyond a + dist, their mean half way, and the fluid inside the hole.
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from util import geom, oracle_models


def ricker(t, f0):
    a = (math.pi * f0 * t) ** 2
    return (1 - 2 * a) * np.exp(-a)


def plane_wave(nrec, nt, dt, spacing, s0, t0, f0, amp=None):
    off = spacing * np.arange(nrec)
    t = np.arange(nt) * dt
    amp = np.ones(nrec) if amp is None else amp
    return np.stack([amp[m] * ricker(t - t0 - s0 * off[m], f0) for m in range(nrec)]), off


def test_whole_sample_moveout_has_unit_coherence_at_its_slowness():
    dt, sp = 1e-5, 0.15
    s0 = 4 * dt / sp  # four samples per receiver
    x, off = plane_wave(8, 600, dt, sp, s0, 1e-3, 5e3)
    dp = s0 / 100
    coh = oracle.semblance(x, dt, off, s0 - 20 * dp, dp, 41, 10, 30, 200)
    j, i = np.unravel_index(np.argmax(coh), coh.shape)
    assert j == 20
    assert coh[20].max() > 1 - 1e-9
    assert coh[[0, 10, 30, 40]].max() < 0.99


@pytest.mark.parametrize("s0", [2.5e-4, 3.17e-4, 6.9e-4])
def test_fractional_moveout_peaks_at_the_nearest_grid_slowness(s0):
    dt, sp = 2e-6, 0.1524
    x, off = plane_wave(13, 3000, dt, sp, s0, 0.6e-3, 8e3)
    p0, dp = 1e-4, 1e-6
    coh = oracle.semblance(x, dt, off, p0, dp, 800, 20, 100, 300)
    p, c = oracle.pick_slowness(coh, p0, dp, 1e-4, 9e-4)
    assert abs(p - s0) <= 0.5 * dp + 1e-12
    assert c > 0.99


def test_scale_invariance_and_noise_level():
    rng = np.random.default_rng(7)
    x = rng.standard_normal((13, 4000))
    off = 0.1524 * np.arange(13)
    args = (1e-6, off, 2e-4, 1e-5, 50, 40, 90, 400)
    c1 = oracle.semblance(x, *args)
    c2 = oracle.semblance(3.5 * x, *args)
    assert np.allclose(c1, c2, rtol=1e-12, atol=0)
    assert abs(c1.mean() - 1 / 13) < 0.01


def test_two_arrivals_are_picked_in_their_bands():
    dt, sp = 1e-6, 0.1524
    xp, off = plane_wave(13, 4000, dt, sp, 1 / 4200, 0.5e-3, 12e3)
    xs, _ = plane_wave(13, 4000, dt, sp, 1 / 2400, 1.1e-3, 12e3, amp=np.full(13, 4.0))
    coh = oracle.semblance(xp + xs, dt, off, 1e-4, 1e-6, 700, 10, 350, 200)
    pP, _ = oracle.pick_slowness(coh, 1e-4, 1e-6, 1 / 6000, 1 / 3000)
    pS, _ = oracle.pick_slowness(coh, 1e-4, 1e-6, 1.4 * pP, 1 / 1500)
    assert abs(pP - 1 / 4200) <= 0.5e-6 + 1e-12
    assert abs(pS - 1 / 2400) <= 0.5e-6 + 1e-12


def test_energy_floor_ignores_faint_windows():
    """A faint early arrival (1e-4 amplitude) is perfectly coherent; with an
    energy floor of 1e-6 of the largest window energy the pick is the strong
    arrival's slowness instead."""
    dt, sp = 1e-6, 0.1524
    faint, off = plane_wave(13, 4000, dt, sp, 1 / 5000, 0.4e-3, 12e3, amp=np.full(13, 1e-4))
    strong, _ = plane_wave(13, 4000, dt, sp, 1 / 3500, 1.5e-3, 12e3)
    rng = np.random.default_rng(3)
    x = faint + strong * rng.uniform(0.5, 1.5, (13, 1)) + 1e-8 * rng.standard_normal((13, 4000))
    coh, en = oracle.semblance(x, dt, off, 1e-4, 1e-6, 400, 10, 360, 300, return_energy=True)
    p_all, _ = oracle.pick_slowness(coh, 1e-4, 1e-6, 1 / 6000, 1 / 3000)
    p_floor, _ = oracle.pick_slowness(coh, 1e-4, 1e-6, 1 / 6000, 1 / 3000, energy=en,
                                      rel_floor=1e-6)
    assert abs(p_all - 1 / 5000) <= 0.5e-6 + 1e-12
    assert abs(p_floor - 1 / 3500) <= 0.5e-6 + 1e-12


def test_starting_model_is_linear_in_radius():
    NR, NZ, dr, a, dist = 300, 3, 5e-3, 0.1, 1.0
    vp, vs = oracle.starting_model(NR, NZ, dr, a, dist, [3000, 3100, 3200], 1700,
                                   [4000, 4100, 4200], 2300, 1500)
    r = (np.arange(NR) + 0.5) * dr
    i_wall = int(np.argmax(r >= a))
    assert np.all(vp[:i_wall] == 1500) and np.all(vs[:i_wall] == 0)
    f = (r[i_wall] - a) / dist
    assert vp[i_wall, 1] == pytest.approx(3100 + f * 1000, rel=1e-14)
    i_mid = int(np.argmin(np.abs(r - (a + dist / 2))))
    f = (r[i_mid] - a) / dist
    assert vs[i_mid, 0] == pytest.approx(1700 + f * 600, rel=1e-14)
    far = r >= a + dist
    assert np.all(vp[far, 2] == 4200) and np.all(vs[far, 2] == 2300)


@pytest.mark.slow
def test_modelled_borehole_waveforms_give_the_formation_velocities():
    """Oracle waveforms of a 10 kHz monopole in a water-filled 0.1 m hole in a
    4000/2300/2300 formation, 13 receivers 0.1524 m apart from 2 m offset."""
    zr = [2.0 + 0.1524 * j for j in range(13)]
    w = workloads.single_shot_homogeneous(nz=900, nt=7000, z_rec=zr, name="semblance")
    sh = w.shots[0]
    lam, mu, rho = oracle_models(w, 0, "start")
    d = oracle.forward(geom(sh), lam, mu, rho, sh.wavelet)
    off = (np.asarray(sh.rec_k) - sh.rec_k[0]) * sh.dz
    win = int(round(0.15e-3 / sh.dt))
    p0, dp, stride = 1.5e-4, 1e-6, 10
    coh, en = oracle.semblance(d, sh.dt, off, p0, dp, 560, stride, (sh.nt - win) // stride + 1,
                               win, return_energy=True)
    pP, _ = oracle.pick_slowness(coh, p0, dp, 1 / 6000, 1 / 2000, energy=en, rel_floor=1e-6)
    pS, _ = oracle.pick_slowness(coh, p0, dp, 1.4 * pP, 0.999 / 1500, energy=en, rel_floor=1e-6)
    assert abs(1 / pP - 4000) / 4000 < 0.015, 1 / pP
    assert abs(1 / pS - 2300) / 2300 < 0.03, 1 / pS
