"""The seeded synthetic workloads against the recipe they stand for: grid,
time step, record, source, receivers, the fluid-filled borehole and the
formation value ranges of each configuration, and determinism of the seeds.
(CPU only: the generators hold no arithmetic of the method.)"""
import math

import numpy as np
import pytest

import workloads as W


def _fluid_ok(w, sh, s=0):
    # water in every cell whose centre radius is below 0.1 m, formation outside
    r = (np.arange(sh.NR) + 0.5) * sh.dr
    fl = r < W.BOREHOLE_RADIUS
    for arr, val in ((w.vp_start, W.FLUID_VP), (w.vs_start, 0.0), (w.rho, W.FLUID_RHO),
                     (w.vp_true, W.FLUID_VP), (w.vs_true, 0.0)):
        win = w.window(arr, s)
        assert np.all(win[fl] == val)
        assert np.all(win[~fl] != val) or val == W.FLUID_VP
    assert np.all(w.window(w.vs_start, s)[~fl] > 0)
    # the inversion mask: formation cells of the physical grid only
    m = w.window(w.mask, s)
    assert not m[fl].any() and not m[sh.nr:].any()
    # the axial PML where the window meets an end of the global model
    # (elsewhere a window's axial PML columns are other shots' formation)
    if sh.win_k0 == 0:
        assert not m[:, :sh.pz].any()
    if sh.win_k0 + sh.NZ == w.NZg:
        assert not m[:, sh.NZ - sh.pz:].any()
    assert m[~fl][: sh.nr - fl.sum(), sh.pz: sh.NZ - sh.pz].all()


def _rows(sh, zs):
    return [W.row_of(z, sh.dz, sh.pz) for z in zs]


def test_single_shot_128x512():
    w = W.make("c1")
    (sh,) = w.shots
    assert (sh.nr, sh.nz, sh.pr, sh.pz, sh.NR, sh.NZ) == (128, 512, 20, 20, 148, 552)
    assert (sh.dr, sh.dz, sh.dt, sh.nt, sh.f0) == (5e-3, 5e-3, 0.5e-6, 4000, 10e3)
    assert sh.src_k == _rows(sh, [0.3])[0] == 80
    assert list(sh.rec_k) == _rows(sh, [1.5 + 0.15 * j for j in range(8)])
    _fluid_ok(w, sh)
    form = (np.arange(sh.NR) + 0.5) * sh.dr >= 0.1
    assert np.all(w.vp_start[form] == 4000) and np.all(w.vs_start[form] == 2300)
    assert np.all(w.rho[form] == 2300)
    # the true model: a 0.1 m damaged zone with Vp and Vs 15 % lower
    r = (np.arange(sh.NR) + 0.5) * sh.dr
    dmg = (r >= 0.1) & (r < 0.2)
    np.testing.assert_allclose(w.vp_true[dmg], 0.85 * 4000)
    np.testing.assert_allclose(w.vs_true[dmg], 0.85 * 2300)
    assert np.all(w.vp_true[form & ~dmg] == 4000)
    # the wavelet: a Ricker of 10 kHz sampled at the half steps
    t = (np.arange(sh.nt) + 0.5) * sh.dt
    a = (math.pi * sh.f0 * (t - 1.5 / sh.f0)) ** 2
    np.testing.assert_allclose(sh.wavelet, (1 - 2 * a) * np.exp(-a), rtol=0, atol=1e-15)


def test_single_shot_320x2048_random_formation():
    w = W.make("c2")
    (sh,) = w.shots
    assert (sh.nr, sh.nz, sh.NR, sh.NZ) == (320, 2048, 340, 2088)
    assert (sh.dr, sh.dt, sh.nt, sh.f0, len(sh.rec_k)) == (2.5e-3, 0.25e-6, 8000, 12e3, 13)
    assert list(sh.rec_k) == _rows(sh, [1.5 + 0.1524 * j for j in range(13)])
    _fluid_ok(w, sh)
    assert w.meta["iters"] == 20 and w.meta["ckpt"] == 250
    r = (np.arange(sh.NR) + 0.5) * sh.dr
    form = r >= 0.1
    vp, vs, rho = w.vp_start[form][0, 0], w.vs_start[form][0, 0], w.rho[form][0, 0]
    assert 3000 <= vp <= 5000 and 1.6 <= vp / vs <= 1.9 and 2200 <= rho <= 2600
    d, pct = w.meta["depth"], w.meta["pct"]
    assert 0.05 <= d <= 0.3 and 0.10 <= pct <= 0.25
    # damage: linear from 1 - pct at the wall to 1 at the wall + depth
    f = w.vp_true[:, 100] / w.vp_start[:, 100]
    inside = form & (r < 0.1 + d)
    np.testing.assert_allclose(f[inside], 1 - pct * (1 - (r[inside] - 0.1) / d))
    np.testing.assert_allclose(w.vs_true[form, 100] / w.vs_start[form, 100], f[form])
    assert np.all(f[r >= 0.1 + d] == 1)


def test_64_shot_layered_batch():
    w = W.make("c3")
    assert len(w.shots) == 64
    step = int(round(0.15 / 2.5e-3))
    for s, sh in enumerate(w.shots):
        assert (sh.nr, sh.nz, sh.NR, sh.NZ, sh.win_k0) == (256, 4096, 276, 4136, s * step)
        assert (sh.dt, sh.nt, sh.f0, len(sh.rec_k)) == (0.25e-6, 8000, 10e3, 13)
        # stability of the staggered step in every window
        assert sh.vmax * sh.dt * math.sqrt(2) / sh.dr < 1
    assert w.NZg == 63 * step + 4136
    for s in (0, 63):
        _fluid_ok(w, w.shots[s], s)
    form = w.mask.astype(bool)
    vp, vs, rho = w.vp_start[form], w.vs_start[form], w.rho[form]
    assert vp.min() >= 2500 and vp.max() <= 5500
    assert (vp / vs).min() >= 1.6 - 1e-12 and (vp / vs).max() <= 2.0 + 1e-12
    assert rho.min() >= 2100 and rho.max() <= 2700
    # layered: several distinct layers along z, each 0.2 - 1.0 m thick
    col = w.vp_start[-1]
    edges = np.flatnonzero(np.diff(col)) + 1
    assert len(edges) >= 10
    thick = np.diff(edges) * 2.5e-3
    assert thick.min() >= 0.2 - 2.5e-3 and thick.max() <= 1.0 + 2.5e-3
    # damage only lowers the velocities, the true model keeps the layering
    assert np.all(w.vp_true[form] <= vp.max()) and np.all(w.vp_true <= w.vp_start + 1e-9)


def test_96_ragged_shots():
    w = W.make("c4")
    assert len(w.shots) == 96
    k0 = 0
    slow = 0
    for s, sh in enumerate(w.shots):
        assert sh.nz in range(1024, 6145, 512) and sh.nr in (128, 256, 384)
        assert 5e3 <= sh.f0 <= 20e3
        assert sh.vmax * sh.dt / sh.dr == pytest.approx(0.5)  # Courant number 0.5
        assert 1e-3 <= sh.nt * sh.dt < 4e-3 + sh.dt
        assert sh.win_k0 == k0  # each shot owns its own stretch of the global model
        k0 += sh.NZ
        form = w.window(w.mask, s).astype(bool)
        vs = w.window(w.vs_start, s)[form]
        if vs.max() < W.FLUID_VP:
            slow += 1
            assert 900 <= vs.min() and vs.max() <= 1400
        assert sh.rec_k.max() < sh.NZ - sh.pz and sh.src_k >= sh.pz
    assert w.NZg == k0
    assert 10 <= slow <= 40  # about a quarter are slow formations
    assert len({(sh.nr, sh.nz, sh.nt) for sh in w.shots}) > 48


def test_128_shot_large_grid_parameters():
    w = W.make("c5", nshot=2)  # the per-shot parameters of the 128-shot batch
    for sh in w.shots:
        assert (sh.nr, sh.nz, sh.NR, sh.NZ) == (512, 16384, 532, 16424)
        assert (sh.dt, sh.nt, sh.f0, len(sh.rec_k)) == (0.25e-6, 16000, 8e3, 13)
    assert w.meta["iters"] == 10 and w.meta["line_search"]


def test_seeds_are_deterministic():
    a, b = W.make("c2"), W.make("c2")
    for f in ("vp_true", "vs_true", "vp_start", "vs_start", "rho", "mask"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    c, d = W.make("c4"), W.make("c4")
    assert [(s.nr, s.nz, s.nt, s.f0) for s in c.shots] == [(s.nr, s.nz, s.nt, s.f0) for s in d.shots]
