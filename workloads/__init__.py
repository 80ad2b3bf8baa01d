"""Seeded synthetic workloads for borehole acoustic FWI.

This module builds INPUTS only: earth models (P velocity, S velocity, density),
acquisition geometry (grid, source and receiver rows), the source wavelet
samples and the time axis.  It holds none of the method's arithmetic (no
moduli, no wave propagation, no gradient), so both the FP64 oracle and the HIP
path can be fed from it without sharing any computation.

There is no public dataset in the paper (every test in it is synthetic and its
model values exist only in figures), so the workloads below stand in for the
paper's layered and flushed-zone models: a fluid-filled borehole of radius
0.1 m (water, 1500 m/s, 1000 kg/m^3) in a formation with radial damage and,
for the batched cases, axial layering.

Conventions shared by every workload:
  * padded grid NR = nr + pr radial rows, NZ = nz + 2 pz axial rows, k contiguous;
  * C cell (i, k) is centred at r = (i + 1/2) dr, z = (k - pz) dz
    (z measured from the first physical row of the shot);
  * a cell is fluid when its centre radius is below the borehole radius;
  * source and receivers sit on the axis; their rows are
    pz + floor(z / dz + 1/2);
  * the wavelet is a Ricker of peak frequency f0 delayed by 1.5 / f0, sampled at
    t = (n + 1/2) dt (the half step where the leapfrog adds the source);
  * every shot is a window of one global model: shot s reads global rows
    [win_k0, win_k0 + NZ) and radial rows [0, NR).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

SEED = 200500281
BOREHOLE_RADIUS = 0.1
FLUID_VP = 1500.0
FLUID_RHO = 1000.0
REC_SPACING_HALF_FOOT = 0.1524


@dataclass
class Shot:
    nr: int
    nz: int
    pr: int
    pz: int
    dr: float
    dz: float
    dt: float
    nt: int
    f0: float          # Ricker peak frequency; also sets the PML frequency shift
    vmax: float        # PML damping reference velocity (max Vp in the window)
    src_k: int
    rec_k: np.ndarray  # int32
    wavelet: np.ndarray  # float64 [nt]
    win_k0: int = 0    # first global row of this shot's window

    @property
    def NR(self) -> int:
        return self.nr + self.pr

    @property
    def NZ(self) -> int:
        return self.nz + 2 * self.pz

    @property
    def cells(self) -> int:
        return self.NR * self.NZ


@dataclass
class Workload:
    name: str
    shots: List[Shot]
    NRg: int
    NZg: int
    vp_true: np.ndarray
    vs_true: np.ndarray
    vp_start: np.ndarray
    vs_start: np.ndarray
    rho: np.ndarray
    mask: np.ndarray   # uint8: 1 on formation cells that the inversion may change
    meta: dict = field(default_factory=dict)

    def window(self, arr: np.ndarray, s: int) -> np.ndarray:
        sh = self.shots[s]
        return arr[: sh.NR, sh.win_k0: sh.win_k0 + sh.NZ]

    @property
    def cell_steps(self) -> int:
        return sum(sh.cells * sh.nt for sh in self.shots)


def ricker(f0: float, dt: float, nt: int) -> np.ndarray:
    t = (np.arange(nt) + 0.5) * dt
    a = (math.pi * f0 * (t - 1.5 / f0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def row_of(z: float, dz: float, pz: int) -> int:
    return int(pz + math.floor(z / dz + 0.5 + 1e-9))


def _radii(NR: int, dr: float) -> np.ndarray:
    return (np.arange(NR) + 0.5) * dr


def _fill_borehole(vp, vs, rho, dr, a=BOREHOLE_RADIUS):
    fl = _radii(vp.shape[0], dr) < a
    vp[fl, :] = FLUID_VP
    vs[fl, :] = 0.0
    rho[fl, :] = FLUID_RHO
    return fl


def _damage_factor(r, a, depth, pct):
    """1 - pct at the wall, rising linearly to 1 at a + depth."""
    f = np.ones_like(r)
    if depth > 0:
        inside = (r >= a) & (r < a + depth)
        f[inside] = 1.0 - pct * (1.0 - (r[inside] - a) / depth)
    return f


def _mask(NRg, NZg, nr, pz, fluid_rows):
    m = np.zeros((NRg, NZg), np.uint8)
    m[:nr, pz: NZg - pz] = 1
    m[fluid_rows, :] = 0
    return m


def _shot(nr, nz, pr, pz, h, dt, nt, f0, vmax, z_src, z_rec, k0=0):
    rec = np.array([row_of(z, h, pz) for z in z_rec], np.int32)
    return Shot(nr, nz, pr, pz, h, h, dt, nt, f0, float(vmax), row_of(z_src, h, pz), rec,
                ricker(f0, dt, nt), k0)


# --------------------------------------------------------------------------
# Single-shot workloads
# --------------------------------------------------------------------------
def single_shot_homogeneous(nr=128, nz=512, h=5e-3, p=20, dt=0.5e-6, nt=4000, f0=10e3,
                            formation=(4000.0, 2300.0, 2300.0), damage=(0.1, 0.15),
                            z_src=0.3, z_rec=None, name="c1") -> Workload:
    """128 x 512 cells of 5 mm, 20-cell PML, homogeneous formation 4000/2300/2300
    around a water-filled hole of 0.1 m; the true model has a 0.1 m damaged zone
    with Vp and Vs reduced by 15 %; 10 kHz Ricker at z = 0.3 m; 8 receivers at
    z = 1.50 ... 2.55 m; dt = 0.5 us, 4000 steps."""
    if z_rec is None:
        z_rec = [1.5 + 0.15 * j for j in range(8)]
    NR, NZ = nr + p, nz + 2 * p
    vp = np.full((NR, NZ), formation[0])
    vs = np.full((NR, NZ), formation[1])
    rho = np.full((NR, NZ), formation[2])
    fl = _fill_borehole(vp, vs, rho, h)
    vp_s, vs_s = vp.copy(), vs.copy()
    r = _radii(NR, h)
    dz_ = (r >= BOREHOLE_RADIUS) & (r < BOREHOLE_RADIUS + damage[0])
    vp_t, vs_t = vp.copy(), vs.copy()
    vp_t[dz_, :] *= 1.0 - damage[1]
    vs_t[dz_, :] *= 1.0 - damage[1]
    shot = _shot(nr, nz, p, p, h, dt, nt, f0, vp_t.max(), z_src, z_rec)
    return Workload(name, [shot], NR, NZ, vp_t, vs_t, vp_s, vs_s, rho,
                    _mask(NR, NZ, nr, p, fl), meta=dict(iters=1, ckpt=250))


def single_shot_random(seed=SEED, name="c2", nr=320, nz=2048, h=2.5e-3, p=20, dt=0.25e-6,
                       nt=8000, f0=12e3, nrec=13, iters=20, ckpt=250) -> Workload:
    """320 x 2048 cells of 2.5 mm; background Vp U[3000,5000], Vs = Vp/U[1.6,1.9],
    rho U[2200,2600]; radial damaged zone of depth U[0.05,0.3] m with Vp and Vs
    reduced linearly by U[10,25] % at the wall; 12 kHz Ricker; 13 receivers at
    0.1524 m from z = 1.5 m; 8000 steps of 0.25 us."""
    rng = np.random.default_rng([seed, 2, 0])
    vpb = rng.uniform(3000, 5000)
    vsb = vpb / rng.uniform(1.6, 1.9)
    rhob = rng.uniform(2200, 2600)
    depth = rng.uniform(0.05, 0.3)
    pct = rng.uniform(0.10, 0.25)
    NR, NZ = nr + p, nz + 2 * p
    vp = np.full((NR, NZ), vpb)
    vs = np.full((NR, NZ), vsb)
    rho = np.full((NR, NZ), rhob)
    fl = _fill_borehole(vp, vs, rho, h)
    vp_s, vs_s = vp.copy(), vs.copy()
    f = _damage_factor(_radii(NR, h), BOREHOLE_RADIUS, depth, pct)
    f[fl] = 1.0
    vp_t, vs_t = vp * f[:, None], vs * f[:, None]
    z_rec = [1.5 + REC_SPACING_HALF_FOOT * j for j in range(nrec)]
    shot = _shot(nr, nz, p, p, h, dt, nt, f0, max(vp_t.max(), vp_s.max()), 0.3, z_rec)
    return Workload(name, [shot], NR, NZ, vp_t, vs_t, vp_s, vs_s, rho,
                    _mask(NR, NZ, nr, p, fl),
                    meta=dict(iters=iters, ckpt=ckpt, depth=depth, pct=pct))


# --------------------------------------------------------------------------
# Layered, batched workloads
# --------------------------------------------------------------------------
def _layers(rng, z0, z1, thick=(0.2, 1.0), vp=(2500, 5500), ratio=(1.6, 2.0),
            rho=(2100, 2700), depth=(0.0, 0.3), pct=(0.10, 0.25)):
    tops, props = [], []
    z = z0
    while z < z1:
        tops.append(z)
        v = rng.uniform(*vp)
        props.append((v, v / rng.uniform(*ratio), rng.uniform(*rho), rng.uniform(*depth),
                      rng.uniform(*pct)))
        z += rng.uniform(*thick)
    return np.array(tops), props


def _layered_model(NR, NZg, h, pz, rng, **kw):
    zc = (np.arange(NZg) - pz) * h
    tops, props = _layers(rng, zc[0] - h, zc[-1] + h, **kw)
    lay = np.searchsorted(tops, zc, side="right") - 1
    r = _radii(NR, h)
    vp_s = np.empty((NR, NZg))
    vs_s = np.empty((NR, NZg))
    rho = np.empty((NR, NZg))
    vp_t = np.empty((NR, NZg))
    vs_t = np.empty((NR, NZg))
    for L, (vp, vs, rh, d, pc) in enumerate(props):
        cols = lay == L
        if not cols.any():
            continue
        f = _damage_factor(r, BOREHOLE_RADIUS, d, pc)
        vp_s[:, cols] = vp
        vs_s[:, cols] = vs
        rho[:, cols] = rh
        vp_t[:, cols] = vp * f[:, None]
        vs_t[:, cols] = vs * f[:, None]
    fl = _fill_borehole(vp_t, vs_t, rho, h)
    vp_s[fl, :] = FLUID_VP
    vs_s[fl, :] = 0.0
    return vp_t, vs_t, vp_s, vs_s, rho, fl


def batched_layered(seed=SEED, name="c3", nshot=64, nr=256, nz=4096, h=2.5e-3, p=20,
                    dt=0.25e-6, nt=8000, f0=10e3, nrec=13, step_m=0.15, iters=1,
                    ckpt=250, cfg_id=3) -> Workload:
    """nshot tool positions every step_m metres over one layered global model:
    layers U[0.2,1.0] m thick, Vp U[2500,5500], Vs = Vp/U[1.6,2.0], rho
    U[2100,2700], each with radial damage of depth U[0,0.3] m reduced linearly by
    U[10,25] %.  Each shot: nr x nz cells of h, Ricker f0 at z = 0.3 m of its
    window, 13 receivers at 0.1524 m from z = 1.5 m.  Start model: the undamaged
    layers."""
    rng = np.random.default_rng([seed, cfg_id, 0])
    step_k = int(round(step_m / h))
    NR, NZ = nr + p, nz + 2 * p
    NZg = (nshot - 1) * step_k + NZ
    vp_t, vs_t, vp_s, vs_s, rho, fl = _layered_model(NR, NZg, h, p, rng)
    z_rec = [1.5 + REC_SPACING_HALF_FOOT * j for j in range(nrec)]
    shots = []
    for s in range(nshot):
        k0 = s * step_k
        vmax = max(vp_t[:, k0:k0 + NZ].max(), vp_s[:, k0:k0 + NZ].max())
        shots.append(_shot(nr, nz, p, p, h, dt, nt, f0, vmax, 0.3, z_rec, k0))
    return Workload(name, shots, NR, NZg, vp_t, vs_t, vp_s, vs_s, rho,
                    _mask(NR, NZg, nr, p, fl), meta=dict(iters=iters, ckpt=ckpt))


def batched_uneven(seed=SEED, name="c4", nshot=96, h=2.5e-3, p=20, nrec=13,
                   nz_choices=tuple(range(1024, 6145, 512)), nr_choices=(128, 256, 384),
                   f0_range=(5e3, 20e3), rec_ms=(1.0, 4.0), slow_frac=0.25,
                   cfl=0.5) -> Workload:
    """nshot independent shots of mixed size: nz from {1024, 1536, ..., 6144}, nr from
    {128, 256, 384}, Ricker peak U[5,20] kHz, record length U[1,4] ms with dt set for
    a Courant number of 0.5.  A quarter are slow formations (Vs U[900,1400] below
    the fluid speed, Vp = Vs U[1.6,2.0]); the rest are layered as in the
    uniform batch.  Each shot owns its own stretch of the global model."""
    specs = []
    for s in range(nshot):
        rng = np.random.default_rng([seed, 4, s])
        nz = int(rng.choice(nz_choices))
        nr = int(rng.choice(nr_choices))
        f0 = rng.uniform(*f0_range)
        T = rng.uniform(*rec_ms) * 1e-3
        slow = rng.uniform() < slow_frac
        specs.append((nz, nr, f0, T, slow, rng))
    NRg = max(nr for _, nr, *_ in specs) + p
    NZg = sum(nz + 2 * p for nz, *_ in specs)
    vp_t = np.full((NRg, NZg), FLUID_VP)
    vs_t = np.zeros((NRg, NZg))
    vp_s = np.full((NRg, NZg), FLUID_VP)
    vs_s = np.zeros((NRg, NZg))
    rho = np.full((NRg, NZg), FLUID_RHO)
    mask = np.zeros((NRg, NZg), np.uint8)
    shots = []
    k0 = 0
    for nz, nr, f0, T, slow, rng in specs:
        NR, NZ = nr + p, nz + 2 * p
        if slow:
            vs_ = rng.uniform(900, 1400)
            vp_ = vs_ * rng.uniform(1.6, 2.0)
            rh = rng.uniform(2100, 2700)
            d, pc = rng.uniform(0, 0.3), rng.uniform(0.10, 0.25)
            f = _damage_factor(_radii(NR, h), BOREHOLE_RADIUS, d, pc)
            a_vp_s = np.full((NR, NZ), vp_)
            a_vs_s = np.full((NR, NZ), vs_)
            a_rho = np.full((NR, NZ), rh)
            a_vp_t = a_vp_s * f[:, None]
            a_vs_t = a_vs_s * f[:, None]
            fl = _fill_borehole(a_vp_t, a_vs_t, a_rho, h)
            a_vp_s[fl, :] = FLUID_VP
            a_vs_s[fl, :] = 0.0
        else:
            a_vp_t, a_vs_t, a_vp_s, a_vs_s, a_rho, fl = _layered_model(NR, NZ, h, p, rng)
        sl = (slice(0, NR), slice(k0, k0 + NZ))
        vp_t[sl], vs_t[sl], vp_s[sl], vs_s[sl], rho[sl] = a_vp_t, a_vs_t, a_vp_s, a_vs_s, a_rho
        m = np.zeros((NR, NZ), np.uint8)
        m[:nr, p:NZ - p] = 1
        m[fl, :] = 0
        mask[sl] = m
        vmax = max(a_vp_t.max(), a_vp_s.max(), FLUID_VP)
        dt = cfl * h / vmax
        nt = int(math.ceil(T / dt))
        Lz = nz * h
        off = min(1.2, Lz - 0.4 - (nrec - 1) * REC_SPACING_HALF_FOOT)
        z_rec = [0.3 + off + REC_SPACING_HALF_FOOT * j for j in range(nrec)]
        shots.append(_shot(nr, nz, p, p, h, dt, nt, f0, vmax, 0.3, z_rec, k0))
        k0 += NZ
    return Workload(name, shots, NRg, NZg, vp_t, vs_t, vp_s, vs_s, rho, mask,
                    meta=dict(iters=1))


# Monopole sources of the acquisition (Numerical Examples section): lower-near,
# far and ultra-far, below a 13-receiver array at 0.5 ft spacing; the tool logs
# every 0.5 ft.  The paper gives no source offsets, only that the realigned
# data form one source with 39 receivers; they are taken as 8, 21 and 34
# receiver spacings (1.22, 3.20, 5.18 m) from the source to the first receiver:
# whole multiples of the logging step (so the three sources realign onto
# common source positions) 13 steps apart (so the three arrays tile one
# contiguous 39-receiver array).
SOURCE_OFFSETS_STEPS = (8, 21, 34)


def realigned_receivers(z_src, nrec=13, spacing=REC_SPACING_HALF_FOOT,
                        offsets_steps=SOURCE_OFFSETS_STEPS):
    """Receiver depths of one realigned gather: every source kind's array, as
    it stood when that source was at z_src (3 x 13 = 39 receivers)."""
    return [z_src + (o + j) * spacing for o in offsets_steps for j in range(nrec)]


def realign(raw, offsets_steps=SOURCE_OFFSETS_STEPS):
    """Data of the logging run, raw[d][q][j] (tool depth d every 0.5 ft, source
    kind q, receiver j), re-sorted into common-source gathers out[s][q*nrec+j]
    for source positions s = 0 .. D - 1 - max(offsets): source kind q at depth
    d sits at position d - offsets_steps[q] (positions counted from the
    array's first receiver at depth 0)."""
    raw = np.asarray(raw)
    D, Q, nrec = raw.shape[:3]
    omax = max(offsets_steps)
    S = D - omax
    if S < 1:
        raise ValueError("the logging run is shorter than the largest source offset")
    out = np.empty((S, Q * nrec) + raw.shape[3:], raw.dtype)
    for s in range(S):
        for q, o in enumerate(offsets_steps):
            # source q at position s: the tool's first receiver was o steps above
            out[s, q * nrec:(q + 1) * nrec] = raw[s + o, q]
    return out


def full_acquisition(seed=SEED, name="acq", nsrc=8, nr=256, h=2.5e-3, p=20, dt=0.25e-6,
                     nt=16000, f0=10e3, nrec=13, cfg_id=6) -> Workload:
    """Realigned full acquisition over the layered formation of the batched
    workloads: nsrc source positions every 0.5 ft, each shot with the 39
    receivers of the near, far and ultra-far arrays (realigned_receivers).
    Each shot's window spans 0.3 m below its source to 0.4 m above its last
    receiver; the record (nt dt = 4 ms by default) covers the S arrival at the
    farthest receiver (7 m)."""
    rng = np.random.default_rng([seed, cfg_id, 0])
    step_k = int(round(REC_SPACING_HALF_FOOT / h))
    z_rec = realigned_receivers(0.3, nrec)
    nz = int(math.ceil((z_rec[-1] + 0.4) / h))
    NR, NZ = nr + p, nz + 2 * p
    NZg = (nsrc - 1) * step_k + NZ
    vp_t, vs_t, vp_s, vs_s, rho, fl = _layered_model(NR, NZg, h, p, rng)
    shots = []
    for s in range(nsrc):
        k0 = s * step_k
        vmax = max(vp_t[:, k0:k0 + NZ].max(), vp_s[:, k0:k0 + NZ].max())
        shots.append(_shot(nr, nz, p, p, h, dt, nt, f0, vmax, 0.3, z_rec, k0))
    return Workload(name, shots, NR, NZg, vp_t, vs_t, vp_s, vs_s, rho,
                    _mask(NR, NZg, nr, p, fl), meta=dict(iters=1, ckpt=250))


def large_layered(seed=SEED, nshot=128, **kw) -> Workload:
    """128 shots of 512 x 16384 cells, 16000 steps, 8 kHz, layered + radial damage."""
    wl = batched_layered(seed=seed, name="c5", nshot=nshot, nr=512, nz=16384, nt=16000,
                         f0=8e3, iters=10, cfg_id=5, **kw)
    wl.meta["line_search"] = True
    return wl


# --------------------------------------------------------------------------
# Tiny grids for brute-force checks
# --------------------------------------------------------------------------
def tiny(seed=1, nr=24, nz=48, h=5e-3, p=6, dt=0.5e-6, nt=240, f0=40e3, nrec=3,
         hetero=True, fluid=True, name="tiny") -> Workload:
    """A small borehole model that many forward runs can afford: random smooth
    perturbations of a 3500/2000/2300 formation, a 4-cell water hole, three
    receivers.  40 kHz keeps about 7 points per S wavelength at 5 mm."""
    rng = np.random.default_rng([seed, 99, 0])
    NR, NZ = nr + p, nz + 2 * p
    vp = np.full((NR, NZ), 3500.0)
    vs = np.full((NR, NZ), 2000.0)
    rho = np.full((NR, NZ), 2300.0)
    if hetero:
        vp *= 1 + 0.05 * rng.standard_normal((NR, NZ))
        vs *= 1 + 0.05 * rng.standard_normal((NR, NZ))
        rho *= 1 + 0.05 * rng.standard_normal((NR, NZ))
    a = 4.0 * h if fluid else 0.0
    if fluid:
        fl = _fill_borehole(vp, vs, rho, h, a)
    else:
        fl = np.zeros(NR, bool)
    vp_s, vs_s = vp.copy(), vs.copy()
    vp_t, vs_t = vp.copy(), vs.copy()
    r = _radii(NR, h)
    band = (r >= a) & (r < a + 4 * h)
    vp_t[band, :] *= 0.9
    vs_t[band, :] *= 0.9
    z_src = 0.25 * nz * h
    z_rec = [(0.55 + 0.12 * j) * nz * h for j in range(nrec)]
    shot = _shot(nr, nz, p, p, h, dt, nt, f0, max(vp_t.max(), vp_s.max()), z_src, z_rec)
    return Workload(name, [shot], NR, NZ, vp_t, vs_t, vp_s, vs_s, rho,
                    _mask(NR, NZ, nr, p, fl), meta=dict(iters=1, ckpt=50))


CONFIGS = {
    "c1": single_shot_homogeneous,
    "c2": single_shot_random,
    "c3": batched_layered,
    "c4": batched_uneven,
    "c5": large_layered,
    "acq": full_acquisition,
}


def make(name: str, **kw) -> Workload:
    if name == "tiny":
        return tiny(**kw)
    return CONFIGS[name](**kw)
