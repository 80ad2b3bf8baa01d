"""FP64 CPU oracle for monopole borehole acoustic FWI -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never does, and shares no code with it.

The wave propagation, the adjoint, the gradients, the finalize, the
preconditioner, the update and the line search live in ``orc.c`` (plain
serial C, double precision), which this module reaches through ctypes.  A few
elementwise extensions are written here in plain float64 numpy instead:
``precondition_diag``, ``radial_taper``, ``update_density`` and
``pick_slowness``.  Each function names the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_SO = os.path.join(_HERE, "liborc.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile liborc.so with gcc (plain -O2, no fast-math, serial)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Geom(C.Structure):
    _fields_ = [
        ("nr", C.c_int32), ("nz", C.c_int32), ("pr", C.c_int32), ("pz", C.c_int32),
        ("dr", C.c_double), ("dz", C.c_double), ("dt", C.c_double),
        ("nt", C.c_int32),
        ("f0", C.c_double), ("vmax", C.c_double),
        ("src_k", C.c_int32), ("nrec", C.c_int32),
        ("rec_k", C.POINTER(C.c_int32)),
    ]


_D = C.POINTER(C.c_double)
_U8 = C.POINTER(C.c_uint8)


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_SO)
        G = C.POINTER(_Geom)
        lib.orc_moduli.argtypes = [C.c_int64, _D, _D, _D, _D, _D]
        lib.orc_velocities.argtypes = [C.c_int64, _D, _D, _D, _D, _D]
        lib.orc_moduli_grad.argtypes = [C.c_int64, _D, _D, _D, _D, _D, _D, _D, _D]
        lib.orc_forward.argtypes = [G, _D, _D, _D, _D, _D, _D]
        lib.orc_forward.restype = C.c_int
        lib.orc_misfit.argtypes = [C.c_int64, _D, _D, _D]
        lib.orc_misfit.restype = C.c_double
        lib.orc_gradient.argtypes = [G, _D, _D, _D, _D, _D, C.c_int32, _D, _D, _D, _D, _D,
                                     _D]
        lib.orc_gradient.restype = C.c_int
        lib.orc_forward_asm.argtypes = [G, C.c_int32, _D, _D, _D, _D, _D, _D]
        lib.orc_forward_asm.restype = C.c_int
        lib.orc_propagate_asm.argtypes = [G, C.c_int32, _D, _D, _D, _D, C.c_int32, C.c_int32]
        lib.orc_propagate_asm.restype = C.c_int
        lib.orc_gradient_asm.argtypes = [G, C.c_int32, _D, _D, _D, _D, _D, C.c_int32, _D, _D,
                                         _D, _D, _D, _D]
        lib.orc_gradient_asm.restype = C.c_int
        lib.orc_source_adjoint.argtypes = [G, _D, _D, _D, _D, _D]
        lib.orc_source_adjoint.restype = C.c_int
        lib.orc_state_len.argtypes = [G]
        lib.orc_state_len.restype = C.c_int64
        lib.orc_propagate.argtypes = [G, _D, _D, _D, _D, C.c_int32]
        lib.orc_propagate.restype = C.c_int
        lib.orc_propagate_adjoint.argtypes = [G, _D, _D, _D, _D, C.c_int32]
        lib.orc_propagate_adjoint.restype = C.c_int
        lib.orc_precondition.argtypes = [C.c_int64, _D, _U8, C.c_double, _D, _D]
        lib.orc_precondition.restype = C.c_double
        lib.orc_line_search.argtypes = [C.c_double] * 4
        I32 = C.c_int32
        lib.orc_semblance.argtypes = [I32, I32, _D, C.c_double, _D, I32, C.c_double, C.c_double,
                                      I32, I32, I32, _D, _D]
        lib.orc_starting_model.argtypes = [I32, I32, C.c_double, C.c_double, C.c_double, _D, _D,
                                           _D, _D, C.c_double, _D, _D]
        lib.orc_line_search.restype = C.c_double
        lib.orc_update.argtypes = [C.c_int64, _D, _D, _D, _D, _D, _U8, C.c_double,
                                   C.c_double, C.c_double, C.c_double, C.c_double,
                                   C.c_double]
        lib.orc_update.restype = C.c_double
        _lib = lib
    return _lib


@dataclass
class Geom:
    """One shot: physical grid nr x nz, PML widths, spacing, time axis, PML
    constants, on-axis source row and receiver rows (padded-grid C rows)."""
    nr: int
    nz: int
    pr: int
    pz: int
    dr: float
    dz: float
    dt: float
    nt: int
    f0: float
    vmax: float
    src_k: int
    rec_k: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))

    @property
    def NR(self) -> int:
        return self.nr + self.pr

    @property
    def NZ(self) -> int:
        return self.nz + 2 * self.pz

    def _c(self):
        rk = np.ascontiguousarray(self.rec_k, dtype=np.int32)
        g = _Geom(self.nr, self.nz, self.pr, self.pz, self.dr, self.dz, self.dt,
                  self.nt, self.f0, self.vmax, self.src_k, len(rk),
                  rk.ctypes.data_as(C.POINTER(C.c_int32)))
        return g, rk  # keep rk alive


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        a = a.reshape(shape)
    return a


def _p(a):
    return a.ctypes.data_as(_D)


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s rejected its input" % what)


def moduli(vp, vs, rho):
    """Eq. 3-4."""
    vp, vs, rho = _f64(vp), _f64(vs), _f64(rho)
    lam, mu = np.empty_like(vp), np.empty_like(vp)
    _load().orc_moduli(vp.size, _p(vp), _p(vs), _p(rho), _p(lam), _p(mu))
    return lam, mu


def moduli_grad(vp, vs, rho, glam, gmu, density=False):
    """Chain rule of Eq. 3-4: (dJ/dVp, dJ/dVs) from (dJ/dlambda, dJ/dmu); with
    density=True also the moduli's share of dJ/drho at fixed velocities."""
    vp, vs, rho, gl, gm = (_f64(a) for a in (vp, vs, rho, glam, gmu))
    gvp, gvs = np.empty_like(vp), np.empty_like(vp)
    gr = np.empty_like(vp) if density else None
    _load().orc_moduli_grad(vp.size, _p(vp), _p(vs), _p(rho), _p(gl), _p(gm), _p(gvp), _p(gvs),
                            _p(gr) if density else None)
    return (gvp, gvs, gr) if density else (gvp, gvs)


def velocities(lam, mu, rho):
    """Eq. 11-12."""
    lam, mu, rho = _f64(lam), _f64(mu), _f64(rho)
    vp, vs = np.empty_like(lam), np.empty_like(lam)
    _load().orc_velocities(lam.size, _p(lam), _p(mu), _p(rho), _p(vp), _p(vs))
    return vp, vs


def forward(g: Geom, lam, mu, rho, wavelet, return_state=False, order=2, assembled=False):
    """Eq. 2 forward modelling; returns traces [nrec, nt] (and the final state,
    14 x NR x NZ, when asked).  order=4, or assembled=True, runs the
    assembled-operator step (orc_forward_asm) of that spatial order."""
    shp = (g.NR, g.NZ)
    lam, mu, rho = _f64(lam, shp), _f64(mu, shp), _f64(rho, shp)
    w = _f64(wavelet)
    assert w.size >= g.nt
    gc, rk = g._c()
    tr = np.zeros((len(rk), g.nt))
    st = np.zeros((14,) + shp) if return_state else None
    if order != 2 or assembled:
        rc = _load().orc_forward_asm(C.byref(gc), int(order), _p(lam), _p(mu), _p(rho), _p(w),
                                     _p(tr), _p(st) if st is not None else None)
        _check(rc, "forward_asm")
        return (tr, st) if return_state else tr
    rc = _load().orc_forward(C.byref(gc), _p(lam), _p(mu), _p(rho), _p(w), _p(tr),
                             _p(st) if st is not None else None)
    _check(rc, "forward")
    return (tr, st) if return_state else tr


def misfit(d, dobs):
    """Eq. 1 and 5: returns (J, resid)."""
    d, dobs = _f64(d), _f64(dobs)
    r = np.empty_like(d)
    J = _load().orc_misfit(d.size, _p(d), _p(dobs), _p(r))
    return J, r


def gradient(g: Geom, lam, mu, rho, wavelet, resid, seg=200, density=False, hessian=False,
             order=2, assembled=False):
    """Eq. 6-8 via the exact discrete transpose; returns (glam, gmu, illum),
    then dJ/drho with density=True, then (H_lambda, H_mu), the
    virtual-source pseudo-Hessian diagonal, with hessian=True.  order=4, or
    assembled=True, uses the assembled operators."""
    shp = (g.NR, g.NZ)
    lam, mu, rho = _f64(lam, shp), _f64(mu, shp), _f64(rho, shp)
    w, r = _f64(wavelet), _f64(resid)
    gc, rk = g._c()
    assert r.size == len(rk) * g.nt
    gl, gm, il = np.zeros(shp), np.zeros(shp), np.zeros(shp)
    gr = np.zeros(shp) if density else None
    hl, hm = (np.zeros(shp), np.zeros(shp)) if hessian else (None, None)
    opt = lambda a: _p(a) if a is not None else None  # noqa: E731
    if order != 2 or assembled:
        rc = _load().orc_gradient_asm(C.byref(gc), int(order), _p(lam), _p(mu), _p(rho), _p(w),
                                      _p(r), int(seg), _p(gl), _p(gm), _p(il), opt(gr),
                                      opt(hl), opt(hm))
        _check(rc, "gradient_asm")
    else:
        rc = _load().orc_gradient(C.byref(gc), _p(lam), _p(mu), _p(rho), _p(w), _p(r),
                                  int(seg), _p(gl), _p(gm), _p(il), opt(gr), opt(hl), opt(hm))
        _check(rc, "gradient")
    out = (gl, gm, il)
    if density:
        out += (gr,)
    if hessian:
        out += (hl, hm)
    return out


def source_adjoint(g: Geom, lam, mu, rho, resid):
    """Transpose of wavelet -> traces (dot-product test)."""
    shp = (g.NR, g.NZ)
    lam, mu, rho = _f64(lam, shp), _f64(mu, shp), _f64(rho, shp)
    r = _f64(resid)
    gc, rk = g._c()
    out = np.zeros(g.nt)
    rc = _load().orc_source_adjoint(C.byref(gc), _p(lam), _p(mu), _p(rho), _p(r), _p(out))
    _check(rc, "source_adjoint")
    return out


def propagate(g: Geom, lam, mu, rho, state, nsteps, adjoint=False, order=2, assembled=False):
    """nsteps source-free steps (or their exact transpose) on a full state."""
    shp = (g.NR, g.NZ)
    lam, mu, rho = _f64(lam, shp), _f64(mu, shp), _f64(rho, shp)
    st = np.array(state, dtype=np.float64, order="C", copy=True)
    gc, rk = g._c()
    lib = _load()
    assert st.size == lib.orc_state_len(C.byref(gc))
    if order != 2 or assembled:
        _check(lib.orc_propagate_asm(C.byref(gc), int(order), _p(lam), _p(mu), _p(rho), _p(st),
                                     int(nsteps), 1 if adjoint else 0), "propagate_asm")
        return st
    fn = lib.orc_propagate_adjoint if adjoint else lib.orc_propagate
    _check(fn(C.byref(gc), _p(lam), _p(mu), _p(rho), _p(st), int(nsteps)), "propagate")
    return st


def precondition(illum, mask, eps, g_lam, g_mu, return_gpg=False):
    """Diagonal preconditioner P = 1/(E + eps max E) applied to both gradients;
    with return_gpg also sum(g . P g) over mask cells."""
    il = _f64(illum)
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    gl, gm = np.array(g_lam, np.float64, order="C"), np.array(g_mu, np.float64, order="C")
    gpg = _load().orc_precondition(il.size, _p(il), m.ctypes.data_as(_U8), float(eps),
                                   _p(gl), _p(gm))
    return (gl, gm, gpg) if return_gpg else (gl, gm)


def precondition_diag(g, mask, eps, diag=None, row_weight=None, return_gpg=False):
    """A general diagonal preconditioner for one gradient [NR, NZ] (the paper
    fixes only that it is diagonal): P = w[i] / (d + eps max_mask d) on mask
    cells, 0 elsewhere, d = diag (P = w without it), w = row_weight per
    radial row (1 without it).  With return_gpg also sum over mask of g P g."""
    g = np.array(g, np.float64)
    mk = np.asarray(mask).astype(bool)
    p = np.ones_like(g)
    if diag is not None:
        d = np.asarray(diag, np.float64)
        p = 1.0 / (d + eps * np.abs(d[mk]).max())
    if row_weight is not None:
        p = p * np.asarray(row_weight, np.float64)[:, None]
    p = np.where(mk, p, 0.0)
    gpg = float((g * p * g).sum())
    out = g * p
    return (out, gpg) if return_gpg else out


def radial_taper(NR, dr, r0, r1):
    """Weight per radial row of C cells (r = (i + 1/2) dr): 0 inside r0,
    sin^2 ramp to 1 at r1, 1 beyond; mutes the gradient next to the
    borehole wall where the guided waves dominate it."""
    r = (np.arange(NR) + 0.5) * dr
    x = np.clip((r - r0) / max(r1 - r0, 1e-30), 0.0, 1.0)
    return np.sin(0.5 * np.pi * x) ** 2


def update_density(rho, g_rho, mask, eta, rho_min, rho_max):
    """Density step of a joint inversion: alpha = eta max|rho| / max|g| over
    mask cells, rho - alpha g clamped to [rho_min, rho_max] there; returns
    (rho, alpha)."""
    r = np.array(rho, np.float64)
    g = np.asarray(g_rho, np.float64)
    mk = np.asarray(mask).astype(bool)
    gmax = np.abs(g[mk]).max()
    alpha = eta * np.abs(r[mk]).max() / gmax if gmax > 0 else 0.0
    r[mk] = np.clip(r[mk] - alpha * g[mk], rho_min, rho_max)
    return r, alpha


def line_search(J0, J1, gpg, alpha1):
    """Parabolic step length (reading of the step rule of Eq. 9-10)."""
    return _load().orc_line_search(float(J0), float(J1), float(gpg), float(alpha1))


def update(lam, mu, rho, g_lam, g_mu, mask, eta, alpha_override=0.0,
           vp_bounds=(0.0, 1e30), vs_bounds=(0.0, 1e30)):
    """Eq. 9-10 with the max-change rule for alpha; returns (lam, mu, alpha)."""
    l, m = np.array(lam, np.float64, order="C"), np.array(mu, np.float64, order="C")
    r, gl, gm = _f64(rho), _f64(g_lam), _f64(g_mu)
    mk = np.ascontiguousarray(mask, dtype=np.uint8)
    a = _load().orc_update(l.size, _p(l), _p(m), _p(r), _p(gl), _p(gm),
                           mk.ctypes.data_as(_U8), float(eta), float(alpha_override),
                           float(vp_bounds[0]), float(vp_bounds[1]),
                           float(vs_bounds[0]), float(vs_bounds[1]))
    return l, m, a


def semblance(traces, dt, offset, p0, dp, np_, tau_stride, ntau, win, return_energy=False):
    """Slowness-time coherence map [np_, ntau] of traces [nrec, nt] (the
    semblance analysis of the Introduction and Fig. 4); with return_energy
    also the window energies (the denominators)."""
    x = _f64(traces)
    nrec, nt = x.shape
    off = _f64(offset)
    assert off.size == nrec
    coh, en = np.zeros((np_, ntau)), np.zeros((np_, ntau))
    _load().orc_semblance(nrec, nt, _p(x), float(dt), _p(off), int(np_), float(p0), float(dp),
                          int(ntau), int(tau_stride), int(win), _p(coh), _p(en))
    return (coh, en) if return_energy else coh


def pick_slowness(coh, p0, dp, p_lo, p_hi, energy=None, rel_floor=0.0):
    """The slowness of the largest coherence among slownesses in [p_lo, p_hi],
    over the windows whose energy is at least rel_floor times the largest
    window energy (all windows without energy): (p, coherence)."""
    c = np.asarray(coh, np.float64)
    if energy is not None:
        e = np.asarray(energy)
        c = np.where(e >= rel_floor * e.max(), c, -1.0)
    p = p0 + dp * np.arange(c.shape[0])
    band = (p >= p_lo) & (p <= p_hi)
    best = c[band].max(axis=1)
    j = int(np.argmax(best))
    return float(p[band][j]), float(best[j])


def starting_model(NR, NZ, dr, a, dist, vp_wall, vs_wall, vp_far, vs_far, vp_fluid):
    """Velocities linear in radius from the wall values to the far values at
    a + dist (Numerical Examples section); per-row inputs of length NZ."""
    args = [_f64(np.broadcast_to(np.asarray(v, np.float64), (NZ,)))
            for v in (vp_wall, vs_wall, vp_far, vs_far)]
    vp, vs = np.zeros((NR, NZ)), np.zeros((NR, NZ))
    _load().orc_starting_model(int(NR), int(NZ), float(dr), float(a), float(dist),
                               *[_p(v) for v in args], float(vp_fluid), _p(vp), _p(vs))
    return vp, vs
