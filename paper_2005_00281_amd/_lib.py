"""ctypes binding of libbhfwi (include/bhfwi.h).  Argument marshalling only:
every step of the path runs in the library's HIP kernels; torch supplies
device memory and the current stream.  Raises if the library is missing --
there is no fallback."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbhfwi.so")

BHFWI_STORE_CKPT = 1
BHFWI_ENOMEM = -3
_ERRORS = {-1: "EINVAL", -2: "ECFL", -3: "ENOMEM", -4: "EHIP", -5: "ENONFINITE",
           -6: "EUNSUPPORTED"}


class BhfwiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("bhfwi %s (%d): %s" % (_ERRORS.get(code, "?"), code, msg))
        self.code = code
        self.name = _ERRORS.get(code, "?")


class Shot(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nz", C.c_int32), ("npml_r", C.c_int32),
                ("npml_z", C.c_int32), ("dr", C.c_float), ("dz", C.c_float),
                ("dt", C.c_float), ("nt", C.c_int32), ("f0", C.c_float),
                ("pml_vmax", C.c_float), ("src_k", C.c_int32), ("nrec", C.c_int32),
                ("rec_off", C.c_int32), ("pad_", C.c_int32), ("model_off", C.c_int64),
                ("model_ld", C.c_int64)]


class Sizes(C.Structure):
    _fields_ = [("fwd_ws_bytes", C.c_int64), ("ckpt_bytes", C.c_int64),
                ("adj_ws_bytes", C.c_int64), ("acc_elems", C.c_int64),
                ("trace_elems", C.c_int64), ("wavelet_elems", C.c_int64),
                ("cells", C.c_int64), ("cell_steps", C.c_int64), ("nt_max", C.c_int32),
                ("ckpt_every", C.c_int32), ("nseg", C.c_int32), ("work_items", C.c_int32)]


class Tune(C.Structure):
    _fields_ = [("rows_per_wave", C.c_int32), ("waves_per_block", C.c_int32),
                ("use_graph", C.c_int32), ("time_kernels", C.c_int32),
                ("tb_steps", C.c_int32), ("tb_rows", C.c_int32), ("tb_waves", C.c_int32),
                ("tile_map", C.c_int32), ("adj_tb_steps", C.c_int32),
                ("adj_tb_rows", C.c_int32), ("adj_tb_waves", C.c_int32),
                ("pml_overlap", C.c_int32), ("rec_overlap", C.c_int32),
                ("full_history", C.c_int32), ("fwd_tile_overlap", C.c_int32)]


class PlanBytes(C.Structure):
    _fields_ = [("ckpt_every", C.c_int32), ("pad_", C.c_int32), ("fwd_ws_bytes", C.c_int64),
                ("ckpt_bytes", C.c_int64), ("adj_ws_bytes", C.c_int64), ("acc_bytes", C.c_int64),
                ("total_bytes", C.c_int64)]


class PlanInfo(C.Structure):
    _fields_ = [("ngroups", C.c_int32), ("pad_", C.c_int32), ("workspace_bytes", C.c_int64),
                ("trace_bytes", C.c_int64)]


class KernelTimes(C.Structure):
    _fields_ = [("fwd_ms", C.c_double), ("rec_ms", C.c_double), ("adj_ms", C.c_double),
                ("fwd_launches", C.c_int64), ("rec_launches", C.c_int64),
                ("adj_launches", C.c_int64)]


class Bounds(C.Structure):
    _fields_ = [("vp_min", C.c_float), ("vp_max", C.c_float), ("vs_min", C.c_float),
                ("vs_max", C.c_float)]


EXPORTS = ["bhfwi_build_id", "bhfwi_create", "bhfwi_destroy", "bhfwi_last_error", "bhfwi_sizes",
           "bhfwi_set_tune", "bhfwi_get_tune", "bhfwi_autotune", "bhfwi_kernel_times",
           "bhfwi_moduli", "bhfwi_moduli_grad", "bhfwi_velocities",
           "bhfwi_fwd_model", "bhfwi_misfit", "bhfwi_adjoint_model", "bhfwi_gradient",
           "bhfwi_precondition", "bhfwi_status", "bhfwi_line_search", "bhfwi_update", "bhfwi_plan_bytes",
           "bhfwi_plan", "bhfwi_kernel_shapes", "bhfwi_semblance", "bhfwi_semblance_pick",
           "bhfwi_starting_model", "bhfwi_adjoint_model_density", "bhfwi_gradient_density",
           "bhfwi_adjoint_model_ex", "bhfwi_gradient_hessian", "bhfwi_precondition_diag",
           "bhfwi_radial_taper", "bhfwi_update_density", "bhfwi_set_order",
           "bhfwi_set_order4_blocks",
           "bhfwi_misfit_noalloc", "bhfwi_adjoint_model_wavelet"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libbhfwi.so; raises if it has not been built, or if it was built
    from sources other than those on disk (its build id differs)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libbhfwi.so is not built (%s); run __graft_entry__.build()" % path)
    L = C.CDLL(path)
    L.bhfwi_build_id.argtypes = []
    L.bhfwi_build_id.restype = C.c_char_p
    if path == LIB_PATH:
        from .build import source_id
        built, want = L.bhfwi_build_id().decode(), source_id()
        if built != want:
            raise RuntimeError("libbhfwi.so is stale: built from sources %s..., the sources on "
                               "disk are %s...; run __graft_entry__.build()" % (built[:12],
                                                                                want[:12]))
    P, V, I64, I32, F = C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_float
    L.bhfwi_create.argtypes = [C.POINTER(C.c_void_p), I32, C.POINTER(Shot), I32,
                               C.POINTER(C.c_int32), I32, I64, I32]
    L.bhfwi_destroy.argtypes = [P]
    L.bhfwi_destroy.restype = None
    L.bhfwi_last_error.argtypes = [P]
    L.bhfwi_last_error.restype = C.c_char_p
    L.bhfwi_sizes.argtypes = [P, C.POINTER(Sizes)]
    L.bhfwi_set_tune.argtypes = [P, C.POINTER(Tune)]
    L.bhfwi_get_tune.argtypes = [P, C.POINTER(Tune)]
    L.bhfwi_kernel_times.argtypes = [P, C.POINTER(KernelTimes), I32]
    L.bhfwi_autotune.argtypes = [P, V, P, P, P, P, P, P, I64, P, I64, P, I32, C.POINTER(Tune),
                                 C.POINTER(C.c_float)]
    L.bhfwi_moduli.argtypes = [V, I64, P, P, P, P, P]
    L.bhfwi_velocities.argtypes = [V, I64, P, P, P, P, P]
    L.bhfwi_moduli_grad.argtypes = [V, I64, P, P, P, P, P, P, P, P]
    L.bhfwi_fwd_model.argtypes = [P, V, P, P, P, P, P, P, I64, P, I64, I32]
    L.bhfwi_misfit.argtypes = [P, V, P, P, P, P, I32]
    L.bhfwi_misfit_noalloc.argtypes = [V, I64, P, P, P, P, I32]
    L.bhfwi_adjoint_model.argtypes = [P, V, P, P, P, P, P, P, I64, P, I64, P, I64, P]
    L.bhfwi_gradient.argtypes = [P, V, P, P, P, P, P, I32]
    L.bhfwi_adjoint_model_density.argtypes = [P, V, P, P, P, P, P, P, I64, P, I64, P, I64, P,
                                              P]
    L.bhfwi_gradient_density.argtypes = [P, V, P, P, P, I32]
    L.bhfwi_adjoint_model_ex.argtypes = [P, V, P, P, P, P, P, P, I64, P, I64, P, I64, P, P, P]
    L.bhfwi_adjoint_model_wavelet.argtypes = [P, V, P, P, P, P, P, P, I64, P, I64, P, I64, P,
                                              P]
    L.bhfwi_gradient_hessian.argtypes = [P, V, P, P, P, I32]
    L.bhfwi_precondition_diag.argtypes = [P, V, I64, I32, P, P, P, F, P, P, I32]
    L.bhfwi_radial_taper.argtypes = [V, I32, F, F, F, P]
    L.bhfwi_set_order.argtypes = [P, I32]
    L.bhfwi_set_order4_blocks.argtypes = [P, I32, I32, I32]
    L.bhfwi_update_density.argtypes = [P, V, I64, P, P, P, F, F, F, P]
    L.bhfwi_precondition.argtypes = [P, V, I64, P, P, F, P, P, P]
    L.bhfwi_line_search.argtypes = [P, V, P, P, P, P, P]
    L.bhfwi_status.argtypes = [P, V]
    L.bhfwi_kernel_shapes.argtypes = [P, C.POINTER(C.c_int32)]
    L.bhfwi_semblance.argtypes = [V, I32, I32, I32, P, F, P, I32, F, F, I32, I32, I32, P, P]
    L.bhfwi_semblance_pick.argtypes = [V, I32, I32, I32, P, P, F, F, F, P, F, F, F, P, P, P]
    L.bhfwi_starting_model.argtypes = [V, I32, I32, F, F, F, P, P, P, P, F, P, P]
    L.bhfwi_plan_bytes.argtypes = [C.POINTER(Shot), I32, I32, C.POINTER(PlanBytes)]
    L.bhfwi_plan.argtypes = [C.POINTER(Shot), I32, I64, I32, I32, C.POINTER(C.c_int32),
                             C.POINTER(C.c_int32), C.POINTER(PlanInfo)]
    L.bhfwi_update.argtypes = [P, V, I64, P, P, P, P, P, P, F, F, P, C.POINTER(Bounds), P]
    for name in EXPORTS:
        if name not in ("bhfwi_destroy", "bhfwi_last_error", "bhfwi_build_id"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _f32(t, n=None):
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous float32 device tensor")
    if n is not None and t.numel() < n:
        raise ValueError("tensor has %d elements, %d needed" % (t.numel(), n))
    return C.c_void_p(t.data_ptr())


def _f64(t):
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 device tensor")
    return C.c_void_p(t.data_ptr())


def _check(rc, ctx=None):
    if rc != 0:
        msg = load().bhfwi_last_error(ctx)
        raise BhfwiError(rc, msg.decode() if msg else "")


def moduli(vp, vs, rho, out=None):
    """Eq. 3-4 on device tensors."""
    lam, mu = out if out is not None else (torch.empty_like(vp), torch.empty_like(vp))
    _check(load().bhfwi_moduli(_stream(), vp.numel(), _f32(vp), _f32(vs), _f32(rho),
                               _f32(lam), _f32(mu)))
    return lam, mu


def moduli_grad(vp, vs, rho, g_lam, g_mu, density=False):
    """Chain rule of Eq. 3-4: (g_vp, g_vs) from (g_lam, g_mu); with density=True
    also the moduli's share of dJ/drho at fixed velocities."""
    g_vp, g_vs = torch.empty_like(vp), torch.empty_like(vp)
    g_rho = torch.empty_like(vp) if density else None
    _check(load().bhfwi_moduli_grad(_stream(), vp.numel(), _f32(vp), _f32(vs), _f32(rho),
                                    _f32(g_lam), _f32(g_mu), _f32(g_vp), _f32(g_vs),
                                    _f32(g_rho) if density else None))
    return (g_vp, g_vs, g_rho) if density else (g_vp, g_vs)


def misfit_noalloc(traces, observed, resid, J, accumulate=False):
    """bhfwi_misfit_noalloc on flat float32 device tensors of one length:
    resid = traces - observed, J (float64 device scalar) = 0.5 sum resid^2
    (or added to it).  Allocates nothing on the device."""
    n = traces.numel()
    if observed.numel() != n or resid.numel() != n:
        raise ValueError("traces, observed and resid must have one length")
    L = load()
    rc = L.bhfwi_misfit_noalloc(_stream(), n, _f32(traces), _f32(observed), _f32(resid),
                                _f64(J), 1 if accumulate else 0)
    _check(rc, None)
    return resid, J


def radial_taper(nrow, dr, r0, r1, device=None):
    """Weights per radial row for precondition_diag (bhfwi_radial_taper)."""
    w = torch.empty(nrow, dtype=torch.float32, device=device or torch.device("cuda", 0))
    _check(load().bhfwi_radial_taper(_stream(), int(nrow), float(dr), float(r0), float(r1),
                                     _f32(w)))
    return w


def semblance(traces, dt, offset, p0, dp, np_, tau_stride, ntau, win, energy=False):
    """Slowness-time coherence (bhfwi_semblance) of gathers [G, nrec, nt] (or
    one gather [nrec, nt]) with receiver offsets [G, nrec] (or [nrec]);
    returns coh [G, np_, ntau] (and the window energies)."""
    one = traces.dim() == 2
    x = traces.unsqueeze(0) if one else traces
    off = (offset.unsqueeze(0).expand(x.shape[0], -1).contiguous()
           if offset.dim() == 1 and not one else offset)
    G, nrec, nt = x.shape
    coh = torch.empty((G, np_, ntau), dtype=torch.float32, device=x.device)
    en = torch.empty_like(coh) if energy else None
    _check(load().bhfwi_semblance(_stream(), G, nrec, nt, _f32(x.contiguous()), float(dt),
                                  _f32(off.contiguous()), int(np_), float(p0), float(dp),
                                  int(ntau), int(tau_stride), int(win), _f32(coh),
                                  _f32(en) if en is not None else None))
    if one:
        coh = coh[0]
        en = en[0] if en is not None else None
    return (coh, en) if energy else coh


def semblance_pick(coh, p0, dp, p_lo, p_hi, p_ref=None, ref_scale=1.0, energy=None,
                   rel_floor=0.0, return_proj=False):
    """Slowness of the largest coherence in [max(p_lo, ref_scale p_ref), p_hi]
    over windows with energy >= rel_floor x the gather's largest, per gather
    (bhfwi_semblance_pick): (p [G], coherence [G]) device tensors, and with
    return_proj the coherence-versus-slowness projection [G, np]."""
    c = coh.unsqueeze(0) if coh.dim() == 2 else coh
    e = None if energy is None else (energy.unsqueeze(0) if energy.dim() == 2 else energy)
    G, np_, ntau = c.shape
    p = torch.empty(G, dtype=torch.float32, device=c.device)
    cc = torch.empty_like(p)
    proj = torch.empty((G, np_), dtype=torch.float32, device=c.device)
    _check(load().bhfwi_semblance_pick(_stream(), G, np_, ntau, _f32(c.contiguous()),
                                       _f32(e.contiguous()) if e is not None else None,
                                       float(rel_floor), float(p0), float(dp),
                                       _f32(p_ref) if p_ref is not None else None,
                                       float(ref_scale), float(p_lo), float(p_hi), _f32(proj),
                                       _f32(p), _f32(cc)))
    return (p, cc, proj) if return_proj else (p, cc)


def starting_model(NR, NZ, dr, a, dist, vp_wall, vs_wall, vp_far, vs_far, vp_fluid):
    """Velocities linear in radius from the wall values (per axial row, device
    tensors of NZ) to the far values at a + dist (bhfwi_starting_model)."""
    dev = vp_wall.device
    vp = torch.empty((NR, NZ), dtype=torch.float32, device=dev)
    vs = torch.empty_like(vp)
    _check(load().bhfwi_starting_model(_stream(), int(NR), int(NZ), float(dr), float(a),
                                       float(dist), _f32(vp_wall, NZ), _f32(vs_wall, NZ),
                                       _f32(vp_far, NZ), _f32(vs_far, NZ), float(vp_fluid),
                                       _f32(vp), _f32(vs)))
    return vp, vs


def velocities(lam, mu, rho, out=None):
    """Eq. 11-12 on device tensors."""
    vp, vs = out if out is not None else (torch.empty_like(lam), torch.empty_like(lam))
    _check(load().bhfwi_velocities(_stream(), lam.numel(), _f32(lam), _f32(mu), _f32(rho),
                                   _f32(vp), _f32(vs)))
    return vp, vs


# Tune fields that are not kernel choices: the history mode decides the
# memory layout (the HBM planner and use_full_history_if_fits set it from the
# budget), time_kernels is an instrumentation switch.  Tune caches neither
# store nor restore them.
NOT_CACHED = ("full_history", "time_kernels")


def cached_kernel_tune(tune):
    """The part of a tune (dict) that a tune cache keeps and re-installs."""
    return {k: v for k, v in tune.items() if k not in NOT_CACHED}


def shot_array(shots, NZg=None):
    """bhfwi_shot array and packed receiver rows for shots (see Survey)."""
    arr = (Shot * len(shots))()
    recs = []
    for s, sh in enumerate(shots):
        rk = np.asarray(sh.rec_k, np.int32)
        NZ = sh.nz + 2 * sh.pz
        arr[s] = Shot(sh.nr, sh.nz, sh.pr, sh.pz, sh.dr, sh.dz, sh.dt, sh.nt, sh.f0,
                      sh.vmax, sh.src_k, len(rk), len(recs), 0,
                      int(getattr(sh, "win_k0", 0)), NZg if NZg is not None else NZ)
        recs.extend(int(x) for x in rk)
    return arr, recs


def plan_bytes(shots, ckpt_every=0):
    """bhfwi_plan_bytes: workspace bytes of shots as one context."""
    arr, _ = shot_array(shots)
    out = PlanBytes()
    _check(load().bhfwi_plan_bytes(arr, len(shots), int(ckpt_every or 0), C.byref(out)), None)
    return out


def plan(shots, budget_bytes, ckpt_every=0, max_groups=0):
    """bhfwi_plan: (group of each shot, interval of each group, PlanInfo)."""
    arr, _ = shot_array(shots)
    n = len(shots)
    gof, kout, info = (C.c_int32 * n)(), (C.c_int32 * n)(), PlanInfo()
    rc = load().bhfwi_plan(arr, n, int(budget_bytes), int(ckpt_every or 0), int(max_groups or 0),
                           gof, kout, C.byref(info))
    if rc == BHFWI_ENOMEM:
        raise MemoryError("no grouping of %d shots fits %.1f GB" % (n, budget_bytes / 1e9))
    _check(rc, None)
    return list(gof), list(kout[:info.ngroups]), info


class Survey:
    """A set of shots over one global model, bound to one HIP device.

    shots: objects with nr, nz, pr, pz, dr, dz, dt, nt, f0, vmax, src_k,
    rec_k (int array) and win_k0 (first global row of the shot's window);
    model_shape: (NRg, NZg) of the global model."""

    def __init__(self, shots, model_shape, ckpt_every=250, device=0, order=2):
        L = load()
        self.model_shape = tuple(int(x) for x in model_shape)
        NRg, NZg = self.model_shape
        for s, sh in enumerate(shots):
            if sh.nr + sh.pr > NRg:
                raise ValueError("shot %d has more radial rows than the model" % s)
        arr, recs = shot_array(shots, NZg)
        rec_arr = (C.c_int32 * max(1, len(recs)))(*recs)
        h = C.c_void_p()
        rc = L.bhfwi_create(C.byref(h), int(device), arr, len(shots), rec_arr, len(recs),
                            NRg * NZg, int(ckpt_every))
        _check(rc, None)
        self._h = h
        self.device = torch.device("cuda", device)
        self.nshot = len(shots)
        self.shots = list(shots)
        self.order = 2
        self.sizes = Sizes()
        _check(L.bhfwi_sizes(h, C.byref(self.sizes)), h)
        self._ws = {}
        self.order4_blocks = (2, 32, 16)  # the library's default fourth-order time blocks
        if order != 2:
            self.set_order(order)

    def set_order(self, order):
        """Spatial order of the step (2 or 4, bhfwi_set_order); refreshes the
        workspace sizes."""
        _check(load().bhfwi_set_order(self._h, int(order)), self._h)
        self.order = int(order)
        _check(load().bhfwi_sizes(self._h, C.byref(self.sizes)), self._h)
        self._ws.clear()

    def set_order4_blocks(self, steps, rows=32, waves=16):
        """Time blocks of the fourth-order forward and adjoint
        (bhfwi_set_order4_blocks): steps per launch (< 2: one step per
        launch), window rows, waves."""
        _check(load().bhfwi_set_order4_blocks(self._h, int(steps), int(rows), int(waves)),
               self._h)
        self.order4_blocks = (int(steps), int(rows), int(waves)) if steps >= 2 else (0, 0, 0)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.bhfwi_destroy(h)
            self._h = None

    # ---------------------------------------------------------------- tuning
    def set_tune(self, **kw):
        """Change any subset of the bhfwi_tune fields (a value of None keeps
        the current one)."""
        names = [n for n, _ in Tune._fields_]
        bad = set(kw) - set(names)
        if bad:
            raise TypeError("unknown tunables %s" % sorted(bad))
        cur = Tune()
        _check(load().bhfwi_get_tune(self._h, C.byref(cur)), self._h)
        t = Tune(**{n: int(getattr(cur, n) if kw.get(n) is None else kw[n]) for n in names})
        _check(load().bhfwi_set_tune(self._h, C.byref(t)), self._h)
        _check(load().bhfwi_sizes(self._h, C.byref(self.sizes)), self._h)

    def device_bytes(self):
        """Device memory one gradient evaluation of this survey needs in the
        current tune: workspaces, checkpoints or full history, accumulators
        and three trace arrays (traces, residuals, observed data)."""
        z = self.sizes
        return (z.fwd_ws_bytes + z.ckpt_bytes + z.adj_ws_bytes + 4 * z.acc_elems +
                12 * z.trace_elems)

    def use_full_history_if_fits(self, budget_bytes):
        """Keep the velocity history of every step (tune full_history: no
        checkpoints, no recompute) when the survey then fits budget_bytes,
        else the checkpoints; returns whether the full history is on."""
        self.set_tune(full_history=1)
        full = self.device_bytes() <= budget_bytes
        if not full:
            self.set_tune(full_history=0)
        return full

    def kernel_shapes(self):
        """{'fwd', 'fwd_pml', 'adj', 'adj_pml', 'adj_x', 'adj_x_pml'}: (T, rows,
        waves) of the temporally blocked kernels the current tune runs, adj_x
        those of the adjoint with extra outputs (T = 0: one step per launch)."""
        out = (C.c_int32 * 18)()
        _check(load().bhfwi_kernel_shapes(self._h, out), self._h)
        names = ("fwd", "fwd_pml", "adj", "adj_pml", "adj_x", "adj_x_pml")
        return {n: tuple(out[3 * q: 3 * q + 3]) for q, n in enumerate(names)}

    def get_tune(self):
        t = Tune()
        _check(load().bhfwi_get_tune(self._h, C.byref(t)), self._h)
        return {name: getattr(t, name) for name, _ in Tune._fields_}

    def shape_key(self, nt=None):
        """Key of the autotune cache: GPU architecture and compute-unit count,
        checkpoint interval and the multiset of shot shapes (with nt, the key
        the same shots would have with records of nt steps)."""
        shapes = sorted((sh.nr + sh.pr, sh.nz + 2 * sh.pz, sh.nt if nt is None else int(nt))
                        for sh in self.shots)
        hist = {}
        for s in shapes:
            hist[s] = hist.get(s, 0) + 1
        p = torch.cuda.get_device_properties(self.device)
        arch = getattr(p, "gcnArchName", "") or torch.cuda.get_device_name(self.device)
        return "%s/%dCU|K%d|%s" % (arch.split(":")[0], p.multi_processor_count,
                                  self.sizes.ckpt_every,
                                  ";".join("%dx%dx%d*%d" % (a, b, c, n)
                                           for (a, b, c), n in sorted(hist.items())))

    def autotune(self, lam, mu, rho, wavelet, probe_steps=None, cache=None, key=None):
        """Pick the fastest kernel shape for this survey (bhfwi_autotune) and
        install it; with cache (a JSON path) reuse and record the choice under
        key (default shape_key()).  The fourth-order kernels have no shapes to
        tune: the current tune is kept."""
        import json
        if self.order != 2:
            return {"tune": self.get_tune(), "ms": None, "cached": False}
        key = key or self.shape_key()
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        if key in table:
            self.set_tune(**cached_kernel_tune(table[key]["tune"]))
            return dict(table[key], cached=True)
        full = self.get_tune()["full_history"]
        if full:  # the probe needs the checkpointed form's history in adj_ws
            self.set_tune(full_history=0)
        z = self.sizes
        if probe_steps is None:
            probe_steps = min(z.ckpt_every, z.nt_max, 256)
        tr = torch.empty(z.trace_elems, dtype=torch.float32, device=self.device)
        acc = torch.empty(z.acc_elems, dtype=torch.float32, device=self.device)
        kept = dict(self._ws)  # the probe's scratch is not kept past the call
        fw, aw = self.workspace("fwd"), self.workspace("adj")
        best, ms = Tune(), C.c_float()
        n = self.model_shape[0] * self.model_shape[1]
        _check(load().bhfwi_autotune(self._h, _stream(), _f32(lam, n), _f32(mu, n),
                                     _f32(rho, n), _f32(wavelet, z.wavelet_elems), _f32(tr),
                                     _ptr(fw), fw.numel(), _ptr(aw), aw.numel(), _f32(acc),
                                     int(probe_steps), C.byref(best), C.byref(ms)), self._h)
        del fw, aw, tr, acc
        self._ws = kept
        if full:
            best.full_history = 1
            self.set_tune(full_history=1)
        _check(load().bhfwi_sizes(self._h, C.byref(self.sizes)), self._h)
        entry = {"tune": cached_kernel_tune({name: getattr(best, name)
                                             for name, _ in Tune._fields_}),
                 "probe_ms": ms.value, "probe_steps": int(probe_steps)}
        if cache:
            table[key] = entry
            tmp = cache + ".tmp%d" % os.getpid()
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return entry

    def kernel_times(self, reset=True):
        """Sums of the per-launch event timings of the instrumented mode."""
        o = KernelTimes()
        _check(load().bhfwi_kernel_times(self._h, C.byref(o), int(reset)), self._h)
        return {"fwd": (o.fwd_ms, o.fwd_launches), "rec": (o.rec_ms, o.rec_launches),
                "adj": (o.adj_ms, o.adj_launches)}

    # ------------------------------------------------------------ workspaces
    def workspace(self, name):
        """Device scratch of this survey (torch allocations, reused; a pool
        shared by several surveys can be installed with use_workspaces)."""
        nbytes = {"fwd": self.sizes.fwd_ws_bytes, "ckpt": self.sizes.ckpt_bytes,
                  "adj": self.sizes.adj_ws_bytes}[name]
        t = self._ws.get(name)
        if t is None or t.numel() < nbytes:
            t = torch.empty(max(1, nbytes), dtype=torch.uint8, device=self.device)
            self._ws[name] = t
        return t

    def use_workspaces(self, pool):
        """Share device scratch: pool maps 'fwd', 'ckpt', 'adj' to uint8 tensors
        at least as large as this survey needs."""
        for name in ("fwd", "ckpt", "adj"):
            need = {"fwd": self.sizes.fwd_ws_bytes, "ckpt": self.sizes.ckpt_bytes,
                    "adj": self.sizes.adj_ws_bytes}[name]
            if pool[name].numel() < need:
                raise ValueError("shared %s workspace too small" % name)
        self._ws = dict(pool)

    def free_workspaces(self):
        self._ws.clear()

    def checkout_ckpt(self):
        """(buffer, token) for the checkpoints of one autograd forward: the
        survey's checkpoint workspace when no other forward holds it, else a
        fresh allocation of the same size (token None)."""
        if getattr(self, "_ckpt_owner", None) is None:
            token = object()
            self._ckpt_owner = token
            return self.workspace("ckpt"), token
        return torch.empty(max(1, self.sizes.ckpt_bytes), dtype=torch.uint8,
                           device=self.device), None

    def release_ckpt(self, token):
        """End the reservation taken by checkout_ckpt (a no-op for a token that
        no longer holds it)."""
        if token is not None and getattr(self, "_ckpt_owner", None) is token:
            self._ckpt_owner = None

    # ---------------------------------------------------------------- steps
    def fwd_model(self, lam, mu, rho, wavelet, store_ckpt=False, ckpt=None, traces=None):
        """Eq. 2 for every shot; returns packed traces (and writes checkpoints)."""
        z = self.sizes
        if traces is None:
            traces = torch.empty(z.trace_elems, dtype=torch.float32, device=self.device)
        fw = self.workspace("fwd")
        if store_ckpt and ckpt is None:
            ckpt = self.workspace("ckpt")
        n = self.model_shape[0] * self.model_shape[1]
        rc = load().bhfwi_fwd_model(
            self._h, _stream(), _f32(lam, n), _f32(mu, n), _f32(rho, n),
            _f32(wavelet, z.wavelet_elems), _f32(traces, z.trace_elems), _ptr(fw), fw.numel(),
            _ptr(ckpt) if store_ckpt else None, ckpt.numel() if store_ckpt else 0,
            BHFWI_STORE_CKPT if store_ckpt else 0)
        _check(rc, self._h)
        return traces

    def misfit(self, traces, observed, resid=None, J=None, accumulate=False):
        """Eq. 1 and 5: returns (resid, J as a 0-d float64 device tensor); with
        accumulate, J (given) is added to."""
        z = self.sizes
        if resid is None:
            resid = torch.empty(z.trace_elems, dtype=torch.float32, device=self.device)
        if J is None:
            J = torch.empty((), dtype=torch.float64, device=self.device)
        _check(load().bhfwi_misfit(self._h, _stream(), _f32(traces, z.trace_elems),
                                   _f32(observed, z.trace_elems), _f32(resid, z.trace_elems),
                                   _ptr(J), 1 if accumulate else 0), self._h)
        return resid, J

    def adjoint_model(self, lam, mu, rho, wavelet, resid, ckpt=None, acc=None):
        """Eq. 6-8 with checkpoint recompute; returns the per-shot accumulators
        [4, cells] (dJ/dlam, C part of dJ/dmu, dJ/dmu_S, illumination)."""
        z = self.sizes
        if acc is None:
            acc = torch.empty(z.acc_elems, dtype=torch.float32, device=self.device)
        if ckpt is None:
            ckpt = self.workspace("ckpt")
        fw, aw = self.workspace("fwd"), self.workspace("adj")
        n = self.model_shape[0] * self.model_shape[1]
        rc = load().bhfwi_adjoint_model(
            self._h, _stream(), _f32(lam, n), _f32(mu, n), _f32(rho, n),
            _f32(wavelet, z.wavelet_elems), _f32(resid, z.trace_elems), _ptr(fw), fw.numel(),
            _ptr(ckpt), ckpt.numel(), _ptr(aw), aw.numel(), _f32(acc, z.acc_elems))
        _check(rc, self._h)
        return acc

    def adjoint_model_density(self, lam, mu, rho, wavelet, resid, ckpt=None, acc=None,
                              acc_rho=None):
        """adjoint_model plus the density correlation: returns (acc, acc_rho),
        acc_rho [2, cells] = b dJ/db at the v_r and v_z nodes."""
        z = self.sizes
        if acc is None:
            acc = torch.empty(z.acc_elems, dtype=torch.float32, device=self.device)
        if acc_rho is None:
            acc_rho = torch.empty(2 * z.cells, dtype=torch.float32, device=self.device)
        if ckpt is None:
            ckpt = self.workspace("ckpt")
        fw, aw = self.workspace("fwd"), self.workspace("adj")
        n = self.model_shape[0] * self.model_shape[1]
        rc = load().bhfwi_adjoint_model_density(
            self._h, _stream(), _f32(lam, n), _f32(mu, n), _f32(rho, n),
            _f32(wavelet, z.wavelet_elems), _f32(resid, z.trace_elems), _ptr(fw), fw.numel(),
            _ptr(ckpt), ckpt.numel(), _ptr(aw), aw.numel(), _f32(acc, z.acc_elems),
            _f32(acc_rho, 2 * z.cells))
        _check(rc, self._h)
        return acc, acc_rho

    def adjoint_model_ex(self, lam, mu, rho, wavelet, resid, ckpt=None, acc=None,
                         density=False, hessian=False, acc_rho=None, acc_h=None):
        """adjoint_model with the optional outputs: returns (acc, acc_rho or
        None, acc_h or None); acc_h [2, cells] is the virtual-source
        pseudo-Hessian diagonal (H_lambda, H_mu) per shot."""
        z = self.sizes
        if acc is None:
            acc = torch.empty(z.acc_elems, dtype=torch.float32, device=self.device)
        if density and acc_rho is None:
            acc_rho = torch.empty(2 * z.cells, dtype=torch.float32, device=self.device)
        if hessian and acc_h is None:
            acc_h = torch.empty(2 * z.cells, dtype=torch.float32, device=self.device)
        if not density:
            acc_rho = None
        if not hessian:
            acc_h = None
        if ckpt is None:
            ckpt = self.workspace("ckpt")
        fw, aw = self.workspace("fwd"), self.workspace("adj")
        n = self.model_shape[0] * self.model_shape[1]
        rc = load().bhfwi_adjoint_model_ex(
            self._h, _stream(), _f32(lam, n), _f32(mu, n), _f32(rho, n),
            _f32(wavelet, z.wavelet_elems), _f32(resid, z.trace_elems), _ptr(fw), fw.numel(),
            _ptr(ckpt), ckpt.numel(), _ptr(aw), aw.numel(), _f32(acc, z.acc_elems),
            _f32(acc_rho, 2 * z.cells) if density else None,
            _f32(acc_h, 2 * z.cells) if hessian else None)
        _check(rc, self._h)
        return acc, acc_rho, acc_h

    def adjoint_model_wavelet(self, lam, mu, rho, wavelet, resid, ckpt=None, acc=None,
                              wgrad=None):
        """adjoint_model plus dJ/dwavelet (bhfwi_adjoint_model_wavelet): returns
        (acc, wgrad), wgrad packed like the wavelets -- the transpose of the
        linear map wavelet -> traces applied to resid."""
        z = self.sizes
        if acc is None:
            acc = torch.empty(z.acc_elems, dtype=torch.float32, device=self.device)
        if wgrad is None:
            wgrad = torch.empty(z.wavelet_elems, dtype=torch.float32, device=self.device)
        if ckpt is None:
            ckpt = self.workspace("ckpt")
        fw, aw = self.workspace("fwd"), self.workspace("adj")
        n = self.model_shape[0] * self.model_shape[1]
        rc = load().bhfwi_adjoint_model_wavelet(
            self._h, _stream(), _f32(lam, n), _f32(mu, n), _f32(rho, n),
            _f32(wavelet, z.wavelet_elems), _f32(resid, z.trace_elems), _ptr(fw), fw.numel(),
            _ptr(ckpt), ckpt.numel(), _ptr(aw), aw.numel(), _f32(acc, z.acc_elems),
            _f32(wgrad, z.wavelet_elems))
        _check(rc, self._h)
        return acc, wgrad

    def gradient_hessian(self, acc_h, out=None, accumulate=False):
        """(H_lambda, H_mu) on the global grid from adjoint_model_ex's acc_h
        (added to `out` when accumulate)."""
        if out is None:
            out = tuple(torch.empty(self.model_shape, dtype=torch.float32, device=self.device)
                        for _ in range(2))
        n = self.model_shape[0] * self.model_shape[1]
        _check(load().bhfwi_gradient_hessian(self._h, _stream(), _f32(acc_h, 2 * self.sizes.cells),
                                             _f32(out[0], n), _f32(out[1], n),
                                             1 if accumulate else 0), self._h)
        return out

    def precondition_diag(self, g, mask, eps, diag=None, row_weight=None, gpg=None,
                          accumulate=False):
        """One gradient through P = w[row] / (d + eps max d) (in place)."""
        n = g.numel()
        _check(load().bhfwi_precondition_diag(
            self._h, _stream(), n, int(g.shape[-1]), _f32(diag, n) if diag is not None else None,
            _f32(row_weight, n // g.shape[-1]) if row_weight is not None else None, _ptr(mask),
            float(eps), _f32(g, n), _ptr(gpg) if gpg is not None else None,
            1 if accumulate else 0), self._h)
        return g

    def update_density(self, rho, g_rho, mask, eta, rho_min, rho_max, alpha=None):
        """Density step (in place); returns alpha as a device scalar."""
        if alpha is None:
            alpha = torch.empty((), dtype=torch.float32, device=self.device)
        n = rho.numel()
        _check(load().bhfwi_update_density(self._h, _stream(), n, _f32(rho, n), _f32(g_rho, n),
                                           _ptr(mask), float(eta), float(rho_min),
                                           float(rho_max), _f32(alpha)), self._h)
        return alpha

    def gradient_density(self, rho, acc_rho, out=None, accumulate=False):
        """dJ/drho on the global grid from adjoint_model_density's acc_rho
        (added to `out` when accumulate)."""
        if out is None:
            out = torch.empty(self.model_shape, dtype=torch.float32, device=self.device)
        n = self.model_shape[0] * self.model_shape[1]
        _check(load().bhfwi_gradient_density(self._h, _stream(), _f32(rho, n),
                                             _f32(acc_rho, 2 * self.sizes.cells), _f32(out, n),
                                             1 if accumulate else 0), self._h)
        return out

    def gradient(self, mu, acc, out=None, accumulate=False):
        """Gradient finalize: returns (g_lam, g_mu, illum) on the global grid
        (added to `out` when accumulate)."""
        shp = self.model_shape
        if out is None:
            out = tuple(torch.empty(shp, dtype=torch.float32, device=self.device)
                        for _ in range(3))
        g_lam, g_mu, illum = out
        _check(load().bhfwi_gradient(self._h, _stream(), _f32(mu), _f32(acc), _f32(g_lam),
                                     _f32(g_mu), _f32(illum), 1 if accumulate else 0),
               self._h)
        return g_lam, g_mu, illum

    def precondition(self, illum, mask, eps, g_lam, g_mu, gpg=None):
        """Diagonal preconditioner, in place on g_lam and g_mu; with gpg (a
        float64 device scalar) also the sum of g . P g over mask cells."""
        if mask.dtype != torch.uint8:
            raise ValueError("mask must be uint8")
        _check(load().bhfwi_precondition(self._h, _stream(), illum.numel(), _f32(illum),
                                         _ptr(mask), float(eps), _f32(g_lam), _f32(g_mu),
                                         _f64(gpg) if gpg is not None else None), self._h)
        return g_lam, g_mu

    def status(self):
        """bhfwi_status on the current stream: raises on non-finite data."""
        _check(load().bhfwi_status(self._h, _stream()), self._h)

    def line_search(self, J0, J1, gpg, alpha1, out=None):
        """Parabolic step length from device scalars (bhfwi_line_search)."""
        out = torch.empty((), dtype=torch.float32, device=self.device) if out is None else out
        _check(load().bhfwi_line_search(self._h, _stream(), _f64(J0), _f64(J1), _f64(gpg),
                                        _f32(alpha1), _f32(out)), self._h)
        return out

    def update(self, lam, mu, rho, g_lam, g_mu, mask, eta, alpha_override=0.0,
               bounds=(0.0, 1e30, 0.0, 1e30), alpha_in=None):
        """Eq. 9-10 in place on lam, mu; returns alpha as a device tensor.
        alpha_in (float32 device scalar) sets alpha directly."""
        alpha = torch.empty((), dtype=torch.float32, device=self.device)
        b = Bounds(*[float(x) for x in bounds])
        _check(load().bhfwi_update(self._h, _stream(), lam.numel(), _f32(lam), _f32(mu),
                                   _f32(rho), _f32(g_lam), _f32(g_mu), _ptr(mask), float(eta),
                                   float(alpha_override),
                                   _f32(alpha_in) if alpha_in is not None else None,
                                   C.byref(b), _ptr(alpha)), self._h)
        return alpha

    # ---------------------------------------------------------------- layout
    def trace_slices(self):
        """(offset, nrec, nt) of each shot in the packed trace arrays."""
        out, off = [], 0
        for sh in self.shots:
            nrec = len(sh.rec_k)
            out.append((off, nrec, sh.nt))
            off += nrec * sh.nt
        return out

    def pack_wavelets(self, wavelets):
        return torch.as_tensor(np.concatenate([np.asarray(w[: sh.nt], np.float32)
                                               for w, sh in zip(wavelets, self.shots)]),
                               device=self.device)

    def unpack_traces(self, traces):
        t = traces.detach().cpu().numpy()
        return [t[o: o + r * nt].reshape(r, nt) for (o, r, nt) in self.trace_slices()]

    def acc_views(self, acc):
        """Per-shot [4, NR, NZ] views of the accumulators (cells are packed
        with 64-float alignment)."""
        z = self.sizes
        a = acc.view(4, z.cells)
        out, off = [], 0
        for sh in self.shots:
            NR, NZ = sh.nr + sh.pr, sh.nz + 2 * sh.pz
            out.append(a[:, off: off + NR * NZ].view(4, NR, NZ))
            off += (NR * NZ + 63) // 64 * 64
        return out
