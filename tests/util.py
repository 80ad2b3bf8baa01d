"""Shared test helpers: glue between the seeded workloads, the FP64 oracle and
(for GPU tests) the HIP binding.  No method arithmetic lives here beyond what a
test states for itself."""
from __future__ import annotations

import json
import math
import os

import numpy as np

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def geom(sh) -> oracle.Geom:
    return oracle.Geom(sh.nr, sh.nz, sh.pr, sh.pz, sh.dr, sh.dz, sh.dt, sh.nt, sh.f0,
                       sh.vmax, sh.src_k, np.asarray(sh.rec_k, np.int32))


def oracle_models(w, s=0, which="start"):
    """(lam, mu, rho) of shot s's window, via the oracle's Eq. 3-4."""
    vp = w.window(w.vp_start if which == "start" else w.vp_true, s)
    vs = w.window(w.vs_start if which == "start" else w.vs_true, s)
    rho = np.ascontiguousarray(w.window(w.rho, s))
    lam, mu = oracle.moduli(vp, vs, rho)
    return lam, mu, rho


def ricker_derivative(f0, t):
    """Analytic time derivative of the Ricker wavelet delayed by 1.5/f0."""
    tt = t - 1.5 / f0
    a = (math.pi * f0 * tt) ** 2
    return 2.0 * math.pi ** 2 * f0 ** 2 * tt * (2.0 * a - 3.0) * np.exp(-a)


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
