"""CPU FP64 oracle of the object priors: l1, reweighted l1 and total variation
regularizers (Eq. tikhonov, Table tab:regularizers) and the finite-support
projection.

TEST INFRASTRUCTURE ONLY: the reference the GPU regularizer kernels are
checked against; only ``tests/``, ``__graft_entry__.smoke()`` and
``bench.py``'s ``cpu_baseline`` leg use it.  Plain NumPy in float64, no code
shared with the HIP library.

Readings (the table is partly garbled; each choice is stated once):

* N_o = S * Ly * Lx, the number of object voxels; every regularizer is a
  mean over voxels, weighted by its coefficient.
* delta/beta objects: l1 = (1/N_o) sum a1 |delta| + a2 |beta|;
  TV = (gamma/N_o) sum (|grad delta|_1 + |grad beta|_1), gamma weighting both
  terms.  Complex (real/imag) objects: the l1 terms act on |O| - mean|O| and
  on arg O; TV acts on |O| and arg O (the table repeats the l1 expression
  for TV; the gradient norm of the same two quantities is the reading).
* |grad C|_1 = |D_x C| + |D_y C| + |D_z C| with forward differences between
  neighbouring voxels inside the array (no term across the boundary).
* mean|O| depends on O and is differentiated through.  arg O is the
  principal value (no unwrapping).
* The derivative of |t| at t = 0 is taken as 0 (a subgradient), as are the
  derivatives of |O| and arg O at O = 0.
* Reweighted l1: W = max|C| / (|C| + eps) per voxel, computed from a
  snapshot of the object and held constant (no gradient through W), as the
  table states; C is the quantity the l1 term acts on.
* Complex gradients are returned as (dR/dRe O, dR/dIm O).
* Finite support: voxels outside the mask are set to the vacuum value
  (delta = beta = 0, or O = 1).
"""
from __future__ import annotations

import numpy as np


def _sign(x):
    return np.sign(x)            # sign(0) = 0


# ---------------------------------------------------------------------------
# the quantities the priors act on
# ---------------------------------------------------------------------------

def l1_quantities(a, b, obj_repr):
    """(C1, C2): delta and beta, or |O| - mean|O| and arg O."""
    if obj_repr == "delta_beta":
        return a, b
    o = a + 1j * b
    mod = np.abs(o)
    return mod - mod.mean(), np.angle(o)


def tv_quantities(a, b, obj_repr):
    """(C1, C2): delta and beta, or |O| and arg O."""
    if obj_repr == "delta_beta":
        return a, b
    o = a + 1j * b
    return np.abs(o), np.angle(o)


def reweight(a, b, obj_repr, eps):
    """Adaptive weights W = max|C| / (|C| + eps) of a snapshot (a, b)."""
    c1, c2 = l1_quantities(a, b, obj_repr)
    return (np.max(np.abs(c1)) / (np.abs(c1) + eps), np.max(np.abs(c2)) / (np.abs(c2) + eps))


# ---------------------------------------------------------------------------
# values
# ---------------------------------------------------------------------------

def l1_value(a, b, obj_repr, a1, a2, w1=None, w2=None):
    c1, c2 = l1_quantities(a, b, obj_repr)
    w1 = 1.0 if w1 is None else w1
    w2 = 1.0 if w2 is None else w2
    return float(np.sum(a1 * w1 * np.abs(c1) + a2 * w2 * np.abs(c2)) / a.size)


def tv_norm(c):
    """sum over voxels of |D_z c| + |D_y c| + |D_x c| (forward differences
    inside the array)."""
    return float(sum(np.sum(np.abs(np.diff(c, axis=ax))) for ax in range(c.ndim)))


def tv_value(a, b, obj_repr, gamma):
    c1, c2 = tv_quantities(a, b, obj_repr)
    return gamma * (tv_norm(c1) + tv_norm(c2)) / a.size


def value(a, b, obj_repr, a1=0.0, a2=0.0, gamma=0.0, w1=None, w2=None):
    """Sum of the l1 (or, with weights, reweighted l1) and TV regularizers."""
    return l1_value(a, b, obj_repr, a1, a2, w1, w2) + tv_value(a, b, obj_repr, gamma)


# ---------------------------------------------------------------------------
# gradients
# ---------------------------------------------------------------------------

def tv_norm_grad(c):
    """d tv_norm / d c: every pair (i, i+1) along an axis adds
    sign(c[i+1] - c[i]) to voxel i+1 and subtracts it from voxel i."""
    g = np.zeros_like(c)
    for ax in range(c.ndim):
        s = _sign(np.diff(c, axis=ax))
        lo = [slice(None)] * c.ndim
        hi = [slice(None)] * c.ndim
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        g[tuple(hi)] += s
        g[tuple(lo)] -= s
    return g


def _complex_chain(a, b, d_mod, d_arg):
    """(dR/dRe, dR/dIm) from dR/d|O| and dR/d arg O:
    d|O| = (Re dRe + Im dIm)/|O|, d arg O = (Re dIm - Im dRe)/|O|^2."""
    mod2 = a * a + b * b
    mod = np.sqrt(mod2)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = np.where(mod > 0, 1.0 / mod, 0.0)
        inv2 = np.where(mod2 > 0, 1.0 / mod2, 0.0)
    return d_mod * a * inv - d_arg * b * inv2, d_mod * b * inv + d_arg * a * inv2


def grad(a, b, obj_repr, a1=0.0, a2=0.0, gamma=0.0, w1=None, w2=None):
    """(dR/da, dR/db) of ``value``."""
    n_o = a.size
    w1 = 1.0 if w1 is None else w1
    w2 = 1.0 if w2 is None else w2
    if obj_repr == "delta_beta":
        ga = a1 * w1 * _sign(a) / n_o + gamma * tv_norm_grad(a) / n_o
        gb = a2 * w2 * _sign(b) / n_o + gamma * tv_norm_grad(b) / n_o
        return ga, gb
    c1, c2 = l1_quantities(a, b, obj_repr)
    # l1 on |O| - m with m = mean|O|: d/d|O_k| = s_k - mean(s), s = W1 sign(c1)
    s = a1 * w1 * _sign(c1) / n_o
    d_mod = s - np.sum(s) / n_o
    d_arg = a2 * w2 * _sign(c2) / n_o
    t1, t2 = tv_quantities(a, b, obj_repr)
    d_mod = d_mod + gamma * tv_norm_grad(t1) / n_o
    d_arg = d_arg + gamma * tv_norm_grad(t2) / n_o
    return _complex_chain(a, b, d_mod, d_arg)


# ---------------------------------------------------------------------------
# finite support
# ---------------------------------------------------------------------------

def support_project(a, b, obj_repr, mask):
    """Voxels where ``mask`` is 0 take the vacuum value."""
    keep = np.asarray(mask).astype(bool)
    vac_a, vac_b = (0.0, 0.0) if obj_repr == "delta_beta" else (1.0, 0.0)
    return np.where(keep, a, vac_a), np.where(keep, b, vac_b)
