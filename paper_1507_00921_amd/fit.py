"""ESSFM coefficient fit (Sec. IV) through the library's adjoint.

Sec. IV obtains the N_c + 1 coefficients c_0..c_Nc of the ESSFM, shared by every step, by
a least-squares fit of its output to that of a multi-step SSFM.  Here the objective is

    F(c) = sum over the samples `sl` of |y - target|^2,   y = dbp_backprop(x; w(c)),

with the taps of every step w(c) = [c_Nc .. c_1, c_0, c_1 .. c_Nc].  Its gradient comes
from dbp_backprop_grad with upstream gradient 2 (y - target) on `sl` (zero elsewhere),
giving dF/dw[s][m] for every step s, which sums over the steps and the two taps of each
symmetric pair into dF/dc.  Forward and reverse run on the GPU; L-BFGS (scipy) updates the
N_c + 1 numbers on the host.  Another loss (e.g. the symbol MSE of a training workload)
can replace the field residual through `loss`.
"""
from __future__ import annotations

import time
from typing import Callable, Optional

import numpy as np


def symmetric_full(c) -> np.ndarray:
    """c_0..c_Nc -> the 2 Nc + 1 taps [c_Nc .. c_1, c_0, c_1 .. c_Nc] (float32)."""
    c = np.asarray(c, dtype=np.float64)
    return np.concatenate([c[:0:-1], c]).astype(np.float32)


def fold_symmetric(g_full: np.ndarray, per_step: bool = False) -> np.ndarray:
    """dF/dw [N_s][2 Nc + 1] -> dF/dc (adjoint of symmetric_full): summed over the steps
    (shared coefficients) or kept per step ([N_s][Nc + 1], flattened)."""
    g = np.asarray(g_full, dtype=np.float64)
    if not per_step:
        g = g.sum(axis=0, keepdims=True)
    nc = (g.shape[1] - 1) // 2
    out = np.empty((g.shape[0], nc + 1))
    out[:, 0] = g[:, nc]
    out[:, 1:] = g[:, nc + 1:] + g[:, nc - 1::-1]
    return out.ravel() if per_step else out[0]


def field_residual_loss(target, sl: slice):
    """Loss head sum_{sl} |y - target|^2 and its gradient dL/dRe + j dL/dIm = 2 (y - target)."""
    import torch

    def loss(y):
        d = y[..., sl] - target[..., sl]
        g = torch.zeros_like(y)
        g[..., sl] = 2.0 * d
        return float(torch.view_as_real(d).double().square().sum()), g

    return loss


def fit_coefficients(plan, x, n_c: int, target=None, sl: Optional[slice] = None,
                     loss: Optional[Callable] = None, c0=None, maxiter: int = 60, per_step: bool = False):
    """Fit the symmetric ESSFM coefficients of an ESSFM plan (2 n_c + 1 taps), shared by
    every step (Sec. IV) or, with per_step, one set per step (N_s (n_c + 1) unknowns, the
    same objective and the same single reverse pass per evaluation).

    x: complex64 CUDA tensor [batch][n_pol][L]; either (target, sl) for the Sec. IV field
    residual or `loss(y) -> (value, dL/dy)`.  Starts from SSFM (c = [1, 0, ..]) unless c0
    is given ([n_c + 1], or [N_s][n_c + 1] with per_step).  Returns (c, info): c is
    [n_c + 1] or [N_s][n_c + 1]; info holds the objective before and after, the number of
    forward + reverse evaluations and the wall time.
    """
    import torch
    from scipy.optimize import minimize

    if loss is None:
        loss = field_residual_loss(target, sl)
    ns = plan.n_steps
    if plan.desc.n_taps != 2 * n_c + 1:
        raise ValueError(f"plan has {plan.desc.n_taps} taps, expected {2 * n_c + 1}")
    if c0 is None:
        c0 = np.zeros(n_c + 1)
        c0[0] = 1.0
    c0 = np.asarray(c0, dtype=np.float64)
    if per_step and c0.ndim == 1:
        c0 = np.tile(c0, (ns, 1))
    shape = c0.shape
    c0 = c0.ravel()
    ws = plan.workspace(grad=True)
    n_eval = [0]

    def taps_of(c):
        if per_step:
            return np.stack([symmetric_full(ci) for ci in c.reshape(shape)])
        return np.tile(symmetric_full(c), (ns, 1))

    def value_and_grad(c):
        w = torch.from_numpy(np.ascontiguousarray(taps_of(c))).cuda()
        y = plan.backprop(x, taps=w)
        f, g = loss(y)
        _, gt, _ = plan.backprop_grad(x, g.contiguous(), taps=w, want_input=False, workspace=ws)
        n_eval[0] += 1
        return f, fold_symmetric(gt.cpu().numpy(), per_step)

    t0 = time.perf_counter()
    f0, _ = value_and_grad(c0)
    scale = 1.0 / f0 if f0 > 0 else 1.0

    def fun(c):
        f, g = value_and_grad(c)
        return f * scale, g * scale

    res = minimize(fun, c0, jac=True, method="L-BFGS-B", options=dict(maxiter=maxiter, ftol=1e-12, gtol=1e-9))
    torch.cuda.synchronize()
    info = {"objective_start": f0, "objective": float(res.fun) / scale, "evaluations": n_eval[0],
            "iterations": int(res.nit), "seconds": time.perf_counter() - t0, "message": str(res.message)}
    return res.x.reshape(shape), info
