"""Least-squares fit of the ESSFM coefficients (Sec. IV), in FP64
(TEST INFRASTRUCTURE ONLY: see oracle/__init__).

Sec. IV obtains the coefficients c_0..c_Nc of the single-step ESSFM by a
least-squares fit of its output to that of a multi-step SSFM on the first part
of the received samples; the same coefficients serve every step.  Here the
residual is the blocked ESSFM output minus a target field on a slice of
samples (both polarizations, real and imaginary parts stacked) and the fit is
scipy's least_squares with its finite-difference Jacobian.  The taps of every
step are the symmetric vector w = [c_Nc .. c_1, c_0, c_1 .. c_Nc].
"""
from __future__ import annotations

from typing import Sequence

import numpy as np
from scipy.optimize import least_squares

from .dbp_ref import Step, run_blocked


def symmetric_full(c: np.ndarray) -> np.ndarray:
    """c_0..c_Nc -> the 2 Nc + 1 taps [c_Nc .. c_1, c_0, c_1 .. c_Nc]."""
    c = np.asarray(c, dtype=np.float64)
    return np.concatenate([c[:0:-1], c])


def essfm_blocked(x: np.ndarray, base: Sequence[Step], c: np.ndarray, fs_thz: float, nb: int, overlap: int,
                  k: int) -> np.ndarray:
    """Blocked ESSFM cascade with the shared symmetric coefficients c on every step of `base`."""
    w = symmetric_full(c)
    steps = [Step(b=st.b, phi=st.phi, w=w) for st in base]
    return run_blocked(x, steps, fs_thz, nb, overlap, k)


def residual(c, x, target, base, fs_thz, nb, overlap, k, sl) -> np.ndarray:
    d = essfm_blocked(x, base, c, fs_thz, nb, overlap, k)[..., sl] - target[..., sl]
    return np.concatenate([d.real.ravel(), d.imag.ravel()])


def fit_coefficients(x: np.ndarray, target: np.ndarray, base: Sequence[Step], fs_thz: float, nb: int,
                     overlap: int, k: int, n_c: int, sl: slice, c0=None) -> np.ndarray:
    """c_0..c_Nc minimizing sum |ESSFM(c; x) - target|^2 over the samples `sl` (Sec. IV).

    Starts from SSFM (c = [1, 0, ..]) unless c0 is given."""
    if c0 is None:
        c0 = np.zeros(n_c + 1)
        c0[0] = 1.0
    res = least_squares(residual, np.asarray(c0, dtype=np.float64),
                        args=(x, target, base, fs_thz, nb, overlap, k, sl),
                        xtol=1e-12, ftol=1e-12, gtol=1e-12)
    return res.x
