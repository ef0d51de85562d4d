"""Reverse-mode gradient of a real loss through the split-step cascade, in FP64
(TEST INFRASTRUCTURE ONLY: see oracle/__init__).

Complex-gradient convention: for a real loss L of a complex array z the
gradient is g = dL/dRe(z) + j dL/dIm(z), so that dL = Re(sum conj(g) dz).
Real parameters (the ESSFM taps w) get ordinary gradients; complex FIR taps h
get gradients in the same convention as fields.

Per step z = u exp(-j phi J), J = w (*) I, I = sum_p |u_p|^2, u = Lin(x):
  g_u   = g_z exp(+j phi J)                       (the phase factor is unitary)
  Jbar  = phi * sum_p Im(conj(g_z,p) z_p)         (dL/dJ)
  wbar  = sum_n Jbar_n I_{n-(m-c)}                (taps: correlation with I)
  Ibar  = w^T (*) Jbar                            (transpose of the tap filter)
  g_u  += 2 Ibar u_p                              (d|u|^2 = 2 Re(conj(u) du))
  FFT linear step: g_x = IDFT(conj(H) DFT(g_u));  FIR: g_x = conj(h)^T (*) g_u,
  hbar[m] = sum_{p,n} g_u[p,n] conj(x[p, n-(m-c)]).
Overlap-and-save: the gather of a block is transposed by a scatter-add of the
block gradient into the signal; the keep-the-centre scatter is transposed by
a gather of the centre gradient with zeros in the halo.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from .dbp_ref import (Step, block_starts, circular_conv, dispersion_response,
                      filtered_intensity, fir_linear_substep, linear_substep, step,
                      total_intensity)


@dataclass
class Grads:
    x: np.ndarray                   # gradient w.r.t. the input field
    w: list                         # per step: gradient w.r.t. the taps (None for SSFM)
    h: list                         # per step: gradient w.r.t. the FIR taps (None for FFT)


def _step_forward(x: np.ndarray, st: Step, fs_thz: float):
    u = fir_linear_substep(x, st.h) if st.h is not None else linear_substep(x, st.b, fs_thz)
    inten = total_intensity(u)
    j = filtered_intensity(inten, st.w)
    z = u * np.exp(-1j * st.phi * j)[..., None, :]
    return u, inten, j, z


def _step_backward(x, st: Step, fs_thz: float, u, inten, j, z, g_z):
    """Returns (g_x, wbar or None, hbar or None), reducing parameter grads over all leading axes."""
    g_u = g_z * np.exp(1j * st.phi * j)[..., None, :]
    jbar = st.phi * np.sum(np.imag(np.conj(g_z) * z), axis=-2)
    wbar = None
    if st.w is not None:
        nt = len(st.w)
        c = (nt - 1) // 2
        wbar = np.array([np.sum(jbar * np.roll(inten, m - c, axis=-1)) for m in range(nt)])
        ibar = circular_conv(jbar, np.asarray(st.w, dtype=np.float64)[::-1])
    else:
        ibar = jbar
    g_u = g_u + 2.0 * ibar[..., None, :] * u
    hbar = None
    if st.h is not None:
        h = np.asarray(st.h, dtype=np.complex128)
        nt = len(h)
        c = (nt - 1) // 2
        g_x = circular_conv(g_u, np.conj(h)[::-1])
        hbar = np.array([np.sum(g_u * np.conj(np.roll(x, m - c, axis=-1))) for m in range(nt)])
    else:
        n = x.shape[-1]
        hconj = np.conj(dispersion_response(n, st.b, fs_thz))
        g_x = np.fft.ifft(np.fft.fft(g_u, axis=-1) * hconj, axis=-1)
    return g_x, wbar, hbar


def _cascade_grad(x0: np.ndarray, steps: Sequence[Step], fs_thz: float, g_out: np.ndarray):
    """Gradient through consecutive steps on one circular field (any leading axes)."""
    states = []
    x = x0
    for st in steps:
        u, inten, j, z = _step_forward(x, st, fs_thz)
        states.append((x, u, inten, j, z))
        x = z
    g = g_out
    wb = [None] * len(steps)
    hb = [None] * len(steps)
    for s in range(len(steps) - 1, -1, -1):
        xs, u, inten, j, z = states[s]
        g, wb[s], hb[s] = _step_backward(xs, steps[s], fs_thz, u, inten, j, z, g)
    return g, wb, hb


def grad_whole(x: np.ndarray, steps: Sequence[Step], fs_thz: float, g_out: np.ndarray) -> Grads:
    """Adjoint of dbp_ref.run_whole."""
    g, wb, hb = _cascade_grad(np.asarray(x, dtype=np.complex128), steps, fs_thz,
                              np.asarray(g_out, dtype=np.complex128))
    return Grads(x=g, w=wb, h=hb)


def grad_blocked(x: np.ndarray, steps: Sequence[Step], fs_thz: float, nb: int, overlap: int,
                 k: int, g_out: np.ndarray) -> Grads:
    """Adjoint of dbp_ref.run_blocked with the same (nb, overlap, k)."""
    y = np.asarray(x, dtype=np.complex128)
    n = y.shape[-1]
    v = nb - overlap
    hh = overlap // 2
    starts = block_starts(n, nb, overlap)
    n_blk = len(starts)
    idx = (starts[:, None] + np.arange(nb)[None, :]) % n
    pass_inputs = []
    for p0 in range(0, len(steps), k):
        pass_inputs.append((p0, y))
        g = np.moveaxis(y[..., idx], -2, 0)
        for st in steps[p0:p0 + k]:
            g = step(g, st, fs_thz)
        g = np.moveaxis(g, 0, -2)
        y = g[..., hh:hh + v].reshape(g.shape[:-2] + (-1,))[..., :n]
    wb = [None] * len(steps)
    hb = [None] * len(steps)
    gsig = np.asarray(g_out, dtype=np.complex128)
    # block b, position m in [hh, hh+V) holds output sample starts[b] + m (if < n)
    out_pos = starts[:, None] + np.arange(nb)[None, :]
    keep = np.zeros((n_blk, nb), dtype=bool)
    keep[:, hh:hh + v] = True
    keep &= out_pos < n
    for p0, y_in in reversed(pass_inputs):
        seg = list(steps[p0:p0 + k])
        gb = np.zeros(gsig.shape[:-1] + (n_blk, nb), dtype=np.complex128)
        gb[..., keep] = gsig[..., out_pos[keep]]
        gblk_in, wseg, hseg = _cascade_grad(np.moveaxis(y_in[..., idx], -2, 0), seg, fs_thz,
                                            np.moveaxis(gb, -2, 0))
        gblk_in = np.moveaxis(gblk_in, 0, -2)                       # [..., n_pol, n_blk, nb]
        gnew = np.zeros_like(gsig)
        flat = gnew.reshape(-1, n)
        src = gblk_in.reshape(-1, n_blk * nb)
        for r in range(flat.shape[0]):
            np.add.at(flat[r], idx.reshape(-1), src[r])
        gsig = flat.reshape(gsig.shape)
        for i, s in enumerate(range(p0, p0 + len(seg))):
            wb[s] = wseg[i]
            hb[s] = hseg[i]
    return Grads(x=gsig, w=wb, h=hb)


# --------------------------------------------------------------------------- loss head

def symbol_mse(z: np.ndarray, s: np.ndarray, p_w: float, mf: np.ndarray, sps: int = 2):
    """Loss of the differentiation workload and its gradient w.r.t. the field z.

    loss = mean |MF(z)[::sps] / a0 - s|^2 over every symbol, with the receive
    filter applied circularly in frequency (mf: real response on the DFT grid)
    and a0 = sqrt(sps * P / n_pol) the symbol amplitude of a launched field of
    total power P (a Nyquist-shaped stream at sps samples per symbol carries
    1/sps of the symbol power per sample).  The filter is real in frequency,
    hence self-adjoint; the adjoint of taking every sps-th sample is zero
    insertion.
    """
    n_pol = z.shape[-2]
    sig = math.sqrt(sps * p_w / n_pol)
    y = np.fft.ifft(np.fft.fft(z, axis=-1) * mf, axis=-1)
    a = y[..., ::sps] / sig - s
    n_tot = a.size
    loss = float(np.sum(np.abs(a) ** 2) / n_tot)
    up = np.zeros(z.shape, dtype=np.complex128)
    up[..., ::sps] = 2.0 * a / (sig * n_tot)
    g = np.fft.ifft(np.fft.fft(up, axis=-1) * mf, axis=-1)
    return loss, g
