"""Reference split-step cascade in FP64 (TEST INFRASTRUCTURE ONLY: see oracle/__init__).

Fields are complex128 arrays of shape [..., n_pol, L] (n_pol = 1 or 2); the
polarization axis is the second to last, time the last.

Conventions (the paper's Sec. II leaves these implicit; the readings are):
  * DFT: X_k = sum_n x_n exp(-j 2 pi k n / L) (numpy), frequency grid f_k =
    fftfreq(L, 1/fs); only f_k^2 enters, so the Nyquist bin's sign is moot.
  * Linear substep, Eq. (1): X_k <- X_k exp(-j 2 pi^2 b f_k^2) with b = beta2*dz.
  * Nonlinear substep, Eqs. (2)-(3): y_p,n <- y_p,n exp(-j phi J_n) with
    I_n = sum_p |y_p,n|^2 (Manakov: total intensity of both polarizations) and
    J = I (SSFM) or J_n = sum_m w[m] I_{n-(m-Nc)} (ESSFM, 2Nc+1 taps, centre Nc;
    the paper's symmetric c_i is w[Nc+i] = w[Nc-i] = c_i).
  * One step = linear substep then nonlinear substep (ops (i)-(iv) of Sec. II).
  * Power-normalized field with ideal amplifiers: attenuation enters only the
    nonlinear weight phi = gamma * exp(-alpha z_a) * (1 - exp(-alpha dz)) / alpha
    (the paper's effective length, generalized to a segment starting at z_a
    inside a span).  Backpropagation runs the same step with b and phi negated,
    segments taken from the receiver end of each span, so the nonlinear phase
    of a segment is applied at its transmitter-side (high-power) end.
  * Overlap-and-save (Sec. III): blocks of Nb samples overlapping by O (even);
    block b covers x[(b V - O/2 + m) mod L], m < Nb, V = Nb - O; each block is
    propagated circularly through k steps and its centre V samples are kept.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np


@dataclass
class Step:
    """One split step: linear part (b, or FIR taps h) then nonlinear part (phi, w)."""
    b: float                         # beta2 * dz  [ps^2]; signed
    phi: float                       # nonlinear weight gamma * dz_eff [1/W]; signed
    w: Optional[np.ndarray] = None   # ESSFM intensity taps (odd length); None = SSFM
    h: Optional[np.ndarray] = None   # complex FIR linear substep (odd length); None = FFT


# --------------------------------------------------------------------------- substeps

def freq_grid(n: int, fs_thz: float) -> np.ndarray:
    """Frequency of each DFT bin in THz (fftfreq ordering)."""
    return np.fft.fftfreq(n, d=1.0 / fs_thz)


def dispersion_response(n: int, b: float, fs_thz: float) -> np.ndarray:
    """All-pass chromatic-dispersion response of Eq. (1): exp(-j 2 pi^2 b f_k^2)."""
    f = freq_grid(n, fs_thz)
    return np.exp(-1j * 2.0 * math.pi ** 2 * b * f * f)


def linear_substep(x: np.ndarray, b: float, fs_thz: float) -> np.ndarray:
    """Ops (i)-(iii) of Sec. II: FFT per polarization, multiply by Eq. (1), inverse FFT."""
    n = x.shape[-1]
    return np.fft.ifft(np.fft.fft(x, axis=-1) * dispersion_response(n, b, fs_thz), axis=-1)


def circular_conv(v: np.ndarray, taps: np.ndarray) -> np.ndarray:
    """out[n] = sum_m taps[m] v[(n - (m - c)) mod L], c = (len(taps)-1)/2, along the last axis."""
    nt = len(taps)
    assert nt % 2 == 1
    c = (nt - 1) // 2
    out = np.zeros(v.shape, dtype=np.result_type(v, taps))
    for m in range(nt):
        out = out + taps[m] * np.roll(v, m - c, axis=-1)
    return out


def fir_linear_substep(x: np.ndarray, h: np.ndarray) -> np.ndarray:
    """Time-domain variant of the linear substep: circular complex FIR per polarization."""
    return circular_conv(x, np.asarray(h, dtype=np.complex128))


def total_intensity(y: np.ndarray) -> np.ndarray:
    """I_n = sum over polarizations of |y_p,n|^2 (Manakov nonlinear term, Sec. II)."""
    return np.sum(y.real ** 2 + y.imag ** 2, axis=-2)


def filtered_intensity(intensity: np.ndarray, w: Optional[np.ndarray]) -> np.ndarray:
    """J of Eq. (3); for SSFM (w is None) J = I as in Eq. (2)."""
    if w is None:
        return intensity
    return circular_conv(intensity, np.asarray(w, dtype=np.float64))


def nonlinear_substep(y: np.ndarray, phi: float, w: Optional[np.ndarray] = None) -> np.ndarray:
    """Op (iv): rotate every polarization by -phi * J (Eq. (2) for SSFM, Eq. (3) for ESSFM)."""
    j = filtered_intensity(total_intensity(y), w)
    return y * np.exp(-1j * phi * j)[..., None, :]


def step(x: np.ndarray, st: Step, fs_thz: float) -> np.ndarray:
    """One split step on a circular field: linear substep, then nonlinear substep."""
    if st.h is not None:
        y = fir_linear_substep(x, st.h)
    else:
        y = linear_substep(x, st.b, fs_thz)
    return nonlinear_substep(y, st.phi, st.w)


# --------------------------------------------------------------------------- schedule

def alpha_lin(alpha_db_km: float) -> float:
    """Power attenuation coefficient in 1/km from dB/km."""
    return alpha_db_km * math.log(10.0) / 10.0


def effective_length(dz: float, alpha: float) -> float:
    """Sec. II: dz_eff = (1 - exp(-alpha dz)) / alpha, -> dz as alpha -> 0."""
    if alpha == 0.0:
        return dz
    return -math.expm1(-alpha * dz) / alpha


def schedule(n_spans: int, span_km: float, steps_per_span: int, beta2_ps2_km: float,
             gamma_w_km: float, alpha_db_km: float, backward: bool = True,
             taps: Optional[Sequence] = None, spans_per_step: int = 1) -> list[Step]:
    """Step list for a homogeneous link (Sec. II step parameters; backward = DBP).

    taps: None (SSFM), one tap vector for every step, or one per step.
    spans_per_step > 1 (with steps_per_span = 1): each step covers that many whole
    spans, as in the experiment of Sec. IV (one step per two spans, one step for the
    whole link).  Such a step applies the dispersion of all its spans at once and one
    nonlinear phase whose weight is the sum of the spans' effective lengths (each
    span's power restarts at its amplifier, so each contributes its full Delta z_eff).
    """
    a = alpha_lin(alpha_db_km)
    m = int(spans_per_step)
    if m < 1 or (m > 1 and (steps_per_span != 1 or n_spans % m != 0)):
        raise ValueError("spans_per_step needs one step per span and must divide n_spans")
    if m > 1:
        n_steps = n_spans // m
        sign = -1.0 if backward else 1.0
        leff = effective_length(span_km, a)
        steps_b = [sign * beta2_ps2_km * span_km * m] * n_steps
        steps_phi = [sign * gamma_w_km * leff * m] * n_steps
    else:
        dz = span_km / steps_per_span
        leff = effective_length(dz, a)
        n_steps = n_spans * steps_per_span
        steps_b, steps_phi = [], []
        for _span in range(n_spans):
            for i in range(steps_per_span):
                if backward:
                    z_a = span_km - (i + 1) * dz     # transmitter-side end of segment i
                    sign = -1.0
                else:
                    z_a = i * dz
                    sign = 1.0
                steps_b.append(sign * beta2_ps2_km * dz)
                steps_phi.append(sign * gamma_w_km * math.exp(-a * z_a) * leff)
    per_step_taps = None
    if taps is not None:
        t = np.asarray(taps, dtype=np.float64)
        per_step_taps = [t] * n_steps if t.ndim == 1 else [np.asarray(v) for v in t]
        assert len(per_step_taps) == n_steps
    return [Step(b=steps_b[s], phi=steps_phi[s], w=None if per_step_taps is None else per_step_taps[s])
            for s in range(n_steps)]


# --------------------------------------------------------------------------- cascades

def run_whole(x: np.ndarray, steps: Sequence[Step], fs_thz: float) -> np.ndarray:
    """Every step applied circularly over the whole signal (the plain definition)."""
    y = np.asarray(x, dtype=np.complex128)
    for st in steps:
        y = step(y, st, fs_thz)
    return y


def block_starts(n: int, nb: int, overlap: int) -> np.ndarray:
    """First sample (before the mod-L wrap) of every overlap-and-save block."""
    v = nb - overlap
    n_blk = -(-n // v)
    return np.arange(n_blk) * v - overlap // 2


def run_blocked(x: np.ndarray, steps: Sequence[Step], fs_thz: float, nb: int, overlap: int,
                k: int) -> np.ndarray:
    """Overlap-and-save cascade (Sec. III) with k steps fused per pass over the signal.

    Each pass gathers blocks g[m] = x[(bV - O/2 + m) mod L], runs up to k steps
    circularly on each block, and keeps the centre samples g[O/2 + m], m < V.
    """
    y = np.asarray(x, dtype=np.complex128)
    n = y.shape[-1]
    if overlap % 2 or overlap < 0 or overlap >= nb or n < nb or k < 1:
        raise ValueError("invalid overlap-and-save geometry")
    v = nb - overlap
    h = overlap // 2
    starts = block_starts(n, nb, overlap)
    idx = (starts[:, None] + np.arange(nb)[None, :]) % n          # [n_blk, nb]
    for p0 in range(0, len(steps), k):
        g = y[..., idx]                                             # [..., n_pol, n_blk, nb]
        g = np.moveaxis(g, -2, 0)                                   # [n_blk, ..., n_pol, nb]
        for st in steps[p0:p0 + k]:
            g = step(g, st, fs_thz)
        g = np.moveaxis(g, 0, -2)                                   # [..., n_pol, n_blk, nb]
        centre = g[..., h:h + v].reshape(g.shape[:-2] + (-1,))
        y = centre[..., :n]
    return y


def run_streaming(x: np.ndarray, steps: Sequence[Step], fs_thz: float, nb: int, overlap: int,
                  k: int) -> np.ndarray:
    """Receiver mode of the overlap-and-save cascade: a stream x[n], n >= 0, preceded by
    silence, with nothing known after its last sample.

    Blocks b have the windows [bV - O/2, bV - O/2 + Nb) of run_blocked, without the wrap, on
    the silence-extended stream: each pass of k steps computes the blocks whose window lies
    inside the samples it has (the silence, then what the previous pass produced) and keeps
    their centres [bV, bV + V).  Returns every output sample n >= 0 computable from x."""
    u = np.asarray(x, dtype=np.complex128)
    v = nb - overlap
    h = overlap // 2
    # silence before the stream, a whole number of blocks, long enough that the first block
    # every pass needs starts inside it: pass p reads from block -(passes - 1 - p) ceil(h/V)
    z = ((passes(len(steps), k) - 1) * (-(-h // v)) + 1) * v
    u = np.concatenate([np.zeros(u.shape[:-1] + (z,), dtype=np.complex128), u], axis=-1)
    for p0 in range(0, len(steps), k):
        e = u.shape[-1]
        n_blk = max((e - h) // v, 0)
        padded = np.concatenate([np.zeros(u.shape[:-1] + (h,), dtype=np.complex128), u], axis=-1)
        out = np.zeros(u.shape[:-1] + (n_blk * v,), dtype=np.complex128)
        for b in range(n_blk):
            g = padded[..., b * v:b * v + nb]                      # samples bV - h .. bV - h + Nb - 1
            for st in steps[p0:p0 + k]:
                g = step(g, st, fs_thz)
            out[..., b * v:(b + 1) * v] = g[..., h:h + v]
        u = out
    return u[..., z:]


def streaming_latency(n_steps: int, nb: int, overlap: int, k: int) -> int:
    """Samples by which the receiver-mode output trails its input: one block per pass."""
    v = nb - overlap
    h = overlap // 2
    return passes(n_steps, k) * (-(-h // v)) * v


def passes(n_steps: int, k: int) -> int:
    return -(-n_steps // k)


# --------------------------------------------------------------------------- link helpers

def ideal_fir_taps(n_taps: int, b: float, fs_thz: float, n_fft: int = 1 << 16) -> np.ndarray:
    """Centre n_taps samples of the impulse response of Eq. (1)'s all-pass filter.

    The L2-optimal truncation: tap m multiplies x[n - (m - c)], c = (n_taps-1)/2,
    and equals the inverse DFT of exp(-j 2 pi^2 b f^2) at lag m - c, computed on a
    fine n_fft-point grid.
    """
    assert n_taps % 2 == 1
    c = (n_taps - 1) // 2
    imp = np.fft.ifft(dispersion_response(n_fft, b, fs_thz))
    return np.array([imp[(m - c) % n_fft] for m in range(n_taps)], dtype=np.complex128)


def ls_fir_taps(n_taps: int, b: float, fs_thz: float, band_thz: float, n_grid: int = 4096,
                oob_weight: float = 1e-3) -> np.ndarray:
    """Least-squares FIR approximation of Eq. (1)'s all-pass response over a band.

    Minimizes sum_k W_k |sum_m h_m exp(-j 2 pi f_k (m - c)/fs) - T_k|^2 on the
    n_grid-point DFT grid, T = exp(-j 2 pi^2 b f^2) and W = 1 for |f| <= band,
    T = 0 and W = oob_weight outside.  (A reading: the learnable dispersion
    taps are initialised from the ideal filter this way because plain
    truncation of the impulse response has gain above one near the band
    edge, which a cascade of steps amplifies.)
    """
    c = (n_taps - 1) // 2
    f = np.fft.fftfreq(n_grid, d=1.0 / fs_thz)
    inb = np.abs(f) <= band_thz
    w = np.where(inb, 1.0, oob_weight)
    t = np.where(inb, np.exp(-1j * 2.0 * math.pi ** 2 * b * f * f), 0.0)
    e = np.exp(-2j * math.pi * np.outer(f / fs_thz, np.arange(n_taps) - c))
    sw = np.sqrt(w)
    h, *_ = np.linalg.lstsq(e * sw[:, None], t * sw, rcond=None)
    return h
