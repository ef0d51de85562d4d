"""Receiver DSP after backpropagation (Sec. IV), in FP64
(TEST INFRASTRUCTURE ONLY: see oracle/__init__).

Sec. IV processes every captured block in this order: backpropagation at the scope's
sampling rate (about 1.8 samples per symbol), digital resampling to two samples per
symbol, a butterfly equalizer that adapts to polarization-mode dispersion and residual
dispersion, then detection at the symbol rate that copes with laser phase noise, and
decisions.  The paper names the blocks, not their algorithms; these are the readings:

  resample     band-limited interpolation by a Kaiser-windowed sinc of K taps, circular over
               the block, for an output/input rate ratio up/down >= 1
  equalizer    2x2 butterfly of T/2-spaced FIRs with N taps per branch,
               y_p[k] = sum_q sum_j W[p, q, j] x_q[2k + j - c] (c = N // 2), its taps the
               data-aided least-squares (Wiener) solution over a training prefix of symbols
  cpr          Viterbi-Viterbi fourth-power phase estimate per polarization over 2W + 1
               symbols, theta_k = arg(-sum y^4) / 4, unwrapped by quarter turns:
               phi_k = theta_0 + sum_{j <= k} wrap(theta_j - theta_{j-1}), then y e^{-j phi},
               the estimate's quarter-turn ambiguity resolved on the training symbols
  decisions    QPSK quadrant decisions, bit errors against the transmitted symbols
"""
from __future__ import annotations

import numpy as np

QUARTER = np.pi / 2


def kaiser_sinc(tau: np.ndarray, k_half: int, beta: float) -> np.ndarray:
    """Interpolation kernel sinc(tau) w(tau), w the Kaiser window of half-width k_half."""
    r = np.clip(tau / k_half, -1.0, 1.0)
    w = np.where(np.abs(tau) < k_half, np.i0(beta * np.sqrt(1.0 - r * r)) / np.i0(beta), 0.0)
    return np.sinc(tau) * w


def resample(x: np.ndarray, up: int, down: int, n_taps: int = 48, beta: float = 8.0) -> np.ndarray:
    """Samples at the rate up/down times the input's: output m sits at input time
    t_m = m down / up; y[m] = sum_k x[(i_m + k) mod n] h(t_m - i_m - k) for
    k = -K/2 + 1 .. K/2, i_m = floor(t_m), h = kaiser_sinc.  x: [..., n], n up / down integer."""
    n = x.shape[-1]
    assert up >= down and (n * up) % down == 0 and n_taps % 2 == 0
    m_out = n * up // down
    kh = n_taps // 2
    m = np.arange(m_out)
    i = (m * down) // up
    frac = (m * down - i * up) / up
    ks = np.arange(-kh + 1, kh + 1)
    idx = (i[:, None] + ks[None, :]) % n
    h = kaiser_sinc(frac[:, None] - ks[None, :], kh, beta)
    return np.einsum("...mk,mk->...m", x[..., idx], h)


def regressors(x2: np.ndarray, n_taps: int, ks: np.ndarray) -> np.ndarray:
    """Rows u_k = [x_0[2k + j - c], x_1[2k + j - c] for j < N] (circular), shape [len(ks), 2N]."""
    n = x2.shape[-1]
    c = n_taps // 2
    j = np.arange(n_taps)
    pos = (2 * ks[:, None] + j[None, :] - c) % n
    return np.concatenate([x2[0][pos], x2[1][pos]], axis=1)


def equalizer_ls(x2: np.ndarray, sym: np.ndarray, n_taps: int, n_train: int) -> np.ndarray:
    """Least-squares butterfly taps W [2, 2, N] from the first n_train symbols:
    W[p] = argmin sum_k |u_k . w - s_p[k]|^2, i.e. (U^H U) w = U^H s_p."""
    U = regressors(x2, n_taps, np.arange(n_train))
    R = U.conj().T @ U
    P = U.conj().T @ sym[:, :n_train].T
    w = np.linalg.solve(R, P)                                     # [2N, 2]
    return w.T.reshape(2, 2, n_taps)


def equalizer_apply(x2: np.ndarray, W: np.ndarray) -> np.ndarray:
    """y_p[k] = sum_q sum_j W[p, q, j] x_q[2k + j - c] for every symbol k < n / 2."""
    n_taps = W.shape[-1]
    U = regressors(x2, n_taps, np.arange(x2.shape[-1] // 2))
    return (U @ W.reshape(2, 2 * n_taps).T).T


def wrap_quarter(a: np.ndarray) -> np.ndarray:
    """a reduced by whole quarter turns into [-pi/4, pi/4]."""
    return a - QUARTER * np.round(a / QUARTER)


def cpr_phase(y: np.ndarray, half_window: int) -> np.ndarray:
    """Unwrapped carrier phase per polarization and symbol (circular window), [n_pol, n_sym]."""
    n = y.shape[-1]
    y4 = y ** 4
    acc = np.zeros_like(y4)
    for j in range(-half_window, half_window + 1):
        acc += np.roll(y4, -j, axis=-1)                            # acc[k] = sum_j y4[(k + j) mod n]
    theta = np.angle(-acc) / 4.0
    d = wrap_quarter(np.diff(theta, axis=-1))
    return theta[..., :1] + np.concatenate([np.zeros(theta.shape[:-1] + (1,)), np.cumsum(d, axis=-1)], axis=-1)


def cpr(y: np.ndarray, half_window: int, sym: np.ndarray = None, n_ref: int = 0) -> np.ndarray:
    """y e^{-j phi}; with n_ref > 0 known symbols the quarter-turn ambiguity of the fourth-power
    estimate is resolved per polarization: the rotation by q pi/2, q the nearest integer to
    arg(sum_{k < n_ref} z_k conj(s_k)) / (pi/2), that best aligns them."""
    z = y * np.exp(-1j * cpr_phase(y, half_window))
    if n_ref > 0:
        c = np.sum(z[:, :n_ref] * np.conj(sym[:, :n_ref]), axis=-1)
        q = np.round(np.angle(c) / QUARTER)
        z = z * np.exp(-1j * QUARTER * q)[:, None]
    return z


def bit_errors(z: np.ndarray, sym: np.ndarray) -> int:
    """Quadrant decisions of z against the transmitted QPSK symbols: wrong signs of the real
    and imaginary parts."""
    return int(np.sum(np.sign(z.real) != np.sign(sym.real)) + np.sum(np.sign(z.imag) != np.sign(sym.imag)))


def receiver_chain(x: np.ndarray, sym: np.ndarray, up: int, down: int, n_taps_rs: int, beta: float, n_eq: int,
                   n_train: int, half_window: int):
    """Resample the backpropagated field to two samples per symbol, equalize, recover the
    carrier phase: (symbols after phase recovery [2, n_sym], equalizer taps)."""
    x2 = resample(x, up, down, n_taps_rs, beta)
    W = equalizer_ls(x2, sym, n_eq, n_train)
    return cpr(equalizer_apply(x2, W), half_window, sym, n_train), W
