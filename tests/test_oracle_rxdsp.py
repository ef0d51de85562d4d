"""Pins of the receiver-DSP oracle (resampling, butterfly equalizer, carrier-phase recovery
and decisions that follow backpropagation in Sec. IV) against exact constructions: FFT
interpolation of band-limited signals, exactly invertible channels, a library least-squares
solver, analytic phase ramps and planted errors."""
import numpy as np
import pytest

import siggen
from oracle import rxdsp as D


def test_resample_at_ratio_one_is_the_identity():
    r = np.random.default_rng(1)
    x = r.standard_normal((2, 500)) + 1j * r.standard_normal((2, 500))
    assert np.max(np.abs(D.resample(x, 25, 25) - x)) <= 1e-14


def test_resample_band_limited_tones_against_their_analytic_values():
    # tones on the period grid up to 62 % of the input Nyquist band (the RRC signal's extent)
    n = 2500
    r = np.random.default_rng(2)
    f = np.array([-0.31, -0.2, -0.05, 0.0, 0.12, 0.27, 0.31]) * n
    f = np.round(f) / n                                        # cycles per input sample
    a = r.standard_normal(f.size) + 1j * r.standard_normal(f.size)
    t_in = np.arange(n)
    x = (a[None, :] * np.exp(2j * np.pi * f[None, :] * t_in[:, None])).sum(1)
    y = D.resample(x, 28, 25)
    t_out = np.arange(n * 28 // 25) * 25 / 28
    ref = (a[None, :] * np.exp(2j * np.pi * f[None, :] * t_out[:, None])).sum(1)
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    assert err <= 2e-4


def test_resample_rrc_signal_against_fft_interpolation():
    # the 50 GSa/s pulse train brought to 56 GSa/s equals the same train generated at 56 GSa/s
    sym = siggen.qpsk_symbols(siggen.rng(30, 0, 0), 2, 1400)
    x50 = siggen.shape_at_rate(sym, 0.050)
    x56 = siggen.shape_at_rate(sym, 0.056)
    y = D.resample(x50, 28, 25)
    assert np.linalg.norm(y - x56) / np.linalg.norm(x56) <= 2e-4


def test_equalizer_inverts_a_polarization_rotation_exactly():
    # even samples carry U s, odd samples are noise: the least-squares butterfly puts U^H
    # on its centre tap and zeros elsewhere, and returns the symbols
    r = np.random.default_rng(3)
    n_sym, n_taps = 3000, 7
    s = siggen.qpsk_symbols(siggen.rng(31, 0, 0), 2, n_sym)
    U = siggen.polarization_rotation(siggen.rng(31, 0, 1))
    x2 = r.standard_normal((2, 2 * n_sym)) + 1j * r.standard_normal((2, 2 * n_sym))
    x2[:, ::2] = U @ s
    W = D.equalizer_ls(x2, s, n_taps, 1000)
    ref = np.zeros((2, 2, n_taps), complex)
    ref[:, :, n_taps // 2] = U.conj().T
    assert np.max(np.abs(W - ref)) <= 1e-10
    assert np.max(np.abs(D.equalizer_apply(x2, W) - s)) <= 1e-10


def test_equalizer_matches_a_library_least_squares_solver():
    r = np.random.default_rng(4)
    x2 = r.standard_normal((2, 4000)) + 1j * r.standard_normal((2, 4000))
    s = siggen.qpsk_symbols(siggen.rng(32, 0, 0), 2, 2000)
    W = D.equalizer_ls(x2, s, 9, 800)
    c = 4
    rows = []
    for k in range(800):                                          # regressors written out anew
        rows.append([x2[q][(2 * k + j - c) % 4000] for q in range(2) for j in range(9)])
    A = np.array(rows)
    for p in range(2):
        w, *_ = np.linalg.lstsq(A, s[p, :800], rcond=None)
        assert np.max(np.abs(W[p].reshape(-1) - w)) <= 1e-10


def test_cpr_recovers_a_constant_phase():
    s = siggen.qpsk_symbols(siggen.rng(33, 0, 0), 2, 2000)
    y = s * np.exp(1j * 0.3)
    assert np.max(np.abs(D.cpr_phase(y, 16) - 0.3)) <= 1e-12
    assert np.max(np.abs(D.cpr(y, 16) - s)) <= 1e-12


def test_cpr_tracks_a_ramp_through_many_quarter_turns():
    # a symmetric window over a linear phase returns the centre phase exactly; the unwrapped
    # estimate follows 5 rad of rotation (about six quarter turns) without a slip
    n = 5000
    s = siggen.qpsk_symbols(siggen.rng(34, 0, 0), 2, n)
    phase = 0.1 + 0.001 * np.arange(n)
    y = s * np.exp(1j * phase)
    est = D.cpr_phase(y, 16)
    inner = slice(16, n - 16)                                    # the window wraps at the ends
    assert np.max(np.abs(est[:, inner] - phase[inner])) <= 1e-9
    assert D.bit_errors(D.cpr(y, 16)[:, inner], s[:, inner]) == 0


def test_cpr_resolves_the_quarter_turn_ambiguity_on_known_symbols():
    # a phase of 0.3 + pi/2 reads as 0.3 to the fourth-power estimate; the reference symbols
    # restore the quarter turn, per polarization
    s = siggen.qpsk_symbols(siggen.rng(37, 0, 0), 2, 2000)
    y = s * np.exp(1j * np.array([[0.3 + np.pi / 2], [-0.2 - np.pi]]))
    assert D.bit_errors(D.cpr(y, 16), s) > 1000
    z = D.cpr(y, 16, s, 100)
    assert np.max(np.abs(z - s)) <= 1e-12


def test_prefix_sum_unwrap_equals_sequential_unwrap():
    r = np.random.default_rng(5)
    theta = D.wrap_quarter(r.uniform(-3, 3, size=(2, 400)))
    seq = np.empty_like(theta)
    seq[:, 0] = theta[:, 0]
    for k in range(1, theta.shape[1]):                            # the textbook loop
        seq[:, k] = seq[:, k - 1] + D.wrap_quarter(theta[:, k] - seq[:, k - 1])
    par = theta[:, :1] + np.concatenate([np.zeros((2, 1)), np.cumsum(D.wrap_quarter(np.diff(theta)), 1)], 1)
    assert np.max(np.abs(seq - par)) <= 1e-12


def test_bit_errors_count_planted_errors():
    s = siggen.qpsk_symbols(siggen.rng(35, 0, 0), 2, 1000)
    z = s.copy()
    z[0, 10] = np.conj(z[0, 10])                                  # one bit (imaginary sign)
    z[1, 20] = -z[1, 20]                                          # two bits
    z[0, 30] = -np.conj(z[0, 30])                                 # one bit (real sign)
    assert D.bit_errors(z, s) == 4


def test_chain_undoes_rotation_and_phase_noise_back_to_back():
    # back to back (no fibre): a rotated, phase-noisy 50 GSa/s capture with 25 dB SNR comes
    # out of resampling, equalizer and phase recovery with no bit errors
    n_sym = 2800
    x, s = siggen.transmitted_field_at_rate(36, 0, 2, n_sym, 0.0, 0.050)
    U = siggen.polarization_rotation(siggen.rng(36, 0, 1))
    ph = siggen.laser_phase_noise(siggen.rng(36, 0, 2), x.shape[-1], 200e3, 0.050)
    y = (U @ x) * np.exp(1j * ph)
    p = np.mean(np.abs(y) ** 2)
    y = siggen.add_awgn(siggen.rng(36, 0, 3), y, p / 10 ** 2.5)
    z, W = D.receiver_chain(y / np.sqrt(p), s, 28, 25, 48, 8.0, 15, 1000, 16)
    assert D.bit_errors(z[:, 20:-20], s[:, 20:-20]) == 0
    evm = siggen.evm(z[:, 20:-20], s[:, 20:-20])
    assert evm < 0.12
