"""Pins of the shared input generator and receiver metric (CPU)."""
import math

import numpy as np

import siggen


def test_rrc_pair_is_nyquist_zero_isi():
    sym = siggen.qpsk_symbols(siggen.rng(92, 0), 2, 1000)
    x = siggen.shape(sym)
    assert np.allclose(siggen.matched_filter_symbols(x), sym, atol=1e-12)


def test_power_scaling_and_seeding():
    x, s = siggen.transmitted_field(92, 1, 2, 4096, 3.0)
    p = siggen.dbm_to_w(3.0)
    assert np.allclose(np.mean(np.abs(x) ** 2, axis=-1), p / 2)
    x2, s2 = siggen.transmitted_field(92, 1, 2, 4096, 3.0)
    assert np.array_equal(x, x2) and np.array_equal(s, s2)
    x3, _ = siggen.transmitted_field(92, 2, 2, 4096, 3.0)
    assert not np.array_equal(x, x3)


def test_evm_of_clean_signal_is_tiny_and_gain_invariant():
    x, s = siggen.transmitted_field(92, 3, 2, 8192, 0.0)
    assert siggen.evm(siggen.matched_filter_symbols(x), s) < 1e-10
    y = x * (0.3 * np.exp(1j * 0.8))
    assert siggen.evm(siggen.matched_filter_symbols(y), s) < 1e-10


def test_awgn_evm_matches_osnr():
    # SNR per symbol after the matched filter = OSNR * ref_bw / symbol rate (two polarizations)
    p = siggen.dbm_to_w(0.0)
    x, s = siggen.transmitted_field(92, 4, 2, 1 << 17, 0.0)
    osnr = 20.0
    y = siggen.add_awgn(siggen.rng(92, 4, 1), x, siggen.awgn_sigma2(p, osnr))
    snr = 10 ** (osnr / 10) * siggen.OSNR_REF_BW_THZ / siggen.SYMBOL_RATE_THZ
    assert abs(siggen.evm_db(y, s) - (-10 * math.log10(snr))) < 0.1


def test_ragged_lengths_range():
    l = siggen.ragged_lengths(siggen.rng(2, 0), 512)
    assert l.min() >= 4096 and l.max() <= 131072 and np.all(l % 2 == 0)
    assert 25000 < l.mean() < 50000


def test_symmetric_taps():
    w = siggen.symmetric_taps(siggen.rng(2, 1), 4)
    assert len(w) == 9 and np.allclose(w, w[::-1]) and abs(w.sum() - 1) < 1e-15
