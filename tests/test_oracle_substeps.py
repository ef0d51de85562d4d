"""Pins of the oracle's substeps against closed forms and brute force (CPU only)."""
import math

import numpy as np
import pytest

from oracle import dbp_ref as R

FS = 0.056


def brute_dft(x):
    n = len(x)
    k = np.arange(n)
    return np.array([np.sum(x * np.exp(-2j * math.pi * kk * k / n)) for kk in range(n)])


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 16, 64])
def test_library_dft_matches_brute_force(n):
    g = np.random.default_rng(n)
    x = g.standard_normal(n) + 1j * g.standard_normal(n)
    assert np.allclose(np.fft.fft(x), brute_dft(x), atol=1e-12, rtol=0)


def test_linear_substep_brute_force_small():
    # Eq. (1) written with an explicit O(L^2) DFT pair on a tiny, odd-length block
    n = 7
    g = np.random.default_rng(1)
    x = g.standard_normal((2, n)) + 1j * g.standard_normal((2, n))
    b = -1734.6
    f = np.array([(k if k < (n + 1) // 2 else k - n) * FS / n for k in range(n)])
    hresp = np.exp(-1j * 2 * math.pi ** 2 * b * f ** 2)
    kk = np.arange(n)
    fwd = np.exp(-2j * math.pi * np.outer(kk, kk) / n)
    inv = np.conj(fwd) / n
    want = np.stack([inv @ (hresp * (fwd @ xp)) for xp in x])
    assert np.allclose(R.linear_substep(x, b, FS), want, atol=1e-13, rtol=0)


def test_single_tone_is_eigenfunction():
    n = 256
    b = -21.68 * 80.0
    for k0 in [0, 1, 17, 128, 200]:
        x = np.exp(2j * math.pi * k0 * np.arange(n) / n)[None, :]
        f = (k0 if k0 < n // 2 else k0 - n) * FS / n
        want = x * np.exp(-1j * 2 * math.pi ** 2 * b * f * f)
        assert np.allclose(R.linear_substep(x, b, FS), want, atol=1e-12, rtol=0)


def test_dispersion_semigroup():
    g = np.random.default_rng(2)
    x = g.standard_normal((2, 512)) + 1j * g.standard_normal((2, 512))
    a = R.linear_substep(R.linear_substep(x, -300.0, FS), 1200.0, FS)
    assert np.allclose(a, R.linear_substep(x, 900.0, FS), atol=1e-12)


def test_gaussian_pulse_closed_form():
    # a(t) = exp(-t^2/(2 T0^2)); after exp(-j beta2 w^2 z / 2) (Eq. (1), w = 2 pi f):
    # a(t) = T0 / sqrt(T0^2 + j b) * exp(-t^2 / (2 (T0^2 + j b))), b = beta2 z.
    n = 4096
    t = (np.arange(n) - n // 2) / FS
    t0 = 100.0
    for b in [-21.6826 * 80.0, 21.6826 * 40.0, -5000.0]:
        x = np.exp(-t ** 2 / (2 * t0 ** 2))[None, :]
        s = t0 ** 2 + 1j * b
        want = t0 / np.sqrt(s) * np.exp(-t ** 2 / (2 * s))
        got = R.linear_substep(x, b, FS)[0]
        assert np.max(np.abs(got - want)) < 1e-12


def test_cw_nonlinear_phase():
    # constant vector input: the FFT step is the identity at DC, the rotation is analytic
    a = np.array([0.03 + 0.01j, -0.02j])
    x = np.repeat(a[:, None], 64, axis=1)
    w = np.array([0.1, 0.2, 0.4, 0.2, 0.1])
    phi = -1.3 * 21.0
    out = R.step(x, R.Step(b=-1734.0, phi=phi, w=w), FS)
    p = np.sum(np.abs(a) ** 2)
    want = x * np.exp(-1j * phi * w.sum() * p)
    assert np.allclose(out, want, atol=1e-15, rtol=1e-13)
    out_ssfm = R.step(x, R.Step(b=-1734.0, phi=phi), FS)
    assert np.allclose(out_ssfm, x * np.exp(-1j * phi * p), atol=1e-15, rtol=1e-13)


def test_zero_dispersion_closed_form_cascade():
    # beta2 = 0: intensity is preserved, phases add: x exp(-j sum_s phi_s (w_s (*) I))
    g = np.random.default_rng(3)
    x = (g.standard_normal((2, 300)) + 1j * g.standard_normal((2, 300))) * 0.03
    steps = []
    for s in range(6):
        w = g.uniform(0, 1, 2 * (s % 3) + 1)
        steps.append(R.Step(b=0.0, phi=-20.0 + s, w=w))
    steps.append(R.Step(b=0.0, phi=-7.0))
    inten = np.sum(np.abs(x) ** 2, axis=0)
    phase = np.zeros(300)
    for st in steps:
        if st.w is None:
            phase += st.phi * inten
        else:
            nt = len(st.w)
            c = nt // 2
            for m in range(nt):      # explicit shifted sum, independent of np.roll
                for n in range(300):
                    phase[n] += st.phi * st.w[m] * inten[(n - (m - c)) % 300]
    want = x * np.exp(-1j * phase)[None, :]
    assert np.allclose(R.run_whole(x, steps, FS), want, atol=1e-14, rtol=1e-12)


def test_essfm_with_delta_taps_equals_ssfm_bitwise():
    g = np.random.default_rng(4)
    x = (g.standard_normal((2, 256)) + 1j * g.standard_normal((2, 256))) * 0.03
    d = np.zeros(9)
    d[4] = 1.0
    a = R.run_whole(x, [R.Step(b=-900.0, phi=-25.0, w=d)] * 3, FS)
    b = R.run_whole(x, [R.Step(b=-900.0, phi=-25.0)] * 3, FS)
    assert np.array_equal(a, b)


def test_step_order_is_linear_then_nonlinear():
    # ops (i)-(iv): the phase is driven by the intensity after dispersion
    g = np.random.default_rng(5)
    x = (g.standard_normal((2, 128)) + 1j * g.standard_normal((2, 128))) * 0.05
    st = R.Step(b=-1500.0, phi=-30.0, w=np.array([0.25, 0.5, 0.25]))
    y = R.linear_substep(x, st.b, FS)
    want = R.nonlinear_substep(y, st.phi, st.w)
    got = R.step(x, st, FS)
    assert np.array_equal(got, want)
    other = R.linear_substep(R.nonlinear_substep(x, st.phi, st.w), st.b, FS)
    assert np.max(np.abs(got - other)) > 1e-4


def test_tap_orientation_asymmetric():
    # w[m] multiplies I[n - (m - c)]: a tap right of centre delays the intensity
    inten = np.zeros(16)
    inten[5] = 1.0
    w = np.array([0.0, 0.0, 0.0, 1.0, 0.0])   # m = 3, c = 2 -> shift by +1
    assert R.filtered_intensity(inten, w)[6] == 1.0


def test_single_polarization_reduction():
    # y = 0: the Manakov step reduces to the scalar step on x alone
    g = np.random.default_rng(6)
    xs = (g.standard_normal(256) + 1j * g.standard_normal(256)) * 0.04
    x2 = np.stack([xs, np.zeros(256)])
    steps = R.schedule(3, 80.0, 1, -21.68, 1.3, 0.2, taps=[0.1, 0.8, 0.1])
    a = R.run_whole(x2, steps, FS)
    b = R.run_whole(xs[None, :], steps, FS)
    assert np.allclose(a[0], b[0], atol=1e-15)
    assert np.all(a[1] == 0)


def test_fir_linear_substep_matches_fft_when_taps_exact():
    # a FIR holding the whole circular impulse response equals the FFT linear step
    n = 33
    b = -600.0
    imp = np.fft.ifft(R.dispersion_response(n, b, FS))
    c = n // 2
    h = np.array([imp[(m - c) % n] for m in range(n)])
    g = np.random.default_rng(7)
    x = g.standard_normal((2, n)) + 1j * g.standard_normal((2, n))
    assert np.allclose(R.fir_linear_substep(x, h), R.linear_substep(x, b, FS), atol=1e-13)


def test_ideal_fir_taps_are_l2_optimal_truncation():
    # the truncated taps minimize sum_f |H(f) - sum_m h_m e^{-j 2pi f (m-c)}|^2 on the fine grid,
    # i.e. they equal the impulse response samples: check energy and centre symmetry
    b = -21.6826 * 80.0
    h = R.ideal_fir_taps(33, b, FS)
    assert np.allclose(h, h[::-1], atol=1e-15)         # even impulse response (f^2 phase)
    assert 0.5 < np.sum(np.abs(h) ** 2) <= 1.0 + 1e-12  # all-pass: total energy 1 over all lags


def test_ls_fir_full_band_is_truncated_impulse_response():
    # with the whole grid in band and unit weight, the least-squares FIR on an N-point DFT grid
    # is the centre of the N-point impulse response (orthogonality of the DFT basis)
    b = -21.6826 * 80.0
    for nt in [9, 33]:
        a = R.ls_fir_taps(nt, b, FS, 1.0, n_grid=4096)
        t = R.ideal_fir_taps(nt, b, FS, n_fft=4096)
        assert np.max(np.abs(a - t)) < 1e-14


def test_ls_fir_band_design_is_stable_and_close_in_band():
    b = -21.6826 * 80.0
    band = 0.0154
    f = np.linspace(-FS / 2, FS / 2, 2001)
    for h, gain_max, err_max in [(R.ls_fir_taps(33, b, FS, band), 1.01, 0.01),
                                 (R.ideal_fir_taps(33, b, FS), 1.4, 0.1)]:
        c = len(h) // 2
        resp = np.exp(-2j * math.pi * np.outer(f / FS, np.arange(len(h)) - c)) @ h
        inb = np.abs(f) <= band
        err = np.sqrt(np.mean(np.abs(resp[inb] - np.exp(-1j * 2 * math.pi ** 2 * b * f[inb] ** 2)) ** 2))
        assert np.abs(resp).max() < gain_max and err < err_max
    # plain truncation of an 80 km response exceeds unit gain (a 40-step cascade would amplify)
    h = R.ideal_fir_taps(33, b, FS)
    resp = np.exp(-2j * math.pi * np.outer(f / FS, np.arange(33) - 16)) @ h
    assert np.abs(resp).max() > 1.2
