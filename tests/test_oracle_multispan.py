"""Pins of the multi-span step schedule (steps covering several whole spans, as in the
experiment of Sec. IV: one step per two spans, or one step for the whole link)."""
import math

import numpy as np
import pytest

import siggen
from oracle import dbp_ref as R

B2 = siggen.beta2_ps2_km()
FS = siggen.FS_THZ


def test_one_span_per_step_is_the_default():
    a = R.schedule(8, 80.0, 1, B2, 1.3, 0.2)
    b = R.schedule(8, 80.0, 1, B2, 1.3, 0.2, spans_per_step=1)
    assert [(s.b, s.phi) for s in a] == [(s.b, s.phi) for s in b]


@pytest.mark.parametrize("m", [2, 4, 8, 40])
def test_link_totals_are_kept(m):
    """Whatever the grouping, the link's total dispersion is -beta2 * N_span * L and the
    total nonlinear weight is -gamma * N_span * L_eff(L) (each span contributes its own
    effective length (1 - e^{-alpha L}) / alpha, Sec. II)."""
    st = R.schedule(40, 80.0, 1, B2, 1.3, 0.2, spans_per_step=m)
    assert len(st) == 40 // m
    alpha = 0.2 * math.log(10) / 10
    leff = (1 - math.exp(-alpha * 80.0)) / alpha
    assert math.isclose(sum(s.b for s in st), -B2 * 3200.0, rel_tol=1e-14)
    assert math.isclose(sum(s.phi for s in st), -1.3 * 40 * leff, rel_tol=1e-14)
    assert math.isclose(leff, 21.169, rel_tol=1e-4)        # the 80 km effective length


@pytest.mark.parametrize("taps", [None, siggen.symmetric_taps(siggen.rng(9, 0), 3)])
def test_dispersionless_link_is_the_closed_form(taps):
    """beta2 = 0: intensity is invariant, so every grouping gives x exp(-j sum(phi) (w * I))."""
    x = siggen.transmitted_field(9, 1, 2, 2048, 3.0)[0]
    st = R.schedule(8, 80.0, 1, 0.0, 1.3, 0.2, spans_per_step=4, taps=taps)
    y = R.run_whole(x, st, FS)
    i = np.abs(x[0]) ** 2 + np.abs(x[1]) ** 2
    j = i if taps is None else sum(taps[m] * np.roll(i, m - (len(taps) - 1) // 2) for m in range(len(taps)))
    phi = sum(s.phi for s in st)
    assert np.allclose(y, x * np.exp(-1j * phi * j)[None, :], rtol=0, atol=1e-13)


def test_linear_link_is_one_dispersion_step():
    """gamma = 0: the steps compose (semigroup of Eq. (1)) into the whole link's dispersion."""
    x = siggen.transmitted_field(9, 2, 2, 4096, 0.0)[0]
    y = R.run_whole(x, R.schedule(40, 80.0, 1, B2, 0.0, 0.2, spans_per_step=40), FS)
    f = np.fft.fftfreq(4096, 1 / FS)
    ref = np.fft.ifft(np.fft.fft(x, axis=-1) * np.exp(1j * 2 * math.pi ** 2 * B2 * 3200.0 * f * f), axis=-1)
    assert np.allclose(y, ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("kw", [dict(n_spans=40, steps_per_span=1, spans_per_step=3),
                                dict(n_spans=40, steps_per_span=2, spans_per_step=2),
                                dict(n_spans=40, steps_per_span=1, spans_per_step=0)])
def test_invalid_groupings_are_refused(kw):
    with pytest.raises(ValueError):
        R.schedule(kw["n_spans"], 80.0, kw["steps_per_span"], B2, 1.3, 0.2, spans_per_step=kw["spans_per_step"])
