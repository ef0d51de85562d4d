"""Pins of the oracle's ESSFM coefficient fit (Sec. IV least squares), CPU only."""
import numpy as np

import siggen
from oracle import dbp_ref as R
from oracle import fit as F

B2 = siggen.beta2_ps2_km()
FS = siggen.FS_THZ


def _field(n=4096, p_dbm=4.0, n_spans=4):
    x, _ = siggen.transmitted_field(5, 0, 2, n, p_dbm)
    fwd = R.schedule(n_spans, 80.0, 4, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM, backward=False)
    return R.run_whole(x, fwd, FS)


def test_symmetric_layout():
    assert np.array_equal(F.symmetric_full([3.0, 2.0, 1.0]), [1.0, 2.0, 3.0, 2.0, 1.0])
    assert np.array_equal(F.symmetric_full([1.0]), [1.0])


def test_fit_recovers_known_coefficients():
    # target made by ESSFM itself with known coefficients: the fit from SSFM (c = delta)
    # returns them (noise-free, so exactly up to the solver's tolerance)
    rx = _field()
    base = R.schedule(4, 80.0, 1, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM)
    c_true = np.array([0.62, 0.15, 0.04])
    target = F.essfm_blocked(rx, base, c_true, FS, 1024, 256, 2)
    sl = slice(1024, 3072)
    c = F.fit_coefficients(rx, target, base, FS, 1024, 256, 2, 2, sl)
    print("recovered", c)
    assert np.max(np.abs(c - c_true)) < 1e-6


def test_fit_to_multistep_ssfm_is_a_stationary_improvement():
    # Sec. IV's use: ESSFM at one step per span fitted to SSFM at 20 steps per span.  The fit
    # starts at plain SSFM (c = delta) and must end no worse, at a stationary point of the
    # objective (central differences of the sum of squares vanish there)
    rx = _field()
    fine = R.schedule(4, 80.0, 20, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM)
    target = R.run_blocked(rx, fine, FS, 1024, 256, 20)
    base = R.schedule(4, 80.0, 1, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM)
    sl = slice(1024, 3072)
    delta = np.array([1.0, 0.0, 0.0])

    def obj(c):
        return float(np.sum(F.residual(c, rx, target, base, FS, 1024, 256, 1, sl) ** 2))

    c = F.fit_coefficients(rx, target, base, FS, 1024, 256, 1, 2, sl)
    print("fitted", c, "objective", obj(c), "vs SSFM-1", obj(delta))
    assert obj(c) < 0.8 * obj(delta)
    h = 1e-5
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        grad = (obj(c + e) - obj(c - e)) / (2 * h)
        curv = (obj(c + e) - 2 * obj(c) + obj(c - e)) / h ** 2
        print(f"  d/dc{i} = {grad:.3e}, curvature {curv:.3e}")
        assert abs(grad) <= 1e-6 * curv      # the step to the minimum along c_i is below 1e-6
