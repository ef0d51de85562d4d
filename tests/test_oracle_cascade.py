"""Pins of the oracle's cascades: invariants, round trips, convergence, overlap-and-save (CPU)."""
import math

import numpy as np
import pytest

import siggen
from oracle import dbp_ref as R

FS = siggen.FS_THZ
B2 = siggen.beta2_ps2_km()


def field(seed, n, n_pol=2, p_dbm=2.0):
    x, _ = siggen.transmitted_field(90, seed, n_pol, n, p_dbm)
    return x


def test_beta2_value():
    assert abs(B2 - (-21.6826)) < 1e-3


def test_schedule_effective_length_one_step_per_span():
    # one step per span: |phi| = gamma * (1 - e^{-alpha L_s}) / alpha, the paper's dz_eff
    st = R.schedule(2, 80.0, 1, B2, 1.3, 0.2)
    a = 0.2 * math.log(10) / 10
    assert abs(st[0].phi - (-1.3 * (1 - math.exp(-a * 80)) / a)) < 1e-12
    assert abs(st[0].b - (-B2 * 80.0)) < 1e-12
    fwd = R.schedule(2, 80.0, 1, B2, 1.3, 0.2, backward=False)
    assert fwd[0].phi == -st[0].phi and fwd[0].b == -st[0].b


def test_schedule_weights_sum_to_span_effective_length():
    # the segment weights of a span add up to the span's effective length, in either direction
    a = 0.2 * math.log(10) / 10
    for n in [1, 4, 20]:
        st = R.schedule(1, 80.0, n, B2, 1.3, 0.2)
        assert abs(sum(s.phi for s in st) + 1.3 * (1 - math.exp(-80 * a)) / a) < 1e-12
        # backward order: first segment is the receiver-side (low-power) one
        assert abs(st[0].phi) <= abs(st[-1].phi)


def test_gamma_zero_round_trip():
    x = field(1, 2048)
    fwd = R.schedule(5, 80.0, 3, B2, 0.0, 0.2, backward=False)
    bwd = R.schedule(5, 80.0, 3, B2, 0.0, 0.2, backward=True)
    y = R.run_whole(R.run_whole(x, fwd, FS), bwd, FS)
    assert np.max(np.abs(y - x)) / np.max(np.abs(x)) < 1e-13


@pytest.mark.parametrize("alpha", [0.0, 0.2])
def test_energy_conserved(alpha):
    x = field(2, 4096, p_dbm=6.0)
    st = R.schedule(4, 80.0, 2, B2, 1.3, alpha, taps=[0.05, 0.2, 0.5, 0.2, 0.05])
    y = R.run_whole(x, st, FS)
    assert abs(np.sum(np.abs(y) ** 2) / np.sum(np.abs(x) ** 2) - 1) < 1e-13


def test_su2_covariance():
    x = field(3, 2048, p_dbm=6.0)
    th, ph, ps = 0.7, 1.1, -0.4
    u = np.array([[math.cos(th) * np.exp(1j * ph), -math.sin(th) * np.exp(1j * ps)],
                  [math.sin(th) * np.exp(-1j * ps), math.cos(th) * np.exp(-1j * ph)]])
    st = R.schedule(3, 80.0, 1, B2, 1.3, 0.2, taps=[0.1, 0.8, 0.1])
    a = R.run_whole(u @ x, st, FS)
    b = u @ R.run_whole(x, st, FS)
    assert np.max(np.abs(a - b)) < 1e-14


def test_time_shift_commutes():
    x = field(4, 1024, p_dbm=6.0)
    st = R.schedule(2, 80.0, 2, B2, 1.3, 0.2, taps=[0.2, 0.6, 0.2])
    a = R.run_whole(np.roll(x, 37, axis=-1), st, FS)
    b = np.roll(R.run_whole(x, st, FS), 37, axis=-1)
    assert np.max(np.abs(a - b)) < 1e-14


def test_ssfm_first_order_convergence():
    # Lie splitting: error against a very fine solution halves per doubling of the step count
    x = field(5, 2048, p_dbm=8.0)
    ref = R.run_whole(x, R.schedule(4, 80.0, 256, B2, 1.3, 0.2), FS)
    errs = []
    for n in [4, 8, 16, 32]:
        y = R.run_whole(x, R.schedule(4, 80.0, n, B2, 1.3, 0.2), FS)
        errs.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(1.6 < r < 2.6 for r in ratios), ratios


def test_backpropagation_inverts_fine_forward():
    # noise-free: DBP(fine forward(x)) -> x as the DBP step count grows
    x = field(6, 4096, p_dbm=6.0)
    rx = R.run_whole(x, R.schedule(4, 80.0, 200, B2, 1.3, 0.2, backward=False), FS)
    errs = []
    for n in [1, 4, 16, 64]:
        y = R.run_whole(rx, R.schedule(4, 80.0, n, B2, 1.3, 0.2), FS)
        errs.append(np.linalg.norm(y - x) / np.linalg.norm(x))
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    cd_only = R.run_whole(rx, R.schedule(4, 80.0, 1, B2, 0.0, 0.2), FS)
    assert errs[0] < np.linalg.norm(cd_only - x) / np.linalg.norm(x)


# ----------------------------------------------------------------- overlap-and-save

def test_blocked_single_block_is_whole():
    x = field(7, 1024)
    st = R.schedule(3, 80.0, 1, B2, 1.3, 0.2, taps=[0.1, 0.8, 0.1])
    a = R.run_blocked(x, st, FS, 1024, 0, 2)
    assert np.array_equal(a, R.run_whole(x, st, FS)) or np.max(np.abs(a - R.run_whole(x, st, FS))) < 1e-15


def test_blocked_exact_without_dispersion():
    # beta2 = 0: the phase rotations leave every intensity unchanged, so the wrapped
    # intensities of a block corrupt only the Nc samples at each edge, for any k:
    # a halo of Nc is exact, a halo of Nc - 1 is not
    x = field(8, 3000)
    w = [0.05, 0.1, 0.2, 0.3, 0.2, 0.1, 0.05]        # Nc = 3
    st = R.schedule(6, 80.0, 1, 0.0, 1.3, 0.2, taps=w)
    want = R.run_whole(x, st, FS)
    for k in [1, 2, 6]:
        got = R.run_blocked(x, st, FS, 256, 2 * 3, k)
        assert np.max(np.abs(got - want)) < 1e-15
        bad = R.run_blocked(x, st, FS, 256, 2 * 2, k)
        assert np.max(np.abs(bad - want)) > 1e-9


def test_blocked_exact_with_fir_linear_substep():
    x = field(9, 2000)
    hf = 4
    nc = 2
    g = np.random.default_rng(9)
    steps = [R.Step(b=0.0, phi=-20.0, w=np.array([0.1, 0.2, 0.4, 0.2, 0.1]),
                    h=(g.standard_normal(2 * hf + 1) + 1j * g.standard_normal(2 * hf + 1)) / 3)
             for _ in range(4)]
    want = R.run_whole(x, steps, FS)
    got = R.run_blocked(x, steps, FS, 128, 2 * 2 * (hf + nc), 2)
    assert np.max(np.abs(got - want)) < 1e-14


def test_blocked_error_decreases_with_overlap():
    x = field(10, 8192)
    st = R.schedule(4, 80.0, 1, B2, 1.3, 0.2, taps=[0.1, 0.8, 0.1])
    want = R.run_whole(x, st, FS)
    errs = [np.linalg.norm(R.run_blocked(x, st, FS, 1024, o, 1) - want) / np.linalg.norm(want)
            for o in [32, 64, 128, 256]]
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    assert errs[-1] < 1e-3


def test_blocked_partial_last_block_and_ragged_length():
    # L not a multiple of V: the last block is partial, every output sample written exactly once
    n = 1000
    x = field(11, n)
    st = [R.Step(b=0.0, phi=0.0)]
    got = R.run_blocked(x, st, FS, 256, 64, 1)     # identity step: blocked must reproduce x
    assert np.max(np.abs(got - x)) < 1e-15
    assert len(R.block_starts(n, 256, 64)) == math.ceil(n / 192)


def test_blocked_rejects_bad_geometry():
    x = field(12, 512)
    for nb, o, k in [(1024, 0, 1), (256, 3, 1), (256, 256, 1), (256, 0, 0)]:
        with pytest.raises(ValueError):
            R.run_blocked(x, [R.Step(0.0, 0.0)], FS, nb, o, k)
