"""GPU parity of the receiver DSP after backpropagation (resampling, least-squares butterfly
equalizer, carrier-phase recovery, decisions) against the FP64 oracle.

Each stage gets the same input on both sides (the GPU's complex64 input, widened for the
oracle).  Tolerances from the arithmetic: resampling and equalizing are FP32 sums of 48 and
30 products (relative L2 <= 1e-6); the equalizer taps come from FP32 chunk sums of the normal
equations solved in FP64 (relative <= 1e-4 at the conditioning of a noisy 20 dB capture);
the carrier phase is an FP32 running sum of wrapped differences (<= 1e-4 rad after 10^5
symbols).  Decisions agree except for symbols within 1e-3 of a decision boundary, which
both sides may legitimately put either way.
"""
import numpy as np
import pytest

import siggen
from oracle import rxdsp as D

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1507_00921_amd as m
    m.lib()
    return m


def capture(seed, n_sym, snr_db=20.0, linewidth=200e3):
    """Back-to-back 50 GSa/s capture: rotated polarizations, laser phase noise, AWGN."""
    x, s = siggen.transmitted_field_at_rate(40, seed, 2, n_sym, 0.0, 0.050)
    U = siggen.polarization_rotation(siggen.rng(40, seed, 1))
    ph = siggen.laser_phase_noise(siggen.rng(40, seed, 2), x.shape[-1], linewidth, 0.050)
    y = (U @ x) * np.exp(1j * ph)
    p = np.mean(np.abs(y) ** 2)
    y = siggen.add_awgn(siggen.rng(40, seed, 3), y, p / 10 ** (snr_db / 10)) / np.sqrt(p)
    return y.astype(np.complex64), s.astype(np.complex64)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy().astype(np.complex128)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def near_boundary(z, tol=1e-3):
    return (np.abs(z.real) < tol) | (np.abs(z.imag) < tol)


@pytest.mark.parametrize("n_sym,taps,beta", [(2800, 48, 8.0), (14014, 32, 7.0), (1400, 64, 9.0)])
def test_resample_matches_oracle(dbp, n_sym, taps, beta):
    x, _ = capture(1, n_sym)
    d = dbp.receiver_dsp(x.shape[-1], resample_taps=taps, kaiser_beta=beta)
    y = host(d.resample(dev(x)))
    ref = D.resample(x.astype(np.complex128), 28, 25, taps, beta)
    err = rel(y, ref)
    print(f"resample n_sym={n_sym} K={taps}: rel L2 {err:.2e}")
    assert y.shape == ref.shape and err <= 1e-6


def test_train_equalize_cpr_match_oracle(dbp):
    n_sym = 28000
    x, s = capture(2, n_sym)
    d = dbp.receiver_dsp(x.shape[-1])
    x2 = d.resample(dev(x))
    sd = dev(s)
    taps = d.train(x2, sd, 4000)
    x2h = host(x2)
    W_ref = D.equalizer_ls(x2h, s.astype(np.complex128), 15, 4000)
    errw = rel(host(taps), W_ref)
    print(f"equalizer taps rel {errw:.2e}")
    assert errw <= 1e-4
    y = d.equalize(x2, taps)
    y_ref = D.equalizer_apply(x2h, host(taps))
    erry = rel(host(y), y_ref)
    print(f"equalizer output rel L2 {erry:.2e}")
    assert erry <= 1e-6
    z, nerr = d.cpr(y, sd, 4000)
    yh = host(y)
    z_ref = D.cpr(yh, 16, s.astype(np.complex128), 4000)
    errz = float(np.max(np.abs(host(z) - z_ref)))
    print(f"phase recovery max |dz| {errz:.2e}, bit errors {nerr}")
    assert errz <= 1e-4
    amb = int(np.sum(near_boundary(z_ref)))
    assert abs(nerr - D.bit_errors(z_ref, s.astype(np.complex128))) <= amb
    assert nerr == D.bit_errors(host(z), s.astype(np.complex128))


def test_chain_at_full_size_matches_oracle_on_sampled_symbols(dbp):
    # 131068 symbols (2 x 234050 samples at 50 GSa/s, the headline field's length in time):
    # BER of the whole block from the GPU, resampling and equalizer output checked on sampled
    # positions against the oracle's formulas, phase against the oracle over the block
    n_sym = 131068
    x, s = capture(3, n_sym, snr_db=16.0)
    d = dbp.receiver_dsp(x.shape[-1])
    x2 = d.resample(dev(x))
    taps = d.train(x2, dev(s), 8000)
    y = d.equalize(x2, taps)
    z, nerr = d.cpr(y, dev(s), 8000)
    torch.cuda.synchronize()
    r = np.random.default_rng(7)
    pick = np.sort(r.choice(x2.shape[-1], 200, replace=False))
    x2h = host(x2)
    ref = D.resample(x.astype(np.complex128), 28, 25)            # whole block, FP64
    assert rel(x2h[:, pick], ref[:, pick]) <= 1e-6
    ks = np.sort(r.choice(n_sym, 200, replace=False))
    Wh = host(taps)
    U = D.regressors(x2h, 15, ks)
    y_ref = (U @ Wh.reshape(2, 30).T).T
    assert rel(host(y)[:, ks], y_ref) <= 1e-6
    zh = host(z)
    z_ref = D.cpr(host(y), 16, s.astype(np.complex128), 8000)
    assert float(np.max(np.abs(zh - z_ref))) <= 1e-4
    ber = nerr / (4 * n_sym)
    print(f"full block: {nerr} bit errors, BER {ber:.2e}")
    assert nerr == D.bit_errors(zh, s.astype(np.complex128))
    assert ber < 1e-3


def test_argument_rules(dbp):
    x, s = capture(4, 1400)
    d = dbp.receiver_dsp(x.shape[-1])
    x2 = d.resample(dev(x))
    with pytest.raises(dbp.DbpError):
        d.train(x2, dev(s), 0)
    with pytest.raises(dbp.DbpError):
        d.train(x2, dev(s), s.shape[-1] + 1)
    import ctypes
    L = dbp.lib()
    y = torch.empty(2, d.n_sym, dtype=torch.complex64, device="cuda")
    # output overlapping the input
    assert L.dbp_dsp_equalize(d._h, ctypes.c_void_p(x2.data_ptr()), ctypes.c_void_p(x2.data_ptr()),
                              ctypes.c_void_p(x2.data_ptr()), None) == 1
    assert L.dbp_dsp_cpr(d._h, ctypes.c_void_p(y.data_ptr()), None, 0, ctypes.c_void_p(y.data_ptr()), None,
                         None) == 1
    z = torch.empty_like(y)
    assert L.dbp_dsp_cpr(d._h, ctypes.c_void_p(y.data_ptr()), None, 10, ctypes.c_void_p(z.data_ptr()), None,
                         None) == 1                                  # reference symbols missing


def test_backpropagation_at_the_scope_rate_then_dsp_matches_oracle(dbp):
    # the paper's order: ESSFM backpropagation at 50 GSa/s (about 1.8 samples per symbol), then
    # resampling, equalizer and phase recovery; 4 x 80 km at +3 dBm, forward channel by the
    # oracle at 20 steps per span, 16 dB OSNR for 0 dBm, rotation and phase noise after it
    from oracle import dbp_ref as R
    fs, n_spans, n_sym = 0.050, 4, 14000
    x, s = siggen.transmitted_field_at_rate(41, 0, 2, n_sym, 3.0, fs)
    fwd = R.schedule(n_spans, 80.0, 20, siggen.beta2_ps2_km(), siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM,
                     backward=False)
    rx = R.run_whole(x, fwd, fs)
    rx = siggen.add_awgn(siggen.rng(41, 0, 1), rx, siggen.awgn_sigma2(siggen.dbm_to_w(0.0), 16.0, fs_thz=fs))
    rx = siggen.polarization_rotation(siggen.rng(41, 0, 2)) @ rx
    rx = (rx * np.exp(1j * siggen.laser_phase_noise(siggen.rng(41, 0, 3), rx.shape[-1], 200e3, fs)))
    rx = rx.astype(np.complex64)
    n = rx.shape[-1]
    taps = siggen.symmetric_taps(siggen.rng(41, 0, 4), 4).astype(np.float32)
    p = dbp.plan(n, n_spans, 1, fs_thz=fs, taps=taps, block=1024, overlap=256, beta2_ps2_km=siggen.beta2_ps2_km())
    y = p.backprop(dev(rx).reshape(1, 2, n)).reshape(2, n).contiguous()
    steps = R.schedule(n_spans, 80.0, 1, siggen.beta2_ps2_km(), siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM,
                       taps=taps.astype(np.float64))
    y_ref = R.run_blocked(rx.astype(np.complex128), steps, fs, p.block, p.overlap, p.steps_per_pass)
    err = rel(host(y), y_ref)
    print(f"ESSFM at 50 GSa/s, Nb={p.block} O={p.overlap} k={p.steps_per_pass}: rel L2 {err:.2e}")
    assert err <= 1e-5
    d = dbp.receiver_dsp(n)
    x2 = d.resample(y)
    taps_eq = d.train(x2, dev(s.astype(np.complex64)), 3000)
    z, nerr = d.cpr(d.equalize(x2, taps_eq), dev(s.astype(np.complex64)), 3000)
    z_ref, _ = D.receiver_chain(y_ref, s, 28, 25, 48, 8.0, 15, 3000, 16)
    zh = host(z)
    amb = int(np.sum(near_boundary(z_ref)))
    print(f"bit errors GPU {nerr}, oracle chain {D.bit_errors(z_ref, s)}, near-boundary {amb}, "
          f"EVM {20 * np.log10(siggen.evm(zh, s)):.3f} / {20 * np.log10(siggen.evm(z_ref, s)):.3f} dB")
    assert abs(nerr - D.bit_errors(z_ref, s)) <= amb
    assert abs(20 * np.log10(siggen.evm(zh, s)) - 20 * np.log10(siggen.evm(z_ref, s))) <= 0.01


def test_degenerate_settings_match_oracle(dbp):
    # ratio 1 (identity resampling), one-tap butterfly (the even samples only), a one-symbol
    # phase window: every stage still equals the oracle's
    x, s = capture(5, 2800)
    n = x.shape[-1]
    d = dbp.receiver_dsp(n, up=25, down=25, resample_taps=2, kaiser_beta=0.0, eq_taps=1, cpr_half_window=0)
    assert (d.n_out, d.n_sym) == (n, n // 2)
    x2 = d.resample(dev(x))
    assert float(np.max(np.abs(host(x2) - x.astype(np.complex128)))) <= 1e-6
    ref2 = D.resample(x.astype(np.complex128), 25, 25, 2, 0.0)
    assert rel(host(x2), ref2) <= 1e-7
    sym2 = s[:, : n // 2].astype(np.complex64)                  # any known sequence of the right length
    taps = d.train(x2, dev(sym2), 1000)
    W_ref = D.equalizer_ls(host(x2), sym2.astype(np.complex128), 1, 1000)
    assert rel(host(taps), W_ref) <= 1e-4
    y = d.equalize(x2, taps)
    assert rel(host(y), D.equalizer_apply(host(x2), host(taps))) <= 1e-6
    z, _ = d.cpr(y)
    z_ref = D.cpr(host(y), 0)
    assert float(np.max(np.abs(host(z) - z_ref))) <= 1e-4


def test_training_flags_a_singular_system(dbp):
    # all-zero input: the normal matrix is zero, the GPU solve reports it and leaves NaN taps;
    # a later well-posed training clears the flag
    d = dbp.receiver_dsp(14625)                 # 16380 samples after resampling, 8190 symbols
    x2 = torch.zeros(2, d.n_out, dtype=torch.complex64, device="cuda")
    s = torch.ones(2, d.n_sym, dtype=torch.complex64, device="cuda")
    taps = d.train(x2, s, 1000)
    torch.cuda.synchronize()
    assert d.status() == 1
    assert torch.isnan(torch.view_as_real(taps)).all()
    g = torch.Generator(device="cuda").manual_seed(3)
    x2 = torch.view_as_complex(torch.randn(2, d.n_out, 2, device="cuda", generator=g)).contiguous()
    taps = d.train(x2, s, 1000)
    torch.cuda.synchronize()
    assert d.status() == 0 and torch.isfinite(torch.view_as_real(taps)).all()
    d.close()
