"""Seeded synthetic inputs and receiver metrics shared by the oracle and the GPU harness.

This module holds none of the backpropagation arithmetic: no dispersion, no
nonlinear phase, no step schedule.  It produces what a receiver would be
handed (a shaped, power-scaled PM-QPSK field plus optical noise), the
fibre constants of the workloads, and the data-aided EVM used to compare
backpropagated fields.  Both sides of a parity check may import it; the
oracle never imports the GPU package and the GPU package never imports the
oracle.

Signal model (the paper's experiment, Sec. IV): 28 GBd QPSK per polarization,
two polarizations (112 Gb/s PM-QPSK), here at 2 samples per symbol with
root-raised-cosine pulses of roll-off 0.1 applied circularly in frequency.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_ROOT = 150700921

# Physical constants and the standard single-mode fibre of the workloads.
C_M_PER_S = 299_792_458.0
SYMBOL_RATE_THZ = 0.028          # 28 GBd
SPS = 2                          # samples per symbol
FS_THZ = SYMBOL_RATE_THZ * SPS   # 0.056 THz sampling rate
ROLLOFF = 0.1
D_PS_NM_KM = 17.0
LAMBDA_NM = 1550.0
GAMMA_W_KM = 1.3
ALPHA_DB_KM = 0.2
SPAN_KM = 80.0
OSNR_REF_BW_THZ = 0.0125         # 12.5 GHz (0.1 nm) OSNR reference bandwidth


def beta2_ps2_km(d_ps_nm_km: float = D_PS_NM_KM, lambda_nm: float = LAMBDA_NM) -> float:
    """Group-velocity dispersion from the dispersion parameter: beta2 = -D lambda^2 / (2 pi c).

    D in ps/(nm km), lambda in nm; returns ps^2/km (negative: anomalous dispersion).
    """
    c_nm_per_ps = C_M_PER_S * 1e9 / 1e12
    return -d_ps_nm_km * lambda_nm ** 2 / (2.0 * math.pi * c_nm_per_ps)


def dbm_to_w(p_dbm: float) -> float:
    return 1e-3 * 10.0 ** (p_dbm / 10.0)


@dataclass(frozen=True)
class Link:
    """A homogeneous link of identical spans with ideal (loss-compensating) amplifiers."""
    n_spans: int
    span_km: float = SPAN_KM
    beta2_ps2_km: float = beta2_ps2_km()
    gamma_w_km: float = GAMMA_W_KM
    alpha_db_km: float = ALPHA_DB_KM
    fs_thz: float = FS_THZ


def rng(cfg: int, idx: int = 0, stream: int = 0) -> np.random.Generator:
    """Counter-style seeding: one independent generator per (workload, item, stream)."""
    return np.random.default_rng([SEED_ROOT, int(cfg), int(idx), int(stream)])


def qpsk_symbols(gen: np.random.Generator, n_pol: int, n_sym: int) -> np.ndarray:
    """Uniform random QPSK symbols (+-1 +-j)/sqrt(2), shape [n_pol, n_sym], complex128."""
    bits = gen.integers(0, 2, size=(n_pol, n_sym, 2))
    return ((2 * bits[..., 0] - 1) + 1j * (2 * bits[..., 1] - 1)) / math.sqrt(2.0)


def raised_cosine(f_norm: np.ndarray, rolloff: float = ROLLOFF) -> np.ndarray:
    """Raised-cosine spectrum RC(f) with unit in-band value; f in units of the symbol rate."""
    a = np.abs(f_norm)
    f1 = (1.0 - rolloff) / 2.0
    f2 = (1.0 + rolloff) / 2.0
    out = np.zeros_like(a, dtype=np.float64)
    out[a <= f1] = 1.0
    band = (a > f1) & (a <= f2)
    out[band] = 0.5 * (1.0 + np.cos(math.pi / rolloff * (a[band] - f1)))
    return out


def rrc_response(n: int, sps: int = SPS, rolloff: float = ROLLOFF) -> np.ndarray:
    """Root-raised-cosine frequency response sqrt(sps * RC(f)) on the length-n DFT grid.

    The factor sps makes transmit RRC times receive RRC a Nyquist pulse with unit
    gain at the symbol instants of a zero-inserted symbol stream.
    """
    f_norm = np.fft.fftfreq(n, d=1.0) * sps   # frequency in units of the symbol rate
    return np.sqrt(sps * raised_cosine(f_norm, rolloff))


def shape(symbols: np.ndarray, sps: int = SPS, rolloff: float = ROLLOFF) -> np.ndarray:
    """Zero-insert to sps samples/symbol and apply RRC circularly in frequency. [..., n_sym*sps]."""
    n_sym = symbols.shape[-1]
    up = np.zeros(symbols.shape[:-1] + (n_sym * sps,), dtype=np.complex128)
    up[..., ::sps] = symbols
    return np.fft.ifft(np.fft.fft(up, axis=-1) * rrc_response(n_sym * sps, sps, rolloff), axis=-1)


def shape_at_rate(symbols: np.ndarray, fs_thz: float, rolloff: float = ROLLOFF,
                  symbol_rate_thz: float = SYMBOL_RATE_THZ) -> np.ndarray:
    """The same RRC pulse train sampled at any rate fs_thz above its bandwidth (e.g. a
    50 GSa/s scope, about 1.8 samples per symbol): the periodic band-limited signal whose
    spectrum on the n-point grid (n = n_sym fs / R, an integer) is the symbols' n_sym-point
    DFT, repeated with period R, times the RRC response, scaled so that every rate samples
    the same continuous signal; at fs = 2R it equals shape()."""
    n_sym = symbols.shape[-1]
    n_f = n_sym * fs_thz / symbol_rate_thz
    n = int(round(n_f))
    assert abs(n - n_f) < 1e-9, "n_sym * fs / R must be an integer"
    assert (1.0 + rolloff) * symbol_rate_thz / 2.0 < fs_thz / 2.0, "rate below the signal bandwidth"
    k = np.fft.fftfreq(n, d=1.0 / n).round().astype(np.int64)    # signed bin index
    S = np.fft.fft(symbols, axis=-1)
    f_norm = k / n_sym                                             # frequency in units of R
    # the DFT of samples of one continuous signal scales with the sampling rate
    X = S[..., k % n_sym] * np.sqrt(2.0 * raised_cosine(f_norm, rolloff)) * (fs_thz / (2.0 * symbol_rate_thz))
    return np.ascontiguousarray(np.fft.ifft(X, axis=-1))


def transmitted_field_at_rate(cfg: int, idx: int, n_pol: int, n_sym: int, p_dbm: float, fs_thz: float,
                              rolloff: float = ROLLOFF):
    """transmitted_field() sampled at fs_thz instead of two samples per symbol."""
    sym = qpsk_symbols(rng(cfg, idx, 0), n_pol, n_sym)
    return set_power(shape_at_rate(sym, fs_thz, rolloff), dbm_to_w(p_dbm)), sym


def polarization_rotation(gen: np.random.Generator) -> np.ndarray:
    """A random constant SU(2) matrix [[a, b], [-conj(b), conj(a)]], |a|^2 + |b|^2 = 1:
    the lossless polarization state change a fibre leaves between transmitter and receiver."""
    v = gen.standard_normal(4)
    v /= np.linalg.norm(v)
    a, b = v[0] + 1j * v[1], v[2] + 1j * v[3]
    return np.array([[a, b], [-np.conj(b), np.conj(a)]])


def laser_phase_noise(gen: np.random.Generator, n: int, linewidth_hz: float, fs_thz: float) -> np.ndarray:
    """Wiener phase of the transmitter and local-oscillator lasers (summed linewidth, Hz),
    one sample per field sample: increments of variance 2 pi linewidth / fs."""
    var = 2.0 * math.pi * linewidth_hz / (fs_thz * 1e12)
    return np.cumsum(gen.standard_normal(n) * math.sqrt(var))


def set_power(field: np.ndarray, p_w: float) -> np.ndarray:
    """Scale each polarization so its empirical mean |x|^2 is p_w / n_pol (total power p_w)."""
    n_pol = field.shape[-2]
    pw = np.mean(np.abs(field) ** 2, axis=-1, keepdims=True)
    return field * np.sqrt((p_w / n_pol) / pw)


def awgn_sigma2(p_w: float, osnr_db: float, fs_thz: float = FS_THZ,
                ref_bw_thz: float = OSNR_REF_BW_THZ) -> float:
    """Noise variance per complex sample per polarization for a given OSNR.

    OSNR = P / (ASE power in both polarizations in ref_bw); the ASE spectral density
    per polarization is white over the sampled band fs, so
    sigma^2 = P * fs / (2 * ref_bw * OSNR_lin).
    """
    return p_w * fs_thz / (2.0 * ref_bw_thz * 10.0 ** (osnr_db / 10.0))


def add_awgn(gen: np.random.Generator, field: np.ndarray, sigma2: float) -> np.ndarray:
    s = math.sqrt(sigma2 / 2.0)
    noise = gen.standard_normal(field.shape) * s + 1j * gen.standard_normal(field.shape) * s
    return field + noise


def transmitted_field(cfg: int, idx: int, n_pol: int, n_samples: int, p_dbm: float,
                      sps: int = SPS, rolloff: float = ROLLOFF):
    """The launched field and its symbols: (field [n_pol, n_samples] complex128, symbols)."""
    assert n_samples % sps == 0
    sym = qpsk_symbols(rng(cfg, idx, 0), n_pol, n_samples // sps)
    return set_power(shape(sym, sps, rolloff), dbm_to_w(p_dbm)), sym


def matched_filter_symbols(r: np.ndarray, sps: int = SPS, rolloff: float = ROLLOFF) -> np.ndarray:
    """Receive RRC (circular, in frequency) followed by sampling at the symbol instants."""
    n = r.shape[-1]
    y = np.fft.ifft(np.fft.fft(r, axis=-1) * rrc_response(n, sps, rolloff), axis=-1)
    return y[..., ::sps]


def evm(r_sym: np.ndarray, s: np.ndarray) -> float:
    """Data-aided EVM: per-polarization least-squares complex gain, pooled over polarizations.

    r_sym, s: [..., n_pol, n_sym].  Returns sqrt(sum|a r - s|^2 / sum|s|^2) (linear).
    """
    num = 0.0
    den = 0.0
    r2 = r_sym.reshape(-1, r_sym.shape[-1])
    s2 = s.reshape(-1, s.shape[-1])
    for rp, sp in zip(r2, s2):
        a = np.vdot(rp, sp) / np.vdot(rp, rp)
        num += float(np.sum(np.abs(a * rp - sp) ** 2))
        den += float(np.sum(np.abs(sp) ** 2))
    return math.sqrt(num / den)


def evm_db(r: np.ndarray, s: np.ndarray, sps: int = SPS, rolloff: float = ROLLOFF) -> float:
    """EVM in dB (20 log10) of a received field r against transmitted symbols s."""
    return 20.0 * math.log10(evm(matched_filter_symbols(r, sps, rolloff), s))


def ragged_lengths(gen: np.random.Generator, n: int, lo_exp: float = 12.0, hi_exp: float = 17.0,
                   multiple: int = SPS) -> np.ndarray:
    """Log-uniform lengths on [2^lo, 2^hi], rounded to a multiple of `multiple`."""
    u = gen.uniform(lo_exp, hi_exp, size=n)
    return (np.round(2.0 ** u / multiple) * multiple).astype(np.int64)


def symmetric_taps(gen: np.random.Generator, n_c: int) -> np.ndarray:
    """A seeded symmetric, positive, unit-sum tap vector of length 2*n_c+1 (centre largest)."""
    half = np.sort(gen.uniform(0.2, 1.0, size=n_c + 1))[::-1]
    half[0] = max(half[0], 1.0)
    full = np.concatenate([half[:0:-1], half])
    return full / full.sum()


def ragged_workload(n_signals: int = 512, seed: int = 0, lo_exp: float = 12.0, hi_exp: float = 17.0,
                    spans=(10, 40), essfm_nc=(2, 6), ssfm_steps=(4, 20)):
    """The ragged-batch workload: per signal a dict with its length (log-uniform on
    [2^lo, 2^hi], even), span count (uniform), and method: the even-indexed half
    ESSFM at one step per span with Nc uniform in essfm_nc (seeded symmetric,
    unit-sum taps), the odd-indexed half SSFM with steps per span uniform in
    ssfm_steps."""
    g = rng(2, seed, 0)
    lengths = ragged_lengths(g, n_signals, lo_exp, hi_exp)
    out = []
    for i in range(n_signals):
        gi = rng(2, seed, 1 + i)
        n_spans = int(gi.integers(spans[0], spans[1] + 1))
        if i % 2 == 0:
            nc = int(gi.integers(essfm_nc[0], essfm_nc[1] + 1))
            out.append(dict(n=int(lengths[i]), n_spans=n_spans, steps_per_span=1,
                            taps=symmetric_taps(gi, nc)))
        else:
            out.append(dict(n=int(lengths[i]), n_spans=n_spans,
                            steps_per_span=int(gi.integers(ssfm_steps[0], ssfm_steps[1] + 1)), taps=None))
    return out
