"""Operation-count model of Sec. III (TEST INFRASTRUCTURE ONLY: see oracle/__init__).

Counting assumptions of the paper (Sec. III and its footnote): radix-2
Cooley-Tukey FFT of N complex samples costs about 8 N log2 N real
multiplications and as many additions for the four FFTs of one step (two
polarizations, forward and inverse); a complex multiplication costs 4 real
multiplications and 2 additions; fixed factors are precomputed and the complex
exponential is a table lookup.  Per block and step:
  linear substep, Eq. (1):              8N mult, 4N add
  squared moduli:                       4N mult, 3N add
  tap combination of Eq. (3):           N*Nc + N mult, 2 N*Nc add
  phase rotation:                       8N mult, 4N add
Of every block of N samples, M are discarded by overlap-and-save, so counts per
received sample are scaled by N / (N - M).  SSFM is ESSFM with Nc = 0; the
frequency-domain FFE for bulk dispersion is one step with the linear substep
only.
"""
from __future__ import annotations

import math


def essfm_mults_per_sample(n: float, m: float, n_c: int) -> float:
    """Real multiplications per received sample per step, ESSFM with Nc coefficients."""
    return n * (8.0 * math.log2(n) + 21.0 + n_c) / (n - m)


def essfm_adds_per_sample(n: float, m: float, n_c: int) -> float:
    """Real additions per received sample per step, ESSFM with Nc coefficients."""
    return n * (8.0 * math.log2(n) + 11.0 + 2.0 * n_c) / (n - m)


def ssfm_mults_per_sample(n: float, m: float) -> float:
    return essfm_mults_per_sample(n, m, 0)


def ssfm_adds_per_sample(n: float, m: float) -> float:
    return essfm_adds_per_sample(n, m, 0)


def ffe_mults_per_sample(n: float, m: float) -> float:
    """Frequency-domain feed-forward equalizer (one linear-only step)."""
    return n * (8.0 * math.log2(n) + 8.0) / (n - m)


def ffe_adds_per_sample(n: float, m: float) -> float:
    return n * (8.0 * math.log2(n) + 4.0) / (n - m)


def channel_memory(beta2_ps2_km: float, length_km: float, bandwidth_thz: float) -> float:
    """M ~ 2 pi |beta2| L B^2 samples (Sec. III)."""
    return 2.0 * math.pi * abs(beta2_ps2_km) * length_km * bandwidth_thz ** 2


def total_mults(n_steps: int, n: float, m: float, n_c: int = 0) -> float:
    """Whole-DBP multiplications per received sample for N_s steps (per-step count x N_s)."""
    return n_steps * essfm_mults_per_sample(n, m, n_c)


def per_step_flops(n: float, m: float, n_c: int) -> float:
    """Multiplications plus additions per received sample per step."""
    return essfm_mults_per_sample(n, m, n_c) + essfm_adds_per_sample(n, m, n_c)
