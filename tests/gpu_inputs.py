"""Seeded workload inputs for the GPU parity tests, built on the CPU from siggen and the
oracle's forward channel (never from the GPU path)."""
import functools

import numpy as np

import siggen
from oracle import dbp_ref as R

B2 = siggen.beta2_ps2_km()
FS = siggen.FS_THZ


@functools.lru_cache(maxsize=16)
def received(cfg: int, idx: int, n_pol: int, n: int, p_dbm: float, n_spans: int,
             fwd_steps_per_span: int, osnr_db: float = 20.0):
    """Launched PM-QPSK field propagated forward by the oracle, plus ASE noise.

    Returns (rx as complex64-rounded complex128 [n_pol, n], symbols).  Noise power is
    fixed at the OSNR referenced to 0 dBm launch (ASE-limited link).
    """
    x, sym = siggen.transmitted_field(cfg, idx, n_pol, n, p_dbm)
    steps = R.schedule(n_spans, 80.0, fwd_steps_per_span, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM,
                       backward=False)
    rx = R.run_whole(x, steps, FS)
    rx = siggen.add_awgn(siggen.rng(cfg, idx, 2), rx, siggen.awgn_sigma2(siggen.dbm_to_w(0.0), osnr_db))
    return rx.astype(np.complex64).astype(np.complex128), sym


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
