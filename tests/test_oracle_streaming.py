"""Pins of the oracle's receiver mode (non-circular overlap-and-save stream), CPU only."""
import numpy as np
import pytest

import siggen
from oracle import dbp_ref as R

B2 = siggen.beta2_ps2_km()
FS = siggen.FS_THZ


def _setup(n=6144, n_spans=4, essfm=True):
    x, _ = siggen.transmitted_field(6, 0, 2, n, 3.0)
    taps = siggen.symmetric_taps(siggen.rng(6, 0, 1), 2) if essfm else None
    steps = R.schedule(n_spans, 80.0, 1, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM, taps=taps)
    return x, steps


@pytest.mark.parametrize("nb,o,k", [(512, 128, 1), (512, 128, 2), (256, 96, 3)])
def test_stream_is_the_circular_cascade_after_silence(nb, o, k):
    # the receiver mode is the circular cascade of the same samples preceded and followed by
    # enough silence (a whole number of blocks): equal bit for bit
    x, steps = _setup()
    v = nb - o
    y = R.run_streaming(x, steps, FS, nb, o, k)
    z = 16 * v
    padded = np.concatenate([np.zeros((2, z)), x, np.zeros((2, z))], axis=-1)
    ref = R.run_blocked(padded, steps, FS, nb, o, k)[:, z:z + y.shape[-1]]
    assert np.array_equal(y, ref)


@pytest.mark.parametrize("nb,o,k", [(512, 128, 1), (1024, 256, 2)])
def test_stream_interior_equals_circular_cascade(nb, o, k):
    x, steps = _setup(n=12288, essfm=False)
    y = R.run_streaming(x, steps, FS, nb, o, k)
    c = R.run_blocked(x, steps, FS, nb, o, k)
    reach = R.passes(len(steps), k) * nb
    assert np.array_equal(y[:, reach:y.shape[-1] - reach], c[:, reach:y.shape[-1] - reach])


@pytest.mark.parametrize("nb,o,k,n_steps", [(512, 128, 1, 4), (1024, 256, 5, 40), (256, 192, 1, 3)])
def test_stream_output_length_is_input_minus_latency(nb, o, k, n_steps):
    v = nb - o
    x = np.zeros((1, 40 * v), dtype=np.complex128)
    steps = [R.Step(b=0.0, phi=0.0)] * n_steps
    y = R.run_streaming(x, steps, FS, nb, o, k)
    assert y.shape[-1] == x.shape[-1] - R.streaming_latency(n_steps, nb, o, k)
