"""GPU receiver mode (an unbounded stream pushed in chunks) against the oracle's streaming
cascade, and against the circular GPU path on the stream surrounded by silence.

The receiver's output trails its input by the latency D: push i returns the output samples
[i C - D, (i + 1) C - D), zeros before n = 0.  FP32 budget as for the circular path:
relative L2 <= 1e-5 against the FP64 oracle for up to 40 steps.
"""
import numpy as np
import pytest

import siggen
from oracle import dbp_ref as R

from gpu_inputs import B2, FS, received, field_err, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TAPS9 = siggen.symmetric_taps(siggen.rng(8, 0, 1), 4)


@pytest.fixture(scope="module")
def dbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1507_00921_amd as m
    m.lib()
    return m


def _stream(dbp, rx, x, chunk):
    outs = []
    for i in range(x.shape[-1] // chunk):
        c = torch.from_numpy(np.ascontiguousarray(x[:, i * chunk:(i + 1) * chunk].astype(np.complex64))).cuda()
        outs.append(rx.push(c).cpu().numpy())
    return np.concatenate(outs, axis=-1)


@pytest.mark.parametrize("nb,o,k,n_pol,taps,n_spans,chunk,n_chunks", [
    (1024, 256, 5, 2, True, 10, 3072, 12),     # headline geometry: 2 passes, latency 1536
    (512, 128, 1, 1, False, 6, 1536, 10),      # SSFM, one polarization, 6 passes
    (256, 192, 1, 2, True, 3, 256, 24),        # halo wider than the valid part: 2 blocks per pass
    (2048, 512, 2, 2, False, 4, 3072, 8),
])
def test_receiver_matches_oracle_stream(dbp, nb, o, k, n_pol, taps, n_spans, chunk, n_chunks):
    n = chunk * n_chunks
    x, _ = received(8, nb + k, n_pol, n, 2.0, n_spans, 2)
    tp = TAPS9 if taps else None
    rx = dbp.receiver(chunk, n_spans, 1, n_pol=n_pol, taps=tp, block=nb, overlap=o, steps_per_pass=k,
                      beta2_ps2_km=B2)
    v, h = nb - o, o // 2
    d = rx.n_passes * (-(-h // v)) * v
    assert (rx.block, rx.overlap, rx.steps_per_pass, rx.latency) == (nb, o, k, d)
    y = _stream(dbp, rx, x, chunk)
    assert not np.any(y[:, :d])                               # before n = 0
    t64 = None if tp is None else np.asarray(tp, np.float32).astype(np.float64)
    steps = R.schedule(n_spans, 80.0, 1, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM, taps=t64)
    ref = R.run_streaming(x, steps, FS, nb, o, k)
    assert ref.shape[-1] == n - d
    err = field_err(y[:, d:].astype(np.complex128), ref)
    print(f"Nb={nb} O={o} k={k} passes={rx.n_passes} latency={d}: rel L2 vs oracle {err:.3e}")
    assert err <= 1e-5


def test_receiver_equals_circular_path_on_stream_with_silence(dbp):
    # the same blocks and arithmetic as dbp_backprop on the stream preceded and followed by
    # silence (a whole number of blocks): bit for bit
    nb, o, k, n_spans, chunk = 1024, 256, 5, 15, 3072
    n = chunk * 10
    x, _ = received(8, 1, 2, n, 3.0, n_spans, 2)
    rx = dbp.receiver(chunk, n_spans, 1, taps=TAPS9, block=nb, overlap=o, steps_per_pass=k, beta2_ps2_km=B2)
    y = _stream(dbp, rx, x, chunk)
    z = 16 * (nb - o)
    padded = np.concatenate([np.zeros((2, z)), x, np.zeros((2, z))], axis=-1).astype(np.complex64)
    p = dbp.plan(padded.shape[-1], n_spans, 1, taps=TAPS9, block=nb, overlap=o, steps_per_pass=k, beta2_ps2_km=B2)
    assert p.kernel.startswith("dbp_pass_kernel<1024, 4, 2, true, 9>")
    c = p.backprop(torch.from_numpy(padded).reshape(1, 2, -1).cuda()).cpu().numpy().reshape(2, -1)
    d = rx.latency
    assert np.array_equal(y[:, d:].view(np.uint32), c[:, z:z + n - d].view(np.uint32))


def test_receiver_chunk_size_and_reset(dbp):
    # the output stream does not depend on the chunk length; reset starts over
    nb, o, k, n_spans = 512, 128, 2, 6
    n = 384 * 48
    x, _ = received(8, 2, 2, n, 2.0, n_spans, 2)
    kw = dict(taps=TAPS9, block=nb, overlap=o, steps_per_pass=k, beta2_ps2_km=B2)
    a = dbp.receiver(768, n_spans, 1, **kw)
    b = dbp.receiver(384 * 12, n_spans, 1, **kw)
    ya = _stream(dbp, a, x, 768)
    yb = _stream(dbp, b, x, 384 * 12)
    assert a.latency == b.latency
    assert np.array_equal(ya.view(np.uint32), yb.view(np.uint32))
    a.reset()
    ya2 = _stream(dbp, a, x, 768)
    assert np.array_equal(ya.view(np.uint32), ya2.view(np.uint32))


def test_receiver_argument_rules(dbp):
    kw = dict(block=1024, overlap=256, beta2_ps2_km=B2)
    for chunk in (1000, 768):            # not a multiple of V; shorter than a block
        with pytest.raises(dbp.DbpError) as e:
            dbp.receiver(chunk, 4, 1, **kw)
        assert e.value.status == 1
    with pytest.raises(dbp.DbpError) as e:
        dbp.receiver(3072, 4, 1, precision=dbp.BF16X3, **kw)
    assert e.value.status == 2
