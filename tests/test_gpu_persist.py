"""The persistent pass loop (DBP_FLAG_PERSISTENT) against the per-pass launches (needs an MI355X).

Both run every block through the same step code on the same inputs, the persistent kernel
only exchanging halo samples bit for bit through memory instead of writing and re-reading
the whole state between passes, so the outputs must be equal bit for bit; the per-pass
path is itself checked against the oracle in test_gpu_parity.py.  Cases: the headline
field (342 blocks, last block partial, halos that wrap around the signal), one polarization,
SSFM with many passes, a batch of signals, repeated calls, and the fallbacks.
"""
import numpy as np
import pytest

import siggen

from gpu_inputs import B2, received

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1507_00921_amd as m
    m.lib()
    return m


TAPS9 = siggen.symmetric_taps(siggen.rng(1, 0, 7), 4)


def _field(x, batch=1):
    a = np.ascontiguousarray(x.astype(np.complex64))
    return torch.from_numpy(a).reshape(batch, *x.shape[-2:]).to("cuda")


@pytest.mark.parametrize("n,n_pol,n_spans,sps,taps,batch", [
    (262144, 2, 40, 1, TAPS9, 1),          # the headline: 342 blocks, 8 passes of 5 steps
    (65536 + 1002, 2, 12, 1, TAPS9, 1),    # ragged tail
    (40000, 1, 10, 1, TAPS9, 1),           # one polarization
    (50000, 2, 8, 20, None, 1),            # SSFM, k = 115 steps per pass, 2 passes
    (30000, 2, 6, 1, TAPS9, 3),            # a batch of three signals (6 steps, 2 passes)
])
def test_persistent_equals_per_pass_launches(dbp, monkeypatch, n, n_pol, n_spans, sps, taps, batch):
    xs = np.stack([received(1, 70 + i, n_pol, n, 2.0, n_spans, 2)[0] for i in range(batch)])
    x = _field(xs, batch)
    kw = dict(n_pol=n_pol, batch=batch, taps=taps, block=1024, overlap=256, beta2_ps2_km=B2)
    # the persistent loop runs whole blocks per workgroup: compare with the plain per-block
    # kernel (small SSFM launches otherwise take the polarization-split one)
    monkeypatch.setenv("DBP_FORCE_SPLIT", "0")
    p0 = dbp.plan(n, n_spans, sps, **kw)
    monkeypatch.delenv("DBP_FORCE_SPLIT")
    p1 = dbp.plan(n, n_spans, sps, persistent=True, **kw)
    assert "persist" in p1.kernel and "persist" not in p0.kernel, (p0.kernel, p1.kernel)
    want = p0.backprop(x)
    got = [p1.backprop(x) for _ in range(3)]        # repeated calls: fresh flags each time
    torch.cuda.synchronize()
    assert p1.persistent_status() == 0
    for g in got:
        assert torch.equal(torch.view_as_real(g), torch.view_as_real(want))
    print(f"persistent {batch}x{n_pol}x{n}: {p1.n_passes} passes, {p1.kernel}: bit for bit")
    p0.close()
    p1.close()


def test_persistent_fallbacks(dbp):
    n = 40000
    x = _field(received(1, 80, 2, n, 2.0, 10, 2)[0])
    p0 = dbp.plan(n, 10, 1, taps=TAPS9, block=1024, overlap=256, beta2_ps2_km=B2)
    p1 = dbp.plan(n, 10, 1, taps=TAPS9, block=1024, overlap=256, beta2_ps2_km=B2, persistent=True)
    want = p0.backprop(x)
    y = x.clone()
    p1.backprop(y, out=y)                               # in place: the per-pass launches
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(y), torch.view_as_real(want))
    # a single pass, a block size without a persistent variant: the plan keeps its launches
    p2 = dbp.plan(n, 10, 1, taps=TAPS9, block=1024, overlap=256, steps_per_pass=10, beta2_ps2_km=B2,
                  persistent=True)
    p3 = dbp.plan(n, 10, 1, taps=TAPS9, block=512, overlap=128, beta2_ps2_km=B2, persistent=True)
    assert "persist" not in p2.kernel and "persist" not in p3.kernel
    for p in (p0, p1, p2, p3):
        p.close()
