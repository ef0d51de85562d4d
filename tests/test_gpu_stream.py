"""GPU parity of the streaming pass kernel (resident grid, next block prefetched).

The streaming kernel runs the same per-block arithmetic as the one-workgroup-
per-block kernel, so on the same plan geometry its output must equal that
kernel's bit for bit, and the FP64 oracle (same geometry) to the FP32 budget.
DBP_STREAM=1 forces it on small launches and DBP_STREAM_GRID sets a small
resident grid, so that every workgroup walks several blocks, the XCD ranges are
uneven and the ragged last block and the circular halo at both signal ends are
covered.
"""
import numpy as np
import pytest

import siggen
from oracle import dbp_ref as R

from gpu_inputs import B2, FS, received, field_err, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TAPS9 = siggen.symmetric_taps(siggen.rng(1, 0, 7), 4)
TAPS7 = siggen.symmetric_taps(siggen.rng(1, 0, 8), 3)


@pytest.fixture(scope="module")
def dbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1507_00921_amd as m
    m.lib()
    return m


def _plans(dbp, monkeypatch, grid, force_e=None, **kw):
    # small SSFM launches would otherwise get the polarization-split kernel, which has no twin
    monkeypatch.setenv("DBP_FORCE_SPLIT", "0")
    if force_e:
        monkeypatch.setenv("DBP_FORCE_E", str(force_e))
    monkeypatch.setenv("DBP_STREAM", "0")
    ref = dbp.plan(**kw)
    monkeypatch.setenv("DBP_STREAM", "1")
    monkeypatch.setenv("DBP_STREAM_GRID", str(grid))
    st = dbp.plan(**kw)
    monkeypatch.delenv("DBP_STREAM")
    monkeypatch.delenv("DBP_STREAM_GRID")
    monkeypatch.delenv("DBP_FORCE_SPLIT")
    if force_e:
        monkeypatch.delenv("DBP_FORCE_E")
    assert ref.kernel.startswith("dbp_pass_kernel<"), ref.kernel
    assert st.kernel.startswith("dbp_stream_kernel<"), st.kernel
    assert (st.block, st.overlap, st.steps_per_pass) == (ref.block, ref.overlap, ref.steps_per_pass)
    return ref, st


@pytest.mark.parametrize("block,overlap,e,n_pol,taps,n_spans,sps,k,n,batch,grid", [
    (512, 128, 8, 2, "9", 6, 1, 1, 40000, 1, 16),           # ESSFM 9 taps, ragged tail
    (512, 128, 8, 1, None, 4, 3, 2, 20000, 3, 24),          # SSFM, one polarization, 3 signals, k = 2
    (512, 128, 8, 2, "7", 6, 1, 1, 30000, 2, 8),            # run-time tap count, 2 signals
    (256, 64, 4, 2, None, 3, 2, 2, 5000, 1, 8),
    (256, 64, 4, 2, "9", 4, 1, 1, 3000, 1, 8),
    (512, 128, 8, 2, "9", 3, 1, 1, 512, 1, 8),              # one block: its halo wraps around the signal
])
def test_stream_matches_block_kernel_and_oracle(dbp, monkeypatch, block, overlap, e, n_pol, taps, n_spans, sps,
                                                k, n, batch, grid):
    tp = {"9": TAPS9, "7": TAPS7, None: None}[taps]
    kw = dict(n_samples=n, n_spans=n_spans, steps_per_span=sps, n_pol=n_pol, batch=batch, taps=tp,
              block=block, overlap=overlap, steps_per_pass=k, beta2_ps2_km=B2)
    ref_plan, st_plan = _plans(dbp, monkeypatch, grid, force_e=e, **kw)
    fields = [received(7, block + i, n_pol, n, 2.0, n_spans, 2)[0] for i in range(batch)]
    x = torch.from_numpy(np.stack(fields).astype(np.complex64)).to("cuda")
    y_ref = ref_plan.backprop(x).cpu().numpy()
    y_st = st_plan.backprop(x).cpu().numpy()
    torch.cuda.synchronize()
    print(f"{st_plan.kernel} grid={grid} Nb={block} k={st_plan.steps_per_pass} batch={batch}")
    assert np.array_equal(y_st.view(np.uint32), y_ref.view(np.uint32)), "stream kernel differs bitwise"
    t64 = None if tp is None else np.asarray(tp, np.float32).astype(np.float64)
    steps = R.schedule(n_spans, 80.0, sps, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM, taps=t64)
    for i in range(batch):
        o = R.run_blocked(fields[i], steps, FS, st_plan.block, st_plan.overlap, st_plan.steps_per_pass)
        err = field_err(y_st[i].astype(np.complex128), o)
        print(f"  signal {i}: rel L2 vs oracle {err:.3e}")
        assert err <= 1e-5


def test_stream_kernel_on_request_for_large_working_set(dbp):
    # the headline field replicated 64 times (256 MiB per state) on 512-point blocks: the
    # planner's default is the per-block kernel, DBP_STREAM=1 selects the streaming twin, and
    # the twin's output equals the per-block kernel's bit for bit
    import os
    n, batch = 262144, 64
    kw = dict(n_samples=n, n_spans=40, steps_per_span=1, batch=batch, taps=TAPS9, block=512, overlap=128,
              steps_per_pass=1, beta2_ps2_km=B2)
    assert "DBP_STREAM" not in os.environ
    q = dbp.plan(**kw)
    assert q.kernel == "dbp_pass_kernel<512, 8, 2, true, 9>", q.kernel
    os.environ["DBP_STREAM"] = "1"
    try:
        p = dbp.plan(**kw)
    finally:
        del os.environ["DBP_STREAM"]
    assert p.kernel == "dbp_stream_kernel<512, 8, 2, true, 9>"
    rx, _ = received(1, 0, 2, n, 0.0, 40, 2)
    x = torch.from_numpy(rx.astype(np.complex64)).to("cuda").reshape(1, 2, n).expand(batch, 2, n).contiguous()
    # distinct signals: rotate each copy in time so no two are equal
    for b in range(batch):
        x[b] = torch.roll(x[b], shifts=97 * b, dims=-1)
    a = p.backprop(x)
    c = q.backprop(x)
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.float32), c.view(torch.float32))
    # and one sampled signal against the oracle
    b = 37
    steps = R.schedule(40, 80.0, 1, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM,
                       taps=np.asarray(TAPS9, np.float32).astype(np.float64))
    o = R.run_blocked(np.roll(rx, 97 * b, axis=-1), steps, FS, 512, 128, 1)
    err = field_err(a[b].cpu().numpy().astype(np.complex128), o)
    print(f"x64 field, signal {b}: rel L2 vs oracle {err:.3e}")
    assert err <= 1e-5
