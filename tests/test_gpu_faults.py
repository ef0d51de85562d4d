"""Allocation failures forced from the host (DBP_FAULT_INJECT) on every object that allocates
device memory (needs an MI355X).

DBP_FAULT_INJECT="<tag>:<n>" makes the library's n-th device allocation since the tag changed
fail as out of memory.  For n = 1, 2, ... the creation must fail with a status (never crash)
until n passes the number of allocations the object makes; then it succeeds.  The device's
free memory afterwards equals its free memory before (what a failed creation had allocated
was released), and the object made last works.
"""
import numpy as np
import pytest

import siggen

from gpu_inputs import B2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MIB = 1 << 20


@pytest.fixture(scope="module")
def dbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1507_00921_amd as m
    m.lib()
    return m


TAPS9 = siggen.symmetric_taps(siggen.rng(1, 0, 7), 4)


def _makers(dbp):
    work = siggen.ragged_workload(6, seed=4, lo_exp=12.0, hi_exp=13.0, spans=(2, 4), essfm_nc=(2, 4),
                                  ssfm_steps=(2, 4))
    descs = [dbp.make_desc(w["n"], w["n_spans"], w["steps_per_span"], taps=w["taps"], beta2_ps2_km=B2)
             for w in work]
    return {
        "plan": lambda: dbp.plan(262144, 40, 1, taps=TAPS9, block=1024, overlap=256, beta2_ps2_km=B2),
        "plan_tuned": lambda: dbp.plan(1 << 20, 8, 1, taps=TAPS9, beta2_ps2_km=B2, tune=True),
        "plan_fir": lambda: dbp.plan(4096, 8, 1, taps=TAPS9, linear=dbp.LINEAR_FIR, n_fir=33, fir_band_thz=0.0154,
                                     beta2_ps2_km=B2),
        "batch": lambda: dbp.plan_batch(descs),
        "receiver": lambda: dbp.receiver(64 * 768, 40, 1, taps=TAPS9, block=1024, overlap=256, beta2_ps2_km=B2),
        "dsp": lambda: dbp.receiver_dsp(234050),
        "mse": lambda: dbp.SymbolMse(32768, 2, 64, siggen.rrc_response(32768), 1.0),
    }


@pytest.mark.parametrize("what", ["plan", "plan_tuned", "plan_fir", "batch", "receiver", "dsp", "mse"])
def test_allocation_failures_are_reported_and_released(dbp, monkeypatch, what):
    make = _makers(dbp)[what]
    make().close()                   # first use: runtime and autotuner state, outside the count
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    failures = 0
    obj = None
    for n in range(1, 400):
        monkeypatch.setenv("DBP_FAULT_INJECT", f"{what}-{n}:{n}")
        try:
            obj = make()
        except dbp.DbpError as e:
            assert e.status in (4, 5), e          # out of memory (or the tuner's HIP error)
            failures += 1
            continue
        break
    monkeypatch.delenv("DBP_FAULT_INJECT")
    assert obj is not None and failures >= 1
    obj.close()
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    print(f"{what}: {failures} injected failures, free memory {free0 / MIB:.1f} -> {free1 / MIB:.1f} MiB")
    assert abs(free1 - free0) <= 4 * MIB
    # the library still works after the failures
    obj = make()
    if what in ("plan", "plan_fir"):
        n = 262144 if what == "plan" else 4096
        x = torch.zeros(1, 2, n, dtype=torch.complex64, device="cuda")
        y = obj.backprop(x)
        torch.cuda.synchronize()
        assert torch.count_nonzero(y).item() == 0
    obj.close()
