"""The allocation-free entry point dbp_backprop_noalloc against dbp_backprop (needs an MI355X).

Both run the same passes with the same kernels; only the workspace differs (the
library's fixed device scratch against a caller-allocated one), so the outputs
must agree bit for bit.  Two calls in a row, the second on a smaller input with
another geometry, check that nothing left in the shared scratch leaks into the
next result; a plan whose workspace exceeds the scratch is refused.
"""
import ctypes

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


def _field(rx, n_pol, n):
    a = np.ascontiguousarray(rx.astype(np.complex64))
    return torch.from_numpy(a).reshape(1, n_pol, n).to("cuda")


def _noalloc(dbp, p, x, out):
    """dbp_backprop_noalloc through the C ABI on the current stream."""
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return dbp.lib().dbp_backprop_noalloc(p._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                          None, None, stream)


def _reference(p, x):
    return p.backprop(x, out=torch.empty_like(x), workspace=p.workspace())


def test_noalloc_matches_backprop_on_two_calls(dbp):
    # first call: the headline geometry (ESSFM, Nb 1024, O 256, 8 passes of 5 steps)
    n1 = 2 * 65536 + 1002
    rx1, _ = received(1, 1024, 2, n1, 2.0, 40, 2)
    p1 = dbp.plan(n1, 40, 1, taps=TAPS9, block=1024, overlap=256, beta2_ps2_km=B2)
    assert p1.workspace_size() <= dbp.NOALLOC_SCRATCH_BYTES
    x1 = _field(rx1, 2, n1)
    want1 = _reference(p1, x1)
    got1 = torch.full_like(x1, complex(np.nan, np.nan))
    assert _noalloc(dbp, p1, x1, got1) == 0
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(got1), torch.view_as_real(want1))

    # second call, smaller input, another geometry (SSFM, one polarization, 512-point blocks)
    n2 = 7777 * 2
    rx2, _ = received(1, 512, 1, n2, 2.0, 4, 2)
    p2 = dbp.plan(n2, 4, 3, n_pol=1, block=512, overlap=128, steps_per_pass=3, beta2_ps2_km=B2)
    x2 = _field(rx2, 1, n2)
    want2 = _reference(p2, x2)
    got2 = torch.full_like(x2, complex(np.nan, np.nan))
    assert _noalloc(dbp, p2, x2, got2) == 0
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(got2), torch.view_as_real(want2))
    print(f"no-alloc: 2x{n1} ({p1.n_passes} passes) then 1x{n2} ({p2.n_passes} passes) bit for bit")
    p1.close()
    p2.close()


def test_noalloc_in_place_and_single_pass(dbp):
    n = 40000
    rx, _ = received(1, 2048, 2, n, 2.0, 10, 2)
    for kw in [dict(block=2048, overlap=512, steps_per_pass=2),          # 5 passes
               dict(block=2048, overlap=512, steps_per_pass=10)]:        # one pass (copies back)
        p = dbp.plan(n, 10, 1, taps=TAPS9, beta2_ps2_km=B2, **kw)
        x = _field(rx, 2, n)
        want = _reference(p, x)
        y = x.clone()
        assert _noalloc(dbp, p, y, y) == 0
        torch.cuda.synchronize()
        assert torch.equal(torch.view_as_real(y), torch.view_as_real(want)), kw
        p.close()


def test_noalloc_refuses_plans_beyond_the_scratch(dbp):
    # two states of 2 x 1200000 complex64 (19.2 MB each) exceed the 32 MiB scratch
    n = 1200000
    p = dbp.plan(n, 4, 1, block=1024, overlap=256, steps_per_pass=1, beta2_ps2_km=B2)
    assert p.workspace_size() > dbp.NOALLOC_SCRATCH_BYTES
    x = torch.zeros(1, 2, n, dtype=torch.complex64, device="cuda")
    out = torch.empty_like(x)
    assert _noalloc(dbp, p, x, out) == 3            # DBP_ERR_WORKSPACE
    with pytest.raises(dbp.DbpError):
        p.backprop_noalloc(x, out)
    p.close()
