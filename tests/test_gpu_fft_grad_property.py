"""Property-based parity of the FFT-step reverse mode (hypothesis, derandomized: every run draws
the same cases).  Each case draws a block size, overlap, steps per pass, length, polarizations,
tap count, launch power and batch size, then checks three properties:

* the gradients with the fields kept by the forward pass equal, bit for bit, those of the
  recompute mode (DBP_FLAG_GRAD_SPARSE), which re-runs every pass from its input;
* the saved forward (dbp_backprop_save) gives dbp_backprop's output bit for bit, and the
  reverse pass from it gives dbp_backprop_grad's gradients bit for bit;
* the input and tap gradients match the oracle's FP64 adjoint of the same blocked cascade
  (Sec. III blocks, Eqs. (1)-(3) steps) to the FP32 budget.
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import siggen
from gpu_inputs import B2, FS, field_err
from oracle import adjoint as A
from oracle import dbp_ref as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1507_00921_amd as m
    m.lib()
    return m


@st.composite
def cases(draw):
    nb = draw(st.sampled_from([256, 512, 1024, 2048, 4096]))
    o = 2 * draw(st.integers(1, nb // 4))                  # even, below Nb / 2
    spans = draw(st.integers(1, 5))
    k = draw(st.integers(1, spans))
    return dict(nb=nb, o=o, spans=spans, k=k, n=draw(st.integers(nb, 4 * nb)),
                n_pol=draw(st.sampled_from([1, 2])), nc=draw(st.sampled_from([None, 1, 3, 4])),
                p_dbm=draw(st.sampled_from([0.0, 4.0])), batch=draw(st.sampled_from([1, 1, 2])),
                seed=draw(st.integers(0, 10**6)))


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a.astype(dtype))).cuda()


@settings(max_examples=20, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.function_scoped_fixture, HealthCheck.too_slow])
@given(c=cases())
def test_reverse_mode_random_geometry(dbp, c):
    g = np.random.default_rng([95, c["seed"]])
    shape = (c["batch"], c["n_pol"], c["n"])
    amp = np.sqrt(siggen.dbm_to_w(c["p_dbm"]) / 2)
    x = ((g.standard_normal(shape) + 1j * g.standard_normal(shape)) * amp).astype(np.complex64)
    gout = (g.standard_normal(shape) + 1j * g.standard_normal(shape)).astype(np.complex64)
    taps = (None if c["nc"] is None else
            np.stack([siggen.symmetric_taps(siggen.rng(95, c["seed"], s), c["nc"]) for s in range(c["spans"])])
            .astype(np.float32))
    kw = dict(n_pol=c["n_pol"], batch=c["batch"], taps=None if taps is None else taps[0], block=c["nb"],
              overlap=c["o"], steps_per_pass=c["k"], beta2_ps2_km=B2)
    p = dbp.plan(c["n"], c["spans"], 1, **kw)
    q = dbp.plan(c["n"], c["spans"], 1, grad_sparse=True, **kw)
    assert (p.block, p.overlap, p.steps_per_pass) == (c["nb"], c["o"], c["k"])
    xd, gd = dev(x, np.complex64), dev(gout, np.complex64)
    td = None if taps is None else dev(taps, np.float32)
    gx, gt, _ = p.backprop_grad(xd, gd, taps=td)
    sx, st_, _ = q.backprop_grad(xd, gd, taps=td)
    out, ws = p.backprop_save(xd, taps=td)
    vx, vt, _ = p.backprop_grad_saved(xd, out, ws, gd, taps=td)
    ref_out = p.backprop(xd, taps=td)
    torch.cuda.synchronize()
    kept = p.workspace_size(grad=True) > q.workspace_size(grad=True)
    print(f"{c}: {p.kernel}, fields kept: {kept}")
    assert torch.equal(torch.view_as_real(gx), torch.view_as_real(sx))
    assert torch.equal(torch.view_as_real(vx), torch.view_as_real(gx))
    assert torch.equal(torch.view_as_real(out), torch.view_as_real(ref_out))
    if taps is None:
        assert gt is None and st_ is None and vt is None
    else:
        assert torch.equal(gt, st_) and torch.equal(vt, gt)
    base = R.schedule(c["spans"], 80.0, 1, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM)
    steps = [R.Step(b=s.b, phi=s.phi, w=None if taps is None else taps[i].astype(np.float64))
             for i, s in enumerate(base)]
    gx = gx.cpu().numpy().astype(np.complex128)
    wsum = 0
    for b in range(c["batch"]):
        ref = A.grad_blocked(x[b].astype(np.complex128), steps, FS, c["nb"], c["o"], c["k"],
                             gout[b].astype(np.complex128))
        assert field_err(gx[b], ref.x) <= 1e-5
        if taps is not None:
            wsum = wsum + np.stack(ref.w)
    if taps is not None:
        assert field_err(gt.cpu().numpy().astype(np.float64), wsum) <= 1e-4
    p.close()
    q.close()
