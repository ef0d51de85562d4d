"""GPU parity of the reverse mode of the overlap-and-save FFT cascade (dbp_backprop_grad on
FFT-step plans) against the oracle's FP64 adjoint of the same blocked cascade.

Both sides take the same complex64-rounded input, the same FP32-rounded taps and the same
seeded upstream gradient; the oracle differentiates exactly the blocked function the GPU
computes (same Nb, O, k).  Tolerances: input gradient relative L2 <= 1e-5 up to 40 steps
(the FP32 budget of the forward path), tap gradients relative L2 <= 1e-4 (sums of
products over every sample, reduced in FP64 on the GPU).
"""
import numpy as np
import pytest

import siggen
from oracle import adjoint as A
from oracle import dbp_ref as R

from gpu_inputs import B2, FS, received, field_err, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1507_00921_amd as m
    m.lib()
    return m


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a.astype(dtype))).cuda()


def case(seed, batch, n_pol, n, n_spans, nc):
    xs = np.stack([received(4, seed * 10 + i, n_pol, n, 3.0, n_spans, 1)[0] for i in range(batch)])
    taps = (np.stack([siggen.symmetric_taps(siggen.rng(4, seed, s), nc) for s in range(n_spans)])
            .astype(np.float32) if nc is not None else None)
    g = np.random.default_rng([4, seed, 99])
    gout = (g.standard_normal(xs.shape) + 1j * g.standard_normal(xs.shape)).astype(np.complex64)
    return xs, taps, gout


@pytest.mark.parametrize("nb,o,k,n_pol,nc,n_spans,n,batch", [
    (1024, 256, 5, 2, 4, 10, 8000, 1),      # headline geometry, 2 passes of 5 steps, ragged tail
    (512, 128, 1, 1, None, 6, 3000, 2),     # SSFM, one polarization, two signals, 6 passes
    (256, 64, 2, 2, 3, 5, 2000, 1),         # 7 taps (run-time tap count), odd pass count
    (2048, 512, 3, 2, 4, 6, 9000, 1),
    (4096, 1024, 2, 2, None, 4, 10000, 1),
    (4096, 1024, 2, 2, 4, 4, 10000, 1),     # the largest adjoint blocks with 9 taps
    (512, 128, 2, 1, 4, 4, 3000, 1),        # ESSFM on one polarization
    (1024, 256, 3, 2, 4, 3, 1024, 1),       # one block: its window wraps around the signal
])
def test_fft_grad_matches_oracle(dbp, nb, o, k, n_pol, nc, n_spans, n, batch):
    xs, taps, gout = case(nb + k, batch, n_pol, n, n_spans, nc)
    kw = dict(batch=batch, n_pol=n_pol, taps=None if taps is None else taps[0], block=nb, overlap=o,
              steps_per_pass=k, beta2_ps2_km=B2)
    p = dbp.plan(n, n_spans, 1, **kw)
    assert (p.block, p.overlap, p.steps_per_pass) == (nb, o, k)
    t_dev = None if taps is None else dev(taps, np.float32)
    gx, gt, gf = p.backprop_grad(dev(xs, np.complex64), dev(gout, np.complex64), taps=t_dev)
    assert gf is None
    # the same gradients, bit for bit, when every reverse pass recomputes its steps from the
    # pass input instead of reading the fields the forward pass kept (the same arithmetic)
    q = dbp.plan(n, n_spans, 1, grad_sparse=True, **kw)
    sx, st_, _ = q.backprop_grad(dev(xs, np.complex64), dev(gout, np.complex64), taps=t_dev)
    kept = p.workspace_size(grad=True) > q.workspace_size(grad=True)
    print(f"Nb={nb} O={o} k={k} pol={n_pol}: kernel {p.kernel}, fields kept by the forward pass: {kept}")
    assert torch.equal(torch.view_as_real(gx), torch.view_as_real(sx))
    assert (gt is None and st_ is None) or torch.equal(gt, st_)
    gx = gx.cpu().numpy().astype(np.complex128)
    base = R.schedule(n_spans, 80.0, 1, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM)
    steps = [R.Step(b=st.b, phi=st.phi, w=None if taps is None else taps[s].astype(np.float64))
             for s, st in enumerate(base)]
    wsum = np.zeros((n_spans, 2 * nc + 1)) if taps is not None else None
    for i in range(batch):
        ref = A.grad_blocked(xs[i], steps, FS, nb, o, k, gout[i].astype(np.complex128))
        err = field_err(gx[i], ref.x)
        print(f"Nb={nb} O={o} k={k} pol={n_pol} signal {i}: grad_in rel L2 {err:.3e}")
        assert err <= 1e-5
        if taps is not None:
            wsum += np.stack(ref.w)
    if taps is not None:
        got = gt.cpu().numpy().astype(np.float64)
        err = field_err(got, wsum)
        print(f"  grad_taps rel L2 {err:.3e}")
        assert err <= 1e-4
    else:
        assert gt is None


def test_fft_grad_is_deterministic_and_matches_autograd(dbp):
    # two runs are bitwise equal, and the autograd Function returns the same gradients
    n, n_spans = 6000, 5
    xs, taps, gout = case(7, 2, 2, n, n_spans, 4)
    p = dbp.plan(n, n_spans, 1, batch=2, taps=taps[0], block=1024, overlap=256, steps_per_pass=2,
                 beta2_ps2_km=B2)
    x = dev(xs, np.complex64)
    t = dev(taps, np.float32)
    g = dev(gout, np.complex64)
    a = p.backprop_grad(x, g, taps=t)
    b = p.backprop_grad(x, g, taps=t)
    torch.cuda.synchronize()
    assert torch.equal(a[0].view(torch.float32), b[0].view(torch.float32))
    assert torch.equal(a[1], b[1])
    fn = dbp.dbp_function()
    xr = x.clone().requires_grad_(True)
    tr = t.clone().requires_grad_(True)
    y = fn.apply(xr, tr, None, p)
    loss = (torch.view_as_real(y) * torch.view_as_real(g)).sum()   # dL/dy = g (real-pair convention)
    loss.backward()
    assert torch.equal(xr.grad.view(torch.float32), a[0].view(torch.float32))
    assert torch.equal(tr.grad, a[1])


@pytest.mark.parametrize("nb,o,k,n_pol,nc,n,sparse", [
    (1024, 256, 2, 2, 4, 5000, False),      # the fields of every step kept by the forward pass
    (1024, 256, 2, 2, 4, 5000, True),       # pass inputs kept, the reverse recomputes
    (256, 64, 3, 1, 3, 3000, False),        # one-wave blocks, 7 taps (run-time tap count)
    (512, 128, 2, 2, None, 200000, False),  # SSFM on 521 blocks (not polarization-split)
    (2048, 512, 2, 2, 4, 9000, False),
    (4096, 1024, 2, 1, 4, 12000, False),
])
def test_fft_saved_forward_then_reverse(dbp, nb, o, k, n_pol, nc, n, sparse):
    # what dbp_backprop_save keeps gives dbp_backprop_grad's gradients bit for bit, and its
    # output is dbp_backprop's, bit for bit, in either mode
    n_spans = 6
    xs, taps, gout = case(8, 1, n_pol, n, n_spans, nc)
    p = dbp.plan(n, n_spans, 1, batch=1, n_pol=n_pol, taps=None if taps is None else taps[0], block=nb,
                 overlap=o, steps_per_pass=k, grad_sparse=sparse, beta2_ps2_km=B2)
    x, g = dev(xs, np.complex64), dev(gout, np.complex64)
    t = None if taps is None else dev(taps, np.float32)
    ref_out = p.backprop(x, taps=t)
    ref = p.backprop_grad(x, g, taps=t)
    out, ws = p.backprop_save(x, taps=t)
    got = p.backprop_grad_saved(x, out, ws, g, taps=t)
    again = p.backprop_grad_saved(x, out, ws, g, taps=t)
    torch.cuda.synchronize()
    print(f"Nb={nb} k={k} pol={n_pol} sparse={sparse}: {p.kernel}, grad workspace {p.workspace_size(grad=True)}")
    assert torch.equal(torch.view_as_real(out), torch.view_as_real(ref_out))
    for r in (got, again):
        assert torch.equal(torch.view_as_real(r[0]), torch.view_as_real(ref[0]))
        assert (r[1] is None and ref[1] is None) or torch.equal(r[1], ref[1])
        assert r[2] is None


def test_fft_kept_fields_budget_and_persistent_plans(dbp):
    # 64 headline-size signals: the kept fields (8 passes x 5 steps x 342 blocks x 64 x 2 x
    # 1024 x 8 B = 14.3 GB) exceed the 4 GiB budget, so the plan keeps pass inputs only
    n, k, nb, V = 262144, 5, 1024, 768
    big = dbp.plan(n, 40, 1, batch=64, taps=np.full(9, 0.1, np.float32), block=nb, overlap=nb - V,
                   beta2_ps2_km=B2)
    assert big.steps_per_pass == k
    n_wg = -(-n // V) * 64
    state = 64 * 2 * n * 8
    window = n_wg * 2 * nb * 8
    assert big.workspace_size(grad=True) == 7 * state + (k - 1) * window + 2 * window + 40 * 9 * n_wg * 4
    big.close()
    # a persistent-launch plan: the forward that keeps the fields gives its output bit for bit
    n_spans = 6
    xs, taps, gout = case(12, 1, 2, 20000, n_spans, 4)
    p = dbp.plan(20000, n_spans, 1, taps=taps[0], block=1024, overlap=256, steps_per_pass=2, persistent=True,
                 beta2_ps2_km=B2)
    x, t, g = dev(xs, np.complex64), dev(taps, np.float32), dev(gout, np.complex64)
    ref_out = p.backprop(x, taps=t)
    out, ws = p.backprop_save(x, taps=t)
    got = p.backprop_grad_saved(x, out, ws, g, taps=t)
    ref = p.backprop_grad(x, g, taps=t)
    torch.cuda.synchronize()
    print(f"persistent plan: {p.kernel}")
    assert torch.equal(torch.view_as_real(out), torch.view_as_real(ref_out))
    assert torch.equal(torch.view_as_real(got[0]), torch.view_as_real(ref[0]))
    assert torch.equal(got[1], ref[1])
    p.close()


def test_fft_grad_finite_difference_of_gpu_forward(dbp):
    # d/dw of <g, DBP(x; w)> along a tap direction, by central differences of the GPU forward
    n, n_spans = 4096, 4
    xs, taps, gout = case(11, 1, 2, n, n_spans, 4)
    p = dbp.plan(n, n_spans, 1, taps=taps[0], block=1024, overlap=256, steps_per_pass=2, beta2_ps2_km=B2)
    x = dev(xs, np.complex64)
    g = dev(gout, np.complex64)
    _, gt, _ = p.backprop_grad(x, g, taps=dev(taps, np.float32))
    d = np.zeros_like(taps)
    d[:, 4] = 1.0      # centre tap of every step
    h = 1e-2

    def f(tp):
        y = p.backprop(x, taps=dev(tp, np.float32)).cpu().numpy().astype(np.complex128)
        return float(np.sum(np.real(np.conj(gout.astype(np.complex128)) * y)))

    fd = (f(taps + h * d) - f(taps - h * d)) / (2 * h)
    an = float(np.sum(gt.cpu().numpy().astype(np.float64) * d))
    print(f"directional derivative: adjoint {an:.6e}, central difference {fd:.6e}")
    assert abs(an - fd) <= 2e-3 * abs(fd) + 1e-6


def test_fft_grad_argument_rules(dbp):
    # workspace sizes, the FIR-only argument, unsupported plans and overlapping buffers
    import ctypes
    n = 4096
    p = dbp.plan(n, 4, 1, taps=np.full(9, 0.1, np.float32), block=1024, overlap=256, steps_per_pass=2,
                 beta2_ps2_km=B2)
    ws = p.workspace_size(grad=True)
    # pass inputs 1..: one state; the fields of the 4 steps kept by the forward pass (2 passes
    # of 2 steps), two window sets, partials
    n_wg = -(-n // 768)
    state = 2 * n * 8
    window = n_wg * 2 * 1024 * 8
    assert ws == state + 4 * window + 2 * window + 4 * 9 * n_wg * 4
    # recomputed passes: the fields of step 0 of one pass only
    sp = dbp.plan(n, 4, 1, taps=np.full(9, 0.1, np.float32), block=1024, overlap=256, steps_per_pass=2,
                  grad_sparse=True, beta2_ps2_km=B2)
    assert sp.workspace_size(grad=True) == state + window + 2 * window + 4 * 9 * n_wg * 4
    x = torch.zeros(1, 2, n, dtype=torch.complex64, device="cuda")
    g = torch.zeros_like(x)
    L = dbp.lib()
    w = p.workspace(grad=True)
    gf = torch.zeros(4, 33, dtype=torch.complex64, device="cuda")
    st = L.dbp_backprop_grad(p.handle, ctypes.c_void_p(x.data_ptr()), None, None, ctypes.c_void_p(g.data_ptr()),
                             None, None, ctypes.c_void_p(gf.data_ptr()), ctypes.c_void_p(w.data_ptr()), w.numel(),
                             None)
    assert st == 1          # grad_fir given for an FFT-step plan
    st = L.dbp_backprop_grad(p.handle, ctypes.c_void_p(x.data_ptr()), None, None, ctypes.c_void_p(g.data_ptr()),
                             ctypes.c_void_p(g.data_ptr()), None, None, ctypes.c_void_p(w.data_ptr()), w.numel(),
                             None)
    assert st == 1          # grad_in overlaps grad_out
    st = L.dbp_backprop_grad(p.handle, ctypes.c_void_p(x.data_ptr()), None, None, ctypes.c_void_p(g.data_ptr()),
                             None, None, None, ctypes.c_void_p(w.data_ptr()), w.numel() - 1, None)
    assert st == 3          # workspace too small
    torch.cuda.synchronize()
    # no reverse kernel: the split-precision variant and 8192-point blocks
    for q in (dbp.plan(n, 4, 1, block=1024, overlap=256, precision=dbp.BF16X3, beta2_ps2_km=B2),
              dbp.plan(16384, 2, 1, block=8192, overlap=1024, beta2_ps2_km=B2)):
        assert q.workspace_size(grad=True) == 0
        with pytest.raises(dbp.DbpError) as e:
            q.backprop_grad(torch.zeros(1, 2, q.shape[2], dtype=torch.complex64, device="cuda"),
                            torch.zeros(1, 2, q.shape[2], dtype=torch.complex64, device="cuda"),
                            workspace=torch.zeros(16, dtype=torch.uint8, device="cuda"))
        assert e.value.status == 2
