"""GPU parity of the loss head (dbp_mse_*) against the oracle's FP64 symbol MSE (needs an MI355X).

The loss is mean |MF(z)[::2] / amp - s|^2 over every symbol with the receive RRC filter
applied circularly in frequency (Sec. IV footnote); the oracle's value and gradient are
pinned by central differences in tests/test_oracle_adjoint.py.  The GPU evaluates it as
half- and quarter-length transforms (no length-L FFT), so its rounding differs from the
oracle's: loss within 1e-5 relative, gradient within 1e-5 relative L2 and the per-sample
bound of the other parity tests.
"""
import math

import numpy as np
import pytest

import siggen
from oracle import adjoint as A
from oracle import dbp_ref as R

from gpu_inputs import B2, FS, field_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1507_00921_amd as m
    m.lib()
    return m


def _inputs(seed, batch, n_pol, n, p_dbm, noise=0.15):
    """Shaped PM-QPSK fields with additive noise (residual of order `noise` per symbol)."""
    zs, syms = [], []
    for b in range(batch):
        x, s = siggen.transmitted_field(3, 1000 * seed + b, n_pol, n, p_dbm)
        g = siggen.rng(3, 1000 * seed + b, 9)
        sig = math.sqrt(siggen.dbm_to_w(p_dbm) / n_pol) * noise
        x = x + sig * (g.standard_normal(x.shape) + 1j * g.standard_normal(x.shape)) / math.sqrt(2)
        zs.append(x)
        syms.append(s)
    z = np.stack(zs).astype(np.complex64).astype(np.complex128)
    s = np.stack(syms).astype(np.complex64).astype(np.complex128)
    return z, s


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).cuda()


def _oracle(z, s, p_w, n):
    """The oracle's loss over the whole batch and its gradient (mean over all symbols)."""
    batch = z.shape[0]
    mf = siggen.rrc_response(n)
    losses, grads = [], []
    for b in range(batch):
        l_b, g_b = A.symbol_mse(z[b], s[b], p_w, mf)
        losses.append(l_b)
        grads.append(g_b / batch)        # each signal's mean is over 1/batch of the symbols
    return float(np.mean(losses)), np.stack(grads)


@pytest.mark.parametrize("batch,n_pol,n", [(1, 2, 2048), (3, 1, 4096), (2, 2, 8192), (1, 2, 16384),
                                           (64, 2, 32768)])
def test_loss_and_gradient_match_oracle(dbp, batch, n_pol, n):
    p_dbm = 1.0
    p_w = siggen.dbm_to_w(p_dbm)
    z, s = _inputs(n, batch, n_pol, n, p_dbm)
    amp = math.sqrt(2 * p_w / n_pol)
    head = dbp.SymbolMse(n, n_pol, batch, siggen.rrc_response(n), amp)
    loss = head.forward(_dev(z), _dev(s))
    g = head.backward()
    torch.cuda.synchronize()
    lref, gref = _oracle(z, s, p_w, n)
    got = g.cpu().numpy().astype(np.complex128)
    el = abs(float(loss.item()) - lref) / lref
    eg = field_err(got, gref)
    print(f"mse {batch}x{n_pol}x{n}: loss {loss.item():.6f} (rel {el:.2e}), grad {eg:.2e}")
    assert el <= 1e-5
    assert eg <= 1e-5
    head.close()


def test_gradient_scale_and_reuse(dbp):
    # backward scales by the device scalar dL/dloss; two forwards in a row (second on other
    # data) leave the second's residual; repeated calls are bitwise reproducible
    n, batch, n_pol = 4096, 2, 2
    p_w = siggen.dbm_to_w(0.0)
    amp = math.sqrt(2 * p_w / n_pol)
    head = dbp.SymbolMse(n, n_pol, batch, siggen.rrc_response(n), amp)
    z1, s1 = _inputs(1, batch, n_pol, n, 0.0)
    z2, s2 = _inputs(2, batch, n_pol, n, 0.0, noise=0.3)
    head.forward(_dev(z2), _dev(s2))
    l1 = head.forward(_dev(z1), _dev(s1)).clone()
    g1 = head.backward().clone()
    scale = torch.tensor([0.375], dtype=torch.float32, device="cuda")
    g1s = head.backward(scale)
    l1b = head.forward(_dev(z1), _dev(s1))
    g1b = head.backward()
    torch.cuda.synchronize()
    assert torch.equal(l1, l1b)
    assert torch.equal(torch.view_as_real(g1), torch.view_as_real(g1b))
    # the scale enters before the transforms: equal to FP32 rounding of the scaled inputs
    assert field_err(g1s.cpu().numpy().astype(np.complex128), 0.375 * g1.cpu().numpy().astype(np.complex128)) <= 1e-6
    lref, gref = _oracle(z1, s1, p_w, n)
    assert abs(float(l1.item()) - lref) <= 1e-5 * lref
    assert field_err(g1.cpu().numpy().astype(np.complex128), gref) <= 1e-5
    head.close()


def test_training_step_through_the_library(dbp):
    # DBP (FIR steps, per-step ESSFM taps) then the loss head, both through autograd: input,
    # tap and FIR gradients against the oracle's chain rule (grad_whole of the loss gradient)
    n, n_spans, n_pol, nf = 4096, 4, 2, 33
    p_dbm = 2.0
    p_w = siggen.dbm_to_w(p_dbm)
    x, sym = siggen.transmitted_field(3, 77, n_pol, n, p_dbm)
    xs = x.astype(np.complex64).astype(np.complex128)
    g = np.random.default_rng(11)
    base = R.schedule(n_spans, 80.0, 1, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM)
    h0 = R.ls_fir_taps(nf, base[0].b, FS, 0.0154)
    fir = np.stack([h0 * (1 + 0.02 * (g.standard_normal(nf) + 1j * g.standard_normal(nf)))
                    for _ in base]).astype(np.complex64)
    taps = np.stack([siggen.symmetric_taps(siggen.rng(3, 77, s), 4) for s in range(n_spans)]).astype(np.float32)
    steps = [R.Step(b=st.b, phi=st.phi, w=taps[s].astype(np.float64), h=fir[s].astype(np.complex128))
             for s, st in enumerate(base)]
    p = dbp.plan(n, n_spans, 1, taps=taps[0], linear=dbp.LINEAR_FIR, fir=fir[0], beta2_ps2_km=B2)
    amp = math.sqrt(2 * p_w / n_pol)
    head = dbp.SymbolMse(n, n_pol, 1, siggen.rrc_response(n), amp)
    xt = _dev(xs).reshape(1, n_pol, n).requires_grad_(True)
    t = torch.from_numpy(taps).cuda().requires_grad_(True)
    f = torch.from_numpy(fir).cuda().requires_grad_(True)
    z = dbp.dbp_function().apply(xt, t, f, p)
    s_dev = _dev(sym.astype(np.complex128)).reshape(1, n_pol, n // 2)
    loss = dbp.mse_function().apply(z, s_dev, head)
    loss.backward()
    torch.cuda.synchronize()
    zo = R.run_whole(xs, steps, FS)
    lref, gz = A.symbol_mse(zo, sym, p_w, siggen.rrc_response(n))
    gr = A.grad_whole(xs, steps, FS, gz)
    assert abs(loss.item() - lref) <= 1e-5 * lref
    ex = field_err(xt.grad[0].cpu().numpy().astype(np.complex128), gr.x)
    et = field_err(t.grad.cpu().numpy().astype(np.float64), np.stack(gr.w))
    ef = field_err(f.grad.cpu().numpy().astype(np.complex128), np.stack(gr.h))
    print(f"training step: loss {loss.item():.6f} grad x {ex:.2e} taps {et:.2e} fir {ef:.2e}")
    assert ex <= 1e-4 and et <= 1e-4 and ef <= 1e-4
    head.close()
    p.close()


def test_reverse_mode_guard(dbp):
    # the reverse mode uses the last forward's residual: a stale autograd graph is refused
    n = 2048
    head = dbp.SymbolMse(n, 2, 1, siggen.rrc_response(n), 1.0)
    z, s = _inputs(5, 1, 2, n, 0.0)
    zt = _dev(z).requires_grad_(True)
    l1 = dbp.mse_function().apply(zt, _dev(s), head)
    dbp.mse_function().apply(zt, _dev(s), head)
    with pytest.raises(RuntimeError):
        l1.backward()
    head.close()
