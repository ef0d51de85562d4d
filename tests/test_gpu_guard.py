"""Guard zones around every device buffer a call reads or writes.

Each buffer the library gets is the middle of a larger allocation.  The guards of inputs and
workspaces hold NaN bit patterns, so a read past a buffer's end (or before its start) puts NaN
into the result; the guards of outputs hold a NaN pattern that arithmetic never produces, so a
write past a buffer changes them.  Every guarded call is checked bit for bit against the same
call on ordinary allocations, and every guard word afterwards.  Covers the pass kernels
(blocked, whole-signal, the 8192-point blocks, both FIR paths), both reverse modes through the
C ABI (FFT steps from kept fields and recomputed), the ragged batch, the receiver mode and the
receiver DSP.
"""
import numpy as np
import pytest

import siggen
from gpu_inputs import B2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PAD = 2048                        # 32-bit words of guard on each side (8 KiB: keeps alignment)
IN_FILL = 0x7FC0DEAD              # quiet NaN with a payload: inputs
WS_FILL = 0x7FC0BEEF              # quiet NaN: workspaces
OUT_FILL = 0x7FA5A5A5             # signalling-NaN pattern (never an arithmetic result): outputs
BAND = 0.0154
T9 = siggen.symmetric_taps(siggen.rng(7, 0, 1), 4).astype(np.float32)


@pytest.fixture(scope="module")
def dbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1507_00921_amd as m
    m.lib()
    return m


class Guarded:
    """A view of `words` 32-bit words in the middle of a guarded int32 allocation."""

    def __init__(self, words, fill):
        self.words, self.fill = words, fill
        self.whole = torch.full((words + 2 * PAD,), fill, dtype=torch.int32, device="cuda")
        self.mid = self.whole[PAD:PAD + words]

    def as_(self, dtype, shape):
        return self.mid.view(torch.float32).view(dtype).view(shape) if dtype != torch.uint8 else \
            self.mid.view(torch.uint8).view(shape)

    def intact(self):
        torch.cuda.synchronize()
        head, tail = self.whole[:PAD], self.whole[PAD + self.words:]
        return bool(torch.all(head == self.fill).item()) and bool(torch.all(tail == self.fill).item())


def guarded_copy(t, fill=IN_FILL):
    """A guarded copy of a complex64 / float32 tensor (same shape and bits)."""
    words = t.numel() * (2 if t.dtype == torch.complex64 else 1)
    g = Guarded(words, fill)
    v = g.as_(t.dtype, t.shape)
    v.copy_(t)
    return g, v


def guarded_out(shape, dtype):
    n = int(np.prod(shape)) * (2 if dtype == torch.complex64 else 1)
    g = Guarded(n, OUT_FILL)
    return g, g.as_(dtype, shape)


def guarded_ws(nbytes):
    g = Guarded(max(1, (nbytes + 3) // 4), WS_FILL)
    return g, g.mid.view(torch.uint8)


def same_bits(a, b):
    if a is None or b is None:
        return a is None and b is None
    return torch.equal(a.contiguous().view(torch.int32) if a.dtype == torch.float32 else
                       a.contiguous().view(torch.float32).view(torch.int32),
                       b.contiguous().view(torch.int32) if b.dtype == torch.float32 else
                       b.contiguous().view(torch.float32).view(torch.int32))


def field(seed, shape):
    g = np.random.default_rng([77, seed])
    a = (g.standard_normal(shape) + 1j * g.standard_normal(shape)) * 0.03
    return torch.from_numpy(a.astype(np.complex64)).cuda()


PLANS = {
    "fft_essfm_1024_ragged_batch2": dict(n=5000, n_spans=6, spp=1, batch=2, taps=T9, block=1024, overlap=256),
    # the reverse pass re-running its steps from the pass inputs instead of reading kept fields
    "fft_essfm_1024_recompute": dict(n=5000, n_spans=6, spp=1, batch=2, taps=T9, block=1024, overlap=256,
                                     grad_sparse=True),
    "fft_ssfm_512_one_pol": dict(n=3001, n_spans=4, spp=2, n_pol=1, block=512, overlap=128),
    "whole_signal_16384": dict(n=16384, n_spans=4, spp=1, n_pol=1, whole=True),
    "blocks_8192_essfm": dict(n=20000, n_spans=4, spp=1, taps=T9, block=8192, overlap=2048),
    "fir_time_domain": dict(n=900, n_spans=3, spp=1, taps=T9, fir_fir=True),
    "fir_fft_blocks": dict(n=2500, n_spans=3, spp=1, taps=T9, fir_fir=True),
}


def make(dbp, kw):
    kw = dict(kw)
    n, ns, spp = kw.pop("n"), kw.pop("n_spans"), kw.pop("spp")
    if kw.pop("fir_fir", False):
        kw.update(linear=dbp.LINEAR_FIR, n_fir=33, fir_band_thz=BAND)
    return dbp.plan(n, ns, spp, beta2_ps2_km=B2, **kw)


@pytest.mark.parametrize("name", list(PLANS))
def test_backprop_stays_inside_its_buffers(dbp, name):
    p = make(dbp, PLANS[name])
    x = field(1, p.shape)
    ref = p.backprop(x, workspace=p.workspace())
    gx, xv = guarded_copy(x)
    go, ov = guarded_out(p.shape, torch.complex64)
    gw, wv = guarded_ws(p.workspace_size())
    y = p.backprop(xv, out=ov, workspace=wv)
    torch.cuda.synchronize()
    print(f"{name}: Nb={p.block} O={p.overlap} k={p.steps_per_pass}")
    assert same_bits(y, ref)
    assert gx.intact() and go.intact() and gw.intact()
    p.close()


@pytest.mark.parametrize("name", ["fft_essfm_1024_ragged_batch2", "fft_essfm_1024_recompute", "fft_ssfm_512_one_pol",
                                  "fir_time_domain", "fir_fft_blocks"])
def test_backprop_grad_stays_inside_its_buffers(dbp, name):
    p = make(dbp, PLANS[name])
    x = field(2, p.shape)
    gout = field(3, p.shape)
    rx, rt, rf = p.backprop_grad(x, gout)
    ns = p.n_steps
    gx_in, xv = guarded_copy(x)
    gg_in, gv = guarded_copy(gout)
    g_gx, gx = guarded_out(p.shape, torch.complex64)
    g_gt, gt = (guarded_out((ns, p.desc.n_taps), torch.float32) if rt is not None else (None, None))
    g_gf, gf = (guarded_out((ns, p.desc.n_fir), torch.complex64) if rf is not None else (None, None))
    g_ws, wv = guarded_ws(p.workspace_size(grad=True))
    st = dbp.lib().dbp_backprop_grad(p._h, dbp._ptr(xv), None, None, dbp._ptr(gv), dbp._ptr(gx), dbp._ptr(gt),
                                     dbp._ptr(gf), dbp._ptr(wv), wv.numel(), dbp._stream_ptr(None))
    assert st == 0
    torch.cuda.synchronize()
    assert same_bits(gx, rx) and same_bits(gt, rt) and same_bits(gf, rf)
    for g in (gx_in, gg_in, g_gx, g_gt, g_gf, g_ws):
        assert g is None or g.intact()
    p.close()


def test_batch_stays_inside_its_buffers(dbp):
    specs = [(3000, 3, 1, T9), (700, 2, 4, None), (9000, 4, 1, T9[1:-1] / T9[1:-1].sum())]
    descs = [dbp.make_desc(n, s, spp, taps=t, beta2_ps2_km=B2) for n, s, spp, t in specs]
    bp = dbp.plan_batch(descs)
    x = field(4, (int(bp.offsets[-1]),))
    ref = bp.backprop(x, workspace=bp.workspace()).clone()
    gx, xv = guarded_copy(x)
    go, ov = guarded_out(x.shape, torch.complex64)
    gw, wv = guarded_ws(bp.workspace_size())
    y = bp.backprop(xv, out=ov, workspace=wv)
    torch.cuda.synchronize()
    assert bp.status() == 0
    assert same_bits(y, ref)
    assert gx.intact() and go.intact() and gw.intact()
    bp.close()


def test_receiver_stays_inside_its_buffers(dbp):
    chunk = 6144
    a = dbp.receiver(chunk, 6, 1, taps=T9, block=1024, overlap=256, beta2_ps2_km=B2)
    b = dbp.receiver(chunk, 6, 1, taps=T9, block=1024, overlap=256, beta2_ps2_km=B2)
    for i in range(3):
        x = field(10 + i, (2, chunk))
        ref = a.push(x)
        gx, xv = guarded_copy(x)
        go, ov = guarded_out((2, chunk), torch.complex64)
        y = b.push(xv, out=ov)
        torch.cuda.synchronize()
        assert same_bits(y, ref), i
        assert gx.intact() and go.intact(), i
    a.close()
    b.close()


def test_receiver_dsp_stays_inside_its_buffers(dbp):
    n_sym = 5600                  # n_sym * 50 / 28 samples: an integer
    x, s = siggen.transmitted_field_at_rate(40, 3, 2, n_sym, 0.0, 0.050)
    x = torch.from_numpy((x / np.sqrt(np.mean(np.abs(x) ** 2))).astype(np.complex64)).cuda()
    sym = torch.from_numpy(s.astype(np.complex64)).cuda()
    d = dbp.receiver_dsp(x.shape[-1])
    x2 = d.resample(x)
    taps = d.train(x2, sym, 2000)
    y = d.equalize(x2, taps)
    z, nerr = d.cpr(y, sym, 2000)
    gx, xv = guarded_copy(x)
    g2, x2v = guarded_out((2, d.n_out), torch.complex64)
    assert same_bits(d.resample(xv, out=x2v), x2)
    gy, yv = guarded_out((2, d.n_sym), torch.complex64)
    gx2, x2in = guarded_copy(x2)
    assert same_bits(d.equalize(x2in, taps, out=yv), y)
    gz, zv = guarded_out((2, d.n_sym), torch.complex64)
    gyin, yin = guarded_copy(y)
    gs, sv = guarded_copy(sym)
    z2, nerr2 = d.cpr(yin, sv, 2000, out=zv)
    torch.cuda.synchronize()
    assert same_bits(z2, z) and nerr2 == nerr
    for g in (gx, g2, gy, gx2, gz, gyin, gs):
        assert g.intact()
    d.close()
