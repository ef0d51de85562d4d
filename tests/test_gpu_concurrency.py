"""Concurrent use from several host threads, under the rule the header states (a plan is
immutable after creation; concurrent calls on one plan are safe when each call has its own
workspace): one plan called at once from four threads, each on its own stream with its own
workspace, and plans created at once from four threads.  Every result is bit for bit the
sequential one.  ctypes releases the interpreter lock during the library's calls, so the threads
do run the library concurrently."""
import threading

import numpy as np
import pytest

import siggen
from gpu_inputs import B2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

T9 = siggen.symmetric_taps(siggen.rng(8, 0, 1), 4).astype(np.float32)
N_THREADS = 4


@pytest.fixture(scope="module")
def dbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1507_00921_amd as m
    m.lib()
    return m


def field(seed, shape):
    g = np.random.default_rng([88, seed])
    a = (g.standard_normal(shape) + 1j * g.standard_normal(shape)) * 0.03
    return torch.from_numpy(a.astype(np.complex64)).cuda()


def run_threads(fn, n=N_THREADS):
    out, errs = [None] * n, []

    def work(i):
        try:
            out[i] = fn(i)
        except BaseException as e:          # re-raised in the test's thread
            errs.append(e)

    ts = [threading.Thread(target=work, args=(i,)) for i in range(n)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    if errs:
        raise errs[0]
    return out


def test_one_fft_plan_from_four_threads(dbp):
    p = dbp.plan(20000, 8, 1, taps=T9, block=1024, overlap=256, beta2_ps2_km=B2)
    xs = [field(i, p.shape) for i in range(N_THREADS)]
    ref = [p.backprop(x).clone() for x in xs]
    torch.cuda.synchronize()

    def work(i):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            ws = p.workspace()
            out = torch.empty_like(xs[i])
            for _ in range(10):
                p.backprop(xs[i], out=out, workspace=ws, stream=s)
            s.synchronize()
            return out

    for i, y in enumerate(run_threads(work)):
        assert torch.equal(y, ref[i]), i
    p.close()


def test_one_fir_plan_forward_and_reverse_from_four_threads(dbp):
    p = dbp.plan(2500, 3, 1, taps=T9, linear=dbp.LINEAR_FIR, n_fir=33, fir_band_thz=0.0154, beta2_ps2_km=B2)
    xs = [field(10 + i, p.shape) for i in range(N_THREADS)]
    gs = [field(20 + i, p.shape) for i in range(N_THREADS)]
    ref_y = [p.backprop(x).clone() for x in xs]
    ref_g = [p.backprop_grad(x, g) for x, g in zip(xs, gs)]
    torch.cuda.synchronize()

    def work(i):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            ws = p.workspace(grad=True)
            for _ in range(4):
                y = p.backprop(xs[i], workspace=ws, stream=s)
                g = p.backprop_grad(xs[i], gs[i], workspace=ws, stream=s)
            s.synchronize()
            return y, g

    for i, (y, (gx, gt, gf)) in enumerate(run_threads(work)):
        rx, rt, rf = ref_g[i]
        assert torch.equal(y, ref_y[i]), i
        assert torch.equal(gx, rx) and torch.equal(gt, rt) and torch.equal(gf, rf), i
    p.close()


def test_plans_created_from_four_threads(dbp):
    kws = [dict(n=5000, spans=6, spp=1, taps=T9, block=1024, overlap=256),
           dict(n=3001, spans=4, spp=2, n_pol=1, block=512, overlap=128),
           dict(n=9000, spans=3, spp=1, taps=T9[1:-1] / T9[1:-1].sum(), block=2048, overlap=512),
           dict(n=900, spans=3, spp=1, linear=dbp.LINEAR_FIR, n_fir=33, fir_band_thz=0.0154)]

    def make(kw):
        kw = dict(kw)
        return dbp.plan(kw.pop("n"), kw.pop("spans"), kw.pop("spp"), beta2_ps2_km=B2, **kw)

    xs = []
    ref = []
    for i, kw in enumerate(kws):
        p = make(kw)
        xs.append(field(30 + i, p.shape))
        ref.append(p.backprop(xs[-1]).clone())
        p.close()
    torch.cuda.synchronize()

    def work(i):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            p = make(kws[i])
            y = p.backprop(xs[i], stream=s)
            s.synchronize()
            geo = (p.block, p.overlap, p.steps_per_pass)
            p.close()
            return y, geo

    for i, (y, geo) in enumerate(run_threads(work)):
        assert torch.equal(y, ref[i]), (i, geo)
