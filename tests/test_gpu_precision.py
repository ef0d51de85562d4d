"""Precision variants against the FP64 oracle (needs an MI355X).

Three arithmetic variants of the same path: FP32 tables and phase, FP32 with
FP64-generated tables and an FP64 phase argument, and the split-precision
variant whose block DFTs run as BF16x3 products on the matrix cores (four-step
1024 = 64 x 16 factorisation, FP32 accumulation).

Tolerance of the split-precision variant, from its arithmetic: each operand is
carried as hi + lo with both parts rounded to BF16 (8-bit significands), which
leaves a relative residual of up to 2^-16 (1.5e-5) per operand, and the dropped
lo*lo term is of the same order.  Through the four products of a 1024-point
transform this is a relative L2 error of about 4.5e-6 per transform (an error
model of exactly these roundings).  The part of it that comes from the constant
DFT fragments is the same at every step, so it adds coherently over a cascade
rather than as a random walk: the bound is 6e-6 per step (two transforms),
linear in N_s, plus 1e-5 for the FP32 rest of the step.
"""
import numpy as np
import pytest

import siggen
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


def split_bound(n_steps):
    return 6e-6 * n_steps + 1e-5


def run(dbp, x, n_spans, sps, precision, taps=None, **kw):
    n_pol, n = x.shape
    p = dbp.plan(n, n_spans, sps, n_pol=n_pol, taps=taps, precision=precision, beta2_ps2_km=B2, **kw)
    xt = torch.from_numpy(np.ascontiguousarray(x.astype(np.complex64))).reshape(1, n_pol, n).cuda()
    y = p.backprop(xt)
    torch.cuda.synchronize()
    return p, y.cpu().numpy().reshape(n_pol, n).astype(np.complex128)


def oracle(x, p, n_spans, sps, taps=None):
    t = None if taps is None else np.asarray(taps, np.float32).astype(np.float64)
    steps = R.schedule(n_spans, 80.0, sps, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM, taps=t)
    if p.overlap == 0 and p.block == x.shape[-1]:
        return R.run_whole(x, steps, FS)
    return R.run_blocked(x, steps, FS, p.block, p.overlap, p.steps_per_pass)


TAPS9 = siggen.symmetric_taps(siggen.rng(4, 0, 7), 4)
TAPS7 = siggen.symmetric_taps(siggen.rng(4, 0, 8), 3)


@pytest.mark.parametrize("n_pol,n,spans,sps,taps", [
    (2, 5 * 1024 + 338, 4, 1, TAPS9),        # ESSFM, compile-time 9 taps, ragged tail
    (2, 7000, 3, 2, None),                   # SSFM, several steps per pass
    (1, 6 * 1024, 5, 1, TAPS7),              # one polarization, run-time taps
    (2, 3000, 40, 1, TAPS9),                 # 40 steps, signal shorter than 3 blocks
])
def test_split_precision_blocked_parity(dbp, n_pol, n, spans, sps, taps):
    x = siggen.transmitted_field(4, n, n_pol, n, 2.0)[0].astype(np.complex64).astype(np.complex128)
    p, y = run(dbp, x, spans, sps, dbp.BF16X3, taps=taps)
    assert p.block == 1024
    ref = oracle(x, p, spans, sps, taps)
    err = field_err(y, ref)
    ns = spans * sps
    print(f"BF16x3 n_pol={n_pol} L={n} steps={ns} k={p.steps_per_pass} O={p.overlap}: rel L2 {err:.3e} "
          f"(bound {split_bound(ns):.2e})")
    assert err <= split_bound(ns)


def test_split_precision_whole_block(dbp):
    x = siggen.transmitted_field(4, 1, 2, 1024, 3.0)[0].astype(np.complex64).astype(np.complex128)
    p, y = run(dbp, x, 2, 2, dbp.BF16X3, taps=TAPS9, whole=True)
    ref = oracle(x, p, 2, 2, TAPS9)
    err = field_err(y, ref)
    print(f"BF16x3 whole 1024: rel L2 {err:.3e}")
    assert err <= split_bound(4)


def test_split_precision_explicit_geometry_and_repeat(dbp):
    x = siggen.transmitted_field(4, 2, 2, 9000, 0.0)[0].astype(np.complex64).astype(np.complex128)
    p, y = run(dbp, x, 6, 1, dbp.BF16X3, taps=TAPS9, block=1024, overlap=384, steps_per_pass=3)
    assert (p.block, p.overlap, p.steps_per_pass) == (1024, 384, 3)
    ref = oracle(x, p, 6, 1, TAPS9)
    assert field_err(y, ref) <= split_bound(6)
    _, y2 = run(dbp, x, 6, 1, dbp.BF16X3, taps=TAPS9, block=1024, overlap=384, steps_per_pass=3)
    assert np.array_equal(y, y2)          # deterministic


def test_precision_report_800_steps(dbp):
    """The precision workload at reduced length: 2 x 65536 samples at 3200 km, SSFM 20
    steps/span (800 steps), received field from the oracle's forward channel (0 dBm, 20 dB
    OSNR).  Per variant: relative L2 error and EVM change against the FP64 oracle."""
    n = 65536
    rx, sym = received(4, 0, 2, n, 0.0, 40, 20)
    report = {}
    ref = None
    for name, prec in [("fp32", dbp.FP32), ("fp32_fp64phase", dbp.FP32_FP64PHASE), ("bf16x3", dbp.BF16X3)]:
        p, y = run(dbp, rx, 40, 20, prec, block=1024, overlap=256)
        if ref is None:
            ref = oracle(rx, p, 40, 20)
            evm_ref = siggen.evm_db(ref, sym)
        err = field_err(y, ref)
        d_evm = siggen.evm_db(y, sym) - evm_ref
        report[name] = (err, d_evm)
        print(f"precision {name}: rel L2 {err:.3e}, EVM change {d_evm:+.5f} dB (oracle EVM {evm_ref:.3f} dB)")
    assert report["fp32_fp64phase"][0] <= 2e-4
    assert report["fp32"][0] <= 3e-4
    assert report["bf16x3"][0] <= split_bound(800)
    for name, (_, d) in report.items():
        assert abs(d) <= 0.01, name


def test_precision_workload_full_size_sampled(dbp):
    """The precision workload at its full size, 2 x 4194304 samples, SSFM 800 steps on
    Nb = 1024, O = 256 with the planner's steps per pass (the launches bench.py times),
    checked on sampled blocks.  A block's output after P passes depends on the input within
    about P blocks of it, so the oracle runs the same blocked cascade on a window aligned to
    the block grid with P + 2 blocks of margin on each side: the window's own circular wrap
    reaches at most one block further per pass, and the centre block is exact.  Input: the
    launched field (the path's arithmetic does not depend on it having crossed the link)."""
    n = 4194304
    x, _ = siggen.transmitted_field(4, 1, 2, n, 0.0)
    x = x.astype(np.complex64).astype(np.complex128)
    steps = R.schedule(40, 80.0, 20, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM)
    for name, prec, tol in [("fp32", dbp.FP32, 2e-4), ("fp32_fp64phase", dbp.FP32_FP64PHASE, 2e-4),
                            ("bf16x3", dbp.BF16X3, split_bound(800))]:
        p, y = run(dbp, x, 40, 20, prec, block=1024, overlap=256)
        v = p.block - p.overlap
        n_blk = -(-n // v)
        m = p.n_passes + 2
        for b in [m, n_blk // 2, n_blk - m - 2]:
            idx = ((b - m) * v + np.arange((2 * m + 1) * v)) % n
            w = R.run_blocked(x[:, idx], steps, FS, p.block, p.overlap, p.steps_per_pass)
            got = y[:, b * v:(b + 1) * v]
            want = w[:, m * v:(m + 1) * v]
            err = field_err(got, want)
            print(f"{name} k={p.steps_per_pass} passes={p.n_passes} block {b}: rel L2 {err:.3e}")
            assert err <= tol
