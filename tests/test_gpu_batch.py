"""GPU parity of the ragged batch (persistent, graph-replayed) against the FP64 oracle.

Each signal is compared with the oracle's overlap-and-save cascade in the
geometry the autotuner chose for it (read back per signal); tolerances as for
single plans: relative L2 <= 1e-5 up to 40 steps, <= 2e-4 beyond.
"""
import numpy as np
import pytest

import siggen
from oracle import dbp_ref as R

from gpu_inputs import B2, FS, field_err, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1507_00921_amd as m
    m.lib()
    return m


def descs_for(dbp, work, **kw):
    return [dbp.make_desc(w["n"], w["n_spans"], w["steps_per_span"], taps=w["taps"], beta2_ps2_km=B2, **kw)
            for w in work]


def fields_for(work, seed):
    return [siggen.transmitted_field(2, seed * 1000 + i, 2, w["n"], 2.0)[0].astype(np.complex64)
            for i, w in enumerate(work)]


def oracle_one(x, w, geo):
    nb, o, k = geo
    taps = None if w["taps"] is None else w["taps"].astype(np.float32).astype(np.float64)
    steps = R.schedule(w["n_spans"], 80.0, w["steps_per_span"], B2, 1.3, 0.2, taps=taps)
    return R.run_blocked(x.astype(np.complex128), steps, FS, nb, o, k), len(steps)


def small_work(seed, n):
    work = siggen.ragged_workload(n, seed=seed, lo_exp=11.5, hi_exp=14.0, spans=(2, 5), essfm_nc=(2, 6),
                                  ssfm_steps=(2, 8))
    work[0]["n"] = 2050            # short signal: partial last block shorter than the halo
    return work


def test_small_ragged_batch_parity(dbp):
    work = small_work(1, 14)
    bp = dbp.plan_batch(descs_for(dbp, work))
    xs = fields_for(work, 1)
    y = bp.unpack(bp.backprop(bp.pack(xs)))
    torch.cuda.synchronize()
    assert bp.status() == 0
    for i, w in enumerate(work):
        ref, ns = oracle_one(xs[i], w, bp.geometry(i))
        err = field_err(y[i].astype(np.complex128), ref)
        print(f"signal {i}: L={w['n']} steps={ns} geo={bp.geometry(i)} rel L2 {err:.3e}")
        assert err <= (1e-5 if ns <= 40 else 2e-4)


def test_graph_replays_and_in_place(dbp):
    work = small_work(2, 10)
    bp = dbp.plan_batch(descs_for(dbp, work))
    xs = fields_for(work, 2)
    x = bp.pack(xs)
    ws = bp.workspace()
    out = torch.empty_like(x)
    first = bp.backprop(x, out=out, workspace=ws).clone()
    for r in range(3):
        # eager work between replays (a torch reduction over many blocks)
        _ = torch.sum(torch.abs(x)).item()
        again = bp.backprop(x, out=out, workspace=ws)
        torch.cuda.synchronize()
        assert torch.equal(again, first), r
    y = x.clone()
    bp.backprop(y, out=y, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(y, first)
    assert bp.status() == 0


def test_explicit_geometry_is_kept(dbp):
    work = small_work(3, 6)
    ds = descs_for(dbp, work, block=512, overlap=128, steps_per_pass=2)
    bp = dbp.plan_batch(ds)
    xs = fields_for(work, 3)
    y = bp.unpack(bp.backprop(bp.pack(xs)))
    for i, w in enumerate(work):
        assert bp.geometry(i) == (512, 128, 2)
        ref, ns = oracle_one(xs[i], w, (512, 128, 2))
        assert field_err(y[i].astype(np.complex128), ref) <= (1e-5 if ns <= 40 else 2e-4)


def test_full_ragged_workload_sampled(dbp):
    # 512 signals (lengths 2^12..2^17, 10-40 spans, half ESSFM 5-13 taps, half SSFM 4-20 steps/span):
    # the shortest, the longest and six more signals against the oracle
    work = siggen.ragged_workload(512, seed=0)
    bp = dbp.plan_batch(descs_for(dbp, work))
    lengths = np.array([w["n"] for w in work])
    steps = np.array([w["n_spans"] * w["steps_per_span"] for w in work])
    cost = lengths * steps
    pick = [int(np.argmin(lengths)), int(np.argmax(lengths))]
    order = np.argsort(cost)
    pick += [int(i) for i in order[[10, 60, 120, 200, 300, 400]] if int(i) not in pick]
    xs = [None] * 512
    for i in range(512):
        xs[i] = siggen.transmitted_field(2, i, 2, work[i]["n"], 0.0)[0].astype(np.complex64) \
            if i in pick else np.zeros((2, work[i]["n"]), np.complex64)
    y = bp.unpack(bp.backprop(bp.pack(xs)))
    torch.cuda.synchronize()
    assert bp.status() == 0
    for i in pick:
        ref, ns = oracle_one(xs[i], work[i], bp.geometry(i))
        err = field_err(y[i].astype(np.complex128), ref)
        print(f"cfg2 signal {i}: L={work[i]['n']} steps={ns} geo={bp.geometry(i)} rel L2 {err:.3e}")
        assert err <= (1e-5 if ns <= 40 else 2e-4)


def test_grouped_blocks_long_signals(dbp):
    # long signals on small blocks: 50..160 blocks each, so work items carry 1..4 blocks
    lengths = [19500, 25000, 40000, 52000, 61440, 33334]
    work = []
    for i, n in enumerate(lengths):
        taps = siggen.symmetric_taps(siggen.rng(2, 900 + i, 0), 2 + i % 3) if i % 2 == 0 else None
        work.append(dict(n=n, n_spans=6, steps_per_span=1 if taps is not None else 3, taps=taps))
    ds = descs_for(dbp, work, block=512, overlap=128, steps_per_pass=2)
    bp = dbp.plan_batch(ds)
    xs = fields_for(work, 9)
    y = bp.unpack(bp.backprop(bp.pack(xs)))
    torch.cuda.synchronize()
    assert bp.status() == 0
    for i, w in enumerate(work):
        ref, ns = oracle_one(xs[i], w, bp.geometry(i))
        err = field_err(y[i].astype(np.complex128), ref)
        print(f"grouped signal {i}: L={w['n']} blocks={-(-w['n'] // 384)} steps={ns} rel L2 {err:.3e}")
        assert err <= 1e-5


def test_batch_kernel_reproduces_the_pass_kernel_on_1024_point_blocks(dbp):
    # the batch kernel runs the same block routine (the in-wave transform at Nb = 1024):
    # per signal, bit for bit the output of a single plan with that geometry, and the oracle
    work = [dict(n=n, n_spans=5, steps_per_span=1, taps=siggen.symmetric_taps(siggen.rng(2, 950 + i, 0), 4))
            for i, n in enumerate((20000, 9000, 31112))]
    ds = descs_for(dbp, work, block=1024, overlap=256, steps_per_pass=3)
    bp = dbp.plan_batch(ds)
    xs = fields_for(work, 11)
    y = bp.unpack(bp.backprop(bp.pack(xs)))
    torch.cuda.synchronize()
    assert bp.status() == 0
    for i, w in enumerate(work):
        assert bp.geometry(i) == (1024, 256, 3)
        p = dbp.plan(w["n"], 5, 1, taps=w["taps"], block=1024, overlap=256, steps_per_pass=3, beta2_ps2_km=B2)
        yp = p.backprop(torch.from_numpy(xs[i]).reshape(1, 2, -1).cuda()).cpu().numpy().reshape(2, -1)
        assert np.array_equal(y[i].view(np.float32), yp.view(np.float32))
        ref, ns = oracle_one(xs[i], w, (1024, 256, 3))
        assert field_err(y[i].astype(np.complex128), ref) <= 1e-5


def test_concurrent_groups_equal_serial_groups(dbp, monkeypatch):
    # the kernel-variant groups (SSFM, ESSFM with 9 and with other tap counts) run as parallel
    # branches of the graph; run one after another instead they give the same bits
    work = small_work(3, 12)
    outs = []
    for serial in ("1", "0"):
        monkeypatch.setenv("DBP_BATCH_SERIAL", serial)
        bp = dbp.plan_batch(descs_for(dbp, work))
        y = bp.backprop(bp.pack(fields_for(work, 3)))
        torch.cuda.synchronize()
        assert bp.status() == 0
        outs.append(y.clone())
        bp.close()
    assert torch.equal(torch.view_as_real(outs[0]), torch.view_as_real(outs[1]))


def test_tune_cache_persists_measured_costs(dbp, tmp_path):
    """DBP_TUNE_CACHE: a first process times the batch kernel variants it needs and appends
    them to the cache; a second process reads them instead of timing (it writes no timing log)
    and chooses the same geometries; a cache that prices 2048-point blocks far below the other
    sizes makes the tuner choose them.  Separate processes: the costs are also kept in memory."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys, json; sys.path.insert(0, %r); import numpy as np; import paper_1507_00921_amd as d\n"
            "bp = d.plan_batch([d.make_desc(300000, 4, 1, taps=np.full(9, 1 / 9, np.float32)),"
            " d.make_desc(200000, 3, 4)])\n"
            "print(json.dumps([bp.geometry(i) for i in range(2)]))\n" % root)

    def run(cache, log):
        env = dict(os.environ, DBP_TUNE_CACHE=str(cache), DBP_AUTOTUNE_LOG=str(log))
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=150,
                           cwd=root)
        assert r.returncode == 0, r.stderr[-2000:]
        return json.loads(r.stdout.strip().splitlines()[-1])

    cache = tmp_path / "tune.jsonl"
    geo1 = run(cache, tmp_path / "log1.jsonl")
    rows = [json.loads(ln) for ln in cache.read_text().splitlines()]
    assert rows and (tmp_path / "log1.jsonl").exists()
    assert all(r["arch"].startswith("gfx950") and r["cus"] > 0 and r["c0_us"] > 0 for r in rows)
    assert {r["nb"] for r in rows} >= {1024, 2048}
    geo2 = run(cache, tmp_path / "log2.jsonl")
    assert not (tmp_path / "log2.jsonl").exists()        # read from the cache, not timed
    assert geo2 == geo1
    forced = tmp_path / "forced.jsonl"
    forced.write_text("".join(json.dumps(dict(r, c0_us=0.01 if r["nb"] == 2048 else 100.0,
                                              c1_us=0.01 if r["nb"] == 2048 else 100.0)) + "\n" for r in rows))
    geo3 = run(forced, tmp_path / "log3.jsonl")
    assert not (tmp_path / "log3.jsonl").exists()
    assert all(g[0] == 2048 for g in geo3), geo3
