"""Host-side checks of the C ABI: exports, validation, schedule and geometry (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

import siggen
from oracle import dbp_ref as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dbp.h")


def _lib_or_skip():
    import paper_1507_00921_amd as dbp
    if not os.path.exists(dbp.LIB_PATH):
        pytest.skip("libdbp.so not built")
    return dbp


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(dbp_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_core_entry_points():
    names = declared_functions()
    for n in ["dbp_plan", "dbp_backprop", "dbp_backprop_grad", "dbp_destroy", "dbp_workspace_size",
              "dbp_plan_batch", "dbp_backprop_batch", "dbp_status_string"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    dbp = _lib_or_skip()
    lib = dbp.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = os.popen(f"nm -D --defined-only {dbp.LIB_PATH}").read()
    for name in declared_functions():
        assert re.search(rf"\bT {name}$", out, flags=re.M), name


def test_status_strings_and_version():
    dbp = _lib_or_skip()
    lib = dbp.lib()
    for s in range(6):
        assert lib.dbp_status_string(s).decode() == dbp.STATUS[s]
    assert lib.dbp_version() == 0x000100


def test_desc_struct_layout_matches_header(tmp_path):
    # compile a probe against the header and compare every field offset with the ctypes mirror
    dbp = _lib_or_skip()
    fields = [f[0] for f in dbp.Desc._fields_]
    body = "\n".join(f'printf("%zu\\n", offsetof(dbp_desc, {f}));' for f in fields)
    src = tmp_path / "probe.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "dbp.h"\nint main(void){'
                   + body + 'printf("%zu\\n", sizeof(dbp_desc));return 0;}\n')
    exe = tmp_path / "probe"
    assert os.system(f"gcc -std=c99 -I{ROOT}/include {src} -o {exe}") == 0
    got = [int(v) for v in os.popen(str(exe)).read().split()]
    want = [getattr(dbp.Desc, f).offset for f in fields] + [ctypes.sizeof(dbp.Desc)]
    assert got == want


def test_dsp_desc_struct_layout_matches_header(tmp_path):
    dbp = _lib_or_skip()
    fields = [f[0] for f in dbp.DspDesc._fields_]
    body = "\n".join(f'printf("%zu\\n", offsetof(dbp_dsp_desc, {f}));' for f in fields)
    src = tmp_path / "probe.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "dbp.h"\nint main(void){'
                   + body + 'printf("%zu\\n", sizeof(dbp_dsp_desc));return 0;}\n')
    exe = tmp_path / "probe"
    assert os.system(f"gcc -std=c99 -I{ROOT}/include {src} -o {exe}") == 0
    got = [int(v) for v in os.popen(str(exe)).read().split()]
    want = [getattr(dbp.DspDesc, f).offset for f in fields] + [ctypes.sizeof(dbp.DspDesc)]
    assert got == want


@pytest.mark.parametrize("kw", [
    dict(up=24), dict(down=0), dict(up=5000, down=1), dict(resample_taps=47), dict(resample_taps=66),
    dict(kaiser_beta=-1.0), dict(eq_taps=14), dict(eq_taps=33), dict(cpr_half_window=-1),
    dict(cpr_half_window=300),
])
def test_invalid_dsp_descriptors_rejected_without_device(kw):
    dbp = _lib_or_skip()
    args = dict(up=28, down=25, resample_taps=48, kaiser_beta=8.0, eq_taps=15, cpr_half_window=16)
    args.update(kw)
    d = dbp.DspDesc(**args)
    h = ctypes.c_void_p(123)
    assert dbp.lib().dbp_dsp_create(ctypes.byref(d), 2500, ctypes.byref(h)) == 1
    assert h.value is None


def test_invalid_dsp_sizes_rejected_without_device():
    dbp = _lib_or_skip()
    d = dbp.DspDesc(28, 25, 48, 8.0, 15, 16)
    h = ctypes.c_void_p(123)
    for n_in in (0, 2501, 10):                # not a whole number of outputs; shorter than the taps
        assert dbp.lib().dbp_dsp_create(ctypes.byref(d), n_in, ctypes.byref(h)) == 1
    d = dbp.DspDesc(3, 2, 4, 8.0, 3, 2)
    assert dbp.lib().dbp_dsp_create(ctypes.byref(d), 102, ctypes.byref(h)) == 1   # 153 outputs: odd


def _desc(**kw):
    dbp = _lib_or_skip()
    args = dict(n_samples=262144, n_spans=40, steps_per_span=1, beta2_ps2_km=siggen.beta2_ps2_km())
    args.update(kw)
    n = args.pop("n_samples")
    s = args.pop("n_spans")
    k = args.pop("steps_per_span")
    return dbp.make_desc(n, s, k, **args)


@pytest.mark.parametrize("mutate", [
    lambda d: setattr(d, "n_pol", 3),
    lambda d: setattr(d, "batch", 0),
    lambda d: setattr(d, "n_samples", 1),
    lambda d: setattr(d, "fs_thz", 0.0),
    lambda d: setattr(d, "n_spans", 0),
    lambda d: setattr(d, "steps_per_span", 0),
    lambda d: setattr(d, "span_km", -1.0),
    lambda d: setattr(d, "gamma_w_km", -1.0),
    lambda d: setattr(d, "alpha_db_km", float("nan")),
    lambda d: setattr(d, "method", 7),
    lambda d: (setattr(d, "method", 1), setattr(d, "n_taps", 4)),
    lambda d: (setattr(d, "method", 1), setattr(d, "n_taps", 9)),          # taps pointer NULL
    lambda d: setattr(d, "linear", 5),
    lambda d: (setattr(d, "linear", 1), setattr(d, "n_fir", 8)),
    lambda d: setattr(d, "precision", 9),
    lambda d: setattr(d, "flags", 0x80),
    lambda d: (setattr(d, "block", 1000), setattr(d, "overlap", 100)),     # not a power of two
    lambda d: (setattr(d, "block", 1024), setattr(d, "overlap", 255)),     # odd overlap
    lambda d: (setattr(d, "block", 1024), setattr(d, "overlap", 1024)),    # overlap >= block
    lambda d: (setattr(d, "block", 1024), setattr(d, "overlap", 256), setattr(d, "n_samples", 512)),
    lambda d: setattr(d, "steps_per_pass", -1),
    lambda d: setattr(d, "spans_per_step", -2),
    lambda d: setattr(d, "spans_per_step", 3),                            # does not divide 40 spans
    lambda d: (setattr(d, "spans_per_step", 2), setattr(d, "steps_per_span", 2)),
])
def test_invalid_descriptors_rejected_without_device(mutate):
    dbp = _lib_or_skip()
    d = _desc()
    mutate(d)
    lib = dbp.lib()
    assert lib.dbp_choose_geometry(ctypes.byref(d), None, None, None) == 1
    h = ctypes.c_void_p(123)
    assert lib.dbp_plan(ctypes.byref(d), ctypes.byref(h)) == 1     # returned before any HIP call
    assert h.value is None


def test_null_arguments():
    dbp = _lib_or_skip()
    lib = dbp.lib()
    assert lib.dbp_plan(None, None) == 1
    assert lib.dbp_backprop(None, None, None, None, None, None, 0, None) == 1
    assert lib.dbp_backprop_grad(None, None, None, None, None, None, None, None, None, 0, None) == 1
    assert lib.dbp_backprop_save(None, None, None, None, None, None, 0, None) == 1
    assert lib.dbp_backprop_grad_saved(None, None, None, None, None, None, None, None, None, None, 0, None) == 1
    assert lib.dbp_workspace_size(None, 0) == 0
    lib.dbp_destroy(None)


def test_receiver_rejects_chunks_beyond_its_ring_masks():
    # rings are indexed with 32-bit masks: a chunk above 2^29 samples is refused before
    # the planner or the device is touched
    import ctypes
    dbp = _lib_or_skip()
    d = dbp.make_desc(1 << 20, 40, 1, block=1024, overlap=256)
    h = ctypes.c_void_p()
    assert dbp.lib().dbp_rx_create(ctypes.byref(d), (1 << 29) + 768, ctypes.byref(h)) == 2
    assert h.value is None
    assert dbp.lib().dbp_rx_create(ctypes.byref(d), 0, ctypes.byref(h)) == 1


@pytest.mark.parametrize("steps_per_span,forward,m", [(1, False, 1), (20, False, 1), (7, True, 1),
                                                      (1, False, 2), (1, True, 8), (1, False, 40)])
def test_planner_schedule_matches_oracle(steps_per_span, forward, m):
    dbp = _lib_or_skip()
    d = _desc(steps_per_span=steps_per_span, forward=forward, spans_per_step=m)
    b, phi = dbp.schedule(d)
    ref = R.schedule(40, 80.0, steps_per_span, siggen.beta2_ps2_km(), 1.3, 0.2, backward=not forward,
                     spans_per_step=m)
    assert len(b) == len(ref)
    assert np.allclose(b, [s.b for s in ref], rtol=1e-15, atol=0)
    assert np.allclose(phi, [s.phi for s in ref], rtol=1e-14, atol=0)


def test_geometry_rules():
    dbp = _lib_or_skip()
    taps = siggen.symmetric_taps(siggen.rng(1, 0), 4)
    # ESSFM 1 step/span, Nb=1024, O=256: spread per side 17.1 + 4 samples, margin 16 -> k = 5
    assert dbp.choose_geometry(_desc(taps=taps, block=1024, overlap=256)) == (1024, 256, 5)
    # SSFM 20 steps/span: spread 0.855 per step -> k_max 130, balanced over 7 passes -> 115
    assert dbp.choose_geometry(_desc(steps_per_span=20, block=1024, overlap=256)) == (1024, 256, 115)
    # explicit k is kept (clamped to N_s)
    assert dbp.choose_geometry(_desc(block=1024, overlap=256, steps_per_pass=3))[2] == 3
    assert dbp.choose_geometry(_desc(block=1024, overlap=256, steps_per_pass=99))[2] == 40
    # whole signal: one block, no overlap, every step in one pass
    d = _desc(n_samples=16384, n_spans=4, n_pol=1, whole=True)
    assert dbp.choose_geometry(d) == (16384, 0, 4)
    # auto geometry covers the accumulated spread of each pass
    nb, o, k = dbp.choose_geometry(_desc(taps=taps))
    assert o // 2 >= k * (np.pi * 21.6826 * 80 * 0.056 ** 2 + 4) + 16 - 1e-9 and nb > o
    # whole-signal sizes without a kernel are refused as unsupported, not invalid
    d = _desc(n_samples=12288, whole=True)
    assert dbp.lib().dbp_choose_geometry(ctypes.byref(d), None, None, None) == 2


@pytest.mark.parametrize("band", [0.0, 0.0154])
def test_planner_fir_design_matches_oracle(band):
    dbp = _lib_or_skip()
    b2 = siggen.beta2_ps2_km()
    d = _desc(n_spans=4, steps_per_span=2, linear=dbp.LINEAR_FIR, n_fir=33, fir_band_thz=band)
    b = R.schedule(4, 80.0, 2, b2, 1.3, 0.2)[3].b
    ref = R.ls_fir_taps(33, b, siggen.FS_THZ, band) if band > 0 else R.ideal_fir_taps(33, b, siggen.FS_THZ)
    got = dbp.fir_taps(d, 3)
    assert np.max(np.abs(got - ref)) < 1e-7 * max(1.0, np.max(np.abs(ref))) + 2e-8
    with pytest.raises(dbp.DbpError):
        dbp.fir_taps(d, 8)      # step out of range

def test_split_precision_geometry_rules():
    """The matrix-core (BF16x3) variant exists for 1024-point blocks with FFT linear steps
    only; everything else is refused as unsupported before any device call."""
    dbp = _lib_or_skip()
    lib = dbp.lib()
    assert dbp.choose_geometry(_desc(precision=dbp.BF16X3))[0] == 1024
    assert dbp.choose_geometry(_desc(precision=dbp.BF16X3, block=1024, overlap=256)) == \
        dbp.choose_geometry(_desc(block=1024, overlap=256))
    for d in (_desc(precision=dbp.BF16X3, block=2048, overlap=512),
              _desc(precision=dbp.BF16X3, n_samples=2048, whole=True)):
        assert lib.dbp_choose_geometry(ctypes.byref(d), None, None, None) == 2
    d = _desc(precision=dbp.BF16X3, linear=dbp.LINEAR_FIR, n_fir=33)
    h = ctypes.c_void_p(123)
    assert lib.dbp_plan(ctypes.byref(d), ctypes.byref(h)) == 2
    assert h.value is None
    arr = (dbp.Desc * 2)(_desc(n_samples=4096, precision=dbp.BF16X3), _desc(n_samples=4096))
    assert lib.dbp_plan_batch(arr, 2, ctypes.byref(h)) == 2



def test_loss_head_validation_on_host():
    # dbp_mse_create rejects bad sizes and arguments before touching the GPU
    dbp = _lib_or_skip()
    lib = dbp.lib()
    h = ctypes.c_void_p()

    def create(n, n_pol=2, batch=1, amp=1.0, mf=None):
        m = np.ones(max(n, 1)) if mf is None else mf
        return lib.dbp_mse_create(n, n_pol, batch, m.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), amp,
                                  ctypes.byref(h))

    assert create(3000) == 1                   # not a power of two
    assert create(1024) == 2                   # below 2048
    assert create(65536) == 2                  # above 32768
    assert create(4096, n_pol=3) == 1
    assert create(4096, batch=0) == 1
    assert create(4096, amp=0.0) == 1
    bad = np.ones(4096)
    bad[7] = np.nan
    assert create(4096, mf=bad) == 1
    assert h.value is None
    assert lib.dbp_mse_forward(None, None, None, None, None) == 1
    assert lib.dbp_mse_backward(None, None, None, None) == 1
    lib.dbp_mse_destroy(None)


def test_tune_flag_is_accepted_and_host_view_is_the_model():
    # DBP_FLAG_TUNE is a valid flag; the host-only view reports the analytic model's choice
    dbp = _lib_or_skip()
    b2 = siggen.beta2_ps2_km()
    for kw in [dict(), dict(spans_per_step=2)]:
        plain = dbp.choose_geometry(dbp.make_desc(262144, 40, 1, beta2_ps2_km=b2, **kw))
        tuned = dbp.choose_geometry(dbp.make_desc(262144, 40, 1, beta2_ps2_km=b2, tune=True, **kw))
        assert plain == tuned
    # the measured cost model keeps 8192-point blocks (several times slower per sample on this
    # chip) for steps that need them: one step per two spans fits 512-1024-point blocks
    assert dbp.choose_geometry(dbp.make_desc(262144, 40, 1, beta2_ps2_km=b2, spans_per_step=2))[0] <= 1024
    assert dbp.choose_geometry(dbp.make_desc(262144, 40, 1, beta2_ps2_km=b2, spans_per_step=40,
                                             taps=np.ones(65, np.float32)))[0] == 4096
