"""GPU ESSFM coefficient fit (Sec. IV) through the library's adjoint, against the oracle's
FP64 least-squares fit of the same blocked cascade.

Both fits see the same complex64-rounded received field and the same target, computed by
the oracle in FP64 (a 20-steps-per-span SSFM, or an ESSFM with known coefficients).  The
GPU objective and gradient are FP32 forward and reverse passes; the fitted coefficients
agree with the oracle's to 1e-4 and the objectives to 1e-4 relative.
"""
import numpy as np
import pytest

import siggen
from oracle import dbp_ref as R
from oracle import fit as F

from gpu_inputs import B2, FS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dbp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1507_00921_amd as m
    m.lib()
    return m


def _field(n=4096, p_dbm=4.0, n_spans=4):
    x, _ = siggen.transmitted_field(5, 0, 2, n, p_dbm)
    fwd = R.schedule(n_spans, 80.0, 4, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM, backward=False)
    return R.run_whole(x, fwd, FS).astype(np.complex64).astype(np.complex128)


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).reshape(1, *a.shape).cuda()


def _gpu_fit(dbp, rx, target, n_c, k, sl):
    from paper_1507_00921_amd import fit as G
    c_start = np.zeros(n_c + 1)
    c_start[0] = 1.0
    p = dbp.plan(rx.shape[-1], 4, 1, taps=G.symmetric_full(c_start), block=1024, overlap=256, steps_per_pass=k,
                 beta2_ps2_km=B2)
    return G.fit_coefficients(p, _gpu(rx), n_c, target=_gpu(target), sl=sl)


def test_gpu_fit_recovers_known_coefficients(dbp):
    rx = _field()
    base = R.schedule(4, 80.0, 1, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM)
    c_true = np.array([0.62, 0.15, 0.04])
    target = F.essfm_blocked(rx, base, c_true, FS, 1024, 256, 2)
    c, info = _gpu_fit(dbp, rx, target, 2, 2, slice(1024, 3072))
    print("recovered", c, info)
    assert np.max(np.abs(c - c_true)) < 1e-4


def test_gpu_fit_matches_oracle_fit_to_multistep_ssfm(dbp):
    rx = _field()
    fine = R.schedule(4, 80.0, 20, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM)
    target = R.run_blocked(rx, fine, FS, 1024, 256, 20)
    base = R.schedule(4, 80.0, 1, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM)
    sl = slice(1024, 3072)
    c_ref = F.fit_coefficients(rx, target, base, FS, 1024, 256, 1, 2, sl)
    obj_ref = float(np.sum(F.residual(c_ref, rx, target, base, FS, 1024, 256, 1, sl) ** 2))
    c, info = _gpu_fit(dbp, rx, target, 2, 1, sl)
    obj = float(np.sum(F.residual(c, rx, target, base, FS, 1024, 256, 1, sl) ** 2))
    print("oracle", c_ref, obj_ref, "gpu", c, obj, info)
    assert np.max(np.abs(c - c_ref)) < 1e-4
    assert abs(obj - obj_ref) <= 1e-4 * obj_ref


def test_gpu_fit_per_step_recovers_known_coefficients(dbp):
    # one coefficient set per step: the target is the oracle's blocked ESSFM with four
    # different symmetric filters, and the per-step fit recovers each of them
    from paper_1507_00921_amd import fit as G
    rx = _field()
    base = R.schedule(4, 80.0, 1, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM)
    c_true = np.array([[0.70, 0.12, 0.03], [0.58, 0.18, 0.03], [0.64, 0.14, 0.04], [0.55, 0.20, 0.025]])
    steps = [R.Step(b=st.b, phi=st.phi, w=F.symmetric_full(c_true[s])) for s, st in enumerate(base)]
    target = R.run_blocked(rx, steps, FS, 1024, 256, 2)
    p = dbp.plan(rx.shape[-1], 4, 1, taps=G.symmetric_full([1.0, 0.0, 0.0]), block=1024, overlap=256,
                 steps_per_pass=2, beta2_ps2_km=B2)
    c, info = G.fit_coefficients(p, _gpu(rx), 2, target=_gpu(target), sl=slice(1024, 3072), per_step=True,
                                 maxiter=200)
    print("recovered", c, info)
    assert c.shape == (4, 3)
    assert np.max(np.abs(c - c_true)) < 1e-3
    assert info["objective"] < 1e-6 * info["objective_start"]
