"""Pins of the oracle's adjoint: central finite differences and the dot-product test (CPU)."""
import numpy as np
import pytest

import siggen
from oracle import adjoint as A
from oracle import dbp_ref as R

FS = siggen.FS_THZ
B2 = siggen.beta2_ps2_km()


def _loss(z, wt):
    """A generic real loss: Re <wt, z> + 0.5 |z|^4 summed (non-quadratic, touches every sample)."""
    return float(np.real(np.vdot(wt, z)) + 0.5 * np.sum(np.abs(z) ** 4))


def _loss_grad(z, wt):
    # d/dz* convention: g = dL/dRe + j dL/dIm
    return wt + 2.0 * np.abs(z) ** 2 * z


def _setup(seed, n=256, fir=False, k_steps=3):
    g = np.random.default_rng(seed)
    x = (g.standard_normal((2, n)) + 1j * g.standard_normal((2, n))) * 0.05
    steps = []
    for s in range(k_steps):
        w = g.uniform(0.0, 1.0, 5)
        h = (g.standard_normal(7) + 1j * g.standard_normal(7)) / 4 if fir else None
        steps.append(R.Step(b=-600.0 * (1 + 0.3 * s), phi=-40.0 + 5 * s, w=w, h=h))
    wt = (g.standard_normal((2, n)) + 1j * g.standard_normal((2, n)))
    return x, steps, wt


def _fd(fun, h=1e-3):
    """Central difference at h = 1e-3, Richardson-extrapolated with h/2 (error O(h^4))."""
    d1 = (fun(h) - fun(-h)) / (2 * h)
    d2 = (fun(h / 2) - fun(-h / 2)) / h
    return (4 * d2 - d1) / 3


@pytest.mark.parametrize("fir", [False, True])
def test_whole_gradient_matches_central_differences(fir):
    x, steps, wt = _setup(1, fir=fir)
    z = R.run_whole(x, steps, FS)
    gr = A.grad_whole(x, steps, FS, _loss_grad(z, wt))
    scale = 1e-3
    for (p, n) in [(0, 3), (1, 100), (0, 255)]:
        for unit in [1.0, 1j]:
            def f(hh):
                xx = x.copy()
                xx[p, n] += unit * hh * scale
                return _loss(R.run_whole(xx, steps, FS), wt)
            fd = _fd(f) / scale
            an = np.real(np.conj(unit) * gr.x[p, n])
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (p, n, unit, fd, an)
    for s in range(len(steps)):
        for m in range(5):
            def f(hh):
                st = [R.Step(q.b, q.phi, None if q.w is None else q.w.copy(), q.h) for q in steps]
                st[s].w[m] += hh
                return _loss(R.run_whole(x, st, FS), wt)
            fd = _fd(f)
            assert abs(fd - gr.w[s][m]) <= 1e-6 * max(1.0, abs(fd)), (s, m, fd, gr.w[s][m])
        if fir:
            for m in [0, 3, 6]:
                for unit in [1.0, 1j]:
                    def f(hh):
                        st = [R.Step(q.b, q.phi, q.w, q.h.copy()) for q in steps]
                        st[s].h[m] += unit * hh
                        return _loss(R.run_whole(x, st, FS), wt)
                    fd = _fd(f)
                    an = np.real(np.conj(unit) * gr.h[s][m])
                    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (s, m, unit, fd, an)


def test_blocked_gradient_matches_central_differences():
    x, steps, wt = _setup(2, n=600, k_steps=4)
    nb, o, k = 128, 32, 2
    z = R.run_blocked(x, steps, FS, nb, o, k)
    gr = A.grad_blocked(x, steps, FS, nb, o, k, _loss_grad(z, wt))
    scale = 1e-3
    for (p, n) in [(0, 0), (1, 95), (0, 96), (1, 599), (0, 300)]:
        for unit in [1.0, 1j]:
            def f(hh):
                xx = x.copy()
                xx[p, n] += unit * hh * scale
                return _loss(R.run_blocked(xx, steps, FS, nb, o, k), wt)
            fd = _fd(f) / scale
            an = np.real(np.conj(unit) * gr.x[p, n])
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (p, n, unit, fd, an)
    for s in range(4):
        for m in [0, 2, 4]:
            def f(hh):
                st = [R.Step(q.b, q.phi, q.w.copy()) for q in steps]
                st[s].w[m] += hh
                return _loss(R.run_blocked(x, st, FS, nb, o, k), wt)
            fd = _fd(f)
            assert abs(fd - gr.w[s][m]) <= 1e-6 * max(1.0, abs(fd)), (s, m, fd, gr.w[s][m])


def test_dot_product_linear_cascade():
    # gamma = 0 makes the cascade C-linear: <F v, w> = <v, F^H w> to rounding
    g = np.random.default_rng(3)
    v = g.standard_normal((2, 512)) + 1j * g.standard_normal((2, 512))
    w = g.standard_normal((2, 512)) + 1j * g.standard_normal((2, 512))
    steps = [R.Step(b=-900.0, phi=0.0), R.Step(b=300.0, phi=0.0, h=np.array([0.1, 1.0, 0.2j]))]
    for blocked in [False, True]:
        if blocked:
            fv = R.run_blocked(v, steps, FS, 128, 32, 1)
            ftw = A.grad_blocked(v, steps, FS, 128, 32, 1, w).x
        else:
            fv = R.run_whole(v, steps, FS)
            ftw = A.grad_whole(v, steps, FS, w).x
        lhs = np.vdot(w, fv)
        rhs = np.vdot(ftw, v)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_symbol_mse_gradient():
    sym = siggen.qpsk_symbols(siggen.rng(91, 0), 2, 128)
    p = siggen.dbm_to_w(0.0)
    z = siggen.set_power(siggen.shape(sym), p)
    g = np.random.default_rng(4)
    z = z + 1e-3 * (g.standard_normal(z.shape) + 1j * g.standard_normal(z.shape))
    mf = siggen.rrc_response(256)
    loss, gz = A.symbol_mse(z, sym, p, mf)
    assert loss < 1e-2
    for (pp, n) in [(0, 1), (1, 77)]:
        for unit in [1.0, 1j]:
            def f(hh):
                zz = z.copy()
                zz[pp, n] += unit * hh * 1e-4
                return A.symbol_mse(zz, sym, p, mf)[0]
            fd = _fd(f) / 1e-4
            an = np.real(np.conj(unit) * gz[pp, n])
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
