"""Host-side pieces of the coefficient fit: the fold of tap gradients onto the symmetric
coefficients is the adjoint of the map c -> w(c), for shared and per-step coefficients."""
import numpy as np

from paper_1507_00921_amd import fit as G


def test_symmetric_full_layout():
    assert np.array_equal(G.symmetric_full([1.0, 0.5, 0.25]), np.float32([0.25, 0.5, 1.0, 0.5, 0.25]))


def test_fold_is_adjoint_of_tap_map_shared():
    # <fold(g), c> = <g, [w(c)] * N_s> for every g and c
    r = np.random.default_rng(3)
    g = r.standard_normal((6, 9))
    c = r.standard_normal(5)
    lhs = float(G.fold_symmetric(g) @ c)
    rhs = float(np.sum(g * np.tile(np.concatenate([c[:0:-1], c]), (6, 1))))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_fold_is_adjoint_of_tap_map_per_step():
    r = np.random.default_rng(4)
    g = r.standard_normal((4, 7))
    c = r.standard_normal((4, 4))
    w = np.stack([np.concatenate([ci[:0:-1], ci]) for ci in c])
    f = G.fold_symmetric(g, per_step=True)
    assert f.shape == (16,)
    assert abs(float(f @ c.ravel()) - float(np.sum(g * w))) <= 1e-12 * float(np.sum(np.abs(g * w)))
    # summing the per-step folds gives the shared fold
    assert np.allclose(f.reshape(4, 4).sum(axis=0), G.fold_symmetric(g))
