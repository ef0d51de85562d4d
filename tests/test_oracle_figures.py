"""The regenerated complexity curves of Figs. 1 and 2 (tests/golden/complexity_curves.json,
written by oracle/figures.py) and the shapes the text states for them (CPU)."""
import json
import os

import numpy as np

from oracle import figures as FG

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "complexity_curves.json")))


def test_stored_curves_match_the_model():
    now = FG.curves()
    for fig in ("fig1_m1024", "fig2_n8m_beta2_21_50ghz"):
        for key, vals in GOLD[fig].items():
            assert np.allclose(vals, now[fig][key], rtol=1e-12), (fig, key)


def test_fig1_shape():
    # every curve falls steeply from N = 1.5M, is within 3 % of its minimum at N = 8M and
    # rises only slowly beyond; ESSFM above SSFM above FFE everywhere
    f = GOLD["fig1_m1024"]
    i8 = f["n_over_m"].index(8)
    for key in ("ffe", "ssfm_step", "essfm_step_nc32"):
        v = np.array(f[key])
        assert v[0] > 1.5 * v.min()
        assert v[i8] < 1.03 * v.min()
        assert v[-1] < 1.2 * v[i8]
    assert np.all(np.array(f["essfm_step_nc32"]) > np.array(f["ssfm_step"]))
    assert np.all(np.array(f["ssfm_step"]) > np.array(f["ffe"]))


def test_fig2_shape():
    # the ESSFM overhead per step over SSFM and FFE shrinks with distance and with fewer
    # coefficients; about +25 % / +40 % at 2000 km for N_c = 32
    f = GOLD["fig2_n8m_beta2_21_50ghz"]
    e, s, ffe = (np.array(f[k]) for k in ("essfm_step_nc32", "ssfm_step", "ffe"))
    assert np.all(np.diff(e / s) < 0) and np.all(np.diff(e / ffe) < 0)
    i = f["length_km"].index(2000)
    assert abs(e[i] / s[i] - 1.25) < 0.03 and abs(e[i] / ffe[i] - 1.40) < 0.03
    for a, b in ((4, 8), (8, 16), (16, 32)):
        assert np.all(np.array(f[f"essfm_step_nc{a}"]) < np.array(f[f"essfm_step_nc{b}"]))
