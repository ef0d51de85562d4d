"""The complexity curves of Figs. 1 and 2 (Sec. III) from the operation-count model
(TEST INFRASTRUCTURE ONLY: see oracle/__init__).  The figures themselves are not available;
their axes and parameters are given in their captions and the text.

Fig. 1: real multiplications per received sample for the FFE, one SSFM step and one ESSFM
step (N_c = 32) against the block length ratio N/M, for a channel memory M = 1024 samples.
Fig. 2: the same for N = 8M against the link length, beta2 = 21 ps^2/km and a 50 GHz
signal (M = 2 pi |beta2| L B^2), ESSFM with several N_c.

Running this module writes tests/golden/complexity_curves.json.
"""
from __future__ import annotations

import json
import os

from . import complexity as C

FIG1_RATIOS = [1.5, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64]
FIG2_LENGTHS_KM = [250, 500, 1000, 1500, 2000, 3000, 4000, 6000, 8000, 10000]
FIG2_NC = [4, 8, 16, 32]


def fig1(m: float = 1024.0, n_c: int = 32, ratios=FIG1_RATIOS) -> dict:
    return {"n_over_m": list(ratios),
            "ffe": [C.ffe_mults_per_sample(r * m, m) for r in ratios],
            "ssfm_step": [C.ssfm_mults_per_sample(r * m, m) for r in ratios],
            f"essfm_step_nc{n_c}": [C.essfm_mults_per_sample(r * m, m, n_c) for r in ratios]}


def fig2(beta2: float = 21.0, band_thz: float = 0.05, lengths=FIG2_LENGTHS_KM, ncs=FIG2_NC) -> dict:
    out = {"length_km": list(lengths), "memory": [], "ffe": [], "ssfm_step": []}
    for nc in ncs:
        out[f"essfm_step_nc{nc}"] = []
    for length in lengths:
        m = C.channel_memory(beta2, length, band_thz)
        n = 8.0 * m
        out["memory"].append(m)
        out["ffe"].append(C.ffe_mults_per_sample(n, m))
        out["ssfm_step"].append(C.ssfm_mults_per_sample(n, m))
        for nc in ncs:
            out[f"essfm_step_nc{nc}"].append(C.essfm_mults_per_sample(n, m, nc))
    return out


def curves() -> dict:
    return {"_source": "oracle/figures.py (operation counts of Sec. III; Figs. 1 and 2)",
            "fig1_m1024": fig1(), "fig2_n8m_beta2_21_50ghz": fig2()}


if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden",
                        "complexity_curves.json")
    with open(path, "w") as f:
        json.dump(curves(), f, indent=1)
    print("wrote", path)
