"""Write fitted_taps_headline.json: ESSFM coefficients for the headline link fitted by the
oracle alone (FP64 least squares of Sec. IV) at the bench's operating point.

Field: the 2 x 262144 PM-QPSK headline field launched at +4 dBm, propagated by the
oracle's forward channel (2 steps per span) plus ASE (tests/gpu_inputs.received).
Target: SSFM with 20 steps per span on the same overlap-and-save blocks (Nb = 1024,
O = 256, 115 steps per pass).  Fit: the N_c + 1 = 5 symmetric coefficients shared by all
40 steps of ESSFM (Nb = 1024, O = 256, 5 steps per pass) minimizing the squared
difference on samples 1024..99999, as Sec. IV fits on the first part of the samples.

    python tests/golden/make_fitted_taps.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import siggen  # noqa: E402
from oracle import dbp_ref as R  # noqa: E402
from oracle import fit as F  # noqa: E402
from gpu_inputs import B2, FS, received  # noqa: E402

N, SPANS, P_DBM, NC = 262144, 40, 4.0, 4


def main():
    t0 = time.time()
    rx, _ = received(1, 0, 2, N, P_DBM, SPANS, 2)
    ssfm = R.schedule(SPANS, 80.0, 20, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM)
    target = R.run_blocked(rx, ssfm, FS, 1024, 256, 115)
    base = R.schedule(SPANS, 80.0, 1, B2, siggen.GAMMA_W_KM, siggen.ALPHA_DB_KM)
    c = F.fit_coefficients(rx, target, base, FS, 1024, 256, 5, NC, slice(1024, 100000))
    out = {
        "_source": "written by tests/golden/make_fitted_taps.py from oracle/ only (FP64 least squares, Sec. IV)",
        "field": "headline 2x262144 PM-QPSK, +4 dBm, 40x80 km, oracle forward channel 2 steps/span, "
                 "ASE 20 dB OSNR at 0 dBm (tests/gpu_inputs.received(1, 0, 2, 262144, 4.0, 40, 2))",
        "target": "SSFM 20 steps/span, Nb 1024, O 256, 115 steps per pass",
        "fit": "c_0..c_4 shared by all 40 ESSFM steps (Nb 1024, O 256, 5 steps per pass), samples 1024..99999",
        "p_dbm": P_DBM, "n_c": NC,
        "c": [float(v) for v in c],
        "taps": [float(v) for v in F.symmetric_full(c)],
    }
    with open(os.path.join(HERE, "fitted_taps_headline.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(f"c = {np.round(c, 6).tolist()} in {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
