"""The operation-count model against the numbers printed in the paper (CPU)."""
import json
import math
import os

import numpy as np

from oracle import complexity as C

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def test_printed_total_multiplications():
    g = GOLD["total_mults_per_sample"]
    n, m = 8192, 1024
    assert round(C.ffe_mults_per_sample(n, m)) == g["ffe"]
    assert round(C.total_mults(1, n, m, 32)) == g["essfm_1step_nc32"]
    assert round(C.total_mults(16, n, m)) == g["ssfm_16step"]
    assert round(C.total_mults(20, n, m)) == g["ssfm_20step"]


def test_printed_reduction_factors():
    n, m = 8192, 1024
    ratio = C.total_mults(20, n, m) / C.total_mults(1, n, m, 32)
    assert round(ratio) == GOLD["complexity_reduction_essfm1_vs_ssfm20"]["value"]
    # latency model: cascaded FFT pairs, one per step
    assert 20 // 1 == GOLD["latency_reduction_essfm1_vs_ssfm20"]["value"]


def test_per_step_increase_at_2000_km():
    g = GOLD["per_step_increase_at_2000km"]
    m = C.channel_memory(21.0, 2000.0, 0.05)
    n = 8 * m
    e = C.essfm_mults_per_sample(n, m, 32)
    s = C.ssfm_mults_per_sample(n, m)
    f = C.ffe_mults_per_sample(n, m)
    assert abs((e / s - 1) - g["essfm_vs_ssfm"]) < 0.03
    assert abs((e / f - 1) - g["essfm_vs_ffe"]) < 0.03
    # "slightly increase at shorter distances, decrease with fewer coefficients"
    m2 = C.channel_memory(21.0, 500.0, 0.05)
    assert C.essfm_mults_per_sample(8 * m2, m2, 32) / C.ssfm_mults_per_sample(8 * m2, m2) > e / s
    assert C.essfm_mults_per_sample(n, m, 8) / s < e / s


def test_memory_examples():
    ex = GOLD["memory_example"]
    mm = C.channel_memory(ex["beta2_ps2_km"], ex["length_km"], ex["bandwidth_thz"])
    assert abs(mm - ex["M"]) / ex["M"] < 0.05
    e2 = GOLD["experiment_memory"]
    mm = C.channel_memory(21.0, e2["length_km"], 0.05)
    assert abs(mm - e2["M"]) / e2["M"] < 0.05
    assert 2 ** round(math.log2(8 * mm)) == e2["N"]


def test_block_rule_near_minimum():
    # N = 8M is within a few percent of the minimum over N/M for every algorithm (Fig. 1)
    m = 1024.0
    r = np.linspace(1.5, 64, 2000)
    for fun in [lambda n: C.ffe_mults_per_sample(n, m),
                lambda n: C.ssfm_mults_per_sample(n, m),
                lambda n: C.essfm_mults_per_sample(n, m, 32)]:
        vals = np.array([fun(ri * m) for ri in r])
        assert fun(GOLD["block_rule"]["n_over_m"] * m) / vals.min() < 1.03
        assert fun(2 * m) / vals.min() > 1.15      # shorter blocks cost significantly more
