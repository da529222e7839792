"""Adaptive time-step driver of the oracle (Section 4, eq. (sencondt) and the retry rule).

The step-size sequence is parity unpinned against the paper (it prints no
history); these tests check the written rule: prediction, retry by 1/sqrt(2)
with zeta doubled, persistence of the doubled zeta, and that a failed attempt
leaves the state untouched.
"""

import math

import numpy as np

from oracle import Oracle, predict_dt
from paper_2209_08001_amd import workloads as W


def test_predict_dt_formula_limits():
    assert predict_dt(0.0, 1e-3, 1.0, 100.0) == 1.0
    assert predict_dt(1e9, 1e-3, 1.0, 100.0) == 1e-3
    r = 0.05
    assert abs(predict_dt(r, 1e-3, 1.0, 100.0) - 1.0 / math.sqrt(1 + 100 * r * r)) < 1e-15


def test_retry_rule_and_state_untouched():
    n = (8, 8)
    c0, e0 = W.init_fields(n, 1)
    o = Oracle(n, W.H, W.DEFAULT_MODEL, c0, e0)
    tried = []

    def hook(step, dt):
        tried.append((step, dt))
        return step == 1 and len([t for t in tried if t[0] == 1]) <= 2

    log = o.advance(3, 1e-3, 1.0, 100.0, fail_hook=hook)
    assert log[0]["dt"] == 1e-3 and log[0]["retries"] == 0
    assert log[1]["retries"] == 2
    first_try = [t[1] for t in tried if t[0] == 1]
    assert abs(first_try[1] - first_try[0] / math.sqrt(2)) < 1e-15
    assert abs(first_try[2] - first_try[0] / 2) < 1e-15
    assert log[1]["zeta"] == 400.0 and log[2]["zeta"] == 400.0
    # the prediction for step 2 uses the doubled zeta
    rate = log[1]["dx_rms"] / log[1]["dt"]
    assert abs(log[2]["dt"] - predict_dt(rate, 1e-3, 1.0, 400.0)) < 1e-15
    assert abs(o.t - sum(r["dt"] for r in log)) < 1e-15
