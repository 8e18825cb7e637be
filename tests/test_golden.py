"""The workloads reuse the parameter values the paper prints."""
import json
import os

import sde_inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load():
    with open(os.path.join(GOLDEN, "paper_parameters.json")) as f:
        return json.load(f)


def test_single_point_uses_fig2_parameters():
    g = _load()["fig2_josephson"]
    p = sde_inputs.jj_single()[0]
    for k_ours, k_paper in [("a", "a"), ("gamma", "gamma"), ("omega", "omega"), ("D", "D0"),
                            ("f", "f")]:
        assert p[k_ours] == g[k_paper]


def test_table1_total():
    t = _load()["table1_flops_per_step"]
    assert sum(c * w for c, _, w in t["rows"]) == t["total"]
    r = _load()["reported_rates"]
    assert abs(r["prog1_steps_per_s"] * t["total"] / 1e9 - r["prog1_gflops"]) < 2.5  # 488 rounds to the printed 490
