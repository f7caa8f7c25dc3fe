"""Host logic of bench.py (no GPU): the one-GPU guard, the per-solve timing
summary, and the per-step byte model of the roofline, pinned to the output
arrays the oracle returns for a small instance (every output written once,
the reference read once)."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from bench import algorithmic_bytes_per_step, stage_bytes_per_step, timing_stats
from paper_2104_03186_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n_gpus", [2, 8])
def test_more_than_one_gpu_exits_with_a_message(n_gpus):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n_gpus)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_timing_stats():
    st = timing_stats([4.0, 1.0, 3.0, 2.0])
    assert st["mean"] == 2.5 and st["median"] == 2.5 and st["min"] == 1.0 and st["runs"] == 4
    assert 3.9 < st["p99"] <= 4.0


@pytest.mark.parametrize("n,m,p", [(4, 2, 4), (3, 1, 2), (6, 3, 5)])
def test_byte_model_matches_the_outputs_per_step(n, m, p):
    T = 12
    prob = inputs.random_problem(n, m, T, seed=5, p=p)
    out = oracle.solve(prob)
    per_step = {f: out[f][0].size for f in ("S", "v", "K", "d", "x", "u")}
    ref_bytes = 8 * prob.r[0].size
    assert prob.r.shape == (T, p)
    for osz in (8, 4):
        want = ref_bytes + osz * sum(per_step.values())
        assert algorithmic_bytes_per_step(n, m, p, osz) == want
        backward = ref_bytes + osz * sum(per_step[f] for f in ("S", "v", "K", "d"))
        assert stage_bytes_per_step("bwd_final", n, m, p, osz) == backward
        forward = osz * sum(per_step[f] for f in ("K", "d", "x", "u"))
        assert stage_bytes_per_step("fwd_final", n, m, p, osz) == forward
    assert stage_bytes_per_step("bwd_final", 4, 2, 4) == 272
    assert np.isclose(algorithmic_bytes_per_step(4, 2, 4), 320)
