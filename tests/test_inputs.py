"""The seeded input generators: determinism, shapes and the stated recipe."""
import numpy as np

from paper_2104_03186_amd import inputs


def test_tracking_problem_recipe():
    a = inputs.tracking_problem(n=4, m=2, T=1000)
    b = inputs.tracking_problem(n=4, m=2, T=1000)
    for f in ("F", "L", "r", "rT", "x0"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    assert np.max(np.abs(np.linalg.eigvals(a.F))) == np.float64(np.max(np.abs(np.linalg.eigvals(a.F))))
    assert abs(np.max(np.abs(np.linalg.eigvals(a.F))) - 0.99) < 1e-12
    assert a.r.shape == (1000, 4) and a.rT.shape == (4,)
    assert np.array_equal(a.X, 10 * np.eye(4)) and np.array_equal(a.U, 0.1 * np.eye(2))
    assert np.array_equal(a.XT, 10 * np.eye(4)) and a.c is None
    # period-200 sinusoid
    assert np.allclose(a.r[0], a.r[200]) and np.allclose(a.r[1], a.r[201])


def test_prefix_stability_across_horizons():
    # the T = 1e4 instance shares dynamics with T = 1e3 (same seed stream order)
    a = inputs.tracking_problem(n=4, m=2, T=1000, workload=1)
    b = inputs.tracking_problem(n=4, m=2, T=10000, workload=1)
    assert np.array_equal(a.F, b.F) and np.array_equal(a.L, b.L)
    assert np.array_equal(a.r, b.r[:1000])


def test_batched_shapes_distribution():
    sh = inputs.batched_shapes(4096)
    ns = np.array([s[0] for s in sh])
    Ts = np.array([s[1] for s in sh])
    assert set(ns.tolist()) == {4, 8, 16}
    assert Ts.min() >= 256 and Ts.max() <= 16384
    assert 3000 < Ts.mean() < 4800
    assert sh == inputs.batched_shapes(4096)


def test_dense_problem_spd():
    p = inputs.dense_problem(n=16, m=8, T=4)
    assert np.min(np.linalg.eigvalsh(p.X)) > 0.09 and np.min(np.linalg.eigvalsh(p.U)) > 0.09
    assert abs(np.max(np.abs(np.linalg.eigvals(p.F))) - 0.98) < 1e-12


def test_serving_stream():
    reqs = inputs.serving_requests(rate_hz=2000.0, seconds=1.0)
    assert 1800 < len(reqs) < 2200
    assert all(4 <= n <= 32 and m == (n + 1) // 2 and 64 <= T <= 65536 for _, n, m, T in reqs)


def test_prefix_problem_is_the_first_steps():
    import oracle

    full = inputs.random_problem(3, 2, 40, seed=4, per_step=1 | 2)
    sub = inputs.prefix_problem(full, 25)
    assert sub.T == 25 and sub.F.shape[0] == 25 and sub.r.shape[0] == 25
    assert np.array_equal(sub.F, full.F[:25]) and np.array_equal(sub.rT, full.rT)
    # its solution is that of a 25-step instance, not a slice of the 40-step one
    assert oracle.solve(sub)["x"].shape == (26, 3)
