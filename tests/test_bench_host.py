"""Host-side logic of bench.py (no GPU): the sets of its LP measurement."""
def test_bench_lp_sets_conjunction_and_polytope():
    # the LP bench's sets: every output row's finite interval ends become
    # halfspaces of one conjunction, and the generator box is cut by
    # sum_j (z_j - zc_j) / r_j <= d / 2
    import math
    import numpy as np
    import bench
    import workloads as W
    p = W.random_symmetric(n=50, k=5, steps=3, ngen=2, o=2, seed=1)
    p.unsafe = np.array([[0.2, math.inf], [-math.inf, 0.7]])
    G, h, U, u = bench.lp_sets(p)
    zc = np.array([g.zc for g in p.gens]); r = np.array([g.radius for g in p.gens])
    np.testing.assert_allclose(G[0], 1.0 / r)
    np.testing.assert_allclose(h[0], float(G[0] @ zc) + 1.0)
    np.testing.assert_array_equal(U, [[-1.0, 0.0], [0.0, 1.0]])
    np.testing.assert_array_equal(u, [-0.2, 0.7])
