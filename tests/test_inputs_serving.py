"""The served contour sweep: 256 requests on 8 circles |k - c| = 0.5 (32 nodes
each), c uniform in [2, 20], star boundaries with N from {512, 1024, 2048,
4096}, interior index 1.5, 16 probing right-hand sides, Poisson arrivals."""
import numpy as np

from paper_2512_14193_amd import inputs as I


def test_serving_workload_shape_and_determinism():
    w = I.serving_workload()
    assert len(w.requests) == 256 and w.n_rhs == 16 and w.nodes_per_contour == 32
    assert np.all((w.centers >= 2.0) & (w.centers <= 20.0))
    assert set(int(n) for n in w.sizes) <= {512, 1024, 2048, 4096}
    pairs = {(r.contour, r.node) for r in w.requests}
    assert len(pairs) == 256  # every node of every contour exactly once
    for r in w.requests:
        c = w.centers[r.contour]
        assert abs(abs(r.physics.k0 - c) - 0.5) < 1e-12
        assert abs(r.physics.k1 - 1.5 * r.physics.k0) < 1e-12
        assert abs(r.physics.eps1 - 2.25) < 1e-12 and r.physics.eps0 == 1.0
        assert abs(r.physics.beta - 1j / r.physics.k0) < 1e-15
        # inside the wavenumber sector the device Hankel functions cover
        for k in (r.physics.k0, r.physics.k1):
            assert k.real > 0 and abs(k.imag) <= 0.5 * k.real
        assert r.n_nodes == int(w.sizes[r.contour])
    assert len({r.rhs_seed for r in w.requests}) == 256
    w2 = I.serving_workload()
    assert [(r.contour, r.node, r.arrival) for r in w.requests] == [(r.contour, r.node, r.arrival) for r in w2.requests]


def test_serving_arrivals_are_poisson():
    w = I.serving_workload(n_contours=64, rate=50.0)  # 2048 arrivals
    t = np.array([r.arrival for r in w.requests])
    gaps = np.diff(t)
    assert t[0] == 0.0 and np.all(gaps >= 0)
    m = gaps.mean()
    assert abs(m - 1 / 50.0) < 4 * (1 / 50.0) / np.sqrt(gaps.size)  # mean gap 1/rate (4 sigma)
    # exponential: coefficient of variation 1, P(gap > mean) = 1/e
    assert abs(gaps.std() / m - 1.0) < 0.1
    assert abs(np.mean(gaps > 1 / 50.0) - np.exp(-1)) < 0.05


def test_contour_nodes():
    k = I.contour_nodes(5.0 + 1.0j, 0.5, 32)
    assert np.allclose(np.abs(k - (5.0 + 1.0j)), 0.5)
    assert abs(k.mean() - (5.0 + 1.0j)) < 1e-14  # symmetric trapezoid nodes
