"""Pins of the FP64 network reference (CPU): its analytic gradient against
central finite differences of its own loss, and the feature encoding against
hand-computed values for one plane, one edge and one paraboloid."""
import numpy as np

from oracle import mlp_ref as R
from paper_2301_06399_amd import workloads as W


def small_params(rng, scale=0.2):
    flat = rng.normal(0, scale, R.NPAR)
    P = R.unpack(flat)
    P["W4"][15] = 0.0
    P["b4"][15] = 0.0
    return P


def test_reference_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    P = small_params(rng)
    X = rng.normal(size=(7, R.F_IN))
    T = rng.normal(size=(7, R.F_OUTP))
    mask = (rng.random((7, R.F_OUTP)) < 0.7).astype(float)
    mask[:, 15] = 0
    loss, G, _ = R.loss_and_grad(P, X, T, mask)
    for name, idx in [("W1", (3, 5)), ("W1", (200, 90)), ("b1", (7,)), ("W2", (10, 20)), ("b2", (100,)),
                      ("W3", (255, 0)), ("b3", (3,)), ("W4", (2, 17)), ("b4", (4,))]:
        h = 1e-6
        Pp = {k: v.copy() for k, v in P.items()}
        Pm = {k: v.copy() for k, v in P.items()}
        Pp[name][idx] += h
        Pm[name][idx] -= h
        fd = (R.loss_and_grad(Pp, X, T, mask)[0] - R.loss_and_grad(Pm, X, T, mask)[0]) / (2 * h)
        assert abs(fd - G[name][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, G[name][idx])


def test_bf16_rounding_is_round_to_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0], np.float64)
    r = R.bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0            # exactly halfway: ties to even (mantissa 0)
    assert r[2] == 1.0 + 2 ** -7  # above halfway rounds up
    assert r[3] == -2.5 and r[4] == 0.0


def test_feature_encoding_by_hand():
    sc = W.Scene(tx=np.array([1.0, 2.0, 3.0]),
                 planes=np.array([W.plane_rect([0, 0, 1], 0.0, [0, 0, 0], [10, 0, 0], [0, 10, 0])]),
                 lines=np.array([W.line_seg([0, 0, 0], [0, 1, 0], 0, 5)]),
                 quadrics=np.array([W.paraboloid([4, 2, 3], [0, 0, 1], 2.0)]),
                 aabb_lo=np.zeros(3), aabb_hi=np.full(3, 10.0))
    b = W.Batch(np.array([[4.0, 6.0, 3.0]]), np.array([0]), np.array([3]), np.array([[0], [1], [2], [-1], [-1]]))
    F = R.features(sc, b)[0]
    L = 5.0  # |RX - TX| = |(3, 4, 0)|
    np.testing.assert_allclose(F[0:6], [3 / L, 4 / L, 0, 0, 0, 0])
    # plane z = 0: type 0, n, (d - n.TX)/L = -3/5
    np.testing.assert_allclose(F[6:11], [1, 0, 0, 0, 0])
    np.testing.assert_allclose(F[10:14], [0, 0, 1, -0.6])
    assert F[22] == 1.0
    # edge along y through the origin: nearest point to TX is (0, 2, 0)
    s = 6 + 17
    assert F[s + 1] == 1.0
    np.testing.assert_allclose(F[s + 4:s + 10], [0, 1, 0, -1 / L, 0, -3 / L])
    # paraboloid vertex (4,2,3), axis z, F = 2: anchor (3,0,0)/L, L*A, b = -axis
    s = 6 + 34
    assert F[s + 2] == 1.0
    np.testing.assert_allclose(F[s + 4:s + 7], [3 / L, 0, 0])
    np.testing.assert_allclose(F[s + 7:s + 13], L * np.array([1 / 8, 0, 0, 1 / 8, 0, 0]))
    np.testing.assert_allclose(F[s + 13:s + 16], [0, 0, -1])
    assert (F[6 + 51:] == 0).all()
