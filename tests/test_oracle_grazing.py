"""Pin of the acceptance rule for grazing reflections (Sec. II: the
reflection law; acceptance in Alg. 1).

A path TX -> corner edge -> the wall between two corners -> the other corner
-> RX, with both corners on the wall, is solved by a whole segment of
points: the ray runs along the wall, where the reflection law leaves it
unchanged, so the reflection point can sit anywhere between the corners.
Such a root is not isolated (the Jacobian is singular there) and its point
is not determined; acceptance rejects it.
"""
import numpy as np

import oracle as O
from paper_2301_06399_amd import workloads as W


def corner_wall_scene():
    wall = W.plane_rect([0, 1, 0], 0.0, [0, 0, 0], [10, 0, 0], [0, 0, 5])
    lines = np.stack([W.line_seg([10, 0, 0], [0, 0, 1], 0.0, 5.0), W.line_seg([0, 0, 0], [0, 0, 1], 0.0, 5.0)])
    return W.Scene(tx=np.array([15.0, -5.0, 1.0]), planes=wall[None, :], lines=lines,
                   aabb_lo=np.array([-10.0, -10.0, 0.0]), aabb_hi=np.array([20.0, 10.0, 5.0]))


def test_grazing_continuum_is_not_accepted():
    sc = corner_wall_scene()
    rx = np.array([-5.0, -5.0, 1.0])
    ids = [1, 0, 2]  # corner x = 10, the wall y = 0, corner x = 0
    # every point of the wall between the corners at z = 1 is a root
    for x2 in (2.0, 5.0, 8.5):
        X = np.array([10.0, 0, 1, x2, 0, 1, 0, 0, 1])
        R, J = O.residual(sc, rx, ids, X)
        assert np.abs(R).max() < 1e-12
        s = np.linalg.svd(J, compute_uv=False)
        assert s[-1] < 1e-9 * s[0]
        assert not O.accept_one(sc, rx, ids, X, O.CONVERGED)
    # the solver reaches the continuum; acceptance rejects the point
    X, c, it, st = O.solve_one(sc, rx, ids)
    assert st == O.CONVERGED and c < 1e-20
    assert not O.accept_one(sc, rx, ids, X, st)
    # a reflection at an angle on the same wall is accepted
    sc.tx = np.array([5.0, -4.0, 1.0])
    X, c, it, st = O.solve_one(sc, np.array([2.0, -3.0, 2.0]), [0])
    assert st == O.CONVERGED and O.accept_one(sc, np.array([2.0, -3.0, 2.0]), [0], X, st)
