"""Pins of the oracle's physical validation: a kept path's segments may not
pass through another object (Alg. 1 keeps paths whose points are valid, and
Sec. II's rays travel in free space between interactions).

The facet-by-facet test of the oracle is checked against an independent
slab-method segment/box test on the street-canyon buildings, and against
closed forms for a paraboloid dish.
"""
import numpy as np

import oracle as O
from paper_2301_06399_amd import workloads as W


def segment_enters_box(P, Q, lo, hi, margin):
    """Slab method: does the open segment P -> Q (trimmed by `margin` metres
    at both ends) pass through the interior of the box [lo, hi]?"""
    d = Q - P
    L = np.linalg.norm(d)
    t0, t1 = margin / L, 1.0 - margin / L
    for i in range(3):
        if abs(d[i]) < 1e-300:
            if not (lo[i] < P[i] < hi[i]):
                return False
            continue
        a, b = (lo[i] - P[i]) / d[i], (hi[i] - P[i]) / d[i]
        t0, t1 = max(t0, min(a, b)), min(t1, max(a, b))
    return t0 < t1


def test_visibility_matches_slab_test_on_buildings():
    """Paths TX -> ground point -> RX in the street canyon: the oracle's
    facet crossings agree with the slab test against every building (the
    ground is the interaction object and is not tested)."""
    sc = W.street_canyon_scene(2)
    rng = np.random.default_rng(5)
    boxes = sc._boxes
    agree = blocked = 0
    for trial in range(3000):
        rx = np.append(sc._free_xy(rng, 1)[0], rng.uniform(0.5, 45.0))
        g = np.append(sc._free_xy(rng, 1)[0], 0.0)
        vis = O.visible_one(sc, rx, [0], g)
        hit = False
        for P, Q in ((sc.tx, g), (g, rx)):
            for cx, cy, w, d, h in boxes:
                lo = np.array([cx - w / 2, cy - d / 2, 0.0])
                hi = np.array([cx + w / 2, cy + d / 2, h])
                hit = hit or segment_enters_box(P, Q, lo, hi, 1e-6)
        agree += (vis == (not hit))
        blocked += hit
    assert agree == 3000
    assert blocked > 300 and 3000 - blocked > 20


def test_visibility_paraboloid_dish_and_endpoints():
    """A dish z = r^2/(4F) (aperture r <= 2F) blocks a vertical segment
    through it inside the aperture and not outside it; a segment that ends
    on a facet is not blocked by that facet."""
    F = 2.0
    sc = W.Scene(tx=np.array([0.5, 0.0, 10.0]),
                 planes=np.array([W.plane_rect([0, 0, 1], -5.0, [-50, -50, -5], [100, 0, 0], [0, 100, 0])]),
                 quadrics=np.array([W.paraboloid([0, 0, 0], [0, 0, 1], F)]),
                 aabb_lo=-50 * np.ones(3), aabb_hi=50 * np.ones(3))
    floor = [0]
    # TX above the dish, reflection point on the floor right below: blocked
    assert not O.visible_one(sc, np.array([0.5, 0.0, 10.0]), floor, np.array([0.5, 0.0, -5.0]))
    # the same outside the aperture (r = 5 > 2F = 4): free
    sc.tx = np.array([5.0, 0.0, 10.0])
    assert O.visible_one(sc, np.array([5.0, 0.0, 10.0]), floor, np.array([5.0, 0.0, -5.0]))
    # reflecting on the dish itself: the dish is not tested for its own segments
    sc.tx = np.array([0.5, 0.0, 10.0])
    X = np.array([0.5, 0.0, 0.25 / (4 * F)])
    assert O.visible_one(sc, np.array([0.5, 0.0, 10.0]), [1], X)
