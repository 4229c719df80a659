"""Seeded synthetic workloads for the batched path solve.

This module only *draws* inputs: scenes of implicit primitives, receiver
positions, interaction sequences and (optionally) random initial guesses.
It holds none of the method's arithmetic (no residuals, projections,
solves or acceptance tests), so both the HIP path and the CPU oracle can
consume its output without sharing any of the method's code.

Scene model (paper Sec. II): every object is an implicit primitive.  The
records below are the flat FP64 layouts the C interfaces take; the global
primitive id is type-major: planes, then straight edges, then quadrics,
then circular edges.

  plane    (13): n(3) unit normal, d with n.x = d, o(3) rectangle corner,
                 eu(3), ev(3) rectangle side vectors (full length)
  line     (8) : p(3) point, e(3) unit direction, s0, s1 (parameter range)
  quadric  (17): p(3) anchor, A(6) = xx,xy,xz,yy,yz,zz of the symmetric
                 matrix, b(3), c, ax(3) patch axis, r_ap aperture radius;
                 f(x) = (x-p)^T A (x-p) + b^T (x-p) + c
  circle   (7) : c(3) centre, n(3) unit normal of its plane, R radius

Optional wedge of each straight edge (7 values, empty array: none): m1(3),
m2(3) unit normals of the two faces that meet at the edge, pointing into
free space, and a kind: 0 a free edge, 1 the outer corner of a solid (the
solid lies where both <x - X, m1> and <x - X, m2> are negative), 2 an inner
corner (the solid lies where either is negative).  Physical validation uses
it to keep diffracted rays out of the solids.

Optional refractive indices of each plane facet (two values, empty array:
none): a facet with both indices positive refracts instead of reflecting
(Snell's law; the first index is that of the side its normal points to, the
second that of the other side); (0, 0) marks a mirror.

Optional side of each plane facet (one value, empty array: none): +1 free
space lies on the side the normal points to, -1 on the other side, 0 on
both (a thin two-sided surface).  The visibility matrix of the candidate
generation uses it.

All seeds derive from S = 230106399 as S + 1000*cfg + stream with the
streams scene=1, rx=2, seq=3, init=4, train=5, heldout=6.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

SEED_BASE = 230106399
STREAM = {"scene": 1, "rx": 2, "seq": 3, "init": 4, "train": 5, "heldout": 6}

PLANE_W, LINE_W, QUAD_W, CIRC_W, WEDGE_W = 13, 8, 17, 7, 7
T_PLANE, T_LINE, T_QUAD, T_CIRC = 0, 1, 2, 3
MAX_ORDER = 5


def seed(cfg: int, stream: str) -> int:
    return SEED_BASE + 1000 * cfg + STREAM[stream]


@dataclass
class Scene:
    tx: np.ndarray
    planes: np.ndarray = field(default_factory=lambda: np.zeros((0, PLANE_W)))
    lines: np.ndarray = field(default_factory=lambda: np.zeros((0, LINE_W)))
    quadrics: np.ndarray = field(default_factory=lambda: np.zeros((0, QUAD_W)))
    circles: np.ndarray = field(default_factory=lambda: np.zeros((0, CIRC_W)))
    wedges: np.ndarray = field(default_factory=lambda: np.zeros((0, WEDGE_W)))
    sides: np.ndarray = field(default_factory=lambda: np.zeros(0))
    aabb_lo: np.ndarray = field(default_factory=lambda: np.zeros(3))
    aabb_hi: np.ndarray = field(default_factory=lambda: np.zeros(3))
    refraction: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))

    def __post_init__(self):
        self.tx = np.ascontiguousarray(self.tx, dtype=np.float64)
        for k in ("planes", "lines", "quadrics", "circles", "wedges", "sides", "refraction"):
            setattr(self, k, np.ascontiguousarray(getattr(self, k), dtype=np.float64))
        if len(self.wedges) and self.wedges.shape != (len(self.lines), WEDGE_W):
            raise ValueError("wedges: one record of 7 values per straight edge, or none")
        if len(self.sides) and self.sides.shape != (len(self.planes),):
            raise ValueError("sides: one value per plane facet, or none")
        if len(self.refraction) and self.refraction.shape != (len(self.planes), 2):
            raise ValueError("refraction: two indices per plane facet, or none")
        self.aabb_lo = np.ascontiguousarray(self.aabb_lo, dtype=np.float64)
        self.aabb_hi = np.ascontiguousarray(self.aabb_hi, dtype=np.float64)

    @property
    def counts(self):
        return (len(self.planes), len(self.lines), len(self.quadrics), len(self.circles))

    @property
    def n_prims(self):
        return sum(self.counts)

    def type_of(self, gid: np.ndarray) -> np.ndarray:
        """Primitive type of global ids (type-major numbering)."""
        c = np.cumsum(self.counts)
        return np.searchsorted(c, gid, side="right").astype(np.int32)


@dataclass
class Batch:
    """A batch of solves: one (RX, interaction list) each.

    rx        [n_rx, 3] FP64 receiver positions
    rx_index  [n] int32 index into rx
    order     [n] int32 number of interactions n_t in 1..5
    prim      [5, n] int32 global primitive ids, -1 beyond the order
    x0        optional [15, n] FP64 initial points (component-major)
    """
    rx: np.ndarray
    rx_index: np.ndarray
    order: np.ndarray
    prim: np.ndarray
    x0: np.ndarray | None = None

    def __post_init__(self):
        self.rx = np.ascontiguousarray(self.rx, dtype=np.float64)
        self.rx_index = np.ascontiguousarray(self.rx_index, dtype=np.int32)
        self.order = np.ascontiguousarray(self.order, dtype=np.int32)
        self.prim = np.ascontiguousarray(self.prim, dtype=np.int32)
        if self.x0 is not None:
            self.x0 = np.ascontiguousarray(self.x0, dtype=np.float64)

    @property
    def n(self):
        return len(self.order)

    def subset(self, idx):
        idx = np.asarray(idx)
        return Batch(self.rx, self.rx_index[idx], self.order[idx], self.prim[:, idx],
                     None if self.x0 is None else self.x0[:, idx])


# ---------------------------------------------------------------- records
def plane_rect(n, d, o, eu, ev):
    return np.concatenate([np.asarray(n, float), [float(d)], np.asarray(o, float),
                           np.asarray(eu, float), np.asarray(ev, float)])


def line_seg(p, e, s0, s1):
    return np.concatenate([np.asarray(p, float), np.asarray(e, float), [float(s0), float(s1)]])


def paraboloid(vertex, axis, focal):
    """Paraboloid of revolution with its vertex, unit axis and focal length F.

    In its own frame z' = (x'^2 + y'^2)/(4F); written as f = 0 with f scaled by
    1/(4F) so that |grad f| = 1 at the vertex.  The patch is r' <= 2F.
    """
    ax = np.asarray(axis, float)
    A = (np.eye(3) - np.outer(ax, ax)) / (4.0 * focal)
    return np.concatenate([np.asarray(vertex, float),
                           [A[0, 0], A[0, 1], A[0, 2], A[1, 1], A[1, 2], A[2, 2]],
                           -ax, [0.0], ax, [2.0 * focal]])


def wedge(m1, m2, kind):
    return np.concatenate([np.asarray(m1, float), np.asarray(m2, float), [float(kind)]])


def circle(c, n, R):
    return np.concatenate([np.asarray(c, float), np.asarray(n, float), [float(R)]])


def _unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


# ---------------------------------------------------------------- helpers
def _no_repeat_sequences(rng, n, order, pool_of_slot):
    """Draw prim ids [5, n]: slot k is drawn from pool_of_slot(k) (array of
    candidate ids per solve, or a 1-D pool), no element equal to the previous."""
    prim = np.full((MAX_ORDER, n), -1, dtype=np.int32)
    for k in range(MAX_ORDER):
        act = order > k
        pool = pool_of_slot(k)
        if isinstance(pool, np.ndarray) and pool.ndim == 1:
            draw = pool[rng.integers(0, len(pool), n)]
        else:
            draw = pool(n)
        prim[k, act] = draw[act]
        if k > 0:
            while True:
                bad = act & (prim[k] == prim[k - 1])
                if not bad.any():
                    break
                nb = int(bad.sum())
                if isinstance(pool, np.ndarray) and pool.ndim == 1:
                    prim[k, bad] = pool[rng.integers(0, len(pool), nb)]
                else:
                    prim[k, bad] = pool(n)[bad]
    return prim


def _near_infinite_object(scene: Scene, pts: np.ndarray, gids: np.ndarray, margin: float):
    """True where a point lies within `margin` of the infinite plane or line of
    the given primitive (input hygiene only: keeps grazing inputs out)."""
    out = np.zeros(len(gids), dtype=bool)
    t = scene.type_of(np.maximum(gids, 0))
    npl, nln = len(scene.planes), len(scene.lines)
    m = (gids >= 0) & (t == T_PLANE)
    if m.any():
        P = scene.planes[gids[m]]
        out[m] = np.abs(np.einsum("ij,ij->i", P[:, 0:3], pts[m]) - P[:, 3]) < margin
    m = (gids >= 0) & (t == T_LINE)
    if m.any():
        L = scene.lines[gids[m] - npl]
        w = pts[m] - L[:, 0:3]
        perp = w - np.einsum("ij,ij->i", w, L[:, 3:6])[:, None] * L[:, 3:6]
        out[m] = np.linalg.norm(perp, axis=1) < margin
    return out


# ---------------------------------------------------------------- config 1
def room_scene() -> Scene:
    """10 x 10 x 3 m room: 6 walls and 2 wall-junction edges, TX at (2,3,1.5)."""
    L, W, H = 10.0, 10.0, 3.0
    planes = np.stack([
        plane_rect([1, 0, 0], 0.0, [0, 0, 0], [0, W, 0], [0, 0, H]),
        plane_rect([1, 0, 0], L, [L, 0, 0], [0, W, 0], [0, 0, H]),
        plane_rect([0, 1, 0], 0.0, [0, 0, 0], [L, 0, 0], [0, 0, H]),
        plane_rect([0, 1, 0], W, [0, W, 0], [L, 0, 0], [0, 0, H]),
        plane_rect([0, 0, 1], 0.0, [0, 0, 0], [L, 0, 0], [0, W, 0]),
        plane_rect([0, 0, 1], H, [0, 0, H], [L, 0, 0], [0, W, 0]),
    ])
    lines = np.stack([
        line_seg([0, 0, 0], [0, 0, 1], 0.0, H),      # vertical corner x=0,y=0
        line_seg([0, W, H], [1, 0, 0], 0.0, L),      # y=10 wall / ceiling junction
    ])
    # inner corners: the room is the free space
    wedges = np.stack([wedge([1, 0, 0], [0, 1, 0], 2), wedge([0, -1, 0], [0, 0, -1], 2)])
    sides = np.array([1.0, -1.0, 1.0, -1.0, 1.0, -1.0])  # the walls face the room
    return Scene(tx=np.array([2.0, 3.0, 1.5]), planes=planes, lines=lines, wedges=wedges, sides=sides,
                 aabb_lo=np.zeros(3), aabb_hi=np.array([L, W, H]))


def config1(n_rx: int = 256) -> tuple[Scene, Batch]:
    """Room, all sequences of length 1-2 over the 8 objects with no immediate
    repeat: 8 + 8*7 = 64 per receiver."""
    sc = room_scene()
    rng = np.random.default_rng(seed(1, "rx"))
    rx = np.column_stack([rng.uniform(0.1, 9.9, n_rx), rng.uniform(0.1, 9.9, n_rx),
                          np.full(n_rx, 1.5)])
    seqs = [(a,) for a in range(8)] + [(a, b) for a in range(8) for b in range(8) if a != b]
    per = len(seqs)
    n = n_rx * per
    order = np.empty(n, np.int32)
    prim = np.full((MAX_ORDER, n), -1, np.int32)
    for j, s in enumerate(seqs):
        order[j::per] = len(s)
        for k, g in enumerate(s):
            prim[k, j::per] = g
    rx_index = np.repeat(np.arange(n_rx, dtype=np.int32), per)
    return sc, Batch(rx, rx_index, order, prim)


# ---------------------------------------------------------------- config 2
def street_canyon_scene(cfg: int = 2, n_boxes: int = 50, tx_height: float = 30.0):
    """Ground [0,200]^2 plus non-overlapping axis-aligned boxes (2 m clearance):
    per box 4 walls + roof (rectangles) and 4 vertical + 4 roof edges."""
    rng = np.random.default_rng(seed(cfg, "scene"))
    size = 200.0
    boxes = []
    while len(boxes) < n_boxes:
        w, d = rng.uniform(10, 30, 2)
        h = rng.uniform(10, 40)
        cx = rng.uniform(w / 2, size - w / 2)
        cy = rng.uniform(d / 2, size - d / 2)
        if abs(h - tx_height) < 1e-2:
            continue
        if all(abs(cx - b[0]) >= (w + b[2]) / 2 + 2 or abs(cy - b[1]) >= (d + b[3]) / 2 + 2
               for b in boxes):
            boxes.append((cx, cy, w, d, h))
    planes = [plane_rect([0, 0, 1], 0.0, [0, 0, 0], [size, 0, 0], [0, size, 0])]
    sides = [1.0]  # the ground faces up, the box faces outwards
    lines, wedges = [], []
    for cx, cy, w, d, h in boxes:
        x0, x1, y0, y1 = cx - w / 2, cx + w / 2, cy - d / 2, cy + d / 2
        planes += [
            plane_rect([1, 0, 0], x0, [x0, y0, 0], [0, d, 0], [0, 0, h]),
            plane_rect([1, 0, 0], x1, [x1, y0, 0], [0, d, 0], [0, 0, h]),
            plane_rect([0, 1, 0], y0, [x0, y0, 0], [w, 0, 0], [0, 0, h]),
            plane_rect([0, 1, 0], y1, [x0, y1, 0], [w, 0, 0], [0, 0, h]),
            plane_rect([0, 0, 1], h, [x0, y0, h], [w, 0, 0], [0, d, 0]),
        ]
        sides += [-1.0, 1.0, -1.0, 1.0, 1.0]
        for (x, y, sx, sy) in ((x0, y0, -1, -1), (x1, y0, 1, -1), (x1, y1, 1, 1), (x0, y1, -1, 1)):
            lines.append(line_seg([x, y, 0], [0, 0, 1], 0.0, h))
            wedges.append(wedge([sx, 0, 0], [0, sy, 0], 1))
        lines += [line_seg([x0, y0, h], [1, 0, 0], 0.0, w), line_seg([x0, y1, h], [1, 0, 0], 0.0, w),
                  line_seg([x0, y0, h], [0, 1, 0], 0.0, d), line_seg([x1, y0, h], [0, 1, 0], 0.0, d)]
        # roof edges: a wall and the roof meet there (outer corners of the box)
        wedges += [wedge([0, -1, 0], [0, 0, 1], 1), wedge([0, 1, 0], [0, 0, 1], 1),
                   wedge([-1, 0, 0], [0, 0, 1], 1), wedge([1, 0, 0], [0, 0, 1], 1)]
    boxes = np.array(boxes)

    def free_xy(r, n, margin=1.0):
        out = np.empty((0, 2))
        while len(out) < n:
            p = r.uniform(0, size, (4 * n + 16, 2))
            inside = np.zeros(len(p), bool)
            for cx, cy, w, d, h in boxes:
                inside |= (np.abs(p[:, 0] - cx) < w / 2 + margin) & (np.abs(p[:, 1] - cy) < d / 2 + margin)
            out = np.vstack([out, p[~inside]])
        return out[:n]

    txy = free_xy(rng, 1)[0]
    sc = Scene(tx=np.array([txy[0], txy[1], tx_height]), planes=np.array(planes),
               lines=np.array(lines), wedges=np.array(wedges), sides=np.array(sides), aabb_lo=np.zeros(3),
               aabb_hi=np.array([size, size, max(40.0, boxes[:, 4].max())]))
    sc._boxes = boxes
    sc._free_xy = free_xy
    return sc


def _resample_near(sc, rx, batch_rx_index, prim, order, rng, pools, margin=1e-3):
    """Redraw sequence elements whose infinite object passes within `margin` of
    TX or of the receiver of that solve."""
    for k in range(MAX_ORDER):
        for _ in range(100):
            act = order > k
            g = prim[k]
            bad = act & (_near_infinite_object(sc, np.broadcast_to(sc.tx, (len(g), 3)), g, margin)
                         | _near_infinite_object(sc, rx[batch_rx_index], g, margin))
            if not bad.any():
                break
            nb = int(bad.sum())
            pool = pools(k)
            new = pool[rng.integers(0, len(pool), nb)] if isinstance(pool, np.ndarray) else pool(nb)
            prim[k, bad] = new
            # keep the no-repeat rule
            for kk in (k, k + 1):
                if 0 < kk < MAX_ORDER:
                    rep = (order > kk) & (prim[kk] == prim[kk - 1])
                    while rep.any():
                        pool2 = pools(kk)
                        nr = int(rep.sum())
                        prim[kk, rep] = (pool2[rng.integers(0, len(pool2), nr)]
                                         if isinstance(pool2, np.ndarray) else pool2(nr))
                        rep = (order > kk) & (prim[kk] == prim[kk - 1])
    return prim


def config2(n_rx: int = 4096, per_rx: int = 64) -> tuple[Scene, Batch]:
    sc = street_canyon_scene(2)
    rng = np.random.default_rng(seed(2, "rx"))
    xy = sc._free_xy(rng, n_rx)
    rx = np.column_stack([xy, np.full(n_rx, 1.5)])
    rs = np.random.default_rng(seed(2, "seq"))
    n = n_rx * per_rx
    order = rs.integers(1, 4, n).astype(np.int32)
    pool = np.arange(sc.n_prims, dtype=np.int32)
    prim = _no_repeat_sequences(rs, n, order, lambda k: pool)
    rx_index = np.repeat(np.arange(n_rx, dtype=np.int32), per_rx)
    prim = _resample_near(sc, rx, rx_index, prim, order, rs, lambda k: pool)
    return sc, Batch(rx, rx_index, order, prim)


# ---------------------------------------------------------------- config 3
def curved_scene(cfg: int = 3, n_quad: int = 200, n_circ: int = 100, rng=None) -> Scene:
    rng = rng or np.random.default_rng(seed(cfg, "scene"))
    lo, hi = np.zeros(3), np.array([200.0, 200.0, 40.0])
    quads = []
    for _ in range(n_quad):
        F = rng.uniform(1, 5)
        v = rng.uniform(lo, hi)
        ax = _unit(rng.normal(size=3))
        quads.append(paraboloid(v, ax, F))
    circs = []
    for _ in range(n_circ):
        R = rng.uniform(0.5, 3)
        c = rng.uniform(lo, hi)
        nn = _unit(rng.normal(size=3))
        circs.append(circle(c, nn, R))
    return Scene(tx=np.array([100.0, 100.0, 20.0]), quadrics=np.array(quads).reshape(-1, QUAD_W),
                 circles=np.array(circs).reshape(-1, CIRC_W), aabb_lo=lo, aabb_hi=hi)


def config3(n_rx: int = 16384, per_rx: int = 64) -> tuple[Scene, Batch]:
    sc = curved_scene(3)
    rng = np.random.default_rng(seed(3, "rx"))
    rx = rng.uniform(sc.aabb_lo, sc.aabb_hi, (n_rx, 3))
    rs = np.random.default_rng(seed(3, "seq"))
    n = n_rx * per_rx
    order = rs.integers(1, 6, n).astype(np.int32)
    pool = np.arange(sc.n_prims, dtype=np.int32)
    prim = _no_repeat_sequences(rs, n, order, lambda k: pool)
    return sc, Batch(rx, np.repeat(np.arange(n_rx, dtype=np.int32), per_rx), order, prim)


# ---------------------------------------------------------------- config 5
def stress_scene() -> Scene:
    sc = street_canyon_scene(5)
    q = curved_scene(5, n_quad=30, n_circ=0, rng=np.random.default_rng(seed(5, "scene") + 77))
    out = Scene(tx=sc.tx, planes=sc.planes, lines=sc.lines, quadrics=q.quadrics, wedges=sc.wedges, sides=sc.sides,
                aabb_lo=sc.aabb_lo, aabb_hi=sc.aabb_hi)
    out._boxes, out._free_xy = sc._boxes, sc._free_xy
    return out


def _stress_lists(sc: Scene, rs, n: int):
    """Lists of order 3-5 with at least two diffractions at random slots:
    diffractions on the box edges, reflections on the facets and the
    paraboloids, no immediate repeat."""
    order = rs.integers(3, 6, n).astype(np.int32)
    nd = (rs.random(n) * (order - 1)).astype(np.int32) + 2       # U{2..order}
    npl, nln, nq, _ = sc.counts
    dpool = np.arange(npl, npl + nln, dtype=np.int32)
    rpool = np.concatenate([np.arange(npl, dtype=np.int32),
                            np.arange(npl + nln, npl + nln + nq, dtype=np.int32)])
    # choose which slots diffract: random permutation keys, the nd smallest
    keys = rs.random((MAX_ORDER, n))
    keys[np.arange(MAX_ORDER)[:, None] >= order[None, :]] = 2.0
    rank = np.argsort(np.argsort(keys, axis=0), axis=0)
    is_d = rank < nd[None, :]
    del keys, rank

    def slot_pool(k):
        def draw(m):
            a = dpool[rs.integers(0, len(dpool), n)]
            b = rpool[rs.integers(0, len(rpool), n)]
            return np.where(is_d[k], a, b)
        return draw
    return order, _no_repeat_sequences(rs, n, order, slot_pool)


def config5(n_rx: int = 16384, per_rx: int = 1024, stream: str = "rx") -> tuple[Scene, Batch]:
    """Orders 3-5 with at least two diffractions; diffractions on the box edges,
    reflections on the facets and the paraboloids.  `stream` "train" or
    "heldout" draws other receivers and lists for the learned start."""
    sc = stress_scene()
    rng = np.random.default_rng(seed(5, stream))
    xy = sc._free_xy(rng, n_rx)
    rx = np.column_stack([xy, np.full(n_rx, 1.5)])
    rs = np.random.default_rng(seed(5, "seq") if stream == "rx" else seed(5, stream) + 500)
    order, prim = _stress_lists(sc, rs, n_rx * per_rx)
    return sc, Batch(rx, np.repeat(np.arange(n_rx, dtype=np.int32), per_rx), order, prim)


# ---------------------------------------------------------------- paper example
def fig5_scene() -> tuple[Scene, Batch]:
    """The two-mirror example of the image-method figure, lifted to 3-D at z=0:
    mirror 1 on y = x for (0,0)-(3.5,3.5), mirror 2 on x = 5 for y in [0.5,4];
    BS (2,-1), UE (2,4)."""
    s2 = np.sqrt(0.5)
    planes = np.stack([
        plane_rect([s2, -s2, 0], 0.0, [0, 0, -1], [3.5, 3.5, 0], [0, 0, 2]),
        plane_rect([1, 0, 0], 5.0, [5, 0.5, -1], [0, 3.5, 0], [0, 0, 2]),
    ])
    sc = Scene(tx=np.array([2.0, -1.0, 0.0]), planes=planes,
               aabb_lo=np.array([-1.0, -1.0, -1.0]), aabb_hi=np.array([11.0, 4.0, 1.0]))
    b = Batch(np.array([[2.0, 4.0, 0.0]]), np.array([0]), np.array([2]),
              np.array([[0], [1], [-1], [-1], [-1]]))
    return sc, b


def fig3_scene(height: float = 5.0) -> tuple[Scene, np.ndarray]:
    """The two-triangle scenario of the visibility figure (Figs. 3-4),
    extruded along z over [-height, height]: triangle 1 with corners
    e1 (-1, .5), e2 (0, .5), e3 (-1, 1.5) and sides s1 = e1e2, s2 = e2e3,
    s3 = e3e1; triangle 2 with e4 (2, -.5), e5 (3.5, -.5), e6 (3.5, 1) and
    s4 = e4e5, s5 = e5e6, s6 = e6e4; BS (-.3, -.5), UE (2, 2) at z = 0.
    Sides are facets facing out of their triangle, corners are vertical
    edges with the wedges of their two sides.  Object ids: s1..s6 = 0..5,
    e1..e6 = 6..11.  Returns the scene and the UE position."""
    tri = [np.array([[-1.0, 0.5], [0.0, 0.5], [-1.0, 1.5]]), np.array([[2.0, -0.5], [3.5, -0.5], [3.5, 1.0]])]
    planes, sides, lines, wedges = [], [], [], []
    outward = []
    for T in tri:
        ctr = T.mean(axis=0)
        nrm = []
        for a in range(3):
            p, q = T[a], T[(a + 1) % 3]
            t = (q - p) / np.linalg.norm(q - p)
            n2 = np.array([t[1], -t[0]])
            if (p - ctr) @ n2 < 0:
                n2 = -n2
            n3 = np.array([n2[0], n2[1], 0.0])
            planes.append(plane_rect(n3, n3[:2] @ p, [p[0], p[1], -height], [q[0] - p[0], q[1] - p[1], 0],
                                     [0, 0, 2 * height]))
            sides.append(1.0)
            nrm.append(n3)
        outward.append(nrm)
    for T, nrm in zip(tri, outward):
        for a in range(3):
            # corner a joins side a-1 (ending there) and side a (starting there)
            lines.append(line_seg([T[a][0], T[a][1], -height], [0, 0, 1], 0.0, 2 * height))
            wedges.append(wedge(nrm[(a - 1) % 3], nrm[a], 1))
    sc = Scene(tx=np.array([-0.3, -0.5, 0.0]), planes=np.array(planes), lines=np.array(lines),
               wedges=np.array(wedges), sides=np.array(sides),
               aabb_lo=np.array([-2.0, -2.0, -height]), aabb_hi=np.array([5.0, 3.0, height]))
    return sc, np.array([2.0, 2.0, 0.0])


def random_init(scene: Scene, batch: Batch, cfg: int, restart: int = 0) -> np.ndarray:
    """Random initial points inside the scene box (the paper's random guess),
    drawn here and passed to both sides as an input."""
    rng = np.random.default_rng([seed(cfg, "init"), restart])
    x0 = np.zeros((3 * MAX_ORDER, batch.n))
    lo, hi = scene.aabb_lo, scene.aabb_hi
    for k in range(MAX_ORDER):
        for c in range(3):
            x0[3 * k + c] = rng.uniform(lo[c], hi[c], batch.n)
    return x0


def training_batch(cfg: int, n_rx: int, per_rx: int = 64, stream: str = "train") -> tuple[Scene, Batch]:
    """Problems for the learned start: the same scene as configuration `cfg`
    (2: street canyon, 3: curved), receivers and interaction lists drawn from
    the separate seed stream `stream` ("train" or "heldout")."""
    if cfg == 2:
        sc = street_canyon_scene(2)
        rng = np.random.default_rng(seed(2, stream))
        xy = sc._free_xy(rng, n_rx)
        rx = np.column_stack([xy, np.full(n_rx, 1.5)])
        lo, hi = 1, 4
    elif cfg == 3:
        sc = curved_scene(3)
        rng = np.random.default_rng(seed(3, stream))
        rx = rng.uniform(sc.aabb_lo, sc.aabb_hi, (n_rx, 3))
        lo, hi = 1, 6
    elif cfg == 5:
        return config5(n_rx=n_rx, per_rx=per_rx, stream=stream)
    else:
        raise ValueError("training batches exist for configurations 2, 3 and 5")
    rs = np.random.default_rng(seed(cfg, stream) + 500)
    n = n_rx * per_rx
    order = rs.integers(lo, hi, n).astype(np.int32)
    pool = np.arange(sc.n_prims, dtype=np.int32)
    prim = _no_repeat_sequences(rs, n, order, lambda k: pool)
    rx_index = np.repeat(np.arange(n_rx, dtype=np.int32), per_rx)
    if cfg == 2:
        prim = _resample_near(sc, rx, rx_index, prim, order, rs, lambda k: pool)
    return sc, Batch(rx, rx_index, order, prim)


# ---------------------------------------------------------------- refraction
def glazed_scene(n_panes: int = 40) -> Scene:
    """The street canyon plus glass panes standing in the streets: each pane
    is a slab of two parallel vertical refracting facets (glass index 1.5
    inside, 1.0 outside), thickness U(0.1, 0.5) m, width U(4, 12) m, height
    U(3, 10) m from the ground, facing x or y, centred in free space.  The
    box facets stay mirrors."""
    sc = street_canyon_scene(6)
    rng = np.random.default_rng(seed(6, "scene") + 91)
    planes, refr, sides = [list(p) for p in sc.planes], [[0.0, 0.0]] * len(sc.planes), list(sc.sides)
    xy = sc._free_xy(rng, n_panes, margin=8.0)
    panes = []
    for (cx, cy) in xy:
        t, w, h = rng.uniform(0.1, 0.5), rng.uniform(4, 12), rng.uniform(3, 10)
        ax = int(rng.integers(0, 2))          # 0: faces along x, 1: along y
        nrm = np.array([1.0, 0.0, 0.0]) if ax == 0 else np.array([0.0, 1.0, 0.0])
        tan = np.array([0.0, 1.0, 0.0]) if ax == 0 else np.array([1.0, 0.0, 0.0])
        c = np.array([cx, cy, 0.0])
        for sgn in (-1.0, 1.0):
            n = sgn * nrm                     # outward normal: air (1.0) in front, glass (1.5) behind
            o = c + 0.5 * t * n - 0.5 * w * tan
            planes.append(plane_rect(n, n @ o, o, w * tan, [0.0, 0.0, h]))
            refr.append([1.0, 1.5])
            sides.append(0.0)
        panes.append((c, nrm, tan, t, w, h))
    out = Scene(tx=sc.tx, planes=np.array(planes), lines=sc.lines, wedges=sc.wedges, sides=np.array(sides),
                refraction=np.array(refr), aabb_lo=sc.aabb_lo, aabb_hi=sc.aabb_hi)
    out._boxes, out._free_xy = sc._boxes, sc._free_xy
    out._n_box_planes = len(sc.planes)
    out._panes = panes
    return out


def config6(n_rx: int = 4096, per_rx: int = 64) -> tuple[Scene, Batch]:
    """Paths through glass panes.  Receiver i stands 1-8 m behind pane
    i mod 40 (on the side away from TX, within its width, at 1.5 m, outside
    the boxes).  Its lists have order 2-4 and hold the two facets of that
    pane back to back in the order a ray from TX crosses them (into the
    glass, out again), at a random position; the other elements are drawn
    uniformly over the box facets and edges, no immediate repeat."""
    sc = glazed_scene()
    rng = np.random.default_rng(seed(6, "rx"))
    nb = sc._n_box_planes
    n_panes = len(sc._panes)
    rx = np.zeros((n_rx, 3))
    first = np.zeros(n_rx, np.int32)
    for i in range(n_rx):
        c, nrm, tan, t, w, h = sc._panes[i % n_panes]
        away = -1.0 if (sc.tx - c) @ nrm > 0 else 1.0     # the side away from TX
        for attempt in range(200):
            # behind the pane; after 100 failed draws (a box or the map's
            # edge behind it) in front of it (then no path crosses the pane)
            side = away if attempt < 100 else -away
            p = c + side * nrm * (0.5 * t + rng.uniform(1.0, 8.0)) + tan * rng.uniform(-0.4, 0.4) * w
            inside = False
            for cx, cy, bw, bd, bh in sc._boxes:
                inside |= abs(p[0] - cx) < bw / 2 + 1.0 and abs(p[1] - cy) < bd / 2 + 1.0
            if not inside and 1 < p[0] < 199 and 1 < p[1] < 199:
                break
        else:
            p = np.append(sc._free_xy(rng, 1)[0], 0.0)
        rx[i] = [p[0], p[1], 1.5]
        # the facet whose outward normal faces TX is crossed first
        first[i] = nb + 2 * (i % n_panes) + (0 if away > 0 else 1)
    rs = np.random.default_rng(seed(6, "seq"))
    n = n_rx * per_rx
    rx_index = np.repeat(np.arange(n_rx, dtype=np.int32), per_rx)
    others = np.concatenate([np.arange(nb), np.arange(len(sc.planes), sc.n_prims)]).astype(np.int32)
    order = rs.integers(2, 5, n).astype(np.int32)
    pos = (rs.random(n) * (order - 1)).astype(np.int32)        # slot of the first pane facet
    f0 = first[rx_index]
    f1 = np.where((f0 - nb) % 2 == 0, f0 + 1, f0 - 1).astype(np.int32)
    prim = -np.ones((MAX_ORDER, n), np.int32)
    for k in range(MAX_ORDER):
        prim[k] = np.where(k < order, others[rs.integers(0, len(others), n)], -1)
    for k in range(MAX_ORDER):
        prim[k] = np.where(pos == k, f0, prim[k])
        prim[k] = np.where(pos + 1 == k, f1, prim[k])
    fixed = lambda k: (pos == k) | (pos + 1 == k)
    for k in range(1, MAX_ORDER):
        rep = (k < order) & (prim[k] == prim[k - 1])
        while rep.any():
            a = rep & ~fixed(k)
            prim[k, a] = others[rs.integers(0, len(others), int(a.sum()))]
            b = rep & fixed(k)
            prim[k - 1, b] = others[rs.integers(0, len(others), int(b.sum()))]
            rep = (k < order) & (prim[k] == prim[k - 1])
    return sc, Batch(rx, rx_index, order, prim)


CONFIGS = {1: config1, 2: config2, 3: config3, 5: config5, 6: config6}
