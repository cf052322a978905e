"""Seeded synthetic chart sets shaped like the paper's packing workloads.

The paper packs UV-unwrapped and texture-space-shading chart sets into square
power-of-two atlases with 1-pixel gutters (Sec. 5, "Experimental Setup"); those
datasets are not redistributable, so every input here is synthetic: star-shaped
polygons, concave L/U shapes and near-rectangular lightmap quads with
log-normal areas, quantised to fixed point (1/256 texel, "Q8").

This module holds no packing arithmetic.  It only draws inputs, and it is the
one module shared by the oracle-side tests and the GPU-side tests / benchmark.
"""
from __future__ import annotations

import dataclasses
import functools
import math

import numpy as np

Q8 = 256  # fixed-point units per texel for input vertex coordinates


@dataclasses.dataclass(frozen=True)
class AtlasInput:
    """One packing problem: charts as a CSR of Q8 polygons plus the atlas."""

    xy: np.ndarray        # int32[2V], interleaved x,y in Q8, y grows downward
    offsets: np.ndarray   # int32[n+1] CSR vertex offsets
    atlas_w: int
    atlas_h: int
    padding: int
    quality: int

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def total_verts(self) -> int:
        return int(self.offsets[-1])

    def chart(self, c: int) -> np.ndarray:
        a, b = int(self.offsets[c]), int(self.offsets[c + 1])
        return self.xy[2 * a:2 * b].reshape(-1, 2)


# Workload recipes.  'mix' entries: (shape, fraction, min_verts, max_verts, max_aspect)
CONFIGS = {
    # 64 stars into 512^2, padding 2
    "stars64": dict(W=512, H=512, p=2, n=64, sigma=0.8, fill=0.6, q=2,
                  mix=[("star", 1.0, 8, 24, 4.0)]),
    # 2,000 charts into 2048^2, padding 2: 70% stars, 30% L/U, area 120% of atlas
    "mixed2k": dict(W=2048, H=2048, p=2, n=2000, sigma=1.2, fill=1.2, q=2,
                   mix=[("star", 0.7, 8, 64, 8.0), ("lu", 0.3, 6, 8, 8.0)]),
    # 20,000 lightmap-style charts into 4096^2, padding 1
    "lightmap20k": dict(W=4096, H=4096, p=1, n=20000, sigma=1.5, fill=1.5, q=2,
                  mix=[("quad", 0.9, 4, 8, 16.0), ("star", 0.1, 16, 48, 4.0)]),
}
CONFIG_INDEX = {"stars64": 1, "mixed2k": 2, "lightmap20k": 3, "batch": 4, "serve": 5, "tss4k": 6}

# Texture-space-shading-like frames (a second workload; the paper's TSS chart
# sets come from camera paths and are not available): screen-space patches of
# a 1920 x 1080 frame clipped to the view frustum, at their on-screen
# orientation (not pre-rotated), packed into a 1024^2 atlas.
TSS = dict(screen=(1920, 1080), W=1024, H=1024, p=2, n=4000, sigma=1.3, cover=0.6, q=2)


def config_seed(name: str, instance: int) -> int:
    """seed = 1000 * config number + instance (instance 0 is the timed input)."""
    return 1000 * CONFIG_INDEX[name] + int(instance)


# --------------------------------------------------------------------------
# exact integer validity test of a quantised polygon
# --------------------------------------------------------------------------
def _orient(ax, ay, bx, by, cx, cy):
    return np.sign((bx - ax) * (cy - ay) - (by - ay) * (cx - ax))


def polygon_is_simple(P: np.ndarray) -> bool:
    """True iff the closed integer polygon P (m x 2) has >= 3 distinct
    consecutive vertices, no zero-length edge and no two edges that touch
    except consecutive edges at their shared vertex (and those do not fold
    back onto each other)."""
    P = np.asarray(P, dtype=np.int64)
    m = P.shape[0]
    if m < 3:
        return False
    Q = np.roll(P, -1, axis=0)
    if np.any(np.all(P == Q, axis=1)):
        return False
    ax, ay = P[:, 0][:, None], P[:, 1][:, None]
    bx, by = Q[:, 0][:, None], Q[:, 1][:, None]
    cx, cy = P[:, 0][None, :], P[:, 1][None, :]
    dx, dy = Q[:, 0][None, :], Q[:, 1][None, :]
    d1 = _orient(ax, ay, bx, by, cx, cy)
    d2 = _orient(ax, ay, bx, by, dx, dy)
    d3 = _orient(cx, cy, dx, dy, ax, ay)
    d4 = _orient(cx, cy, dx, dy, bx, by)
    proper = (d1 * d2 < 0) & (d3 * d4 < 0)

    def on_seg(px, py, qx, qy, rx, ry):  # r on segment pq given collinear
        return ((np.minimum(px, qx) <= rx) & (rx <= np.maximum(px, qx)) &
                (np.minimum(py, qy) <= ry) & (ry <= np.maximum(py, qy)))

    touch = ((d1 == 0) & on_seg(ax, ay, bx, by, cx, cy)) | \
            ((d2 == 0) & on_seg(ax, ay, bx, by, dx, dy)) | \
            ((d3 == 0) & on_seg(cx, cy, dx, dy, ax, ay)) | \
            ((d4 == 0) & on_seg(cx, cy, dx, dy, bx, by))
    hit = proper | touch
    idx = np.arange(m)
    same = idx[:, None] == idx[None, :]
    nxt = (idx[:, None] + 1) % m == idx[None, :]
    prv = (idx[None, :] + 1) % m == idx[:, None]
    bad = hit & ~same & ~nxt & ~prv
    if np.any(bad):
        return False
    # consecutive edges must not fold back (collinear with opposite direction)
    R = np.roll(P, -2, axis=0)
    e1 = Q - P
    e2 = R - Q
    cross = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    dot = e1[:, 0] * e2[:, 0] + e1[:, 1] * e2[:, 1]
    if np.any((cross == 0) & (dot < 0)):
        return False
    if m == 3 and np.all(cross == 0):
        return False
    return True


def _shoelace(P: np.ndarray) -> float:
    x, y = P[:, 0], P[:, 1]
    return 0.5 * abs(float(np.dot(x, np.roll(y, -1)) - np.dot(np.roll(x, -1), y)))


# --------------------------------------------------------------------------
# shape primitives (float, unit-ish size; scaled to the target area later)
# --------------------------------------------------------------------------
def _rot(P, phi):
    c, s = math.cos(phi), math.sin(phi)
    return P @ np.array([[c, s], [-s, c]])


def _star(rng, m, amax):
    ang = 2.0 * np.pi * (np.arange(m) + rng.uniform(-0.3, 0.3, m)) / m
    ang.sort()
    r = 1.0 + rng.uniform(-0.4, 0.4, m)
    P = np.stack([r * np.cos(ang), r * np.sin(ang)], axis=1)
    a = rng.uniform(1.0, amax)
    P[:, 0] *= math.sqrt(a)
    P[:, 1] /= math.sqrt(a)
    return _rot(P, rng.uniform(0.0, np.pi))


def _lu(rng, amax):
    a = rng.uniform(1.0, amax)
    w, h = math.sqrt(a), 1.0 / math.sqrt(a)
    fx, fy = rng.uniform(0.3, 0.7, 2)
    if rng.uniform() < 0.5:   # L: rectangle minus a corner block
        P = np.array([[0, 0], [w, 0], [w, h * fy], [w * fx, h * fy], [w * fx, h], [0, h]], float)
    else:                     # U: rectangle minus a centred notch
        nw = w * fx
        x0 = 0.5 * (w - nw)
        P = np.array([[0, 0], [x0, 0], [x0, h * fy], [x0 + nw, h * fy], [x0 + nw, 0],
                      [w, 0], [w, h], [0, h]], float)
    t = rng.integers(0, 4)
    P = _rot(P, t * np.pi / 2)
    if rng.uniform() < 0.5:
        P[:, 0] = -P[:, 0]
        P = P[::-1].copy()
    if rng.uniform() < 0.5:
        P = _rot(P, rng.uniform(0.0, np.pi))
    return P


def _quad(rng, mv, amax):
    a = rng.uniform(1.0, amax)
    w, h = math.sqrt(a), 1.0 / math.sqrt(a)
    short = min(w, h)
    corners = np.array([[0, 0], [w, 0], [w, h], [0, h]], float)
    corners += rng.uniform(-0.05, 0.05, corners.shape) * short
    extra = int(rng.integers(0, mv - 4 + 1))
    pts = []
    per_edge = np.zeros(4, int)
    for _ in range(extra):
        per_edge[rng.integers(0, 4)] += 1
    for e in range(4):
        p0, p1 = corners[e], corners[(e + 1) % 4]
        pts.append(p0)
        if per_edge[e]:
            ts = np.sort(rng.uniform(0.15, 0.85, per_edge[e]))
            d = p1 - p0
            nrm = np.array([-d[1], d[0]]) / (np.hypot(*d) + 1e-30)
            for t in ts:
                pts.append(p0 + t * d + nrm * rng.uniform(-0.02, 0.02) * short)
    P = np.array(pts)
    return _rot(P, rng.uniform(-np.pi / 18, np.pi / 18))


def _draw_shape(rng, kind, vmin, vmax, amax):
    if kind == "star":
        return _star(rng, int(rng.integers(vmin, vmax + 1)), amax)
    if kind == "lu":
        return _lu(rng, amax)
    if kind == "quad":
        return _quad(rng, vmax, amax)
    raise ValueError(kind)


def _quantise(P_float, area_tex, rng, place_w, place_h):
    """Scale a float shape to area_tex texel^2, place it at a random spot and
    round to Q8.  Returns None if the result is degenerate or not simple."""
    A = _shoelace(P_float)
    if A <= 0:
        return None
    P = P_float * math.sqrt(area_tex / A)
    P -= P.min(axis=0)
    off = np.array([rng.uniform(0, place_w), rng.uniform(0, place_h)])
    Q = np.rint((P + off) * Q8).astype(np.int64)
    ext = Q.max(axis=0) - Q.min(axis=0)
    if ext.min() < 4 or np.abs(Q).max() >= (1 << 21):
        return None
    if not polygon_is_simple(Q):
        return None
    return Q


def generate_charts(n, W, H, sigma, fill, mix, seed):
    """n charts with log-normal areas summing to fill*W*H texel^2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    areas = np.exp(sigma * rng.standard_normal(n))
    areas *= fill * W * H / areas.sum()
    fracs = np.array([m[1] for m in mix], float)
    kinds = rng.choice(len(mix), size=n, p=fracs / fracs.sum())
    polys = []
    for i in range(n):
        kind, _, vmin, vmax, amax = mix[kinds[i]]
        for _attempt in range(64):
            Q = _quantise(_draw_shape(rng, kind, vmin, vmax, amax), areas[i], rng, W, H)
            if Q is not None:
                break
        else:  # pragma: no cover - vanishingly rare
            raise RuntimeError("could not draw a valid chart")
        polys.append(Q)
    return polys


def clip_to_rect(P, x0, y0, x1, y1):
    """Sutherland-Hodgman clip of a float polygon to the box [x0,x1] x [y0,y1]."""
    def clip(poly, inside, cross):
        out = []
        m = len(poly)
        for i in range(m):
            a, b = poly[i], poly[(i + 1) % m]
            ia, ib = inside(a), inside(b)
            if ia:
                out.append(a)
            if ia != ib:
                out.append(cross(a, b))
        return out

    def xcut(xv):
        return lambda a, b: (xv, a[1] + (b[1] - a[1]) * (xv - a[0]) / (b[0] - a[0]))

    def ycut(yv):
        return lambda a, b: (a[0] + (b[0] - a[0]) * (yv - a[1]) / (b[1] - a[1]), yv)
    poly = [tuple(p) for p in np.asarray(P, float)]
    for inside, cross in ((lambda q: q[0] >= x0, xcut(x0)), (lambda q: q[0] <= x1, xcut(x1)),
                          (lambda q: q[1] >= y0, ycut(y0)), (lambda q: q[1] <= y1, ycut(y1))):
        if len(poly) < 3:
            return np.zeros((0, 2))
        poly = clip(poly, inside, cross)
    return np.array(poly, float) if len(poly) >= 3 else np.zeros((0, 2))


def _tss_patch(rng):
    """A projected surface patch: a perspective-distorted quad (a planar
    rectangle seen at an angle), a convex fan of 5-9 vertices, or a concave
    L-shaped patch, at a random on-screen angle."""
    r = rng.uniform()
    if r < 0.5:
        a = rng.uniform(1.0, 6.0)
        w, h = math.sqrt(a), 1.0 / math.sqrt(a)
        t = rng.uniform(0.4, 1.0)  # far edge shrunk by perspective
        P = np.array([[-w / 2, 0], [w / 2, 0], [t * w / 2, h], [-t * w / 2, h]], float)
    elif r < 0.8:
        m = int(rng.integers(5, 10))
        ang = np.sort(2 * np.pi * (np.arange(m) + rng.uniform(-0.25, 0.25, m)) / m)
        rr = 1.0 + rng.uniform(-0.15, 0.15, m)
        P = np.stack([rr * np.cos(ang), rr * np.sin(ang) * rng.uniform(0.3, 1.0)], axis=1)
    else:
        P = _lu(rng, 4.0)
    return _rot(P, rng.uniform(0.0, 2 * np.pi))


def generate_tss_charts(n, screen, sigma, cover, seed):
    """n clipped screen-space patches whose areas (log-normal, sigma) sum to
    about `cover` of the screen; patch centres fall on the screen grown by a
    fifth of its size on every side, so the border patches are clipped to
    the frustum (straight edges along the screen edges)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    SW, SH = screen
    areas = np.exp(sigma * rng.standard_normal(n))
    areas *= cover * SW * SH / areas.sum()
    polys = []
    i = 0
    while len(polys) < n:
        P = _tss_patch(rng)
        A = _shoelace(P)
        P = P * math.sqrt(areas[i % n] / A)
        c = np.array([rng.uniform(-0.2 * SW, 1.2 * SW), rng.uniform(-0.2 * SH, 1.2 * SH)])
        C = clip_to_rect(P + c, 0.0, 0.0, float(SW), float(SH))
        i += 1
        if C.shape[0] < 3 or _shoelace(C) < 1.0:
            continue  # outside the frustum, or a sliver
        Q = np.rint(C * Q8).astype(np.int64)
        keep = np.any(Q != np.roll(Q, 1, axis=0), axis=1)  # merge repeated points
        Q = Q[keep]
        ext = Q.max(axis=0) - Q.min(axis=0) if Q.shape[0] else np.zeros(2)
        if Q.shape[0] < 3 or ext.min() < 4 or not polygon_is_simple(Q):
            continue
        polys.append(Q)
    return polys


@functools.lru_cache(maxsize=16)
def make_tss(instance: int = 0, n: int | None = None, atlas: int | None = None,
             quality: int | None = None) -> AtlasInput:
    """A TSS-like frame (see TSS): instance 0 is the timed input."""
    nn = TSS["n"] if n is None else int(n)
    seed = config_seed("tss4k", instance) + (0 if n is None else 7919 * nn)
    polys = generate_tss_charts(nn, TSS["screen"], TSS["sigma"],
                                TSS["cover"] * nn / TSS["n"], seed)
    xy, offs = pack_csr(polys)
    side = TSS["W"] if atlas is None else int(atlas)
    return AtlasInput(xy, offs, side, side, TSS["p"], TSS["q"] if quality is None else quality)


@dataclasses.dataclass
class LoopsInput:
    """Charts of one or more boundary loops each: loop l is vertices
    [loop_offsets[l], loop_offsets[l+1]) of xy (Q8), chart c is loops
    [chart_loops[c], chart_loops[c+1])."""

    xy: np.ndarray
    loop_offsets: np.ndarray
    chart_loops: np.ndarray
    atlas_w: int
    atlas_h: int
    padding: int
    quality: int

    @property
    def n(self) -> int:
        return int(self.chart_loops.shape[0] - 1)

    def loops(self, c: int):
        out = []
        for l in range(int(self.chart_loops[c]), int(self.chart_loops[c + 1])):
            a, b = int(self.loop_offsets[l]), int(self.loop_offsets[l + 1])
            out.append(self.xy[2 * a:2 * b].reshape(-1, 2))
        return out


def loops_csr(charts, W, H, p, q):
    """LoopsInput from a list of charts, each a list of Q8 loops."""
    loops = [L for ch in charts for L in ch]
    xy, lofs = pack_csr(loops)
    cl = np.zeros(len(charts) + 1, np.int32)
    cl[1:] = np.cumsum([len(ch) for ch in charts])
    return LoopsInput(xy, lofs, cl, W, H, p, q)


def make_loops(n, W, H, p, q, seed, hole_frac=0.4, island_frac=0.2, fill=0.9):
    """Mesh-like charts: stars and L/U shapes, some with one or two holes
    (smaller loops inside, opposite orientation), some made of two islands
    side by side; log-normal areas (sigma 1.2) summing to `fill` of the
    atlas.  Returns (LoopsInput, the charts' outer loops only as an
    AtlasInput; islands have no single outer loop, that entry is None)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    mix = CONFIGS["mixed2k"]["mix"]
    base = generate_charts(n, W, H, 1.2, fill, mix, seed + 1)
    charts, outers = [], []
    for P in base:
        P = P.astype(np.int64)
        r = rng.uniform()
        c = P.mean(axis=0)
        if r < hole_frac:
            holes = []
            for _ in range(int(rng.integers(1, 3))):
                # a small square well inside: shrink towards an inner point until it fits
                ext = (P.max(0) - P.min(0)).min()
                hs = max(2, int(ext * rng.uniform(0.05, 0.12)))
                for t in np.linspace(0.0, 0.8, 9):
                    o = (c + t * (P[int(rng.integers(0, len(P)))] - c)).astype(np.int64)
                    Hq = np.array([o, o + [0, hs], o + [hs, hs], o + [hs, 0]], np.int64)
                    if _inside_all(Hq, P) and all(not _overlap_box(Hq, h2) for h2 in holes):
                        holes.append(Hq)
                        break
            charts.append([P] + holes)
            outers.append(P)
        elif r < hole_frac + island_frac:
            # two islands: the shape and a shifted, smaller copy beside it
            ext = P.max(0) - P.min(0)
            Q = ((P - P.min(0)) // 2 + P.min(0) + [ext[0] + 4 * 256, 0]).astype(np.int64)
            if polygon_is_simple(Q) and np.abs(Q).max() < (1 << 21):
                charts.append([P, Q])
                outers.append(None)
            else:
                charts.append([P])
                outers.append(P)
        else:
            charts.append([P])
            outers.append(P)
    return loops_csr(charts, W, H, p, q), outers


def _inside_all(Q, P):
    """Every vertex of Q strictly inside polygon P, and no edge of Q crossing P
    (even-odd test on the vertices; edges checked against P's edges)."""
    def inside(pt):
        x, y = pt
        c = False
        m = len(P)
        for i in range(m):
            (x1, y1), (x2, y2) = P[i], P[(i + 1) % m]
            if (y1 > y) != (y2 > y):
                xc = x1 + (x2 - x1) * (y - y1) / (y2 - y1)
                if xc == x:
                    return False
                if xc > x:
                    c = not c
        return c
    if not all(inside(q) for q in Q):
        return False
    both = np.concatenate([P, Q])
    return polygon_is_simple(P) and not _edges_cross(P, Q)


def _edges_cross(P, Q):
    for i in range(len(P)):
        a, b = P[i], P[(i + 1) % len(P)]
        for j in range(len(Q)):
            c, d = Q[j], Q[(j + 1) % len(Q)]
            d1 = _orient(*a, *b, *c)
            d2 = _orient(*a, *b, *d)
            d3 = _orient(*c, *d, *a)
            d4 = _orient(*c, *d, *b)
            if d1 * d2 <= 0 and d3 * d4 <= 0:
                return True
    return False


def _overlap_box(A, B):
    return not (A[:, 0].max() < B[:, 0].min() or B[:, 0].max() < A[:, 0].min() or
                A[:, 1].max() < B[:, 1].min() or B[:, 1].max() < A[:, 1].min())


def pack_csr(polys):
    offs = np.zeros(len(polys) + 1, np.int32)
    offs[1:] = np.cumsum([p.shape[0] for p in polys])
    xy = np.concatenate([p.reshape(-1) for p in polys]).astype(np.int32) if polys \
        else np.zeros(0, np.int32)
    return xy, offs


@functools.lru_cache(maxsize=64)
def make_input(name: str, instance: int = 0, quality: int | None = None,
               n: int | None = None) -> AtlasInput:
    """A named workload ('small', 'medium', 'large'); n overrides the chart
    count (same recipe) for reduced-size parity cases."""
    cfg = CONFIGS[name]
    nn = cfg["n"] if n is None else int(n)
    seed = config_seed(name, instance) + (0 if n is None else 7919 * nn)
    polys = generate_charts(nn, cfg["W"], cfg["H"], cfg["sigma"], cfg["fill"] * nn / cfg["n"]
                            if n is not None else cfg["fill"], cfg["mix"], seed)
    xy, offs = pack_csr(polys)
    return AtlasInput(xy, offs, cfg["W"], cfg["H"], cfg["p"],
                      cfg["q"] if quality is None else int(quality))


def make_custom(n, W, H, p, q, sigma, fill, mix, seed, fast=False) -> AtlasInput:
    polys = (generate_charts_fast if fast else generate_charts)(n, W, H, sigma, fill, mix, seed)
    xy, offs = pack_csr(polys)
    return AtlasInput(xy, offs, W, H, p, q)


def make_batch(count: int = 256, seed: int = 4000, nmin: int = 50, nmax: int = 5000):
    """Independent atlases with side drawn from {512,1024,2048} and chart counts
    uniform in [nmin, nmax], each drawn with the 2,000-chart recipe (70% stars,
    30% L/U, sigma 1.2, area 120% of the atlas)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sides = rng.choice([512, 1024, 2048], size=count)
    ns = rng.integers(nmin, nmax + 1, size=count)
    mix = CONFIGS["mixed2k"]["mix"]
    out = []
    for a in range(count):
        out.append(make_custom(int(ns[a]), int(sides[a]), int(sides[a]), 2, 2, 1.2, 1.2, mix,
                               seed * 1000 + a, fast=True))
    return out


def rect_input(n, a_q8, b_q8, W, H, p, q=2, seed=0, jitter_xy=True) -> AtlasInput:
    """n identical axis-aligned a x b rectangles (Q8 sides), at random offsets."""
    rng = np.random.Generator(np.random.PCG64(seed))
    polys = []
    for _ in range(n):
        ox, oy = (rng.integers(0, 1 << 18, 2) if jitter_xy else (0, 0))
        polys.append(np.array([[ox, oy], [ox + a_q8, oy], [ox + a_q8, oy + b_q8],
                               [ox, oy + b_q8]], np.int64))
    xy, offs = pack_csr(polys)
    return AtlasInput(xy, offs, W, H, p, q)


# --------------------------------------------------------------------------
# vectorised generation for large batches (same recipes, drawn family by
# family; a different random stream from generate_charts)
# --------------------------------------------------------------------------
def _simple_many(P: np.ndarray) -> np.ndarray:
    """polygon_is_simple over a stack of polygons P (B, m, 2) of equal m.
    Charts whose test involves a collinear triple are re-checked exactly one
    by one (rare)."""
    P = P.astype(np.int64)
    B, m, _ = P.shape
    ok = np.ones(B, bool)
    Q = np.roll(P, -1, axis=1)
    if np.any(np.all(P == Q, axis=2), axis=1).any():
        ok &= ~np.any(np.all(P == Q, axis=2), axis=1)
    ax, ay = P[:, :, None, 0], P[:, :, None, 1]
    bx, by = Q[:, :, None, 0], Q[:, :, None, 1]
    cx, cy = P[:, None, :, 0], P[:, None, :, 1]
    dx, dy = Q[:, None, :, 0], Q[:, None, :, 1]
    d1 = np.sign((bx - ax) * (cy - ay) - (by - ay) * (cx - ax))
    d2 = np.sign((bx - ax) * (dy - ay) - (by - ay) * (dx - ax))
    d3 = np.sign((dx - cx) * (ay - cy) - (dy - cy) * (ax - cx))
    d4 = np.sign((dx - cx) * (by - cy) - (dy - cy) * (bx - cx))
    idx = np.arange(m)
    far = ~((idx[:, None] == idx[None, :]) | ((idx[:, None] + 1) % m == idx[None, :]) |
            ((idx[None, :] + 1) % m == idx[:, None]))
    proper = (d1 * d2 < 0) & (d3 * d4 < 0) & far[None]
    ok &= ~proper.reshape(B, -1).any(axis=1)
    zero = ((d1 == 0) | (d2 == 0) | (d3 == 0) | (d4 == 0)) & far[None]
    suspect = zero.reshape(B, -1).any(axis=1)
    R = np.roll(P, -2, axis=1)
    e1, e2 = Q - P, R - Q
    cross = e1[..., 0] * e2[..., 1] - e1[..., 1] * e2[..., 0]
    dot = e1[..., 0] * e2[..., 0] + e1[..., 1] * e2[..., 1]
    ok &= ~((cross == 0) & (dot < 0)).any(axis=1)
    for b in np.nonzero(ok & suspect)[0]:
        ok[b] = polygon_is_simple(P[b])
    return ok


def _stars_many(rng, cnt, m, amax):
    ang = 2.0 * np.pi * (np.arange(m)[None, :] + rng.uniform(-0.3, 0.3, (cnt, m))) / m
    ang.sort(axis=1)
    r = 1.0 + rng.uniform(-0.4, 0.4, (cnt, m))
    a = rng.uniform(1.0, amax, cnt)
    x = r * np.cos(ang) * np.sqrt(a)[:, None]
    y = r * np.sin(ang) / np.sqrt(a)[:, None]
    phi = rng.uniform(0.0, np.pi, cnt)
    c, s = np.cos(phi)[:, None], np.sin(phi)[:, None]
    return np.stack([x * c - y * s, x * s + y * c], axis=2)


def _star_shaped(Q, C):
    """Exact sufficient test of simplicity: every vertex turns strictly
    counter-clockwise around the integer point C and the loop winds once."""
    D = Q - C[:, None, :]
    E = np.roll(D, -1, axis=1)
    cr = D[..., 0] * E[..., 1] - D[..., 1] * E[..., 0]
    # crossings of the ray from C along +x, counted upward
    up = (D[..., 1] < 0) & (E[..., 1] >= 0)
    winds = (cr > 0).all(axis=1) & (up.sum(axis=1) == 1)
    return winds


def _place_many(rng, P, areas, W, H, centre=None):
    x, y = P[..., 0], P[..., 1]
    A = 0.5 * np.abs((x * np.roll(y, -1, 1) - np.roll(x, -1, 1) * y).sum(1))
    sc = np.sqrt(areas / A)[:, None, None]
    P = P * sc
    lo = P.min(axis=1, keepdims=True)
    P = P - lo
    off = np.stack([rng.uniform(0, W, len(areas)), rng.uniform(0, H, len(areas))], 1)
    Q = np.rint((P + off[:, None, :]) * Q8).astype(np.int64)
    ext = Q.max(axis=1) - Q.min(axis=1)
    good = (ext.min(axis=1) >= 4) & (np.abs(Q).max(axis=(1, 2)) < (1 << 21))
    if centre is not None:
        C = np.rint((-lo[:, 0, :] + off) * Q8).astype(np.int64)
        fast = _star_shaped(Q, C)
        # counter-clockwise in (x, y) coordinates; the fast test proves simplicity
        rest = good & ~fast
        if rest.any():
            good[rest] = _simple_many(Q[rest])
    else:
        good &= _simple_many(Q)
    return Q, good


def generate_charts_fast(n, W, H, sigma, fill, mix, seed):
    """Vectorised counterpart of generate_charts for large batches."""
    rng = np.random.Generator(np.random.PCG64(seed))
    areas = np.exp(sigma * rng.standard_normal(n))
    areas *= fill * W * H / areas.sum()
    fracs = np.array([m[1] for m in mix], float)
    kinds = rng.choice(len(mix), size=n, p=fracs / fracs.sum())
    out = [None] * n
    for ki, (kind, _, vmin, vmax, amax) in enumerate(mix):
        ids = np.nonzero(kinds == ki)[0]
        if kind == "star":
            ms = rng.integers(vmin, vmax + 1, ids.size)
            for m in np.unique(ms):
                sel = ids[ms == m]
                for _attempt in range(64):
                    if sel.size == 0:
                        break
                    Q, good = _place_many(rng, _stars_many(rng, sel.size, int(m), amax),
                                          areas[sel], W, H, centre=True)
                    for j in np.nonzero(good)[0]:
                        out[sel[j]] = Q[j]
                    sel = sel[~good]
        else:
            sel = ids
            for _attempt in range(64):
                if sel.size == 0:
                    break
                polys = _lu_many(rng, sel.size, amax) if kind == "lu" else \
                    _quads_many(rng, sel.size, vmax, amax)
                left = []
                for m in sorted({p.shape[0] for p in polys}):
                    js = [j for j, p in enumerate(polys) if p.shape[0] == m]
                    Q, good = _place_many(rng, np.stack([polys[j] for j in js]), areas[sel[js]],
                                          W, H)
                    for jj, j in enumerate(js):
                        if good[jj]:
                            out[sel[j]] = Q[jj]
                        else:
                            left.append(sel[j])
                sel = np.array(sorted(left), dtype=np.int64)
    if any(p is None for p in out):  # pragma: no cover - vanishingly rare
        raise RuntimeError("could not draw a valid chart")
    return out


def _lu_many(rng, cnt, amax):
    """cnt L or U shapes (list of float polygons), as _lu draws them."""
    a = rng.uniform(1.0, amax, cnt)
    w, h = np.sqrt(a), 1.0 / np.sqrt(a)
    fx, fy = rng.uniform(0.3, 0.7, cnt), rng.uniform(0.3, 0.7, cnt)
    isL = rng.uniform(size=cnt) < 0.5
    turn = rng.integers(0, 4, cnt)
    mirror = rng.uniform(size=cnt) < 0.5
    free = rng.uniform(size=cnt) < 0.5
    phi = rng.uniform(0.0, np.pi, cnt)
    out = []
    for i in range(cnt):
        if isL[i]:
            P = np.array([[0, 0], [w[i], 0], [w[i], h[i] * fy[i]], [w[i] * fx[i], h[i] * fy[i]],
                          [w[i] * fx[i], h[i]], [0, h[i]]])
        else:
            nw = w[i] * fx[i]
            x0 = 0.5 * (w[i] - nw)
            P = np.array([[0, 0], [x0, 0], [x0, h[i] * fy[i]], [x0 + nw, h[i] * fy[i]], [x0 + nw, 0],
                          [w[i], 0], [w[i], h[i]], [0, h[i]]])
        P = _rot(P, turn[i] * np.pi / 2)
        if mirror[i]:
            P[:, 0] = -P[:, 0]
            P = P[::-1].copy()
        if free[i]:
            P = _rot(P, phi[i])
        out.append(P)
    return out


def _quads_many(rng, cnt, mv, amax):
    """cnt near-rectangular quads with 0..mv-4 extra edge vertices."""
    a = rng.uniform(1.0, amax, cnt)
    w, h = np.sqrt(a), 1.0 / np.sqrt(a)
    short = np.minimum(w, h)
    jit = rng.uniform(-0.05, 0.05, (cnt, 4, 2)) * short[:, None, None]
    extra = rng.integers(0, mv - 4 + 1, cnt)
    phi = rng.uniform(-np.pi / 18, np.pi / 18, cnt)
    out = []
    for i in range(cnt):
        corners = np.array([[0, 0], [w[i], 0], [w[i], h[i]], [0, h[i]]]) + jit[i]
        per_edge = np.bincount(rng.integers(0, 4, extra[i]), minlength=4)
        pts = []
        for e in range(4):
            p0, p1 = corners[e], corners[(e + 1) % 4]
            pts.append(p0)
            if per_edge[e]:
                ts = np.sort(rng.uniform(0.15, 0.85, per_edge[e]))
                d = p1 - p0
                nrm = np.array([-d[1], d[0]]) / (np.hypot(*d) + 1e-30)
                for t in ts:
                    pts.append(p0 + t * d + nrm * rng.uniform(-0.02, 0.02) * short[i])
        out.append(_rot(np.array(pts), phi[i]))
    return out
