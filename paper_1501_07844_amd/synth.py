"""Seeded synthetic workloads for the pseudo-flow continuous max-flow solvers.

This module only builds inputs: images, data terms D, smoothness terms S,
label graphs and ground-truth maps.  It contains none of the solver's
arithmetic (no divergence, projection, softmax or energy) and is imported by
both the tests of the reference CPU implementation and the GPU path, so that
the two always see identical float32 arrays.

Conventions
-----------
* Every array is float32 (int32 for label maps), laid out [B][L][Z][Y][X]
  with x fastest.  2-D problems have Z == 1 and ``ndim == 2``.
* Label graphs number the source 0.  Leaves (end-labels, nodes without
  children) are indexed in ascending node id; the data term D holds one field
  per leaf in that order.  Potts problems are the flat graph source -> leaves.
* The data term of every workload is a Gaussian negative log-likelihood with
  a shared sigma, D_L = (I - mu_L)^2 / (2 sigma^2); the label-independent
  constant is dropped, so D >= 0.
* All random draws come from ``numpy.random.default_rng(seed)`` in float64 and
  are cast to float32 once, in a fixed draw order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "LabelGraph", "Problem", "potts_graph", "potts2d_rects", "potts3d_voronoi",
    "hmf_ellipsoids", "dagmf_blobs", "diff_batch", "random_potts",
    "random_tree", "random_dag", "random_problem", "CONFIGS", "make_config",
    "ishikawa_levels", "hmf_tree", "dagmf_graph",
]


@dataclass
class LabelGraph:
    """A rooted label DAG as a plain edge list (source = node 0).

    ``weight`` may be None, meaning the default w_(A,B) = 1/|parents(B)|.
    """
    n_nodes: int
    parent: np.ndarray          # int32 [n_edges]
    child: np.ndarray           # int32 [n_edges]
    weight: Optional[np.ndarray] = None   # float64 [n_edges] or None

    @property
    def n_edges(self) -> int:
        return int(self.parent.shape[0])

    def leaves(self) -> List[int]:
        has_child = set(int(p) for p in self.parent)
        return [a for a in range(1, self.n_nodes) if a not in has_child]

    @property
    def n_leaf(self) -> int:
        return len(self.leaves())

    @property
    def n_node(self) -> int:
        """Non-source nodes."""
        return self.n_nodes - 1


@dataclass
class Problem:
    name: str
    ndim: int
    D: np.ndarray                      # float32 [B][n_leaf][Z][Y][X]
    S: np.ndarray                      # see s_mode
    s_mode: str                        # "node_scalar" | "shared_field" | "node_field"
    graph: LabelGraph
    gt: np.ndarray                     # int32 [B][Z][Y][X], leaf index of the truth
    c: float
    tau: float
    iters: int
    kind: str = "potts"                # "potts" | "hmf" | "dagmf"
    extra: dict = field(default_factory=dict)

    @property
    def shape(self) -> Tuple[int, int, int, int]:
        B, _, Z, Y, X = self.D.shape
        return B, Z, Y, X

    @property
    def n_leaf(self) -> int:
        return int(self.D.shape[1])

    @property
    def n_node(self) -> int:
        if self.kind == "ishikawa":
            return self.n_leaf - 1
        return self.graph.n_node

    @property
    def voxels(self) -> int:
        B, Z, Y, X = self.shape
        return B * Z * Y * X


# ---------------------------------------------------------------- helpers ---

def potts_graph(n_labels: int) -> LabelGraph:
    """Flat graph: source -> n_labels leaves, unit weights."""
    par = np.zeros(n_labels, np.int32)
    chi = np.arange(1, n_labels + 1, dtype=np.int32)
    return LabelGraph(n_labels + 1, par, chi, np.ones(n_labels))


def _gaussian_nll(I: np.ndarray, mu: Sequence[float], sigma: float) -> np.ndarray:
    """[..., Z, Y, X] float64 image -> float32 [..., L, Z, Y, X] data terms."""
    mu = np.asarray(mu, np.float64)
    out = np.empty(I.shape[:-3] + (len(mu),) + I.shape[-3:], np.float32)
    for k, m in enumerate(mu):
        out[..., k, :, :, :] = ((I - m) ** 2 / (2.0 * sigma * sigma)).astype(np.float32)
    return out


def _voronoi_labels(rng, shape, n_sites: int, n_classes: int) -> np.ndarray:
    """Nearest-site class map; sites uniform in the box, distances to voxel
    centres, ties to the lowest site index."""
    Z, Y, X = shape
    sites = rng.uniform(0.0, 1.0, size=(n_sites, 3)) * np.array([Z, Y, X], np.float64)
    cls = (np.arange(n_sites) % n_classes).astype(np.int32)
    yy = (np.arange(Y) + 0.5)[:, None, None]
    xx = (np.arange(X) + 0.5)[None, :, None]
    out = np.empty(shape, np.int32)
    sy = sites[None, None, :, 1]
    sx = sites[None, None, :, 2]
    dyx = (yy - sy) ** 2 + (xx - sx) ** 2          # [Y, X, n_sites]
    for z in range(Z):
        d = dyx + ((z + 0.5) - sites[:, 0]) ** 2
        out[z] = cls[np.argmin(d, axis=-1)]
    return out


# ----------------------------------------------------------- the configs ---

def potts2d_rects(seed: int = 1, ny: int = 64, nx: int = 64, iters: int = 200) -> Problem:
    """Potts 2-D, 3 labels: background class 0 and three axis-aligned
    rectangles painted class 1, 2, then 0; means 0.2/0.5/0.8, noise 0.1,
    constant S = 0.5."""
    rng = np.random.default_rng(seed)
    mu = (0.2, 0.5, 0.8)
    g = np.zeros((ny, nx), np.int32)
    lo, hi = max(2, (16 * ny) // 64), max(3, (40 * ny) // 64)
    for cls in (1, 2, 0):
        h, w = rng.integers(lo, hi + 1, size=2)
        h, w = min(int(h), ny), min(int(w), nx)
        y0 = int(rng.integers(0, ny - h + 1))
        x0 = int(rng.integers(0, nx - w + 1))
        g[y0:y0 + h, x0:x0 + w] = cls
    I = np.asarray(mu)[g] + 0.1 * rng.standard_normal((ny, nx))
    D = _gaussian_nll(I[None, None], mu, 0.1)          # [1][3][1][Y][X]
    S = np.full(3, 0.5, np.float32)
    return Problem("potts2d_rects", 2, D, S, "node_scalar", potts_graph(3),
                   g[None, None].astype(np.int32), c=4.0, tau=0.125, iters=iters)


def potts3d_voronoi(seed: int = 2, n: int = 256, iters: int = 500,
                    shape: Optional[Tuple[int, int, int]] = None) -> Problem:
    """Potts 3-D, 8 labels: 64-site Voronoi map (site j has class j mod 8),
    class means uniform in [0, 1], noise 0.15, S(x) = 0.3 exp(-|grad I|^2/0.01)
    from forward differences (zero on the last index) of the noisy image."""
    rng = np.random.default_rng(seed)
    shape = shape or (n, n, n)
    g = _voronoi_labels(rng, shape, 64, 8)
    mu = rng.uniform(0.0, 1.0, size=8)
    I = mu[g] + 0.15 * rng.standard_normal(shape)
    D = _gaussian_nll(I, mu, 0.15)[None]
    g2 = np.zeros(shape, np.float64)
    for ax in range(3):
        dif = np.diff(I, axis=ax)
        pad = [(0, 0)] * 3
        pad[ax] = (0, 1)
        g2 += np.pad(dif, pad) ** 2
    S = (0.3 * np.exp(-g2 / 0.01)).astype(np.float32)[None]
    return Problem("potts3d_voronoi", 3, D, S, "shared_field", potts_graph(8),
                   g[None].astype(np.int32), c=1.0, tau=0.125, iters=iters,
                   extra={"mu": mu})


def hmf_tree() -> LabelGraph:
    """S -> {1,2,3}; 1 -> {4,5,6}; 2 -> {7,8,9}; 3 -> {10,11}; unit weights."""
    edges = [(0, 1), (0, 2), (0, 3), (1, 4), (1, 5), (1, 6),
             (2, 7), (2, 8), (2, 9), (3, 10), (3, 11)]
    par = np.array([e[0] for e in edges], np.int32)
    chi = np.array([e[1] for e in edges], np.int32)
    return LabelGraph(12, par, chi, np.ones(len(edges)))


def hmf_ellipsoids(seed: int = 3, shape: Tuple[int, int, int] = (128, 256, 256),
                   iters: int = 300) -> Problem:
    """HMF 3-D on the 3 -> 8 tree: seven nested ellipsoids around a jittered
    centre (class = innermost containing shell, 0 outside), leaf means
    (k + 0.5)/8, noise 0.1, per-node constant S ~ U[0.1, 1.0]."""
    rng = np.random.default_rng(seed)
    Z, Y, X = shape
    ext = np.array([Z, Y, X], np.float64)
    centre = (ext - 1.0) / 2.0 + rng.uniform(-8.0, 8.0, size=3) * (ext / np.array([128., 256., 256.]))
    r1 = 0.45 * ext * rng.uniform(0.8, 1.0, size=3)
    radii = [r1]
    for j in range(2, 8):
        radii.append(r1 * (8 - j) / 8.0 * rng.uniform(0.9, 1.0, size=3))
    zz = np.arange(Z, dtype=np.float64)[:, None, None]
    yy = np.arange(Y, dtype=np.float64)[None, :, None]
    xx = np.arange(X, dtype=np.float64)[None, None, :]
    g = np.zeros(shape, np.int32)
    for j, r in enumerate(radii, start=1):
        inside = (((zz - centre[0]) / r[0]) ** 2 + ((yy - centre[1]) / r[1]) ** 2
                  + ((xx - centre[2]) / r[2]) ** 2) <= 1.0
        g[inside] = j
    mu = (np.arange(8) + 0.5) / 8.0
    I = mu[g] + 0.1 * rng.standard_normal(shape)
    D = _gaussian_nll(I, mu, 0.1)[None]
    S = rng.uniform(0.1, 1.0, size=11).astype(np.float32)
    return Problem("hmf_ellipsoids", 3, D, S, "node_scalar", hmf_tree(),
                   g[None].astype(np.int32), c=8.0, tau=0.125, iters=iters, kind="hmf")


def dagmf_graph(rng) -> LabelGraph:
    """S -> P1..P4 (w = 1); leaves 5..16 each pick two distinct parents
    uniformly (whole assignment redrawn until every parent has a child);
    w_(P, L) = 1/2."""
    while True:
        picks = [rng.choice(4, size=2, replace=False) + 1 for _ in range(12)]
        used = set(int(p) for pk in picks for p in pk)
        if used == {1, 2, 3, 4}:
            break
    par, chi, w = [], [], []
    for p in range(1, 5):
        par.append(0); chi.append(p); w.append(1.0)
    for i, pk in enumerate(picks):
        for p in sorted(int(v) for v in pk):
            par.append(p); chi.append(5 + i); w.append(0.5)
    return LabelGraph(17, np.array(par, np.int32), np.array(chi, np.int32), np.array(w))


def dagmf_blobs(seed: int = 4, shape: Tuple[int, int, int] = (256, 512, 512),
                iters: int = 300) -> Problem:
    """DAGMF 3-D, 4 shared parents x 12 leaves: background class 0 and 64
    painted balls (centre uniform, radius U[16, 64] at full size, class
    U{1..11}), leaf means (k + 0.5)/12, noise 0.1, per-node S ~ U[0.1, 1.0]."""
    rng = np.random.default_rng(seed)
    graph = dagmf_graph(rng)
    Z, Y, X = shape
    ext = np.array([Z, Y, X], np.float64)
    scale = float(np.min(ext / np.array([256., 512., 512.])))
    g = np.zeros(shape, np.int32)
    for _ in range(64):
        c = rng.uniform(0.0, 1.0, size=3) * ext
        r = rng.uniform(16.0, 64.0) * scale
        cls = int(rng.integers(1, 12))
        lo = np.maximum(np.floor(c - r), 0).astype(int)
        hi = np.minimum(np.ceil(c + r) + 1, ext).astype(int)
        if np.any(hi <= lo):
            continue
        zz = np.arange(lo[0], hi[0], dtype=np.float64)[:, None, None]
        yy = np.arange(lo[1], hi[1], dtype=np.float64)[None, :, None]
        xx = np.arange(lo[2], hi[2], dtype=np.float64)[None, None, :]
        m = (zz - c[0]) ** 2 + (yy - c[1]) ** 2 + (xx - c[2]) ** 2 <= r * r
        sub = g[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        sub[m] = cls
    mu = (np.arange(12) + 0.5) / 12.0
    I = mu[g] + 0.1 * rng.standard_normal(shape)
    D = _gaussian_nll(I, mu, 0.1)[None]
    S = rng.uniform(0.1, 1.0, size=16).astype(np.float32)
    return Problem("dagmf_blobs", 3, D, S, "node_scalar", graph,
                   g[None].astype(np.int32), c=8.0, tau=1.0 / 12.0, iters=iters, kind="dagmf")


def diff_batch(seed: int = 5, batch: int = 16, ny: int = 256, nx: int = 256,
               iters: int = 100) -> Problem:
    """Batch of 2-D Potts problems, 5 labels: 16-site Voronoi maps (class =
    site mod 5), means (k + 0.5)/5, noise 0.1, S a per-voxel field of 0.5."""
    rng = np.random.default_rng(seed)
    g = np.stack([_voronoi_labels(rng, (1, ny, nx), 16, 5) for _ in range(batch)])
    mu = (np.arange(5) + 0.5) / 5.0
    I = mu[g] + 0.1 * rng.standard_normal(g.shape)
    D = _gaussian_nll(I, mu, 0.1)                       # [B][5][1][Y][X]
    S = np.full((batch, 1, ny, nx), 0.5, np.float32)
    return Problem("diff_batch", 2, D, S, "shared_field", potts_graph(5),
                   g.astype(np.int32), c=2.0, tau=0.125, iters=iters,
                   extra={"checkpoint_every": 10})


def ishikawa_levels(seed: int = 6, shape: Tuple[int, int, int] = (1, 96, 128),
                    n_levels: int = 4, iters: int = 200) -> Problem:
    """Ordered-label workload for the Ishikawa chain: a smooth random field
    (sum of 12 Gaussian bumps) quantised into n_levels + 1 ordered levels,
    level means i / n_levels, noise 0.1, Gaussian-NLL data terms and one
    constant S per flow drawn from U[0.2, 0.6].  2-D when Z == 1."""
    rng = np.random.default_rng(seed)
    Z, Y, X = shape
    ext = np.array([Z, Y, X], np.float64)
    zz = np.arange(Z, dtype=np.float64)[:, None, None]
    yy = np.arange(Y, dtype=np.float64)[None, :, None]
    xx = np.arange(X, dtype=np.float64)[None, None, :]
    f = np.zeros(shape)
    for _ in range(12):
        c = rng.uniform(0.0, 1.0, size=3) * ext
        r = rng.uniform(0.1, 0.3) * float(np.max(ext))
        f += rng.uniform(-1.0, 1.0) * np.exp(-((zz - c[0]) ** 2 + (yy - c[1]) ** 2
                                               + (xx - c[2]) ** 2) / (2 * r * r))
    f = (f - f.min()) / max(f.max() - f.min(), 1e-12)
    g = np.minimum((f * (n_levels + 1)).astype(np.int32), n_levels)
    mu = np.arange(n_levels + 1) / n_levels
    I = mu[g] + 0.1 * rng.standard_normal(shape)
    D = _gaussian_nll(I, mu, 0.1)[None]
    S = rng.uniform(0.2, 0.6, size=n_levels).astype(np.float32)
    return Problem("ishikawa_levels", 2 if Z == 1 else 3, D, S, "node_scalar",
                   potts_graph(n_levels + 1), g[None].astype(np.int32), c=2.0, tau=0.0625,
                   iters=iters, kind="ishikawa")


# ------------------------------------------------------ generic fixtures ---

def random_tree(rng, n_internal: int, n_leaf: int) -> LabelGraph:
    """Random rooted tree with unit weights whose leaves are exactly the
    last n_leaf node ids (internal nodes first, each internal node gets at
    least one child)."""
    n = 1 + n_internal + n_leaf
    par, chi = [], []
    for a in range(1, 1 + n_internal):
        par.append(int(rng.integers(0, a))); chi.append(a)
    # guarantee every internal node has a child, then place the rest
    leaves = list(range(1 + n_internal, n))
    owners = list(range(1, 1 + n_internal)) if n_internal else [0]
    childless = [a for a in owners if a not in par]
    for i, L in enumerate(leaves):
        p = childless[i] if i < len(childless) else owners[int(rng.integers(0, len(owners)))]
        par.append(p); chi.append(L)
    return LabelGraph(n, np.array(par, np.int32), np.array(chi, np.int32), np.ones(len(par)))


def random_dag(rng, n_internal: int, n_leaf: int, max_parents: int = 2) -> LabelGraph:
    """Random rooted DAG: internal node a gets parents among {0..a-1}, each
    leaf 1..max_parents parents among the internal nodes (or the source),
    every internal node keeps at least one child; default weights."""
    n = 1 + n_internal + n_leaf
    par, chi = [], []
    for a in range(1, 1 + n_internal):
        k = int(rng.integers(1, min(max_parents, a) + 1))
        for p in rng.choice(a, size=k, replace=False):
            par.append(int(p)); chi.append(a)
    pool = list(range(1, 1 + n_internal)) if n_internal else [0]
    for L in range(1 + n_internal, n):
        k = int(rng.integers(1, min(max_parents, len(pool)) + 1))
        for p in rng.choice(pool, size=k, replace=False):
            par.append(int(p)); chi.append(L)
    has_child = set(par)
    for a in range(1, 1 + n_internal):
        if a not in has_child:
            par.append(a); chi.append(1 + n_internal + int(rng.integers(0, n_leaf)))
    return LabelGraph(n, np.array(par, np.int32), np.array(chi, np.int32), None)


def random_problem(seed: int, shape: Tuple[int, int, int], ndim: int, graph: LabelGraph,
                   batch: int = 1, s_mode: str = "node_scalar", d_scale: float = 4.0,
                   s_range: Tuple[float, float] = (0.1, 1.0), c: float = 4.0,
                   tau: float = 0.0625, iters: int = 20, kind: str = "dagmf") -> Problem:
    """Uniform-random D in [0, d_scale) and S in s_range, any graph."""
    rng = np.random.default_rng(seed)
    Z, Y, X = shape
    nl = graph.n_leaf
    D = rng.uniform(0.0, d_scale, size=(batch, nl, Z, Y, X)).astype(np.float32)
    if s_mode == "node_scalar":
        S = rng.uniform(*s_range, size=graph.n_node).astype(np.float32)
    elif s_mode == "shared_field":
        S = rng.uniform(*s_range, size=(batch, Z, Y, X)).astype(np.float32)
    elif s_mode == "node_field":
        S = rng.uniform(*s_range, size=(batch, graph.n_node, Z, Y, X)).astype(np.float32)
    else:
        raise ValueError(s_mode)
    gt = np.argmin(D, axis=1).astype(np.int32)
    return Problem(f"random_{seed}", ndim, D, S, s_mode, graph, gt, c, tau, iters, kind=kind)


def random_potts(seed: int, shape: Tuple[int, int, int], ndim: int, n_labels: int,
                 **kw) -> Problem:
    return random_problem(seed, shape, ndim, potts_graph(n_labels), kind="potts", **kw)


# Full-size workloads (the reduced parity sizes pass shape/n arguments).
CONFIGS = {
    1: potts2d_rects,
    2: potts3d_voronoi,
    3: hmf_ellipsoids,
    4: dagmf_blobs,
    5: diff_batch,
}


def make_config(k: int, **kw) -> Problem:
    return CONFIGS[k](**kw)
