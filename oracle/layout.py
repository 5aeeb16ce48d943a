"""Tile layout, consensus weights and PSF-interpolation weights (FP64).

Coordinates: the observed image y covers [0, M) per axis.  The unknown image
x lives on the larger domain X = [-r, M + r) (the sensor sees less than the
optics, Eq. (2) footnote; the dashed extra pixels of Fig. 1), stored with an
offset of r so X-array index = coordinate + r.

Tiles (Section III-A, "N overlapping blocks"): along one axis block a is
B_a = [a p, min(a p + p + o, M)) for a < T-1 and B_{T-1} = [(T-1) p, M).
Its support P_a = B_a dilated by r on both sides is the set of unknowns the
node estimates; neighbouring supports overlap by o + 2r pixels.

Consensus weights omega (Fig. 1, first-order interpolation weights in [0, 1]
summing to one): 1 inside a support except over each overlap with a
neighbour, where the lower tile ramps (L - s - 1/2)/L and the upper tile
ramps (s + 1/2)/L, s = 0..L-1 from the overlap start.  The half-pixel offset
keeps omega > 0 so the metric alpha = gamma * omega is positive definite
(Section III-B needs V positive definite).

Grid layout (Section III-C, smooth shift-variant blur): one tile per PSF
node, T = G, and block a spans the grid points a - 1 .. a + 1: the pixels
strictly between c_{a-1} and c_{a+1} (c_k the node centres below), the first
block from 0 and the last to M.  Adjacent blocks overlap by half an interior
block, so an observed pixel lies in two blocks per axis (four in 2-D), and
near a node, within r, the supports of three tiles meet.  The consensus
weight there is the node's tent widened to reach over its support,
phi_a(i) = max(0, 1 - |i - c_a| / (q + r + 1/2)), normalised over the tiles
covering i: omega_a = phi_a / sum_b phi_b.  It is positive on the support
and sums to one over the covering tiles; between two nodes, where only two
tiles cover, it is linear.  Requires 2r <= q (at most three tiles meet).

PSF-interpolation weights (Section II-B, first-order interpolation between
PSFs sampled on a regular grid): G nodes per axis at c_k = (k + 1/2) q - 1/2
with q = M / G; the tent w_k(i) = max(0, 1 - |i - c_k| / q), held at 1 beyond
the outer nodes, so sum_k w_k = 1 on the whole of X.  2-D weights are
products of the 1-D ones.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class AxisLayout:
    """One axis of the tiling and of the PSF grid."""

    M: int       # observed length
    T: int       # tiles
    p: int       # tile pitch
    o: int       # overlap of blocks
    r: int       # PSF half-width
    G: int       # PSF nodes
    kind: str = "pitch"   # "pitch": blocks from p and o; "grid": one block per node (Section III-C)

    def __post_init__(self):
        if self.T < 1 or self.G < 1 or self.r < 0:
            raise ValueError("bad axis layout")
        if self.kind not in ("pitch", "grid"):
            raise ValueError("kind must be 'pitch' or 'grid'")
        if self.kind == "grid":
            if self.T != self.G:
                raise ValueError("the grid layout has one tile per PSF node")
            if self.G > 1 and 2 * self.r > self.M / self.G:
                raise ValueError("the grid layout needs 2r <= the node spacing")
        elif self.T > 1:
            if self.o + 2 * self.r > self.p:
                raise ValueError("overlap + 2r must not exceed the pitch")
            if self.M - (self.T - 1) * self.p <= self.o:
                raise ValueError("last block must extend past the previous one")
        for a in range(self.T):
            s, e = self.block(a)
            if e - s < 2 * self.r + 1:
                raise ValueError("block smaller than the PSF")

    # --- tiles ------------------------------------------------------------
    def block(self, a):
        """Observed-pixel interval [start, end) of block a."""
        if self.kind == "grid":
            start = 0 if a == 0 else int(np.floor(self.node_centre(a - 1))) + 1
            end = self.M if a == self.T - 1 else int(np.ceil(self.node_centre(a + 1)))
            return start, end
        start = a * self.p
        end = self.M if a == self.T - 1 else min(a * self.p + self.p + self.o, self.M)
        return start, end

    def support(self, a):
        """Interval of unknowns P_a = block dilated by r (observed coordinates)."""
        s, e = self.block(a)
        return s - self.r, e + self.r

    def support_len(self, a):
        s, e = self.support(a)
        return e - s

    def _grid_phi(self, a, coords):
        h = self.M / self.G + self.r + 0.5
        return np.maximum(0.0, 1.0 - np.abs(np.asarray(coords, dtype=np.float64) - self.node_centre(a)) / h)

    def omega(self, a):
        """Consensus weight of tile a on its support (1-D, float64)."""
        s0, s1 = self.support(a)
        if self.kind == "grid":
            coords = np.arange(s0, s1)
            den = np.zeros(s1 - s0)
            for b in range(self.T):
                b0, b1 = self.support(b)
                inside = (coords >= b0) & (coords < b1)
                den += np.where(inside, self._grid_phi(b, coords), 0.0)
            return self._grid_phi(a, coords) / den
        w = np.ones(s1 - s0)
        if a > 0:
            _, prev_end = self.support(a - 1)
            L = prev_end - s0
            s = np.arange(L)
            w[:L] = (s + 0.5) / L
        if a < self.T - 1:
            nxt_start, _ = self.support(a + 1)
            L = s1 - nxt_start
            s = np.arange(L)
            w[nxt_start - s0:] = (L - s - 0.5) / L
        return w

    # --- PSF grid -----------------------------------------------------------
    def node_centre(self, k):
        q = self.M / self.G
        return (k + 0.5) * q - 0.5

    def tent(self, k, coords):
        """First-order interpolation weight of node k at observed coordinates."""
        coords = np.asarray(coords, dtype=np.float64)
        q = self.M / self.G
        c = self.node_centre(k)
        w = np.maximum(0.0, 1.0 - np.abs(coords - c) / q)
        if k == 0:
            w = np.where(coords <= c, 1.0, w)
        if k == self.G - 1:
            w = np.where(coords >= c, 1.0, w)
        return w

    def tile_nodes(self, a):
        """Nodes whose tent is non-zero somewhere on the support of tile a."""
        s0, s1 = self.support(a)
        coords = np.arange(s0, s1)
        return [k for k in range(self.G) if np.any(self.tent(k, coords) > 0.0)]


@dataclasses.dataclass(frozen=True)
class Layout:
    """2-D layout: tile t = a * T_x + b covers rows of axis y, columns of axis x."""

    ay: AxisLayout
    ax: AxisLayout
    model: str = "interp"   # "interp": sum over the nodes of the tile; "local": node t only

    def __post_init__(self):
        if self.model not in ("interp", "local"):
            raise ValueError("model must be 'interp' or 'local'")
        if self.model == "local" and (self.ay.G != self.ay.T or self.ax.G != self.ax.T):
            raise ValueError("local model needs one PSF per tile")

    @property
    def n_tiles(self):
        return self.ay.T * self.ax.T

    @property
    def r(self):
        return self.ay.r

    @property
    def X_shape(self):
        return (self.ay.M + 2 * self.ay.r, self.ax.M + 2 * self.ax.r)

    def tile_ab(self, t):
        return divmod(t, self.ax.T)

    def block(self, t):
        a, b = self.tile_ab(t)
        return self.ay.block(a), self.ax.block(b)

    def support(self, t):
        a, b = self.tile_ab(t)
        return self.ay.support(a), self.ax.support(b)

    def support_shape(self, t):
        a, b = self.tile_ab(t)
        return self.ay.support_len(a), self.ax.support_len(b)

    def block_shape(self, t):
        (y0, y1), (x0, x1) = self.block(t)
        return y1 - y0, x1 - x0

    def omega(self, t):
        """2-D consensus weight omega_t on the support of tile t."""
        a, b = self.tile_ab(t)
        return np.outer(self.ay.omega(a), self.ax.omega(b))

    def terms(self, t):
        """Cached list of (node index, weight on the support); see _terms."""
        cache = self.__dict__.setdefault("_terms_cache", {})
        if t not in cache:
            cache[t] = self._terms(t)
        return cache[t]

    def _terms(self, t):
        """List of (node index ky * G_x + kx, w_k on the support) for tile t.

        Interp model: every node whose tent touches the support, with the
        tent product as weight (the restriction of the global interpolated
        operator to the tile).  Local model: the tile's own node, weight 1
        (the paper's H_i = C_i calH_i of Section II-B).
        """
        a, b = self.tile_ab(t)
        shape = self.support_shape(t)
        if self.model == "local":
            return [(a * self.ax.G + b, np.ones(shape))]
        (y0, y1), (x0, x1) = self.support(t)
        ry, rx = np.arange(y0, y1), np.arange(x0, x1)
        out = []
        for ky in self.ay.tile_nodes(a):
            wy = self.ay.tent(ky, ry)
            for kx in self.ax.tile_nodes(b):
                wx = self.ax.tent(kx, rx)
                out.append((ky * self.ax.G + kx, np.outer(wy, wx)))
        return out

    def restrict(self, x_global, t):
        """S_t: the support of tile t cut out of an array on X."""
        (y0, y1), (x0, x1) = self.support(t)
        r = self.r
        return x_global[y0 + r:y1 + r, x0 + r:x1 + r].copy()

    def block_of(self, y_global, t):
        """The observed block B_t cut out of an array on [0, M)^2."""
        (y0, y1), (x0, x1) = self.block(t)
        return y_global[y0:y1, x0:x1].copy()


def make_layout(M, T, p, o, P, G, model="interp", M_x=None, T_x=None, G_x=None, kind="pitch"):
    """Square-by-default layout helper (P = PSF size 2r+1).  kind="grid": the
    Section III-C layout (one tile per node; p and o unused)."""
    r = P // 2
    ay = AxisLayout(M, T, p, o, r, G, kind)
    ax = AxisLayout(M if M_x is None else M_x, T if T_x is None else T_x, p, o, r,
                    G if G_x is None else G_x, kind)
    return Layout(ay, ax, model)
