"""Gridding NUFFT (Kaiser-Bessel, oversampled FFT) in FP64, plus binning.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The NUFFT approximates the exact SENSE operator of Problem Setup
(Eq. model_i) and is built "following Beatty et al." with oversampling alpha
and kernel width W (Experiments section).  The steps, in order:

Forward  y = A x
  1. z_c[n] = x[n] s_c[n] / (sqrt(N) prod_a Chat(n_a / G_a)), placed at grid
     position n mod G (centred n, no shift).
  2. Z_c = unnormalised forward DFT of z_c over the G grid (numpy.fft).
  3. y_c[i] = sum over the W^d taps j of prod_a C(g_ia - j_a) Z_c[(j - G/2) mod G].

Adjoint  x = A^H y  (the exact transpose of the above)
  1. Spread: Z'_c[(j - G/2) mod G] += prod_a C(g_ia - j_a) y_c[i].
  2. Unnormalised inverse DFT (sign +, no 1/G).
  3. Crop n, multiply by conj(s_c) / (sqrt(N) prod Chat), sum over coils.

Canonical grid coordinates (exact float32 pipeline, no fused multiply-add):
  c_a = fl32(G_a / (2 pi))            (computed in float64, rounded once)
  t   = fl32(omega_a * c_a)
  g_a = fl32(t + G_a / 2)
  if g_a <  0:   g_a = fl32(g_a + G_a)
  if g_a >= G_a: g_a = fl32(g_a - G_a)
A coordinate whose g_a is still outside [0, G_a) (|omega| beyond about 3 pi,
NaN, inf) is rejected.  The shifted coordinate g = omega G / (2 pi) + G/2
places k = 0 at grid cell G/2; tap j then addresses DFT bin (j - G/2) mod G.
The taps of a sample are j_a = cell_a - W/2 + 1 + t_a, t_a = 0..W-1, with
cell_a = floor(g_a); weights are evaluated in float64 at u = (double)g_a - j_a.

Binning: tile (bin) of a sample = (cell_a // B_a) per axis, linear key
row-major (last axis fastest); the permutation is the stable argsort of the
key and the bin offsets its exclusive prefix count.  The tile touch list of
tile T is the ascending list of sorted sample positions whose W^d footprint
(taken mod G) meets T.

Pins: NUFFT vs the exact NDFT on small grids with errors shrinking as W
grows; adjoint identity to 1e-12; on-grid Cartesian samples; the sort
against its defining properties (tests/test_oracle_operators.py).
"""
from __future__ import annotations

import copy
import itertools
import math

import numpy as np

from . import kb


def grid_shape(shape, alpha):
    return tuple(kb.grid_size(n, alpha) for n in shape)


def canonical_coords(coords, G):
    """float32 (M, d) grid coordinates in [0, G_a); raises on invalid input."""
    k = np.asarray(coords)
    if k.dtype != np.float32:
        raise TypeError("coordinates must be float32")
    M, d = k.shape
    g = np.empty((M, d), dtype=np.float32)
    for a in range(d):
        Ga = int(G[a])
        c = np.float32(Ga / (2.0 * math.pi))
        t = np.multiply(k[:, a], c, dtype=np.float32)
        ga = np.add(t, np.float32(Ga // 2), dtype=np.float32)
        neg = ga < 0
        ga = np.where(neg, np.add(ga, np.float32(Ga), dtype=np.float32), ga)
        big = ga >= np.float32(Ga)
        ga = np.where(big, np.subtract(ga, np.float32(Ga), dtype=np.float32), ga)
        bad = ~((ga >= 0) & (ga < np.float32(Ga)))
        if np.any(bad):
            raise ValueError("coordinate out of range on axis %d" % a)
        g[:, a] = ga
    return g


def cells(g):
    return np.floor(g.astype(np.float64)).astype(np.int64)


def bin_keys(g, G, B):
    """Row-major linear tile index of each sample's cell."""
    cl = cells(g)
    d = g.shape[1]
    nb = [int(G[a]) // int(B[a]) for a in range(d)]
    key = np.zeros(g.shape[0], dtype=np.int64)
    for a in range(d):
        key = key * nb[a] + cl[:, a] // int(B[a])
    return key, nb


def sort_by_bin(g, G, B):
    """(perm, offsets): stable argsort of the bin key and bin start offsets."""
    key, nb = bin_keys(g, G, B)
    nbins = int(np.prod(nb))
    perm = np.argsort(key, kind="stable")
    counts = np.bincount(key, minlength=nbins)
    offsets = np.concatenate([[0], np.cumsum(counts)])
    return perm.astype(np.int64), offsets.astype(np.int64)


def tile_touch_lists(g_sorted, G, B, W):
    """For each tile, the ascending sorted-sample positions touching it.

    Returned in CSR form (offsets[ntiles+1], entries[...]).
    """
    M, d = g_sorted.shape
    cl = cells(g_sorted)
    nb = [int(G[a]) // int(B[a]) for a in range(d)]
    per_axis = []
    for a in range(d):
        tl = [((cl[:, a] - W // 2 + 1 + t) % int(G[a])) // int(B[a]) for t in range(W)]
        per_axis.append(np.stack(tl, axis=1))            # (M, W) tile index per tap
    pairs_t, pairs_s = [], []
    idx = np.arange(M, dtype=np.int64)
    seen = set()
    keys = []
    for combo in itertools.product(range(W), repeat=d):
        key = np.zeros(M, dtype=np.int64)
        for a in range(d):
            key = key * nb[a] + per_axis[a][:, combo[a]]
        keys.append(key)
    K = np.stack(keys, axis=1)                           # (M, W^d)
    # unique (tile, sample) pairs
    flat_t = K.ravel()
    flat_s = np.repeat(idx, K.shape[1])
    pair = np.unique(flat_t * M + flat_s)
    tiles = pair // M
    samples = pair % M
    ntiles = int(np.prod(nb))
    counts = np.bincount(tiles, minlength=ntiles)
    offsets = np.concatenate([[0], np.cumsum(counts)])
    return offsets.astype(np.int64), samples.astype(np.int64)


class Nufft:
    """Plain gridding NUFFT for a fixed trajectory, image shape and maps."""

    def __init__(self, coords, shape, maps=None, alpha=2.0, width=4):
        self.shape = tuple(int(n) for n in shape)
        self.d = len(self.shape)
        self.N = int(np.prod(self.shape))
        self.alpha = float(np.float32(alpha))
        self.W = int(width)
        self.G = grid_shape(self.shape, alpha)
        self.beta = kb.kb_beta(alpha, width)
        self.maps = None if maps is None else np.asarray(maps, dtype=np.complex128)
        self.C = 1 if maps is None else self.maps.shape[0]
        self.coords = np.asarray(coords, dtype=np.float32)
        self.M = self.coords.shape[0]
        self.g = canonical_coords(self.coords, self.G)
        self.cell = cells(self.g)
        # deapodisation: 1 / (sqrt(N) prod_a Chat(n_a / G_a)), separable
        scale = np.ones(self.shape)
        for a, n in enumerate(self.shape):
            nu = (np.arange(n) - n // 2) / self.G[a]
            s = 1.0 / kb.kb_ft(nu, self.W, self.beta)
            sh = [1] * self.d
            sh[a] = n
            scale = scale * s.reshape(sh)
        self.scale = scale / math.sqrt(self.N)
        # grid positions n mod G of the centred image
        self.pos = [(np.arange(n) - n // 2) % self.G[a] for a, n in enumerate(self.shape)]
        # taps: flat grid index and weight for every (sample, tap)
        self._taps = self._make_taps()

    def with_maps(self, maps):
        """The same operator (trajectory, grid, taps) with other coil maps."""
        other = copy.copy(self)
        other.maps = None if maps is None else np.asarray(maps, dtype=np.complex128)
        other.C = 1 if maps is None else other.maps.shape[0]
        return other

    def _make_taps(self):
        taps = []
        for combo in itertools.product(range(self.W), repeat=self.d):
            w = np.ones(self.M)
            flat = np.zeros(self.M, dtype=np.int64)
            for a in range(self.d):
                j = self.cell[:, a] - self.W // 2 + 1 + combo[a]
                u = self.g[:, a].astype(np.float64) - j
                w = w * kb.kb_kernel(u, self.W, self.beta)
                flat = flat * self.G[a] + (j - self.G[a] // 2) % self.G[a]
            taps.append((flat, w))
        return taps

    def _maps(self):
        if self.maps is None:
            return np.ones((1,) + self.shape, dtype=np.complex128)
        return self.maps

    def interp(self, Z):
        """y[i] = sum_taps w Z[flat] for one grid Z."""
        Zf = Z.ravel()
        y = np.zeros(self.M, dtype=np.complex128)
        for flat, w in self._taps:
            y += w * Zf[flat]
        return y

    def spread(self, y):
        """Transpose of interp: a G-grid."""
        size = int(np.prod(self.G))
        re = np.zeros(size)
        im = np.zeros(size)
        for flat, w in self._taps:
            re += np.bincount(flat, weights=w * y.real, minlength=size)
            im += np.bincount(flat, weights=w * y.imag, minlength=size)
        return (re + 1j * im).reshape(self.G)

    def pad(self, img):
        z = np.zeros(self.G, dtype=np.complex128)
        z[np.ix_(*self.pos)] = img
        return z

    def crop(self, Z):
        return Z[np.ix_(*self.pos)]

    def forward_image(self, z_img):
        """Forward for one coil image (maps already applied), no 1/sqrt(N) loss."""
        Z = np.fft.fftn(self.pad(z_img * self.scale))
        return self.interp(Z)

    def adjoint_image(self, y):
        Z = self.spread(y)
        img = self.crop(np.fft.ifftn(Z) * float(np.prod(self.G)))
        return img * self.scale

    def forward(self, x):
        x = np.asarray(x, dtype=np.complex128).reshape(self.shape)
        S = self._maps()
        return np.stack([self.forward_image(S[c] * x) for c in range(S.shape[0])])

    def adjoint(self, y):
        S = self._maps()
        y = np.asarray(y, dtype=np.complex128).reshape(S.shape[0], self.M)
        x = np.zeros(self.shape, dtype=np.complex128)
        for c in range(S.shape[0]):
            x += np.conj(S[c]) * self.adjoint_image(y[c])
        return x

    # multichannel forms without coil maps (one image per channel)
    def forward_channels(self, imgs):
        return np.stack([self.forward_image(im) for im in imgs])

    def adjoint_channels(self, y):
        return np.stack([self.adjoint_image(yc) for yc in y])
