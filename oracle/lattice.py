"""Lattice geometry for the oracle (test infrastructure).

The paper puts quark fields on lattice sites and gauge links on the links
between them (Sec. II, Fig. 1) and leaves the storage order to its companion
single-GPU paper, which is not available.  The reading used here:

* dims = (Lx, Ly, Lz, Lt), every extent even and >= 2, periodic in all four
  directions;
* lexicographic index lex = x + Lx*(y + Ly*(z + Lz*t))  (x fastest);
* parity p = (x+y+z+t) mod 2;
* even-odd index eo = p*N/2 + lex//2 (all even sites first).  Because Lx is
  even, lex//2 is a bijection on each parity class;
* direction d in 0..7: d<4 is the forward hop +mu (mu = d, 0..3 = x,y,z,t),
  d>=4 the backward hop -mu (mu = d-4).
"""
from __future__ import annotations

import numpy as np


class Lattice:
    def __init__(self, dims):
        dims = tuple(int(d) for d in dims)
        if len(dims) != 4 or any(d < 2 or d % 2 for d in dims):
            raise ValueError("every lattice extent must be even and >= 2: %r" % (dims,))
        self.dims = dims
        self.N = dims[0] * dims[1] * dims[2] * dims[3]
        # array shape of a lexicographic field: t slowest, x fastest
        self.shape = (dims[3], dims[2], dims[1], dims[0])

    # -- single-site helpers (plain Python, used for hand examples) --------
    def lex(self, x, y, z, t) -> int:
        lx, ly, lz, _ = self.dims
        return x + lx * (y + ly * (z + lz * t))

    def coords(self, lex):
        lx, ly, lz, _ = self.dims
        x = lex % lx
        y = (lex // lx) % ly
        z = (lex // (lx * ly)) % lz
        t = lex // (lx * ly * lz)
        return (x, y, z, t)

    def parity(self, x, y, z, t) -> int:
        return (x + y + z + t) % 2

    def eo(self, x, y, z, t) -> int:
        return self.parity(x, y, z, t) * (self.N // 2) + self.lex(x, y, z, t) // 2

    def hop(self, coords, d):
        """Coordinates of the neighbour of `coords` in direction d (periodic)."""
        c = list(coords)
        mu = d % 4
        step = 1 if d < 4 else -1
        c[mu] = (c[mu] + step) % self.dims[mu]
        return tuple(c)

    # -- whole-lattice tables ------------------------------------------------
    def eo_of_lex(self) -> np.ndarray:
        """eo index of every site, indexed by lex (int64 [N])."""
        out = np.empty(self.N, dtype=np.int64)
        for lex in range(self.N):
            out[lex] = self.eo(*self.coords(lex))
        return out

    def neighbor_table(self) -> np.ndarray:
        """int32 [8][N]: table[d][eo(s)] = eo(neighbour of s in direction d).

        Built site by site from the definition above, without any of the
        shortcuts an optimised kernel would use.
        """
        table = np.empty((8, self.N), dtype=np.int32)
        for lex in range(self.N):
            c = self.coords(lex)
            e = self.eo(*c)
            for d in range(8):
                table[d, e] = self.eo(*self.hop(c, d))
        return table

    # -- layout conversion between lexicographic and even-odd order ---------
    def to_eo(self, field_lex: np.ndarray) -> np.ndarray:
        """Reorder a [N,...] lexicographic field into even-odd site order."""
        out = np.empty_like(field_lex)
        out[self.eo_of_lex()] = field_lex
        return out

    def from_eo(self, field_eo: np.ndarray) -> np.ndarray:
        return field_eo[self.eo_of_lex()]
