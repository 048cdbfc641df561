"""Periodic atomic structures for seeded synthetic workloads.

Every generator takes a ``numpy.random.Generator`` and returns
``(cell, positions, types)``: ``cell`` is 3x3 with rows a, b, c (Angstrom),
``positions`` is ``[n, 3]`` Cartesian and wrapped into the cell, ``types`` is
``int32 [n]``.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

_FCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
_BCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])


@dataclass
class Batch:
    """A packed batch of structures (all arrays host-side numpy)."""

    positions: np.ndarray  # float64 [Na, 3]
    types: np.ndarray  # int32 [Na]
    cells: np.ndarray  # float64 [Ns, 3, 3], rows a, b, c
    atom_offset: np.ndarray  # int64 [Ns + 1]
    num_types: int

    @property
    def num_structures(self) -> int:
        return int(self.cells.shape[0])

    @property
    def num_atoms(self) -> int:
        return int(self.positions.shape[0])

    def counts(self) -> np.ndarray:
        return np.diff(self.atom_offset)

    def structure(self, s: int):
        a, b = int(self.atom_offset[s]), int(self.atom_offset[s + 1])
        return self.cells[s], self.positions[a:b], self.types[a:b]

    def subset(self, idx) -> "Batch":
        return pack([self.structure(int(s)) for s in idx], self.num_types)


def pack(structs, num_types: int) -> Batch:
    cells = np.stack([np.asarray(c, dtype=np.float64) for c, _, _ in structs])
    pos = np.concatenate([np.asarray(p, dtype=np.float64) for _, p, _ in structs])
    typ = np.concatenate([np.asarray(t, dtype=np.int32) for _, _, t in structs])
    off = np.zeros(len(structs) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(p) for _, p, _ in structs])
    return Batch(pos, typ, cells, off, int(num_types))


def wrap(cell: np.ndarray, pos: np.ndarray) -> np.ndarray:
    frac = pos @ np.linalg.inv(cell)
    frac -= np.floor(frac)
    frac[frac >= 1.0] = 0.0
    return frac @ cell


def near_cubic_dims(sites_per_cell: int, n: int):
    """Smallest supercell (n1 <= n2 <= n3, n3 - n1 <= 1) holding at least n sites."""
    best = None
    for n1 in range(1, 64):
        for n2 in (n1, n1 + 1):
            for n3 in (n2, n2 + 1):
                if n3 - n1 > 1:
                    continue
                cap = sites_per_cell * n1 * n2 * n3
                if cap >= n and (best is None or n1 * n2 * n3 < best[0]):
                    best = (n1 * n2 * n3, (n1, n2, n3))
        if best is not None and sites_per_cell * n1 ** 3 > n:
            break
    return best[1]


def lattice_sites(basis: np.ndarray, dims, a: float):
    n1, n2, n3 = dims
    g = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), -1)
    g = g.reshape(-1, 1, 3) + basis[None, :, :]
    frac = g.reshape(-1, 3) / np.array([n1, n2, n3], dtype=np.float64)
    cell = np.diag([n1 * a, n2 * a, n3 * a]).astype(np.float64)
    return cell, frac @ cell


def symmetric_strain(rng: np.random.Generator, max_abs: float) -> np.ndarray:
    e = rng.uniform(-max_abs, max_abs, size=(3, 3))
    return np.triu(e) + np.triu(e, 1).T


def assign_species(rng: np.random.Generator, n: int, num_types: int) -> np.ndarray:
    if num_types == 1:
        return np.zeros(n, dtype=np.int32)
    frac = rng.dirichlet(np.ones(num_types))
    raw = frac * n
    cnt = np.floor(raw).astype(np.int64)
    rem = n - int(cnt.sum())
    order = np.argsort(-(raw - cnt), kind="stable")
    cnt[order[:rem]] += 1
    types = np.repeat(np.arange(num_types, dtype=np.int32), cnt)
    return types[rng.permutation(n)].astype(np.int32)


def _crystal(rng, basis, a, n, sigma, strain, num_types, exact_dims=None):
    dims = exact_dims if exact_dims is not None else near_cubic_dims(len(basis), n)
    cell, pos = lattice_sites(basis, dims, a)
    if len(pos) > n:
        keep = np.sort(rng.choice(len(pos), size=n, replace=False))
        pos = pos[keep]
    if strain > 0.0:
        f = np.eye(3) + symmetric_strain(rng, strain)
        cell = cell @ f.T
        pos = pos @ f.T
    if sigma > 0.0:
        pos = pos + rng.normal(0.0, sigma, size=pos.shape)
    types = assign_species(rng, n, num_types)
    return cell, wrap(cell, pos), types


def fcc_structure(rng, n, a=4.0, sigma=0.15, strain=0.0, num_types=1, exact_dims=None):
    return _crystal(rng, _FCC_BASIS, a, n, sigma, strain, num_types, exact_dims)


def bcc_structure(rng, n, a=3.2, sigma=0.1, strain=0.0, num_types=1, exact_dims=None):
    return _crystal(rng, _BCC_BASIS, a, n, sigma, strain, num_types, exact_dims)


def _min_image_d2(box, pts, p):
    d = pts - p
    d -= box * np.round(d / box)
    return np.einsum("ij,ij->i", d, d)


def random_packing(rng, n, density=0.0625, d_min=1.8, num_types=1, max_tries=200000):
    """Random sequential addition in a cubic periodic box at number density ``density``."""
    side = (n / density) ** (1.0 / 3.0)
    box = np.full(3, side)
    pts = np.empty((0, 3))
    tries = 0
    while len(pts) < n:
        p = rng.uniform(0.0, side, size=3)
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random packing did not converge")
        if len(pts) == 0 or _min_image_d2(box, pts, p).min() >= d_min * d_min:
            pts = np.vstack([pts, p])
    cell = np.diag(box)
    return cell, wrap(cell, pts), assign_species(rng, n, num_types)


def dense_liquid(rng, n, density=0.11, sigma=0.3, d_min=1.8, num_types=1):
    """fcc lattice at ``density`` with Gaussian noise; atoms closer than d_min are redrawn."""
    from scipy.spatial import cKDTree

    a = (4.0 / density) ** (1.0 / 3.0)
    cell, pos, types = fcc_structure(rng, n, a=a, sigma=sigma, num_types=num_types)
    box = np.diag(cell).copy()
    for _ in range(64):
        tree = cKDTree(pos, boxsize=box)
        pairs = tree.query_pairs(d_min, output_type="ndarray")
        if len(pairs) == 0:
            break
        bad = np.unique(pairs[:, 1])
        pos[bad] = rng.uniform(0.0, 1.0, size=(len(bad), 3)) * box
    return cell, wrap(cell, pos), types


def make_batch(structs, num_types):
    return pack(structs, num_types)
