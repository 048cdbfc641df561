"""The five seeded synthetic workloads and their model hyper-parameters.

Each workload stands in for a training set of the kind the paper fits (its
datasets are not available): crystalline and liquid-like periodic cells of
uneven size, one to five species. Seeds: master seed per workload; structure
s uses child s of ``SeedSequence(master)``; structure sizes use the last child;
initial parameters use master+1000, teacher parameters master+2000,
finite-difference indices master+3000, minibatch shuffles master+4000+epoch.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .structures import (
    bcc_structure,
    dense_liquid,
    fcc_structure,
    pack,
    random_packing,
)


@dataclass(frozen=True)
class Workload:
    name: str
    seed: int
    num_structures: int
    dtype: str  # "f64" or "f32": bulk precision of the GPU path
    model: dict = field(default_factory=dict)
    lambdas: tuple = (1.0, 1.0, 0.1)
    about: str = ""
    minibatch: int = 0  # > 0: a training epoch in minibatches of this size

    @property
    def description(self) -> str:
        m = self.model
        extra = (" + 4-body" if m["l_max_4b"] == 2 else "") + (" + 5-body" if m["l_max_5b"] == 1 else "")
        return (f"{self.about}; {m['num_types']} species, rc {m['rc_r']:g}/{m['rc_a']:g} A, "
                f"n_max {m['n_max_r']}/{m['n_max_a']}, basis {m['basis_r']}/{m['basis_a']}, "
                f"l_max {m['l_max']}{extra}, {m['hidden']} hidden, {self.dtype}")


def _model(T, rc_r, rc_a, n_r, n_a, b_r, b_a, l_max, l4, l5, hidden):
    return dict(num_types=T, rc_r=rc_r, rc_a=rc_a, n_max_r=n_r, n_max_a=n_a,
                basis_r=b_r, basis_a=b_a, l_max=l_max, l_max_4b=l4, l_max_5b=l5,
                hidden=hidden)


WORKLOADS = {
    # 8 single-element 64-atom bcc cells (4x4x2 conventional cells), FP64.
    "bcc64x8": Workload("bcc64x8", 1, 8, "f64",
                        _model(1, 5.0, 4.0, 4, 4, 8, 8, 4, 0, 0, 30),
                        about="8 bcc cells of 64 atoms"),
    # 256 single-element fcc cells with 32..256 atoms, strain and noise, FP32.
    "fcc_uneven_256": Workload("fcc_uneven_256", 2, 256, "f32",
                               _model(1, 6.0, 4.0, 6, 4, 8, 8, 4, 0, 0, 30),
                               about="256 fcc cells of 32-256 atoms"),
    # 1024 four-species fcc/bcc alloys with 16..512 atoms, 4-body and 5-body terms.
    "alloy4_1024": Workload("alloy4_1024", 3, 1024, "f32",
                            _model(4, 6.0, 4.0, 8, 6, 12, 10, 4, 2, 1, 50),
                            about="1024 fcc/bcc alloy cells of 16-512 atoms"),
    # 4096 three-species cells, half crystalline and half liquid-like packings.
    "mixed3_4096": Workload("mixed3_4096", 4, 4096, "f32",
                            _model(3, 6.0, 4.0, 8, 8, 12, 12, 4, 0, 0, 80),
                            about="4096 crystalline and liquid-like cells of 32-256 atoms, minibatch 64",
                            minibatch=64),
    # 32 five-species cells with 4000..16000 atoms (alloy and dense liquid).
    "large5_32": Workload("large5_32", 5, 32, "f32",
                          _model(5, 6.0, 5.0, 10, 8, 12, 12, 4, 0, 0, 100),
                          about="32 alloy and dense-liquid cells of 4000-16000 atoms"),
}


def _children(seed: int, n: int):
    return np.random.SeedSequence(seed).spawn(n + 1)


def _gen_structure(name: str, rng: np.random.Generator, n: int, T: int):
    if name == "bcc64x8":
        return bcc_structure(rng, 64, a=3.2, sigma=0.1, exact_dims=(4, 4, 2))
    if name == "fcc_uneven_256":
        return fcc_structure(rng, n, a=4.0, sigma=0.15, strain=0.02)
    if name == "alloy4_1024":
        if rng.uniform() < 0.5:
            return fcc_structure(rng, n, a=4.0, sigma=0.2, num_types=T)
        return bcc_structure(rng, n, a=3.2, sigma=0.2, num_types=T)
    if name == "mixed3_4096":
        if rng.uniform() < 0.5:
            if rng.uniform() < 0.5:
                return fcc_structure(rng, n, a=4.0, sigma=0.15, num_types=T)
            return bcc_structure(rng, n, a=3.2, sigma=0.15, num_types=T)
        return random_packing(rng, n, density=0.0625, d_min=1.8, num_types=T)
    if name == "large5_32":
        if rng.uniform() < 0.5:
            return fcc_structure(rng, n, a=(4.0 / 0.11) ** (1.0 / 3.0), sigma=0.1, num_types=T)
        return dense_liquid(rng, n, density=0.11, sigma=0.3, d_min=1.8, num_types=T)
    raise KeyError(name)


_SIZE_RANGE = {
    "bcc64x8": (64, 64),
    "fcc_uneven_256": (32, 256),
    "alloy4_1024": (16, 512),
    "mixed3_4096": (32, 256),
    "large5_32": (4000, 16000),
}


def structure_sizes(name: str, count: int | None = None) -> np.ndarray:
    w = WORKLOADS[name]
    kids = _children(w.seed, w.num_structures)
    rng = np.random.Generator(np.random.PCG64(kids[-1]))
    lo, hi = _SIZE_RANGE[name]
    sizes = rng.integers(lo, hi + 1, size=w.num_structures)
    return sizes if count is None else sizes[:count]


def workload_batch(name: str, indices=None):
    """Generate (a subset of) a workload's structures, packed as one batch."""
    w = WORKLOADS[name]
    kids = _children(w.seed, w.num_structures)
    sizes = structure_sizes(name)
    idx = range(w.num_structures) if indices is None else indices
    T = w.model["num_types"]
    structs = []
    for s in idx:
        rng = np.random.Generator(np.random.PCG64(kids[int(s)]))
        structs.append(_gen_structure(name, rng, int(sizes[int(s)]), T))
    return pack(structs, T)


def draw_theta(num_params: int, seed: int, std: float = 0.1) -> np.ndarray:
    """Seeded N(0, std^2) draw of every parameter (float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(0.0, std, size=int(num_params))


def random_targets(batch, seed: int, e_std: float = 0.1, f_std: float = 0.5, w_std: float = 0.05):
    """Seeded random reference data for a packed batch: energies E_s = N_s * N(0, e_std^2),
    forces N(0, f_std^2) per component, symmetric virials N_s * N(0, w_std^2) per entry
    (N_s = atoms of the structure). Values only; no potential is evaluated."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = np.diff(np.asarray(batch.atom_offset)).astype(np.float64)
    E = n * rng.normal(0.0, e_std, size=len(n))
    F = rng.normal(0.0, f_std, size=(int(batch.num_atoms), 3))
    w = rng.normal(0.0, w_std, size=(len(n), 3, 3))
    W = (n[:, None, None] * 0.5 * (w + w.transpose(0, 2, 1))).reshape(len(n), 9)
    return E, F, W
