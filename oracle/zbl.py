"""FP64 oracle of the ZBL short-range repulsion added to NEP predictions.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle``): the GPU library never
imports it and shares no code with it.

The paper lists a ZBL correction among the potential's supported terms without
giving its form. The form used here is the universal screened-Coulomb pair
potential of Ziegler, Biersack and Littmark ("The Stopping and Range of Ions
in Solids", 1985):

    phi(r) = k_e Z_a Z_b / r * Phi(r / a_ab),   a_ab = 0.8854 a_0 / (Z_a^0.23 + Z_b^0.23),
    Phi(x) = 0.18175 e^{-3.19980 x} + 0.50986 e^{-0.94229 x}
           + 0.28022 e^{-0.40290 x} + 0.02817 e^{-0.20162 x},

with k_e = e^2 / (4 pi eps_0) = 14.399645 eV A and the Bohr radius a_0 =
0.529177210903 A (CODATA). Readings (the paper does not fix these):
  * the pair energy is switched off smoothly by f(r) = 1 below r_inner,
    (1 + cos(pi (r - r_inner) / (r_outer - r_inner))) / 2 up to r_outer and
    0 beyond, i.e. phi_c(r) = phi(r) f(r);
  * each ordered pair gives half its energy to the centre atom, so a pair
    potential summed over the neighbour lists counts every bond once:
    E_i = 1/2 sum_j phi_c(r_ij);
  * the term has no trainable parameter: forces F_i = -dE/dr_i and virials
    W_s = -sum_{i in s, j} r_ij (x) dE_i/dr_ij follow the same conventions as
    the NEP predictions, and it is added to them;
  * a pair at distance exactly 0 contributes nothing (phi is unbounded there).

Pins (``tests/test_oracle_pins.py``): Phi(0) = 1 and the Coulomb limit of
r phi(r) at r -> 0; forces against central finite differences of the energy;
virials against the energy's derivative under a homogeneous strain; the
switching function's end values; zero net force; and the dimer energy counted
once.
"""

from __future__ import annotations

import numpy as np

from . import neighbors

K_E = 14.399645  # e^2 / (4 pi eps_0), eV A
A_0 = 0.529177210903  # Bohr radius, A
_C = np.array([0.18175, 0.50986, 0.28022, 0.02817])
_D = np.array([3.19980, 0.94229, 0.40290, 0.20162])


def screening(x):
    """Universal screening function Phi(x) and its derivative."""
    x = np.asarray(x, dtype=np.float64)[..., None]
    e = _C * np.exp(-_D * x)
    return e.sum(-1), -(e * _D).sum(-1)


def switch(r, r_inner, r_outer):
    """Smooth cutoff f(r) and f'(r)."""
    r = np.asarray(r, dtype=np.float64)
    t = np.clip((r - r_inner) / (r_outer - r_inner), 0.0, 1.0)
    f = 0.5 * (1.0 + np.cos(np.pi * t))
    fp = np.where((r > r_inner) & (r < r_outer), -0.5 * np.pi / (r_outer - r_inner) * np.sin(np.pi * t), 0.0)
    return f, fp


def pair(za, zb, r, r_inner, r_outer):
    """phi_c(r) and d phi_c / dr for nuclear charges za, zb (arrays broadcast)."""
    za, zb, r = (np.asarray(v, dtype=np.float64) for v in (za, zb, r))
    inv_a = (za ** 0.23 + zb ** 0.23) / (0.8854 * A_0)
    pre = K_E * za * zb
    x = r * inv_a
    s, sp = screening(x)
    phi = pre * s / r
    dphi = pre * (sp * inv_a / r - s / (r * r))
    f, fp = switch(r, r_inner, r_outer)
    return phi * f, dphi * f + phi * fp


def zbl(atomic_numbers, r_inner, r_outer, batch):
    """E [Ns], F [Na, 3], W [Ns, 9] of the ZBL term over a packed batch."""
    Z = np.asarray(atomic_numbers, dtype=np.float64)
    Ns, Na = batch.num_structures, batch.num_atoms
    E = np.zeros(Ns)
    F = np.zeros((Na, 3))
    W = np.zeros((Ns, 9))
    for s in range(Ns):
        cell, pos, typ = batch.structure(s)
        a = int(batch.atom_offset[s])
        i, j, _, rv = neighbors(cell, pos, r_outer)
        r = np.linalg.norm(rv, axis=1)
        keep = r > 0.0
        i, j, rv, r = i[keep], j[keep], rv[keep], r[keep]
        typ = np.asarray(typ)
        phi, dphi = pair(Z[typ[i]], Z[typ[j]], r, r_inner, r_outer)
        E[s] = 0.5 * phi.sum()
        # dE_i/dr_ij = phi'(r) r_ij / (2 r); F_k = sum_j h_kj - sum_i h_ik = sum_j phi'(r_kj) r_kj / r
        g = (dphi / r)[:, None] * rv
        np.add.at(F, a + i, g)
        W[s] = -0.5 * np.einsum("p,pa,pb->ab", dphi / r, rv, rv).ravel()
    return E, F, W
