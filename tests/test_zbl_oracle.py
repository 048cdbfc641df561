"""Pins of the ZBL oracle against the mathematics and the constants' definitions.

The paper names a ZBL term without giving its form; the oracle takes the
universal Ziegler-Biersack-Littmark pair potential with a cosine switch
(readings listed in ``oracle/zbl.py``). These tests check it against things
other than itself: SI constants, limits, the switch's end values, finite
differences of the energy, the strain derivative, and the dimer.
"""

import numpy as np
import pytest

import oracle as O
from oracle import zbl as Z
from synth import structures as S

Z_OF_TYPE = [26.0, 24.0, 28.0]  # Fe, Cr, Ni
R_IN, R_OUT = 2.4, 3.0


def _bcc(seed, T=3, strain=0.0, sigma=0.15):
    rng = np.random.default_rng(seed)
    return S.bcc_structure(rng, 16, a=3.2, sigma=sigma, strain=strain, num_types=T, exact_dims=(2, 2, 2))


def _energy(cell, pos, typ):
    b = S.pack([(cell, pos, typ)], 3)
    return Z.zbl(Z_OF_TYPE, R_IN, R_OUT, b)[0][0]


def test_constants_from_si():
    e, eps0 = 1.602176634e-19, 8.8541878128e-12  # C, F/m (SI, CODATA 2018)
    assert abs(Z.K_E - e / (4 * np.pi * eps0 * 1e-10)) < 1e-5  # eV A
    assert abs(Z.A_0 - 0.529177210903) < 1e-12


def test_screening_unit_at_origin_and_decay():
    s, sp = Z.screening(0.0)
    assert abs(s - 1.0) < 1e-12  # the four weights sum to one: bare Coulomb at r -> 0
    assert sp < 0
    x = np.linspace(0.0, 30.0, 301)
    v, _ = Z.screening(x)
    assert np.all(np.diff(v) < 0) and v[-1] < 1e-2


def test_coulomb_limit():
    for za, zb in [(1, 1), (26, 28), (74, 74)]:
        r = 1e-7
        phi, _ = Z.pair(za, zb, r, R_IN, R_OUT)
        assert abs(phi * r / (Z.K_E * za * zb) - 1.0) < 1e-5


def test_switch_end_values_and_continuity():
    f, fp = Z.switch([0.0, R_IN, 0.5 * (R_IN + R_OUT), R_OUT, R_OUT + 1.0], R_IN, R_OUT)
    assert np.allclose(f, [1.0, 1.0, 0.5, 0.0, 0.0], atol=1e-15)
    assert abs(fp[0]) == 0 and abs(fp[1]) < 1e-12 and abs(fp[3]) < 1e-12 and fp[2] < 0
    # the pair energy goes to zero smoothly at r_outer
    lo, _ = Z.pair(26, 28, R_OUT - 1e-6, R_IN, R_OUT)
    hi, _ = Z.pair(26, 28, R_OUT + 1e-6, R_IN, R_OUT)
    assert abs(lo) < 1e-9 and hi == 0.0


def test_pair_derivative_fd():
    r = np.array([0.3, 1.0, 2.0, 2.5, 2.7, 2.95])
    _, dphi = Z.pair(26, 24, r, R_IN, R_OUT)
    h = 1e-6
    fd = (Z.pair(26, 24, r + h, R_IN, R_OUT)[0] - Z.pair(26, 24, r - h, R_IN, R_OUT)[0]) / (2 * h)
    assert np.allclose(dphi, fd, rtol=1e-7, atol=1e-9)


def test_dimer_counts_bond_once():
    L = 30.0
    d = np.array([0.7, 1.3, -1.1])
    pos = np.array([[L / 2] * 3, L / 2 + d])
    b = S.pack([(np.eye(3) * L, pos, np.array([0, 2], np.int32))], 3)
    E, F, W = Z.zbl(Z_OF_TYPE, R_IN, R_OUT, b)
    r = np.linalg.norm(d)
    phi, dphi = Z.pair(26, 28, r, R_IN, R_OUT)
    assert abs(E[0] - phi) < 1e-12 * abs(phi)
    # repulsion pushes atom 0 away from atom 1: F_0 = phi'(r) d / r with phi' < 0
    assert np.allclose(F[0], dphi * d / r) and np.allclose(F[1], -F[0])
    assert np.allclose(W[0].reshape(3, 3), -dphi * np.outer(d, d) / r)


def test_forces_finite_difference():
    cell, pos, typ = _bcc(3)
    b = S.pack([(cell, pos, typ)], 3)
    E, F, W = Z.zbl(Z_OF_TYPE, R_IN, R_OUT, b)
    assert np.abs(F).max() > 0.1  # pairs inside and across the switch
    h = 1e-6
    for i in (0, 7, 13):
        for c in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, c] += h
            pm[i, c] -= h
            fd = -(_energy(cell, pp, typ) - _energy(cell, pm, typ)) / (2 * h)
            assert np.isclose(F[i, c], fd, rtol=1e-6, atol=1e-7 * np.abs(F).max())
    assert np.abs(F.sum(0)).max() < 1e-11 * np.abs(F).max() * len(F)


def test_virial_strain_derivative():
    cell, pos, typ = _bcc(4, strain=0.02)
    b = S.pack([(cell, pos, typ)], 3)
    _, _, W = Z.zbl(Z_OF_TYPE, R_IN, R_OUT, b)
    Wm = W[0].reshape(3, 3)
    assert np.abs(Wm - Wm.T).max() < 1e-12 * np.abs(Wm).max()
    h = 1e-6
    for al in range(3):
        for be in range(3):
            eps = np.zeros((3, 3))
            eps[al, be] = h
            Fp, Fm = np.eye(3) + eps, np.eye(3) - eps
            ep = _energy(cell @ Fp.T, pos @ Fp.T, typ)
            em = _energy(cell @ Fm.T, pos @ Fm.T, typ)
            assert np.isclose(-(ep - em) / (2 * h), Wm[be, al], rtol=1e-6, atol=1e-7 * np.abs(Wm).max())


def test_translation_and_image_invariance():
    cell, pos, typ = _bcc(5)
    e0 = _energy(cell, pos, typ)
    assert np.isclose(_energy(cell, pos + np.array([0.3, -1.7, 2.2]), typ), e0, rtol=1e-12)
    shifted = pos.copy()
    shifted[3] += cell[1] - 2 * cell[2]  # another periodic image of atom 3
    assert np.isclose(_energy(cell, shifted, typ), e0, rtol=1e-12)


@pytest.mark.parametrize("k", [0, 1])
def test_target_shift_equals_added_term(k):
    """Training against targets minus the ZBL term gives the loss of the NEP
    prediction plus the ZBL term against the original targets (the term has no
    trainable parameter), so the loss is unchanged by where the term is added."""
    m = O.Model(num_types=3, rc_r=4.5, rc_a=3.8, n_max_r=3, n_max_a=3, basis_r=5, basis_a=4, l_max=4, hidden=7)
    rng = np.random.default_rng(9 + k)
    b = S.pack([_bcc(20 + k), _bcc(30 + k, strain=0.02)], 3)
    P, _ = O.dims(m)
    th = rng.normal(0.0, 0.1, P)
    s = O.scaler(O.descriptors(m, th, b))
    Et = rng.normal(size=2)
    Ft = rng.normal(size=(b.num_atoms, 3))
    Wt = rng.normal(size=(2, 9))
    Ez, Fz, Wz = Z.zbl(Z_OF_TYPE, R_IN, R_OUT, b)
    loss, _, E, F, W = O.loss_and_grad(m, th, s, b, Et - Ez, Ft - Fz, Wt - Wz, want_grad=False)
    # the loss written out (Eqs. 4-7) for predictions E + Ez against the raw targets
    n = np.diff(b.atom_offset)
    dE = np.mean(((E + Ez - Et) / n) ** 2)
    dF = np.mean((F + Fz - Ft) ** 2)
    dV = np.mean(((W + Wz - Wt) / n[:, None]) ** 2)
    assert np.allclose(loss[1:], [dE, dF, dV], rtol=1e-12)
