"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (Table II parameter counts, Adam defaults), closed forms, library
routines (scipy spherical harmonics and Legendre polynomials, torch's Adam),
invariances stated in the Methods, finite differences, and brute force.
"""

import json
import os

import numpy as np
import pytest
import scipy.special as sp

import oracle as O
from synth import structures as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def model_1s(**kw):
    base = dict(num_types=1, rc_r=5.0, rc_a=4.0, n_max_r=4, n_max_a=4, basis_r=8, basis_a=8, l_max=4, hidden=12)
    base.update(kw)
    return O.Model(**base)


def model_alloy(**kw):
    base = dict(num_types=3, rc_r=4.5, rc_a=3.8, n_max_r=3, n_max_a=3, basis_r=5, basis_a=4, l_max=4,
                l_max_4b=2, l_max_5b=1, hidden=7)
    base.update(kw)
    return O.Model(**base)


def small_bcc(seed=0, dims=(2, 2, 2), sigma=0.12, T=1, strain=0.0):
    rng = np.random.default_rng(seed)
    return S.bcc_structure(rng, 2 * dims[0] * dims[1] * dims[2], a=3.2, sigma=sigma, strain=strain,
                           num_types=T, exact_dims=dims)


def theta_and_scale(m, batch, seed=0, std=0.1):
    P, _ = O.dims(m)
    theta = np.random.default_rng(seed).normal(0.0, std, P)
    q = O.descriptors(m, theta, batch)
    return theta, O.scaler(q)


# ----------------------------------------------------------------- layout


def test_table2_parameter_counts():
    """Table II: 16 species, basis 8/8, l_max 4 2 1, 80 neurons -> 70,401 / 97,537 / 124,673."""
    g = json.load(open(os.path.join(GOLDEN, "table2_param_counts.json")))
    for case in g["cases"]:
        m = O.Model(num_types=g["num_types"], rc_r=5.0, rc_a=4.0, n_max_r=case["n_max"][0],
                    n_max_a=case["n_max"][1], basis_r=g["basis"][0], basis_a=g["basis"][1],
                    l_max=g["l_max"][0], l_max_4b=g["l_max"][1], l_max_5b=g["l_max"][2], hidden=g["hidden"])
        P, D = O.dims(m)
        assert P == case["params"], case["label"]


def test_invalid_models_rejected():
    with pytest.raises(ValueError):
        O.dims(model_1s(rc_a=6.0))  # angular cutoff beyond radial
    with pytest.raises(ValueError):
        O.dims(model_1s(l_max_4b=3))
    with pytest.raises(ValueError):
        O.dims(model_1s(l_max_4b=2, l_max=1))


# ------------------------------------------------------------------ basis


def test_basis_closed_forms():
    """Eqs. (17)-(18): f_k(0) = 1; f_k and f_k' vanish at r_c; T_k(cos phi) = cos(k phi)."""
    rc, K = 4.3, 12
    f0, _ = O.basis(0.0, rc, K)
    assert np.allclose(f0, 1.0, atol=1e-15)
    f1, fp1 = O.basis(rc * (1 - 1e-12), rc, K)
    assert np.abs(f1).max() < 1e-15 and np.abs(fp1).max() < 1e-9
    fo, fpo = O.basis(rc * 1.01, rc, K)
    assert not fo.any() and not fpo.any()
    for phi in (0.3, 1.1, 2.5):
        x = np.cos(phi)
        r = rc * (1.0 - np.sqrt((1.0 + x) / 2.0))
        fc = 0.5 * (np.cos(np.pi * r / rc) + 1.0)
        f, _ = O.basis(r, rc, K)
        want = 0.5 * (np.cos(np.arange(K) * phi) + 1.0) * fc
        assert np.allclose(f, want, rtol=0, atol=1e-14)


def test_basis_derivative_fd():
    rc, K, h = 5.0, 10, 1e-6
    for r in (0.7, 2.2, 4.1, 4.95):
        _, fp = O.basis(r, rc, K)
        fpl, _ = O.basis(r + h, rc, K)
        fmi, _ = O.basis(r - h, rc, K)
        assert np.allclose(fp, (fpl - fmi) / (2 * h), atol=1e-8)


# -------------------------------------------------------- spherical harmonics


def _scipy_real_sh(L, u):
    th, ph = np.arccos(u[2]), np.arctan2(u[1], u[0])
    out = []
    for l in range(1, L + 1):
        for m in range(-l, l + 1):
            c = sp.sph_harm_y(l, abs(m), th, ph)
            if m > 0:
                out.append(np.sqrt(2) * (-1) ** m * c.real)
            elif m < 0:
                out.append(np.sqrt(2) * (-1) ** m * c.imag)
            else:
                out.append(c.real)
    return np.array(out)


def test_real_sh_matches_scipy_and_addition_theorem():
    rng = np.random.default_rng(1)
    L = 6
    for _ in range(10):
        r1, r2 = rng.normal(size=3) * 2, rng.normal(size=3) * 2
        Y1, _ = O.real_sh(L, r1)
        Y2, _ = O.real_sh(L, r2)
        u1, u2 = r1 / np.linalg.norm(r1), r2 / np.linalg.norm(r2)
        assert np.allclose(Y1, _scipy_real_sh(L, u1), atol=1e-13)
        for l in range(1, L + 1):
            sl = slice(l * l - 1, (l + 1) ** 2 - 1)
            # Unsold: sum_m Y_lm^2 = (2l+1)/4pi ; addition theorem with Legendre P_l
            assert np.isclose((Y1[sl] ** 2).sum(), (2 * l + 1) / (4 * np.pi), atol=1e-13)
            assert np.isclose((Y1[sl] * Y2[sl]).sum(), (2 * l + 1) / (4 * np.pi) * sp.eval_legendre(l, u1 @ u2),
                              atol=1e-13)


def test_real_sh_gradient_fd():
    rng = np.random.default_rng(2)
    h = 1e-6
    for _ in range(5):
        r = rng.normal(size=3) * 1.5
        _, dY = O.real_sh(4, r)
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            fd = (O.real_sh(4, r + e)[0] - O.real_sh(4, r - e)[0]) / (2 * h)
            assert np.allclose(dY[:, c], fd, atol=1e-8)


def test_complex_sh2_matches_scipy():
    rng = np.random.default_rng(3)
    for _ in range(5):
        r = rng.normal(size=3)
        u = r / np.linalg.norm(r)
        th, ph = np.arccos(u[2]), np.arctan2(u[1], u[0])
        want = np.array([sp.sph_harm_y(2, m, th, ph) for m in range(-2, 3)])
        assert np.allclose(O.complex_sh2(r), want, atol=1e-14)


# ---------------------------------------------------------------- Wigner 3j


def _three_j_zero(j1, j2, j3):
    """Closed form of (j1 j2 j3; 0 0 0) for even J = j1 + j2 + j3."""
    J = j1 + j2 + j3
    if J % 2:
        return 0.0
    g = J // 2
    f = sp.factorial
    return (-1) ** g * np.sqrt(f(J - 2 * j1) * f(J - 2 * j2) * f(J - 2 * j3) / f(J + 1)) * f(g) / (
        f(g - j1) * f(g - j2) * f(g - j3))


def test_wigner3j_closed_form_and_orthogonality():
    for js in [(2, 2, 2), (1, 1, 2), (2, 2, 4), (3, 2, 1), (4, 4, 4)]:
        assert np.isclose(O.wigner3j(*js, 0, 0, 0), _three_j_zero(*js), atol=1e-14)
    assert np.isclose(O.wigner3j(2, 2, 2, 0, 0, 0), -np.sqrt(2.0 / 35.0), atol=1e-15)
    j1 = j2 = 2
    for j3 in range(0, 5):
        for j3p in range(0, 5):
            for m3 in range(-min(j3, j3p), min(j3, j3p) + 1):
                s = sum(O.wigner3j(j1, j2, j3, m1, m3 * 0 - m1 - m3, m3) *
                        O.wigner3j(j1, j2, j3p, m1, -m1 - m3, m3)
                        for m1 in range(-j1, j1 + 1) if abs(-m1 - m3) <= j2)
                want = (1.0 / (2 * j3 + 1)) if j3 == j3p else 0.0
                assert np.isclose(s, want, atol=1e-13)


KAPPA = -4.5 * np.sqrt(2.0 / 35.0) * (5.0 / (4.0 * np.pi)) ** 1.5


def test_q4_equals_cartesian_cubic_invariant():
    """The (2 2 2) contraction of complex l=2 moments is real and equals kappa tr(S^3),
    S = sum_j g_j (u_j u_j^T - I/3): the cubic invariants of l=2 form a 1-D space."""
    rng = np.random.default_rng(4)
    for _ in range(8):
        n = rng.integers(1, 9)
        g = rng.normal(size=n)
        rs = rng.normal(size=(n, 3))
        mom = sum(gj * O.complex_sh2(rj) for gj, rj in zip(g, rs))
        q4 = O.q4_of_moments(mom)
        Smat = sum(gj * (np.outer(rj, rj) / (rj @ rj) - np.eye(3) / 3) for gj, rj in zip(g, rs))
        assert abs(q4.imag) < 1e-13
        assert np.isclose(q4.real, KAPPA * np.trace(Smat @ Smat @ Smat), rtol=1e-12, atol=1e-14)


# ------------------------------------------------------ descriptor closed forms


def _big_box(points, types=None, L=40.0):
    cell = np.eye(3) * L
    pos = np.asarray(points, dtype=float) + L / 2
    t = np.zeros(len(pos), np.int32) if types is None else np.asarray(types, np.int32)
    return S.pack([(cell, pos, t)], int(t.max()) + 1)


def _g(theta, m, r, n, kind, a=0, b=0):
    """g_n(r) from the coefficients (Eq. 16) and the pinned basis."""
    P, D = O.dims(m)
    T = m.num_types
    if kind == "R":
        K, N, rc, off = m.basis_r + 1, m.n_max_r + 1, m.rc_r, 0
    else:
        K, N, rc = m.basis_a + 1, m.n_max_a + 1, m.rc_a
        off = T * T * (m.n_max_r + 1) * (m.basis_r + 1)
    f, _ = O.basis(r, rc, K)
    c = theta[off + ((a * T + b) * N + n) * K: off + ((a * T + b) * N + n) * K + K]
    return float(c @ f)


def test_dimer_descriptor_closed_form():
    """One neighbour: q_n = g_n(r); q_nl = g_n^A(r)^2 (2l+1)/4pi; q5 = q_n1^2;
    q4 along z = (2 2 2; 0 0 0) (5/4pi)^(3/2) g^3."""
    m = model_alloy(num_types=1)
    P, D = O.dims(m)
    theta = np.random.default_rng(5).normal(0, 0.3, P)
    r = 2.7
    b = _big_box([[0, 0, 0], [0, 0, r]])
    q = O.descriptors(m, theta, b)[0]
    NR, NA, L = m.n_max_r + 1, m.n_max_a + 1, m.l_max
    for n in range(NR):
        assert np.isclose(q[n], _g(theta, m, r, n, "R"), atol=1e-14)
    for n in range(NA):
        g = _g(theta, m, r, n, "A")
        for l in range(1, L + 1):
            assert np.isclose(q[NR + (l - 1) * NA + n], g * g * (2 * l + 1) / (4 * np.pi), atol=1e-14)
        q4 = q[NR + L * NA + n]
        assert np.isclose(q4, -np.sqrt(2 / 35) * (5 / (4 * np.pi)) ** 1.5 * g ** 3, atol=1e-14)
        assert np.isclose(q[NR + (L + 1) * NA + n], (3 / (4 * np.pi) * g * g) ** 2, atol=1e-14)


def test_trimer_descriptor_legendre():
    """Two neighbours at angle theta: q_nl = (2l+1)/4pi [g1^2 + g2^2 + 2 g1 g2 P_l(cos theta)]."""
    m = model_1s(l_max=5)
    P, D = O.dims(m)
    theta = np.random.default_rng(6).normal(0, 0.3, P)
    r1, r2, ang = 2.3, 3.1, 1.1
    pts = [[0, 0, 0], [r1, 0, 0], [r2 * np.cos(ang), r2 * np.sin(ang), 0]]
    # atoms 1 and 2 are 2.92 A apart; descriptor of atom 0 only sees both.
    q = O.descriptors(m, theta, _big_box(pts))[0]
    NR, NA = m.n_max_r + 1, m.n_max_a + 1
    for n in range(NA):
        g1, g2 = _g(theta, m, r1, n, "A"), _g(theta, m, r2, n, "A")
        for l in range(1, m.l_max + 1):
            want = (2 * l + 1) / (4 * np.pi) * (g1 ** 2 + g2 ** 2 + 2 * g1 * g2 * sp.eval_legendre(l, np.cos(ang)))
            assert np.isclose(q[NR + (l - 1) * NA + n], want, atol=1e-13)


def test_zero_input_weights():
    """W0 = 0: E_i = sum_mu w1 tanh(-b0) - b1 and forces, virial vanish."""
    m = model_alloy()
    batch = S.pack([small_bcc(7, T=3)], 3)
    P, D = O.dims(m)
    T, H = m.num_types, m.hidden
    theta = np.random.default_rng(8).normal(0, 0.2, P)
    offN = P - 1 - T * (D + 2) * H
    for t in range(T):
        base = offN + t * (D + 2) * H
        theta[base:base + H * D] = 0.0
    E, F, W, Ei = O.forward(m, theta, np.ones(D), batch, per_atom=True)
    for i, t in enumerate(batch.types):
        base = offN + t * (D + 2) * H
        b0, w1 = theta[base + H * D: base + H * D + H], theta[base + H * D + H: base + H * D + 2 * H]
        assert np.isclose(Ei[i], np.sum(w1 * np.tanh(-b0)) - theta[-1], atol=1e-14)
    assert np.abs(F).max() < 1e-14 and np.abs(W).max() < 1e-14


# ------------------------------------------------------------- neighbours


@pytest.mark.parametrize("lat,a,rc,want", [("bcc", 3.2, 5.0, 26), ("bcc", 3.2, 4.0, 14),
                                           ("fcc", 4.0, 6.0, 54), ("fcc", 4.0, 3.0, 12)])
def test_lattice_shell_counts(lat, a, rc, want):
    """Perfect lattices, including cells thinner than 2 r_c: every atom sees its shells."""
    rng = np.random.default_rng(0)
    maker = S.bcc_structure if lat == "bcc" else S.fcc_structure
    for dims in [(1, 1, 1), (2, 1, 1), (3, 2, 2)]:
        nsites = (2 if lat == "bcc" else 4) * dims[0] * dims[1] * dims[2]
        cell, pos, _ = maker(rng, nsites, a=a, sigma=0.0, exact_dims=dims)
        i, j, s, r = O.neighbors(cell, pos, rc)
        assert np.all(np.bincount(i, minlength=len(pos)) == want)


def test_neighbors_match_independent_search():
    """Noisy strained cell thinner than 2 r_c vs an independent image search."""
    rng = np.random.default_rng(9)
    cell, pos, _ = S.fcc_structure(rng, 30, a=4.0, sigma=0.2, strain=0.02)
    rc = 6.0
    i, j, s, r = O.neighbors(cell, pos, rc)
    got = sorted(zip(i.tolist(), j.tolist(), map(tuple, s.tolist())))
    rng_img = range(-3, 4)
    want = []
    for a in range(len(pos)):
        for b in range(len(pos)):
            for n0 in rng_img:
                for n1 in rng_img:
                    for n2 in rng_img:
                        if a == b and n0 == n1 == n2 == 0:
                            continue
                        d = pos[b] + n0 * cell[0] + n1 * cell[1] + n2 * cell[2] - pos[a]
                        if d @ d < rc * rc:
                            want.append((a, b, (n0, n1, n2)))
    assert got == sorted(want)
    assert np.allclose(r, np.array([pos[b] + np.array(n) @ cell - pos[a] for a, b, n in got]), atol=1e-12)


# ------------------------------------------------- forces, virial, invariances


@pytest.mark.parametrize("mk,T", [(model_1s, 1), (model_alloy, 3)])
def test_forces_finite_difference(mk, T):
    m = mk()
    cell, pos, typ = small_bcc(10, T=T)
    batch = S.pack([(cell, pos, typ)], T)
    theta, s = theta_and_scale(m, batch)
    E, F, W = O.forward(m, theta, s, batch)
    h = 1e-5
    for i in (0, 5, 11):
        for c in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, c] += h
            pm[i, c] -= h
            fd = -(O.energy(m, theta, s, cell, pp, typ) - O.energy(m, theta, s, cell, pm, typ)) / (2 * h)
            assert np.isclose(F[i, c], fd, rtol=1e-7, atol=1e-8 * np.abs(F).max())
    assert np.abs(F.sum(0)).max() < 1e-12 * np.abs(F).max() * len(F)


@pytest.mark.parametrize("mk,T", [(model_1s, 1), (model_alloy, 3)])
def test_virial_strain_derivative(mk, T):
    """W = -dE/d(strain) under r -> (I+e) r, H -> H (I+e)^T; symmetric."""
    m = mk()
    cell, pos, typ = small_bcc(11, T=T, strain=0.02)
    batch = S.pack([(cell, pos, typ)], T)
    theta, s = theta_and_scale(m, batch)
    E, F, W = O.forward(m, theta, s, batch)
    Wm = W[0].reshape(3, 3)
    assert np.abs(Wm - Wm.T).max() < 1e-12 * np.abs(Wm).max()
    h = 1e-6
    for al in range(3):
        for be in range(3):
            eps = np.zeros((3, 3))
            eps[al, be] = h
            Fp, Fm = np.eye(3) + eps, np.eye(3) - eps
            ep = O.energy(m, theta, s, cell @ Fp.T, pos @ Fp.T, typ)
            em = O.energy(m, theta, s, cell @ Fm.T, pos @ Fm.T, typ)
            assert np.isclose(-(ep - em) / (2 * h), Wm[be, al], rtol=1e-6, atol=1e-7 * np.abs(Wm).max())


def test_rotation_translation_permutation_invariance():
    m = model_alloy()
    cell, pos, typ = small_bcc(12, T=3, strain=0.02)
    batch = S.pack([(cell, pos, typ)], 3)
    theta, s = theta_and_scale(m, batch)
    E, F, W = O.forward(m, theta, s, batch)
    # rotation of positions and cell
    Q, _ = np.linalg.qr(np.random.default_rng(13).normal(size=(3, 3)))
    Er, Fr, Wr = O.forward(m, theta, s, S.pack([(cell @ Q.T, pos @ Q.T, typ)], 3))
    assert np.isclose(Er[0], E[0], rtol=1e-12)
    assert np.allclose(Fr, F @ Q.T, atol=1e-11)
    assert np.allclose(Wr[0].reshape(3, 3), Q @ W[0].reshape(3, 3) @ Q.T, atol=1e-10)
    # translation (positions leave the cell: images must still be found)
    Et, Ft, _ = O.forward(m, theta, s, S.pack([(cell, pos + np.array([0.7, -1.3, 2.9]), typ)], 3))
    assert np.isclose(Et[0], E[0], rtol=1e-12) and np.allclose(Ft, F, atol=1e-11)
    # permutation
    perm = np.random.default_rng(14).permutation(len(pos))
    Ep, Fp, _ = O.forward(m, theta, s, S.pack([(cell, pos[perm], typ[perm])], 3))
    assert np.isclose(Ep[0], E[0], rtol=1e-12) and np.allclose(Fp, F[perm], atol=1e-11)


def test_supercell_extensivity():
    """E(n1 x n2 x n3 replica) = n1 n2 n3 E(cell) and forces replicate (tests image handling)."""
    m = model_alloy()
    cell, pos, typ = small_bcc(15, dims=(1, 2, 1), T=3)
    batch = S.pack([(cell, pos, typ)], 3)
    theta, s = theta_and_scale(m, batch)
    E, F, W = O.forward(m, theta, s, batch)
    reps = (2, 1, 3)
    shifts = [np.array([a, b, c]) @ cell for a in range(reps[0]) for b in range(reps[1]) for c in range(reps[2])]
    big = (np.diag(reps) @ cell, np.concatenate([pos + sh for sh in shifts]), np.tile(typ, len(shifts)))
    Eb, Fb, Wb = O.forward(m, theta, s, S.pack([big], 3))
    assert np.isclose(Eb[0], len(shifts) * E[0], rtol=1e-12)
    assert np.allclose(Fb, np.tile(F, (len(shifts), 1)), atol=1e-11)
    assert np.allclose(Wb[0], len(shifts) * W[0], rtol=1e-10, atol=1e-10)


def test_scaler_rescaling_invariance():
    """Eq. (2): multiplying one radial channel's coefficients by c scales q_n by c and the
    recomputed scaler by 1/c, leaving every energy unchanged."""
    m = model_1s()
    batch = S.pack([small_bcc(16), small_bcc(17)], 1)
    theta, s = theta_and_scale(m, batch)
    E, F, W = O.forward(m, theta, s, batch)
    th2 = theta.copy()
    K = m.basis_r + 1
    th2[2 * K:3 * K] *= 3.7  # radial channel n = 2
    s2 = O.scaler(O.descriptors(m, th2, batch))
    assert np.isclose(s2[2], s[2] / 3.7, rtol=1e-12)
    E2, F2, W2 = O.forward(m, th2, s2, batch)
    assert np.allclose(E2, E, rtol=1e-12) and np.allclose(F2, F, atol=1e-11)


# ------------------------------------------------------- loss and gradient


def _targets(batch, seed):
    rng = np.random.default_rng(seed)
    return (rng.normal(0, 1.0, batch.num_structures), rng.normal(0, 0.3, (batch.num_atoms, 3)),
            rng.normal(0, 1.0, (batch.num_structures, 9)))


@pytest.mark.parametrize("mk,T", [(model_1s, 1), (model_alloy, 3)])
@pytest.mark.parametrize("lam", [(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0), (1.0, 1.0, 0.1)])
def test_loss_gradient_finite_difference(mk, T, lam):
    """Central differences (h = 1e-6) on seeded random parameter indices; one-hot weights
    isolate the energy, force and virial adjoints."""
    m = mk()
    batch = S.pack([small_bcc(20, T=T, strain=0.02), small_bcc(21, dims=(2, 1, 2), T=T)], T)
    theta, s = theta_and_scale(m, batch, seed=1, std=0.3)
    Et, Ft, Wt = _targets(batch, 2)
    hv = np.array([1, 0], np.uint8)
    loss, g, *_ = O.loss_and_grad(m, theta, s, batch, Et, Ft, Wt, lam, has_virial=hv)
    P = len(theta)
    rng = np.random.default_rng(3003)
    T_, NR, KR = m.num_types, m.n_max_r + 1, m.basis_r + 1
    nCR = T_ * T_ * NR * KR
    nCA = T_ * T_ * (m.n_max_a + 1) * (m.basis_a + 1)
    idx = np.concatenate([rng.choice(nCR, 6, replace=False), nCR + rng.choice(nCA, 8, replace=False),
                          nCR + nCA + rng.choice(P - nCR - nCA, 10, replace=False), [P - 1]])
    h = 1e-6
    scale = np.abs(g).max()
    for p in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        lp = O.loss_and_grad(m, tp, s, batch, Et, Ft, Wt, lam, has_virial=hv, want_grad=False)[0][0]
        lm = O.loss_and_grad(m, tm, s, batch, Et, Ft, Wt, lam, has_virial=hv, want_grad=False)[0][0]
        fd = (lp - lm) / (2 * h)
        assert abs(g[p] - fd) <= 1e-7 * scale + 1e-6 * abs(fd), (p, g[p], fd)


def test_loss_value_definition():
    """Eqs. (4)-(7) with hand-computed residuals."""
    m = model_1s()
    batch = S.pack([small_bcc(30), small_bcc(31, dims=(2, 2, 1))], 1)
    theta, s = theta_and_scale(m, batch)
    Et, Ft, Wt = _targets(batch, 4)
    lam = (0.7, 1.3, 0.2)
    loss, _, E, F, W = O.loss_and_grad(m, theta, s, batch, Et, Ft, Wt, lam, want_grad=False)
    na = batch.counts()
    dE = np.mean(((E - Et) / na) ** 2)
    dF = np.sum((F - Ft) ** 2) / (3 * batch.num_atoms)
    dV = np.sum(((W - Wt) / na[:, None]) ** 2) / (9 * batch.num_structures)
    assert np.allclose(loss, [lam[0] * dE + lam[1] * dF + lam[2] * dV, dE, dF, dV], rtol=1e-13)


def test_empty_structures_take_no_part():
    """A structure without atoms has no per-atom residual in Eqs. (4)-(7) (N_a^s = 0):
    inserting empty structures, labelled or not, leaves the loss and its gradient
    unchanged, and the hand-computed loss of the non-empty ones holds."""
    m = model_alloy()
    rng = np.random.default_rng(3)
    full = [S.fcc_structure(rng, 9, a=4.0, sigma=0.2, num_types=3), S.bcc_structure(rng, 8, a=3.2, sigma=0.2,
                                                                                  num_types=3)]
    empty = (np.eye(3) * 7.0, np.zeros((0, 3)), np.zeros(0, np.int32))
    b0 = S.pack(full, 3)
    b1 = S.pack([empty, full[0], empty, full[1], empty], 3)
    theta, s = theta_and_scale(m, b0)
    Et, Ft, Wt = _targets(b0, 5)
    hv0 = np.array([1, 0], np.uint8)
    lam = (1.0, 1.0, 0.1)
    l0, g0, E0, F0, W0 = O.loss_and_grad(m, theta, s, b0, Et, Ft, Wt, lam, has_virial=hv0)
    Et1 = np.array([3.0, Et[0], -2.0, Et[1], 1.0])
    Wt1 = np.stack([np.full(9, 5.0), Wt[0], np.ones(9), Wt[1], np.zeros(9)])
    hv1 = np.array([1, 1, 0, 0, 1], np.uint8)
    l1, g1, E1, F1, W1 = O.loss_and_grad(m, theta, s, b1, Et1, Ft, Wt1, lam, has_virial=hv1)
    assert np.allclose(l1, l0, rtol=1e-14, atol=0) and np.allclose(g1, g0, rtol=1e-12, atol=1e-15)
    assert np.array_equal(E1[[0, 2, 4]], np.zeros(3)) and np.array_equal(W1[[0, 2, 4]], np.zeros((3, 9)))
    na = b0.counts()
    dE = np.mean(((E0 - Et) / na) ** 2)
    dV = np.sum(((W0[0] - Wt[0]) / na[0]) ** 2) / 9.0
    assert np.allclose(l0[[1, 3]], [dE, dV], rtol=1e-13)


# ------------------------------------------------------------------- Adam


def test_adam_defaults_and_first_step():
    """Eqs. (8)-(13) with the printed defaults: at t = 1 theta_1 = theta_0 - lr g/(|g| + eps)."""
    d = json.load(open(os.path.join(GOLDEN, "adam_defaults.json")))
    rng = np.random.default_rng(40)
    th, g = rng.normal(size=50), rng.normal(size=50)
    z = np.zeros(50)
    t1, m1, v1, vm1 = O.adam_step(th, g, z, z, z, 1, lr=5e-3, beta1=d["beta1"], beta2=d["beta2"], eps=d["eps"])
    assert np.allclose(t1, th - 5e-3 * g / (np.abs(g) + d["eps"]), rtol=0, atol=1e-15)


@pytest.mark.parametrize("mode", ["torch", "off"])
def test_adam_matches_torch(mode):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(41)
    th = rng.normal(size=40)
    p = torch.tensor(th.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8, amsgrad=(mode == "torch"))
    m = v = vm = np.zeros(40)
    for t in range(1, 8):
        g = rng.normal(size=40) * (1.0 + t)
        p.grad = torch.tensor(g)
        opt.step()
        th, m, v, vm = O.adam_step(th, g, m, v, vm, t, lr=3e-3, mode=mode)
        assert np.allclose(th, p.detach().numpy(), rtol=1e-14, atol=1e-16)


def test_adam_paper_mode_running_max():
    """Paper mode keeps the max of the bias-corrected second moment (Eq. 12)."""
    g1, g2 = np.array([1.0]), np.array([1e-3])
    z = np.zeros(1)
    _, m1, v1, vm1 = O.adam_step(z, g1, z, z, z, 1, lr=1e-3)
    _, m2, v2, vm2 = O.adam_step(z, g2, m1, v1, vm1, 2, lr=1e-3)
    assert np.isclose(vm1[0], 1.0) and np.isclose(vm2[0], max(1.0, v2[0] / (1 - 0.999 ** 2)))
