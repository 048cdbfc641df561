"""FP64 CPU oracle for NEP energies, forces, virials, loss and loss gradient.

TEST INFRASTRUCTURE ONLY: the slow, obviously-correct reference that the GPU
path is checked against. Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import it; the GPU library never does, and the two
share no code. The arithmetic lives in ``nep_oracle.c`` (see its header for
the equations it follows); this module marshals numpy arrays through ctypes
and adds the descriptor scaler (Eq. 2) and Adam/AMSGrad (``adam.py``).
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from .adam import adam_step  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "liborc.so")
_lib = None


class _Model(C.Structure):
    _fields_ = [
        ("num_types", C.c_int), ("n_max_r", C.c_int), ("n_max_a", C.c_int),
        ("basis_r", C.c_int), ("basis_a", C.c_int), ("l_max", C.c_int),
        ("l_max_4b", C.c_int), ("l_max_5b", C.c_int), ("hidden", C.c_int),
        ("rc_r", C.c_double), ("rc_a", C.c_double),
    ]


@dataclass(frozen=True)
class Model:
    num_types: int
    rc_r: float
    rc_a: float
    n_max_r: int
    n_max_a: int
    basis_r: int
    basis_a: int
    l_max: int
    l_max_4b: int = 0
    l_max_5b: int = 0
    hidden: int = 30

    def c(self) -> _Model:
        return _Model(self.num_types, self.n_max_r, self.n_max_a, self.basis_r, self.basis_a,
                      self.l_max, self.l_max_4b, self.l_max_5b, self.hidden, self.rc_r, self.rc_a)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from .build import build
            build()
        L = C.CDLL(_LIB_PATH)
        dp, ip, lp = C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_long)
        mp = C.POINTER(_Model)
        L.orc_dims.argtypes = [mp, lp, lp]
        L.orc_neighbors.argtypes = [C.c_int, dp, dp, C.c_double, C.c_long, ip, ip, ip, dp]
        L.orc_neighbors.restype = C.c_long
        L.orc_descriptors.argtypes = [mp, dp, C.c_int, dp, dp, ip, dp]
        L.orc_forward.argtypes = [mp, dp, dp, C.c_int, dp, dp, ip, dp, dp, dp, dp]
        L.orc_vjp.argtypes = [mp, dp, dp, C.c_int, dp, dp, ip, C.c_double, dp, dp, dp]
        L.orc_batch_loss_grad.argtypes = [mp, dp, dp, C.c_int, lp, dp, dp, ip, dp, dp, dp,
                                          C.POINTER(C.c_ubyte), C.c_double, C.c_double, C.c_double,
                                          dp, dp, dp, dp, dp, C.c_int]
        L.orc_search_seconds.argtypes = [C.c_int]
        L.orc_search_seconds.restype = C.c_double
        L.orc_wigner3j.argtypes = [C.c_int] * 6
        L.orc_wigner3j.restype = C.c_double
        L.orc_real_sh.argtypes = [C.c_int, dp, dp, dp]
        L.orc_basis.argtypes = [C.c_double, C.c_double, C.c_int, dp, dp]
        L.orc_q4_of_moments.argtypes = [dp, dp, dp]
        L.orc_complex_sh2.argtypes = [dp, dp, dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def dims(model: Model):
    P, D = C.c_long(), C.c_long()
    if lib().orc_dims(C.byref(model.c()), C.byref(P), C.byref(D)):
        raise ValueError("invalid model")
    return int(P.value), int(D.value)


def neighbors(cell, pos, rc):
    """Brute-force list of every (i, j, image shift, r_ij) with |r_ij| < rc."""
    cell, pos = _f64(cell), _f64(pos)
    n = pos.shape[0]
    cnt = lib().orc_neighbors(n, _d(cell), _d(pos), float(rc), 0, None, None, None, None)
    if cnt < 0:
        raise ValueError("singular cell")
    i = np.zeros(cnt, np.int32)
    j = np.zeros(cnt, np.int32)
    s = np.zeros((cnt, 3), np.int32)
    r = np.zeros((cnt, 3), np.float64)
    lib().orc_neighbors(n, _d(cell), _d(pos), float(rc), cnt, _i(i), _i(j), _i(s), _d(r))
    return i, j, s, r


def descriptors(model: Model, theta, batch):
    """Descriptor q [Na, D] of every atom (Eqs. 15-20)."""
    P, D = dims(model)
    theta = _f64(theta)
    out = np.zeros((batch.num_atoms, D))
    for s in range(batch.num_structures):
        cell, pos, typ = batch.structure(s)
        a = int(batch.atom_offset[s])
        q = np.zeros((len(pos), D))
        rc = lib().orc_descriptors(C.byref(model.c()), _d(theta), len(pos), _d(_f64(cell)), _d(_f64(pos)),
                                   _i(_i32(typ)), _d(q))
        if rc:
            raise RuntimeError(f"orc_descriptors failed ({rc})")
        out[a:a + len(pos)] = q
    return out


def scaler(q, floor: float = 1e-10):
    """Eq. (2): s_nu = 1/(max_nu - min_nu) over all atoms; 1 where the range is below ``floor``."""
    q = np.asarray(q, dtype=np.float64)
    rng = q.max(axis=0) - q.min(axis=0)
    return np.where(rng < floor, 1.0, 1.0 / np.where(rng < floor, 1.0, rng))


def forward(model: Model, theta, qscale, batch, per_atom: bool = False):
    """E [Ns], F [Na, 3], W [Ns, 9] (and per-atom energies when asked)."""
    theta, qscale = _f64(theta), _f64(qscale)
    Ns, Na = batch.num_structures, batch.num_atoms
    E = np.zeros(Ns)
    Ei = np.zeros(Na)
    F = np.zeros((Na, 3))
    W = np.zeros((Ns, 9))
    for s in range(Ns):
        cell, pos, typ = batch.structure(s)
        a = int(batch.atom_offset[s])
        n = len(pos)
        e = np.zeros(1)
        ei = np.zeros(n)
        f = np.zeros((n, 3))
        w = np.zeros(9)
        rc = lib().orc_forward(C.byref(model.c()), _d(theta), _d(qscale), n, _d(_f64(cell)), _d(_f64(pos)),
                               _i(_i32(typ)), _d(e), _d(ei), _d(f), _d(w))
        if rc:
            raise RuntimeError(f"orc_forward failed ({rc})")
        E[s], Ei[a:a + n], F[a:a + n], W[s] = e[0], ei, f, w
    return (E, F, W, Ei) if per_atom else (E, F, W)


def energy(model: Model, theta, qscale, cell, pos, types):
    """Energy of a single structure (for finite differences)."""
    e = np.zeros(1)
    n = len(pos)
    rc = lib().orc_forward(C.byref(model.c()), _d(_f64(theta)), _d(_f64(qscale)), n, _d(_f64(cell)),
                           _d(_f64(pos)), _i(_i32(types)), _d(e), None, None, None)
    if rc:
        raise RuntimeError(f"orc_forward failed ({rc})")
    return float(e[0])


def vjp(model: Model, theta, qscale, batch, ebar, ubar, Ubar):
    """grad = sum_s ebar_s dE_s/dtheta + sum_i ubar_i . dF_i/dtheta + sum_s Ubar_s : dW_s/dtheta."""
    P, _ = dims(model)
    theta, qscale = _f64(theta), _f64(qscale)
    ebar, ubar, Ubar = _f64(ebar), _f64(ubar).reshape(-1, 3), _f64(Ubar).reshape(-1, 9)
    g = np.zeros(P)
    for s in range(batch.num_structures):
        cell, pos, typ = batch.structure(s)
        a = int(batch.atom_offset[s])
        n = len(pos)
        rc = lib().orc_vjp(C.byref(model.c()), _d(theta), _d(qscale), n, _d(_f64(cell)), _d(_f64(pos)),
                           _i(_i32(typ)), float(ebar[s]), _d(np.ascontiguousarray(ubar[a:a + n])),
                           _d(np.ascontiguousarray(Ubar[s])), _d(g))
        if rc:
            raise RuntimeError(f"orc_vjp failed ({rc})")
    return g


def loss_and_grad(model: Model, theta, qscale, batch, E_t, F_t, W_t, lambdas=(1.0, 1.0, 0.1),
                  has_virial=None, nthreads: int = 1, want_grad: bool = True):
    """Loss (Eqs. 4-7) as [L, dE, dF, dV], its gradient, and the predictions E, F, W."""
    P, _ = dims(model)
    Ns, Na = batch.num_structures, batch.num_atoms
    theta, qscale = _f64(theta), _f64(qscale)
    off = np.ascontiguousarray(batch.atom_offset, dtype=np.int64)
    E = np.zeros(Ns)
    F = np.zeros((Na, 3))
    W = np.zeros((Ns, 9))
    loss = np.zeros(4)
    grad = np.zeros(P) if want_grad else None
    hv = None
    if has_virial is not None:
        hv_arr = np.ascontiguousarray(has_virial, dtype=np.uint8)
        hv = hv_arr.ctypes.data_as(C.POINTER(C.c_ubyte))
    rc = lib().orc_batch_loss_grad(
        C.byref(model.c()), _d(theta), _d(qscale), Ns, off.ctypes.data_as(C.POINTER(C.c_long)),
        _d(_f64(batch.cells)), _d(_f64(batch.positions)), _i(_i32(batch.types)),
        _d(_f64(E_t)), _d(_f64(F_t)), _d(_f64(W_t)), hv,
        float(lambdas[0]), float(lambdas[1]), float(lambdas[2]),
        _d(E), _d(F), _d(W), _d(loss), _d(grad) if want_grad else None, int(nthreads))
    if rc:
        raise RuntimeError(f"orc_batch_loss_grad failed ({rc})")
    return loss, grad, E, F, W


def search_seconds(reset: bool = False) -> float:
    """Seconds the brute-force neighbour search has taken so far, summed over
    threads (timing only); ``reset`` zeroes the counter."""
    return float(lib().orc_search_seconds(1 if reset else 0))


def wigner3j(j1, j2, j3, m1, m2, m3):
    return float(lib().orc_wigner3j(j1, j2, j3, m1, m2, m3))


def real_sh(L, rvec):
    LM = (L + 1) ** 2 - 1
    Y = np.zeros(LM)
    dY = np.zeros((LM, 3))
    lib().orc_real_sh(L, _d(_f64(rvec)), _d(Y), _d(dY))
    return Y, dY


def basis(r, rc, K):
    f = np.zeros(K)
    fp = np.zeros(K)
    lib().orc_basis(float(r), float(rc), int(K), _d(f), _d(fp))
    return f, fp


def q4_of_moments(moments):
    m = np.asarray(moments, dtype=np.complex128)
    out = np.zeros(2)
    lib().orc_q4_of_moments(_d(_f64(m.real)), _d(_f64(m.imag)), _d(out))
    return complex(out[0], out[1])


def complex_sh2(rvec):
    re = np.zeros(5)
    im = np.zeros(5)
    lib().orc_complex_sh2(_d(_f64(rvec)), _d(re), _d(im))
    return re + 1j * im
