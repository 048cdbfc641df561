"""Thin ctypes binding of libnep (``include/nep.h``).

Argument marshalling only: every step of the computation runs in the HIP
library. PyTorch supplies device memory (tensors) and the current stream.
The functions named ``nep_*`` mirror the C entry points one to one; the
classes hold the device tensors the C structs point to.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnep.so")

NEP_OK, NEP_ERR_INVALID_ARG, NEP_ERR_UNSUPPORTED, NEP_ERR_CAPACITY, NEP_ERR_WORKSPACE, NEP_ERR_HIP = 0, -1, -2, -3, -4, -5
NEP_F32, NEP_F64 = 0, 1

EXPORTS = ("nep_param_count", "nep_workspace_size", "nep_build_neighbors", "nep_gather_batch", "nep_forward",
           "nep_loss_and_grad", "nep_backward", "nep_autotune", "nep_adam_step", "nep_descriptor_scale",
           "nep_last_error", "nep_profile_enable", "nep_profile_read", "nep_zbl_add", "nep_train_step",
           "nep_train_step_noalloc", "nep_profile_only")


class NepError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libnep error {code}: {msg}")
        self.code = code


class c_plan(C.Structure):
    _fields_ = [("team_descriptor", C.c_int32), ("team_force", C.c_int32), ("team_tangent", C.c_int32),
                ("team_coeff_grad", C.c_int32), ("coeff_grad_blocks", C.c_int32), ("outer_chunk", C.c_int32),
                ("network", C.c_int32), ("coeff_grad_rows", C.c_int32)]


class c_model(C.Structure):
    _fields_ = [("num_types", C.c_int32), ("n_max_r", C.c_int32), ("n_max_a", C.c_int32),
                ("basis_r", C.c_int32), ("basis_a", C.c_int32), ("l_max", C.c_int32),
                ("l_max_4b", C.c_int32), ("l_max_5b", C.c_int32), ("hidden", C.c_int32),
                ("dtype", C.c_int32), ("rc_r", C.c_double), ("rc_a", C.c_double),
                ("plan", C.POINTER(c_plan))]


class c_batch(C.Structure):
    _fields_ = [("num_structures", C.c_int32), ("num_atoms", C.c_int64), ("atom_offset", C.c_void_p),
                ("positions", C.c_void_p), ("types", C.c_void_p), ("cells", C.c_void_p)]


class c_neighbors(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("row_offset", C.c_void_p), ("seg_count", C.c_void_p),
                ("pairs", C.c_void_p), ("reverse", C.c_void_p), ("atom_struct", C.c_void_p),
                ("species_order", C.c_void_p),
                ("species_offset", C.c_void_p), ("num_pairs", C.c_int64), ("num_angular_pairs", C.c_int64),
                ("species_runs", C.c_void_p)]


class c_targets(C.Structure):
    _fields_ = [("energy", C.c_void_p), ("force", C.c_void_p), ("virial", C.c_void_p),
                ("has_virial", C.c_void_p), ("lambda_e", C.c_double), ("lambda_f", C.c_double),
                ("lambda_v", C.c_double)]


class c_adam(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("amsgrad", C.c_int32), ("amsgrad_mode", C.c_int32)]


class c_zbl(C.Structure):
    _fields_ = [("atomic_number", C.POINTER(C.c_int32)), ("r_inner", C.c_double), ("r_outer", C.c_double)]


_lib = None


def lib():
    """Load libnep.so; raise if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2606_19557_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.nep_param_count.argtypes = [C.POINTER(c_model), C.POINTER(i64), C.POINTER(i64)]
        L.nep_workspace_size.argtypes = [C.POINTER(c_model), i32, i64, i64, C.POINTER(C.c_size_t)]
        L.nep_build_neighbors.argtypes = [C.POINTER(c_model), C.POINTER(c_batch), C.POINTER(c_neighbors), vp,
                                          C.c_size_t, vp]
        L.nep_gather_batch.argtypes = [C.POINTER(c_model), C.POINTER(c_batch), C.POINTER(c_neighbors),
                                       C.POINTER(c_targets), vp, i32, i64, vp, vp, vp, vp, C.POINTER(c_neighbors),
                                       vp, vp, vp, vp, vp, C.c_size_t, vp]
        L.nep_forward.argtypes = [C.POINTER(c_model), vp, vp, C.POINTER(c_batch), C.POINTER(c_neighbors), vp, vp,
                                  vp, vp, vp, C.c_size_t, vp]
        L.nep_loss_and_grad.argtypes = [C.POINTER(c_model), vp, vp, C.POINTER(c_batch), C.POINTER(c_neighbors),
                                        C.POINTER(c_targets), vp, vp, vp, vp, vp, vp, C.c_size_t, vp]
        L.nep_backward.argtypes = [C.POINTER(c_model), vp, vp, C.POINTER(c_batch), C.POINTER(c_neighbors), vp, vp,
                                   vp, vp, vp, C.c_size_t, vp]
        L.nep_autotune.argtypes = [C.POINTER(c_model), vp, vp, C.POINTER(c_batch), C.POINTER(c_neighbors),
                                   C.POINTER(c_targets), vp, vp, vp, C.c_size_t, i32, C.POINTER(c_plan), vp]
        L.nep_adam_step.argtypes = [i64, i32, vp, vp, vp, vp, vp, i64, C.POINTER(c_adam), vp]
        L.nep_train_step.argtypes = [C.POINTER(c_model), vp, vp, C.POINTER(c_batch), C.POINTER(c_neighbors),
                                     C.POINTER(c_targets), vp, vp, vp, i64, C.POINTER(c_adam), vp, vp, vp,
                                     C.c_size_t, vp]
        L.nep_train_step_noalloc.argtypes = [C.POINTER(c_model), vp, vp, C.POINTER(c_batch), C.POINTER(c_neighbors),
                                             C.POINTER(c_targets), vp, vp, vp, i64, C.POINTER(c_adam), vp, vp, vp]
        L.nep_descriptor_scale.argtypes = [i64, i64, i32, vp, vp, vp]
        L.nep_zbl_add.argtypes = [C.POINTER(c_model), C.POINTER(c_zbl), C.POINTER(c_batch), C.POINTER(c_neighbors),
                                  C.c_double, vp, vp, vp, vp, C.c_size_t, vp]
        L.nep_last_error.restype = C.c_char_p
        L.nep_profile_enable.argtypes = [i32]
        L.nep_profile_read.argtypes = [i32, vp, vp, vp, C.POINTER(i32)]
        L.nep_profile_only.argtypes = [C.c_char_p]
        for name in EXPORTS:
            getattr(L, name).restype = C.c_char_p if name == "nep_last_error" else i32
        _lib = L
    return _lib


def _check(code: int):
    if code != NEP_OK:
        raise NepError(code, lib().nep_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


# ------------------------------------------------------------------ model


@dataclass(frozen=True)
class Plan:
    """Launch plan (nep_plan); 0 = the library default."""
    team_descriptor: int = 0
    team_force: int = 0
    team_tangent: int = 0
    team_coeff_grad: int = 0
    coeff_grad_blocks: int = 0
    outer_chunk: int = 0
    network: int = 0  # 1 = matrix-core tiles, 2 = one lane per atom, 3 = inside the sweeps
    coeff_grad_rows: int = 0  # 0 = pair-per-lane coefficient sweep; 1-3 = moment rows per lane

    def c(self) -> c_plan:
        return c_plan(self.team_descriptor, self.team_force, self.team_tangent, self.team_coeff_grad,
                      self.coeff_grad_blocks, self.outer_chunk, self.network, self.coeff_grad_rows)

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k in self.__dataclass_fields__}


@dataclass(frozen=True)
class Model:
    num_types: int
    rc_r: float
    rc_a: float
    n_max_r: int
    n_max_a: int
    basis_r: int
    basis_a: int
    l_max: int = 4
    l_max_4b: int = 0
    l_max_5b: int = 0
    hidden: int = 30
    dtype: str = "f32"
    plan: Plan | None = None

    @property
    def torch_dtype(self):
        return torch.float64 if self.dtype == "f64" else torch.float32

    def with_plan(self, plan: Plan | None) -> "Model":
        from dataclasses import replace

        return replace(self, plan=plan)

    def c(self) -> c_model:
        # the pointer object keeps the plan struct alive as long as the model struct
        plan = C.pointer(self.plan.c()) if self.plan is not None else C.POINTER(c_plan)()
        return c_model(self.num_types, self.n_max_r, self.n_max_a, self.basis_r, self.basis_a, self.l_max,
                       self.l_max_4b, self.l_max_5b, self.hidden, NEP_F64 if self.dtype == "f64" else NEP_F32,
                       float(self.rc_r), float(self.rc_a), plan)

    @classmethod
    def from_dict(cls, d: dict, dtype: str = "f32") -> "Model":
        keys = ("num_types", "rc_r", "rc_a", "n_max_r", "n_max_a", "basis_r", "basis_a", "l_max", "l_max_4b",
                "l_max_5b", "hidden")
        return cls(**{k: d[k] for k in keys}, dtype=dtype)


def nep_param_count(model: Model):
    P, D = C.c_int64(), C.c_int64()
    m = model.c()
    _check(lib().nep_param_count(C.byref(m), C.byref(P), C.byref(D)))
    return int(P.value), int(D.value)


# ----------------------------------------------------------------- batch


class Batch:
    """Device-resident packed batch (positions in the model dtype)."""

    def __init__(self, positions, types, cells, atom_offset, dtype=torch.float32, device="cuda"):
        self.positions = torch.as_tensor(positions).to(device=device, dtype=dtype).contiguous()
        self.types = torch.as_tensor(types).to(device=device, dtype=torch.int32).contiguous()
        self.cells = torch.as_tensor(cells).to(device=device, dtype=torch.float64).reshape(-1, 3, 3).contiguous()
        self.atom_offset = torch.as_tensor(atom_offset).to(device=device, dtype=torch.int64).contiguous()
        self.num_structures = int(self.cells.shape[0])
        self.num_atoms = int(self.positions.shape[0])

    @property
    def counts(self):
        """Atoms per structure (host tensor; reads the offsets back)."""
        return torch.diff(self.atom_offset.cpu())

    @classmethod
    def from_host(cls, b, dtype=torch.float32, device="cuda"):
        return cls(b.positions, b.types, b.cells, b.atom_offset, dtype=dtype, device=device)

    def c(self) -> c_batch:
        return c_batch(self.num_structures, self.num_atoms, _ptr(self.atom_offset), _ptr(self.positions),
                       _ptr(self.types), _ptr(self.cells))


class Neighbors:
    """Device-resident neighbour lists (see nep_neighbors in nep.h)."""

    def __init__(self, model: Model, batch: Batch, capacity: int, species_runs: bool = False):
        self._alloc(model.num_types, batch.num_atoms, capacity, model.torch_dtype, batch.positions.device)
        if species_runs:
            self.species_runs = torch.zeros((max(batch.num_structures, 1), model.num_types, 2), dtype=torch.int32,
                                            device=batch.positions.device)

    @classmethod
    def empty(cls, num_types: int, num_atoms: int, capacity: int, dtype, device) -> "Neighbors":
        nb = cls.__new__(cls)
        nb._alloc(num_types, num_atoms, capacity, dtype, device, zero=False)
        return nb

    def _alloc(self, T, Na, capacity, dtype, dev, zero=True):
        new = torch.zeros if zero else torch.empty
        self.row_offset = new(Na + 1, dtype=torch.int64, device=dev)
        self.seg_count = new((Na, T, 2), dtype=torch.int32, device=dev)
        self.pairs = new((max(capacity, 1), 4), dtype=dtype, device=dev)
        self.reverse = new(max(capacity, 1), dtype=torch.int32, device=dev)
        self.atom_struct = new(max(Na, 1), dtype=torch.int32, device=dev)
        self.species_order = new(max(Na, 1), dtype=torch.int32, device=dev)
        self.species_offset = new(T + 1, dtype=torch.int64, device=dev)
        self.species_runs = None
        self.capacity = capacity
        self.num_pairs = -1
        self.num_angular_pairs = -1

    def c(self) -> c_neighbors:
        return c_neighbors(self.capacity, _ptr(self.row_offset), _ptr(self.seg_count), _ptr(self.pairs),
                           _ptr(self.reverse), _ptr(self.atom_struct), _ptr(self.species_order),
                           _ptr(self.species_offset),
                           self.num_pairs, self.num_angular_pairs, _ptr(self.species_runs))

    def neighbor_index(self):
        """j of every pair (host int64), decoded from the 4th slot."""
        w = self.pairs[: self.num_pairs, 3].contiguous()
        if w.dtype == torch.float32:
            return w.view(torch.int32).to(torch.int64).cpu()
        return w.view(torch.int64).cpu()


def nep_workspace_size(model: Model, num_structures: int, num_atoms: int, num_pairs: int) -> int:
    n = C.c_size_t()
    m = model.c()
    _check(lib().nep_workspace_size(C.byref(m), int(num_structures), int(num_atoms), int(num_pairs), C.byref(n)))
    return int(n.value)


def workspace(model: Model, batch: Batch, nbr: Neighbors | None = None):
    pairs = nbr.num_pairs if nbr is not None and nbr.num_pairs > 0 else 0
    n = nep_workspace_size(model, batch.num_structures, batch.num_atoms, pairs)
    return torch.empty(max(n, 256), dtype=torch.uint8, device=batch.positions.device)


def nep_build_neighbors(model: Model, batch: Batch, capacity: int | None = None, ws=None,
                        species_runs: bool = False) -> Neighbors:
    """Build the lists; grows the pair buffer once when the first guess is short.
    species_runs: also keep each structure's species runs (for a dataset that
    minibatches are gathered from)."""
    if capacity is None:
        capacity = max(1024, batch.num_atoms * 64)
    ws = ws if ws is not None else workspace(model, batch)
    for _ in range(2):
        nb = Neighbors(model, batch, capacity, species_runs=species_runs)
        m, b, cn = model.c(), batch.c(), nb.c()
        code = lib().nep_build_neighbors(C.byref(m), C.byref(b), C.byref(cn), _ptr(ws), ws.numel(), _stream())
        nb.num_pairs, nb.num_angular_pairs = int(cn.num_pairs), int(cn.num_angular_pairs)
        if code == NEP_ERR_CAPACITY:
            capacity = nb.num_pairs
            continue
        _check(code)
        return nb
    raise NepError(NEP_ERR_CAPACITY, "neighbour capacity retry failed")


def nep_gather_batch(model: Model, src: Batch, src_nbr: Neighbors, src_targets, ids, num_atoms: int,
                     num_pairs: int, num_angular_pairs: int, ws=None):
    """Minibatch of structures `ids` (device int32 tensor) of a packed dataset:
    (Batch, Neighbors, Targets or None). num_atoms / num_pairs / num_angular_pairs
    are the sums of the selected structures' counts (see Dataset)."""
    dev, dt = src.positions.device, model.torch_dtype
    n = int(ids.numel())
    ids = ids.to(device=dev, dtype=torch.int32).contiguous()
    T = model.num_types
    off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    pos = torch.empty((num_atoms, 3), dtype=dt, device=dev)
    typ = torch.empty(num_atoms, dtype=torch.int32, device=dev)
    cells = torch.empty((n, 3, 3), dtype=torch.float64, device=dev)
    nb = Neighbors.empty(T, num_atoms, num_pairs, dt, dev)
    tg = None
    E = F = W = hv = None
    if src_targets is not None:
        E = torch.empty(n, dtype=torch.float64, device=dev)
        F = torch.empty((num_atoms, 3), dtype=dt, device=dev)
        W = torch.empty((n, 9), dtype=torch.float64, device=dev)
        hv = torch.empty(n, dtype=torch.uint8, device=dev)
    need = 8 * (n + 1) + (4 * T * (n + 1) if src_nbr.species_runs is not None else 0)
    ws = ws if ws is not None and ws.numel() >= need else torch.empty(need, dtype=torch.uint8, device=dev)
    m, sb, sn, cn = model.c(), src.c(), src_nbr.c(), nb.c()
    stg = src_targets.c() if src_targets is not None else None
    _check(lib().nep_gather_batch(C.byref(m), C.byref(sb), C.byref(sn), C.byref(stg) if stg is not None else None,
                                  _ptr(ids), n, int(num_atoms), _ptr(off), _ptr(pos), _ptr(typ), _ptr(cells),
                                  C.byref(cn), _ptr(E), _ptr(F), _ptr(W), _ptr(hv), _ptr(ws), ws.numel(), _stream()))
    nb.num_pairs, nb.num_angular_pairs = int(num_pairs), int(num_angular_pairs)
    b = Batch.__new__(Batch)
    b.positions, b.types, b.cells, b.atom_offset = pos, typ, cells, off
    b.num_structures, b.num_atoms = n, int(num_atoms)
    if src_targets is not None:
        tg = Targets.__new__(Targets)
        tg.energy, tg.force, tg.virial, tg.has_virial = E, F, W, hv
        tg.lambdas = src_targets.lambdas
    return b, nb, tg


# --------------------------------------------------------------- compute


def nep_forward(model: Model, theta, q_scale, batch: Batch, nbr: Neighbors, ws=None, want_force=True,
                want_virial=True, want_descriptor=False, zbl=None):
    """E [Ns] f64, F [Na,3], W [Ns,9] f64 (None when not asked) and optionally q [Na,D];
    with `zbl` (a Zbl) the ZBL term is added to E, F and W (nep_zbl_add)."""
    dev, dt = batch.positions.device, model.torch_dtype
    P, D = nep_param_count(model)
    ws = ws if ws is not None else workspace(model, batch, nbr)
    E = torch.empty(batch.num_structures, dtype=torch.float64, device=dev)
    F = torch.empty((batch.num_atoms, 3), dtype=dt, device=dev) if want_force else None
    W = torch.empty((batch.num_structures, 9), dtype=torch.float64, device=dev) if want_virial else None
    q = torch.empty((batch.num_atoms, D), dtype=dt, device=dev) if want_descriptor else None
    m, b, cn = model.c(), batch.c(), nbr.c()
    _check(lib().nep_forward(C.byref(m), _ptr(theta), _ptr(q_scale), C.byref(b), C.byref(cn), _ptr(E), _ptr(F),
                             _ptr(W), _ptr(q), _ptr(ws), ws.numel(), _stream()))
    if zbl is not None:
        nep_zbl_add(model, zbl, batch, nbr, E, F, W, ws=ws)
    return (E, F, W, q) if want_descriptor else (E, F, W)


@dataclass(frozen=True)
class Zbl:
    """ZBL pair term: nuclear charge of each species and the switch range (A)."""

    atomic_numbers: tuple
    r_inner: float
    r_outer: float


def nep_zbl_add(model: Model, zbl: Zbl, batch: Batch, nbr: Neighbors, energy=None, force=None, virial=None,
                scale: float = 1.0, ws=None):
    """Adds scale * (E, F, W) of the ZBL term to the given tensors in place
    (energy [Ns] f64, force [Na,3] model dtype, virial [Ns,9] f64; any may be None)."""
    if len(zbl.atomic_numbers) != model.num_types:
        raise ValueError(f"{len(zbl.atomic_numbers)} atomic numbers for {model.num_types} species")
    dev = batch.positions.device
    need = 80 * batch.num_atoms
    ws = ws if ws is not None and ws.numel() >= need else torch.empty(max(need, 8), dtype=torch.uint8, device=dev)
    z = (C.c_int32 * max(1, model.num_types))(*[int(v) for v in zbl.atomic_numbers])
    cz = c_zbl(C.cast(z, C.POINTER(C.c_int32)), float(zbl.r_inner), float(zbl.r_outer))
    m, b, cn = model.c(), batch.c(), nbr.c()
    _check(lib().nep_zbl_add(C.byref(m), C.byref(cz), C.byref(b), C.byref(cn), float(scale), _ptr(energy),
                             _ptr(force), _ptr(virial), _ptr(ws), ws.numel(), _stream()))


def nep_descriptors(model: Model, theta, batch: Batch, nbr: Neighbors, ws=None):
    dev, dt = batch.positions.device, model.torch_dtype
    _, D = nep_param_count(model)
    ws = ws if ws is not None else workspace(model, batch, nbr)
    q = torch.empty((batch.num_atoms, D), dtype=dt, device=dev)
    m, b, cn = model.c(), batch.c(), nbr.c()
    _check(lib().nep_forward(C.byref(m), _ptr(theta), None, C.byref(b), C.byref(cn), None, None, None, _ptr(q),
                             _ptr(ws), ws.numel(), _stream()))
    return q


def nep_descriptor_scale(q):
    s = torch.empty(q.shape[1], dtype=q.dtype, device=q.device)
    _check(lib().nep_descriptor_scale(q.shape[0], q.shape[1], NEP_F64 if q.dtype == torch.float64 else NEP_F32,
                                      _ptr(q), _ptr(s), _stream()))
    return s


class Targets:
    def __init__(self, energy, force, virial, has_virial=None, lambdas=(1.0, 1.0, 0.1), dtype=torch.float32,
                 device="cuda"):
        self.energy = torch.as_tensor(energy).to(device=device, dtype=torch.float64).contiguous()
        self.force = torch.as_tensor(force).to(device=device, dtype=dtype).reshape(-1, 3).contiguous()
        self.virial = torch.as_tensor(virial).to(device=device, dtype=torch.float64).reshape(-1, 9).contiguous()
        self.has_virial = None if has_virial is None else \
            torch.as_tensor(has_virial).to(device=device, dtype=torch.uint8).contiguous()
        self.lambdas = tuple(float(x) for x in lambdas)

    def c(self) -> c_targets:
        return c_targets(_ptr(self.energy), _ptr(self.force), _ptr(self.virial), _ptr(self.has_virial),
                         *self.lambdas)


def nep_loss_and_grad(model: Model, theta, q_scale, batch: Batch, nbr: Neighbors, targets: Targets, ws=None,
                      grad=None, loss=None, want_predictions=False):
    """Returns (loss[4] f64 device, grad [P]) and, when asked, (E, F, W)."""
    dev, dt = batch.positions.device, model.torch_dtype
    P, _ = nep_param_count(model)
    ws = ws if ws is not None else workspace(model, batch, nbr)
    grad = grad if grad is not None else torch.empty(P, dtype=dt, device=dev)
    loss = loss if loss is not None else torch.empty(4, dtype=torch.float64, device=dev)
    E = F = W = None
    if want_predictions:
        E = torch.empty(batch.num_structures, dtype=torch.float64, device=dev)
        F = torch.empty((batch.num_atoms, 3), dtype=dt, device=dev)
        W = torch.empty((batch.num_structures, 9), dtype=torch.float64, device=dev)
    m, b, cn, tg = model.c(), batch.c(), nbr.c(), targets.c()
    _check(lib().nep_loss_and_grad(C.byref(m), _ptr(theta), _ptr(q_scale), C.byref(b), C.byref(cn), C.byref(tg),
                                   _ptr(loss), _ptr(grad), _ptr(E), _ptr(F), _ptr(W), _ptr(ws), ws.numel(),
                                   _stream()))
    return (loss, grad, E, F, W) if want_predictions else (loss, grad)


def nep_backward(model: Model, theta, q_scale, batch: Batch, nbr: Neighbors, dE=None, dF=None, dW=None, ws=None):
    dev, dt = batch.positions.device, model.torch_dtype
    P, _ = nep_param_count(model)
    ws = ws if ws is not None else workspace(model, batch, nbr)
    grad = torch.empty(P, dtype=dt, device=dev)
    dE = None if dE is None else dE.to(dtype=torch.float64).contiguous()
    dF = None if dF is None else dF.to(dtype=dt).contiguous()
    dW = None if dW is None else dW.to(dtype=torch.float64).reshape(-1, 9).contiguous()
    m, b, cn = model.c(), batch.c(), nbr.c()
    _check(lib().nep_backward(C.byref(m), _ptr(theta), _ptr(q_scale), C.byref(b), C.byref(cn), _ptr(dE), _ptr(dF),
                              _ptr(dW), _ptr(grad), _ptr(ws), ws.numel(), _stream()))
    return grad


def nep_autotune(model: Model, theta, q_scale, batch: Batch, nbr: Neighbors, targets: Targets, ws=None,
                 repeats: int = 5) -> Plan:
    """Time candidate launch plans on this batch (see nep.h) and return the fastest."""
    dev, dt = batch.positions.device, model.torch_dtype
    P, _ = nep_param_count(model)
    if ws is None:
        # room for the largest candidate (more partial rows than the default)
        big = model.with_plan(Plan(4, 4, 4, 4, 4096, 32))
        n = max(nep_workspace_size(model, batch.num_structures, batch.num_atoms, max(nbr.num_pairs, 0)),
                nep_workspace_size(big, batch.num_structures, batch.num_atoms, max(nbr.num_pairs, 0)))
        ws = torch.empty(n, dtype=torch.uint8, device=dev)
    grad = torch.empty(P, dtype=dt, device=dev)
    loss = torch.empty(4, dtype=torch.float64, device=dev)
    out = c_plan()
    m, b, cn, tg = model.c(), batch.c(), nbr.c(), targets.c()
    _check(lib().nep_autotune(C.byref(m), _ptr(theta), _ptr(q_scale), C.byref(b), C.byref(cn), C.byref(tg),
                              _ptr(loss), _ptr(grad), _ptr(ws), ws.numel(), int(repeats), C.byref(out), _stream()))
    return Plan(out.team_descriptor, out.team_force, out.team_tangent, out.team_coeff_grad, out.coeff_grad_blocks,
                out.outer_chunk, out.network, out.coeff_grad_rows)


@dataclass
class AdamConfig:
    lr: float = 5e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    amsgrad: bool = True
    mode: str = "paper"  # "paper" (max of bias-corrected v, Eq. 12) or "torch"

    def c(self) -> c_adam:
        return c_adam(self.lr, self.beta1, self.beta2, self.eps, 1 if self.amsgrad else 0,
                      0 if self.mode == "paper" else 1)


def nep_adam_step(theta, grad, m, v, vmax, t: int, cfg: AdamConfig):
    dt = NEP_F64 if theta.dtype == torch.float64 else NEP_F32
    c = cfg.c()
    _check(lib().nep_adam_step(theta.numel(), dt, _ptr(theta), _ptr(grad), _ptr(m), _ptr(v), _ptr(vmax), int(t),
                               C.byref(c), _stream()))


def nep_train_step(model: Model, theta, q_scale, batch: Batch, nbr: Neighbors, targets: Targets, m, v, vmax,
                   t: int, cfg: AdamConfig, ws=None, grad=None, loss=None):
    """nep_loss_and_grad + nep_adam_step in one call (theta, m, v, vmax updated in
    place); returns (loss[4] f64, grad [P]) with grad taken at the old theta."""
    dev, dt = batch.positions.device, model.torch_dtype
    P, _ = nep_param_count(model)
    ws = ws if ws is not None else workspace(model, batch, nbr)
    grad = grad if grad is not None else torch.empty(P, dtype=dt, device=dev)
    loss = loss if loss is not None else torch.empty(4, dtype=torch.float64, device=dev)
    mm, b, cn, tg, c = model.c(), batch.c(), nbr.c(), targets.c(), cfg.c()
    _check(lib().nep_train_step(C.byref(mm), _ptr(theta), _ptr(q_scale), C.byref(b), C.byref(cn), C.byref(tg),
                                _ptr(m), _ptr(v), _ptr(vmax), int(t), C.byref(c), _ptr(loss), _ptr(grad), _ptr(ws),
                                ws.numel(), _stream()))
    return loss, grad


def nep_train_step_noalloc(model: Model, theta, q_scale, batch: Batch, nbr: Neighbors, targets: Targets, m, v,
                           vmax, t: int, cfg: AdamConfig, grad, loss):
    """nep_train_step with the library's static device workspace (no allocation
    anywhere in the call): the caller passes every output (grad [P], loss [4]
    f64); returns (loss, grad)."""
    mm, b, cn, tg, c = model.c(), batch.c(), nbr.c(), targets.c(), cfg.c()
    _check(lib().nep_train_step_noalloc(C.byref(mm), _ptr(theta), _ptr(q_scale), C.byref(b), C.byref(cn),
                                        C.byref(tg), _ptr(m), _ptr(v), _ptr(vmax), int(t), C.byref(c), _ptr(loss),
                                        _ptr(grad), _stream()))
    return loss, grad


def nep_profile_enable(on: bool):
    _check(lib().nep_profile_enable(1 if on else 0))


def nep_profile_only(kernel: str | None):
    """Time only launches of `kernel` (None: every kernel) while profiling is on."""
    _check(lib().nep_profile_only(None if kernel is None else kernel.encode()))


def nep_profile_read(cap: int = 64):
    names = (C.c_char * 64 * cap)()
    launches = (C.c_int64 * cap)()
    total = (C.c_double * cap)()
    count = C.c_int32()
    _check(lib().nep_profile_read(cap, C.cast(names, C.c_void_p), C.cast(launches, C.c_void_p),
                                  C.cast(total, C.c_void_p), C.byref(count)))
    return {bytes(names[k]).split(b"\0")[0].decode(): (int(launches[k]), float(total[k]))
            for k in range(min(cap, count.value))}


# ------------------------------------------------------- autograd function


class NEPFunction(torch.autograd.Function):
    """theta -> (E, F, W) with a hand-written backward (nep_backward, a VJP
    whose force and virial parts are the mixed second derivative d^2E/dtheta dr)."""

    @staticmethod
    def forward(ctx, theta, model, q_scale, batch, nbr, ws):
        E, F, W = nep_forward(model, theta.detach(), q_scale, batch, nbr, ws)
        ctx.save_for_backward(theta)
        ctx.meta = (model, q_scale, batch, nbr, ws)
        return E, F, W

    @staticmethod
    def backward(ctx, dE, dF, dW):
        (theta,) = ctx.saved_tensors
        model, q_scale, batch, nbr, ws = ctx.meta
        g = nep_backward(model, theta.detach(), q_scale, batch, nbr, dE, dF, dW, ws)
        return g, None, None, None, None, None
