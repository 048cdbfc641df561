"""Mini-batch training on top of the hot path: Adam/AMSGrad steps (Eqs. 8-13)
over shuffled minibatches, the two-stage loss-weight / learning-rate protocol
(Methods, Training; Table I) and the epoch-level plateau scheduler (Eq. 14),
with checkpoint and resume.

The dataset and its neighbour lists live in HBM and are built once; each
minibatch is packed on the device by nep_gather_batch. Host work per step is
argument marshalling only; the loss is read back once per epoch.
"""

from __future__ import annotations

from dataclasses import asdict, dataclass, field

import numpy as np
import torch

from .nep import (AdamConfig, Batch, Model, Targets, Zbl, nep_build_neighbors, nep_gather_batch,
                  nep_param_count, nep_train_step, nep_workspace_size, nep_zbl_add)


class Dataset:
    """A packed set of structures with targets, resident on the device, plus the
    per-structure atom / pair / angular-pair counts the minibatch packer needs
    (kept on the host, so packing a minibatch needs no device read-back)."""

    def __init__(self, model: Model, host_batch, energy, force, virial, has_virial=None, device="cuda",
                 capacity: int | None = None, zbl: Zbl | None = None):
        batch = Batch.from_host(host_batch, dtype=model.torch_dtype, device=device)
        nbr = nep_build_neighbors(model, batch, capacity, species_runs=True)
        targets = Targets(energy, force, virial, has_virial, dtype=model.torch_dtype, device=device)
        if zbl is not None:
            # the ZBL term has no parameter: training NEP on targets minus ZBL is
            # training NEP + ZBL on the targets (same residuals, loss, gradient);
            # the copies keep the caller's tensors unchanged
            targets.energy, targets.force, targets.virial = (t.clone() for t in
                                                             (targets.energy, targets.force, targets.virial))
            nep_zbl_add(model, zbl, batch, nbr, targets.energy, targets.force, targets.virial, scale=-1.0)
        self._init(model, batch, nbr, targets, host_batch.atom_offset)

    @classmethod
    def from_device(cls, model: Model, batch, nbr, targets, atom_offset) -> "Dataset":
        """Wrap a batch, its neighbour lists and targets already on the device."""
        d = cls.__new__(cls)
        d._init(model, batch, nbr, targets, atom_offset)
        return d

    def _init(self, model, batch, nbr, targets, atom_offset):
        self.model, self.batch, self.nbr, self.targets = model, batch, nbr, targets
        off = np.asarray(atom_offset, dtype=np.int64)
        row = self.nbr.row_offset.cpu().numpy()
        seg = self.nbr.seg_count.cpu().numpy()  # [Na][T][2]
        self.atoms = np.diff(off)
        self.pairs = row[off[1:]] - row[off[:-1]]
        ang = np.concatenate([[0], np.cumsum(seg[:, :, 1].sum(axis=1, dtype=np.int64))])
        self.angular = ang[off[1:]] - ang[off[:-1]]

    @property
    def num_structures(self) -> int:
        return self.batch.num_structures

    def sizes(self, ids) -> tuple[int, int, int]:
        ids = np.asarray(ids, dtype=np.int64)
        return int(self.atoms[ids].sum()), int(self.pairs[ids].sum()), int(self.angular[ids].sum())

    def minibatch(self, ids, lambdas=None, ws=None, ids_device=None):
        """(Batch, Neighbors, Targets) of structures `ids`, packed on the device.
        `ids_device` may hold the same ids as a device int32 tensor: a copy from
        pageable host memory waits for the stream's earlier work, so callers
        stepping through an epoch upload its order once and pass slices."""
        na, npairs, nang = self.sizes(ids)
        if ids_device is not None:
            idt = ids_device
        else:
            idt = torch.as_tensor(np.asarray(ids, dtype=np.int32)).to(self.batch.positions.device)
        b, nb, tg = nep_gather_batch(self.model, self.batch, self.nbr, self.targets, idt, na, npairs, nang, ws)
        if lambdas is not None:
            tg.lambdas = tuple(float(x) for x in lambdas)
        return b, nb, tg


class PlateauScheduler:
    """Eq. 14: the learning rate is held for an epoch; after the epoch-averaged
    loss has failed to improve on its best value for more than `patience`
    consecutive epochs it becomes max(factor * lr, min_lr). "Improve" means a
    relative decrease by more than `threshold`; a reduction smaller than `eps`
    is skipped (the semantics of the ReduceLROnPlateau scheduler the paper uses)."""

    def __init__(self, lr: float, factor: float = 0.5, patience: int = 15, min_lr: float = 1e-6,
                 threshold: float = 1e-4, eps: float = 1e-8):
        if not 0.0 < factor < 1.0:
            raise ValueError("factor must be in (0, 1)")
        self.lr, self.factor, self.patience, self.min_lr = float(lr), float(factor), int(patience), float(min_lr)
        self.threshold, self.eps = float(threshold), float(eps)
        self.best = float("inf")
        self.bad_epochs = 0

    def step(self, loss: float) -> float:
        loss = float(loss)
        if loss < self.best * (1.0 - self.threshold):
            self.best = loss
            self.bad_epochs = 0
        else:
            self.bad_epochs += 1
        if self.bad_epochs > self.patience:
            new = max(self.lr * self.factor, self.min_lr)
            if self.lr - new > self.eps:
                self.lr = new
            self.bad_epochs = 0
        return self.lr

    def state_dict(self) -> dict:
        return {k: getattr(self, k) for k in ("lr", "factor", "patience", "min_lr", "threshold", "eps", "best",
                                              "bad_epochs")}

    def load_state_dict(self, d: dict):
        for k, v in d.items():
            setattr(self, k, v)


@dataclass
class TrainConfig:
    """Training hyper-parameters; the defaults are Table I's Stage I / Stage II values."""
    epochs: int = 600
    batch_size: int = 16
    lr: float = 5e-3
    lambdas: tuple = (1.0, 100.0, 1.0)
    patience: int = 15
    factor: float = 0.5
    min_lr: float = 1e-6
    stage2: bool = True
    start_stage2: int = 300
    stage2_lr: float = 5e-4
    stage2_lambdas: tuple = (100.0, 5.0, 30.0)
    seed: int = 0
    adam: AdamConfig = field(default_factory=AdamConfig)


class Trainer:
    """Adam/AMSGrad over shuffled minibatches of a Dataset. Stage 2 starts at
    epoch `start_stage2` with its own learning rate, loss weights and a fresh
    plateau scheduler; the Adam moments carry over. Shuffle of epoch e uses
    numpy PCG64 seeded with seed + 4000 + e."""

    def __init__(self, model: Model, theta, q_scale, cfg: TrainConfig, data: Dataset):
        self.model, self.cfg = model, cfg
        dev, dt = theta.device, theta.dtype
        self.P = nep_param_count(model)[0]
        self.theta = theta.detach().clone()
        self.q_scale = q_scale
        self.m = torch.zeros(self.P, dtype=dt, device=dev)
        self.v = torch.zeros(self.P, dtype=dt, device=dev)
        self.vmax = torch.zeros(self.P, dtype=dt, device=dev)
        self.grad = torch.empty(self.P, dtype=dt, device=dev)
        self.loss = torch.empty(4, dtype=torch.float64, device=dev)
        self.t = 0
        self.epoch = 0
        self.stage = 1
        self.sched = PlateauScheduler(cfg.lr, cfg.factor, cfg.patience, cfg.min_lr)
        # one workspace for the largest possible minibatch of this dataset
        k = min(cfg.batch_size, data.num_structures)
        na = int(np.sort(data.atoms)[::-1][:k].sum())
        npairs = int(np.sort(data.pairs)[::-1][:k].sum())
        self.ws = torch.empty(max(256, nep_workspace_size(model, k, na, npairs)), dtype=torch.uint8, device=dev)

    @property
    def lambdas(self):
        return self.cfg.stage2_lambdas if self.stage == 2 else self.cfg.lambdas

    def epoch_order(self, n: int) -> np.ndarray:
        return np.random.Generator(np.random.PCG64(self.cfg.seed + 4000 + self.epoch)).permutation(n)

    def step(self, b, nb, tg):
        """One optimisation step on a packed minibatch (loss stays on the device):
        the loss gradient and the Adam update in one call (nep_train_step)."""
        self.t += 1
        a = self.cfg.adam
        cfg = AdamConfig(lr=self.sched.lr, beta1=a.beta1, beta2=a.beta2, eps=a.eps, amsgrad=a.amsgrad, mode=a.mode)
        nep_train_step(self.model, self.theta, self.q_scale, b, nb, tg, self.m, self.v, self.vmax, self.t, cfg,
                       self.ws, grad=self.grad, loss=self.loss)

    def run_epoch(self, data: Dataset) -> np.ndarray:
        """One epoch; returns the epoch-averaged [L, Delta_E, Delta_F, Delta_V]."""
        if self.cfg.stage2 and self.stage == 1 and self.epoch >= self.cfg.start_stage2:
            self.stage = 2
            self.sched = PlateauScheduler(self.cfg.stage2_lr, self.cfg.factor, self.cfg.patience, self.cfg.min_lr)
        order = self.epoch_order(data.num_structures)
        bs = self.cfg.batch_size
        acc = torch.zeros(4, dtype=torch.float64, device=self.theta.device)
        nmb = 0
        order_dev = torch.as_tensor(np.asarray(order, dtype=np.int32)).to(self.theta.device)  # one copy per epoch
        for lo in range(0, len(order), bs):
            b, nb, tg = data.minibatch(order[lo:lo + bs], lambdas=self.lambdas, ids_device=order_dev[lo:lo + bs])
            self.step(b, nb, tg)
            acc += self.loss
            nmb += 1
        parts = (acc / max(nmb, 1)).cpu().numpy()
        self.sched.step(parts[0])
        self.epoch += 1
        return parts

    def state_dict(self) -> dict:
        return {"theta": self.theta, "m": self.m, "v": self.v, "vmax": self.vmax, "t": self.t, "epoch": self.epoch,
                "stage": self.stage, "sched": self.sched.state_dict(),
                "cfg": {k: (v if not isinstance(v, AdamConfig) else asdict(v)) for k, v in asdict(self.cfg).items()}}

    def load_state_dict(self, d: dict):
        for k in ("theta", "m", "v", "vmax"):
            getattr(self, k).copy_(d[k])
        self.t, self.epoch, self.stage = int(d["t"]), int(d["epoch"]), int(d["stage"])
        self.sched.load_state_dict(d["sched"])

    def save(self, path: str):
        torch.save(self.state_dict(), path)

    def load(self, path: str):
        self.load_state_dict(torch.load(path, map_location=self.theta.device, weights_only=True))
