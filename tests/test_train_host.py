"""Host logic of training: the plateau scheduler (Eq. 14) against torch's
ReduceLROnPlateau, and the default protocol against Table I."""

import json
import os

import numpy as np
import pytest
import torch

train = pytest.importorskip("paper_2606_19557_amd.train")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _torch_lrs(losses, lr, **kw):
    p = torch.nn.Parameter(torch.zeros(1))
    opt = torch.optim.SGD([p], lr=lr)
    sch = torch.optim.lr_scheduler.ReduceLROnPlateau(opt, mode="min", **kw)
    out = []
    for x in losses:
        sch.step(x)
        out.append(opt.param_groups[0]["lr"])
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plateau_matches_torch(seed):
    rng = np.random.default_rng(seed)
    # noisy decay with long flat stretches, so reductions happen several times
    x = np.exp(-np.arange(400) / 80.0) + 0.02 * rng.random(400)
    x[150:260] = x[150]
    x[300:] = x[300] * (1 + 1e-5 * rng.random(100))
    ours = train.PlateauScheduler(5e-3, factor=0.5, patience=15, min_lr=1e-6)
    got = [ours.step(v) for v in x]
    ref = _torch_lrs(x, 5e-3, factor=0.5, patience=15, min_lr=1e-6)
    assert np.allclose(got, ref, rtol=0, atol=0)
    assert min(got) < 5e-3 / 4  # it did reduce


def test_plateau_floor_and_state():
    s = train.PlateauScheduler(1e-3, factor=0.1, patience=0, min_lr=2e-6)
    for _ in range(10):
        s.step(1.0)
    assert s.lr == pytest.approx(2e-6)
    t = train.PlateauScheduler(0.5)
    t.load_state_dict(s.state_dict())
    assert t.state_dict() == s.state_dict()


def test_defaults_are_table1():
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "table1_training.json")))
    c = train.TrainConfig()
    s1, s2 = g["stage1"], g["stage2"]
    assert (c.epochs, c.lr, c.batch_size, c.patience, c.factor) == (s1["epoch"], s1["lr"], s1["batch"],
                                                                    s1["scheduler_patience"], s1["scheduler_factor"])
    assert c.lambdas == (s1["lambda_e"], s1["lambda_f"], s1["lambda_v"])
    assert (c.start_stage2, c.stage2_lr) == (s2["start_stage2"], s2["stage2_lr"])
    assert c.stage2_lambdas == (s2["stage2_lambda_e"], s2["stage2_lambda_f"], s2["stage2_lambda_v"])
