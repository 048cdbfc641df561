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


def test_plan_cache_roundtrip(tmp_path):
    """The tuned-plan cache: a miss tunes and stores, a hit for the same kind of
    batch returns the stored plan without tuning; a different density misses."""
    from types import SimpleNamespace

    from paper_2606_19557_amd import nep, tuning

    calls = []

    def fake_tuner(model, theta, qs, batch, nbr, targets, repeats=3):
        calls.append(repeats)
        return nep.Plan(4, 8, 16, 8, 1024, 128, 2)

    m = nep.Model(num_types=1, rc_r=6.0, rc_a=4.0, n_max_r=6, n_max_a=4, basis_r=8, basis_a=8, hidden=30)
    path = str(tmp_path / "plans.json")
    b1, n1 = SimpleNamespace(num_atoms=36391), SimpleNamespace(num_pairs=1757148)
    p, cached = tuning.tuned_plan(m, None, None, b1, n1, None, path=path, tuner=fake_tuner)
    assert not cached and p == nep.Plan(4, 8, 16, 8, 1024, 128, 2) and calls == [3]
    b2, n2 = SimpleNamespace(num_atoms=40000), SimpleNamespace(num_pairs=1900000)  # same buckets
    p2, cached2 = tuning.tuned_plan(m, None, None, b2, n2, None, path=path, tuner=fake_tuner)
    assert cached2 and p2 == p and calls == [3]
    b3, n3 = SimpleNamespace(num_atoms=36391), SimpleNamespace(num_pairs=36391 * 100)  # denser
    _, cached3 = tuning.tuned_plan(m, None, None, b3, n3, None, path=path, tuner=fake_tuner)
    assert not cached3 and len(calls) == 2
    assert len(tuning.load(path)) == 2
    # a read-only shipped file answers misses of the user cache, which wins on a hit
    shipped = str(tmp_path / "shipped.json")
    b4, n4 = SimpleNamespace(num_atoms=300000), SimpleNamespace(num_pairs=300000 * 100)
    key4 = tuning.plan_key(m, b4.num_atoms, n4.num_pairs)
    tuning.store({key4: nep.Plan(16, 16, 16, 32, 512, 256, 3).as_dict(),
                  tuning.plan_key(m, b1.num_atoms, n1.num_pairs): nep.Plan(8, 8, 8, 8, 64, 64, 1).as_dict()}, shipped)
    p4, cached4 = tuning.tuned_plan(m, None, None, b4, n4, None, path=path, tuner=fake_tuner, shipped=shipped)
    assert cached4 and p4 == nep.Plan(16, 16, 16, 32, 512, 256, 3) and len(calls) == 2
    p5, _ = tuning.tuned_plan(m, None, None, b1, n1, None, path=path, tuner=fake_tuner, shipped=shipped)
    assert p5 == p
    assert len(tuning.load(path)) == 2  # shipped plans are not copied into the user cache
