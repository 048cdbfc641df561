"""Launch plans (team sizes 4/8/16 per pair sweep, coefficient-gradient grid,
outer-product chunk) all reproduce the oracle, and the autotuner returns a
valid plan whose results match the default plan's."""

import numpy as np
import pytest
import torch

import oracle as O
from helpers import SMALL_ALLOY, device_inputs, fixture, rel_err, small_alloy_batch

pytestmark = pytest.mark.gpu

N = pytest.importorskip("paper_2606_19557_amd")

PLANS = [
    N.Plan(4, 4, 4, 4, 512, 32, 1),
    N.Plan(16, 16, 16, 16, 4096, 256, 2),
    N.Plan(4, 16, 8, 16, 1, 8, 1),
    N.Plan(16, 4, 16, 8, 7, 100, 2),
    N.Plan(8, 8, 8, 32, 300, 64, 1),
    N.Plan(4, 8, 16, 8, 2048, 64, 3),
    N.Plan(16, 8, 4, 16, 64, 16, 3),
]


def _case(which):
    if which == "small_alloy":
        return fixture(SMALL_ALLOY, seed=7, batch=small_alloy_batch()), "f64", 1e-9
    return fixture("fcc_uneven_256", list(range(10))), "f32", None


@pytest.mark.parametrize("plan", PLANS, ids=lambda p: "-".join(str(v) for v in p.as_dict().values()))
@pytest.mark.parametrize("which", ["small_alloy", "fcc"])
def test_plan_parity(which, plan):
    print(f"plan {which} {plan}", flush=True)
    (md, m, b, th, s, tg), dtype, tol = _case(which)
    b, th, s, tg = device_inputs(dtype, b, th, s, tg)
    model = N.Model.from_dict(md, dtype=dtype).with_plan(plan)
    td = model.torch_dtype
    gb = N.Batch.from_host(b, dtype=td)
    nb = N.nep_build_neighbors(model, gb)
    ws = N.workspace(model, gb, nb)
    theta = torch.tensor(th, dtype=td, device="cuda")
    qs = torch.tensor(s, dtype=td, device="cuda")
    Et, Ft, Wt = tg
    targets = N.Targets(Et, Ft, Wt, lambdas=(1.0, 1.0, 0.1), dtype=td)
    loss, g, E, F, W = N.nep_loss_and_grad(model, theta, qs, gb, nb, targets, ws, want_predictions=True)
    lo, go, Eo, Fo, Wo = O.loss_and_grad(m, th, s, b, Et, Ft, Wt, (1.0, 1.0, 0.1), nthreads=8)
    t = dict(E=tol or 1e-5, F=tol or 1e-4, G=tol or 1e-4, L=tol or 1e-5)
    assert rel_err(E.cpu().numpy(), Eo) < t["E"]
    assert rel_err(F.double().cpu().numpy(), Fo) < t["F"]
    assert rel_err(W.cpu().numpy(), Wo) < t["F"]
    assert rel_err(loss.cpu().numpy(), lo) < t["L"]
    assert rel_err(g.double().cpu().numpy(), go) < t["G"]
    q = N.nep_descriptors(model, theta, gb, nb, ws)
    assert rel_err(q.double().cpu().numpy(), O.descriptors(m, th, b)) < t["F"]
    # the forward-only call under the same plan (fused plans run the force
    # pass inside the descriptor sweep there too)
    E2, F2, W2 = N.nep_forward(model, theta, qs, gb, nb, ws)
    assert rel_err(E2.cpu().numpy(), Eo) < t["E"]
    assert rel_err(F2.double().cpu().numpy(), Fo) < t["F"]
    assert rel_err(W2.cpu().numpy(), Wo) < t["F"]


def test_autotune_returns_valid_plan():
    print("autotune fcc", flush=True)
    md, m, b, th, s, tg = fixture("fcc_uneven_256", list(range(24)))
    b, th, s, tg = device_inputs("f32", b, th, s, tg)
    model = N.Model.from_dict(md, dtype="f32")
    gb = N.Batch.from_host(b)
    nb = N.nep_build_neighbors(model, gb)
    theta = torch.tensor(th, dtype=torch.float32, device="cuda")
    qs = torch.tensor(s, dtype=torch.float32, device="cuda")
    targets = N.Targets(*tg)
    plan = N.nep_autotune(model, theta, qs, gb, nb, targets, repeats=2)
    for k in ("team_descriptor", "team_force", "team_tangent"):
        assert getattr(plan, k) in (4, 8, 16)
    assert plan.team_coeff_grad in (4, 8, 16, 32)
    assert plan.coeff_grad_blocks in (512, 1024, 2048, 4096) and plan.outer_chunk in (32, 64, 128, 256)
    assert plan.network in (1, 2, 3)
    tuned = model.with_plan(plan)
    l0, g0 = N.nep_loss_and_grad(model, theta, qs, gb, nb, targets)
    l1, g1 = N.nep_loss_and_grad(tuned, theta, qs, gb, nb, targets)
    assert rel_err(g1.double().cpu().numpy(), g0.double().cpu().numpy()) < 1e-4
    assert rel_err(l1.cpu().numpy(), l0.cpu().numpy()) < 1e-5
