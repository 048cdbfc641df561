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


# the row-owned angular coefficient sweep (FP32): 1, 2 or 3 moment rows per
# lane on every compiled kernel shape used by a workload, with grids small
# enough that each wavefront walks several tiles and blocks sum several
# wavefronts' accumulators
ROWS_CASES = [
    ("fcc_uneven_256", list(range(10)), 1, 0),
    ("fcc_uneven_256", list(range(10)), 2, 3),
    ("fcc_uneven_256", list(range(10)), 3, 0),
    ("small_alloy", None, 1, 2),
    ("small_alloy", None, 2, 0),
    ("small_alloy", None, 3, 1),
    ("alloy4_1024", [4, 0, 1, 3], 2, 0),
    ("alloy4_1024", [4, 0, 1, 3], 3, 5),
    ("mixed3_4096", [0, 1, 2, 4, 5], 2, 0),
    ("mixed3_4096", [0, 1, 2, 4, 5], 3, 2),
    ("large5_32", [20], 2, 0),
    ("large5_32", [20], 3, 0),
]


@pytest.mark.parametrize("name,idx,rows,blocks", ROWS_CASES)
def test_rows_coeff_sweep_parity(name, idx, rows, blocks):
    print(f"rows coefficient sweep {name} rows {rows} blocks {blocks}", flush=True)
    if name == "small_alloy":
        md, m, b, th, s, tg = fixture(SMALL_ALLOY, seed=7, batch=small_alloy_batch())
    else:
        md, m, b, th, s, tg = fixture(name, idx)
    b, th, s, tg = device_inputs("f32", b, th, s, tg)
    base = N.Model.from_dict(md, dtype="f32")
    gb = N.Batch.from_host(b)
    nb = N.nep_build_neighbors(base, gb)
    theta = torch.tensor(th, dtype=torch.float32, device="cuda")
    qs = torch.tensor(s, dtype=torch.float32, device="cuda")
    targets = N.Targets(*tg, lambdas=(1.0, 1.0, 0.1))
    model = base.with_plan(N.Plan(network=3, coeff_grad_rows=rows, coeff_grad_blocks=blocks))
    ws = N.workspace(model, gb, nb)
    loss, g = N.nep_loss_and_grad(model, theta, qs, gb, nb, targets, ws)[:2]
    g1 = g.clone()
    loss2, g2 = N.nep_loss_and_grad(model, theta, qs, gb, nb, targets, ws)[:2]
    # bitwise repeatable: the wavefront's accumulator takes its additions in a fixed order
    assert torch.equal(g1, g2) and torch.equal(loss, loss2)
    lo, go, _, _, _ = O.loss_and_grad(m, th, s, b, *tg, (1.0, 1.0, 0.1), nthreads=8)
    assert rel_err(loss.cpu().numpy(), lo) < 1e-5
    assert rel_err(g.double().cpu().numpy(), go) < 1e-4
    # the angular-coefficient block alone, against the pair-per-lane sweep's
    ref = base.with_plan(N.Plan(network=3))
    gr = N.nep_loss_and_grad(ref, theta, qs, gb, nb, targets, N.workspace(ref, gb, nb))[1]
    P = O.dims(m)[0]
    T, NR, NA, KR, KA = md["num_types"], md["n_max_r"] + 1, md["n_max_a"] + 1, md["basis_r"] + 1, md["basis_a"] + 1
    a0, a1 = T * T * NR * KR, T * T * (NR * KR + NA * KA)
    assert a1 < P
    assert rel_err(g[a0:a1].double().cpu().numpy(), go[a0:a1]) < 1e-4
    assert rel_err(g[a0:a1].double().cpu().numpy(), gr[a0:a1].double().cpu().numpy()) < 1e-4


def test_rows_coeff_sweep_fp64_refused():
    md, m, b, th, s, tg = fixture("bcc64x8")
    model = N.Model.from_dict(md, dtype="f64").with_plan(N.Plan(coeff_grad_rows=2))
    gb = N.Batch.from_host(b, dtype=torch.float64)
    nb = N.nep_build_neighbors(model, gb)
    theta = torch.tensor(th, device="cuda")
    qs = torch.tensor(s, device="cuda")
    with pytest.raises(N.NepError) as e:
        N.nep_loss_and_grad(model, theta, qs, gb, nb, N.Targets(*tg, dtype=torch.float64), N.workspace(model, gb, nb))
    assert e.value.code == -2  # NEP_ERR_UNSUPPORTED
