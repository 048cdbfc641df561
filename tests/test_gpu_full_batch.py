"""Whole benchmark batches against the oracle: the loss, its gradient with
respect to every parameter, every structure's energy and virial, and forces on
4096 evenly spaced atoms, for the 1024-structure 4-species alloy (4-body and
5-body terms) and the 32 large cells (5 species, ~100 neighbours per atom),
in the launch configuration a benchmark run uses (the shipped autotuned plan,
one call over the whole batch). The oracle's values were written by
``tests/golden/make_full_batch.py`` from the same seeded, float32-rounded
inputs (Eqs. 4-7 for the loss, and the gradient that the analytic adjoint
must equal)."""

import os
import sys

import numpy as np
import pytest
import torch

from helpers import rel_err, rel_err_plain

pytestmark = pytest.mark.gpu

N = pytest.importorskip("paper_2606_19557_amd")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLDEN)


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("name", ["alloy4_1024", "large5_32"])
def test_full_batch_loss_grad(name):
    from make_full_batch import input_digest, rounded_inputs

    from paper_2606_19557_amd import tuning

    _say(f"full batch {name}: loss, gradient, E, W, sampled F against the oracle")
    ref = np.load(os.path.join(GOLDEN, f"full_{name}.npz"))
    w, m, b, theta, tg = rounded_inputs(name)
    assert str(ref["digest"]) == input_digest(b, theta, tg), "regenerated inputs differ from the golden's"
    model = N.Model.from_dict(w.model, dtype="f32")
    gb = N.Batch.from_host(b, dtype=torch.float32)
    nb = N.nep_build_neighbors(model, gb)
    key = tuning.plan_key(model, b.num_atoms, nb.num_pairs)
    plan = tuning._entry(tuning.load(tuning.SHIPPED_PLANS), key)
    assert plan is not None, f"no shipped plan for {key}"
    model = model.with_plan(plan)
    _say(f"  plan {plan.as_dict()}")
    ws = N.workspace(model, gb, nb)
    th = torch.tensor(theta, dtype=torch.float32, device="cuda")
    qs = torch.tensor(ref["qscale"], dtype=torch.float32, device="cuda")
    targets = N.Targets(*tg, lambdas=w.lambdas, dtype=torch.float32)
    loss, g, E, F, W = N.nep_loss_and_grad(model, th, qs, gb, nb, targets, ws, want_predictions=True)
    torch.cuda.synchronize()
    loss, g = loss.cpu().numpy(), g.double().cpu().numpy()
    E, W = E.cpu().numpy(), W.cpu().numpy()
    F = F.double().cpu().numpy()[ref["f_idx"]]
    errs = {"loss": rel_err(loss, ref["loss"]), "E": rel_err(E, ref["E"]), "W": rel_err(W, ref["W"]),
            "F": rel_err(F, ref["F"]), "grad": rel_err(g, ref["grad"])}
    plain = rel_err_plain(g, ref["grad"], 1e-2)
    _say(f"  errors {errs}; gradient entries above 1% of the largest: max plain relative error {plain:.2e}")
    assert errs["loss"] < 1e-5 and errs["E"] < 1e-5
    assert errs["W"] < 1e-4 and errs["F"] < 1e-4 and errs["grad"] < 1e-4
    assert plain < 1e-4
