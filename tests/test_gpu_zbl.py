"""The ZBL pair term on the GPU against the FP64 oracle: parity of E, F, W in
both precisions, its add-with-scale semantics, NEP + ZBL predictions, and a
training dataset whose targets carry the term."""

import numpy as np
import pytest
import torch

import oracle as O
from oracle import zbl as OZ
from helpers import SMALL_ALLOY, device_inputs, fixture, rel_err, small_alloy_batch

pytestmark = pytest.mark.gpu

N = pytest.importorskip("paper_2606_19557_amd")

ZS = (26, 24, 28)
R_IN, R_OUT = 2.4, 3.0


def _setup(dtype):
    (md, m, b, th, s, tg) = fixture(SMALL_ALLOY, seed=7, batch=small_alloy_batch())
    b, th, s, tg = device_inputs(dtype, b, th, s, tg)
    model = N.Model.from_dict(md, dtype=dtype)
    gb = N.Batch.from_host(b, dtype=model.torch_dtype)
    nb = N.nep_build_neighbors(model, gb)
    return md, m, b, th, s, tg, model, gb, nb


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_zbl_parity(dtype, tol):
    print(f"zbl parity {dtype}", flush=True)
    md, m, b, th, s, tg, model, gb, nb = _setup(dtype)
    td = model.torch_dtype
    Ez, Fz, Wz = OZ.zbl(ZS, R_IN, R_OUT, b)
    assert np.abs(Fz).max() > 1.0  # pairs inside the switch and across it
    E = torch.zeros(gb.num_structures, dtype=torch.float64, device="cuda")
    F = torch.zeros((gb.num_atoms, 3), dtype=td, device="cuda")
    W = torch.zeros((gb.num_structures, 9), dtype=torch.float64, device="cuda")
    N.nep_zbl_add(model, N.Zbl(ZS, R_IN, R_OUT), gb, nb, E, F, W)
    assert rel_err(E.cpu().numpy(), Ez) < tol
    assert rel_err(F.double().cpu().numpy(), Fz) < 10 * tol
    assert rel_err(W.cpu().numpy(), Wz.reshape(-1, 9)) < 10 * tol
    # add-with-scale onto existing values; NULL outputs are skipped
    E0 = torch.randn(gb.num_structures, dtype=torch.float64, device="cuda")
    F0 = torch.randn((gb.num_atoms, 3), dtype=td, device="cuda")
    E1, F1 = E0.clone(), F0.clone()
    N.nep_zbl_add(model, N.Zbl(ZS, R_IN, R_OUT), gb, nb, E1, F1, None, scale=-0.5)
    # the results against the starting values plus the scaled oracle term (no
    # difference of the outputs, whose cancellation would loosen the check)
    assert rel_err(E1.cpu().numpy(), E0.cpu().numpy() - 0.5 * Ez) < tol
    assert rel_err(F1.double().cpu().numpy(), F0.double().cpu().numpy() - 0.5 * Fz) < 10 * tol
    # and the added part alone, to the tolerance of the plain call
    assert rel_err((E1 - E0).cpu().numpy(), -0.5 * Ez) < tol


def test_zbl_outside_switch_is_zero_and_forward_sum():
    print("zbl forward f64", flush=True)
    md, m, b, th, s, tg, model, gb, nb = _setup("f64")
    z = N.Zbl(ZS, 0.5, 1.0)  # no pair closer than 1 A
    E = torch.zeros(gb.num_structures, dtype=torch.float64, device="cuda")
    F = torch.zeros((gb.num_atoms, 3), dtype=torch.float64, device="cuda")
    W = torch.zeros((gb.num_structures, 9), dtype=torch.float64, device="cuda")
    N.nep_zbl_add(model, z, gb, nb, E, F, W)
    assert E.abs().max().item() == 0.0 and F.abs().max().item() == 0.0 and W.abs().max().item() == 0.0
    # NEP + ZBL predictions
    theta = torch.tensor(th, dtype=torch.float64, device="cuda")
    qs = torch.tensor(s, dtype=torch.float64, device="cuda")
    E, F, W = N.nep_forward(model, theta, qs, gb, nb, zbl=N.Zbl(ZS, R_IN, R_OUT))
    Eo, Fo, Wo = O.forward(m, th, s, b)
    Ez, Fz, Wz = OZ.zbl(ZS, R_IN, R_OUT, b)
    assert rel_err(E.cpu().numpy(), Eo + Ez) < 1e-9
    assert rel_err(F.cpu().numpy(), Fo + Fz) < 1e-9
    assert rel_err(W.cpu().numpy(), Wo + Wz) < 1e-9


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_dataset_with_zbl_trains_nep_plus_zbl(dtype):
    """A dataset built with the ZBL term gives the loss and gradient of NEP + ZBL
    against the raw targets (the oracle computes that loss with the term moved to
    its targets, which its own pins show to be the same loss)."""
    print(f"zbl dataset {dtype}", flush=True)
    from paper_2606_19557_amd.train import Dataset

    md, m, b, th, s, tg, model, gb, nb = _setup(dtype)
    Et, Ft, Wt = tg
    rng = np.random.default_rng(3)
    Et = Et + rng.normal(0.0, 1.0, Et.shape)  # targets away from the teacher
    data = Dataset(model, b, Et, Ft, Wt, zbl=N.Zbl(ZS, R_IN, R_OUT))
    td = model.torch_dtype
    theta = torch.tensor(th, dtype=td, device="cuda")
    qs = torch.tensor(s, dtype=td, device="cuda")
    loss, g = N.nep_loss_and_grad(model, theta, qs, data.batch, data.nbr, data.targets)
    Ez, Fz, Wz = OZ.zbl(ZS, R_IN, R_OUT, b)
    lo, go, _, _, _ = O.loss_and_grad(m, th, s, b, Et - Ez, Ft - Fz, Wt - Wz, nthreads=8)
    tl, tg_ = (1e-9, 1e-9) if dtype == "f64" else (1e-5, 1e-4)
    assert rel_err(loss.cpu().numpy(), lo) < tl
    assert rel_err(g.double().cpu().numpy(), go) < tg_


def test_zbl_self_images_and_empty_batch():
    """A one-atom cell whose only ZBL partners are its own periodic images, a
    two-atom cell and a bcc cell, FP64 against the oracle; an empty batch is a
    no-op."""
    print("zbl edge cases", flush=True)
    from synth import structures as S

    rng = np.random.default_rng(17)
    structs = [
        (np.diag([2.3, 2.6, 3.3]), np.array([[0.2, 0.1, 0.3]]), np.array([0], np.int32)),
        (np.diag([2.9, 4.0, 3.2]), np.array([[0.1, 0.2, 0.3], [1.2, 1.4, 1.1]]), np.array([0, 0], np.int32)),
        S.bcc_structure(rng, 15, a=3.2, sigma=0.15, exact_dims=(2, 2, 2)),
    ]
    b = S.pack(structs, 1)
    md = dict(num_types=1, rc_r=5.0, rc_a=4.0, n_max_r=4, n_max_a=4, basis_r=8, basis_a=8, l_max=4, l_max_4b=0,
              l_max_5b=0, hidden=30)
    model = N.Model.from_dict(md, dtype="f64")
    gb = N.Batch.from_host(b, dtype=torch.float64)
    nb = N.nep_build_neighbors(model, gb)
    z = N.Zbl((26,), 2.0, 3.0)
    E = torch.zeros(3, dtype=torch.float64, device="cuda")
    F = torch.zeros((b.num_atoms, 3), dtype=torch.float64, device="cuda")
    W = torch.zeros((3, 9), dtype=torch.float64, device="cuda")
    N.nep_zbl_add(model, z, gb, nb, E, F, W)
    Ez, Fz, Wz = OZ.zbl((26,), 2.0, 3.0, b)
    assert Ez[0] > 0 and np.abs(Fz[0]).max() < 1e-9 * Ez[0]  # a lone atom's images pull evenly
    assert rel_err(E.cpu().numpy(), Ez) < 1e-10
    assert np.abs(F.cpu().numpy() - Fz).max() < 1e-9 * max(1.0, np.abs(Fz).max())
    assert rel_err(W.cpu().numpy(), Wz) < 1e-9
    empty = N.Batch(np.zeros((0, 3)), np.zeros(0, np.int32), np.zeros((0, 3, 3)), np.zeros(1, np.int64),
                    dtype=torch.float64)
    enb = N.nep_build_neighbors(model, empty)
    N.nep_zbl_add(model, z, empty, enb, None, None, None)
    torch.cuda.synchronize()
