"""Sixteen species on the GPU: the Table II NEP44 model shape (16 elements,
n_max 4/4, basis 8/8, l_max 4 2 1, 80 hidden neurons) on a small seeded batch
of uneven fcc and bcc cells with every species present. This runs the
neighbour build compiled for up to 16 species and the coefficient-gradient
layout of T^2 = 256 species pairs, against the FP64 oracle (FP64: 1e-9; FP32:
energies 1e-5, forces, virials and gradients 1e-4)."""

from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle as O
from helpers import device_inputs, fixture, rel_err
from synth import structures as S

pytestmark = pytest.mark.gpu

N = pytest.importorskip("paper_2606_19557_amd")

NEP44 = dict(num_types=16, rc_r=6.0, rc_a=4.0, n_max_r=4, n_max_a=4, basis_r=8, basis_a=8, l_max=4, l_max_4b=2,
             l_max_5b=1, hidden=80)


def _batch(seed=16):
    rng = np.random.default_rng(seed)
    structs = []
    for k, n in enumerate((40, 29, 36, 24, 31, 18)):
        if k % 3 == 2:
            structs.append(S.bcc_structure(rng, n, a=3.2, sigma=0.15, strain=0.02, num_types=16))
        else:
            structs.append(S.fcc_structure(rng, n, a=4.0, sigma=0.2, strain=0.02, num_types=16))
    b = S.pack(structs, 16)
    # every species present at least once: relabel the first 16 atoms
    types = b.types.copy()
    types[:16] = np.arange(16, dtype=types.dtype)
    return replace(b, types=types)


def test_nep44_param_count_is_table2():
    P, D = O.dims(O.Model(**NEP44))
    assert P == 70401 and D == 35


# f32-force4: the force sweep with 4-lane teams, 64 atoms per block, whose
# per-team radial coefficients and segment tables for 16 species take more
# than 64 KB of LDS beside the static B blocks
@pytest.mark.parametrize("dtype,plan", [("f64", None), ("f32", None), ("f32", N.Plan(network=3, coeff_grad_rows=2)),
                                        ("f32", N.Plan(4, 16, 8, 32, 7, 16, 1)),
                                        ("f32", N.Plan(team_force=4, network=2))],
                         ids=["f64", "f32", "f32-rows2", "f32-teams", "f32-force4"])
def test_sixteen_species_parity(dtype, plan):
    print(f"16 species {dtype} {plan}", flush=True)
    md, m, b, th, s, tg = fixture(NEP44, seed=44, batch=_batch())
    assert len(np.unique(b.types)) == 16
    b, th, s, tg = device_inputs(dtype, b, th, s, tg)
    model = N.Model.from_dict(md, dtype=dtype).with_plan(plan)
    td = model.torch_dtype
    gb = N.Batch.from_host(b, dtype=td)
    nb = N.nep_build_neighbors(model, gb)
    # neighbour lists: per-species counts and the multiset of neighbours of
    # every row equal those of the brute-force search (index work: exact)
    torch.cuda.synchronize()
    row = nb.row_offset.cpu().numpy()
    seg = nb.seg_count.cpu().numpy()
    js = nb.neighbor_index().numpy()
    total = 0
    for st in range(b.num_structures):
        cell, pos, typ = b.structure(st)
        a0 = int(b.atom_offset[st])
        oi, oj, osh, orr = O.neighbors(cell, pos, md["rc_r"])
        total += len(oi)
        for i in range(len(pos)):
            sel = oi == i
            d = np.linalg.norm(orr[sel], axis=1)
            for t in range(16):
                mask = typ[oj[sel]] == t
                assert seg[a0 + i, t, 0] == mask.sum()
                assert seg[a0 + i, t, 1] == (d[mask] < md["rc_a"]).sum()
            assert sorted((js[row[a0 + i]:row[a0 + i + 1]] - a0).tolist()) == sorted(oj[sel].tolist())
    assert nb.num_pairs == total
    ws = N.workspace(model, gb, nb)
    theta = torch.tensor(th, dtype=td, device="cuda")
    qs = torch.tensor(s, dtype=td, device="cuda")
    targets = N.Targets(*tg, lambdas=(1.0, 1.0, 0.1), dtype=td)
    loss, g, E, F, W = N.nep_loss_and_grad(model, theta, qs, gb, nb, targets, ws, want_predictions=True)
    lo, go, Eo, Fo, Wo = O.loss_and_grad(m, th, s, b, *tg, (1.0, 1.0, 0.1), nthreads=8)
    tol = dict(E=1e-9, F=1e-9, G=1e-9, L=1e-9) if dtype == "f64" else dict(E=1e-5, F=1e-4, G=1e-4, L=1e-5)
    assert rel_err(E.cpu().numpy(), Eo) < tol["E"]
    assert rel_err(F.double().cpu().numpy(), Fo) < tol["F"]
    assert rel_err(W.cpu().numpy(), Wo) < tol["F"]
    assert rel_err(loss.cpu().numpy(), lo) < tol["L"]
    assert rel_err(g.double().cpu().numpy(), go) < tol["G"]
    # every one of the 256 angular coefficient blocks took part
    T, NR, KR, NA, KA = 16, 5, 9, 5, 9
    cA = np.asarray(go[T * T * NR * KR:T * T * (NR * KR + NA * KA)]).reshape(T, T, NA * KA)
    assert (np.abs(cA).sum(axis=2) > 0).sum() >= 200
    E2, F2, W2 = N.nep_forward(model, theta, qs, gb, nb, ws)
    assert rel_err(E2.cpu().numpy(), Eo) < tol["E"]
    assert rel_err(F2.double().cpu().numpy(), Fo) < tol["F"]
