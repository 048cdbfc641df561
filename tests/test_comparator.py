"""The plain-PyTorch autograd (double backward) implementation against the
oracle on the CPU in FP64: an independent second route to E, F, W, the loss
and its parameter gradient."""

import numpy as np
import pytest
import torch

import oracle as O
from comparator import AutogradNEP
from helpers import SMALL_ALLOY, fixture, rel_err, small_alloy_batch


def _pairs(m, b):
    I, J, R = [], [], []
    for s in range(b.num_structures):
        cell, pos, typ = b.structure(s)
        a0 = int(b.atom_offset[s])
        i, j, sh, r = O.neighbors(cell, pos, m.rc_r)
        I.append(i + a0)
        J.append(j + a0)
        R.append(r)
    return (torch.tensor(np.concatenate(I)), torch.tensor(np.concatenate(J)),
            torch.tensor(np.concatenate(R), dtype=torch.float64))


@pytest.mark.parametrize("case", ["bcc", "alloy"])
def test_autograd_matches_oracle(case):
    if case == "bcc":
        md, m, b, th, s, tg = fixture("bcc64x8", [0, 1, 2])
    else:
        md, m, b, th, s, tg = fixture(SMALL_ALLOY, seed=7, batch=small_alloy_batch())
    pi, pj, pr = _pairs(m, b)
    net = AutogradNEP(md, torch.tensor(b.types), torch.tensor(b.atom_offset), pi, pj, pr)
    theta = torch.tensor(th)
    qs = torch.tensor(s)
    E, F, W = net.energy_forces_virial(theta, qs)
    Eo, Fo, Wo = O.forward(m, th, s, b)
    assert rel_err(E.numpy(), Eo) < 1e-12
    assert rel_err(F.numpy(), Fo) < 1e-11
    assert rel_err(W.numpy(), Wo) < 1e-11
    Et, Ft, Wt = tg
    hv = np.ones(b.num_structures, np.uint8)
    hv[0] = 0
    parts, g = net.loss_and_grad(theta, qs, torch.tensor(Et), torch.tensor(Ft), torch.tensor(Wt), (1.0, 1.0, 0.1),
                                 torch.tensor(hv))
    lo, go, *_ = O.loss_and_grad(m, th, s, b, Et, Ft, Wt, (1.0, 1.0, 0.1), has_virial=hv)
    assert rel_err(parts.numpy(), lo) < 1e-12
    assert rel_err(g.numpy(), go) < 1e-10
