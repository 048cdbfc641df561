"""Per-workload GPU checks beyond element-wise oracle parity on small subsets:
central finite differences of the GPU loss against the GPU gradient (FP64, 32
seeded parameters, step 1e-6), the plain-PyTorch autograd double-backward
comparator on the same GPU, and full-size batches checked on sampled structures
against the oracle computed one structure at a time."""

import numpy as np
import pytest
import torch

import oracle as O
from helpers import device_inputs, fixture, rel_err
from synth import WORKLOADS, workload_batch
from synth.workloads import draw_theta

pytestmark = pytest.mark.gpu

N = pytest.importorskip("paper_2606_19557_amd")


def _say(msg):
    print(msg, flush=True)


def _gpu(md, b, dtype):
    model = N.Model.from_dict(md, dtype=dtype)
    gb = N.Batch.from_host(b, dtype=model.torch_dtype)
    nb = N.nep_build_neighbors(model, gb)
    ws = N.workspace(model, gb, nb)
    return model, gb, nb, ws


def test_finite_differences_alloy_fp64():
    """dL/dtheta from the hand-written adjoint against central differences of the
    GPU loss, step 1e-6, on 32 parameters drawn with the workload's FD seed."""
    _say("fd alloy4_1024 f64")
    md, m, b, th, s, tg = fixture("alloy4_1024", [4, 0, 1])
    model, gb, nb, ws = _gpu(md, b, "f64")
    targets = N.Targets(*tg, lambdas=(1.0, 1.0, 0.1), dtype=torch.float64)
    theta = torch.tensor(th, device="cuda")
    qs = torch.tensor(s, device="cuda")
    loss, g = N.nep_loss_and_grad(model, theta, qs, gb, nb, targets, ws)
    g = g.cpu().numpy().copy()
    rng = np.random.default_rng(WORKLOADS["alloy4_1024"].seed + 3000)
    P = len(th)
    assert N.nep_param_count(model)[0] == P
    idx = rng.choice(P, size=32, replace=False)
    h = 1e-6
    scale = np.abs(g).max()
    for k in idx:
        tp, tm = theta.clone(), theta.clone()
        tp[k] += h
        tm[k] -= h
        lp = N.nep_loss_and_grad(model, tp, qs, gb, nb, targets, ws)[0][0].item()
        lm = N.nep_loss_and_grad(model, tm, qs, gb, nb, targets, ws)[0][0].item()
        fd = (lp - lm) / (2 * h)
        # FP64 rounding of the loss over 2h gives ~1e-10 absolute noise
        assert abs(fd - g[k]) <= 1e-5 * abs(g[k]) + 1e-8 * scale, (k, fd, g[k])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_autograd_comparator_alloy(dtype):
    """The same loss and gradient through torch autograd double backward on the GPU."""
    from comparator import AutogradNEP, pairs_from_csr

    _say(f"comparator alloy4_1024 {dtype}")
    md, m, b, th, s, tg = fixture("alloy4_1024", [4, 0, 1, 3])
    b, th, s, tg = device_inputs(dtype, b, th, s, tg)
    model, gb, nb, ws = _gpu(md, b, dtype)
    td = model.torch_dtype
    theta = torch.tensor(th, dtype=td, device="cuda")
    qs = torch.tensor(s, dtype=td, device="cuda")
    Et, Ft, Wt = tg
    targets = N.Targets(Et, Ft, Wt, lambdas=(1.0, 1.0, 0.1), dtype=td)
    loss, g = N.nep_loss_and_grad(model, theta, qs, gb, nb, targets, ws)
    pi, pj, pr = pairs_from_csr(nb.row_offset[: b.num_atoms + 1], nb.neighbor_index().to("cuda"),
                                nb.pairs[: nb.num_pairs, :3])
    net = AutogradNEP(md, gb.types, gb.atom_offset, pi, pj, pr.to(td))
    parts, gc = net.loss_and_grad(theta, qs, torch.tensor(Et, dtype=td, device="cuda"), targets.force,
                                  torch.tensor(Wt, dtype=td, device="cuda"), (1.0, 1.0, 0.1))
    tol = 1e-9 if dtype == "f64" else 1e-4
    assert rel_err(gc.double().cpu().numpy(), g.double().cpu().numpy()) < tol
    assert rel_err(parts.double().cpu().numpy(), loss.cpu().numpy()) < tol


@pytest.mark.parametrize("name,sample", [("alloy4_1024", [0, 511, 684, 1023]), ("large5_32", [20, 3])])
def test_full_workload_sampled(name, sample):
    """The whole batch in one call (the launch configuration of a benchmark run);
    energies, forces and virials of sampled structures against the oracle run
    on those structures alone (structures are independent)."""
    _say(f"full {name} sampled {sample}")
    w = WORKLOADS[name]
    md = dict(w.model)
    b = workload_batch(name)
    m = O.Model(**md)
    P, D = O.dims(m)
    th = draw_theta(P, w.seed + 1000)
    b, th, _, _ = device_inputs("f32", b, th, np.ones(D))
    model, gb, nb, ws = _gpu(md, b, "f32")
    theta = torch.tensor(th, dtype=torch.float32, device="cuda")
    q = N.nep_descriptors(model, theta, gb, nb, ws)
    qs = N.nep_descriptor_scale(q)
    E, F, W = N.nep_forward(model, theta, qs, gb, nb, ws)
    s = qs.double().cpu().numpy()
    E, F, W = E.cpu().numpy(), F.double().cpu().numpy(), W.cpu().numpy()
    for st in sample:
        sub = b.subset([st])
        Eo, Fo, Wo = O.forward(m, th, s, sub)
        a0, a1 = int(b.atom_offset[st]), int(b.atom_offset[st + 1])
        assert rel_err(E[st:st + 1], Eo) < 1e-5, st
        assert rel_err(F[a0:a1], Fo) < 1e-4, st
        assert rel_err(W[st], Wo) < 1e-4, st


@pytest.mark.parametrize("name,sample", [("mixed3_4096", [0, 2047, 4095]), ("large5_32", [31])])
def test_full_size_neighbor_lists(name, sample):
    """Full-size neighbour build (many-block scans, species sort and reverse
    search): invariants over every pair, and sampled structures' per-atom
    counts against the oracle's brute-force search."""
    _say(f"neighbors full {name}")
    w = WORKLOADS[name]
    host = workload_batch(name)
    model = N.Model.from_dict(w.model, dtype=w.dtype)
    gb = N.Batch.from_host(host, dtype=model.torch_dtype)
    nb = N.nep_build_neighbors(model, gb)
    torch.cuda.synchronize()
    T, Na, P = w.model["num_types"], host.num_atoms, nb.num_pairs
    row = nb.row_offset.cpu().numpy()
    seg = nb.seg_count.cpu().numpy()
    assert row[0] == 0 and row[-1] == P
    assert np.array_equal(np.diff(row), seg[:, :, 0].sum(axis=1))
    assert nb.num_angular_pairs == int(seg[:, :, 1].sum())
    typ = np.asarray(host.types)
    assert np.array_equal(nb.species_order.cpu().numpy(), np.argsort(typ, kind="stable"))
    want_off = np.concatenate([[0], np.cumsum(np.bincount(typ, minlength=T))])
    assert np.array_equal(nb.species_offset.cpu().numpy(), want_off)
    owner = np.repeat(np.arange(Na), np.diff(row))
    j = nb.neighbor_index().numpy()
    rev = nb.reverse[:P].cpu().numpy().astype(np.int64)
    r = nb.pairs[:P, :3].double().cpu().numpy()
    ok = rev >= 0
    assert ok.mean() > 0.9999  # a pair at the cutoff may lose its partner to rounding
    p = np.nonzero(ok)[0]
    q = rev[p]
    assert np.array_equal(rev[q], p)
    assert np.array_equal(owner[q], j[p]) and np.array_equal(j[q], owner[p])
    assert np.abs(r[q] + r[p]).max() < 1e-4
    for s in sample:
        cell, pos, t = host.structure(s)
        a0 = int(host.atom_offset[s])
        oi, _, _, _ = O.neighbors(cell, pos, w.model["rc_r"])
        assert np.array_equal(np.diff(row)[a0:a0 + len(pos)], np.bincount(oi, minlength=len(pos)))
