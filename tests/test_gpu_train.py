"""Minibatch packing on the device and the training driver: a gathered
minibatch equals the one built from scratch, bit for bit (lists and results);
training lowers the loss, switches stage at the configured epoch, and a run
resumed from a checkpoint continues bit for bit like the uninterrupted run."""

import os
import tempfile

import numpy as np
import pytest
import torch

from helpers import device_inputs, fixture
from synth import workload_batch

pytestmark = pytest.mark.gpu

N = pytest.importorskip("paper_2606_19557_amd")
from paper_2606_19557_amd import train  # noqa: E402


def _say(msg):
    print(msg, flush=True)


def _dataset(name, idx, dtype="f32", runs=True):
    md, m, b, th, s, tg = fixture(name, idx)
    b, th, s, tg = device_inputs(dtype, b, th, s, tg)
    model = N.Model.from_dict(md, dtype=dtype)
    if runs:
        data = train.Dataset(model, b, *tg)
    else:
        # lists without species runs: the gather sorts each minibatch by species
        gb = N.Batch.from_host(b, dtype=model.torch_dtype)
        nb = N.nep_build_neighbors(model, gb)
        data = train.Dataset.from_device(model, gb, nb, N.Targets(*tg, dtype=model.torch_dtype), b.atom_offset)
    td = model.torch_dtype
    return md, model, data, torch.tensor(th, dtype=td, device="cuda"), torch.tensor(s, dtype=td, device="cuda"), b, tg


def test_species_runs_match_species_order():
    """Each structure's run {start, end} in species_order, recomputed on the host."""
    _say("species runs alloy4_1024")
    md, model, data, theta, qs, b, tg = _dataset("alloy4_1024", list(range(12)))
    nb = data.nbr
    assert nb.species_runs is not None
    runs = nb.species_runs.cpu().numpy()
    order = nb.species_order.cpu().numpy()[: b.num_atoms]
    soff = nb.species_offset.cpu().numpy()
    struct = nb.atom_struct.cpu().numpy()
    T = model.num_types
    want = np.zeros((b.num_structures, T, 2), dtype=np.int64)
    for t in range(T):
        for p in range(soff[t], soff[t + 1]):
            s = struct[order[p]]
            if want[s, t, 1] == 0:
                want[s, t, 0] = p
            want[s, t, 1] = p + 1
    assert np.array_equal(runs, want)


def test_gather_more_ids_than_one_scan_chunk():
    """1,100 ids (more than the gather's 1,024-structure scan chunk, with
    repeats): the species order gathered from the dataset's runs equals a
    stable sort of the gathered species, the species offsets their counts, and
    everything equals the minibatch gathered without the runs (sorted)."""
    _say("gather 1100 ids alloy4_1024")
    md, model, data, theta, qs, b, tg = _dataset("alloy4_1024", list(range(10)))
    _, _, data2, _, _, _, _ = _dataset("alloy4_1024", list(range(10)), runs=False)
    pick = np.random.default_rng(7).integers(0, 10, size=1100).tolist()
    gb, gnb, gtg = data.minibatch(pick)
    gb2, gnb2, gtg2 = data2.minibatch(pick)
    types = gb.types.cpu().numpy()
    T = model.num_types
    assert np.array_equal(gnb.species_order.cpu().numpy()[: gb.num_atoms], np.argsort(types, kind="stable"))
    want_off = np.concatenate([[0], np.cumsum(np.bincount(types, minlength=T))])
    assert np.array_equal(gnb.species_offset.cpu().numpy(), want_off)
    assert torch.equal(gb.atom_offset, gb2.atom_offset) and torch.equal(gb.positions, gb2.positions)
    for k in ("row_offset", "seg_count", "atom_struct", "species_order", "species_offset"):
        assert torch.equal(getattr(gnb, k), getattr(gnb2, k)), k
    P = gnb.num_pairs
    assert torch.equal(gnb.pairs[:P], gnb2.pairs[:P]) and torch.equal(gnb.reverse[:P], gnb2.reverse[:P])


@pytest.mark.parametrize("name,dtype,runs", [("fcc_uneven_256", "f32", True), ("alloy4_1024", "f64", True),
                                             ("alloy4_1024", "f32", False)])
def test_gather_equals_direct_build(name, dtype, runs):
    _say(f"gather {name} {dtype} runs={runs}")
    idx = list(range(10))
    md, model, data, theta, qs, b, tg = _dataset(name, idx, dtype, runs)
    pick = [7, 2, 9, 0, 4]
    gb, gnb, gtg = data.minibatch(pick, lambdas=(1.0, 1.0, 0.1))
    sub = b.subset(pick)
    db = N.Batch.from_host(sub, dtype=model.torch_dtype)
    dnb = N.nep_build_neighbors(model, db)
    assert (gnb.num_pairs, gnb.num_angular_pairs) == (dnb.num_pairs, dnb.num_angular_pairs)
    P = dnb.num_pairs
    assert torch.equal(gb.atom_offset, db.atom_offset)
    assert torch.equal(gb.positions, db.positions) and torch.equal(gb.types, db.types)
    assert torch.equal(gb.cells, db.cells)
    for k in ("row_offset", "seg_count", "atom_struct", "species_order", "species_offset"):
        assert torch.equal(getattr(gnb, k), getattr(dnb, k)), k
    assert torch.equal(gnb.pairs[:P], dnb.pairs[:P]) and torch.equal(gnb.reverse[:P], dnb.reverse[:P])
    Et, Ft, Wt = tg
    a0 = np.concatenate([np.arange(b.atom_offset[s], b.atom_offset[s + 1]) for s in pick])
    dtg = N.Targets(Et[pick], Ft[a0], Wt[pick], lambdas=(1.0, 1.0, 0.1), dtype=model.torch_dtype)
    assert torch.equal(gtg.energy, dtg.energy) and torch.equal(gtg.force, dtg.force)
    assert torch.equal(gtg.virial, dtg.virial) and bool(torch.all(gtg.has_virial == 1))
    l1, g1 = N.nep_loss_and_grad(model, theta, qs, gb, gnb, gtg)
    l2, g2 = N.nep_loss_and_grad(model, theta, qs, db, dnb, dtg)
    assert torch.equal(l1, l2) and torch.equal(g1, g2)


def test_training_epochs_stage_switch_and_resume():
    _say("train fcc 24 structures")
    md, model, data, theta, qs, b, tg = _dataset("fcc_uneven_256", list(range(24)))
    cfg = train.TrainConfig(epochs=4, batch_size=8, lr=2e-3, lambdas=(1.0, 1.0, 0.1), start_stage2=2,
                            stage2_lr=1e-3, stage2_lambdas=(10.0, 1.0, 1.0), seed=3)
    tr = train.Trainer(model, theta, qs, cfg, data)
    first = tr.run_epoch(data)
    second = tr.run_epoch(data)
    assert tr.stage == 1 and tr.t == 6 and second[0] < first[0]
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ckpt.pt")
        tr.save(path)
        third = tr.run_epoch(data)
        assert tr.stage == 2 and tr.sched.lr == pytest.approx(1e-3)
        fourth = tr.run_epoch(data)
        tr2 = train.Trainer(model, theta, qs, cfg, data)
        tr2.load(path)
        assert tr2.epoch == 2 and tr2.t == 6
        assert np.array_equal(tr2.run_epoch(data), third)
        assert np.array_equal(tr2.run_epoch(data), fourth)
        assert torch.equal(tr2.theta, tr.theta) and torch.equal(tr2.vmax, tr.vmax)


def test_gather_out_of_range_ids_are_empty_structures():
    """An id outside [0, Ns) selects an empty structure (no atoms, zero targets,
    virial mask 0) and the other structures are packed as usual."""
    _say("gather out-of-range ids")
    md, model, data, theta, qs, b, tg = _dataset("fcc_uneven_256", [0, 1, 2])
    na, npairs, nang = data.sizes([2, 0])
    ids = torch.tensor([2, -5, 0, 99], dtype=torch.int32, device="cuda")
    gb, gnb, gtg = N.nep_gather_batch(model, data.batch, data.nbr, data.targets, ids, na, npairs, nang)
    off = gb.atom_offset.cpu().numpy()
    assert list(np.diff(off)) == [data.atoms[2], 0, data.atoms[0], 0]
    assert gtg.has_virial.cpu().tolist() == [1, 0, 1, 0]
    assert float(gtg.energy[1]) == 0.0 and float(gtg.energy[3]) == 0.0
    direct = N.Batch.from_host(b.subset([2, 0]), dtype=model.torch_dtype)
    dnb = N.nep_build_neighbors(model, direct)
    P = dnb.num_pairs
    assert torch.equal(gnb.pairs[:P], dnb.pairs[:P]) and torch.equal(gnb.reverse[:P], dnb.reverse[:P])
    assert torch.equal(gb.positions, direct.positions)
    # the empty structures take no part in the loss: the gathered batch's loss and
    # gradient equal the oracle's on the two structures alone (and on the
    # gathered batch with its empty entries)
    import oracle as O
    from helpers import rel_err

    m = O.Model(**md)
    sub = b.subset([2, 0])
    a0 = np.concatenate([np.arange(b.atom_offset[s], b.atom_offset[s + 1]) for s in (2, 0)])
    Et, Ft, Wt = tg
    lam = (1.0, 1.0, 0.1)
    gtg.lambdas = lam
    loss, g = N.nep_loss_and_grad(model, theta, qs, gb, gnb, gtg)
    lo, go, *_ = O.loss_and_grad(m, theta.double().cpu().numpy(), qs.double().cpu().numpy(), sub, Et[[2, 0]],
                                 Ft[a0], Wt[[2, 0]], lam)
    assert rel_err(loss.cpu().numpy(), lo) < 1e-5
    assert rel_err(g.double().cpu().numpy(), go) < 1e-4
