"""Input-file parsing and the model file (save / load) on the host.

Pins: the paper's example input file (Table I) parses to its printed model
and training values; the parameter count from the model keys equals Table II's
printed counts and the oracle's own count; a save/load round trip returns
theta and the scaler bit for bit in FP32 and FP64, so the oracle's energies,
forces and virials from a reloaded model are identical. Compatibility with the
model files of other NEP programs is parity unpinned (no such file or format
is in the paper)."""

import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2606_19557_amd import model_io as io
from synth.workloads import draw_theta

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _text(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return f.read()


def test_table1_input_parses_to_printed_values():
    inp = io.parse_input(_text("table1_input.txt"))
    assert inp.species == ["C"]
    assert inp.model == dict(num_types=1, rc_r=4.2, rc_a=3.7, n_max_r=10, n_max_a=8, basis_r=10, basis_a=8,
                             l_max=4, l_max_4b=2, l_max_5b=1, hidden=100)
    t1 = json.loads(_text("table1_training.json"))
    for k, v in {**t1["stage1"], **t1["stage2"]}.items():
        assert inp.train[k] == v, k
    assert inp.train["stage2"] == 1


def test_param_count_matches_table2_and_oracle():
    t2 = json.loads(_text("table2_param_counts.json"))
    for case in t2["cases"]:
        md = dict(num_types=t2["num_types"], rc_r=6.0, rc_a=4.0, n_max_r=case["n_max"][0], n_max_a=case["n_max"][1],
                  basis_r=t2["basis"][0], basis_a=t2["basis"][1], l_max=t2["l_max"][0], l_max_4b=t2["l_max"][1],
                  l_max_5b=t2["l_max"][2], hidden=t2["hidden"])
        assert io.num_params(md)[0] == case["params"], case["label"]
        assert io.num_params(md) == O.dims(O.Model(**md))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_round_trip_bitwise(tmp_path, dtype):
    inp = io.parse_input(_text("table1_input.txt"))
    md = dict(inp.model, num_types=3)
    P, D = io.num_params(md)
    npt = np.float32 if dtype == "f32" else np.float64
    theta = draw_theta(P, 7).astype(npt)
    # values that a decimal format most easily gets wrong
    special = np.array([0.0, -0.0, 1.0 / 3.0, -2.0 ** -126, 2.0 ** -149 if dtype == "f32" else 5e-324,
                        np.finfo(npt).max, np.finfo(npt).tiny, 1e-7, 123456789.0], dtype=npt)
    theta[:special.size] = special
    qs = np.abs(draw_theta(D, 8)).astype(npt) + npt(0.5)
    path = str(tmp_path / "model.txt")
    io.save_model(path, md, ["Al", "Cu", "Ni"], theta, qs, dtype=dtype, zbl=(1.0, 2.0))
    got, gd, th2, qs2 = io.load_model(path)
    assert gd == dtype and got.species == ["Al", "Cu", "Ni"] and got.zbl == (1.0, 2.0)
    assert got.model == md
    assert th2.dtype == npt and qs2.dtype == npt
    assert th2.tobytes() == theta.tobytes()
    assert qs2.tobytes() == qs.tobytes()


def test_reloaded_model_gives_identical_oracle_predictions(tmp_path):
    from helpers import SMALL_ALLOY, small_alloy_batch

    md = dict(SMALL_ALLOY)
    m = O.Model(**md)
    P, D = O.dims(m)
    b = small_alloy_batch(n_struct=2)
    theta = draw_theta(P, 11)
    s = O.scaler(O.descriptors(m, theta, b))
    path = str(tmp_path / "m.txt")
    io.save_model(path, md, ["A", "B", "C"], theta, s, dtype="f64")
    inp, _, th2, s2 = io.load_model(path)
    E, F, W = O.forward(O.Model(**inp.model), th2, s2, b)
    E0, F0, W0 = O.forward(m, theta, s, b)
    assert np.array_equal(E, E0) and np.array_equal(F, F0) and np.array_equal(W, W0)


@pytest.mark.parametrize("bad", ["version 3", "l_max 4 1 1", "l_max 4 2 2", "cutoff 4 5", "frobnicate 1",
                                 "type 2 C"])
def test_invalid_input_rejected(bad):
    text = _text("table1_input.txt")
    key = bad.split()[0]
    lines = [ln for ln in text.splitlines() if not ln.startswith(key + " ")]
    with pytest.raises(ValueError):
        io.parse_input("\n".join(lines + [bad]))


def test_missing_key_and_size_mismatch_rejected(tmp_path):
    text = "\n".join(ln for ln in _text("table1_input.txt").splitlines() if not ln.startswith("neuron"))
    with pytest.raises(ValueError):
        io.parse_input(text)
    md = io.parse_input(_text("table1_input.txt")).model
    P, D = io.num_params(md)
    with pytest.raises(ValueError):
        io.save_model(str(tmp_path / "x.txt"), md, ["C"], np.zeros(P - 1), np.ones(D))


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_reloaded_model_gives_identical_gpu_predictions(tmp_path, dtype):
    """Save, load, and evaluate on the GPU: E, F, W bitwise those of the
    parameters before saving (the round trip is exact, so the kernels see the
    same bits)."""
    import torch

    import paper_2606_19557_amd as N
    from helpers import SMALL_ALLOY, device_inputs, small_alloy_batch

    md = dict(SMALL_ALLOY)
    m = O.Model(**md)
    P, D = O.dims(m)
    b = small_alloy_batch(n_struct=3)
    theta = draw_theta(P, 13)
    s = O.scaler(O.descriptors(m, theta, b))
    b, theta, s, _ = device_inputs(dtype, b, theta, s)
    npt = np.float32 if dtype == "f32" else np.float64
    path = str(tmp_path / "m.txt")
    io.save_model(path, md, ["A", "B", "C"], theta.astype(npt), s.astype(npt), dtype=dtype)
    inp, gd, th2, s2 = io.load_model(path)
    assert gd == dtype
    model = N.Model.from_dict(md, dtype=dtype)
    td = model.torch_dtype
    gb = N.Batch.from_host(b, dtype=td)
    nb = N.nep_build_neighbors(model, gb)
    ws = N.workspace(model, gb, nb)
    outs = []
    for th, qs in ((theta, s), (th2, s2)):
        E, F, W = N.nep_forward(N.Model.from_dict(inp.model if th is th2 else md, dtype=dtype),
                                torch.tensor(np.asarray(th, dtype=npt), device="cuda"),
                                torch.tensor(np.asarray(qs, dtype=npt), device="cuda"), gb, nb, ws)
        outs.append((E.cpu(), F.cpu(), W.cpu()))
    for a, c in zip(*outs):
        assert torch.equal(a, c)
