"""NEP input files and model files.

Input file: the model keys of the paper's input file (Table I, "Example
TorchNEP input file") -- ``type``, ``version``, ``cutoff``, ``n_max``,
``basis_size``, ``l_max``, ``neuron`` -- and its Stage I / Stage II training
keys, one ``key value...`` line each; ``#`` starts a comment. ``l_max``
takes one to three numbers: the three-body l_max, then 2 to switch the
4-body term on and 1 for the 5-body term (Methods, "NEP descriptors").

Model file (this library's own text format, written and read here): the same
model keys, ``dtype``, then the parameter vector theta in the order of the C
ABI (c_R[a][b][n][k], c_A[a][b][n][k], for each species W0, b0, w1, then b1)
and the frozen descriptor scaler of Eq. 2, one value per line. Values are
written as the shortest decimal that reads back to the same float32 or
float64, so a save/load round trip is bitwise. Compatibility with model
files of other NEP programs is not claimed: their format is not given by
the paper.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MODEL_KEYS = ("type", "version", "cutoff", "n_max", "basis_size", "l_max", "neuron")
# Stage I / Stage II keys of the input file and the type of their values
TRAIN_KEYS = {
    "epoch": int, "lr": float, "lambda_e": float, "lambda_f": float, "lambda_v": float, "batch": int,
    "scheduler_patience": int, "scheduler_factor": float, "stage2": int, "start_stage2": int,
    "stage2_lr": float, "stage2_lambda_e": float, "stage2_lambda_f": float, "stage2_lambda_v": float,
}
MAGIC = "nep_model_file 1"


@dataclass
class NepInput:
    """A parsed input file: the model hyper-parameters (the dict taken by
    ``Model.from_dict``), the species names, optional ZBL switch radii and the
    training keys present in the file."""

    model: dict
    species: list
    train: dict = field(default_factory=dict)
    zbl: tuple | None = None


def _model_lines(model: dict, species) -> list:
    l4 = 2 if model.get("l_max_4b", 0) == 2 else 0
    l5 = 1 if model.get("l_max_5b", 0) == 1 else 0
    return [
        f"type {len(species)} {' '.join(species)}",
        "version 4",
        f"cutoff {model['rc_r']!r} {model['rc_a']!r}",
        f"n_max {model['n_max_r']} {model['n_max_a']}",
        f"basis_size {model['basis_r']} {model['basis_a']}",
        f"l_max {model['l_max']} {l4} {l5}",
        f"neuron {model['hidden']}",
    ]


def _parse_model_key(key: str, vals: list, model: dict, out: dict):
    if key == "type":
        n = int(vals[0])
        names = vals[1:]
        if n < 1 or len(names) != n:
            raise ValueError(f"type: {n} species but {len(names)} names")
        out["species"] = names
        model["num_types"] = n
    elif key == "version":
        if int(vals[0]) != 4:
            raise ValueError(f"version {vals[0]}: only NEP version 4 is supported")
    elif key == "cutoff":
        model["rc_r"], model["rc_a"] = float(vals[0]), float(vals[1])
        if not 0.0 < model["rc_a"] <= model["rc_r"]:
            raise ValueError("cutoff: need 0 < angular <= radial")
    elif key == "n_max":
        model["n_max_r"], model["n_max_a"] = int(vals[0]), int(vals[1])
    elif key == "basis_size":
        model["basis_r"], model["basis_a"] = int(vals[0]), int(vals[1])
    elif key == "l_max":
        l3 = int(vals[0])
        l4 = int(vals[1]) if len(vals) > 1 else 0
        l5 = int(vals[2]) if len(vals) > 2 else 0
        if l4 not in (0, 2) or l5 not in (0, 1):
            raise ValueError(f"l_max {' '.join(vals)}: the 4-body entry must be 0 or 2, the 5-body 0 or 1")
        model["l_max"], model["l_max_4b"], model["l_max_5b"] = l3, l4, l5
    elif key == "neuron":
        model["hidden"] = int(vals[0])


def _tokens(text: str):
    for raw in text.splitlines():
        line = raw.split("#", 1)[0].strip()
        if line:
            parts = line.split()
            yield parts[0], parts[1:]


def parse_input(text: str) -> NepInput:
    """Parse an input file's text (model keys required, training keys optional)."""
    model, meta, train, zbl = {}, {}, {}, None
    for key, vals in _tokens(text):
        if key in MODEL_KEYS:
            _parse_model_key(key, vals, model, meta)
        elif key in TRAIN_KEYS:
            train[key] = TRAIN_KEYS[key](vals[0])
        elif key == "zbl":
            zbl = (float(vals[0]), float(vals[1]))
        else:
            raise ValueError(f"unknown key {key!r}")
    missing = [k for k in MODEL_KEYS if k != "version" and not _has(k, model, meta)]
    if missing:
        raise ValueError(f"input file lacks {', '.join(missing)}")
    return NepInput(model=model, species=meta["species"], train=train, zbl=zbl)


def _has(key, model, meta):
    return {"type": "species" in meta, "cutoff": "rc_r" in model, "n_max": "n_max_r" in model,
            "basis_size": "basis_r" in model, "l_max": "l_max" in model, "neuron": "hidden" in model}[key]


def num_params(model: dict) -> tuple[int, int]:
    """(P, D) of a model: the parameter count and descriptor length of the C ABI's layout."""
    T = model["num_types"]
    NR, NA = model["n_max_r"] + 1, model["n_max_a"] + 1
    KR, KA = model["basis_r"] + 1, model["basis_a"] + 1
    L = model["l_max"] + (model.get("l_max_4b", 0) == 2) + (model.get("l_max_5b", 0) == 1)
    D = NR + NA * L
    H = model["hidden"]
    return T * T * (NR * KR + NA * KA) + T * (D + 2) * H + 1, D


def _fmt(x, dtype) -> str:
    return np.format_float_scientific(dtype(x), unique=True)


def save_model(path: str, model: dict, species, theta, q_scale, dtype: str = "f32", zbl=None):
    """Write a model file: the model keys, dtype ("f32" or "f64"), theta [P] and the scaler [D]."""
    P, D = num_params(model)
    if len(species) != model["num_types"]:
        raise ValueError("one species name per type")
    if dtype not in ("f32", "f64"):
        raise ValueError("dtype is f32 or f64")
    npt = np.float32 if dtype == "f32" else np.float64
    th = np.asarray(theta).ravel()
    qs = np.asarray(q_scale).ravel()
    if th.size != P or qs.size != D:
        raise ValueError(f"theta has {th.size} values and the scaler {qs.size}; the model needs {P} and {D}")
    lines = [MAGIC, *_model_lines(model, list(species)), f"dtype {dtype}"]
    if zbl is not None:
        lines.append(f"zbl {float(zbl[0])!r} {float(zbl[1])!r}")
    lines.append(f"theta {P}")
    lines += [_fmt(x, npt) for x in th]
    lines.append(f"q_scale {D}")
    lines += [_fmt(x, npt) for x in qs]
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def load_model(path: str):
    """Read a model file: (NepInput with the model keys, dtype, theta, q_scale) with
    theta and q_scale as numpy arrays of the file's dtype."""
    with open(path) as f:
        lines = f.read().splitlines()
    if not lines or lines[0].strip() != MAGIC:
        raise ValueError(f"{path}: not a model file of this library")
    k = 1
    head = []
    while k < len(lines) and not lines[k].startswith("theta "):
        head.append(lines[k])
        k += 1
    dtype, body = "f32", []
    for ln in head:
        if ln.startswith("dtype "):
            dtype = ln.split()[1]
        else:
            body.append(ln)
    inp = parse_input("\n".join(body))
    npt = np.float32 if dtype == "f32" else np.float64
    P, D = num_params(inp.model)
    n = int(lines[k].split()[1])
    if n != P:
        raise ValueError(f"{path}: {n} parameters, the model keys give {P}")
    theta = np.array([npt(s) for s in lines[k + 1:k + 1 + P]], dtype=npt)
    k += 1 + P
    m = int(lines[k].split()[1])
    if m != D or not lines[k].startswith("q_scale "):
        raise ValueError(f"{path}: scaler of {m} values, the model keys give {D}")
    q_scale = np.array([npt(s) for s in lines[k + 1:k + 1 + D]], dtype=npt)
    if theta.size != P or q_scale.size != D:
        raise ValueError(f"{path}: truncated")
    return inp, dtype, theta, q_scale
