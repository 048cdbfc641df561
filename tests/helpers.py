"""Shared test utilities: tolerance semantics, seeded fixtures, oracle targets."""

from __future__ import annotations

from dataclasses import replace

import numpy as np

import oracle as O
from synth import workload_batch, WORKLOADS
from synth.workloads import draw_theta

# Small 3-species model with 4-body and 5-body terms (a compiled kernel shape).
SMALL_ALLOY = dict(num_types=3, rc_r=4.5, rc_a=3.8, n_max_r=3, n_max_a=3, basis_r=5, basis_a=4, l_max=4,
                   l_max_4b=2, l_max_5b=1, hidden=7)


def rel_err(x, ref):
    """max_i |x_i - ref_i| / max(|ref_i|, rms(ref)): relative error with an rms floor so
    components near zero are judged against the array's typical size."""
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    if ref.size == 0:
        return 0.0
    rms = np.sqrt(np.mean(ref * ref))
    den = np.maximum(np.abs(ref), rms)
    den = np.where(den == 0.0, 1.0, den)
    return float(np.max(np.abs(x - ref) / den))


def oracle_model(model_dict):
    return O.Model(**model_dict)


def fixture(name_or_model, indices=None, seed=0, batch=None, T=None):
    """(oracle model, host batch, theta, q_scale, targets E/F/W) for a workload or model dict."""
    if isinstance(name_or_model, str):
        w = WORKLOADS[name_or_model]
        md = dict(w.model)
        batch = workload_batch(name_or_model, indices) if batch is None else batch
        base = w.seed
    else:
        md = dict(name_or_model)
        base = seed
    m = oracle_model(md)
    P, D = O.dims(m)
    theta = draw_theta(P, base + 1000)
    q = O.descriptors(m, theta, batch)
    s = O.scaler(q)
    teacher = draw_theta(P, base + 2000)
    Et, Ft, Wt = O.forward(m, teacher, s, batch)
    return md, m, batch, theta, s, (Et, Ft, Wt)


def device_inputs(dtype, batch, theta, scale, targets=None):
    """The inputs exactly as a device run in `dtype` receives them. For FP32 the
    positions, parameters, scaler and force targets are rounded to float32 (cells,
    energies and virials stay FP64, as in the C ABI), so the oracle and the HIP path
    are compared on bit-identical inputs and the tolerance measures arithmetic only."""
    if dtype != "f32":
        return batch, theta, scale, targets
    r = lambda x: np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)
    b = replace(batch, positions=r(batch.positions))
    tg = None if targets is None else (targets[0], r(targets[1]), targets[2])
    return b, r(theta), r(scale), tg


def small_alloy_batch(seed=5, n_struct=5):
    """Uneven 3-species bcc/fcc cells (some thinner than twice the cutoff)."""
    from synth import structures as S

    rng = np.random.default_rng(seed)
    structs = []
    for k in range(n_struct):
        if k % 2 == 0:
            dims = [(1, 1, 2), (2, 2, 1), (2, 1, 2)][k % 3]
            structs.append(S.bcc_structure(rng, 2 * int(np.prod(dims)) - (k % 3), a=3.2, sigma=0.15, strain=0.02,
                                           num_types=3, exact_dims=dims))
        else:
            structs.append(S.fcc_structure(rng, 10 + 3 * k, a=4.0, sigma=0.2, strain=0.02, num_types=3))
    return S.pack(structs, 3)


def rel_err_plain(x, ref, floor_frac):
    """max_i |x_i - ref_i| / |ref_i| over the entries with |ref_i| >= floor_frac * max|ref|:
    the plain per-element relative error of the components that carry the array."""
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    big = np.abs(ref) >= floor_frac * np.abs(ref).max() if ref.size else np.zeros(0, bool)
    if not big.any():
        return 0.0
    return float(np.max(np.abs(x[big] - ref[big]) / np.abs(ref[big])))
