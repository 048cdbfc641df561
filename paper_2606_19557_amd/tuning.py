"""Launch plans chosen by the autotuner, kept in a JSON cache.

A plan depends on the model shape and precision and on the batch's size and
neighbour density, so the key holds those (atoms and pairs per atom in
power-of-two buckets): a new batch of the same kind reuses the plan without
timing again. The cache is a plain JSON object {key: plan fields}; its path is
$NEP_PLAN_CACHE, else ~/.cache/nep_mi355x/plans.json. `plans_mi355x.json`
beside this module holds plans the autotuner chose on an MI355X for the
benchmark workloads; callers may pass it as a read-only fallback.
"""

from __future__ import annotations

import json
import math
import os
import tempfile

from .nep import Batch, Model, Neighbors, Plan, Targets, nep_autotune

_FIELDS = tuple(Plan.__dataclass_fields__)
SHIPPED_PLANS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "plans_mi355x.json")


def cache_path() -> str:
    p = os.environ.get("NEP_PLAN_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "nep_mi355x", "plans.json")


def plan_key(model: Model, num_atoms: int, num_pairs: int) -> str:
    shape = (model.num_types, model.n_max_r, model.n_max_a, model.basis_r, model.basis_a, model.l_max,
             model.l_max_4b, model.l_max_5b, model.hidden)
    atoms_b = 0 if num_atoms <= 0 else int(math.log2(num_atoms))
    ppa_b = 0 if num_atoms <= 0 or num_pairs <= 0 else int(math.log2(num_pairs / num_atoms))
    return f"{model.dtype}|{'-'.join(map(str, shape))}|atoms2^{atoms_b}|pairs_per_atom2^{ppa_b}"


def load(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def store(entries: dict, path: str | None = None):
    """Atomic rewrite of the cache file."""
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(path) or ".", suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(entries, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _entry(entries: dict, key: str) -> Plan | None:
    hit = entries.get(key)
    if isinstance(hit, dict) and set(hit) >= set(_FIELDS):
        return Plan(**{k: int(hit[k]) for k in _FIELDS})
    return None


def tuned_plan(model: Model, theta, q_scale, batch: Batch, nbr: Neighbors, targets: Targets, repeats: int = 3,
               path: str | None = None, tuner=nep_autotune, shipped: str | None = None) -> tuple[Plan, bool]:
    """(plan, from_cache): the cached plan for this kind of batch, else the one
    in the read-only `shipped` file, else a freshly tuned one (then stored)."""
    key = plan_key(model, batch.num_atoms, nbr.num_pairs)
    entries = load(path)
    plan = _entry(entries, key)
    if plan is None and shipped:
        plan = _entry(load(shipped), key)
    if plan is not None:
        return plan, True
    plan = tuner(model, theta, q_scale, batch, nbr, targets, repeats=repeats)
    entries[key] = plan.as_dict()
    store(entries, path)
    return plan, False
