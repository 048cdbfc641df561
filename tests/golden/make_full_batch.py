"""Writes the oracle's loss, gradient and predictions for whole benchmark batches
(``full_<workload>.npz`` beside this script), against which the full-batch GPU
parity test compares the HIP path under the launch plan a benchmark run uses.

Calls only ``oracle/`` (FP64 CPU) and ``synth/`` (seeded inputs). The inputs
are rounded to float32 exactly as an FP32 device run receives them: positions,
parameters, the descriptor scaler and the force targets (cells, energies and
virials stay float64, as in the C ABI). The scaler is Eq. 2 over every atom of
the batch with the initial parameters; the targets are seeded random values
(``synth.random_targets``), which exercise the energy, force and virial terms
of Eqs. 4-7 alike.

Stored: the scaler, the loss [L, dE, dF, dV], the gradient [P], E [Ns],
W [Ns, 9], F on 4096 evenly spaced atoms, and a digest of the inputs so the
test can tell that it regenerated the same batch.

    python tests/golden/make_full_batch.py alloy4_1024 large5_32 [--threads 8]
"""

from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from synth import WORKLOADS, random_targets, workload_batch  # noqa: E402
from synth.workloads import draw_theta  # noqa: E402

F_SAMPLE = 4096
TARGET_SEED_OFFSET = 5000


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def rounded_inputs(name):
    """Batch, parameters and targets of a workload as an FP32 device run gets them."""
    from dataclasses import replace

    w = WORKLOADS[name]
    b = workload_batch(name)
    b = replace(b, positions=f32(b.positions))
    m = O.Model(**w.model)
    P, D = O.dims(m)
    theta = f32(draw_theta(P, w.seed + 1000))
    Et, Ft, Wt = random_targets(b, w.seed + TARGET_SEED_OFFSET)
    return w, m, b, theta, (Et, f32(Ft), Wt)


def input_digest(b, theta, targets):
    h = hashlib.sha256()
    for a in (b.positions, b.types, b.cells, b.atom_offset, theta, *targets):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def _desc_chunk(args):
    name, idx, theta = args
    from dataclasses import replace

    w = WORKLOADS[name]
    b = workload_batch(name, idx)
    b = replace(b, positions=f32(b.positions))
    return O.descriptors(O.Model(**w.model), theta, b)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workloads", nargs="+")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    for name in args.workloads:
        t0 = time.time()
        w, m, b, theta, tg = rounded_inputs(name)
        Ns = b.num_structures
        # Eq. 2 scaler over every atom, structures spread over worker processes
        chunks = [list(range(s, Ns, args.threads)) for s in range(min(args.threads, Ns))]
        with ProcessPoolExecutor(len(chunks)) as ex:
            parts = list(ex.map(_desc_chunk, [(name, c, theta) for c in chunks]))
        q = np.zeros((b.num_atoms, parts[0].shape[1]))
        for c, qc in zip(chunks, parts):
            sub_off = np.concatenate([[0], np.cumsum(np.diff(b.atom_offset)[c])])
            for k, s in enumerate(c):
                q[b.atom_offset[s]:b.atom_offset[s + 1]] = qc[sub_off[k]:sub_off[k + 1]]
        s = f32(O.scaler(q))
        print(f"[golden] {name}: descriptors of {b.num_atoms} atoms in {time.time() - t0:.0f} s", flush=True)
        loss, grad, E, F, W = O.loss_and_grad(m, theta, s, b, *tg, w.lambdas, nthreads=args.threads)
        f_idx = np.unique(np.linspace(0, b.num_atoms - 1, F_SAMPLE).astype(np.int64))
        out = os.path.join(HERE, f"full_{name}.npz")
        np.savez_compressed(out, workload=np.array(name), digest=np.array(input_digest(b, theta, tg)),
                            target_seed=np.array(w.seed + TARGET_SEED_OFFSET), qscale=s, loss=loss, grad=grad,
                            E=E, W=W, f_idx=f_idx, F=F[f_idx])
        print(f"[golden] {name}: loss {loss[0]:.9e}, |grad| {np.linalg.norm(grad):.6e}, "
              f"{time.time() - t0:.0f} s -> {out}", flush=True)


if __name__ == "__main__":
    main()
