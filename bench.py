"""Benchmark of the NEP training step on one MI355X.

One step = nep_loss_and_grad (descriptors, network, forces, virials, loss,
analytic parameter gradient) + nep_adam_step over the whole batch (as the one
call nep_train_step, which takes the update in the gradient's last kernel), with the
batch and its neighbour lists already resident in HBM (the lists are built
once per dataset and timed separately, as the paper caches them).

Default workload: the large-cell configuration, 32 periodic cells of
4000-16000 atoms (277,380 atoms; half random 5-species alloys on an fcc
lattice at 0.11 atoms/A^3, half dense liquids), radial/angular cutoff 6/5 A,
n_max 10/8, basis 12/12, l_max 4, 100 hidden neurons, ~90 radial neighbours
per atom; FP32 bulk arithmetic with FP64 per-structure and loss reductions;
synthetic structures, random-initialised parameters and teacher-model
targets. Other workloads: --workload.

Prints one JSON line (rank 0) with the throughput in structures/s, the
per-step spread, the roofline position of the dominant kernel and of the
whole step, the plain-PyTorch autograd double-backward comparator on the same
GPU, and the FP64 CPU oracle baseline; beside them, outside the timed steps,
the neighbour build (first and warm) and the forward-only path (E, F, W per
call, and with the lists rebuilt before every call as in a molecular-dynamics
loop).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3  # MI355X published dense FP32 vector peak
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=None,
                   help="timed steps (default 50; a whole epoch of minibatches for a minibatch workload)")
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--workload", default="large5_32")
    p.add_argument("--comparator-steps", type=int, default=3)
    p.add_argument("--no-comparator", action="store_true")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-autotune", action="store_true", help="use the default launch plan")
    p.add_argument("--retune", action="store_true", help="tune the launch plan even when one is cached")
    p.add_argument("--plan", default=None, metavar="JSON",
                   help='override fields of the chosen launch plan, e.g. \'{"coeff_grad_rows": 3}\'')
    p.add_argument("--cpu-structures", type=int, default=0,
                   help="oracle sample: the first N structures (default: 16 large cells, 64 alloy cells, else 256)")
    p.add_argument("--cpu-threads", type=int, default=0,
                   help="oracle threads for the CPU baseline (default: the host's cores, at most 16)")
    p.add_argument("--cpu-seconds", type=float, default=10.0,
                   help="repeat the all-thread oracle run over the sample until this much time has passed")
    p.add_argument("--json-out", default=None, help="also write the result line to this file")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="also run one device-to-device copy of this many MiB (a known-size kernel that "
                        "calibrates hardware byte counters)")
    return p.parse_args()


# ------------------------------------------------------------ work model
#
# Algorithmic work of each kernel per launch, counted from the formulas it
# evaluates: FLOPs with FMA = 2 and every other arithmetic operation or
# transcendental = 1; bytes = every array the kernel must read or write, each
# counted once (neighbour records 4 reals per pair; per-atom and per-structure
# arrays at their size; gathers of neighbour data and block-partial reduction
# rows are not algorithmic and are not counted).
# K = basis size + 1, N = radial/angular channels, LM = 24 harmonics (l <= 4),
# D = descriptor length, H = hidden units, T = species.

Y_VAL = 82      # the 24 real solid harmonics of a unit vector
Y_DIR = 214     # harmonics and their derivative along one vector (dual numbers)
Y_CGRAD = 241   # gradient of one linear combination of the 24 harmonics (closed form)
PAIR_GEOM = 9   # |r| (3 FMA + sqrt), 1/r, unit vector


def basis_flops(K, deriv):
    # setup (y, x, sincospi, cutoff and its slope) 13; per k: f_k and the
    # recurrence 4 (+ f_k' and the derivative recurrence 8)
    return 13 + K * (12 if deriv else 4)


def work_model(name, md, n, fused=False):
    """(flops, bytes) of one launch of kernel `name`; n holds the batch counts.
    `fused`: the network runs inside the descriptor and tangent sweeps (plan
    network 3), which then also do the network passes' work, and the
    descriptor sweep the force pass's."""
    if fused and name in ("descriptor", "tangent"):
        fl, by = work_model(name, md, n)
        nf, nb = work_model("network_forward" if name == "descriptor" else "network_backward", md, n)
        D = md["n_max_r"] + 1 + (md["n_max_a"] + 1) * (md["l_max"] + (md["l_max_4b"] == 2) + (md["l_max_5b"] == 1))
        # the descriptor (or its tangent) is in registers: not read again
        fl, by = fl + nf, by + nb - n["atoms"] * (4 + n["real_bytes"] * D)
        if name == "descriptor":
            ff, fb = work_model("force", md, n)
            LM = (md["l_max"] + 1) ** 2 - 1
            NA, r = md["n_max_a"] + 1, n["real_bytes"]
            # records, moments, e and the per-atom indices were read or made
            # by the same kernel
            fb -= 4 * r * n["pairs"] + n["atoms"] * (8 + 4 + 4 + 8 * md["num_types"] + r * (NA * LM + D))
            fl, by = fl + ff, by + fb
        return fl, by
    KR, KA = md["basis_r"] + 1, md["basis_a"] + 1
    NR, NA = md["n_max_r"] + 1, md["n_max_a"] + 1
    T, H, L = md["num_types"], md["hidden"], md["l_max"]
    LM = (L + 1) ** 2 - 1
    h4, h5 = md["l_max_4b"] == 2, md["l_max_5b"] == 1
    D = NR + NA * (L + h4 + h5)
    npr, nang, na, ns, r = n["pairs"], n["angular_pairs"], n["atoms"], n["structures"], n["real_bytes"]
    rec = 4 * r * npr                    # neighbour records
    rec_ang = 4 * r * nang               # angular records only
    idx = na * (8 + 4 + 4 + 8 * T)       # row offset, type, structure, per-species counts
    B_atom = 2 * NA * LM + (50 * NA if h4 else 0) + (15 * NA if h5 else 0)  # dE/dA from e and A
    if name == "descriptor":
        pair_r = PAIR_GEOM + basis_flops(KR, False) + KR
        pair_a = basis_flops(KA, False) + Y_VAL + 2 * NA * KA + 2 * NA * LM
        atom = T * 2 * NR * KR + 2 * NA * LM + (40 * NA if h4 else 0)
        return (npr * pair_r + nang * pair_a + na * atom,
                rec + idx + na * r * (D + NA * LM + T * KR))
    if name == "network_forward":
        return (na * (2 * D + H * (2 * D + 2) + H * (2 * D + 4) + 2 * H),
                na * (4 + r * (D + 1 + D + H)))
    if name == "force":
        pair_r = PAIR_GEOM + basis_flops(KR, True) + 2 * KR + 3 + 6 + 18
        pair_a = basis_flops(KA, True) + Y_VAL + Y_CGRAD + 4 * NA * KA + 4 * NA * LM + 2 * LM + 5 + 12
        atom = B_atom + T * 2 * NR * KR
        return (npr * pair_r + nang * pair_a + na * atom,
                rec + 4 * npr + idx + na * r * (NA * LM + D + 3 + 9) + rec)
    if name == "force_gather":
        return (npr * 3, rec + na * (8 + 2 * 3 * r))
    if name == "tangent":
        pair_r = PAIR_GEOM + 24 + basis_flops(KR, True) + 5 + 2 * KR
        pair_a = basis_flops(KA, True) + Y_DIR + 4 * LM + 4 * NA * KA + NA + 4 * NA * LM
        atom = T * 2 * NR * KR + 4 * NA * LM + (60 * NA if h4 else 0)
        return (npr * pair_r + nang * pair_a + na * atom,
                rec + idx + na * r * (3 + NA * LM + D + NA * LM + T * KR) + ns * 72)
    if name == "network_backward":
        return (na * (H * (2 * D) + H * 14 + H * (2 * D) + 3 * D),
                na * (4 + r * (3 * D + H + 3 * H)) + ns * 8)
    if name == "angular_coeff_grad":
        pair = (PAIR_GEOM + 24 + 5 + basis_flops(KA, True) + Y_DIR + 4 * LM
                + 6 * NA * LM + NA + 4 * NA * KA)
        atom = 3 * B_atom
        return (nang * pair + na * atom,
                rec_ang + idx + na * r * (3 + 2 * NA * LM + 2 * D) + ns * 72)
    if name == "outer_grad":
        return (na * (4 * H * D + 2 * H + 4 * T * NR * KR),
                na * (4 + r * (4 * D + 3 * H + 2 * T * KR)))
    return None


def source_digest():
    """SHA-256 over the HIP sources of the library (any edit changes it)."""
    import hashlib

    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2606_19557_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".inc", ".h")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel, workload, plan=None):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when there is none, the sources changed since it was taken, or it was
    taken under another launch plan than `plan` (a dict of plan fields)."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    # the summary's row for this kernel as the plan builds it
    label = "k_" + kernel
    if plan is not None and plan.get("network") == 3 and kernel in ("descriptor", "tangent"):
        label += "+network+force" if kernel == "descriptor" else "+network"
    digest, val = None, None
    for line in open(path):
        if line.startswith("plan:") and plan is not None:
            taken = json.loads(line.split(":", 1)[1])
            if any(taken.get(k) != v for k, v in plan.items()):
                return None
        if line.startswith("source-sha256:"):
            digest = line.split(":", 1)[1].strip()
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 6 and cells[0] == label:
            try:
                val = float(cells[5])
            except ValueError:
                pass
    if digest != source_digest() or val is None:
        return None
    return val


# --------------------------------------------------------------- CPU baseline


def host_cpu():
    """(logical CPUs, CPU model name) of this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count() or 1, model


def cpu_baseline(args, w, host, th, qs, targets, log):
    """The FP64 oracle's loss + gradient on a bounded sample of the workload:
    one run on all threads (repeated up to --cpu-seconds) and one on a single
    thread over the sample's first n/threads structures. The oracle's brute-force
    neighbour search is timed by the oracle itself (thread-seconds) and left
    out of the rates: single thread, wall minus search; all threads, wall
    minus search thread-seconds over the threads in use."""
    import oracle as O

    default_n = {"large5_32": 16, "alloy4_1024": 64}.get(args.workload, 256)
    n_s = min(args.cpu_structures or default_n, host.num_structures)
    sub = host.subset(range(n_s))
    om = O.Model(**w.model)
    nproc, cpu_model = host_cpu()
    threads = min(args.cpu_threads if args.cpu_threads > 0 else min(nproc, 16), n_s)
    th_h = th.double().cpu().numpy()
    qs_h = qs.double().cpu().numpy()
    a0 = int(sub.atom_offset[-1])
    Et_h = targets.energy[:n_s].cpu().numpy()
    Ft_h = targets.force[:a0].double().cpu().numpy()
    Wt_h = targets.virial[:n_s].cpu().numpy()
    lam = w.lambdas

    def run(batch, nthreads, seconds):
        Et, Ft, Wt = Et_h[:batch.num_structures], Ft_h[:batch.num_atoms], Wt_h[:batch.num_structures]
        O.search_seconds(reset=True)
        reps, t0 = 0, time.perf_counter()
        while True:
            O.loss_and_grad(om, th_h, qs_h, batch, Et, Ft, Wt, lam, nthreads=nthreads)
            reps += 1
            wall = time.perf_counter() - t0
            if wall >= seconds:
                break
        return reps, wall, O.search_seconds()

    reps, wall, search = run(sub, threads, args.cpu_seconds)
    compute = wall - search / threads
    rate = reps * n_s / compute
    one = sub.subset(range(max(1, n_s // threads)))
    r1, wall1, search1 = run(one, 1, args.cpu_seconds / 4)
    rate1 = r1 * one.num_structures / (wall1 - search1)
    atoms = reps * a0 / compute
    log(f"cpu oracle {rate:.3f} structures/s on {threads} threads ({reps} x {n_s} structures, {wall:.1f} s, "
        f"search {search:.1f} thread-s excluded); 1 thread {rate1:.4f} structures/s; {nproc} CPUs: {cpu_model}")
    return {"value": round(rate, 4), "unit": "structures/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n_s} structures ({a0} atoms) of the workload x {reps}, FP64 loss + gradient; "
                      f"the oracle's brute-force neighbour search excluded ({search:.1f} of "
                      f"{wall * threads:.1f} thread-seconds); single-thread rate on the first "
                      f"{one.num_structures} structures ({one.num_atoms} atoms) x {r1}",
            "atoms_per_s": round(atoms, 1),
            "value_with_search": round(reps * n_s / wall, 4),
            "search_thread_s": round(search, 2),
            "single_thread": {"value": round(rate1, 5), "unit": "structures/s",
                              "atoms_per_s": round(one.num_atoms * r1 / (wall1 - search1), 1),
                              "search_s": round(search1, 2), "wall_s": round(wall1, 2)},
            "host": {"nproc": nproc, "cpu_model": cpu_model}}


# ------------------------------------------------------------------- main


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported by this build "
              "(structures are independent; the multi-GPU design is documented, not built).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2606_19557_amd as N
    from synth import WORKLOADS, workload_batch
    from synth.workloads import draw_theta

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    w = WORKLOADS[args.workload]
    model = N.Model.from_dict(w.model, dtype=w.dtype)
    td = model.torch_dtype
    P, D = N.nep_param_count(model)
    host = workload_batch(args.workload)
    log(f"workload {args.workload}: {host.num_structures} structures, {host.num_atoms} atoms, P={P}, D={D}")
    dev = torch.device("cuda:0")
    gb = N.Batch.from_host(host, dtype=td, device=dev)

    # neighbour lists, built once (timed separately)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # (a minibatch workload's dataset lists also keep each structure's species
    # runs, from which a minibatch's species order is gathered)
    runs = w.minibatch > 0
    nb = N.nep_build_neighbors(model, gb, capacity=host.num_atoms * 80, species_runs=runs)
    torch.cuda.synchronize()
    nbr_first_ms = (time.perf_counter() - t0) * 1e3
    # again, warm (code objects loaded, buffers cached): the cost of a rebuild,
    # e.g. per step of a forward-only MD loop
    nbw_ws = N.workspace(model, gb)
    t0 = time.perf_counter()
    nb = N.nep_build_neighbors(model, gb, capacity=nb.num_pairs, ws=nbw_ws, species_runs=runs)
    torch.cuda.synchronize()
    nbr_ms = (time.perf_counter() - t0) * 1e3
    del nbw_ws
    log(f"neighbour build {nbr_first_ms:.1f} ms first, {nbr_ms:.2f} ms warm: {nb.num_pairs} pairs, "
        f"{nb.num_angular_pairs} angular")

    ws = N.workspace(model, gb, nb)
    theta = torch.tensor(draw_theta(P, w.seed + 1000), dtype=td, device=dev)
    teacher = torch.tensor(draw_theta(P, w.seed + 2000), dtype=td, device=dev)
    q = N.nep_descriptors(model, theta, gb, nb, ws)
    qs = N.nep_descriptor_scale(q)
    Et, Ft, Wt = N.nep_forward(model, teacher, qs, gb, nb, ws)
    targets = N.Targets(Et, Ft, Wt, lambdas=w.lambdas, dtype=td, device=dev)
    epoch_mode = w.minibatch > 0
    if epoch_mode:
        # a training epoch: shuffled minibatches packed on the device from the
        # dataset's lists (built once), one Adam step each
        from paper_2606_19557_amd.train import Dataset

        data = Dataset.from_device(model, gb, nb, targets, host.atom_offset)
        order = np.random.Generator(np.random.PCG64(w.seed + 4000)).permutation(host.num_structures)
        mbs = [order[lo:lo + w.minibatch] for lo in range(0, len(order), w.minibatch)]
        # the epoch's order goes to the device once (a copy from pageable host
        # memory per step would wait for the previous step's kernels)
        order_dev = torch.as_tensor(order.astype(np.int32)).to(dev)
        mbs_dev = [order_dev[lo:lo + w.minibatch] for lo in range(0, len(order), w.minibatch)]
        sizes = np.array([data.sizes(ids) for ids in mbs])
        tune_b, tune_nb, tune_tg = data.minibatch(mbs[0])
        log(f"epoch of {len(mbs)} minibatches of {w.minibatch}: mean {sizes[:, 0].mean():.0f} atoms, "
            f"{sizes[:, 1].mean():.0f} pairs")
    else:
        tune_b, tune_nb, tune_tg = gb, nb, targets
    plan, plan_cached, plan_key = None, False, None
    if not args.no_autotune:
        from paper_2606_19557_amd import tuning

        t0 = time.perf_counter()
        if args.retune:
            plan = N.nep_autotune(model, theta, qs, tune_b, tune_nb, tune_tg, repeats=3)
        else:
            plan, plan_cached = tuning.tuned_plan(model, theta, qs, tune_b, tune_nb, tune_tg, repeats=3,
                                                  shipped=tuning.SHIPPED_PLANS)
        if args.plan:
            from dataclasses import replace

            plan, plan_cached = replace(plan, **{k: int(v) for k, v in json.loads(args.plan).items()}), False
        model = model.with_plan(plan)
        plan_key = tuning.plan_key(model, tune_b.num_atoms, tune_nb.num_pairs)
        log(f"{'cached' if plan_cached else 'autotuned'} plan in {time.perf_counter() - t0:.2f} s: {plan.as_dict()}")
    if epoch_mode:
        data.model = model
        big = int(np.argmax(sizes[:, 1]))
        ws = torch.empty(max(256, N.nep_workspace_size(model, w.minibatch, int(sizes[:, 0].max()),
                                                       int(sizes[:, 1].max()))), dtype=torch.uint8, device=dev)
        structs_per_step = w.minibatch
        counts = {"pairs": float(sizes[:, 1].mean()), "angular_pairs": float(sizes[:, 2].mean()),
                  "atoms": float(sizes[:, 0].mean()), "structures": w.minibatch, "real_bytes": 8 if w.dtype == "f64" else 4}
        del big
    else:
        ws = N.workspace(model, gb, nb)
        structs_per_step = host.num_structures
        counts = {"pairs": nb.num_pairs, "angular_pairs": nb.num_angular_pairs, "atoms": host.num_atoms,
                  "structures": host.num_structures, "real_bytes": 8 if w.dtype == "f64" else 4}
    if args.steps is None:
        args.steps = len(mbs) if epoch_mode else 50
    m_ = torch.zeros(P, dtype=td, device=dev)
    v_ = torch.zeros(P, dtype=td, device=dev)
    vm_ = torch.zeros(P, dtype=td, device=dev)
    grad = torch.empty(P, dtype=td, device=dev)
    loss = torch.empty(4, dtype=torch.float64, device=dev)
    adam = N.AdamConfig(lr=5e-3)
    th = theta.clone()
    step_no = [0]

    def step():
        if epoch_mode:
            k = step_no[0] % len(mbs)
            b_, nb_, tg_ = data.minibatch(mbs[k], ids_device=mbs_dev[k])
        else:
            b_, nb_, tg_ = gb, nb, targets
        step_no[0] += 1
        # nep_loss_and_grad + nep_adam_step, the update taken in the kernel that
        # finishes the gradient
        N.nep_train_step(model, th, qs, b_, nb_, tg_, m_, v_, vm_, step_no[0], adam, ws, grad=grad, loss=loss)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done, loss {loss[0].item():.6e}")
    # every kernel's duration, from HIP events around each launch on the launch
    # stream over a profiled pass of the same steps (outside the timed region:
    # events around every launch would add to the step time of small batches)
    N.nep_profile_enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = N.nep_profile_read()
    N.nep_profile_enable(False)
    # the dominant kernel by time per step, re-timed inside the timed region
    dom_name = max(prof.items(), key=lambda kv: kv[1][1])[0]
    # timed region: an event after every step (per-step spread) and HIP events
    # around every launch of the dominant kernel only (its live duration)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    N.nep_profile_only(dom_name)
    N.nep_profile_enable(True)
    torch.cuda.synchronize()
    evs[0].record()
    for k in range(args.steps):
        step()
        evs[k + 1].record()
    torch.cuda.synchronize()
    ms = evs[0].elapsed_time(evs[-1]) / args.steps
    per_step = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])
    live = N.nep_profile_read()
    N.nep_profile_enable(False)
    N.nep_profile_only(None)
    prof[dom_name] = live[dom_name]
    sps = structs_per_step / (ms * 1e-3)
    p10, p50, p90 = (float(np.percentile(per_step, q)) for q in (10, 50, 90))
    log(f"timed {args.steps} steps: {ms:.4f} ms/step (median {p50:.4f}, p10 {p10:.4f}, p90 {p90:.4f}), "
        f"{sps:.1f} structures/s, loss {loss[0].item():.6e}")

    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nbytes} bytes read and written once")
        del src, dst

    rows = []
    for name, (n, tot) in prof.items():
        rows.append((name, n, tot / n))
        log(f"  kernel {name:22s} launches {n:4d}  avg {tot / n * 1e3:9.2f} us")
    used_plan = plan.as_dict() if plan is not None else dict(
        team_descriptor=8, team_force=8, team_tangent=8, team_coeff_grad=8, coeff_grad_blocks=2048, outer_chunk=64,
        network=1, coeff_grad_rows=0)
    fused = used_plan["network"] == 3
    peak_alu = PEAK_FP64_TFLOPS if w.dtype == "f64" else PEAK_FP32_TFLOPS
    # whole step: algorithmic FLOPs and bytes of every kernel launched per step
    step_fl = step_by = 0.0
    for name, n, _ in rows:
        wk = work_model(name, w.model, counts, fused=fused)
        if wk is not None:
            step_fl += wk[0] * n / args.steps
            step_by += wk[1] * n / args.steps
    step_roof = {"gflop": round(step_fl / 1e9, 3), "alg_mb": round(step_by / 1e6, 2),
                 "flop_per_byte": round(step_fl / max(step_by, 1.0), 2),
                 "alu_frac": round(step_fl / (ms * 1e-3) / 1e12 / peak_alu, 4),
                 "hbm_frac": round(step_by / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    dom = next(r for r in rows if r[0] == dom_name)
    name, n, avg_ms = dom
    work = work_model(name, w.model, counts, fused=fused)
    roof = None
    if work is not None:
        fl, by = work
        sec = avg_ms * 1e-3
        traffic = measured_traffic(name, args.workload, used_plan)
        # the bound: the kernel's algorithmic FLOPs at the vector peak against
        # its algorithmic bytes at the HBM peak (the work model's FLOP/byte
        # against the ridge); the measured HBM bytes, when a counter summary of
        # these sources exists, are reported beside it (traffic and
        # hbm_frac_measured) -- bytes above the algorithmic ones are re-reads
        # and partial-line writes, not the method's work
        t_alu = fl / (peak_alu * 1e12)
        t_hbm = by / (PEAK_HBM_GBS * 1e9)
        if t_alu >= t_hbm:
            achieved, peak = fl / sec / 1e12, peak_alu
            roof = {"kernel": name, "bound": "alu", "achieved": round(achieved, 3), "peak": peak,
                    "unit": "TFLOP/s"}
        else:
            achieved, peak = by / sec / 1e9, PEAK_HBM_GBS
            roof = {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": peak,
                    "unit": "GB/s"}
        roof.update({"frac": round(achieved / peak, 4), "traffic": None if traffic is None else int(traffic),
                     "flops_per_launch": int(fl), "bytes_per_launch": int(by),
                     "alu_frac": round(fl / sec / 1e12 / peak_alu, 4),
                     # the kernels are built without packed FP32 instructions:
                     # the vector rate they can reach is half the published peak
                     "alu_frac_nonpacked": round(fl / sec / 1e12 / (peak_alu / 2 if w.dtype == "f32" else peak_alu),
                                                 4),
                     "hbm_frac": round(by / sec / 1e9 / PEAK_HBM_GBS, 4),
                     "hbm_frac_measured": None if traffic is None else round(traffic / sec / 1e9 / PEAK_HBM_GBS, 4),
                     "avg_launch_us": round(avg_ms * 1e3, 2),
                     "timing": "HIP events around each launch of this kernel inside the timed steps",
                     "step": step_roof})
    kernel_table = {r[0]: round(r[2] * 1e3, 2) for r in rows}

    # forward-only path (inference, MD): E, F, W per call on the resident lists,
    # and with the lists rebuilt before every call as an MD step would
    fb, fnb = (tune_b, tune_nb) if epoch_mode else (gb, nb)
    fws, nbws, reps = N.workspace(model, fb, fnb), N.workspace(model, fb), 20
    for _ in range(2):
        N.nep_forward(model, th, qs, fb, fnb, fws)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        N.nep_forward(model, th, qs, fb, fnb, fws)
    b.record()
    torch.cuda.synchronize()
    fwd_ms = a.elapsed_time(b) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        nb_md = N.nep_build_neighbors(model, fb, capacity=fnb.num_pairs, ws=nbws)
        N.nep_forward(model, th, qs, fb, nb_md, fws)
    torch.cuda.synchronize()
    md_ms = (time.perf_counter() - t0) * 1e3 / reps
    del nb_md, fws, nbws
    forward = {"ms_per_call": round(fwd_ms, 4), "structures_per_s": round(fb.num_structures / (fwd_ms * 1e-3), 1),
               "ms_per_call_with_neighbor_rebuild": round(md_ms, 3)}
    log(f"forward only: {fwd_ms:.4f} ms per call, {md_ms:.3f} ms with the neighbour lists rebuilt")

    # comparator: plain PyTorch autograd double backward on the same GPU
    comp = None
    if not args.no_comparator:
        from comparator import AutogradNEP, pairs_from_csr

        try:
            # the timed batch (the first minibatch of the epoch in epoch mode)
            cb, cnb, ctg = tune_b, tune_nb, tune_tg
            pi, pj, pr = pairs_from_csr(cnb.row_offset[: cb.num_atoms + 1], cnb.neighbor_index().to(dev),
                                        cnb.pairs[: cnb.num_pairs, :3])
            net = AutogradNEP(w.model, cb.types, cb.atom_offset, pi, pj, pr.to(td))
            Ft_c = ctg.force
            for _ in range(1):
                net.loss_and_grad(th, qs, ctg.energy.to(td), Ft_c, ctg.virial.to(td), w.lambdas)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(args.comparator_steps):
                parts, gc = net.loss_and_grad(th, qs, ctg.energy.to(td), Ft_c, ctg.virial.to(td), w.lambdas)
            b.record()
            torch.cuda.synchronize()
            cms = a.elapsed_time(b) / args.comparator_steps
            wsc = N.workspace(model, cb, cnb)
            N.nep_loss_and_grad(model, th, qs, cb, cnb, ctg, wsc, grad=grad, loss=loss)
            rel = float((gc - grad).abs().max() / grad.abs().max())
            comp = {"kind": "torch autograd double backward", "value": round(cb.num_structures / (cms * 1e-3), 1),
                    "unit": "structures/s", "ms_per_step": round(cms, 3), "speedup": round(cms / ms, 2),
                    "grad_max_rel_diff": rel}
            log(f"comparator {cms:.3f} ms/step -> speedup {cms / ms:.2f}x (grad rel diff {rel:.2e})")
        except Exception as e:  # report, do not hide
            comp = {"kind": "torch autograd double backward", "error": repr(e)[:200]}
            log(f"comparator failed: {e!r}")

    # CPU baseline: the FP64 oracle on the host cores, on the first structures
    # of the workload, timed with its brute-force neighbour search excluded
    # (the GPU step excludes the list build too); the search's own time and
    # the rate with it are reported beside
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, w, host, th, qs, targets, log)

    out = {
        "metric": "structures/s for NEP E/F/virial loss+param-grad; % HBM/VALU roofline",
        "value": round(sps, 1),
        "unit": "structures/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "ms_per_step_spread": {"median": round(p50, 4), "p10": round(p10, 4), "p90": round(p90, 4)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w.dtype == "f32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {w.description}",
                   "structures": host.num_structures, "atoms": host.num_atoms, "pairs": nb.num_pairs,
                   "angular_pairs": nb.num_angular_pairs, "parallelism": "single GPU",
                   "plan": None if plan is None else dict(plan.as_dict(), from_cache=plan_cached, key=plan_key),
                   **({"minibatch": w.minibatch, "steps_per_epoch": len(mbs),
                       "epoch_s": round(ms * len(mbs) * 1e-3, 5)} if epoch_mode else {})},
        "roofline": roof,
        "cpu_baseline": cpu,
        "autograd_comparator": comp,
        "kernels_avg_us": kernel_table,
        "neighbor_build_ms": round(nbr_ms, 2),
        "neighbor_build_first_ms": round(nbr_first_ms, 2),
        "forward_only": forward,
    }
    print(json.dumps(out), flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(json.dumps(out) + "\n")


if __name__ == "__main__":
    main()
