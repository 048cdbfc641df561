"""Benchmark of the NEP training step on one MI355X.

One step = nep_loss_and_grad (descriptors, network, forces, virials, loss,
analytic parameter gradient) + nep_adam_step over the whole batch, with the
batch and its neighbour lists already resident in HBM (the lists are built
once per dataset and timed separately, as the paper caches them).

Workload: 256 single-species periodic fcc cells with 32..256 atoms (noise
0.15 A, strain up to 2%), radial/angular cutoff 6/4 A, n_max 6/4, basis 8/8,
l_max 4, 30 hidden neurons, FP32 bulk arithmetic with FP64 per-structure and
loss reductions; synthetic structures, random-initialised parameters and
teacher-model targets.

Prints one JSON line (rank 0) with the throughput in structures/s, the
roofline position of the dominant kernel, the plain-PyTorch autograd
double-backward comparator on the same GPU, and the FP64 CPU oracle baseline.
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
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--workload", default="fcc_uneven_256")
    p.add_argument("--profile-steps", type=int, default=5)
    p.add_argument("--comparator-steps", type=int, default=3)
    p.add_argument("--no-comparator", action="store_true")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-structures", type=int, default=256)
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="also run one device-to-device copy of this many MiB (a known-size kernel that "
                        "calibrates hardware byte counters)")
    return p.parse_args()


# ------------------------------------------------------------ FLOP model
#
# Algorithmic FLOPs per unit of work of each kernel, counted from the formulas
# the kernel evaluates (FMA = 2, other arithmetic and transcendental = 1).
# K = basis size + 1, N = channels, LM = 24 harmonics (l <= 4), D descriptors.

Y_VAL = 82      # the 24 real solid harmonics of a unit vector
Y_DIR = 214     # harmonics and their derivative along one vector (dual numbers)
Y_GRAD = 478    # harmonics and their full gradient (dual numbers)


def basis_flops(K, deriv):
    # x, y, sincospi, cutoff (~13) + per k: value 3 (+ derivative 6) + recurrence 2 (+ 4)
    return 13 + K * (3 + (6 if deriv else 0)) + (K - 1) * (2 + (4 if deriv else 0))


def kernel_flops(name, md, npairs, nang, natoms):
    KR, KA = md["basis_r"] + 1, md["basis_a"] + 1
    NR, NA = md["n_max_r"] + 1, md["n_max_a"] + 1
    T, H, L = md["num_types"], md["hidden"], md["l_max"]
    LM = (L + 1) ** 2 - 1
    D = NR + NA * (L + (md["l_max_4b"] == 2) + (md["l_max_5b"] == 1))
    if name == "descriptor":
        rad = 6 + basis_flops(KR, False) + KR
        ang = 4 + basis_flops(KA, False) + Y_VAL + 2 * NA * KA + 2 * NA * LM
        atom = T * 2 * NR * KR + 2 * NA * LM
        return npairs * rad + nang * ang + natoms * atom
    if name == "force":
        rad = 6 + 1 + 3 + basis_flops(KR, True) + 3 * KR + 3
        ang = basis_flops(KA, True) + Y_GRAD + 8 * NA * KA + 8 * NA * LM + 2 * LM * 5 + 12
        return npairs * (rad + 18) + nang * ang
    if name == "tangent":
        rad = 6 + 1 + 3 + 15 + 5 + basis_flops(KR, True) + 2 * KR
        ang = basis_flops(KA, True) + Y_DIR + 4 * LM + 4 * NA * KA + 4 * NA * LM + NA
        atom = T * 2 * NR * KR + 4 * NA * LM
        return npairs * rad + nang * ang + natoms * atom
    if name == "angular_coeff_grad":
        per = 6 + 1 + 3 + 15 + 5 + basis_flops(KA, True) + Y_DIR + 4 * LM + 6 * NA * LM + NA + 4 * NA * KA
        return nang * per
    if name == "network_forward":
        return natoms * (D + H * (4 * D + 6) + 2 * NA * LM + T * 2 * NR * KR)
    if name == "network_backward":
        return natoms * (D + H * (4 * D + 14) + 3 * D + 4 * NA * LM)
    if name == "outer_grad":
        return natoms * (T * NR * KR * 4 + H * D * 4 + 2 * H)
    return None


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
    nb = N.nep_build_neighbors(model, gb, capacity=host.num_atoms * 80)
    torch.cuda.synchronize()
    nbr_ms = (time.perf_counter() - t0) * 1e3
    log(f"neighbour build {nbr_ms:.1f} ms: {nb.num_pairs} pairs, {nb.num_angular_pairs} angular")

    ws = N.workspace(model, gb, nb)
    theta = torch.tensor(draw_theta(P, w.seed + 1000), dtype=td, device=dev)
    teacher = torch.tensor(draw_theta(P, w.seed + 2000), dtype=td, device=dev)
    q = N.nep_descriptors(model, theta, gb, nb, ws)
    qs = N.nep_descriptor_scale(q)
    Et, Ft, Wt = N.nep_forward(model, teacher, qs, gb, nb, ws)
    targets = N.Targets(Et, Ft, Wt, lambdas=w.lambdas, dtype=td, device=dev)
    m_ = torch.zeros(P, dtype=td, device=dev)
    v_ = torch.zeros(P, dtype=td, device=dev)
    vm_ = torch.zeros(P, dtype=td, device=dev)
    grad = torch.empty(P, dtype=td, device=dev)
    loss = torch.empty(4, dtype=torch.float64, device=dev)
    adam = N.AdamConfig(lr=5e-3)
    th = theta.clone()
    step_no = [0]

    def step():
        N.nep_loss_and_grad(model, th, qs, gb, nb, targets, ws, grad=grad, loss=loss)
        step_no[0] += 1
        N.nep_adam_step(th, grad, m_, v_, vm_, step_no[0], adam)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done, loss {loss[0].item():.6e}")
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    sps = host.num_structures / (ms * 1e-3)
    log(f"timed {args.steps} steps: {ms:.4f} ms/step, {sps:.1f} structures/s, loss {loss[0].item():.6e}")

    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nbytes} bytes read and written once")
        del src, dst

    # per-kernel event timing on the launch stream
    N.nep_profile_enable(True)
    for _ in range(args.profile_steps):
        step()
    prof = N.nep_profile_read()
    N.nep_profile_enable(False)
    rows = []
    for name, (n, tot) in prof.items():
        rows.append((name, n, tot / n))
        log(f"  kernel {name:22s} launches {n:4d}  avg {tot / n * 1e3:9.2f} us")
    dom = max(rows, key=lambda r: r[2] * (r[1] / args.profile_steps))
    name, n, avg_ms = dom
    fl = kernel_flops(name, w.model, nb.num_pairs, nb.num_angular_pairs, host.num_atoms)
    peak = PEAK_FP64_TFLOPS if w.dtype == "f64" else PEAK_FP32_TFLOPS
    roof = None
    if fl is not None:
        achieved = fl / (avg_ms * 1e-3) / 1e12
        roof = {"kernel": name, "bound": "alu", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                "flops_per_launch": int(fl), "avg_launch_us": round(avg_ms * 1e3, 2)}
    kernel_table = {r[0]: round(r[2] * 1e3, 2) for r in rows}

    # comparator: plain PyTorch autograd double backward on the same GPU
    comp = None
    if not args.no_comparator:
        from comparator import AutogradNEP, pairs_from_csr

        try:
            pi, pj, pr = pairs_from_csr(nb.row_offset[: host.num_atoms + 1], nb.neighbor_index().to(dev),
                                        nb.pairs[: nb.num_pairs, :3])
            net = AutogradNEP(w.model, gb.types, gb.atom_offset, pi, pj, pr.to(td))
            Ft_c = targets.force
            for _ in range(1):
                net.loss_and_grad(th, qs, targets.energy.to(td), Ft_c, targets.virial.to(td), w.lambdas)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(args.comparator_steps):
                parts, gc = net.loss_and_grad(th, qs, targets.energy.to(td), Ft_c, targets.virial.to(td), w.lambdas)
            b.record()
            torch.cuda.synchronize()
            cms = a.elapsed_time(b) / args.comparator_steps
            N.nep_loss_and_grad(model, th, qs, gb, nb, targets, ws, grad=grad, loss=loss)
            rel = float((gc - grad).abs().max() / grad.abs().max())
            comp = {"kind": "torch autograd double backward", "value": round(host.num_structures / (cms * 1e-3), 1),
                    "unit": "structures/s", "ms_per_step": round(cms, 3), "speedup": round(cms / ms, 2),
                    "grad_max_rel_diff": rel}
            log(f"comparator {cms:.3f} ms/step -> speedup {cms / ms:.2f}x (grad rel diff {rel:.2e})")
        except Exception as e:  # report, do not hide
            comp = {"kind": "torch autograd double backward", "error": repr(e)[:200]}
            log(f"comparator failed: {e!r}")

    # CPU baseline: the FP64 oracle on the host cores
    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O

        n_s = min(args.cpu_structures, host.num_structures)
        sub = host.subset(range(n_s))
        om = O.Model(**w.model)
        cores = min(os.cpu_count() or 1, 16)
        th_h = th.double().cpu().numpy()
        qs_h = qs.double().cpu().numpy()
        a0 = int(sub.atom_offset[-1])
        Et_h = targets.energy[:n_s].cpu().numpy()
        Ft_h = targets.force[:a0].double().cpu().numpy()
        Wt_h = targets.virial[:n_s].cpu().numpy()
        t0 = time.perf_counter()
        O.loss_and_grad(om, th_h, qs_h, sub, Et_h, Ft_h, Wt_h, w.lambdas, nthreads=cores)
        dt = time.perf_counter() - t0
        cpu = {"value": round(n_s / dt, 2), "unit": "structures/s", "cores": cores, "kind": "oracle",
               "sample": f"first {n_s} structures of the workload, FP64 loss + gradient, {dt:.2f} s"}
        log(f"cpu oracle {n_s / dt:.1f} structures/s on {cores} threads")

    out = {
        "metric": "structures/s for NEP E/F/virial loss+param-grad; % HBM/VALU roofline",
        "value": round(sps, 1),
        "unit": "structures/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w.dtype == "f32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {host.num_structures} fcc cells, {host.num_atoms} atoms, "
                               f"{nb.num_pairs} pairs (rc 6/4 A, n_max 6/4, basis 8/8, l_max 4, 30 neurons)",
                   "structures": host.num_structures, "atoms": host.num_atoms, "pairs": nb.num_pairs,
                   "angular_pairs": nb.num_angular_pairs, "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "autograd_comparator": comp,
        "kernels_avg_us": kernel_table,
        "neighbor_build_ms": round(nbr_ms, 2),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
