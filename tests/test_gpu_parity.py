"""GPU parity: every output of the HIP path against the FP64 oracle, element by
element, on seeded inputs; bit-exact for index work, the stated relative
tolerances for floating point (FP64: 1e-9; FP32: energies 1e-5, forces,
virials and parameter gradients 1e-4, relative with an rms floor)."""

import numpy as np
import pytest
import torch

import oracle as O
from helpers import SMALL_ALLOY, device_inputs, fixture, rel_err, small_alloy_batch
from synth import structures as S

pytestmark = pytest.mark.gpu

N = pytest.importorskip("paper_2606_19557_amd")

TOL = {"f64": dict(E=1e-9, F=1e-9, W=1e-9, G=1e-9, L=1e-9),
       "f32": dict(E=1e-5, F=1e-4, W=1e-4, G=1e-4, L=1e-5)}

CASES = [
    ("bcc64x8", None, "f64"),
    ("fcc_uneven_256", list(range(12)), "f32"),
    ("fcc_uneven_256", list(range(12)), "f64"),
    ("small_alloy", None, "f64"),
    ("small_alloy", None, "f32"),
    # subsets of the larger workloads, in their own kernel shapes: 4 species with
    # 4-body and 5-body terms; 3 species with liquid-like packings; 5 species
    # with ~100 neighbours per atom (the smallest 4250-atom cell)
    ("alloy4_1024", [4, 0, 1, 3], "f32"),
    ("alloy4_1024", [4, 0, 1, 3], "f64"),
    ("mixed3_4096", [0, 1, 2, 4, 5], "f32"),
    ("large5_32", [20], "f32"),
]


def _setup(name, idx, dtype):
    if name == "small_alloy":
        md, m, b, th, s, tg = fixture(SMALL_ALLOY, seed=7, batch=small_alloy_batch())
    else:
        md, m, b, th, s, tg = fixture(name, idx)
    b, th, s, tg = device_inputs(dtype, b, th, s, tg)
    model = N.Model.from_dict(md, dtype=dtype)
    td = model.torch_dtype
    gb = N.Batch.from_host(b, dtype=td)
    nb = N.nep_build_neighbors(model, gb)
    ws = N.workspace(model, gb, nb)
    theta = torch.tensor(th, dtype=td, device="cuda")
    qs = torch.tensor(s, dtype=td, device="cuda")
    return md, m, b, th, s, tg, model, gb, nb, ws, theta, qs


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("name,idx,dtype", CASES)
def test_neighbor_lists_match_bruteforce(name, idx, dtype):
    _say(f"neighbors {name} {dtype}")
    md, m, b, th, s, tg, model, gb, nb, ws, theta, qs = _setup(name, idx, dtype)
    torch.cuda.synchronize()
    row = nb.row_offset.cpu().numpy()
    seg = nb.seg_count.cpu().numpy()
    js = nb.neighbor_index().numpy()
    rv = nb.pairs[: nb.num_pairs, :3].double().cpu().numpy()
    astruct = nb.atom_struct.cpu().numpy()
    T = md["num_types"]
    total = 0
    for st in range(b.num_structures):
        cell, pos, typ = b.structure(st)
        a0 = int(b.atom_offset[st])
        oi, oj, osh, orr = O.neighbors(cell, pos, md["rc_r"])
        total += len(oi)
        for i in range(len(pos)):
            gi = a0 + i
            assert astruct[gi] == st
            sel = oi == i
            got_j = js[row[gi]:row[gi + 1]] - a0
            got_r = rv[row[gi]:row[gi + 1]]
            # per-species counts and angular counts (index work: exact)
            for t in range(T):
                mask = typ[oj[sel]] == t
                d = np.linalg.norm(orr[sel][mask], axis=1)
                assert seg[gi, t, 0] == mask.sum()
                assert seg[gi, t, 1] == (d < md["rc_a"]).sum()
            # row grouped by species, angular pairs first inside each group
            off = 0
            for t in range(T):
                cnt, ang = seg[gi, t]
                blk_j, blk_r = got_j[off:off + cnt], got_r[off:off + cnt]
                assert np.all(typ[blk_j] == t)
                dist = np.linalg.norm(blk_r, axis=1)
                assert np.all(dist[:ang] < md["rc_a"] + 1e-5) and np.all(dist[ang:] >= md["rc_a"] - 1e-5)
                off += cnt
            # same multiset of (j, r_ij)
            key_g = sorted(zip(got_j.tolist(), np.round(got_r, 4).tolist()))
            key_o = sorted(zip(oj[sel].tolist(), np.round(orr[sel], 4).tolist()))
            assert [k[0] for k in key_g] == [k[0] for k in key_o]
            assert np.allclose(np.array([k[1] for k in key_g]), np.array([k[1] for k in key_o]), atol=2e-4)
    assert nb.num_pairs == total


@pytest.mark.parametrize("name,idx,dtype", CASES)
def test_forward_parity(name, idx, dtype):
    _say(f"forward {name} {dtype}")
    md, m, b, th, s, tg, model, gb, nb, ws, theta, qs = _setup(name, idx, dtype)
    E, F, W, q = N.nep_forward(model, theta, qs, gb, nb, ws, want_descriptor=True)
    Eo, Fo, Wo = O.forward(m, th, s, b)
    qo = O.descriptors(m, th, b)
    tol = TOL[dtype]
    assert rel_err(q.cpu().numpy(), qo) < tol["F"]
    assert rel_err(E.cpu().numpy(), Eo) < tol["E"]
    assert rel_err(F.double().cpu().numpy(), Fo) < tol["F"]
    assert rel_err(W.cpu().numpy(), Wo) < tol["W"]


@pytest.mark.parametrize("name,idx,dtype", CASES)
def test_loss_and_grad_parity(name, idx, dtype):
    _say(f"loss_and_grad {name} {dtype}")
    md, m, b, th, s, tg, model, gb, nb, ws, theta, qs = _setup(name, idx, dtype)
    Et, Ft, Wt = tg
    hv = np.ones(b.num_structures, np.uint8)
    hv[::3] = 0
    lam = (1.0, 1.0, 0.1)
    targets = N.Targets(Et, Ft, Wt, has_virial=hv, lambdas=lam, dtype=model.torch_dtype)
    loss, g, E, F, W = N.nep_loss_and_grad(model, theta, qs, gb, nb, targets, ws, want_predictions=True)
    lo, go, Eo, Fo, Wo = O.loss_and_grad(m, th, s, b, Et, Ft, Wt, lam, has_virial=hv, nthreads=8)
    tol = TOL[dtype]
    assert rel_err(loss.cpu().numpy(), lo) < tol["L"]
    assert rel_err(E.cpu().numpy(), Eo) < tol["E"]
    assert rel_err(F.double().cpu().numpy(), Fo) < tol["F"]
    assert rel_err(W.cpu().numpy(), Wo) < tol["W"]
    assert rel_err(g.double().cpu().numpy(), go) < tol["G"]


@pytest.mark.parametrize("name,idx,dtype", [CASES[0], CASES[3], CASES[4]])
def test_backward_vjp_parity(name, idx, dtype):
    _say(f"backward {name} {dtype}")
    md, m, b, th, s, tg, model, gb, nb, ws, theta, qs = _setup(name, idx, dtype)
    rng = np.random.default_rng(11)
    dE = rng.normal(size=b.num_structures)
    dF = rng.normal(size=(b.num_atoms, 3))
    dW = rng.normal(size=(b.num_structures, 9))
    g = N.nep_backward(model, theta, qs, gb, nb, torch.tensor(dE, device="cuda"),
                       torch.tensor(dF, device="cuda"), torch.tensor(dW, device="cuda"), ws)
    go = O.vjp(m, th, s, b, dE, dF, dW)
    assert rel_err(g.double().cpu().numpy(), go) < TOL[dtype]["G"]


def test_full_bench_workload_fp32():
    """The whole 256-structure uneven fcc batch, in the launch configuration the benchmark times."""
    _say("full fcc_uneven_256 f32")
    md, m, b, th, s, tg, model, gb, nb, ws, theta, qs = _setup("fcc_uneven_256", None, "f32")
    Et, Ft, Wt = tg
    targets = N.Targets(Et, Ft, Wt, lambdas=(1.0, 1.0, 0.1))
    loss, g, E, F, W = N.nep_loss_and_grad(model, theta, qs, gb, nb, targets, ws, want_predictions=True)
    lo, go, Eo, Fo, Wo = O.loss_and_grad(m, th, s, b, Et, Ft, Wt, (1.0, 1.0, 0.1), nthreads=16)
    assert rel_err(E.cpu().numpy(), Eo) < 1e-5
    assert rel_err(F.double().cpu().numpy(), Fo) < 1e-4
    assert rel_err(W.cpu().numpy(), Wo) < 1e-4
    assert rel_err(loss.cpu().numpy(), lo) < 1e-5
    assert rel_err(g.double().cpu().numpy(), go) < 1e-4


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_descriptor_scale_parity(dtype):
    md, m, b, th, s, tg, model, gb, nb, ws, theta, qs = _setup("fcc_uneven_256", list(range(6)), dtype)
    q = N.nep_descriptors(model, theta, gb, nb, ws)
    sg = N.nep_descriptor_scale(q)
    assert rel_err(sg.double().cpu().numpy(), s) < (1e-9 if dtype == "f64" else 1e-4)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("mode", ["paper", "torch", "off"])
def test_adam_parity(dtype, mode):
    rng = np.random.default_rng(12)
    P = 1000
    td = torch.float64 if dtype == "f64" else torch.float32
    th = rng.normal(size=P)
    cfg = N.AdamConfig(lr=5e-3, amsgrad=mode != "off", mode="torch" if mode == "torch" else "paper")
    t_th = torch.tensor(th, dtype=td, device="cuda")
    m_ = torch.zeros(P, dtype=td, device="cuda")
    v_ = torch.zeros(P, dtype=td, device="cuda")
    vm_ = torch.zeros(P, dtype=td, device="cuda")
    om = ov = ovm = np.zeros(P)
    for t in range(1, 6):
        g = rng.normal(size=P) * (0.1 + t)
        N.nep_adam_step(t_th, torch.tensor(g, dtype=td, device="cuda"), m_, v_, vm_, t, cfg)
        th, om, ov, ovm = O.adam_step(th, g, om, ov, ovm, t, lr=5e-3, mode=mode)
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert rel_err(t_th.double().cpu().numpy(), th) < tol


def test_edge_cases_single_atom_and_ragged():
    """A one-atom cell (only periodic self-images as neighbours), a two-atom cell and a
    ragged mix, FP64 against the oracle."""
    rng = np.random.default_rng(13)
    structs = [
        (np.diag([3.0, 3.1, 3.3]), np.array([[0.2, 0.1, 0.3]]), np.array([0], np.int32)),
        (np.diag([2.9, 4.0, 3.2]), np.array([[0.1, 0.2, 0.3], [1.5, 1.9, 1.7]]), np.array([0, 0], np.int32)),
        S.bcc_structure(rng, 15, a=3.2, sigma=0.15, exact_dims=(2, 2, 2)),
    ]
    b = S.pack(structs, 1)
    md, m, b, th, s, tg = fixture("bcc64x8", batch=b)
    model = N.Model.from_dict(md, dtype="f64")
    gb = N.Batch.from_host(b, dtype=torch.float64)
    nb = N.nep_build_neighbors(model, gb)
    ws = N.workspace(model, gb, nb)
    theta = torch.tensor(th, device="cuda")
    qs = torch.tensor(s, device="cuda")
    Et, Ft, Wt = tg
    loss, g, E, F, W = N.nep_loss_and_grad(model, theta, qs, gb, nb, N.Targets(Et, Ft, Wt, dtype=torch.float64),
                                           ws, want_predictions=True)
    lo, go, Eo, Fo, Wo = O.loss_and_grad(m, th, s, b, Et, Ft, Wt, (1.0, 1.0, 0.1))
    assert rel_err(E.cpu().numpy(), Eo) < 1e-9
    assert rel_err(F.cpu().numpy(), Fo) < 1e-9
    assert rel_err(g.cpu().numpy(), go) < 1e-9


def test_empty_batch():
    model = N.Model(num_types=1, rc_r=5.0, rc_a=4.0, n_max_r=4, n_max_a=4, basis_r=8, basis_a=8, hidden=30,
                    dtype="f64")
    gb = N.Batch(np.zeros((0, 3)), np.zeros(0, np.int32), np.zeros((0, 3, 3)), np.zeros(1, np.int64),
                 dtype=torch.float64)
    nb = N.nep_build_neighbors(model, gb)
    assert nb.num_pairs == 0
    P, D = N.nep_param_count(model)
    theta = torch.zeros(P, dtype=torch.float64, device="cuda")
    qs = torch.ones(D, dtype=torch.float64, device="cuda")
    tg = N.Targets(np.zeros(0), np.zeros((0, 3)), np.zeros((0, 9)), dtype=torch.float64)
    loss, g = N.nep_loss_and_grad(model, theta, qs, gb, nb, tg)
    assert torch.all(g == 0) and torch.all(loss == 0)


def test_repeatable_bitwise():
    md, m, b, th, s, tg, model, gb, nb, ws, theta, qs = _setup("fcc_uneven_256", list(range(8)), "f32")
    targets = N.Targets(*tg)
    g1 = N.nep_loss_and_grad(model, theta, qs, gb, nb, targets, ws)[1].clone()
    g2 = N.nep_loss_and_grad(model, theta, qs, gb, nb, targets, ws)[1].clone()
    assert torch.equal(g1, g2)


def test_autograd_function_matches_loss_and_grad():
    """A torch loss composed on NEPFunction's outputs back-propagates through the
    hand-written VJP to the same gradient as nep_loss_and_grad."""
    md, m, b, th, s, tg, model, gb, nb, ws, theta, qs = _setup("small_alloy", None, "f64")
    Et, Ft, Wt = (torch.tensor(x, device="cuda") for x in tg)
    th_t = theta.clone().requires_grad_(True)
    E, F, W = N.NEPFunction.apply(th_t, model, qs, gb, nb, ws)
    na = gb.counts.to("cuda").double()
    Ns, Na = gb.num_structures, gb.num_atoms
    L = (((E - Et) / na) ** 2).mean() + ((F - Ft) ** 2).sum() / (3 * Na) + \
        0.1 * (((W - Wt) / na[:, None]) ** 2).sum() / (9 * Ns)
    L.backward()
    loss, g = N.nep_loss_and_grad(model, theta, qs, gb, nb, N.Targets(*tg, dtype=torch.float64), ws)
    assert rel_err(th_t.grad.cpu().numpy(), g.cpu().numpy()) < 1e-10
    assert abs(L.item() - loss[0].item()) < 1e-12 * abs(L.item())


# The fused plan (network inside the sweeps, force pass inside the descriptor
# sweep) on every kernel shape, with the team sizes the autotuner picks there
# and the other register / LDS variants of the fused force pass (from
# registers for three-body models, through the stored rows for 4-lane teams of
# large moment blocks and for 4/5-body models).
FUSED = [
    ("bcc64x8", None, "f64", (16, 16, 16, 32, 2048, 64, 3)),
    ("alloy4_1024", [4, 0, 1, 3], "f32", (4, 4, 4, 8, 1024, 128, 3)),
    ("mixed3_4096", [0, 1, 2, 4, 5], "f32", (8, 8, 8, 16, 2048, 64, 3)),
    ("mixed3_4096", [0, 1, 2, 4, 5], "f32", (4, 4, 16, 32, 512, 32, 3)),
    ("large5_32", [20], "f32", (4, 4, 8, 16, 1024, 128, 3)),
    ("large5_32", [20], "f32", (16, 16, 4, 8, 4096, 256, 3)),
]


@pytest.mark.parametrize("name,idx,dtype,plan", FUSED)
def test_fused_plan_parity(name, idx, dtype, plan):
    _say(f"fused plan {name} {dtype} {plan}")
    md, m, b, th, s, tg, model, gb, nb, ws, theta, qs = _setup(name, idx, dtype)
    model = model.with_plan(N.Plan(*plan))
    ws = N.workspace(model, gb, nb)
    Et, Ft, Wt = tg
    lam = (1.0, 1.0, 0.1)
    targets = N.Targets(Et, Ft, Wt, lambdas=lam, dtype=model.torch_dtype)
    loss, g, E, F, W = N.nep_loss_and_grad(model, theta, qs, gb, nb, targets, ws, want_predictions=True)
    lo, go, Eo, Fo, Wo = O.loss_and_grad(m, th, s, b, Et, Ft, Wt, lam, nthreads=8)
    tol = TOL[dtype]
    assert rel_err(loss.cpu().numpy(), lo) < tol["L"]
    assert rel_err(E.cpu().numpy(), Eo) < tol["E"]
    assert rel_err(F.double().cpu().numpy(), Fo) < tol["F"]
    assert rel_err(W.cpu().numpy(), Wo) < tol["W"]
    assert rel_err(g.double().cpu().numpy(), go) < tol["G"]
    E2, F2, W2 = N.nep_forward(model, theta, qs, gb, nb, ws)
    assert rel_err(E2.cpu().numpy(), Eo) < tol["E"]
    assert rel_err(F2.double().cpu().numpy(), Fo) < tol["F"]
    assert rel_err(W2.cpu().numpy(), Wo) < tol["W"]
    rng = np.random.default_rng(11)
    dE = rng.normal(size=b.num_structures)
    dF = rng.normal(size=(b.num_atoms, 3))
    dW = rng.normal(size=(b.num_structures, 9))
    gv = N.nep_backward(model, theta, qs, gb, nb, torch.tensor(dE, device="cuda"),
                        torch.tensor(dF, device="cuda"), torch.tensor(dW, device="cuda"), ws)
    assert rel_err(gv.double().cpu().numpy(), O.vjp(m, th, s, b, dE, dF, dW)) < tol["G"]


@pytest.mark.parametrize("bad", [3, -1])
def test_build_rejects_species_out_of_range(bad):
    """A species outside [0, T) is found on the device and reported with the
    pair count; the lists of a valid batch built afterwards are unaffected."""
    _say(f"neighbors species {bad}")
    from dataclasses import replace

    md, m, b, th, s, tg = fixture(SMALL_ALLOY, seed=7, batch=small_alloy_batch())
    model = N.Model.from_dict(md, dtype="f32")
    typ = np.array(b.types, copy=True)
    typ[len(typ) // 2] = bad
    with pytest.raises(N.NepError) as e:
        N.nep_build_neighbors(model, N.Batch.from_host(replace(b, types=typ)))
    assert e.value.code == N.nep.NEP_ERR_INVALID_ARG and "species" in str(e.value)
    ok = N.nep_build_neighbors(model, N.Batch.from_host(b))
    ref = N.nep_build_neighbors(model, N.Batch.from_host(b))
    assert ok.num_pairs == ref.num_pairs > 0
    assert torch.equal(ok.row_offset, ref.row_offset) and torch.equal(ok.reverse[:ok.num_pairs], ref.reverse[:ref.num_pairs])


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("amsgrad,mode", [(False, "paper"), (True, "paper"), (True, "torch")])
def test_train_step_matches_loss_grad_then_adam(dtype, amsgrad, mode):
    """nep_train_step is nep_loss_and_grad followed by nep_adam_step, bit for bit,
    over three steps, under the plain and the fused launch plans."""
    _say(f"train step {dtype} amsgrad={amsgrad} {mode}")
    md, m, b, th, s, tg, model, gb, nb, ws, theta, qs = _setup("small_alloy", None, dtype)
    targets = N.Targets(*tg, lambdas=(1.0, 1.0, 0.1), dtype=model.torch_dtype)
    cfg = N.AdamConfig(lr=1e-2, amsgrad=amsgrad, mode=mode)
    for plan in (None, N.Plan(8, 8, 8, 8, 2048, 64, 3)):
        mdl = model.with_plan(plan)
        w = N.workspace(mdl, gb, nb)
        a = [theta.clone()] + [torch.zeros_like(theta) for _ in range(3)]
        f = [theta.clone()] + [torch.zeros_like(theta) for _ in range(3)]
        for t in (1, 2, 3):
            la, ga = N.nep_loss_and_grad(mdl, a[0], qs, gb, nb, targets, w)
            ga = ga.clone()
            N.nep_adam_step(a[0], ga, a[1], a[2], a[3], t, cfg)
            lf, gf = N.nep_train_step(mdl, f[0], qs, gb, nb, targets, f[1], f[2], f[3], t, cfg, w)
            torch.cuda.synchronize()
            assert torch.equal(la, lf) and torch.equal(ga, gf)
            for x, y in zip(a, f):
                assert torch.equal(x, y)
        assert not torch.equal(a[0], theta)  # the parameters did move
