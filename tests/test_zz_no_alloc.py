"""nep_train_step_noalloc (the allocation-free training step whose workspace is
the library's static device array) against nep_train_step with a caller
workspace: identical loss, gradient and updated parameters and moments, on two
calls in a row, the second with a smaller batch (the array keeps the first
call's contents). A batch that needs more workspace than the array holds is
refused on the host."""

import ctypes as C

import numpy as np
import pytest
import torch

from helpers import device_inputs, fixture

N = pytest.importorskip("paper_2606_19557_amd")
from paper_2606_19557_amd import nep as NP  # noqa: E402


def _lib_or_skip():
    import os

    if not os.path.exists(NP.LIB_PATH):
        pytest.skip("libnep.so not built")
    return NP.lib()


def test_noalloc_refuses_oversize_batch_on_host():
    """The size check runs before any device call (no GPU needed): the 32 large
    cells (277,380 atoms, 24.9 M pairs) need ~1.8 GiB of workspace."""
    L = _lib_or_skip()
    from synth import WORKLOADS

    model = NP.Model.from_dict(WORKLOADS["large5_32"].model, dtype="f32")
    na, npairs, ns = 277380, 24868090, 32
    need = NP.nep_workspace_size(model, ns, na, npairs)
    assert need > (128 << 20)
    fake = C.c_void_p(0x1000)  # never dereferenced: the call returns before touching memory
    b = NP.c_batch(ns, na, fake, fake, fake, fake)
    nb = NP.c_neighbors(npairs, fake, fake, fake, fake, fake, fake, fake, npairs, npairs // 2)
    tg = NP.c_targets(fake, fake, fake, None, 1.0, 1.0, 0.1)
    cfg = NP.AdamConfig().c()
    mm = model.c()
    code = L.nep_train_step_noalloc(C.byref(mm), fake, fake, C.byref(b), C.byref(nb), C.byref(tg), fake, fake, fake,
                                    1, C.byref(cfg), fake, fake, None)
    assert code == NP.NEP_ERR_WORKSPACE
    msg = L.nep_last_error().decode()
    assert "128" in msg or str(128 << 20) in msg, msg


def _inputs(indices, dtype):
    md, m, b, th, s, tg = fixture("fcc_uneven_256", indices)
    b, th, s, tg = device_inputs(dtype, b, th, s, tg)
    model = N.Model.from_dict(md, dtype=dtype)
    td = model.torch_dtype
    gb = N.Batch.from_host(b, dtype=td)
    nb = N.nep_build_neighbors(model, gb)
    targets = N.Targets(*tg, dtype=td, device="cuda")
    theta = torch.tensor(th, dtype=td, device="cuda")
    qs = torch.tensor(s, dtype=td, device="cuda")
    return model, gb, nb, targets, theta, qs


def _state(theta, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    P = theta.numel()
    m = (0.01 * torch.randn(P, generator=g, dtype=torch.float64)).to(theta)
    v = (1e-4 * torch.rand(P, generator=g, dtype=torch.float64)).to(theta)
    vmax = v * 1.5
    return [theta.clone(), m, v, vmax]


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_matches_train_step_twice(dtype):
    cfg = N.AdamConfig(lr=1e-3)
    for call, idx in enumerate((list(range(48)), list(range(40, 52)))):
        print(f"noalloc {dtype} call {call}: {len(idx)} structures", flush=True)
        model, gb, nb, targets, theta, qs = _inputs(idx, dtype)
        ws = N.workspace(model, gb, nb)
        assert ws.numel() <= (128 << 20)
        P = theta.numel()
        ref = _state(theta, 11 + call)
        got = [x.clone() for x in ref]
        t = 3 + call
        loss_r, grad_r = N.nep_train_step(model, *ref[:1], qs, gb, nb, targets, *ref[1:], t, cfg, ws)
        grad = torch.full((P,), float("nan"), dtype=theta.dtype, device="cuda")
        loss = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
        N.nep_train_step_noalloc(model, got[0], qs, gb, nb, targets, got[1], got[2], got[3], t, cfg, grad, loss)
        torch.cuda.synchronize()
        # the same kernels on the same inputs: every output bitwise equal
        assert torch.equal(loss, loss_r), (loss, loss_r)
        assert torch.equal(grad, grad_r)
        for name, a, r in zip(("theta", "m", "v", "vmax"), got, ref):
            assert torch.equal(a, r), name
        assert np.isfinite(loss.cpu().numpy()).all()
