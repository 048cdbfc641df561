"""NEP energy, forces, virial and loss in plain PyTorch ops, differentiated by
autograd: forces come from torch.autograd.grad(E, r_ij, create_graph=True) and
the parameter gradient from a second backward pass through them (the
"autograd force training" the paper compares its analytic gradients with,
Results, "Training efficiency").

Descriptor definitions (TorchNEP paper, Methods): Chebyshev basis with cosine
cutoff (Eqs. 17-18), radial q_n (Eqs. 15-16), angular moments with real
orthonormal harmonics (Eq. 19), q_nl = sum_m A_nlm^2 (Eq. 20), 4-body term
kappa tr(S^3) with S = sum_j g_n (u u^T - I/3) (equal to the (2 2 2) Wigner-3j
contraction of the complex l = 2 moments), 5-body term q_n1^2; network Eq. (3);
loss Eqs. (4)-(7). Parameter and descriptor order as in include/nep.h.
"""

from __future__ import annotations

import math

import torch

KAPPA4 = -4.5 * math.sqrt(2.0 / 35.0) * (5.0 / (4.0 * math.pi)) ** 1.5


def pairs_from_csr(row_offset, neighbor_index, pair_vectors):
    """(i, j, r_ij) from CSR neighbour lists."""
    counts = torch.diff(row_offset)
    i = torch.repeat_interleave(torch.arange(len(counts), device=row_offset.device), counts)
    return i, neighbor_index.to(row_offset.device), pair_vectors


def _chebyshev(d, rc, K):
    """f_k(d), k < K: (T_k(x) + 1)/2 * (cos(pi d/rc) + 1)/2, zero beyond rc."""
    x = 2.0 * (d / rc - 1.0) ** 2 - 1.0
    fc = torch.where(d < rc, 0.5 * (torch.cos(math.pi * d / rc) + 1.0), torch.zeros_like(d))
    T = [torch.ones_like(d), x]
    for _ in range(2, K):
        T.append(2.0 * x * T[-1] - T[-2])
    return torch.stack([0.5 * (t + 1.0) * fc for t in T[:K]], dim=-1)


def _real_harmonics(u, L):
    """Real orthonormal Y_lm(u), l = 1..L (L <= 4), columns ordered m = -l..l."""
    x, y, z = u[:, 0], u[:, 1], u[:, 2]
    pi = math.pi
    out = [math.sqrt(3 / (4 * pi)) * y, math.sqrt(3 / (4 * pi)) * z, math.sqrt(3 / (4 * pi)) * x]
    if L >= 2:
        out += [0.5 * math.sqrt(15 / pi) * x * y, 0.5 * math.sqrt(15 / pi) * y * z,
                0.25 * math.sqrt(5 / pi) * (3 * z * z - 1), 0.5 * math.sqrt(15 / pi) * x * z,
                0.25 * math.sqrt(15 / pi) * (x * x - y * y)]
    if L >= 3:
        out += [0.25 * math.sqrt(35 / (2 * pi)) * y * (3 * x * x - y * y), 0.5 * math.sqrt(105 / pi) * x * y * z,
                0.25 * math.sqrt(21 / (2 * pi)) * y * (5 * z * z - 1), 0.25 * math.sqrt(7 / pi) * (5 * z ** 3 - 3 * z),
                0.25 * math.sqrt(21 / (2 * pi)) * x * (5 * z * z - 1), 0.25 * math.sqrt(105 / pi) * z * (x * x - y * y),
                0.25 * math.sqrt(35 / (2 * pi)) * x * (x * x - 3 * y * y)]
    if L >= 4:
        out += [0.75 * math.sqrt(35 / pi) * x * y * (x * x - y * y),
                0.75 * math.sqrt(35 / (2 * pi)) * y * z * (3 * x * x - y * y),
                0.75 * math.sqrt(5 / pi) * x * y * (7 * z * z - 1),
                0.75 * math.sqrt(5 / (2 * pi)) * y * z * (7 * z * z - 3),
                (3 / 16) * math.sqrt(1 / pi) * (35 * z ** 4 - 30 * z * z + 3),
                0.75 * math.sqrt(5 / (2 * pi)) * x * z * (7 * z * z - 3),
                0.375 * math.sqrt(5 / pi) * (x * x - y * y) * (7 * z * z - 1),
                0.75 * math.sqrt(35 / (2 * pi)) * x * z * (x * x - 3 * y * y),
                (3 / 16) * math.sqrt(35 / pi) * (x * x * (x * x - 3 * y * y) - y * y * (3 * x * x - y * y))]
    return torch.stack(out, dim=-1)


class AutogradNEP:
    """NEP of one model on one packed batch with cached neighbour pairs."""

    def __init__(self, model: dict, types, atom_offset, pair_i, pair_j, pair_r):
        self.m = dict(model)
        T = model["num_types"]
        self.T = T
        self.NR, self.NA = model["n_max_r"] + 1, model["n_max_a"] + 1
        self.KR, self.KA = model["basis_r"] + 1, model["basis_a"] + 1
        self.L = model["l_max"]
        self.h4, self.h5 = model.get("l_max_4b", 0) == 2, model.get("l_max_5b", 0) == 1
        self.H = model["hidden"]
        self.D = self.NR + self.NA * (self.L + self.h4 + self.h5)
        self.offA = T * T * self.NR * self.KR
        self.offN = self.offA + T * T * self.NA * self.KA
        self.P = self.offN + T * (self.D + 2) * self.H + 1
        dev = pair_r.device
        self.types = types.to(dev).long()
        self.atom_offset = atom_offset.to(dev).long()
        self.Na = len(self.types)
        self.Ns = len(self.atom_offset) - 1
        counts = torch.diff(self.atom_offset)
        self.na_s = counts.to(pair_r.dtype)
        self.struct_of = torch.repeat_interleave(torch.arange(self.Ns, device=dev), counts)
        self.pi, self.pj, self.r = pair_i.to(dev).long(), pair_j.to(dev).long(), pair_r
        d = self.r.norm(dim=1)
        self.ang = torch.nonzero(d < model["rc_a"]).flatten()
        ti, tj = self.types[self.pi], self.types[self.pj]
        self.tpair = ti * T + tj
        self.tpair_a = self.tpair[self.ang]
        self.tpair_groups = self._groups(self.tpair)
        self.tpair_a_groups = self._groups(self.tpair_a)

    def _groups(self, tp):
        """Pair indices of each species pair present (None when there is one species)."""
        if self.T == 1:
            return None
        return [(int(ab), torch.nonzero(tp == ab).flatten()) for ab in torch.unique(tp).tolist()]

    @staticmethod
    def _expand(f, c, groups):
        """g[p, n] = sum_k c[ab(p), n, k] f[p, k], one matmul per species pair."""
        if groups is None:
            return f @ c[0].T
        g = torch.zeros(f.shape[0], c.shape[1], dtype=f.dtype, device=f.device)
        for ab, idx in groups:
            g = g.index_put((idx,), f[idx] @ c[ab].T)
        return g

    # -------------------------------------------------------------- pieces

    def descriptors(self, theta, r):
        T, NR, NA, KR, KA, L = self.T, self.NR, self.NA, self.KR, self.KA, self.L
        cR = theta[: self.offA].reshape(T * T, NR, KR)
        cA = theta[self.offA: self.offN].reshape(T * T, NA, KA)
        d = r.norm(dim=1)
        fR = _chebyshev(d, self.m["rc_r"], KR)  # [p, KR]
        gR = self._expand(fR, cR, self.tpair_groups)
        q_rad = torch.zeros(self.Na, NR, dtype=r.dtype, device=r.device).index_add(0, self.pi, gR)
        ra = r[self.ang]
        da = d[self.ang]
        u = ra / da[:, None]
        fA = _chebyshev(da, self.m["rc_a"], KA)
        gA = self._expand(fA, cA, self.tpair_a_groups)  # [pa, NA]
        Y = _real_harmonics(u, L)  # [pa, LM]
        A = torch.zeros(self.Na, NA, Y.shape[1], dtype=r.dtype, device=r.device)
        A = A.index_add(0, self.pi[self.ang], gA[:, :, None] * Y[:, None, :])
        parts = [q_rad]
        for l in range(1, L + 1):
            parts.append((A[:, :, l * l - 1:(l + 1) ** 2 - 1] ** 2).sum(-1))
        if self.h4:
            Tm = u[:, :, None] * u[:, None, :] - torch.eye(3, dtype=r.dtype, device=r.device) / 3.0
            Smat = torch.zeros(self.Na, NA, 3, 3, dtype=r.dtype, device=r.device)
            Smat = Smat.index_add(0, self.pi[self.ang], gA[:, :, None, None] * Tm[:, None, :, :])
            parts.append(KAPPA4 * torch.einsum("anij,anjk,anki->an", Smat, Smat, Smat))
        if self.h5:
            parts.append(parts[1] ** 2)  # q_n1^2
        return torch.cat(parts, dim=1)

    def site_energies(self, theta, q, q_scale):
        T, H, D = self.T, self.H, self.D
        net = theta[self.offN: self.offN + T * (D + 2) * H].reshape(T, (D + 2) * H)
        W0 = net[:, :H * D].reshape(T, H, D)
        b0 = net[:, H * D:H * D + H]
        w1 = net[:, H * D + H:]
        b1 = theta[-1]
        qs = q * q_scale
        E = torch.zeros(self.Na, dtype=q.dtype, device=q.device)
        for t in range(T):
            sel = torch.nonzero(self.types == t).flatten()
            if len(sel) == 0:
                continue
            a = qs[sel] @ W0[t].T - b0[t]
            E = E.index_put((sel,), torch.tanh(a) @ w1[t] - b1)
        return E

    # ------------------------------------------------------------- public

    def energy_forces_virial(self, theta, q_scale, create_graph=False):
        r = self.r.detach().clone().requires_grad_(True)
        q = self.descriptors(theta, r)
        Ei = self.site_energies(theta, q, q_scale)
        E = torch.zeros(self.Ns, dtype=Ei.dtype, device=Ei.device).index_add(0, self.struct_of, Ei)
        (h,) = torch.autograd.grad(Ei.sum(), r, create_graph=create_graph)  # h_ij = dE_i/dr_ij
        F = torch.zeros(self.Na, 3, dtype=h.dtype, device=h.device).index_add(0, self.pi, h)
        F = F.index_add(0, self.pj, -h)
        outer = -(r[:, :, None] * h[:, None, :]).reshape(-1, 9)
        W = torch.zeros(self.Ns, 9, dtype=h.dtype, device=h.device).index_add(0, self.struct_of[self.pi], outer)
        if not create_graph:
            return E.detach(), F.detach(), W.detach()
        return E, F, W

    def loss(self, theta, q_scale, E_t, F_t, W_t, lambdas=(1.0, 1.0, 0.1), has_virial=None):
        E, F, W = self.energy_forces_virial(theta, q_scale, create_graph=True)
        # structures without atoms take no part (N_s and N_v count structures with atoms)
        nz = self.na_s > 0
        dE = (((E - E_t)[nz] / self.na_s[nz]) ** 2).mean()
        dF = ((F - F_t) ** 2).sum() / (3 * self.Na)
        rw = ((W - W_t)[nz] / self.na_s[nz][:, None]) ** 2
        hv = (has_virial[nz] if has_virial is not None else torch.ones_like(self.na_s[nz])).to(rw.dtype)
        nv = hv.sum()
        dV = (rw.sum(1) * hv).sum() / (9 * nv) if nv > 0 else rw.sum() * 0
        L = lambdas[0] * dE + lambdas[1] * dF + lambdas[2] * dV
        return L, torch.stack([L, dE, dF, dV]).detach()

    def loss_and_grad(self, theta, q_scale, E_t, F_t, W_t, lambdas=(1.0, 1.0, 0.1), has_virial=None):
        th = theta.detach().clone().requires_grad_(True)
        L, parts = self.loss(th, q_scale, E_t, F_t, W_t, lambdas, has_virial)
        (g,) = torch.autograd.grad(L, th)
        return parts, g
