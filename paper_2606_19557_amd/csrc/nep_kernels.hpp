// NEP kernels for gfx950.
//
// Pair sweeps (descriptor, force, tangent, coefficient gradient) give each
// atom a team of S consecutive lanes: the lanes stride over the atom's CSR row
// (grouped by neighbour species, angular pairs first in each group), keep
// their partial sums in registers, and reduce across the team with
// cross-lane shuffles. Forces use the gather form (each atom sums both
// directions of its own pairs), so no force atomics are needed.
//
// Per-atom kernels (network forward / backward) run one lane per atom.
// Reductions over atoms into parameter gradients go through per-block partial
// rows that a final kernel sums in a fixed order in double precision.
#pragma once

#include "nep_device.hpp"

namespace nep {

template <typename R>
__device__ __forceinline__ R load_theta(const R* __restrict__ th, long idx) {
    return th[idx];
}

// Occupancy requests of the pair sweeps (waves per SIMD that their registers
// must allow; 1 leaves the allocation unconstrained). FP32 sweeps of large
// moment blocks (N_A x 24 > 120) come out a few registers above 256, i.e.
// one wave per SIMD; asking for two costs at most a small spill. The tangent
// sweep of small blocks with teams of 8 fits 3 waves with 28 bytes per lane
// spilled, which measures faster than 2 waves without. The coefficient
// sweep with 16- or 32-lane teams is a few registers above 3 waves. FP64
// sweeps would spill hundreds of bytes per lane and are left alone.
template <typename R, class Sh, int S>
struct SweepWaves {
    static constexpr bool f32 = sizeof(R) == 4;
    static constexpr bool big = Sh::NA * Sh::LM > 120;
    static constexpr int descriptor = (f32 && big) ? 2 : 1;
    static constexpr int tangent = !f32 ? 1 : big ? 2 : S == 8 ? 3 : 1;
    static constexpr int coeff_grad = (f32 && S >= 16) ? 3 : 1;
};

// Work item b of the species-sorted atom list: chunk k of species t, i.e.
// sorted positions [soff[t] + k*chunk, min(soff[t+1], soff[t] + (k+1)*chunk)).
// Items beyond the last chunk get t = -1.
__device__ __forceinline__ void species_chunk(const int64_t* __restrict__ soff, int T, int chunk, int b, int* t_out,
                                              long* lo, long* hi) {
    *t_out = -1;
    for (int t = 0; t < T; ++t) {
        const long n = soff[t + 1] - soff[t];
        const int c = int((n + chunk - 1) / chunk);
        if (b < c) {
            *t_out = t;
            *lo = soff[t] + long(b) * chunk;
            *hi = min(soff[t + 1], *lo + chunk);
            return;
        }
        b -= c;
    }
}

// ------------------------------------------------ network inside the sweeps

// The per-species network of one atom split over its team (the fused plan):
// lane l takes hidden units mu = l, l + S, ... and the team sums the rest.
// Per-unit rows (t, alpha, beta, gamma) are indexed by atom.

// Eqs. 2-3: E_i = sum_mu w1 tanh(W0 (s q) - b0) - b1 and e = dE_i/dq; every
// lane holds the atom's descriptor qv.
template <typename R, int D, int S>
__device__ __forceinline__ void team_network_forward(int lane, const Dims& dm, const R* __restrict__ theta, int a,
                                                     const R* __restrict__ qscale, const R (&qv)[D], long i,
                                                     R* __restrict__ E_out, R* __restrict__ e_out,
                                                     R* __restrict__ t_out, R (&e)[D]) {
    const int H = dm.H;
    const R* __restrict__ W0 = theta + dm.offN + (long)a * (D + 2) * H;
    const R* __restrict__ b0 = W0 + (long)H * D;
    const R* __restrict__ w1 = b0 + H;
    R qs[D], ev[D];
#pragma unroll
    for (int v = 0; v < D; ++v) {
        qs[v] = qscale[v] * qv[v];
        ev[v] = R(0);
    }
    R E = R(0);
    // two hidden units per step (mu and mu + S), so that both weight rows
    // are in flight together; a missing second unit reads the first's row
    for (int mu = lane; mu < H; mu += 2 * S) {
        const bool two = mu + S < H;
        const int mu2 = two ? mu + S : mu;
        const R* __restrict__ w = W0 + (long)mu * D;
        const R* __restrict__ w2 = W0 + (long)mu2 * D;
        R acc = -b0[mu], acc2 = -b0[mu2];
#pragma unroll
        for (int v = 0; v < D; ++v) {
            acc += w[v] * qs[v];
            acc2 += w2[v] * qs[v];
        }
        const R t = tanh_<R>(acc), t2 = tanh_<R>(acc2);
        const R wm = w1[mu], wm2 = two ? w1[mu2] : R(0);
        E += wm * t;
        E += wm2 * t2;
        const R c = wm * (R(1) - t * t), c2 = wm2 * (R(1) - t2 * t2);
#pragma unroll
        for (int v = 0; v < D; ++v) {
            // two separate accumulations: each one fused multiply-add
            ev[v] += w[v] * c;
            ev[v] += w2[v] * c2;
        }
        t_out[i * H + mu] = t;
        if (two) t_out[i * H + mu2] = t2;
    }
    E = team_sum<S>(E);
#pragma unroll
    for (int v = 0; v < D; ++v) ev[v] = team_sum<S>(ev[v]);
    if (lane == 0) E_out[i] = E - theta[dm.offB1];
#pragma unroll
    for (int v = 0; v < D; ++v) {
        e[v] = qscale[v] * ev[v];  // every lane
        if (v % S == lane) e_out[i * D + v] = e[v];
    }
}

// Loads of the first step of team_network_backward (units mu = lane and
// lane + S, their weight rows, activations, the atom's e entries and ebar),
// issued by the caller ahead of other work so their latency overlaps it.
template <typename R, int D, int S>
struct NetBackFirst {
    static constexpr int OWNV = (D + S - 1) / S;
    R w[D], w2[D], t, t2, wm, wm2, eo[OWNV], eb;
    bool two;
    __device__ __forceinline__ void load(int lane, const Dims& dm, const R* __restrict__ theta, int a,
                                         const R* __restrict__ t_in, const R* __restrict__ e_in,
                                         const double* __restrict__ ebar_s, int s, long i) {
        const int H = dm.H;
        const R* __restrict__ W0 = theta + dm.offN + (long)a * (D + 2) * H;
        const R* __restrict__ w1 = W0 + (long)H * D + H;
        const int mu = lane < H ? lane : 0;  // lanes past H run one discarded step
        two = lane + S < H;
        const int mu2 = two ? lane + S : mu;
#pragma unroll
        for (int v = 0; v < D; ++v) {
            w[v] = W0[(long)mu * D + v];
            w2[v] = W0[(long)mu2 * D + v];
        }
        t = t_in[i * H + mu];
        t2 = t_in[i * H + mu2];
        wm = lane < H ? w1[mu] : R(0);
        wm2 = two ? w1[mu2] : R(0);
#pragma unroll
        for (int o = 0; o < OWNV; ++o) eo[o] = lane + S * o < D ? e_in[i * D + lane + S * o] : R(0);
        eb = R(ebar_s[s]);
    }
};

// The Hessian-vector product and weight-gradient factors of the force/virial
// adjoint for one atom (as the network backward pass): da = W0 (s dq),
// alpha = w1 s'(ebar - 2 t da), beta = w1 s', gamma = ebar t + s' da,
// abar = ebar e + s (W0^T (-2 w1 t s' da)); every lane holds dq. Two hidden
// units per step (mu and mu + S); the first step's operands come in `f`.
template <typename R, int D, int S>
__device__ __forceinline__ void team_network_backward(int lane, const Dims& dm, const R* __restrict__ theta, int a,
                                                      const R* __restrict__ qscale, const R (&dq)[D], long i,
                                                      const NetBackFirst<R, D, S>& f, const R* __restrict__ t_in,
                                                      R* __restrict__ abar_out, R* __restrict__ alpha_out,
                                                      R* __restrict__ beta_out, R* __restrict__ gamma_out) {
    const int H = dm.H;
    const R* __restrict__ W0 = theta + dm.offN + (long)a * (D + 2) * H;
    const R* __restrict__ w1 = W0 + (long)H * D + H;
    const R eb = f.eb;
    R dk[D], z[D];
#pragma unroll
    for (int v = 0; v < D; ++v) {
        dk[v] = qscale[v] * dq[v];
        z[v] = R(0);
    }
    // one step: units mu (and mu2 when `two`), rows read through wr / wr2
    auto step = [&](int mu, int mu2, bool two, R t, R t2, R wm, R wm2, auto wr, auto wr2) {
        R da = R(0), da2 = R(0);
#pragma unroll
        for (int v = 0; v < D; ++v) {
            da += wr(v) * dk[v];
            da2 += wr2(v) * dk[v];
        }
        const R sp = R(1) - t * t, sp2 = R(1) - t2 * t2;
        alpha_out[i * H + mu] = wm * sp * (eb - R(2) * t * da);
        beta_out[i * H + mu] = wm * sp;
        gamma_out[i * H + mu] = eb * t + sp * da;
        if (two) {
            alpha_out[i * H + mu2] = wm2 * sp2 * (eb - R(2) * t2 * da2);
            beta_out[i * H + mu2] = wm2 * sp2;
            gamma_out[i * H + mu2] = eb * t2 + sp2 * da2;
        }
        const R c = R(-2) * wm * t * sp * da, c2 = R(-2) * wm2 * t2 * sp2 * da2;
#pragma unroll
        for (int v = 0; v < D; ++v) {
            z[v] += wr(v) * c;
            z[v] += wr2(v) * c2;
        }
    };
    if (lane < H)
        step(lane, f.two ? lane + S : lane, f.two, f.t, f.t2, f.wm, f.wm2, [&](int v) { return f.w[v]; },
             [&](int v) { return f.w2[v]; });
    for (int mu = lane + 2 * S; mu < H; mu += 2 * S) {
        const bool two = mu + S < H;
        const int mu2 = two ? mu + S : mu;
        const R* __restrict__ w = W0 + (long)mu * D;
        const R* __restrict__ w2 = W0 + (long)mu2 * D;
        step(mu, mu2, two, t_in[i * H + mu], t_in[i * H + mu2], w1[mu], two ? w1[mu2] : R(0),
             [&](int v) { return w[v]; }, [&](int v) { return w2[v]; });
    }
#pragma unroll
    for (int v = 0; v < D; ++v) z[v] = team_sum<S>(z[v]);
#pragma unroll
    for (int v = 0; v < D; ++v)
        if (v % S == lane) abar_out[i * D + v] = eb * f.eo[v / S] + qscale[v] * z[v];
}

// defined further down, used by the descriptor sweep when it also runs the
// force pass
template <typename R, class Sh, int S, bool WITH_BP>
__device__ __forceinline__ void moment_adjoints(int lane, const R* __restrict__ A, const R* __restrict__ dA,
                                                const R* __restrict__ e, const R* __restrict__ ab, R* B, R* Bp);
template <typename R, class Sh, int S>
__device__ __forceinline__ void force_pass(int lane, const Dims& dm, const R* __restrict__ theta, int i, bool live,
                                           int a, const int64_t* __restrict__ row, const int* __restrict__ seg,
                                           const Rec<R>* __restrict__ pairs, const int* __restrict__ reverse,
                                           const R* Bk, const R* __restrict__ ei, Rec<R>* __restrict__ h_in,
                                           R* __restrict__ Fown_out, R* __restrict__ Wat_out);

// LDS per team of the descriptor sweep: the moment exchange, grown when the
// sweep also runs the force pass (the team's B = dE/dA, N_A x 24 values,
// and e's N_R radial entries) by whole 128-byte steps, so team blocks keep
// the exchange's bank pattern.
template <typename R, int NA, int LM, int NR, int S, int FUSE>
struct DescTeamLds {
    static constexpr int TF = MomentExchange<R, NA, LM, S>::TEAM_FLOATS, STEP = 128 / int(sizeof(R));
    static constexpr int need = NA * LM + NR;  // B, then e's radial entries
    static constexpr int floats = (FUSE < 2 || TF >= need) ? TF : TF + (need - TF + STEP - 1) / STEP * STEP;
};

// ------------------------------------------------------------------ descriptor

// q (radial, Eqs. 15-16; angular invariants, Eqs. 19-20 and the 4/5-body
// contractions), the angular moments A[n][lm], and the per-neighbour-species
// radial basis sums S0[b][k] = sum_{j in b} f_k(r_ij) used by the gradient.
// Angular pairs are processed S at a time by the team and their (g_n, Y_lm)
// exchanged through LDS; each lane owns the moments lm = lane + S*o.
// FUSE >= 1: the team then evaluates the atom's network (E_i, e_i, t_i);
// FUSE == 2: and runs the atom's force pass (h, own-direction F, virial).
template <typename R, class Sh, int S, int FUSE>
__global__ void __launch_bounds__(kBlock, (SweepWaves<R, Sh, S>::descriptor))
k_descriptor(const Dims dm, const R* __restrict__ theta, const int* __restrict__ order,
             const int64_t* __restrict__ soff, int Na,
             const int64_t* __restrict__ row, const int* __restrict__ seg, const Rec<R>* __restrict__ pairs,
             R* __restrict__ q_out, R* __restrict__ A_out, R* __restrict__ S0_out, const R* __restrict__ qscale,
             R* __restrict__ E_out, R* __restrict__ e_out, R* __restrict__ t_out, const int* __restrict__ reverse,
             Rec<R>* __restrict__ h_in, R* __restrict__ Fown_out, R* __restrict__ Wat_out) {
    constexpr int NR = Sh::NR, NA = Sh::NA, KR = Sh::KR, KA = Sh::KA, LM = Sh::LM, D = Sh::D, L = Sh::L;
    using X = MomentExchange<R, NA, LM, S>;
    constexpr int OWN = X::OWN, TEAMS = kBlock / S, XR = DescTeamLds<R, NA, LM, NR, S, FUSE>::floats;
    __shared__ R xbuf[TEAMS * XR];
    const int team = threadIdx.x / S, lane = threadIdx.x % S;
    R* tbuf = xbuf + team * XR;
    const int T = dm.T;
    // a block takes TEAMS atoms of one species from the species-sorted list:
    // the species, and with it every coefficient address, is uniform over the
    // block (scalar loads)
    int a;
    long lo = 0, hi = 0;
    species_chunk(soff, T, TEAMS, xcd_tile(blockIdx.x, gridDim.x), &a, &lo, &hi);
    if (a < 0) return;
    const bool live = lo + team < hi;
    const int i = live ? order[lo + team] : 0;
    const R rcR = R(dm.rcR), rcA = R(dm.rcA), irR = R(1.0 / dm.rcR), irA = R(1.0 / dm.rcA);
    int64_t p = live ? row[i] : 0;
    // without the network in the sweep a lane needs only the radial rows it
    // stores, n = lane + S o: NR_OWN of them
    constexpr int NR_OWN = FUSE == 0 ? (NR + S - 1) / S : NR;
    R qR[NR_OWN];
#pragma unroll
    for (int n = 0; n < NR_OWN; ++n) qR[n] = R(0);
    R acc[NA][OWN];
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int o = 0; o < OWN; ++o) acc[n][o] = R(0);

    for (int b = 0; b < T; ++b) {
        const int tot = live ? seg[(i * T + b) * 2] : 0;
        const int ang = live ? seg[(i * T + b) * 2 + 1] : 0;
        const R* __restrict__ cA = theta + dm.offA + (long)((a * T + b) * NA) * KA;
        R Sb[KR];
#pragma unroll
        for (int k = 0; k < KR; ++k) Sb[k] = R(0);
        // batches of S pairs (team-uniform trip count); the record of the next
        // batch is loaded one batch ahead. Batches that start inside the
        // angular prefix go through the moment exchange.
        Rec<R> nx{};
        if (lane < tot) nx = pairs[p + lane];
        for (int base = 0; base < tot; base += S) {
            const int k = base + lane;
            const Rec<R> pr = nx;
            if (k + S < tot) nx = pairs[p + k + S];
            const bool angb = base < ang;
            R g[NA], Y[LM];
#pragma unroll
            for (int n = 0; n < NA; ++n) g[n] = R(0);
#pragma unroll
            for (int lm = 0; lm < LM; ++lm) Y[lm] = R(0);
            if (k < tot) {
                const R r = sqrt(pr.x * pr.x + pr.y * pr.y + pr.z * pr.z);
                R f[KR];
                cheb_basis<R, KR, false>(r, rcR, irR, f, nullptr);
#pragma unroll
                for (int kk = 0; kk < KR; ++kk) Sb[kk] += f[kk];
                if (k < ang) {
                    R fa[KA];
                    cheb_basis<R, KA, false>(r, rcA, irA, fa, nullptr);
                    const R ir = R(1) / r;
                    solid_harmonics<R, R, L>(pr.x * ir, pr.y * ir, pr.z * ir, Y);
#pragma unroll
                    for (int n = 0; n < NA; ++n)
#pragma unroll
                        for (int kk = 0; kk < KA; ++kk) g[n] += cA[n * KA + kk] * fa[kk];
                }
            }
            if (angb) X::accumulate(tbuf, lane, g, Y, acc);
        }
        p += tot;
#pragma unroll
        for (int kk = 0; kk < KR; ++kk) Sb[kk] = team_sum<S>(Sb[kk]);
        const R* __restrict__ cR = theta + (long)((a * T + b) * NR) * KR;
        if constexpr (FUSE == 0) {
            // the lane's own coefficient rows (vector loads; a row past N_R
            // reads the last one and is never stored)
#pragma unroll
            for (int o = 0; o < NR_OWN; ++o) {
                const int n = lane + S * o;
                const R* __restrict__ cr = cR + (n < NR ? n : NR - 1) * KR;
#pragma unroll
                for (int kk = 0; kk < KR; ++kk) qR[o] += cr[kk] * Sb[kk];
            }
        } else {
#pragma unroll
            for (int n = 0; n < NR; ++n)
#pragma unroll
                for (int kk = 0; kk < KR; ++kk) qR[n] += cR[n * KR + kk] * Sb[kk];
        }
        if (live) {
#pragma unroll
            for (int kk = 0; kk < KR; ++kk)
                if (kk % S == lane) S0_out[((long)i * T + b) * KR + kk] = Sb[kk];
        }
    }
    // invariants: partial sums over owned harmonics, summed over the team
    R qA[NA * L];
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int l = 1; l <= L; ++l) {
            R s2 = R(0);
#pragma unroll
            for (int o = 0; o < OWN; ++o) {
                const int lm = lane + S * o;
                if (lm < LM && lm_degree<LM>(lm) == l) s2 += acc[n][o] * acc[n][o];
            }
            qA[(l - 1) * NA + n] = team_sum<S>(s2);
        }
    R q4v[NA];
    if (Sh::H4) {
#pragma unroll
        for (int n = 0; n < NA; ++n) {
            R a2[5];
#pragma unroll
            for (int m = 0; m < 5; ++m) a2[m] = __shfl(acc[n][(3 + m) / S], (threadIdx.x & ~(S - 1)) + (3 + m) % S, 64);
            q4v[n] = q4_value<R>(a2);
        }
    }
    if (!live) return;
    // the whole descriptor is known to every lane of the team
    R qv[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if (d < NR) {
            // (FUSE 0: right only in the lane that stores entry d, d % S == lane)
            if constexpr (FUSE == 0)
                qv[d] = qR[d / S];
            else
                qv[d] = qR[d];
        } else if (d < NR + L * NA) {
            qv[d] = qA[d - NR];
        } else if (Sh::H4 && d < NR + (L + 1) * NA) {
            qv[d] = q4v[d - NR - L * NA];
        } else {
            const R P = qA[d - NR - (L + (Sh::H4 ? 1 : 0)) * NA];  // l = 1 three-body term
            qv[d] = P * P;
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d)
        if (d % S == lane) q_out[(long)i * D + d] = qv[d];
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int o = 0; o < OWN; ++o) {
            const int lm = lane + S * o;
            if (lm < LM) A_out[((long)i * NA + n) * LM + lm] = acc[n][o];
        }
    R e[D];
    if (FUSE >= 1) team_network_forward<R, D, S>(lane, dm, theta, a, qscale, qv, i, E_out, e_out, t_out, e);
    if (FUSE == 2) {
        // B = dE_i/dA into the team's LDS block, whose exchange use has ended
        if constexpr (!Sh::H4 && !Sh::H5 && (Sh::NA * Sh::LM <= 120 || S >= 8)) {
            // three-body invariants only: B_nlm = 2 e_(n,l) A_nlm, each lane
            // for the harmonics it owns, from registers; e's radial entries
            // beside it for the radial force coefficients (4-lane teams of
            // large moment blocks would spill holding e)
#pragma unroll
            for (int n = 0; n < NA; ++n)
#pragma unroll
                for (int o = 0; o < OWN; ++o) {
                    const int lm = lane + S * o;
                    if (lm >= LM) continue;
                    const int l = lm < 3 ? 1 : lm < 8 ? 2 : lm < 15 ? 3 : 4;
                    R el = e[NR + n];
#pragma unroll
                    for (int ll = 2; ll <= L; ++ll)
                        if (l == ll) el = e[NR + (ll - 1) * NA + n];
                    tbuf[n * LM + lm] = R(2) * el * acc[n][o];
                }
#pragma unroll
            for (int d = 0; d < NR; ++d)
                if (d % S == lane) tbuf[NA * LM + d] = e[d];
            X::wave_fence();
            force_pass<R, Sh, S>(lane, dm, theta, i, true, a, row, seg, pairs, reverse, tbuf, tbuf + NA * LM, h_in,
                                 Fown_out, Wat_out);
        } else {
            // from the team's just-stored A and e rows (a workgroup-scope
            // fence makes each lane's stores visible to the other lanes)
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            moment_adjoints<R, Sh, S, false>(lane, A_out + (long)i * NA * LM, nullptr, e_out + (long)i * D, nullptr,
                                             tbuf, nullptr);
            X::wave_fence();
            force_pass<R, Sh, S>(lane, dm, theta, i, true, a, row, seg, pairs, reverse, tbuf, e_out + (long)i * D,
                                 h_in, Fown_out, Wat_out);
        }
    }
}

// ------------------------------------------------ per-atom moment adjoints

// B = dE_i/dA[n][lm] (Eq. 20 and the 4/5-body terms, with e = dE_i/dq) and,
// when WITH_BP, Bp = dPsi/dA[n][lm] for Psi = abar . q + e . dq (abar = dPsi/dq,
// dA the tangent of the moments). The S lanes of a team take entries
// x = lane, lane + S, ... of the atom's NA x LM block.
template <typename R, class Sh, int S, bool WITH_BP>
__device__ __forceinline__ void moment_adjoints(int lane, const R* __restrict__ A, const R* __restrict__ dA,
                                                const R* __restrict__ e, const R* __restrict__ ab, R* B, R* Bp) {
    constexpr int NR = Sh::NR, NA = Sh::NA, LM = Sh::LM, L = Sh::L;
    for (int x = lane; x < NA * LM; x += S) {
        const int n = x / LM, lm = x % LM;
        const int l = lm < 3 ? 1 : lm < 8 ? 2 : lm < 15 ? 3 : 4;
        const int idx = NR + (l - 1) * NA + n;
        const R a = A[x];
        R b = R(2) * e[idx] * a;
        R bp = R(0);
        if (WITH_BP) bp = R(2) * ab[idx] * a + R(2) * e[idx] * dA[x];
        if (Sh::H4 && l == 2) {
            R a2[5], g4[5];
#pragma unroll
            for (int m = 0; m < 5; ++m) a2[m] = A[n * LM + 3 + m];
            q4_grad<R>(a2, g4);
            R gm = g4[0];
#pragma unroll
            for (int m = 1; m < 5; ++m)
                if (lm - 3 == m) gm = g4[m];
            const int i4 = NR + L * NA + n;
            b += e[i4] * gm;
            if (WITH_BP) {
                R d2[5], h4[5];
#pragma unroll
                for (int m = 0; m < 5; ++m) d2[m] = dA[n * LM + 3 + m];
                q4_hess_vec<R>(a2, d2, h4);
                R hm = h4[0];
#pragma unroll
                for (int m = 1; m < 5; ++m)
                    if (lm - 3 == m) hm = h4[m];
                bp += ab[i4] * gm + e[i4] * hm;
            }
        }
        if (Sh::H5 && l == 1) {
            const R a0 = A[n * LM], a1 = A[n * LM + 1], a2 = A[n * LM + 2];
            const R P = a0 * a0 + a1 * a1 + a2 * a2;
            const int i5 = NR + (L + (Sh::H4 ? 1 : 0)) * NA + n;
            b += e[i5] * R(4) * P * a;
            if (WITH_BP) {
                const R dd = a0 * dA[n * LM] + a1 * dA[n * LM + 1] + a2 * dA[n * LM + 2];
                bp += ab[i5] * R(4) * P * a + e[i5] * (R(8) * dd * a + R(4) * P * dA[x]);
            }
        }
        B[x] = b;
        if (WITH_BP) Bp[x] = bp;
    }
}

// ------------------------------------------------------------------- force

// One pair of atom i's row in the force pass: h_ij = dE_i/dr_ij from the
// radial force coefficients eps_k = sum_n e_n c_R[a][b][n][k] (epsk) and, for
// an angular pair, from c^A[a][b] (cA) and the atom's own B = dE_i/dA (Bk);
// -h_ij goes to the slot q of the reverse pair (j, i) (zero to the pair's own
// slot pos when it has none), h_ij to the atom's own-direction sum F and
// -r_ij (x) h_ij to its virial Wv.
template <typename R, class Sh>
__device__ __forceinline__ void force_pair(const Rec<R>& pr, int q, int64_t pos, bool angular, const R* epsk,
                                           const R* cA, const R* Bk, R rcR, R irR, R rcA, R irA,
                                           Rec<R>* __restrict__ h_in, R* F, R* Wv) {
    constexpr int NA = Sh::NA, KR = Sh::KR, KA = Sh::KA, LM = Sh::LM;
    const R r = sqrt(pr.x * pr.x + pr.y * pr.y + pr.z * pr.z);
    const R ir = R(1) / r;
    const R u[3] = {pr.x * ir, pr.y * ir, pr.z * ir};
    R f[KR], fp[KR];
    cheb_basis<R, KR, true>(r, rcR, irR, f, fp);
    R sr = R(0);
#pragma unroll
    for (int kk = 0; kk < KR; ++kk) sr += epsk[kk] * fp[kk];
    R hv[3] = {sr * u[0], sr * u[1], sr * u[2]};
    if (angular) {
        R fa[KA], fap[KA];
        cheb_basis<R, KA, true>(r, rcA, irA, fa, fap);
        R c[LM], cp[LM];
#pragma unroll
        for (int lm = 0; lm < LM; ++lm) c[lm] = cp[lm] = R(0);
#pragma unroll
        for (int n = 0; n < NA; ++n) {
            R g = R(0), gp = R(0);
#pragma unroll
            for (int kk = 0; kk < KA; ++kk) {
                g += cA[n * KA + kk] * fa[kk];
                gp += cA[n * KA + kk] * fap[kk];
            }
#pragma unroll
            for (int lm = 0; lm < LM; ++lm) {
                c[lm] += Bk[n * LM + lm] * g;
                cp[lm] += Bk[n * LM + lm] * gp;
            }
        }
        // G = grad_u sum_lm c_lm Y_lm(u); Y_lm is homogeneous of degree l, so
        // u . G = sum_lm l c_lm Y_lm (Euler) and the tangential part of
        // the gradient is G - (u . G) u.
        R Y[LM], G[3];
        solid_harmonics<R, R, Sh::L>(u[0], u[1], u[2], Y);
        R sY = R(0);
#pragma unroll
        for (int lm = 0; lm < LM; ++lm) sY += cp[lm] * Y[lm];
        solid_harmonics_grad<R, Sh::L>(u[0], u[1], u[2], c, G);
        const R lY = u[0] * G[0] + u[1] * G[1] + u[2] * G[2];
#pragma unroll
        for (int d = 0; d < 3; ++d) hv[d] += sY * u[d] + (G[d] - lY * u[d]) * ir;
    }
    if (q >= 0) {
        Rec<R> ho;
        ho.x = -hv[0];
        ho.y = -hv[1];
        ho.z = -hv[2];
        ho.w = R(0);
        h_in[q] = ho;  // -dE_i/dr_ij is the pair's contribution to F_j
    } else {
        // no reverse pair (|r| at the cutoff in one direction only):
        // nothing else writes this pair's own slot
        h_in[pos] = Rec<R>{};
    }
    const R rv[3] = {pr.x, pr.y, pr.z};
#pragma unroll
    for (int d = 0; d < 3; ++d) F[d] += hv[d];
#pragma unroll
    for (int al = 0; al < 3; ++al)
#pragma unroll
        for (int be = 0; be < 3; ++be) Wv[al * 3 + be] -= rv[al] * hv[be];
}

// The team sums of an atom's own-direction force and virial, stored by the
// lanes that own each component.
template <typename R, int S>
__device__ __forceinline__ void force_store(int lane, bool live, int i, R* F, R* Wv, R* __restrict__ Fown_out,
                                            R* __restrict__ Wat_out) {
#pragma unroll
    for (int d = 0; d < 3; ++d) F[d] = team_sum<S>(F[d]);
#pragma unroll
    for (int c = 0; c < 9; ++c) Wv[c] = team_sum<S>(Wv[c]);
    if (live) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
            if (d % S == lane) Fown_out[(long)i * 3 + d] = F[d];
#pragma unroll
        for (int c = 0; c < 9; ++c)
            if (c % S == lane) Wat_out[(long)i * 9 + c] = Wv[c];
    }
}

// The force pass of one atom's team inside the descriptor sweep: for every
// pair of atom i's row, h_ij = dE_i/dr_ij from the atom's own B = dE_i/dA (Bk,
// the team's LDS copy) and e = dE_i/dq (ei), the radial part through eps_k =
// sum_n e_n c_R[a][b][n][k] (one direction per pair); the atom's
// own-direction sum sum_j h_ij, its virial -sum_j r_ij (x) h_ij, and -h_ij
// written into the slot of the reverse pair (j, i), so that k_force_gather
// completes F_j = sum h_jk + sum (-h_kj) with contiguous reads and no atomics.
// The teams of a wavefront walk the neighbour-species segments in lock step
// (coefficient addresses uniform over the block).
template <typename R, class Sh, int S>
__device__ __forceinline__ void force_pass(int lane, const Dims& dm, const R* __restrict__ theta, int i, bool live,
                                           int a, const int64_t* __restrict__ row, const int* __restrict__ seg,
                                           const Rec<R>* __restrict__ pairs, const int* __restrict__ reverse,
                                           const R* Bk, const R* __restrict__ ei, Rec<R>* __restrict__ h_in,
                                           R* __restrict__ Fown_out, R* __restrict__ Wat_out) {
    constexpr int NR = Sh::NR, NA = Sh::NA, KR = Sh::KR, KA = Sh::KA;
    const int T = dm.T;
    const R rcR = R(dm.rcR), rcA = R(dm.rcA), irR = R(1.0 / dm.rcR), irA = R(1.0 / dm.rcA);
    int64_t p = live ? row[i] : 0;
    R F[3] = {R(0), R(0), R(0)};
    R Wv[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) Wv[c] = R(0);
    for (int b = 0; b < T; ++b) {
        const int tot = live ? seg[(i * T + b) * 2] : 0;
        const int ang = live ? seg[(i * T + b) * 2 + 1] : 0;
        // radial force coefficients eps_k = sum_n e_n c_R[a][b][n][k]: each
        // lane of the team sums its columns k = lane + S o (a column past K_R
        // reads the last one and is dropped), then the team gathers them
        R epsk[KR];
        const R* __restrict__ cRab = theta + (long)((a * T + b) * NR) * KR;
        {
            constexpr int KO = (KR + S - 1) / S;
            R mine[KO];
#pragma unroll
            for (int o = 0; o < KO; ++o) mine[o] = R(0);
            if (live) {
#pragma unroll
                for (int n = 0; n < NR; ++n) {
                    const R en = ei[n];
#pragma unroll
                    for (int o = 0; o < KO; ++o) {
                        const int kk = lane + S * o;
                        mine[o] += en * cRab[n * KR + (kk < KR ? kk : KR - 1)];
                    }
                }
            }
            const int base = int(threadIdx.x) & ~(S - 1);
#pragma unroll
            for (int kk = 0; kk < KR; ++kk) epsk[kk] = __shfl(mine[kk / S], base + kk % S, 64);
        }
        const R* __restrict__ cA = theta + dm.offA + (long)((a * T + b) * NA) * KA;
        // the next record and reverse index are loaded one iteration ahead,
        // with no branch around the loads (the last iteration reads the
        // segment's last pair again and drops it)
        Rec<R> nx{};
        int nrev = -1;
        if (lane < tot) {
            nx = pairs[p + lane];
            nrev = reverse[p + lane];
        }
        for (int k = lane; k < tot; k += S) {
            const Rec<R> pr = nx;
            const int q = nrev;
            {
                const int kn = min(k + S, tot - 1);
                nx = pairs[p + kn];
                nrev = reverse[p + kn];
            }
            force_pair<R, Sh>(pr, q, p + k, k < ang, epsk, cA, Bk, rcR, irR, rcA, irA, h_in, F, Wv);
        }
        p += tot;
    }
    force_store<R, S>(lane, live, i, F, Wv, Fown_out, Wat_out);
}

// Forces and virials (Eq. 1) in their own sweep, the teams of a wavefront in
// lock step over the neighbour-species segments (c^A[a][b] and c_R[a][b]
// read at addresses uniform over the block): each team builds its atom's
// B = dE_i/dA in LDS from the stored moments and e, then runs force_pass.
// The FP64 sweep (its pair body held in registers with c^A in VGPRs instead
// of scalar registers would spill).
template <typename R, class Sh, int S>
__global__ void __launch_bounds__(kBlock)
k_force_lockstep(const Dims dm, const R* __restrict__ theta, const int* __restrict__ order,
                 const int64_t* __restrict__ soff, int Na, const int64_t* __restrict__ row,
                 const int* __restrict__ seg, const Rec<R>* __restrict__ pairs, const int* __restrict__ reverse,
                 const R* __restrict__ A_in, const R* __restrict__ e_in, Rec<R>* __restrict__ h_in,
                 R* __restrict__ Fown_out, R* __restrict__ Wat_out) {
    constexpr int NA = Sh::NA, LM = Sh::LM, D = Sh::D;
    constexpr int TEAMS = kBlock / S;
    __shared__ R Bsh[TEAMS][NA * LM];
    const int team = threadIdx.x / S, lane = threadIdx.x % S;
    int a;
    long lo = 0, hi = 0;
    species_chunk(soff, dm.T, TEAMS, xcd_tile(blockIdx.x, gridDim.x), &a, &lo, &hi);
    if (a < 0) return;
    const bool live = lo + team < hi;
    const int i = live ? order[lo + team] : 0;
    const R* __restrict__ ei = e_in + (long)(live ? i : 0) * D;
    if (live) {
        moment_adjoints<R, Sh, S, false>(lane, A_in + (long)i * NA * LM, nullptr, ei, nullptr, Bsh[team], nullptr);
    } else {
        for (int x = lane; x < NA * LM; x += S) Bsh[team][x] = R(0);
    }
    __syncthreads();
    force_pass<R, Sh, S>(lane, dm, theta, i, live, a, row, seg, pairs, reverse, Bsh[team], ei, h_in, Fown_out,
                         Wat_out);
}

// One of the force sweep's two walks over a team's row (ANG: the angular
// pairs of every neighbour-species segment, else the radial-only pairs):
// the walk's k-th pair lies in the segment b whose table entry is the first
// with end > k (end: .x for the angular walk, .z for the radial one), at row
// offset k + off (.y, .w). Lane l takes k = l, l + S, ...; the next pair's
// segment, record and reverse index are found one iteration ahead, with no
// branch around the loads (the last iteration reads the walk's last pair
// again and drops it).
template <typename R, class Sh, int S, bool ANG>
__device__ __forceinline__ void force_walk(int lane, int total, const int4* tab, int64_t p0,
                                           const Rec<R>* __restrict__ pairs, const int* __restrict__ reverse,
                                           const R* cAs, int cas, const R* eps, const R* Bk, R rcR, R irR, R rcA,
                                           R irA, Rec<R>* __restrict__ h_in, R* F, R* Wv) {
    constexpr int KR = Sh::KR;
    if (total <= 0) return;
    int bn = 0;
    int4 tn = tab[0];
    int kn = min(lane, total - 1);
    while (kn >= (ANG ? tn.x : tn.z)) tn = tab[++bn];
    int64_t posn = p0 + kn + (ANG ? tn.y : tn.w);
    Rec<R> nx = pairs[posn];
    int nrev = reverse[posn];
    // a wait for all vector memory at the walk's start: the compiler merges
    // its wait counts where the loop is entered, and without this wait the
    // merged count made every iteration begin by waiting for the previous
    // pair's h store; with it, that wait comes after the pair's arithmetic
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    for (int k = lane; k < total; k += S) {
        const Rec<R> pr = nx;
        const int q = nrev, b = bn;
        const int64_t pos = posn;
        kn = min(k + S, total - 1);
        while (kn >= (ANG ? tn.x : tn.z)) tn = tab[++bn];
        posn = p0 + kn + (ANG ? tn.y : tn.w);
        nx = pairs[posn];
        nrev = reverse[posn];
        // B's reads stay in the loop (hoisted, N_A x 24 values would take
        // registers from the occupancy): an offset opaque to the compiler
        int bo = 0;
        asm volatile("" : "+v"(bo));
        force_pair<R, Sh>(pr, q, pos, ANG, eps + b * KR, cAs + b * cas, Bk + bo, rcR, irR, rcA, irA, h_in, F, Wv);
    }
}

// Forces and virials (Eq. 1) in their own sweep. Each team builds its atom's
// B = dE_i/dA in LDS from the stored moments and e and walks its row twice,
// across the neighbour-species segments: first the angular pairs of every
// segment, then the radial-only pairs. The teams of a wavefront then pad
// only at the end of each walk instead of at the end of every segment (and
// no wavefront runs the angular part for one team while another is on its
// radial-only pairs). A pair's segment b selects c^A[a][b] (staged for the
// whole block) and the team's eps_k[b] in LDS.
template <typename R, class Sh, int S>
__global__ void __launch_bounds__(kBlock)
k_force(const Dims dm, const R* __restrict__ theta, const int* __restrict__ order, const int64_t* __restrict__ soff,
        int Na, const int64_t* __restrict__ row, const int* __restrict__ seg, const Rec<R>* __restrict__ pairs,
        const int* __restrict__ reverse, const R* __restrict__ A_in, const R* __restrict__ e_in,
        Rec<R>* __restrict__ h_in, R* __restrict__ Fown_out, R* __restrict__ Wat_out) {
    constexpr int NR = Sh::NR, NA = Sh::NA, KR = Sh::KR, KA = Sh::KA, LM = Sh::LM, D = Sh::D;
    constexpr int TEAMS = kBlock / S;
    __shared__ R Bsh[TEAMS][NA * LM];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int T = dm.T;
    const ForceLds g = force_lds(T, NA, KA, KR, TEAMS, int(sizeof(R)));
    R* cAs = reinterpret_cast<R*>(smem_raw);
    const int team = threadIdx.x / S, lane = threadIdx.x % S;
    R* eps = reinterpret_cast<R*>(smem_raw + g.off_eps) + team * g.eps_team;
    int4* tab = reinterpret_cast<int4*>(smem_raw + g.off_tab) + team * (T + 1);
    // one species per block, as in the sweeps
    int a;
    long lo = 0, hi = 0;
    species_chunk(soff, T, TEAMS, xcd_tile(blockIdx.x, gridDim.x), &a, &lo, &hi);
    if (a < 0) return;
    const bool live = lo + team < hi;
    const int i = live ? order[lo + team] : 0;
    const R* __restrict__ ei = e_in + (long)i * D;
    // c^A[a][b] for every neighbour species b
    {
        const R* __restrict__ cAa = theta + dm.offA + (long)(a * T) * NA * KA;
        for (int x = threadIdx.x; x < T * NA * KA; x += kBlock) {
            const int b = x / (NA * KA);
            cAs[b * g.cas + (x - b * NA * KA)] = cAa[x];
        }
    }
    // the team's eps_k[b] = sum_n e_n c_R[a][b][n][k], column (b, k) per lane
    {
        R en[NR];
#pragma unroll
        for (int n = 0; n < NR; ++n) en[n] = live ? ei[n] : R(0);
        const R* __restrict__ cRa = theta + (long)(a * T) * NR * KR;
        for (int c = lane; c < T * KR; c += S) {
            const int b = c / KR;
            const R* __restrict__ col = cRa + (long)b * NR * KR + (c - b * KR);
            R sum = R(0);
#pragma unroll
            for (int n = 0; n < NR; ++n) sum += en[n] * col[n * KR];
            eps[c] = sum;
        }
    }
    // the team's segment table: entry b = (end of b's angular pairs in the
    // angular walk, their row offset, end of b's radial-only pairs in the
    // radial walk, their row offset); entry T = the two walks' lengths
    if (lane == 0) {
        int preA = 0, preR = 0, rel = 0;
        for (int b = 0; b < T; ++b) {
            const int tot = live ? seg[(i * T + b) * 2] : 0;
            const int ang = live ? seg[(i * T + b) * 2 + 1] : 0;
            tab[b] = make_int4(preA + ang, rel - preA, preR + (tot - ang), rel + ang - preR);
            preA += ang;
            preR += tot - ang;
            rel += tot;
        }
        tab[T] = make_int4(preA, preR, 0, 0);
    }
    if (live) {
        moment_adjoints<R, Sh, S, false>(lane, A_in + (long)i * NA * LM, nullptr, ei, nullptr, Bsh[team], nullptr);
    } else {
        for (int x = lane; x < NA * LM; x += S) Bsh[team][x] = R(0);
    }
    __syncthreads();
    const R rcR = R(dm.rcR), rcA = R(dm.rcA), irR = R(1.0 / dm.rcR), irA = R(1.0 / dm.rcA);
    const int64_t p0 = live ? row[i] : 0;
    const int4 len = tab[T];
    R F[3] = {R(0), R(0), R(0)};
    R Wv[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) Wv[c] = R(0);
    force_walk<R, Sh, S, true>(lane, len.x, tab, p0, pairs, reverse, cAs, g.cas, eps, Bsh[team], rcR, irR, rcA, irA,
                               h_in, F, Wv);
    force_walk<R, Sh, S, false>(lane, len.y, tab, p0, pairs, reverse, cAs, g.cas, eps, Bsh[team], rcR, irR, rcA,
                                irA, h_in, F, Wv);
    force_store<R, S>(lane, live, i, F, Wv, Fown_out, Wat_out);
}

// F_i = (own-direction sum) + sum_{p in row i} h_in[p]: team of S lanes per
// atom over its (contiguous) row, team sum in fixed shuffle order. Slots of
// pairs without a reverse partner hold zeros (written by the force sweep).
template <typename R, int S>
__global__ void __launch_bounds__(kBlock)
k_force_gather(int Na, const int64_t* __restrict__ row, const Rec<R>* __restrict__ h_in,
               const R* __restrict__ Fown, R* __restrict__ F_out) {
    const int team = threadIdx.x / S, lane = threadIdx.x % S;
    const int i = xcd_tile(blockIdx.x, gridDim.x) * (kBlock / S) + team;
    const bool live = i < Na;
    const int64_t p0 = live ? row[i] : 0, p1 = live ? row[i + 1] : 0;
    R f[3] = {R(0), R(0), R(0)};
    // every slot is written by the force sweep (zero for unpaired pairs), so
    // the loads are unconditional and several are in flight at once
#pragma unroll 4
    for (int64_t p = p0 + lane; p < p1; p += S) {
        const Rec<R> a = h_in[p];
        f[0] += a.x;
        f[1] += a.y;
        f[2] += a.z;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) f[d] = team_sum<S>(f[d]);
    if (live && lane < 3) F_out[(long)i * 3 + lane] = Fown[(long)i * 3 + lane] + (lane == 0 ? f[0] : (lane == 1 ? f[1] : f[2]));
}

// ----------------------------------------------------------------- tangent

// Directional derivative of the descriptor along v_ij = u_i - u_j - U_s^T r_ij:
// dq (radial and invariants), dA[n][lm] = sum_j [g_n' (v.r^) Y_lm + g_n v.dY_lm],
// and S1[b][k] = sum_{j in b} (v.r^) f_k'. Angular pairs go through the team
// exchange (two terms per pair); each lane owns the moments lm = lane + S*o.
// With NET the team then runs the atom's network Hessian-vector product.
template <typename R, class Sh, int S, bool NET>
__global__ void __launch_bounds__(kBlock, (SweepWaves<R, Sh, S>::tangent))
k_tangent(const Dims dm, const R* __restrict__ theta, const int* __restrict__ order,
          const int64_t* __restrict__ soff, const int* __restrict__ atom_struct, int Na, const int64_t* __restrict__ row, const int* __restrict__ seg,
          const Rec<R>* __restrict__ pairs, const R* __restrict__ ubar, const double* __restrict__ Ubar,
          const R* __restrict__ A_in, R* __restrict__ dq_out, R* __restrict__ dA_out, R* __restrict__ S1_out,
          const R* __restrict__ qscale, const double* __restrict__ ebar_s, const R* __restrict__ e_in,
          const R* __restrict__ t_in, R* __restrict__ abar_out, R* __restrict__ alpha_out, R* __restrict__ beta_out,
          R* __restrict__ gamma_out) {
    constexpr int NR = Sh::NR, NA = Sh::NA, KR = Sh::KR, KA = Sh::KA, LM = Sh::LM, D = Sh::D, L = Sh::L;
    using X = MomentExchange<R, NA, LM, S>;
    constexpr int OWN = X::OWN, TEAMS = kBlock / S;
    constexpr int DANG = NA * (L + (Sh::H4 ? 1 : 0) + (Sh::H5 ? 1 : 0));
    __shared__ R xbuf[TEAMS * X::TEAM_FLOATS];
    const int team = threadIdx.x / S, lane = threadIdx.x % S;
    R* tbuf = xbuf + team * X::TEAM_FLOATS;
    const int T = dm.T;
    // one species per block, as in the descriptor sweep
    int a;
    long lo = 0, hi = 0;
    species_chunk(soff, T, TEAMS, xcd_tile(blockIdx.x, gridDim.x), &a, &lo, &hi);
    if (a < 0) return;
    const bool live = lo + team < hi;
    const int i = live ? order[lo + team] : 0;
    const R rcR = R(dm.rcR), rcA = R(dm.rcA), irR = R(1.0 / dm.rcR), irA = R(1.0 / dm.rcA);
    const int s = live ? atom_struct[i] : 0;
    int64_t p = live ? row[i] : 0;
    R ui[3], U[9];
#pragma unroll
    for (int d = 0; d < 3; ++d) ui[d] = live ? ubar[(long)i * 3 + d] : R(0);
#pragma unroll
    for (int c = 0; c < 9; ++c) U[c] = live ? R(Ubar[(long)s * 9 + c]) : R(0);
    // without the network in the sweep a lane needs only the radial rows it
    // stores, n = lane + S o
    constexpr int NR_OWN = NET ? NR : (NR + S - 1) / S;
    R dqR[NR_OWN];
#pragma unroll
    for (int n = 0; n < NR_OWN; ++n) dqR[n] = R(0);
    R acc[NA][OWN];
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int o = 0; o < OWN; ++o) acc[n][o] = R(0);

    for (int b = 0; b < T; ++b) {
        const int tot = live ? seg[(i * T + b) * 2] : 0;
        const int ang = live ? seg[(i * T + b) * 2 + 1] : 0;
        const R* __restrict__ cA = theta + dm.offA + (long)((a * T + b) * NA) * KA;
        R Sb[KR];
#pragma unroll
        for (int kk = 0; kk < KR; ++kk) Sb[kk] = R(0);
        // the next batch's record is loaded one batch ahead; the neighbour's
        // seed (a dependent load) is issued before the basis is evaluated.
        // Inside the loop no branch guards a load (a lane past the segment's
        // end reads its last pair, or atom 0's seed, and drops the values), so
        // the compiler waits only for the loads a value needs.
        Rec<R> nx{};
        if (lane < tot) nx = pairs[p + lane];
        for (int base = 0; base < tot; base += S) {
            const int k = base + lane;
            const bool angb = base < ang;  // team-uniform: this batch starts inside the angular prefix
            const Rec<R> pr = nx;
            R uj[3];
            {
                const long j = rec_j(pr);
#pragma unroll
                for (int be = 0; be < 3; ++be) uj[be] = ubar[j * 3 + be];
            }
            nx = pairs[p + min(k + S, tot - 1)];
            R gpv[NA], g[NA], Y[LM], vdY[LM];
#pragma unroll
            for (int n = 0; n < NA; ++n) gpv[n] = g[n] = R(0);
#pragma unroll
            for (int lm = 0; lm < LM; ++lm) Y[lm] = vdY[lm] = R(0);
            if (k < tot) {
                const R rv[3] = {pr.x, pr.y, pr.z};
                const R r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
                const R ir = R(1) / r;
                const R u[3] = {rv[0] * ir, rv[1] * ir, rv[2] * ir};
                R f[KR], fp[KR];
                cheb_basis<R, KR, true>(r, rcR, irR, f, fp);
                R fa[KA], fap[KA];
                if (k < ang) cheb_basis<R, KA, true>(r, rcA, irA, fa, fap);
                R v[3];
#pragma unroll
                for (int be = 0; be < 3; ++be)
                    v[be] = ui[be] - uj[be] - (U[be] * rv[0] + U[3 + be] * rv[1] + U[6 + be] * rv[2]);
                const R vu = v[0] * u[0] + v[1] * u[1] + v[2] * u[2];
#pragma unroll
                for (int kk = 0; kk < KR; ++kk) Sb[kk] += vu * fp[kk];
                if (k < ang) {
                    const D1<R> dx = {u[0], v[0]}, dy = {u[1], v[1]}, dz = {u[2], v[2]};
                    D1<R> Yd[LM];
                    solid_harmonics<D1<R>, R, L>(dx, dy, dz, Yd);
#pragma unroll
                    for (int lm = 0; lm < LM; ++lm) {
                        Y[lm] = Yd[lm].v;
                        vdY[lm] = (Yd[lm].d - R(lm_degree<LM>(lm)) * Yd[lm].v * vu) * ir;
                    }
#pragma unroll
                    for (int n = 0; n < NA; ++n) {
                        R gg = R(0), gp = R(0);
#pragma unroll
                        for (int kk = 0; kk < KA; ++kk) {
                            gg += cA[n * KA + kk] * fa[kk];
                            gp += cA[n * KA + kk] * fap[kk];
                        }
                        g[n] = gg;
                        gpv[n] = gp * vu;
                    }
                }
            }
            if (angb) {
                X::accumulate(tbuf, lane, gpv, Y, acc);
                X::accumulate(tbuf, lane, g, vdY, acc);
            }
        }
        p += tot;
#pragma unroll
        for (int kk = 0; kk < KR; ++kk) Sb[kk] = team_sum<S>(Sb[kk]);
        const R* __restrict__ cR = theta + (long)((a * T + b) * NR) * KR;
        if constexpr (!NET) {
#pragma unroll
            for (int o = 0; o < NR_OWN; ++o) {
                const int n = lane + S * o;
                const R* __restrict__ cr = cR + (n < NR ? n : NR - 1) * KR;
#pragma unroll
                for (int kk = 0; kk < KR; ++kk) dqR[o] += cr[kk] * Sb[kk];
            }
        } else {
#pragma unroll
            for (int n = 0; n < NR; ++n)
#pragma unroll
                for (int kk = 0; kk < KR; ++kk) dqR[n] += cR[n * KR + kk] * Sb[kk];
        }
        if (live) {
#pragma unroll
            for (int kk = 0; kk < KR; ++kk)
                if (kk % S == lane) S1_out[((long)i * T + b) * KR + kk] = Sb[kk];
        }
    }
    // the network step's first operands load while the invariant tangents
    // below wait for the moments
    NetBackFirst<R, D, S> nf;
    if (NET && live) nf.load(lane, dm, theta, a, t_in, e_in, ebar_s, s, i);
    // invariant tangents: contractions with the atom's own moments A, split
    // over the owned harmonics and summed over the team
    R part[DANG];
#pragma unroll
    for (int x = 0; x < DANG; ++x) part[x] = R(0);
#pragma unroll
    for (int n = 0; n < NA; ++n) {
        R An[OWN];
#pragma unroll
        for (int o = 0; o < OWN; ++o) {
            const int lm = lane + S * o;
            An[o] = (live && lm < LM) ? A_in[((long)i * NA + n) * LM + lm] : R(0);
        }
#pragma unroll
        for (int l = 1; l <= L; ++l)
#pragma unroll
            for (int o = 0; o < OWN; ++o) {
                const int lm = lane + S * o;
                if (lm < LM && lm_degree<LM>(lm) == l) part[(l - 1) * NA + n] += R(2) * An[o] * acc[n][o];
            }
        if (Sh::H4) {
            R a2[5], g4[5];
#pragma unroll
            for (int m = 0; m < 5; ++m) a2[m] = live ? A_in[((long)i * NA + n) * LM + 3 + m] : R(0);
            q4_grad<R>(a2, g4);
#pragma unroll
            for (int o = 0; o < OWN; ++o)
#pragma unroll
                for (int m = 0; m < 5; ++m)
                    if (lane + S * o == 3 + m) part[L * NA + n] += g4[m] * acc[n][o];
        }
        if (Sh::H5) {
            R P = R(0);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                const R am = live ? A_in[((long)i * NA + n) * LM + m] : R(0);
                P += am * am;
            }
#pragma unroll
            for (int o = 0; o < OWN; ++o) {
                const int lm = lane + S * o;
                if (lm < 3) part[(L + (Sh::H4 ? 1 : 0)) * NA + n] += R(4) * P * An[o] * acc[n][o];
            }
        }
    }
#pragma unroll
    for (int x = 0; x < DANG; ++x) part[x] = team_sum<S>(part[x]);
    if (!live) return;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if (d % S != lane) continue;
        if constexpr (!NET)
            dq_out[(long)i * D + d] = d < NR ? dqR[d / S] : part[d - NR];
        else
            dq_out[(long)i * D + d] = d < NR ? dqR[d] : part[d - NR];
    }
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int o = 0; o < OWN; ++o) {
            const int lm = lane + S * o;
            if (lm < LM) dA_out[((long)i * NA + n) * LM + lm] = acc[n][o];
        }
    if constexpr (NET) {
        R dq[D];
#pragma unroll
        for (int d = 0; d < D; ++d) dq[d] = d < NR ? dqR[d] : part[d - NR];
        team_network_backward<R, D, S>(lane, dm, theta, a, qscale, dq, i, nf, t_in, abar_out, alpha_out, beta_out,
                                       gamma_out);
    }
}

// -------------------------------------------------- angular coefficient grad

// dL/dc_A[a][b][n][k] = sum_{i in a} sum_{j in b, angular}
//     [ f_k P_n + f_k' R_n ],  P_n = sum_lm (Bp_nlm Y_lm + Q_nlm v.dY_lm),
//     R_n = (v.r^) sum_lm Q_nlm Y_lm,  Q = B = dE_i/dA.
// The atom's Bp and Q sit in LDS; each lane evaluates one pair of a batch and
// the team exchanges (P, f) and (R, f') so each lane owns k = lane + S*o.
// Per neighbour species the team's sums go to a team slot and are added into
// the block accumulator in team order (bitwise repeatable); one partial row
// (double) per block over a grid-stride loop of atom tiles.
template <typename R, class Sh, int S>
struct CoeffGradSmem {
    static constexpr int NA = Sh::NA, KA = Sh::KA, LM = Sh::LM, TEAMS = kBlock / S;
    using X = MomentExchange<R, NA, KA, S>;
    // 16-byte vectors of R for the broadcast loads of Bp and Q
    static constexpr int VEC = 16 / int(sizeof(R));
    // per-team [Bp | Q] block: 2 NA LM values padded to a whole number of
    // vectors and to 8 (mod 32) 4-byte words, so the teams of a wave read
    // distinct banks
    static constexpr int WORDS = 2 * NA * LM * int(sizeof(R)) / 4;
    static constexpr int BQ_STRIDE = (WORDS + ((8 - WORDS) % 32 + 32) % 32) * 4 / int(sizeof(R));
    // per-team region holding the exchange during a segment's pair loop and
    // the team's N_A x K_A sums after it; grown past the exchange by whole
    // 128-byte steps, so team regions keep the exchange's bank pattern
    static constexpr int NK = NA * KA, STEP = 128 / int(sizeof(R));
    static constexpr int REGION =
        X::TEAM_FLOATS >= NK ? X::TEAM_FLOATS : X::TEAM_FLOATS + (NK - X::TEAM_FLOATS + STEP - 1) / STEP * STEP;
    __host__ __device__ static constexpr size_t align16(size_t n) { return (n * sizeof(R) + 15) / 16 * 16 / sizeof(R); }
    // offsets (in R) of the regions: G, Bp/Q blocks, team regions
    __host__ __device__ static size_t off_bq(int T) { return align16(size_t(T) * T * NK); }
    __host__ __device__ static size_t off_x(int T) { return off_bq(T) + size_t(TEAMS) * BQ_STRIDE; }
    __host__ __device__ static size_t bytes(int T) { return sizeof(R) * (off_x(T) + size_t(TEAMS) * REGION) + sizeof(int) * TEAMS; }
};
static_assert(CoeffGradSmem<float, Shape<9, 9, 7, 5, 4, 0, 0>, 8>::BQ_STRIDE % 4 == 0, "vector alignment");

template <typename R, class Sh, int S>
__global__ void __launch_bounds__(kBlock, (SweepWaves<R, Sh, S>::coeff_grad))
k_angular_coeff_grad(const Dims dm, const int* __restrict__ types, const int* __restrict__ atom_struct, int Na,
                     const int64_t* __restrict__ row, const int* __restrict__ seg, const Rec<R>* __restrict__ pairs,
                     const R* __restrict__ ubar, const double* __restrict__ Ubar, const R* __restrict__ A_in,
                     const R* __restrict__ dA_in, const R* __restrict__ e_in, const R* __restrict__ abar,
                     double* __restrict__ partial) {
    constexpr int NA = Sh::NA, KA = Sh::KA, LM = Sh::LM, L = Sh::L, D = Sh::D;
    using SM = CoeffGradSmem<R, Sh, S>;
    using X = typename SM::X;
    using V = typename VecOf<R>::type;
    constexpr int OWN = X::OWN, NK = NA * KA, TEAMS = kBlock / S, VEC = SM::VEC;
    static_assert(LM % VEC == 0, "harmonic rows are whole vectors");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int T = dm.T;
    const int G_len = T * T * NK;
    R* G = reinterpret_cast<R*>(smem_raw);
    R* BQ = G + SM::off_bq(T);                // [TEAMS][BQ_STRIDE]: Bp[NA][LM], Q[NA][LM]
    R* xb = G + SM::off_x(T);                 // [TEAMS][REGION]: exchange, then the team's sums
    int* team_type = reinterpret_cast<int*>(xb + TEAMS * SM::REGION);
    for (int x = threadIdx.x; x < G_len; x += kBlock) G[x] = R(0);
    const int team = threadIdx.x / S, lane = threadIdx.x % S;
    R* myBp = BQ + team * SM::BQ_STRIDE;
    R* myQ = myBp + NA * LM;
    R* tbuf = xb + team * SM::REGION;
    const R rcA = R(dm.rcA), irA = R(1.0 / dm.rcA);
    const int tiles = (Na + TEAMS - 1) / TEAMS;
    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int i = tile * TEAMS + team;
        const bool live = i < Na;
        const int a = live ? types[i] : 0;
        const int s = live ? atom_struct[i] : 0;
        int64_t p = live ? row[i] : 0;
        R ui[3], U[9];
#pragma unroll
        for (int d = 0; d < 3; ++d) ui[d] = live ? ubar[(long)i * 3 + d] : R(0);
#pragma unroll
        for (int c = 0; c < 9; ++c) U[c] = live ? R(Ubar[(long)s * 9 + c]) : R(0);
        __syncthreads();
        if (live) {
            moment_adjoints<R, Sh, S, true>(lane, A_in + (long)i * NA * LM, dA_in + (long)i * NA * LM,
                                            e_in + (long)i * D, abar + (long)i * D, myQ, myBp);
        } else {
            for (int x = lane; x < NA * LM; x += S) myBp[x] = myQ[x] = R(0);
        }
        __syncthreads();
        for (int b = 0; b < T; ++b) {
            const int tot = live ? seg[(i * T + b) * 2] : 0;
            const int ang = live ? seg[(i * T + b) * 2 + 1] : 0;
            R acc[NA][OWN];
#pragma unroll
            for (int n = 0; n < NA; ++n)
#pragma unroll
                for (int o = 0; o < OWN; ++o) acc[n][o] = R(0);
            // record one batch ahead; the neighbour's seed before the basis; no
            // branch guards a load inside the loop (as in the tangent sweep)
            Rec<R> nx{};
            if (lane < ang) nx = pairs[p + lane];
            for (int base = 0; base < ang; base += S) {
                const int k = base + lane;
                const Rec<R> pr = nx;
                R uj[3];
                {
                    const long j = rec_j(pr);
#pragma unroll
                    for (int be = 0; be < 3; ++be) uj[be] = ubar[j * 3 + be];
                }
                nx = pairs[p + min(k + S, ang - 1)];
                R P[NA], Rn[NA], fa[KA], fap[KA];
#pragma unroll
                for (int n = 0; n < NA; ++n) P[n] = Rn[n] = R(0);
#pragma unroll
                for (int kk = 0; kk < KA; ++kk) fa[kk] = fap[kk] = R(0);
                if (k < ang) {
                    const R rv[3] = {pr.x, pr.y, pr.z};
                    const R r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
                    const R ir = R(1) / r;
                    const R u[3] = {rv[0] * ir, rv[1] * ir, rv[2] * ir};
                    cheb_basis<R, KA, true>(r, rcA, irA, fa, fap);
                    R v[3];
#pragma unroll
                    for (int be = 0; be < 3; ++be)
                        v[be] = ui[be] - uj[be] - (U[be] * rv[0] + U[3 + be] * rv[1] + U[6 + be] * rv[2]);
                    const R vu = v[0] * u[0] + v[1] * u[1] + v[2] * u[2];
                    const D1<R> dx = {u[0], v[0]}, dy = {u[1], v[1]}, dz = {u[2], v[2]};
                    D1<R> Yd[LM];
                    solid_harmonics<D1<R>, R, L>(dx, dy, dz, Yd);
                    R vdy[LM];
#pragma unroll
                    for (int lm = 0; lm < LM; ++lm)
                        vdy[lm] = (Yd[lm].d - R(lm_degree<LM>(lm)) * Yd[lm].v * vu) * ir;
#pragma unroll
                    for (int n = 0; n < NA; ++n) {
                        R pn = R(0), rn = R(0);
                        const V* bp = reinterpret_cast<const V*>(myBp + n * LM);
                        const V* qq = reinterpret_cast<const V*>(myQ + n * LM);
#pragma unroll
                        for (int c = 0; c < LM / VEC; ++c) {
                            const V bv = bp[c], qv = qq[c];
#pragma unroll
                            for (int e = 0; e < VEC; ++e) {
                                const int lm = c * VEC + e;
                                pn += bv[e] * Yd[lm].v;
                                pn += qv[e] * vdy[lm];
                                rn += qv[e] * Yd[lm].v;
                            }
                        }
                        P[n] = pn;
                        Rn[n] = rn * vu;
                    }
                }
                X::accumulate(tbuf, lane, P, fa, acc);
                X::accumulate(tbuf, lane, Rn, fap, acc);
            }
            p += tot;
#pragma unroll
            for (int n = 0; n < NA; ++n)
#pragma unroll
                for (int o = 0; o < OWN; ++o) {
                    const int kk = lane + S * o;
                    if (kk < KA) tbuf[n * KA + kk] = live ? acc[n][o] : R(0);
                }
            if (lane == 0) team_type[team] = a;
            __syncthreads();
            for (int x = threadIdx.x; x < NK; x += kBlock)
                for (int tm = 0; tm < TEAMS; ++tm) G[(team_type[tm] * T + b) * NK + x] += xb[tm * SM::REGION + x];
            __syncthreads();
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < G_len; x += kBlock) partial[(long)blockIdx.x * G_len + x] = double(G[x]);
}

// ------------------------------------- angular coefficient grad, rows per lane

// The moment adjoints of one row n of an atom (the terms of moment_adjoints
// for entries n*LM .. n*LM + LM - 1): Q = dE_i/dA[n][.] and Bp = dPsi/dA[n][.].
template <typename R, class Sh>
__device__ __forceinline__ void row_adjoints(int n, const R* __restrict__ A, const R* __restrict__ dA,
                                             const R* __restrict__ e, const R* __restrict__ ab, R (&Q)[Sh::LM],
                                             R (&Bp)[Sh::LM]) {
    constexpr int NR = Sh::NR, NA = Sh::NA, LM = Sh::LM, L = Sh::L;
    const R* __restrict__ An = A + n * LM;
    const R* __restrict__ dAn = dA + n * LM;
    R el[L], al[L];
#pragma unroll
    for (int l = 1; l <= L; ++l) {
        el[l - 1] = e[NR + (l - 1) * NA + n];
        al[l - 1] = ab[NR + (l - 1) * NA + n];
    }
    R a[LM], d[LM];
#pragma unroll
    for (int lm = 0; lm < LM; ++lm) {
        a[lm] = An[lm];
        d[lm] = dAn[lm];
    }
#pragma unroll
    for (int lm = 0; lm < LM; ++lm) {
        const int l = lm_degree<LM>(lm);
        Q[lm] = R(2) * el[l - 1] * a[lm];
        Bp[lm] = R(2) * al[l - 1] * a[lm] + R(2) * el[l - 1] * d[lm];
    }
    if (Sh::H4) {
        const int i4 = NR + L * NA + n;
        const R e4 = e[i4], a4 = ab[i4];
        R g4[5], h4[5];
        q4_grad<R>(a + 3, g4);
        q4_hess_vec<R>(a + 3, d + 3, h4);
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            Q[3 + m] += e4 * g4[m];
            Bp[3 + m] += a4 * g4[m] + e4 * h4[m];
        }
    }
    if (Sh::H5) {
        const int i5 = NR + (L + (Sh::H4 ? 1 : 0)) * NA + n;
        const R e5 = e[i5], a5 = ab[i5];
        const R P = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
        const R dd = a[0] * d[0] + a[1] * d[1] + a[2] * d[2];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            Q[m] += e5 * R(4) * P * a[m];
            Bp[m] += a5 * R(4) * P * a[m] + e5 * (R(8) * dd * a[m] + R(4) * P * d[m]);
        }
    }
}

// A small integer carried bit for bit in a slot's spare value.
template <typename R>
__device__ __forceinline__ R slot_tag(int b);
template <>
__device__ __forceinline__ float slot_tag<float>(int b) { return __int_as_float(b); }
template <>
__device__ __forceinline__ double slot_tag<double>(int b) { return __longlong_as_double((long long)b); }
template <typename R>
__device__ __forceinline__ int slot_untag(R v);
template <>
__device__ __forceinline__ int slot_untag<float>(float v) { return __float_as_int(v); }
template <>
__device__ __forceinline__ int slot_untag<double>(double v) { return (int)__double_as_longlong(v); }

// dL/dc_A[a][b][n][k] (the sum of k_angular_coeff_grad), rows per lane: a team
// of S = ceil(N_A / ROWS) lanes per atom, lane l holding rows
// n = l ROWS .. l ROWS + ROWS - 1 of the atom's Bp and Q in registers. Each
// batch, the team's lanes evaluate one pair each (basis, harmonics and their
// derivative along v) and publish (Y, v.dY, f, (v.r^) f', segment) in their
// LDS slots; every lane then runs the whole batch for its own rows, forming
// P_n and R_n in full, so the outer product over k needs neither an exchange
// nor a team sum. A batch takes the atom's next S angular pairs whatever
// their neighbour species; a lane adds its sums into the wavefront's
// accumulator G[a][b] (LDS atomics, in the wavefront's fixed instruction
// order: bitwise repeatable) when the pairs move to another segment b. Pair
// records are loaded two batches ahead and the neighbours' seeds one batch
// ahead. Each wavefront owns one G and walks its own tiles; the block's
// wavefronts add their G in wavefront order into the block's partial row.
template <typename R, class Sh, int ROWS>
__global__ void __launch_bounds__(kBlock)
k_angular_coeff_grad_rows(const Dims dm, const int* __restrict__ order, const int64_t* __restrict__ soff,
                          const int* __restrict__ atom_struct, int Na, const int64_t* __restrict__ row,
                          const int* __restrict__ seg, const Rec<R>* __restrict__ pairs,
                          const R* __restrict__ ubar, const double* __restrict__ Ubar, const R* __restrict__ A_in,
                          const R* __restrict__ dA_in, const R* __restrict__ e_in, const R* __restrict__ abar,
                          int group_tiles, double* __restrict__ partial) {
    constexpr int NA = Sh::NA, KA = Sh::KA, LM = Sh::LM, L = Sh::L, D = Sh::D;
    constexpr CgRowsGeom GM = cg_rows_slots(NA, KA, LM, int(sizeof(R)), ROWS);
    constexpr int S = GM.S, TEAMS = GM.teams, VEC = GM.vec, KFP = GM.kfp, SLOT = GM.slot, TSTRIDE = GM.tstride;
    static_assert(LM % VEC == 0 && KFP % VEC == 0 && SLOT % VEC == 0 && TSTRIDE % VEC == 0 && VEC % 2 == 0,
                  "vector layout");
    using V = typename VecOf<R>::type;
    using X = MomentExchange<R, NA, LM, S>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int T = dm.T;
    const CgRowsGeom gm = cg_rows_place(GM, T, NA, KA, int(sizeof(R)));
    const int nw = blockDim.x / 64, wave = threadIdx.x / 64, wl = threadIdx.x % 64;
    unsigned char* wbase = smem_raw + size_t(wave) * gm.wave_bytes;
    // the wavefront's accumulator for its current species a: G[b][n][k]
    R* G = reinterpret_cast<R*>(wbase);
    const int G_len = T * NA * KA;
    for (int x = wl; x < G_len; x += 64) G[x] = R(0);
    const int team = wl / S, lane = wl % S;
    const bool in_team = team < TEAMS;
    R* myslots = reinterpret_cast<R*>(wbase + gm.off_slots) + (in_team ? team : 0) * TSTRIDE;
    int* tab = reinterpret_cast<int*>(wbase + gm.off_tab) + (in_team ? team : 0) * (2 * T + 1);
    const R rcA = R(dm.rcA), irA = R(1.0 / dm.rcA);
    // tiles of TEAMS atoms of one species from the species-sorted list; each
    // wavefront walks one contiguous range of them (so it meets each species in
    // one run) and owns partial row gw, whose section for species a it writes
    // when its run of species a ends; sections it never meets are zero
    const int gw = blockIdx.x * nw + wave, GW = gridDim.x * nw;
    const int tiles_ub = (Na + TEAMS - 1) / TEAMS + T;
    const int per_wave = (tiles_ub + GW - 1) / GW;
    const int wave_end = min((gw + 1) * per_wave, tiles_ub);
    // With group_tiles > 0 (at most kCgSortTiles), the atoms of a group of up
    // to group_tiles consecutive tiles of one species are ordered by their
    // angular pair counts (largest first, ties in species order), then cut
    // into tiles again: the teams of a tile then have similar pair counts
    // and pad less at the end of their atoms. The group's tiles keep their
    // sizes and species; perm holds the order, keys (in the slots, free
    // between tiles) the counts. With 0 the tiles keep the species order.
    int* perm = reinterpret_cast<int*>(wbase + gm.off_perm);
    int* keys = reinterpret_cast<int*>(wbase + gm.off_slots);
    static_assert(size_t(kCgSortTiles) * TEAMS * 4 <= size_t(TEAMS) * TSTRIDE * sizeof(R), "keys fit the slots");
    int group_end = -1;
    long group_lo = 0;
    double* __restrict__ prow = partial + (long)gw * T * G_len;
    unsigned met = 0;  // species whose section this wavefront has written
    int cur_a = -1;
    auto flush_species = [&]() {
        if (cur_a < 0) return;
        X::wave_fence();
        for (int x = wl; x < G_len; x += 64) {
            prow[(long)cur_a * G_len + x] = double(G[x]);
            G[x] = R(0);
        }
        met |= 1u << cur_a;
        X::wave_fence();
    };
    for (int tile = gw * per_wave; tile < (gw + 1) * per_wave && tile < tiles_ub; ++tile) {
        int a;
        long lo = 0, hi = 0;
        species_chunk(soff, T, TEAMS, tile, &a, &lo, &hi);
        if (a < 0) break;
        if (a != cur_a) {
            flush_species();
            cur_a = a;
        }
        if (group_tiles > 0 && tile >= group_end) {
            // a new group: this tile and the next ones of species a in the
            // wavefront's range, at most kCgSortTiles
            const long a_hi = soff[a + 1];
            const int left = int((a_hi - lo + TEAMS - 1) / TEAMS);
            const int nt = min(min(group_tiles, left), wave_end - tile);
            const int n = int(min(a_hi, lo + long(nt) * TEAMS) - lo);
            group_end = tile + nt;
            group_lo = lo;
            for (int x = wl; x < n; x += 64) {
                const int ii = order[lo + x];
                int c = 0;
                for (int b = 0; b < T; ++b) c += seg[((long)ii * T + b) * 2 + 1];
                keys[x] = c;
            }
            X::wave_fence();
            for (int x = wl; x < n; x += 64) {
                const int kx = keys[x];
                int rk = 0;
                for (int y = 0; y < n; ++y) {
                    const int ky = keys[y];
                    rk += (ky > kx || (ky == kx && y < x)) ? 1 : 0;
                }
                perm[rk] = order[lo + x];
            }
            X::wave_fence();
        }
        const bool live = in_team && lo + team < hi;
        // The atom's data: every lane loads (a lane without an atom reads the
        // tile's first one, lo < hi, and drops what it read), so that the loads
        // go out together rather than one after another behind branches.
        const int k0 = int(lo - group_lo);
        const int i = group_tiles > 0 ? perm[k0 + (live ? team : 0)] : order[live ? lo + team : lo];
        const int s = atom_struct[i];
        const int64_t p0 = row[i];
        R ui[3], U[9];
#pragma unroll
        for (int d = 0; d < 3; ++d) ui[d] = ubar[(long)i * 3 + d];
#pragma unroll
        for (int c = 0; c < 9; ++c) U[c] = R(Ubar[(long)s * 9 + c]);
        if (live && lane == 0) {
            const int2* __restrict__ sg = reinterpret_cast<const int2*>(seg) + (long)i * T;
            int2 v[kMaxTypes];
#pragma unroll
            for (int b = 0; b < kMaxTypes; ++b) v[b] = sg[b < T ? b : T - 1];
            int cum = 0, pos = 0;
#pragma unroll
            for (int b = 0; b < kMaxTypes; ++b) {
                if (b < T) {
                    tab[b] = cum;
                    tab[T + 1 + b] = pos;
                    cum += v[b].y;
                    pos += v[b].x;
                }
            }
            tab[T] = cum;
        }
        // this lane's rows of the atom's moment adjoints (rows past N_A and
        // lanes without an atom load row N_A - 1 and keep zeros)
        R Q[ROWS][LM], Bp[ROWS][LM];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int n = lane * ROWS + r;
            const bool own = live && n < NA;
            row_adjoints<R, Sh>(n < NA ? n : NA - 1, A_in + (long)i * NA * LM, dA_in + (long)i * NA * LM,
                                e_in + (long)i * D, abar + (long)i * D, Q[r], Bp[r]);
#pragma unroll
            for (int lm = 0; lm < LM; ++lm) {
                Q[r][lm] = own ? Q[r][lm] : R(0);
                Bp[r][lm] = own ? Bp[r][lm] : R(0);
            }
        }
        X::wave_fence();
        // The atom's angular pairs in batches of S taken across its neighbour-
        // species segments (kappa = 0 .. A-1 numbers them segment after
        // segment): a batch pads only at the atom's end, not at every
        // segment's. locate(kappa) gives the pair's row index and segment b
        // from the team's table (cum[b] = first kappa of segment b).
        const int A = live ? tab[T] : 0;
        auto locate = [&](int kap, int* bo) -> int64_t {
            int bb = 0;
            for (int t = 1; t < T; ++t) bb = tab[t] <= kap ? t : bb;
            *bo = bb;
            return p0 + tab[T + 1 + bb] + (kap - tab[bb]);
        };
        // records of batches t and t+1 and the neighbours' seeds of t; a lane
        // past the atom's last pair reads that pair again and drops it
        int bA = 0, bB = 0;
        Rec<R> recA{}, recB{};
        R ujA[3] = {R(0), R(0), R(0)};
        if (A > 0) {
            recA = pairs[locate(lane < A ? lane : A - 1, &bA)];
            recB = pairs[locate(S + lane < A ? S + lane : A - 1, &bB)];
            const long j = rec_j(recA);
#pragma unroll
            for (int d = 0; d < 3; ++d) ujA[d] = ubar[j * 3 + d];
        }
        int cur_b = -1;
        R acc[ROWS][KA];
#pragma unroll
        for (int r = 0; r < ROWS; ++r)
#pragma unroll
            for (int k = 0; k < KA; ++k) acc[r][k] = R(0);
        auto flush = [&]() {
            if (cur_b < 0) return;
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const int n = lane * ROWS + r;
                if (n >= NA) continue;
                R* g = G + (cur_b * NA + n) * KA;
#pragma unroll
                for (int k = 0; k < KA; ++k) {
                    __hip_atomic_fetch_add(g + k, acc[r][k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    acc[r][k] = R(0);
                }
            }
        };
        for (int base = 0; base < A; base += S) {
            // loads for the next batches: the records of t+2, then the
            // neighbours' seeds of t+1 (issued last, so that waiting for them
            // at the next batch does not also wait for the records), by every
            // lane with no branch around them: the compiler then waits for
            // exactly the loads a value needs instead of all of them
            int bC;
            const int kC = base + 2 * S + lane;
            const Rec<R> recC = pairs[locate(kC < A ? kC : A - 1, &bC)];
            R ujB[3];
            {
                const long j = rec_j(recB);
#pragma unroll
                for (int d = 0; d < 3; ++d) ujB[d] = ubar[j * 3 + d];
            }
            // phase 1: this lane's pair of batch t into its slot, with its segment
            const int nq = A - base < S ? A - base : S;
            if (lane < nq) {
                const R rv[3] = {recA.x, recA.y, recA.z};
                const R r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
                const R ir = R(1) / r;
                const R u[3] = {rv[0] * ir, rv[1] * ir, rv[2] * ir};
                R v[3];
#pragma unroll
                for (int be = 0; be < 3; ++be)
                    v[be] = ui[be] - ujA[be] - (U[be] * rv[0] + U[3 + be] * rv[1] + U[6 + be] * rv[2]);
                const R vu = v[0] * u[0] + v[1] * u[1] + v[2] * u[2];
                // each value goes to the slot as soon as it is known, which keeps
                // the basis and the harmonics from being live at once
                // (whole 16-byte vectors: one LDS write per vector)
                V* sl = reinterpret_cast<V*>(myslots + lane * SLOT);
                {
                    R fa[KA], fap[KA];
                    cheb_basis<R, KA, true>(r, rcA, irA, fa, fap);
#pragma unroll
                    for (int c = 0; c < KFP / VEC; ++c) {
                        V w;
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            const int x = c * VEC + e, k = x / 2;
                            w[e] = k < KA ? ((x & 1) ? fap[k] * vu : fa[k]) : x == 2 * KA ? slot_tag<R>(bA) : R(0);
                        }
                        sl[2 * LM / VEC + c] = w;
                    }
                }
                const D1<R> dx = {u[0], v[0]}, dy = {u[1], v[1]}, dz = {u[2], v[2]};
                D1<R> Yd[LM];
                solid_harmonics<D1<R>, R, L>(dx, dy, dz, Yd);
#pragma unroll
                for (int c = 0; c < LM / VEC; ++c) {
                    V y, dv;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const int lm = c * VEC + e;
                        y[e] = Yd[lm].v;
                        dv[e] = (Yd[lm].d - R(lm_degree<LM>(lm)) * Yd[lm].v * vu) * ir;
                    }
                    sl[c] = y;
                    sl[LM / VEC + c] = dv;
                }
            }
            X::wave_fence();
            // phase 2: the batch's pairs for this lane's rows; the sums go to
            // G[a][b] whenever the pairs move to another segment b
#pragma unroll 1
            for (int q = 0; q < nq; ++q) {
                const V* sl = reinterpret_cast<const V*>(myslots + q * SLOT);
                R pn[ROWS], rn[ROWS];
#pragma unroll
                for (int r = 0; r < ROWS; ++r) pn[r] = rn[r] = R(0);
#pragma unroll
                for (int c = 0; c < LM / VEC; ++c) {
                    const V y = sl[c], dv = sl[LM / VEC + c];
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
#pragma unroll
                        for (int r = 0; r < ROWS; ++r) {
                            // one fused multiply-add per term
                            pn[r] += Bp[r][c * VEC + e] * y[e];
                            pn[r] += Q[r][c * VEC + e] * dv[e];
                            rn[r] += Q[r][c * VEC + e] * y[e];
                        }
                }
                const int bq = slot_untag<R>(myslots[q * SLOT + 2 * LM + 2 * KA]);
                if (bq != cur_b) {
                    flush();
                    cur_b = bq;
                }
#pragma unroll
                for (int c = 0; c < KFP / VEC; ++c) {
                    const V w = sl[2 * LM / VEC + c];  // (f_k, (v.r^) f'_k) pairs
#pragma unroll
                    for (int e = 0; e < VEC; e += 2) {
                        const int k = (c * VEC + e) / 2;
                        if (k >= KA) continue;
#pragma unroll
                        for (int r = 0; r < ROWS; ++r) {
                            acc[r][k] += pn[r] * w[e];
                            acc[r][k] += rn[r] * w[e + 1];
                        }
                    }
                }
            }
            X::wave_fence();
            recA = recB;
            recB = recC;
            bA = bB;
            bB = bC;
#pragma unroll
            for (int d = 0; d < 3; ++d) ujA[d] = ujB[d];
        }
        flush();
        X::wave_fence();
    }
    flush_species();
    for (int t = 0; t < T; ++t)
        if (!(met >> t & 1u))
            for (int x = wl; x < G_len; x += 64) prow[(long)t * G_len + x] = 0.0;
}

// ------------------------------------------ network and radial coefficient grad

// Matrix-core tile C[M][M] += A[M][KPI] B[KPI][M] of one wavefront.
// FP32: v_mfma_f32_32x32x2f32 (M = 32, K = 2 per instruction);
// FP64: v_mfma_f64_16x16x4f64 (M = 16, K = 4 per instruction).
// Operand lane l supplies A[l mod M][l / M] and B[l / M][l mod M]; accumulator
// register v of lane l holds C[c_row(l, v)][l mod M].
template <typename R>
struct Mfma;

template <>
struct Mfma<float> {
    static constexpr int M = 32, KPI = 2, NV = 16;
    typedef float Acc __attribute__((ext_vector_type(16)));
    __device__ static Acc mma(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }
    __device__ static int c_row(int lane, int v) { return (v & 3) + 4 * (lane >> 5) + 8 * (v >> 2); }
};

template <>
struct Mfma<double> {
    static constexpr int M = 16, KPI = 4, NV = 4;
    typedef double Acc __attribute__((ext_vector_type(4)));
    __device__ static Acc mma(double a, double b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int c_row(int lane, int v) { return 4 * v + (lane >> 4); }
};

// For the per-atom outer products sum_i X1_i (x) Y1_i + X2_i (x) Y2_i the K
// slots of one instruction are (atom, term) pairs: KPI / 2 atoms per instruction.
template <typename R>
struct OuterMma : Mfma<R> {
    static constexpr int ATOMS = Mfma<R>::KPI / 2;
    __device__ static int slot_atom(int lane) { return (lane / Mfma<R>::M) >> 1; }
    __device__ static int slot_term(int lane) { return (lane / Mfma<R>::M) & 1; }
};

// One partial row per work item (a chunk of atoms of one species a):
//   row[0] = a (or -1 for an empty item), then W1 = (D+2) H + T NR KR columns:
//   W0[mu][nu] = sum_i alpha_mu (s q)_nu + beta_mu (s dq)_nu     (matrix cores),
//   b0[mu] = -sum_i alpha_mu, w1[mu] = sum_i gamma_mu,
//   c_R[a][b][n][k] = sum_i abar_n S0[b][k] + e_n S1[b][k]        (matrix cores).
// The block walks its chunk in sub-chunks of SC atoms (32 in FP32 when their
// operand rows fit 64 KB of LDS, else 16, so that rows of wide networks and
// many species still leave room for several blocks per CU): every operand row of a
// sub-chunk is copied once into LDS with coalesced loads (rows of the
// per-unit arrays are contiguous in the species-sorted list), then each wave
// updates the 32 x 32 (16 x 16 in FP64) output tiles it owns from LDS. A tile
// belongs to one wave for the whole chunk, so its sums need no cross-wave step.
template <typename R, int SC_ = 16>
struct OuterTiles {
    static constexpr int SC = SC_;  // atoms per staged sub-chunk
    static constexpr int MAXTW = 6;                        // tiles per wave at most
    // accumulator slots the kernel is built with for a network: the smallest
    // of 1, 2, 4, 6 covering its tiles (fewer slots, fewer registers)
    __host__ __device__ static int tiles_per_wave(const Dims& d) {
        const int t = (tiles(d) + WAVES - 1) / WAVES;
        return t <= 1 ? 1 : t <= 2 ? 2 : t <= 4 ? 4 : 6;
    }
    static constexpr int WAVES = kBlock / 64;
    __host__ __device__ static int floats_per_atom(const Dims& d) {
        return 3 * d.H + 2 * d.D + 2 * d.NR + 2 * d.T * d.KR;
    }
    __host__ __device__ static size_t lds_bytes(const Dims& d) { return sizeof(R) * size_t(SC) * floats_per_atom(d); }
    __host__ __device__ static int tiles(const Dims& d) {
        const int M = Mfma<R>::M;
        return ((d.H + M - 1) / M) * ((d.D + M - 1) / M) + ((d.NR + M - 1) / M) * ((d.T * d.KR + M - 1) / M);
    }
};

template <typename R, class Sh, int MAXTW, int SCA>
__global__ void __launch_bounds__(kBlock)
k_outer_grad(const Dims dm, const R* __restrict__ qscale, const int* __restrict__ order,
             const int64_t* __restrict__ soff, int chunk, const R* __restrict__ q_in, const R* __restrict__ dq_in,
             const R* __restrict__ abar, const R* __restrict__ e_in, const R* __restrict__ alpha,
             const R* __restrict__ beta, const R* __restrict__ gam, const R* __restrict__ S0,
             const R* __restrict__ S1, int units_by_atom, double* __restrict__ partial) {
    using MM = OuterMma<R>;
    using OT = OuterTiles<R, SCA>;
    constexpr int M = MM::M, NR = Sh::NR, KR = Sh::KR, D = Sh::D, SC = OT::SC;
    constexpr int WAVES = OT::WAVES, KSTEPS = 2 * SC / MM::KPI;
    extern __shared__ __align__(16) unsigned char outer_smem[];
    const int T = dm.T, H = dm.H, TK = T * KR;
    const int W1 = (D + 2) * H + T * NR * KR;
    double* __restrict__ rowp = partial + (long)blockIdx.x * (W1 + 1);
    int a;
    long lo = 0, hi = 0;
    species_chunk(soff, T, chunk, blockIdx.x, &a, &lo, &hi);
    if (threadIdx.x == 0) rowp[0] = double(a);
    if (a < 0) return;
    // LDS sub-chunk: alpha, beta, gamma [SC][H]; s q, s dq [SC][D]; abar, e [SC][NR]; S0, S1 [SC][TK]
    R* Xa = reinterpret_cast<R*>(outer_smem);
    R* Xb = Xa + SC * H;
    R* Xg = Xb + SC * H;
    R* Yq = Xg + SC * H;
    R* Yd = Yq + SC * D;
    R* Ra = Yd + SC * D;
    R* Re = Ra + SC * NR;
    R* C0 = Re + SC * NR;
    R* C1 = C0 + SC * TK;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int srow = lane % M, satom = MM::slot_atom(lane), sterm = MM::slot_term(lane);
    const int tilesD = (D + M - 1) / M, tilesC = (TK + M - 1) / M;
    const int nW = ((H + M - 1) / M) * tilesD, ntiles = nW + ((NR + M - 1) / M) * tilesC;
    typename MM::Acc acc[MAXTW];
#pragma unroll
    for (int k = 0; k < MAXTW; ++k)
#pragma unroll
        for (int v = 0; v < MM::NV; ++v) acc[k][v] = R(0);
    // atom index of each sub-chunk slot, double-buffered: the next
    // sub-chunk's indices load during the current staging. Slots
    // past the chunk hold 0, a valid atom, so every staging load below is
    // unconditional (its value is then replaced by zero).
    __shared__ int ord[2][SC];
    if (threadIdx.x < SC) ord[0][threadIdx.x] = lo + threadIdx.x < hi ? order[lo + threadIdx.x] : 0;
    int buf = 0;
    constexpr int U = 4;  // staging iterations whose loads are issued together
    R sa = R(0), sg = R(0);  // b0 / w1 column sums of unit mu = threadIdx.x (H <= kBlock)
    for (long s0 = lo; s0 < hi; s0 += SC, buf ^= 1) {
        const int n = int(hi - s0 < SC ? hi - s0 : SC);
        const int* os = ord[buf];
        __syncthreads();
        // the next sub-chunk's atom indices, issued before this one's staging
        int nxt = 0;
        if (threadIdx.x < SC && s0 + SC + threadIdx.x < hi) nxt = order[s0 + SC + threadIdx.x];
        // One staging loop for every operand array: each thread first issues
        // the loads of U iterations of all of them (slots past an array's
        // end read its element 0 and are not stored), then stores them, so a
        // sub-chunk costs one memory wait per thread, not one per array.
        // Per-unit rows are contiguous in the species-sorted list, or
        // (written by the sweeps) indexed by atom; per-atom rows are gathered
        // by atom index.
        const int nX = SC * H, nY = SC * D, nR = SC * NR, nC = SC * TK;
        const int nMax = nX > nY ? (nX > nC ? nX : nC) : (nY > nC ? nY : nC);
        for (int x0 = threadIdx.x; x0 < nMax; x0 += U * kBlock) {
            R va[U], vb[U], vg[U], vq[U], vd[U], ra[U], re[U], c0[U], c1[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int x = x0 + u * kBlock;
                {
                    const bool in = x < n * H;
                    const int sl = in ? x / H : 0, c = in ? x % H : 0;
                    const long src = units_by_atom ? long(os[sl]) * H + c : (s0 + sl) * H + c;
                    va[u] = alpha[src];
                    vb[u] = beta[src];
                    vg[u] = gam[src];
                }
                {
                    const bool in = x < n * D;
                    const int v = in ? x % D : 0;
                    const long i = os[in ? x / D : 0];
                    const R sv = qscale[v];
                    vq[u] = sv * q_in[i * D + v];
                    vd[u] = sv * dq_in[i * D + v];
                }
                {
                    const bool in = x < n * NR;
                    const int r = in ? x % NR : 0;
                    const long i = os[in ? x / NR : 0];
                    ra[u] = abar[i * D + r];
                    re[u] = e_in[i * D + r];
                }
                {
                    const bool in = x < n * TK;
                    const int c = in ? x % TK : 0;
                    const long i = os[in ? x / TK : 0];
                    c0[u] = S0[i * TK + c];
                    c1[u] = S1[i * TK + c];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int x = x0 + u * kBlock;
                if (x < nX) {
                    const bool in = x < n * H;
                    Xa[x] = in ? va[u] : R(0);
                    Xb[x] = in ? vb[u] : R(0);
                    Xg[x] = in ? vg[u] : R(0);
                }
                if (x < nY) {
                    const bool in = x < n * D;
                    Yq[x] = in ? vq[u] : R(0);
                    Yd[x] = in ? vd[u] : R(0);
                }
                if (x < nR) {
                    const bool in = x < n * NR;
                    Ra[x] = in ? ra[u] : R(0);
                    Re[x] = in ? re[u] : R(0);
                }
                if (x < nC) {
                    const bool in = x < n * TK;
                    C0[x] = in ? c0[u] : R(0);
                    C1[x] = in ? c1[u] : R(0);
                }
            }
        }
        if (threadIdx.x < SC) ord[buf ^ 1][threadIdx.x] = nxt;
        __syncthreads();
        if (threadIdx.x < H)
            for (int sl = 0; sl < n; ++sl) {
                sa += Xa[sl * H + threadIdx.x];
                sg += Xg[sl * H + threadIdx.x];
            }
#pragma unroll
        for (int k = 0; k < MAXTW; ++k) {
            const int tl = wave + WAVES * k;
            if (tl >= ntiles) continue;
            const bool wtile = tl < nW;
            const int r0 = (wtile ? tl / tilesD : (tl - nW) / tilesC) * M;
            const int c0 = (wtile ? tl % tilesD : (tl - nW) % tilesC) * M;
            const int rr = r0 + srow, cc = c0 + srow;
            const int RN = wtile ? H : NR, CN = wtile ? D : TK;
            const R* Xs = wtile ? (sterm ? Xb : Xa) : (sterm ? Re : Ra);
            const R* Ys = wtile ? (sterm ? Yd : Yq) : (sterm ? C1 : C0);
#pragma unroll 4
            for (int kb = 0; kb < KSTEPS; ++kb) {
                const int sl = kb * MM::ATOMS + satom;
                const R xv = rr < RN ? Xs[sl * RN + rr] : R(0);
                const R yv = cc < CN ? Ys[sl * CN + cc] : R(0);
                acc[k] = MM::mma(xv, yv, acc[k]);
            }
        }
    }
    // each wave writes the tiles it owns
#pragma unroll
    for (int k = 0; k < MAXTW; ++k) {
        const int tl = wave + WAVES * k;
        if (tl >= ntiles) continue;
        const bool wtile = tl < nW;
        const int r0 = (wtile ? tl / tilesD : (tl - nW) / tilesC) * M;
        const int c0 = (wtile ? tl % tilesD : (tl - nW) % tilesC) * M;
#pragma unroll
        for (int v = 0; v < MM::NV; ++v) {
            const int r = r0 + MM::c_row(lane, v), c = c0 + lane % M;
            if (wtile) {
                if (r < H && c < D) rowp[1 + r * D + c] = double(acc[k][v]);
            } else if (r < NR && c < TK) {
                const int b = c / KR, kk = c % KR;
                rowp[1 + (D + 2) * H + (b * NR + r) * KR + kk] = double(acc[k][v]);
            }
        }
    }
    if (threadIdx.x < H) {
        rowp[1 + H * D + threadIdx.x] = -double(sa);
        rowp[1 + H * D + H + threadIdx.x] = double(sg);
    }
}

// ------------------------------------------------- network on matrix cores

// One 64-lane block per tile of M atoms of one species (species-sorted list).
// The hidden pre-activations are computed transposed, a^T = W0 (s q)^T, so the
// M x M accumulator holds hidden rows x atom columns and each atom's values
// sit in the lanes that share its column. The second product of each pass
// (W0^T times a per-hidden-unit factor) is fed through an LDS transpose.

// Per-hidden-unit arrays (t, alpha, beta, gamma) are stored by position in the
// species-sorted atom list, row s = H units. A block's M atoms are rows
// lo .. lo + nat - 1, so its tile is one contiguous span: it moves through an
// LDS tile [atom][unit] (padded to M + 1) with whole-line coalesced accesses.
template <typename R, int M>
__device__ __forceinline__ void store_unit_tile(const R* tile, R* __restrict__ out, long lo, int nat, int H,
                                                int mu0, int lane) {
    const int nrow = H - mu0 < M ? H - mu0 : M;
    for (int x = lane; x < nat * nrow; x += 64) {
        const int jj = x / nrow, r = x % nrow;
        out[(lo + jj) * H + mu0 + r] = tile[jj * (M + 1) + r];
    }
}

template <typename R, int M>
__device__ __forceinline__ void load_unit_tile(const R* __restrict__ in, R* tile, long lo, int nat, int H, int mu0,
                                               int lane) {
    const int nrow = H - mu0 < M ? H - mu0 : M;
    for (int x = lane; x < nat * nrow; x += 64) {
        const int jj = x / nrow, r = x % nrow;
        tile[jj * (M + 1) + r] = in[(lo + jj) * H + mu0 + r];
    }
}

// E_i, e_i = dE_i/dq_i and tanh activations (Eqs. 2-3).
template <typename R, class Sh>
__global__ void __launch_bounds__(64)
k_network_forward(const Dims dm, const R* __restrict__ theta, const R* __restrict__ qscale,
                  const int* __restrict__ order, const int64_t* __restrict__ soff, const R* __restrict__ q_in,
                  R* __restrict__ E_out, R* __restrict__ e_out, R* __restrict__ t_out) {
    using MM = Mfma<R>;
    constexpr int M = MM::M, KPI = MM::KPI, NV = MM::NV, D = Sh::D;
    constexpr int DT = (D + M - 1) / M, DK = (D + KPI - 1) / KPI;
    __shared__ R cbuf[M * M];
    __shared__ R obuf[M * (M + 1)];
    const int T = dm.T, H = dm.H;
    int a;
    long lo = 0, hi = 0;
    species_chunk(soff, T, M, blockIdx.x, &a, &lo, &hi);
    if (a < 0) return;
    const int lane = threadIdx.x, j = lane % M, kk = lane / M;
    const long ia = (lo + j < hi) ? long(order[lo + j]) : -1;
    const int nat = int(hi - lo < M ? hi - lo : M);
    const R* __restrict__ W0 = theta + dm.offN + (long)a * (D + 2) * H;
    const R* __restrict__ b0 = W0 + (long)H * D;
    const R* __restrict__ w1 = b0 + H;
    R qk[DK];
#pragma unroll
    for (int s = 0; s < DK; ++s) {
        const int k = s * KPI + kk;
        qk[s] = (ia >= 0 && k < D) ? qscale[k] * q_in[ia * D + k] : R(0);
    }
    typename MM::Acc eacc[DT];
#pragma unroll
    for (int dt = 0; dt < DT; ++dt)
#pragma unroll
        for (int v = 0; v < NV; ++v) eacc[dt][v] = R(0);
    R Ej = R(0);
    for (int mu0 = 0; mu0 < H; mu0 += M) {
        typename MM::Acc acc;
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = R(0);
        const int mrow = mu0 + j;
#pragma unroll
        for (int s = 0; s < DK; ++s) {
            const int k = s * KPI + kk;
            const R x = (mrow < H && k < D) ? W0[(long)mrow * D + k] : R(0);
            acc = MM::mma(x, qk[s], acc);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int r = MM::c_row(lane, v), mu = mu0 + r;
            R c = R(0);
            if (mu < H) {
                const R t = tanh_<R>(acc[v] - b0[mu]);
                obuf[j * (M + 1) + r] = t;
                const R w = w1[mu];
                Ej += w * t;
                c = w * (R(1) - t * t);
            }
            cbuf[r * M + j] = c;
        }
        __syncthreads();
        store_unit_tile<R, M>(obuf, t_out, lo, nat, H, mu0, lane);
#pragma unroll
        for (int dt = 0; dt < DT; ++dt) {
            const int nu = dt * M + j;
#pragma unroll
            for (int s = 0; s < M / KPI; ++s) {
                const int k = s * KPI + kk;
                const R x = (nu < D && mu0 + k < H) ? W0[(long)(mu0 + k) * D + nu] : R(0);
                eacc[dt] = MM::mma(x, cbuf[k * M + j], eacc[dt]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int o = M; o < 64; o <<= 1) Ej += __shfl_xor(Ej, o, 64);
    if (kk == 0 && ia >= 0) E_out[ia] = Ej - theta[dm.offB1];
#pragma unroll
    for (int dt = 0; dt < DT; ++dt)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int nu = dt * M + MM::c_row(lane, v);
            if (nu < D && ia >= 0) e_out[ia * D + nu] = qscale[nu] * eacc[dt][v];
        }
}

// For Psi = sum_i ebar_s E_i + e(q_i) . dq_i (the force/virial adjoint): the
// Hessian-vector product da = W0 (s dq), per-unit weight-gradient factors
// alpha = w1 s'(ebar - 2 t da), beta = w1 s', gamma = ebar t + s' da, and
// abar = dPsi/dq = ebar e + s (W0^T (-2 w1 t s' da)).
template <typename R, class Sh>
__global__ void __launch_bounds__(64)
k_network_backward(const Dims dm, const R* __restrict__ theta, const R* __restrict__ qscale,
                   const int* __restrict__ order, const int64_t* __restrict__ soff, const int* __restrict__ atom_struct,
                   const double* __restrict__ ebar_s, const R* __restrict__ dq_in, const R* __restrict__ e_in,
                   const R* __restrict__ t_in, R* __restrict__ abar_out, R* __restrict__ alpha_out,
                   R* __restrict__ beta_out, R* __restrict__ gamma_out) {
    using MM = Mfma<R>;
    constexpr int M = MM::M, KPI = MM::KPI, NV = MM::NV, D = Sh::D;
    constexpr int DT = (D + M - 1) / M, DK = (D + KPI - 1) / KPI;
    __shared__ R cbuf[M * M];
    __shared__ R obuf[4][M * (M + 1)];
    const int T = dm.T, H = dm.H;
    int a;
    long lo = 0, hi = 0;
    species_chunk(soff, T, M, blockIdx.x, &a, &lo, &hi);
    if (a < 0) return;
    const int lane = threadIdx.x, j = lane % M, kk = lane / M;
    const long ia = (lo + j < hi) ? long(order[lo + j]) : -1;
    const int nat = int(hi - lo < M ? hi - lo : M);
    const R eb = ia >= 0 ? R(ebar_s[atom_struct[ia]]) : R(0);
    const R* __restrict__ W0 = theta + dm.offN + (long)a * (D + 2) * H;
    const R* __restrict__ w1 = W0 + (long)H * D + H;
    R dk[DK];
#pragma unroll
    for (int s = 0; s < DK; ++s) {
        const int k = s * KPI + kk;
        dk[s] = (ia >= 0 && k < D) ? qscale[k] * dq_in[ia * D + k] : R(0);
    }
    typename MM::Acc zacc[DT];
#pragma unroll
    for (int dt = 0; dt < DT; ++dt)
#pragma unroll
        for (int v = 0; v < NV; ++v) zacc[dt][v] = R(0);
    for (int mu0 = 0; mu0 < H; mu0 += M) {
        load_unit_tile<R, M>(t_in, obuf[3], lo, nat, H, mu0, lane);
        typename MM::Acc acc;
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = R(0);
        const int mrow = mu0 + j;
#pragma unroll
        for (int s = 0; s < DK; ++s) {
            const int k = s * KPI + kk;
            const R x = (mrow < H && k < D) ? W0[(long)mrow * D + k] : R(0);
            acc = MM::mma(x, dk[s], acc);
        }
        __syncthreads();
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int r = MM::c_row(lane, v), mu = mu0 + r;
            R c2 = R(0);
            if (mu < H && ia >= 0) {
                const R t = obuf[3][j * (M + 1) + r], sp = R(1) - t * t, w = w1[mu], da = acc[v];
                obuf[0][j * (M + 1) + r] = w * sp * (eb - R(2) * t * da);
                obuf[1][j * (M + 1) + r] = w * sp;
                obuf[2][j * (M + 1) + r] = eb * t + sp * da;
                c2 = R(-2) * w * t * sp * da;
            }
            cbuf[r * M + j] = c2;
        }
        __syncthreads();
        store_unit_tile<R, M>(obuf[0], alpha_out, lo, nat, H, mu0, lane);
        store_unit_tile<R, M>(obuf[1], beta_out, lo, nat, H, mu0, lane);
        store_unit_tile<R, M>(obuf[2], gamma_out, lo, nat, H, mu0, lane);
#pragma unroll
        for (int dt = 0; dt < DT; ++dt) {
            const int nu = dt * M + j;
#pragma unroll
            for (int s = 0; s < M / KPI; ++s) {
                const int k = s * KPI + kk;
                const R x = (nu < D && mu0 + k < H) ? W0[(long)(mu0 + k) * D + nu] : R(0);
                zacc[dt] = MM::mma(x, cbuf[k * M + j], zacc[dt]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int dt = 0; dt < DT; ++dt)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int nu = dt * M + MM::c_row(lane, v);
            if (nu < D && ia >= 0) abar_out[ia * D + nu] = eb * e_in[ia * D + nu] + qscale[nu] * zacc[dt][v];
        }
}

// ------------------------------------------------- network, one lane per atom

// The same network passes with one lane per atom: a block is one wavefront of
// up to 64 atoms of one species (species-sorted list), so every lane reads the
// same weight row at the same time (wave-uniform addresses, scalar loads) and
// the loop over hidden units needs no exchange between lanes. Per-unit values
// go through an LDS tile [atom][unit] to whole-line stores.
template <typename R>
struct LaneNet {
    static constexpr int MC = sizeof(R) == 4 ? 32 : 16;  // hidden units per LDS tile
    // the backward pass stages three outputs per unit: half the units per
    // tile keep its LDS (13 KB per FP32 wavefront) from capping the waves
    // per SIMD below what its registers allow
    static constexpr int MCB = MC / 2;
    static_assert((MC & (MC - 1)) == 0 && (MCB & (MCB - 1)) == 0, "unit tiles of a power of two");
};

template <typename R, class Sh>
__global__ void __launch_bounds__(64)
k_network_forward_lane(const Dims dm, const R* __restrict__ theta, const R* __restrict__ qscale,
                       const int* __restrict__ order, const int64_t* __restrict__ soff, const R* __restrict__ q_in,
                       R* __restrict__ E_out, R* __restrict__ e_out, R* __restrict__ t_out) {
    constexpr int D = Sh::D, MC = LaneNet<R>::MC;
    __shared__ R tb[64 * (MC + 1)];
    const int T = dm.T, H = dm.H;
    int a;
    long lo = 0, hi = 0;
    species_chunk(soff, T, 64, blockIdx.x, &a, &lo, &hi);
    if (a < 0) return;
    const int l = threadIdx.x;
    const int nat = int(hi - lo);
    const bool live = l < nat;
    const long ia = order[live ? lo + l : lo];
    const R* __restrict__ W0 = theta + dm.offN + (long)a * (D + 2) * H;
    const R* __restrict__ b0 = W0 + (long)H * D;
    const R* __restrict__ w1 = b0 + H;
    R qv[D], ev[D];
#pragma unroll
    for (int v = 0; v < D; ++v) {
        qv[v] = qscale[v] * q_in[ia * D + v];
        ev[v] = R(0);
    }
    R E = R(0);
    for (int mu0 = 0; mu0 < H; mu0 += MC) {
        const int mn = H - mu0 < MC ? H - mu0 : MC;
        for (int m = 0; m < mn; ++m) {
            const R* __restrict__ w = W0 + (long)(mu0 + m) * D;
            R acc = -b0[mu0 + m];
#pragma unroll
            for (int v = 0; v < D; ++v) acc += w[v] * qv[v];
            const R t = tanh_<R>(acc);
            const R wm = w1[mu0 + m];
            E += wm * t;
            const R c = wm * (R(1) - t * t);
#pragma unroll
            for (int v = 0; v < D; ++v) ev[v] += w[v] * c;
            tb[l * (MC + 1) + m] = t;
        }
        __syncthreads();
        // element x of the tile is unit x % MC of atom x / MC (MC a power of
        // two: shifts, no division); units past the layer's end are skipped
        for (int x = l; x < nat * MC; x += 64) {
            const int sl = x / MC, m = x % MC;
            if (m < mn) t_out[(lo + sl) * H + mu0 + m] = tb[sl * (MC + 1) + m];
        }
        __syncthreads();
    }
    if (!live) return;
    E_out[ia] = E - theta[dm.offB1];
#pragma unroll
    for (int v = 0; v < D; ++v) e_out[ia * D + v] = qscale[v] * ev[v];
}

template <typename R, class Sh>
__global__ void __launch_bounds__(64)
k_network_backward_lane(const Dims dm, const R* __restrict__ theta, const R* __restrict__ qscale,
                        const int* __restrict__ order, const int64_t* __restrict__ soff,
                        const int* __restrict__ atom_struct, const double* __restrict__ ebar_s,
                        const R* __restrict__ dq_in, const R* __restrict__ e_in, const R* __restrict__ t_in,
                        R* __restrict__ abar_out, R* __restrict__ alpha_out, R* __restrict__ beta_out,
                        R* __restrict__ gamma_out) {
    constexpr int D = Sh::D, MC = LaneNet<R>::MCB, LD = MC + 1;
    __shared__ R tb[3][64 * LD];
    const int T = dm.T, H = dm.H;
    int a;
    long lo = 0, hi = 0;
    species_chunk(soff, T, 64, blockIdx.x, &a, &lo, &hi);
    if (a < 0) return;
    const int l = threadIdx.x;
    const int nat = int(hi - lo);
    const bool live = l < nat;
    const long ia = order[live ? lo + l : lo];
    const R eb = live ? R(ebar_s[atom_struct[ia]]) : R(0);
    const R* __restrict__ W0 = theta + dm.offN + (long)a * (D + 2) * H;
    const R* __restrict__ w1 = W0 + (long)H * D + H;
    R dk[D], z[D];
#pragma unroll
    for (int v = 0; v < D; ++v) {
        dk[v] = qscale[v] * dq_in[ia * D + v];
        z[v] = R(0);
    }
    for (int mu0 = 0; mu0 < H; mu0 += MC) {
        const int mn = H - mu0 < MC ? H - mu0 : MC;
        // the tile's activations t[atom][unit], read along the atoms' rows
        // (coalesced) into the gamma tile, whose slot each unit overwrites
        // after reading it; the unit loop then stays rolled, so each weight
        // row arrives in a few wide scalar loads
        for (int x = l; x < nat * MC; x += 64) {
            const int sl = x / MC, m = x % MC;
            if (m < mn) tb[2][sl * LD + m] = t_in[(lo + sl) * H + mu0 + m];
        }
        __syncthreads();
        for (int m = 0; m < mn; ++m) {
            const R* __restrict__ w = W0 + (long)(mu0 + m) * D;
            R da = R(0);
#pragma unroll
            for (int v = 0; v < D; ++v) da += w[v] * dk[v];
            const R t = live ? tb[2][l * LD + m] : R(0);
            const R sp = R(1) - t * t, wm = w1[mu0 + m];
            tb[0][l * LD + m] = wm * sp * (eb - R(2) * t * da);
            tb[1][l * LD + m] = wm * sp;
            tb[2][l * LD + m] = eb * t + sp * da;
            const R c2 = R(-2) * wm * t * sp * da;
#pragma unroll
            for (int v = 0; v < D; ++v) z[v] += w[v] * c2;
        }
        __syncthreads();
        for (int x = l; x < nat * MC; x += 64) {
            const int sl = x / MC, m = x % MC;
            if (m < mn) {
                const long o = (lo + sl) * H + mu0 + m;
                alpha_out[o] = tb[0][sl * LD + m];
                beta_out[o] = tb[1][sl * LD + m];
                gamma_out[o] = tb[2][sl * LD + m];
            }
        }
        __syncthreads();
    }
    if (!live) return;
#pragma unroll
    for (int v = 0; v < D; ++v) abar_out[ia * D + v] = eb * e_in[ia * D + v] + qscale[v] * z[v];
}

}  // namespace nep
