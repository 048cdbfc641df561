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

// ------------------------------------------------------------------ descriptor

// q (radial, Eqs. 15-16; angular invariants, Eqs. 19-20 and the 4/5-body
// contractions), the angular moments A[n][lm], and the per-neighbour-species
// radial basis sums S0[b][k] = sum_{j in b} f_k(r_ij) used by the gradient.
template <typename R, class Sh, int S>
__global__ void __launch_bounds__(kBlock)
k_descriptor(const Dims dm, const R* __restrict__ theta, const int* __restrict__ types, int Na,
             const int64_t* __restrict__ row, const int* __restrict__ seg, const Rec<R>* __restrict__ pairs,
             R* __restrict__ q_out, R* __restrict__ A_out, R* __restrict__ S0_out) {
    constexpr int NR = Sh::NR, NA = Sh::NA, KR = Sh::KR, KA = Sh::KA, LM = Sh::LM, D = Sh::D;
    const int team = threadIdx.x / S, lane = threadIdx.x % S;
    const int i = blockIdx.x * (kBlock / S) + team;
    const bool live = i < Na;
    const int T = dm.T;
    const R rcR = R(dm.rcR), rcA = R(dm.rcA), irR = R(1.0 / dm.rcR), irA = R(1.0 / dm.rcA);
    const int a = live ? types[i] : 0;
    int64_t p = live ? row[i] : 0;
    R qR[NR];
    R A[NA][LM];
#pragma unroll
    for (int n = 0; n < NR; ++n) qR[n] = R(0);
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int lm = 0; lm < LM; ++lm) A[n][lm] = R(0);

    for (int b = 0; b < T; ++b) {
        const int tot = live ? seg[(i * T + b) * 2] : 0;
        const int ang = live ? seg[(i * T + b) * 2 + 1] : 0;
        const R* __restrict__ cA = theta + dm.offA + (long)((a * T + b) * NA) * KA;
        R Sb[KR];
#pragma unroll
        for (int k = 0; k < KR; ++k) Sb[k] = R(0);
        for (int k = lane; k < tot; k += S) {
            const Rec<R> pr = pairs[p + k];
            const R r = sqrt(pr.x * pr.x + pr.y * pr.y + pr.z * pr.z);
            R f[KR];
            cheb_basis<R, KR, false>(r, rcR, irR, f, nullptr);
#pragma unroll
            for (int kk = 0; kk < KR; ++kk) Sb[kk] += f[kk];
            if (k < ang) {
                R fa[KA];
                cheb_basis<R, KA, false>(r, rcA, irA, fa, nullptr);
                const R ir = R(1) / r;
                const R ux = pr.x * ir, uy = pr.y * ir, uz = pr.z * ir;
                R Y[LM];
                solid_harmonics<R, R, Sh::L>(ux, uy, uz, Y);
#pragma unroll
                for (int n = 0; n < NA; ++n) {
                    R g = R(0);
#pragma unroll
                    for (int kk = 0; kk < KA; ++kk) g += cA[n * KA + kk] * fa[kk];
#pragma unroll
                    for (int lm = 0; lm < LM; ++lm) A[n][lm] += g * Y[lm];
                }
            }
        }
        p += tot;
#pragma unroll
        for (int kk = 0; kk < KR; ++kk) Sb[kk] = team_sum<S>(Sb[kk]);
        const R* __restrict__ cR = theta + (long)((a * T + b) * NR) * KR;
#pragma unroll
        for (int n = 0; n < NR; ++n)
#pragma unroll
            for (int kk = 0; kk < KR; ++kk) qR[n] += cR[n * KR + kk] * Sb[kk];
        if (live) {
#pragma unroll
            for (int kk = 0; kk < KR; ++kk)
                if (kk % S == lane) S0_out[((long)i * T + b) * KR + kk] = Sb[kk];
        }
    }
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int lm = 0; lm < LM; ++lm) A[n][lm] = team_sum<S>(A[n][lm]);

    R q[D];
#pragma unroll
    for (int n = 0; n < NR; ++n) q[n] = qR[n];
#pragma unroll
    for (int n = 0; n < NA; ++n) {
#pragma unroll
        for (int l = 1; l <= Sh::L; ++l) {
            R s = R(0);
#pragma unroll
            for (int lm = l * l - 1; lm < (l + 1) * (l + 1) - 1; ++lm) s += A[n][lm] * A[n][lm];
            q[NR + (l - 1) * NA + n] = s;
        }
        if (Sh::H4) q[NR + Sh::L * NA + n] = q4_value<R>(&A[n][3]);
        if (Sh::H5) {
            const R P = q[NR + n];
            q[NR + (Sh::L + (Sh::H4 ? 1 : 0)) * NA + n] = P * P;
        }
    }
    if (live) {
#pragma unroll
        for (int d = 0; d < D; ++d)
            if (d % S == lane) q_out[(long)i * D + d] = q[d];
#pragma unroll
        for (int n = 0; n < NA; ++n)
#pragma unroll
            for (int lm = 0; lm < LM; ++lm)
                if ((n * LM + lm) % S == lane) A_out[((long)i * NA + n) * LM + lm] = A[n][lm];
    }
}

// -------------------------------------------------------------- network fwd

// E_i, e = dE_i/dq (Eqs. 2-3), tanh activations, B = dE_i/dA[n][lm] and the
// radial force coefficients eps[b][k] = sum_n e_n c_R[a][b][n][k].
template <typename R, class Sh>
__global__ void __launch_bounds__(kBlock)
k_network_forward(const Dims dm, const R* __restrict__ theta, const R* __restrict__ qscale,
                  const int* __restrict__ types, int Na, const R* __restrict__ q_in, const R* __restrict__ A_in,
                  R* __restrict__ E_out, R* __restrict__ e_out, R* __restrict__ t_out, R* __restrict__ B_out,
                  R* __restrict__ eps_out) {
    constexpr int NR = Sh::NR, NA = Sh::NA, KR = Sh::KR, LM = Sh::LM, D = Sh::D;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= Na) return;
    const int T = dm.T, H = dm.H;
    const int a = types[i];
    R qs[D], e[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        qs[d] = q_in[(long)i * D + d] * qscale[d];
        e[d] = R(0);
    }
    const R* __restrict__ W0 = theta + dm.offN + (long)a * (D + 2) * H;
    const R* __restrict__ b0 = W0 + (long)H * D;
    const R* __restrict__ w1 = b0 + H;
    R E = -theta[dm.offB1];
    for (int mu = 0; mu < H; ++mu) {
        R acc = -b0[mu];
#pragma unroll
        for (int d = 0; d < D; ++d) acc += W0[(long)mu * D + d] * qs[d];
        const R t = tanh_<R>(acc);
        t_out[(long)i * H + mu] = t;
        const R w = w1[mu];
        E += w * t;
        const R c = w * (R(1) - t * t);
#pragma unroll
        for (int d = 0; d < D; ++d) e[d] += c * W0[(long)mu * D + d];
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
        e[d] *= qscale[d];
        e_out[(long)i * D + d] = e[d];
    }
    E_out[i] = E;
    // B = dE/dA
#pragma unroll
    for (int n = 0; n < NA; ++n) {
        R An[LM], Bn[LM];
#pragma unroll
        for (int lm = 0; lm < LM; ++lm) An[lm] = A_in[((long)i * NA + n) * LM + lm];
#pragma unroll
        for (int lm = 0; lm < LM; ++lm) Bn[lm] = R(2) * e[NR + (lm_degree<LM>(lm) - 1) * NA + n] * An[lm];
        if (Sh::H4) {
            R g4[5];
            q4_grad<R>(&An[3], g4);
            const R e4 = e[NR + Sh::L * NA + n];
#pragma unroll
            for (int m = 0; m < 5; ++m) Bn[3 + m] += e4 * g4[m];
        }
        if (Sh::H5) {
            const R P = An[0] * An[0] + An[1] * An[1] + An[2] * An[2];
            const R e5 = e[NR + (Sh::L + (Sh::H4 ? 1 : 0)) * NA + n];
#pragma unroll
            for (int m = 0; m < 3; ++m) Bn[m] += e5 * R(4) * P * An[m];
        }
#pragma unroll
        for (int lm = 0; lm < LM; ++lm) B_out[((long)i * NA + n) * LM + lm] = Bn[lm];
    }
    // radial force coefficients for every neighbour species
    for (int b = 0; b < T; ++b) {
        const R* __restrict__ cR = theta + (long)((a * T + b) * NR) * KR;
#pragma unroll
        for (int kk = 0; kk < KR; ++kk) {
            R s = R(0);
#pragma unroll
            for (int n = 0; n < NR; ++n) s += e[n] * cR[n * KR + kk];
            eps_out[((long)i * T + b) * KR + kk] = s;
        }
    }
}

// ------------------------------------------------------------------- force

// F_k = sum_{j in N(k)} (dE_k/dr_kj - dE_j/dr_jk) (gather form over k's row)
// and the per-atom virial -1/2 sum_j r_kj (x) (that pair force), which sums
// over a structure to W = -sum_{i,j} r_ij (x) dE_i/dr_ij.
template <typename R, class Sh, int S>
__global__ void __launch_bounds__(kBlock)
k_force(const Dims dm, const R* __restrict__ theta, const int* __restrict__ types, int Na,
        const int64_t* __restrict__ row, const int* __restrict__ seg, const Rec<R>* __restrict__ pairs,
        const R* __restrict__ B_in, const R* __restrict__ eps_in, R* __restrict__ F_out, R* __restrict__ Wat_out) {
    constexpr int NA = Sh::NA, KR = Sh::KR, KA = Sh::KA, LM = Sh::LM;
    const int team = threadIdx.x / S, lane = threadIdx.x % S;
    const int i = blockIdx.x * (kBlock / S) + team;
    const bool live = i < Na;
    const int T = dm.T;
    const R rcR = R(dm.rcR), rcA = R(dm.rcA), irR = R(1.0 / dm.rcR), irA = R(1.0 / dm.rcA);
    const int a = live ? types[i] : 0;
    int64_t p = live ? row[i] : 0;
    R F[3] = {R(0), R(0), R(0)};
    R Wv[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) Wv[c] = R(0);
    const R* __restrict__ Bk = B_in + (long)i * NA * LM;

    for (int b = 0; b < T; ++b) {
        const int tot = live ? seg[(i * T + b) * 2] : 0;
        const int ang = live ? seg[(i * T + b) * 2 + 1] : 0;
        R epsk[KR];
#pragma unroll
        for (int kk = 0; kk < KR; ++kk) epsk[kk] = live ? eps_in[((long)i * T + b) * KR + kk] : R(0);
        const R* __restrict__ cAab = theta + dm.offA + (long)((a * T + b) * NA) * KA;
        const R* __restrict__ cAba = theta + dm.offA + (long)((b * T + a) * NA) * KA;
        for (int k = lane; k < tot; k += S) {
            const Rec<R> pr = pairs[p + k];
            const int j = rec_j(pr);
            const R r = sqrt(pr.x * pr.x + pr.y * pr.y + pr.z * pr.z);
            const R ir = R(1) / r;
            const R u[3] = {pr.x * ir, pr.y * ir, pr.z * ir};
            R f[KR], fp[KR];
            cheb_basis<R, KR, true>(r, rcR, irR, f, fp);
            const R* __restrict__ epsj = eps_in + ((long)j * T + a) * KR;
            R s = R(0);
#pragma unroll
            for (int kk = 0; kk < KR; ++kk) s += (epsk[kk] + epsj[kk]) * fp[kk];
            R fv[3] = {s * u[0], s * u[1], s * u[2]};
            if (k < ang) {
                R fa[KA], fap[KA];
                cheb_basis<R, KA, true>(r, rcA, irA, fa, fap);
                const G3<R> gx = {u[0], R(1), R(0), R(0)}, gy = {u[1], R(0), R(1), R(0)},
                            gz = {u[2], R(0), R(0), R(1)};
                G3<R> Yg[LM];
                solid_harmonics<G3<R>, R, Sh::L>(gx, gy, gz, Yg);
                R c[LM], cp[LM];
#pragma unroll
                for (int lm = 0; lm < LM; ++lm) c[lm] = cp[lm] = R(0);
                const R* __restrict__ Bj = B_in + (long)j * NA * LM;
#pragma unroll
                for (int n = 0; n < NA; ++n) {
                    R g1 = R(0), gp1 = R(0), g2 = R(0), gp2 = R(0);
#pragma unroll
                    for (int kk = 0; kk < KA; ++kk) {
                        const R c1 = cAab[n * KA + kk], c2 = cAba[n * KA + kk];
                        g1 += c1 * fa[kk];
                        gp1 += c1 * fap[kk];
                        g2 += c2 * fa[kk];
                        gp2 += c2 * fap[kk];
                    }
#pragma unroll
                    for (int lm = 0; lm < LM; ++lm) {
                        const R bk = Bk[n * LM + lm];
                        const R bj = (lm_degree<LM>(lm) & 1) ? -Bj[n * LM + lm] : Bj[n * LM + lm];
                        c[lm] += bk * g1 + bj * g2;
                        cp[lm] += bk * gp1 + bj * gp2;
                    }
                }
                R sY = R(0), lY = R(0), G[3] = {R(0), R(0), R(0)};
#pragma unroll
                for (int lm = 0; lm < LM; ++lm) {
                    sY += cp[lm] * Yg[lm].v;
                    lY += R(lm_degree<LM>(lm)) * c[lm] * Yg[lm].v;
                    G[0] += c[lm] * Yg[lm].x;
                    G[1] += c[lm] * Yg[lm].y;
                    G[2] += c[lm] * Yg[lm].z;
                }
#pragma unroll
                for (int d = 0; d < 3; ++d) fv[d] += sY * u[d] + (G[d] - lY * u[d]) * ir;
            }
            const R rv[3] = {pr.x, pr.y, pr.z};
#pragma unroll
            for (int d = 0; d < 3; ++d) F[d] += fv[d];
#pragma unroll
            for (int al = 0; al < 3; ++al)
#pragma unroll
                for (int be = 0; be < 3; ++be) Wv[al * 3 + be] -= R(0.5) * rv[al] * fv[be];
        }
        p += tot;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) F[d] = team_sum<S>(F[d]);
#pragma unroll
    for (int c = 0; c < 9; ++c) Wv[c] = team_sum<S>(Wv[c]);
    if (live) {
#pragma unroll
        for (int d = 0; d < 3; ++d)
            if (d % S == lane) F_out[(long)i * 3 + d] = F[d];
#pragma unroll
        for (int c = 0; c < 9; ++c)
            if (c % S == lane) Wat_out[(long)i * 9 + c] = Wv[c];
    }
}

// ----------------------------------------------------------------- tangent

// Directional derivative of the descriptor along v_ij = u_i - u_j - U_s^T r_ij:
// dq (radial and invariants), dA[n][lm], and S1[b][k] = sum_{j in b} (v.r^) f_k'.
template <typename R, class Sh, int S>
__global__ void __launch_bounds__(kBlock)
k_tangent(const Dims dm, const R* __restrict__ theta, const int* __restrict__ types,
          const int* __restrict__ atom_struct, int Na, const int64_t* __restrict__ row, const int* __restrict__ seg,
          const Rec<R>* __restrict__ pairs, const R* __restrict__ ubar, const double* __restrict__ Ubar,
          const R* __restrict__ A_in, R* __restrict__ dq_out, R* __restrict__ dA_out, R* __restrict__ S1_out) {
    constexpr int NR = Sh::NR, NA = Sh::NA, KR = Sh::KR, KA = Sh::KA, LM = Sh::LM, D = Sh::D;
    const int team = threadIdx.x / S, lane = threadIdx.x % S;
    const int i = blockIdx.x * (kBlock / S) + team;
    const bool live = i < Na;
    const int T = dm.T;
    const R rcR = R(dm.rcR), rcA = R(dm.rcA), irR = R(1.0 / dm.rcR), irA = R(1.0 / dm.rcA);
    const int a = live ? types[i] : 0;
    const int s = live ? atom_struct[i] : 0;
    int64_t p = live ? row[i] : 0;
    R ui[3], U[9];
#pragma unroll
    for (int d = 0; d < 3; ++d) ui[d] = live ? ubar[(long)i * 3 + d] : R(0);
#pragma unroll
    for (int c = 0; c < 9; ++c) U[c] = live ? R(Ubar[(long)s * 9 + c]) : R(0);
    R dqR[NR];
    R dA[NA][LM];
#pragma unroll
    for (int n = 0; n < NR; ++n) dqR[n] = R(0);
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int lm = 0; lm < LM; ++lm) dA[n][lm] = R(0);

    for (int b = 0; b < T; ++b) {
        const int tot = live ? seg[(i * T + b) * 2] : 0;
        const int ang = live ? seg[(i * T + b) * 2 + 1] : 0;
        const R* __restrict__ cA = theta + dm.offA + (long)((a * T + b) * NA) * KA;
        R Sb[KR];
#pragma unroll
        for (int kk = 0; kk < KR; ++kk) Sb[kk] = R(0);
        for (int k = lane; k < tot; k += S) {
            const Rec<R> pr = pairs[p + k];
            const int j = rec_j(pr);
            const R rv[3] = {pr.x, pr.y, pr.z};
            R v[3];
#pragma unroll
            for (int be = 0; be < 3; ++be)
                v[be] = ui[be] - ubar[(long)j * 3 + be] - (U[be] * rv[0] + U[3 + be] * rv[1] + U[6 + be] * rv[2]);
            const R r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
            const R ir = R(1) / r;
            const R u[3] = {rv[0] * ir, rv[1] * ir, rv[2] * ir};
            const R vu = v[0] * u[0] + v[1] * u[1] + v[2] * u[2];
            R f[KR], fp[KR];
            cheb_basis<R, KR, true>(r, rcR, irR, f, fp);
#pragma unroll
            for (int kk = 0; kk < KR; ++kk) Sb[kk] += vu * fp[kk];
            if (k < ang) {
                R fa[KA], fap[KA];
                cheb_basis<R, KA, true>(r, rcA, irA, fa, fap);
                const D1<R> dx = {u[0], v[0]}, dy = {u[1], v[1]}, dz = {u[2], v[2]};
                D1<R> Yd[LM];
                solid_harmonics<D1<R>, R, Sh::L>(dx, dy, dz, Yd);
                R Y[LM], vdY[LM];
#pragma unroll
                for (int lm = 0; lm < LM; ++lm) {
                    Y[lm] = Yd[lm].v;
                    vdY[lm] = (Yd[lm].d - R(lm_degree<LM>(lm)) * Yd[lm].v * vu) * ir;
                }
#pragma unroll
                for (int n = 0; n < NA; ++n) {
                    R g = R(0), gp = R(0);
#pragma unroll
                    for (int kk = 0; kk < KA; ++kk) {
                        g += cA[n * KA + kk] * fa[kk];
                        gp += cA[n * KA + kk] * fap[kk];
                    }
                    const R gpv = gp * vu;
#pragma unroll
                    for (int lm = 0; lm < LM; ++lm) dA[n][lm] += gpv * Y[lm] + g * vdY[lm];
                }
            }
        }
        p += tot;
#pragma unroll
        for (int kk = 0; kk < KR; ++kk) Sb[kk] = team_sum<S>(Sb[kk]);
        const R* __restrict__ cR = theta + (long)((a * T + b) * NR) * KR;
#pragma unroll
        for (int n = 0; n < NR; ++n)
#pragma unroll
            for (int kk = 0; kk < KR; ++kk) dqR[n] += cR[n * KR + kk] * Sb[kk];
        if (live) {
#pragma unroll
            for (int kk = 0; kk < KR; ++kk)
                if (kk % S == lane) S1_out[((long)i * T + b) * KR + kk] = Sb[kk];
        }
    }
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int lm = 0; lm < LM; ++lm) dA[n][lm] = team_sum<S>(dA[n][lm]);
    if (!live) return;
    R dq[D];
#pragma unroll
    for (int n = 0; n < NR; ++n) dq[n] = dqR[n];
#pragma unroll
    for (int n = 0; n < NA; ++n) {
        R An[LM];
#pragma unroll
        for (int lm = 0; lm < LM; ++lm) An[lm] = A_in[((long)i * NA + n) * LM + lm];
#pragma unroll
        for (int l = 1; l <= Sh::L; ++l) {
            R s2 = R(0);
#pragma unroll
            for (int lm = l * l - 1; lm < (l + 1) * (l + 1) - 1; ++lm) s2 += An[lm] * dA[n][lm];
            dq[NR + (l - 1) * NA + n] = R(2) * s2;
        }
        if (Sh::H4) {
            R g4[5];
            q4_grad<R>(&An[3], g4);
            R s4 = R(0);
#pragma unroll
            for (int m = 0; m < 5; ++m) s4 += g4[m] * dA[n][3 + m];
            dq[NR + Sh::L * NA + n] = s4;
        }
        if (Sh::H5) {
            const R P = An[0] * An[0] + An[1] * An[1] + An[2] * An[2];
            const R dd = An[0] * dA[n][0] + An[1] * dA[n][1] + An[2] * dA[n][2];
            dq[NR + (Sh::L + (Sh::H4 ? 1 : 0)) * NA + n] = R(4) * P * dd;
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d)
        if (d % S == lane) dq_out[(long)i * D + d] = dq[d];
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int lm = 0; lm < LM; ++lm)
            if ((n * LM + lm) % S == lane) dA_out[((long)i * NA + n) * LM + lm] = dA[n][lm];
}

// ------------------------------------------------------------- network bwd

// For Psi = sum_i ebar_s E_i + e(q_i) . dq_i: per-atom factors of the network
// weight gradients (alpha, beta, gamma), abar = dPsi/dq and
// Bp = dPsi/dA[n][lm] (the angular moments' adjoint).
template <typename R, class Sh>
__global__ void __launch_bounds__(kBlock)
k_network_backward(const Dims dm, const R* __restrict__ theta, const R* __restrict__ qscale,
                   const int* __restrict__ types, const int* __restrict__ atom_struct, int Na,
                   const double* __restrict__ ebar_s, const R* __restrict__ q_in, const R* __restrict__ dq_in,
                   const R* __restrict__ e_in, const R* __restrict__ t_in, const R* __restrict__ A_in,
                   const R* __restrict__ dA_in, R* __restrict__ abar_out, R* __restrict__ alpha_out,
                   R* __restrict__ beta_out, R* __restrict__ gamma_out, R* __restrict__ Bp_out) {
    constexpr int NR = Sh::NR, NA = Sh::NA, LM = Sh::LM, D = Sh::D;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= Na) return;
    const int H = dm.H;
    const int a = types[i];
    const R eb = R(ebar_s[atom_struct[i]]);
    R dqs[D], z[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        dqs[d] = dq_in[(long)i * D + d] * qscale[d];
        z[d] = R(0);
    }
    const R* __restrict__ W0 = theta + dm.offN + (long)a * (D + 2) * H;
    const R* __restrict__ w1 = W0 + (long)H * D + H;
    for (int mu = 0; mu < H; ++mu) {
        R da = R(0);
#pragma unroll
        for (int d = 0; d < D; ++d) da += W0[(long)mu * D + d] * dqs[d];
        const R t = t_in[(long)i * H + mu];
        const R sp = R(1) - t * t;
        const R w = w1[mu];
        alpha_out[(long)i * H + mu] = w * sp * (eb - R(2) * t * da);
        beta_out[(long)i * H + mu] = w * sp;
        gamma_out[(long)i * H + mu] = eb * t + sp * da;
        const R c = R(-2) * w * t * sp * da;
#pragma unroll
        for (int d = 0; d < D; ++d) z[d] += c * W0[(long)mu * D + d];
    }
    R ab[D], e[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        e[d] = e_in[(long)i * D + d];
        ab[d] = eb * e[d] + z[d] * qscale[d];
        abar_out[(long)i * D + d] = ab[d];
    }
#pragma unroll
    for (int n = 0; n < NA; ++n) {
        R An[LM], dAn[LM], Bn[LM];
#pragma unroll
        for (int lm = 0; lm < LM; ++lm) {
            An[lm] = A_in[((long)i * NA + n) * LM + lm];
            dAn[lm] = dA_in[((long)i * NA + n) * LM + lm];
        }
#pragma unroll
        for (int lm = 0; lm < LM; ++lm) {
            const int idx = NR + (lm_degree<LM>(lm) - 1) * NA + n;
            Bn[lm] = R(2) * ab[idx] * An[lm] + R(2) * e[idx] * dAn[lm];
        }
        if (Sh::H4) {
            R g4[5], h4[5];
            q4_grad<R>(&An[3], g4);
            q4_hess_vec<R>(&An[3], &dAn[3], h4);
            const int idx = NR + Sh::L * NA + n;
#pragma unroll
            for (int m = 0; m < 5; ++m) Bn[3 + m] += ab[idx] * g4[m] + e[idx] * h4[m];
        }
        if (Sh::H5) {
            const R P = An[0] * An[0] + An[1] * An[1] + An[2] * An[2];
            const R dd = An[0] * dAn[0] + An[1] * dAn[1] + An[2] * dAn[2];
            const int idx = NR + (Sh::L + (Sh::H4 ? 1 : 0)) * NA + n;
#pragma unroll
            for (int m = 0; m < 3; ++m)
                Bn[m] += ab[idx] * R(4) * P * An[m] + e[idx] * (R(8) * dd * An[m] + R(4) * P * dAn[m]);
        }
#pragma unroll
        for (int lm = 0; lm < LM; ++lm) Bp_out[((long)i * NA + n) * LM + lm] = Bn[lm];
    }
}

// -------------------------------------------------- angular coefficient grad

// dL/dc_A[a][b][n][k] = sum_{i in a} sum_{j in b, angular}
//     [ f_k (sum_lm Bp_nlm Y_lm + Q_nlm v.dY_lm) + f_k' (v.r^) sum_lm Q_nlm Y_lm ],
// Q = B = dE_i/dA. Per-block partial rows (double) over a grid-stride loop.
// Each team's per-segment sums go to its own LDS slot and are then added into
// the block accumulator in team order, so the result is bitwise repeatable.
template <typename R, class Sh, int S>
__global__ void __launch_bounds__(kBlock)
k_angular_coeff_grad(const Dims dm, const int* __restrict__ types, const int* __restrict__ atom_struct, int Na,
                     const int64_t* __restrict__ row, const int* __restrict__ seg, const Rec<R>* __restrict__ pairs,
                     const R* __restrict__ ubar, const double* __restrict__ Ubar, const R* __restrict__ Bp_in,
                     const R* __restrict__ Q_in, double* __restrict__ partial) {
    constexpr int NA = Sh::NA, KA = Sh::KA, LM = Sh::LM;
    constexpr int NK = NA * KA, TEAMS = kBlock / S;
    extern __shared__ unsigned char smem_raw[];
    R* G = reinterpret_cast<R*>(smem_raw);
    const int T = dm.T;
    const int G_len = T * T * NK;
    R* slot = G + G_len;                   // [TEAMS][NK]
    int* team_type = reinterpret_cast<int*>(slot + TEAMS * NK);  // [TEAMS]
    for (int x = threadIdx.x; x < G_len; x += kBlock) G[x] = R(0);
    __syncthreads();
    const int team = threadIdx.x / S, lane = threadIdx.x % S;
    const R rcA = R(dm.rcA), irA = R(1.0 / dm.rcA);
    const int tiles = (Na + kBlock / S - 1) / (kBlock / S);
    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int i = tile * (kBlock / S) + team;
        const bool live = i < Na;
        const int a = live ? types[i] : 0;
        const int s = live ? atom_struct[i] : 0;
        int64_t p = live ? row[i] : 0;
        R ui[3], U[9];
#pragma unroll
        for (int d = 0; d < 3; ++d) ui[d] = live ? ubar[(long)i * 3 + d] : R(0);
#pragma unroll
        for (int c = 0; c < 9; ++c) U[c] = live ? R(Ubar[(long)s * 9 + c]) : R(0);
        const R* __restrict__ Bpi = Bp_in + (long)i * NA * LM;
        const R* __restrict__ Qi = Q_in + (long)i * NA * LM;
        for (int b = 0; b < T; ++b) {
            const int tot = live ? seg[(i * T + b) * 2] : 0;
            const int ang = live ? seg[(i * T + b) * 2 + 1] : 0;
            R acc[NA][KA];
#pragma unroll
            for (int n = 0; n < NA; ++n)
#pragma unroll
                for (int kk = 0; kk < KA; ++kk) acc[n][kk] = R(0);
            for (int k = lane; k < ang; k += S) {
                const Rec<R> pr = pairs[p + k];
                const int j = rec_j(pr);
                const R rv[3] = {pr.x, pr.y, pr.z};
                R v[3];
#pragma unroll
                for (int be = 0; be < 3; ++be)
                    v[be] = ui[be] - ubar[(long)j * 3 + be] - (U[be] * rv[0] + U[3 + be] * rv[1] + U[6 + be] * rv[2]);
                const R r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
                const R ir = R(1) / r;
                const R u[3] = {rv[0] * ir, rv[1] * ir, rv[2] * ir};
                const R vu = v[0] * u[0] + v[1] * u[1] + v[2] * u[2];
                R fa[KA], fap[KA];
                cheb_basis<R, KA, true>(r, rcA, irA, fa, fap);
                const D1<R> dx = {u[0], v[0]}, dy = {u[1], v[1]}, dz = {u[2], v[2]};
                D1<R> Yd[LM];
                solid_harmonics<D1<R>, R, Sh::L>(dx, dy, dz, Yd);
                R Y[LM], vdY[LM];
#pragma unroll
                for (int lm = 0; lm < LM; ++lm) {
                    Y[lm] = Yd[lm].v;
                    vdY[lm] = (Yd[lm].d - R(lm_degree<LM>(lm)) * Yd[lm].v * vu) * ir;
                }
#pragma unroll
                for (int n = 0; n < NA; ++n) {
                    R P = R(0), Rn = R(0);
#pragma unroll
                    for (int lm = 0; lm < LM; ++lm) {
                        const R q = Qi[n * LM + lm];
                        P += Bpi[n * LM + lm] * Y[lm] + q * vdY[lm];
                        Rn += q * Y[lm];
                    }
                    Rn *= vu;
#pragma unroll
                    for (int kk = 0; kk < KA; ++kk) acc[n][kk] += P * fa[kk] + Rn * fap[kk];
                }
            }
            p += tot;
#pragma unroll
            for (int n = 0; n < NA; ++n)
#pragma unroll
                for (int kk = 0; kk < KA; ++kk) {
                    const R vsum = team_sum<S>(acc[n][kk]);
                    if ((n * KA + kk) % S == lane) slot[team * NK + n * KA + kk] = live ? vsum : R(0);
                }
            if (lane == 0) team_type[team] = a;
            __syncthreads();
            for (int x = threadIdx.x; x < NK; x += kBlock)
                for (int tm = 0; tm < TEAMS; ++tm) G[(team_type[tm] * T + b) * NK + x] += slot[tm * NK + x];
            __syncthreads();
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < G_len; x += kBlock) partial[(long)blockIdx.x * G_len + x] = double(G[x]);
}

// ------------------------------------------ network and radial coefficient grad

// Partial rows over chunks of the species-sorted atom list. Row layout:
// [0, offA): c_R[a][b][n][k] -> sum_i abar_n S0[b][k] + e_n S1[b][k];
// [offA, offA + T (D+2) H): per species W0 -> alpha (x) s.q + beta (x) s.dq,
// b0 -> -alpha, w1 -> gamma.
template <typename R, class Sh>
__global__ void __launch_bounds__(kBlock)
k_outer_grad(const Dims dm, const R* __restrict__ qscale, const int* __restrict__ types,
             const int* __restrict__ order, int Na, int chunk, const R* __restrict__ q_in,
             const R* __restrict__ dq_in, const R* __restrict__ abar, const R* __restrict__ e_in,
             const R* __restrict__ alpha, const R* __restrict__ beta, const R* __restrict__ gam,
             const R* __restrict__ S0, const R* __restrict__ S1, double* __restrict__ partial) {
    constexpr int NR = Sh::NR, KR = Sh::KR, D = Sh::D;
    const int T = dm.T, H = dm.H;
    const long nR = dm.offA;
    const long rowlen = nR + (long)T * (D + 2) * H;
    const int nchunks = (Na + chunk - 1) / chunk;
    for (long col = threadIdx.x; col < rowlen; col += kBlock) {
        // decode the column
        int kind, a, x0, x1, x2;
        if (col < nR) {
            kind = 0;
            long c = col;
            x2 = int(c % KR);
            c /= KR;
            x1 = int(c % NR);
            c /= NR;
            x0 = int(c % T);
            a = int(c / T);
        } else {
            long c = col - nR;
            a = int(c / ((long)(D + 2) * H));
            c %= (long)(D + 2) * H;
            if (c < (long)H * D) {
                kind = 1;
                x0 = int(c / D);
                x1 = int(c % D);
            } else if (c < (long)H * D + H) {
                kind = 2;
                x0 = int(c - (long)H * D);
            } else {
                kind = 3;
                x0 = int(c - (long)H * D - H);
            }
            x2 = 0;
        }
        double acc = 0.0;
        for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
            const int lo = ch * chunk, hi = min(Na, lo + chunk);
            R part = R(0);
            for (int ii = lo; ii < hi; ++ii) {
                const int i = order[ii];
                if (types[i] != a) continue;
                if (kind == 0) {
                    part += abar[(long)i * D + x1] * S0[((long)i * T + x0) * KR + x2] +
                            e_in[(long)i * D + x1] * S1[((long)i * T + x0) * KR + x2];
                } else if (kind == 1) {
                    const R s = qscale[x1];
                    part += alpha[(long)i * H + x0] * s * q_in[(long)i * D + x1] +
                            beta[(long)i * H + x0] * s * dq_in[(long)i * D + x1];
                } else if (kind == 2) {
                    part -= alpha[(long)i * H + x0];
                } else {
                    part += gam[(long)i * H + x0];
                }
            }
            acc += double(part);
        }
        partial[(long)blockIdx.x * rowlen + col] = acc;
    }
}

}  // namespace nep
