// Per-structure FP64 reductions, the loss and its seeds (Eqs. 4-7), the final
// deterministic gradient reduction, Adam/AMSGrad (Eqs. 8-13) and the
// descriptor scaler (Eq. 2).
#pragma once

#include "nep_device.hpp"

namespace nep {

constexpr int kRedBlock = 256;

// One block per structure: E_s = sum E_i and W_s = sum of per-atom virials in
// double. With `loss` set: the loss pieces of the structure and the seeds
//   ebar_s = dL/dE_s = 2 lam_e (E_s - E*_s) / (N_s N_a^s^2),
//   ubar_i = dL/dF_i = 2 lam_f (F_i - F*_i) / (3 N_a),
//   Ubar_s = dL/dW_s = 2 lam_v (W_s - W*_s) / (9 N_v N_a^s^2)  (labelled s only).
// Structures without atoms take no part: N_s and N_v count only structures
// with atoms (N_a^s = 0 leaves Eq. 4's per-atom residual undefined).
template <typename R>
__global__ void __launch_bounds__(kRedBlock)
k_structure(int Ns, long Na, const int64_t* __restrict__ off, const R* __restrict__ E_at,
            const R* __restrict__ W_at, const R* __restrict__ F, int loss, const double* __restrict__ Et,
            const R* __restrict__ Ft, const double* __restrict__ Wt, const uint8_t* __restrict__ has_v,
            double lam_e, double lam_f, double lam_v, double* __restrict__ E_out, double* __restrict__ W_out,
            double* __restrict__ ebar, double* __restrict__ Ubar, R* __restrict__ ubar,
            double* __restrict__ lossp) {
    // E, W[9], the force residual, the number of labelled structures and the
    // number of structures with atoms
    constexpr int NV = 13, WAVES = kRedBlock / 64;
    __shared__ double part[WAVES][NV];
    const int s = blockIdx.x;
    const long a0 = off[s], a1 = off[s + 1];
    const double na = double(a1 - a0);
    // the structure's targets are loaded first, so their latency overlaps the sums
    double Ets = 0.0, Wts[9];
    bool hv = true;
#pragma unroll
    for (int c = 0; c < 9; ++c) Wts[c] = 0.0;
    if (loss && threadIdx.x == 0) {
        Ets = Et[s];
#pragma unroll
        for (int c = 0; c < 9; ++c) Wts[c] = Wt[s * 9 + c];
        hv = has_v ? has_v[s] != 0 : true;
    }
    double acc[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) acc[c] = 0.0;
    const double cf = 2.0 * lam_f / (3.0 * double(Na));
    // UN atoms per thread per round, every load of the round issued before
    // the first sum (an atom past the structure's end reads its last atom and
    // adds nothing), so a large structure is not one load latency per atom
    constexpr int UN = 4;
    for (long i0 = a0 + threadIdx.x; i0 < a1; i0 += UN * kRedBlock) {
        R e[UN], wv[UN][9], f[UN][3], ft[UN][3];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const long i = min(i0 + long(u) * kRedBlock, a1 - 1);
            e[u] = E_at[i];
#pragma unroll
            for (int c = 0; c < 9; ++c) wv[u][c] = W_at[i * 9 + c];
            if (loss) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    f[u][d] = F[i * 3 + d];
                    ft[u][d] = Ft[i * 3 + d];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const long i = i0 + long(u) * kRedBlock;
            if (i >= a1) continue;
            acc[0] += double(e[u]);
#pragma unroll
            for (int c = 0; c < 9; ++c) acc[1 + c] += double(wv[u][c]);
            if (loss) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double r = double(f[u][d]) - double(ft[u][d]);
                    acc[10] += r * r;
                    ubar[i * 3 + d] = R(cf * r);
                }
            }
        }
    }
    if (loss)
        for (int t = threadIdx.x; t < Ns; t += kRedBlock) {
            const bool atoms = off[t + 1] > off[t];
            acc[11] += (atoms && (has_v ? has_v[t] != 0 : true)) ? 1.0 : 0.0;
            acc[12] += atoms ? 1.0 : 0.0;
        }
    // wave sums by shuffles, one barrier, then the waves' sums in wave order
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        double v = acc[c];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (l == 0) part[w][c] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double res[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < WAVES; ++k) t += part[k][c];
        res[c] = t;
    }
    const double E = res[0];
    if (E_out) E_out[s] = E;
    if (W_out)
        for (int c = 0; c < 9; ++c) W_out[s * 9 + c] = res[1 + c];
    if (!loss) return;
    if (na == 0.0) {
        ebar[s] = 0.0;
        for (int c = 0; c < 9; ++c) Ubar[s * 9 + c] = 0.0;
        lossp[s * 3 + 0] = 0.0;
        lossp[s * 3 + 1] = 0.0;
        lossp[s * 3 + 2] = 0.0;
        return;
    }
    const double Nv = res[11], Nsa = res[12];
    const double dE = E - Ets;
    ebar[s] = 2.0 * lam_e * dE / (Nsa * na * na);
    lossp[s * 3 + 0] = (dE / na) * (dE / na) / Nsa;
    lossp[s * 3 + 1] = res[10] / (3.0 * double(Na));
    double dv = 0.0;
    for (int c = 0; c < 9; ++c) {
        const double dw = res[1 + c] - Wts[c];
        if (hv && Nv > 0.0) {
            dv += (dw / na) * (dw / na) / (9.0 * Nv);
            Ubar[s * 9 + c] = 2.0 * lam_v * dw / (9.0 * Nv * na * na);
        } else {
            Ubar[s * 9 + c] = 0.0;
        }
    }
    lossp[s * 3 + 2] = dv;
}

// Seeds given directly (vector-Jacobian product): ebar = dE, Ubar = dW, ubar = dF.
template <typename R>
__global__ void __launch_bounds__(kRedBlock)
k_seeds(int Ns, long Na, const double* __restrict__ dE, const R* __restrict__ dF, const double* __restrict__ dW,
        double* __restrict__ ebar, double* __restrict__ Ubar, R* __restrict__ ubar) {
    const long t = (long)blockIdx.x * kRedBlock + threadIdx.x;
    if (t < Ns) ebar[t] = dE ? dE[t] : 0.0;
    if (t < 9L * Ns) Ubar[t] = dW ? dW[t] : 0.0;
    if (t < 3 * Na) ubar[t] = dF ? dF[t] : R(0);
}

// Gradient reduction, stage 1: block (x, g) sums, for 64 consecutive
// parameters (one per lane, coalesced), the partial rows r = 4 g + w,
// 4 g + w + 4 G, ... (w = wave) and adds the four wave sums in wave order into
// stage[g][p]. Network and radial-coefficient columns of species a come from
// species a's rows of the outer reduction only (its chunks of the
// species-sorted atom list, in species order; soff and chunk give the range),
// angular coefficients from the angular rows.
constexpr int kStageGroups = 16;

template <int WAVES_PER_BLOCK>
__global__ void __launch_bounds__(kRedBlock)
k_reduce_stage(Dims dm, int NRKR, const double* __restrict__ outer_part, int outer_rows,
               const double* __restrict__ ang_part, int ang_rows, double* __restrict__ stage,
               const int64_t* __restrict__ soff, int chunk) {
    __shared__ double red[kRedBlock];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, waves = WAVES_PER_BLOCK;
    const int g = blockIdx.y, G = gridDim.y;
    const long p = (long)blockIdx.x * 64 + lane;
    const int T = dm.T, H = dm.H, D = dm.D;
    const long net_w = long(D + 2) * H;
    const long W1 = net_w + long(T) * NRKR;
    double s = 0.0;
    if (p < dm.offB1) {
        long col = -1;
        int a = 0;
        if (p < dm.offA) {
            a = int(p / (long(T) * NRKR));
            col = net_w + p % (long(T) * NRKR);
        } else if (p >= dm.offN) {
            a = int((p - dm.offN) / net_w);
            col = (p - dm.offN) % net_w;
        }
        const int step = waves * G;
        // unconditional loads in unrolled loops: the rows' loads are in
        // flight together instead of one round trip per row
        if (col >= 0) {
            // only species a's rows: the outer-product rows are the chunks of
            // the species-sorted atom list in species order
            int r0 = 0;
            for (int t = 0; t < a; ++t) r0 += int((soff[t + 1] - soff[t] + chunk - 1) / chunk);
            int r1 = r0 + int((soff[a + 1] - soff[a] + chunk - 1) / chunk);
            r1 = r1 < outer_rows ? r1 : outer_rows;
#pragma unroll 4
            for (int r = r0 + g * waves + wave; r < r1; r += step) s += outer_part[(long)r * (W1 + 1) + 1 + col];
        } else {
            const long angw = dm.offN - dm.offA;
#pragma unroll 8
            for (int r = g * waves + wave; r < ang_rows; r += step) s += ang_part[(long)r * angw + (p - dm.offA)];
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (wave == 0 && p < dm.offB1) {
        double t = 0.0;
        for (int w = 0; w < waves; ++w) t += red[w * 64 + lane];
        stage[(long)g * dm.offB1 + p] = t;
    }
}

// Stage 2: grad[p] = sum over groups in order; b1 gets -sum_s N_a^s ebar_s;
// block 0 also writes loss[4] = {L, Delta_E, Delta_F, Delta_V}. With `adam`
// set, the lane that finishes a parameter's gradient then takes its Adam step
// (theta, m, v, vmax in place), as k_adam would after this kernel.
template <typename R>
__global__ void __launch_bounds__(kRedBlock)
k_final_reduce(Dims dm, int Ns, const int64_t* __restrict__ off, const double* __restrict__ stage, int G,
               const double* __restrict__ ebar, const double* __restrict__ lossp, double lam_e, double lam_f,
               double lam_v, R* __restrict__ grad, double* __restrict__ loss, int adam, AdamArgs aa,
               R* __restrict__ theta, R* __restrict__ m, R* __restrict__ v, R* __restrict__ vmax) {
    const long p = (long)blockIdx.x * kRedBlock + threadIdx.x;
    if (p < dm.offB1) {
        double t = 0.0;
#pragma unroll 8
        for (int g = 0; g < G; ++g) t += stage[(long)g * dm.offB1 + p];
        grad[p] = R(t);
        if (adam) adam_update<R>(p, R(t), aa, theta, m, v, vmax);
    }
    if (blockIdx.x != 0) return;
    // -sum_s N_a^s ebar_s and the three loss parts: wave sums, one barrier,
    // then the waves' sums in wave order
    constexpr int WAVES = kRedBlock / 64;
    __shared__ double part[WAVES][4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int t = threadIdx.x; t < Ns; t += kRedBlock) {
        acc[0] -= double(off[t + 1] - off[t]) * ebar[t];
        if (loss) {
            acc[1] += lossp[t * 3 + 0];
            acc[2] += lossp[t * 3 + 1];
            acc[3] += lossp[t * 3 + 2];
        }
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double v = acc[c];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (l == 0) part[w][c] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double res[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < WAVES; ++k) t += part[k][c];
        res[c] = t;
    }
    grad[dm.offB1] = R(res[0]);
    if (adam) adam_update<R>(dm.offB1, R(res[0]), aa, theta, m, v, vmax);
    if (!loss) return;
    loss[0] = lam_e * res[1] + lam_f * res[2] + lam_v * res[3];
    loss[1] = res[1];
    loss[2] = res[2];
    loss[3] = res[3];
}

// One Adam/AMSGrad step (Eqs. 8-13) of parameter p with gradient gp.
template <typename R>
__device__ __forceinline__ void adam_update(long p, R gp, const AdamArgs& a, R* __restrict__ theta,
                                            R* __restrict__ m, R* __restrict__ v, R* __restrict__ vmax) {
    const R mp = R(a.b1) * m[p] + R(1.0 - a.b1) * gp;
    const R vp = R(a.b2) * v[p] + R(1.0 - a.b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    const R mhat = mp / R(a.bc1);
    R denom;
    if (!a.amsgrad) {
        denom = sqrt(vp / R(a.bc2)) + R(a.eps);
    } else if (a.mode == 0) {
        const R vm = fmax(vmax[p], vp / R(a.bc2));
        vmax[p] = vm;
        denom = sqrt(vm) + R(a.eps);
    } else {
        const R vm = fmax(vmax[p], vp);
        vmax[p] = vm;
        denom = sqrt(vm) / sqrt(R(a.bc2)) + R(a.eps);
    }
    theta[p] -= R(a.lr) * mhat / denom;
}

// The step over all parameters, one lane each.
template <typename R>
__global__ void __launch_bounds__(kRedBlock)
k_adam(long P, R* __restrict__ theta, const R* __restrict__ g, R* __restrict__ m, R* __restrict__ v,
       R* __restrict__ vmax, AdamArgs a) {
    const long p = (long)blockIdx.x * kRedBlock + threadIdx.x;
    if (p >= P) return;
    adam_update<R>(p, g[p], a, theta, m, v, vmax);
}

// q_scale[d] = 1/(max - min) over atoms, 1 for ranges below 1e-10 (Eq. 2).
template <typename R>
__global__ void __launch_bounds__(kRedBlock)
k_scale(long Na, int D, const R* __restrict__ q, R* __restrict__ out) {
    __shared__ double lo_s[kRedBlock], hi_s[kRedBlock];
    const int d = blockIdx.x;
    double lo = 1e300, hi = -1e300;
    for (long i = threadIdx.x; i < Na; i += kRedBlock) {
        const double x = double(q[i * D + d]);
        lo = fmin(lo, x);
        hi = fmax(hi, x);
    }
    lo_s[threadIdx.x] = lo;
    hi_s[threadIdx.x] = hi;
    __syncthreads();
    for (int s = kRedBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            lo_s[threadIdx.x] = fmin(lo_s[threadIdx.x], lo_s[threadIdx.x + s]);
            hi_s[threadIdx.x] = fmax(hi_s[threadIdx.x], hi_s[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double r = hi_s[0] - lo_s[0];
        out[d] = (Na > 0 && r >= 1e-10) ? R(1.0 / r) : R(1);
    }
}

}  // namespace nep
