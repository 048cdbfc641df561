// Per-structure FP64 reductions, the loss and its seeds (Eqs. 4-7), the final
// deterministic gradient reduction, Adam/AMSGrad (Eqs. 8-13) and the
// descriptor scaler (Eq. 2).
#pragma once

#include "nep_device.hpp"

namespace nep {

constexpr int kRedBlock = 256;

// Block-wide sum of a double (wave64 shuffles, then one value per wave in LDS).
__device__ __forceinline__ double block_sum(double v, double* scratch) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) scratch[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += scratch[k];
    return t;  // valid in thread 0
}

// One block per structure: E_s = sum E_i and W_s = sum of per-atom virials in
// double. With `loss` set: the loss pieces of the structure and the seeds
//   ebar_s = dL/dE_s = 2 lam_e (E_s - E*_s) / (N_s N_a^s^2),
//   ubar_i = dL/dF_i = 2 lam_f (F_i - F*_i) / (3 N_a),
//   Ubar_s = dL/dW_s = 2 lam_v (W_s - W*_s) / (9 N_v N_a^s^2)  (labelled s only).
// Structures without atoms contribute nothing.
template <typename R>
__global__ void __launch_bounds__(kRedBlock)
k_structure(int Ns, long Na, const int64_t* __restrict__ off, const R* __restrict__ E_at,
            const R* __restrict__ W_at, const R* __restrict__ F, int loss, const double* __restrict__ Et,
            const R* __restrict__ Ft, const double* __restrict__ Wt, const uint8_t* __restrict__ has_v,
            double lam_e, double lam_f, double lam_v, double* __restrict__ E_out, double* __restrict__ W_out,
            double* __restrict__ ebar, double* __restrict__ Ubar, R* __restrict__ ubar,
            double* __restrict__ lossp) {
    __shared__ double scratch[kRedBlock / 64];
    __shared__ double res[11];
    const int s = blockIdx.x;
    const long a0 = off[s], a1 = off[s + 1];
    const double na = double(a1 - a0);
    double acc[11];
#pragma unroll
    for (int c = 0; c < 11; ++c) acc[c] = 0.0;
    const double cf = 2.0 * lam_f / (3.0 * double(Na));
    for (long i = a0 + threadIdx.x; i < a1; i += kRedBlock) {
        const R fi[3] = {F[i * 3], F[i * 3 + 1], F[i * 3 + 2]};
        acc[0] += double(E_at[i]);
#pragma unroll
        for (int c = 0; c < 9; ++c) acc[1 + c] += double(W_at[i * 9 + c]);
        if (loss) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double r = double(fi[d]) - double(Ft[i * 3 + d]);
                acc[10] += r * r;
                ubar[i * 3 + d] = R(cf * r);
            }
        }
    }
    // number of structures with a virial label
    double nv = 0.0;
    if (loss) {
        for (int t = threadIdx.x; t < Ns; t += kRedBlock) nv += has_v ? double(has_v[t] != 0) : 1.0;
    }
#pragma unroll
    for (int c = 0; c < 11; ++c) {
        const double t = block_sum(acc[c], scratch);
        if (threadIdx.x == 0) res[c] = t;
    }
    const double Nv = loss ? block_sum(nv, scratch) : 0.0;
    if (threadIdx.x != 0) return;
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
    const double dE = E - Et[s];
    ebar[s] = 2.0 * lam_e * dE / (double(Ns) * na * na);
    lossp[s * 3 + 0] = (dE / na) * (dE / na) / double(Ns);
    lossp[s * 3 + 1] = res[10] / (3.0 * double(Na));
    const bool hv = has_v ? has_v[s] != 0 : true;
    double dv = 0.0;
    for (int c = 0; c < 9; ++c) {
        const double dw = res[1 + c] - Wt[s * 9 + c];
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
// stage[g][p]. Network and radial-coefficient columns come from the
// species-tagged rows of the outer reduction, angular coefficients from the
// angular rows.
constexpr int kStageGroups = 16;

template <int WAVES_PER_BLOCK>
__global__ void __launch_bounds__(kRedBlock)
k_reduce_stage(Dims dm, int NRKR, const double* __restrict__ outer_part, int outer_rows,
               const double* __restrict__ ang_part, int ang_rows, double* __restrict__ stage) {
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
        if (col >= 0) {
            for (int r = g * waves + wave; r < outer_rows; r += step) {
                const double* row = outer_part + (long)r * (W1 + 1);
                if (row[0] == double(a)) s += row[1 + col];
            }
        } else {
            const long angw = dm.offN - dm.offA;
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
// block 0 also writes loss[4] = {L, Delta_E, Delta_F, Delta_V}.
template <typename R>
__global__ void __launch_bounds__(kRedBlock)
k_final_reduce(Dims dm, int Ns, const int64_t* __restrict__ off, const double* __restrict__ stage, int G,
               const double* __restrict__ ebar, const double* __restrict__ lossp, double lam_e, double lam_f,
               double lam_v, R* __restrict__ grad, double* __restrict__ loss) {
    __shared__ double scratch[kRedBlock / 64];
    const long p = (long)blockIdx.x * kRedBlock + threadIdx.x;
    if (p < dm.offB1) {
        double t = 0.0;
        for (int g = 0; g < G; ++g) t += stage[(long)g * dm.offB1 + p];
        grad[p] = R(t);
    }
    if (blockIdx.x != 0) return;
    double sb = 0.0, dE = 0.0, dF = 0.0, dV = 0.0;
    for (int t = threadIdx.x; t < Ns; t += kRedBlock) {
        sb -= double(off[t + 1] - off[t]) * ebar[t];
        if (loss) {
            dE += lossp[t * 3 + 0];
            dF += lossp[t * 3 + 1];
            dV += lossp[t * 3 + 2];
        }
    }
    sb = block_sum(sb, scratch);
    if (threadIdx.x == 0) grad[dm.offB1] = R(sb);
    if (!loss) return;
    dE = block_sum(dE, scratch);
    dF = block_sum(dF, scratch);
    dV = block_sum(dV, scratch);
    if (threadIdx.x == 0) {
        loss[0] = lam_e * dE + lam_f * dF + lam_v * dV;
        loss[1] = dE;
        loss[2] = dF;
        loss[3] = dV;
    }
}

// One Adam/AMSGrad step (Eqs. 8-13), elementwise.
template <typename R>
__global__ void __launch_bounds__(kRedBlock)
k_adam(long P, R* __restrict__ theta, const R* __restrict__ g, R* __restrict__ m, R* __restrict__ v,
       R* __restrict__ vmax, double lr, double b1, double b2, double eps, double bc1, double bc2, int amsgrad,
       int mode) {
    const long p = (long)blockIdx.x * kRedBlock + threadIdx.x;
    if (p >= P) return;
    const R gp = g[p];
    const R mp = R(b1) * m[p] + R(1.0 - b1) * gp;
    const R vp = R(b2) * v[p] + R(1.0 - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    const R mhat = mp / R(bc1);
    R denom;
    if (!amsgrad) {
        denom = sqrt(vp / R(bc2)) + R(eps);
    } else if (mode == 0) {
        const R vm = fmax(vmax[p], vp / R(bc2));
        vmax[p] = vm;
        denom = sqrt(vm) + R(eps);
    } else {
        const R vm = fmax(vmax[p], vp);
        vmax[p] = vm;
        denom = sqrt(vm) / sqrt(R(bc2)) + R(eps);
    }
    theta[p] -= R(lr) * mhat / denom;
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
