// ZBL short-range repulsion: the universal screened-Coulomb pair potential of
// Ziegler, Biersack and Littmark (1985), which the paper lists among the
// potential's supported terms, switched off by a cosine between r_inner and
// r_outer. It has no trainable parameter, so the same kernels serve inference
// (add it to the NEP energies, forces and virials) and training (subtract it
// from the targets once per dataset: the loss residuals, and hence the loss
// and its gradient, are then those of NEP + ZBL against the raw targets).
//
// Per pair, with a = 0.8854 a_0 / (Z_i^0.23 + Z_j^0.23) and x = r / a:
//   phi(r) = k_e Z_i Z_j / r * sum_k c_k exp(-d_k x) * f(r),
// and atom i takes half of each of its pairs' energy, E_i = 1/2 sum_j phi(r_ij),
// so each bond counts once. A pair potential's h_ij = dE_i/dr_ij is
// phi'(r) r_ij / (2r) and h_ji = -h_ij, so F_i = sum_j phi'(r_ij) r_ij / r
// needs no reverse-pair gather, and W_s = -1/2 sum phi'(r)/r r_ij (x) r_ij.
#include "nep_internal.hpp"

namespace nep {
namespace {

constexpr int kZblTeam = 8;    // lanes per atom
constexpr int kZblBlock = 256;
constexpr int kZblReduce = 256;

// e^2 / (4 pi eps_0) in eV A and the Bohr radius in A (CODATA); the universal
// screening function's four weights and decay rates (ZBL).
constexpr double kCoulomb = 14.399645;
constexpr double kBohr = 0.529177210903;
constexpr double kScrC[4] = {0.18175, 0.50986, 0.28022, 0.02817};
constexpr double kScrD[4] = {3.19980, 0.94229, 0.40290, 0.20162};

struct ZblArgs {
    double z[kMaxTypes];   // nuclear charge of each species
    double zp[kMaxTypes];  // Z^0.23 / (0.8854 a_0): inverse screening length = zp_i + zp_j
    double r_in, r_out2, pi_over_width;
};

// phi(r) and phi'(r) of one pair (switch included).
__device__ __forceinline__ void zbl_pair(double zz, double inv_a, double r, const ZblArgs& a, double& phi,
                                         double& dphi) {
    const double x = r * inv_a;
    double s = 0.0, ds = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double t = kScrC[k] * exp(-kScrD[k] * x);
        s += t;
        ds -= kScrD[k] * t;
    }
    const double ir = 1.0 / r;
    const double pre = kCoulomb * zz;
    const double v = pre * s * ir;
    const double dv = pre * ir * (ds * inv_a - s * ir);
    if (r <= a.r_in) {
        phi = v;
        dphi = dv;
    } else {
        double sn, cs;
        sincos(a.pi_over_width * (r - a.r_in), &sn, &cs);
        const double f = 0.5 * (1.0 + cs), fp = -0.5 * a.pi_over_width * sn;
        phi = v * f;
        dphi = dv * f + v * fp;
    }
}

// One team of kZblTeam lanes per atom: the team's lanes take the pairs of each
// neighbour-species group in turn, then sum their partials with DPP moves.
// Writes E_i and the atom's 9 virial terms (unscaled) and adds scale * F_i.
template <typename R>
__global__ void __launch_bounds__(kZblBlock)
k_zbl_atoms(long Na, int T, const int* __restrict__ types, const int64_t* __restrict__ row,
            const int* __restrict__ seg, const Rec<R>* __restrict__ pairs, ZblArgs a, double scale,
            R* __restrict__ force, double* __restrict__ e_at, double* __restrict__ w_at) {
    constexpr int S = kZblTeam, TEAMS = kZblBlock / S;
    const int team = threadIdx.x / S, lane = threadIdx.x % S;
    const long i = (long)xcd_tile(blockIdx.x, gridDim.x) * TEAMS + team;
    if (i >= Na) return;  // whole teams leave together: the DPP sums stay inside a team
    const int ti = types[i];
    const double zi = a.z[ti], zpi = a.zp[ti];
    // e, f[3], w = {xx, yy, zz, xy, xz, yz} of sum phi'(r)/r r (x) r
    double acc[10];
#pragma unroll
    for (int c = 0; c < 10; ++c) acc[c] = 0.0;
    int64_t p = row[i];
    for (int b = 0; b < T; ++b) {
        const int n = seg[(i * T + b) * 2];
        const double zz = zi * a.z[b], inv_a = zpi + a.zp[b];
        for (int q = lane; q < n; q += S) {
            const Rec<R> rc = pairs[p + q];
            const double x = rc.x, y = rc.y, z = rc.z;
            const double r2 = x * x + y * y + z * z;
            if (r2 < a.r_out2 && r2 > 0.0) {
                const double r = sqrt(r2);
                double phi, dphi;
                zbl_pair(zz, inv_a, r, a, phi, dphi);
                const double g = dphi / r;
                acc[0] += phi;
                acc[1] += g * x;
                acc[2] += g * y;
                acc[3] += g * z;
                acc[4] += g * x * x;
                acc[5] += g * y * y;
                acc[6] += g * z * z;
                acc[7] += g * x * y;
                acc[8] += g * x * z;
                acc[9] += g * y * z;
            }
        }
        p += n;
    }
#pragma unroll
    for (int c = 0; c < 10; ++c) acc[c] = team_sum<S>(acc[c]);
    if (lane != 0) return;
    e_at[i] = 0.5 * acc[0];
    double* w = w_at + i * 9;
    w[0] = -0.5 * acc[4];
    w[4] = -0.5 * acc[5];
    w[8] = -0.5 * acc[6];
    w[1] = w[3] = -0.5 * acc[7];
    w[2] = w[6] = -0.5 * acc[8];
    w[5] = w[7] = -0.5 * acc[9];
    if (force) {
#pragma unroll
        for (int d = 0; d < 3; ++d) force[i * 3 + d] = R(double(force[i * 3 + d]) + scale * acc[1 + d]);
    }
}

// One block per structure: E_s and W_s over its atoms, in a fixed order, added
// with the given sign and scale.
__global__ void __launch_bounds__(kZblReduce)
k_zbl_structure(const int64_t* __restrict__ off, const double* __restrict__ e_at, const double* __restrict__ w_at,
                double scale, double* __restrict__ energy, double* __restrict__ virial) {
    constexpr int NV = 10, WAVES = kZblReduce / 64;
    __shared__ double part[WAVES][NV];
    const int s = blockIdx.x;
    const long a0 = off[s], a1 = off[s + 1];
    double acc[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) acc[c] = 0.0;
    for (long i = a0 + threadIdx.x; i < a1; i += kZblReduce) {
        acc[0] += e_at[i];
#pragma unroll
        for (int c = 0; c < 9; ++c) acc[1 + c] += w_at[i * 9 + c];
    }
#pragma unroll
    for (int c = 0; c < NV; ++c) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc[c] += __shfl_xor(acc[c], o, 64);
    }
    const int wave = threadIdx.x / 64;
    if (threadIdx.x % 64 == 0) {
#pragma unroll
        for (int c = 0; c < NV; ++c) part[wave][c] = acc[c];
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = 0.0;
        for (int w = 0; w < WAVES; ++w) t += part[w][threadIdx.x];
        if (threadIdx.x == 0) {
            if (energy) energy[s] += scale * t;
        } else if (virial) {
            virial[s * 9 + threadIdx.x - 1] += scale * t;
        }
    }
}

template <typename R>
nep_status launch_zbl(const ZblArgs& a, int T, int Ns, long Na, const int64_t* off, const int* types,
                      const int64_t* row, const int* seg, const void* pairs, double scale, double* energy,
                      void* force, double* virial, void* ws, hipStream_t st) {
    double* e_at = static_cast<double*>(ws);
    double* w_at = e_at + Na;
    if (Na > 0) {
        const long teams = kZblBlock / kZblTeam;
        const int grid = int((Na + teams - 1) / teams);
        NEP_LAUNCH("zbl_atoms", k_zbl_atoms<R>, dim3(grid), dim3(kZblBlock), 0, st, Na, T, types, row, seg,
                   static_cast<const Rec<R>*>(pairs), a, scale, static_cast<R*>(force), e_at, w_at);
    }
    if (Ns > 0 && (energy || virial))
        NEP_LAUNCH("zbl_structure", k_zbl_structure, dim3(Ns), dim3(kZblReduce), 0, st, off, e_at, w_at, scale,
                   energy, virial);
    return NEP_OK;
}

}  // namespace

size_t zbl_workspace_bytes(long Na) { return size_t(Na) * 10 * sizeof(double); }

nep_status zbl_add(const Dims& dm, bool f64, const nep_zbl* z, const nep_batch* b, const nep_neighbors* nb,
                   double scale, double* energy, void* force, double* virial, void* ws, hipStream_t st) {
    ZblArgs a{};
    for (int t = 0; t < dm.T; ++t) {
        a.z[t] = double(z->atomic_number[t]);
        a.zp[t] = std::pow(a.z[t], 0.23) / (0.8854 * kBohr);
    }
    a.r_in = z->r_inner;
    a.r_out2 = z->r_outer * z->r_outer;
    a.pi_over_width = M_PI / (z->r_outer - z->r_inner);
    const long Na = long(b->num_atoms);
    return f64 ? launch_zbl<double>(a, dm.T, b->num_structures, Na, b->atom_offset, b->types, nb->row_offset,
                                    nb->seg_count, nb->pairs, scale, energy, force, virial, ws, st)
               : launch_zbl<float>(a, dm.T, b->num_structures, Na, b->atom_offset, b->types, nb->row_offset,
                                   nb->seg_count, nb->pairs, scale, energy, force, virial, ws, st);
}

}  // namespace nep
