// Neighbour lists of a packed batch of periodic structures.
//
// One lane per atom scans every atom of its structure and every periodic image
// n with |s_j - s_i + n|_d < rc / w_d in each lattice direction d (s are
// fractional coordinates, w the perpendicular cell widths), which is necessary
// for |r_ij| < rc; the distance test is done in double precision. Rows are
// written grouped by neighbour species, pairs inside the angular cutoff first
// in each group, in (j, image) scan order, so the result is deterministic.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "nep_device.hpp"
#include "nep_internal.hpp"

namespace nep {

namespace {

constexpr int kNbBlock = 128;

struct CellInfo {
    double H[9], Hi[9], w[3];
};

__device__ __forceinline__ CellInfo cell_info(const double* __restrict__ c) {
    CellInfo ci;
    for (int k = 0; k < 9; ++k) ci.H[k] = c[k];
    const double* H = ci.H;
    const double det = H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                       H[2] * (H[3] * H[7] - H[4] * H[6]);
    const double id = 1.0 / det;
    ci.Hi[0] = (H[4] * H[8] - H[5] * H[7]) * id;
    ci.Hi[1] = (H[2] * H[7] - H[1] * H[8]) * id;
    ci.Hi[2] = (H[1] * H[5] - H[2] * H[4]) * id;
    ci.Hi[3] = (H[5] * H[6] - H[3] * H[8]) * id;
    ci.Hi[4] = (H[0] * H[8] - H[2] * H[6]) * id;
    ci.Hi[5] = (H[2] * H[3] - H[0] * H[5]) * id;
    ci.Hi[6] = (H[3] * H[7] - H[4] * H[6]) * id;
    ci.Hi[7] = (H[1] * H[6] - H[0] * H[7]) * id;
    ci.Hi[8] = (H[0] * H[4] - H[1] * H[3]) * id;
    // width along lattice direction d = volume / |cross of the other two rows|
    //   = 1 / |column d of H^-1|
    for (int d = 0; d < 3; ++d) {
        const double x = ci.Hi[d], y = ci.Hi[3 + d], z = ci.Hi[6 + d];
        ci.w[d] = 1.0 / sqrt(x * x + y * y + z * z);
    }
    return ci;
}

__device__ __forceinline__ int find_struct(const int64_t* __restrict__ off, int Ns, long i) {
    int lo = 0, hi = Ns;  // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

template <typename R, bool FILL>
__global__ void __launch_bounds__(kNbBlock)
k_neighbors(int Ns, long Na, int T, const int64_t* __restrict__ off, const R* __restrict__ pos,
            const int* __restrict__ types, const double* __restrict__ cells, double rcR, double rcA,
            int* __restrict__ seg, int64_t* __restrict__ count_or_row, int* __restrict__ atom_struct,
            Rec<R>* __restrict__ pairs) {
    const long i = (long)blockIdx.x * kNbBlock + threadIdx.x;
    if (i >= Na) return;
    const int s = find_struct(off, Ns, i);
    const CellInfo ci = cell_info(cells + 9L * s);
    const long j0 = off[s], j1 = off[s + 1];
    const double ri[3] = {double(pos[3 * i]), double(pos[3 * i + 1]), double(pos[3 * i + 2])};
    double fi[3];
    for (int d = 0; d < 3; ++d) fi[d] = ri[0] * ci.Hi[d] + ri[1] * ci.Hi[3 + d] + ri[2] * ci.Hi[6 + d];
    const double rc2R = rcR * rcR, rc2A = rcA * rcA;
    int cur[2 * kMaxTypes];  // FILL: write cursors {angular, radial-only} per species
    int64_t base = 0;
    if (FILL) {
        base = count_or_row[i];
        int acc = 0;
        for (int b = 0; b < T; ++b) {
            cur[2 * b] = acc;
            cur[2 * b + 1] = acc + seg[(i * T + b) * 2 + 1];
            acc += seg[(i * T + b) * 2];
        }
    } else {
        for (int b = 0; b < 2 * T; ++b) cur[b] = 0;
        atom_struct[i] = s;
    }
    for (long j = j0; j < j1; ++j) {
        const double rj[3] = {double(pos[3 * j]), double(pos[3 * j + 1]), double(pos[3 * j + 2])};
        const int tb = types[j];
        int lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            const double fj = rj[0] * ci.Hi[d] + rj[1] * ci.Hi[3 + d] + rj[2] * ci.Hi[6 + d];
            const double ds = fj - fi[d];
            const double h = rcR / ci.w[d] + 1e-9;
            lo[d] = (int)ceil(-ds - h);
            hi[d] = (int)floor(-ds + h);
        }
        for (int n0 = lo[0]; n0 <= hi[0]; ++n0)
            for (int n1 = lo[1]; n1 <= hi[1]; ++n1)
                for (int n2 = lo[2]; n2 <= hi[2]; ++n2) {
                    if (j == i && n0 == 0 && n1 == 0 && n2 == 0) continue;
                    double r[3];
                    for (int d = 0; d < 3; ++d)
                        r[d] = rj[d] + n0 * ci.H[d] + n1 * ci.H[3 + d] + n2 * ci.H[6 + d] - ri[d];
                    const double d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                    if (!(d2 < rc2R)) continue;
                    const bool ang = d2 < rc2A;
                    if (FILL) {
                        const int slot = ang ? cur[2 * tb]++ : cur[2 * tb + 1]++;
                        Rec<R> rec;
                        rec.x = R(r[0]);
                        rec.y = R(r[1]);
                        rec.z = R(r[2]);
                        if constexpr (sizeof(R) == 4)
                            rec.w = __int_as_float((int)j);
                        else
                            rec.w = __longlong_as_double((long long)j);
                        pairs[base + slot] = rec;
                    } else {
                        cur[2 * tb] += 1;
                        if (ang) cur[2 * tb + 1] += 1;
                    }
                }
    }
    if (!FILL) {
        int64_t tot = 0;
        for (int b = 0; b < T; ++b) {
            seg[(i * T + b) * 2] = cur[2 * b];
            seg[(i * T + b) * 2 + 1] = cur[2 * b + 1];
            tot += cur[2 * b];
        }
        count_or_row[i + 1] = tot;
    }
}

// reverse[p] = index of the pair (j, i, -n) for pair p = (i, j, n): the entry
// of row j with neighbour i whose vector is closest to -r_ij (exactly -r_ij up
// to rounding; other images of the same atom differ by a lattice vector).
// -1 if the reverse pair was not kept (possible only at |r_ij| = rc to rounding).
template <typename R>
__global__ void __launch_bounds__(kNbBlock)
k_reverse(long Na, const int64_t* __restrict__ row, const Rec<R>* __restrict__ pairs, int* __restrict__ reverse) {
    const long i = (long)blockIdx.x * kNbBlock + threadIdx.x;
    if (i >= Na) return;
    for (int64_t p = row[i]; p < row[i + 1]; ++p) {
        const Rec<R> a = pairs[p];
        const long j = rec_j(a);
        int64_t best = -1;
        double bd = 1e300;
        for (int64_t q = row[j]; q < row[j + 1]; ++q) {
            const Rec<R> b = pairs[q];
            if (rec_j(b) != i) continue;
            const double dx = double(a.x) + double(b.x), dy = double(a.y) + double(b.y), dz = double(a.z) + double(b.z);
            const double d = dx * dx + dy * dy + dz * dz;
            if (d < bd) {
                bd = d;
                best = q;
            }
        }
        reverse[p] = (best >= 0 && bd < 1e-6) ? int(best) : -1;
    }
}

// Exclusive scan row[0..Na] of the per-row counts in row[1..Na] (row[0] = 0),
// one block; also sums the angular counts into totals[1] (totals[0] = pairs).
constexpr int kScanBlock = 1024;

__global__ void __launch_bounds__(kScanBlock)
k_scan_rows(long Na, int T, int64_t* __restrict__ row, const int* __restrict__ seg, int64_t* __restrict__ totals) {
    __shared__ int64_t buf[kScanBlock];
    __shared__ int64_t carry_s;
    if (threadIdx.x == 0) {
        carry_s = 0;
        row[0] = 0;
    }
    int64_t ang = 0;
    for (long i = threadIdx.x; i < Na * T; i += kScanBlock) ang += seg[2 * i + 1];
    __syncthreads();
    for (long base = 0; base < Na; base += kScanBlock) {
        const long i = base + threadIdx.x;
        const int64_t v = (i < Na) ? row[i + 1] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < kScanBlock; o <<= 1) {
            const int64_t t = (threadIdx.x >= (unsigned)o) ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        const int64_t incl = buf[threadIdx.x] + carry_s;
        if (i < Na) row[i + 1] = incl;
        __syncthreads();
        if (threadIdx.x == kScanBlock - 1) carry_s = incl;
        __syncthreads();
    }
    // angular total
    buf[threadIdx.x] = ang;
    __syncthreads();
    for (int s = kScanBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < (unsigned)s) buf[threadIdx.x] += buf[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        totals[0] = row[Na];
        totals[1] = buf[0];
    }
}

// Stable sort of atom indices by species, one block: each thread owns a
// contiguous chunk, counts per species, and scatters after a block scan.
__global__ void __launch_bounds__(kScanBlock)
k_species_sort(long Na, int T, const int* __restrict__ types, int* __restrict__ order, int64_t* __restrict__ soff) {
    __shared__ int cnt[kScanBlock];
    __shared__ int64_t tot_s[kMaxTypes + 1];
    const long per = (Na + kScanBlock - 1) / kScanBlock;
    const long c0 = threadIdx.x * per, c1 = min(Na, c0 + per);
    if (threadIdx.x == 0) tot_s[0] = 0;
    for (int t = 0; t < T; ++t) {
        int c = 0;
        for (long i = c0; i < c1; ++i) c += types[i] == t;
        cnt[threadIdx.x] = c;
        __syncthreads();
        // inclusive scan of cnt
        for (int o = 1; o < kScanBlock; o <<= 1) {
            const int x = (threadIdx.x >= (unsigned)o) ? cnt[threadIdx.x - o] : 0;
            __syncthreads();
            cnt[threadIdx.x] += x;
            __syncthreads();
        }
        const int64_t start = tot_s[t] + (cnt[threadIdx.x] - c);
        int64_t w = start;
        for (long i = c0; i < c1; ++i)
            if (types[i] == t) order[w++] = (int)i;
        __syncthreads();
        if (threadIdx.x == kScanBlock - 1) tot_s[t + 1] = tot_s[t] + cnt[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x <= (unsigned)T) soff[threadIdx.x] = tot_s[threadIdx.x];
}

template <typename R>
nep_status build_neighbors_impl(const Ctx& c, const nep_batch* b, nep_neighbors* nb, void* ws, size_t ws_bytes) {
    const long Na = b->num_atoms;
    const int Ns = b->num_structures, T = c.dm.T;
    if (ws_bytes < sizeof(int64_t) * 2) return fail(NEP_ERR_WORKSPACE, "workspace too small for neighbour totals");
    int64_t* totals = static_cast<int64_t*>(ws);
    hipStream_t st = c.stream;
    const R* pos = static_cast<const R*>(b->positions);
    const int grid = int((Na + kNbBlock - 1) / kNbBlock);
    // Host-side validation of the index arrays every later kernel trusts:
    // offsets must run 0 .. Na without decreasing and species must lie in [0, T).
    {
        std::vector<int64_t> off(static_cast<size_t>(Ns) + 1);
        NEP_HIP(hipMemcpyAsync(off.data(), b->atom_offset, sizeof(int64_t) * off.size(), hipMemcpyDeviceToHost, st));
        std::vector<int> typ(static_cast<size_t>(Na));
        if (Na > 0) NEP_HIP(hipMemcpyAsync(typ.data(), b->types, sizeof(int) * typ.size(), hipMemcpyDeviceToHost, st));
        NEP_HIP(hipStreamSynchronize(st));
        if (off[0] != 0 || off[Ns] != Na) return fail(NEP_ERR_INVALID_ARG, "atom_offset must run from 0 to num_atoms");
        for (int s = 0; s < Ns; ++s)
            if (off[s + 1] < off[s]) return fail(NEP_ERR_INVALID_ARG, "atom_offset decreases at structure %d", s);
        for (long i = 0; i < Na; ++i)
            if (typ[i] < 0 || typ[i] >= T) return fail(NEP_ERR_INVALID_ARG, "atom %ld has species %d outside [0, %d)", i, typ[i], T);
    }
    if (Na > 0) {
        NEP_LAUNCH("neighbors_count", (k_neighbors<R, false>), dim3(grid), dim3(kNbBlock), 0, st, Ns, Na, T,
                   b->atom_offset, pos, b->types, b->cells, c.dm.rcR, c.dm.rcA, nb->seg_count, nb->row_offset,
                   nb->atom_struct, (Rec<R>*)nullptr);
    }
    NEP_LAUNCH("neighbors_scan", k_scan_rows, dim3(1), dim3(kScanBlock), 0, st, Na, T, nb->row_offset, nb->seg_count,
               totals);
    NEP_LAUNCH("species_sort", k_species_sort, dim3(1), dim3(kScanBlock), 0, st, Na, T, b->types, nb->species_order,
               nb->species_offset);
    int64_t host_tot[2] = {0, 0};
    NEP_HIP(hipMemcpyAsync(host_tot, totals, sizeof(host_tot), hipMemcpyDeviceToHost, st));
    NEP_HIP(hipStreamSynchronize(st));
    nb->num_pairs = host_tot[0];
    nb->num_angular_pairs = host_tot[1];
    if (host_tot[0] >= (int64_t(1) << 31)) return fail(NEP_ERR_UNSUPPORTED, "more than 2^31-1 pairs in one batch");
    if (host_tot[0] > nb->capacity) {
        return fail(NEP_ERR_CAPACITY, "neighbour capacity too small: need %lld pairs, have %lld",
                    (long long)host_tot[0], (long long)nb->capacity);
    }
    if (Na > 0 && host_tot[0] > 0) {
        NEP_LAUNCH("neighbors_fill", (k_neighbors<R, true>), dim3(grid), dim3(kNbBlock), 0, st, Ns, Na, T,
                   b->atom_offset, pos, b->types, b->cells, c.dm.rcR, c.dm.rcA, nb->seg_count, nb->row_offset,
                   nb->atom_struct, static_cast<Rec<R>*>(nb->pairs));
        NEP_LAUNCH("neighbors_reverse", (k_reverse<R>), dim3(grid), dim3(kNbBlock), 0, st, Na, nb->row_offset,
                   static_cast<const Rec<R>*>(nb->pairs), nb->reverse);
    }
    return NEP_OK;
}

}  // namespace

nep_status build_neighbors(const Ctx& c, const nep_batch* b, nep_neighbors* nb, void* ws, size_t ws_bytes) {
    return c.f64 ? build_neighbors_impl<double>(c, b, nb, ws, ws_bytes)
                 : build_neighbors_impl<float>(c, b, nb, ws, ws_bytes);
}

}  // namespace nep
