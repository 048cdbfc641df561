// Neighbour lists of a packed batch of periodic structures, built with cell lists.
//
// Each structure's cell is cut into n_d >= 1 bins along every lattice
// direction d, each at least r_c wide across (n_d = floor(w_d / r_c), w_d the
// perpendicular width), at most one bin per atom. Atoms are binned by their
// wrapped fractional coordinates; a bin's atoms are kept in index order. A
// team of lanes per atom then scans the bins c + delta, |delta_d| <= ceil(r_c n_d / w_d):
// bin (c + delta) mod n lies in periodic image floor((c + delta) / n), so thin
// cells (n_d = 1, w_d < r_c) get their extra images from the same loop, and
// each (j, image) is visited once. Distances are tested in double precision.
// Rows are written grouped by neighbour species, pairs inside the angular
// cutoff first in each group, in scan order, so the result is deterministic.
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

// An atom as the neighbour search reads it, stored in bin order: wrapped
// position, index and species (one contiguous record per candidate).
struct alignas(16) BinRec {
    double x, y, z;
    int j, t;
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

// Per structure: bins per lattice direction and the structure's bin count.
__global__ void __launch_bounds__(kNbBlock)
k_cell_setup(int Ns, const int64_t* __restrict__ off, const double* __restrict__ cells, double rc,
             int* __restrict__ sbins, int64_t* __restrict__ bin_base) {
    const int s = blockIdx.x * kNbBlock + threadIdx.x;
    if (s >= Ns) return;
    const CellInfo ci = cell_info(cells + 9L * s);
    const long n_at = off[s + 1] - off[s];
    long nb[3];
    for (int d = 0; d < 3; ++d) {
        const double q = floor(ci.w[d] / rc);
        nb[d] = q < 1.0 ? 1 : (q > 1024.0 ? 1024 : long(q));
    }
    const long cap = n_at > 1 ? n_at : 1;
    while (nb[0] * nb[1] * nb[2] > cap) {  // at most one bin per atom
        int dm = 0;
        for (int d = 1; d < 3; ++d)
            if (nb[d] > nb[dm]) dm = d;
        nb[dm] -= 1;
    }
    for (int d = 0; d < 3; ++d) sbins[3 * s + d] = int(nb[d]);
    bin_base[s + 1] = nb[0] * nb[1] * nb[2];
}

// Single-block exclusive scan in place: a[0] = 0, a[1..n] counts -> running sums.
constexpr int kScanBlock = 1024;

__global__ void __launch_bounds__(kScanBlock)
k_scan_counts(long n, int64_t* __restrict__ a) {
    __shared__ int64_t buf[kScanBlock];
    __shared__ int64_t carry_s;
    if (threadIdx.x == 0) {
        carry_s = 0;
        a[0] = 0;
    }
    __syncthreads();
    for (long base = 0; base < n; base += kScanBlock) {
        const long i = base + threadIdx.x;
        buf[threadIdx.x] = (i < n) ? a[i + 1] : 0;
        __syncthreads();
        for (int o = 1; o < kScanBlock; o <<= 1) {
            const int64_t t = (threadIdx.x >= (unsigned)o) ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        const int64_t incl = buf[threadIdx.x] + carry_s;
        if (i < n) a[i + 1] = incl;
        __syncthreads();
        if (threadIdx.x == kScanBlock - 1) carry_s = incl;
        __syncthreads();
    }
}

template <typename I>
__global__ void __launch_bounds__(kNbBlock) k_zero(long n, I* __restrict__ a) {
    const long i = (long)blockIdx.x * kNbBlock + threadIdx.x;
    if (i < n) a[i] = 0;
}

// Per atom: structure, wrapped position r - floor(f) H (f = r H^-1 the
// fractional coordinates, wrapped into [0, 1)) and global bin index; counts
// atoms per bin (bin_count[b + 1]).
template <typename R>
__global__ void __launch_bounds__(kNbBlock)
k_bin_atoms(int Ns, long Na, const int64_t* __restrict__ off, const R* __restrict__ pos,
            const double* __restrict__ cells, const int* __restrict__ sbins, const int64_t* __restrict__ bin_base,
            int* __restrict__ atom_struct, int* __restrict__ atom_bin, double* __restrict__ wpos,
            unsigned long long* __restrict__ bin_count) {
    const long i = (long)blockIdx.x * kNbBlock + threadIdx.x;
    if (i >= Na) return;
    const int s = find_struct(off, Ns, i);
    const CellInfo ci = cell_info(cells + 9L * s);
    const double r[3] = {double(pos[3 * i]), double(pos[3 * i + 1]), double(pos[3 * i + 2])};
    double sh[3];
    int c[3];
    for (int d = 0; d < 3; ++d) {
        const double f = r[0] * ci.Hi[d] + r[1] * ci.Hi[3 + d] + r[2] * ci.Hi[6 + d];
        double n = floor(f), fw = f - n;
        if (fw >= 1.0) {
            n += 1.0;
            fw = 0.0;
        }
        sh[d] = n;
        const int nb = sbins[3 * s + d];
        const int cd = int(fw * nb);
        c[d] = cd < nb ? cd : nb - 1;
    }
    for (int x = 0; x < 3; ++x) wpos[3 * i + x] = r[x] - (sh[0] * ci.H[x] + sh[1] * ci.H[3 + x] + sh[2] * ci.H[6 + x]);
    const int gb = int(bin_base[s] + (long(c[0]) * sbins[3 * s + 1] + c[1]) * sbins[3 * s + 2] + c[2]);
    atom_struct[i] = s;
    atom_bin[i] = gb;
    atomicAdd(bin_count + gb + 1, 1ull);
}

// bad != 0 after the launch if a species lies outside [0, T).
__global__ void __launch_bounds__(kNbBlock)
k_check_types(long Na, int T, const int* __restrict__ types, unsigned int* __restrict__ bad) {
    const long i = (long)blockIdx.x * kNbBlock + threadIdx.x;
    if (i < Na && (types[i] < 0 || types[i] >= T)) atomicOr(bad, 1u);
}

// Scatter atoms into their bins (arbitrary order within a bin, fixed below).
__global__ void __launch_bounds__(kNbBlock)
k_bin_fill(long Na, const int* __restrict__ atom_bin, const int64_t* __restrict__ bin_start,
           unsigned int* __restrict__ cursor, int* __restrict__ bin_tmp) {
    const long i = (long)blockIdx.x * kNbBlock + threadIdx.x;
    if (i >= Na) return;
    const int gb = atom_bin[i];
    const unsigned int k = atomicAdd(cursor + gb, 1u);
    bin_tmp[bin_start[gb] + k] = int(i);
}

// Each bin's atoms in increasing index order: atom i's rank in its bin is the
// number of members with a smaller index (one lane per atom); its record goes
// to that slot.
__global__ void __launch_bounds__(kNbBlock)
k_bin_rank(long Na, const int* __restrict__ atom_bin, const int64_t* __restrict__ bin_start,
           const int* __restrict__ bin_tmp, const double* __restrict__ wpos, const int* __restrict__ types,
           BinRec* __restrict__ bin_rec) {
    const long i = (long)blockIdx.x * kNbBlock + threadIdx.x;
    if (i >= Na) return;
    const int gb = atom_bin[i];
    const int64_t lo = bin_start[gb], hi = bin_start[gb + 1];
    int64_t rank = 0;
    for (int64_t q = lo; q < hi; ++q) rank += bin_tmp[q] < i;
    BinRec br;
    br.x = wpos[3 * i];
    br.y = wpos[3 * i + 1];
    br.z = wpos[3 * i + 2];
    br.j = int(i);
    br.t = types[i];
    bin_rec[lo + rank] = br;
}

__device__ __forceinline__ int floordiv(int a, int n) { return a >= 0 ? a / n : -((-a + n - 1) / n); }

// One team of kNbTeam lanes per atom: the team walks the bins c + delta
// together and splits each bin's atoms over its lanes, kNbTeam candidates at
// a time in bin order. COUNT (FILL = false) writes the per-species
// {all, angular} counts and the row length; FILL writes the records, each
// (species, angular or not) group filled in candidate order: a lane's slot is
// the group's cursor plus the hits of lower lanes in the same batch (team
// ballots), so the rows are those of a scan of the bins one candidate at a time;
// COUNT tallies per lane and sums over the team once at the end.
// MT >= T bounds the per-species cursors (4, 8 or 16: fewer registers, more
// waves per SIMD for batches with few species).
constexpr int kNbTeam = 16;

template <typename R, bool FILL, int MT>
__global__ void __launch_bounds__(kNbBlock)
k_neighbors(long Na, int T, const double* __restrict__ cells, double rcR,
            double rcA, const int* __restrict__ atom_struct, const int* __restrict__ atom_bin,
            const double* __restrict__ wpos, const int* __restrict__ sbins, const int64_t* __restrict__ bin_base,
            const int64_t* __restrict__ bin_start, const BinRec* __restrict__ bin_rec, int* __restrict__ seg,
            int64_t* __restrict__ count_or_row, Rec<R>* __restrict__ pairs) {
    constexpr int S = kNbTeam, TEAMS = kNbBlock / S;
    const int team = threadIdx.x / S, lane = threadIdx.x % S;
    const long i = (long)blockIdx.x * TEAMS + team;
    if (i >= Na) return;  // whole teams
    const int tshift = (threadIdx.x & 63) / S * S;  // the team's first bit in a wave ballot
    const unsigned long long below = (1ull << lane) - 1ull;
    const int s = atom_struct[i];
    const CellInfo ci = cell_info(cells + 9L * s);
    const int nb[3] = {sbins[3 * s], sbins[3 * s + 1], sbins[3 * s + 2]};
    int c[3];
    {
        int loc = int(atom_bin[i] - bin_base[s]);
        c[2] = loc % nb[2];
        loc /= nb[2];
        c[1] = loc % nb[1];
        c[0] = loc / nb[1];
    }
    const double ri[3] = {wpos[3 * i], wpos[3 * i + 1], wpos[3 * i + 2]};
    // Bin t along direction d is the slab t/n_d <= f_d < (t+1)/n_d between two
    // lattice planes; an atom at fractional coordinate f is at least
    // w_d * (distance in f) from every point of it. Slabs that far or farther
    // (with a 1e-9 A margin) are dropped from both ends of the range the
    // bins c +- kk would cover, per direction.
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        const int kk = int(ceil(rcR * nb[d] / ci.w[d] + 1e-9));
        const double f = ri[0] * ci.Hi[d] + ri[1] * ci.Hi[3 + d] + ri[2] * ci.Hi[6 + d];
        const double rcut = rcR + 1e-9;
        lo[d] = c[d] - kk;
        hi[d] = c[d] + kk;
        while (lo[d] < c[d] && ci.w[d] * (f - double(lo[d] + 1) / nb[d]) >= rcut) ++lo[d];
        while (hi[d] > c[d] && ci.w[d] * (double(hi[d]) / nb[d] - f) >= rcut) --hi[d];
    }
    const double rc2R = rcR * rcR, rc2A = rcA * rcA;
    // per species {angular, radial-only}: FILL write cursors, COUNT {all, angular} counts
    int cur[2 * MT];
    int64_t base = 0;
#pragma unroll
    for (int b = 0; b < 2 * MT; ++b) cur[b] = 0;
    if (FILL) {
        base = count_or_row[i];
        int acc = 0;
#pragma unroll
        for (int b = 0; b < MT; ++b) {
            if (b >= T) break;
            cur[2 * b] = acc;
            cur[2 * b + 1] = acc + seg[(i * T + b) * 2 + 1];
            acc += seg[(i * T + b) * 2];
        }
    }
    for (int t0 = lo[0]; t0 <= hi[0]; ++t0) {
        const int m0 = floordiv(t0, nb[0]), b0 = t0 - m0 * nb[0];
        for (int t1 = lo[1]; t1 <= hi[1]; ++t1) {
            const int m1 = floordiv(t1, nb[1]), b1 = t1 - m1 * nb[1];
            for (int t2 = lo[2]; t2 <= hi[2]; ++t2) {
                const int m2 = floordiv(t2, nb[2]), b2 = t2 - m2 * nb[2];
                double sh[3];
                for (int x = 0; x < 3; ++x) sh[x] = m0 * ci.H[x] + m1 * ci.H[3 + x] + m2 * ci.H[6 + x] - ri[x];
                const bool self_image = m0 == 0 && m1 == 0 && m2 == 0;
                const long gb = bin_base[s] + (long(b0) * nb[1] + b1) * nb[2] + b2;
                const int64_t q1 = bin_start[gb + 1];
                for (int64_t qb = bin_start[gb]; qb < q1; qb += S) {
                    const int64_t q = qb + lane;
                    bool hit = false, ang = false;
                    int tb = -1, j = 0;
                    double r[3] = {0.0, 0.0, 0.0};
                    if (q < q1) {
                        const BinRec br = bin_rec[q];
                        j = br.j;
                        if (!(self_image && j == i)) {
                            r[0] = br.x + sh[0];
                            r[1] = br.y + sh[1];
                            r[2] = br.z + sh[2];
                            const double d2v = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                            hit = d2v < rc2R;
                            ang = d2v < rc2A;
                            if (hit) tb = br.t;
                        }
                    }
                    if (!FILL) {  // counting: per-lane tallies, summed over the team at the end
#pragma unroll
                        for (int b = 0; b < MT; ++b) {
                            cur[2 * b] += tb == b;
                            cur[2 * b + 1] += tb == b && ang;
                        }
                        continue;
                    }
#pragma unroll
                    for (int b = 0; b < MT; ++b) {
                        if (b >= T) break;
                        const unsigned long long ma = (__ballot(tb == b && ang) >> tshift) & ((1ull << S) - 1ull);
                        const unsigned long long mr = (__ballot(tb == b && !ang) >> tshift) & ((1ull << S) - 1ull);
                        if (tb == b) {
                            const int slot = ang ? cur[2 * b] + __popcll(ma & below)
                                                 : cur[2 * b + 1] + __popcll(mr & below);
                            Rec<R> rec;
                            rec.x = R(r[0]);
                            rec.y = R(r[1]);
                            rec.z = R(r[2]);
                            if constexpr (sizeof(R) == 4)
                                rec.w = __int_as_float(j);
                            else
                                rec.w = __longlong_as_double((long long)j);
                            pairs[base + slot] = rec;
                        }
                        cur[2 * b] += __popcll(ma);
                        cur[2 * b + 1] += __popcll(mr);
                    }
                }
            }
        }
    }
    if (!FILL) {
#pragma unroll
        for (int b = 0; b < 2 * MT; ++b) {
#pragma unroll
            for (int o = 1; o < S; o <<= 1) cur[b] += __shfl_xor(cur[b], o, 64);
        }
    }
    if (!FILL && lane == 0) {
        int64_t tot = 0;
#pragma unroll
        for (int b = 0; b < MT; ++b) {
            if (b >= T) break;
            seg[(i * T + b) * 2] = cur[2 * b];
            seg[(i * T + b) * 2 + 1] = cur[2 * b + 1];
            tot += cur[2 * b];
        }
        count_or_row[i + 1] = tot;
    }
}

// Reverse pair of every pair: p = (i -> j, image n) is matched with the pair
// q = (j -> i, -n) in row j's group of species(i), the one with r_q = -r_p
// (other images of i in that group differ from -r_p by a lattice vector, so
// at most one record lies within 1e-3 A of it). One lane per pair, the group
// read kRevBatch records at a time so that many loads are in flight. Each
// unordered pair is searched once, from its end with the lower atom index,
// which writes both reverse[p] and reverse[q]; pairs of an atom with its own
// images search for themselves. reverse[] starts at -1 (k_fill), which stays
// where no partner was kept (possible only at |r_ij| = r_c, to rounding).
constexpr int kRevBatch = 8;

__global__ void __launch_bounds__(kNbBlock) k_fill(long n, int v, int* __restrict__ a) {
    const long i = (long)blockIdx.x * kNbBlock + threadIdx.x;
    if (i < n) a[i] = v;
}

template <typename R>
__global__ void __launch_bounds__(kNbBlock)
k_reverse(long Na, long npairs, int T, const int* __restrict__ types, const int* __restrict__ seg,
          const int64_t* __restrict__ row, const Rec<R>* __restrict__ pairs, int* __restrict__ reverse) {
    // the block's pairs belong to a short run of rows: two lanes find the rows
    // of its first and last pair by bisection over all rows, every lane then
    // bisects only inside that run (row[lo] <= p < row[hi] throughout)
    __shared__ long run_s[2];
    const long p0 = (long)blockIdx.x * kNbBlock;
    const long p = p0 + threadIdx.x;
    if (threadIdx.x < 2) {
        const long key = threadIdx.x == 0 ? p0 : min(p0 + kNbBlock, npairs) - 1;
        long lo = 0, hi = Na;
        while (hi - lo > 1) {
            const long mid = (lo + hi) >> 1;
            if (row[mid] <= key)
                lo = mid;
            else
                hi = mid;
        }
        run_s[threadIdx.x] = lo;
    }
    __syncthreads();
    if (p >= npairs) return;
    long lo = run_s[0], hi = run_s[1] + 1;
    while (hi - lo > 1) {
        const long mid = (lo + hi) >> 1;
        if (row[mid] <= p)
            lo = mid;
        else
            hi = mid;
    }
    const long i = lo;
    const Rec<R> a = pairs[p];
    const long j = rec_j(a);
    if (j < i) return;  // searched from the other end
    const int ti = types[i];
    if (ti < 0 || ti >= T) return;  // reported by k_check_types
    int64_t g0 = row[j];
    for (int b = 0; b < ti; ++b) g0 += seg[(j * T + b) * 2];
    const int n = seg[(j * T + ti) * 2];
    long found = -1;
    for (int base = 0; base < n && found < 0; base += kRevBatch) {
        Rec<R> b[kRevBatch];
#pragma unroll
        for (int u = 0; u < kRevBatch; ++u) b[u] = pairs[g0 + min(base + u, n - 1)];  // in the group
#pragma unroll
        for (int u = 0; u < kRevBatch; ++u) {
            if (base + u >= n || rec_j(b[u]) != i) continue;
            const double dx = double(a.x) + double(b[u].x), dy = double(a.y) + double(b[u].y),
                         dz = double(a.z) + double(b[u].z);
            if (found < 0 && dx * dx + dy * dy + dz * dz < 1e-6) found = g0 + base + u;
        }
    }
    if (found < 0) return;
    reverse[p] = int(found);
    if (j != i) reverse[found] = int(p);
}

// Multi-block form of the same exclusive scan, for long arrays: tiles of
// kTile counts get their sums (k_tile_sums), a one-block scan turns those into
// tile offsets (k_scan_counts on tile[0..ntiles]), and each tile then scans
// itself from its offset (k_tile_apply). Every block touches only its own tile.
constexpr int kTileThreads = 256, kTileItems = 8, kTile = kTileThreads * kTileItems;

__device__ __forceinline__ int64_t block_sum_256(int64_t v, int64_t* part) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (threadIdx.x % 64 == 0) part[threadIdx.x / 64] = v;
    __syncthreads();
    return part[0] + part[1] + part[2] + part[3];
}

// tile[b + 1] = sum of the counts a[1 + b*kTile ...]; with seg != nullptr
// (the row scan) also adds the angular counts of the tile's atoms to *ang.
__global__ void __launch_bounds__(kTileThreads)
k_tile_sums(long n, const int64_t* __restrict__ a, int64_t* __restrict__ tile, int T, const int* __restrict__ seg,
            unsigned long long* __restrict__ ang) {
    __shared__ int64_t part[kTileThreads / 64];
    const long base = (long)blockIdx.x * kTile;
    int64_t s = 0, g = 0;
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
        const long i = base + k * kTileThreads + threadIdx.x;
        if (i < n) {
            s += a[i + 1];
            if (seg)
                for (int b = 0; b < T; ++b) g += seg[(i * T + b) * 2 + 1];
        }
    }
    const int64_t tot = block_sum_256(s, part);
    if (threadIdx.x == 0) tile[blockIdx.x + 1] = tot;
    if (seg) {
        __syncthreads();
        const int64_t gt = block_sum_256(g, part);
        if (threadIdx.x == 0) atomicAdd(ang, (unsigned long long)gt);
    }
}

// a[1 + i] = tile offset + inclusive sum inside the tile; a[0] = 0. With
// last != nullptr the grand total a[n] is also stored there.
__global__ void __launch_bounds__(kTileThreads)
k_tile_apply(long n, int64_t* __restrict__ a, const int64_t* __restrict__ tile, int64_t* __restrict__ last) {
    __shared__ int64_t wsum[kTileThreads / 64];
    const long i0 = (long)blockIdx.x * kTile + (long)threadIdx.x * kTileItems;
    int64_t v[kTileItems], s = 0;
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
        v[k] = (i0 + k < n) ? a[i0 + k + 1] : 0;
        s += v[k];
    }
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    int64_t incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int64_t run = tile[blockIdx.x] + incl - s;
    for (int w = 0; w < wave; ++w) run += wsum[w];
#pragma unroll
    for (int k = 0; k < kTileItems; ++k) {
        run += v[k];
        if (i0 + k < n) {
            a[i0 + k + 1] = run;
            if (last && i0 + k == n - 1) *last = run;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) a[0] = 0;
}

// Stable sort of atom indices by species over many blocks: one wavefront per
// tile of kSortTile atoms counts each species with ballots, one block turns the
// counts into each tile's first slot per species, and the wavefronts then
// place their atoms in index order (slot = tile base + running count + rank
// among the lower lanes with the same species). Same result as the one-block
// sort below.
constexpr int kSortTile = 1024;

__global__ void __launch_bounds__(64)
k_species_count(long Na, int T, const int* __restrict__ types, int* __restrict__ cnt) {
    const long base = (long)blockIdx.x * kSortTile;
    int c[kMaxTypes];
#pragma unroll
    for (int t = 0; t < kMaxTypes; ++t) c[t] = 0;
    for (int st = 0; st < kSortTile / 64; ++st) {
        const long i = base + st * 64 + threadIdx.x;
        const int ty = i < Na ? types[i] : -1;
#pragma unroll
        for (int t = 0; t < kMaxTypes; ++t) {
            if (t >= T) break;
            c[t] += __popcll(__ballot(ty == t));
        }
    }
    int mine = 0;
#pragma unroll
    for (int t = 0; t < kMaxTypes; ++t)
        if ((int)threadIdx.x == t) mine = c[t];
    if ((int)threadIdx.x < T) cnt[blockIdx.x * T + threadIdx.x] = mine;
}

// cnt[k][t] -> first slot of species t in tile k; soff[0..T] species starts.
__global__ void __launch_bounds__(kScanBlock)
k_species_base(long ntiles, int T, int* __restrict__ cnt, int64_t* __restrict__ soff) {
    __shared__ int buf[kScanBlock];
    __shared__ int tot_s[kMaxTypes + 1];
    for (int t = 0; t < T; ++t) {
        int carry = 0;
        for (long b0 = 0; b0 < ntiles; b0 += kScanBlock) {
            const long k = b0 + threadIdx.x;
            const int v = k < ntiles ? cnt[k * T + t] : 0;
            buf[threadIdx.x] = v;
            __syncthreads();
            for (int o = 1; o < kScanBlock; o <<= 1) {
                const int x = (threadIdx.x >= (unsigned)o) ? buf[threadIdx.x - o] : 0;
                __syncthreads();
                buf[threadIdx.x] += x;
                __syncthreads();
            }
            if (k < ntiles) cnt[k * T + t] = carry + buf[threadIdx.x] - v;
            carry += buf[kScanBlock - 1];
            __syncthreads();
        }
        if (threadIdx.x == 0) tot_s[t] = carry;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t o = 0;
        for (int t = 0; t < T; ++t) {
            const int c = tot_s[t];
            soff[t] = o;
            tot_s[t] = int(o);
            o += c;
        }
        soff[T] = o;
    }
    __syncthreads();
    for (long k = threadIdx.x; k < ntiles * T; k += kScanBlock) cnt[k] += tot_s[k % T];
}

__global__ void __launch_bounds__(64)
k_species_scatter(long Na, int T, const int* __restrict__ types, const int* __restrict__ cnt, int* __restrict__ order) {
    const long base = (long)blockIdx.x * kSortTile;
    int run[kMaxTypes];
#pragma unroll
    for (int t = 0; t < kMaxTypes; ++t) run[t] = t < T ? cnt[blockIdx.x * T + t] : 0;
    const unsigned long long below = (1ull << threadIdx.x) - 1ull;
    for (int st = 0; st < kSortTile / 64; ++st) {
        const long i = base + st * 64 + threadIdx.x;
        const int ty = i < Na ? types[i] : -1;
#pragma unroll
        for (int t = 0; t < kMaxTypes; ++t) {
            if (t >= T) break;
            const unsigned long long m = __ballot(ty == t);
            if (ty == t) order[run[t] + __popcll(m & below)] = (int)i;
            run[t] += __popcll(m);
        }
    }
}

// Exclusive scan row[0..Na] of the per-row counts in row[1..Na] (row[0] = 0),
// one block; also sums the angular counts into totals[1] (totals[0] = pairs).

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

// Stable sort of atom indices by species, one block: each of its wavefronts
// owns a contiguous slice of whole 64-atom steps and counts each species with
// ballots; one thread per species then sets where each wavefront's share of
// it starts, and the wavefronts place their atoms in index order (rank among
// the lower lanes of the same species from the same ballots).
__global__ void __launch_bounds__(kScanBlock)
k_species_sort(long Na, int T, const int* __restrict__ types, int* __restrict__ order, int64_t* __restrict__ soff) {
    constexpr int WAVES = kScanBlock / 64;
    __shared__ int cnt_s[WAVES][kMaxTypes];
    __shared__ int base_s[WAVES][kMaxTypes];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const long per = ((Na + WAVES - 1) / WAVES + 63) / 64 * 64;  // whole 64-atom steps per wave
    const long a0 = min(Na, wave * per), a1 = min(Na, a0 + per);
    int c[kMaxTypes];
#pragma unroll
    for (int t = 0; t < kMaxTypes; ++t) c[t] = 0;
    // up to REG steps per wave keep their species in registers for both
    // passes (all loads in flight at once); longer slices reload them
    constexpr int REG = 16;
    const bool held = per <= REG * 64;  // the same for the whole block
    int tr[REG];
    if (held) {
#pragma unroll
        for (int k = 0; k < REG; ++k) {
            const long i = a0 + k * 64 + lane;
            tr[k] = i < a1 ? types[i] : -1;
        }
#pragma unroll
        for (int k = 0; k < REG; ++k) {
            if (a0 + k * 64 >= a1) break;
#pragma unroll
            for (int t = 0; t < kMaxTypes; ++t) {
                if (t >= T) break;
                c[t] += __popcll(__ballot(tr[k] == t));
            }
        }
    } else {
#pragma unroll 4
        for (long i0 = a0; i0 < a1; i0 += 64) {
            const long i = i0 + lane;
            const int ty = i < a1 ? types[i] : -1;
#pragma unroll
            for (int t = 0; t < kMaxTypes; ++t) {
                if (t >= T) break;
                c[t] += __popcll(__ballot(ty == t));
            }
        }
    }
#pragma unroll
    for (int t = 0; t < kMaxTypes; ++t)
        if (lane == t && t < T) cnt_s[wave][t] = c[t];
    __syncthreads();
    // thread t: start of species t, then of each wave's share of it
    if (threadIdx.x < (unsigned)T) {
        const int t = threadIdx.x;
        int64_t o = 0;
        for (int u = 0; u < t; ++u)
            for (int w = 0; w < WAVES; ++w) o += cnt_s[w][u];
        soff[t] = o;
        for (int w = 0; w < WAVES; ++w) {
            base_s[w][t] = int(o);
            o += cnt_s[w][t];
        }
        if (t == T - 1) soff[T] = o;
    }
    __syncthreads();
    int run[kMaxTypes];
#pragma unroll
    for (int t = 0; t < kMaxTypes; ++t) run[t] = t < T ? base_s[wave][t] : 0;
    const unsigned long long below = (1ull << lane) - 1ull;
    if (held) {
#pragma unroll
        for (int k = 0; k < REG; ++k) {
            if (a0 + k * 64 >= a1) break;
            const long i = a0 + k * 64 + lane;
            const int ty = tr[k];
#pragma unroll
            for (int t = 0; t < kMaxTypes; ++t) {
                if (t >= T) break;
                const unsigned long long m = __ballot(ty == t);
                if (ty == t) order[run[t] + __popcll(m & below)] = (int)i;
                run[t] += __popcll(m);
            }
        }
        return;
    }
#pragma unroll 4
    for (long i0 = a0; i0 < a1; i0 += 64) {
        const long i = i0 + lane;
        const int ty = i < a1 ? types[i] : -1;
#pragma unroll
        for (int t = 0; t < kMaxTypes; ++t) {
            if (t >= T) break;
            const unsigned long long m = __ballot(ty == t);
            if (ty == t) order[run[t] + __popcll(m & below)] = (int)i;
            run[t] += __popcll(m);
        }
    }
}

// Per structure s and species t of a batch, the run of s's atoms of species t
// inside species_order: the stable sort keeps them together, in index order,
// since a structure's atoms are one index range. runs[s][t] = {start, end},
// zeroed beforehand so that a species absent from s has an empty run.
// Species are valid here (checked before the launch), so order is a
// permutation of the atoms.
__global__ void __launch_bounds__(kNbBlock)
k_species_runs(long Na, int T, const int* __restrict__ types, const int* __restrict__ atom_struct,
               const int* __restrict__ order, const int64_t* __restrict__ soff, int* __restrict__ runs) {
    const long p = (long)blockIdx.x * kNbBlock + threadIdx.x;
    if (p >= Na) return;
    const int i = order[p], t = types[i], s = atom_struct[i];
    int* r = runs + 2L * s * T + 2 * t;
    if (p == soff[t] || atom_struct[order[p - 1]] != s) r[0] = int(p);
    if (p + 1 == soff[t + 1] || atom_struct[order[p + 1]] != s) r[1] = int(p + 1);
}

// ------------------------------------------------------------- minibatches

// Per selected structure k (one block, chunked scan): atom and pair counts of
// structure ids[k] -> minibatch atom offsets and pair bases; per-structure
// cells and targets. ids outside [0, Ns) select an empty structure.
__global__ void __launch_bounds__(kScanBlock)
k_gather_structs(int n, const int* __restrict__ ids, int Ns, const int64_t* __restrict__ src_off,
                 const int64_t* __restrict__ src_row, const double* __restrict__ src_cells,
                 const double* __restrict__ src_E, const double* __restrict__ src_W, const uint8_t* __restrict__ src_hv,
                 int64_t* __restrict__ dst_off, int64_t* __restrict__ pair_base, double* __restrict__ dst_cells,
                 double* __restrict__ dst_E, double* __restrict__ dst_W, uint8_t* __restrict__ dst_hv, int T,
                 const int* __restrict__ src_runs, int* __restrict__ run_base, int64_t* __restrict__ dst_soff) {
    __shared__ int64_t ba[kScanBlock], bp[kScanBlock];
    __shared__ int64_t carry_a, carry_p;
    if (threadIdx.x == 0) {
        carry_a = carry_p = 0;
        dst_off[0] = 0;
        pair_base[0] = 0;
    }
    __syncthreads();
    for (int base = 0; base < n; base += kScanBlock) {
        const int k = base + threadIdx.x;
        int64_t ca = 0, cp = 0;
        if (k < n) {
            const int sid = ids[k];
            if (sid >= 0 && sid < Ns) {
                ca = src_off[sid + 1] - src_off[sid];
                cp = src_row[src_off[sid + 1]] - src_row[src_off[sid]];
                for (int x = 0; x < 9; ++x) dst_cells[9L * k + x] = src_cells[9L * sid + x];
                if (dst_E && src_E) dst_E[k] = src_E[sid];
                if (dst_W && src_W)
                    for (int x = 0; x < 9; ++x) dst_W[9L * k + x] = src_W[9L * sid + x];
                if (dst_hv) dst_hv[k] = src_hv ? src_hv[sid] : uint8_t(1);
            } else {
                for (int x = 0; x < 9; ++x) dst_cells[9L * k + x] = x % 4 == 0 ? 1.0 : 0.0;
                if (dst_E) dst_E[k] = 0.0;
                if (dst_W)
                    for (int x = 0; x < 9; ++x) dst_W[9L * k + x] = 0.0;
                if (dst_hv) dst_hv[k] = 0;
            }
        }
        ba[threadIdx.x] = ca;
        bp[threadIdx.x] = cp;
        __syncthreads();
        for (int o = 1; o < kScanBlock; o <<= 1) {
            const int64_t ta = (threadIdx.x >= (unsigned)o) ? ba[threadIdx.x - o] : 0;
            const int64_t tp = (threadIdx.x >= (unsigned)o) ? bp[threadIdx.x - o] : 0;
            __syncthreads();
            ba[threadIdx.x] += ta;
            bp[threadIdx.x] += tp;
            __syncthreads();
        }
        const int64_t ia = ba[threadIdx.x] + carry_a, ip = bp[threadIdx.x] + carry_p;
        if (k < n) {
            dst_off[k + 1] = ia;
            pair_base[k + 1] = ip;
        }
        __syncthreads();
        if (threadIdx.x == kScanBlock - 1) {
            carry_a = ia;
            carry_p = ip;
        }
        __syncthreads();
    }
    if (!src_runs) return;
    // With the dataset's species runs: per species t, the exclusive scan over
    // the selected structures of their runs' lengths, run_base[t][k] (and the
    // species total in run_base[t][n]); the species offsets follow.
    constexpr int WAVES = kScanBlock / 64;
    __shared__ int wsum[WAVES];
    __shared__ int carry_t[kMaxTypes];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (threadIdx.x < kMaxTypes) carry_t[threadIdx.x] = 0;
    __syncthreads();
    for (int base = 0; base < n; base += kScanBlock) {
        const int k = base + threadIdx.x;
        int sid = -1;
        if (k < n) {
            const int s = ids[k];
            if (s >= 0 && s < Ns) sid = s;
        }
        for (int t = 0; t < T; ++t) {
            const int c = sid >= 0 ? src_runs[2L * sid * T + 2 * t + 1] - src_runs[2L * sid * T + 2 * t] : 0;
            int x = c;  // inclusive scan over the wavefront
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o, 64);
                if (lane >= o) x += y;
            }
            if (lane == 63) wsum[wave] = x;
            __syncthreads();
            int pre = carry_t[t];
            for (int w = 0; w < wave; ++w) pre += wsum[w];
            if (k < n) run_base[(long)t * (n + 1) + k] = pre + x - c;
            __syncthreads();
            if (threadIdx.x == kScanBlock - 1) carry_t[t] = pre + x;
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        int64_t o = 0;
        for (int t = 0; t < T; ++t) {
            dst_soff[t] = o;
            run_base[(long)t * (n + 1) + n] = carry_t[t];
            o += carry_t[t];
        }
        dst_soff[T] = o;
    }
}

// Per minibatch atom a < min(Na, dst_off[n]): position, species, per-species
// pair counts, force target, structure index and row end.
template <typename R>
__device__ __forceinline__ void gather_atoms_block(
    long blk, long Na, int n, int T, const int* __restrict__ ids, const int64_t* __restrict__ src_off,
    const int64_t* __restrict__ src_row, const R* __restrict__ src_pos, const int* __restrict__ src_types,
    const int* __restrict__ src_seg, const R* __restrict__ src_F, const int64_t* __restrict__ dst_off,
    const int64_t* __restrict__ pair_base, R* __restrict__ dst_pos, int* __restrict__ dst_types,
    int* __restrict__ dst_seg, R* __restrict__ dst_F, int* __restrict__ dst_struct, int64_t* __restrict__ dst_row,
    const int* __restrict__ src_runs, const int* __restrict__ src_order, const int* __restrict__ run_base,
    const int64_t* __restrict__ dst_soff, int* __restrict__ dst_order) {
    const long a = blk * kNbBlock + threadIdx.x;
    if (a == 0) dst_row[0] = 0;
    if (a >= Na || a >= dst_off[n]) return;
    if (src_runs) {
        // entry a of the minibatch's species order: species t and rank r in
        // it, the structure k whose run holds rank r (the last k with
        // run_base[t][k] <= r; run_base[t][n] is the total), then the atom
        // that run holds in the dataset's species order, renumbered
        int t = 0;
        while (t + 1 < T && dst_soff[t + 1] <= a) ++t;
        const int r = int(a - dst_soff[t]);
        const int* __restrict__ bt = run_base + (long)t * (n + 1);
        int lo = 0, hi = n;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (bt[mid] <= r)
                lo = mid;
            else
                hi = mid;
        }
        const int sid = ids[lo];
        const int src_atom = src_order[src_runs[2L * sid * T + 2 * t] + (r - bt[lo])];
        dst_order[a] = int(dst_off[lo] + (src_atom - src_off[sid]));
    }
    int lo = 0, hi = n;  // dst_off[lo] <= a < dst_off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (dst_off[mid] <= a)
            lo = mid;
        else
            hi = mid;
    }
    const int k = lo, sid = ids[k];
    const long sa = src_off[sid] + (a - dst_off[k]);
    for (int x = 0; x < 3; ++x) dst_pos[3 * a + x] = src_pos[3 * sa + x];
    if (dst_F && src_F)
        for (int x = 0; x < 3; ++x) dst_F[3 * a + x] = src_F[3 * sa + x];
    dst_types[a] = src_types[sa];
    for (int x = 0; x < 2 * T; ++x) dst_seg[2L * T * a + x] = src_seg[2L * T * sa + x];
    dst_struct[a] = k;
    dst_row[a + 1] = pair_base[k] + (src_row[sa + 1] - src_row[src_off[sid]]);
}

// Per minibatch pair p < min(P, pair_base[n]): a structure's pairs form one
// contiguous range in the dataset's lists and in the minibatch's, so the pair
// is found by its structure k (pair_base[k] <= p < pair_base[k + 1]) and
// copied with j renumbered and the reverse index moved to the minibatch's
// pair numbering.
template <typename R>
__device__ __forceinline__ void gather_pairs_block(long blk, long P, int n, const int* __restrict__ ids,
                                                   const int64_t* __restrict__ src_off,
                                                   const int64_t* __restrict__ src_row,
                                                   const Rec<R>* __restrict__ src_pairs,
                                                   const int* __restrict__ src_rev, const int64_t* __restrict__ dst_off,
                                                   const int64_t* __restrict__ pair_base, Rec<R>* __restrict__ dst_pairs,
                                                   int* __restrict__ dst_rev) {
    const long lim = min(P, (long)pair_base[n]);
    const long p0 = blk * kNbBlock;
    if (p0 >= lim) return;  // the whole block
    // the block's pairs lie in a short run of structures: two lanes bisect
    // pair_base for its first and last pair, every lane then bisects inside it
    __shared__ int run_s[2];
    if (threadIdx.x < 2) {
        const long key = threadIdx.x == 0 ? p0 : min(p0 + kNbBlock, lim) - 1;
        int lo = 0, hi = n;  // pair_base[lo] <= key < pair_base[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pair_base[mid] <= key)
                lo = mid;
            else
                hi = mid;
        }
        run_s[threadIdx.x] = lo;
    }
    __syncthreads();
    const long p = p0 + threadIdx.x;
    if (p >= lim) return;
    int lo = run_s[0], hi = run_s[1] + 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pair_base[mid] <= p)
            lo = mid;
        else
            hi = mid;
    }
    const int k = lo, sid = ids[k];
    const long s0 = src_row[src_off[sid]];  // the structure's first pair in the dataset
    const long sp = s0 + (p - pair_base[k]);
    Rec<R> r = src_pairs[sp];
    const long j = long(rec_j(r)) - src_off[sid] + dst_off[k];
    if constexpr (sizeof(R) == 4)
        r.w = __int_as_float(int(j));
    else
        r.w = __longlong_as_double((long long)j);
    dst_pairs[p] = r;
    const int rv = src_rev[sp];
    dst_rev[p] = rv < 0 ? -1 : int(rv - s0 + pair_base[k]);
}

// One launch for both copies: blocks below atom_blocks take atoms, the rest
// take pairs (both need only the structure offsets and pair bases).
template <typename R>
__global__ void __launch_bounds__(kNbBlock)
k_gather_atoms_pairs(long atom_blocks, long Na, int n, int T, const int* __restrict__ ids,
                     const int64_t* __restrict__ src_off, const int64_t* __restrict__ src_row,
                     const R* __restrict__ src_pos, const int* __restrict__ src_types, const int* __restrict__ src_seg,
                     const R* __restrict__ src_F, const int64_t* __restrict__ dst_off,
                     const int64_t* __restrict__ pair_base, R* __restrict__ dst_pos, int* __restrict__ dst_types,
                     int* __restrict__ dst_seg, R* __restrict__ dst_F, int* __restrict__ dst_struct,
                     int64_t* __restrict__ dst_row, const int* __restrict__ src_runs, const int* __restrict__ src_order,
                     const int* __restrict__ run_base, const int64_t* __restrict__ dst_soff, int* __restrict__ dst_order,
                     long P, const Rec<R>* __restrict__ src_pairs, const int* __restrict__ src_rev,
                     Rec<R>* __restrict__ dst_pairs, int* __restrict__ dst_rev) {
    const long b = blockIdx.x;
    if (b < atom_blocks)
        gather_atoms_block<R>(b, Na, n, T, ids, src_off, src_row, src_pos, src_types, src_seg, src_F, dst_off,
                              pair_base, dst_pos, dst_types, dst_seg, dst_F, dst_struct, dst_row, src_runs, src_order,
                              run_base, dst_soff, dst_order);
    else
        gather_pairs_block<R>(b - atom_blocks, P, n, ids, src_off, src_row, src_pairs, src_rev, dst_off, pair_base,
                              dst_pairs, dst_rev);
}

nep_status species_sort(long Na, int T, const int* types, int* order, int64_t* soff, int* cnt, hipStream_t st);

template <typename R>
nep_status gather_impl(const Ctx& c, const nep_batch* src, const nep_neighbors* sn, const nep_targets* st_,
                       const int* ids, int n, long Na, int64_t* dst_off, void* dst_pos, int* dst_types,
                       double* dst_cells, nep_neighbors* dn, double* dst_E, void* dst_F, double* dst_W,
                       uint8_t* dst_hv, void* ws, size_t ws_bytes) {
    const int T = c.dm.T;
    hipStream_t st = c.stream;
    // with the dataset's species runs the minibatch's species order is
    // gathered (run_base [T][n+1] after pair_base); without, it is sorted
    const int* runs = sn->species_runs;
    const size_t need = sizeof(int64_t) * (size_t(n) + 1) + (runs ? sizeof(int) * size_t(T) * (size_t(n) + 1) : 0);
    if (ws_bytes < need) return fail(NEP_ERR_WORKSPACE, "workspace holds %zu bytes, the gather needs %zu", ws_bytes, need);
    int64_t* pair_base = static_cast<int64_t*>(ws);
    int* run_base = runs ? reinterpret_cast<int*>(pair_base + n + 1) : nullptr;
    const double* sE = st_ ? st_->energy : nullptr;
    const double* sW = st_ ? st_->virial : nullptr;
    const uint8_t* sH = st_ ? st_->has_virial : nullptr;
    const R* sF = st_ ? static_cast<const R*>(st_->force) : nullptr;
    NEP_LAUNCH("gather_structs", k_gather_structs, dim3(1), dim3(kScanBlock), 0, st, n, ids, src->num_structures,
               src->atom_offset, sn->row_offset, src->cells, sE, sW, sH, dst_off, pair_base, dst_cells, dst_E, dst_W,
               dst_hv, T, runs, run_base, dn->species_offset);
    const long P = dn->capacity;
    const long atom_blocks = Na > 0 ? (Na + kNbBlock - 1) / kNbBlock : 1, pair_blocks = (P + kNbBlock - 1) / kNbBlock;
    NEP_LAUNCH("gather_atoms_pairs", (k_gather_atoms_pairs<R>), dim3(int(atom_blocks + pair_blocks)), dim3(kNbBlock),
               0, st, atom_blocks, Na, n, T, ids, src->atom_offset, sn->row_offset,
               static_cast<const R*>(src->positions), src->types, sn->seg_count, sF, dst_off, pair_base,
               static_cast<R*>(dst_pos), dst_types, dn->seg_count, static_cast<R*>(dst_F), dn->atom_struct,
               dn->row_offset, runs, sn->species_order, run_base, dn->species_offset, dn->species_order, P,
               static_cast<const Rec<R>*>(sn->pairs), sn->reverse, static_cast<Rec<R>*>(dn->pairs), dn->reverse);
    if (runs) return NEP_OK;
    return species_sort(Na, T, dst_types, dn->species_order, dn->species_offset, nullptr, st);
}

template <class F>
nep_status with_max_types(int T, F&& f) {
    if (T <= 4) return f(std::integral_constant<int, 4>{});
    if (T <= 8) return f(std::integral_constant<int, 8>{});
    return f(std::integral_constant<int, kMaxTypes>{});
}

// Exclusive scan of a[1..n] in place (a[0] = 0); tile holds ceil(n / kTile) + 1 values.
nep_status scan_counts(const char* name, long n, int64_t* a, int64_t* tile, hipStream_t st) {
    const long ntiles = (n + kTile - 1) / kTile;
    if (ntiles <= 1) {
        NEP_LAUNCH(name, k_scan_counts, dim3(1), dim3(kScanBlock), 0, st, n, a);
        return NEP_OK;
    }
    NEP_LAUNCH(name, k_tile_sums, dim3(int(ntiles)), dim3(kTileThreads), 0, st, n, (const int64_t*)a, tile, 0,
               (const int*)nullptr, (unsigned long long*)nullptr);
    NEP_LAUNCH(name, k_scan_counts, dim3(1), dim3(kScanBlock), 0, st, ntiles, tile);
    NEP_LAUNCH(name, k_tile_apply, dim3(int(ntiles)), dim3(kTileThreads), 0, st, n, a, (const int64_t*)tile,
               (int64_t*)nullptr);
    return NEP_OK;
}

// Stable species sort; cnt (ceil(Na / kSortTile) * T ints) selects the
// multi-block form, nullptr the one-block form.
nep_status species_sort(long Na, int T, const int* types, int* order, int64_t* soff, int* cnt, hipStream_t st) {
    const long ntiles = (Na + kSortTile - 1) / kSortTile;
    if (!cnt || ntiles <= 16) {
        NEP_LAUNCH("species_sort", k_species_sort, dim3(1), dim3(kScanBlock), 0, st, Na, T, types, order, soff);
        return NEP_OK;
    }
    NEP_LAUNCH("species_sort", k_species_count, dim3(int(ntiles)), dim3(64), 0, st, Na, T, types, cnt);
    NEP_LAUNCH("species_sort", k_species_base, dim3(1), dim3(kScanBlock), 0, st, ntiles, T, cnt, soff);
    NEP_LAUNCH("species_sort", k_species_scatter, dim3(int(ntiles)), dim3(64), 0, st, Na, T, types,
               (const int*)cnt, order);
    return NEP_OK;
}

template <typename R>
nep_status build_neighbors_impl(const Ctx& c, const nep_batch* b, nep_neighbors* nb, void* ws, size_t ws_bytes) {
    const long Na = b->num_atoms;
    const int Ns = b->num_structures, T = c.dm.T;
    if (ws_bytes < sizeof(int64_t) * 3) return fail(NEP_ERR_WORKSPACE, "workspace too small for neighbour totals");
    int64_t* totals = static_cast<int64_t*>(ws);
    hipStream_t st = c.stream;
    const R* pos = static_cast<const R*>(b->positions);
    const int grid = int((Na + kNbBlock - 1) / kNbBlock);
    const int team_grid = int((Na + kNbBlock / kNbTeam - 1) / (kNbBlock / kNbTeam));
    // The offsets, which size the bins below, are checked on the host: they
    // must run 0 .. Na without decreasing. Species are checked on the device
    // (totals[2] flags one outside [0, T), read back with the pair count); every
    // kernel below stays inside its arrays whatever the species, and the call
    // fails before the lists are filled.
    {
        std::vector<int64_t> off(static_cast<size_t>(Ns) + 1);
        NEP_HIP(hipMemcpyAsync(off.data(), b->atom_offset, sizeof(int64_t) * off.size(), hipMemcpyDeviceToHost, st));
        NEP_HIP(hipStreamSynchronize(st));
        if (off[0] != 0 || off[Ns] != Na) return fail(NEP_ERR_INVALID_ARG, "atom_offset must run from 0 to num_atoms");
        for (int s = 0; s < Ns; ++s)
            if (off[s + 1] < off[s]) return fail(NEP_ERR_INVALID_ARG, "atom_offset decreases at structure %d", s);
    }
    NEP_LAUNCH("neighbors_check", k_zero<int64_t>, dim3(1), dim3(kNbBlock), 0, st, 3L, totals);
    if (Na > 0)
        NEP_LAUNCH("neighbors_check", k_check_types, dim3(grid), dim3(kNbBlock), 0, st, Na, T, b->types,
                   reinterpret_cast<unsigned int*>(totals + 2));
    // cell-list scratch in the workspace after the totals
    const long max_bins = Na + Ns;
    size_t o = 64;
    auto carve = [&](size_t bytes) {
        const size_t at = o;
        o += (bytes + 255) / 256 * 256;
        return static_cast<char*>(ws) + at;
    };
    int* sbins = reinterpret_cast<int*>(carve(sizeof(int) * 3 * size_t(Ns)));
    int64_t* bin_base = reinterpret_cast<int64_t*>(carve(sizeof(int64_t) * (size_t(Ns) + 1)));
    int64_t* bin_start = reinterpret_cast<int64_t*>(carve(sizeof(int64_t) * (size_t(max_bins) + 1)));
    unsigned int* cursor = reinterpret_cast<unsigned int*>(carve(sizeof(unsigned int) * size_t(max_bins)));
    int* atom_bin = reinterpret_cast<int*>(carve(sizeof(int) * size_t(Na)));
    BinRec* bin_rec = reinterpret_cast<BinRec*>(carve(sizeof(BinRec) * size_t(Na)));
    int* bin_tmp = reinterpret_cast<int*>(carve(sizeof(int) * size_t(Na)));
    double* wpos = reinterpret_cast<double*>(carve(sizeof(double) * 3 * size_t(Na)));
    int64_t* tile = reinterpret_cast<int64_t*>(carve(sizeof(int64_t) * (size_t(max_bins) / kTile + 2)));
    int* sort_cnt = reinterpret_cast<int*>(carve(sizeof(int) * (size_t(Na) / kSortTile + 1) * size_t(T)));
    if (o > ws_bytes) return fail(NEP_ERR_WORKSPACE, "workspace holds %zu bytes, the neighbour build needs %zu", ws_bytes, o);
    if (Na > 0) {
        const int sgrid = (Ns + kNbBlock - 1) / kNbBlock;
        const int bgrid = int((max_bins + 1 + kNbBlock - 1) / kNbBlock);
        NEP_LAUNCH("cell_setup", k_cell_setup, dim3(sgrid), dim3(kNbBlock), 0, st, Ns, b->atom_offset, b->cells,
                   c.dm.rcR, sbins, bin_base);
        nep_status e;
        if ((e = scan_counts("cell_scan", long(Ns), bin_base, tile, st))) return e;
        NEP_LAUNCH("cell_zero", k_zero<int64_t>, dim3(bgrid), dim3(kNbBlock), 0, st, max_bins + 1, bin_start);
        NEP_LAUNCH("cell_zero", k_zero<unsigned int>, dim3(bgrid), dim3(kNbBlock), 0, st, max_bins, cursor);
        NEP_LAUNCH("cell_bin", (k_bin_atoms<R>), dim3(grid), dim3(kNbBlock), 0, st, Ns, Na, b->atom_offset, pos,
                   b->cells, sbins, bin_base, nb->atom_struct, atom_bin, wpos,
                   reinterpret_cast<unsigned long long*>(bin_start));
        if ((e = scan_counts("cell_scan", max_bins, bin_start, tile, st))) return e;
        NEP_LAUNCH("cell_fill", k_bin_fill, dim3(grid), dim3(kNbBlock), 0, st, Na, atom_bin, bin_start, cursor,
                   bin_tmp);
        NEP_LAUNCH("cell_rank", k_bin_rank, dim3(grid), dim3(kNbBlock), 0, st, Na, atom_bin, bin_start, bin_tmp,
                   (const double*)wpos, b->types, bin_rec);
        nep_status e2 = with_max_types(T, [&](auto mt) -> nep_status {
            NEP_LAUNCH("neighbors_count", (k_neighbors<R, false, decltype(mt)::value>), dim3(team_grid),
                       dim3(kNbBlock), 0, st, Na, T, b->cells, c.dm.rcR, c.dm.rcA, nb->atom_struct,
                       atom_bin, wpos, sbins, bin_base, bin_start, bin_rec, nb->seg_count, nb->row_offset,
                       (Rec<R>*)nullptr);
            return NEP_OK;
        });
        if (e2) return e2;
    }
    if (Na <= kTile) {
        NEP_LAUNCH("neighbors_scan", k_scan_rows, dim3(1), dim3(kScanBlock), 0, st, Na, T, nb->row_offset,
                   nb->seg_count, totals);
    } else {
        // row offsets over many blocks; totals[0] = pairs (the last offset),
        // totals[1] = angular pairs (block sums added atomically, in integers,
        // onto the zero written before the species check)
        const long ntiles = (Na + kTile - 1) / kTile;
        NEP_LAUNCH("neighbors_scan", k_tile_sums, dim3(int(ntiles)), dim3(kTileThreads), 0, st, Na,
                   (const int64_t*)nb->row_offset, tile, T, (const int*)nb->seg_count,
                   reinterpret_cast<unsigned long long*>(totals + 1));
        NEP_LAUNCH("neighbors_scan", k_scan_counts, dim3(1), dim3(kScanBlock), 0, st, ntiles, tile);
        NEP_LAUNCH("neighbors_scan", k_tile_apply, dim3(int(ntiles)), dim3(kTileThreads), 0, st, Na, nb->row_offset,
                   (const int64_t*)tile, totals);
    }
    {
        nep_status e = species_sort(Na, T, b->types, nb->species_order, nb->species_offset, sort_cnt, st);
        if (e) return e;
    }
    int64_t host_tot[3] = {0, 0, 0};
    NEP_HIP(hipMemcpyAsync(host_tot, totals, sizeof(host_tot), hipMemcpyDeviceToHost, st));
    NEP_HIP(hipStreamSynchronize(st));
    if (host_tot[2] != 0) return fail(NEP_ERR_INVALID_ARG, "an atom's species lies outside [0, %d)", T);
    nb->num_pairs = host_tot[0];
    nb->num_angular_pairs = host_tot[1];
    if (host_tot[0] >= (int64_t(1) << 31)) return fail(NEP_ERR_UNSUPPORTED, "more than 2^31-1 pairs in one batch");
    if (host_tot[0] > nb->capacity) {
        return fail(NEP_ERR_CAPACITY, "neighbour capacity too small: need %lld pairs, have %lld",
                    (long long)host_tot[0], (long long)nb->capacity);
    }
    if (nb->species_runs && Ns > 0) {
        const long nr = 2L * Ns * T;
        NEP_LAUNCH("species_runs", k_zero<int>, dim3(int((nr + kNbBlock - 1) / kNbBlock)), dim3(kNbBlock), 0, st, nr,
                   nb->species_runs);
        if (Na > 0)
            NEP_LAUNCH("species_runs", k_species_runs, dim3(grid), dim3(kNbBlock), 0, st, Na, T, b->types,
                       nb->atom_struct, nb->species_order, nb->species_offset, nb->species_runs);
    }
    if (Na > 0 && host_tot[0] > 0) {
        nep_status e2 = with_max_types(T, [&](auto mt) -> nep_status {
            NEP_LAUNCH("neighbors_fill", (k_neighbors<R, true, decltype(mt)::value>), dim3(team_grid),
                       dim3(kNbBlock), 0, st, Na, T, b->cells, c.dm.rcR, c.dm.rcA, nb->atom_struct,
                       atom_bin, wpos, sbins, bin_base, bin_start, bin_rec, nb->seg_count, nb->row_offset,
                       static_cast<Rec<R>*>(nb->pairs));
            return NEP_OK;
        });
        if (e2) return e2;
        const long np = host_tot[0];
        NEP_LAUNCH("neighbors_reverse", k_fill, dim3(int((np + kNbBlock - 1) / kNbBlock)), dim3(kNbBlock), 0, st, np,
                   -1, nb->reverse);
        NEP_LAUNCH("neighbors_reverse", (k_reverse<R>), dim3(int((np + kNbBlock - 1) / kNbBlock)), dim3(kNbBlock), 0,
                   st, Na, np, T, b->types, nb->seg_count, nb->row_offset, static_cast<const Rec<R>*>(nb->pairs),
                   nb->reverse);
    }
    return NEP_OK;
}

}  // namespace

nep_status build_neighbors(const Ctx& c, const nep_batch* b, nep_neighbors* nb, void* ws, size_t ws_bytes) {
    return c.f64 ? build_neighbors_impl<double>(c, b, nb, ws, ws_bytes)
                 : build_neighbors_impl<float>(c, b, nb, ws, ws_bytes);
}

nep_status gather_batch(const Ctx& c, const nep_batch* src, const nep_neighbors* sn, const nep_targets* st,
                        const int* ids, int n, long Na, int64_t* dst_off, void* dst_pos, int* dst_types,
                        double* dst_cells, nep_neighbors* dn, double* dst_E, void* dst_F, double* dst_W,
                        uint8_t* dst_hv, void* ws, size_t ws_bytes) {
    return c.f64 ? gather_impl<double>(c, src, sn, st, ids, n, Na, dst_off, dst_pos, dst_types, dst_cells, dn, dst_E,
                                       dst_F, dst_W, dst_hv, ws, ws_bytes)
                 : gather_impl<float>(c, src, sn, st, ids, n, Na, dst_off, dst_pos, dst_types, dst_cells, dn, dst_E,
                                      dst_F, dst_W, dst_hv, ws, ws_bytes);
}

}  // namespace nep
