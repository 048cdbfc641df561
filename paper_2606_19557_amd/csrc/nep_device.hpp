// Device building blocks of the NEP kernels for gfx950: model dimensions,
// the neighbour-pair record, the Chebyshev basis with cosine cutoff,
// real solid harmonics up to l = 4 evaluated on value / directional-derivative
// / gradient number types, the 4-body algebra on the l = 2 moments, and
// team (sub-wavefront) reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace nep {

// Threads per block of the atom and pair-sweep kernels.
constexpr int kBlock = 256;
// s_waitcnt immediate that waits for vmcnt 0 only (gfx9 encoding: vmcnt in
// bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at their maxima)
constexpr int kWaitVm0 = 0x0F70;

// Runtime model dimensions (host computes, kernels take by value).
struct Dims {
    int T, H, D;
    int NR, NA, KR, KA, L, LM;
    int has4, has5;
    long offA, offN, offB1, P;
    double rcR, rcA;
};

// Compile-time shape of the descriptor; every pair-sweep kernel is
// instantiated for one shape so all per-lane arrays live in registers.
template <int KR_, int KA_, int NR_, int NA_, int L_, int H4_, int H5_>
struct Shape {
    static constexpr int KR = KR_, KA = KA_, NR = NR_, NA = NA_, L = L_;
    static constexpr bool H4 = H4_ != 0, H5 = H5_ != 0;
    static constexpr int LM = (L + 1) * (L + 1) - 1;
    static constexpr int D = NR + NA * (L + (H4 ? 1 : 0) + (H5 ? 1 : 0));
    static_assert(L >= 1 && L <= 4, "solid harmonics are written out for l <= 4");
    static_assert(!H4 || L >= 2, "4-body term needs l = 2 moments");
};

// One neighbour pair: r_ij and the neighbour index j, bit-cast into the 4th slot.
template <typename R>
struct alignas(4 * sizeof(R)) Rec {
    R x, y, z, w;
};

__device__ __forceinline__ int rec_j(const Rec<float>& r) { return __float_as_int(r.w); }
__device__ __forceinline__ int rec_j(const Rec<double>& r) { return (int)__double_as_longlong(r.w); }

template <typename R>
__device__ __forceinline__ R rsqrt_(R x);
template <>
__device__ __forceinline__ float rsqrt_<float>(float x) { return 1.0f / sqrtf(x); }
template <>
__device__ __forceinline__ double rsqrt_<double>(double x) { return 1.0 / sqrt(x); }

template <typename R>
__device__ __forceinline__ void sincospi_(R x, R* s, R* c);
template <>
__device__ __forceinline__ void sincospi_<float>(float x, float* s, float* c) { sincospif(x, s, c); }
template <>
__device__ __forceinline__ void sincospi_<double>(double x, double* s, double* c) { sincospi(x, s, c); }

template <typename R>
__device__ __forceinline__ R tanh_(R x);
template <>
__device__ __forceinline__ float tanh_<float>(float x) { return tanhf(x); }
template <>
__device__ __forceinline__ double tanh_<double>(double x) { return tanh(x); }

// f_k(r) = (T_k(x) + 1)/2 f_c(r) with x = 2(r/rc - 1)^2 - 1 and
// f_c = (cos(pi r/rc) + 1)/2 (Eqs. 17-18); zero at and beyond rc.
// With D set, also f_k'(r), via T'_{k+1} = 2 T_k + 2x T'_k - T'_{k-1}.
template <typename R, int K, bool DERIV>
__device__ __forceinline__ void cheb_basis(R r, R rc, R inv_rc, R* f, R* fp) {
    const R y = r * inv_rc - R(1);
    const R x = R(2) * y * y - R(1);
    R s, c;
    sincospi_<R>(r * inv_rc, &s, &c);
    const bool in = r < rc;
    const R fc = in ? R(0.5) * (c + R(1)) : R(0);
    const R fcp = in ? R(-0.5 * 3.14159265358979323846) * inv_rc * s : R(0);
    const R xp = R(4) * y * inv_rc;
    R t0 = R(1), t1 = x, d0 = R(0), d1 = R(1);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const R tk = (k == 0) ? t0 : t1;
        const R dk = (k == 0) ? d0 : d1;
        f[k] = R(0.5) * (tk + R(1)) * fc;
        if (DERIV) fp[k] = R(0.5) * (dk * xp * fc + (tk + R(1)) * fcp);
        if (k >= 1) {
            const R t2 = R(2) * x * t1 - t0;
            const R d2 = R(2) * t1 + R(2) * x * d1 - d0;
            t0 = t1;
            t1 = t2;
            d0 = d1;
            d1 = d2;
        }
    }
}

// 16-byte vector of R (LDS and global vector loads)
template <typename R>
struct VecOf;
template <>
struct VecOf<float> {
    typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct VecOf<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};

// ---------------------------------------------------------------- number types

// Value and one directional derivative.
template <typename R>
struct D1 {
    R v, d;
};
template <typename R>
__device__ __forceinline__ D1<R> operator+(D1<R> a, D1<R> b) { return {a.v + b.v, a.d + b.d}; }
template <typename R>
__device__ __forceinline__ D1<R> operator-(D1<R> a, D1<R> b) { return {a.v - b.v, a.d - b.d}; }
template <typename R>
__device__ __forceinline__ D1<R> operator*(D1<R> a, D1<R> b) { return {a.v * b.v, a.v * b.d + a.d * b.v}; }
template <typename R>
__device__ __forceinline__ D1<R> operator*(R s, D1<R> a) { return {s * a.v, s * a.d}; }

// Real orthonormal solid harmonics R_lm(x, y, z), homogeneous of degree l,
// equal to Y_lm on the unit sphere; order l = 1..L, m = -l..l.
// N is any number type with +, -, * and scalar multiplication.
template <typename N, typename R, int L>
__device__ __forceinline__ void solid_harmonics(const N& x, const N& y, const N& z, N* Y) {
    constexpr double C1 = 0.4886025119029199;
    constexpr double C2A = 1.0925484305920792, C20 = 0.31539156525252005, C22 = 0.5462742152960396;
    constexpr double C33 = 0.5900435899266435, C32 = 2.890611442640554, C31 = 0.4570457994644658;
    constexpr double C30 = 0.3731763325901154, C32B = 1.445305721320277;
    constexpr double C44 = 2.5033429417967046, C43 = 1.7701307697799304, C42 = 0.9461746957575601;
    constexpr double C41 = 0.6690465435572892, C40 = 0.10578554691520431, C42B = 0.47308734787878004;
    constexpr double C44B = 0.6258357354491761;
    Y[0] = R(C1) * y;
    Y[1] = R(C1) * z;
    Y[2] = R(C1) * x;
    if (L < 2) return;
    const N x2 = x * x, y2 = y * y, z2 = z * z, xy = x * y, xz = x * z, yz = y * z;
    const N x2my2 = x2 - y2, x2py2 = x2 + y2;
    Y[3] = R(C2A) * xy;
    Y[4] = R(C2A) * yz;
    Y[5] = R(C20) * (R(2) * z2 - x2py2);
    Y[6] = R(C2A) * xz;
    Y[7] = R(C22) * x2my2;
    if (L < 3) return;
    const N t3 = R(4) * z2 - x2py2;  // 5z^2 - r^2
    Y[8] = R(C33) * (y * (R(3) * x2 - y2));
    Y[9] = R(C32) * (xy * z);
    Y[10] = R(C31) * (y * t3);
    Y[11] = R(C30) * (z * (R(2) * z2 - R(3) * x2py2));
    Y[12] = R(C31) * (x * t3);
    Y[13] = R(C32B) * (z * x2my2);
    Y[14] = R(C33) * (x * (x2 - R(3) * y2));
    if (L < 4) return;
    const N t42 = R(6) * z2 - x2py2;              // 7z^2 - r^2
    const N t41 = R(4) * z2 - R(3) * x2py2;       // 7z^2 - 3r^2
    const N r2 = x2py2 + z2;
    Y[15] = R(C44) * (xy * x2my2);
    Y[16] = R(C43) * (yz * (R(3) * x2 - y2));
    Y[17] = R(C42) * (xy * t42);
    Y[18] = R(C41) * (yz * t41);
    Y[19] = R(C40) * (R(35) * (z2 * z2) - R(30) * (z2 * r2) + R(3) * (r2 * r2));
    Y[20] = R(C41) * (xz * t41);
    Y[21] = R(C42B) * (x2my2 * t42);
    Y[22] = R(C43) * (xz * (x2 - R(3) * y2));
    Y[23] = R(C44B) * (x2 * (x2 - R(3) * y2) - y2 * (R(3) * x2 - y2));
}

// g = grad_(x,y,z) sum_lm c[lm] R_lm(x, y, z): the gradient of one
// combination of the solid harmonics above, from the partial derivatives of
// their polynomial forms (cheaper than carrying the full gradient through
// every harmonic when only this contraction is needed).
template <typename R, int L>
__device__ __forceinline__ void solid_harmonics_grad(R x, R y, R z, const R* c, R* g) {
    constexpr double C1 = 0.4886025119029199;
    constexpr double C2A = 1.0925484305920792, C20 = 0.31539156525252005, C22 = 0.5462742152960396;
    constexpr double C33 = 0.5900435899266435, C32 = 2.890611442640554, C31 = 0.4570457994644658;
    constexpr double C30 = 0.3731763325901154, C32B = 1.445305721320277;
    constexpr double C44 = 2.5033429417967046, C43 = 1.7701307697799304, C42 = 0.9461746957575601;
    constexpr double C41 = 0.6690465435572892, C40 = 0.10578554691520431, C42B = 0.47308734787878004;
    constexpr double C44B = 0.6258357354491761;
    R gx = R(C1) * c[2], gy = R(C1) * c[0], gz = R(C1) * c[1];
    if (L >= 2) {
        const R a3 = R(C2A) * c[3], a4 = R(C2A) * c[4], a5 = R(C20) * c[5], a6 = R(C2A) * c[6], a7 = R(C22) * c[7];
        gx += a3 * y + a6 * z + R(2) * x * (a7 - a5);
        gy += a3 * x + a4 * z - R(2) * y * (a5 + a7);
        gz += a4 * y + a6 * x + R(4) * z * a5;
    }
    if (L >= 3) {
        const R x2 = x * x, y2 = y * y, z2 = z * z, xy = x * y, xz = x * z, yz = y * z;
        const R a8 = R(C33) * c[8], a9 = R(C32) * c[9], a10 = R(C31) * c[10], a11 = R(C30) * c[11];
        const R a12 = R(C31) * c[12], a13 = R(C32B) * c[13], a14 = R(C33) * c[14];
        const R t3 = R(4) * z2 - x2 - y2;  // 5z^2 - r^2
        gx += R(6) * xy * a8 + yz * a9 - R(2) * xy * a10 - R(6) * xz * a11 + (t3 - R(2) * x2) * a12 +
              R(2) * xz * a13 + R(3) * (x2 - y2) * a14;
        gy += R(3) * (x2 - y2) * a8 + xz * a9 + (t3 - R(2) * y2) * a10 - R(6) * yz * a11 - R(2) * xy * a12 -
              R(2) * yz * a13 - R(6) * xy * a14;
        gz += xy * a9 + R(8) * yz * a10 + R(3) * (R(2) * z2 - x2 - y2) * a11 + R(8) * xz * a12 + (x2 - y2) * a13;
        if (L >= 4) {
            const R a15 = R(C44) * c[15], a16 = R(C43) * c[16], a17 = R(C42) * c[17], a18 = R(C41) * c[18];
            const R a19 = R(C40) * c[19], a20 = R(C41) * c[20], a21 = R(C42B) * c[21], a22 = R(C43) * c[22];
            const R a23 = R(C44B) * c[23];
            const R r2 = x2 + y2 + z2, d = x2 - y2;
            const R t42 = R(6) * z2 - x2 - y2;            // 7z^2 - r^2
            const R t41 = R(4) * z2 - R(3) * (x2 + y2);   // 7z^2 - 3r^2
            const R p19 = R(12) * r2 - R(60) * z2;
            gx += (R(3) * x2 - y2) * y * a15 + R(6) * xy * z * a16 + y * (t42 - R(2) * x2) * a17 - R(6) * xy * z * a18 +
                  x * p19 * a19 + z * (t41 - R(6) * x2) * a20 + R(2) * x * (t42 - d) * a21 +
                  R(3) * d * z * a22 + R(4) * x * (x2 - R(3) * y2) * a23;
            gy += x * (x2 - R(3) * y2) * a15 + R(3) * d * z * a16 + x * (t42 - R(2) * y2) * a17 +
                  z * (t41 - R(6) * y2) * a18 + y * p19 * a19 - R(6) * xy * z * a20 - R(2) * y * (t42 + d) * a21 -
                  R(6) * xy * z * a22 + R(4) * y * (y2 - R(3) * x2) * a23;
            gz += y * (R(3) * x2 - y2) * a16 + R(12) * xy * z * a17 + y * (t41 + R(8) * z2) * a18 +
                  z * (R(80) * z2 - R(48) * r2) * a19 + x * (t41 + R(8) * z2) * a20 + R(12) * d * z * a21 +
                  x * (x2 - R(3) * y2) * a22;
        }
    }
    g[0] = gx;
    g[1] = gy;
    g[2] = gz;
}

template <int LM>
__device__ __forceinline__ constexpr int lm_degree(int lm) {
    return lm < 3 ? 1 : lm < 8 ? 2 : lm < 15 ? 3 : 4;
}

// ------------------------------------------------------------------ 4-body

// Symmetric traceless 3x3 matrix S = sum_j g_j (u_j u_j^T - I/3) rebuilt from
// the real l = 2 moments a[m+2] of the solid harmonics above.
template <typename R>
struct Sym3 {
    R xx, yy, zz, xy, xz, yz;
};

template <typename R>
__device__ __forceinline__ Sym3<R> sym_from_l2(const R* a) {
    constexpr double C2A = 1.0925484305920792, C20 = 0.31539156525252005, C22 = 0.5462742152960396;
    Sym3<R> s;
    s.xy = a[0] * R(1.0 / C2A);
    s.yz = a[1] * R(1.0 / C2A);
    s.zz = a[2] * R(1.0 / (3.0 * C20));
    s.xz = a[3] * R(1.0 / C2A);
    const R d = a[4] * R(1.0 / C22);
    s.xx = R(0.5) * (d - s.zz);
    s.yy = R(0.5) * (-d - s.zz);
    return s;
}

// Adjoint of sym_from_l2: out[m] = <X, dS/da_m> (Frobenius) for symmetric X.
template <typename R>
__device__ __forceinline__ void l2_from_sym_adj(const Sym3<R>& X, R* out) {
    constexpr double C2A = 1.0925484305920792, C20 = 0.31539156525252005, C22 = 0.5462742152960396;
    out[0] = R(2.0 / C2A) * X.xy;
    out[1] = R(2.0 / C2A) * X.yz;
    out[2] = R(1.0 / (3.0 * C20)) * X.zz - R(1.0 / (6.0 * C20)) * (X.xx + X.yy);
    out[3] = R(2.0 / C2A) * X.xz;
    out[4] = R(1.0 / (2.0 * C22)) * (X.xx - X.yy);
}

// A B + B A for symmetric A, B.
template <typename R>
__device__ __forceinline__ Sym3<R> sym_anticomm(const Sym3<R>& A, const Sym3<R>& B) {
    Sym3<R> o;
    o.xx = R(2) * (A.xx * B.xx + A.xy * B.xy + A.xz * B.xz);
    o.yy = R(2) * (A.xy * B.xy + A.yy * B.yy + A.yz * B.yz);
    o.zz = R(2) * (A.xz * B.xz + A.yz * B.yz + A.zz * B.zz);
    o.xy = A.xx * B.xy + A.xy * B.yy + A.xz * B.yz + B.xx * A.xy + B.xy * A.yy + B.xz * A.yz;
    o.xz = A.xx * B.xz + A.xy * B.yz + A.xz * B.zz + B.xx * A.xz + B.xy * A.yz + B.xz * A.zz;
    o.yz = A.xy * B.xz + A.yy * B.yz + A.yz * B.zz + B.xy * A.xz + B.yy * A.yz + B.yz * A.zz;
    return o;
}

template <typename R>
__device__ __forceinline__ R sym_det(const Sym3<R>& s) {
    return s.xx * (s.yy * s.zz - s.yz * s.yz) - s.xy * (s.xy * s.zz - s.yz * s.xz) + s.xz * (s.xy * s.yz - s.yy * s.xz);
}

// kappa such that the (2 2 2) Wigner-3j contraction of the complex l = 2
// moments equals kappa tr(S^3): fixed by one neighbour along z, where the
// contraction is (2 2 2; 0 0 0)(5/4pi)^(3/2) g^3 and tr(S^3) = 2 g^3 / 9.
constexpr double KAPPA4 = -0.26998130975990764;

// q4 = kappa tr(S^3) = 3 kappa det(S) for traceless S.
template <typename R>
__device__ __forceinline__ R q4_value(const R* a) {
    return R(3.0 * KAPPA4) * sym_det(sym_from_l2(a));
}
// dq4/da = 3 kappa M*(S^2).
template <typename R>
__device__ __forceinline__ void q4_grad(const R* a, R* g) {
    const Sym3<R> S = sym_from_l2(a);
    Sym3<R> S2 = sym_anticomm(S, S);  // 2 S^2
    l2_from_sym_adj(S2, g);
#pragma unroll
    for (int m = 0; m < 5; ++m) g[m] *= R(1.5 * KAPPA4);
}
// d(dq4)/da along da: 3 kappa M*(S dS + dS S).
template <typename R>
__device__ __forceinline__ void q4_hess_vec(const R* a, const R* da, R* out) {
    const Sym3<R> S = sym_from_l2(a), dS = sym_from_l2(da);
    l2_from_sym_adj(sym_anticomm(S, dS), out);
#pragma unroll
    for (int m = 0; m < 5; ++m) out[m] *= R(3.0 * KAPPA4);
}

// ------------------------------------------------------------ team reduce

// Sum over the S consecutive lanes of a team (S a power of two <= 64).
// Workgroups are dispatched to the 8 XCDs round-robin by block index, each
// XCD with its own L2. xcd_tile maps block b of an nb-block grid to a tile so
// that every XCD walks one contiguous range of tiles (a bijection on
// [0, nb)): neighbouring atoms, and the pair slots they write for each other,
// then share an L2.
// Constants of one Adam/AMSGrad step t (Eqs. 8-13): bc1 = 1 - beta1^t and
// bc2 = 1 - beta2^t are the bias corrections; mode 0 keeps the running maximum
// of the bias-corrected second moment, mode 1 that of the raw one.
struct AdamArgs {
    double lr, b1, b2, eps, bc1, bc2;
    int amsgrad, mode;
};

constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int per = nb / kXcds, rem = nb % kXcds, x = b % kXcds, k = b / kXcds;
    return x * per + (x < rem ? x : rem) + k;
}

// Lane permutes of the DPP modifier (encodings of the dpp_ctrl field):
// exchange with lane ^ 1 and lane ^ 2 inside each quad, and the mirror of the
// lane inside its half row (8 lanes) and its row (16 lanes).
constexpr int kDppXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;  // lane i <- lane 7 - i in each group of 8
constexpr int kDppMirror = 0x140;      // lane i <- lane 15 - i in each row of 16

template <int CTRL>
__device__ __forceinline__ float dpp_read(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_read(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, int(b), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(unsigned(lo)) | ((long long)hi << 32));
}

// Sum over the S consecutive lanes of a team (S a power of two <= 32), every
// lane getting the same bits: a butterfly whose partner reads are DPP lane
// permutes inside the add (xor 1, xor 2, then the half-row and row mirrors,
// which pair each group with the other half of its next-larger group); only
// the step across 16 lanes of a 32-lane team goes through a cross-lane
// shuffle. Each step adds two equal-rank partial sums, so partners agree.
template <int S, typename R>
__device__ __forceinline__ R team_sum(R v) {
    static_assert(S == 1 || S == 2 || S == 4 || S == 8 || S == 16 || S == 32, "team size");
    if (S >= 2) v += dpp_read<kDppXor1>(v);
    if (S >= 4) v += dpp_read<kDppXor2>(v);
    if (S >= 8) v += dpp_read<kDppHalfMirror>(v);
    if (S >= 16) v += dpp_read<kDppMirror>(v);
    if (S >= 32) v += __shfl_xor(v, 16, 64);
    return v;
}

// --------------------------------------------------------- team exchange

// Per-atom moment accumulation M[n][lm] += sum_pairs u_n(p) Y_lm(p) without
// per-lane copies of all of M: the S lanes of a team each evaluate one pair,
// publish (u, Y) in the team's LDS slots, and every lane then accumulates only
// the harmonics it owns, lm = lane + S*o, over all S pairs of the batch.
template <typename R, int NA, int LM, int S>
struct MomentExchange {
    static constexpr int OWN = (LM + S - 1) / S;
    // Lane slot of NA + LM values padded to 1 (mod 4) elements: the slots of
    // one team and the team blocks of one wave then fall on distinct LDS banks
    // for the stores and for both the broadcast and the per-lane loads.
    static constexpr int SLOT = NA + LM + ((1 - (NA + LM)) % 4 + 4) % 4;
    static constexpr int TEAM_FLOATS = S * SLOT;

    __device__ static void wave_fence() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // acc[n][o] += sum over the team's lanes q of u_q[n] * Y_q[lane + S*o]
    __device__ static void accumulate(R* team_buf, int lane, const R* u, const R* Y, R (&acc)[NA][OWN]) {
        R* mine = team_buf + lane * SLOT;
#pragma unroll
        for (int n = 0; n < NA; ++n) mine[n] = u[n];
#pragma unroll
        for (int lm = 0; lm < LM; ++lm) mine[NA + lm] = Y[lm];
        wave_fence();
        // unrolled by at most 8 pairs: wide teams would otherwise hold the
        // loads of every pair of the batch in registers at once
#pragma unroll 8
        for (int q = 0; q < S; ++q) {
            const R* src = team_buf + q * SLOT;
            R yv[OWN];
#pragma unroll
            for (int o = 0; o < OWN; ++o) {
                const int lm = lane + S * o;
                yv[o] = (lm < LM) ? src[NA + lm] : R(0);
            }
#pragma unroll
            for (int n = 0; n < NA; ++n) {
                const R un = src[n];
#pragma unroll
                for (int o = 0; o < OWN; ++o) acc[n][o] += un * yv[o];
            }
        }
        wave_fence();
    }
};


// ------------------------------------------- row-owned coefficient sweep

// Geometry of the row-owned angular coefficient sweep (k_angular_coeff_grad_rows)
// for a model of T species, N_A angular channels, K_A basis functions and LM
// harmonics in reals of rbytes bytes, `rows` moment rows per lane: S lanes per
// atom, TEAMS atoms per wavefront, each lane's LDS slot of SLOT reals
// (Y[LM], v.dY[LM], f[KAP], (v.r^) f'[KAP], the basis rows padded to whole
// 16-byte vectors), team blocks of TSTRIDE reals (a team stride of 4 words
// modulo 32, so the broadcast reads of different teams spread over the banks),
// and the bytes of one wavefront's LDS: its accumulator G[T][N_A][K_A] for one
// atom species, the slots, and per team the segment table (angular starts
// [T+1], row offsets [T]), and the atom order of the wavefront's current
// group of up to kCgSortTiles tiles. Host and device use the same function.
struct CgRowsGeom {
    int S, teams, vec, kfp, slot, tstride;
    size_t off_slots, off_tab, off_perm, wave_bytes;
};
// Tiles per group whose atoms the row-owned coefficient sweep orders by their
// angular pair counts before cutting them into tiles again.
constexpr int kCgSortTiles = 8;
// Bank-conflict count of one wavefront's 16-byte LDS accesses to the slots:
// lane (team t, lane q) writes its own slot at t*ts + q*slot and every lane
// of team t reads one slot of its team, chunk by chunk (all sizes in 4-byte
// words). Lanes are served `group` at a time by `banks` banks; a group costs
// the largest number of distinct 16-byte addresses that share a bank quad.
__host__ __device__ constexpr int cg_slot_conflicts(int S, int slot_w, int ts_w, int banks, int group) {
    const int teams = 64 / S, quads = banks / 4;
    int cost = 0;
    for (int c = 0; c < slot_w; c += 4)
        for (int g0 = 0; g0 < 64; g0 += group) {
            int wq[16] = {}, rq[16] = {}, last_t = -1;
            for (int l = g0; l < g0 + group && l < teams * S; ++l) {
                const int t = l / S, q = l % S;
                ++wq[((t * ts_w + q * slot_w + c) / 4) % quads];
                if (t != last_t) ++rq[((t * ts_w + c) / 4) % quads];  // one address per team
                last_t = t;
            }
            int mw = 0, mr = 0;
            for (int b = 0; b < quads; ++b) {
                mw = wq[b] > mw ? wq[b] : mw;
                mr = rq[b] > mr ? rq[b] : mr;
            }
            cost += mw + mr;
        }
    return cost;
}
// LDS layout of the row-owned angular coefficient sweep (one region per
// wavefront): G [T][N_A][K_A]; a slot per lane holding one pair's Y [24],
// (v.grad) Y [24], the interleaved (f_k, (v.r^) f'_k) pairs and the pair's
// neighbour-species segment, padded to whole 16-byte vectors; the team stride padded by whole vectors to the
// fewest bank conflicts for 8-lane groups on 32 banks and 16-lane groups on
// 64 banks; then the teams' segment tables. cg_rows_slots fixes the slots
// (no dependence on T: kernels take it as a compile-time constant, the
// search never runs on the device), cg_rows_place the offsets for T species.
__host__ __device__ constexpr CgRowsGeom cg_rows_slots(int NA, int KA, int LM, int rbytes, int rows) {
    CgRowsGeom g{};
    g.S = (NA + rows - 1) / rows;
    g.teams = 64 / g.S;
    g.vec = 16 / rbytes;
    g.kfp = (2 * KA + 1 + g.vec - 1) / g.vec * g.vec;  // f, f' pairs and the pair's segment
    g.slot = 2 * LM + g.kfp;
    const int sw = g.slot * rbytes / 4;
    int best = -1, best_pad = 0;
    for (int pad = 0; pad < 32; pad += 4) {
        const int c = cg_slot_conflicts(g.S, sw, g.S * sw + pad, 32, 8) + cg_slot_conflicts(g.S, sw, g.S * sw + pad, 64, 16);
        if (best < 0 || c < best) {
            best = c;
            best_pad = pad;
        }
    }
    g.tstride = (g.S * sw + best_pad) * 4 / rbytes;
    return g;
}
__host__ __device__ constexpr CgRowsGeom cg_rows_place(CgRowsGeom g, int T, int NA, int KA, int rbytes) {
    const size_t G = size_t(T) * NA * KA * rbytes;
    g.off_slots = (G + 15) / 16 * 16;
    g.off_tab = g.off_slots + size_t(g.teams) * g.tstride * rbytes;
    g.off_perm = (g.off_tab + size_t(g.teams) * (2 * T + 1) * 4 + 15) / 16 * 16;
    g.wave_bytes = (g.off_perm + size_t(kCgSortTiles) * g.teams * 4 + 15) / 16 * 16;
    return g;
}
__host__ __device__ constexpr CgRowsGeom cg_rows_geom(int T, int NA, int KA, int LM, int rbytes, int rows) {
    return cg_rows_place(cg_rows_slots(NA, KA, LM, rbytes, rows), T, NA, KA, rbytes);
}
// Wavefronts per block of that sweep: four, two or one, the most that still
// lets a CU's 160 KB of LDS hold as many wavefronts as single-wavefront blocks
// would (blocks are placed whole).
__host__ __device__ constexpr int cg_rows_waves(size_t wave_bytes) {
    const size_t cu = 160 * 1024, per_cu = cu / wave_bytes;
    return (cu / (4 * wave_bytes)) * 4 == per_cu ? 4 : (cu / (2 * wave_bytes)) * 2 == per_cu ? 2 : 1;
}

// LDS of the force sweep beyond its static blocks of B, for a model of T
// species with N_A angular channels, K_A angular and K_R radial basis
// functions, TEAMS atoms per block and reals of rbytes bytes: c^A[a][b] of
// the block's species a for every neighbour species b (rows of N_A K_A reals
// padded by one 16-byte vector, so that teams at different b read different
// banks), each team's radial force coefficients eps_k[b][K_R] (whole 16-byte
// vectors per team), and each team's segment table (T + 1 int4 entries).
struct ForceLds {
    int cas, eps_team;
    size_t off_eps, off_tab, bytes;
};
__host__ __device__ constexpr ForceLds force_lds(int T, int NA, int KA, int KR, int teams, int rbytes) {
    ForceLds g{};
    const int vec = 16 / rbytes;
    g.cas = (NA * KA + vec - 1) / vec * vec + vec;
    g.eps_team = (T * KR + vec - 1) / vec * vec;
    g.off_eps = size_t(T) * g.cas * rbytes;
    g.off_tab = g.off_eps + size_t(teams) * g.eps_team * rbytes;
    g.bytes = g.off_tab + size_t(teams) * (T + 1) * 16;
    return g;
}

}  // namespace nep
