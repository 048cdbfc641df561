/*
 * Plain FP64 CPU oracle for neuroevolution-potential (NEP) energies, forces,
 * virials, the weighted energy/force/virial loss and its gradient with
 * respect to every model parameter.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, obviously-correct
 * reference that the GPU path is checked against. It shares no code, header,
 * table or constant with the GPU library, and nothing on the product path may
 * call it. Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.
 *
 * What it follows (TorchNEP paper, arXiv 2606.19557):
 *   - site energies, Eq. (1); descriptor scaling, Eq. (2); per-species
 *     one-hidden-layer tanh network with a shared output bias, Eq. (3);
 *   - loss, Eqs. (4)-(7); Adam/AMSGrad lives in adam.py (Eqs. (8)-(13));
 *   - radial descriptor, Eqs. (15)-(16); Chebyshev basis and cosine cutoff,
 *     Eqs. (17)-(18); angular moments with spherical harmonics, Eq. (19);
 *     three-body invariant, Eq. (20); higher-order contractions (Methods,
 *     "NEP descriptors"): 4-body = the (2 2 2) Wigner-3j contraction of the
 *     complex l = 2 moments, 5-body = the square of the l = 1 three-body term.
 *
 * Everything is computed from the definitions in plain loops:
 *   - neighbours by brute force over every atom pair and every periodic image
 *     that can lie within the cutoff (self-images included, only the zero-shift
 *     self pair excluded);
 *   - real orthonormal spherical harmonics from the closed form of the
 *     associated Legendre functions, complex l = 2 harmonics with the
 *     Condon-Shortley phase, Wigner 3j symbols from the Racah formula;
 *   - forces F = -dE/dr by the chain rule, scattered pair by pair;
 *     virial W = -sum_pairs r_ij (x) dE_i/dr_ij;
 *   - the loss gradient by the chain rule: dL/dtheta = sum_s dL/dE_s dE_s/dtheta
 *     + sum_i dL/dF_i . dF_i/dtheta + sum_s dL/dW_s : dW_s/dtheta, where the
 *     force and virial terms are expanded pair by pair into the derivative
 *     of dE_i/dr_ij with respect to each parameter block.
 *
 * Descriptor order: radial n = 0..n_max_r, then for l = 1..l_max and
 * n = 0..n_max_a the three-body q_nl, then the 4-body terms (n = 0..n_max_a),
 * then the 5-body terms. Parameter order: c_R[a][b][n][k], c_A[a][b][n][k],
 * then per species t: W0[t][mu][nu], b0[t][mu], w1[t][mu]; b1 last.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define ORC_KMAX 33
#define ORC_LMAX 8
#define ORC_LM ((ORC_LMAX + 1) * (ORC_LMAX + 1) - 1)
#define ORC_PI 3.14159265358979323846

typedef struct {
    int num_types, n_max_r, n_max_a, basis_r, basis_a;
    int l_max, l_max_4b, l_max_5b, hidden;
    double rc_r, rc_a;
} orc_model;

typedef struct {
    int T, NR, NA, KR, KA, L, has4, has5, H, D, LM;
    long offA, offN, offB1, P;
} dims_t;

static int make_dims(const orc_model* m, dims_t* d) {
    if (m->num_types < 1 || m->n_max_r < 0 || m->n_max_a < 0) return -1;
    if (m->basis_r < 0 || m->basis_a < 0 || m->basis_r + 1 > ORC_KMAX || m->basis_a + 1 > ORC_KMAX) return -1;
    if (m->l_max < 0 || m->l_max > ORC_LMAX || m->hidden < 1) return -1;
    if (m->l_max_4b != 0 && m->l_max_4b != 2) return -1;
    if (m->l_max_5b != 0 && m->l_max_5b != 1) return -1;
    if ((m->l_max_4b && m->l_max < 2) || (m->l_max_5b && m->l_max < 1)) return -1;
    if (!(m->rc_a > 0.0) || !(m->rc_r >= m->rc_a)) return -1;
    d->T = m->num_types;
    d->NR = m->n_max_r + 1;
    d->NA = m->n_max_a + 1;
    d->KR = m->basis_r + 1;
    d->KA = m->basis_a + 1;
    d->L = m->l_max;
    d->has4 = m->l_max_4b == 2;
    d->has5 = m->l_max_5b == 1;
    d->H = m->hidden;
    d->D = d->NR + d->NA * (d->L + d->has4 + d->has5);
    d->LM = (d->L + 1) * (d->L + 1) - 1;
    d->offA = (long)d->T * d->T * d->NR * d->KR;
    d->offN = d->offA + (long)d->T * d->T * d->NA * d->KA;
    d->offB1 = d->offN + (long)d->T * (d->D + 2) * d->H;
    d->P = d->offB1 + 1;
    return 0;
}

int orc_dims(const orc_model* m, long* P, long* D) {
    dims_t d;
    if (make_dims(m, &d)) return -1;
    *P = d.P;
    *D = d.D;
    return 0;
}

/* index helpers */
static inline int lm_index(int l, int m) { return l * l - 1 + (m + l); }
static inline int q3_index(const dims_t* d, int l, int n) { return d->NR + (l - 1) * d->NA + n; }
static inline int q4_index(const dims_t* d, int n) { return d->NR + d->L * d->NA + n; }
static inline int q5_index(const dims_t* d, int n) { return d->NR + (d->L + d->has4) * d->NA + n; }
static inline long cR_index(const dims_t* d, int a, int b, int n, int k) {
    return (((long)a * d->T + b) * d->NR + n) * d->KR + k;
}
static inline long cA_index(const dims_t* d, int a, int b, int n, int k) {
    return d->offA + (((long)a * d->T + b) * d->NA + n) * d->KA + k;
}
static inline long W0_index(const dims_t* d, int t, int mu, int nu) {
    return d->offN + (long)t * (d->D + 2) * d->H + (long)mu * d->D + nu;
}
static inline long b0_index(const dims_t* d, int t, int mu) {
    return d->offN + (long)t * (d->D + 2) * d->H + (long)d->H * d->D + mu;
}
static inline long w1_index(const dims_t* d, int t, int mu) {
    return d->offN + (long)t * (d->D + 2) * d->H + (long)d->H * d->D + d->H + mu;
}

/* ---------------------------------------------------------------- maths */

static double factorial(int n) {
    double r = 1.0;
    for (int i = 2; i <= n; i++) r *= i;
    return r;
}

static double binom(int n, int k) {
    if (k < 0 || k > n) return 0.0;
    return factorial(n) / (factorial(k) * factorial(n - k));
}

/* Eqs. (17)-(18): f_k(r) = (T_k(x) + 1)/2 * f_c(r), x = 2(r/rc - 1)^2 - 1,
 * f_c = (cos(pi r/rc) + 1)/2 for r <= rc and 0 beyond; fp = d f_k / d r.
 * T_k' = k U_{k-1} (Chebyshev polynomials of the second kind). */
static void cheb_basis(double r, double rc, int K, double* f, double* fp) {
    if (r >= rc) {
        for (int k = 0; k < K; k++) f[k] = fp[k] = 0.0;
        return;
    }
    double fc = 0.5 * (cos(ORC_PI * r / rc) + 1.0);
    double fcp = -0.5 * ORC_PI / rc * sin(ORC_PI * r / rc);
    double y = r / rc - 1.0;
    double x = 2.0 * y * y - 1.0;
    double xp = 4.0 * y / rc;
    double T[ORC_KMAX + 1], U[ORC_KMAX + 1];
    T[0] = 1.0;
    T[1] = x;
    U[0] = 1.0;
    U[1] = 2.0 * x;
    for (int k = 1; k < K; k++) {
        T[k + 1] = 2.0 * x * T[k] - T[k - 1];
        U[k + 1] = 2.0 * x * U[k] - U[k - 1];
    }
    for (int k = 0; k < K; k++) {
        double Tp = (k == 0) ? 0.0 : k * U[k - 1];
        f[k] = 0.5 * (T[k] + 1.0) * fc;
        fp[k] = 0.5 * Tp * xp * fc + 0.5 * (T[k] + 1.0) * fcp;
    }
}

/* The z-polynomial of the associated Legendre function on the unit sphere:
 * d^m/dz^m P_l(z) with P_l(z) = 2^-l sum_k (-1)^k C(l,k) C(2l-2k,l) z^(l-2k).
 * Returns value and derivative in z. */
static void legendre_dm(int l, int m, double z, double* val, double* dval) {
    double v = 0.0, dv = 0.0;
    for (int k = 0; 2 * k <= l - m; k++) {
        int p = l - 2 * k - m;
        double c = pow(2.0, -l) * ((k % 2) ? -1.0 : 1.0) * binom(l, k) * binom(2 * l - 2 * k, l) *
                   factorial(l - 2 * k) / factorial(p);
        v += c * pow(z, p);
        if (p > 0) dv += c * p * pow(z, p - 1);
    }
    *val = v;
    *dval = dv;
}

/* w^p for an integer p >= 0 by repeated multiplication (exact at w = 0). */
static double complex ipow(double complex w, int p) {
    double complex r = 1.0;
    for (int i = 0; i < p; i++) r *= w;
    return r;
}

static double sh_norm(int l, int m) {
    return sqrt((2.0 * l + 1.0) / (4.0 * ORC_PI) * factorial(l - m) / factorial(l + m));
}

/* Project the gradient of an extension of Y(u) onto the sphere tangent and
 * divide by r: d Y(r/|r|) / d r = (I - u u^T) grad_u / r. */
static void tangent(const double u[3], double r, const double g[3], double out[3]) {
    double ug = u[0] * g[0] + u[1] * g[1] + u[2] * g[2];
    for (int a = 0; a < 3; a++) out[a] = (g[a] - u[a] * ug) / r;
}

/* Real orthonormal spherical harmonics Y_lm(u) for l = 1..L and their
 * gradients with respect to the bond vector (|r| = r, direction u):
 *   m = 0: N_l0 P_l(z);  m > 0: sqrt2 N_lm Re[(x+iy)^m] P_l^(m)(z);
 *   m < 0: sqrt2 N_l|m| Im[(x+iy)^|m|] P_l^(|m|)(z). */
static void real_sh(int L, const double u[3], double r, double* Y, double (*dY)[3]) {
    double complex w = u[0] + I * u[1];
    for (int l = 1; l <= L; l++) {
        for (int m = 0; m <= l; m++) {
            double Pz, dPz;
            legendre_dm(l, m, u[2], &Pz, &dPz);
            double N = sh_norm(l, m);
            if (m == 0) {
                double g[3] = {0.0, 0.0, N * dPz};
                Y[lm_index(l, 0)] = N * Pz;
                tangent(u, r, g, dY[lm_index(l, 0)]);
            } else {
                double complex wm = ipow(w, m);
                double complex dwm = m * ipow(w, m - 1);
                double s = sqrt(2.0) * N;
                /* d/dx w^m = m w^(m-1), d/dy w^m = i m w^(m-1) */
                double gp[3] = {s * creal(dwm) * Pz, s * creal(I * dwm) * Pz, s * creal(wm) * dPz};
                double gm[3] = {s * cimag(dwm) * Pz, s * cimag(I * dwm) * Pz, s * cimag(wm) * dPz};
                Y[lm_index(l, m)] = s * creal(wm) * Pz;
                Y[lm_index(l, -m)] = s * cimag(wm) * Pz;
                tangent(u, r, gp, dY[lm_index(l, m)]);
                tangent(u, r, gm, dY[lm_index(l, -m)]);
            }
        }
    }
}

/* Complex Y_2^m (Condon-Shortley phase), m = -2..2 stored at m + 2, and the
 * gradients with respect to the bond vector. Y_l^-m = (-1)^m conj(Y_l^m). */
static void complex_sh2(const double u[3], double r, double complex* Y, double complex (*dY)[3]) {
    double complex w = u[0] + I * u[1];
    for (int m = 0; m <= 2; m++) {
        double Pz, dPz;
        legendre_dm(2, m, u[2], &Pz, &dPz);
        double N = ((m % 2) ? -1.0 : 1.0) * sh_norm(2, m);
        double complex wm = ipow(w, m);
        double complex dwm = (m == 0) ? 0.0 : m * ipow(w, m - 1);
        double complex g[3] = {N * dwm * Pz, N * I * dwm * Pz, N * wm * dPz};
        double complex t[3];
        double complex ug = u[0] * g[0] + u[1] * g[1] + u[2] * g[2];
        for (int a = 0; a < 3; a++) t[a] = (g[a] - u[a] * ug) / r;
        Y[m + 2] = N * wm * Pz;
        for (int a = 0; a < 3; a++) dY[m + 2][a] = t[a];
        if (m > 0) {
            double sg = (m % 2) ? -1.0 : 1.0;
            Y[2 - m] = sg * conj(Y[m + 2]);
            for (int a = 0; a < 3; a++) dY[2 - m][a] = sg * conj(t[a]);
        }
    }
}

/* Wigner 3j symbol (j1 j2 j3; m1 m2 m3) for integer arguments, Racah formula. */
double orc_wigner3j(int j1, int j2, int j3, int m1, int m2, int m3) {
    if (m1 + m2 + m3 != 0) return 0.0;
    if (j3 < abs(j1 - j2) || j3 > j1 + j2) return 0.0;
    if (abs(m1) > j1 || abs(m2) > j2 || abs(m3) > j3) return 0.0;
    double tri = factorial(j1 + j2 - j3) * factorial(j1 - j2 + j3) * factorial(-j1 + j2 + j3) /
                 factorial(j1 + j2 + j3 + 1);
    double pre = sqrt(tri * factorial(j1 + m1) * factorial(j1 - m1) * factorial(j2 + m2) * factorial(j2 - m2) *
                      factorial(j3 + m3) * factorial(j3 - m3));
    double sum = 0.0;
    for (int k = 0; k <= j1 + j2 + j3; k++) {
        int a1 = j3 - j2 + k + m1, a2 = j3 - j1 + k - m2, a3 = j1 + j2 - j3 - k, a4 = j1 - k - m1, a5 = j2 - k + m2;
        if (a1 < 0 || a2 < 0 || a3 < 0 || a4 < 0 || a5 < 0) continue;
        double den = factorial(k) * factorial(a1) * factorial(a2) * factorial(a3) * factorial(a4) * factorial(a5);
        sum += ((k % 2) ? -1.0 : 1.0) / den;
    }
    int ph = j1 - j2 - m3;
    return ((ph % 2) ? -1.0 : 1.0) * pre * sum;
}

/* The (2 2 2) coupling tensor C[m1][m2][m3] (indices m + 2). */
static double C222[5][5][5];
static int C222_ready = 0;

static void init_c222(void) {
    if (C222_ready) return;
    for (int a = 0; a < 5; a++)
        for (int b = 0; b < 5; b++)
            for (int c = 0; c < 5; c++) C222[a][b][c] = orc_wigner3j(2, 2, 2, a - 2, b - 2, c - 2);
    C222_ready = 1;
}

/* q4 = sum_{m1 m2 m3} C x_m1 x_m2 x_m3 with its gradient and Hessian in x. */
static void cubic222(const double complex* x, double complex* q, double complex* g, double complex (*h)[5]) {
    double complex v = 0.0;
    for (int a = 0; a < 5; a++)
        for (int b = 0; b < 5; b++)
            for (int c = 0; c < 5; c++) v += C222[a][b][c] * x[a] * x[b] * x[c];
    *q = v;
    for (int m = 0; m < 5; m++) {
        double complex s = 0.0;
        for (int b = 0; b < 5; b++)
            for (int c = 0; c < 5; c++)
                s += (C222[m][b][c] + C222[b][m][c] + C222[b][c][m]) * x[b] * x[c];
        g[m] = s;
    }
    for (int m = 0; m < 5; m++)
        for (int n = 0; n < 5; n++) {
            double complex s = 0.0;
            for (int c = 0; c < 5; c++)
                s += (C222[m][n][c] + C222[m][c][n] + C222[n][m][c] + C222[c][m][n] + C222[n][c][m] + C222[c][n][m]) *
                     x[c];
            h[m][n] = s;
        }
}

/* ------------------------------------------------------------ neighbours */

static int inv3(const double* H, double* Hi) {
    double det = H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                 H[2] * (H[3] * H[7] - H[4] * H[6]);
    if (fabs(det) < 1e-12) return -1;
    Hi[0] = (H[4] * H[8] - H[5] * H[7]) / det;
    Hi[1] = (H[2] * H[7] - H[1] * H[8]) / det;
    Hi[2] = (H[1] * H[5] - H[2] * H[4]) / det;
    Hi[3] = (H[5] * H[6] - H[3] * H[8]) / det;
    Hi[4] = (H[0] * H[8] - H[2] * H[6]) / det;
    Hi[5] = (H[2] * H[3] - H[0] * H[5]) / det;
    Hi[6] = (H[3] * H[7] - H[4] * H[6]) / det;
    Hi[7] = (H[1] * H[6] - H[0] * H[7]) / det;
    Hi[8] = (H[0] * H[4] - H[1] * H[3]) / det;
    return 0;
}

typedef struct {
    int i, j, s[3];
    double r[3];
} raw_pair;

/* Every (i, j, image) with 0 < |r_j + n.H - r_i| < rc. Cell rows a, b, c. */
static long brute_neighbors(int n, const double* cell, const double* pos, double rc, raw_pair** out) {
    double Hi[9];
    if (inv3(cell, Hi)) return -1;
    const double *A = cell, *B = cell + 3, *C = cell + 6;
    double cross[3][3];
    const double* rows[3] = {A, B, C};
    for (int d = 0; d < 3; d++) {
        const double* p = rows[(d + 1) % 3];
        const double* q = rows[(d + 2) % 3];
        cross[d][0] = p[1] * q[2] - p[2] * q[1];
        cross[d][1] = p[2] * q[0] - p[0] * q[2];
        cross[d][2] = p[0] * q[1] - p[1] * q[0];
    }
    double vol = fabs(A[0] * cross[0][0] + A[1] * cross[0][1] + A[2] * cross[0][2]);
    double width[3];
    for (int d = 0; d < 3; d++)
        width[d] = vol / sqrt(cross[d][0] * cross[d][0] + cross[d][1] * cross[d][1] + cross[d][2] * cross[d][2]);
    double* frac = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; i++)
        for (int d = 0; d < 3; d++)
            frac[3 * i + d] = pos[3 * i] * Hi[d] + pos[3 * i + 1] * Hi[3 + d] + pos[3 * i + 2] * Hi[6 + d];
    long cap = 1024, cnt = 0;
    raw_pair* list = (raw_pair*)malloc(sizeof(raw_pair) * cap);
    for (int i = 0; i < n; i++) {
        for (int j = 0; j < n; j++) {
            int lo[3], hi[3];
            for (int d = 0; d < 3; d++) {
                double ds = frac[3 * j + d] - frac[3 * i + d];
                lo[d] = (int)floor(-ds - rc / width[d]);
                hi[d] = (int)ceil(-ds + rc / width[d]);
            }
            for (int a = lo[0]; a <= hi[0]; a++)
                for (int b = lo[1]; b <= hi[1]; b++)
                    for (int c = lo[2]; c <= hi[2]; c++) {
                        if (i == j && a == 0 && b == 0 && c == 0) continue;
                        double r[3];
                        for (int d = 0; d < 3; d++)
                            r[d] = pos[3 * j + d] + a * A[d] + b * B[d] + c * C[d] - pos[3 * i + d];
                        double d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                        if (d2 < rc * rc) {
                            if (cnt == cap) {
                                cap *= 2;
                                list = (raw_pair*)realloc(list, sizeof(raw_pair) * cap);
                            }
                            raw_pair* p = &list[cnt++];
                            p->i = i;
                            p->j = j;
                            p->s[0] = a;
                            p->s[1] = b;
                            p->s[2] = c;
                            p->r[0] = r[0];
                            p->r[1] = r[1];
                            p->r[2] = r[2];
                        }
                    }
        }
    }
    free(frac);
    *out = list;
    return cnt;
}

/* Exported: brute-force neighbour list of one structure. Returns the count;
 * writes min(count, cap) entries when the output pointers are non-NULL. */
long orc_neighbors(int n, const double* cell, const double* pos, double rc, long cap, int* oi, int* oj, int* oshift,
                   double* orv) {
    raw_pair* list = NULL;
    long cnt = brute_neighbors(n, cell, pos, rc, &list);
    if (cnt < 0) return cnt;
    if (oi)
        for (long p = 0; p < cnt && p < cap; p++) {
            oi[p] = list[p].i;
            oj[p] = list[p].j;
            for (int d = 0; d < 3; d++) {
                oshift[3 * p + d] = list[p].s[d];
                orv[3 * p + d] = list[p].r[d];
            }
        }
    free(list);
    return cnt;
}

/* ------------------------------------------------- one atom's environment */

typedef struct {
    int j, tj, ang;
    double r[3], d, u[3];
    double fR[ORC_KMAX], fRp[ORC_KMAX];
    double fA[ORC_KMAX], fAp[ORC_KMAX];
    double Y[ORC_LM], dY[ORC_LM][3];
    double complex Yc[5], dYc[5][3];
} env_pair;

typedef struct {
    int np;
    env_pair* p;
    double* q;      /* [D] */
    double* dq;     /* [np][D][3] */
    double* A;      /* [NA][LM] */
    double complex* Ac; /* [NA][5] */
    double* gR;     /* [np][NR]  g^R_n(r_p) */
    double* gRp;    /* [np][NR]  */
    double* gA;     /* [np][NA]  */
    double* gAp;    /* [np][NA]  */
} atom_env;

/* Build atom i's environment from the structure's pair list [first, last). */
static void build_env(const dims_t* d, const orc_model* m, const double* theta, const int* types, int i,
                      const raw_pair* pl, long first, long last, atom_env* e) {
    int np = (int)(last - first);
    int a = types[i];
    e->np = np;
    e->p = (env_pair*)calloc((size_t)(np > 0 ? np : 1), sizeof(env_pair));
    e->q = (double*)calloc((size_t)d->D, sizeof(double));
    e->dq = (double*)calloc((size_t)(np > 0 ? np : 1) * d->D * 3, sizeof(double));
    e->A = (double*)calloc((size_t)d->NA * (d->LM > 0 ? d->LM : 1), sizeof(double));
    e->Ac = (double complex*)calloc((size_t)d->NA * 5, sizeof(double complex));
    e->gR = (double*)calloc((size_t)(np > 0 ? np : 1) * d->NR, sizeof(double));
    e->gRp = (double*)calloc((size_t)(np > 0 ? np : 1) * d->NR, sizeof(double));
    e->gA = (double*)calloc((size_t)(np > 0 ? np : 1) * d->NA, sizeof(double));
    e->gAp = (double*)calloc((size_t)(np > 0 ? np : 1) * d->NA, sizeof(double));
    for (int k = 0; k < np; k++) {
        const raw_pair* rp = &pl[first + k];
        env_pair* p = &e->p[k];
        p->j = rp->j;
        p->tj = types[rp->j];
        for (int c = 0; c < 3; c++) p->r[c] = rp->r[c];
        p->d = sqrt(p->r[0] * p->r[0] + p->r[1] * p->r[1] + p->r[2] * p->r[2]);
        for (int c = 0; c < 3; c++) p->u[c] = p->r[c] / p->d;
        p->ang = p->d < m->rc_a;
        cheb_basis(p->d, m->rc_r, d->KR, p->fR, p->fRp);
        for (int n = 0; n < d->NR; n++) {
            double g = 0.0, gp = 0.0;
            for (int kk = 0; kk < d->KR; kk++) {
                double c = theta[cR_index(d, a, p->tj, n, kk)];
                g += c * p->fR[kk];
                gp += c * p->fRp[kk];
            }
            e->gR[k * d->NR + n] = g;
            e->gRp[k * d->NR + n] = gp;
        }
        if (p->ang) {
            cheb_basis(p->d, m->rc_a, d->KA, p->fA, p->fAp);
            real_sh(d->L, p->u, p->d, p->Y, p->dY);
            if (d->has4) complex_sh2(p->u, p->d, p->Yc, p->dYc);
            for (int n = 0; n < d->NA; n++) {
                double g = 0.0, gp = 0.0;
                for (int kk = 0; kk < d->KA; kk++) {
                    double c = theta[cA_index(d, a, p->tj, n, kk)];
                    g += c * p->fA[kk];
                    gp += c * p->fAp[kk];
                }
                e->gA[k * d->NA + n] = g;
                e->gAp[k * d->NA + n] = gp;
            }
        }
    }
    /* Eq. (15): radial descriptor */
    for (int k = 0; k < np; k++)
        for (int n = 0; n < d->NR; n++) e->q[n] += e->gR[k * d->NR + n];
    /* Eq. (19): angular moments */
    for (int k = 0; k < np; k++) {
        env_pair* p = &e->p[k];
        if (!p->ang) continue;
        for (int n = 0; n < d->NA; n++) {
            double g = e->gA[k * d->NA + n];
            for (int lm = 0; lm < d->LM; lm++) e->A[n * d->LM + lm] += g * p->Y[lm];
            if (d->has4)
                for (int mm = 0; mm < 5; mm++) e->Ac[n * 5 + mm] += g * p->Yc[mm];
        }
    }
    /* Eq. (20) and the higher-order contractions */
    for (int n = 0; n < d->NA; n++) {
        for (int l = 1; l <= d->L; l++) {
            double s = 0.0;
            for (int mm = -l; mm <= l; mm++) {
                double v = e->A[n * d->LM + lm_index(l, mm)];
                s += v * v;
            }
            e->q[q3_index(d, l, n)] = s;
        }
        if (d->has4) {
            double complex q4, g4[5], h4[5][5];
            cubic222(&e->Ac[n * 5], &q4, g4, h4);
            e->q[q4_index(d, n)] = creal(q4);
        }
        if (d->has5) {
            double P = e->q[q3_index(d, 1, n)];
            e->q[q5_index(d, n)] = P * P;
        }
    }
    /* Jacobian dq/dr_p for every neighbour p of atom i */
    for (int k = 0; k < np; k++) {
        env_pair* p = &e->p[k];
        double* J = &e->dq[(size_t)k * d->D * 3];
        for (int n = 0; n < d->NR; n++)
            for (int c = 0; c < 3; c++) J[n * 3 + c] = e->gRp[k * d->NR + n] * p->u[c];
        if (!p->ang) continue;
        for (int n = 0; n < d->NA; n++) {
            double g = e->gA[k * d->NA + n], gp = e->gAp[k * d->NA + n];
            for (int l = 1; l <= d->L; l++) {
                double acc[3] = {0.0, 0.0, 0.0};
                for (int mm = -l; mm <= l; mm++) {
                    int lm = lm_index(l, mm);
                    double Anlm = e->A[n * d->LM + lm];
                    for (int c = 0; c < 3; c++) acc[c] += 2.0 * Anlm * (gp * p->Y[lm] * p->u[c] + g * p->dY[lm][c]);
                }
                for (int c = 0; c < 3; c++) J[q3_index(d, l, n) * 3 + c] = acc[c];
            }
            if (d->has4) {
                double complex q4, g4[5], h4[5][5];
                cubic222(&e->Ac[n * 5], &q4, g4, h4);
                double complex acc[3] = {0.0, 0.0, 0.0};
                for (int mm = 0; mm < 5; mm++)
                    for (int c = 0; c < 3; c++) acc[c] += g4[mm] * (gp * p->Yc[mm] * p->u[c] + g * p->dYc[mm][c]);
                for (int c = 0; c < 3; c++) J[q4_index(d, n) * 3 + c] = creal(acc[c]);
            }
            if (d->has5) {
                double P = e->q[q3_index(d, 1, n)];
                for (int c = 0; c < 3; c++) J[q5_index(d, n) * 3 + c] = 2.0 * P * J[q3_index(d, 1, n) * 3 + c];
            }
        }
    }
}

static void free_env(atom_env* e) {
    free(e->p);
    free(e->q);
    free(e->dq);
    free(e->A);
    free(e->Ac);
    free(e->gR);
    free(e->gRp);
    free(e->gA);
    free(e->gAp);
}

/* Eqs. (2)-(3): per-species network. Returns E_i; fills t = tanh(a) and
 * e = dE_i/dq. */
static double network(const dims_t* d, const double* theta, const double* qscale, int t, const double* q, double* tv,
                      double* e) {
    double E = -theta[d->offB1];
    for (int nu = 0; nu < d->D; nu++) e[nu] = 0.0;
    for (int mu = 0; mu < d->H; mu++) {
        double a = -theta[b0_index(d, t, mu)];
        for (int nu = 0; nu < d->D; nu++) a += theta[W0_index(d, t, mu, nu)] * qscale[nu] * q[nu];
        double th = tanh(a);
        tv[mu] = th;
        double w1 = theta[w1_index(d, t, mu)];
        E += w1 * th;
        for (int nu = 0; nu < d->D; nu++) e[nu] += w1 * (1.0 - th * th) * theta[W0_index(d, t, mu, nu)] * qscale[nu];
    }
    return E;
}

/* pair list of one structure, sorted by centre atom (brute force order is). */
typedef struct {
    long np;
    raw_pair* list;
    long* first; /* [n+1] */
} struct_pairs;

/* Seconds spent in the brute-force search, summed over threads (timing only:
 * lets a benchmark report the evaluation without the search). */
static double g_search_seconds = 0.0;

double orc_search_seconds(int reset) {
    double v;
#pragma omp critical(orc_search_timer)
    {
        v = g_search_seconds;
        if (reset) g_search_seconds = 0.0;
    }
    return v;
}

static int make_struct_pairs(const orc_model* m, int n, const double* cell, const double* pos, struct_pairs* sp) {
    const double t0 = omp_get_wtime();
    sp->np = brute_neighbors(n, cell, pos, m->rc_r, &sp->list);
    const double dt = omp_get_wtime() - t0;
#pragma omp critical(orc_search_timer)
    g_search_seconds += dt;
    if (sp->np < 0) return -1;
    sp->first = (long*)calloc((size_t)n + 1, sizeof(long));
    for (long p = 0; p < sp->np; p++) sp->first[sp->list[p].i + 1]++;
    for (int i = 0; i < n; i++) sp->first[i + 1] += sp->first[i];
    return 0;
}

static void free_struct_pairs(struct_pairs* sp) {
    free(sp->list);
    free(sp->first);
}

/* ------------------------------------------------------------ exported */

int orc_descriptors(const orc_model* m, const double* theta, int n, const double* cell, const double* pos,
                    const int* types, double* q) {
    dims_t d;
    if (make_dims(m, &d)) return -1;
    init_c222();
    struct_pairs sp;
    if (make_struct_pairs(m, n, cell, pos, &sp)) return -2;
    for (int i = 0; i < n; i++) {
        atom_env e;
        build_env(&d, m, theta, types, i, sp.list, sp.first[i], sp.first[i + 1], &e);
        memcpy(&q[(size_t)i * d.D], e.q, sizeof(double) * d.D);
        free_env(&e);
    }
    free_struct_pairs(&sp);
    return 0;
}

/* Energy (Eq. 1), forces F_k = -dE/dr_k and virial W = -sum r_ij (x) dE_i/dr_ij
 * of one structure. Ei, F, W may be NULL. */
int orc_forward(const orc_model* m, const double* theta, const double* qscale, int n, const double* cell,
                const double* pos, const int* types, double* E, double* Ei, double* F, double* W) {
    dims_t d;
    if (make_dims(m, &d)) return -1;
    init_c222();
    struct_pairs sp;
    if (make_struct_pairs(m, n, cell, pos, &sp)) return -2;
    double* tv = (double*)malloc(sizeof(double) * d.H);
    double* ev = (double*)malloc(sizeof(double) * d.D);
    double Es = 0.0;
    if (F) memset(F, 0, sizeof(double) * 3 * n);
    if (W) memset(W, 0, sizeof(double) * 9);
    for (int i = 0; i < n; i++) {
        atom_env e;
        build_env(&d, m, theta, types, i, sp.list, sp.first[i], sp.first[i + 1], &e);
        double Eat = network(&d, theta, qscale, types[i], e.q, tv, ev);
        if (Ei) Ei[i] = Eat;
        Es += Eat;
        for (int k = 0; k < e.np; k++) {
            const double* J = &e.dq[(size_t)k * d.D * 3];
            double h[3] = {0.0, 0.0, 0.0};
            for (int nu = 0; nu < d.D; nu++)
                for (int c = 0; c < 3; c++) h[c] += ev[nu] * J[nu * 3 + c];
            int j = e.p[k].j;
            if (F)
                for (int c = 0; c < 3; c++) {
                    F[3 * i + c] += h[c];
                    F[3 * j + c] -= h[c];
                }
            if (W)
                for (int al = 0; al < 3; al++)
                    for (int be = 0; be < 3; be++) W[al * 3 + be] -= e.p[k].r[al] * h[be];
        }
        free_env(&e);
    }
    *E = Es;
    free(tv);
    free(ev);
    free_struct_pairs(&sp);
    return 0;
}

/* Vector-Jacobian product of one structure:
 *   grad += ebar dE/dtheta + sum_i ubar_i . dF_i/dtheta + Ubar : dW/dtheta.
 * F_i = sum_j h_ij - sum_{k: i in N(k)} h_ki and W = -sum r_ij (x) h_ij are
 * linear in h_ij = dE_i/dr_ij, so the force and virial terms collect into
 * sum_pairs v_ij . dh_ij/dtheta with v_ij = ubar_i - ubar_j - Ubar^T r_ij.
 * For atom i, sum_j v_ij . dh_ij/dtheta = d/dtheta (e(q_i) . dq_i) where
 * dq_i = sum_j (dq_i/dr_ij) v_ij, and each parameter block is
 * differentiated explicitly below. */
int orc_vjp(const orc_model* m, const double* theta, const double* qscale, int n, const double* cell,
            const double* pos, const int* types, double ebar, const double* ubar, const double* Ubar, double* grad) {
    dims_t d;
    if (make_dims(m, &d)) return -1;
    init_c222();
    struct_pairs sp;
    if (make_struct_pairs(m, n, cell, pos, &sp)) return -2;
    int D = d.D, H = d.H, T = d.T, NA = d.NA, LM = d.LM, KA = d.KA, KR = d.KR, NR = d.NR;
    double* tv = (double*)malloc(sizeof(double) * H);
    double* ev = (double*)malloc(sizeof(double) * D);
    double* dq = (double*)malloc(sizeof(double) * D);
    double* da = (double*)malloc(sizeof(double) * H);
    double* z = (double*)malloc(sizeof(double) * D);
    double* abar = (double*)malloc(sizeof(double) * D);
    double* v = NULL;
    double* dA = (double*)malloc(sizeof(double) * NA * (LM > 0 ? LM : 1));          /* delta A[n][lm] */
    double complex* dAc = (double complex*)malloc(sizeof(double complex) * NA * 5); /* delta A~ [n][m] */
    /* per (b, k): dA/dc and d(deltaA)/dc of the angular moments */
    double* MA = (double*)malloc(sizeof(double) * T * KA * (LM > 0 ? LM : 1));
    double* MdA = (double*)malloc(sizeof(double) * T * KA * (LM > 0 ? LM : 1));
    double complex* MAc = (double complex*)malloc(sizeof(double complex) * T * KA * 5);
    double complex* MdAc = (double complex*)malloc(sizeof(double complex) * T * KA * 5);
    double* SR = (double*)malloc(sizeof(double) * T * KR);  /* sum_p f_k */
    double* SdR = (double*)malloc(sizeof(double) * T * KR); /* sum_p v.u f_k' */

    for (int i = 0; i < n; i++) {
        atom_env e;
        build_env(&d, m, theta, types, i, sp.list, sp.first[i], sp.first[i + 1], &e);
        int a = types[i];
        network(&d, theta, qscale, a, e.q, tv, ev);
        v = (double*)realloc(v, sizeof(double) * 3 * (e.np > 0 ? e.np : 1));
        for (int k = 0; k < e.np; k++) {
            int j = e.p[k].j;
            for (int be = 0; be < 3; be++) {
                double s = ubar[3 * i + be] - ubar[3 * j + be];
                for (int al = 0; al < 3; al++) s -= Ubar[al * 3 + be] * e.p[k].r[al];
                v[3 * k + be] = s;
            }
        }
        /* tangent of the descriptor along v */
        for (int nu = 0; nu < D; nu++) {
            double s = 0.0;
            for (int k = 0; k < e.np; k++)
                for (int c = 0; c < 3; c++) s += e.dq[((size_t)k * D + nu) * 3 + c] * v[3 * k + c];
            dq[nu] = s;
        }
        /* network parameters: d/dtheta [ebar E_i + e(q) . dq] */
        for (int mu = 0; mu < H; mu++) {
            double s = 0.0;
            for (int nu = 0; nu < D; nu++) s += theta[W0_index(&d, a, mu, nu)] * qscale[nu] * dq[nu];
            da[mu] = s;
        }
        for (int nu = 0; nu < D; nu++) z[nu] = 0.0;
        for (int mu = 0; mu < H; mu++) {
            double th = tv[mu], sp1 = 1.0 - th * th, w1 = theta[w1_index(&d, a, mu)];
            grad[w1_index(&d, a, mu)] += ebar * th + sp1 * da[mu];
            grad[b0_index(&d, a, mu)] += -ebar * w1 * sp1 + 2.0 * w1 * th * sp1 * da[mu];
            for (int nu = 0; nu < D; nu++) {
                double sq = qscale[nu] * e.q[nu], sd = qscale[nu] * dq[nu];
                grad[W0_index(&d, a, mu, nu)] += ebar * w1 * sp1 * sq + w1 * sp1 * sd - 2.0 * w1 * th * sp1 * da[mu] * sq;
                z[nu] += -2.0 * w1 * th * sp1 * da[mu] * theta[W0_index(&d, a, mu, nu)] * qscale[nu];
            }
        }
        grad[d.offB1] += -ebar;
        /* descriptor coefficients: dL/dc = abar . dq/dc + e . d(dq)/dc */
        for (int nu = 0; nu < D; nu++) abar[nu] = ebar * ev[nu] + z[nu];

        /* radial block: q_n = sum_p sum_k c^{ab}_nk f_k, dq_n = sum_p sum_k c^{ab}_nk f_k' (u.v) */
        memset(SR, 0, sizeof(double) * T * KR);
        memset(SdR, 0, sizeof(double) * T * KR);
        for (int k = 0; k < e.np; k++) {
            env_pair* p = &e.p[k];
            double uv = p->u[0] * v[3 * k] + p->u[1] * v[3 * k + 1] + p->u[2] * v[3 * k + 2];
            for (int kk = 0; kk < KR; kk++) {
                SR[p->tj * KR + kk] += p->fR[kk];
                SdR[p->tj * KR + kk] += p->fRp[kk] * uv;
            }
        }
        for (int b = 0; b < T; b++)
            for (int nn = 0; nn < NR; nn++)
                for (int kk = 0; kk < KR; kk++)
                    grad[cR_index(&d, a, b, nn, kk)] += abar[nn] * SR[b * KR + kk] + ev[nn] * SdR[b * KR + kk];

        /* angular block */
        if (NA > 0 && (LM > 0)) {
            memset(dA, 0, sizeof(double) * NA * LM);
            memset(dAc, 0, sizeof(double complex) * NA * 5);
            memset(MA, 0, sizeof(double) * T * KA * LM);
            memset(MdA, 0, sizeof(double) * T * KA * LM);
            memset(MAc, 0, sizeof(double complex) * T * KA * 5);
            memset(MdAc, 0, sizeof(double complex) * T * KA * 5);
            for (int k = 0; k < e.np; k++) {
                env_pair* p = &e.p[k];
                if (!p->ang) continue;
                double uv = p->u[0] * v[3 * k] + p->u[1] * v[3 * k + 1] + p->u[2] * v[3 * k + 2];
                for (int lm = 0; lm < LM; lm++) {
                    double dYv = p->dY[lm][0] * v[3 * k] + p->dY[lm][1] * v[3 * k + 1] + p->dY[lm][2] * v[3 * k + 2];
                    for (int nn = 0; nn < NA; nn++)
                        dA[nn * LM + lm] += e.gAp[k * NA + nn] * p->Y[lm] * uv + e.gA[k * NA + nn] * dYv;
                    for (int kk = 0; kk < KA; kk++) {
                        MA[(p->tj * KA + kk) * LM + lm] += p->fA[kk] * p->Y[lm];
                        MdA[(p->tj * KA + kk) * LM + lm] += p->fAp[kk] * p->Y[lm] * uv + p->fA[kk] * dYv;
                    }
                }
                if (d.has4)
                    for (int mm = 0; mm < 5; mm++) {
                        double complex dYv = p->dYc[mm][0] * v[3 * k] + p->dYc[mm][1] * v[3 * k + 1] +
                                             p->dYc[mm][2] * v[3 * k + 2];
                        for (int nn = 0; nn < NA; nn++)
                            dAc[nn * 5 + mm] += e.gAp[k * NA + nn] * p->Yc[mm] * uv + e.gA[k * NA + nn] * dYv;
                        for (int kk = 0; kk < KA; kk++) {
                            MAc[(p->tj * KA + kk) * 5 + mm] += p->fA[kk] * p->Yc[mm];
                            MdAc[(p->tj * KA + kk) * 5 + mm] += p->fAp[kk] * p->Yc[mm] * uv + p->fA[kk] * dYv;
                        }
                    }
            }
            for (int b = 0; b < T; b++)
                for (int nn = 0; nn < NA; nn++)
                    for (int kk = 0; kk < KA; kk++) {
                        const double* mA = &MA[(b * KA + kk) * LM];
                        const double* mdA = &MdA[(b * KA + kk) * LM];
                        const double* An = &e.A[nn * LM];
                        const double* dAn = &dA[nn * LM];
                        double gsum = 0.0;
                        double dq1 = 0.0, ddq1 = 0.0; /* l = 1 pieces for the 5-body term */
                        for (int l = 1; l <= d.L; l++) {
                            double dqc = 0.0, ddqc = 0.0;
                            for (int mm = -l; mm <= l; mm++) {
                                int lm = lm_index(l, mm);
                                dqc += 2.0 * An[lm] * mA[lm];
                                ddqc += 2.0 * (mA[lm] * dAn[lm] + An[lm] * mdA[lm]);
                            }
                            int nu = q3_index(&d, l, nn);
                            gsum += abar[nu] * dqc + ev[nu] * ddqc;
                            if (l == 1) {
                                dq1 = dqc;
                                ddq1 = ddqc;
                            }
                        }
                        if (d.has4) {
                            double complex q4, g4[5], h4[5][5];
                            cubic222(&e.Ac[nn * 5], &q4, g4, h4);
                            const double complex* mAc = &MAc[(b * KA + kk) * 5];
                            const double complex* mdAc = &MdAc[(b * KA + kk) * 5];
                            double complex dqc = 0.0, ddqc = 0.0;
                            for (int mm = 0; mm < 5; mm++) {
                                dqc += g4[mm] * mAc[mm];
                                double complex hd = 0.0;
                                for (int m2 = 0; m2 < 5; m2++) hd += h4[mm][m2] * mAc[m2];
                                ddqc += hd * dAc[nn * 5 + mm] + g4[mm] * mdAc[mm];
                            }
                            int nu = q4_index(&d, nn);
                            gsum += abar[nu] * creal(dqc) + ev[nu] * creal(ddqc);
                        }
                        if (d.has5) {
                            double P = e.q[q3_index(&d, 1, nn)];
                            double dP = dq[q3_index(&d, 1, nn)];
                            int nu = q5_index(&d, nn);
                            gsum += abar[nu] * 2.0 * P * dq1 + ev[nu] * (2.0 * dq1 * dP + 2.0 * P * ddq1);
                        }
                        grad[cA_index(&d, a, b, nn, kk)] += gsum;
                    }
        }
        free_env(&e);
    }
    free(tv);
    free(ev);
    free(dq);
    free(da);
    free(z);
    free(abar);
    free(v);
    free(dA);
    free(dAc);
    free(MA);
    free(MdA);
    free(MAc);
    free(MdAc);
    free(SR);
    free(SdR);
    free_struct_pairs(&sp);
    return 0;
}

/* Eqs. (4)-(7) over a batch, then the gradient. N_s, N_a and N_a^s are taken
 * over the batch; Delta_V averages over the structures that carry a virial
 * label (has_virial may be NULL = all). loss[4] = {L, Delta_E, Delta_F,
 * Delta_V}. E_out, F_out, W_out and grad may be NULL. */
int orc_batch_loss_grad(const orc_model* m, const double* theta, const double* qscale, int Ns, const long* off,
                        const double* cells, const double* pos, const int* types, const double* Et, const double* Ft,
                        const double* Wt, const unsigned char* has_virial, double lam_e, double lam_f, double lam_v,
                        double* E_out, double* F_out, double* W_out, double* loss, double* grad, int nthreads) {
    dims_t d;
    if (make_dims(m, &d)) return -1;
    init_c222();
    long Na = off[Ns];
    double* E = (double*)malloc(sizeof(double) * (Ns > 0 ? Ns : 1));
    double* F = (double*)malloc(sizeof(double) * 3 * (Na > 0 ? Na : 1));
    double* W = (double*)malloc(sizeof(double) * 9 * (Ns > 0 ? Ns : 1));
    int err = 0;
#pragma omp parallel for schedule(dynamic) num_threads(nthreads) reduction(| : err)
    for (int s = 0; s < Ns; s++) {
        int n = (int)(off[s + 1] - off[s]);
        err |= orc_forward(m, theta, qscale, n, &cells[9 * s], &pos[3 * off[s]], &types[off[s]], &E[s], NULL,
                           &F[3 * off[s]], &W[9 * s]) != 0;
    }
    if (err) {
        free(E);
        free(F);
        free(W);
        return -2;
    }
    /* Eqs. 4-7 average per-atom residuals over the batch's structures; a
     * structure without atoms has no per-atom residual (N_a^s = 0) and is not
     * counted in N_s, nor in the number N_v of labelled structures. */
    int Nv = 0, Nsa = 0;
    for (int s = 0; s < Ns; s++) {
        if (off[s + 1] == off[s]) continue;
        Nsa++;
        Nv += has_virial ? (has_virial[s] != 0) : 1;
    }
    double dE = 0.0, dF = 0.0, dV = 0.0;
    double* ebar = (double*)malloc(sizeof(double) * (Ns > 0 ? Ns : 1));
    double* ub = (double*)malloc(sizeof(double) * 3 * (Na > 0 ? Na : 1));
    double* Ub = (double*)malloc(sizeof(double) * 9 * (Ns > 0 ? Ns : 1));
    for (int s = 0; s < Ns; s++) {
        double na = (double)(off[s + 1] - off[s]);
        if (na == 0.0) {
            ebar[s] = 0.0;
            for (int c = 0; c < 9; c++) Ub[9 * s + c] = 0.0;
            continue;
        }
        double r = (E[s] - Et[s]) / na;
        dE += r * r / Nsa;
        ebar[s] = lam_e * 2.0 * (E[s] - Et[s]) / (Nsa * na * na);
        int hv = has_virial ? (has_virial[s] != 0) : 1;
        for (int c = 0; c < 9; c++) {
            double rw = (W[9 * s + c] - Wt[9 * s + c]) / na;
            if (hv && Nv > 0) {
                dV += rw * rw / (9.0 * Nv);
                Ub[9 * s + c] = lam_v * 2.0 * (W[9 * s + c] - Wt[9 * s + c]) / (9.0 * Nv * na * na);
            } else {
                Ub[9 * s + c] = 0.0;
            }
        }
    }
    for (long i = 0; i < 3 * Na; i++) {
        double r = F[i] - Ft[i];
        dF += r * r / (3.0 * Na);
        ub[i] = lam_f * 2.0 * r / (3.0 * Na);
    }
    loss[1] = dE;
    loss[2] = dF;
    loss[3] = dV;
    loss[0] = lam_e * dE + lam_f * dF + lam_v * dV;
    if (E_out) memcpy(E_out, E, sizeof(double) * Ns);
    if (F_out) memcpy(F_out, F, sizeof(double) * 3 * Na);
    if (W_out) memcpy(W_out, W, sizeof(double) * 9 * Ns);
    if (grad) {
        double* gs = (double*)calloc((size_t)(Ns > 0 ? Ns : 1) * d.P, sizeof(double));
#pragma omp parallel for schedule(dynamic) num_threads(nthreads) reduction(| : err)
        for (int s = 0; s < Ns; s++) {
            int n = (int)(off[s + 1] - off[s]);
            err |= orc_vjp(m, theta, qscale, n, &cells[9 * s], &pos[3 * off[s]], &types[off[s]], ebar[s],
                           &ub[3 * off[s]], &Ub[9 * s], &gs[(size_t)s * d.P]) != 0;
        }
        for (long p = 0; p < d.P; p++) {
            double acc = 0.0;
            for (int s = 0; s < Ns; s++) acc += gs[(size_t)s * d.P + p];
            grad[p] = acc;
        }
        free(gs);
    }
    free(E);
    free(F);
    free(W);
    free(ebar);
    free(ub);
    free(Ub);
    return err ? -2 : 0;
}

/* Real orthonormal Y_lm and gradients of one bond vector (for pins). */
int orc_real_sh(int L, const double* rv, double* Y, double* dY) {
    if (L < 1 || L > ORC_LMAX) return -1;
    double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
    double u[3] = {rv[0] / r, rv[1] / r, rv[2] / r};
    double Yl[ORC_LM], dYl[ORC_LM][3];
    real_sh(L, u, r, Yl, dYl);
    int LM = (L + 1) * (L + 1) - 1;
    for (int i = 0; i < LM; i++) {
        Y[i] = Yl[i];
        for (int c = 0; c < 3; c++) dY[3 * i + c] = dYl[i][c];
    }
    return 0;
}

/* Chebyshev basis values and derivatives at one distance (for pins). */
int orc_basis(double r, double rc, int K, double* f, double* fp) {
    if (K < 1 || K > ORC_KMAX) return -1;
    cheb_basis(r, rc, K, f, fp);
    return 0;
}

/* The 4-body invariant of one set of complex l=2 moments, as re, im. */
int orc_q4_of_moments(const double* re, const double* im, double* out) {
    init_c222();
    double complex x[5], q, g[5], h[5][5];
    for (int mm = 0; mm < 5; mm++) x[mm] = re[mm] + I * im[mm];
    cubic222(x, &q, g, h);
    out[0] = creal(q);
    out[1] = cimag(q);
    return 0;
}

/* Complex l=2 spherical harmonics at a direction, as re/im pairs (for pins). */
int orc_complex_sh2(const double* rv, double* re, double* im) {
    double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
    double u[3] = {rv[0] / r, rv[1] / r, rv[2] / r};
    double complex Y[5], dY[5][3];
    complex_sh2(u, r, Y, dY);
    for (int mm = 0; mm < 5; mm++) {
        re[mm] = creal(Y[mm]);
        im[mm] = cimag(Y[mm]);
    }
    return 0;
}
