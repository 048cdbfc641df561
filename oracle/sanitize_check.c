/*
 * Memory and undefined-behaviour check of the oracle (test infrastructure):
 * built together with nep_oracle.c under -fsanitize=address,undefined by the
 * CPU test suite, it runs every exported oracle routine on small periodic
 * cells -- one cell thinner than twice the cutoff (many images), a one-atom
 * cell, an empty structure, three species with the 4-body and 5-body terms --
 * and exits 0 when the sanitizers report nothing (they abort otherwise).
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int num_types, n_max_r, n_max_a, basis_r, basis_a;
    int l_max, l_max_4b, l_max_5b, hidden;
    double rc_r, rc_a;
} orc_model;

int orc_dims(const orc_model* m, long* P, long* D);
double orc_wigner3j(int j1, int j2, int j3, int m1, int m2, int m3);
long orc_neighbors(int n, const double* cell, const double* pos, double rc, long cap, int* oi, int* oj, int* oshift,
                   double* orv);
int orc_descriptors(const orc_model* m, const double* theta, int n, const double* cell, const double* pos,
                    const int* types, double* q);
int orc_forward(const orc_model* m, const double* theta, const double* qscale, int n, const double* cell,
                const double* pos, const int* types, double* E, double* Ei, double* F, double* W);
int orc_vjp(const orc_model* m, const double* theta, const double* qscale, int n, const double* cell,
            const double* pos, const int* types, double ebar, const double* ubar, const double* Ubar, double* grad);
int orc_batch_loss_grad(const orc_model* m, const double* theta, const double* qscale, int Ns, const long* off,
                        const double* cells, const double* pos, const int* types, const double* Et, const double* Ft,
                        const double* Wt, const unsigned char* has_virial, double lam_e, double lam_f, double lam_v,
                        double* E_out, double* F_out, double* W_out, double* loss, double* grad, int nthreads);
int orc_real_sh(int L, const double* rv, double* Y, double* dY);
int orc_basis(double r, double rc, int K, double* f, double* fp);
int orc_q4_of_moments(const double* re, const double* im, double* out);
int orc_complex_sh2(const double* rv, double* re, double* im);
double orc_search_seconds(int reset);

static unsigned long long g_state = 88172645463325252ULL;
static double urand(void) { /* xorshift64, uniform in [0, 1) */
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (double)(g_state >> 11) / 9007199254740992.0;
}

#define CHECK(x)                                                        \
    do {                                                                \
        if (!(x)) {                                                     \
            fprintf(stderr, "sanitize_check: %s failed (line %d)\n", #x, __LINE__); \
            return 1;                                                   \
        }                                                               \
    } while (0)

int main(void) {
    const orc_model m = {3, 3, 3, 5, 4, 4, 2, 1, 7, 4.5, 3.8};
    long P = 0, D = 0;
    CHECK(orc_dims(&m, &P, &D) == 0);
    /* structures: a 2x2x1 bcc cell (thin along c), one atom, empty, a 9-atom cell */
    enum { NS = 4 };
    const int counts[NS] = {8, 1, 0, 9};
    long off[NS + 1] = {0};
    for (int s = 0; s < NS; s++) off[s + 1] = off[s] + counts[s];
    const int Na = (int)off[NS];
    double cells[NS * 9] = {0};
    const double edge[NS][3] = {{6.4, 6.4, 3.2}, {3.0, 3.1, 3.3}, {7.0, 7.0, 7.0}, {6.0, 6.2, 5.8}};
    for (int s = 0; s < NS; s++)
        for (int d = 0; d < 3; d++) cells[9 * s + 4 * d] = edge[s][d];
    cells[9 * 0 + 3] = 0.3; /* a sheared cell */
    double* pos = malloc(sizeof(double) * 3 * Na);
    int* types = malloc(sizeof(int) * Na);
    for (int s = 0; s < NS; s++)
        for (long i = off[s]; i < off[s + 1]; i++) {
            for (int d = 0; d < 3; d++) pos[3 * i + d] = urand() * edge[s][d];
            types[i] = (int)(urand() * 3.0) % 3;
        }
    double* theta = malloc(sizeof(double) * P);
    for (long p = 0; p < P; p++) theta[p] = 0.2 * (urand() - 0.5);
    double* qs = malloc(sizeof(double) * D);
    for (long d = 0; d < D; d++) qs[d] = 0.5 + urand();
    double* q = malloc(sizeof(double) * D * (Na > 0 ? Na : 1));
    double* F = malloc(sizeof(double) * 3 * Na);
    double* Ei = malloc(sizeof(double) * Na);
    double* grad = calloc((size_t)P, sizeof(double));
    double E, W[9];
    for (int s = 0; s < NS; s++) {
        const int n = counts[s];
        const double* c = &cells[9 * s];
        const double* x = &pos[3 * off[s]];
        const int* t = &types[off[s]];
        long cnt = orc_neighbors(n, c, x, m.rc_r, 0, NULL, NULL, NULL, NULL);
        CHECK(cnt >= 0);
        int* oi = malloc(sizeof(int) * (cnt + 1));
        int* oj = malloc(sizeof(int) * (cnt + 1));
        int* sh = malloc(sizeof(int) * 3 * (cnt + 1));
        double* rv = malloc(sizeof(double) * 3 * (cnt + 1));
        CHECK(orc_neighbors(n, c, x, m.rc_r, cnt, oi, oj, sh, rv) == cnt);
        free(oi);
        free(oj);
        free(sh);
        free(rv);
        CHECK(orc_descriptors(&m, theta, n, c, x, t, q) == 0);
        CHECK(orc_forward(&m, theta, qs, n, c, x, t, &E, Ei, F, W) == 0);
        CHECK(orc_forward(&m, theta, qs, n, c, x, t, &E, NULL, NULL, NULL) == 0);
        double ub[3 * 16], Ub[9];
        for (int k = 0; k < 3 * n; k++) ub[k] = urand() - 0.5;
        for (int k = 0; k < 9; k++) Ub[k] = urand() - 0.5;
        CHECK(orc_vjp(&m, theta, qs, n, c, x, t, 0.3, ub, Ub, grad) == 0);
    }
    double* Ft = malloc(sizeof(double) * 3 * Na);
    for (int k = 0; k < 3 * Na; k++) Ft[k] = urand() - 0.5;
    double Et[NS], Wt[NS * 9];
    for (int s = 0; s < NS; s++) Et[s] = urand() - 0.5;
    for (int k = 0; k < NS * 9; k++) Wt[k] = urand() - 0.5;
    unsigned char hv[NS] = {1, 0, 1, 1};
    double Eo[NS], Wo[NS * 9], loss[4];
    for (int threads = 1; threads <= 2; threads++) {
        CHECK(orc_batch_loss_grad(&m, theta, qs, NS, off, cells, pos, types, Et, Ft, Wt, hv, 1.0, 1.0, 0.1, Eo, F, Wo,
                                  loss, grad, threads) == 0);
        CHECK(isfinite(loss[0]));
        CHECK(orc_batch_loss_grad(&m, theta, qs, NS, off, cells, pos, types, Et, Ft, Wt, NULL, 1.0, 1.0, 0.1, NULL,
                                  NULL, NULL, loss, NULL, threads) == 0);
    }
    double Y[80], dY[240], f[33], fp[33], re[5], im[5], out[2];
    const double r3[3] = {0.3, -1.2, 0.7};
    for (int L = 1; L <= 8; L++) CHECK(orc_real_sh(L, r3, Y, dY) == 0);
    CHECK(orc_basis(2.0, 4.5, 33, f, fp) == 0);
    CHECK(orc_complex_sh2(r3, re, im) == 0);
    CHECK(orc_q4_of_moments(re, im, out) == 0);
    CHECK(fabs(orc_wigner3j(2, 2, 2, 0, 0, 0) + sqrt(2.0 / 35.0)) < 1e-14);
    CHECK(orc_search_seconds(1) >= 0.0);
    free(pos);
    free(types);
    free(theta);
    free(qs);
    free(q);
    free(F);
    free(Ei);
    free(grad);
    free(Ft);
    printf("sanitize_check ok: P %ld, D %ld, loss %.6e\n", P, D, loss[0]);
    return 0;
}
