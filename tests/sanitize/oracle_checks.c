/*
 * The C oracle (oracle/oracle_cpu.c) under AddressSanitizer and UndefinedBehaviorSanitizer,
 * on a small seeded catalogue: every output of zo_multipoles (with and without the optional
 * arrays), zo_zeta and zo_setup_seconds, an empty pivot set, and a check of the pair counts
 * against a direct double loop and of zeta's Hermitian symmetry.  Built and run by
 * tests/test_sanitizers.py; exit status 0 when every check holds.
 */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int zo_multipoles(int64_t n, const double *x, const double *y, const double *z, const double *w, const double *v,
                  int64_t np, const double *px, const double *py, const double *pz, int nb, const double *edges,
                  int m_max, double *a_re, double *a_im, double *W, int64_t *cnt, uint64_t *idsum, uint64_t *idhash,
                  int nthreads);
double zo_setup_seconds(int64_t n, const double *x, const double *y, const double *z, const double *w,
                        const double *v, int nb, const double *edges, int m_max);
int zo_zeta(int64_t n, const double *x, const double *y, const double *z, const double *w, const double *v,
            int64_t np, const double *px, const double *py, const double *pz, const double *pw, const double *pv,
            int nb, const double *edges, int m_max, double *zeta, int64_t *pairs, int nthreads);

static uint64_t state = 12345;
static double uniform(void)
{   /* 64-bit LCG (Knuth's MMIX constants), top 53 bits */
    state = state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}

int main(void)
{
    enum { N = 600, NP = 150, NB = 4, M = 6 };
    const double cap = 5.0 * M_PI / 180.0;
    double *x = malloc(N * sizeof(double)), *y = malloc(N * sizeof(double)), *z = malloc(N * sizeof(double));
    double *w = malloc(N * sizeof(double)), *v = malloc(N * sizeof(double));
    for (int i = 0; i < N; ++i) {
        const double ca = 1.0 - uniform() * (1.0 - cos(cap)), sa = sqrt(1.0 - ca * ca), b = 2.0 * M_PI * uniform();
        x[i] = ca;
        y[i] = sa * cos(b);
        z[i] = sa * sin(b);
        w[i] = 0.5 + uniform();
        v[i] = w[i] * (uniform() - 0.3);
    }
    double edges[NB + 1];
    for (int b = 0; b <= NB; ++b) {
        const double t = (0.2 + 0.6 * b) * M_PI / 180.0, s = 2.0 * sin(t / 2.0);
        edges[b] = s * s;
    }
    const size_t A = (size_t)(M + 1) * NB;
    double *are = malloc(NP * A * sizeof(double)), *aim = malloc(NP * A * sizeof(double));
    double *W = malloc(NP * NB * sizeof(double));
    int64_t *cnt = malloc(NP * NB * sizeof(int64_t));
    uint64_t *ids = malloc(NP * NB * sizeof(uint64_t)), *idh = malloc(NP * NB * sizeof(uint64_t));
    int bad = 0;
    if (zo_multipoles(N, x, y, z, w, v, NP, x, y, z, NB, edges, M, are, aim, W, cnt, ids, idh, 4)) bad |= 1;
    if (zo_multipoles(N, x, y, z, w, v, NP, x, y, z, NB, edges, M, are, aim, NULL, NULL, NULL, NULL, 2)) bad |= 2;
    if (zo_multipoles(N, x, y, z, w, v, 0, x, y, z, NB, edges, M, are, aim, W, cnt, NULL, NULL, 1)) bad |= 4;
    /* counts against a direct double loop over the same d2 rule */
    for (int p = 0; p < NP; ++p)
        for (int b = 0; b < NB; ++b) {
            int64_t c = 0;
            for (int j = 0; j < N; ++j) {
                const double dx = x[j] - x[p], dy = y[j] - y[p], dz = z[j] - z[p];
                const double d2 = (dx * dx + dy * dy) + dz * dz;
                if (d2 >= edges[b] && d2 < edges[b + 1]) ++c;
            }
            if (c != cnt[p * NB + b]) bad |= 8;
        }
    double *zeta = calloc(A * NB * 2, sizeof(double));
    double *pw = malloc(NP * sizeof(double)), *pv = malloc(NP * sizeof(double));
    for (int p = 0; p < NP; ++p) { pw[p] = w[p]; pv[p] = v[p]; }
    int64_t pairs = 0, total = 0;
    if (zo_zeta(N, x, y, z, w, v, NP, x, y, z, pw, pv, NB, edges, M, zeta, &pairs, 3)) bad |= 16;
    for (int i = 0; i < NP * NB; ++i) total += cnt[i];
    if (pairs != total || pairs == 0) bad |= 32;
    for (int m = 0; m <= M; ++m)
        for (int b1 = 0; b1 < NB; ++b1)
            for (int b2 = 0; b2 < NB; ++b2) {
                const double *z12 = zeta + (((size_t)m * NB + b1) * NB + b2) * 2;
                const double *z21 = zeta + (((size_t)m * NB + b2) * NB + b1) * 2;
                if (fabs(z12[0] - z21[0]) > 1e-12 * (fabs(z12[0]) + 1e-300) || fabs(z12[1] + z21[1]) > 1e-12)
                    bad |= 64;
            }
    double *zeta0 = calloc(A * NB * 2, sizeof(double));
    int64_t pairs0 = -1;
    if (zo_zeta(N, x, y, z, w, v, 0, x, y, z, pw, pv, NB, edges, M, zeta0, &pairs0, 1) || pairs0 != 0) bad |= 128;
    if (zo_setup_seconds(N, x, y, z, w, v, NB, edges, M) < 0.0) bad |= 256;
    free(x); free(y); free(z); free(w); free(v); free(are); free(aim); free(W); free(cnt); free(ids); free(idh);
    free(zeta); free(zeta0); free(pw); free(pv);
    if (bad) fprintf(stderr, "oracle checks failed: mask %d\n", bad);
    else printf("oracle checks ok (%lld pairs)\n", (long long)pairs);
    return bad ? 1 : 0;
}
