/*
 * oracle_cpu.c -- plain C + OpenMP FP64 estimator of the harmonic-basis 3PCF.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py.  Shares no code with the GPU library.
 *
 * Computes exactly what oracle/ref.py computes (binned estimator of the paper's
 * "3PCF binned estimator" subsection: eqs. Xm.binned, Ym/Zm.binned, zetamEst,
 * zetamEst2, with the readings stated in oracle/__init__.py), for catalogues too
 * large for NumPy:
 *
 *   d2 = (dx*dx + dy*dy) + dz*dz   (FP64, built with -ffp-contract=off: no FMA)
 *   pair kept iff E_0 <= d2 < E_nb, bin b: E_b <= d2 < E_{b+1}
 *   phi = atan2(delta.e_E, delta.e_N)         (position angle, north through east)
 *   a_{m,b} += w_j x_j (cos(m phi) - i sin(m phi))   (direct libm trigonometry)
 *   W_{p,b} += w_j, N_{p,b} += 1
 *   X = a / W (0 where W = 0);  zeta_m(b1,b2) += w_p x_p X(b1) conj X(b2)
 *
 * Neighbour search: a uniform grid of cubes over [-1,1]^3 whose side L is at least
 * the largest chord sqrt(E_nb).  Every neighbour within chord L of a pivot then lies
 * in the 3x3x3 block of cubes around the pivot's cube, so visiting those 27 cubes and
 * applying the d2 rule above finds exactly the pairs of the definition.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
    int g;            /* cubes per axis */
    double inv_side;  /* g / 2 */
    int64_t *start;   /* [g^3 + 1] */
    int64_t *order;   /* catalogue indices sorted by cube */
} cube_grid;

static int cube_coord(double v, const cube_grid *cg)
{
    int c = (int)floor((v + 1.0) * cg->inv_side);
    if (c < 0) c = 0;
    if (c >= cg->g) c = cg->g - 1;
    return c;
}

static int grid_build(cube_grid *cg, int64_t n, const double *x, const double *y,
                      const double *z, double max_chord)
{
    double side = max_chord * (1.0 + 1e-9) + 1e-12;
    if (side < 2.0 / 256.0) side = 2.0 / 256.0;
    int g = (int)floor(2.0 / side);
    if (g < 1) g = 1;
    cg->g = g;
    cg->inv_side = g / 2.0; /* cube side 2/g >= side */
    int64_t ncube = (int64_t)g * g * g;
    cg->start = (int64_t *)calloc((size_t)ncube + 1, sizeof(int64_t));
    cg->order = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *key = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!cg->start || !cg->order || !key) { free(key); return -1; }
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = ((int64_t)cube_coord(x[i], cg) * g + cube_coord(y[i], cg)) * g + cube_coord(z[i], cg);
        key[i] = k;
        cg->start[k + 1]++;
    }
    for (int64_t k = 0; k < ncube; ++k) cg->start[k + 1] += cg->start[k];
    int64_t *fill = (int64_t *)malloc((size_t)ncube * sizeof(int64_t));
    if (!fill) { free(key); return -1; }
    memcpy(fill, cg->start, (size_t)ncube * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) cg->order[fill[key[i]]++] = i;
    free(fill);
    free(key);
    return 0;
}

static void grid_free(cube_grid *cg)
{
    free(cg->start);
    free(cg->order);
}

static uint64_t mix64(uint64_t v)
{   /* SplitMix64 finaliser (Steele, Lea & Flood 2014) */
    v += 0x9E3779B97F4A7C15ull;
    v = (v ^ (v >> 30)) * 0xBF58476D1CE4E5B9ull;
    v = (v ^ (v >> 27)) * 0x94D049BB133111EBull;
    return v ^ (v >> 31);
}

typedef struct {
    int64_t n;
    const double *x, *y, *z, *w, *v; /* neighbour catalogue; v = w * value */
    int nb;
    const double *edges;             /* chord^2 edges [nb + 1] */
    int m_max;
    cube_grid cg;
} catalogue;

/* Multipoles of one pivot.  a_re/a_im: [m_max+1][nb], W: [nb], cnt: [nb]. */
static void pivot_multipoles(const catalogue *c, double px, double py, double pz,
                             double *a_re, double *a_im, double *W, int64_t *cnt,
                             uint64_t *idsum, uint64_t *idhash)
{
    const int nb = c->nb, M = c->m_max;
    memset(a_re, 0, sizeof(double) * (size_t)(M + 1) * nb);
    memset(a_im, 0, sizeof(double) * (size_t)(M + 1) * nb);
    memset(W, 0, sizeof(double) * (size_t)nb);
    memset(cnt, 0, sizeof(int64_t) * (size_t)nb);
    if (idsum) memset(idsum, 0, sizeof(uint64_t) * (size_t)nb);
    if (idhash) memset(idhash, 0, sizeof(uint64_t) * (size_t)nb);

    /* local north and east at the pivot */
    double nx = -pz * px, ny = -pz * py, nz = 1.0 - pz * pz;
    double nn = sqrt(nx * nx + ny * ny + nz * nz);
    if (nn < 1e-12) {
        nx = 1.0 - px * px; ny = -px * py; nz = -px * pz;
        nn = sqrt(nx * nx + ny * ny + nz * nz);
    }
    nx /= nn; ny /= nn; nz /= nn;
    double ex = ny * pz - nz * py, ey = nz * px - nx * pz, ez = nx * py - ny * px;

    const cube_grid *cg = &c->cg;
    int cx = cube_coord(px, cg), cy = cube_coord(py, cg), cz = cube_coord(pz, cg);
    for (int ix = cx - 1; ix <= cx + 1; ++ix) {
        if (ix < 0 || ix >= cg->g) continue;
        for (int iy = cy - 1; iy <= cy + 1; ++iy) {
            if (iy < 0 || iy >= cg->g) continue;
            for (int iz = cz - 1; iz <= cz + 1; ++iz) {
                if (iz < 0 || iz >= cg->g) continue;
                int64_t k = ((int64_t)ix * cg->g + iy) * cg->g + iz;
                for (int64_t s = cg->start[k]; s < cg->start[k + 1]; ++s) {
                    int64_t j = cg->order[s];
                    double dx = c->x[j] - px, dy = c->y[j] - py, dz = c->z[j] - pz;
                    double d2 = (dx * dx + dy * dy) + dz * dz;
                    if (!(d2 >= c->edges[0] && d2 < c->edges[nb])) continue;
                    int b = 0;
                    while (d2 >= c->edges[b + 1]) ++b;
                    double u1 = dx * nx + dy * ny + dz * nz;
                    double u2 = dx * ex + dy * ey + dz * ez;
                    double phi = atan2(u2, u1);
                    double v = c->v[j];
                    for (int m = 0; m <= M; ++m) {
                        a_re[m * nb + b] += v * cos(m * phi);
                        a_im[m * nb + b] -= v * sin(m * phi);
                    }
                    W[b] += c->w[j];
                    cnt[b] += 1;
                    if (idsum) idsum[b] += (uint64_t)j;
                    if (idhash) idhash[b] += mix64((uint64_t)j);
                }
            }
        }
    }
}

static int catalogue_init(catalogue *c, int64_t n, const double *x, const double *y,
                          const double *z, const double *w, const double *v, int nb,
                          const double *edges, int m_max)
{
    c->n = n; c->x = x; c->y = y; c->z = z; c->w = w; c->v = v;
    c->nb = nb; c->edges = edges; c->m_max = m_max;
    return grid_build(&c->cg, n, x, y, z, sqrt(edges[nb]));
}

/*
 * Per-pivot multipoles.  Outputs (row-major, all optional except a_re/a_im):
 *   a_re, a_im [np][m_max+1][nb] raw sums; W [np][nb]; cnt [np][nb];
 *   idsum, idhash [np][nb]: sum of neighbour indices and of mix64(index) per bin.
 */
int zo_multipoles(int64_t n, const double *x, const double *y, const double *z,
                  const double *w, const double *v,
                  int64_t np, const double *px, const double *py, const double *pz,
                  int nb, const double *edges, int m_max,
                  double *a_re, double *a_im, double *W, int64_t *cnt,
                  uint64_t *idsum, uint64_t *idhash, int nthreads)
{
    catalogue c;
    if (catalogue_init(&c, n, x, y, z, w, v, nb, edges, m_max)) return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const size_t A = (size_t)(m_max + 1) * nb;
    int err = 0;
#pragma omp parallel
    {
        double *Wl = (double *)malloc(sizeof(double) * (size_t)nb);
        int64_t *cl = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
        if (!Wl || !cl) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t p = 0; p < np; ++p) {
                pivot_multipoles(&c, px[p], py[p], pz[p], a_re + (size_t)p * A, a_im + (size_t)p * A,
                                 Wl, cl, idsum ? idsum + (size_t)p * nb : NULL,
                                 idhash ? idhash + (size_t)p * nb : NULL);
                if (W) memcpy(W + (size_t)p * nb, Wl, sizeof(double) * (size_t)nb);
                if (cnt) memcpy(cnt + (size_t)p * nb, cl, sizeof(int64_t) * (size_t)nb);
            }
        }
        free(Wl);
        free(cl);
    }
    grid_free(&c.cg);
    return err ? -1 : 0;
}

/*
 * Wall time of the oracle's catalogue set-up alone (the cube grid over all n neighbours,
 * which zo_zeta and zo_multipoles build on every call), in seconds; -1 on failure.
 */
double zo_setup_seconds(int64_t n, const double *x, const double *y, const double *z,
                        const double *w, const double *v, int nb, const double *edges, int m_max)
{
    const double t0 = omp_get_wtime();
    catalogue c;
    if (catalogue_init(&c, n, x, y, z, w, v, nb, edges, m_max)) return -1.0;
    grid_free(&c.cg);
    return omp_get_wtime() - t0;
}

/*
 * zeta over the given pivots: zeta[m][b1][b2][2] = (1/sum w_p) sum_p v_p X(b1) conj X(b2)
 * (pivot values vp = w_p x_p, pivot weights pw).  Pivots are processed in blocks of
 * 1024; each block's partial sum is added in block order, so the result does not
 * depend on the thread count.  *pairs receives the total pair count.
 */
int zo_zeta(int64_t n, const double *x, const double *y, const double *z,
            const double *w, const double *v,
            int64_t np, const double *px, const double *py, const double *pz,
            const double *pw, const double *pv,
            int nb, const double *edges, int m_max,
            double *zeta, int64_t *pairs, int nthreads)
{
    catalogue c;
    if (catalogue_init(&c, n, x, y, z, w, v, nb, edges, m_max)) return -1;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const int64_t BLK = 1024;
    const int64_t nblk = (np + BLK - 1) / BLK;
    const size_t Z = (size_t)(m_max + 1) * nb * nb * 2;
    const size_t A = (size_t)(m_max + 1) * nb;
    double *part = (double *)calloc((size_t)(nblk > 0 ? nblk : 1) * Z, sizeof(double));
    int64_t *pcnt = (int64_t *)calloc((size_t)(nblk > 0 ? nblk : 1), sizeof(int64_t));
    if (!part || !pcnt) { free(part); free(pcnt); grid_free(&c.cg); return -1; }
    int err = 0;
#pragma omp parallel
    {
        double *ar = (double *)malloc(sizeof(double) * A), *ai = (double *)malloc(sizeof(double) * A);
        double *Wl = (double *)malloc(sizeof(double) * (size_t)nb);
        int64_t *cl = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
        if (!ar || !ai || !Wl || !cl) {
#pragma omp atomic write
            err = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t bk = 0; bk < nblk; ++bk) {
                double *zp = part + (size_t)bk * Z;
                int64_t e = (bk + 1) * BLK < np ? (bk + 1) * BLK : np;
                for (int64_t p = bk * BLK; p < e; ++p) {
                    pivot_multipoles(&c, px[p], py[p], pz[p], ar, ai, Wl, cl, NULL, NULL);
                    for (int b = 0; b < nb; ++b) {
                        pcnt[bk] += cl[b];
                        double inv = Wl[b] > 0.0 ? 1.0 / Wl[b] : 0.0;
                        for (int m = 0; m <= m_max; ++m) {
                            ar[m * nb + b] = Wl[b] > 0.0 ? ar[m * nb + b] * inv : 0.0;
                            ai[m * nb + b] = Wl[b] > 0.0 ? ai[m * nb + b] * inv : 0.0;
                        }
                    }
                    for (int m = 0; m <= m_max; ++m)
                        for (int b1 = 0; b1 < nb; ++b1)
                            for (int b2 = 0; b2 < nb; ++b2) {
                                double r1 = ar[m * nb + b1], i1 = ai[m * nb + b1];
                                double r2 = ar[m * nb + b2], i2 = ai[m * nb + b2];
                                /* (r1 + i i1)(r2 - i i2) */
                                double re = r1 * r2 + i1 * i2;
                                double im = i1 * r2 - r1 * i2;
                                size_t o = (((size_t)m * nb + b1) * nb + b2) * 2;
                                zp[o] += pv[p] * re;
                                zp[o + 1] += pv[p] * im;
                            }
                }
            }
        }
        free(ar); free(ai); free(Wl); free(cl);
    }
    double sw = 0.0;
    for (int64_t p = 0; p < np; ++p) sw += pw[p];
    memset(zeta, 0, sizeof(double) * Z);
    int64_t tot = 0;
    for (int64_t bk = 0; bk < nblk; ++bk) {
        for (size_t o = 0; o < Z; ++o) zeta[o] += part[(size_t)bk * Z + o];
        tot += pcnt[bk];
    }
    if (sw != 0.0)
        for (size_t o = 0; o < Z; ++o) zeta[o] /= sw;
    if (pairs) *pairs = tot;
    free(part);
    free(pcnt);
    grid_free(&c.cg);
    return err ? -1 : 0;
}
