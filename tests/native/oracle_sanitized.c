/*
 * Driver for a sanitizer build of the oracle (tests/test_oracle_sanitized.py
 * compiles oracle/vlasov_oracle.c together with this file under
 * -fsanitize=address,undefined and runs it).  It exercises every entry point
 * on small cases: the line remap with all optional outputs, dense and sparse
 * steps in both ghost schemes, pruning with 0, 6 and 26 neighbours, GT
 * levels, simulation edges, Courant overrides, the longest pencil (256 padded
 * cells, whose per-line arrays live on the stack) and the moments, and checks
 * the invariants that hold exactly (mass balance with the pruned mass).
 * Prints "ok" and returns 0 on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void vlo_ppm_line(const double *a, int L, double c, double *out, double *face_out, double *al_out,
                  double *ar_out, double *a6_out, double *flux_out);
void *vlo_create(const int32_t *n, const int32_t *nblk, const double *dx, const double *vmin,
                 const double *dv, const int32_t *order, double sparse_min, int32_t vbuffer);
void vlo_destroy(void *h);
int vlo_set_cell(void *h, int32_t x, int32_t y, int32_t z, int32_t count, const int32_t *ids,
                 const double *f);
int32_t vlo_cell_count(void *h, int32_t x, int32_t y, int32_t z);
int vlo_get_cell(void *h, int32_t x, int32_t y, int32_t z, int32_t *ids, double *f);
int vlo_load_local(void *h, const int64_t *offsets, const int32_t *ids, const double *f);
int64_t vlo_local_blocks(void *h);
void vlo_export_local(void *h, int64_t *offsets, int32_t *ids, double *f);
void vlo_set_courant_override(void *h, const double *table, int32_t stride);
void vlo_fill_ghosts(void *h);
void vlo_mark_ghosts_valid(void *h);
void vlo_update_box(void *h, int32_t mode, int32_t s, int32_t *lo, int32_t *hi);
int32_t vlo_set_edges(void *h, int32_t mask);
int32_t vlo_set_gt_level(void *h, int32_t k);
double vlo_local_mass(void *h);
int vlo_step(void *h, double dt, int32_t mode, double *stats);
void vlo_moments(void *h, double *dens, double *V, double *P, double *total);

static int failures = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            printf("check failed at line %d: %s\n", __LINE__, #c);      \
            failures++;                                                  \
        }                                                                \
    } while (0)

static uint64_t rng_state = 0x2504214500000001ull;
static double urand(void)
{
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

/* random sparse state: each cell holds each block with probability density */
static void *make_state(const int32_t n[3], const int32_t nblk[3], double density, double smin, int vb,
                        const int32_t order[3])
{
    const double dx[3] = {6.0, 5.0, 7.0}, dv[3] = {1.0, 1.0, 1.0};
    double vmin[3];
    for (int d = 0; d < 3; d++) vmin[d] = -2.0 * nblk[d];
    void *h = vlo_create(n, nblk, dx, vmin, dv, order, smin, vb);
    const int NB = nblk[0] * nblk[1] * nblk[2];
    const int64_t nc = (int64_t)n[0] * n[1] * n[2];
    int64_t *off = calloc((size_t)nc + 1, sizeof(int64_t));
    int32_t *ids = malloc(sizeof(int32_t) * (size_t)(nc * NB + 1));
    double *f = malloc(sizeof(double) * (size_t)(nc * NB * 64 + 64));
    int64_t m = 0;
    for (int64_t c = 0; c < nc; c++) {
        for (int b = 0; b < NB; b++)
            if (urand() < density) {
                ids[m] = b;
                for (int l = 0; l < 64; l++) f[m * 64 + l] = urand() < 0.2 ? 0.0 : 1e-9 * urand();
                m++;
            }
        off[c + 1] = m;
    }
    CHECK(vlo_load_local(h, off, ids, f) == 0);
    free(off);
    free(ids);
    free(f);
    return h;
}

/* exact_mass: the step conserves the local mass up to the pruned mass (not
 * so for GT1/GT2, whose stale ghost layers feed the local cells) */
static void run_steps(void *h, int steps, int mode, double dt, int exact_mass)
{
    for (int k = 0; k < steps; k++) {
        double st[8];
        if (mode == 0) vlo_fill_ghosts(h);
        CHECK(vlo_step(h, dt, mode, st) == 0);
        if (exact_mass) CHECK(fabs(st[1] + st[2] - st[0]) <= 1e-12 * (st[0] > 0 ? st[0] : 1.0));
    }
}

int main(void)
{
    /* line remap, every optional output, several Courant numbers */
    {
        const int L = 40;
        double a[40], out[40], face[40], al[40], ar[40], a6[40], fl[40];
        for (int i = 0; i < L; i++) a[i] = (i > 10 && i < 25) ? 1.0 + urand() : 0.0;
        const double cs[] = {-1.0, -0.7, -0.2, 0.0, 0.3, 0.5, 1.0};
        for (int k = 0; k < 7; k++) {
            vlo_ppm_line(a, L, cs[k], out, face, al, ar, a6, fl);
            double m0 = 0.0, m1 = 0.0;
            for (int i = 3; i < L - 3; i++) {
                m0 += a[i];
                m1 += out[i];
            }
            CHECK(fabs(m1 - m0) <= 1e-13 * m0);
        }
    }
    const int32_t o012[3] = {0, 1, 2}, o201[3] = {2, 0, 1};
    /* sparse steps, both schemes, three buffers */
    {
        const int32_t n[3] = {5, 4, 6}, nblk[3] = {3, 2, 3};
        const int vbs[3] = {0, 6, 26};
        for (int v = 0; v < 3; v++)
            for (int mode = 0; mode < 2; mode++) {
                void *h = make_state(n, nblk, 0.4, 6e-10, vbs[v], v == 1 ? o201 : o012);
                run_steps(h, 2, mode, 1.0, 1);
                const int64_t nb = vlo_local_blocks(h);
                int64_t *off = malloc(sizeof(int64_t) * (5 * 4 * 6 + 1));
                int32_t *ids = malloc(sizeof(int32_t) * (size_t)(nb + 1));
                double *f = malloc(sizeof(double) * (size_t)(nb + 1) * 64);
                vlo_export_local(h, off, ids, f);
                CHECK(off[5 * 4 * 6] == nb);
                double dens[120], V[360], P[720], tot;
                vlo_moments(h, dens, V, P, &tot);
                CHECK(tot >= 0.0);
                free(off);
                free(ids);
                free(f);
                vlo_destroy(h);
            }
    }
    /* GT levels, edges (boundary cells set explicitly), Courant override */
    {
        const int32_t n[3] = {4, 5, 3}, nblk[3] = {2, 2, 2};
        for (int k = 1; k <= 3; k++) {
            void *h = make_state(n, nblk, 0.5, 0.0, 0, o012);
            CHECK(vlo_set_gt_level(h, k) == 0);
            int32_t lo[3], hi[3];
            for (int s = 0; s < 3; s++) vlo_update_box(h, 0, s, lo, hi);
            run_steps(h, 2, 0, 1.0, k == 3);
            vlo_destroy(h);
        }
        void *h = make_state(n, nblk, 0.5, 0.0, 0, o012);
        CHECK(vlo_set_edges(h, 0x3) == 0);
        CHECK(vlo_set_edges(h, 64) == -1);
        const int32_t id0 = 3;
        double blk[64];
        for (int l = 0; l < 64; l++) blk[l] = 1e-9;
        for (int z = 0; z < 9; z++)
            for (int y = 0; y < 11; y++)
                for (int x = 0; x < 3; x++) {
                    CHECK(vlo_set_cell(h, x, y, z, 1, &id0, blk) == 0);
                    CHECK(vlo_set_cell(h, x + 7, y, z, 0, &id0, blk) == 0);
                }
        vlo_mark_ghosts_valid(h);
        double st[8];
        CHECK(vlo_step(h, 1.0, 0, st) == 0);
        double tab[3 * 8];
        for (int i = 0; i < 24; i++) tab[i] = (i % 3) - 1.0;
        vlo_set_courant_override(h, tab, 8);
        vlo_fill_ghosts(h);
        CHECK(vlo_step(h, 1.0, 0, st) == 0);
        vlo_set_courant_override(h, NULL, 0);
        int32_t cid[8];
        double cf[8 * 64];
        CHECK(vlo_get_cell(h, 3, 3, 3, cid, cf) == vlo_cell_count(h, 3, 3, 3));
        CHECK(vlo_step(h, 1.0, 0, st) == -4);  /* ghosts consumed */
        vlo_destroy(h);
    }
    /* the longest pencil: 250 local cells along x (256 padded) */
    {
        const int32_t n[3] = {250, 1, 1}, nblk[3] = {1, 1, 1};
        void *h = make_state(n, nblk, 1.0, 0.0, 0, o012);
        run_steps(h, 2, 0, 1.0, 1);
        run_steps(h, 1, 1, 1.0, 1);
        vlo_destroy(h);
    }
    if (failures) {
        printf("%d checks failed\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
