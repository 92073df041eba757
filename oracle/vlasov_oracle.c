/*
 * Plain FP64 CPU oracle for the Vlasov translation step with a coalesced
 * ghost domain (Battarbee et al., "Coalescing MPI communication in 6D Vlasov
 * simulations: solving ghost domains in Vlasiator").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the HIP library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never calls it.  It shares no code, header or constant with
 * the HIP library.
 *
 * What it computes (paper sections in brackets):
 *  - The translation part of the Vlasov equation (Section 2, eq. 1: the
 *    v . grad_x f term) split into three Cartesian shears, one per spatial
 *    axis, in a fixed order (Section 2.1).
 *  - Each shear is a conservative semi-Lagrangian remap along straight
 *    pencils of spatial cells: a piecewise-parabolic (PPM) profile is fitted
 *    to the cell averages with a stencil of 2 cells on each side, shifted by
 *    the velocity of the phase-space cell and integrated back into cell
 *    averages (Section 2.1).  The paper names no PPM variant; this oracle uses
 *    the textbook one of Colella & Woodward (1984), J. Comput. Phys. 54:174:
 *    limited slopes (their eq. 1.7-1.8), fourth-order face values (eq. 1.6 on
 *    a uniform grid), the monotonicity limiter (eq. 1.10) and the integrated
 *    flux (eq. 1.12).  The time step keeps |v dt / dx| <= 1, so each cell only
 *    exchanges mass with its face neighbours (Section 2.1).
 *  - The flux form used here (each cell's new average is its old average
 *    plus the difference of its two face fluxes) is the same update as the
 *    paper's push form, in which a cell writes into itself and its downwind
 *    face neighbour (Section 2.1).
 *  - Velocity space is sparse: 64-cell (4x4x4) blocks are added and removed
 *    as needed (Section 2).  Before each shear a cell gains every block that
 *    its upwind face neighbour holds and that moves into it; after the step a
 *    block is kept if one of its values is >= sparse_min, together with a
 *    buffer of neighbouring blocks in velocity space.
 *  - Ghost Translation (Section 3, 3.1, Fig. 3): the partition is padded by
 *    3 ghost layers; one ghost update per step, after which the first shear
 *    is also computed on the ghost cells that later shears read, and the
 *    second shear on those the third shear reads (the "full" variant, GT3,
 *    Section 3.2).  The classical mode (Section 2.1, Fig. 1) instead
 *    refreshes the ghost faces of the current direction before each shear and
 *    computes local cells only.
 *  - Velocity moments (density, bulk velocity, pressure tensor) in two passes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define VLO_H 3          /* ghost depth: 2-cell stencil + 1 face neighbour */
#define VLO_BLK 64       /* phase-space cells per velocity block (4x4x4) */

#define VLO_OK 0
#define VLO_ERR_ARG (-1)
#define VLO_ERR_CFL (-2)
#define VLO_ERR_STALE (-4)

#define VLO_COALESCED 0
#define VLO_PER_SWEEP 1

static const double VLO_MP = 1.67262192e-27; /* proton mass [kg] */

typedef struct {
    int32_t n;     /* number of blocks */
    int32_t *ids;  /* ascending block ids */
    double *f;     /* n * 64 values */
} vlo_cell;

typedef struct {
    int32_t n[3];      /* local cells per axis */
    int32_t P[3];      /* padded cells per axis = n + 2H */
    int32_t nblk[3];   /* velocity blocks per axis */
    int32_t nv[3];     /* velocity cells per axis */
    int32_t NB;        /* number of block ids */
    double dx[3], vmin[3], dv[3];
    int32_t order[3];
    double sparse_min;
    int32_t vbuffer;
    int32_t ghosts_valid;
    int32_t gt_level;  /* Ghost Translation level k = 1, 2, 3 (Section 3.2) */
    int32_t edges;     /* faces at the simulation edge: bit 2d low, 2d+1 high face of axis d */
    vlo_cell *cells;   /* padded box, x fastest */
    double *cover[3];  /* optional Courant table override per axis (nv[d]) */
} vlo_part;

/* ------------------------------------------------------------------------ */
/* small helpers                                                             */
/* ------------------------------------------------------------------------ */
static int64_t cidx(const vlo_part *p, int x, int y, int z)
{
    return (int64_t)x + (int64_t)p->P[0] * ((int64_t)y + (int64_t)p->P[1] * z);
}

static int is_local(const vlo_part *p, int x, int y, int z)
{
    return x >= VLO_H && x < VLO_H + p->n[0] && y >= VLO_H && y < VLO_H + p->n[1] &&
           z >= VLO_H && z < VLO_H + p->n[2];
}

static int find_block(const vlo_cell *c, int32_t id)
{
    int lo = 0, hi = c->n - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (c->ids[mid] == id) return mid;
        if (c->ids[mid] < id) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

static void cell_free(vlo_cell *c)
{
    free(c->ids);
    free(c->f);
    c->ids = NULL;
    c->f = NULL;
    c->n = 0;
}

static void cell_assign(vlo_cell *c, int32_t n, const int32_t *ids, const double *f)
{
    cell_free(c);
    c->n = n;
    if (n > 0) {
        c->ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        c->f = (double *)malloc(sizeof(double) * (size_t)n * VLO_BLK);
        memcpy(c->ids, ids, sizeof(int32_t) * (size_t)n);
        if (f) memcpy(c->f, f, sizeof(double) * (size_t)n * VLO_BLK);
        else memset(c->f, 0, sizeof(double) * (size_t)n * VLO_BLK);
    }
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* velocity-cell index along axis d of lane l of block b */
static int vel_index(const vlo_part *p, int d, int32_t b, int l)
{
    int bd;
    if (d == 0) bd = b % p->nblk[0];
    else if (d == 1) bd = (b / p->nblk[0]) % p->nblk[1];
    else bd = b / (p->nblk[0] * p->nblk[1]);
    int ld = (d == 0) ? (l & 3) : (d == 1) ? ((l >> 2) & 3) : (l >> 4);
    return 4 * bd + ld;
}

/* Courant number of velocity index j along axis d: v_j dt / dx with the
 * cell-centre velocity v_j = vmin + (j + 1/2) dv. */
static double courant(const vlo_part *p, int d, int j, double dt)
{
    if (p->cover[d]) return p->cover[d][j];
    double v = p->vmin[d] + ((double)j + 0.5) * p->dv[d];
    return v * dt / p->dx[d];
}

/* ------------------------------------------------------------------------ */
/* 1D PPM remap of one line (Colella & Woodward 1984, uniform grid)          */
/* ------------------------------------------------------------------------ */
/*
 * a[0..L): cell averages along a pencil.  Cells [3, L-3) are updated:
 *   out[i] = a[i] + F[i-1/2] - F[i+1/2]
 * where F is the fraction of a cell's content (in units of the cell average)
 * crossing a face towards +d during the step.  Optional outputs (may be
 * NULL): face[i] = a_{i+1/2} for i in [1, L-3]; al/ar/a6 = limited profile of
 * cell i for i in [2, L-3]; flux[i] = F_{i+1/2} for i in [2, L-4].
 */
void vlo_ppm_line(const double *a, int L, double c, double *out, double *face_out,
                  double *al_out, double *ar_out, double *a6_out, double *flux_out)
{
    double da[L], face[L], al[L], ar[L], a6[L], F[L];
    for (int i = 0; i < L; i++) da[i] = face[i] = al[i] = ar[i] = a6[i] = F[i] = 0.0;

    /* limited slope (CW84 eq. 1.7-1.8) */
    for (int i = 1; i <= L - 2; i++) {
        double dl = a[i] - a[i - 1];
        double dr = a[i + 1] - a[i];
        if (dr * dl > 0.0) {
            double central = 0.5 * (a[i + 1] - a[i - 1]);
            double m = fabs(central);
            if (2.0 * fabs(dl) < m) m = 2.0 * fabs(dl);
            if (2.0 * fabs(dr) < m) m = 2.0 * fabs(dr);
            da[i] = central > 0.0 ? m : -m;
        } else {
            da[i] = 0.0;
        }
    }
    /* face value a_{i+1/2} (CW84 eq. 1.6, uniform grid) */
    for (int i = 1; i <= L - 3; i++)
        face[i] = a[i] + 0.5 * (a[i + 1] - a[i]) - (da[i + 1] - da[i]) / 6.0;

    /* monotonicity limiter (CW84 eq. 1.10) */
    for (int i = 2; i <= L - 3; i++) {
        double l = face[i - 1], r = face[i], ai = a[i];
        if ((r - ai) * (ai - l) <= 0.0) {
            l = ai;
            r = ai;
        } else {
            double d = r - l;
            double m = ai - 0.5 * (l + r);
            if (d * m > d * d / 6.0) {
                l = 3.0 * ai - 2.0 * r;
            } else if (-(d * d) / 6.0 > d * m) {
                r = 3.0 * ai - 2.0 * l;
            }
        }
        al[i] = l;
        ar[i] = r;
        a6[i] = 6.0 * (ai - 0.5 * (l + r));
    }
    /* flux through face i+1/2 (CW84 eq. 1.12), as a fraction of a cell */
    for (int i = 2; i <= L - 4; i++) {
        if (c > 0.0) {
            double dA = ar[i] - al[i];
            F[i] = c * (ar[i] - 0.5 * c * (dA - (1.0 - 2.0 * c / 3.0) * a6[i]));
        } else if (c < 0.0) {
            double s = -c;
            double dA = ar[i + 1] - al[i + 1];
            F[i] = c * (al[i + 1] + 0.5 * s * (dA + (1.0 - 2.0 * s / 3.0) * a6[i + 1]));
        } else {
            F[i] = 0.0;
        }
    }
    for (int i = 3; i <= L - 4; i++) out[i] = a[i] + (F[i - 1] - F[i]);

    if (face_out) for (int i = 1; i <= L - 3; i++) face_out[i] = face[i];
    if (al_out) for (int i = 2; i <= L - 3; i++) al_out[i] = al[i];
    if (ar_out) for (int i = 2; i <= L - 3; i++) ar_out[i] = ar[i];
    if (a6_out) for (int i = 2; i <= L - 3; i++) a6_out[i] = a6[i];
    if (flux_out) for (int i = 2; i <= L - 4; i++) flux_out[i] = F[i];
}

/* ------------------------------------------------------------------------ */
/* partition lifecycle                                                       */
/* ------------------------------------------------------------------------ */
void *vlo_create(const int32_t *n, const int32_t *nblk, const double *dx, const double *vmin,
                 const double *dv, const int32_t *order, double sparse_min, int32_t vbuffer)
{
    vlo_part *p = (vlo_part *)calloc(1, sizeof(vlo_part));
    for (int d = 0; d < 3; d++) {
        p->n[d] = n[d];
        p->P[d] = n[d] + 2 * VLO_H;
        p->nblk[d] = nblk[d];
        p->nv[d] = 4 * nblk[d];
        p->dx[d] = dx[d];
        p->vmin[d] = vmin[d];
        p->dv[d] = dv[d];
        p->order[d] = order[d];
    }
    p->NB = nblk[0] * nblk[1] * nblk[2];
    p->sparse_min = sparse_min;
    p->vbuffer = vbuffer;
    p->gt_level = VLO_H;
    p->cells = (vlo_cell *)calloc((size_t)p->P[0] * p->P[1] * p->P[2], sizeof(vlo_cell));
    return p;
}

void vlo_destroy(void *h)
{
    vlo_part *p = (vlo_part *)h;
    if (!p) return;
    int64_t N = (int64_t)p->P[0] * p->P[1] * p->P[2];
    for (int64_t i = 0; i < N; i++) cell_free(&p->cells[i]);
    free(p->cells);
    for (int d = 0; d < 3; d++) free(p->cover[d]);
    free(p);
}

/* Set one cell of the padded box (coordinates in [0, P)); ids ascending. */
int vlo_set_cell(void *h, int32_t x, int32_t y, int32_t z, int32_t count, const int32_t *ids,
                 const double *f)
{
    vlo_part *p = (vlo_part *)h;
    if (x < 0 || y < 0 || z < 0 || x >= p->P[0] || y >= p->P[1] || z >= p->P[2]) return VLO_ERR_ARG;
    for (int i = 1; i < count; i++)
        if (ids[i] <= ids[i - 1]) return VLO_ERR_ARG;
    for (int i = 0; i < count; i++)
        if (ids[i] < 0 || ids[i] >= p->NB) return VLO_ERR_ARG;
    cell_assign(&p->cells[cidx(p, x, y, z)], count, ids, f);
    return VLO_OK;
}

int32_t vlo_cell_count(void *h, int32_t x, int32_t y, int32_t z)
{
    vlo_part *p = (vlo_part *)h;
    return p->cells[cidx(p, x, y, z)].n;
}

int vlo_get_cell(void *h, int32_t x, int32_t y, int32_t z, int32_t *ids, double *f)
{
    vlo_part *p = (vlo_part *)h;
    vlo_cell *c = &p->cells[cidx(p, x, y, z)];
    if (c->n > 0) {
        memcpy(ids, c->ids, sizeof(int32_t) * (size_t)c->n);
        memcpy(f, c->f, sizeof(double) * (size_t)c->n * VLO_BLK);
    }
    return c->n;
}

/* Load the local cells (x fastest) from a CSR state. */
int vlo_load_local(void *h, const int64_t *offsets, const int32_t *ids, const double *f)
{
    vlo_part *p = (vlo_part *)h;
    int64_t q = 0;
    for (int z = 0; z < p->n[2]; z++)
        for (int y = 0; y < p->n[1]; y++)
            for (int x = 0; x < p->n[0]; x++, q++) {
                int64_t b0 = offsets[q], b1 = offsets[q + 1];
                int rc = vlo_set_cell(h, x + VLO_H, y + VLO_H, z + VLO_H, (int32_t)(b1 - b0), ids + b0,
                                      f + b0 * VLO_BLK);
                if (rc) return rc;
            }
    p->ghosts_valid = 0;
    return VLO_OK;
}

/* Number of blocks in the local cells (x fastest) — to size an export. */
int64_t vlo_local_blocks(void *h)
{
    vlo_part *p = (vlo_part *)h;
    int64_t s = 0;
    for (int z = 0; z < p->n[2]; z++)
        for (int y = 0; y < p->n[1]; y++)
            for (int x = 0; x < p->n[0]; x++) s += p->cells[cidx(p, x + VLO_H, y + VLO_H, z + VLO_H)].n;
    return s;
}

/* Export the local cells (x fastest) as CSR; arrays sized by the caller. */
void vlo_export_local(void *h, int64_t *offsets, int32_t *ids, double *f)
{
    vlo_part *p = (vlo_part *)h;
    int64_t q = 0, b = 0;
    offsets[0] = 0;
    for (int z = 0; z < p->n[2]; z++)
        for (int y = 0; y < p->n[1]; y++)
            for (int x = 0; x < p->n[0]; x++, q++) {
                vlo_cell *c = &p->cells[cidx(p, x + VLO_H, y + VLO_H, z + VLO_H)];
                if (c->n > 0) {
                    memcpy(ids + b, c->ids, sizeof(int32_t) * (size_t)c->n);
                    memcpy(f + b * VLO_BLK, c->f, sizeof(double) * (size_t)c->n * VLO_BLK);
                }
                b += c->n;
                offsets[q + 1] = b;
            }
}

/* Courant-number override: table[d * stride + j] for velocity index j along
 * axis d (used to drive exact integer shifts); NULL restores v dt / dx. */
void vlo_set_courant_override(void *h, const double *table, int32_t stride)
{
    vlo_part *p = (vlo_part *)h;
    for (int d = 0; d < 3; d++) {
        free(p->cover[d]);
        p->cover[d] = NULL;
        if (table) {
            p->cover[d] = (double *)malloc(sizeof(double) * (size_t)p->nv[d]);
            for (int j = 0; j < p->nv[d]; j++) p->cover[d][j] = table[(size_t)d * stride + j];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* ghost updates (periodic partition: the ghost is the image g mod n)        */
/* ------------------------------------------------------------------------ */
static int wrap(int g, int n)
{
    int l = (g - VLO_H) % n;
    if (l < 0) l += n;
    return l + VLO_H;
}

static void copy_cell(vlo_part *p, int64_t dst, int64_t src)
{
    vlo_cell *s = &p->cells[src];
    cell_assign(&p->cells[dst], s->n, s->ids, s->f);
}

/* A padded cell beyond a face at the simulation edge is a boundary cell
 * (Section 2.1): it provides stencil data but is not translated, and ghost
 * updates leave it as it was loaded. */
static int beyond_edge(const vlo_part *p, int x, int y, int z)
{
    const int g[3] = {x, y, z};
    for (int e = 0; e < 3; e++) {
        if (g[e] < VLO_H && (p->edges >> (2 * e) & 1)) return 1;
        if (g[e] >= VLO_H + p->n[e] && (p->edges >> (2 * e + 1) & 1)) return 1;
    }
    return 0;
}

/* Coalesced ghost update: every padded cell outside the local box becomes a
 * copy of its periodic image (Section 3, Fig. 3a). */
void vlo_fill_ghosts(void *h)
{
    vlo_part *p = (vlo_part *)h;
    for (int z = 0; z < p->P[2]; z++)
        for (int y = 0; y < p->P[1]; y++)
            for (int x = 0; x < p->P[0]; x++) {
                if (is_local(p, x, y, z) || beyond_edge(p, x, y, z)) continue;
                copy_cell(p, cidx(p, x, y, z),
                          cidx(p, wrap(x, p->n[0]), wrap(y, p->n[1]), wrap(z, p->n[2])));
            }
    p->ghosts_valid = 1;
}

/* Declare an explicitly supplied ghost domain (set with vlo_set_cell) as the
 * ghost update of the next step, e.g. when the partition is one of several
 * sub-domains whose halo comes from its neighbours. */
void vlo_mark_ghosts_valid(void *h)
{
    ((vlo_part *)h)->ghosts_valid = 1;
}

/* Classical ghost update along axis d before its shear (Section 2.1, step 1):
 * the 3 ghost layers on both sides of the local box along d. */
static void fill_faces(vlo_part *p, int d)
{
    int lo[3], hi[3];
    for (int e = 0; e < 3; e++) {
        lo[e] = VLO_H;
        hi[e] = VLO_H + p->n[e];
    }
    lo[d] = 0;
    hi[d] = p->P[d];
    for (int z = lo[2]; z < hi[2]; z++)
        for (int y = lo[1]; y < hi[1]; y++)
            for (int x = lo[0]; x < hi[0]; x++) {
                if (is_local(p, x, y, z) || beyond_edge(p, x, y, z)) continue;
                copy_cell(p, cidx(p, x, y, z),
                          cidx(p, wrap(x, p->n[0]), wrap(y, p->n[1]), wrap(z, p->n[2])));
            }
}

/* ------------------------------------------------------------------------ */
/* one shear along axis d on the update box [lo, hi) (padded coordinates)     */
/* ------------------------------------------------------------------------ */
/* sign content of block b along d: bit0 = some lane moves towards +d,
 * bit1 = some lane moves towards -d */
static int block_dirs(const vlo_part *p, int d, int32_t b, double dt)
{
    int r = 0;
    for (int l = 0; l < VLO_BLK; l++) {
        double c = courant(p, d, vel_index(p, d, b, l), dt);
        if (c > 0.0) r |= 1;
        if (c < 0.0) r |= 2;
    }
    return r;
}

static void sweep(vlo_part *p, int d, const int lo[3], const int hi[3], double dt, int64_t *updates)
{
    int e1 = (d == 0) ? 1 : 0;
    int e2 = (d == 2) ? 1 : 2;
    int L = p->P[d];
    int n1 = hi[e1] - lo[e1], n2 = hi[e2] - lo[e2];
    int64_t stride = (d == 0) ? 1 : (d == 1) ? p->P[0] : (int64_t)p->P[0] * p->P[1];
    int64_t total_updates = 0;

    /* per-block direction content, indexed by block id */
    int *dirs = (int *)malloc(sizeof(int) * (size_t)p->NB);
    for (int32_t b = 0; b < p->NB; b++) dirs[b] = block_dirs(p, d, b, dt);

#pragma omp parallel for collapse(2) schedule(dynamic) reduction(+ : total_updates)
    for (int t2 = 0; t2 < n2; t2++)
        for (int t1 = 0; t1 < n1; t1++) {
            int co[3];
            co[e1] = lo[e1] + t1;
            co[e2] = lo[e2] + t2;
            co[d] = 0;
            int64_t base = cidx(p, co[0], co[1], co[2]);
            vlo_cell **cl = (vlo_cell **)malloc(sizeof(vlo_cell *) * (size_t)L);
            for (int i = 0; i < L; i++) cl[i] = &p->cells[base + (int64_t)i * stride];

            /* block growth, from the lists before this shear: a cell gains the
             * blocks of its upwind face neighbours that move into it */
            int32_t **nid = (int32_t **)calloc((size_t)L, sizeof(int32_t *));
            int *nn = (int *)calloc((size_t)L, sizeof(int));
            for (int i = lo[d]; i < hi[d]; i++) {
                int cap = cl[i]->n + cl[i - 1]->n + cl[i + 1]->n;
                int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
                int m = 0;
                for (int k = 0; k < cl[i]->n; k++) tmp[m++] = cl[i]->ids[k];
                for (int k = 0; k < cl[i - 1]->n; k++)
                    if (dirs[cl[i - 1]->ids[k]] & 1) tmp[m++] = cl[i - 1]->ids[k];
                for (int k = 0; k < cl[i + 1]->n; k++)
                    if (dirs[cl[i + 1]->ids[k]] & 2) tmp[m++] = cl[i + 1]->ids[k];
                qsort(tmp, (size_t)m, sizeof(int32_t), cmp_i32);
                int u = 0;
                for (int k = 0; k < m; k++)
                    if (u == 0 || tmp[k] != tmp[u - 1]) tmp[u++] = tmp[k];
                nid[i] = tmp;
                nn[i] = u;
            }
            for (int i = lo[d]; i < hi[d]; i++) {
                if (nn[i] == cl[i]->n) {
                    free(nid[i]);
                    continue;
                }
                double *nf = (double *)calloc((size_t)nn[i] * VLO_BLK, sizeof(double));
                for (int k = 0; k < nn[i]; k++) {
                    int old = find_block(cl[i], nid[i][k]);
                    if (old >= 0) memcpy(nf + (size_t)k * VLO_BLK, cl[i]->f + (size_t)old * VLO_BLK,
                                         sizeof(double) * VLO_BLK);
                }
                free(cl[i]->ids);
                free(cl[i]->f);
                cl[i]->ids = nid[i];
                cl[i]->f = nf;
                cl[i]->n = nn[i];
            }
            free(nid);
            free(nn);

            /* every block held by an updated cell of this pencil */
            int cap = 0;
            for (int i = lo[d]; i < hi[d]; i++) cap += cl[i]->n;
            int32_t *ub = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
            int m = 0;
            for (int i = lo[d]; i < hi[d]; i++)
                for (int k = 0; k < cl[i]->n; k++) ub[m++] = cl[i]->ids[k];
            qsort(ub, (size_t)m, sizeof(int32_t), cmp_i32);
            int nu = 0;
            for (int k = 0; k < m; k++)
                if (nu == 0 || ub[k] != ub[nu - 1]) ub[nu++] = ub[k];

            double *a = (double *)malloc(sizeof(double) * (size_t)L);
            double *out = (double *)malloc(sizeof(double) * (size_t)L);
            int *pos = (int *)malloc(sizeof(int) * (size_t)L);
            for (int q = 0; q < nu; q++) {
                int32_t b = ub[q];
                for (int i = 0; i < L; i++) pos[i] = find_block(cl[i], b);
                for (int l = 0; l < VLO_BLK; l++) {
                    double c = courant(p, d, vel_index(p, d, b, l), dt);
                    for (int i = 0; i < L; i++)
                        a[i] = pos[i] >= 0 ? cl[i]->f[(size_t)pos[i] * VLO_BLK + l] : 0.0;
                    vlo_ppm_line(a, L, c, out, NULL, NULL, NULL, NULL, NULL);
                    for (int i = lo[d]; i < hi[d]; i++)
                        if (pos[i] >= 0) cl[i]->f[(size_t)pos[i] * VLO_BLK + l] = out[i];
                }
                for (int i = lo[d]; i < hi[d]; i++)
                    if (pos[i] >= 0) total_updates += VLO_BLK;
            }
            free(a);
            free(out);
            free(pos);
            free(ub);
            free(cl);
        }
    free(dirs);
    if (updates) *updates += total_updates;
}

/* Update box of shear s (0, 1, 2 in sweep order) in padded coordinates.
 * Coalesced: shear s also covers the ghost layers of the axes swept after it,
 * since those cells feed the later stencils (Section 3.1); Ghost Translation
 * of level k computes only the k layers nearest the local domain and leaves
 * the others at their ghost-update values (Section 3.2: GT3 all three, GT1
 * one); a domain at the simulation edge needs no layers there (Section 3.3).
 * Classical: the local box. */
void vlo_update_box(void *h, int32_t mode, int32_t s, int32_t *lo, int32_t *hi)
{
    vlo_part *p = (vlo_part *)h;
    for (int e = 0; e < 3; e++) {
        lo[e] = VLO_H;
        hi[e] = VLO_H + p->n[e];
    }
    if (mode == VLO_COALESCED)
        for (int t = s + 1; t < 3; t++) {
            int e = p->order[t];
            /* no ghost layers are translated beyond a simulation edge */
            lo[e] = (p->edges >> (2 * e) & 1) ? VLO_H : VLO_H - p->gt_level;
            hi[e] = (p->edges >> (2 * e + 1) & 1) ? VLO_H + p->n[e] : VLO_H + p->n[e] + p->gt_level;
        }
}

/* Faces at the simulation edge (bit 2d: low face of axis d, bit 2d+1: high
 * face); the padded cells beyond them are boundary cells.  Returns 0, or -1
 * for a mask outside 0..63. */
int32_t vlo_set_edges(void *h, int32_t mask)
{
    vlo_part *p = (vlo_part *)h;
    if (mask < 0 || mask > 63) return -1;
    p->edges = mask;
    return 0;
}

/* Ghost Translation level of the coalesced mode: 1, 2 or 3 (default 3).
 * Returns 0, or -1 for another value. */
int32_t vlo_set_gt_level(void *h, int32_t k)
{
    vlo_part *p = (vlo_part *)h;
    if (k < 1 || k > VLO_H) return -1;
    p->gt_level = k;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* end-of-step block pruning (Section 2: blocks added and removed as needed) */
/* ------------------------------------------------------------------------ */
static double prune_cell(vlo_part *p, vlo_cell *c, double vol)
{
    if (p->sparse_min <= 0.0 || c->n == 0) return 0.0;
    char *keep = (char *)calloc((size_t)p->NB, 1);
    for (int k = 0; k < c->n; k++) {
        int content = 0;
        for (int l = 0; l < VLO_BLK; l++)
            if (c->f[(size_t)k * VLO_BLK + l] >= p->sparse_min) content = 1;
        if (!content) continue;
        int32_t b = c->ids[k];
        int bx = b % p->nblk[0], by = (b / p->nblk[0]) % p->nblk[1], bz = b / (p->nblk[0] * p->nblk[1]);
        for (int oz = -1; oz <= 1; oz++)
            for (int oy = -1; oy <= 1; oy++)
                for (int ox = -1; ox <= 1; ox++) {
                    int nz = (ox != 0) + (oy != 0) + (oz != 0);
                    if (nz > 1 && p->vbuffer != 26) continue;
                    if (nz == 1 && p->vbuffer == 0) continue;
                    int x = bx + ox, y = by + oy, z = bz + oz;
                    if (x < 0 || y < 0 || z < 0 || x >= p->nblk[0] || y >= p->nblk[1] || z >= p->nblk[2])
                        continue;
                    keep[x + p->nblk[0] * (y + p->nblk[1] * z)] = 1;
                }
    }
    int nn = 0;
    for (int32_t b = 0; b < p->NB; b++) nn += keep[b];
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nn > 0 ? nn : 1));
    double *f = (double *)calloc((size_t)(nn > 0 ? nn : 1) * VLO_BLK, sizeof(double));
    int q = 0;
    for (int32_t b = 0; b < p->NB; b++)
        if (keep[b]) {
            ids[q] = b;
            int old = find_block(c, b);
            if (old >= 0) memcpy(f + (size_t)q * VLO_BLK, c->f + (size_t)old * VLO_BLK, sizeof(double) * VLO_BLK);
            q++;
        }
    double removed = 0.0;
    for (int k = 0; k < c->n; k++)
        if (!keep[c->ids[k]])
            for (int l = 0; l < VLO_BLK; l++) removed += c->f[(size_t)k * VLO_BLK + l];
    free(keep);
    free(c->ids);
    free(c->f);
    c->ids = ids;
    c->f = f;
    c->n = nn;
    return removed * vol;
}

/* phase-space volume of one cell: dx dy dz dvx dvy dvz */
static double ps_volume(const vlo_part *p)
{
    return p->dx[0] * p->dx[1] * p->dx[2] * p->dv[0] * p->dv[1] * p->dv[2];
}

double vlo_local_mass(void *h)
{
    vlo_part *p = (vlo_part *)h;
    double s = 0.0;
    for (int z = 0; z < p->n[2]; z++)
        for (int y = 0; y < p->n[1]; y++)
            for (int x = 0; x < p->n[0]; x++) {
                vlo_cell *c = &p->cells[cidx(p, x + VLO_H, y + VLO_H, z + VLO_H)];
                for (int64_t k = 0; k < (int64_t)c->n * VLO_BLK; k++) s += c->f[k];
            }
    return s * ps_volume(p);
}

/*
 * One translation step.  stats (may be NULL) receives
 *  [0] local mass before, [1] local mass after, [2] pruned mass,
 *  [3] phase-space cell updates of shear 1, [4] of shear 2, [5] of shear 3,
 *  [6] local blocks after the step.
 */
int vlo_step(void *h, double dt, int32_t mode, double *stats)
{
    vlo_part *p = (vlo_part *)h;
    if (mode != VLO_COALESCED && mode != VLO_PER_SWEEP) return VLO_ERR_ARG;
    for (int d = 0; d < 3; d++)
        for (int j = 0; j < p->nv[d]; j++)
            if (fabs(courant(p, d, j, dt)) > 1.0) return VLO_ERR_CFL;
    if (mode == VLO_COALESCED && !p->ghosts_valid) return VLO_ERR_STALE;
    double m0 = stats ? vlo_local_mass(h) : 0.0;

    for (int s = 0; s < 3; s++) {
        int d = p->order[s];
        int lo[3], hi[3];
        vlo_update_box(h, mode, s, lo, hi);
        if (mode == VLO_PER_SWEEP) fill_faces(p, d);
        int64_t upd = 0;
        sweep(p, d, lo, hi, dt, &upd);
        if (stats) stats[3 + s] = (double)upd;
    }
    p->ghosts_valid = 0;

    double pruned = 0.0, vol = ps_volume(p);
    int64_t nblocks = 0;
    for (int z = 0; z < p->n[2]; z++)
        for (int y = 0; y < p->n[1]; y++)
            for (int x = 0; x < p->n[0]; x++) {
                vlo_cell *c = &p->cells[cidx(p, x + VLO_H, y + VLO_H, z + VLO_H)];
                pruned += prune_cell(p, c, vol);
                nblocks += c->n;
            }
    if (stats) {
        stats[0] = m0;
        stats[1] = vlo_local_mass(h);
        stats[2] = pruned;
        stats[6] = (double)nblocks;
    }
    return VLO_OK;
}

/* ------------------------------------------------------------------------ */
/* velocity moments of the local cells (two passes, FP64)                    */
/* ------------------------------------------------------------------------ */
/*
 * Per local cell (x fastest): number density n = dv^3 sum f, bulk velocity
 * V = dv^3 sum f v / n, pressure tensor P_ab = m_p dv^3 sum f (v_a - V_a)(v_b - V_b)
 * stored as (xx, yy, zz, xy, xz, yz).  total = sum n dx dy dz.
 */
void vlo_moments(void *h, double *dens, double *V, double *P, double *total)
{
    vlo_part *p = (vlo_part *)h;
    double dv3 = p->dv[0] * p->dv[1] * p->dv[2];
    double tot = 0.0;
    int64_t q = 0;
    for (int z = 0; z < p->n[2]; z++)
        for (int y = 0; y < p->n[1]; y++)
            for (int x = 0; x < p->n[0]; x++, q++) {
                vlo_cell *c = &p->cells[cidx(p, x + VLO_H, y + VLO_H, z + VLO_H)];
                double s0 = 0.0, s1[3] = {0.0, 0.0, 0.0};
                for (int k = 0; k < c->n; k++)
                    for (int l = 0; l < VLO_BLK; l++) {
                        double fv = c->f[(size_t)k * VLO_BLK + l];
                        s0 += fv;
                        for (int d = 0; d < 3; d++) {
                            double v = p->vmin[d] + ((double)vel_index(p, d, c->ids[k], l) + 0.5) * p->dv[d];
                            s1[d] += fv * v;
                        }
                    }
                double nd = dv3 * s0;
                double Vc[3] = {0.0, 0.0, 0.0};
                if (s0 != 0.0)
                    for (int d = 0; d < 3; d++) Vc[d] = s1[d] / s0;
                double s2[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                for (int k = 0; k < c->n; k++)
                    for (int l = 0; l < VLO_BLK; l++) {
                        double fv = c->f[(size_t)k * VLO_BLK + l];
                        double u[3];
                        for (int d = 0; d < 3; d++)
                            u[d] = p->vmin[d] + ((double)vel_index(p, d, c->ids[k], l) + 0.5) * p->dv[d] - Vc[d];
                        s2[0] += fv * u[0] * u[0];
                        s2[1] += fv * u[1] * u[1];
                        s2[2] += fv * u[2] * u[2];
                        s2[3] += fv * u[0] * u[1];
                        s2[4] += fv * u[0] * u[2];
                        s2[5] += fv * u[1] * u[2];
                    }
                dens[q] = nd;
                for (int d = 0; d < 3; d++) V[3 * q + d] = Vc[d];
                for (int k = 0; k < 6; k++) P[6 * q + k] = VLO_MP * dv3 * s2[k];
                tot += nd * p->dx[0] * p->dx[1] * p->dx[2];
            }
    *total = tot;
}

/* ------------------------------------------------------------------------ */
/* acceleration: the Lorentz-force term of the Vlasov equation (Section 2,  */
/* eq. 1) over one time step, as three velocity-axis shears (SLICE-3D,      */
/* Zerroukat & Allen 2012, which Section 2 names for this solver)           */
/* ------------------------------------------------------------------------ */
/*
 * In fields E, B that are constant over the step, every velocity moves along
 * its characteristic dv/dt = (q/m)(E + v x B): the part along b = B/|B|
 * gains (q/m)(E.b) t, the rest gyrates about the E x B drift velocity
 * vE = E x B / |B|^2 by the angle -(q/m)|B| t.  Over dt this is the affine
 * map v' = A v + c with A the rotation by theta = -(q/m)|B| dt about b and
 * c = (I - A) vE + (q/m)(E.b) dt b; with B = 0 it is v' = v + (q/m) E dt.
 * Rotation about a unit axis b by theta (Rodrigues):
 *   A = cos(theta) I + sin(theta) [b]x + (1 - cos(theta)) b b^T.
 */
void vlo_accel_map(const double *E, const double *B, double qm, double dt, double *A, double *c)
{
    double Bm = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    for (int i = 0; i < 9; i++) A[i] = (i % 4 == 0) ? 1.0 : 0.0;
    if (Bm == 0.0) {
        for (int d = 0; d < 3; d++) c[d] = qm * E[d] * dt;
        return;
    }
    double b[3] = {B[0] / Bm, B[1] / Bm, B[2] / Bm};
    double th = -qm * Bm * dt;
    double co = cos(th), si = sin(th);
    double cross[9] = {0.0, -b[2], b[1], b[2], 0.0, -b[0], -b[1], b[0], 0.0};
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            A[3 * i + j] = (i == j ? co : 0.0) + si * cross[3 * i + j] + (1.0 - co) * b[i] * b[j];
    double vE[3] = {(E[1] * B[2] - E[2] * B[1]) / (Bm * Bm), (E[2] * B[0] - E[0] * B[2]) / (Bm * Bm),
                    (E[0] * B[1] - E[1] * B[0]) / (Bm * Bm)};
    double Epar = E[0] * b[0] + E[1] * b[1] + E[2] * b[2];
    for (int i = 0; i < 3; i++) {
        double Av = A[3 * i] * vE[0] + A[3 * i + 1] * vE[1] + A[3 * i + 2] * vE[2];
        c[i] = vE[i] - Av + qm * Epar * dt * b[i];
    }
}

/*
 * SLICE-3D splits the map into three maps that each change one velocity
 * coordinate, in the order o[0], o[1], o[2]: the k-th sets coordinate o[k] to
 * its final value, written as an affine function of the coordinates the
 * velocity has after the maps before it.  With the homogeneous 4x4 form T of
 * the map (rows A | c), step k's row is T's row o[k] times the inverses of the
 * steps before it, so the three steps compose to T exactly.
 * M[4k .. 4k+3] receives step k's row (coefficients of coordinates 0, 1, 2 and
 * the constant).  Returns 0, or -1 if a step's own coefficient is not
 * positive (the step would not be invertible and order-preserving).
 */
static void inv_step(const double *row, int d, double *Minv)
{
    /* inverse of the identity with row d replaced by row (4x4, row-major) */
    for (int i = 0; i < 16; i++) Minv[i] = (i % 5 == 0) ? 1.0 : 0.0;
    for (int j = 0; j < 4; j++) Minv[4 * d + j] = (j == d) ? 1.0 / row[d] : -row[j] / row[d];
}

static void row_times(const double *row, const double *M, double *out)
{
    for (int j = 0; j < 4; j++) {
        double s = 0.0;
        for (int i = 0; i < 4; i++) s += row[i] * M[4 * i + j];
        out[j] = s;
    }
}

int vlo_slice_factors(const double *A, const double *c, const int32_t *o, double *M)
{
    double T[3][4];
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) T[i][j] = A[3 * i + j];
        T[i][3] = c[i];
    }
    double r0[4], r1[4], r2[4], t[4], I0[16], I1[16];
    for (int j = 0; j < 4; j++) r0[j] = T[o[0]][j];
    if (!(r0[o[0]] > 0.0)) return -1;
    inv_step(r0, o[0], I0);
    row_times(T[o[1]], I0, r1);
    if (!(r1[o[1]] > 0.0)) return -1;
    inv_step(r1, o[1], I1);
    row_times(T[o[2]], I0, t);
    row_times(t, I1, r2);
    if (!(r2[o[2]] > 0.0)) return -1;
    for (int j = 0; j < 4; j++) {
        M[j] = r0[j];
        M[4 + j] = r1[j];
        M[8 + j] = r2[j];
    }
    return 0;
}

/*
 * Conservative remap of one column of N cells of unit width: cell i covers
 * [i, i+1) and holds the average a[i]; values outside [0, N) are zero.  The
 * column moves by u -> alpha u + sigma (alpha > 0), so cell i of the result
 * receives the mass of the source interval [(i - sigma)/alpha,
 * (i + 1 - sigma)/alpha] under the CW84 parabolas of a (the same slopes,
 * faces and limiter as the spatial remap), divided by its unit width.  A
 * source cell covered whole contributes its average exactly.
 */
void vlo_remap_column(const double *a, int N, double alpha, double sigma, double *out)
{
    int L = N + 6;
    double pad[L], al[L], ar[L], a6[L], tmp[L];
    for (int i = 0; i < L; i++) pad[i] = (i >= 3 && i < N + 3) ? a[i - 3] : 0.0;
    for (int i = 0; i < L; i++) al[i] = ar[i] = a6[i] = 0.0;
    vlo_ppm_line(pad, L, 0.0, tmp, NULL, al, ar, a6, NULL);
    for (int i = 0; i < N; i++) {
        double lo = ((double)i - sigma) / alpha, hi = ((double)i + 1.0 - sigma) / alpha;
        double m = 0.0;
        int j0 = (int)floor(lo), j1 = (int)floor(hi);
        if (j0 < 0) j0 = 0;
        if (j1 > N - 1) j1 = N - 1;
        for (int j = j0; j <= j1; j++) {
            double xa = lo - j, xb = hi - j;
            if (xa < 0.0) xa = 0.0;
            if (xb > 1.0) xb = 1.0;
            if (!(xb > xa)) continue;
            int q = j + 3;
            if (xa == 0.0 && xb == 1.0) {
                m += pad[q];
                continue;
            }
            double dA = ar[q] - al[q];
            m += al[q] * (xb - xa) + 0.5 * (dA + a6[q]) * (xb * xb - xa * xa) -
                 a6[q] * (xb * xb * xb - xa * xa * xa) / 3.0;
        }
        out[i] = m;
    }
}

/*
 * One acceleration step of every local cell: the fields of cell q are
 * EB[6q .. 6q+5] = (Ex, Ey, Ez, Bx, By, Bz), qm the charge-to-mass ratio.  The
 * cell's velocity space is remapped densely (absent blocks read as zero) by
 * the three steps of vlo_slice_factors in the order o; a column along axis d
 * (fixed cells of the other two axes, at their centre velocities w) moves by
 * w_d -> alpha w_d + s with alpha and s from the step's row.  The new block
 * list is the old list plus every block holding a nonzero value; then the
 * end-of-step pruning (as after a translation step).  Mass leaving the
 * velocity mesh is lost.  stats (may be NULL): [0] local mass before,
 * [1] after, [2] pruned, [3] local blocks after.  Returns 0, or -1 if a
 * cell's map cannot be split (see vlo_slice_factors).
 */
int vlo_accelerate(void *h, double dt, double qm, const double *EB, const int32_t *o, double *stats)
{
    vlo_part *p = (vlo_part *)h;
    const int nv0 = p->nv[0], nv1 = p->nv[1], nv2 = p->nv[2];
    const int64_t NV = (int64_t)nv0 * nv1 * nv2;
    const int64_t ncell = (int64_t)p->n[0] * p->n[1] * p->n[2];
    double m0 = stats ? vlo_local_mass(h) : 0.0;
    int bad = 0;
#pragma omp parallel for schedule(dynamic) reduction(| : bad)
    for (int64_t q = 0; q < ncell; q++) {
        int x = (int)(q % p->n[0]), y = (int)((q / p->n[0]) % p->n[1]), z = (int)(q / ((int64_t)p->n[0] * p->n[1]));
        vlo_cell *cl = &p->cells[cidx(p, x + VLO_H, y + VLO_H, z + VLO_H)];
        double A[9], c[3], M[12];
        vlo_accel_map(EB + 6 * q, EB + 6 * q + 3, qm, dt, A, c);
        if (vlo_slice_factors(A, c, o, M)) {
            bad = 1;
            continue;
        }
        /* dense velocity space of the cell, j = j0 + nv0 (j1 + nv1 j2) */
        double *f = (double *)calloc((size_t)NV, sizeof(double));
        for (int k = 0; k < cl->n; k++)
            for (int l = 0; l < VLO_BLK; l++) {
                int j0 = vel_index(p, 0, cl->ids[k], l), j1 = vel_index(p, 1, cl->ids[k], l),
                    j2 = vel_index(p, 2, cl->ids[k], l);
                f[j0 + (int64_t)nv0 * (j1 + (int64_t)nv1 * j2)] = cl->f[(size_t)k * VLO_BLK + l];
            }
        const int nv[3] = {nv0, nv1, nv2};
        const int64_t stride[3] = {1, nv0, (int64_t)nv0 * nv1};
        int maxn = nv0 > nv1 ? (nv0 > nv2 ? nv0 : nv2) : (nv1 > nv2 ? nv1 : nv2);
        double *col = (double *)malloc(sizeof(double) * (size_t)maxn);
        double *res = (double *)malloc(sizeof(double) * (size_t)maxn);
        for (int k = 0; k < 3; k++) {
            const int d = o[k];
            const int e1 = (d == 0) ? 1 : 0, e2 = (d == 2) ? 1 : 2;
            const double *row = M + 4 * k;
            const double alpha = row[d];
            for (int i2 = 0; i2 < nv[e2]; i2++)
                for (int i1 = 0; i1 < nv[e1]; i1++) {
                    double w1 = p->vmin[e1] + ((double)i1 + 0.5) * p->dv[e1];
                    double w2 = p->vmin[e2] + ((double)i2 + 0.5) * p->dv[e2];
                    double s = row[e1] * w1 + row[e2] * w2 + row[3];
                    /* in cell units along d: u -> alpha u + sigma */
                    double sigma = ((alpha - 1.0) * p->vmin[d] + s) / p->dv[d];
                    int64_t base = (int64_t)i1 * stride[e1] + (int64_t)i2 * stride[e2];
                    int any = 0;
                    for (int i = 0; i < nv[d]; i++) {
                        col[i] = f[base + (int64_t)i * stride[d]];
                        any |= col[i] != 0.0;
                    }
                    if (!any) continue;
                    vlo_remap_column(col, nv[d], alpha, sigma, res);
                    for (int i = 0; i < nv[d]; i++) f[base + (int64_t)i * stride[d]] = res[i];
                }
        }
        free(col);
        free(res);
        /* new list: the old blocks and every block holding a nonzero value */
        char *keep = (char *)calloc((size_t)p->NB, 1);
        for (int k = 0; k < cl->n; k++) keep[cl->ids[k]] = 1;
        for (int32_t b = 0; b < p->NB; b++) {
            if (keep[b]) continue;
            for (int l = 0; l < VLO_BLK && !keep[b]; l++) {
                int j0 = vel_index(p, 0, b, l), j1 = vel_index(p, 1, b, l), j2 = vel_index(p, 2, b, l);
                if (f[j0 + (int64_t)nv0 * (j1 + (int64_t)nv1 * j2)] != 0.0) keep[b] = 1;
            }
        }
        int nn = 0;
        for (int32_t b = 0; b < p->NB; b++) nn += keep[b];
        int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nn > 0 ? nn : 1));
        double *nf = (double *)malloc(sizeof(double) * (size_t)(nn > 0 ? nn : 1) * VLO_BLK);
        int u = 0;
        for (int32_t b = 0; b < p->NB; b++)
            if (keep[b]) {
                ids[u] = b;
                for (int l = 0; l < VLO_BLK; l++) {
                    int j0 = vel_index(p, 0, b, l), j1 = vel_index(p, 1, b, l), j2 = vel_index(p, 2, b, l);
                    nf[(size_t)u * VLO_BLK + l] = f[j0 + (int64_t)nv0 * (j1 + (int64_t)nv1 * j2)];
                }
                u++;
            }
        free(keep);
        free(f);
        free(cl->ids);
        free(cl->f);
        cl->ids = ids;
        cl->f = nf;
        cl->n = nn;
    }
    if (bad) return -1;
    double pruned = 0.0, vol = ps_volume(p);
    int64_t nblocks = 0;
    for (int z = 0; z < p->n[2]; z++)
        for (int y = 0; y < p->n[1]; y++)
            for (int x = 0; x < p->n[0]; x++) {
                vlo_cell *cl = &p->cells[cidx(p, x + VLO_H, y + VLO_H, z + VLO_H)];
                pruned += prune_cell(p, cl, vol);
                nblocks += cl->n;
            }
    p->ghosts_valid = 0;
    if (stats) {
        stats[0] = m0;
        stats[1] = vlo_local_mass(h);
        stats[2] = pruned;
        stats[3] = (double)nblocks;
    }
    return 0;
}
