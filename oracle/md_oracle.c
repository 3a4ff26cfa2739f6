/*
 * md_oracle.c -- plain FP64 CPU oracle for soft-sphere molecular dynamics
 * (Rapaport, "Enhanced molecular dynamics performance with a programmable
 * graphics processor", arXiv:0911.5631).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library product links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the HIP path.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared (no FMA
 * contraction, IEEE round-to-nearest-even, single thread).
 *
 * What it computes, and where the paper defines it:
 *   - the soft-sphere potential: Eq. (1) truncated at r_c = 2^(1/6) with the
 *     constant epsilon added so that u(r_c) = 0 (Sec. 3.1, Eq. 1 and the
 *     sentence after it); reduced units sigma = epsilon = m = 1;
 *   - region geometry: edge L, cell grid G = floor(L / r_n) per edge, cell
 *     edge w = L / G, region centred at the origin (Sec. 3.1);
 *   - cell assignment by linked lists (Sec. 3.2, first algorithm);
 *   - the half neighbour-pair list over 14 cells with periodic image codes
 *     (Sec. 3.2, second algorithm) and the Newton's-third-law force loop over
 *     it (Sec. 3.2, third algorithm);
 *   - layer assignment (Sec. 3.4, first algorithm) and the cell-order
 *     reordering scan of the cell-layer matrix (Sec. 3.5, reorder algorithm),
 *     used to state what a stable cell binning must produce;
 *   - the leapfrog MD loop, steps (a)-(e), with the neighbour list rebuilt
 *     once the accumulated maximum displacement passes delta/2 (Sec. 3.1), and
 *     step (f), the velocity adjustment of the equilibration period (Sec. 5.1);
 *   - brute-force O(N^2) definitions of the pair set and of the forces over
 *     all 27 periodic images, used to pin the cell algorithms above.
 *
 * Readings where the paper is silent (kept identical in the HIP path so that
 * integer results can be compared bit for bit):
 *   - cell coordinate: c = (int)((x + L/2) * invW) with invW = G / L computed
 *     once in FP64, clamped to [0, G-1]; scalar index (c_z*G + c_y)*G + c_x;
 *   - wrap: x >= L/2 -> x - L, x < -L/2 -> x + L (exact by Sterbenz), applied
 *     at every rebuild (every step in cell-list-only mode);
 *   - pair separation d = (x_i - x_j) + b with b in {-L, 0, +L}, b = -L when
 *     the neighbour cell index wrapped past G-1 and +L when it wrapped below 0;
 *     r^2 = (d_x*d_x + d_y*d_y) + d_z*d_z; both cutoff tests strict;
 *   - virial W = sum over pairs of f(r) r^2 (the paper does not define it);
 *   - the create-time evaluation is step 0's (b)-(e): wrap, bin, list, forces,
 *     properties, then disp = vmax*dt and the rebuild flag from it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_BOX_TOO_SMALL (-2)
#define OR_ERR_NOMEM (-3)
#define OR_ERR_PAIR_CAP (-5)

/* ------------------------------------------------------------------------ */
/* Pair potential, Eq. (1) with the soft-sphere shift.                      */
/* Input r^2 (s); returns f such that the force on i is f * d, d = r_i-r_j, */
/* and the pair energy in *u.  ushift = 1 for soft spheres, 0 for plain LJ. */
/* ------------------------------------------------------------------------ */
static double pair_fu(double s, double ushift, double *u)
{
    double rri = 1.0 / s;
    double rri3 = rri * rri * rri;
    double f = 48.0 * rri3 * (rri3 - 0.5) * rri;
    *u = 4.0 * rri3 * (rri3 - 1.0) + ushift;
    return f;
}

/* u(r) and the radial force magnitude -du/dr for a single distance (pins). */
void or_pair_potential(double r, double rc, double ushift, double *u, double *fr)
{
    double s = r * r;
    if (!(s < rc * rc)) { *u = 0.0; *fr = 0.0; return; }
    double uu;
    double f = pair_fu(s, ushift, &uu);
    *u = uu;
    *fr = f * r;
}

/* ------------------------------------------------------------------------ */
/* Several species: the extension the paper names in Sec. 3.5 (no  */
/* parameters given there).  Each species pair (a, b) has its own epsilon,  */
/* sigma, cutoff and energy shift: u = 4 eps ((sigma/r)^12 - (sigma/r)^6) + */
/* shift inside the cutoff, i.e. Eq. (1) in units of sigma_ab and eps_ab.   */
/* ------------------------------------------------------------------------ */
#define OR_MAXSP 4
typedef struct {
    int32_t ns;                     /* number of species */
    int32_t pad;
    const int32_t *sp;              /* species of each atom, in the caller's order */
    double eps[OR_MAXSP * OR_MAXSP], sig2[OR_MAXSP * OR_MAXSP];
    double rc2[OR_MAXSP * OR_MAXSP], shift[OR_MAXSP * OR_MAXSP];
} or_mix;

/* f (force on i = f d) and u of pair type k at r^2 = s:
 * f = -(1/r) du/dr = 48 eps (sigma/r)^6 ((sigma/r)^6 - 1/2) / r^2. */
static double pair_fu_mix(const or_mix *mx, int k, double s, double *u)
{
    double rri = mx->sig2[k] / s;
    double rri3 = rri * rri * rri;
    double f = 48.0 * mx->eps[k] * rri3 * (rri3 - 0.5) / s;
    *u = 4.0 * mx->eps[k] * rri3 * (rri3 - 1.0) + mx->shift[k];
    return f;
}

/* ------------------------------------------------------------------------ */
/* Geometry (Sec. 3.1)                                                       */
/* ------------------------------------------------------------------------ */

/* Cells per edge: floor(L / r_n); with even != 0, the largest even number
 * not above that (the rule that reproduces the cell counts of Tables 1, 5). */
int or_cells_per_edge(double L, double rn, int even)
{
    double q = floor(L / rn);
    int G = (int)q;
    if (even) G -= (G & 1);
    return G;
}

/* Periodic wrap into [-L/2, L/2), once per call. */
void or_wrap(int64_t n, double *x, double *y, double *z, double L)
{
    double h = 0.5 * L;
    double *c[3] = {x, y, z};
    for (int a = 0; a < 3; ++a)
        for (int64_t i = 0; i < n; ++i) {
            if (c[a][i] >= h) c[a][i] = c[a][i] - L;
            else if (c[a][i] < -h) c[a][i] = c[a][i] + L;
        }
}

static int cell_coord(double x, double L, double invW, int G)
{
    int c = (int)((x + 0.5 * L) * invW);
    if (c < 0) c = 0;
    if (c > G - 1) c = G - 1;
    return c;
}

/* Scalar cell index of every atom (x fastest), 0-based. */
void or_cell_ids(int64_t n, const double *x, const double *y, const double *z,
                 double L, int G, int32_t *cell)
{
    double invW = (double)G / L;
    for (int64_t i = 0; i < n; ++i) {
        int cx = cell_coord(x[i], L, invW, G);
        int cy = cell_coord(y[i], L, invW, G);
        int cz = cell_coord(z[i], L, invW, G);
        cell[i] = (int32_t)(((int64_t)cz * G + cy) * G + cx);
    }
}

/* Layer assignment (Sec. 3.4): k_c counts the occupants of cell c seen so
 * far in index order, l_i is atom i's 0-based layer.  Then the reorder scan
 * (Sec. 3.5): H_{c,l} = i, read in cell order and, within a cell, in layer
 * order, gives the new storage order.  Outputs: layer[n], order[n] (order[p]
 * = index of the atom stored at position p after reordering), cell_start
 * [N_c + 1] (first position of each cell) and the layer count N_l. */
int or_layers_reorder(int64_t n, const int32_t *cell, int G, int32_t *layer,
                      int64_t *order, int64_t *cell_start, int32_t *n_layers)
{
    int64_t nc = (int64_t)G * G * G;
    int32_t *k = (int32_t *)calloc((size_t)nc, sizeof(int32_t));
    if (!k) return OR_ERR_NOMEM;
    int32_t nl = 0;
    for (int64_t i = 0; i < n; ++i) {
        k[cell[i]] += 1;
        layer[i] = k[cell[i]] - 1;
        if (k[cell[i]] > nl) nl = k[cell[i]];
    }
    int64_t *H = (int64_t *)malloc((size_t)(nc * (nl > 0 ? nl : 1)) * sizeof(int64_t));
    if (!H) { free(k); return OR_ERR_NOMEM; }
    for (int64_t e = 0; e < nc * nl; ++e) H[e] = -1;
    for (int64_t i = 0; i < n; ++i) H[(int64_t)cell[i] * nl + layer[i]] = i;
    int64_t p = 0;
    for (int64_t c = 0; c < nc; ++c) {
        cell_start[c] = p;
        for (int32_t l = 0; l < nl; ++l) {
            int64_t i = H[c * nl + l];
            if (i < 0) break;
            order[p++] = i;
        }
    }
    cell_start[nc] = p;
    *n_layers = nl;
    free(H);
    free(k);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Linked-list cells and the 14-cell half pair list (Sec. 3.2)               */
/* ------------------------------------------------------------------------ */

/* The 14 offsets: the cell itself and the 13 with (oz, oy, ox)
 * lexicographically positive, so every adjacent pair of cells is visited
 * exactly once. */
static const int HALF_OFF[14][3] = {
    {0, 0, 0},
    {1, 0, 0},
    {-1, 1, 0}, {0, 1, 0}, {1, 1, 0},
    {-1, -1, 1}, {0, -1, 1}, {1, -1, 1},
    {-1, 0, 1}, {0, 0, 1}, {1, 0, 1},
    {-1, 1, 1}, {0, 1, 1}, {1, 1, 1},
};  /* {ox, oy, oz} */

typedef struct {
    int64_t n;
    int G;
    int32_t *head;  /* N_c entries, -1 = empty */
    int32_t *next;  /* n entries,  -1 = end   */
} cells_t;

static int build_linked_cells(cells_t *cl, int64_t n, const double *x, const double *y,
                              const double *z, double L, int G)
{
    int64_t nc = (int64_t)G * G * G;
    cl->n = n;
    cl->G = G;
    cl->head = (int32_t *)malloc((size_t)nc * sizeof(int32_t));
    cl->next = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *cell = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!cl->head || !cl->next || !cell) {
        free(cl->head); free(cl->next); free(cell);
        return OR_ERR_NOMEM;
    }
    for (int64_t c = 0; c < nc; ++c) cl->head[c] = -1;
    or_cell_ids(n, x, y, z, L, G, cell);
    for (int64_t i = 0; i < n; ++i) {  /* Sec. 3.2, linked-list assignment */
        cl->next[i] = cl->head[cell[i]];
        cl->head[cell[i]] = (int32_t)i;
    }
    free(cell);
    return OR_OK;
}

static void free_linked_cells(cells_t *cl)
{
    free(cl->head);
    free(cl->next);
}

/* Visit every pair (i', i'') of atoms in the same or adjacent cells once,
 * with the periodic image shift b (in units of L) of i''.  Calls `visit`
 * with the FP64 separation d = r_i' - r_i'' + b and s = |d|^2; the visitor
 * decides what to keep. */
typedef void (*pair_visitor)(void *ctx, int32_t i, int32_t j, const int8_t img[3],
                             const double d[3], double s);

static void half_pairs(const cells_t *cl, const double *x, const double *y, const double *z,
                       double L, pair_visitor visit, void *ctx)
{
    int G = cl->G;
    for (int cz = 0; cz < G; ++cz)
        for (int cy = 0; cy < G; ++cy)
            for (int cx = 0; cx < G; ++cx) {
                int64_t c1 = ((int64_t)cz * G + cy) * G + cx;
                for (int k = 0; k < 14; ++k) {
                    int cc[3] = {cx + HALF_OFF[k][0], cy + HALF_OFF[k][1], cz + HALF_OFF[k][2]};
                    int8_t img[3];
                    double b[3];
                    for (int a = 0; a < 3; ++a) {
                        img[a] = 0;
                        if (cc[a] >= G) { cc[a] -= G; img[a] = -1; }
                        else if (cc[a] < 0) { cc[a] += G; img[a] = 1; }
                        b[a] = img[a] == 0 ? 0.0 : (img[a] > 0 ? L : -L);
                    }
                    int64_t c2 = ((int64_t)cc[2] * G + cc[1]) * G + cc[0];
                    for (int32_t i1 = cl->head[c1]; i1 >= 0; i1 = cl->next[i1]) {
                        for (int32_t i2 = cl->head[c2]; i2 >= 0; i2 = cl->next[i2]) {
                            if (c1 == c2 && !(i1 < i2)) continue;
                            double d[3];
                            d[0] = (x[i1] - x[i2]) + b[0];
                            d[1] = (y[i1] - y[i2]) + b[1];
                            d[2] = (z[i1] - z[i2]) + b[2];
                            double s = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                            visit(ctx, i1, i2, img, d, s);
                        }
                    }
                }
            }
}

typedef struct {
    double rn2;
    int64_t cap, m;
    int32_t *pi, *pj;
    int8_t *img;
} list_ctx;

static void list_visit(void *vctx, int32_t i, int32_t j, const int8_t img[3],
                       const double d[3], double s)
{
    (void)d;
    list_ctx *c = (list_ctx *)vctx;
    if (s < c->rn2) {
        if (c->m < c->cap) {
            c->pi[c->m] = i;
            c->pj[c->m] = j;
            c->img[3 * c->m + 0] = img[0];
            c->img[3 * c->m + 1] = img[1];
            c->img[3 * c->m + 2] = img[2];
        }
        c->m += 1;
    }
}

/* Half neighbour-pair list with r^2 < r_n^2 (Sec. 3.2).  img holds, per pair,
 * the image shift of atom j in units of L (-1, 0, +1 per dimension).
 * Returns the number of pairs found; only the first `cap` are stored. */
int64_t or_pairs_cells(int64_t n, const double *x, const double *y, const double *z,
                       double L, int G, double rn, int64_t cap,
                       int32_t *pi, int32_t *pj, int8_t *img)
{
    if (G < 3) return OR_ERR_BOX_TOO_SMALL;
    cells_t cl;
    if (build_linked_cells(&cl, n, x, y, z, L, G) != OR_OK) return OR_ERR_NOMEM;
    list_ctx c = {rn * rn, cap, 0, pi, pj, img};
    half_pairs(&cl, x, y, z, L, list_visit, &c);
    free_linked_cells(&cl);
    return c.m;
}

/* Brute force: all i < j over all 27 periodic images; r^2 < r_n^2. */
int64_t or_pairs_brute(int64_t n, const double *x, const double *y, const double *z,
                       double L, double rn, int64_t cap,
                       int32_t *pi, int32_t *pj, int8_t *img)
{
    double rn2 = rn * rn;
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j)
            for (int bz = -1; bz <= 1; ++bz)
                for (int by = -1; by <= 1; ++by)
                    for (int bx = -1; bx <= 1; ++bx) {
                        double dx = (x[i] - x[j]) + (bx == 0 ? 0.0 : (bx > 0 ? L : -L));
                        double dy = (y[i] - y[j]) + (by == 0 ? 0.0 : (by > 0 ? L : -L));
                        double dz = (z[i] - z[j]) + (bz == 0 ? 0.0 : (bz > 0 ? L : -L));
                        double s = (dx * dx + dy * dy) + dz * dz;
                        if (s < rn2) {
                            if (m < cap) {
                                pi[m] = (int32_t)i;
                                pj[m] = (int32_t)j;
                                img[3 * m + 0] = (int8_t)bx;
                                img[3 * m + 1] = (int8_t)by;
                                img[3 * m + 2] = (int8_t)bz;
                            }
                            m += 1;
                        }
                    }
    return m;
}

/* ------------------------------------------------------------------------ */
/* Forces                                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    double *fx, *fy, *fz;   /* per-atom force */
    double *ua, *wa;        /* per-atom energy and virial (each pair counted on both atoms) */
    double U, W;            /* totals over pairs */
    int64_t n_inter;        /* pairs inside r_c */
    const or_mix *mix;      /* several species, or NULL */
} force_acc;

static void acc_pair(force_acc *a, int32_t i, int32_t j, const double d[3], double s,
                     double ushift)
{
    double u, f;
    if (a->mix) {
        const int k = a->mix->sp[i] * OR_MAXSP + a->mix->sp[j];
        if (!(s < a->mix->rc2[k])) return;
        f = pair_fu_mix(a->mix, k, s, &u);
    } else {
        f = pair_fu(s, ushift, &u);
    }
    a->fx[i] += f * d[0];
    a->fy[i] += f * d[1];
    a->fz[i] += f * d[2];
    a->fx[j] -= f * d[0];
    a->fy[j] -= f * d[1];
    a->fz[j] -= f * d[2];
    a->U += u;
    a->W += f * s;
    if (a->ua) { a->ua[i] += u; a->ua[j] += u; }
    if (a->wa) { a->wa[i] += f * s; a->wa[j] += f * s; }
    a->n_inter += 1;
}

static void acc_zero(force_acc *a, int64_t n)
{
    memset(a->fx, 0, (size_t)n * sizeof(double));
    memset(a->fy, 0, (size_t)n * sizeof(double));
    memset(a->fz, 0, (size_t)n * sizeof(double));
    if (a->ua) memset(a->ua, 0, (size_t)n * sizeof(double));
    if (a->wa) memset(a->wa, 0, (size_t)n * sizeof(double));
    a->U = 0.0;
    a->W = 0.0;
    a->n_inter = 0;
}

/* Pair-list force loop with Newton's third law (Sec. 3.2): for each stored
 * pair with r^2 < r_c^2, f_i += f d, f_j -= f d, U += u, W += f r^2.
 * With mix (may be NULL) the pair's own cutoff and parameters apply (rc is
 * then the largest cutoff).  The cell and brute-force versions below take
 * mix in the same way.
 * ua/wa (may be NULL) receive per-atom sums with each pair counted on both
 * atoms, so sum(ua) = 2U and sum(wa) = 2W.  out[0] = U, out[1] = W,
 * out[2] = number of pairs inside r_c. */
void or_forces_pairs(int64_t n, const double *x, const double *y, const double *z, double L,
                     int64_t np, const int32_t *pi, const int32_t *pj, const int8_t *img,
                     double rc, double ushift, double *fx, double *fy, double *fz,
                     double *ua, double *wa, double *out, const or_mix *mix)
{
    force_acc a = {fx, fy, fz, ua, wa, 0.0, 0.0, 0, mix};
    acc_zero(&a, n);
    double rc2 = rc * rc;
    for (int64_t m = 0; m < np; ++m) {
        int32_t i = pi[m], j = pj[m];
        double d[3];
        d[0] = (x[i] - x[j]) + (img[3 * m + 0] == 0 ? 0.0 : (img[3 * m + 0] > 0 ? L : -L));
        d[1] = (y[i] - y[j]) + (img[3 * m + 1] == 0 ? 0.0 : (img[3 * m + 1] > 0 ? L : -L));
        d[2] = (z[i] - z[j]) + (img[3 * m + 2] == 0 ? 0.0 : (img[3 * m + 2] > 0 ? L : -L));
        double s = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
        if (s < rc2) acc_pair(&a, i, j, d, s, ushift);
    }
    out[0] = a.U;
    out[1] = a.W;
    out[2] = (double)a.n_inter;
}

typedef struct {
    force_acc *a;
    double rc2, ushift;
} cellforce_ctx;

static void cellforce_visit(void *vctx, int32_t i, int32_t j, const int8_t img[3],
                            const double d[3], double s)
{
    (void)img;
    cellforce_ctx *c = (cellforce_ctx *)vctx;
    if (s < c->rc2) acc_pair(c->a, i, j, d, s, c->ushift);
}

/* Forces straight from the cells, no stored list (the cell method of
 * Sec. 3.1): same enumeration as the half list with r_n = r_c. */
int or_forces_cells(int64_t n, const double *x, const double *y, const double *z, double L,
                    int G, double rc, double ushift, double *fx, double *fy, double *fz,
                    double *ua, double *wa, double *out, const or_mix *mix)
{
    if (G < 3) return OR_ERR_BOX_TOO_SMALL;
    cells_t cl;
    if (build_linked_cells(&cl, n, x, y, z, L, G) != OR_OK) return OR_ERR_NOMEM;
    force_acc a = {fx, fy, fz, ua, wa, 0.0, 0.0, 0, mix};
    acc_zero(&a, n);
    cellforce_ctx c = {&a, rc * rc, ushift};
    half_pairs(&cl, x, y, z, L, cellforce_visit, &c);
    free_linked_cells(&cl);
    out[0] = a.U;
    out[1] = a.W;
    out[2] = (double)a.n_inter;
    return OR_OK;
}

/* Brute-force forces: every i < j over all 27 images. */
void or_forces_brute(int64_t n, const double *x, const double *y, const double *z, double L,
                     double rc, double ushift, double *fx, double *fy, double *fz,
                     double *ua, double *wa, double *out, const or_mix *mix)
{
    force_acc a = {fx, fy, fz, ua, wa, 0.0, 0.0, 0, mix};
    acc_zero(&a, n);
    double rc2 = rc * rc;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j)
            for (int bz = -1; bz <= 1; ++bz)
                for (int by = -1; by <= 1; ++by)
                    for (int bx = -1; bx <= 1; ++bx) {
                        double d[3];
                        d[0] = (x[i] - x[j]) + (bx == 0 ? 0.0 : (bx > 0 ? L : -L));
                        d[1] = (y[i] - y[j]) + (by == 0 ? 0.0 : (by > 0 ? L : -L));
                        d[2] = (z[i] - z[j]) + (bz == 0 ? 0.0 : (bz > 0 ? L : -L));
                        double s = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                        if (s < rc2) acc_pair(&a, (int32_t)i, (int32_t)j, d, s, ushift);
                    }
    out[0] = a.U;
    out[1] = a.W;
    out[2] = (double)a.n_inter;
}

/* Minimum-image shift of a coordinate difference, in units of L.  For a
 * region with L > 2 r_n only one image of a pair can lie within r_n, and it
 * is this one. */
static double min_image_shift(double dd, double L)
{
    if (dd > 0.5 * L) return -L;
    if (dd < -0.5 * L) return L;
    return 0.0;
}

/* Force, energy and virial of selected atoms, each computed on its own over
 * every other atom (minimum image).  Intended for spot checks of large
 * systems.  u and w count each pair once per atom (full-list convention). */
void or_force_on_atoms(int64_t n, const double *x, const double *y, const double *z, double L,
                       double rc, double ushift, int64_t ns, const int64_t *idx,
                       double *fx, double *fy, double *fz, double *u, double *w, int32_t *n_inter)
{
    double rc2 = rc * rc;
    for (int64_t k = 0; k < ns; ++k) {
        int64_t i = idx[k];
        double ax = 0, ay = 0, az = 0, au = 0, aw = 0;
        int32_t cnt = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
            dx = dx + min_image_shift(dx, L);
            dy = dy + min_image_shift(dy, L);
            dz = dz + min_image_shift(dz, L);
            double s = (dx * dx + dy * dy) + dz * dz;
            if (s < rc2) {
                double uu;
                double f = pair_fu(s, ushift, &uu);
                ax += f * dx; ay += f * dy; az += f * dz;
                au += uu; aw += f * s;
                cnt += 1;
            }
        }
        fx[k] = ax; fy[k] = ay; fz[k] = az; u[k] = au; w[k] = aw;
        n_inter[k] = cnt;
    }
}

/* All j != i with r^2 < r_n^2 (minimum image), ascending.  Returns the count;
 * stores at most `cap`. */
int64_t or_neighbors_of_atom(int64_t n, const double *x, const double *y, const double *z,
                             double L, double rn, int64_t i, int64_t cap, int32_t *out)
{
    double rn2 = rn * rn;
    int64_t m = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double dx = x[i] - x[j], dy = y[i] - y[j], dz = z[i] - z[j];
        dx = dx + min_image_shift(dx, L);
        dy = dy + min_image_shift(dy, L);
        dz = dz + min_image_shift(dz, L);
        double s = (dx * dx + dy * dy) + dz * dz;
        if (s < rn2) {
            if (m < cap) out[m] = (int32_t)j;
            m += 1;
        }
    }
    return m;
}

/* ------------------------------------------------------------------------ */
/* The MD loop (Sec. 3.1, steps (a)-(e))                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    double L, rc, shell, dt, ushift;
    int32_t G;            /* cells per edge for r_n = r_c + shell */
    int32_t cell_only;    /* 1: no stored list, forces from cells each step */
    int32_t check_missed; /* 1: count pairs inside r_c absent from the list (slow) */
    int32_t pad;
} or_params;

/* Mutable loop state besides positions/velocities/forces. */
typedef struct {
    double disp;          /* accumulated sum of vmax*dt since the last rebuild */
    int64_t step;
    int64_t n_rebuilds;
    int64_t n_missed;     /* pairs inside r_c absent from the list (check_missed) */
    int32_t rebuild;      /* rebuild due at the next step */
    int32_t pad;
} or_state;

/* Per-step trace record: ke, pe, virial, vmax^2 (totals), pairs in list,
 * rebuilt-this-step flag. */
#define OR_TRACE 6

typedef struct {
    int64_t n;
    double *x, *y, *z, *vx, *vy, *vz, *fx, *fy, *fz;
    const or_params *p;
    or_state *st;
    int64_t cap, np;
    int32_t *pi, *pj;
    int8_t *img;
    double U, W;
    const or_mix *mix;    /* several species, or NULL */
} loop_t;

static int rebuild_list(loop_t *lp)
{
    const or_params *p = lp->p;
    for (;;) {
        int64_t m = or_pairs_cells(lp->n, lp->x, lp->y, lp->z, p->L, p->G, p->rc + p->shell,
                                   lp->cap, lp->pi, lp->pj, lp->img);
        if (m < 0) return (int)m;
        if (m <= lp->cap) { lp->np = m; return OR_OK; }
        int64_t ncap = m + m / 4 + 16;
        int32_t *npi = (int32_t *)realloc(lp->pi, (size_t)ncap * sizeof(int32_t));
        if (npi) lp->pi = npi;
        int32_t *npj = (int32_t *)realloc(lp->pj, (size_t)ncap * sizeof(int32_t));
        if (npj) lp->pj = npj;
        int8_t *nimg = (int8_t *)realloc(lp->img, (size_t)ncap * 3);
        if (nimg) lp->img = nimg;
        if (!npi || !npj || !nimg) return OR_ERR_NOMEM;
        lp->cap = ncap;
    }
}

static int compute_forces(loop_t *lp)
{
    const or_params *p = lp->p;
    double out[3];
    if (p->cell_only) {
        int rc = or_forces_cells(lp->n, lp->x, lp->y, lp->z, p->L, p->G, p->rc, p->ushift,
                                 lp->fx, lp->fy, lp->fz, NULL, NULL, out, lp->mix);
        if (rc != OR_OK) return rc;
    } else {
        or_forces_pairs(lp->n, lp->x, lp->y, lp->z, p->L, lp->np, lp->pi, lp->pj, lp->img,
                        p->rc, p->ushift, lp->fx, lp->fy, lp->fz, NULL, NULL, out, lp->mix);
        if (p->check_missed) {
            /* Every pair inside r_c must be in the list: count pairs inside r_c
             * by brute force; list pairs are a subset with the same r^2, so
             * equal counts mean nothing is missing. */
            double *tx = (double *)malloc((size_t)lp->n * 3 * sizeof(double));
            if (!tx) return OR_ERR_NOMEM;
            double bo[3];
            or_forces_brute(lp->n, lp->x, lp->y, lp->z, p->L, p->rc, p->ushift, tx,
                            tx + lp->n, tx + 2 * lp->n, NULL, NULL, bo, lp->mix);
            lp->st->n_missed += (int64_t)(bo[2] - out[2]);
            free(tx);
        }
    }
    lp->U = out[0];
    lp->W = out[1];
    return OR_OK;
}

/* Step (e): kinetic energy, maximum v^2, and the rebuild decision. */
static void props_and_decide(loop_t *lp, double *rec)
{
    const or_params *p = lp->p;
    double kin = 0.0, vv_max = 0.0;
    for (int64_t i = 0; i < lp->n; ++i) {
        double vv = (lp->vx[i] * lp->vx[i] + lp->vy[i] * lp->vy[i]) + lp->vz[i] * lp->vz[i];
        kin += vv;
        if (vv > vv_max) vv_max = vv;
    }
    if (rec) {
        rec[0] = 0.5 * kin;
        rec[1] = lp->U;
        rec[2] = lp->W;
        rec[3] = vv_max;
        rec[4] = (double)lp->np;
    }
    if (!p->cell_only) {
        lp->st->disp += sqrt(vv_max) * p->dt;
        lp->st->rebuild = lp->st->disp > 0.5 * p->shell;
    }
}

static int loop_init(loop_t *lp, int64_t n, double *x, double *y, double *z, double *vx,
                     double *vy, double *vz, double *fx, double *fy, double *fz,
                     const or_params *p, or_state *st)
{
    if (n < 0 || !(p->L > 0) || !(p->dt > 0) || p->G < 3) return OR_ERR_ARG;
    memset(lp, 0, sizeof(*lp));
    lp->n = n;
    lp->x = x; lp->y = y; lp->z = z;
    lp->vx = vx; lp->vy = vy; lp->vz = vz;
    lp->fx = fx; lp->fy = fy; lp->fz = fz;
    lp->p = p;
    lp->st = st;
    lp->cap = n * 8 + 64;
    lp->pi = (int32_t *)malloc((size_t)lp->cap * sizeof(int32_t));
    lp->pj = (int32_t *)malloc((size_t)lp->cap * sizeof(int32_t));
    lp->img = (int8_t *)malloc((size_t)lp->cap * 3);
    if (!lp->pi || !lp->pj || !lp->img) return OR_ERR_NOMEM;
    return OR_OK;
}

static void loop_free(loop_t *lp)
{
    free(lp->pi);
    free(lp->pj);
    free(lp->img);
}

/* A simulation handle: the loop state lives here between calls, so the list
 * built at a rebuild is the one used until the next rebuild. */
typedef struct {
    loop_t lp;
    or_params p;
    or_state st;
    double *buf;  /* 9 n doubles: x y z vx vy vz fx fy fz */
    or_mix mix;
    int32_t *sp;  /* the mixture's own copy of the species */
} or_sim;

void or_sim_free(or_sim *s)
{
    if (!s) return;
    loop_free(&s->lp);
    free(s->buf);
    free(s->sp);
    free(s);
}

/* Give the atoms species and the species pairs their parameters (a copy is
 * kept), then evaluate the forces of the current state again (the list, built
 * for r_n, stays).  Every cutoff must be at most the r_c of the parameters.
 * Returns 0, or OR_ERR_ARG. */
int or_sim_set_mix(or_sim *s, const or_mix *mx)
{
    const int64_t n = s->lp.n;
    if (mx->ns < 1 || mx->ns > OR_MAXSP) return OR_ERR_ARG;
    for (int k = 0; k < OR_MAXSP * OR_MAXSP; ++k)
        if (mx->rc2[k] > s->p.rc * s->p.rc) return OR_ERR_ARG;
    int32_t *sp = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!sp) return OR_ERR_NOMEM;
    for (int64_t i = 0; i < n; ++i) {
        if (mx->sp[i] < 0 || mx->sp[i] >= mx->ns) { free(sp); return OR_ERR_ARG; }
        sp[i] = mx->sp[i];
    }
    free(s->sp);
    s->sp = sp;
    s->mix = *mx;
    s->mix.sp = sp;
    s->lp.mix = &s->mix;
    return compute_forces(&s->lp);
}

/* Create a simulation from positions/velocities (n x 3, row-major) and run
 * step 0: wrap, bin, build the list, forces, properties and the first
 * rebuild decision (disp = vmax*dt).  rec (may be NULL) gets one trace
 * record.  Returns NULL on failure, with *err set. */
or_sim *or_sim_new(int64_t n, const double *pos, const double *vel, const or_params *p,
                   double *rec, int *err)
{
    or_sim *s = (or_sim *)calloc(1, sizeof(or_sim));
    *err = OR_ERR_NOMEM;
    if (!s) return NULL;
    s->p = *p;
    s->buf = (double *)malloc((size_t)(n > 0 ? n : 1) * 9 * sizeof(double));
    if (!s->buf) { free(s); return NULL; }
    double *b = s->buf;
    int rc = loop_init(&s->lp, n, b, b + n, b + 2 * n, b + 3 * n, b + 4 * n, b + 5 * n,
                       b + 6 * n, b + 7 * n, b + 8 * n, &s->p, &s->st);
    if (rc != OR_OK) { *err = rc; or_sim_free(s); return NULL; }
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            b[a * n + i] = pos[3 * i + a];
            b[(3 + a) * n + i] = vel[3 * i + a];
        }
    loop_t *lp = &s->lp;
    or_wrap(n, lp->x, lp->y, lp->z, p->L);
    if (!p->cell_only) rc = rebuild_list(lp);
    if (rc == OR_OK) rc = compute_forces(lp);
    if (rc != OR_OK) { *err = rc; or_sim_free(s); return NULL; }
    props_and_decide(lp, rec);
    if (rec) rec[5] = 1.0;
    *err = OR_OK;
    return s;
}

/* Advance nsteps leapfrog steps (a)-(e).  trace (may be NULL) receives
 * OR_TRACE doubles per step. */
int or_sim_run(or_sim *s, int64_t nsteps, double *trace)
{
    loop_t *lp = &s->lp;
    const or_params *p = &s->p;
    or_state *st = &s->st;
    const int64_t n = lp->n;
    double *x = lp->x, *y = lp->y, *z = lp->z;
    double *vx = lp->vx, *vy = lp->vy, *vz = lp->vz;
    double *fx = lp->fx, *fy = lp->fy, *fz = lp->fz;
    const double hdt = 0.5 * p->dt;
    int rc = OR_OK;
    for (int64_t t = 0; t < nsteps; ++t) {
        /* (a) half kick, full drift */
        for (int64_t i = 0; i < n; ++i) {
            vx[i] = vx[i] + hdt * fx[i];
            vy[i] = vy[i] + hdt * fy[i];
            vz[i] = vz[i] + hdt * fz[i];
            x[i] = x[i] + p->dt * vx[i];
            y[i] = y[i] + p->dt * vy[i];
            z[i] = z[i] + p->dt * vz[i];
        }
        /* (b) periodic correction and rebuild when due */
        int rebuilt = 0;
        if (p->cell_only) {
            or_wrap(n, x, y, z, p->L);
            rebuilt = 1;
        } else if (st->rebuild) {
            or_wrap(n, x, y, z, p->L);
            st->disp = 0.0;
            st->rebuild = 0;
            st->n_rebuilds += 1;
            rebuilt = 1;
            rc = rebuild_list(lp);
            if (rc != OR_OK) break;
        }
        /* (c) forces */
        rc = compute_forces(lp);
        if (rc != OR_OK) break;
        /* (d) half kick */
        for (int64_t i = 0; i < n; ++i) {
            vx[i] = vx[i] + hdt * fx[i];
            vy[i] = vy[i] + hdt * fy[i];
            vz[i] = vz[i] + hdt * fz[i];
        }
        st->step += 1;
        /* (e) properties, rebuild decision */
        double *rec = trace ? trace + OR_TRACE * t : NULL;
        props_and_decide(lp, rec);
        if (rec) rec[5] = (double)rebuilt;
    }
    return rc;
}

/* Step (f) of the loop (Sec. 3.1), as used during the equilibration period
 * of Sec. 5.1: scale every velocity by one factor so that the kinetic
 * temperature equals T.  With the centre of mass at rest the velocities carry
 * 3 (N - 1) degrees of freedom, so the target is sum v^2 = 3 (N - 1) T.
 * The sum is the plain sequential one.  Returns the factor (1 when there is
 * nothing to scale: N < 2 or every velocity zero). */
double or_sim_adjust_temp(or_sim *s, double temperature)
{
    loop_t *lp = &s->lp;
    const int64_t n = lp->n;
    double vv = 0.0;
    for (int64_t i = 0; i < n; ++i)
        vv += (lp->vx[i] * lp->vx[i] + lp->vy[i] * lp->vy[i]) + lp->vz[i] * lp->vz[i];
    if (n < 2 || !(vv > 0.0)) return 1.0;
    const double fac = sqrt(3.0 * (double)(n - 1) * temperature / vv);
    for (int64_t i = 0; i < n; ++i) {
        lp->vx[i] *= fac;
        lp->vy[i] *= fac;
        lp->vz[i] *= fac;
    }
    return fac;
}

/* Copy out positions, velocities, forces (n x 3, row-major, may be NULL)
 * and the loop state. */
void or_sim_get(const or_sim *s, double *pos, double *vel, double *force, or_state *st)
{
    const loop_t *lp = &s->lp;
    const int64_t n = lp->n;
    for (int64_t i = 0; i < n; ++i) {
        if (pos) { pos[3 * i] = lp->x[i]; pos[3 * i + 1] = lp->y[i]; pos[3 * i + 2] = lp->z[i]; }
        if (vel) { vel[3 * i] = lp->vx[i]; vel[3 * i + 1] = lp->vy[i]; vel[3 * i + 2] = lp->vz[i]; }
        if (force) { force[3 * i] = lp->fx[i]; force[3 * i + 1] = lp->fy[i]; force[3 * i + 2] = lp->fz[i]; }
    }
    if (st) *st = s->st;
}

/* Current pair list (half list, i' before i''), as stored at the last
 * rebuild.  Returns the count; stores at most cap. */
int64_t or_sim_pairs(const or_sim *s, int64_t cap, int32_t *pi, int32_t *pj, int8_t *img)
{
    const loop_t *lp = &s->lp;
    for (int64_t m = 0; m < lp->np && m < cap; ++m) {
        pi[m] = lp->pi[m];
        pj[m] = lp->pj[m];
        img[3 * m] = lp->img[3 * m];
        img[3 * m + 1] = lp->img[3 * m + 1];
        img[3 * m + 2] = lp->img[3 * m + 2];
    }
    return lp->np;
}
