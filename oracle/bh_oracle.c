/*
 * Plain FP64 CPU oracle for Barnes-Hut gravitational potentials on an octree AMR
 * mesh (Lukat & Banerjee, "A GPU accelerated Barnes-Hut Tree Code for FLASH4").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code, header or table with the
 * GPU path: it builds its own octree from the block list, computes every
 * node's moments directly from the node's own cells, and walks each group with
 * a per-cell opening test.  It is written to be checked by eye, not to be fast
 * (OpenMP over independent targets is the only concession).
 *
 * What it computes (paper sections cited; readings of unclear passages noted):
 *
 *  O1 cells   - a leaf block of level L with lower corner lo has edge
 *               Lb = box / (nbase 2^L); cell (i,j,k) has h = Lb/8, centre
 *               lo + (i + 1/2) h and mass rho h^3 (cells act as point masses,
 *               section 2, footnote on "particles").
 *  O2 direct  - phi_i = -G sum_{j != i} m_j / |r_i - r_j|  (Eq. 2 of section 1,
 *               read without its factor 1/2, which belongs to the energy).
 *  O3 nodes   - every node is a cube with centre c and edge l; M = sum m,
 *               X = sum m r / M (the centre-of-mass equation of section 3.2.3,
 *               the centers-of-gravitation kernel), traceless quadrupole about X,
 *               Q = sum m (3 D D^T - |D|^2 I), D = r - X, and
 *               delta = |X - c| (section 2, Eq. THETA2).  M = 0 gives X = c,
 *               Q = 0, delta = 0.
 *  O4 groups  - the cells of each leaf block, in Morton order (x bit lowest),
 *               split into aligned runs of group_cells cells; each group has
 *               its own opening angle theta_g.
 *  O5 MAC     - node n is accepted for group g iff every cell i of g has
 *               d^2 > s^2, d = |r_i - X_n|, s = l (1/theta_g) + delta
 *               (Eq. THETA2 combined with the all() vote of the potential
 *               kernel, section 3.3; equality opens).
 *  O5b        - the variant the paper uses between a node and a region: d is
 *               the smallest distance from X_n to the group's cube.
 *  O6 walk    - depth-first from the root; accepted -> far list, rejected
 *               bottom node (children are cells) -> near list, rejected
 *               internal node -> visit its 8 children.  Zero-mass nodes are
 *               skipped.
 *  O7 sum     - phi_i = -G [ sum_far (M/d + R^T Q R / (2 d^5))
 *                            + sum_{near cells j != i} m_j / |r_i - r_j| ],
 *               R = r_i - X_n, with Neumaier-compensated sums.
 *  O8 accel   - g_i = -grad_i phi_i, the gradient of O7 term by term (an
 *               extension: the paper's method yields the potential only;
 *               forces are the item its section 3.1 writes back next to it).
 *  O9 Ewald   - the periodic Green's function of the appendix (below).
 *  O10 periodic BH - O5-O7 in a periodic box (below).
 *
 * Tree shape: the box is the root (depth 0); log2(nbase) virtual levels lead
 * down to the level-0 blocks; an AMR block of level L sits at depth
 * log2(nbase) + L; a leaf block has 8 octant nodes (4^3 cells each) and 64
 * bottom nodes (2^3 cells each) below it.  Node identity across
 * implementations is the key (depth, ix, iy, iz) of the node's lower corner
 * in units of its own edge.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NB 8
#define NCB 512 /* cells per block */

typedef struct {
    int depth;
    int64_t ix, iy, iz;
    double c[3];
    double l;
    int bottom;     /* 1: children are the 8 cells below */
    int child[8];   /* node ids (internal) */
    int64_t cell[8]; /* canonical cell ids (bottom) */
    double M, X[3], Q[6], delta; /* Q order: xx yy zz xy xz yz */
    double S;                    /* sum m |r - X|^2 (trace of the second moments about X) */
} onode;

typedef struct {
    int n;
    int cap;
    int *v;
} ivec;

typedef struct otree {
    int nblk, nbase, vlev;
    double box_lo[3], box;
    int nleaf;
    int *leaf_of_block; /* block -> leaf ordinal or -1 */
    double *leaf_h;     /* cell edge per leaf */
    int *block_of_leaf;
    int nnodes, capnodes;
    onode *nodes;
    int root;
    /* cells, canonical order leaf*512 + z*64 + y*8 + x */
    int64_t ncells;
    double *cx, *cy, *cz, *cm;
    /* sorted keys for lookup */
    uint64_t *skeys;
    int *sidx;
    /* walk results */
    int group_cells;
    int64_t ngroups;
    ivec *far, *near;
    int64_t *counts; /* [g][4] visited, far, near, marginal */
    /* marginal band of the next walks: |d^2 - s^2| <= tau s^2 + tau_lin s
     * (the linear term bounds rounding that scales with the coordinates, not
     * with s; 0 unless set) */
    double tau_lin;
} otree;

static void ivec_push(ivec *a, int x) {
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 64;
        a->v = (int *)realloc(a->v, sizeof(int) * (size_t)a->cap);
    }
    a->v[a->n++] = x;
}

/* Neumaier compensated summation */
typedef struct { double s, c; } nsum;
static inline void nadd(nsum *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static inline double nval(const nsum *a) { return a->s + a->c; }

uint64_t ot_make_key(int depth, int64_t ix, int64_t iy, int64_t iz) {
    return ((uint64_t)depth << 57) | ((uint64_t)ix << 38) | ((uint64_t)iy << 19) | (uint64_t)iz;
}

static int new_node(otree *t, int depth, int64_t ix, int64_t iy, int64_t iz) {
    if (t->nnodes == t->capnodes) {
        t->capnodes = t->capnodes ? 2 * t->capnodes : 1024;
        t->nodes = (onode *)realloc(t->nodes, sizeof(onode) * (size_t)t->capnodes);
    }
    onode *n = &t->nodes[t->nnodes];
    memset(n, 0, sizeof(*n));
    n->depth = depth;
    n->ix = ix; n->iy = iy; n->iz = iz;
    n->l = t->box / (double)((int64_t)1 << depth);
    n->c[0] = t->box_lo[0] + ((double)ix + 0.5) * n->l;
    n->c[1] = t->box_lo[1] + ((double)iy + 0.5) * n->l;
    n->c[2] = t->box_lo[2] + ((double)iz + 0.5) * n->l;
    for (int o = 0; o < 8; o++) n->child[o] = -1;
    return t->nnodes++;
}

/* in-block node of a leaf block: sub-level 1 = octant (4^3 cells), 2 = bottom (2^3 cells) */
static int build_inblock(otree *t, int leaf, int depth, int64_t ix, int64_t iy, int64_t iz,
                         int sub, int i0, int j0, int k0) {
    int id = new_node(t, depth, ix, iy, iz);
    int half = NB >> (sub + 1); /* cells per edge of each child */
    if (sub == 2) {
        t->nodes[id].bottom = 1;
        for (int o = 0; o < 8; o++) {
            int i = i0 + (o & 1), j = j0 + ((o >> 1) & 1), k = k0 + ((o >> 2) & 1);
            t->nodes[id].cell[o] = (int64_t)leaf * NCB + (int64_t)k * 64 + j * 8 + i;
        }
        return id;
    }
    for (int o = 0; o < 8; o++) {
        int ox = o & 1, oy = (o >> 1) & 1, oz = (o >> 2) & 1;
        int c = build_inblock(t, leaf, depth + 1, 2 * ix + ox, 2 * iy + oy, 2 * iz + oz, sub + 1,
                              i0 + ox * half, j0 + oy * half, k0 + oz * half);
        t->nodes[id].child[o] = c;
    }
    return id;
}

static int build_block(otree *t, const int *child, int b, int depth, int64_t ix, int64_t iy, int64_t iz) {
    if (t->leaf_of_block[b] >= 0) {
        /* the leaf block itself is the sub-level-0 node */
        int leaf = t->leaf_of_block[b];
        int id = new_node(t, depth, ix, iy, iz);
        for (int o = 0; o < 8; o++) {
            int ox = o & 1, oy = (o >> 1) & 1, oz = (o >> 2) & 1;
            int c = build_inblock(t, leaf, depth + 1, 2 * ix + ox, 2 * iy + oy, 2 * iz + oz, 1,
                                  ox * 4, oy * 4, oz * 4);
            t->nodes[id].child[o] = c;
        }
        return id;
    }
    int id = new_node(t, depth, ix, iy, iz);
    for (int o = 0; o < 8; o++) {
        int ox = o & 1, oy = (o >> 1) & 1, oz = (o >> 2) & 1;
        int c = build_block(t, child, child[8 * b + o], depth + 1, 2 * ix + ox, 2 * iy + oy, 2 * iz + oz);
        t->nodes[id].child[o] = c;
    }
    return id;
}

static int build_virtual(otree *t, const int *child, const int *base_at, int depth, int64_t ix, int64_t iy,
                         int64_t iz) {
    if (depth == t->vlev) {
        int b = base_at[(iz * t->nbase + iy) * t->nbase + ix];
        return build_block(t, child, b, depth, ix, iy, iz);
    }
    int id = new_node(t, depth, ix, iy, iz);
    for (int o = 0; o < 8; o++) {
        int ox = o & 1, oy = (o >> 1) & 1, oz = (o >> 2) & 1;
        int c = build_virtual(t, child, base_at, depth + 1, 2 * ix + ox, 2 * iy + oy, 2 * iz + oz);
        t->nodes[id].child[o] = c;
    }
    return id;
}

static uint64_t *g_sort_keys;
static int cmp_by_key(const void *a, const void *b) {
    uint64_t ka = g_sort_keys[*(const int *)a], kb = g_sort_keys[*(const int *)b];
    return ka < kb ? -1 : (ka > kb ? 1 : 0);
}

/* The block list is assumed valid (the product library validates its input;
 * the oracle only reads it). */
otree *ot_create(int nblk, const int *level, const double *lo, const int *parent, const int *child,
                 const unsigned char *is_leaf, const double *box_lo, double box, int nbase) {
    (void)parent;
    otree *t = (otree *)calloc(1, sizeof(otree));
    t->nblk = nblk;
    t->nbase = nbase;
    t->vlev = 0;
    while ((1 << t->vlev) < nbase) t->vlev++;
    for (int d = 0; d < 3; d++) t->box_lo[d] = box_lo[d];
    t->box = box;
    t->leaf_of_block = (int *)malloc(sizeof(int) * (size_t)nblk);
    t->nleaf = 0;
    for (int b = 0; b < nblk; b++) t->leaf_of_block[b] = is_leaf[b] ? t->nleaf++ : -1;
    t->block_of_leaf = (int *)malloc(sizeof(int) * (size_t)(t->nleaf > 0 ? t->nleaf : 1));
    for (int b = 0; b < nblk; b++)
        if (is_leaf[b]) t->block_of_leaf[t->leaf_of_block[b]] = b;
    int *base_at = (int *)malloc(sizeof(int) * (size_t)(nbase * nbase * nbase));
    double e0 = box / nbase;
    for (int b = 0; b < nblk; b++) {
        if (level[b] != 0) continue;
        int ix = (int)llround((lo[3 * b] - box_lo[0]) / e0);
        int iy = (int)llround((lo[3 * b + 1] - box_lo[1]) / e0);
        int iz = (int)llround((lo[3 * b + 2] - box_lo[2]) / e0);
        base_at[(iz * nbase + iy) * nbase + ix] = b;
    }
    t->root = build_virtual(t, child, base_at, 0, 0, 0, 0);
    free(base_at);
    /* cell geometry (O1) */
    t->ncells = (int64_t)t->nleaf * NCB;
    t->cx = (double *)malloc(sizeof(double) * (size_t)t->ncells);
    t->cy = (double *)malloc(sizeof(double) * (size_t)t->ncells);
    t->cz = (double *)malloc(sizeof(double) * (size_t)t->ncells);
    t->cm = (double *)calloc((size_t)t->ncells, sizeof(double));
    t->leaf_h = (double *)malloc(sizeof(double) * (size_t)(t->nleaf > 0 ? t->nleaf : 1));
    for (int f = 0; f < t->nleaf; f++) {
        int b = t->block_of_leaf[f];
        double Lb = box / ((double)nbase * (double)((int64_t)1 << level[b]));
        double h = Lb / NB;
        t->leaf_h[f] = h;
        for (int k = 0; k < NB; k++)
            for (int j = 0; j < NB; j++)
                for (int i = 0; i < NB; i++) {
                    int64_t c = (int64_t)f * NCB + k * 64 + j * 8 + i;
                    t->cx[c] = lo[3 * b] + (i + 0.5) * h;
                    t->cy[c] = lo[3 * b + 1] + (j + 0.5) * h;
                    t->cz[c] = lo[3 * b + 2] + (k + 0.5) * h;
                }
    }
    /* key lookup table */
    t->skeys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)t->nnodes);
    t->sidx = (int *)malloc(sizeof(int) * (size_t)t->nnodes);
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)t->nnodes);
    for (int n = 0; n < t->nnodes; n++) {
        keys[n] = ot_make_key(t->nodes[n].depth, t->nodes[n].ix, t->nodes[n].iy, t->nodes[n].iz);
        t->sidx[n] = n;
    }
    g_sort_keys = keys;
    qsort(t->sidx, (size_t)t->nnodes, sizeof(int), cmp_by_key);
    for (int n = 0; n < t->nnodes; n++) t->skeys[n] = keys[t->sidx[n]];
    free(keys);
    return t;
}

static void free_walk(otree *t) {
    if (t->far) {
        for (int64_t g = 0; g < t->ngroups; g++) { free(t->far[g].v); free(t->near[g].v); }
        free(t->far); free(t->near); free(t->counts);
    }
    t->far = t->near = NULL;
    t->counts = NULL;
    t->ngroups = 0;
}

void ot_destroy(otree *t) {
    if (!t) return;
    free_walk(t);
    free(t->leaf_of_block); free(t->block_of_leaf); free(t->leaf_h); free(t->nodes);
    free(t->cx); free(t->cy); free(t->cz); free(t->cm);
    free(t->skeys); free(t->sidx);
    free(t);
}

int ot_num_nodes(const otree *t) { return t->nnodes; }
int64_t ot_num_cells(const otree *t) { return t->ncells; }
int ot_num_leaves(const otree *t) { return t->nleaf; }

/* node i's key, depth, bottom flag, centre and edge */
void ot_node_info(const otree *t, uint64_t *key, int *depth, int *bottom, double *centre, double *edge) {
    for (int n = 0; n < t->nnodes; n++) {
        const onode *a = &t->nodes[n];
        key[n] = ot_make_key(a->depth, a->ix, a->iy, a->iz);
        depth[n] = a->depth;
        bottom[n] = a->bottom;
        for (int d = 0; d < 3; d++) centre[3 * n + d] = a->c[d];
        edge[n] = a->l;
    }
}

int ot_lookup(const otree *t, uint64_t key) {
    int lo = 0, hi = t->nnodes - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (t->skeys[mid] == key) return t->sidx[mid];
        if (t->skeys[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* O1: masses from densities (rho in caller layout [leaf][z][y][x]) */
void ot_set_density(otree *t, const double *rho) {
    for (int f = 0; f < t->nleaf; f++) {
        double h = t->leaf_h[f];
        double vol = h * h * h;
        for (int c = 0; c < NCB; c++) t->cm[(int64_t)f * NCB + c] = rho[(int64_t)f * NCB + c] * vol;
    }
}

/* enumerate the cells below node n */
typedef void (*cell_fn)(const otree *, int64_t, void *);
static void for_cells(const otree *t, int n, cell_fn fn, void *ctx) {
    const onode *a = &t->nodes[n];
    if (a->bottom) {
        for (int o = 0; o < 8; o++) fn(t, a->cell[o], ctx);
        return;
    }
    for (int o = 0; o < 8; o++) for_cells(t, a->child[o], fn, ctx);
}

typedef struct { nsum m, sx, sy, sz; } acc1;
static void acc1_fn(const otree *t, int64_t c, void *p) {
    acc1 *a = (acc1 *)p;
    double m = t->cm[c];
    nadd(&a->m, m);
    nadd(&a->sx, m * t->cx[c]);
    nadd(&a->sy, m * t->cy[c]);
    nadd(&a->sz, m * t->cz[c]);
}
typedef struct { double X[3]; nsum q[6]; nsum s; } acc2;
static void acc2_fn(const otree *t, int64_t c, void *p) {
    acc2 *a = (acc2 *)p;
    double m = t->cm[c];
    double dx = t->cx[c] - a->X[0], dy = t->cy[c] - a->X[1], dz = t->cz[c] - a->X[2];
    double r2 = dx * dx + dy * dy + dz * dz;
    nadd(&a->q[0], m * (3.0 * dx * dx - r2));
    nadd(&a->q[1], m * (3.0 * dy * dy - r2));
    nadd(&a->q[2], m * (3.0 * dz * dz - r2));
    nadd(&a->q[3], m * (3.0 * dx * dy));
    nadd(&a->q[4], m * (3.0 * dx * dz));
    nadd(&a->q[5], m * (3.0 * dy * dz));
    nadd(&a->s, m * r2);
}

/* O3: every node's moments straight from its own cells */
void ot_moments(otree *t) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int n = 0; n < t->nnodes; n++) {
        onode *a = &t->nodes[n];
        acc1 s1;
        memset(&s1, 0, sizeof(s1));
        for_cells(t, n, acc1_fn, &s1);
        double M = nval(&s1.m);
        a->M = M;
        if (M > 0.0) {
            a->X[0] = nval(&s1.sx) / M;
            a->X[1] = nval(&s1.sy) / M;
            a->X[2] = nval(&s1.sz) / M;
            acc2 s2;
            memset(&s2, 0, sizeof(s2));
            for (int d = 0; d < 3; d++) s2.X[d] = a->X[d];
            for_cells(t, n, acc2_fn, &s2);
            for (int q = 0; q < 6; q++) a->Q[q] = nval(&s2.q[q]);
            a->S = nval(&s2.s);
            double ex = a->X[0] - a->c[0], ey = a->X[1] - a->c[1], ez = a->X[2] - a->c[2];
            a->delta = sqrt(ex * ex + ey * ey + ez * ez);
        } else {
            for (int d = 0; d < 3; d++) a->X[d] = a->c[d];
            for (int q = 0; q < 6; q++) a->Q[q] = 0.0;
            a->delta = 0.0;
            a->S = 0.0;
        }
    }
}

/* S of every node (see onode), by node id */
void ot_get_trace(const otree *t, double *S) {
    for (int n = 0; n < t->nnodes; n++) S[n] = t->nodes[n].S;
}

void ot_get_moments(const otree *t, double *M, double *X, double *Q, double *delta) {
    for (int n = 0; n < t->nnodes; n++) {
        const onode *a = &t->nodes[n];
        M[n] = a->M;
        for (int d = 0; d < 3; d++) X[3 * n + d] = a->X[d];
        for (int q = 0; q < 6; q++) Q[6 * n + q] = a->Q[q];
        delta[n] = a->delta;
    }
}

/* Morton decode of a 9-bit in-block index: bit 3p is x, 3p+1 is y, 3p+2 is z */
static void morton_decode(int m, int *i, int *j, int *k) {
    *i = *j = *k = 0;
    for (int p = 0; p < 3; p++) {
        *i |= ((m >> (3 * p)) & 1) << p;
        *j |= ((m >> (3 * p + 1)) & 1) << p;
        *k |= ((m >> (3 * p + 2)) & 1) << p;
    }
}

/* canonical cell ids of group g (O4) */
static void group_cells_of(const otree *t, int64_t g, int G, int64_t *out) {
    (void)t;
    int per = NCB / G;
    int64_t leaf = g / per;
    int s = (int)(g % per);
    for (int q = 0; q < G; q++) {
        int i, j, k;
        morton_decode(s * G + q, &i, &j, &k);
        out[q] = leaf * NCB + k * 64 + j * 8 + i;
    }
}

typedef struct {
    const otree *t;
    const int64_t *cells;
    int G;
    double inv_theta;
    double tau, tau_lin;
    ivec *far, *near;
    int64_t visited, marginal;
    int mac;            /* 0: every cell of the group (O5); 1: the group's cube (O5b) */
    double box[6];      /* O5b: lower and upper corner of the group's cube */
} walkctx;

/* O5b (the paper's test between a node and a whole region, section 3.2
 * "Find Essential Nodes" and Fig. opening_angles2): d_c is the smallest
 * distance from the node's centre of mass to the group's cube, whose faces are
 * the outer faces of its cells; the node is accepted iff d_c^2 > s^2. */
static void group_cube(const otree *t, const int64_t *cells, int G, double *box) {
    int64_t leaf = cells[0] / NCB;
    double h = t->leaf_h[leaf];
    for (int d = 0; d < 3; d++) { box[d] = INFINITY; box[3 + d] = -INFINITY; }
    for (int q = 0; q < G; q++) {
        double p[3] = {t->cx[cells[q]], t->cy[cells[q]], t->cz[cells[q]]};
        for (int d = 0; d < 3; d++) {
            if (p[d] - 0.5 * h < box[d]) box[d] = p[d] - 0.5 * h;
            if (p[d] + 0.5 * h > box[3 + d]) box[3 + d] = p[d] + 0.5 * h;
        }
    }
}

/* O5 + O6 */
static void walk_node(walkctx *w, int n) {
    const otree *t = w->t;
    const onode *a = &t->nodes[n];
    if (a->M == 0.0) return;
    w->visited++;
    double s = a->l * w->inv_theta + a->delta;
    double s2 = s * s;
    int accept = 1;
    double dmin2 = INFINITY;
    if (w->mac == 1) {
        double g[3];
        for (int d = 0; d < 3; d++) {
            double below = w->box[d] - a->X[d], above = a->X[d] - w->box[3 + d];
            g[d] = below > 0.0 ? below : (above > 0.0 ? above : 0.0);
        }
        dmin2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        accept = dmin2 > s2;
    } else {
        for (int q = 0; q < w->G; q++) {
            int64_t c = w->cells[q];
            double dx = t->cx[c] - a->X[0];
            double dy = t->cy[c] - a->X[1];
            double dz = t->cz[c] - a->X[2];
            double d2 = dx * dx + dy * dy + dz * dz;
            if (!(d2 > s2)) accept = 0;
            if (d2 < dmin2) dmin2 = d2;
        }
    }
    if (fabs(dmin2 - s2) <= w->tau * s2 + w->tau_lin * s) w->marginal++;
    if (accept) {
        ivec_push(w->far, n);
    } else if (a->bottom) {
        ivec_push(w->near, n);
    } else {
        for (int o = 0; o < 8; o++) walk_node(w, a->child[o]);
    }
}

/* Walk every group; theta_group[g] per group (canonical group order:
 * leaf-major, then Morton run).  Returns the number of groups. */
int64_t ot_walk_mac(otree *t, int group_cells, const double *theta_group, double tau, int mac) {
    free_walk(t);
    int G = group_cells;
    t->group_cells = G;
    t->ngroups = (int64_t)t->nleaf * (NCB / G);
    t->far = (ivec *)calloc((size_t)t->ngroups, sizeof(ivec));
    t->near = (ivec *)calloc((size_t)t->ngroups, sizeof(ivec));
    t->counts = (int64_t *)calloc((size_t)t->ngroups * 4, sizeof(int64_t));
#pragma omp parallel
    {
        int64_t *cells = (int64_t *)malloc(sizeof(int64_t) * (size_t)G);
#pragma omp for schedule(dynamic, 4)
        for (int64_t g = 0; g < t->ngroups; g++) {
            group_cells_of(t, g, G, cells);
            walkctx w;
            w.t = t; w.cells = cells; w.G = G;
            w.inv_theta = 1.0 / theta_group[g];
            w.tau = tau;
            w.tau_lin = t->tau_lin;
            w.far = &t->far[g]; w.near = &t->near[g];
            w.visited = 0; w.marginal = 0;
            w.mac = mac;
            if (mac == 1) group_cube(t, cells, G, w.box);
            walk_node(&w, t->root);
            t->counts[4 * g + 0] = w.visited;
            t->counts[4 * g + 1] = t->far[g].n;
            t->counts[4 * g + 2] = t->near[g].n;
            t->counts[4 * g + 3] = w.marginal;
        }
        free(cells);
    }
    return t->ngroups;
}

int64_t ot_walk(otree *t, int group_cells, const double *theta_group, double tau) {
    return ot_walk_mac(t, group_cells, theta_group, tau, 0);
}

void ot_walk_sizes(const otree *t, int64_t *total_far, int64_t *total_near) {
    int64_t a = 0, b = 0;
    for (int64_t g = 0; g < t->ngroups; g++) { a += t->far[g].n; b += t->near[g].n; }
    *total_far = a;
    *total_near = b;
}

void ot_walk_export(const otree *t, int64_t *far_off, uint64_t *far_keys, int64_t *near_off, uint64_t *near_keys,
                    int64_t *counts) {
    int64_t a = 0, b = 0;
    for (int64_t g = 0; g < t->ngroups; g++) {
        far_off[g] = a;
        near_off[g] = b;
        for (int q = 0; q < t->far[g].n; q++) {
            const onode *n = &t->nodes[t->far[g].v[q]];
            far_keys[a++] = ot_make_key(n->depth, n->ix, n->iy, n->iz);
        }
        for (int q = 0; q < t->near[g].n; q++) {
            const onode *n = &t->nodes[t->near[g].v[q]];
            near_keys[b++] = ot_make_key(n->depth, n->ix, n->iy, n->iz);
        }
    }
    far_off[t->ngroups] = a;
    near_off[t->ngroups] = b;
    memcpy(counts, t->counts, sizeof(int64_t) * 4 * (size_t)t->ngroups);
}

/* O7 for one group given its lists (node ids).  phi is indexed by canonical
 * cell id, or by the cell's position in the group when local != 0. */
static void sum_group_to(const otree *t, int64_t g, int G, const int *far, int nfar, const int *near, int nnear,
                         double Gc, int order, double *phi, int64_t *cells, int local) {
    group_cells_of(t, g, G, cells);
    for (int q = 0; q < G; q++) {
        int64_t i = cells[q];
        double xi = t->cx[i], yi = t->cy[i], zi = t->cz[i];
        nsum acc = {0.0, 0.0};
        for (int f = 0; f < nfar; f++) {
            const onode *a = &t->nodes[far[f]];
            double rx = xi - a->X[0], ry = yi - a->X[1], rz = zi - a->X[2];
            double d2 = rx * rx + ry * ry + rz * rz;
            double d = sqrt(d2);
            double rqr = a->Q[0] * rx * rx + a->Q[1] * ry * ry + a->Q[2] * rz * rz
                         + 2.0 * (a->Q[3] * rx * ry + a->Q[4] * rx * rz + a->Q[5] * ry * rz);
            nadd(&acc, a->M / d);
            if (order >= 2) nadd(&acc, rqr / (2.0 * d2 * d2 * d));
        }
        for (int b = 0; b < nnear; b++) {
            const onode *a = &t->nodes[near[b]];
            for (int o = 0; o < 8; o++) {
                int64_t j = a->cell[o];
                if (j == i) continue;
                double rx = xi - t->cx[j], ry = yi - t->cy[j], rz = zi - t->cz[j];
                nadd(&acc, t->cm[j] / sqrt(rx * rx + ry * ry + rz * rz));
            }
        }
        phi[local ? q : i] = -Gc * nval(&acc);
    }
}

static void sum_group(const otree *t, int64_t g, int G, const int *far, int nfar, const int *near, int nnear,
                      double Gc, int order, double *phi, int64_t *cells) {
    sum_group_to(t, g, G, far, nfar, near, nnear, Gc, order, phi, cells, 0);
}

/* O7 using the lists of the last ot_walk; phi in caller layout.
 * order 2 = monopole + quadrupole (the method), 0 = monopole only (the
 * paper's own far field, kept for the convergence-order checks). */
void ot_potential(const otree *t, double Gc, int order, double *phi) {
    int G = t->group_cells;
#pragma omp parallel
    {
        int64_t *cells = (int64_t *)malloc(sizeof(int64_t) * (size_t)G);
#pragma omp for schedule(dynamic, 4)
        for (int64_t g = 0; g < t->ngroups; g++)
            sum_group(t, g, G, t->far[g].v, t->far[g].n, t->near[g].v, t->near[g].n, Gc, order, phi, cells);
        free(cells);
    }
}

/* O7 on externally supplied lists (node keys, CSR per group): evaluates
 * another implementation's interaction lists in FP64.  Returns 0, or -1 if a
 * key names no node, or -2 if a near key is not a bottom node. */
int ot_potential_lists(const otree *t, int group_cells, const int64_t *far_off, const uint64_t *far_keys,
                       const int64_t *near_off, const uint64_t *near_keys, double Gc, int order, double *phi) {
    int G = group_cells;
    int64_t ng = (int64_t)t->nleaf * (NCB / G);
    int err = 0;
#pragma omp parallel
    {
        int64_t *cells = (int64_t *)malloc(sizeof(int64_t) * (size_t)G);
        int *fl = NULL, *nl = NULL;
        int fcap = 0, ncap = 0;
#pragma omp for schedule(dynamic, 4)
        for (int64_t g = 0; g < ng; g++) {
            int nf = (int)(far_off[g + 1] - far_off[g]);
            int nn = (int)(near_off[g + 1] - near_off[g]);
            if (nf > fcap) { fcap = nf; fl = (int *)realloc(fl, sizeof(int) * (size_t)fcap); }
            if (nn > ncap) { ncap = nn; nl = (int *)realloc(nl, sizeof(int) * (size_t)ncap); }
            int bad = 0;
            for (int q = 0; q < nf; q++) {
                fl[q] = ot_lookup(t, far_keys[far_off[g] + q]);
                if (fl[q] < 0) bad = -1;
            }
            for (int q = 0; q < nn; q++) {
                nl[q] = ot_lookup(t, near_keys[near_off[g] + q]);
                if (nl[q] < 0) bad = -1;
                else if (!t->nodes[nl[q]].bottom) bad = -2;
            }
            if (bad) {
#pragma omp critical
                err = bad;
                continue;
            }
            sum_group(t, g, G, fl, nf, nl, nn, Gc, order, phi, cells);
        }
        free(fl); free(nl); free(cells);
    }
    return err;
}

/* O5-O7 for a subset of groups only (sampled checks on large grids):
 * counts[4 * q + ...] as in ot_walk for groups[q]; phi[q * G + c] for the
 * group's c-th cell in Morton order.  theta_group is indexed by canonical
 * group id, as in ot_walk. */
void ot_solve_groups_mac(const otree *t, int group_cells, const double *theta_group, const int64_t *groups,
                         int64_t n, double tau, double Gc, int order, int mac, int64_t *counts, double *phi) {
    int G = group_cells;
#pragma omp parallel
    {
        int64_t *cells = (int64_t *)malloc(sizeof(int64_t) * (size_t)G);
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < n; q++) {
            int64_t g = groups[q];
            group_cells_of(t, g, G, cells);
            ivec far = {0, 0, NULL}, near = {0, 0, NULL};
            walkctx w;
            w.t = t; w.cells = cells; w.G = G;
            w.inv_theta = 1.0 / theta_group[g];
            w.tau = tau;
            w.tau_lin = t->tau_lin;
            w.far = &far; w.near = &near;
            w.visited = 0; w.marginal = 0;
            w.mac = mac;
            if (mac == 1) group_cube(t, cells, G, w.box);
            walk_node(&w, t->root);
            counts[4 * q + 0] = w.visited;
            counts[4 * q + 1] = far.n;
            counts[4 * q + 2] = near.n;
            counts[4 * q + 3] = w.marginal;
            sum_group_to(t, g, G, far.v, far.n, near.v, near.n, Gc, order, phi + q * G, cells, 1);
            free(far.v);
            free(near.v);
        }
        free(cells);
    }
}

void ot_solve_groups(const otree *t, int group_cells, const double *theta_group, const int64_t *groups, int64_t n,
                     double tau, double Gc, int order, int64_t *counts, double *phi) {
    ot_solve_groups_mac(t, group_cells, theta_group, groups, n, tau, Gc, order, 0, counts, phi);
}

/* O2 for selected targets (canonical cell ids) */
void ot_direct(const otree *t, const int64_t *targets, int64_t ntargets, double Gc, double *phi) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t q = 0; q < ntargets; q++) {
        int64_t i = targets[q];
        double xi = t->cx[i], yi = t->cy[i], zi = t->cz[i];
        nsum acc = {0.0, 0.0};
        for (int64_t j = 0; j < t->ncells; j++) {
            if (j == i) continue;
            double rx = xi - t->cx[j], ry = yi - t->cy[j], rz = zi - t->cz[j];
            nadd(&acc, t->cm[j] / sqrt(rx * rx + ry * ry + rz * rz));
        }
        phi[q] = -Gc * nval(&acc);
    }
}

/* cell geometry as the oracle sees it (for tests) */
void ot_cells(const otree *t, double *x, double *y, double *z, double *m) {
    memcpy(x, t->cx, sizeof(double) * (size_t)t->ncells);
    memcpy(y, t->cy, sizeof(double) * (size_t)t->ncells);
    memcpy(z, t->cz, sizeof(double) * (size_t)t->ncells);
    memcpy(m, t->cm, sizeof(double) * (size_t)t->ncells);
}

/*
 * O8 accelerations g = -grad phi (beyond the paper, whose method computes
 * the potential only): the gradient of O7 taken term by term with respect to
 * the target position r_i.  For a far node with R = r_i - X, d = |R|:
 *   d/dr (M / d)                  = -M R / d^3
 *   d/dr (R^T Q R / (2 d^5))      =  Q R / d^5 - (5/2) (R^T Q R) R / d^7
 * so g_i += G [ Q R / d^5 - (M / d^3 + (5/2) R^T Q R / d^7) R ]  (order 2;
 * order 0 keeps the monopole part), and for a near cell j != i
 *   g_i -= G m_j (r_i - r_j) / |r_i - r_j|^3.
 * Each component is a Neumaier sum; acc is [..][3].
 */
static void accel_group_to(const otree *t, int64_t g, int G, const int *far, int nfar, const int *near, int nnear,
                           double Gc, int order, double *acc, int64_t *cells, int local) {
    group_cells_of(t, g, G, cells);
    for (int q = 0; q < G; q++) {
        int64_t i = cells[q];
        double xi = t->cx[i], yi = t->cy[i], zi = t->cz[i];
        nsum ax = {0.0, 0.0}, ay = {0.0, 0.0}, az = {0.0, 0.0};
        for (int f = 0; f < nfar; f++) {
            const onode *a = &t->nodes[far[f]];
            double rx = xi - a->X[0], ry = yi - a->X[1], rz = zi - a->X[2];
            double d2 = rx * rx + ry * ry + rz * rz;
            double d = sqrt(d2);
            double d3 = d2 * d;
            double cx = -a->M / d3 * rx, cy = -a->M / d3 * ry, cz = -a->M / d3 * rz;
            if (order >= 2) {
                /* Q R with Q in the order xx yy zz xy xz yz */
                double qx = a->Q[0] * rx + a->Q[3] * ry + a->Q[4] * rz;
                double qy = a->Q[3] * rx + a->Q[1] * ry + a->Q[5] * rz;
                double qz = a->Q[4] * rx + a->Q[5] * ry + a->Q[2] * rz;
                double rqr = rx * qx + ry * qy + rz * qz;
                double d5 = d3 * d2, d7 = d5 * d2;
                cx += qx / d5 - 2.5 * rqr / d7 * rx;
                cy += qy / d5 - 2.5 * rqr / d7 * ry;
                cz += qz / d5 - 2.5 * rqr / d7 * rz;
            }
            nadd(&ax, cx);
            nadd(&ay, cy);
            nadd(&az, cz);
        }
        for (int b = 0; b < nnear; b++) {
            const onode *a = &t->nodes[near[b]];
            for (int o = 0; o < 8; o++) {
                int64_t j = a->cell[o];
                if (j == i) continue;
                double rx = xi - t->cx[j], ry = yi - t->cy[j], rz = zi - t->cz[j];
                double d2 = rx * rx + ry * ry + rz * rz;
                double w = t->cm[j] / (d2 * sqrt(d2));
                nadd(&ax, -w * rx);
                nadd(&ay, -w * ry);
                nadd(&az, -w * rz);
            }
        }
        int64_t o = local ? q : i;
        acc[3 * o + 0] = Gc * nval(&ax);
        acc[3 * o + 1] = Gc * nval(&ay);
        acc[3 * o + 2] = Gc * nval(&az);
    }
}

/* O8 with the lists of the last ot_walk; acc in caller layout [cell][3]. */
void ot_accel(const otree *t, double Gc, int order, double *acc) {
    int G = t->group_cells;
#pragma omp parallel
    {
        int64_t *cells = (int64_t *)malloc(sizeof(int64_t) * (size_t)G);
#pragma omp for schedule(dynamic, 4)
        for (int64_t g = 0; g < t->ngroups; g++)
            accel_group_to(t, g, G, t->far[g].v, t->far[g].n, t->near[g].v, t->near[g].n, Gc, order, acc, cells, 0);
        free(cells);
    }
}

/* O5, O6 and O8 for a subset of groups: counts as in ot_solve_groups,
 * acc[(q * G + c) * 3 + k] for the group's c-th cell in Morton order. */
void ot_solve_groups_accel(const otree *t, int group_cells, const double *theta_group, const int64_t *groups,
                           int64_t n, double tau, double Gc, int order, int64_t *counts, double *acc) {
    int G = group_cells;
#pragma omp parallel
    {
        int64_t *cells = (int64_t *)malloc(sizeof(int64_t) * (size_t)G);
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < n; q++) {
            int64_t g = groups[q];
            group_cells_of(t, g, G, cells);
            ivec far = {0, 0, NULL}, near = {0, 0, NULL};
            walkctx w;
            w.t = t; w.cells = cells; w.G = G;
            w.inv_theta = 1.0 / theta_group[g];
            w.tau = tau;
            w.tau_lin = t->tau_lin;
            w.far = &far; w.near = &near;
            w.visited = 0; w.marginal = 0;
            w.mac = 0;
            walk_node(&w, t->root);
            counts[4 * q + 0] = w.visited;
            counts[4 * q + 1] = far.n;
            counts[4 * q + 2] = near.n;
            counts[4 * q + 3] = w.marginal;
            accel_group_to(t, g, G, far.v, far.n, near.v, near.n, Gc, order, acc + 3 * q * G, cells, 1);
            free(far.v);
            free(near.v);
        }
        free(cells);
    }
}

/* Exact acceleration of the direct sum at selected cells: -G sum_{j != i}
 * m_j (r_i - r_j) / |r_i - r_j|^3, acc[q][3]. */
void ot_direct_accel(const otree *t, const int64_t *targets, int64_t ntargets, double Gc, double *acc) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t q = 0; q < ntargets; q++) {
        int64_t i = targets[q];
        double xi = t->cx[i], yi = t->cy[i], zi = t->cz[i];
        nsum ax = {0.0, 0.0}, ay = {0.0, 0.0}, az = {0.0, 0.0};
        for (int64_t j = 0; j < t->ncells; j++) {
            if (j == i) continue;
            double rx = xi - t->cx[j], ry = yi - t->cy[j], rz = zi - t->cz[j];
            double d2 = rx * rx + ry * ry + rz * rz;
            double w = t->cm[j] / (d2 * sqrt(d2));
            nadd(&ax, -w * rx);
            nadd(&ay, -w * ry);
            nadd(&az, -w * rz);
        }
        acc[3 * q + 0] = Gc * nval(&ax);
        acc[3 * q + 1] = Gc * nval(&ay);
        acc[3 * q + 2] = Gc * nval(&az);
    }
}

/* Direct-sum potential at arbitrary points p[q][3], leaving out cell
 * exclude[q] (if >= 0): the reference for finite-difference checks. */
void ot_direct_at(const otree *t, const double *p, const int64_t *exclude, int64_t n, double Gc, double *phi) {
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t q = 0; q < n; q++) {
        nsum acc = {0.0, 0.0};
        for (int64_t j = 0; j < t->ncells; j++) {
            if (j == exclude[q]) continue;
            double rx = p[3 * q] - t->cx[j], ry = p[3 * q + 1] - t->cy[j], rz = p[3 * q + 2] - t->cz[j];
            nadd(&acc, t->cm[j] / sqrt(rx * rx + ry * ry + rz * rz));
        }
        phi[q] = -Gc * nval(&acc);
    }
}

/*
 * O9 periodic boundaries (appendix "Periodic boundaries"): the potential of a
 * unit mass in a cubic box of side L repeated in all three directions, with
 * the mean density removed, split with the error function into a short-range
 * sum over images and a long-range sum over wave vectors (Ewald):
 *   psi(r) = sum_n erfc(a |r + nL|) / |r + nL|
 *          + 1/(pi L) sum_{m != 0} exp(-pi^2 |m|^2 / (a L)^2) / |m|^2 cos(2 pi m.r / L)
 *          - pi / (a^2 L^3),
 * independent of the splitting constant a.  D(r) = psi(r) - 1/|r| is smooth
 * near r = 0, with D(0) the self term psi_0.  Sums run over |n_i| <= nreal and
 * 0 < |m_i| <= nrecip (each component).
 */
/* Adds the value, gradient and Hessian (order xx yy zz xy xz yz) of a radial
 * function f(|p|) given f, f' and f'' at d = |p| > 0. */
static void add_radial(const double *p, double d, double f, double f1, double f2, nsum *s, nsum *g, nsum *h) {
    nadd(s, f);
    for (int k = 0; k < 3; k++) nadd(&g[k], f1 * p[k] / d);
    if (!h) return;
    const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
    for (int q = 0; q < 6; q++) {
        double pp = p[ia[q]] * p[ib[q]] / (d * d);
        nadd(&h[q], f2 * pp + f1 * ((ia[q] == ib[q] ? 1.0 : 0.0) - pp) / d);
    }
}

static void ewald_at(double L, double a, int nreal, int nrecip, const double *r, double *D, double *g, double *H) {
    const double sqpi = 1.7724538509055160273;
    const double c = 2.0 * a / sqpi;
    double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    nsum s = {0.0, 0.0}, gs[3], hs[6];
    memset(gs, 0, sizeof(gs));
    memset(hs, 0, sizeof(hs));
    /* image n = 0 minus 1/r: g(r) = -erf(a r)/r, a smooth even function.
     * Near 0 by its series, g = -c sum_k a_k u^k, u = (a r)^2,
     * a_k = (-1)^k / (k! (2k + 1)), with grad g = G1 r and
     * Hessian G1 I + G2 r r^T (G1 = g'/r, G2 = G1'/r); terms to u^7 leave
     * below 1e-16 for a r < 0.1.  Elsewhere from erf directly. */
    if (a * rr < 0.1) {
        double u = a * a * rr * rr;
        double gv = 0.0, g1 = 0.0, g2 = 0.0;
        double ak = 1.0, uk = 1.0, uk1 = 1.0, uk2 = 1.0;  /* (-1)^k / k!, u^k, u^(k-1), u^(k-2) */
        for (int k = 0; k <= 7; k++) {
            if (k > 0) ak *= -1.0 / k;
            double coef = ak / (2 * k + 1);
            gv += coef * uk;
            if (k >= 1) {
                g1 += coef * 2.0 * k * a * a * uk1;
                uk1 *= u;
            }
            if (k >= 2) {
                g2 += coef * 2.0 * k * (2.0 * k - 2.0) * a * a * a * a * uk2;
                uk2 *= u;
            }
            uk *= u;
        }
        nadd(&s, -c * gv);
        for (int k = 0; k < 3; k++) nadd(&gs[k], -c * g1 * r[k]);
        if (H) {
            const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
            for (int q = 0; q < 6; q++)
                nadd(&hs[q], -c * ((ia[q] == ib[q] ? g1 : 0.0) + g2 * r[ia[q]] * r[ib[q]]));
        }
    } else {
        double E = exp(-a * a * rr * rr), ef = erf(a * rr);
        double f = -ef / rr;
        double f1 = ef / (rr * rr) - c * E / rr;
        double f2 = 2.0 * c * a * a * E + 2.0 * c * E / (rr * rr) - 2.0 * ef / (rr * rr * rr);
        add_radial(r, rr, f, f1, f2, &s, gs, H ? hs : NULL);
    }
    /* images n != 0; beyond a |r + nL| of 6.5, erfc is below 1e-19 and the
     * image is left out */
    for (int i = -nreal; i <= nreal; i++)
        for (int j = -nreal; j <= nreal; j++)
            for (int k = -nreal; k <= nreal; k++) {
                if (i == 0 && j == 0 && k == 0) continue;
                double p[3] = {r[0] + i * L, r[1] + j * L, r[2] + k * L};
                double d = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
                if (a * d > 6.5) continue;
                double E = exp(-a * a * d * d), ec = erfc(a * d);
                double f1 = -ec / (d * d) - c * E / d;
                double f2 = 2.0 * c * a * a * E + 2.0 * c * E / (d * d) + 2.0 * ec / (d * d * d);
                add_radial(p, d, ec / d, f1, f2, &s, gs, H ? hs : NULL);
            }
    /* wave vectors m != 0: the weight exp(-pi^2 |m|^2 / (aL)^2) and the phase
     * exp(2 pi i m.r / L) both factor over the axes, so each term is a
     * product of per-axis tables */
    const double pi = 3.14159265358979323846;
    const double kk = 2.0 * pi / L;
    enum { NM = 16 };
    double ew[2 * NM + 1], cph[3][2 * NM + 1], sph[3][2 * NM + 1];
    if (nrecip > NM) nrecip = NM;
    for (int i = -nrecip; i <= nrecip; i++) {
        ew[i + NM] = exp(-pi * pi * (double)(i * i) / (a * a * L * L));
        for (int d = 0; d < 3; d++) {
            cph[d][i + NM] = cos(kk * i * r[d]);
            sph[d][i + NM] = sin(kk * i * r[d]);
        }
    }
    for (int i = -nrecip; i <= nrecip; i++)
        for (int j = -nrecip; j <= nrecip; j++) {
            /* phase of the x and y factors: (cx + i sx)(cy + i sy) */
            double cxy = cph[0][i + NM] * cph[1][j + NM] - sph[0][i + NM] * sph[1][j + NM];
            double sxy = sph[0][i + NM] * cph[1][j + NM] + cph[0][i + NM] * sph[1][j + NM];
            for (int k = -nrecip; k <= nrecip; k++) {
                if (i == 0 && j == 0 && k == 0) continue;
                double m2 = (double)(i * i + j * j + k * k);
                double w = ew[i + NM] * ew[j + NM] * ew[k + NM] / (pi * L * m2);
                double cs = cxy * cph[2][k + NM] - sxy * sph[2][k + NM];
                double sn = sxy * cph[2][k + NM] + cxy * sph[2][k + NM];
                nadd(&s, w * cs);
                double m[3] = {(double)i, (double)j, (double)k};
                for (int q = 0; q < 3; q++) nadd(&gs[q], -w * sn * kk * m[q]);
                if (H) {
                    const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
                    for (int q = 0; q < 6; q++) nadd(&hs[q], -w * cs * kk * kk * m[ia[q]] * m[ib[q]]);
                }
            }
        }
    nadd(&s, -pi / (a * a * L * L * L));
    *D = nval(&s);
    for (int q = 0; q < 3; q++) g[q] = nval(&gs[q]);
    if (H)
        for (int q = 0; q < 6; q++) H[q] = nval(&hs[q]);
}

/* D and grad D at n points r[n][3] (any r: the sums are periodic). */
void ot_ewald(double L, double alpha, int nreal, int nrecip, const double *r, int64_t n, double *D, double *grad) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n; q++) ewald_at(L, alpha, nreal, nrecip, r + 3 * q, D + q, grad + 3 * q, NULL);
}

/* D, grad D and the Hessian H[n][6] (xx yy zz xy xz yz) at n points. */
void ot_ewald_hessian(double L, double alpha, int nreal, int nrecip, const double *r, int64_t n, double *D,
                      double *grad, double *H) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n; q++) ewald_at(L, alpha, nreal, nrecip, r + 3 * q, D + q, grad + 3 * q, H + 6 * q);
}

/* splitting constant a = 2 / L: images beyond 3 boxes and wave vectors with a
 * component beyond 4 add less than 1e-17 relative */
#define EW_ALPHA 2.0
#define EW_NREAL 3
#define EW_NRECIP 4

/* Exact periodic direct sum at selected cells:
 *   phi_i = -G [ sum_{j != i} m_j psi(r_i - r_j) + m_i psi_0 ],
 * psi = 1/|r'| + D(r') with r' the nearest image, psi_0 = D(0). */
void ot_direct_periodic(const otree *t, const int64_t *targets, int64_t ntargets, double Gc, double *phi) {
    const double L = t->box;
    double D0, g0[3], zero[3] = {0.0, 0.0, 0.0};
    ewald_at(L, EW_ALPHA / L, EW_NREAL, EW_NRECIP, zero, &D0, g0, NULL);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < ntargets; q++) {
        int64_t i = targets[q];
        nsum acc = {0.0, 0.0};
        nadd(&acc, t->cm[i] * D0);
        for (int64_t j = 0; j < t->ncells; j++) {
            if (j == i || t->cm[j] == 0.0) continue;
            double r[3] = {t->cx[i] - t->cx[j], t->cy[i] - t->cy[j], t->cz[i] - t->cz[j]};
            for (int d = 0; d < 3; d++) r[d] -= L * nearbyint(r[d] / L);
            double D, gr[3];
            ewald_at(L, EW_ALPHA / L, EW_NREAL, EW_NRECIP, r, &D, gr, NULL);
            nadd(&acc, t->cm[j] * (1.0 / sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) + D));
        }
        phi[q] = -Gc * nval(&acc);
    }
}

/*
 * O10 periodic Barnes-Hut: O5-O7 in a box of side L repeated in every
 * direction (appendix "Periodic boundaries": every node or cell contributes
 * through the periodic Green's function psi = 1/|r| + D(r) of O9; read here
 * with this method's group walk and quadrupoles).  Every pair (cell, node)
 * and (cell, cell) is taken at its nearest image: R = r_i - X reduced per
 * axis by L rint(R_a / L).
 *  - MAC: node n is accepted iff every cell of g has |R|^2 > s^2 (O5 with the
 *    nearest-image distance).  All other images are then farther, and so is
 *    every singularity of psi seen from R, so the expansion below converges
 *    as the isolated one does.  A rejected bottom node goes to the near list,
 *    any other rejected node is opened.
 *  - Far node:
 *      M (1/|R| + D(R)) + R^T Q R / (2 |R|^5) + Q:H(R) / 6 + (2 pi / (3 L^3)) S,
 *    the expansion of sum_j m_j psi(r_i - x_j) about X to second order: the
 *    quadrupole meets the Hessians of 1/|r| and of D (H), the trace of the
 *    second moments (S) the Laplacian 4 pi / L^3 of D.  Near the half-box
 *    planes D holds the neighbouring image's 1/|r|, and its Hessian term is
 *    of the same order as the quadrupole term of 1/|r|.
 *  - Near node n: the periodic Green's function cell by cell,
 *      sum_{j != i} m_j / |R_ij| + sum_j m_j D(R_ij),
 *    the cell itself included in the second sum (D(0) = psi_0, its images).
 *  - phi_i = -G (far + near), compensated sums.
 * Marginal: an opening test within tau of its threshold, as in O5.
 */
typedef struct {
    const otree *t;
    const int64_t *cells;
    int G;
    double inv_theta, tau, tau_lin, L;
    ivec *far, *near;
    int64_t visited, marginal;
} pwalkctx;

/* nearest image of the vector a - b */
static void nearest_image(const double *a, const double *b, double L, double *R) {
    for (int d = 0; d < 3; d++) {
        R[d] = a[d] - b[d];
        R[d] -= L * nearbyint(R[d] / L);
    }
}

static void pwalk_node(pwalkctx *w, int n) {
    const otree *t = w->t;
    const onode *a = &t->nodes[n];
    if (a->M == 0.0) return;
    w->visited++;
    double s = a->l * w->inv_theta + a->delta;
    double s2 = s * s;
    int accept = 1;
    double dmin2 = INFINITY;
    for (int q = 0; q < w->G; q++) {
        int64_t c = w->cells[q];
        double r[3] = {t->cx[c], t->cy[c], t->cz[c]}, R[3];
        nearest_image(r, a->X, w->L, R);
        double d2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
        if (!(d2 > s2)) accept = 0;
        if (d2 < dmin2) dmin2 = d2;
    }
    if (fabs(dmin2 - s2) <= w->tau * s2 + w->tau_lin * s) w->marginal++;
    if (accept) {
        ivec_push(w->far, n);
    } else if (a->bottom) {
        ivec_push(w->near, n);
    } else {
        for (int o = 0; o < 8; o++) pwalk_node(w, a->child[o]);
    }
}

/* the smooth part of node a at R: M D(R) + Q:H(R)/6 + (2 pi/(3 L^3)) S */
static double smooth_node(const onode *a, const double *R, double L) {
    double D, g[3], H[6];
    ewald_at(L, EW_ALPHA / L, EW_NREAL, EW_NRECIP, R, &D, g, H);
    double qh = a->Q[0] * H[0] + a->Q[1] * H[1] + a->Q[2] * H[2] + 2.0 * (a->Q[3] * H[3] + a->Q[4] * H[4] + a->Q[5] * H[5]);
    const double pi = 3.14159265358979323846;
    return a->M * D + qh / 6.0 + 2.0 * pi / (3.0 * L * L * L) * a->S;
}

static void psum_group(const otree *t, const int64_t *cells, int G, const ivec *far, const ivec *near, double Gc,
                       double *phi) {
    const double L = t->box;
    for (int q = 0; q < G; q++) {
        int64_t i = cells[q];
        double ri[3] = {t->cx[i], t->cy[i], t->cz[i]};
        nsum acc = {0.0, 0.0};
        for (int f = 0; f < far->n; f++) {
            const onode *a = &t->nodes[far->v[f]];
            double R[3];
            nearest_image(ri, a->X, L, R);
            double d2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
            double dd = sqrt(d2);
            double rqr = a->Q[0] * R[0] * R[0] + a->Q[1] * R[1] * R[1] + a->Q[2] * R[2] * R[2]
                         + 2.0 * (a->Q[3] * R[0] * R[1] + a->Q[4] * R[0] * R[2] + a->Q[5] * R[1] * R[2]);
            nadd(&acc, a->M / dd);
            nadd(&acc, rqr / (2.0 * d2 * d2 * dd));
            nadd(&acc, smooth_node(a, R, L));
        }
        for (int b = 0; b < near->n; b++) {
            const onode *a = &t->nodes[near->v[b]];
            for (int o = 0; o < 8; o++) {
                int64_t j = a->cell[o];
                if (t->cm[j] == 0.0) continue;
                double xj[3] = {t->cx[j], t->cy[j], t->cz[j]}, R[3];
                nearest_image(ri, xj, L, R);
                if (j != i) nadd(&acc, t->cm[j] / sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]));
                double D, g[3];
                ewald_at(L, EW_ALPHA / L, EW_NREAL, EW_NRECIP, R, &D, g, NULL);
                nadd(&acc, t->cm[j] * D);
            }
        }
        phi[q] = -Gc * nval(&acc);
    }
}

/* O10 for selected canonical groups: phi[q * G + c] for the group's c-th cell
 * in Morton order, counts[4 q + ...] = visited, far, near, marginal, and
 * (if qsum is not NULL) qsum[q] = sum over the group's far nodes of
 * sum_ab |Q_ab| / 6 (the weight of the Hessian in the far terms, for error
 * bounds). */
void ot_solve_groups_periodic(const otree *t, int group_cells, const double *theta_group, const int64_t *groups,
                              int64_t n, double tau, double Gc, int64_t *counts, double *phi, double *qsum) {
    int G = group_cells;
#pragma omp parallel
    {
        int64_t *cells = (int64_t *)malloc(sizeof(int64_t) * (size_t)G);
#pragma omp for schedule(dynamic, 1)
        for (int64_t q = 0; q < n; q++) {
            int64_t g = groups[q];
            group_cells_of(t, g, G, cells);
            ivec far = {0, 0, NULL}, near = {0, 0, NULL};
            pwalkctx w;
            w.t = t; w.cells = cells; w.G = G;
            w.inv_theta = 1.0 / theta_group[g];
            w.tau = tau;
            w.tau_lin = t->tau_lin;
            w.L = t->box;
            w.far = &far; w.near = &near;
            w.visited = 0; w.marginal = 0;
            pwalk_node(&w, t->root);
            counts[4 * q + 0] = w.visited;
            counts[4 * q + 1] = far.n;
            counts[4 * q + 2] = near.n;
            counts[4 * q + 3] = w.marginal;
            psum_group(t, cells, G, &far, &near, Gc, phi + q * G);
            if (qsum) {
                double w = 0.0;
                for (int f = 0; f < far.n; f++) {
                    const double *Q = t->nodes[far.v[f]].Q;
                    w += (fabs(Q[0]) + fabs(Q[1]) + fabs(Q[2]) + 2.0 * (fabs(Q[3]) + fabs(Q[4]) + fabs(Q[5]))) / 6.0;
                }
                qsum[q] = w;
            }
            free(far.v);
            free(near.v);
        }
        free(cells);
    }
}

/* O10 far term of node n at point p (image nearest to p), by part:
 * out = [M (1/|R| + D(R)), R^T Q R / (2 |R|^5), Q:H(R) / 6, 2 pi S / (3 L^3)]. */
void ot_node_far_periodic(const otree *t, int n, const double *p, double *out) {
    const onode *a = &t->nodes[n];
    const double L = t->box;
    double R[3];
    nearest_image(p, a->X, L, R);
    double d2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2], dd = sqrt(d2);
    double D, g[3], H[6];
    ewald_at(L, EW_ALPHA / L, EW_NREAL, EW_NRECIP, R, &D, g, H);
    double rqr = a->Q[0] * R[0] * R[0] + a->Q[1] * R[1] * R[1] + a->Q[2] * R[2] * R[2]
                 + 2.0 * (a->Q[3] * R[0] * R[1] + a->Q[4] * R[0] * R[2] + a->Q[5] * R[1] * R[2]);
    double qh = a->Q[0] * H[0] + a->Q[1] * H[1] + a->Q[2] * H[2] + 2.0 * (a->Q[3] * H[3] + a->Q[4] * H[4] + a->Q[5] * H[5]);
    const double pi = 3.14159265358979323846;
    out[0] = a->M * (1.0 / dd + D);
    out[1] = rqr / (2.0 * d2 * d2 * dd);
    out[2] = qh / 6.0;
    out[3] = 2.0 * pi / (3.0 * L * L * L) * a->S;
}

/* Threads of the OpenMP parallel regions (for timing the oracle on a given
 * number of host cores): set, and read back what the runtime will use. */
void ot_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int ot_get_threads(void) { return omp_get_max_threads(); }

/* Linear term of the marginal band of the following walks (see otree). */
void ot_set_tau_lin(otree *t, double lin) { t->tau_lin = lin; }
