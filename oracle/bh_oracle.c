/*
 * Oracle for the Barnes-Hut force step of Bedorf, Gaburov & Portegies Zwart,
 * "Bonsai: A GPU Tree-Code" (arXiv:1204.2280).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, sequential-per-group CPU
 * implementation in float64 that the GPU library is checked against.  Only the
 * test-suite, the package smoke check and the benchmark's CPU-baseline leg may
 * load it; the GPU library never links, imports or calls it, and the two share
 * no code, headers or tables.
 *
 * It follows the method step by step, in the order the paper lists the parts
 * of a force step (Results section: sorting along a Morton space-filling
 * curve, moving the particle properties, tree construction, multipole
 * moments, tree traverse).  The paper leaves most constants unstated; the
 * readings used here are:
 *   - keys: 20 bits per axis (60-bit Morton key), x -> bit 3b+2, y -> 3b+1,
 *     z -> 3b; the root cube is anchored at the per-axis minimum and has a
 *     power-of-two side L strictly larger than the largest extent;
 *   - sort: stable (ties keep input order);
 *   - tree: sparse octree, a cell splits iff it holds more than ncrit
 *     particles and its level is below 20; breadth-first cell numbering;
 *   - groups: maximal tree cells holding at most gcap particles (a level-20
 *     leaf with more is cut into consecutive chunks of gcap);
 *   - multipoles: monopole + traceless quadrupole about the centre of mass,
 *     summed bottom-up in a fixed order with explicit fma only;
 *   - MAC (Barnes 1994 group criterion combined with the vector-machine
 *     grouping of Barnes 1990, named in the Results section): a cell is
 *     accepted for a group iff the squared distance from the group's
 *     bounding box to the cell's centre of mass exceeds r_open^2 with
 *     r_open = l'/theta + delta (l' = max(l, 2 * the largest per-axis distance
 *     of the cell's particles from its geometric centre), l: cell side,
 *     delta: distance from the centre of mass to the geometric centre; l' = l
 *     for a freshly built tree, whose cells contain their particles);
 *     equality opens; every ancestor-or-self of the group's own cell is
 *     opened.
 *   - refit (block time steps, Discussion section): the tree of the last
 *     build is kept, its particles take new positions in the same sorted
 *     order and the multipoles, l' and delta are recomputed;  The predicate is evaluated in
 *     float32 with a fixed operation order so that any implementation can
 *     reproduce the same interaction sets bit for bit;
 *   - interactions: float64 here, G and Plummer softening eps2 as parameters,
 *     self pairs and exactly coincident pairs skipped.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no contraction of
 * a*b+c into fma other than the explicit fma() calls).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_KEY_BITS 20 /* bits per axis; maximum tree level */

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ENONFINITE = -6 };

typedef struct {
    int64_t n;
    int ncrit, gcap;
    /* root cube (step "sorting": domain of the space-filling curve) */
    float lo[3];
    int k;      /* L = 2^k */
    double L;
    /* keys, permutation, moved particles */
    uint64_t *keys; /* sorted */
    int64_t *perm;  /* sorted position -> input index */
    float *sposf;   /* sorted float32 positions [n][3] */
    double *spos;   /* the same, widened [n][3] */
    double *smass;  /* sorted masses, widened */
    /* cells, breadth-first */
    int64_t ncells, cap_cells;
    int *level;
    int64_t *first, *count, *child_first;
    int *nchild;
    int64_t *parent;
    /* groups, ordered by first particle */
    int64_t ngroups;
    int64_t *gfirst, *gcount, *gcell;
    int *glevel;
    /* multipoles */
    double *M, *com, *S, *Q, *delta; /* com [c][3], S and Q [c][6]: xx yy zz xy xz yz */
    float *bmin, *bmax;              /* per cell: bounding box of its particles [c][3] */
    double *lside;                   /* per cell: l' = max(l, 2 * reach from the geometric centre) */
    /* MAC data for the last theta */
    float *com32, *r2open;
    /* per-group list sizes for the last walk */
    int64_t *n_pc, *n_pp;
    /* results, sorted order and input order */
    double *sacc, *spot, *acc, *pot;
} orc_tree;

/* ------------------------------------------------------------------ */
/* small helpers                                                        */
/* ------------------------------------------------------------------ */

static void *xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

/* Octant of the key at level lev (1..20): 3 bits, 4*x + 2*y + z. */
static int octant_at(uint64_t key, int lev) {
    return (int)((key >> (3 * (ORC_KEY_BITS - lev))) & 7u);
}

/* Integer coordinate of a level-lev cell along axis a (0=x,1=y,2=z), read
 * back from the key prefix one bit per level. */
static uint64_t cell_coord(uint64_t key, int lev, int a) {
    uint64_t q = 0;
    for (int b = 0; b < lev; b++) {
        /* level b+1 digit sits at bits 3*(19-b) .. 3*(19-b)+2 */
        int dig = octant_at(key, b + 1);
        int bit = (dig >> (2 - a)) & 1;
        q = (q << 1) | (uint64_t)bit;
    }
    return q;
}

void orc_free(orc_tree *t) {
    if (!t) return;
    free(t->keys); free(t->perm); free(t->sposf); free(t->spos); free(t->smass);
    free(t->level); free(t->first); free(t->count); free(t->child_first);
    free(t->nchild); free(t->parent);
    free(t->gfirst); free(t->gcount); free(t->gcell); free(t->glevel);
    free(t->M); free(t->com); free(t->S); free(t->Q); free(t->delta);
    free(t->bmin); free(t->bmax); free(t->lside);
    free(t->com32); free(t->r2open); free(t->n_pc); free(t->n_pp);
    free(t->sacc); free(t->spot); free(t->acc); free(t->pot);
    free(t);
}

orc_tree *orc_new(void) { return (orc_tree *)calloc(1, sizeof(orc_tree)); }

/* ------------------------------------------------------------------ */
/* Step 1: root cube (part of "sorting")                                */
/* ------------------------------------------------------------------ */

/* Per-axis min/max in float32 (exact), extent in float64, L = 2^k with
 * L > extent strictly (k from frexp), k = 0 for a zero extent. */
int orc_root_cube(const float *pos, int64_t n, float lo[3], int *k_out) {
    float mn[3], mx[3];
    for (int a = 0; a < 3; a++) { mn[a] = pos[a]; mx[a] = pos[a]; }
    for (int64_t i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) {
            float v = pos[3 * i + a];
            if (!isfinite(v)) return ORC_ENONFINITE;
            if (v < mn[a]) mn[a] = v;
            if (v > mx[a]) mx[a] = v;
        }
    double ext = 0.0;
    for (int a = 0; a < 3; a++) {
        double e = (double)mx[a] - (double)mn[a];
        if (e > ext) ext = e;
    }
    int k = 0;
    if (ext > 0.0) frexp(ext, &k); /* ext = f * 2^k, f in [0.5, 1) => 2^k > ext */
    for (int a = 0; a < 3; a++) lo[a] = mn[a];
    *k_out = k;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Step 2: Morton keys (part of "sorting")                              */
/* ------------------------------------------------------------------ */

/* q_a = min(floor((x_a - lo_a) * 2^(20-k)), 2^20 - 1); the key interleaves
 * the 20 bits of each q with x the most significant of every triple. */
uint64_t orc_key(const float x[3], const float lo[3], int k) {
    double s = ldexp(1.0, ORC_KEY_BITS - k);
    uint64_t q[3];
    for (int a = 0; a < 3; a++) {
        double f = floor(((double)x[a] - (double)lo[a]) * s);
        if (f > (double)((1u << ORC_KEY_BITS) - 1)) f = (double)((1u << ORC_KEY_BITS) - 1);
        if (f < 0.0) f = 0.0;
        q[a] = (uint64_t)f;
    }
    uint64_t key = 0;
    for (int b = 0; b < ORC_KEY_BITS; b++) {
        key |= ((q[0] >> b) & 1u) << (3 * b + 2);
        key |= ((q[1] >> b) & 1u) << (3 * b + 1);
        key |= ((q[2] >> b) & 1u) << (3 * b);
    }
    return key;
}

/* ------------------------------------------------------------------ */
/* Step 3: stable sort by key (the rest of "sorting")                   */
/* ------------------------------------------------------------------ */

typedef struct { uint64_t key; int64_t idx; } kv_t;

static int kv_cmp(const void *a, const void *b) {
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx); /* ties: input order */
}

/* ------------------------------------------------------------------ */
/* Step 5: octree ("tree-construction"), breadth first                  */
/* ------------------------------------------------------------------ */

static int push_cell(orc_tree *t, int lev, int64_t first, int64_t count, int64_t parent) {
    if (t->ncells == t->cap_cells) {
        int64_t cap = t->cap_cells ? 2 * t->cap_cells : 1024;
        int *lv = realloc(t->level, cap * sizeof(int));
        if (lv) t->level = lv;
        int64_t *f = realloc(t->first, cap * sizeof(int64_t));
        if (f) t->first = f;
        int64_t *c = realloc(t->count, cap * sizeof(int64_t));
        if (c) t->count = c;
        int64_t *cf = realloc(t->child_first, cap * sizeof(int64_t));
        if (cf) t->child_first = cf;
        int *nc = realloc(t->nchild, cap * sizeof(int));
        if (nc) t->nchild = nc;
        int64_t *p = realloc(t->parent, cap * sizeof(int64_t));
        if (p) t->parent = p;
        if (!lv || !f || !c || !cf || !nc || !p) return ORC_ENOMEM;
        t->cap_cells = cap;
    }
    int64_t c = t->ncells++;
    t->level[c] = lev;
    t->first[c] = first;
    t->count[c] = count;
    t->child_first[c] = 0;
    t->nchild[c] = 0;
    t->parent[c] = parent;
    return ORC_OK;
}

/* A cell splits iff count > ncrit and level < 20; its children are its
 * non-empty octants in octant order, appended to the breadth-first array, so
 * cells come out ordered by level and, within a level, by key. */
static int build_tree(orc_tree *t) {
    t->ncells = 0;
    if (push_cell(t, 0, 0, t->n, -1)) return ORC_ENOMEM;
    for (int64_t c = 0; c < t->ncells; c++) {
        int lev = t->level[c];
        if (!(t->count[c] > t->ncrit && lev < ORC_KEY_BITS)) continue;
        int64_t b = t->first[c], e = t->first[c] + t->count[c];
        t->child_first[c] = t->ncells;
        int64_t i = b;
        while (i < e) {
            int oct = octant_at(t->keys[i], lev + 1);
            int64_t j = i;
            while (j < e && octant_at(t->keys[j], lev + 1) == oct) j++;
            if (push_cell(t, lev + 1, i, j - i, c)) return ORC_ENOMEM;
            t->nchild[c]++;
            i = j;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Step 6: groups (vector-machine walk: one list per group)            */
/* ------------------------------------------------------------------ */

static int cmp_i64_pair(const void *a, const void *b) {
    const int64_t *x = (const int64_t *)a, *y = (const int64_t *)b;
    return (x[0] > y[0]) - (x[0] < y[0]);
}

/* A cell is a group iff count <= gcap and it is the root or its parent holds
 * more than gcap; a level-20 leaf holding more than gcap is cut into
 * consecutive chunks of gcap.  Groups are ordered by first particle. */
static int build_groups(orc_tree *t) {
    int64_t cap = 16, ng = 0;
    int64_t *rec = malloc(cap * 4 * sizeof(int64_t)); /* first, count, cell, level */
    if (!rec) return ORC_ENOMEM;
    for (int64_t c = 0; c < t->ncells; c++) {
        int parent_big = (t->parent[c] < 0) || (t->count[t->parent[c]] > t->gcap);
        if (!parent_big) continue;
        int64_t pieces = 0, f = t->first[c], cnt = t->count[c];
        if (cnt <= t->gcap) pieces = 1;
        else if (t->nchild[c] == 0) pieces = (cnt + t->gcap - 1) / t->gcap; /* level-20 leaf */
        for (int64_t p = 0; p < pieces; p++) {
            if (ng == cap) {
                cap *= 2;
                int64_t *r = realloc(rec, cap * 4 * sizeof(int64_t));
                if (!r) { free(rec); return ORC_ENOMEM; }
                rec = r;
            }
            int64_t pf = f + p * t->gcap;
            int64_t pc = cnt - p * t->gcap < t->gcap ? cnt - p * t->gcap : t->gcap;
            if (pieces == 1) { pf = f; pc = cnt; }
            rec[4 * ng + 0] = pf;
            rec[4 * ng + 1] = pc;
            rec[4 * ng + 2] = c;
            rec[4 * ng + 3] = t->level[c];
            ng++;
        }
    }
    qsort(rec, ng, 4 * sizeof(int64_t), cmp_i64_pair);
    t->ngroups = ng;
    t->gfirst = xcalloc(ng, sizeof(int64_t));
    t->gcount = xcalloc(ng, sizeof(int64_t));
    t->gcell = xcalloc(ng, sizeof(int64_t));
    t->glevel = xcalloc(ng, sizeof(int));
    if (!t->gfirst || !t->gcount || !t->gcell || !t->glevel) { free(rec); return ORC_ENOMEM; }
    for (int64_t g = 0; g < ng; g++) {
        t->gfirst[g] = rec[4 * g + 0];
        t->gcount[g] = rec[4 * g + 1];
        t->gcell[g] = rec[4 * g + 2];
        t->glevel[g] = (int)rec[4 * g + 3];
    }
    free(rec);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Step 7: multipole moments ("tree-properties")                        */
/* ------------------------------------------------------------------ */

/* Geometric centre of a cell: corner = lo + q*l per axis, centre = corner + l/2. */
static void cell_centre(const orc_tree *t, int64_t c, double centre[3], double *side) {
    int lev = t->level[c];
    double l = ldexp(1.0, t->k - lev);
    uint64_t key = t->keys[t->first[c]];
    for (int a = 0; a < 3; a++) {
        double q = (double)cell_coord(key, lev, a);
        double corner = (double)t->lo[a] + q * l;
        centre[a] = corner + 0.5 * l;
    }
    *side = l;
}

/* Leaves from their particles, internal cells from their children in
 * child order, deepest cells first (reverse breadth-first order):
 *   M   = sum m
 *   com = (sum fma(m, x, .)) / M           (geometric centre if M == 0)
 *   S   = sum fma(m*d_a, d_b, .), d = x - com            (leaf)
 *   S   = sum (S_c + (M_c*e_a)*e_b), e = com_c - com     (internal)
 *   Q   = 3 S - tr(S) I,  tr(S) = (Sxx + Syy) + Szz
 *   delta = sqrt((dx*dx + dy*dy) + dz*dz), d = com - centre
 *   box = float32 min/max of the cell's particles (children's boxes for an
 *         internal cell), reach = max_a max(centre_a - min_a, max_a - centre_a),
 *   l'  = max(l, 2 reach). */
static void compute_multipoles(orc_tree *t) {
    static const int IA[6] = {0, 1, 2, 0, 0, 1}, IB[6] = {0, 1, 2, 1, 2, 2};
    for (int64_t c = t->ncells - 1; c >= 0; c--) {
        double centre[3], l;
        cell_centre(t, c, centre, &l);
        double M = 0.0, cm[3] = {0, 0, 0}, S[6] = {0, 0, 0, 0, 0, 0};
        double *com = &t->com[3 * c];
        float *bn = &t->bmin[3 * c], *bx = &t->bmax[3 * c];
        if (t->nchild[c] == 0) {
            int64_t b = t->first[c], e = t->first[c] + t->count[c];
            for (int a = 0; a < 3; a++) bn[a] = bx[a] = t->sposf[3 * b + a];
            for (int64_t j = b; j < e; j++)
                for (int a = 0; a < 3; a++) {
                    float v = t->sposf[3 * j + a];
                    if (v < bn[a]) bn[a] = v;
                    if (v > bx[a]) bx[a] = v;
                }
            for (int64_t j = b; j < e; j++) {
                M = M + t->smass[j];
                for (int a = 0; a < 3; a++) cm[a] = fma(t->smass[j], t->spos[3 * j + a], cm[a]);
            }
            for (int a = 0; a < 3; a++) com[a] = M > 0.0 ? cm[a] / M : centre[a];
            for (int64_t j = b; j < e; j++) {
                double d[3];
                for (int a = 0; a < 3; a++) d[a] = t->spos[3 * j + a] - com[a];
                for (int s = 0; s < 6; s++) S[s] = fma(t->smass[j] * d[IA[s]], d[IB[s]], S[s]);
            }
        } else {
            int64_t cb = t->child_first[c], ce = cb + t->nchild[c];
            for (int a = 0; a < 3; a++) {
                bn[a] = t->bmin[3 * cb + a];
                bx[a] = t->bmax[3 * cb + a];
            }
            for (int64_t ch = cb; ch < ce; ch++)
                for (int a = 0; a < 3; a++) {
                    if (t->bmin[3 * ch + a] < bn[a]) bn[a] = t->bmin[3 * ch + a];
                    if (t->bmax[3 * ch + a] > bx[a]) bx[a] = t->bmax[3 * ch + a];
                }
            for (int64_t ch = cb; ch < ce; ch++) {
                M = M + t->M[ch];
                for (int a = 0; a < 3; a++) cm[a] = fma(t->M[ch], t->com[3 * ch + a], cm[a]);
            }
            for (int a = 0; a < 3; a++) com[a] = M > 0.0 ? cm[a] / M : centre[a];
            for (int64_t ch = cb; ch < ce; ch++) {
                double e[3];
                for (int a = 0; a < 3; a++) e[a] = t->com[3 * ch + a] - com[a];
                for (int s = 0; s < 6; s++) {
                    double shift = (t->M[ch] * e[IA[s]]) * e[IB[s]];
                    S[s] = S[s] + (t->S[6 * ch + s] + shift);
                }
            }
        }
        t->M[c] = M;
        for (int s = 0; s < 6; s++) t->S[6 * c + s] = S[s];
        double tr = (S[0] + S[1]) + S[2];
        for (int s = 0; s < 3; s++) t->Q[6 * c + s] = 3.0 * S[s] - tr;
        for (int s = 3; s < 6; s++) t->Q[6 * c + s] = 3.0 * S[s];
        double dx = com[0] - centre[0], dy = com[1] - centre[1], dz = com[2] - centre[2];
        t->delta[c] = sqrt((dx * dx + dy * dy) + dz * dz);
        double reach = 0.0;
        for (int a = 0; a < 3; a++) {
            double lo_d = centre[a] - (double)bn[a], hi_d = (double)bx[a] - centre[a];
            if (lo_d > reach) reach = lo_d;
            if (hi_d > reach) reach = hi_d;
        }
        t->lside[c] = 2.0 * reach > l ? 2.0 * reach : l;
    }
}

/* ------------------------------------------------------------------ */
/* Steps 1-7 driver                                                     */
/* ------------------------------------------------------------------ */

int orc_build(orc_tree *t, const float *pos, const float *mass, int64_t n, int ncrit, int gcap) {
    if (!t || !pos || !mass || n < 1 || ncrit < 1 || gcap < ncrit) return ORC_EINVAL;
    for (int64_t i = 0; i < n; i++)
        if (!isfinite(mass[i])) return ORC_ENONFINITE;
    for (int64_t i = 0; i < n; i++)
        if (mass[i] < 0.0f) return ORC_EINVAL;
    t->n = n;
    t->ncrit = ncrit;
    t->gcap = gcap;
    int st = orc_root_cube(pos, n, t->lo, &t->k);
    if (st) return st;
    t->L = ldexp(1.0, t->k);

    kv_t *kv = malloc(n * sizeof(kv_t));
    if (!kv) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; i++) {
        kv[i].key = orc_key(&pos[3 * i], t->lo, t->k);
        kv[i].idx = i;
    }
    qsort(kv, n, sizeof(kv_t), kv_cmp);

    t->keys = malloc(n * sizeof(uint64_t));
    t->perm = malloc(n * sizeof(int64_t));
    t->sposf = malloc(3 * n * sizeof(float));
    t->spos = malloc(3 * n * sizeof(double));
    t->smass = malloc(n * sizeof(double));
    if (!t->keys || !t->perm || !t->sposf || !t->spos || !t->smass) { free(kv); return ORC_ENOMEM; }
    /* "moving": particle properties follow the permutation */
    for (int64_t i = 0; i < n; i++) {
        t->keys[i] = kv[i].key;
        t->perm[i] = kv[i].idx;
        for (int a = 0; a < 3; a++) {
            t->sposf[3 * i + a] = pos[3 * kv[i].idx + a];
            t->spos[3 * i + a] = (double)pos[3 * kv[i].idx + a];
        }
        t->smass[i] = (double)mass[kv[i].idx];
    }
    free(kv);

    if ((st = build_tree(t))) return st;
    if ((st = build_groups(t))) return st;

    int64_t nc = t->ncells;
    t->M = xcalloc(nc, sizeof(double));
    t->com = xcalloc(3 * nc, sizeof(double));
    t->S = xcalloc(6 * nc, sizeof(double));
    t->Q = xcalloc(6 * nc, sizeof(double));
    t->delta = xcalloc(nc, sizeof(double));
    t->bmin = xcalloc(3 * nc, sizeof(float));
    t->bmax = xcalloc(3 * nc, sizeof(float));
    t->lside = xcalloc(nc, sizeof(double));
    t->com32 = xcalloc(3 * nc, sizeof(float));
    t->r2open = xcalloc(nc, sizeof(float));
    t->n_pc = xcalloc(t->ngroups, sizeof(int64_t));
    t->n_pp = xcalloc(t->ngroups, sizeof(int64_t));
    t->sacc = xcalloc(3 * n, sizeof(double));
    t->spot = xcalloc(n, sizeof(double));
    t->acc = xcalloc(3 * n, sizeof(double));
    t->pot = xcalloc(n, sizeof(double));
    if (!t->M || !t->com || !t->S || !t->Q || !t->delta || !t->com32 || !t->r2open ||
        !t->bmin || !t->bmax || !t->lside ||
        !t->n_pc || !t->n_pp || !t->sacc || !t->spot || !t->acc || !t->pot)
        return ORC_ENOMEM;
    compute_multipoles(t);
    return ORC_OK;
}

/* Refit (block time steps): the particles of the last build take new
 * positions and masses (input order, same particles); the sorted order,
 * cells and groups stay, the moved properties and the multipoles are
 * recomputed. */
int orc_refit(orc_tree *t, const float *pos, const float *mass) {
    if (!t || !t->keys || !pos || !mass) return ORC_EINVAL;
    for (int64_t i = 0; i < 3 * t->n; i++)
        if (!isfinite(pos[i])) return ORC_ENONFINITE;
    for (int64_t i = 0; i < t->n; i++) {
        if (!isfinite(mass[i])) return ORC_ENONFINITE;
        if (mass[i] < 0.0f) return ORC_EINVAL;
    }
    for (int64_t k = 0; k < t->n; k++) {
        int64_t i = t->perm[k];
        for (int a = 0; a < 3; a++) {
            t->sposf[3 * k + a] = pos[3 * i + a];
            t->spos[3 * k + a] = (double)pos[3 * i + a];
        }
        t->smass[k] = (double)mass[i];
    }
    compute_multipoles(t);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Step 8: MAC data for one theta                                       */
/* ------------------------------------------------------------------ */

/* r_open = l'/theta + delta in float64 (theta is the float32 input widened),
 * stored squared and rounded to float32; the centre of mass is rounded to
 * float32 for the float32 predicate. */
int orc_mac_prep(orc_tree *t, float theta) {
    if (!(theta > 0.0f) || !isfinite(theta)) return ORC_EINVAL;
    for (int64_t c = 0; c < t->ncells; c++) {
        double ro = t->lside[c] / (double)theta + t->delta[c];
        t->r2open[c] = (float)(ro * ro);
        for (int a = 0; a < 3; a++) t->com32[3 * c + a] = (float)t->com[3 * c + a];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Step 9: group walk ("tree-traverse")                                 */
/* ------------------------------------------------------------------ */

typedef struct { int64_t *v; int64_t n, cap; } vec_t;

static int vpush(vec_t *s, int64_t x) {
    if (s->n == s->cap) {
        int64_t cap = s->cap ? 2 * s->cap : 256;
        int64_t *v = realloc(s->v, cap * sizeof(int64_t));
        if (!v) return ORC_ENOMEM;
        s->v = v;
        s->cap = cap;
    }
    s->v[s->n++] = x;
    return ORC_OK;
}

/* Float32 predicate with every operation rounded to nearest:
 * d_a = max(max(bmin_a - c_a, c_a - bmax_a), 0); d2 = (dx*dx + dy*dy) + dz*dz;
 * accept iff d2 > r2open. */
static int mac_accept(const float bmin[3], const float bmax[3], const float c[3], float r2open) {
    float d[3];
    for (int a = 0; a < 3; a++) {
        float u = bmin[a] - c[a];
        float v = c[a] - bmax[a];
        float m = u > v ? u : v;
        d[a] = m > 0.0f ? m : 0.0f;
    }
    float d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    return d2 > r2open;
}

/* Interaction lists of one group: PC = accepted cells, PP = opened leaves.
 * Depth-first with an explicit stack; the visiting order does not change the
 * sets.  Returns n_pc and n_pp (particles in the PP leaves, self included). */
static int group_lists(const orc_tree *t, int64_t g, vec_t *stack, vec_t *pc, vec_t *pp) {
    int64_t gf = t->gfirst[g], gn = t->gcount[g];
    int glev = t->glevel[g];
    float bmin[3], bmax[3];
    for (int a = 0; a < 3; a++) { bmin[a] = t->sposf[3 * gf + a]; bmax[a] = bmin[a]; }
    for (int64_t i = gf; i < gf + gn; i++)
        for (int a = 0; a < 3; a++) {
            float v = t->sposf[3 * i + a];
            if (v < bmin[a]) bmin[a] = v;
            if (v > bmax[a]) bmax[a] = v;
        }
    stack->n = pc->n = pp->n = 0;
    if (vpush(stack, 0)) return ORC_ENOMEM;
    while (stack->n > 0) {
        int64_t c = stack->v[--stack->n];
        int ancestor = t->first[c] <= gf && gf < t->first[c] + t->count[c] && t->level[c] <= glev;
        int accept = !ancestor && mac_accept(bmin, bmax, &t->com32[3 * c], t->r2open[c]);
        if (accept) {
            if (vpush(pc, c)) return ORC_ENOMEM;
        } else if (t->nchild[c] == 0) {
            if (vpush(pp, c)) return ORC_ENOMEM;
        } else {
            for (int64_t ch = t->child_first[c] + t->nchild[c] - 1; ch >= t->child_first[c]; ch--)
                if (vpush(stack, ch)) return ORC_ENOMEM;
        }
    }
    return ORC_OK;
}

/* Cell (monopole + traceless quadrupole) field at a point, R = x - com:
 *   a   += G [ -M R / r^3 + Q R / r^5 - (5/2) (R.Q.R) R / r^7 ]
 *   phi -= G [  M / r    + (R.Q.R) / (2 r^5) ],  r^2 = R.R + eps2. */
static void pc_interaction(const orc_tree *t, int64_t c, const double x[3], double eps2, double G,
                           double a[3], double *phi) {
    const double *cm = &t->com[3 * c], *Q = &t->Q[6 * c];
    double R[3] = {x[0] - cm[0], x[1] - cm[1], x[2] - cm[2]};
    double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2] + eps2;
    double rinv = 1.0 / sqrt(r2);
    double rinv2 = rinv * rinv;
    double rinv3 = rinv * rinv2, rinv5 = rinv3 * rinv2, rinv7 = rinv5 * rinv2;
    double QR[3];
    QR[0] = Q[0] * R[0] + Q[3] * R[1] + Q[4] * R[2];
    QR[1] = Q[3] * R[0] + Q[1] * R[1] + Q[5] * R[2];
    QR[2] = Q[4] * R[0] + Q[5] * R[1] + Q[2] * R[2];
    double RQR = R[0] * QR[0] + R[1] * QR[1] + R[2] * QR[2];
    double M = t->M[c];
    for (int d = 0; d < 3; d++)
        a[d] += G * (-M * R[d] * rinv3 + QR[d] * rinv5 - 2.5 * RQR * R[d] * rinv7);
    *phi -= G * (M * rinv + 0.5 * RQR * rinv5);
}

/* Particle-particle term; j == i and exactly coincident pairs are skipped. */
static void pp_interaction(const double xj[3], double mj, const double x[3], double eps2, double G,
                           double a[3], double *phi) {
    double d[3] = {xj[0] - x[0], xj[1] - x[1], xj[2] - x[2]};
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 == 0.0) return;
    double rinv = 1.0 / sqrt(r2 + eps2);
    double rinv3 = rinv * rinv * rinv;
    for (int k = 0; k < 3; k++) a[k] += G * mj * d[k] * rinv3;
    *phi -= G * mj * rinv;
}

/* Lists and interactions of group g (after orc_mac_prep): fills n_pc/n_pp of
 * the group and the sorted accelerations and potentials of its particles. */
static int walk_group(orc_tree *t, int64_t g, double eps2, double G, vec_t *stack, vec_t *pc, vec_t *pp) {
    if (group_lists(t, g, stack, pc, pp)) return ORC_ENOMEM;
    int64_t npp = 0;
    for (int64_t k = 0; k < pp->n; k++) npp += t->count[pp->v[k]];
    t->n_pc[g] = pc->n;
    t->n_pp[g] = npp;
    for (int64_t i = t->gfirst[g]; i < t->gfirst[g] + t->gcount[g]; i++) {
        const double *x = &t->spos[3 * i];
        double a[3] = {0, 0, 0}, phi = 0.0;
        for (int64_t k = 0; k < pc->n; k++) pc_interaction(t, pc->v[k], x, eps2, G, a, &phi);
        for (int64_t k = 0; k < pp->n; k++) {
            int64_t c = pp->v[k];
            for (int64_t j = t->first[c]; j < t->first[c] + t->count[c]; j++) {
                if (j == i) continue;
                pp_interaction(&t->spos[3 * j], t->smass[j], x, eps2, G, a, &phi);
            }
        }
        for (int d = 0; d < 3; d++) t->sacc[3 * i + d] = a[d];
        t->spot[i] = phi;
    }
    return ORC_OK;
}

/* Walk the groups glist[0..ng) (glist NULL: groups g_begin + 0..ng) with
 * nthreads threads (<= 0: runtime default), after orc_mac_prep. */
static int walk_groups(orc_tree *t, double eps2, double G, const int64_t *glist, int64_t g_begin, int64_t ng,
                       int nthreads) {
    int err = ORC_OK;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
#endif
    {
        vec_t stack = {0}, pc = {0}, pp = {0};
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int64_t k = 0; k < ng; k++) {
            int64_t g = glist ? glist[k] : g_begin + k;
            if (walk_group(t, g, eps2, G, &stack, &pc, &pp)) err = ORC_ENOMEM;
        }
        free(stack.v); free(pc.v); free(pp.v);
    }
    return err;
}

/* Walk groups [g_begin, g_end), after MAC data for theta. */
int orc_walk(orc_tree *t, float theta, double eps2, double G, int64_t g_begin, int64_t g_end,
             int nthreads) {
    int st = orc_mac_prep(t, theta);
    if (st) return st;
    if (g_begin < 0) g_begin = 0;
    if (g_end > t->ngroups) g_end = t->ngroups;
    if (g_end <= g_begin) return ORC_OK;
    return walk_groups(t, eps2, G, NULL, g_begin, g_end - g_begin, nthreads);
}

/* Walk the listed groups (each at most once; any order). */
int orc_walk_list(orc_tree *t, float theta, double eps2, double G, const int64_t *glist, int64_t ng,
                  int nthreads) {
    int st = orc_mac_prep(t, theta);
    if (st) return st;
    for (int64_t k = 0; k < ng; k++)
        if (glist[k] < 0 || glist[k] >= t->ngroups) return ORC_EINVAL;
    return walk_groups(t, eps2, G, glist, 0, ng, nthreads);
}

/* Interaction lists of one group (after orc_mac_prep), for brute-force checks:
 * writes up to cap_pc accepted cells and cap_pp opened leaves, returns the
 * true sizes in *npc and *npp_leaves. */
int orc_group_lists(orc_tree *t, int64_t g, int64_t *pc_out, int64_t cap_pc, int64_t *pp_out,
                    int64_t cap_pp, int64_t *npc, int64_t *npp_leaves) {
    if (g < 0 || g >= t->ngroups) return ORC_EINVAL;
    vec_t stack = {0}, pc = {0}, pp = {0};
    int st = group_lists(t, g, &stack, &pc, &pp);
    if (!st) {
        for (int64_t k = 0; k < pc.n && k < cap_pc; k++) pc_out[k] = pc.v[k];
        for (int64_t k = 0; k < pp.n && k < cap_pp; k++) pp_out[k] = pp.v[k];
        *npc = pc.n;
        *npp_leaves = pp.n;
    }
    free(stack.v); free(pc.v); free(pp.v);
    return st;
}

/* ------------------------------------------------------------------ */
/* Step 10: back to input order; energies                               */
/* ------------------------------------------------------------------ */

void orc_unsort(orc_tree *t) {
    for (int64_t k = 0; k < t->n; k++) {
        int64_t i = t->perm[k];
        for (int d = 0; d < 3; d++) t->acc[3 * i + d] = t->sacc[3 * k + d];
        t->pot[i] = t->spot[k];
    }
}

/* W = 1/2 sum m phi and T = 1/2 sum m |v|^2, float64, input order. */
void orc_energy(const float *mass, const double *pot, const float *vel, int64_t n, double *T,
                double *W) {
    double w = 0.0, k = 0.0;
    for (int64_t i = 0; i < n; i++) {
        w += (double)mass[i] * pot[i];
        if (vel) {
            double v2 = 0.0;
            for (int d = 0; d < 3; d++) v2 += (double)vel[3 * i + d] * (double)vel[3 * i + d];
            k += (double)mass[i] * v2;
        }
    }
    *W = 0.5 * w;
    *T = 0.5 * k;
}

/* ------------------------------------------------------------------ */
/* Direct O(N^2) summation (the brute-force method of the Introduction) */
/* ------------------------------------------------------------------ */

/* For each target index, sum over every j != i with a non-zero separation. */
int orc_direct(const float *pos, const float *mass, int64_t n, const int64_t *targets, int64_t nt,
               double eps2, double G, double *acc, double *pot, int nthreads) {
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads)
#endif
    for (int64_t t = 0; t < nt; t++) {
        int64_t i = targets ? targets[t] : t;
        double x[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
        double a[3] = {0, 0, 0}, phi = 0.0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double xj[3] = {pos[3 * j], pos[3 * j + 1], pos[3 * j + 2]};
            pp_interaction(xj, (double)mass[j], x, eps2, G, a, &phi);
        }
        for (int d = 0; d < 3; d++) acc[3 * t + d] = a[d];
        pot[t] = phi;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* accessors for the ctypes wrapper                                     */
/* ------------------------------------------------------------------ */

int64_t orc_n(const orc_tree *t) { return t->n; }
int64_t orc_ncells(const orc_tree *t) { return t->ncells; }
int64_t orc_ngroups(const orc_tree *t) { return t->ngroups; }
int orc_k(const orc_tree *t) { return t->k; }
const float *orc_lo(const orc_tree *t) { return t->lo; }
const uint64_t *orc_keys(const orc_tree *t) { return t->keys; }
const int64_t *orc_perm(const orc_tree *t) { return t->perm; }
const int *orc_level(const orc_tree *t) { return t->level; }
const int64_t *orc_first(const orc_tree *t) { return t->first; }
const int64_t *orc_count(const orc_tree *t) { return t->count; }
const int64_t *orc_child_first(const orc_tree *t) { return t->child_first; }
const int *orc_nchild(const orc_tree *t) { return t->nchild; }
const int64_t *orc_parent(const orc_tree *t) { return t->parent; }
const int64_t *orc_gfirst(const orc_tree *t) { return t->gfirst; }
const int64_t *orc_gcount(const orc_tree *t) { return t->gcount; }
const int64_t *orc_gcell(const orc_tree *t) { return t->gcell; }
const int *orc_glevel(const orc_tree *t) { return t->glevel; }
const double *orc_M(const orc_tree *t) { return t->M; }
const double *orc_com(const orc_tree *t) { return t->com; }
const double *orc_S(const orc_tree *t) { return t->S; }
const double *orc_Q(const orc_tree *t) { return t->Q; }
const double *orc_delta(const orc_tree *t) { return t->delta; }
const float *orc_bmin(const orc_tree *t) { return t->bmin; }
const float *orc_bmax(const orc_tree *t) { return t->bmax; }
const double *orc_lside(const orc_tree *t) { return t->lside; }
const float *orc_com32(const orc_tree *t) { return t->com32; }
const float *orc_r2open(const orc_tree *t) { return t->r2open; }
const int64_t *orc_n_pc(const orc_tree *t) { return t->n_pc; }
const int64_t *orc_n_pp(const orc_tree *t) { return t->n_pp; }
const double *orc_sacc(const orc_tree *t) { return t->sacc; }
const double *orc_spot(const orc_tree *t) { return t->spot; }
const double *orc_acc(const orc_tree *t) { return t->acc; }
const double *orc_pot(const orc_tree *t) { return t->pot; }
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
