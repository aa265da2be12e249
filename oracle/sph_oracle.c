/*
 * sph_oracle.c -- reference implementation of grouped ("recycled") SPH
 * neighbour search, from Ragagnin, Tchipev, Bader, Dolag, Hammer,
 * "Exploiting the Space Filling Curve Ordering of Particles in the
 * Neighbour Search of Gadget3".
 *
 * TEST INFRASTRUCTURE.  This file is the oracle that the GPU path is checked
 * against.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header, table or constant
 * with the GPU library.
 *
 * Style: plain C, FP64 throughout, brute-force O(N^2) neighbour sets.  Build
 * with -ffp-contract=off so that every product and sum is rounded exactly as
 * written; fma() appears only where the canonical distance formula asks for
 * it.  OpenMP is used only across independent target particles.
 *
 * The paper gives the neighbour definitions (section "Phases of Neighbour
 * Search": density neighbours are closer than h_i, hydro neighbours closer
 * than max(h_i,h_j)), the Hilbert ordering of particles, the greedy grouping
 * rule (section "Implementation of Neighbour Recycling using a Space Filling
 * Curve"), the superset radius R + max(h_i) and the adaptive R = f h_0
 * (section "Adaptive Neighbour Recycling", Eq. 1).  It does not print SPH
 * kernels, density or force equations; those follow the Gadget-2 paper it
 * cites (Springel 2005) and are marked READING below.  Every reading is also
 * listed in the design notes.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* threads of the OpenMP loops over targets (timing on one core or all) */
void orc_set_threads(int32_t n) { omp_set_num_threads(n > 0 ? n : 1); }
int32_t orc_get_threads(void) { return (int32_t)omp_get_max_threads(); }

/* ------------------------------------------------------------------ */
/* Periodic minimum-image displacement (READING: the test box is a     */
/* cosmological, hence periodic, box; the paper does not say so).      */
/* d = x_j - x_i, folded once into [-L/2, L/2).                        */
/* ------------------------------------------------------------------ */
static inline double orc_fold(double d, double L)
{
    double half = 0.5 * L;
    if (d >= half)
        d = d - L;
    else if (d < -half)
        d = d + L;
    return d;
}

/* canonical squared distance: fma(dz,dz, fma(dy,dy, dx*dx)) */
static inline double orc_r2(double xi, double yi, double zi,
                            double xj, double yj, double zj, double L)
{
    double dx = orc_fold(xj - xi, L);
    double dy = orc_fold(yj - yi, L);
    double dz = orc_fold(zj - zi, L);
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

/* ------------------------------------------------------------------ */
/* Hilbert keys.  The paper orders particles along the Peano-Hilbert   */
/* curve (section "Impact of the Neighbour Search ...").  It does not  */
/* say which Hilbert variant; READING: J. Skilling, "Programming the    */
/* Hilbert curve", AIP Conf. Proc. 707 (2004): convert the axes to the  */
/* "transposed" Hilbert index, then interleave bits, axis 0 first.      */
/* ------------------------------------------------------------------ */
uint64_t orc_hilbert_key_cell(uint32_t ix, uint32_t iy, uint32_t iz, int32_t bits)
{
    uint32_t X[3] = {ix, iy, iz};
    uint32_t M = 1u << (bits - 1);
    /* undo excess work: walk the bit planes from the top */
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        uint32_t P = Q - 1;
        for (int i = 0; i < 3; i++) {
            if (X[i] & Q) {
                X[0] ^= P; /* invert low bits of axis 0 */
            } else {
                uint32_t t = (X[0] ^ X[i]) & P; /* swap low bits of 0 and i */
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    /* Gray encode */
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q)
            t ^= Q - 1;
    X[0] ^= t;
    X[1] ^= t;
    X[2] ^= t;
    /* interleave: most significant bit plane first, axis 0 leading */
    uint64_t key = 0;
    for (int b = bits - 1; b >= 0; b--)
        for (int i = 0; i < 3; i++)
            key = (key << 1) | (uint64_t)((X[i] >> b) & 1u);
    return key;
}

/* cell index along one axis: floor(x/L * 2^bits), clamped */
static inline uint32_t orc_cell(double x, double L, int32_t bits)
{
    double s = (x / L) * (double)(1u << bits);
    double top = (double)((1u << bits) - 1u);
    if (!(s >= 0.0))
        return 0u;
    if (s >= top)
        return (uint32_t)top;
    return (uint32_t)s; /* s >= 0: truncation is floor */
}

void orc_hilbert_keys(int64_t n, const double *x, const double *y, const double *z,
                      const int32_t *box, const double *box_L, int32_t bits,
                      uint64_t *key)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double L = box_L[box ? box[i] : 0];
        key[i] = orc_hilbert_key_cell(orc_cell(x[i], L, bits), orc_cell(y[i], L, bits),
                                      orc_cell(z[i], L, bits), bits);
    }
}

/* ------------------------------------------------------------------ */
/* Octree (the paper's tree over the particles, sections "Impact ..."  */
/* and "Neighbour Recycling in Gadget3").  Definition used here: a     */
/* node is a Hilbert cell at level l (all keys sharing the top 3l      */
/* bits) that holds at least one particle; the box is the level-0      */
/* node; a node is a leaf when it holds <= n_leaf particles or l ==    */
/* bits; otherwise its children are its non-empty sub-cells in key     */
/* order.  Nodes are emitted in depth-first pre-order; skip[k] is the  */
/* first node after k's subtree.  Box = per-node min/max of the        */
/* particle coordinates; hmax = max h over the node (READING: the      */
/* hydro walk needs it for the max(h_i,h_j) rule).                     */
/* ------------------------------------------------------------------ */
typedef struct {
    const uint64_t *key;
    const double *x, *y, *z, *h;
    int32_t n_leaf, bits;
    int64_t cap, nn;
    int32_t *first, *count, *level, *leaf, *skip;
    double *bbox, *hmax;
} orc_tree_ctx;

static void orc_tree_rec(orc_tree_ctx *c, int64_t a, int64_t b, int32_t l)
{
    int64_t me = c->nn++;
    int is_leaf = (b - a <= c->n_leaf) || (l == c->bits);
    if (me < c->cap) {
        c->first[me] = (int32_t)a;
        c->count[me] = (int32_t)(b - a);
        c->level[me] = l;
        c->leaf[me] = is_leaf;
        double lo[3] = {INFINITY, INFINITY, INFINITY};
        double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        double hm = -INFINITY;
        for (int64_t i = a; i < b; i++) {
            double p[3] = {c->x[i], c->y[i], c->z[i]};
            for (int d = 0; d < 3; d++) {
                if (p[d] < lo[d]) lo[d] = p[d];
                if (p[d] > hi[d]) hi[d] = p[d];
            }
            if (c->h[i] > hm) hm = c->h[i];
        }
        for (int d = 0; d < 3; d++) {
            c->bbox[6 * me + d] = lo[d];
            c->bbox[6 * me + 3 + d] = hi[d];
        }
        c->hmax[me] = hm;
    }
    if (!is_leaf) {
        int shift = 3 * (c->bits - l - 1);
        int64_t s = a;
        while (s < b) {
            uint64_t dig = (c->key[s] >> shift) & 7u;
            int64_t e = s;
            while (e < b && ((c->key[e] >> shift) & 7u) == dig)
                e++;
            orc_tree_rec(c, s, e, l + 1);
            s = e;
        }
    }
    if (me < c->cap)
        c->skip[me] = (int32_t)c->nn;
}

/* returns the number of nodes; writes at most cap nodes */
int64_t orc_octree(int64_t n, const uint64_t *key, int32_t nbox, const int64_t *box_off,
                   int32_t n_leaf, int32_t bits, const double *x, const double *y,
                   const double *z, const double *h, int64_t cap, int32_t *first,
                   int32_t *count, int32_t *level, int32_t *leaf, int32_t *skip,
                   double *bbox, double *hmax)
{
    (void)n;
    orc_tree_ctx c = {key, x, y, z, h, n_leaf, bits, cap, 0,
                      first, count, level, leaf, skip, bbox, hmax};
    for (int32_t b = 0; b < nbox; b++)
        if (box_off[b + 1] > box_off[b])
            orc_tree_rec(&c, box_off[b], box_off[b + 1], 0);
    return c.nn;
}

/* ------------------------------------------------------------------ */
/* Grouping (section "Implementation of Neighbour Recycling using a    */
/* Space Filling Curve"): walk the active particles in curve order;    */
/* the first one opens a group; each next one joins while it is closer */
/* than R to the group's first particle; the first one that is not     */
/* opens the next group, until no particle is left: one pass over the  */
/* whole active list.  R = f h_0 (section "Adaptive Neighbour          */
/* Recycling"), READING h_0 = h of the group's first particle, strict  */
/* "<".  Additional closing rules (READINGS): a group never crosses a  */
/* box and never exceeds n_group_max members.                          */
/* policy 0 ("count") drops the distance test.                         */
/* policy 2 ("tree", section "Adaptive Neighbour Recycling": a group   */
/* is the set of leaves inside a node of one tree depth): a particle   */
/* joins while it lies in the same octree node as the group's first    */
/* particle, the node being that particle's ancestor of depth          */
/* level[b], or its leaf when the leaf is shallower (leaf_level[i] =   */
/* depth of the leaf holding particle i).  Nodes are cubes of the      */
/* 2^l grid, so "same node of depth l" = same cell index >> (bits-l)  */
/* on every axis.                                                      */
/* gstart[0..G] receives group starts (positions in act), gstart[G]=A. */
/* ------------------------------------------------------------------ */
int64_t orc_groups(int64_t A, const int32_t *act, const double *x, const double *y,
                   const double *z, const double *h, const int32_t *box,
                   const double *box_L, const int32_t *policy, const int32_t *n_group_max,
                   const double *f, const int32_t *level,
                   const int32_t *leaf_level, int32_t bits, int32_t *gstart)
{
    int64_t G = 0;
    int64_t k0 = -1, size = 0;
    for (int64_t k = 0; k < A; k++) {
        int32_t i = act[k];
        int32_t b = box ? box[i] : 0;
        int open = 0;
        if (k0 < 0) {
            open = 1;
        } else {
            int32_t i0 = act[k0];
            int32_t b0 = box ? box[i0] : 0;
            if (b != b0) {
                open = 1;
            } else if (size >= n_group_max[b]) {
                open = 1;
            } else if (policy[b] == 1) {
                double L = box_L[b];
                double r2 = orc_r2(x[i0], y[i0], z[i0], x[i], y[i], z[i], L);
                double R = f[b] * h[i0];
                if (!(r2 < R * R))
                    open = 1;
            } else if (policy[b] == 2) {
                double L = box_L[b];
                int32_t d = level[b] < leaf_level[i0] ? level[b] : leaf_level[i0];
                int32_t sh = bits - d;
                if ((orc_cell(x[i], L, bits) >> sh) != (orc_cell(x[i0], L, bits) >> sh) ||
                    (orc_cell(y[i], L, bits) >> sh) != (orc_cell(y[i0], L, bits) >> sh) ||
                    (orc_cell(z[i], L, bits) >> sh) != (orc_cell(z[i0], L, bits) >> sh))
                    open = 1;
            }
        }
        if (open) {
            gstart[G++] = (int32_t)k;
            k0 = k;
            size = 0;
        }
        size++;
    }
    gstart[G] = (int32_t)A;
    return G;
}

/* ------------------------------------------------------------------ */
/* Neighbour sets (section "Phases of Neighbour Search").              */
/*  mode 0, density: N_i = { j : r_ij < h_i }, self included (READING).*/
/*  mode 1, hydro:   H_i = { j != i : r_ij < max(h_i, h_j) }.          */
/* Brute force over every particle of the target's box, or, with      */
/* use_grid, over the cells of a uniform grid that cover the ball; the */
/* predicate is the same, the grid only prunes.                        */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t nc;
    double cs, L;
    int64_t base, nb;
    int32_t *start; /* nc^3 + 1 */
    int32_t *idx;   /* box-local particle order by cell, ascending within a cell */
    double hmax;
} orc_grid;

static void orc_grid_build(orc_grid *g, int64_t base, int64_t nb, double L,
                           const double *x, const double *y, const double *z,
                           const double *h, double cell_hint)
{
    g->base = base;
    g->nb = nb;
    g->L = L;
    double hm = 0.0;
    for (int64_t i = 0; i < nb; i++)
        if (h[base + i] > hm) hm = h[base + i];
    g->hmax = hm;
    int64_t nc = (int64_t)floor(L / (cell_hint > 0 ? cell_hint : L));
    if (nc < 1) nc = 1;
    if (nc > 256) nc = 256;
    int64_t want = (int64_t)cbrt((double)nb / 2.0) + 1; /* ~2 particles per cell at most */
    if (nc > want) nc = want;
    g->nc = (int32_t)nc;
    g->cs = L / (double)nc;
    int64_t nc3 = nc * nc * nc;
    g->start = (int32_t *)calloc((size_t)(nc3 + 1), sizeof(int32_t));
    g->idx = (int32_t *)malloc((size_t)(nb > 0 ? nb : 1) * sizeof(int32_t));
    int32_t *cell = (int32_t *)malloc((size_t)(nb > 0 ? nb : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < nb; i++) {
        int64_t c[3];
        double p[3] = {x[base + i], y[base + i], z[base + i]};
        for (int d = 0; d < 3; d++) {
            int64_t q = (int64_t)floor(p[d] / g->cs);
            if (q < 0) q = 0;
            if (q >= nc) q = nc - 1;
            c[d] = q;
        }
        cell[i] = (int32_t)((c[0] * nc + c[1]) * nc + c[2]);
        g->start[cell[i] + 1]++;
    }
    for (int64_t c = 0; c < nc3; c++)
        g->start[c + 1] += g->start[c];
    int32_t *fill = (int32_t *)malloc((size_t)nc3 * sizeof(int32_t));
    memcpy(fill, g->start, (size_t)nc3 * sizeof(int32_t));
    for (int64_t i = 0; i < nb; i++)
        g->idx[fill[cell[i]]++] = (int32_t)i;
    free(fill);
    free(cell);
}

static void orc_grid_free(orc_grid *g)
{
    free(g->start);
    free(g->idx);
}

static int orc_cmp_i32(const void *a, const void *b)
{
    int32_t u = *(const int32_t *)a, v = *(const int32_t *)b;
    return (u > v) - (u < v);
}

/* Candidates j (global indices) whose cells may hold a point within
 * radius r of p, sorted ascending.  Returns count; *buf grows as needed. */
static int64_t orc_grid_candidates(const orc_grid *g, const double p[3], double r,
                                   int32_t **buf, int64_t *cap)
{
    int64_t nc = g->nc;
    int64_t lo[3], hi[3];
    int full = 0;
    for (int d = 0; d < 3; d++) {
        lo[d] = (int64_t)floor((p[d] - r) / g->cs) - 1;
        hi[d] = (int64_t)floor((p[d] + r) / g->cs) + 1;
        if (hi[d] - lo[d] + 1 >= nc) {
            lo[d] = 0;
            hi[d] = nc - 1;
        }
        if (nc <= 3) full = 1;
    }
    int64_t m = 0;
    if (full) {
        if (*cap < g->nb) {
            *cap = g->nb;
            *buf = (int32_t *)realloc(*buf, (size_t)*cap * sizeof(int32_t));
        }
        for (int64_t i = 0; i < g->nb; i++)
            (*buf)[m++] = (int32_t)(g->base + i);
        return m;
    }
    for (int64_t a = lo[0]; a <= hi[0]; a++) {
        int64_t ca = ((a % nc) + nc) % nc;
        for (int64_t b = lo[1]; b <= hi[1]; b++) {
            int64_t cb = ((b % nc) + nc) % nc;
            for (int64_t c = lo[2]; c <= hi[2]; c++) {
                int64_t cc = ((c % nc) + nc) % nc;
                int64_t cell = (ca * nc + cb) * nc + cc;
                int32_t s = g->start[cell], e = g->start[cell + 1];
                if (m + (e - s) > *cap) {
                    *cap = 2 * (m + (e - s)) + 1024;
                    *buf = (int32_t *)realloc(*buf, (size_t)*cap * sizeof(int32_t));
                }
                for (int32_t t = s; t < e; t++)
                    (*buf)[m++] = (int32_t)(g->base + g->idx[t]);
            }
        }
    }
    qsort(*buf, (size_t)m, sizeof(int32_t), orc_cmp_i32);
    return m;
}

static inline int64_t orc_box_of(int32_t nbox, const int64_t *box_off, int64_t i)
{
    int64_t lo = 0, hi = nbox; /* find b with box_off[b] <= i < box_off[b+1] */
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) / 2;
        if (box_off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

static inline int orc_is_ngb(int mode, int64_t i, int64_t j, double r2, double hi_,
                             double hj)
{
    if (mode == 0)
        return r2 < hi_ * hi_;
    if (j == i)
        return 0;
    double hm = hi_ > hj ? hi_ : hj;
    return r2 < hm * hm;
}

static inline uint64_t orc_splitmix64(uint64_t v)
{
    uint64_t z = v + 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

typedef struct {
    int32_t nbox;
    const int64_t *box_off;
    const double *box_L;
    orc_grid *grids; /* NULL: brute force */
} orc_space;

static void orc_space_init(orc_space *s, int32_t nbox, const int64_t *box_off,
                           const double *box_L, int32_t use_grid, const double *x,
                           const double *y, const double *z, const double *h)
{
    s->nbox = nbox;
    s->box_off = box_off;
    s->box_L = box_L;
    s->grids = NULL;
    if (!use_grid)
        return;
    s->grids = (orc_grid *)calloc((size_t)nbox, sizeof(orc_grid));
    for (int32_t b = 0; b < nbox; b++) {
        int64_t base = box_off[b], nb = box_off[b + 1] - box_off[b];
        double hs = 0.0;
        for (int64_t i = 0; i < nb; i++) hs += h[base + i];
        double hmean = nb > 0 ? hs / (double)nb : box_L[b];
        orc_grid_build(&s->grids[b], base, nb, box_L[b], x, y, z, h, hmean);
    }
}

static void orc_space_free(orc_space *s)
{
    if (!s->grids) return;
    for (int32_t b = 0; b < s->nbox; b++) orc_grid_free(&s->grids[b]);
    free(s->grids);
}

/* Visit the neighbours of target i, ascending j, calling the body macro. */
typedef struct {
    int32_t *buf;
    int64_t cap;
} orc_scratch;

/* Returns candidate range: either [b0,b1) of the box (brute force) or a
 * sorted list in scr->buf (grid).  r is the largest radius any neighbour
 * can have for this query. */
static int64_t orc_candidates(const orc_space *s, int64_t i, const double *x,
                              const double *y, const double *z, double r,
                              orc_scratch *scr, int64_t *b0, int64_t *b1, double *L)
{
    int64_t b = orc_box_of(s->nbox, s->box_off, i);
    *L = s->box_L[b];
    if (!s->grids) {
        *b0 = s->box_off[b];
        *b1 = s->box_off[b + 1];
        return -1;
    }
    double p[3] = {x[i], y[i], z[i]};
    return orc_grid_candidates(&s->grids[b], p, r, &scr->buf, &scr->cap);
}

#define ORC_FOR_CAND(m, b0, b1, scr, j, ...)                                   \
    do {                                                                       \
        if ((m) < 0) {                                                         \
            for (int64_t j = (b0); j < (b1); j++) { __VA_ARGS__ }              \
        } else {                                                               \
            for (int64_t t_ = 0; t_ < (m); t_++) {                             \
                int64_t j = (scr).buf[t_];                                     \
                __VA_ARGS__                                                    \
            }                                                                  \
        }                                                                      \
    } while (0)

static double orc_box_hmax(const orc_space *s, int64_t i, const double *h)
{
    int64_t b = orc_box_of(s->nbox, s->box_off, i);
    if (s->grids) return s->grids[b].hmax;
    double hm = 0.0;
    for (int64_t j = s->box_off[b]; j < s->box_off[b + 1]; j++)
        if (h[j] > hm) hm = h[j];
    return hm;
}

/* counts and fingerprints (n_i, sum_j splitmix64(orig_j) mod 2^64) */
void orc_ngb_count(int32_t mode, int64_t n, const double *x, const double *y,
                   const double *z, const double *h, const uint32_t *orig, int32_t nbox,
                   const int64_t *box_off, const double *box_L, int64_t nt,
                   const int32_t *tgt, int32_t use_grid, int32_t *cnt, uint64_t *fp)
{
    (void)n;
    orc_space s;
    orc_space_init(&s, nbox, box_off, box_L, use_grid, x, y, z, h);
    double *bh = (double *)malloc((size_t)nbox * sizeof(double));
    for (int32_t b = 0; b < nbox; b++)
        bh[b] = (box_off[b + 1] > box_off[b]) ? orc_box_hmax(&s, box_off[b], h) : 0.0;
#pragma omp parallel
    {
        orc_scratch scr = {NULL, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t t = 0; t < nt; t++) {
            int64_t i = tgt[t], b0 = 0, b1 = 0;
            double L;
            double r = h[i];
            if (mode == 1) {
                double hb = bh[orc_box_of(nbox, box_off, i)];
                if (hb > r) r = hb;
            }
            int64_t m = orc_candidates(&s, i, x, y, z, r, &scr, &b0, &b1, &L);
            int32_t c = 0;
            uint64_t acc = 0;
            ORC_FOR_CAND(m, b0, b1, scr, j, {
                double r2 = orc_r2(x[i], y[i], z[i], x[j], y[j], z[j], L);
                if (orc_is_ngb(mode, i, j, r2, h[i], h[j])) {
                    c++;
                    acc += orc_splitmix64(orig ? (uint64_t)orig[j] : (uint64_t)j);
                }
            });
            cnt[t] = c;
            if (fp) fp[t] = acc;
        }
        free(scr.buf);
    }
    free(bh);
    orc_space_free(&s);
}

/* neighbour lists, ascending j, into out[off[t] .. off[t+1]) */
void orc_ngb_fill(int32_t mode, int64_t n, const double *x, const double *y,
                  const double *z, const double *h, int32_t nbox, const int64_t *box_off,
                  const double *box_L, int64_t nt, const int32_t *tgt, int32_t use_grid,
                  const int64_t *off, int32_t *out)
{
    (void)n;
    orc_space s;
    orc_space_init(&s, nbox, box_off, box_L, use_grid, x, y, z, h);
    double *bh = (double *)malloc((size_t)nbox * sizeof(double));
    for (int32_t b = 0; b < nbox; b++)
        bh[b] = (box_off[b + 1] > box_off[b]) ? orc_box_hmax(&s, box_off[b], h) : 0.0;
#pragma omp parallel
    {
        orc_scratch scr = {NULL, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t t = 0; t < nt; t++) {
            int64_t i = tgt[t], b0 = 0, b1 = 0;
            double L;
            double r = h[i];
            if (mode == 1) {
                double hb = bh[orc_box_of(nbox, box_off, i)];
                if (hb > r) r = hb;
            }
            int64_t m = orc_candidates(&s, i, x, y, z, r, &scr, &b0, &b1, &L);
            int64_t w = off[t];
            ORC_FOR_CAND(m, b0, b1, scr, j, {
                double r2 = orc_r2(x[i], y[i], z[i], x[j], y[j], z[j], L);
                if (orc_is_ngb(mode, i, j, r2, h[i], h[j]) && w < off[t + 1])
                    out[w++] = (int32_t)j;
            });
        }
        free(scr.buf);
    }
    free(bh);
    orc_space_free(&s);
}

/* ------------------------------------------------------------------ */
/* SPH kernels (READING: the paper prints none).  Support radius h,    */
/* q = r/h, W = C w(q) / h^3.                                           */
/*  0: cubic spline M4 in the Gadget form, C = 8/pi.                   */
/*  1: Wendland C6 (Dehnen & Aly 2012), C = 1365/(64 pi).              */
/* ------------------------------------------------------------------ */
double orc_kernel_norm(int32_t kernel)
{
    return kernel == 0 ? 8.0 / ORC_PI : 1365.0 / (64.0 * ORC_PI);
}

void orc_kernel_w(int32_t kernel, double q, double *w, double *dw)
{
    if (!(q < 1.0)) {
        *w = 0.0;
        *dw = 0.0;
        return;
    }
    if (kernel == 0) {
        if (q < 0.5) {
            *w = 1.0 - 6.0 * q * q + 6.0 * q * q * q;
            *dw = -12.0 * q + 18.0 * q * q;
        } else {
            double u = 1.0 - q;
            *w = 2.0 * u * u * u;
            *dw = -6.0 * u * u;
        }
    } else {
        double u = 1.0 - q;
        double u2 = u * u, u4 = u2 * u2, u7 = u4 * u2 * u, u8 = u4 * u4;
        *w = u8 * (1.0 + 8.0 * q + 25.0 * q * q + 32.0 * q * q * q);
        *dw = -22.0 * q * u7 * (1.0 + 7.0 * q + 16.0 * q * q);
    }
}

/* ------------------------------------------------------------------ */
/* Smoothing-length iteration.  The paper: the number of neighbours    */
/* within h_i is held fixed and varies locally by a few percent; the   */
/* particles that are done leave the active list and the search is     */
/* repeated for the rest (sections "Phases of Neighbour Search",       */
/* "Adaptive Neighbour Recycling").  READING, deterministic and made   */
/* of IEEE basic operations only (so that every implementation lands   */
/* on the same h):                                                      */
/*   repeat: n = |N_i(h)|; stop if |n - n_ngb| <= dn or after max_iter */
/*   evaluations; otherwise tighten the bracket (lo = h if n is low,   */
/*   hi = h if high) and scale h by g ~ (n_ngb/n)^(1/3) (since n grows */
/*   like h^3), g from two Halley steps for y^3 = t = n_ngb/n started  */
/*   at y = 1:  y = (1+2t)/(2+t);  g = y (y^3 + 2t) / (2y^3 + t).      */
/*   If h*g leaves the open bracket (lo, hi), take its midpoint.       */
/* ------------------------------------------------------------------ */
double orc_h_step(int32_t n, int32_t n_ngb, int32_t dn, double h, double *lo, double *hi)
{
    if (n < n_ngb - dn)
        *lo = h;
    else
        *hi = h;
    double t = (double)n_ngb / (double)n;
    double y = (1.0 + 2.0 * t) / (2.0 + t);
    double y3 = (y * y) * y;
    double g = (y * (y3 + 2.0 * t)) / (2.0 * y3 + t);
    double hn = h * g;
    if (!(hn > *lo && hn < *hi))
        hn = 0.5 * (*lo + *hi);
    return hn;
}

static int32_t orc_count_density(const orc_space *s, int64_t i, double h,
                                 const double *x, const double *y, const double *z,
                                 orc_scratch *scr)
{
    int64_t b0 = 0, b1 = 0;
    double L;
    int64_t m = orc_candidates(s, i, x, y, z, h, scr, &b0, &b1, &L);
    int32_t c = 0;
    double h2 = h * h;
    ORC_FOR_CAND(m, b0, b1, (*scr), j, {
        double r2 = orc_r2(x[i], y[i], z[i], x[j], y[j], z[j], L);
        if (r2 < h2) c++;
    });
    return c;
}

/* Density (READING after Springel 2005 / Springel & Hernquist 2002):
 *   rho_i   = sum_{j in N_i} m_j W(r_ij, h_i)
 *   drho/dh = -sum m_j (C/h^4) (3 w(q) + q w'(q))
 *   f_i     = 1 / (1 + h_i/(3 rho_i) drho/dh)
 * summed in ascending particle order, FP64.  The h loop above runs
 * first unless fixed_h. */
void orc_density(int64_t n, const double *x, const double *y, const double *z,
                 const double *h_in, const double *m, int32_t nbox,
                 const int64_t *box_off, const double *box_L, int64_t nt,
                 const int32_t *tgt, int32_t use_grid, int32_t kernel, int32_t n_ngb,
                 int32_t dn, int32_t max_iter, int32_t fixed_h, double *h_out,
                 int32_t *nngb, int32_t *iters, int32_t *converged, double *rho,
                 double *drhodh, double *fgrad, double *abs_drhodh)
{
    (void)n;
    orc_space s;
    orc_space_init(&s, nbox, box_off, box_L, use_grid, x, y, z, h_in);
    double C = orc_kernel_norm(kernel);
#pragma omp parallel
    {
        orc_scratch scr = {NULL, 0};
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < nt; t++) {
            int64_t i = tgt[t];
            double h = h_in[i], lo = 0.0, hi = INFINITY;
            int32_t it = 0, nc = 0, conv = 0;
            for (;;) {
                it++;
                nc = orc_count_density(&s, i, h, x, y, z, &scr);
                if (fixed_h) {
                    conv = 1;
                    break;
                }
                if (nc >= n_ngb - dn && nc <= n_ngb + dn) {
                    conv = 1;
                    break;
                }
                if (it >= max_iter)
                    break;
                h = orc_h_step(nc, n_ngb, dn, h, &lo, &hi);
            }
            /* sums at the final h */
            int64_t b0 = 0, b1 = 0;
            double L;
            int64_t mm = orc_candidates(&s, i, x, y, z, h, &scr, &b0, &b1, &L);
            double sw = 0.0, sd = 0.0, sa = 0.0, h2 = h * h;
            ORC_FOR_CAND(mm, b0, b1, scr, j, {
                double r2 = orc_r2(x[i], y[i], z[i], x[j], y[j], z[j], L);
                if (r2 < h2) {
                    double q = sqrt(r2) / h, w, dw;
                    orc_kernel_w(kernel, q, &w, &dw);
                    sw += m[j] * w;
                    double dd = m[j] * (3.0 * w + q * dw);
                    sd += dd;
                    sa += fabs(dd);
                }
            });
            double h3 = h * h * h, h4 = h3 * h;
            double r = C * sw / h3;
            double d = -C * sd / h4;
            h_out[t] = h;
            nngb[t] = nc;
            iters[t] = it;
            converged[t] = conv;
            rho[t] = r;
            drhodh[t] = d;
            fgrad[t] = 1.0 / (1.0 + h / (3.0 * r) * d);
            if (abs_drhodh) abs_drhodh[t] = C * sa / h4;
        }
        free(scr.buf);
    }
    orc_space_free(&s);
}

/* Hydro force (READING: Gadget-2 equations of Springel 2005 in energy
 * form, the paper's citation for the SPH method; no Balsara switch):
 *   P = (gamma-1) rho u,  c = sqrt(gamma P / rho),  Pf = f P / rho^2
 *   grad_i W(r,h) = r_ij/r * C w'(r/h)/h^4      (r_ij = x_i - x_j)
 *   w_ij = v_ij.r_ij / r if negative else 0,  v_sig = c_i + c_j - 3 w_ij
 *   Pi_ij = -(alpha/2) v_sig w_ij / ((rho_i + rho_j)/2)
 *   a_i    = -sum m_j [Pf_i dW(h_i) + Pf_j dW(h_j) + Pi_ij dWbar] r_ij/r
 *   du_i/dt =  Pf_i sum m_j v_ij.r_ij/r dW(h_i) + 1/2 sum m_j Pi_ij v_ij.r_ij/r dWbar
 *   vsigmax_i = max_j v_sig (0 without neighbours)
 * with dWbar = (dW(h_i) + dW(h_j))/2 over H_i, ascending j.
 * abs_a / abs_du: sums of the magnitudes of the per-pair terms. */
void orc_hydro(int64_t n, const double *x, const double *y, const double *z,
               const double *h, const double *m, const double *vx, const double *vy,
               const double *vz, const double *u, const double *rho, const double *fgrad,
               int32_t nbox, const int64_t *box_off, const double *box_L, int64_t nt,
               const int32_t *tgt, int32_t use_grid, int32_t kernel, double gamma,
               double alpha, double *ax, double *ay, double *az, double *dudt,
               double *vsigmax, double *abs_a, double *abs_du)
{
    (void)n;
    orc_space s;
    orc_space_init(&s, nbox, box_off, box_L, use_grid, x, y, z, h);
    double C = orc_kernel_norm(kernel);
    double *bh = (double *)malloc((size_t)nbox * sizeof(double));
    for (int32_t b = 0; b < nbox; b++)
        bh[b] = (box_off[b + 1] > box_off[b]) ? orc_box_hmax(&s, box_off[b], h) : 0.0;
#pragma omp parallel
    {
        orc_scratch scr = {NULL, 0};
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < nt; t++) {
            int64_t i = tgt[t], b0 = 0, b1 = 0;
            double L;
            double rq = h[i], hb = bh[orc_box_of(nbox, box_off, i)];
            if (hb > rq) rq = hb;
            int64_t mm = orc_candidates(&s, i, x, y, z, rq, &scr, &b0, &b1, &L);
            double Pi = (gamma - 1.0) * rho[i] * u[i];
            double ci = sqrt(gamma * Pi / rho[i]);
            double Pfi = fgrad[i] * Pi / (rho[i] * rho[i]);
            double sax = 0, say = 0, saz = 0, sdu = 0, vmax = 0, sabs = 0, sdabs = 0;
            ORC_FOR_CAND(mm, b0, b1, scr, j, {
                double dx = orc_fold(x[i] - x[j], L);
                double dy = orc_fold(y[i] - y[j], L);
                double dz = orc_fold(z[i] - z[j], L);
                double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                if (orc_is_ngb(1, i, j, r2, h[i], h[j])) {
                    double Pj = (gamma - 1.0) * rho[j] * u[j];
                    double cj = sqrt(gamma * Pj / rho[j]);
                    if (r2 > 0.0) {
                        double r = sqrt(r2);
                        double w, dwi, dwj;
                        orc_kernel_w(kernel, r / h[i], &w, &dwi);
                        orc_kernel_w(kernel, r / h[j], &w, &dwj);
                        double hi4 = h[i] * h[i] * h[i] * h[i];
                        double hj4 = h[j] * h[j] * h[j] * h[j];
                        double dWi = C * dwi / hi4, dWj = C * dwj / hj4;
                        double dWb = 0.5 * (dWi + dWj);
                        double vdx = vx[i] - vx[j], vdy = vy[i] - vy[j], vdz = vz[i] - vz[j];
                        double vr = vdx * dx + vdy * dy + vdz * dz;
                        double wij = vr < 0.0 ? vr / r : 0.0;
                        double vsig = ci + cj - 3.0 * wij;
                        double Pfj = fgrad[j] * Pj / (rho[j] * rho[j]);
                        double visc = -(alpha / 2.0) * vsig * wij / (0.5 * (rho[i] + rho[j]));
                        double fac = m[j] * (Pfi * dWi + Pfj * dWj + visc * dWb);
                        sax -= fac * dx / r;
                        say -= fac * dy / r;
                        saz -= fac * dz / r;
                        double d1 = m[j] * Pfi * (vr / r) * dWi;
                        double d2 = 0.5 * m[j] * visc * (vr / r) * dWb;
                        sdu += d1 + d2;
                        sabs += fabs(fac);
                        sdabs += fabs(d1) + fabs(d2);
                        if (vsig > vmax) vmax = vsig;
                    } else {
                        double vsig = ci + cj;
                        if (vsig > vmax) vmax = vsig;
                    }
                }
            });
            ax[t] = sax;
            ay[t] = say;
            az[t] = saz;
            dudt[t] = sdu;
            vsigmax[t] = vmax;
            if (abs_a) abs_a[t] = sabs;
            if (abs_du) abs_du[t] = sdabs;
        }
        free(scr.buf);
    }
    free(bh);
    orc_space_free(&s);
}

/* Gadget3's production SPH, after the scheme the paper cites for it in its
 * introduction (Beck et al.): the hydro force of orc_hydro with
 *  - a viscosity coefficient per particle, alpha_ij = (alpha_i + alpha_j)/2
 *    in place of alpha (the coefficient is evolved in time by the caller);
 *  - artificial conduction of internal energy (Price 2008):
 *      du_i/dt += sum_j m_j alpha_u v_ij^u (u_i - u_j) F_ij / rho_ij,
 *    v_ij^u = sqrt(|P_i - P_j| / rho_ij), rho_ij = (rho_i + rho_j)/2,
 *    F_ij = (W'(r, h_i) + W'(r, h_j))/2 (the radial kernel derivative, <= 0);
 *  - the velocity divergence
 *      div v_i = -(1/rho_i) sum_j m_j (v_i - v_j) . (x_i - x_j)/r W'(r, h_i);
 *  - the rate of the viscosity switch (Morris & Monaghan 1997)
 *      dalpha_i/dt = -(alpha_i - alpha_min) ell c_i / h_i
 *                    + max(-div v_i, 0) (alpha_max - alpha_i).
 * The paper prints none of these formulas: parity unpinned against the
 * paper (pinned by the tests through the standard case, conservation and
 * closed forms). */
void orc_hydro_prod(int64_t n, const double *x, const double *y, const double *z,
                    const double *h, const double *m, const double *vx, const double *vy,
                    const double *vz, const double *u, const double *rho, const double *fgrad,
                    const double *alpha_p, int32_t nbox, const int64_t *box_off,
                    const double *box_L, int64_t nt, const int32_t *tgt, int32_t use_grid,
                    int32_t kernel, double gamma, double alpha_u, double alpha_min,
                    double alpha_max, double ell, double *ax, double *ay, double *az,
                    double *dudt, double *vsigmax, double *divv, double *dalphadt,
                    double *abs_a, double *abs_du, double *abs_divv)
{
    (void)n;
    orc_space s;
    orc_space_init(&s, nbox, box_off, box_L, use_grid, x, y, z, h);
    double C = orc_kernel_norm(kernel);
    double *bh = (double *)malloc((size_t)nbox * sizeof(double));
    for (int32_t b = 0; b < nbox; b++)
        bh[b] = (box_off[b + 1] > box_off[b]) ? orc_box_hmax(&s, box_off[b], h) : 0.0;
#pragma omp parallel
    {
        orc_scratch scr = {NULL, 0};
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < nt; t++) {
            int64_t i = tgt[t], b0 = 0, b1 = 0;
            double L;
            double rq = h[i], hb = bh[orc_box_of(nbox, box_off, i)];
            if (hb > rq) rq = hb;
            int64_t mm = orc_candidates(&s, i, x, y, z, rq, &scr, &b0, &b1, &L);
            double Pi = (gamma - 1.0) * rho[i] * u[i];
            double ci = sqrt(gamma * Pi / rho[i]);
            double Pfi = fgrad[i] * Pi / (rho[i] * rho[i]);
            double sax = 0, say = 0, saz = 0, sdu = 0, vmax = 0, sabs = 0, sdabs = 0, sdiv = 0,
                   sdivabs = 0;
            ORC_FOR_CAND(mm, b0, b1, scr, j, {
                double dx = orc_fold(x[i] - x[j], L);
                double dy = orc_fold(y[i] - y[j], L);
                double dz = orc_fold(z[i] - z[j], L);
                double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                if (orc_is_ngb(1, i, j, r2, h[i], h[j])) {
                    double Pj = (gamma - 1.0) * rho[j] * u[j];
                    double cj = sqrt(gamma * Pj / rho[j]);
                    if (r2 > 0.0) {
                        double r = sqrt(r2);
                        double w, dwi, dwj;
                        orc_kernel_w(kernel, r / h[i], &w, &dwi);
                        orc_kernel_w(kernel, r / h[j], &w, &dwj);
                        double hi4 = h[i] * h[i] * h[i] * h[i];
                        double hj4 = h[j] * h[j] * h[j] * h[j];
                        double dWi = C * dwi / hi4, dWj = C * dwj / hj4;
                        double dWb = 0.5 * (dWi + dWj);
                        double rhob = 0.5 * (rho[i] + rho[j]);
                        double vdx = vx[i] - vx[j], vdy = vy[i] - vy[j], vdz = vz[i] - vz[j];
                        double vr = vdx * dx + vdy * dy + vdz * dz;
                        double wij = vr < 0.0 ? vr / r : 0.0;
                        double vsig = ci + cj - 3.0 * wij;
                        double Pfj = fgrad[j] * Pj / (rho[j] * rho[j]);
                        double aij = 0.5 * (alpha_p[i] + alpha_p[j]);
                        double visc = -(aij / 2.0) * vsig * wij / rhob;
                        double fac = m[j] * (Pfi * dWi + Pfj * dWj + visc * dWb);
                        sax -= fac * dx / r;
                        say -= fac * dy / r;
                        saz -= fac * dz / r;
                        double d1 = m[j] * Pfi * (vr / r) * dWi;
                        double d2 = 0.5 * m[j] * visc * (vr / r) * dWb;
                        double vu = sqrt(fabs(Pi - Pj) / rhob);
                        double d3 = m[j] * alpha_u * vu * (u[i] - u[j]) * dWb / rhob;
                        sdu += d1 + d2 + d3;
                        sdiv += m[j] * (vr / r) * dWi;
                        sdivabs += fabs(m[j] * (vr / r) * dWi);
                        sabs += fabs(fac);
                        sdabs += fabs(d1) + fabs(d2) + fabs(d3);
                        if (vsig > vmax) vmax = vsig;
                    } else {
                        double vsig = ci + cj;
                        if (vsig > vmax) vmax = vsig;
                    }
                }
            });
            double dv = -sdiv / rho[i];
            ax[t] = sax;
            ay[t] = say;
            az[t] = saz;
            dudt[t] = sdu;
            vsigmax[t] = vmax;
            divv[t] = dv;
            dalphadt[t] = -(alpha_p[i] - alpha_min) * ell * ci / h[i] +
                          (dv < 0.0 ? -dv : 0.0) * (alpha_max - alpha_p[i]);
            if (abs_a) abs_a[t] = sabs;
            if (abs_du) abs_du[t] = sdabs;
            if (abs_divv) abs_divv[t] = sdivabs / rho[i];
        }
        free(scr.buf);
    }
    free(bh);
    orc_space_free(&s);
}

/* Candidate superset of one group (section "Implementation of Neighbour
 * Recycling ..."): every particle of the box closer than R + max(h_i) to
 * the group's first particle, with R the largest member distance
 * (READING: the measured group radius; the paper's nominal R also works).
 * Returns the count; used by the statistical pin of Eq. (1). */
int64_t orc_group_superset_size(int64_t n, const double *x, const double *y,
                                const double *z, const double *h, int32_t nbox,
                                const int64_t *box_off, const double *box_L,
                                const int32_t *act, int64_t g0, int64_t g1,
                                double R_nominal)
{
    (void)n;
    int64_t i0 = act[g0];
    int64_t b = orc_box_of(nbox, box_off, i0);
    double L = box_L[b];
    double R2 = 0.0, hm = 0.0;
    for (int64_t k = g0; k < g1; k++) {
        int64_t i = act[k];
        double r2 = orc_r2(x[i0], y[i0], z[i0], x[i], y[i], z[i], L);
        if (r2 > R2) R2 = r2;
        if (h[i] > hm) hm = h[i];
    }
    double R = R_nominal > 0.0 ? R_nominal : sqrt(R2);
    double rad = R + hm;
    int64_t c = 0;
    for (int64_t j = box_off[b]; j < box_off[b + 1]; j++) {
        double r2 = orc_r2(x[i0], y[i0], z[i0], x[j], y[j], z[j], L);
        if (r2 < rad * rad) c++;
    }
    return c;
}
