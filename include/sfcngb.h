/*
 * sfcngb.h -- grouped ("recycled") SPH neighbour search on one AMD MI355X.
 *
 * The method is that of Ragagnin, Tchipev, Bader, Dolag, Hammer,
 * "Exploiting the Space Filling Curve Ordering of Particles in the
 * Neighbour Search of Gadget3" (arXiv:1810.09898): particles are ordered
 * along the Peano-Hilbert curve, active particles that follow each other on
 * the curve and lie close together are grouped, each group walks the octree
 * once with an enlarged radius to obtain a common candidate superset, and
 * every member filters that superset down to its own neighbours before the
 * density and hydro-force sums.
 *
 * Conventions shared by every call
 *  - Every array pointer in sfc_particles, sfc_density_out, sfc_hydro_out and
 *    sfc_verify is a DEVICE pointer owned by the caller; the library never
 *    allocates or frees device memory.  Host pointers are marked "host".
 *  - All work is enqueued asynchronously on the context's HIP stream; no call
 *    except sfc_status_read synchronises, so a sequence of calls may be
 *    captured into a HIP graph (sfc_graph_begin / sfc_graph_end).
 *  - Return codes: SFC_OK, or a negative code.  Host-detected errors are
 *    returned synchronously and nothing is enqueued; sfc_ctx_last_error()
 *    gives a message.  Conditions detected on the device are accumulated in a
 *    status block read by sfc_status_read().
 *  - A particle set is a concatenation of independent periodic boxes; box b
 *    owns particles [box_off[b], box_off[b+1]) and has side box_L[b].  Every
 *    coordinate must lie in [0, box_L[b]).  A single box is a batch of one.
 *  - Positions and smoothing lengths are FP64; masses, velocities, internal
 *    energies, densities and forces are FP32.
 *  - Not thread-safe per context: one context per stream.
 */
#ifndef SFCNGB_H
#define SFCNGB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SFC_API __attribute__((visibility("default")))

#define SFC_OK 0
#define SFC_EINVAL (-1)     /* bad argument (null pointer, size, parameter range) */
#define SFC_EWORKSPACE (-2) /* no workspace bound, or too small for the call */
#define SFC_EHIP (-3)       /* a HIP runtime call or kernel launch failed */
#define SFC_EOVERFLOW (-4)  /* device-side capacity exceeded (reported by sfc_status_read) */
#define SFC_EORDER (-5)     /* call out of order (e.g. density before group_ngb_search) */

#define SFC_WAVE_GROUP_MAX 64 /* a group is processed by one 64-lane wavefront */

/* ---------------------------------------------------------------------- */
/* Context and workspace                                                   */
/* ---------------------------------------------------------------------- */
typedef struct sfc_ctx sfc_ctx;

/* Create a context bound to `hip_stream` (a hipStream_t; NULL = the null
 * stream) on the current HIP device.  *out receives the handle. */
SFC_API int sfc_ctx_create(sfc_ctx **out, void *hip_stream);
SFC_API void sfc_ctx_destroy(sfc_ctx *ctx);
SFC_API int sfc_ctx_set_stream(sfc_ctx *ctx, void *hip_stream);
/* Schedule statistics (sfc_status.sched_*): on = 1 makes every workgroup of
 * the density group kernel and every wave of the hydro member kernel record
 * its start and end on the device's constant clock (four atomics each, into
 * one of eight per-XCD slots of the status block); on = 0 (the default)
 * records nothing.  SFC_EINVAL for other values. */
SFC_API int sfc_ctx_set_trace(sfc_ctx *ctx, int on);
/* Message of the last host-detected error (static storage of the context). */
SFC_API const char *sfc_ctx_last_error(const sfc_ctx *ctx);
/* Number of compute units of the context's device. */
SFC_API int32_t sfc_ctx_cu_count(const sfc_ctx *ctx);

/* Sizes that fix the workspace layout. */
typedef struct {
    int64_t n;           /* particles over all boxes, >= 1, < 2^30; the octree's node
                            capacity, n + 22 n / (n_leaf_min + 1) + n_boxes + 64, must
                            stay below 2^28 (SFC_EINVAL otherwise) */
    int32_t n_boxes;     /* >= 1 */
    int32_t n_leaf_min;  /* smallest leaf size tree_build will be given (>= 1) */
    int32_t t_cand_max;  /* largest candidate tile any call will use (64..8192, multiple of 64) */
    int32_t cand_per_particle; /* capacity of the candidate buffer that holds every group's
                                  superset, in candidates per particle (0 = 96; 1..4096).
                                  Groups that do not fit finish member by member (slower,
                                  same results) and are counted in sfc_status.n_overflow. */
    int32_t keep_supersets;    /* 1: the density and the hydro pass keep their group supersets
                                  in buffers of their own (twice the candidate memory), so
                                  that later calls with reuse = 1 filter them again instead
                                  of walking; 0: one buffer, no reuse */
} sfc_dims;

/* Bytes of device workspace needed for `dims` (0 on invalid dims). */
SFC_API size_t sfc_workspace_bytes(const sfc_dims *dims);
/* Bind a caller-owned device workspace of ws_bytes >= sfc_workspace_bytes(dims)
 * to the context and clear its status block.  The workspace holds the sort
 * buffers, the octree, the active list and groups, the candidate supersets
 * of the groups, per-particle hydro records and the status block; it must
 * stay alive while the context uses it. */
SFC_API int sfc_workspace_bind(sfc_ctx *ctx, const sfc_dims *dims, void *ws, size_t ws_bytes);

/* ---------------------------------------------------------------------- */
/* Particles                                                               */
/* ---------------------------------------------------------------------- */
typedef struct {
    int64_t n;                   /* must equal the bound dims.n */
    int32_t n_boxes;             /* must equal the bound dims.n_boxes */
    const int64_t *box_off_host; /* host [n_boxes+1], box_off_host[0] = 0, ends at n */
    const int64_t *box_off;      /* device copy of box_off_host */
    const double *box_L;         /* device [n_boxes], > 0 */
    double *x, *y, *z;           /* [n] positions in [0, L) */
    double *h;                   /* [n] smoothing length = kernel support radius, > 0 */
    float *m;                    /* [n] masses */
    float *vx, *vy, *vz, *u;     /* [n] velocities, internal energy (hydro only; else NULL) */
    float *rho, *fgrad;          /* [n] density and grad-h factor f (state; hydro reads them) */
    uint8_t *active;             /* [n] nonzero = active this step */
    uint32_t *orig;              /* [n] caller's particle id, carried through the sort (nullable) */
} sfc_particles;

/* Peano-Hilbert keys and the stable (box, key) order (the paper's
 * space-filling-curve ordering, section "Impact of the Neighbour Search in
 * the Gadget3 Performance"; Hilbert variant: Skilling's transpose algorithm,
 * 21 bits per axis, cell = floor(x/L * 2^21) clamped).  Out of place: every
 * non-NULL array of `in` is gathered into the same array of `out` in sorted
 * order (equal keys keep input order); out->active receives 1 where
 * in->active is nonzero, else 0.  out->orig receives in->orig permuted,
 * or the input index if in->orig is NULL.  keys_out: device [n], the sorted
 * keys.  perm_out: device [n] or NULL, the input index of each output slot.
 * in and out must not alias. */
SFC_API int sfc_sort(sfc_ctx *ctx, const sfc_particles *in, sfc_particles *out, uint64_t *keys_out,
             uint32_t *perm_out);

/* The sort of sfc_sort without any device allocation or bound workspace,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments and the same results, bit for bit, as sfc_sort; the records,
 * keys, payloads and histograms live in a static device array of
 * SFC_STATIC_SCRATCH_BYTES that the library holds on every device it runs on
 * (from the first sfc_ctx_create there) until the process ends.  Limit:
 * 1 <= in->n <= SFC_SORT_STATIC_MAX_N, else SFC_EINVAL with nothing
 * enqueued.  Every call on one device shares that device's scratch: calls
 * that overlap on one device (other streams, other contexts) race, so
 * serialise them.  Leaves the context's tree, groups and kept supersets as
 * they were. */
#define SFC_STATIC_SCRATCH_BYTES (32u << 20)
#define SFC_SORT_STATIC_MAX_N 262144
SFC_API int sfc_sort_static(sfc_ctx *ctx, const sfc_particles *in, sfc_particles *out,
                            uint64_t *keys_out, uint32_t *perm_out);

/* Octree over sorted particles (the tree of section "Neighbour Search in
 * Gadget3"): a node is a non-empty Hilbert cell (keys sharing the top 3l bits
 * at level l), the box is the root, a node with <= n_leaf particles (or at
 * level 21) is a leaf, nodes are stored in depth-first pre-order with skip
 * links, and each node keeps the min/max of its particles' coordinates and
 * the max of their h.  keys: the sorted keys from sfc_sort.  n_leaf >=
 * dims.n_leaf_min. */
SFC_API int tree_build(sfc_ctx *ctx, const sfc_particles *p, const uint64_t *keys, int32_t n_leaf);
/* Recompute every node's max h from p->h (hydro_force and the hydro
 * verify pass do this themselves). */
SFC_API int tree_refit_hmax(sfc_ctx *ctx, const sfc_particles *p);
/* Recompute every node's bounding box and max h after the particles moved
 * (same order, same tree structure: a node still holds the same particles,
 * its box is whatever they now span).  Kept supersets stay kept. */
SFC_API int tree_refit(sfc_ctx *ctx, const sfc_particles *p);

/* ---------------------------------------------------------------------- */
/* Grouping and neighbour search                                           */
/* ---------------------------------------------------------------------- */
#define SFC_POLICY_COUNT 0 /* n_group_max consecutive actives */
#define SFC_POLICY_PAPER 1 /* greedy radius rule, R = f h_0 */
#define SFC_POLICY_TREE 2  /* the actives of one octree node of depth `level` */

typedef struct {
    int32_t policy;      /* SFC_POLICY_COUNT, SFC_POLICY_PAPER or SFC_POLICY_TREE */
    int32_t n_group_max; /* 1..64 members per group */
    double f;            /* paper policy: a particle joins while closer than f*h_0 to the
                            group's first member (section "Adaptive Neighbour Recycling") */
    int32_t level;       /* tree policy (0..21): a particle joins while it lies in the octree
                            node of depth `level` that holds the group's first member, or, when
                            that member's leaf is shallower, in that leaf (section "Neighbour
                            Recycling": groups as the leaves inside nodes of one tree depth).
                            Node = Hilbert cell of the last tree_build, so the tree and its
                            n_leaf decide the leaves. */
    int32_t t_cand;      /* in a per-box table only: the most candidates a group superset of
                            this box may hold in the density and hydro calls that follow
                            (0 = the call's t_cand; else clamped to [64, the call's t_cand]);
                            a group whose superset exceeds it finishes member by member */
} sfc_group_params;

/* Optional neighbour-set dump (testing): for every active particle i,
 * count[i] = |neighbour set| and fingerprint[i] = sum over neighbours j of
 * splitmix64(orig[j]) mod 2^64 (orig = the sorted particles' orig array);
 * with list != NULL the neighbours' sorted indices, ascending, are written to
 * list[list_off[i] .. list_off[i+1]).  Inactive slots are left untouched.
 * mode 0: density set  { j : |x_j - x_i| < h_i }  (self included);
 * mode 1: hydro set    { j != i : |x_j - x_i| < max(h_i, h_j) }
 * (section "Phases of Neighbour Search"). */
typedef struct {
    int32_t mode;
    int32_t *count;          /* device [n] */
    uint64_t *fingerprint;   /* device [n] or NULL */
    const int64_t *list_off; /* device [n+1] or NULL */
    int32_t *list;           /* device [list_cap] or NULL */
    int64_t list_cap;
} sfc_verify;

/* Active list (curve order) and groups (section "Implementation of
 * Neighbour Recycling using a Space Filling Curve"): one greedy pass over
 * the actives in curve order, as the paper runs it: the first active opens
 * a group, the next active joins while the policy allows and the group has
 * fewer than n_group_max members, otherwise it opens the next group; a box
 * boundary also opens a group.  (Computed in parallel; the groups are those
 * of the sequential pass exactly.)  gp: host pointer to one parameter set used for every box,
 * or NULL when gp_box is given.  gp_box: device [n_boxes] per-box parameters
 * or NULL.  With verify != NULL the walk and filter run once for every group
 * and write the neighbour sets (no physics); t_cand is the candidate tile
 * for that pass. */
SFC_API int group_ngb_search(sfc_ctx *ctx, const sfc_particles *p, const sfc_group_params *gp,
                     const sfc_group_params *gp_box, const sfc_verify *verify, int32_t t_cand);

/* ---------------------------------------------------------------------- */
/* Density and hydro force                                                 */
/* ---------------------------------------------------------------------- */
#define SFC_KERNEL_CUBIC 0 /* cubic spline M4, support h */
#define SFC_KERNEL_WC6 1   /* Wendland C6, support h */
#define SFC_ACCUM_F32 0    /* FP32 pair terms, compensated (Kahan) sums */
#define SFC_ACCUM_F64 1    /* FP64 pair terms and sums */

typedef struct {
    int32_t kernel;   /* SFC_KERNEL_* */
    int32_t n_ngb;    /* target neighbour number */
    int32_t dn;       /* accepted window |n - n_ngb| <= dn */
    int32_t max_iter; /* h evaluations per particle (>= 1) */
    int32_t fixed_h;  /* 1: keep h, evaluate once */
    int32_t accum;    /* SFC_ACCUM_* */
    double skin;      /* group walk radius = R_g + skin * max h (>= 1) */
    int32_t t_cand;   /* candidate tile (multiple of 64, <= dims.t_cand_max) */
    int32_t reuse;    /* 1: filter the supersets kept by the last walking density call
                         (dims.keep_supersets; same groups, same t_cand) instead of walking */
} sfc_density_params;

typedef struct {
    float *drhodh;       /* device [n] or NULL */
    int32_t *nngb;       /* device [n] or NULL: final neighbour count */
    int32_t *iters;      /* device [n] or NULL: h evaluations */
    uint8_t *converged;  /* device [n] or NULL */
    double *rho64, *drhodh64, *fgrad64; /* device [n] or NULL (written with SFC_ACCUM_F64) */
} sfc_density_out;

/* Superset reuse across steps: the Verlet-list idea that section "Neighbour
 * Recycling in Gadget3" recalls (one superset kept over several steps),
 * applied to the group supersets.  With
 * dims.keep_supersets, a walking density or hydro call keeps its supersets,
 * the group centres and radii, and a snapshot of x, y, z (density) and h
 * (hydro).  The particles may then move and change h (keeping their order;
 * call tree_refit), and a call with reuse = 1 skips the walks: with delta =
 * the largest displacement since the snapshot (minimum image) and, for
 * hydro, dh = the largest growth of any h, a member keeps its group's
 * superset while
 *   density: h_i + |x_i - c| + delta <= R_g + skin * max h
 *   hydro:   h_i + |x_i - c| + delta <= R_g + (skin - 1) max h + max h  and
 *            |x_i - c| + delta + dh <= R_g + (skin - 1) max h
 * (c the group's centre; R_g and max h as at the walk), and otherwise
 * finishes as a member whose h outgrew the superset.  A reuse call computes
 * only the members whose active flag is set now, so that a finer timestep
 * bin (a subset of the grouped particles) reuses the supersets of the step
 * that grouped them all; an active particle outside the kept groups sets
 * SFC_ST_REUSE_ACTIVE.  Results are those of a walking call.  sfc_sort,
 * tree_build and group_ngb_search drop the kept supersets.
 * The particle arrays are the ones the walking call saw, in the same order
 * (moved in place by the caller).  density and hydro_force with reuse = 1
 * refit the node boxes themselves (tree_refit).  Errors (host side,
 * nothing enqueued): SFC_EORDER when no superset is kept, SFC_EINVAL for a
 * t_cand other than the walking call's.  keep_supersets enlarges the
 * workspace (a second candidate buffer and group records, snapshots);
 * sfc_workspace_bytes includes it. */

/* Density pass over the active particles of the last group_ngb_search
 * (sections "Phases of Neighbour Search" and "Adaptive Neighbour
 * Recycling"): each group walks the octree once (ball R_g + skin * max h
 * around its first member) and keeps the candidate superset; every member
 * iterates its h on that superset with integer neighbour counts n = |{j :
 * r_ij < h}|: stop when |n - n_ngb| <= dn or after max_iter evaluations,
 * otherwise narrow a bracket (lo = h if n is low, hi = h if high) and move
 * to h * g, g two Halley steps for (n_ngb/n)^(1/3), or to the bracket's
 * midpoint when h * g leaves it.  A member whose h outgrows the superset
 * walks once for a superset of its own.  Then
 *   rho_i = sum_j m_j W(r_ij, h_i),  drho/dh_i,  f_i = 1/(1 + h_i/(3 rho_i) drho/dh_i)
 * are written to p->h, p->rho, p->fgrad and `out` at the active slots.
 * Uses the candidate buffer of the workspace; the tree's max h is left as it
 * was (hydro_force refreshes it). */
SFC_API int density(sfc_ctx *ctx, sfc_particles *p, const sfc_density_params *dp,
            sfc_density_out *out);

#define SFC_HYDRO_STANDARD 0   /* one viscosity coefficient alpha */
#define SFC_HYDRO_PRODUCTION 1 /* Gadget3's production SPH, see hydro_force */

typedef struct {
    int32_t kernel; /* SFC_KERNEL_* */
    double gamma;   /* adiabatic index */
    double alpha;   /* artificial viscosity (SFC_HYDRO_STANDARD) */
    int32_t accum;  /* SFC_ACCUM_* */
    int32_t t_cand; /* candidate tile */
    double skin;    /* group walk radius = R_g + (skin - 1) * max h + max(max h, h_j), skin >= 1 */
    int32_t reuse;  /* 1: filter the supersets kept by the last walking hydro call */
    int32_t physics;           /* SFC_HYDRO_*; the fields below are read by SFC_HYDRO_PRODUCTION */
    const float *alpha_i;      /* device [n]: each particle's viscosity coefficient (>= 0),
                                  evolved in time by the caller from out->dalphadt */
    double alpha_u;            /* artificial conduction coefficient (>= 0) */
    double alpha_min, alpha_max; /* the viscosity switch's floor and ceiling */
    double ell;                /* the switch's decay: rate ell * c_i / h_i (>= 0) */
} sfc_hydro_params;

typedef struct {
    float *ax, *ay, *az, *dudt, *vsigmax;     /* device [n] */
    double *ax64, *ay64, *az64, *dudt64;      /* device [n] or NULL (SFC_ACCUM_F64) */
    float *divv, *dalphadt;                   /* device [n] or NULL (SFC_HYDRO_PRODUCTION):
                                                 velocity divergence, d alpha_i / dt */
} sfc_hydro_out;

/* Hydro force over the active particles of the last group_ngb_search:
 * neighbours j != i closer than max(h_i, h_j) (section "Phases of Neighbour
 * Search"); SPH pressure force with artificial viscosity in the Gadget-2
 * form:  P_i = (gamma - 1) rho_i u_i,  c_i = sqrt(gamma P_i / rho_i),
 *   a_i = -sum_j m_j (f_i P_i/rho_i^2 W'_i + f_j P_j/rho_j^2 W'_j + Pi_ij W'_ij) x_ij / r,
 *   du_i/dt = sum_j m_j (f_i P_i/rho_i^2 W'_i + Pi_ij W'_ij / 2) v_ij . x_ij / r,
 * W'_i = dW(r, h_i)/dr, W'_ij = (W'_i + W'_j)/2, Pi_ij = -(alpha/2) v_sig w_ij / rho_ij,
 * w_ij = min(v_ij . x_ij / r, 0), v_sig = c_i + c_j - 3 w_ij, rho_ij = (rho_i + rho_j)/2.
 * SFC_HYDRO_PRODUCTION is Gadget3's production SPH after the scheme the
 * paper cites for it in its introduction (no formula of it is printed in
 * the paper): alpha is replaced by (alpha_i + alpha_j)/2, du_i/dt gains the
 * artificial conduction sum_j m_j alpha_u sqrt(|P_i - P_j| / rho_ij)
 * (u_i - u_j) W'_ij / rho_ij, and out->divv, out->dalphadt (when not NULL)
 * receive div v_i = -(1/rho_i) sum_j m_j W'_i v_ij . x_ij / r and the switch's
 * rate -(alpha_i - alpha_min) ell c_i / h_i + max(-div v_i, 0) (alpha_max - alpha_i).
 * Requires vx, vy, vz, u, rho, fgrad.  First recomputes every node's max h
 * from p->h (h may have changed since the tree was built), then each group
 * walks once with R_g + max(max member h, h_j). */
SFC_API int hydro_force(sfc_ctx *ctx, const sfc_particles *p, const sfc_hydro_params *hp,
                sfc_hydro_out *out);

/* ---------------------------------------------------------------------- */
/* Status, inspection, graphs                                              */
/* ---------------------------------------------------------------------- */
#define SFC_ST_LIST_OVERFLOW 0x1u   /* verify list capacity exceeded */
#define SFC_ST_NODE_OVERFLOW 0x2u   /* octree larger than its workspace bound */
#define SFC_ST_BAD_INPUT 0x4u       /* coordinate outside its box or h <= 0 */
#define SFC_ST_GUARD 0x8u           /* a loop hit its trip limit (corrupt tree or h loop) */
#define SFC_ST_REUSE_ACTIVE 0x10u   /* a reuse call found active particles outside the kept
                                       groups (they were not computed) */

typedef struct {
    uint32_t flags;          /* SFC_ST_* bits */
    int32_t n_nodes;         /* nodes of the last tree */
    int32_t n_active;        /* actives of the last group_ngb_search */
    int32_t n_groups;        /* groups of the last group_ngb_search */
    int64_t n_deferred;      /* members finished on their own walk (since bind) */
    int64_t n_overflow;      /* groups whose superset exceeded t_cand (since bind) */
    int64_t n_not_converged; /* particles that hit max_iter (since bind) */
    int64_t sum_cand;        /* sum of group superset sizes (since bind) */
    int64_t n_walks;         /* tree walks (since bind) */
    int64_t sum_iters;       /* h evaluations (since bind) */
    int64_t sum_tests;       /* member x superset-candidate tests of the filters (since bind) */
    int64_t sum_pairs;       /* neighbour pairs summed by density and hydro (since bind) */
    /* With sfc_ctx_set_trace(ctx, 1): the schedule of the last density pass
     * [0] and the last hydro pass [1] (device's constant clock; zero while
     * tracing is off): the workgroups of the density group
     * kernel, resp. the waves of the hydro member kernel, that ran, the time
     * from the first one's start to the last one's end, and the tail: the
     * last end minus the mean end (how long the device ran for its slowest
     * unit after the average one had finished). */
    int64_t sched_units[2];
    double sched_span_us[2];
    double sched_tail_us[2];
} sfc_status;

/* Synchronise the stream and copy the status block to *out.  Returns
 * SFC_EOVERFLOW if an overflow flag is set, SFC_OK otherwise. */
SFC_API int sfc_status_read(sfc_ctx *ctx, sfc_status *out);
/* Zero the flags and the counters of the status block (enqueued;
 * capturable).  n_nodes, n_active and n_groups describe the current tree and
 * grouping and are kept. */
SFC_API int sfc_status_clear(sfc_ctx *ctx);

/* Device pointers into the bound workspace (valid until re-bind). */
typedef struct {
    int32_t capacity;   /* node capacity */
    const int32_t *n_nodes;     /* device scalar */
    const int32_t *info;        /* [capacity][4]: first, count, skip, level | leaf<<8 */
    const double *lo;           /* [capacity][4]: min x, min y, min z, max h */
    const double *hi;           /* [capacity][4]: max x, max y, max z, 0 */
    const int32_t *box_root;    /* [n_boxes+1]: first node of each box, then n_nodes */
    const int32_t *act;         /* [n]: sorted indices of the actives */
    const int32_t *n_act;       /* device scalar */
    const int32_t *goff;        /* [n+1]: group g = act[goff[g] .. goff[g+1]) */
    const int32_t *n_groups;    /* device scalar */
} sfc_views;
SFC_API int sfc_get_views(const sfc_ctx *ctx, sfc_views *out);

typedef struct sfc_graph sfc_graph;
/* Begin capturing the context's stream; the calls until sfc_graph_end are
 * recorded, not run. */
SFC_API int sfc_graph_begin(sfc_ctx *ctx);
SFC_API int sfc_graph_end(sfc_ctx *ctx, sfc_graph **out);
SFC_API int sfc_graph_launch(sfc_ctx *ctx, sfc_graph *g);
SFC_API void sfc_graph_destroy(sfc_graph *g);

#ifdef __cplusplus
}
#endif
#endif /* SFCNGB_H */
