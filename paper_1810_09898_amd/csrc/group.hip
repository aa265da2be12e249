// group.hip -- active list and the greedy grouping along the Hilbert curve.
//
// The grouping is the paper's sequential loop (section "Implementation of
// Neighbour Recycling using a Space Filling Curve"): walking the actives in
// curve order, the first one opens a group, each next one joins while the
// policy allows (paper policy: closer than f*h_0 to the group's first
// member, h_0 being that member's h; count policy: no distance test; tree
// policy: same octree node of a chosen depth), at most n_group_max members,
// never across a box, and the first one that may not join opens the next
// group.  Its result is computed in parallel without changing it:
//
//  1. nxt(k) for every active k: the position that would open the next
//     group if k opened one (the first later active that fails the test
//     against k, or k + n_group_max, or the box's end).  The group starts are
//     then exactly the orbit of the first active under nxt.
//  2. The actives are cut into blocks of GB1 positions.  Since nxt(k) - k <=
//     64, the orbit enters a block within its first 64 positions, so each
//     block is described by a map: for each entry e in [0, 64), the position
//     where the orbit leaves the block and the number of starts on the way.
//     One wave follows the 64 chains of a block in LDS.
//  3. Maps of 64 consecutive blocks compose into the map of a block 64 times
//     larger (lane e follows entry e through the 64 maps), up to one map for
//     the whole list, whose entry 0 gives the number of groups.
//  4. Top-down, each block gets its true entry and the number of groups
//     before it; one wave per block then writes its starts into goff.
#include "internal.h"

__global__ void k_act_flags(int64_t n, const uint8_t *__restrict__ active,
                            uint32_t *__restrict__ flag)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = active[i] ? 1u : 0u;
    else if (i == n) flag[n] = 0u;
}

__global__ void k_act_scatter(int64_t n, const uint8_t *__restrict__ active,
                              const uint32_t *__restrict__ fscan, int32_t *__restrict__ act,
                              int32_t *__restrict__ n_act)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && active[i]) act[fscan[i]] = (int32_t)i;
    if (i == 0) *n_act = (int32_t)fscan[n];
}

struct GroupCfg {
    const double *x, *y, *z, *h;
    const int64_t *box_off;
    const double *box_L;
    int nb;
    const uint32_t *fscan; // exclusive scan of active flags [n+1]
    const int32_t *act;
    const int32_t *n_act;
    sfc_group_params gp;   // used when gp_box == NULL
    const sfc_group_params *gp_box;
    const int8_t *dlev;    // per particle: deepest level whose cell holds more than n_leaf
                           // particles (-1: none), so its leaf lies at min(21, dlev + 1)
};

__device__ __forceinline__ sfc_group_params group_params(const GroupCfg &c, int b)
{
    sfc_group_params gp = c.gp_box ? c.gp_box[b] : c.gp;
    // per-box tables are device data: keep them in range
    gp.n_group_max = min(max(gp.n_group_max, 1), SFC_WAVE_GROUP_MAX);
    gp.level = min(max(gp.level, 0), SFC_KEY_BITS);
    return gp;
}

// ------------------------------------------------------------------ nxt
constexpr int NX_THREADS = 256;
constexpr int NX_STAGE = NX_THREADS + SFC_WAVE_GROUP_MAX; // positions a block reads

// nxt[k] for the NX_THREADS positions of a block; the positions of the
// actives it reads sit in LDS (staged with independent, coalesced-index
// loads), so the test loop of each position costs no global round trip
__global__ __launch_bounds__(NX_THREADS) void k_group_next(GroupCfg c, int32_t *__restrict__ nxt)
{
    __shared__ double sx[NX_STAGE], sy[NX_STAGE], sz[NX_STAGE];
    __shared__ uint32_t sc[NX_STAGE][3]; // tree policy: key cells of the staged actives
    const int A = *c.n_act;
    const int k0 = (int)blockIdx.x * NX_THREADS;
    if (k0 >= A) return;
    const int nst = min(NX_STAGE, A - k0);
    const int t = threadIdx.x;
    const bool tree = c.gp_box != nullptr || c.gp.policy == SFC_POLICY_TREE;
    for (int j = t; j < nst; j += NX_THREADS) {
        const int i = c.act[k0 + j];
        sx[j] = c.x[i];
        sy[j] = c.y[i];
        sz[j] = c.z[i];
        if (tree) {
            const double L = c.box_L[c.nb > 1 ? box_of(c.box_off, c.nb, i) : 0];
            sc[j][0] = key_cell(sx[j], L);
            sc[j][1] = key_cell(sy[j], L);
            sc[j][2] = key_cell(sz[j], L);
        }
    }
    __syncthreads();
    const int k = k0 + t;
    if (k >= A) return;
    const int i0 = c.act[k];
    const int b = c.nb > 1 ? box_of(c.box_off, c.nb, i0) : 0;
    const sfc_group_params gp = group_params(c, b);
    // first active position of the next box: a group never crosses a box
    const int a1 = (int)c.fscan[c.box_off[b + 1]];
    const int lim = min(k + gp.n_group_max, a1);
    int next = lim;
    if (gp.policy == SFC_POLICY_PAPER) {
        const double L = c.box_L[b];
        const double x0 = sx[t], y0 = sy[t], z0 = sz[t];
        const double R = gp.f * c.h[i0];
        const double R2 = R * R;
        for (int j = k + 1; j < lim; j++) {
            const int s = j - k0;
            const double dx = fold(sx[s] - x0, L), dy = fold(sy[s] - y0, L),
                         dz = fold(sz[s] - z0, L);
            const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            if (!(r2 < R2)) {
                next = j;
                break;
            }
        }
    } else if (gp.policy == SFC_POLICY_TREE) {
        // same cell as the first member at the depth of its node: the chosen
        // level, or its leaf's when that is shallower
        const int leaf = min((int)c.dlev[i0] + 1, SFC_KEY_BITS);
        const int sh = SFC_KEY_BITS - min(gp.level, leaf);
        const uint32_t cx = sc[t][0] >> sh, cy = sc[t][1] >> sh, cz = sc[t][2] >> sh;
        for (int j = k + 1; j < lim; j++) {
            const int s = j - k0;
            if ((sc[s][0] >> sh) != cx || (sc[s][1] >> sh) != cy || (sc[s][2] >> sh) != cz) {
                next = j;
                break;
            }
        }
    }
    nxt[k] = next;
}

// ------------------------------------------------------------------ block maps
// level-1 block of GB1 positions; a map entry e is the orbit entering the
// block at its position e (absolute exit position, starts on the way)
constexpr int GB1 = 1024;

__global__ __launch_bounds__(64) void k_group_map1(const int32_t *__restrict__ n_act,
                                                   const int32_t *__restrict__ nxt,
                                                   GMap *__restrict__ map)
{
    __shared__ int32_t sn[GB1];
    const int A = *n_act;
    const int q = (int)blockIdx.x;
    const int s0 = q * GB1;
    if (s0 >= A) return;
    const int end = min(s0 + GB1, A);
    const int lane = lane_id();
    for (int j = lane; j < end - s0; j += 64) sn[j] = nxt[s0 + j];
    wave_lds_sync();
    int p = s0 + lane, cnt = 0;
    // nxt(k) > k: at most GB1 steps
    for (int guard = 0; p < end && guard <= GB1; guard++) {
        cnt++;
        p = sn[p - s0];
    }
    map[q].exit[lane] = p;
    map[q].cnt[lane] = cnt;
}

// map of item I of a level = the maps of its 64 children (the items of the
// level below, span `cspan` positions each) followed one after the other
__global__ __launch_bounds__(64) void k_group_compose(const int32_t *__restrict__ n_act,
                                                      const GMap *__restrict__ child, int n_child,
                                                      int64_t cspan, GMap *__restrict__ map)
{
    const int A = *n_act;
    const int I = (int)blockIdx.x;
    const int64_t s0 = (int64_t)I * 64 * cspan;
    if (s0 >= A) return;
    const int lane = lane_id();
    int p = (int)s0 + lane, cnt = 0;
    for (int k = 0; k < 64; k++) {
        const int ch = 64 * I + k;
        if (ch >= n_child || p >= A) break;
        const int e = p - (int)((int64_t)ch * cspan); // in [0, 64)
        cnt += child[ch].cnt[e];
        p = child[ch].exit[e];
    }
    map[I].exit[lane] = p;
    map[I].cnt[lane] = cnt;
}

// the orbit's entry into each child of item I, and the groups before it
__global__ void k_group_expand(const int32_t *__restrict__ n_act, int n_item,
                               const int32_t *__restrict__ ent, const int32_t *__restrict__ before,
                               const GMap *__restrict__ child, int n_child, int64_t cspan,
                               int32_t *__restrict__ cent, int32_t *__restrict__ cbefore)
{
    const int A = *n_act;
    const int I = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (I >= n_item || (int64_t)I * 64 * cspan >= A) return;
    int p = ent[I], cnt = before[I];
    for (int k = 0; k < 64; k++) {
        const int ch = 64 * I + k;
        const int64_t cs = (int64_t)ch * cspan;
        if (ch >= n_child || cs >= A) break;
        cent[ch] = p;
        cbefore[ch] = cnt;
        if (p < A) {
            const int e = p - (int)cs;
            cnt += child[ch].cnt[e];
            p = child[ch].exit[e];
        }
    }
}

// top of the hierarchy: one item entered at position 0 with no group before
__global__ void k_group_top(const int32_t *__restrict__ n_act, const GMap *__restrict__ top,
                            int32_t *__restrict__ ent, int32_t *__restrict__ before,
                            int32_t *__restrict__ goff, int32_t *__restrict__ n_groups,
                            DevStatus *st)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int A = *n_act;
    const int G = A > 0 ? top[0].cnt[0] : 0;
    ent[0] = 0;
    before[0] = 0;
    *n_groups = G;
    goff[G] = A;
    st->n_groups = G;
    st->n_active = A;
}

// the starts of one level-1 block, from its entry, into goff
__global__ __launch_bounds__(64) void k_group_emit(const int32_t *__restrict__ n_act,
                                                   const int32_t *__restrict__ nxt,
                                                   const int32_t *__restrict__ ent,
                                                   const int32_t *__restrict__ before,
                                                   int32_t *__restrict__ goff)
{
    __shared__ int32_t sn[GB1];
    const int A = *n_act;
    const int q = (int)blockIdx.x;
    const int s0 = q * GB1;
    if (s0 >= A) return;
    const int end = min(s0 + GB1, A);
    const int lane = lane_id();
    for (int j = lane; j < end - s0; j += 64) sn[j] = nxt[s0 + j];
    wave_lds_sync();
    if (lane != 0) return;
    int p = ent[q], g = before[q];
    for (int guard = 0; p < end && guard <= GB1; guard++) {
        goff[g++] = p;
        p = sn[p - s0];
    }
}

// ------------------------------------------------------------------ launcher
int group_levels(int64_t n, int64_t *n_items, int64_t *span)
{
    int L = 0;
    int64_t m = (n + GB1 - 1) / GB1, s = GB1;
    for (;;) {
        n_items[L] = m < 1 ? 1 : m;
        span[L] = s;
        L++;
        if (m <= 1 || L == GROUP_LEVELS_MAX) break;
        m = (m + 63) / 64;
        s *= 64;
    }
    return L;
}

// the per-box superset caps of a per-box table (0 without one)
__global__ void k_box_tiles(const sfc_group_params *gp_box, int nb, int32_t *box_T)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) box_T[b] = gp_box ? gp_box[b].t_cand : 0;
}

hipError_t launch_groups(hipStream_t s, const PartDev &p, const sfc_group_params *gp,
                         const sfc_group_params *gp_box, const int8_t *dlev, GroupBufs &g,
                         uint32_t *scan_tmp, DevStatus *st)
{
    int64_t n = p.n;
    unsigned gb = (unsigned)((n + 1 + 255) / 256);
    // flags into goff's storage (n+1 entries; goff is written last)
    uint32_t *flag = (uint32_t *)g.goff;
    k_act_flags<<<gb, 256, 0, s>>>(n, p.active, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_scan_excl_u32(s, flag, g.flag_scan, n + 1, scan_tmp, nullptr);
    if (e != hipSuccess) return e;
    k_act_scatter<<<gb, 256, 0, s>>>(n, p.active, g.flag_scan, g.act, g.n_act);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    GroupCfg c;
    c.x = p.x; c.y = p.y; c.z = p.z; c.h = p.h;
    c.box_off = p.box_off;
    c.box_L = p.box_L;
    c.nb = p.nb;
    c.fscan = g.flag_scan;
    c.act = g.act;
    c.n_act = g.n_act;
    if (gp) c.gp = *gp;
    else c.gp = sfc_group_params{SFC_POLICY_COUNT, 1, 0.0, 0, 0};
    c.gp_box = gp_box;
    c.dlev = dlev;
    k_group_next<<<(unsigned)((n + NX_THREADS - 1) / NX_THREADS), NX_THREADS, 0, s>>>(c, g.nxt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int64_t ni[GROUP_LEVELS_MAX], sp[GROUP_LEVELS_MAX];
    const int L = group_levels(n, ni, sp);
    k_group_map1<<<(unsigned)ni[0], 64, 0, s>>>(g.n_act, g.nxt, g.map[0]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int l = 1; l < L; l++) {
        k_group_compose<<<(unsigned)ni[l], 64, 0, s>>>(g.n_act, g.map[l - 1], (int)ni[l - 1],
                                                       sp[l - 1], g.map[l]);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    k_group_top<<<1, 64, 0, s>>>(g.n_act, g.map[L - 1], g.ent[L - 1], g.before[L - 1], g.goff,
                                 g.n_groups, st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int l = L - 1; l >= 1; l--) {
        k_group_expand<<<(unsigned)((ni[l] + 63) / 64), 64, 0, s>>>(
            g.n_act, (int)ni[l], g.ent[l], g.before[l], g.map[l - 1], (int)ni[l - 1], sp[l - 1],
            g.ent[l - 1], g.before[l - 1]);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    k_group_emit<<<(unsigned)ni[0], 64, 0, s>>>(g.n_act, g.nxt, g.ent[0], g.before[0], g.goff);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_box_tiles<<<(unsigned)((p.nb + 255) / 256), 256, 0, s>>>(gp_box, p.nb, g.box_T);
    return hipGetLastError();
}
