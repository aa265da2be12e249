// group.hip -- active list and greedy grouping along the Hilbert curve.
//
// The actives of a box, in curve order, are cut into slices of `chunk`
// actives; one wave runs the paper's greedy scan over each slice: the first
// active of a slice opens a group, the following ones join while the policy
// allows (paper policy: closer than f*h_0 to the group's first member, h_0
// being that member's h; count policy: no distance test), at most
// n_group_max members, and the first one that may not join opens the next
// group.  The 64 lanes test the next 63 actives against the group's first
// member at once, so one step of the scan places a whole group.
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

// chunks per box -> cnt[b]; cnt[nb] = 0 (scanned into chunk_base)
__global__ void k_chunk_counts(int nb, const int64_t *__restrict__ box_off,
                               const uint32_t *__restrict__ fscan, int chunk,
                               const sfc_group_params *__restrict__ gp_box, uint32_t *cnt)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nb) return;
    if (b == nb) {
        cnt[nb] = 0;
        return;
    }
    int c = gp_box ? max(gp_box[b].chunk, 64) : chunk;
    uint32_t a = fscan[box_off[b + 1]] - fscan[box_off[b]];
    cnt[b] = (a + (uint32_t)c - 1u) / (uint32_t)c;
}

struct GroupCfg {
    const double *x, *y, *z, *h;
    const int64_t *box_off;
    const double *box_L;
    int nb;
    const uint32_t *fscan;     // exclusive scan of active flags [n+1]
    const int32_t *act;
    const uint32_t *chunk_base; // [nb+1]
    int32_t *gs_local;
    uint32_t *gcount;
    int64_t max_chunks;
    sfc_group_params gp;          // used when gp_box == NULL
    const sfc_group_params *gp_box;
    const int8_t *dlev; // per particle: deepest level whose cell holds more than n_leaf
                        // particles (-1: none), so its leaf lies at min(21, dlev + 1)
};

// actives of a chunk whose positions sit in LDS at a time
constexpr int GSTAGE = 512;

// one wave per chunk; the greedy scan reads positions from LDS, staged
// GSTAGE actives at a time with independent (coalesced-index) loads, so
// that each group costs no global-memory round trip
__global__ __launch_bounds__(64) void k_group_chunks(GroupCfg c)
{
    __shared__ double sx[GSTAGE], sy[GSTAGE], sz[GSTAGE], sh[GSTAGE];
    __shared__ int sl[GSTAGE]; // tree policy: leaf level of each staged active
    int64_t q = (int64_t)blockIdx.x;
    int lane = lane_id();
    int64_t nch = c.chunk_base[c.nb];
    if (q >= nch) {
        if (q < c.max_chunks && lane == 0) c.gcount[q] = 0;
        return;
    }
    // box of chunk q
    int lo = 0, hi = c.nb;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if ((int64_t)c.chunk_base[mid] <= q) lo = mid; else hi = mid;
    }
    int b = lo;
    sfc_group_params gp = c.gp_box ? c.gp_box[b] : c.gp;
    gp.chunk = max(gp.chunk, 64); // per-box tables are device data: keep them in range
    gp.n_group_max = min(max(gp.n_group_max, 1), 64);
    gp.level = min(max(gp.level, 0), SFC_KEY_BITS);
    int64_t a0 = c.fscan[c.box_off[b]], a1 = c.fscan[c.box_off[b + 1]];
    int64_t start = a0 + (q - (int64_t)c.chunk_base[b]) * gp.chunk;
    int64_t end = min(start + (int64_t)gp.chunk, a1);
    double L = c.box_L[b];
    int cap = gp.n_group_max;
    int64_t k = start;
    int64_t t0 = 0, t1 = 0; // staged actives [t0, t1)
    int ng = 0;
    while (k < end) {
        if (lane == 0) c.gs_local[start + ng] = (int32_t)k;
        ng++;
        int lim = (int)min((int64_t)cap, end - k);
        int size;
        if (gp.policy == SFC_POLICY_COUNT) {
            size = lim;
        } else {
            if (k + lim > t1) { // restage from k
                t0 = k;
                t1 = min(k + (int64_t)GSTAGE, end);
                wave_lds_sync();
                for (int j = lane; j < (int)(t1 - t0); j += 64) {
                    const int i = c.act[t0 + j];
                    sx[j] = c.x[i];
                    sy[j] = c.y[i];
                    sz[j] = c.z[i];
                    sh[j] = c.h[i];
                    if (gp.policy == SFC_POLICY_TREE) sl[j] = min((int)c.dlev[i] + 1, SFC_KEY_BITS);
                }
                wave_lds_sync();
            }
            const int s0 = (int)(k - t0);
            double x0 = sx[s0], y0 = sy[s0], z0 = sz[s0];
            bool pass = lane == 0;
            if (gp.policy == SFC_POLICY_TREE) {
                // same cell as the first member at the depth of its node: the
                // chosen level, or its leaf's when that is shallower
                const int sh3 = SFC_KEY_BITS - min(gp.level, sl[s0]);
                const uint32_t cx = key_cell(x0, L) >> sh3, cy = key_cell(y0, L) >> sh3,
                               cz = key_cell(z0, L) >> sh3;
                if (lane > 0 && lane < lim)
                    pass = (key_cell(sx[s0 + lane], L) >> sh3) == cx &&
                           (key_cell(sy[s0 + lane], L) >> sh3) == cy &&
                           (key_cell(sz[s0 + lane], L) >> sh3) == cz;
            } else {
                double R = gp.f * sh[s0];
                double R2 = R * R;
                if (lane > 0 && lane < lim) {
                    double dx = fold(sx[s0 + lane] - x0, L);
                    double dy = fold(sy[s0 + lane] - y0, L);
                    double dz = fold(sz[s0 + lane] - z0, L);
                    double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
                    pass = r2 < R2;
                }
            }
            size = ctz64(~ballot(pass));
        }
        k += size;
    }
    if (lane == 0) c.gcount[q] = (uint32_t)ng;
}

__global__ __launch_bounds__(64) void k_group_scatter(GroupCfg c, const uint32_t *__restrict__ gscan,
                                                      int32_t *__restrict__ goff,
                                                      int32_t *__restrict__ n_groups,
                                                      const int32_t *__restrict__ n_act,
                                                      DevStatus *st)
{
    int64_t q = (int64_t)blockIdx.x;
    int lane = lane_id();
    int64_t nch = c.chunk_base[c.nb];
    if (q == 0 && lane == 0) {
        int G = (int)gscan[c.max_chunks];
        *n_groups = G;
        goff[G] = *n_act;
        st->n_groups = G;
        st->n_active = *n_act;
    }
    if (q >= nch) return;
    int lo = 0, hi = c.nb;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if ((int64_t)c.chunk_base[mid] <= q) lo = mid; else hi = mid;
    }
    int b = lo;
    int chunk = c.gp_box ? max(c.gp_box[b].chunk, 64) : c.gp.chunk;
    int64_t a0 = c.fscan[c.box_off[b]];
    int64_t start = a0 + (q - (int64_t)c.chunk_base[b]) * chunk;
    uint32_t base = gscan[q];
    int ng = (int)c.gcount[q];
    for (int g = lane; g < ng; g += 64) goff[base + g] = c.gs_local[start + g];
}

hipError_t launch_groups(hipStream_t s, const PartDev &p, const sfc_group_params *gp,
                         const sfc_group_params *gp_box, const int8_t *dlev, GroupBufs &g,
                         uint32_t *scan_tmp, DevStatus *st)
{
    int64_t n = p.n;
    unsigned gb = (unsigned)((n + 1 + 255) / 256);
    // flags into gscan's sibling buffer: reuse goff as u32 flags (n+1 entries)
    uint32_t *flag = (uint32_t *)g.goff;
    k_act_flags<<<gb, 256, 0, s>>>(n, p.active, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_scan_excl_u32(s, flag, g.flag_scan, n + 1, scan_tmp, nullptr);
    if (e != hipSuccess) return e;
    k_act_scatter<<<gb, 256, 0, s>>>(n, p.active, g.flag_scan, g.act, g.n_act);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int chunk = gp ? gp->chunk : 64;
    k_chunk_counts<<<(p.nb + 1 + 255) / 256, 256, 0, s>>>(p.nb, p.box_off, g.flag_scan, chunk,
                                                         gp_box, g.gcount);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    uint32_t *chunk_base = (uint32_t *)g.chunk_base;
    e = launch_scan_excl_u32(s, g.gcount, chunk_base, p.nb + 1, scan_tmp, nullptr);
    if (e != hipSuccess) return e;
    GroupCfg c;
    c.x = p.x; c.y = p.y; c.z = p.z; c.h = p.h;
    c.box_off = p.box_off;
    c.box_L = p.box_L;
    c.nb = p.nb;
    c.fscan = g.flag_scan;
    c.act = g.act;
    c.chunk_base = chunk_base;
    c.gs_local = g.gs_local;
    c.gcount = g.gcount;
    c.max_chunks = g.max_chunks;
    if (gp) c.gp = *gp;
    else c.gp = sfc_group_params{SFC_POLICY_COUNT, 1, 0.0, 64, 0};
    c.gp_box = gp_box;
    c.dlev = dlev;
    k_group_chunks<<<(unsigned)g.max_chunks, 64, 0, s>>>(c);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // gcount[max_chunks] = 0 so that the scan's last entry is the group total
    e = launch_fill_i32(s, (int32_t *)(g.gcount + g.max_chunks), 0, 1);
    if (e != hipSuccess) return e;
    e = launch_scan_excl_u32(s, g.gcount, g.gscan, g.max_chunks + 1, scan_tmp, nullptr);
    if (e != hipSuccess) return e;
    k_group_scatter<<<(unsigned)g.max_chunks, 64, 0, s>>>(c, g.gscan, g.goff, g.n_groups, g.n_act,
                                                         st);
    return hipGetLastError();
}
