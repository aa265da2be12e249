// internal.h -- shared device helpers and workspace views of the sfcngb
// library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sfcngb.h"

#define SFC_KEY_BITS 21
// node indices fit in the 28 low bits of a walk item
#define TREE_ITEM_NODE 0x0fffffff
#define SFC_WG 256 // threads per workgroup in the persistent kernels (4 waves)

// cell of a coordinate along one axis at the deepest level: floor(x/L 2^21),
// clamped to [0, 2^21 - 1]; the level-l cell is this >> (21 - l)
__device__ __forceinline__ uint32_t key_cell(double x, double L)
{
    double s = (x / L) * 2097152.0; // 2^21
    if (!(s >= 0.0)) return 0u;
    if (s >= 2097151.0) return 2097151u;
    return (uint32_t)s;
}

// ---------------------------------------------------------------- wave ops
__device__ __forceinline__ int lane_id()
{
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
// number of set bits of m below this lane
__device__ __forceinline__ int mbcnt(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ int popc64(uint64_t m) { return __builtin_popcountll(m); }
__device__ __forceinline__ int ctz64(uint64_t m) { return m ? __builtin_ctzll(m) : 64; }
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ double readlane_d(double v, int l)
{
    union { double d; int i[2]; } a, b;
    a.d = v;
    b.i[0] = __builtin_amdgcn_readlane(a.i[0], l);
    b.i[1] = __builtin_amdgcn_readlane(a.i[1], l);
    return b.d;
}
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l)
{
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}
// write the uniform value s into lane l of v
__device__ __forceinline__ uint64_t writelane_u64(uint64_t v, uint64_t s, int l)
{
    return lane_id() == l ? s : v;
}
// order LDS accesses of the lanes of one wave (each wave owns its LDS slice)
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ float wave_sum_f(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_max_f(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_max_d(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_sum_f_or_d(float v) { return wave_sum_f(v); }
__device__ __forceinline__ double wave_sum_f_or_d(double v) { return wave_sum_d(v); }
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t lo = __shfl_xor((unsigned)(uint32_t)v, o, 64);
        uint32_t hi = __shfl_xor((unsigned)(uint32_t)(v >> 32), o, 64);
        v += ((uint64_t)hi << 32) | lo;
    }
    return v;
}

// ------------------------------------------------------- box helpers
// box b with box_off[b] <= i < box_off[b+1] (boxes may be empty)
__device__ __forceinline__ int box_of(const int64_t *box_off, int nb, int64_t i)
{
    int lo = 0, hi = nb;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (box_off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// minimum-image fold of a coordinate difference into [-L/2, L/2)
__device__ __forceinline__ double fold(double d, double L)
{
    double half = 0.5 * L;
    if (d >= half) d = d - L;
    else if (d < -half) d = d + L;
    return d;
}

// ------------------------------------------------------- status block
// cost classes of the density group kernel's order of the groups, and the
// groups per workgroup of the kernels that make it
constexpr int GO_K = 16;
constexpr int GO_CH = 512;

struct DevStatus {
    uint32_t flags;
    int32_t n_nodes;
    int32_t n_active;
    int32_t n_groups;
    unsigned long long n_deferred;
    unsigned long long n_overflow;
    unsigned long long n_not_converged;
    unsigned long long sum_cand;
    unsigned long long n_walks;
    unsigned long long sum_iters;
    unsigned long long sum_tests;
    unsigned long long sum_pairs;
    unsigned long long n_dfr; // per pass: hydro members deferred to their own walks
    unsigned long long n_glist; // reuse density pass: groups holding a member active now
    // with tracing on, per pass, for the density group kernel [0] and the
    // hydro member kernel [1], per XCD (each on a 128-byte line of its own):
    // the earliest start and the latest end of a workgroup (density) or wave
    // (hydro) on the device's constant clock, the sum of their end times and
    // their number
    unsigned long long sched[2][8][16];
    // Per-pass counters of the search kernels, one per eighth of the work
    // items, each on its own 128-byte line so that the eighths do not
    // serialise on one address: bump pointers of the eight regions of the
    // candidate buffer and the walk kernel's work counters.
    unsigned long long cand_top[8 * 16]; // cand_top[16 * x]
    int32_t qctr[8 * 32];                // qctr[32 * x]: the walk kernel's
    int32_t qctr2[8 * 32];               // qctr2[32 * x]: the group kernels'
    int32_t qctr3[8 * 32];               // qctr3[32 * x]: the density solo kernel's
    // per density pass, the order of the groups for the group kernel: the
    // total cost, and per eighth and cost class the groups and the slots
    // handed out so far
    unsigned long long go_wtot;
    int32_t go_on; // the order was written (else the index order holds)
    int32_t go_tot[8 * GO_K];
    int32_t go_cur[8 * GO_K];
};

// per-group record written by the walk kernel
#define GSUP_WRAP 1 // pairs of this group need the periodic fold
#define GSUP_SOLO 2 // superset not kept (tile or buffer overflow): members walk alone
#define GSUP_FRESH 4 // a member's own superset, walked at the current positions
struct GSup {
    double cx, cy, cz; // centre: the group's first member
    double cov;        // walk radius (density: R_g + skin * max member h; hydro: rs + max h)
    double rs;         // hydro: R_g + (skin - 1) * max member h
    int64_t c0;        // first candidate in the candidate buffer
    int32_t nc;        // number of candidates
    int32_t flags;
};

// ------------------------------------------------------- tree view
struct TreeDev {
    int4 *info;     // first, count, skip, level | leaf << 8
    int32_t *kids;  // [8 * capacity]: children of a node in order, -1 past the last
    double4 *lo;    // min x, min y, min z, hmax
    double4 *hi;    // max x, max y, max z, 0
    float4 *box32;  // [2 * capacity]: the box in FP32 rounded outwards (min down, max and
                    // max h up): (min x, min y, min z, max h), (max x, max y, max z, 0)
    int32_t *nchild;
    // [16 * capacity]: for child slot s of node p, at 2 (8 p + s), the child's
    // FP32 box as in box32, with the .w of the second float4 holding the
    // child's item (bit pattern of an int: node index | (child count - 1)
    // << 28, leaf flag in bit 31); empty slots hold a box no ball reaches
    float4 *krec;
    int32_t *box_root; // [nb+1]
    int32_t capacity;
};

// ------------------------------------------------------- particle view
struct PartDev {
    int64_t n;
    int nb;
    const int64_t *box_off;
    const double *box_L;
    const double *x, *y, *z;
    double *h;
    const float *m, *vx, *vy, *vz, *u;
    float *rho, *fgrad;
    const uint8_t *active;
    const uint32_t *orig;
};

// splitmix64 finaliser (Steele, Lea, Flood 2014) for neighbour fingerprints
__device__ __forceinline__ uint64_t mix64(uint64_t v)
{
    v += 0x9e3779b97f4a7c15ull;
    v = (v ^ (v >> 30)) * 0xbf58476d1ce4e5b9ull;
    v = (v ^ (v >> 27)) * 0x94d049bb133111ebull;
    return v ^ (v >> 31);
}

// ------------------------------------------------------- host-side launchers
// (defined in the .hip files, called by the C-ABI layer)
// a particle's fields in one 64-byte record (the gather's unit)
struct __align__(64) PRec {
    double x, y, z, h;
    float m, vx, vy, vz, u, rho, fgrad;
    uint32_t orig;
};
static_assert(sizeof(PRec) == 64, "PRec is one 64-byte record");

struct SortBufs {
    PRec *rec;               // [n] input-order records
    uint64_t *key_a, *key_b;
    uint32_t *val_a, *val_b;
    uint32_t *box_a, *box_b; // box ids (batched sort only)
    uint32_t *hist;          // 256 * ntiles
    uint32_t *scan_tmp;      // scratch for the device scan
};

hipError_t launch_keys(hipStream_t s, const sfc_particles *in, SortBufs &b);
hipError_t launch_radix_sort(hipStream_t s, int64_t n, int nb, SortBufs &b, uint64_t *keys_out,
                             uint32_t **perm_out);
hipError_t launch_gather(hipStream_t s, const sfc_particles *in, sfc_particles *out,
                         const uint32_t *perm, const PRec *rec, uint32_t *perm_out);
size_t scan_tmp_elems(int64_t n);
hipError_t launch_scan_excl_u32(hipStream_t s, const uint32_t *in, uint32_t *out, int64_t n,
                                uint32_t *tmp, uint32_t *total);
hipError_t launch_fill_i32(hipStream_t s, int32_t *p, int32_t v, int64_t n);

struct TreeBufs {
    int8_t *lcp;     // [n]
    int8_t *dlev;    // [n]
    uint32_t *cnt;   // [n+1]
    uint32_t *start; // [n+1]
};
hipError_t launch_tree_build(hipStream_t s, const PartDev &p, const uint64_t *keys, int n_leaf,
                             TreeBufs &tb, TreeDev &t, uint32_t *scan_tmp, DevStatus *st);
hipError_t launch_tree_refit(hipStream_t s, const PartDev &p, TreeDev &t, bool bbox,
                             DevStatus *st, int64_t n);

// Grouping: per active the position that would open the next group, and
// per block of the active list (GB1 = 1024 positions at level 0, 64 times
// more per level above) the map of the orbit through it, its true entry
// and the number of groups before it.
#define GROUP_LEVELS_MAX 6
struct GMap {
    int32_t exit[64]; // entry e (the block's position e) -> where the orbit leaves the block
    int32_t cnt[64];  // -> group starts on the way
};
struct GroupBufs {
    uint32_t *flag_scan; // [n+1] exclusive scan of active flags
    int32_t *act;        // [n]
    int32_t *nxt;        // [n]
    GMap *map[GROUP_LEVELS_MAX];
    int32_t *ent[GROUP_LEVELS_MAX];
    int32_t *before[GROUP_LEVELS_MAX];
    int32_t *goff;       // [n+1]
    int32_t *box_T;      // [n_boxes] per-box superset cap of the last grouping (0: the call's)
    int32_t *n_act;      // device scalar
    int32_t *n_groups;   // device scalar
};
// items and span (positions) of each level of the maps for n actives at most;
// returns the number of levels
int group_levels(int64_t n, int64_t *n_items, int64_t *span);
hipError_t launch_groups(hipStream_t s, const PartDev &p, const sfc_group_params *gp,
                         const sfc_group_params *gp_box, const int8_t *dlev, GroupBufs &g,
                         uint32_t *scan_tmp, DevStatus *st);

struct SearchBufs {
    int32_t *cand;    // [cand_cap] candidate supersets of all groups
    int64_t cand_cap;
    GSup *sup;        // [n] per group
    int32_t *grp;     // [n] per active: its group
    float4 *pa, *pb;  // [n] hydro records: (m, v) and (rho, f P / rho^2, c, h)
    float4 *pc;       // [n] production SPH: (alpha_i, u, P)
    float4 *pos4;     // [n] FP32 x, y, z and (density) m or (hydro) h, for the walks
    double4 *p64;     // [n] FP64 x, y, z and the mass (density: group staging, pair
                      // terms) or h (hydro: pair terms)
    double4 *dstate;  // [n] per active: h, bracket lo, hi, evaluations (members that leave
                      // their group superset)
    double4 *snap;    // [n] kept supersets: x, y, z (and h) when they were walked, or NULL
    unsigned long long *drift; // [4 + 3 * 512] largest displacement, largest h growth since
                               // (FP64 bits), active particles now, members active now;
                               // then per-block partials
    int32_t *sel;     // [n] reuse: positions in the active list of the members active now
    int32_t *dfr;     // [n] hydro: positions in the active list of the members that walk alone
    int32_t *gmark;   // [n] reuse: 1 for a kept group holding a member active now
    int32_t *glist;   // [n] reuse: those groups (st->n_glist of them); otherwise every group,
                      // in the density group kernel's order (when st->go_on is set)
    int32_t cu_count;
};
struct DensityArgs {
    sfc_density_params dp;
    sfc_density_out out;
    bool keep; // snapshot x, y, z for a later reuse
    bool trace; // schedule statistics
};
struct HydroArgs {
    sfc_hydro_params hp;
    sfc_hydro_out out;
    bool keep; // snapshot x, y, z, h for a later reuse
    bool trace; // schedule statistics
};
hipError_t launch_density(hipStream_t s, const PartDev &p, const TreeDev &t, const GroupBufs &g,
                          SearchBufs &sb, const DensityArgs &a, DevStatus *st);
hipError_t launch_hydro(hipStream_t s, const PartDev &p, const TreeDev &t, const GroupBufs &g,
                        SearchBufs &sb, const HydroArgs &a, DevStatus *st);
hipError_t launch_verify(hipStream_t s, const PartDev &p, const TreeDev &t, const GroupBufs &g,
                         SearchBufs &sb, const sfc_verify &v, int t_cand, DevStatus *st);
