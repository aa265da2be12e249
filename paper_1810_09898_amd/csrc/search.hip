// search.hip -- grouped neighbour search, density and hydro force.
//
// A group is a run of active particles along the Hilbert curve (section
// "Implementation of Neighbour Recycling using a Space Filling Curve").
// Every pass (density, hydro, verify) is two kernels:
//
//  k_walk: one wavefront per group walks the octree ONCE with the group
//    ball (centre = first member, radius = R_g + skin * max h for density,
//    R_g + max(max h, h_j) for hydro): a descent to the deepest node that
//    holds the whole ball, then level by level over an ordered list of the
//    reached nodes (a pre-order window walk when the list outgrows its
//    slots).  Particles of reached leaves are tested against the ball (FP32
//    copies, radius widened past their rounding) and written in ascending
//    order straight into the wave's chunk of the global candidate buffer:
//    the group's candidate superset.  A per-group record and the member ->
//    group map are written.
//
//  k_density / k_hydro / k_verify: one wavefront per active particle.  The
//    lanes hold 64 candidates of the particle's group at a time; one test
//    each (FP32 where provably on the same side as the FP64 test, FP64
//    otherwise) gives the neighbour mask of that chunk.  Density iterates h
//    on the superset while h + |x_i - x_0| stays inside the walk radius
//    (masks of the last evaluation are kept in LDS), then streams the
//    neighbours through an LDS FIFO in which the k-th neighbour always lands
//    on lane k mod 64: each lane accumulates a fixed subsequence in a fixed
//    order, so the sums do not depend on the group the particle was in.
//
// A particle whose h outgrows the superset, and every member of a group
// whose superset overflows the tile or the candidate buffer, takes a
// superset of its own (density: up to three times), and else finishes
// alone: one walk per h evaluation, neighbours streamed through the same
// FIFO.
//
// Every data-dependent loop has a hard trip limit; hitting one sets
// SFC_ST_GUARD in the status block instead of spinning.
#include <cstring>

#include "internal.h"

#define INFL (1.0 + 0x1p-30)

namespace {

// kernel normalisations, W = C w(q) / h^3 with 4 pi C int_0^1 w q^2 dq = 1
constexpr double PI_D = 3.14159265358979323846;
constexpr double C_CUBIC = 8.0 / PI_D;            // cubic spline M4
constexpr double C_WC6 = 1365.0 / (64.0 * PI_D);  // Wendland C6

template <int KER> __host__ __device__ constexpr double knorm() { return KER == 0 ? C_CUBIC : C_WC6; }

template <typename T> __device__ __forceinline__ T mad(T a, T b, T c);
template <> __device__ __forceinline__ float mad<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double mad<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ double uni_d(double v)
{
    union { double d; int i[2]; } a;
    a.d = v;
    a.i[0] = __builtin_amdgcn_readfirstlane(a.i[0]);
    a.i[1] = __builtin_amdgcn_readfirstlane(a.i[1]);
    return a.d;
}
__device__ __forceinline__ bool uni_b(bool v) { return __builtin_amdgcn_readfirstlane((int)v) != 0; }

// kernel shape w(q) and w'(q), support q < 1
template <int KER, typename T> __device__ __forceinline__ void kern_eval(T q, T &w, T &dw)
{
    const T u = q < T(1) ? T(1) - q : T(0);
    if (KER == 0) {
        T wo = T(2) * u * u * u;
        T dwo = T(-6) * u * u;
        T wi = mad(q * q, mad(T(6), q, T(-6)), T(1));
        T dwi = q * mad(T(18), q, T(-12));
        bool inner = q < T(0.5);
        w = inner ? wi : wo;
        dw = inner ? dwi : dwo;
    } else {
        T u2 = u * u, u4 = u2 * u2, u7 = u4 * u2 * u, u8 = u4 * u4;
        w = u8 * mad(q, mad(q, mad(T(32), q, T(25)), T(8)), T(1));
        dw = T(-22) * q * u7 * mad(q, mad(T(16), q, T(7)), T(1));
    }
}

// the same from q and an accurate u = 1 - q (0 outside the support): the
// pair terms form u as (h^2 - r^2) / (h^2 (1 + q)) with the difference taken
// in FP64, so the tail (1 - q)^k keeps its relative accuracy up to the edge
template <int KER, typename T> __device__ __forceinline__ void kern_eval_u(T q, T u, T &w, T &dw)
{
    if (KER == 0) {
        T wo = T(2) * u * u * u;
        T dwo = T(-6) * u * u;
        T wi = mad(q * q, mad(T(6), q, T(-6)), T(1));
        T dwi = q * mad(T(18), q, T(-12));
        bool inner = q < T(0.5);
        w = inner ? wi : wo;
        dw = inner ? dwi : dwo;
    } else {
        T u2 = u * u, u4 = u2 * u2, u7 = u4 * u2 * u, u8 = u4 * u4;
        w = u8 * mad(q, mad(q, mad(T(32), q, T(25)), T(8)), T(1));
        dw = T(-22) * q * u7 * mad(q, mad(T(16), q, T(7)), T(1));
    }
}

// w'(q) alone from q and u = 1 - q (the force terms need no w)
template <int KER, typename T> __device__ __forceinline__ T kern_deval_u(T q, T u)
{
    if (KER == 0) return q < T(0.5) ? q * mad(T(18), q, T(-12)) : T(-6) * u * u;
    const T u2 = u * u, u4 = u2 * u2, u7 = u4 * u2 * u;
    return T(-22) * q * u7 * mad(q, mad(T(16), q, T(7)), T(1));
}

// 1 - q for q = sqrt(r2) / h, from the FP64 r2 and h2 = h^2: the difference
// h2 - r2 is exact near the edge (the two are within a factor 2), so the
// result has a small relative error even where it is tiny; 0 outside
template <typename T> __device__ __forceinline__ T tail_u(double h2, double r2, T inv_h2, T q);
template <> __device__ __forceinline__ float tail_u<float>(double h2, double r2, float inv_h2, float q)
{
    const double dd = h2 - r2;
    return dd > 0.0 ? (float)dd * inv_h2 * __builtin_amdgcn_rcpf(1.0f + q) : 0.0f;
}
template <> __device__ __forceinline__ double tail_u<double>(double h2, double r2, double inv_h2, double q)
{
    (void)h2;
    (void)r2;
    (void)inv_h2;
    return q < 1.0 ? 1.0 - q : 0.0;
}

// square root and reciprocal of the pair arithmetic: the hardware's
// single-instruction forms (1 ulp) in FP32, the exact ones in FP64
template <typename T> __device__ __forceinline__ T acc_sqrt(T x);
template <> __device__ __forceinline__ float acc_sqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ __forceinline__ double acc_sqrt<double>(double x) { return sqrt(x); }
template <typename T> __device__ __forceinline__ T acc_rcp(T x);
template <> __device__ __forceinline__ float acc_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double acc_rcp<double>(double x) { return 1.0 / x; }

// the same from the FP64 difference h^2 - r^2 already rounded to T
template <typename T> __device__ __forceinline__ T tail_g(T d, T inv_h2, T q);
template <> __device__ __forceinline__ float tail_g<float>(float d, float inv_h2, float q)
{
    return d > 0.0f ? d * inv_h2 * __builtin_amdgcn_rcpf(1.0f + q) : 0.0f;
}
template <> __device__ __forceinline__ double tail_g<double>(double d, double inv_h2, double q)
{
    (void)d;
    (void)inv_h2;
    return q < 1.0 ? 1.0 - q : 0.0;
}

template <typename T> struct Kahan {
    T s = T(0), c = T(0);
    __device__ __forceinline__ void add(T v)
    {
        T y = v - c;
        T t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ T value() const { return s - c; }
};
template <> struct Kahan<double> {
    double s = 0.0;
    __device__ __forceinline__ void add(double v) { s += v; }
    __device__ __forceinline__ double value() const { return s; }
};

__device__ __forceinline__ double sq(double a) { return a * a; }

// smoothing-length step: bracket, then h * g with g a two-step Halley
// estimate of (n_ngb/n)^(1/3); the bracket midpoint when h*g leaves it.
// IEEE basic operations only, in this order, so that every implementation
// lands on the same h.
__device__ __forceinline__ double h_step(int n, int n_ngb, int dn, double h, double &lo, double &hi)
{
    if (n < n_ngb - dn) lo = h; else hi = h;
    double t = (double)n_ngb / (double)n;
    double y = (1.0 + 2.0 * t) / (2.0 + t);
    double y3 = (y * y) * y;
    double g = (y * (y3 + 2.0 * t)) / (2.0 * y3 + t);
    double hn = h * g;
    if (!(hn > lo && hn < hi)) hn = 0.5 * (lo + hi);
    return hn;
}

__device__ __forceinline__ void guard_hit(DevStatus *st)
{
    if (lane_id() == 0) atomicOr(&st->flags, (unsigned)SFC_ST_GUARD);
}

__device__ __forceinline__ unsigned long long uni_u64(unsigned long long v)
{
    return ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v)) |
           ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32)) << 32);
}

// Statistics of one wave, added to the status block once, when the wave
// leaves: a status counter updated by every particle or group would
// serialise the whole grid on one address.
struct WaveStats {
    uint32_t walks = 0, overflow = 0, deferred = 0, iters = 0, not_conv = 0;
    unsigned long long cand = 0, tests = 0, pairs = 0;
    __device__ __forceinline__ void flush(DevStatus *st) const
    {
        if (lane_id() != 0) return;
        if (walks) atomicAdd(&st->n_walks, (unsigned long long)walks);
        if (cand) atomicAdd(&st->sum_cand, cand);
        if (overflow) atomicAdd(&st->n_overflow, (unsigned long long)overflow);
        if (deferred) atomicAdd(&st->n_deferred, (unsigned long long)deferred);
        if (iters) atomicAdd(&st->sum_iters, (unsigned long long)iters);
        if (not_conv) atomicAdd(&st->n_not_converged, (unsigned long long)not_conv);
        if (tests) atomicAdd(&st->sum_tests, tests);
        if (pairs) atomicAdd(&st->sum_pairs, pairs);
    }
};

} // namespace

// --------------------------------------------------------------- kernel args
struct Geom {
    const double *x, *y, *z;
    double *h;
    const int64_t *box_off;
    const double *box_L;
    const int4 *info;
    const double4 *lo, *hi;
    const float4 *box32; // node boxes in FP32, rounded outwards
    const float4 *krec;  // per child slot: the child's FP32 box and its item (tree.hip)
    const int32_t *kids, *nchild;
    const int32_t *box_root;
    int nb;
};
struct GroupArg {
    const int32_t *act, *goff, *n_groups, *n_act;
    const int32_t *box_T; // per-box superset caps (0: T)
    int T;
};
struct CandArg {
    int32_t *cand; // global candidate buffer
    int64_t cap;   // its capacity
    GSup *sup;     // per group
    int32_t *grp;  // per active: its group
};

namespace {

// ------------------------------------------------------------------ scheduling
// Workgroups are dealt to the 8 XCDs round-robin (block b on XCD b mod 8),
// and each XCD has its own L2.  The work items (groups, or active particles,
// both in Hilbert order) are cut into 8 contiguous ranges, one per XCD, each
// a compact region of space, so the waves of one XCD share the tree nodes
// and particles they read.  A wave takes the next item of its XCD's range
// from a counter; when that range is used up it takes items from the other
// ranges, so no XCD idles while another has work.  Every take advances a
// counter, and a wave leaves after all 8 ranges are used up: the loop ends.
// A take hands out QB consecutive items, so the counters see one atomic per
// QB items.
constexpr int QB = 1;
struct Queue {
    int32_t *ctr; // [8 * 32]: counter x at ctr[32 * x]
    int n, per, xcd, xs;
    int cur, end; // items left of the current take
    int qb;       // items per take
};
__device__ __forceinline__ Queue queue_open(int32_t *ctr, int n_items, int qb = QB)
{
    Queue q;
    q.ctr = ctr;
    q.qb = qb;
    q.n = n_items;
    q.per = (n_items + 7) >> 3;
    q.xcd = blockIdx.x & 7;
    q.xs = 0;
    q.cur = q.end = 0;
    return q;
}
// Items per take: GQB per atomic when there are many items per taker (the
// walk: at least WQ_MANY per wave; the density group kernel: at least
// GQ_MANY per workgroup, its groups cost more and vary more), so the
// atomics are fewer and the few items that one take holds back at the end
// are a small part of a taker's work; otherwise one, so that every taker
// gets work when the items are few.
constexpr int GQB = 4;
constexpr int WQ_MANY = 8;
constexpr int GQ_MANY = 256;
__device__ __forceinline__ int queue_qb(int n_items, int takers, int qb, int many)
{
    return (int64_t)n_items >= (int64_t)many * takers ? qb : 1;
}
// next item, or -1 when every range is used up
__device__ __forceinline__ int queue_next(Queue &q)
{
    if (q.cur < q.end) return q.cur++;
    while (q.xs < 8) {
        const int x = (q.xcd + q.xs) & 7;
        int t = 0;
        if (lane_id() == 0) t = atomicAdd(&q.ctr[32 * x], q.qb);
        t = uni(t);
        const int item = x * q.per + t;
        if (t < q.per && item < q.n) {
            q.cur = item + 1;
            q.end = min(min(x * q.per + q.per, q.n), item + q.qb);
            return item;
        }
        q.xs++;
    }
    return -1;
}

// The particle kernels keep a static split instead: the waves of one
// workgroup (one CU) take consecutive particles, which mostly belong to the
// same group and read the same candidates at the same time, so the CU's L1
// serves them.
struct ItemRange {
    int i, end, stride;
};
__device__ __forceinline__ ItemRange item_range(int n_items)
{
    const int wpg = (int)(blockDim.x >> 6);
    const int wave = uni((int)(threadIdx.x >> 6));
    const int nblk = (int)gridDim.x;
    ItemRange r;
    if (nblk < 8 || (nblk & 7)) {
        r.i = (int)blockIdx.x * wpg + wave;
        r.end = n_items;
        r.stride = nblk * wpg;
        return r;
    }
    const int xcd = blockIdx.x & 7;
    const int per = (n_items + 7) >> 3;
    r.i = xcd * per + (int)(blockIdx.x >> 3) * wpg + wave;
    r.end = min(n_items, (xcd + 1) * per);
    r.stride = (nblk >> 3) * wpg;
    return r;
}

// ------------------------------------------------------------------ walk
struct Ball {
    double cx, cy, cz, L;
    double W2;     // density: squared walk radius
    double Rg, Hg; // hydro: node radius R_g + max(H_g, node hmax)
    int hydro;
    int nowrap;    // the ball lies inside the box: no candidate needs the periodic fold
};


// position (and h) of a walked particle
struct Pos {
    double x, y, z, h;
};

// Leaves `vl` (lane mask) of the current window: flatten their particles and
// hand them to `visit` 64 at a time, ascending.  A prefix sum of the leaf
// sizes gives each leaf its first flattened position; in a batch of 64
// positions only a few leaves start, so each lane finds its leaf by walking
// the (uniform) list of those starts, and reads the leaf's first particle
// from the leaf's lane.  V::EB batches per step: their loads (visit.fetch)
// are in flight together before visit.take consumes them in order.
template <class V> __device__ __forceinline__ void emit_leaves(uint64_t vl, int4 inf, V &visit)
{
    constexpr int EB = V::EB;
    const int lane = lane_id();
    const bool isl = (vl >> lane) & 1ull;
    const int c = isl ? inf.y : 0;
    int incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    const int total = uni(readlane_i(incl, 63));
    const int pre = incl - c; // first flattened position of this lane's leaf
    int carry = 0;            // lane of the leaf covering the position before the batch
    for (int t0 = 0; t0 < total; t0 += 64 * EB) {
        int j[EB];
#pragma unroll
        for (int u = 0; u < EB; u++) {
            const int b0 = t0 + 64 * u;
            int own = carry;
            uint64_t st = ballot(isl && c > 0 && pre >= b0 && pre < b0 + 64);
            for (int it = 0; it < 65 && st; it++) { // one round per leaf starting here
                const int ln = ctz64(st);
                st &= st - 1ull;
                const int off = uni(readlane_i(pre, ln)) - b0;
                if (lane >= off) own = ln;
            }
            carry = uni(readlane_i(own, 63));
            const int qc = min(b0 + lane, total - 1); // clamped: no divergence
            const int f = __shfl(inf.x, own, 64);
            const int p0 = __shfl(pre, own, 64);
            j[u] = f + (qc - p0);
        }
        decltype(visit.fetch(0)) p[EB];
#pragma unroll
        for (int u = 0; u < EB; u++)
            if (u == 0 || t0 + 64 * u < total) p[u] = visit.fetch(j[u]);
#pragma unroll
        for (int u = 0; u < EB; u++)
            if (u == 0 || t0 + 64 * u < total) visit.take(j[u], t0 + 64 * u + lane < total, p[u]);
    }
}

// inclusive prefix maximum over the lanes of a wave
__device__ __forceinline__ int wave_incl_max(int v)
{
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o, 64);
        if (lane >= o) v = max(v, t);
    }
    return v;
}

// Stackless pre-order walk of nodes [root, root_end): `visit` receives the
// particles of every opened leaf, in ascending order.
//
// The 64 lanes test the 64 consecutive pre-order nodes [k, k+64) at once.
// The window start is always on the walk (all its ancestors are open).  A
// closed node c hides its subtree, the node range (c, skip(c)); a node j of
// the window is on the walk iff no closed node before it in the window hides
// it, i.e. iff the prefix maximum of the skip links of the closed nodes
// before j does not exceed j (ancestors before the window are ancestors of
// the window start, hence open).  The next window starts at the larger of
// k + 64 and the largest skip link of a closed node in the window: every
// node in between is hidden.  Each window advances k by at least 64.
// does the ball reach node c's bounding box (hydro: with the node's max h)?
// In FP32 on the outward-rounded boxes, against the squared radius widened
// by 2^-16 relative + 2^-18 L rad (the rounding of the centre, of the gaps
// and their squares): every node the FP64 test on the exact box opens is
// opened (a few more at the rim only cost their tests).
__device__ __forceinline__ float axis_gap32(float c, float lo, float hi, float L)
{
    float a = lo - c, b = c - hi;
    float d = fmaxf(fmaxf(a, b), 0.0f);
    d = fminf(d, a + L);
    d = fminf(d, b + L);
    return d;
}
__device__ __forceinline__ bool box_open(const float4 &lo, const float4 &hi, const Ball &B)
{
    const float L = (float)B.L;
    const float gx = axis_gap32((float)B.cx, lo.x, hi.x, L);
    const float gy = axis_gap32((float)B.cy, lo.y, hi.y, L);
    const float gz = axis_gap32((float)B.cz, lo.z, hi.z, L);
    const float d2 = __builtin_fmaf(gz, gz, __builtin_fmaf(gy, gy, gx * gx));
    float lim;
    if (B.hydro) {
        const float rad = ((float)B.Rg + fmaxf((float)B.Hg, lo.w)) * (float)INFL;
        lim = __builtin_fmaf(rad * rad, 0x1p-16f, rad * rad) + 0x1p-18f * L * rad;
    } else {
        const float w2 = (float)B.W2;
        lim = __builtin_fmaf(w2, 0x1p-16f, w2) + 0x1p-18f * L * sqrtf(w2);
    }
    return d2 < lim;
}
__device__ __forceinline__ bool node_open(const Geom &g, int c, const Ball &B)
{
    return box_open(g.box32[2 * (int64_t)c], g.box32[2 * (int64_t)c + 1], B);
}

// The item of a node in the walks' lists: its index, its child count less
// one, and a leaf flag in the sign bit (the format of the child records).
__device__ __forceinline__ int item_node(int it) { return it & TREE_ITEM_NODE; }
__device__ __forceinline__ int item_kids(int it) { return ((it >> 28) & 7) + 1; }
__device__ __forceinline__ int root_item(const Geom &g, int root)
{
    const int4 ir = g.info[root];
    const int nc = g.nchild[root];
    return (ir.w >> 8) ? (root | (int)0x80000000u) : (root | ((max(nc, 1) - 1) << 28));
}

// Entry node of a walk (its item): from the root, step down while exactly
// one child of the current node is reached by the ball; every node the ball
// reaches then lies in the entry node's subtree, [entry, skip(entry)).  Lanes
// 0-7 test the children of the current node together, on the child records
// of the node (one load per level).
__device__ __forceinline__ int walk_entry(const Geom &g, int root, const Ball &B)
{
    const int lane = lane_id();
    int it = uni(root_item(g, root));
#pragma unroll 1
    for (int d = 0; d < 24; d++) { // 21 key levels below a root
        if (it < 0) break;         // a leaf
        const int p = item_node(it);
        bool open = false;
        int ci = -1;
        if (lane < item_kids(it)) {
            const int64_t r = 2 * (8 * (int64_t)p + lane);
            const float4 lo = g.krec[r], hi = g.krec[r + 1];
            open = box_open(lo, hi, B);
            ci = __float_as_int(hi.w);
        }
        const uint64_t m = ballot(open);
        if (popc64(m) != 1) break;
        const int nit = uni(readlane_i(ci, ctz64(m)));
        if (item_node(nit) <= p) break; // a child always follows its parent
        it = nit;
    }
    return it;
}

template <class V>
__device__ void walk(const Geom &g, int root, int root_end, const Ball &B, V &visit,
                     DevStatus *st)
{
    const int lane = lane_id();
    int k = uni(item_node(walk_entry(g, uni(root), B)));
    if (k != root) root_end = min(uni(root_end), uni(g.info[k].z));
    root_end = uni(root_end);
    int steps = 0;
    const int max_steps = (root_end - k) / 64 + 2;
    while (k < root_end) {
        if (visit.stop()) break;
        if (++steps > max_steps) {
            guard_hit(st);
            break;
        }
        const int node = k + lane;
        const bool inr = node < root_end;
        int4 inf = make_int4(0, 0, 0, 0);
        bool open = false;
        if (inr) {
            inf = g.info[node];
            open = node_open(g, node, B);
        }
        const int hide = (inr && !open) ? inf.z : -1;
        const int incl = wave_incl_max(hide);
        int excl = __shfl_up(incl, 1, 64);
        if (lane == 0) excl = -1;
        const bool on_walk = inr && excl <= node;
        const uint64_t vl = ballot(on_walk && open && (inf.w >> 8));
        const int far = uni(readlane_i(incl, 63));
        int nk = max(k + 64, far);
        if (vl) emit_leaves(vl, inf, visit);
        k = uni(min(nk, root_end));
    }
}

// Level-by-level walk for the group kernel.  An ordered list of items (in
// LDS) holds, in pre-order, the leaves reached so far and the internal nodes
// of the current level that the ball reaches; each round replaces every
// internal node by its reached children, in order, so the list stays in
// pre-order.  Only the children of reached nodes are tested (the window walk
// also tests the nodes hidden below closed ones).  At the end the list holds
// the reached leaves in ascending particle order, and they are emitted like
// the window walk emits them, so both walks hand the visitor the same
// particles in the same order.  Returns false, having emitted nothing, when
// the list would outgrow its LCAP slots; the caller then takes the window
// walk.
constexpr int LCAP = 256;

template <class V>
__device__ bool walk_levels(const Geom &g, int root, const Ball &B, int *la, int *lb, int *mk,
                            V &visit)
{
    const int lane = lane_id();
    const int ent = uni(walk_entry(g, uni(root), B));
    // a node other than the root was entered because the ball reaches it
    if (item_node(ent) == root && !uni_b(node_open(g, root, B))) return true; // reaches nothing
    if (lane == 0) la[0] = ent;
    int m = 1;
    wave_lds_sync();
    for (int level = 0; level < 24; level++) {
        int mb = 0;
        bool inner = false; // an internal node was kept: one more round
        for (int c0 = 0; c0 < m; c0 += 64) {
            const int idx = c0 + lane;
            const bool vi = idx < m;
            const int it = vi ? la[idx] : 0;
            const bool lf = it < 0;
            const int cnt = vi ? (lf ? 1 : item_kids(it)) : 0;
            int incl = cnt;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                int t = __shfl_up(incl, o, 64);
                if (lane >= o) incl += t;
            }
            const int total = uni(readlane_i(incl, 63));
            const int pre = incl - cnt;
            int carry = 0;
            for (int b0 = 0; b0 < total; b0 += 64) {
                // owner of each slot of this batch: the last item whose first
                // slot is at or before it (items in ascending order, distinct
                // first slots), by a prefix maximum over marks in LDS
                mk[lane] = -1;
                wave_lds_sync();
                if (cnt > 0 && pre >= b0 && pre < b0 + 64) mk[pre - b0] = lane;
                wave_lds_sync();
                int own = max(mk[lane], carry);
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int t = __shfl_up(own, o, 64);
                    if (lane >= o) own = max(own, t);
                }
                wave_lds_sync();
                carry = uni(readlane_i(own, 63));
                const bool valid = b0 + lane < total;
                const int oit = __shfl(it, own, 64);
                const int slot = b0 + lane - __shfl(pre, own, 64);
                int ci = oit; // a leaf item is carried over
                bool keep = valid;
                if (oit >= 0) { // an internal item: test its child `slot` on its record
                    keep = false;
                    if (valid) {
                        const int64_t r = 2 * (8 * (int64_t)item_node(oit) + min(max(slot, 0), 7));
                        const float4 lo = g.krec[r], hi = g.krec[r + 1];
                        keep = box_open(lo, hi, B);
                        ci = __float_as_int(hi.w);
                    }
                }
                const uint64_t km = ballot(keep);
                if (ballot(keep && ci >= 0)) inner = true;
                const int nk = popc64(km);
                if (mb + nk > LCAP) return false;
                if (keep) lb[mb + mbcnt(km)] = ci;
                mb = uni(mb + nk);
            }
        }
        wave_lds_sync();
        int *t = la;
        la = lb;
        lb = t;
        m = mb;
        if (!uni_b(inner)) break;
    }
    // the list now holds leaves only, ascending
    for (int c0 = 0; c0 < m; c0 += 64) {
        if (visit.stop()) break;
        const int idx = c0 + lane;
        const bool vi = idx < m;
        int4 inf = make_int4(0, 0, 0, 0);
        if (vi) inf = g.info[item_node(la[idx])];
        const uint64_t vl = ballot(vi);
        emit_leaves(vl, inf, visit);
    }
    wave_lds_sync();
    return true;
}

// minimum-image fold in FP32 (the FP32 copies of the positions)
__device__ __forceinline__ float fold32(float d, float L)
{
    const float half = 0.5f * L;
    if (d >= half) d = d - L;
    else if (d < -half) d = d + L;
    return d;
}

// canonical squared distance of x_j relative to x_i (fold when `wrap`)
__device__ __forceinline__ double r2_of(double xj, double yj, double zj, double xi, double yi,
                                        double zi, double L, bool wrap)
{
    double dx = xj - xi, dy = yj - yi, dz = zj - zi;
    if (wrap) {
        dx = fold(dx, L);
        dy = fold(dy, L);
        dz = fold(dz, L);
    }
    return __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
}

// Candidate collection for a group ball, straight into the candidate buffer.
// The test runs on the FP32 copies of the positions (and, for hydro, of h)
// against the ball's squared radius widened by 2^-16 relative plus
// 2^-18 L rad: that covers the rounding of the FP32 coordinates (at most
// 2^-24 L each), of their differences and squares and of the radius, so
// every particle of the exact ball is kept; the few extra ones at the rim
// cost a filter test and change no result (the filters are exact).  Also
// records whether a kept candidate needed the periodic fold relative to the
// centre and the largest per-axis displacement of a kept candidate
// (lane-wise, see pair_wrap).
// The walk kernel's chunk of the candidate buffer, [cur, end): a superset
// starts in what is left of it and, when it outgrows that, moves to a fresh
// chunk (what it wrote so far is copied), so that no group leaves a tile's
// worth of slots unused behind it.
struct CandChunk {
    DevStatus *st;
    int32_t *cand; // the whole buffer
    int64_t cap;   // its capacity
    int64_t cur, end;
    int size;      // slots of a fresh chunk (>= T)
    int x;         // XCD of the wave: its region of the buffer first
};

// Bump allocation of cnt candidates in region x (of 8) of the candidate
// buffer; -1 when every region is full.
__device__ __forceinline__ int64_t cand_alloc(DevStatus *st, int64_t cap, int x, int cnt)
{
    const int64_t rcap = cap >> 3;
    // the own region first, then the others: a region fills up before the
    // rest where its XCD took more than its share of the work
#pragma unroll 1
    for (int t = 0; t < 8; t++) {
        const int r = (x + t) & 7;
        unsigned long long off = 0ull;
        if (lane_id() == 0) off = atomicAdd(&st->cand_top[16 * r], (unsigned long long)cnt);
        off = uni_u64(off);
        if ((int64_t)off + cnt <= rcap) return (int64_t)r * rcap + (int64_t)off;
    }
    return -1;
}

struct AppendCand {
    static constexpr int EB = 3; // leaf batches in flight (emit_leaves)
    const float4 *p4; // x, y, z and, for hydro, h in FP32
    int *cand;
    int T;            // most candidates a superset may hold
    int room;         // slots at cand (<= T)
    int n;
    bool over;
    bool folded;
    Ball B;
    double ext;
    CandChunk *ck;    // the walk's chunk (grows into a fresh one), or NULL: room is all
    float cx, cy, cz, L, Rg, Hg, w2; // w2: widened density limit
    __device__ AppendCand(const float4 *p4_, int *cand_, int T_, const Ball &B_, double ext_,
                          int room_ = -1, CandChunk *ck_ = nullptr)
        : p4(p4_), cand(cand_), T(T_), room(room_ < 0 ? T_ : room_), n(0), over(false),
          folded(false), B(B_), ext(ext_), ck(ck_)
    {
        cx = (float)B.cx;
        cy = (float)B.cy;
        cz = (float)B.cz;
        L = (float)B.L;
        Rg = (float)B.Rg;
        Hg = (float)B.Hg;
        w2 = (float)(B.W2 * (1.0 + 0x1p-16) + 0x1p-18 * B.L * sqrt(B.W2));
    }
    __device__ bool stop() const { return over; }
    __device__ __forceinline__ float4 fetch(int j) const { return p4[j]; }
    __device__ __forceinline__ float lim(float hj) const
    {
        if (!B.hydro) return w2;
        const float rad = (Rg + fmaxf(Hg, hj)) * (float)INFL;
        return __builtin_fmaf(rad * rad, 0x1p-16f, rad * rad) + 0x1p-18f * L * rad;
    }
    __device__ void take(int j, bool valid, const float4 &p)
    {
        bool keep = false, fl = false;
        float e = 0.0f;
        if (B.nowrap) {
            // the ball lies inside the box: raw differences are the minimum
            // images of every candidate it can keep (and a particle whose
            // raw difference is not is farther than the ball radius either
            // way); `ext` already holds the ball radius
            if (valid) {
                const float dx = p.x - cx, dy = p.y - cy, dz = p.z - cz;
                keep = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)) < lim(p.w);
            }
        } else if (valid) {
            const float rx = p.x - cx, ry = p.y - cy, rz = p.z - cz;
            const float dx = fold32(rx, L), dy = fold32(ry, L), dz = fold32(rz, L);
            keep = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)) < lim(p.w);
            fl = (dx != rx) | (dy != ry) | (dz != rz);
            e = fmaxf(fabsf(dx), fmaxf(fabsf(dy), fabsf(dz)));
        }
        if (keep) ext = fmax(ext, (double)e * (1.0 + 0x1p-20));
        const uint64_t m = ballot(keep);
        if (ballot(keep && fl)) folded = true;
        const int cnt = popc64(m);
        if (n + cnt > room) {
            if (n + cnt > T || !ck || !grow()) {
                over = true;
                return;
            }
        }
        if (keep) cand[n + mbcnt(m)] = j;
        n = uni(n + cnt);
    }
    // move the superset to a fresh chunk of the buffer (room becomes T)
    __device__ bool grow()
    {
        const int64_t base = cand_alloc(ck->st, ck->cap, ck->x, ck->size);
        if (base < 0) {
            ck->cur = ck->end = -1;
            return false;
        }
        int *dst = ck->cand + base;
        // this wave wrote the first n entries: order them before the reads
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        for (int t = lane_id(); t < n; t += 64) dst[t] = cand[t];
        cand = dst;
        room = T;
        ck->cur = base;
        ck->end = base + ck->size;
        return true;
    }
};

// The raw difference x_j - x_i equals its minimum image (no fold needed) for
// every member i and candidate j when no one needed a fold relative to the
// centre and the two largest per-axis displacements add up to less than
// L/2 (with a margin for rounding); otherwise pairs fold.
__device__ __forceinline__ bool pair_wrap(bool folded, double cand_ext_lane, bool mfold, double mext,
                                          double L)
{
    const double ext = uni_d(wave_max_d(cand_ext_lane));
    return folded || mfold || !(ext + mext < 0.49 * L);
}

// box of particle i: side and octree root range
struct BoxInfo {
    double L;
    int root, root_end;
    int b;
};
__device__ __forceinline__ BoxInfo box_info(const Geom &geo, int i)
{
    const int b = geo.nb > 1 ? uni(box_of(geo.box_off, geo.nb, i)) : 0;
    BoxInfo bi;
    bi.L = uni_d(geo.box_L[b]);
    bi.root = uni(geo.box_root[b]);
    bi.root_end = uni(geo.box_root[b + 1]);
    bi.b = b;
    return bi;
}

} // namespace

// ================================================================== walk kernel
struct WalkK {
    Geom g;
    GroupArg ga;
    CandArg ca;
    DevStatus *st;
    const float4 *pos4; // FP32 x, y, z and (hydro) h per particle
    double skin;        // density ball: R_g + skin * max h; hydro: R_g + (skin - 1) * max h
    int hydro;          // 1: hydro ball R_s + max(max member h, h_j), R_s = R_g + (skin - 1) max h
};

// per-pass reset of the candidate buffer and the work counters (a kernel,
// not a memset, so that the step can be captured in a graph)
__global__ void k_reset_pass(DevStatus *st, int pass)
{
    const int t = threadIdx.x;
    if (blockIdx.x != 0) return;
    if (t < 32) st->sched[pass][t >> 2][t & 3] = (t & 3) == 0 ? ~0ull : 0ull;
    if (t < 8) {
        st->cand_top[16 * t] = 0ull;
        st->qctr[32 * t] = 0;
        st->qctr2[32 * t] = 0;
        st->qctr3[32 * t] = 0;
    }
    if (t == 8) st->n_dfr = 0ull;
    if (t == 9) st->n_glist = 0ull;
    if (t == 10) st->go_wtot = 0ull;
    for (int j = t; j < 8 * GO_K; j += blockDim.x) {
        st->go_tot[j] = 0;
        st->go_cur[j] = 0;
    }
}

// Reuse: the positions in the active list of the members whose active flag
// is set now, appended to sel (count in *cnt, zeroed before).  A wave takes
// SEL_CH consecutive blocks of 64 members, counts them, reserves their
// slots with one atomic (a single counter serialises its atomics) and
// writes them in order.
constexpr int SEL_CH = 8;
__global__ __launch_bounds__(256) void k_sel_members(const int32_t *__restrict__ n_act,
                                                     const int32_t *__restrict__ act,
                                                     const uint8_t *__restrict__ active,
                                                     int32_t *__restrict__ sel,
                                                     unsigned long long *__restrict__ cnt)
{
    const int A = *n_act;
    const int lane = lane_id();
    const int nw = (int)(gridDim.x * blockDim.x) >> 6;
    const int wv = (int)(blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    for (int c0 = wv * 64 * SEL_CH; c0 < A; c0 += nw * 64 * SEL_CH) {
        uint64_t m[SEL_CH];
        int total = 0;
#pragma unroll
        for (int u = 0; u < SEL_CH; u++) {
            const int a = c0 + 64 * u + lane;
            m[u] = ballot(a < A && active[act[a < A ? a : 0]] != 0);
            total += popc64(m[u]);
        }
        if (total == 0) continue;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(cnt, (unsigned long long)total);
        int b = readlane_i((int)base, 0);
#pragma unroll
        for (int u = 0; u < SEL_CH; u++) {
            if ((m[u] >> lane) & 1ull) sel[b + mbcnt(m[u])] = c0 + 64 * u + lane;
            b += popc64(m[u]);
        }
    }
}

// Reuse: the kept groups that hold a member active now.  First each
// selected member marks its group (gmark cleared before), then the marked
// groups are listed like the members (one atomic per SEL_CH blocks of 64).
__global__ __launch_bounds__(256) void k_gmark(const int32_t *__restrict__ sel,
                                               const unsigned long long *__restrict__ cnt,
                                               const int32_t *__restrict__ grp,
                                               int32_t *__restrict__ gmark)
{
    const int n = (int)*cnt;
    const int stride = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) gmark[grp[sel[i]]] = 1;
}
__global__ __launch_bounds__(256) void k_glist(const int32_t *__restrict__ n_groups,
                                               const int32_t *__restrict__ gmark,
                                               int32_t *__restrict__ glist,
                                               unsigned long long *__restrict__ cnt)
{
    const int G = *n_groups;
    const int lane = lane_id();
    const int nw = (int)(gridDim.x * blockDim.x) >> 6;
    const int wv = (int)(blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    for (int c0 = wv * 64 * SEL_CH; c0 < G; c0 += nw * 64 * SEL_CH) {
        uint64_t m[SEL_CH];
        int total = 0;
#pragma unroll
        for (int u = 0; u < SEL_CH; u++) {
            const int g = c0 + 64 * u + lane;
            m[u] = ballot(g < G && gmark[g] != 0);
            total += popc64(m[u]);
        }
        if (total == 0) continue;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(cnt, (unsigned long long)total);
        int b = readlane_i((int)base, 0);
#pragma unroll
        for (int u = 0; u < SEL_CH; u++) {
            if ((m[u] >> lane) & 1ull) glist[b + mbcnt(m[u])] = c0 + 64 * u + lane;
            b += popc64(m[u]);
        }
    }
}

// Order of the groups for the density group kernel.  Its queues hand each
// XCD the groups of one eighth of the index range, in index order
// (neighbouring groups share candidates in that XCD's L2).  A large group
// taken near the end of an eighth then runs alone while the other
// workgroups have finished.  So the heavy groups of each eighth move to its
// front, costliest first; every other group keeps its index order after
// them.  A group's cost is its member count times its
// superset size, w; class c holds the groups with w in
// [2^(c+GO_LOG0), 2^(c+GO_LOG0+1)) (the lowest and the highest class
// open-ended; a group without a kept superset in class 0), and a class is
// heavy when its upper bound reaches 1/GO_BETA of a workgroup's fair share
// of the total cost (sum of w over the number of workgroups).  Two passes
// over chunks of GO_CH groups: class totals per eighth and the total cost
// (atomics into the status block, cleared by the pass reset), then each
// chunk takes its slots per class with one atomic and scatters its groups
// in index order; the chunks of one class follow each other in the order
// of their atomics.  With many groups per workgroup (GQ_MANY or more) the
// groups are small against a workgroup's share and the order stays the
// index order (go_on = 0): no pass writes it and the group kernel reads no
// list.
constexpr int GO_LOG0 = 9;
constexpr int GO_BETA = 32;
struct GoSpan {
    int x, g0, g1; // eighth, chunk [g0, g1)
};
__device__ __forceinline__ GoSpan go_span(int G)
{
    const int per = (G + 7) >> 3;
    const int nch = (per + GO_CH - 1) / GO_CH;
    GoSpan sp;
    sp.x = nch > 0 ? (int)blockIdx.x / nch : 8;
    const int c = nch > 0 ? (int)blockIdx.x % nch : 0;
    const int e0 = sp.x * per, e1 = min((sp.x + 1) * per, G);
    sp.g0 = e0 + c * GO_CH;
    sp.g1 = sp.x < 8 ? min(sp.g0 + GO_CH, e1) : sp.g0;
    return sp;
}
// cost class of group g
__device__ __forceinline__ int go_raw(const GroupArg &ga, const GSup *sup, int g, int64_t &w)
{
    const GSup &sp = sup[g];
    w = (sp.flags & GSUP_SOLO) ? 0 : (int64_t)(ga.goff[g + 1] - ga.goff[g]) * sp.nc;
    const int lg = w > 0 ? 63 - __clzll(w) : 0;
    return min(max(lg - GO_LOG0, 0), GO_K - 1);
}
// grid: 8 x (groups per eighth / GO_CH) workgroups at least
__device__ __forceinline__ bool go_wanted(int G, int units)
{
    return (int64_t)G < (int64_t)GQ_MANY * units;
}
__global__ __launch_bounds__(256) void k_gcount(GroupArg ga, const GSup *__restrict__ sup, int units,
                                               DevStatus *st)
{
    __shared__ int h[GO_K];
    __shared__ unsigned long long ws;
    const int G = *ga.n_groups;
    if (!go_wanted(G, units)) return;
    const GoSpan sp = go_span(G);
    if (sp.g0 >= sp.g1) return;
    if (threadIdx.x < GO_K) h[threadIdx.x] = 0;
    if (threadIdx.x == 0) ws = 0ull;
    __syncthreads();
    unsigned long long mine = 0ull;
    for (int g = sp.g0 + (int)threadIdx.x; g < sp.g1; g += 256) {
        int64_t w;
        atomicAdd(&h[go_raw(ga, sup, g, w)], 1);
        mine += (unsigned long long)w;
    }
    if (mine) atomicAdd(&ws, mine);
    __syncthreads();
    if (threadIdx.x < GO_K && h[threadIdx.x]) atomicAdd(&st->go_tot[sp.x * GO_K + threadIdx.x], h[threadIdx.x]);
    if (threadIdx.x == 0 && ws) atomicAdd(&st->go_wtot, ws);
}
// the same grid: the positions of the chunk's groups in the order, for
// `units` workgroups of the group kernel; block 0 also sets go_on
__global__ __launch_bounds__(256) void k_gorder(GroupArg ga, const GSup *__restrict__ sup, int units,
                                               int32_t *__restrict__ order, DevStatus *st)
{
    __shared__ int base[GO_K], hk[GO_K], wc[4][GO_K];
    __shared__ int kmin_s;
    const int G = *ga.n_groups;
    const int t = threadIdx.x, lane = lane_id(), wv = t >> 6;
    if (blockIdx.x == 0 && t == 0) st->go_on = go_wanted(G, units) ? 1 : 0;
    if (!go_wanted(G, units)) return;
    const GoSpan sp = go_span(G);
    if (sp.g0 >= sp.g1) return;
    const int per = (G + 7) >> 3;
    if (t == 0) {
        const double share = (double)st->go_wtot / max(units, 1);
        int km = 0; // heavy: 2^(k + GO_LOG0 + 1) >= share / GO_BETA
        while (km < GO_K - 1 && ldexp(1.0, km + GO_LOG0 + 1) * GO_BETA < share) km++;
        kmin_s = km;
    }
    if (t < GO_K) hk[t] = 0;
    __syncthreads();
    const int kmin = kmin_s;
    // effective class: a heavy class, or kmin - 1 for every other group
    int kk[(GO_CH + 255) / 256];
#pragma unroll
    for (int u = 0; u < (GO_CH + 255) / 256; u++) {
        const int g = sp.g0 + 256 * u + t;
        int64_t w;
        kk[u] = g < sp.g1 ? max(go_raw(ga, sup, g, w), kmin - 1) : -2;
        if (kk[u] >= 0) atomicAdd(&hk[kk[u]], 1);
    }
    __syncthreads();
    if (t < GO_K) {
        int above = 0; // groups of the eighth in higher effective classes
        for (int k = max(t + 1, kmin); k < GO_K; k++) above += st->go_tot[sp.x * GO_K + k];
        base[t] = hk[t] ? sp.x * per + above + atomicAdd(&st->go_cur[sp.x * GO_K + t], hk[t]) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < (GO_CH + 255) / 256; u++) {
        const int g = sp.g0 + 256 * u + t;
        const int k = kk[u];
        int r = 0;
#pragma unroll
        for (int q = 0; q < GO_K; q++) {
            const uint64_t m = ballot(k == q);
            if (k == q) r = mbcnt(m);
            if (lane == 0) wc[wv][q] = popc64(m);
        }
        __syncthreads();
        if (k >= 0) {
            int o = base[k] + r;
            for (int w = 0; w < wv; w++) o += wc[w][k];
            order[o] = g;
        }
        __syncthreads();
        if (t < GO_K) base[t] += wc[0][t] + wc[1][t] + wc[2][t] + wc[3][t];
        __syncthreads();
    }
}

// After a reuse pass: every particle active now was a member of a kept group
__global__ void k_reuse_check(const unsigned long long *drift, DevStatus *st)
{
    if (blockIdx.x == 0 && threadIdx.x == 0 && drift[3] != drift[2])
        atomicOr(&st->flags, (unsigned)SFC_ST_REUSE_ACTIVE);
}

// One wave per group: the walk, the superset straight into the global
// buffer, the group record and the member -> group map.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(7))) void k_walk(WalkK k)
{
    extern __shared__ __align__(16) char lds_raw[];
    const int T = k.ga.T;
    int *lst = (int *)lds_raw; // [2 * LCAP + 64]: item lists of the level walk, owner marks
    const int lane = lane_id();
    const int G = uni(*k.ga.n_groups);
    Queue wq = queue_open(k.st->qctr, G, queue_qb(G, (int)gridDim.x, GQB, WQ_MANY));
    WaveStats ws;
    // candidates are placed in chunks taken by this wave: up to 8192 slots,
    // at most a quarter of a wave's fair share of the buffer, at least a tile
    CandChunk ck;
    ck.st = k.st;
    ck.cand = k.ca.cand;
    ck.cap = k.ca.cap;
    ck.size = (int)max((int64_t)T, min((int64_t)8192, k.ca.cap / (4 * (int64_t)gridDim.x)));
    ck.x = blockIdx.x & 7;
    ck.cur = ck.end = 0;
    for (int g = queue_next(wq); g >= 0; g = queue_next(wq)) {
        const int a = uni(k.ga.goff[g]);
        const int nm = min(uni(k.ga.goff[g + 1]) - a, 64);
        const bool mem = lane < nm;
        const int i = mem ? k.ga.act[a + lane] : 0;
        const int i0 = uni(readlane_i(i, 0));
        const BoxInfo bx = box_info(k.g, i0);
        double xi = 0.0, yi = 0.0, zi = 0.0, hi = 0.0;
        if (mem) {
            xi = k.g.x[i];
            yi = k.g.y[i];
            zi = k.g.z[i];
            hi = k.g.h[i];
        }
        const double cx = uni_d(readlane_d(xi, 0));
        const double cy = uni_d(readlane_d(yi, 0));
        const double cz = uni_d(readlane_d(zi, 0));
        const double rx = xi - cx, ry = yi - cy, rz = zi - cz;
        const double dx = fold(rx, bx.L), dy = fold(ry, bx.L), dz = fold(rz, bx.L);
        const bool mfold = ballot(mem && ((dx != rx) | (dy != ry) | (dz != rz))) != 0ull;
        const double mext =
            uni_d(wave_max_d(mem ? fmax(fabs(dx), fmax(fabs(dy), fabs(dz))) : 0.0));
        const double d = mem ? sqrt(__builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx))) : 0.0;
        const double R = uni_d(wave_max_d(d));
        const double H = uni_d(wave_max_d(hi));
        // hydro: the group radius widened by the skin (kept supersets stay
        // valid while members and neighbours move and h grows within it)
        const double Rs = k.hydro ? R + (k.skin - 1.0) * H : R;
        const double cov = k.hydro ? Rs + H : R + k.skin * H;
        // largest distance a kept candidate can have; the ball needs no
        // periodic fold when it stays inside the box on every axis
        const double rad =
            (k.hydro ? (Rs + fmax(H, uni_d(k.g.lo[bx.root].w))) * INFL : cov * INFL) * (1.0 + 0x1p-20);
        const int nowrap = cx - rad >= 0.0 && cx + rad < bx.L && cy - rad >= 0.0 &&
                           cy + rad < bx.L && cz - rad >= 0.0 && cz + rad < bx.L;
        Ball B{cx, cy, cz, bx.L, sq(cov * INFL), Rs, H, k.hydro, nowrap};
        // the superset goes straight to what is left of the wave's current
        // chunk of the buffer (a fresh chunk when that is nearly used up;
        // a superset that outgrows it moves to a fresh one)
        if (ck.cur >= 0 && ck.end - ck.cur < 64) {
            const int64_t base = cand_alloc(k.st, k.ca.cap, ck.x, ck.size);
            ck.cur = base;
            ck.end = base < 0 ? base : base + ck.size;
        }
        int flags = 0;
        int64_t c0 = 0;
        int nc = 0;
        const bool walked = ck.cur >= 0;
        if (!walked) { // the buffer is used up: the members walk on their own
            flags = GSUP_SOLO;
        } else {
            // the box's own cap on the superset, if its grouping table set one
            const int tb = k.ga.box_T ? uni(k.ga.box_T[bx.b]) : 0;
            const int Tb = tb > 0 ? min(max(tb, 64), T) : T;
            AppendCand ap(k.pos4, k.ca.cand + ck.cur, Tb, B, nowrap ? rad : 0.0,
                          (int)min((int64_t)Tb, ck.end - ck.cur), &ck);
            if (!walk_levels(k.g, bx.root, B, lst, lst + LCAP, lst + 2 * LCAP, ap)) // list too long: window walk
                walk(k.g, bx.root, bx.root_end, B, ap, k.st);
            nc = uni(ap.n);
            if (uni_b(ap.over)) {
                flags = GSUP_SOLO;
            } else {
                c0 = ck.cur;
                ck.cur += nc;
                if (pair_wrap(uni_b(ap.folded), ap.ext, mfold, mext, bx.L)) flags |= GSUP_WRAP;
            }
        }
        if (lane == 0) {
            GSup sp;
            sp.cx = cx;
            sp.cy = cy;
            sp.cz = cz;
            sp.cov = cov;
            sp.rs = Rs;
            sp.c0 = c0;
            sp.nc = (flags & GSUP_SOLO) ? 0 : nc;
            sp.flags = flags;
            k.ca.sup[g] = sp;
        }
        if (walked) ws.walks++;
        if (!(flags & GSUP_SOLO)) ws.cand += (unsigned long long)nc;
        if (flags & GSUP_SOLO) ws.overflow++;
        if (mem) k.ca.grp[a + lane] = g;
        wave_lds_sync();
    }
    ws.flush(k.st);
}

namespace {

// ------------------------------------------------------------------ per-member set-up
constexpr int FIFO_B = 2; // neighbour batches of 64 consumed together

// LDS of one member wave (the passes of members that walk alone):
// neighbour masks of the last filter pass, the FIFO and the squared-distance
// cache of the count passes.
// squared distances kept (as FP32) for the first R2C_MAX candidates
constexpr int R2C_MAX = 1024;
__host__ __device__ constexpr int r2c_len(int T, bool cache) { return cache ? (T < R2C_MAX ? T : R2C_MAX) : 0; }

constexpr int FIFO_BYTES = 64 * (FIFO_B + 1) * 4; // the larger FIFO (density: FIFO_B + 1 batches of ints)

struct MemLds {
    uint64_t *masks; // [T/64]
    void *fifo;      // FIFO_BYTES
    float *r2c;      // [r2c_len]: squared distances of the first pass
    int rc;
};
__host__ __device__ constexpr size_t mem_lds_bytes(int T, bool cache)
{
    return (size_t)8 * (T / 64) + (size_t)FIFO_BYTES + (size_t)4 * r2c_len(T, cache);
}
__device__ __forceinline__ MemLds mem_carve(char *base, int T, bool cache)
{
    const int wave = uni((int)(threadIdx.x >> 6));
    char *p = base + (size_t)wave * mem_lds_bytes(T, cache);
    MemLds m;
    m.masks = (uint64_t *)p;
    m.fifo = (void *)(m.masks + T / 64);
    m.r2c = (float *)((char *)m.fifo + FIFO_BYTES);
    m.rc = r2c_len(T, cache);
    return m;
}

struct Member {
    int i, g;
    double xi, yi, zi, h;
    double d;     // |x_i - x_0|
    GSup s;
    BoxInfo bx;
};
__device__ __forceinline__ GSup load_gsup(const GSup *sp)
{
    GSup s;
    s.cx = uni_d(sp->cx);
    s.cy = uni_d(sp->cy);
    s.cz = uni_d(sp->cz);
    s.cov = uni_d(sp->cov);
    s.rs = uni_d(sp->rs);
    const int64_t c0 = sp->c0;
    s.c0 = ((int64_t)uni((int)(c0 >> 32)) << 32) | (uint32_t)uni((int)(uint32_t)c0);
    s.nc = uni(sp->nc);
    s.flags = uni(sp->flags);
    return s;
}
__device__ __forceinline__ Member member(const Geom &geo, const GroupArg &ga, const CandArg &ca, int a)
{
    Member M;
    M.i = uni(ga.act[a]);
    M.g = uni(ca.grp[a]);
    M.s = load_gsup(ca.sup + M.g);
    M.bx = box_info(geo, M.i);
    M.xi = uni_d(geo.x[M.i]);
    M.yi = uni_d(geo.y[M.i]);
    M.zi = uni_d(geo.z[M.i]);
    M.h = uni_d(geo.h[M.i]);
    const double dx = fold(M.xi - M.s.cx, M.bx.L), dy = fold(M.yi - M.s.cy, M.bx.L),
                 dz = fold(M.zi - M.s.cz, M.bx.L);
    M.d = sqrt(__builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx)));
    return M;
}

// The walk of one particle inside the per-particle kernels: level by level
// with its item lists in the squared-distance cache (idle during the walk),
// the window walk when that cache is too small or the lists overflow.  Both
// give the same particles in the same order.
template <class V>
__device__ __forceinline__ void solo_walk(const Geom &g, const MemLds &S, const Member &M,
                                          const Ball &B, V &visit, DevStatus *st)
{
    int *lst = (int *)S.r2c;
    if (S.rc >= 2 * LCAP + 64 && walk_levels(g, M.bx.root, B, lst, lst + LCAP, lst + 2 * LCAP, visit))
        return;
    walk(g, M.bx.root, M.bx.root_end, B, visit, st);
}

// FIFO entries: a neighbour.  The pair's values (r^2 for density, the
// displacement for hydro) are formed when its term is computed, from the
// FP64 positions of the two particles only, so a particle's sums do not
// depend on the path that found the pair (group superset, own superset or
// own walk) nor on the group it was in.
struct DEnt {
    int j;
};
struct HEnt {
    int j;
};

// FIFO of neighbour entries; the k-th pushed entry is consumed by lane k%64.
// It holds up to B batches of 64 and hands them to the consumer together, so
// that the loads of B batches are in flight at once; each lane still adds its
// terms in push order.  The consumer provides term(entry) (loads and
// arithmetic of one pair) and add(term) (the accumulation).
template <int B, class E> struct FifoB {
    static constexpr int SIZE = 64 * (B + 1); // ring of SIZE entries
    E *buf;
    int np;       // entries held
    int head = 0; // ring position of the oldest entry
    __device__ __forceinline__ static int wrap(int i) { return i >= SIZE ? i - SIZE : i; }
    template <class F> __device__ __forceinline__ void run(F &f, int cnt)
    {
        const int lane = lane_id();
        typename F::Term t[B];
        bool v[B];
#pragma unroll
        for (int b = 0; b < B; b++) {
            const int idx = (b << 6) + lane;
            v[b] = idx < cnt;
            if ((b << 6) < cnt) t[b] = f.term(v[b] ? buf[wrap(head + idx)] : E{0});
        }
#pragma unroll
        for (int b = 0; b < B; b++)
            if ((b << 6) < cnt && v[b]) f.add(t[b]);
    }
    template <class F> __device__ __forceinline__ void push(bool hit, const E &e, F &f)
    {
        const uint64_t m = ballot(hit);
        if (!m) return;
        if (hit) buf[wrap(wrap(head + np) + mbcnt(m))] = e;
        np = uni(np + popc64(m));
        if (np >= 64 * B) {
            wave_lds_sync();
            run(f, 64 * B);
            head = uni(wrap(head + 64 * B));
            np -= 64 * B;
            wave_lds_sync();
        }
    }
    template <class F> __device__ __forceinline__ void flush(F &f)
    {
        wave_lds_sync();
        if (np > 0) run(f, np);
        np = 0;
        head = 0;
        wave_lds_sync();
    }
};
typedef FifoB<FIFO_B, DEnt> Fifo;
typedef FifoB<2, HEnt> FifoH; // hydro terms are larger: two batches at a time
static_assert(FifoB<FIFO_B, DEnt>::SIZE * sizeof(DEnt) <= FIFO_BYTES, "density FIFO fits");
static_assert(FifoB<2, HEnt>::SIZE * sizeof(HEnt) <= FIFO_BYTES, "hydro FIFO fits");

constexpr int UNR = 4; // candidate chunks loaded together

// Pair r^2 in FP32 from the FP32 copies of the positions (rounded to
// nearest), folded in FP32 when `wrap`: the screen of the count passes.
__device__ __forceinline__ float r2_f32(float xj, float yj, float zj, float xi, float yi, float zi,
                                        float L, bool wrap)
{
    float dx = xj - xi, dy = yj - yi, dz = zj - zi;
    if (wrap) {
        dx = fold32(dx, L);
        dy = fold32(dy, L);
        dz = fold32(dz, L);
    }
    return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

// density count pass over a member's own superset: masks of r2 < h2, their
// count.  The test is decided on the FP32 r^2 of the FP32 positions wherever
// that is safely away from h^2, and on the canonical FP64 r^2 otherwise, so
// the result is exactly that of the FP64 test.  Bound: each coordinate is
// off by at most u L (u = 2^-24, coordinates in [0, L)), a (folded)
// difference by 4 u L + u |d|, so near r = h the FP32 r^2 is within
// 14 u L h + 5 u h^2 of the FP64 one; the band is E = 16 u (L h + h^2).  The
// first pass keeps the FP32 r^2 of the first S.rc candidates in LDS for the
// later passes.
__device__ __forceinline__ int count_pass(const Geom &geo, const float4 *P, const int32_t *cand,
                                          const Member &M, double h, bool wrap, const MemLds &S,
                                          bool first)
{
    const int lane = lane_id();
    const int nc = M.s.nc;
    const int nch = (nc + 63) >> 6;
    const int32_t *cg = cand + M.s.c0;
    const double h2 = h * h;
    const double E = 0x1p-20 * (M.bx.L * h + h2);
    // the band's ends in FP32, rounded outwards: a candidate decided in FP32
    // is decided as before; the few that the rounding moves into the band
    // take the FP64 test
    const float lo_b = __double2float_rd(h2 - E), hi_b = __double2float_ru(h2 + E);
    const float xf = (float)M.xi, yf = (float)M.yi, zf = (float)M.zi, Lf = (float)M.bx.L;
    const int cached = first ? 0 : min(nch, S.rc >> 6);
    int cnt = 0;
    for (int c = 0; c < cached; c++) {
        const int slot = (c << 6) + lane;
        const bool v = slot < nc;
        const float r2f = v ? S.r2c[slot] : 0.0f;
        bool hit = r2f < lo_b;
        const bool amb = v && !hit && !(r2f > hi_b);
        if (ballot(amb)) {
            if (amb) {
                const int j = cg[slot];
                hit = r2_of(geo.x[j], geo.y[j], geo.z[j], M.xi, M.yi, M.zi, M.bx.L, wrap) < h2;
            }
        }
        const uint64_t hm = ballot(v && hit);
        if (lane == 0) S.masks[c] = hm;
        cnt += popc64(hm);
    }
    int jn[UNR];
#pragma unroll
    for (int u = 0; u < UNR; u++) jn[u] = cg[min(((cached + u) << 6) + lane, nc - 1)];
    for (int c0 = cached; c0 < nch; c0 += UNR) {
        int j[UNR];
        bool v[UNR];
#pragma unroll
        for (int u = 0; u < UNR; u++) {
            v[u] = ((c0 + u) << 6) + lane < nc;
            j[u] = jn[u];
        }
        float4 pj[UNR];
#pragma unroll
        for (int u = 0; u < UNR; u++) pj[u] = P[j[u]];
#pragma unroll
        for (int u = 0; u < UNR; u++) jn[u] = cg[min(((c0 + UNR + u) << 6) + lane, nc - 1)];
#pragma unroll
        for (int u = 0; u < UNR; u++) {
            const int slot = ((c0 + u) << 6) + lane;
            const float r2f = r2_f32(pj[u].x, pj[u].y, pj[u].z, xf, yf, zf, Lf, wrap);
            if (first && v[u] && slot < S.rc) S.r2c[slot] = r2f;
            bool hit = r2f < lo_b;
            const bool amb = v[u] && !hit && !(r2f > hi_b);
            if (ballot(amb)) {
                if (amb) {
                    const int jj = j[u];
                    hit = r2_of(geo.x[jj], geo.y[jj], geo.z[jj], M.xi, M.yi, M.zi, M.bx.L, wrap) < h2;
                }
            }
            const uint64_t hm = ballot(v[u] && hit);
            if (c0 + u < nch) {
                if (lane == 0) S.masks[c0 + u] = hm;
                cnt += popc64(hm);
            }
        }
    }
    wave_lds_sync();
    return uni(cnt);
}

// stream the neighbours recorded in the masks through the FIFO
template <class F>
__device__ __forceinline__ void stream_masks(const int32_t *cand, int64_t c0, int nc,
                                             const uint64_t *masks, Fifo &q, F &consume)
{
    const int lane = lane_id();
    const int nch = (nc + 63) >> 6;
    const int32_t *cg = cand + c0;
    for (int cb = 0; cb < nch; cb += UNR) {
        uint64_t mk[UNR];
        int j[UNR];
#pragma unroll
        for (int u = 0; u < UNR; u++) {
            mk[u] = cb + u < nch ? readlane_u64(masks[cb + u], 0) : 0ull;
            j[u] = mk[u] ? cg[min(((cb + u) << 6) + lane, nc - 1)] : 0;
        }
#pragma unroll
        for (int u = 0; u < UNR; u++) q.push((mk[u] >> lane) & 1ull, DEnt{j[u]}, consume);
    }
    q.flush(consume);
}

// counts |{j : r2 < h2}| over walked particles (solo path)
struct CountVisit {
    static constexpr int EB = 2; // leaf batches in flight (emit_leaves)
    const double *x, *y, *z;
    double xi, yi, zi, L, h2;
    int cnt;
    __device__ bool stop() const { return false; }
    __device__ __forceinline__ Pos fetch(int j) const
    {
        Pos p;
        p.x = x[j];
        p.y = y[j];
        p.z = z[j];
        p.h = 0.0;
        return p;
    }
    __device__ void take(int j, bool valid, const Pos &p)
    {
        (void)j;
        const bool hit = valid && r2_of(p.x, p.y, p.z, xi, yi, zi, L, true) < h2;
        cnt = uni(cnt + popc64(ballot(hit)));
    }
};

// filter walked particles against one particle and push the neighbours
template <int MODE, class F, class Q = Fifo> struct StreamVisit {
    static constexpr int EB = 2; // leaf batches in flight (emit_leaves)
    const double *x, *y, *z, *h;
    double xi, yi, zi, L, hi;
    int i;
    Q q;
    F *consume;
    __device__ bool stop() const { return false; }
    __device__ __forceinline__ Pos fetch(int j) const
    {
        Pos p;
        p.x = x[j];
        p.y = y[j];
        p.z = z[j];
        p.h = MODE == 1 ? h[j] : 0.0;
        return p;
    }
    __device__ void take(int j, bool valid, const Pos &p)
    {
        if constexpr (MODE == 0) {
            const double r2 = r2_of(p.x, p.y, p.z, xi, yi, zi, L, true);
            q.push(valid && r2 < hi * hi, DEnt{j}, *consume);
        } else {
            const double r2 = r2_of(p.x, p.y, p.z, xi, yi, zi, L, true);
            const double hm = fmax(hi, p.h);
            q.push(valid && (j != i) && (r2 < hm * hm), HEnt{j}, *consume);
        }
    }
};

// ------------------------------------------------------------------ group workgroups
// One workgroup of W waves per group (four; two for small neighbour counts,
// with at most GC_SMALL candidates staged, so that eight groups share a CU),
// groups taken from per-XCD work
// queues.  The group's superset is staged once into LDS: the FP64 positions
// of its first C candidates, with the mass (density) or h_j and the particle
// index (hydro); a superset larger than C reads the rest from global memory.
// Chunks of 64 consecutive candidates lie on the lanes.
//
// The membership test is the canonical FP64 one.  In a group that needs no
// periodic fold the raw differences are the minimum images, so the test is
// exact as written; in a group that does, every coordinate is moved into
// the frame of the group's centre (x - s L, s in {-1, 0, 1} per axis), and
// the test decides on those differences outside a band E = 2^-44 (L h + h^2)
// around h^2 (the two evaluations differ by less than 2^-48 L h + 2^-50 h^2),
// and on the canonical r^2 of the raw coordinates inside it.
constexpr int GW = 4;               // waves per group workgroup (2 for small neighbour counts)
constexpr int GKB = 4;              // candidate chunks a wave holds during a round
constexpr int GSTG = 4;             // candidates a thread stages per pass
constexpr int GC_MAX = 1024;        // staged candidates at most
constexpr int GC_SMALL = 512;       // staged candidates at most for two waves per group
constexpr int GMR = 32;             // members whose masks over the staged chunks are kept
constexpr int GFB = 2;              // batches a group wave's FIFO hands over at once

// shift of a coordinate into the frame of the centre c: x - L when it lies
// more than L/2 above c, x + L when more than L/2 below
__device__ __forceinline__ double to_frame(double x, double c, double L)
{
    const double d = x - c;
    return d >= 0.5 * L ? x - L : (d < -0.5 * L ? x + L : x);
}

__device__ __forceinline__ int wave_sum_i(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// append the members in `dm` (lanes) to the list of members that finish on
// their own, one atomic per group

__device__ __forceinline__ void defer_members(uint64_t dm, int a, int32_t *dfr, DevStatus *st)
{
    if (!dm) return;
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(&st->n_dfr, (unsigned long long)popc64(dm));
    const int b = (int)uni_u64(base);
    if ((dm >> lane_id()) & 1ull) dfr[b + mbcnt(dm)] = a;
}

// LDS of a group workgroup
struct GLds {
    double *cx, *cy, *cz; // [C] staged candidates: raw FP64 positions (NaN past the superset)
    uint64_t *rows;       // [GMR][C / 64]: the masks of member m over the staged chunks
    double *fin;          // [2][64] the lane-reduced sums of member m (W, its h derivative)
    float *cm;            // [C] staged candidates: m_j
    int32_t *mcnt;        // [3][64] neighbour counts of member m in round r (row r % 3)
    int32_t *ctl;         // [8]: the group taken
    char *fifo;           // one FIFO of 128 * (batches at once) entries per wave
    int C;
};
__host__ __device__ constexpr size_t glds_bytes(int C, int W)
{
    return (size_t)C * 28 + (size_t)8 * GMR * (C / 64) + 8 * 64 * 2 + 3 * 64 * 4 + 8 * 4 +
           (size_t)W * 128 * GFB * 4;
}
__device__ __forceinline__ GLds glds_carve(char *p, int C)
{
    GLds S;
    S.C = C;
    S.cx = (double *)p;
    p += 8 * (size_t)C;
    S.cy = (double *)p;
    p += 8 * (size_t)C;
    S.cz = (double *)p;
    p += 8 * (size_t)C;
    S.rows = (uint64_t *)p;
    p += (size_t)8 * GMR * (C / 64);
    S.fin = (double *)p;
    p += 8 * 128;
    S.cm = (float *)p;
    p += 4 * (size_t)C;
    S.mcnt = (int32_t *)p;
    p += 3 * 64 * 4;
    S.ctl = (int32_t *)p;
    p += 4 * 8;
    S.fifo = p;
    return S;
}

// The group's superset in global memory
struct GCand {
    const int32_t *cg; // its candidate indices
    int nc;
    const double4 *p64;
};

// Stage the first min(nc, C) candidates (all threads of the workgroup):
// their positions and masses.  The slots past nc up to the end of its chunk
// get NaN positions, on which every test fails.  Each pass loads GSTG
// indices per thread, then their records.
template <int W> __device__ __forceinline__ void stage_cands(const GLds &S, const GCand &gc)
{
    const int n = min(gc.nc, S.C);
    const int npad = min((gc.nc + 63) & ~63, S.C);
    const double nan = __builtin_nan("");
    for (int base = 0; base < npad; base += GSTG * W * 64) {
        int j[GSTG];
#pragma unroll
        for (int u = 0; u < GSTG; u++) {
            const int t = base + u * W * 64 + (int)threadIdx.x;
            j[u] = t < n ? gc.cg[t] : -1;
        }
        double4 p[GSTG];
#pragma unroll
        for (int u = 0; u < GSTG; u++) p[u] = gc.p64[j[u] < 0 ? 0 : j[u]];
#pragma unroll
        for (int u = 0; u < GSTG; u++) {
            const int t = base + u * W * 64 + (int)threadIdx.x;
            if (t < npad) {
                const bool v = j[u] >= 0;
                S.cx[t] = v ? p[u].x : nan;
                S.cy[t] = v ? p[u].y : nan;
                S.cz[t] = v ? p[u].z : nan;
                S.cm[t] = v ? (float)p[u].w : 0.0f;
            }
        }
    }
}

// candidate `slot` (one per lane): staged, or from global memory past the
// staged part; NaN past the superset
// (the LDS is read unconditionally at a clamped slot, so that the LDS and
// global paths never merge into one generic pointer)
__device__ __forceinline__ void cand_xyz(const GLds &S, const GCand &gc, int slot, double &x, double &y,
                                         double &z)
{
    const int sl = min(slot, S.C - 1);
    x = S.cx[sl];
    y = S.cy[sl];
    z = S.cz[sl];
    if (slot >= S.C) {
        const bool v = slot < gc.nc;
        const double4 p = gc.p64[gc.cg[v ? slot : gc.nc - 1]];
        const double nan = __builtin_nan("");
        x = v ? p.x : nan;
        y = v ? p.y : nan;
        z = v ? p.z : nan;
    }
}

// Is the candidate (frame coordinates fx, fy, fz) within sqrt(lim) of the
// member (frame coordinates xm, ym, zm)?  With WRAP, inside the band E the
// canonical squared distance of the raw coordinates, raw_r2(), decides.
template <bool WRAP, class R>
__device__ __forceinline__ bool in_ball(double fx, double fy, double fz, double xm, double ym,
                                        double zm, double lim, double E, const R &raw_r2)
{
    const double dx = fx - xm, dy = fy - ym, dz = fz - zm;
    const double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
    if (!WRAP) return r2 < lim;
    bool hit = r2 < lim - E;
    const bool amb = !hit && r2 <= lim + E;
    if (ballot(amb)) {
        if (amb) hit = raw_r2() < lim;
    }
    return hit;
}

// FIFO of a group workgroup's wave: a ring of 128 B entries in LDS; the k-th
// entry pushed is consumed by lane k % 64, B batches of 64 at a time (their
// loads in flight together), and each lane adds its terms in push order (the
// order of FifoB, so both give the same sums).
template <class E, int B> struct GFifo {
    static constexpr int RING = 128 * B; // a power of two for B = 1, 2, 4
    E *buf;
    int head, np; // ring position of the oldest entry (a multiple of 64), entries held
    template <class F> __device__ __forceinline__ void run(F &f, int cnt)
    {
        const int lane = lane_id();
        typename F::Term t[B];
        bool v[B];
#pragma unroll
        for (int b = 0; b < B; b++) {
            const int idx = (b << 6) + lane;
            v[b] = idx < cnt;
            if ((b << 6) < cnt) t[b] = f.term(v[b] ? buf[(head + idx) & (RING - 1)] : E{0});
        }
#pragma unroll
        for (int b = 0; b < B; b++)
            if ((b << 6) < cnt && v[b]) f.add(t[b]);
    }
    // push entry e of every lane set in the (uniform) mask mk
    template <class F> __device__ __forceinline__ void push(uint64_t mk, const E &e, F &f)
    {
        if (!mk) return;
        if ((mk >> lane_id()) & 1ull) buf[(head + np + mbcnt(mk)) & (RING - 1)] = e;
        np = uni(np + popc64(mk));
        if (np >= 64 * B) {
            wave_lds_sync();
            run(f, 64 * B);
            head = uni((head + 64 * B) & (RING - 1));
            np -= 64 * B;
            wave_lds_sync();
        }
    }
    template <class F> __device__ __forceinline__ void flush(F &f)
    {
        wave_lds_sync();
        if (np > 0) run(f, np);
        np = 0;
        head = 0;
        wave_lds_sync();
    }
};

// The members of a group in the lanes of every wave of its workgroup (each
// wave loads them; lane m holds member m)
struct GMem {
    double rx, ry, rz; // raw position
    double h;          // density: h of the current round
    double d;          // distance to the group centre (density: plus the drift)
    int i;             // particle
    bool live;         // takes part (a reuse pass: active now)
};
__device__ __forceinline__ GMem grp_members(const Geom &geo, const GroupArg &ga, const uint8_t *active,
                                            int a0, int M, const GSup &s, double L, double dl)
{
    const int lane = lane_id();
    GMem gm;
    gm.live = lane < M;
    gm.i = 0;
    gm.rx = gm.ry = gm.rz = gm.h = gm.d = 0.0;
    if (gm.live) {
        gm.i = ga.act[a0 + lane];
        gm.rx = geo.x[gm.i];
        gm.ry = geo.y[gm.i];
        gm.rz = geo.z[gm.i];
        gm.h = geo.h[gm.i];
        if (active) gm.live = active[gm.i] != 0; // reuse: the members active now
        const double dx = fold(gm.rx - s.cx, L), dy = fold(gm.ry - s.cy, L), dz = fold(gm.rz - s.cz, L);
        gm.d = sqrt(__builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx))) + dl;
    }
    return gm;
}

// One filter round (all waves of the workgroup) of the members in `ev`: wave
// w takes blocks w, w + W, ... of GKB chunks, holds their candidates in
// registers and tests them against every member of ev (r < h_m; member data
// from lane m by readlane).  Member m's mask over staged chunk c goes to
// S.rows[m * (C / 64) + c] (m < GMR); the counts are added to cnt_m[m].
template <bool WRAP, int W>
__device__ __forceinline__ void grp_round(const GLds &S, const GCand &gc, const GSup &s, double L,
                                          uint64_t ev, const GMem &gm, int32_t *cnt_m)
{
    const int lane = lane_id();
    const int wv = uni((int)(threadIdx.x >> 6));
    const int nch = (gc.nc + 63) >> 6;
    const int RC = S.C >> 6;
    const double xm = WRAP ? to_frame(gm.rx, s.cx, L) : gm.rx;
    const double ym = WRAP ? to_frame(gm.ry, s.cy, L) : gm.ry;
    const double zm = WRAP ? to_frame(gm.rz, s.cz, L) : gm.rz;
    const double limv = gm.h * gm.h;
    const double Ev = WRAP ? 0x1p-44 * (L * gm.h + gm.h * gm.h) : 0.0;
    int cntv = 0;
    for (int cb = wv * GKB; cb < nch; cb += W * GKB) {
        double x[GKB], y[GKB], z[GKB];
#pragma unroll
        for (int u = 0; u < GKB; u++) {
            if (cb + u < nch) {
                cand_xyz(S, gc, ((cb + u) << 6) + lane, x[u], y[u], z[u]);
                if (WRAP) {
                    x[u] = to_frame(x[u], s.cx, L);
                    y[u] = to_frame(y[u], s.cy, L);
                    z[u] = to_frame(z[u], s.cz, L);
                }
            }
        }
        uint64_t rest = ev;
        while (rest) {
            const int m = ctz64(rest);
            rest &= rest - 1ull;
            const double xmm = readlane_d(xm, m), ymm = readlane_d(ym, m), zmm = readlane_d(zm, m);
            const double lim = readlane_d(limv, m);
            const double E = WRAP ? readlane_d(Ev, m) : 0.0;
            int cnt = 0;
#pragma unroll
            for (int u = 0; u < GKB; u++) {
                if (cb + u < nch) {
                    const int slot = ((cb + u) << 6) + lane;
                    const bool hit = in_ball<WRAP>(x[u], y[u], z[u], xmm, ymm, zmm, lim, E, [&]() {
                        double px, py, pz;
                        cand_xyz(S, gc, slot, px, py, pz);
                        return r2_of(px, py, pz, readlane_d(gm.rx, m), readlane_d(gm.ry, m),
                                     readlane_d(gm.rz, m), L, true);
                    });
                    const uint64_t mk = ballot(hit);
                    cnt += popc64(mk);
                    if (m < GMR && cb + u < RC && lane == 0) S.rows[m * RC + cb + u] = mk;
                }
            }
            cntv += lane == m ? cnt : 0;
        }
    }
    if ((ev >> lane) & 1ull) atomicAdd(&cnt_m[lane], cntv);
}

// the start and end of one workgroup or wave of a scheduled kernel (slot k
// of DevStatus::sched), on the device's constant clock: the spread of the
// ends is the tail that the work queues leave
__device__ __forceinline__ void sched_mark(DevStatus *st, int k, unsigned long long t0)
{
    const unsigned long long t1 = wall_clock64();
    unsigned long long *q = st->sched[k][blockIdx.x & 7];
    atomicMin(&q[0], t0);
    atomicMax(&q[1], t1);
    atomicAdd(&q[2], t1);
    atomicAdd(&q[3], 1ull);
}

// The groups of a workgroup: wave 0 takes them from the queue and looks
// each up in the list `gl` (NULL: the item is the group), one group ahead,
// so that the look-up of the next group runs while the workgroup works on
// the current one.

struct WgTake {
    Queue q;
    const int32_t *gl;
    int next; // wave 0: the group after the current one (-1: none left)
};
__device__ __forceinline__ int wg_resolve(WgTake &w)
{
    const int item = queue_next(w.q);
    return item < 0 ? -1 : (w.gl ? w.gl[item] : item);
}
__device__ __forceinline__ WgTake wg_open(int32_t *ctr, int n_items, const int32_t *gl)
{
    WgTake w;
    w.q = queue_open(ctr, n_items, queue_qb(n_items, (int)gridDim.x, GQB, GQ_MANY));
    w.gl = gl;
    w.next = threadIdx.x < 64 ? wg_resolve(w) : -1;
    return w;
}
// the group taken by the workgroup (-1: none left)
__device__ __forceinline__ int wg_take(WgTake &w, const GLds &S)
{
    if (threadIdx.x < 64) {
        if (threadIdx.x == 0) S.ctl[0] = w.next;
        w.next = w.next < 0 ? -1 : wg_resolve(w);
    }
    __syncthreads();
    return uni(S.ctl[0]);
}
} // namespace

// ================================================================== density
struct DensK {
    Geom g;
    GroupArg ga;
    CandArg ca;
    const float4 *pos4;  // FP32 x, y, z and m per particle (walks, own-superset count passes)
    const double4 *p64;  // FP64 x, y, z and the mass per particle (group staging, pair terms)
    const float *m;
    float *rho, *fgrad;
    sfc_density_out out;
    DevStatus *st;
    int64_t priv; // offset in the candidate buffer of the private slots (T per wave), -1: none
    const unsigned long long *drift; // reused supersets: [0] largest displacement (FP64 bits), or NULL
    const uint8_t *active;           // reused supersets: the members computed now
    int32_t *dfr;                    // members that finish on their own (st->n_dfr of them)
    double4 *dstate;                 // per active: h, bracket lo, hi and evaluations so far
    const int32_t *glist;            // reuse: the groups holding a member active now
                                     // (st->n_glist of them), or NULL
    const int32_t *gord;             // otherwise: every group, in the order to take them
                                     // when st->go_on is set
    int n_ngb, dn, max_iter, fixed_h;
    int C;                           // candidates a group workgroup stages in LDS
    int trace; // schedule statistics (DevStatus::sched)
};

namespace {

template <int KER, typename ACC> struct DensAcc {
    double xi, yi, zi, L;
    bool wrap;
    double h2;
    ACC hinv, inv_h2;
    Kahan<ACC> sw, sd;
    struct Term {
        ACC w, d;
    };
    __device__ __forceinline__ void init(double x, double y, double z, double Lb, double h, bool wr)
    {
        xi = x;
        yi = y;
        zi = z;
        L = Lb;
        wrap = wr;
        h2 = h * h;
        hinv = (ACC)(1.0 / h);
        inv_h2 = (ACC)(1.0 / (h * h));
    }
    // the pair term from the neighbour's FP64 position and mass: the
    // canonical FP64 r^2 of the pair, rounded once for the FP32 sums
    __device__ __forceinline__ Term make(double xj, double yj, double zj, float mjf) const
    {
        const double r2 = r2_of(xj, yj, zj, xi, yi, zi, L, wrap);
        const ACC q = acc_sqrt((ACC)r2) * hinv;
        ACC w, dw;
        kern_eval_u<KER, ACC>(q, tail_u<ACC>(h2, r2, inv_h2, q), w, dw);
        const ACC mj = (ACC)mjf;
        Term t;
        t.w = mj * w;
        t.d = mj * mad(q, dw, ACC(3) * w);
        return t;
    }
    __device__ __forceinline__ void add(const Term &t)
    {
        sw.add(t.w);
        sd.add(t.d);
    }
};

// neighbours given by particle index
template <int KER, typename ACC> struct DensPair : DensAcc<KER, ACC> {
    using Term = typename DensAcc<KER, ACC>::Term;
    const double4 *p64;
    const float *m;
    __device__ __forceinline__ Term term(const DEnt &e) const
    {
        const double4 pj = p64[e.j];
        return this->make(pj.x, pj.y, pj.z, (float)pj.w);
    }
};

// neighbours given by their slot in a staged group superset
template <int KER, typename ACC> struct DensPairS : DensAcc<KER, ACC> {
    using Term = typename DensAcc<KER, ACC>::Term;
    GLds S;
    GCand gc;
    const float *m;
    __device__ __forceinline__ Term term(const DEnt &e) const
    {
        const int s = e.j;
        const int sl = min(s, S.C - 1);
        double xj = S.cx[sl], yj = S.cy[sl], zj = S.cz[sl];
        float mj = S.cm[sl];
        if (s >= S.C) {
            const int j = gc.cg[s];
            const double4 pj = gc.p64[j];
            xj = pj.x;
            yj = pj.y;
            zj = pj.z;
            mj = (float)pj.w;
        }
        return this->make(xj, yj, zj, mj);
    }
};

template <int KER, typename ACC>
__device__ __forceinline__ DensPair<KER, ACC> dens_pair(const DensK &k, double xi, double yi,
                                                        double zi, double L, double h, bool wrap)
{
    DensPair<KER, ACC> pp;
    pp.init(xi, yi, zi, L, h, wrap);
    pp.p64 = k.p64;
    pp.m = k.m;
    return pp;
}

// rho, drho/dh and f of particle i at its final h from its lane-reduced sums
// of m_j w and m_j (q w' + 3 w) (any lane)
template <int KER>
__device__ void dens_finish(const DensK &k, int i, double h, double Sw, double Sd)
{
    constexpr double C = knorm<KER>();
    double h3 = h * h * h;
    double rho = C * Sw / h3;
    double drho = -C * Sd / (h3 * h);
    double f = 1.0 / (1.0 + h / (3.0 * rho) * drho);
    k.rho[i] = (float)rho;
    k.fgrad[i] = (float)f;
    if (k.out.drhodh) k.out.drhodh[i] = (float)drho;
    if (k.out.rho64) k.out.rho64[i] = rho;
    if (k.out.drhodh64) k.out.drhodh64[i] = drho;
    if (k.out.fgrad64) k.out.fgrad64[i] = f;
}

template <int KER, typename ACC, class P>
__device__ void dens_write(const DensK &k, int i, double h, int nn, int it, bool conv,
                           const P &pp, WaveStats &ws)
{
    ws.iters += (uint32_t)it;
    ws.pairs += (unsigned)nn;
    if (!conv) ws.not_conv++;
    double Sw = (double)wave_sum_f_or_d(pp.sw.value());
    double Sd = (double)wave_sum_f_or_d(pp.sd.value());
    if (lane_id() != 0) return;
    constexpr double C = knorm<KER>();
    double h3 = h * h * h;
    double rho = C * Sw / h3;
    double drho = -C * Sd / (h3 * h);
    double f = 1.0 / (1.0 + h / (3.0 * rho) * drho);
    k.g.h[i] = h;
    k.rho[i] = (float)rho;
    k.fgrad[i] = (float)f;
    if (k.out.drhodh) k.out.drhodh[i] = (float)drho;
    if (k.out.nngb) k.out.nngb[i] = nn;
    if (k.out.iters) k.out.iters[i] = it;
    if (k.out.converged) k.out.converged[i] = conv ? 1 : 0;
    if (k.out.rho64) k.out.rho64[i] = rho;
    if (k.out.drhodh64) k.out.drhodh64[i] = drho;
    if (k.out.fgrad64) k.out.fgrad64[i] = f;
}

// one particle on its own: one walk per h evaluation, then the sums
template <int KER, typename ACC>
__device__ void dens_solo(const DensK &k, const MemLds &S, const Member &M, double h, double lo,
                          double hi, int it, WaveStats &ws)
{
    int nn = 0;
    bool conv = false;
    for (int guard = 0; guard <= k.max_iter; guard++) {
        Ball B{M.xi, M.yi, M.zi, M.bx.L, sq(h * INFL), 0.0, 0.0, 0};
        CountVisit cv{k.g.x, k.g.y, k.g.z, M.xi, M.yi, M.zi, M.bx.L, h * h, 0};
        walk(k.g, M.bx.root, M.bx.root_end, B, cv, k.st);
        ws.walks++;
        nn = uni(cv.cnt);
        it++;
        if (k.fixed_h || (nn >= k.n_ngb - k.dn && nn <= k.n_ngb + k.dn)) {
            conv = true;
            break;
        }
        if (it >= k.max_iter) break;
        h = uni_d(h_step(nn, k.n_ngb, k.dn, h, lo, hi));
        lo = uni_d(lo);
        hi = uni_d(hi);
    }
    DensPair<KER, ACC> pp = dens_pair<KER, ACC>(k, M.xi, M.yi, M.zi, M.bx.L, h, true);
    StreamVisit<0, DensPair<KER, ACC>> sv{k.g.x, k.g.y, k.g.z, k.g.h, M.xi, M.yi, M.zi, M.bx.L, h, M.i,
                                          Fifo{(DEnt *)S.fifo, 0}, &pp};
    Ball B{M.xi, M.yi, M.zi, M.bx.L, sq(h * INFL), 0.0, 0.0, 0};
    walk(k.g, M.bx.root, M.bx.root_end, B, sv, k.st);
    sv.q.flush(pp);
    ws.walks++;
    dens_write<KER, ACC>(k, M.i, h, nn, it, conv, pp, ws);
}

// h iteration on the (own) superset of M: 1 when h is final (in the window,
// or max_iter evaluations), 0 when h has outgrown the superset (h + d > cov);
// the masks of the last evaluation stay in LDS
__device__ __forceinline__ int iterate(const DensK &k, const Member &M, const MemLds &S, double &h,
                                       double &lo, double &hi, int &it, int &nn, bool &conv,
                                       WaveStats &ws)
{
    bool first = true;
    while (it < k.max_iter) {
        if (!(h + M.d <= M.s.cov)) return 0;
        // own supersets carry GSUP_WRAP; a reused one may fold after the drift
        const bool wrap = (M.s.flags & GSUP_WRAP) || k.drift;
        nn = count_pass(k.g, k.pos4, k.ca.cand, M, h, wrap, S, first);
        ws.tests += (unsigned)M.s.nc;
        first = false;
        it++;
        if (k.fixed_h || (nn >= k.n_ngb - k.dn && nn <= k.n_ngb + k.dn)) {
            conv = true;
            return 1;
        }
        if (it >= k.max_iter) return 1;
        h = uni_d(h_step(nn, k.n_ngb, k.dn, h, lo, hi));
        lo = uni_d(lo);
        hi = uni_d(hi);
    }
    return 1;
}

// A private superset for one particle: one walk with radius `rad` around
// x_i, straight into the wave's private slot of T candidates (a fixed area
// behind the group supersets, reused particle after particle: a private
// superset is dead once its particle is done).  False if the slot is too
// small or there are no slots.
__device__ __forceinline__ bool own_superset(const DensK &k, const MemLds &S, Member &M, double rad,
                                             WaveStats &ws)
{
    const int T = k.ga.T;
    if (k.priv < 0) return false;
    const int wave = (int)blockIdx.x * (int)(blockDim.x >> 6) + uni((int)(threadIdx.x >> 6));
    const int64_t base = k.priv + (int64_t)wave * T;
    Ball B{M.xi, M.yi, M.zi, M.bx.L, sq(rad * INFL), 0.0, 0.0, 0};
    AppendCand ap(k.pos4, k.ca.cand + base, T, B, 0.0);
    solo_walk(k.g, S, M, B, ap, k.st);
    ws.walks++;
    if (uni_b(ap.over)) return false;
    M.s.cx = M.xi;
    M.s.cy = M.yi;
    M.s.cz = M.zi;
    M.s.cov = rad;
    M.s.c0 = (int64_t)base;
    M.s.nc = uni(ap.n);
    M.s.flags = GSUP_WRAP | GSUP_FRESH;
    M.d = 0.0;
    return true;
}

constexpr int ST_ITER = 0, ST_DONE = 1, ST_DEFER = 2;

// Member m's neighbours (one wave): its masks of the last round (re-tested
// for members past GMR and chunks past the staged ones) pushed in candidate
// order through the wave's FIFO into the sums.  Returns the neighbour count.
template <int KER, typename ACC, bool WRAP>
__device__ __forceinline__ int dens_emit(const DensK &k, const GLds &S, const GCand &gc, const GSup &s,
                                         double L, bool wrap, const GMem &gm, int m, DEnt *fifo)
{
    const int lane = lane_id();
    const double rx = uni_d(readlane_d(gm.rx, m)), ry = uni_d(readlane_d(gm.ry, m)),
                 rz = uni_d(readlane_d(gm.rz, m));
    const double h = uni_d(readlane_d(gm.h, m));
    const double lim = h * h;
    const double E = WRAP ? 0x1p-44 * (L * h + h * h) : 0.0;
    const double xm = WRAP ? to_frame(rx, s.cx, L) : rx;
    const double ym = WRAP ? to_frame(ry, s.cy, L) : ry;
    const double zm = WRAP ? to_frame(rz, s.cz, L) : rz;
    DensPairS<KER, ACC> pp;
    pp.init(rx, ry, rz, L, h, wrap);
    pp.S = S;
    pp.gc = gc;
    pp.m = k.m;
    GFifo<DEnt, GFB> q{fifo, 0, 0};
    const int nch = (gc.nc + 63) >> 6;
    const int RC = S.C >> 6;
    // the member's masks over the staged chunks, word c in lane c
    const uint64_t row = (m < GMR && lane < RC) ? S.rows[m * RC + lane] : 0ull;
    int nn = 0;
    for (int c = 0; c < nch; c++) {
        const int slot = (c << 6) + lane;
        uint64_t mk;
        if (m < GMR && c < RC) {
            mk = uni_u64(readlane_u64(row, c));
        } else {
            double x, y, z;
            cand_xyz(S, gc, slot, x, y, z);
            const double fx = WRAP ? to_frame(x, s.cx, L) : x;
            const double fy = WRAP ? to_frame(y, s.cy, L) : y;
            const double fz = WRAP ? to_frame(z, s.cz, L) : z;
            mk = ballot(in_ball<WRAP>(fx, fy, fz, xm, ym, zm, lim, E,
                                      [&]() { return r2_of(x, y, z, rx, ry, rz, L, true); }));
        }
        nn += popc64(mk);
        q.push(mk, DEnt{slot}, pp);
    }
    q.flush(pp);
    // the lanes' sums, reduced by the fixed butterfly, for the workgroup's
    // lane-parallel finish
    const double Sw = (double)wave_sum_f_or_d(pp.sw.value());
    const double Sd = (double)wave_sum_f_or_d(pp.sd.value());
    if (lane == 0) {
        S.fin[m] = Sw;
        S.fin[64 + m] = Sd;
    }
    return nn;
}
} // namespace

// Density, one workgroup per group: the members iterate h together on the
// staged superset, one filter round at a time.  Every wave keeps the h loop
// state of all members in its lanes (lane m: member m) and applies the same
// h step after the round's barrier, so one barrier per round suffices (the
// counts of round r go to row r % 3 of S.mcnt; wave 0 clears row r + 1 in
// round r, when every wave has read it in round r - 2).  Members whose h
// outgrows the superset, or whose group kept none, are listed for
// k_dens_solo with the state they reached; every member that finished is
// then streamed by one wave into its sums from its masks of the last round,
// and wave 0 finishes rho, drho/dh and f of all of them, one lane each.
template <int KER, typename ACC, int W>
__global__ __launch_bounds__(W * 64) __attribute__((amdgpu_waves_per_eu(4))) void k_dgrp(DensK k)
{
    extern __shared__ __align__(16) char lds_raw[];
    const unsigned long long t_start = wall_clock64();
    const GLds S = glds_carve(lds_raw, k.C);
    const int lane = lane_id();
    const int wv = uni((int)(threadIdx.x >> 6));
    DEnt *fifo = (DEnt *)(S.fifo + (size_t)wv * 128 * GFB * sizeof(DEnt));
    // a reuse pass takes only the groups that hold a member active now
    const int32_t *gl = k.glist ? k.glist : (k.gord && uni(k.st->go_on) ? k.gord : nullptr);
    WgTake wq = wg_open(k.st->qctr2, k.glist ? uni((int)k.st->n_glist) : uni(*k.ga.n_groups), gl);
    WaveStats ws;
    // a reused superset: every particle may have moved by dl since the walk
    const double dl = k.drift ? __longlong_as_double((long long)*k.drift) : 0.0;
    for (;;) {
        const int g = wg_take(wq, S);
        if (g < 0) break;
        const GSup s = load_gsup(k.ca.sup + g);
        const int a0 = uni(k.ga.goff[g]);
        const int M = min(uni(k.ga.goff[g + 1]) - a0, 64);
        const BoxInfo bx = box_info(k.g, uni(k.ga.act[a0]));
        const bool wrap = (s.flags & GSUP_WRAP) || k.drift;
        const GCand gc{k.ca.cand + s.c0, s.nc, k.p64};
        GMem gm = grp_members(k.g, k.ga, k.active, a0, M, s, bx.L, dl);
        // the h loop state of member `lane` (the same in every wave)
        int it = 0, nn = 0;
        int stt = gm.live ? ((s.flags & GSUP_SOLO) ? ST_DEFER : ST_ITER) : ST_DONE;
        if (stt == ST_ITER && !(gm.h + gm.d <= s.cov)) stt = ST_DEFER;
        double lo = 0.0, hi = INFINITY;
        bool conv = false;
        uint64_t ev = ballot(stt == ST_ITER);
        if (wv == 0) {
            S.mcnt[lane] = 0;
            S.mcnt[64 + lane] = 0;
        }
        if (!(s.flags & GSUP_SOLO)) stage_cands<W>(S, gc);
        __syncthreads();
        for (int round = 0; ev && round <= k.max_iter; round++) {
            int32_t *cnt = S.mcnt + 64 * (round % 3);
            if (wv == 0) S.mcnt[64 * ((round + 1) % 3) + lane] = 0;
            if (wrap)
                grp_round<true, W>(S, gc, s, bx.L, ev, gm, cnt);
            else
                grp_round<false, W>(S, gc, s, bx.L, ev, gm, cnt);
            __syncthreads();
            if (wv == 0) ws.tests += (unsigned long long)popc64(ev) * (unsigned long long)s.nc;
            if ((ev >> lane) & 1ull) {
                it++;
                nn = cnt[lane];
                if (k.fixed_h || (nn >= k.n_ngb - k.dn && nn <= k.n_ngb + k.dn)) {
                    conv = true;
                    stt = ST_DONE;
                } else if (it >= k.max_iter) {
                    stt = ST_DONE;
                } else {
                    gm.h = h_step(nn, k.n_ngb, k.dn, gm.h, lo, hi);
                    if (!(gm.h + gm.d <= s.cov)) stt = ST_DEFER;
                }
            }
            ev = ballot(stt == ST_ITER);
        }
        const bool done = gm.live && stt == ST_DONE;
        const uint64_t dn = ballot(done);
        if (wv == 0) {
            // a member still iterating here has hit the round limit: impossible
            // while every round advances it, kept as a guard
            if (ballot(stt == ST_ITER)) guard_hit(k.st);
            const uint64_t dm = ballot(gm.live && stt == ST_DEFER);
            if ((dm >> lane) & 1ull) k.dstate[a0 + lane] = make_double4(gm.h, lo, hi, (double)it);
            defer_members(dm, a0 + lane, k.dfr, k.st);
            ws.deferred += (uint32_t)popc64(dm);
            if (done) {
                k.g.h[gm.i] = gm.h;
                if (k.out.nngb) k.out.nngb[gm.i] = nn;
                if (k.out.iters) k.out.iters[gm.i] = it;
                if (k.out.converged) k.out.converged[gm.i] = conv ? 1 : 0;
            }
            ws.iters += (uint32_t)uni(wave_sum_i(done ? it : 0));
            ws.not_conv += (uint32_t)popc64(ballot(done && !conv));
        }
        // the r-th member that finished is streamed by wave r mod W (the
        // masks and the staged superset are complete since the last barrier)
        uint64_t rest = dn;
        for (int r = 0; rest; r++) {
            const int m = ctz64(rest);
            rest &= rest - 1ull;
            if (r % W != wv) continue;
            const int c = wrap ? dens_emit<KER, ACC, true>(k, S, gc, s, bx.L, wrap, gm, m, fifo)
                               : dens_emit<KER, ACC, false>(k, S, gc, s, bx.L, wrap, gm, m, fifo);
            ws.pairs += (unsigned long long)c;
        }
        __syncthreads();
        if (wv == 0 && done) dens_finish<KER>(k, gm.i, gm.h, S.fin[lane], S.fin[64 + lane]);
    }
    ws.flush(k.st);
    if (k.trace && threadIdx.x == 0) sched_mark(k.st, 0, t_start);
}

// One wave per member that left its group superset: a superset of its own
// (radius: the bracket's upper end, or 1.25 h while there is none), walked
// up to three times, and the h loop continued on it from where the group
// left it; only when that fails too does it walk once per h evaluation.
constexpr int SOLO_PER_CU = 5; // workgroups of k_dens_solo per CU
template <int KER, typename ACC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SOLO_PER_CU))) void k_dens_solo(DensK k)
{
    extern __shared__ __align__(16) char lds_raw[];
    const MemLds S = mem_carve(lds_raw, k.ga.T, true);
    const int D = uni((int)k.st->n_dfr);
    // the members cost from one superset pass to a walk per h evaluation:
    // taken one at a time from the per-XCD queues
    Queue dq = queue_open(k.st->qctr3, D, 1);
    WaveStats ws;
    for (int item = queue_next(dq); item >= 0; item = queue_next(dq)) {
        const int a = uni(k.dfr[item]);
        Member M = member(k.g, k.ga, k.ca, a);
        const double4 ds = k.dstate[a];
        double h = uni_d(ds.x), lo = uni_d(ds.y), hi = uni_d(ds.z);
        int it = uni((int)ds.w), nn = 0;
        bool conv = false, done = false, usable = false;
        for (int round = 0; round < 4; round++) {
            if (usable && iterate(k, M, S, h, lo, hi, it, nn, conv, ws)) {
                done = true;
                break;
            }
            if (round == 3) break;
            const double rad = hi < INFINITY ? hi : 1.25 * h;
            usable = own_superset(k, S, M, rad, ws);
            if (!usable) break;
        }
        if (!done) {
            dens_solo<KER, ACC>(k, S, M, h, lo, hi, it, ws);
            continue;
        }
        DensPair<KER, ACC> pp = dens_pair<KER, ACC>(k, M.xi, M.yi, M.zi, M.bx.L, h, true);
        Fifo q{(DEnt *)S.fifo, 0};
        stream_masks(k.ca.cand, M.s.c0, M.s.nc, S.masks, q, pp);
        dens_write<KER, ACC>(k, M.i, h, nn, it, conv, pp, ws);
    }
    ws.flush(k.st);
}

// ================================================================== hydro
struct HydroK {
    Geom g;
    GroupArg ga;
    CandArg ca;
    const float *m, *vx, *vy, *vz, *u, *rho, *fgrad;
    const float4 *pa;   // per particle: m, vx, vy, vz
    const float4 *pb;   // per particle: rho, f P / rho^2, sound speed, h
    const float4 *pos4; // per particle: FP32 x, y, z, h (walks, the filter's screen)
    const double4 *p64; // per particle: FP64 x, y, z, h (pair terms)
    const unsigned long long *drift; // reused supersets: largest displacement, h growth, or NULL
    const uint8_t *active;           // reused supersets: the members computed now
    const int32_t *sel;              // reused supersets: the members active now, or NULL
    int32_t *dfr;                    // members that walk alone (st->n_dfr of them)
    sfc_hydro_out out;
    DevStatus *st;
    double gamma, alpha;
    // production SPH: per particle (alpha_i, u, P) in pc, conduction, switch
    const float4 *pc;
    const float *alpha_i;
    double alpha_u, alpha_min, alpha_max, ell;
    int trace; // schedule statistics (DevStatus::sched)
};

namespace {
// PHYS 0: the standard force; 1: the production SPH (a per-particle
// viscosity coefficient, artificial conduction, the velocity divergence)
template <int KER, typename ACC, int PHYS = 0> struct HydroAcc {
    static constexpr int phys = PHYS;
    const HydroK *k;
    double xi, yi, zi, L;
    bool wrap;
    double h2;
    ACC hinv, hinv4, vx, vy, vz, rho, pf, cs;
    ACC al, ui, Pi; // production: alpha_i, u_i, P_i
    Kahan<ACC> ax, ay, az, du, dv;
    ACC vmax;
    struct Term {
        ACC ax, ay, az, du, vs, dv;
    };
    // the pair geometry from the neighbour's FP64 position and h: x_i - x_j
    // (the force direction) and r^2 in FP64 rounded once, and the FP64
    // differences h_i^2 - r^2, h_j^2 - r^2 rounded once (the kernel tails)
    struct Geo {
        ACC dx, dy, dz, r2, ti, tj;
    };
    __device__ __forceinline__ Geo geom(const double4 &pj) const
    {
        double dxd = xi - pj.x, dyd = yi - pj.y, dzd = zi - pj.z;
        if (wrap) {
            dxd = fold(dxd, L);
            dyd = fold(dyd, L);
            dzd = fold(dzd, L);
        }
        const double r2d = __builtin_fma(dzd, dzd, __builtin_fma(dyd, dyd, dxd * dxd));
        Geo g;
        g.dx = (ACC)dxd;
        g.dy = (ACC)dyd;
        g.dz = (ACC)dzd;
        g.r2 = (ACC)r2d;
        g.ti = (ACC)(h2 - r2d);
        g.tj = (ACC)(pj.w * pj.w - r2d);
        return g;
    }
    __device__ __forceinline__ Term make(int j, const double4 &pj) const { return make_g(j, geom(pj), pj.w); }
    // the pair term of neighbour j from its geometry (hj64: its FP64 h, read
    // by the FP64 variant only)
    __device__ __forceinline__ Term make_g(int j, const Geo &g, double hj64) const
    {
        constexpr ACC C = (ACC)knorm<KER>();
        const ACC dx = g.dx, dy = g.dy, dz = g.dz;
        ACC mj, vxj, vyj, vzj, rhoj, pfj, csj, hj;
        ACC alj = ACC(0), uj = ACC(0), Pj = ACC(0);
        if (sizeof(ACC) == 8) {
            double gm1 = k->gamma - 1.0;
            double ujd = k->u[j];
            rhoj = (ACC)k->rho[j];
            pfj = (ACC)(k->fgrad[j] * gm1 * ujd / (double)k->rho[j]);
            csj = (ACC)sqrt(k->gamma * gm1 * ujd);
            hj = (ACC)hj64;
            mj = (ACC)k->m[j];
            vxj = (ACC)k->vx[j];
            vyj = (ACC)k->vy[j];
            vzj = (ACC)k->vz[j];
            if (PHYS) {
                alj = (ACC)k->alpha_i[j];
                uj = (ACC)ujd;
                Pj = (ACC)(gm1 * (double)k->rho[j] * ujd);
            }
        } else {
            const float4 a = k->pa[j];
            const float4 b = k->pb[j];
            mj = (ACC)a.x;
            vxj = (ACC)a.y;
            vyj = (ACC)a.z;
            vzj = (ACC)a.w;
            rhoj = (ACC)b.x;
            pfj = (ACC)b.y;
            csj = (ACC)b.z;
            hj = (ACC)b.w;
            if (PHYS) {
                const float4 c = k->pc[j];
                alj = (ACC)c.x;
                uj = (ACC)c.y;
                Pj = (ACC)c.z;
            }
        }
        ACC r = acc_sqrt(g.r2);
        ACC rinv = r > ACC(0) ? acc_rcp(r) : ACC(0);
        const ACC qi = r * hinv;
        const ACC dwi = kern_deval_u<KER, ACC>(qi, tail_g<ACC>(g.ti, hinv * hinv, qi));
        ACC hjinv = acc_rcp(hj);
        const ACC qj = r * hjinv;
        const ACC dwj = kern_deval_u<KER, ACC>(qj, tail_g<ACC>(g.tj, hjinv * hjinv, qj));
        ACC hj2 = hjinv * hjinv;
        ACC dWi = C * dwi * hinv4;
        ACC dWj = C * dwj * (hj2 * hj2);
        ACC dWb = ACC(0.5) * (dWi + dWj);
        ACC vdx = vx - vxj, vdy = vy - vyj, vdz = vz - vzj;
        ACC vr = mad(vdz, dz, mad(vdy, dy, vdx * dx));
        ACC wij = vr < ACC(0) ? vr * rinv : ACC(0);
        ACC vsig = cs + csj - ACC(3) * wij;
        const ACC rr = acc_rcp(rho + rhoj); // 1 / (2 rho_ij)
        const ACC aij = PHYS ? ACC(0.5) * (al + alj) : (ACC)k->alpha;
        ACC visc = -aij * vsig * wij * rr;
        ACC fac = mj * (pf * dWi + pfj * dWj + visc * dWb);
        ACC fr = fac * rinv;
        Term t;
        t.ax = -fr * dx;
        t.ay = -fr * dy;
        t.az = -fr * dz;
        t.du = mj * (pf * dWi + ACC(0.5) * visc * dWb) * vr * rinv;
        t.vs = vsig;
        t.dv = ACC(0);
        if (PHYS) {
            // conduction at the signal speed sqrt(|P_i - P_j| / rho_ij)
            const ACC vu = acc_sqrt(fabs(Pi - Pj) * ACC(2) * rr);
            t.du += mj * (ACC)k->alpha_u * vu * (ui - uj) * dWb * ACC(2) * rr;
            t.dv = mj * vr * rinv * dWi;
        }
        return t;
    }
    __device__ __forceinline__ void add(const Term &t)
    {
        ax.add(t.ax);
        ay.add(t.ay);
        az.add(t.az);
        du.add(t.du);
        if (PHYS) dv.add(t.dv);
        vmax = t.vs > vmax ? t.vs : vmax;
    }
    __device__ __forceinline__ void init(const HydroK &kk, int i, double x, double y, double z,
                                         double Lb, double h, bool wr)
    {
        k = &kk;
        xi = x;
        yi = y;
        zi = z;
        L = Lb;
        wrap = wr;
        double hv = 1.0 / h;
        h2 = h * h;
        hinv = (ACC)hv;
        hinv4 = (ACC)(hv * hv * hv * hv);
        vx = (ACC)kk.vx[i];
        vy = (ACC)kk.vy[i];
        vz = (ACC)kk.vz[i];
        rho = (ACC)kk.rho[i];
        double gm1 = kk.gamma - 1.0;
        double u = kk.u[i];
        pf = (ACC)(kk.fgrad[i] * gm1 * u / (double)kk.rho[i]);
        cs = (ACC)sqrt(kk.gamma * gm1 * u);
        vmax = ACC(0);
        al = ui = Pi = ACC(0);
        if (PHYS) {
            al = (ACC)kk.alpha_i[i];
            ui = (ACC)u;
            Pi = (ACC)(gm1 * (double)kk.rho[i] * u);
        }
    }
};

// neighbours given by particle index
template <int KER, typename ACC, int PHYS = 0> struct HydroPair : HydroAcc<KER, ACC, PHYS> {
    using Term = typename HydroAcc<KER, ACC, PHYS>::Term;
    __device__ __forceinline__ Term term(const HEnt &e) const
    {
        return this->make(e.j, this->k->p64[e.j]);
    }
};


template <int KER, typename ACC, int PHYS>
__device__ __forceinline__ HydroPair<KER, ACC, PHYS> hydro_pair(const HydroK &k, int i, double xi,
                                                                double yi, double zi, double L,
                                                                double h, bool wrap)
{
    HydroPair<KER, ACC, PHYS> hp;
    hp.init(k, i, xi, yi, zi, L, h, wrap);
    return hp;
}

template <int KER, typename ACC, class P>
__device__ void hydro_write(const HydroK &k, int i, const P &hp)
{
    double ax = (double)wave_sum_f_or_d(hp.ax.value());
    double ay = (double)wave_sum_f_or_d(hp.ay.value());
    double az = (double)wave_sum_f_or_d(hp.az.value());
    double du = (double)wave_sum_f_or_d(hp.du.value());
    double dvs = 0.0;
    if (P::phys) dvs = (double)wave_sum_f_or_d(hp.dv.value());
    ACC vm = hp.vmax;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        ACC t = __shfl_xor(vm, o, 64);
        vm = t > vm ? t : vm;
    }
    if (lane_id() != 0) return;
    if (P::phys) {
        // the velocity divergence and the viscosity switch's rate
        const double divv = -dvs / (double)k.rho[i];
        const double al = (double)k.alpha_i[i];
        const double c = sqrt(k.gamma * (k.gamma - 1.0) * (double)k.u[i]);
        const double rate = -(al - k.alpha_min) * k.ell * c / k.g.h[i] +
                            (divv < 0.0 ? -divv : 0.0) * (k.alpha_max - al);
        if (k.out.divv) k.out.divv[i] = (float)divv;
        if (k.out.dalphadt) k.out.dalphadt[i] = (float)rate;
    }
    k.out.ax[i] = (float)ax;
    k.out.ay[i] = (float)ay;
    k.out.az[i] = (float)az;
    k.out.dudt[i] = (float)du;
    k.out.vsigmax[i] = (float)vm;
    if (k.out.ax64) k.out.ax64[i] = ax;
    if (k.out.ay64) k.out.ay64[i] = ay;
    if (k.out.az64) k.out.az64[i] = az;
    if (k.out.dudt64) k.out.dudt64[i] = du;
}

} // namespace

__global__ void k_dens_prep(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                            const double *__restrict__ z, const double *__restrict__ h,
                            const float *__restrict__ m, float4 *__restrict__ pos4,
                            double4 *__restrict__ p64, double4 *__restrict__ snap)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xi = x[i], yi = y[i], zi = z[i];
    pos4[i] = make_float4((float)xi, (float)yi, (float)zi, m[i]);
    p64[i] = make_double4(xi, yi, zi, (double)m[i]); // the mass in one block with x
    if (snap) snap[i] = make_double4(xi, yi, zi, 0.0);
}

// Drift since the snapshot of kept supersets: the largest displacement
// (minimum image in its box) and the largest growth of h, as the bit
// patterns of non-negative doubles (whose order is the numbers' order), and
// the number of active particles.  First per block into part[3 * block],
// then k_drift_final.
constexpr int DRIFT_BLOCKS = 512;
__global__ __launch_bounds__(256) void k_drift_part(int64_t n, int nb, const int64_t *__restrict__ box_off,
                                                    const double *__restrict__ box_L,
                                                    const double *__restrict__ x, const double *__restrict__ y,
                                                    const double *__restrict__ z, const double *__restrict__ h,
                                                    const uint8_t *__restrict__ active,
                                                    const double4 *__restrict__ snap,
                                                    unsigned long long *__restrict__ part)
{
    __shared__ unsigned long long red[3][256];
    unsigned long long dm = 0, hm = 0, na = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double L = box_L[nb > 1 ? box_of(box_off, nb, (int)i) : 0];
        const double4 s = snap[i];
        const double dx = fold(x[i] - s.x, L), dy = fold(y[i] - s.y, L), dz = fold(z[i] - s.z, L);
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        dm = max(dm, (unsigned long long)__double_as_longlong(d));
        if (h) hm = max(hm, (unsigned long long)__double_as_longlong(fmax(h[i] - s.w, 0.0)));
        na += active[i] != 0;
    }
    red[0][threadIdx.x] = dm;
    red[1][threadIdx.x] = hm;
    red[2][threadIdx.x] = na;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] = max(red[0][threadIdx.x], red[0][threadIdx.x + w]);
            red[1][threadIdx.x] = max(red[1][threadIdx.x], red[1][threadIdx.x + w]);
            red[2][threadIdx.x] += red[2][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 3) part[3 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_drift_final(const unsigned long long *__restrict__ part,
                                                     unsigned long long *__restrict__ out)
{
    __shared__ unsigned long long red[3][256];
    unsigned long long dm = 0, hm = 0, na = 0;
    for (int b = threadIdx.x; b < DRIFT_BLOCKS; b += 256) {
        dm = max(dm, part[3 * b]);
        hm = max(hm, part[3 * b + 1]);
        na += part[3 * b + 2];
    }
    red[0][threadIdx.x] = dm;
    red[1][threadIdx.x] = hm;
    red[2][threadIdx.x] = na;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] = max(red[0][threadIdx.x], red[0][threadIdx.x + w]);
            red[1][threadIdx.x] = max(red[1][threadIdx.x], red[1][threadIdx.x + w]);
            red[2][threadIdx.x] += red[2][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
}

// FP32 copies of x, y, z and h (the verify pass's walk)
__global__ void k_pos_h(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                        const double *__restrict__ z, const double *__restrict__ h,
                        float4 *__restrict__ pos4)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    pos4[i] = make_float4((float)x[i], (float)y[i], (float)z[i], (float)h[i]);
}

__global__ void k_hydro_prep(int64_t n, const float *__restrict__ m, const float *__restrict__ vx,
                             const float *__restrict__ vy, const float *__restrict__ vz,
                             const float *__restrict__ rho, const float *__restrict__ fgrad,
                             const float *__restrict__ u, const double *__restrict__ h,
                             const double *__restrict__ x, const double *__restrict__ y,
                             const double *__restrict__ z, double gamma, float4 *__restrict__ pa,
                             float4 *__restrict__ pb, float4 *__restrict__ pos4,
                             double4 *__restrict__ p64, double4 *__restrict__ snap,
                             const float *__restrict__ alpha_i, float4 *__restrict__ pc)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xi = x[i], yi = y[i], zi = z[i], hi = h[i];
    if (snap) snap[i] = make_double4(xi, yi, zi, hi);
    double gm1 = gamma - 1.0;
    double uu = u[i];
    pa[i] = make_float4(m[i], vx[i], vy[i], vz[i]);
    pos4[i] = make_float4((float)xi, (float)yi, (float)zi, (float)hi);
    p64[i] = make_double4(xi, yi, zi, hi);
    pb[i] = make_float4(rho[i], (float)(fgrad[i] * gm1 * uu / (double)rho[i]),
                        (float)sqrt(gamma * gm1 * uu), (float)hi);
    // production SPH: alpha_i, u_i, P_i
    if (alpha_i) pc[i] = make_float4(alpha_i[i], (float)uu, (float)(gm1 * (double)rho[i] * uu), 0.0f);
}


constexpr int HQB = 8; // members per take in the hydro member kernel's dynamic part

// Hydro, one wave per active particle: the group superset filtered to
// r < max(h_i, h_j), j != i, decided on the FP32 positions and h wherever
// that is safely away from the edge and by the FP64 test inside the band,
// the pairs streamed through the FIFO into the force sums.  Members the
// superset does not cover are listed for k_hydro_solo.
template <int KER, typename ACC, int PHYS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(ACC) == 4 ? 4 : 1))) void k_hmem(HydroK k)
{
    extern __shared__ __align__(16) char lds_raw[];
    const unsigned long long t_start = wall_clock64();
    HEnt *fifo = (HEnt *)(lds_raw + (size_t)uni((int)(threadIdx.x >> 6)) * FIFO_BYTES);
    const int lane = lane_id();
    // a reuse pass takes only the members active now (listed in sel)
    const int A = k.sel ? uni((int)k.drift[3]) : uni(*k.ga.n_act);
    // the first seven eighths in a static split (the waves of a workgroup
    // on consecutive members, which share a superset in the CU's L1), the
    // rest from the per-XCD queues, HQB members per take, so that the waves
    // that finish their share early absorb the spread of the others
    const int As = A - (A >> 3);
    const ItemRange ar = item_range(As);
    WaveStats ws;
    // reused supersets: the largest displacement and h growth since the walk
    const double dl = k.drift ? __longlong_as_double((long long)k.drift[0]) : 0.0;
    const double dh = k.drift ? __longlong_as_double((long long)k.drift[1]) : 0.0;
    auto one = [&](int item) {
        const int a = k.sel ? uni(k.sel[item]) : item;
        const Member M = member(k.g, k.ga, k.ca, a);
        if (k.active && !uni(k.active[M.i])) return; // reuse: the members active now
        const bool kept = !k.drift || (M.h + M.d + dl <= M.s.cov && M.d + dl + dh <= M.s.rs);
        if ((M.s.flags & GSUP_SOLO) || !kept) {
            ws.deferred++;
            if (lane == 0) k.dfr[atomicAdd(&k.st->n_dfr, 1ull)] = a;
            return;
        }
        const bool wrap = (M.s.flags & GSUP_WRAP) || k.drift;
        HydroPair<KER, ACC, PHYS> hp = hydro_pair<KER, ACC, PHYS>(k, M.i, M.xi, M.yi, M.zi, M.bx.L, M.h,
                                                                  wrap);
        FifoH q{fifo, 0};
        // the FP32 screen: coordinates off by at most 2^-24 L each, h by
        // 2^-24 h; near r = max(h_i, h_j) the FP32 r^2 is within
        // 2^-19 (L hm + hm^2) of the FP64 one
        const float xf = (float)M.xi, yf = (float)M.yi, zf = (float)M.zi, Lf = (float)M.bx.L,
                    hf = (float)M.h;
        const int nc = M.s.nc;
        const int nch = (nc + 63) >> 6;
        const int32_t *cg = k.ca.cand + M.s.c0;
        ws.tests += (unsigned)nc;
        int jn[UNR];
#pragma unroll
        for (int u = 0; u < UNR; u++) jn[u] = cg[min((u << 6) + lane, nc - 1)];
        for (int c0 = 0; c0 < nch; c0 += UNR) {
            int j[UNR];
            bool v[UNR];
#pragma unroll
            for (int u = 0; u < UNR; u++) {
                v[u] = ((c0 + u) << 6) + lane < nc;
                j[u] = jn[u];
            }
            float4 pj[UNR]; // x, y, z, h
#pragma unroll
            for (int u = 0; u < UNR; u++) pj[u] = k.pos4[j[u]];
#pragma unroll
            for (int u = 0; u < UNR; u++) jn[u] = cg[min(((c0 + UNR + u) << 6) + lane, nc - 1)];
#pragma unroll
            for (int u = 0; u < UNR; u++) {
                if (c0 + u >= nch) break;
                const float r2f = r2_f32(pj[u].x, pj[u].y, pj[u].z, xf, yf, zf, Lf, wrap);
                const float hmf = fmaxf(hf, pj[u].w);
                const float hm2f = hmf * hmf;
                const float E = 0x1p-19f * __builtin_fmaf(Lf, hmf, hm2f);
                bool hit = r2f < hm2f - E;
                const bool amb = v[u] && !hit && !(r2f > hm2f + E);
                if (ballot(amb)) { // inside the band: the FP64 test decides
                    if (amb) {
                        const int jj = j[u];
                        const double hm = fmax(M.h, k.g.h[jj]);
                        hit = r2_of(k.g.x[jj], k.g.y[jj], k.g.z[jj], M.xi, M.yi, M.zi, M.bx.L, wrap) <
                              hm * hm;
                    }
                }
                const bool pair = v[u] && j[u] != M.i && hit;
                ws.pairs += (unsigned)popc64(ballot(pair));
                q.push(pair, HEnt{j[u]}, hp);
            }
        }
        q.flush(hp);
        hydro_write<KER, ACC>(k, M.i, hp);
    };
    for (int item = ar.i; item < ar.end; item += ar.stride) one(item);
    Queue tq = queue_open(k.st->qctr2, A - As, HQB);
    for (int t = queue_next(tq); t >= 0; t = queue_next(tq)) one(As + t);
    ws.flush(k.st);
    if (k.trace && lane == 0) sched_mark(k.st, 1, t_start);
}

// The hydro members that their group's superset does not cover (their group
// kept none, or a reused one no longer covers them): one wave each walks the
// tree level by level and streams its pairs into the sums.
constexpr int HSOLO_WAVE_LDS = FIFO_BYTES + 4 * (2 * LCAP + 64);
template <int KER, typename ACC, int PHYS> __global__ __launch_bounds__(256) void k_hydro_solo(HydroK k)
{
    extern __shared__ __align__(16) char lds_raw[];
    const int wave = uni((int)(threadIdx.x >> 6));
    MemLds S;
    S.masks = nullptr;
    S.fifo = (void *)(lds_raw + (size_t)wave * HSOLO_WAVE_LDS);
    S.r2c = (float *)((char *)S.fifo + FIFO_BYTES);
    S.rc = 2 * LCAP + 64;
    const int D = uni((int)k.st->n_dfr);
    const ItemRange ar = item_range(D);
    WaveStats ws;
    for (int item = ar.i; item < ar.end; item += ar.stride) {
        const Member M = member(k.g, k.ga, k.ca, uni(k.dfr[item]));
        HydroPair<KER, ACC, PHYS> hp = hydro_pair<KER, ACC, PHYS>(k, M.i, M.xi, M.yi, M.zi, M.bx.L, M.h,
                                                                  true);
        StreamVisit<1, HydroPair<KER, ACC, PHYS>, FifoH> sv{k.g.x, k.g.y, k.g.z, k.g.h, M.xi, M.yi, M.zi,
                                               M.bx.L, M.h, M.i, FifoH{(HEnt *)S.fifo, 0}, &hp};
        Ball B{M.xi, M.yi, M.zi, M.bx.L, 0.0, 0.0, M.h, 1};
        solo_walk(k.g, S, M, B, sv, k.st);
        ws.walks++;
        sv.q.flush(hp);
        hydro_write<KER, ACC>(k, M.i, hp);
    }
    ws.flush(k.st);
}

// ================================================================== verify
struct VerK {
    Geom g;
    GroupArg ga;
    CandArg ca;
    sfc_verify ver;
    const uint32_t *orig;
    DevStatus *st;
};

namespace {
struct VerifyAcc {
    const VerK *k;
    int64_t w1; // end of this particle's list window
    int64_t pos;
    uint64_t fp;
    int cnt;
    bool over;
    __device__ void operator()(int j, bool valid)
    {
        const uint64_t m = ballot(valid);
        if (valid) {
            fp += mix64((uint64_t)(k->orig ? k->orig[j] : (uint32_t)j));
            if (k->ver.list) {
                int64_t at = pos + mbcnt(m);
                if (at < w1 && at < k->ver.list_cap) k->ver.list[at] = j;
                else over = true;
            }
        }
        pos += popc64(m);
        cnt += popc64(m);
    }
};

__device__ __forceinline__ VerifyAcc verify_init(const VerK &k, int i)
{
    VerifyAcc va;
    va.k = &k;
    va.pos = k.ver.list ? k.ver.list_off[i] : 0;
    va.w1 = k.ver.list ? k.ver.list_off[i + 1] : 0;
    va.fp = 0ull;
    va.cnt = 0;
    va.over = false;
    return va;
}

__device__ void verify_write(const VerK &k, int i, VerifyAcc &va)
{
    uint64_t fp = wave_sum_u64(va.fp);
    bool over = ballot(va.over) != 0ull;
    if (lane_id() != 0) return;
    k.ver.count[i] = va.cnt;
    if (k.ver.fingerprint) k.ver.fingerprint[i] = fp;
    if (over || (k.ver.list && va.pos != va.w1)) atomicOr(&k.st->flags, (unsigned)SFC_ST_LIST_OVERFLOW);
}

struct VerVisit {
    static constexpr int EB = 2; // leaf batches in flight (emit_leaves)
    const double *x, *y, *z, *h;
    double xi, yi, zi, L, hi;
    int i, mode;
    VerifyAcc *va;
    __device__ bool stop() const { return false; }
    __device__ __forceinline__ Pos fetch(int j) const
    {
        Pos p;
        p.x = x[j];
        p.y = y[j];
        p.z = z[j];
        p.h = h[j];
        return p;
    }
    __device__ void take(int j, bool valid, const Pos &p)
    {
        bool hit = false;
        if (valid) {
            double r2 = r2_of(p.x, p.y, p.z, xi, yi, zi, L, true);
            if (mode == 0) {
                hit = r2 < hi * hi;
            } else {
                double hm = fmax(hi, p.h);
                hit = (j != i) && (r2 < hm * hm);
            }
        }
        (*va)(j, hit);
    }
};
} // namespace

// One wave per active particle: its neighbour set from the group superset
// (count, fingerprint, optional list in ascending order).
__global__ __launch_bounds__(256) void k_verify(VerK k)
{
    extern __shared__ __align__(16) char lds_raw[];
    const MemLds S = mem_carve(lds_raw, k.ga.T, false);
    const int lane = lane_id();
    const int mode = k.ver.mode;
    const int A = uni(*k.ga.n_act);
    const ItemRange ar = item_range(A);
    for (int a = ar.i; a < ar.end; a += ar.stride) {
        const Member M = member(k.g, k.ga, k.ca, a);
        VerifyAcc va = verify_init(k, M.i);
        if (M.s.flags & GSUP_SOLO) {
            VerVisit vv{k.g.x, k.g.y, k.g.z, k.g.h, M.xi, M.yi, M.zi, M.bx.L, M.h, M.i, mode, &va};
            Ball B = mode == 0 ? Ball{M.xi, M.yi, M.zi, M.bx.L, sq(M.h * INFL), 0.0, 0.0, 0}
                               : Ball{M.xi, M.yi, M.zi, M.bx.L, 0.0, 0.0, M.h, 1};
            walk(k.g, M.bx.root, M.bx.root_end, B, vv, k.st);
            verify_write(k, M.i, va);
            continue;
        }
        const bool wrap = (M.s.flags & GSUP_WRAP) != 0;
        const int nc = M.s.nc;
        const int nch = (nc + 63) >> 6;
        const int32_t *cg = k.ca.cand + M.s.c0;
        for (int ch = 0; ch < nch; ch++) {
            const int slot = (ch << 6) + lane;
            const bool v = slot < nc;
            const int j = cg[min(slot, nc - 1)];
            const double r2 = r2_of(k.g.x[j], k.g.y[j], k.g.z[j], M.xi, M.yi, M.zi, M.bx.L, wrap);
            bool hit;
            if (mode == 0) {
                hit = r2 < M.h * M.h;
            } else {
                const double hm = fmax(M.h, k.g.h[j]);
                hit = j != M.i && r2 < hm * hm;
            }
            va(j, v && hit);
        }
        verify_write(k, M.i, va);
    }
}

// ================================================================== launchers
namespace {
Geom make_geom(const PartDev &p, const TreeDev &t)
{
    Geom g;
    g.x = p.x;
    g.y = p.y;
    g.z = p.z;
    g.h = p.h;
    g.box_off = p.box_off;
    g.box_L = p.box_L;
    g.info = t.info;
    g.lo = t.lo;
    g.hi = t.hi;
    g.box32 = t.box32;
    g.krec = t.krec;
    g.kids = t.kids;
    g.nchild = t.nchild;
    g.box_root = t.box_root;
    g.nb = p.nb;
    return g;
}

GroupArg make_groups(const GroupBufs &gb, int T)
{
    GroupArg a;
    a.act = gb.act;
    a.goff = gb.goff;
    a.n_groups = gb.n_groups;
    a.n_act = gb.n_act;
    a.box_T = gb.box_T;
    a.T = T;
    return a;
}

CandArg make_cand(const SearchBufs &sb)
{
    CandArg c;
    c.cand = sb.cand;
    c.cap = sb.cand_cap;
    c.sup = sb.sup;
    c.grp = sb.grp;
    return c;
}

template <class Kern> hipError_t allow_lds(Kern kern, size_t lds)
{
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// persistent grid: as many workgroups as fit on the chip at once (a multiple
// of 8), so that every wave is resident and keeps its XCD's items
template <class Kern>
unsigned grid_size(Kern kern, int threads, size_t lds, int cu, int64_t max_items)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 2;
    int64_t w = (int64_t)cu * per_cu;
    const int64_t need = (max_items + threads / 64 - 1) / (threads / 64);
    const int64_t cap = ((need + 7) / 8) * 8;
    if (cap < w) w = cap;
    w = (w / 8) * 8;
    return (unsigned)(w < 8 ? 8 : w);
}

template <class Kern, class Arg>
hipError_t launch_persistent(Kern kern, hipStream_t s, const Arg &a, int threads, size_t lds, int cu,
                             int64_t max_items)
{
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    kern<<<grid_size(kern, threads, lds, cu, max_items), threads, lds, s>>>(a);
    return hipGetLastError();
}

constexpr int MEM_WAVES = 4; // member waves per workgroup of the solo kernels

hipError_t launch_walk(hipStream_t s, const PartDev &p, const TreeDev &t, const GroupBufs &g,
                       SearchBufs &sb, DevStatus *st, int T, double skin, int hydro)
{
    k_reset_pass<<<1, 64, 0, s>>>(st, hydro);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    WalkK k;
    memset(&k, 0, sizeof(k));
    k.g = make_geom(p, t);
    k.ga = make_groups(g, T);
    k.ca = make_cand(sb);
    k.st = st;
    k.pos4 = sb.pos4;
    k.skin = skin;
    k.hydro = hydro;
    const size_t lds = (size_t)4 * (2 * LCAP + 64);
    // every wave that takes a group first takes a chunk of at least T slots
    // of the buffer: no more waves than half the buffer has chunks for
    const int64_t waves = min(p.n, max((int64_t)8, sb.cand_cap / (2 * (int64_t)T)));
    return launch_persistent(k_walk, s, k, 64, lds, sb.cu_count, waves);
}

// the drift bounds of kept supersets and the active count into
// sb.drift[0..2] (h: NULL for none); the members active now into sb.sel,
// their count into sb.drift[3]
hipError_t launch_drift(hipStream_t s, const PartDev &p, const double *h, const GroupBufs &g,
                        const SearchBufs &sb)
{
    k_drift_part<<<DRIFT_BLOCKS, 256, 0, s>>>(p.n, p.nb, p.box_off, p.box_L, p.x, p.y, p.z, h,
                                              p.active, sb.snap, sb.drift + 4);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_drift_final<<<1, 256, 0, s>>>(sb.drift + 4, sb.drift);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_fill_i32(s, (int32_t *)(sb.drift + 3), 0, 2)) != hipSuccess) return e;
    const int64_t wg = (p.n + 256 * SEL_CH - 1) / (256 * SEL_CH);
    k_sel_members<<<(unsigned)(wg < 4096 ? wg : 4096), 256, 0, s>>>(g.n_act, g.act, p.active, sb.sel,
                                                                   sb.drift + 3);
    return hipGetLastError();
}

// The density pass: the walk of the groups, k_dgrp (the h loop and the sums
// of every group's members on its superset, one workgroup per group) and
// k_dens_solo (the members that left their group superset).  Each wave of
// k_dens_solo owns a private slot of T candidates at the end of the
// candidate buffer (when the slots take at most half of it); the group
// supersets use the rest.
template <int KER, typename ACC>
hipError_t run_density(hipStream_t s, const PartDev &p, const TreeDev &t, const GroupBufs &g,
                       const SearchBufs &sb, const DensityArgs &a, DevStatus *st)
{
    const sfc_density_params &dp = a.dp;
    const int T = dp.t_cand;
    auto ks = k_dens_solo<KER, ACC>;
    const size_t lds_s = MEM_WAVES * mem_lds_bytes(T, true);
    hipError_t e = allow_lds(ks, lds_s);
    if (e != hipSuccess) return e;
    // the members that leave their group walk the tree alone, latency
    // bound: SOLO_PER_CU workgroups per CU (five waves per SIMD, as many as
    // fit its registers without spills), each wave
    // with a private slot; fewer workgroups when the slots would take more
    // than half the buffer, and SOLO_PER_CU without slots when not even one
    // per CU fits
    int per_cu = SOLO_PER_CU;
    while (per_cu > 1 && (int64_t)per_cu * sb.cu_count * MEM_WAVES * T > sb.cand_cap / 2) per_cu--;
    unsigned grid_s = (unsigned)((per_cu * sb.cu_count + 7) / 8 * 8);
    int64_t priv = (int64_t)grid_s * MEM_WAVES * T;
    if (priv > sb.cand_cap / 2) {
        grid_s = (unsigned)((SOLO_PER_CU * sb.cu_count + 7) / 8 * 8);
        priv = sb.cand_cap; // no private slots
    }
    SearchBufs gs = sb;
    if (priv <= sb.cand_cap / 2) gs.cand_cap = sb.cand_cap - priv;
    // small neighbour counts give small supersets (about (1 + f)^3 N_ngb, a
    // few N_ngb): then two waves per group and at most 512 staged candidates
    // (19 KB of LDS), so that eight groups share a CU; the rest of a larger
    // superset is read from global memory
    const bool small = 4 * dp.n_ngb <= GC_SMALL;
    const int C = min(T, small ? GC_SMALL : GC_MAX);
    auto kg = small ? k_dgrp<KER, ACC, 2> : k_dgrp<KER, ACC, GW>;
    const int wgt = 64 * (small ? 2 : GW);
    const size_t lds_g = glds_bytes(C, small ? 2 : GW);
    if ((e = allow_lds(kg, lds_g)) != hipSuccess) return e;
    const unsigned units = grid_size(kg, wgt, lds_g, sb.cu_count, p.n * (wgt / 64));
    k_dens_prep<<<(unsigned)((p.n + 255) / 256), 256, 0, s>>>(p.n, p.x, p.y, p.z, p.h, p.m, sb.pos4,
                                                              sb.p64, a.keep ? sb.snap : nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (dp.reuse) {
        // the kept supersets: the walk is skipped, the drift bounds them
        k_reset_pass<<<1, 64, 0, s>>>(st, 0);
        e = launch_drift(s, p, nullptr, g, sb);
        // the groups holding a member active now
        if (e == hipSuccess) e = launch_fill_i32(s, sb.gmark, 0, p.n);
        if (e == hipSuccess) {
            k_gmark<<<1024, 256, 0, s>>>(sb.sel, sb.drift + 3, gs.grp, sb.gmark);
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            const int64_t wg = (p.n + 256 * SEL_CH - 1) / (256 * SEL_CH);
            k_glist<<<(unsigned)(wg < 4096 ? wg : 4096), 256, 0, s>>>(g.n_groups, sb.gmark, sb.glist,
                                                                     &st->n_glist);
            e = hipGetLastError();
        }
    } else {
        e = launch_walk(s, p, t, g, gs, st, T, dp.skin, 0);
        // every group; the heavy ones of an eighth first
        const unsigned go_grid = (unsigned)(8 * (((p.n + 7) / 8 + GO_CH - 1) / GO_CH));
        if (e == hipSuccess) {
            const GroupArg ga = make_groups(g, T);
            k_gcount<<<go_grid, 256, 0, s>>>(ga, gs.sup, (int)units, st);
            k_gorder<<<go_grid, 256, 0, s>>>(ga, gs.sup, (int)units, sb.glist, st);
            e = hipGetLastError();
        }
    }
    if (e != hipSuccess) return e;
    DensK k;
    memset(&k, 0, sizeof(k));
    k.g = make_geom(p, t);
    k.ga = make_groups(g, T);
    k.ca = make_cand(gs);
    k.priv = gs.cand_cap < sb.cand_cap ? gs.cand_cap : -1;
    k.pos4 = sb.pos4;
    k.p64 = sb.p64;
    k.m = p.m;
    k.rho = p.rho;
    k.fgrad = p.fgrad;
    k.out = a.out;
    k.st = st;
    k.n_ngb = dp.n_ngb;
    k.dn = dp.dn;
    k.max_iter = dp.max_iter;
    k.fixed_h = dp.fixed_h;
    k.trace = a.trace ? 1 : 0;
    k.C = C;
    k.drift = dp.reuse ? sb.drift : nullptr;
    k.active = dp.reuse ? p.active : nullptr;
    k.glist = dp.reuse ? sb.glist : nullptr;
    k.gord = dp.reuse ? nullptr : sb.glist;
    k.dfr = sb.dfr;
    k.dstate = sb.dstate;
    kg<<<units, wgt, lds_g, s>>>(k);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    ks<<<grid_s, 64 * MEM_WAVES, lds_s, s>>>(k);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (!dp.reuse) return hipSuccess;
    k_reuse_check<<<1, 64, 0, s>>>(sb.drift, st);
    return hipGetLastError();
}

template <int KER, typename ACC, int PHYS>
hipError_t run_hydro(hipStream_t s, const HydroK &k, const SearchBufs &sb, int64_t n)
{
    const size_t lds_s = (size_t)MEM_WAVES * HSOLO_WAVE_LDS;
    hipError_t e = launch_persistent(k_hmem<KER, ACC, PHYS>, s, k, 256, (size_t)MEM_WAVES * FIFO_BYTES,
                                     sb.cu_count, n);
    if (e == hipSuccess)
        e = launch_persistent(k_hydro_solo<KER, ACC, PHYS>, s, k, 64 * MEM_WAVES, lds_s, sb.cu_count,
                              n);
    return e;
}
} // namespace

hipError_t launch_density(hipStream_t s, const PartDev &p, const TreeDev &t, const GroupBufs &g,
                          SearchBufs &sb, const DensityArgs &a, DevStatus *st)
{
    const sfc_density_params &dp = a.dp;
    if (dp.kernel == 0 && dp.accum == SFC_ACCUM_F32) return run_density<0, float>(s, p, t, g, sb, a, st);
    if (dp.kernel == 0) return run_density<0, double>(s, p, t, g, sb, a, st);
    if (dp.accum == SFC_ACCUM_F32) return run_density<1, float>(s, p, t, g, sb, a, st);
    return run_density<1, double>(s, p, t, g, sb, a, st);
}

hipError_t launch_hydro(hipStream_t s, const PartDev &p, const TreeDev &t, const GroupBufs &g,
                        SearchBufs &sb, const HydroArgs &a, DevStatus *st)
{
    const sfc_hydro_params &hp = a.hp;
    k_hydro_prep<<<(unsigned)((p.n + 255) / 256), 256, 0, s>>>(p.n, p.m, p.vx, p.vy, p.vz, p.rho,
                                                               p.fgrad, p.u, p.h, p.x, p.y, p.z,
                                                               hp.gamma, sb.pa, sb.pb, sb.pos4,
                                                               sb.p64, a.keep ? sb.snap : nullptr,
                                                               hp.physics == SFC_HYDRO_PRODUCTION
                                                                   ? hp.alpha_i
                                                                   : nullptr,
                                                               sb.pc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (hp.reuse) {
        k_reset_pass<<<1, 64, 0, s>>>(st, 1);
        e = launch_drift(s, p, p.h, g, sb);
    } else {
        e = launch_walk(s, p, t, g, sb, st, hp.t_cand, hp.skin, 1);
    }
    if (e != hipSuccess) return e;
    HydroK k;
    memset(&k, 0, sizeof(k));
    k.g = make_geom(p, t);
    k.ga = make_groups(g, hp.t_cand);
    k.ca = make_cand(sb);
    k.m = p.m;
    k.vx = p.vx;
    k.vy = p.vy;
    k.vz = p.vz;
    k.u = p.u;
    k.rho = p.rho;
    k.fgrad = p.fgrad;
    k.pa = sb.pa;
    k.pb = sb.pb;
    k.pos4 = sb.pos4;
    k.p64 = sb.p64;
    k.out = a.out;
    k.st = st;
    k.gamma = hp.gamma;
    k.alpha = hp.alpha;
    k.trace = a.trace ? 1 : 0;
    k.pc = sb.pc;
    k.alpha_i = hp.alpha_i;
    k.alpha_u = hp.alpha_u;
    k.alpha_min = hp.alpha_min;
    k.alpha_max = hp.alpha_max;
    k.ell = hp.ell;
    k.drift = hp.reuse ? sb.drift : nullptr;
    k.active = hp.reuse ? p.active : nullptr;
    k.sel = hp.reuse ? sb.sel : nullptr;
    k.dfr = sb.dfr;
    const int64_t n = p.n;
    const bool f32 = hp.accum == SFC_ACCUM_F32;
    if (hp.physics == SFC_HYDRO_PRODUCTION) {
        if (hp.kernel == 0) e = f32 ? run_hydro<0, float, 1>(s, k, sb, n) : run_hydro<0, double, 1>(s, k, sb, n);
        else e = f32 ? run_hydro<1, float, 1>(s, k, sb, n) : run_hydro<1, double, 1>(s, k, sb, n);
    } else {
        if (hp.kernel == 0) e = f32 ? run_hydro<0, float, 0>(s, k, sb, n) : run_hydro<0, double, 0>(s, k, sb, n);
        else e = f32 ? run_hydro<1, float, 0>(s, k, sb, n) : run_hydro<1, double, 0>(s, k, sb, n);
    }
    if (e != hipSuccess || !hp.reuse) return e;
    k_reuse_check<<<1, 64, 0, s>>>(sb.drift, st);
    return hipGetLastError();
}

hipError_t launch_verify(hipStream_t s, const PartDev &p, const TreeDev &t, const GroupBufs &g,
                         SearchBufs &sb, const sfc_verify &v, int t_cand, DevStatus *st)
{
    // the walk tests FP32 copies of x, y, z and h
    k_pos_h<<<(unsigned)((p.n + 255) / 256), 256, 0, s>>>(p.n, p.x, p.y, p.z, p.h, sb.pos4);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_walk(s, p, t, g, sb, st, t_cand, 1.0, v.mode == 1 ? 1 : 0);
    if (e != hipSuccess) return e;
    VerK k;
    memset(&k, 0, sizeof(k));
    k.g = make_geom(p, t);
    k.ga = make_groups(g, t_cand);
    k.ca = make_cand(sb);
    k.ver = v;
    k.orig = p.orig;
    k.st = st;
    return launch_persistent(k_verify, s, k, 64 * MEM_WAVES, MEM_WAVES * mem_lds_bytes(t_cand, false),
                             sb.cu_count, p.n);
}
