// tree.hip -- octree over Hilbert-sorted particles.
//
// Node = non-empty Hilbert cell.  With keys sorted, the cell of level l that
// holds particle i starts where the level-l key prefix changes.  Two
// per-particle numbers give the whole tree without recursion:
//   lcp(i)  levels shared by key[i-1] and key[i] (-1 at a box start): the
//           cells starting at i are those of level > lcp(i);
//   d(i)    deepest level whose cell around i holds more than n_leaf
//           particles = max over the windows [s, s+n_leaf] that contain i of
//           the levels shared by key[s] and key[s+n_leaf].
// Nodes starting at i are the levels lcp(i)+1 .. min(21, d(i)+1); the last
// one is a leaf.  Emitting them for every i in order, levels ascending, is a
// depth-first pre-order of the octree, so an exclusive scan of the counts
// numbers the nodes, a node's first child is the next node and its skip link
// is the first node starting at the end of its cell.  Bounding boxes and
// max(h) are reduced from the leaves (one launch over all of them) to the
// root, three levels per launch.
#include "internal.h"

__device__ __forceinline__ int common_levels(uint64_t a, uint64_t b)
{
    uint64_t x = a ^ b;
    if (x == 0) return SFC_KEY_BITS;
    return (__builtin_clzll(x) - 1) / 3; // bit 63 is always clear
}

__global__ void k_tree_prefix(int64_t n, int nb, const int64_t *__restrict__ box_off,
                              const uint64_t *__restrict__ key, int n_leaf,
                              int8_t *__restrict__ lcp, int8_t *__restrict__ cwin)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = nb > 1 ? box_of(box_off, nb, i) : 0;
    int64_t bs = box_off[b], be = box_off[b + 1];
    uint64_t k = key[i];
    lcp[i] = (int8_t)(i == bs ? -1 : common_levels(key[i - 1], k));
    cwin[i] = (int8_t)(i + n_leaf < be ? common_levels(k, key[i + n_leaf]) : -1);
}

__global__ void k_tree_count(int64_t n, int nb, const int64_t *__restrict__ box_off,
                             int n_leaf, const int8_t *__restrict__ lcp,
                             const int8_t *__restrict__ cwin, int8_t *__restrict__ dlev,
                             uint32_t *__restrict__ cnt)
{
    // the block's windows reach n_leaf entries back: stage them in LDS
    extern __shared__ int8_t win[]; // [blockDim.x + n_leaf]
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t w0 = i0 - n_leaf > 0 ? i0 - n_leaf : 0;
    const int64_t w1 = i0 + blockDim.x < n ? i0 + blockDim.x : n;
    for (int64_t s = w0 + threadIdx.x; s < w1; s += blockDim.x) win[s - w0] = cwin[s];
    __syncthreads();
    int64_t i = i0 + threadIdx.x;
    if (i > n) return;
    if (i == n) {
        cnt[n] = 0;
        return;
    }
    int b = nb > 1 ? box_of(box_off, nb, i) : 0;
    int64_t bs = box_off[b];
    int64_t s0 = i - n_leaf > bs ? i - n_leaf : bs;
    int d = -1;
    for (int64_t s = s0; s <= i; s++) d = max(d, (int)win[s - w0]);
    dlev[i] = (int8_t)d;
    int lo = lcp[i] + 1;
    int hi = min(SFC_KEY_BITS, d + 1);
    cnt[i] = hi >= lo ? (uint32_t)(hi - lo + 1) : 0u;
}

// first index in (i, be) whose key differs from key[i] above bit `sh`
__device__ __forceinline__ int64_t cell_end(const uint64_t *key, int64_t i, int64_t be, int sh)
{
    uint64_t pref = key[i] >> sh;
    int64_t good = i, step = 1, probe = i + 1;
    while (probe < be && (key[probe] >> sh) == pref) {
        good = probe;
        step <<= 1;
        probe = i + step;
    }
    int64_t bad = probe < be ? probe : be; // key[bad] differs or bad == be
    while (bad - good > 1) {
        int64_t mid = good + ((bad - good) >> 1);
        if ((key[mid] >> sh) == pref) good = mid; else bad = mid;
    }
    return bad;
}

__global__ void k_tree_emit(int64_t n, int nb, const int64_t *__restrict__ box_off,
                            const uint64_t *__restrict__ key, const int8_t *__restrict__ lcp,
                            const int8_t *__restrict__ dlev, const uint32_t *__restrict__ start,
                            TreeDev t, DevStatus *st)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = lcp[i] + 1;
    int hi = min(SFC_KEY_BITS, (int)dlev[i] + 1);
    if (hi < lo) return;
    int b = nb > 1 ? box_of(box_off, nb, i) : 0;
    int64_t bs = box_off[b], be = box_off[b + 1];
    uint32_t base = start[i];
    for (int l = lo; l <= hi; l++) {
        int64_t id = (int64_t)base + (l - lo);
        if (id >= t.capacity) {
            atomicOr(&st->flags, SFC_ST_NODE_OVERFLOW);
            return;
        }
        int sh = 3 * (SFC_KEY_BITS - l);
        int64_t end = l == 0 ? be : cell_end(key, i, be, sh);
        int leaf = l == hi;
        int4 inf;
        inf.x = (int)i;
        inf.y = (int)(end - i);
        inf.z = (int)start[end];
        inf.w = l | (leaf << 8);
        t.info[id] = inf;
    }
}

__global__ void k_tree_roots(int nb, const int64_t *__restrict__ box_off,
                             const uint32_t *__restrict__ start, int32_t *__restrict__ box_root,
                             DevStatus *st, int64_t n)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b <= nb) box_root[b] = (int32_t)start[box_off[b]];
    if (b == 0) st->n_nodes = (int32_t)start[n];
}

// child count and child table of node id (children follow each other by
// skip links: the first is id + 1, the next one starts where a subtree ends)
__device__ __forceinline__ void tree_children(const TreeDev &t, int id, int nn)
{
    int4 inf = t.info[id];
    int k = 0;
    int kid[8];
#pragma unroll
    for (int s = 0; s < 8; s++) kid[s] = -1;
    if (!(inf.w >> 8)) {
        int c = id + 1;
        int end = min(inf.z, nn);
        while (c < end && k < 8) { // the children follow each other by skip links
            kid[k] = c;
            k++;
            c = t.info[c].z;
        }
    }
    t.nchild[id] = k;
    int4 *kp = (int4 *)(t.kids + 8 * (int64_t)id);
    kp[0] = make_int4(kid[0], kid[1], kid[2], kid[3]);
    kp[1] = make_int4(kid[4], kid[5], kid[6], kid[7]);
}

__global__ void k_tree_nchild(const TreeDev t, const DevStatus *st)
{
    const int nn = min(st->n_nodes, t.capacity);
    const int stride = gridDim.x * blockDim.x;
    for (int id = blockIdx.x * blockDim.x + threadIdx.x; id < nn; id += stride)
        tree_children(t, id, nn);
}


// min / max over aligned groups of W lanes (W a power of two; the lanes of a
// group are those that differ in the low log2(W) bits)
template <int LO, int HI> __device__ __forceinline__ double xmin(double v)
{
#pragma unroll
    for (int o = LO; o < HI; o <<= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}
template <int LO, int HI> __device__ __forceinline__ double xmax(double v)
{
#pragma unroll
    for (int o = LO; o < HI; o <<= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

struct NodeBox {
    double lx, ly, lz, hx, hy, hz, hm;
};
__device__ __forceinline__ NodeBox box_empty()
{
    return NodeBox{INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
}
__device__ __forceinline__ void box_add(NodeBox &b, const double4 &lo, const double4 &hi, bool bbox)
{
    b.hm = fmax(b.hm, lo.w);
    if (bbox) {
        b.lx = fmin(b.lx, lo.x); b.ly = fmin(b.ly, lo.y); b.lz = fmin(b.lz, lo.z);
        b.hx = fmax(b.hx, hi.x); b.hy = fmax(b.hy, hi.y); b.hz = fmax(b.hz, hi.z);
    }
}
template <int LO, int HI> __device__ __forceinline__ void box_reduce(NodeBox &b, bool bbox)
{
    b.hm = xmax<LO, HI>(b.hm);
    if (bbox) {
        b.lx = xmin<LO, HI>(b.lx); b.ly = xmin<LO, HI>(b.ly); b.lz = xmin<LO, HI>(b.lz);
        b.hx = xmax<LO, HI>(b.hx); b.hy = xmax<LO, HI>(b.hy); b.hz = xmax<LO, HI>(b.hz);
    }
}
__device__ __forceinline__ void box_store(const TreeDev &t, int id, const NodeBox &b, bool bbox)
{
    if (bbox) {
        t.lo[id] = make_double4(b.lx, b.ly, b.lz, b.hm);
        t.hi[id] = make_double4(b.hx, b.hy, b.hz, 0.0);
        t.box32[2 * (int64_t)id] = make_float4(__double2float_rd(b.lx), __double2float_rd(b.ly),
                                               __double2float_rd(b.lz), __double2float_ru(b.hm));
        t.box32[2 * (int64_t)id + 1] = make_float4(__double2float_ru(b.hx), __double2float_ru(b.hy),
                                                   __double2float_ru(b.hz), 0.0f);
    } else {
        t.lo[id].w = b.hm;
        t.box32[2 * (int64_t)id].w = __double2float_ru(b.hm);
    }
}

// Leaves: a group of eight lanes per node id (grid-stride); a leaf's group
// strides through its particles, eight at a time.
__global__ void k_tree_leaves(const PartDev p, const TreeDev t, const DevStatus *st_in,
                              DevStatus *st, int with_bbox)
{
    const int nn = min(st_in->n_nodes, t.capacity);
    const int lane = lane_id();
    const int sub = lane & 7;
    const bool bbox = with_bbox != 0;
    const int ng = (int)(gridDim.x * blockDim.x) >> 3;
    // every lane runs the same number of rounds, so the group reductions
    // below always see all their lanes active
    const int rounds = (nn + ng - 1) / ng;
    int id = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 3);
    for (int r = 0; r < rounds; r++, id += ng) {
        const int4 inf = id < nn ? t.info[id] : make_int4(0, 0, 0, 0);
        const bool leaf = id < nn && (inf.w >> 8);
        const int first = inf.x, cnt = leaf ? inf.y : 0;
        const int b = p.nb > 1 && leaf ? box_of(p.box_off, p.nb, first) : 0;
        const double L = p.box_L[b];
        NodeBox bx = box_empty();
        bool bad = false;
        for (int i = first + sub; i < first + cnt; i += 8) {
            const double hh = p.h[i];
            bx.hm = fmax(bx.hm, hh);
            bad |= !(hh > 0.0);
            if (bbox) {
                const double x = p.x[i], y = p.y[i], z = p.z[i];
                bx.lx = fmin(bx.lx, x); bx.hx = fmax(bx.hx, x);
                bx.ly = fmin(bx.ly, y); bx.hy = fmax(bx.hy, y);
                bx.lz = fmin(bx.lz, z); bx.hz = fmax(bx.hz, z);
                bad |= !(x >= 0.0 && x < L && y >= 0.0 && y < L && z >= 0.0 && z < L);
            }
        }
        if (ballot(bad) != 0ull && lane == 0) atomicOr(&st->flags, SFC_ST_BAD_INPUT);
        box_reduce<1, 8>(bx, bbox);
        if (sub == 0 && leaf) box_store(t, id, bx, bbox);
    }
}

// Internal nodes of `level` together with their children and grandchildren:
// one wave per node, lane 8c + g holding grandchild g of child c.  A
// grandchild that is internal reduces its own children (level + 3: leaves, or
// done by the launch before), a child reduces its eight lanes, the node its
// eight children.  Launches go from level 18 up to 0 in steps of three.
__global__ void k_tree_up3(const TreeDev t, const DevStatus *st_in, int with_bbox, int level)
{
    const int nn = min(st_in->n_nodes, t.capacity);
    const int lane = lane_id();
    const bool bbox = with_bbox != 0;
    const int c = lane >> 3, g = lane & 7;
    const int nw = (int)(gridDim.x * blockDim.x) >> 6;
    for (int base = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64; base < nn;
         base += nw * 64) {
        const int id = base + lane;
        const int4 inf = id < nn ? t.info[id] : make_int4(0, 0, 0, 0);
        uint64_t m = ballot(id < nn && !(inf.w >> 8) && (inf.w & 255) == level);
        while (m) {
            const int s = ctz64(m);
            m &= m - 1;
            const int nd = base + s;
            const int ch = t.kids[8 * (int64_t)nd + c];
            const bool ch_ok = ch >= 0 && ch < nn;
            const bool ch_leaf = ch_ok && (t.info[ch].w >> 8);
            NodeBox bx = box_empty();
            if (ch_ok && ch_leaf) {
                if (g == 0) box_add(bx, t.lo[ch], t.hi[ch], bbox);
            } else if (ch_ok) {
                const int gc = t.kids[8 * (int64_t)ch + g];
                if (gc >= 0 && gc < nn) {
                    if (t.info[gc].w >> 8) {
                        box_add(bx, t.lo[gc], t.hi[gc], bbox);
                    } else {
                        const int4 *kp = (const int4 *)(t.kids + 8 * (int64_t)gc);
                        const int4 ka = kp[0], kb = kp[1];
                        const int kid[8] = {ka.x, ka.y, ka.z, ka.w, kb.x, kb.y, kb.z, kb.w};
#pragma unroll
                        for (int k = 0; k < 8; k++)
                            if (kid[k] >= 0 && kid[k] < nn) box_add(bx, t.lo[kid[k]], t.hi[kid[k]], bbox);
                        box_store(t, gc, bx, bbox);
                    }
                }
            }
            box_reduce<1, 8>(bx, bbox); // the child
            if (ch_ok && !ch_leaf && g == 0) box_store(t, ch, bx, bbox);
            box_reduce<8, 64>(bx, bbox); // the node
            if (lane == 0) box_store(t, nd, bx, bbox);
        }
    }
}

// The child records of every node (after its children's boxes are final):
// slot s of node p gets child s's outward-rounded FP32 box and its item, so
// that a walk tests all children of a node with one load per child.
__global__ void k_tree_krec(const TreeDev t, const DevStatus *st)
{
    const int nn = min(st->n_nodes, t.capacity);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < 8 * (int64_t)nn; q += stride) {
        const int c = t.kids[q];
        float4 lo = make_float4(INFINITY, INFINITY, INFINITY, 0.0f);
        float4 hi = make_float4(-INFINITY, -INFINITY, -INFINITY, __int_as_float(-1));
        if (c >= 0 && c < nn) {
            const int leaf = t.info[c].w >> 8;
            const int nc = t.nchild[c];
            lo = t.box32[2 * (int64_t)c];
            hi = t.box32[2 * (int64_t)c + 1];
            hi.w = __int_as_float(leaf ? (c | (int)0x80000000u) : (c | ((max(nc, 1) - 1) << 28)));
        }
        t.krec[2 * q] = lo;
        t.krec[2 * q + 1] = hi;
    }
}

hipError_t launch_tree_build(hipStream_t s, const PartDev &p, const uint64_t *keys, int n_leaf,
                             TreeBufs &tb, TreeDev &t, uint32_t *scan_tmp, DevStatus *st)
{
    int64_t n = p.n;
    unsigned gb = (unsigned)((n + 256) / 256);
    k_tree_prefix<<<gb, 256, 0, s>>>(n, p.nb, p.box_off, keys, n_leaf, tb.lcp, (int8_t *)tb.start);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // cwin lives in the (not yet used) start buffer
    k_tree_count<<<gb, 256, 256 + n_leaf, s>>>(n, p.nb, p.box_off, n_leaf, tb.lcp,
                                               (const int8_t *)tb.start, tb.dlev, tb.cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = launch_scan_excl_u32(s, tb.cnt, tb.start, n + 1, scan_tmp, nullptr);
    if (e != hipSuccess) return e;
    k_tree_emit<<<gb, 256, 0, s>>>(n, p.nb, p.box_off, keys, tb.lcp, tb.dlev, tb.start, t, st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_tree_roots<<<(p.nb + 1 + 255) / 256, 256, 0, s>>>(p.nb, p.box_off, tb.start, t.box_root,
                                                       st, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_tree_refit(s, p, t, true, st, n);
}

hipError_t launch_tree_refit(hipStream_t s, const PartDev &p, TreeDev &t, bool bbox,
                             DevStatus *st, int64_t n)
{
    (void)n;
    // grid-stride kernels over the nodes (their number is known on the device only)
    int64_t g = (t.capacity + 255) / 256;
    const unsigned gnodes = (unsigned)(g < 1024 ? g : 1024);
    hipError_t e;
    if (bbox) { // a new tree: child counts and the child table
        k_tree_nchild<<<gnodes, 256, 0, s>>>(t, st);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // eight lanes per node id: up to 8192 workgroups of 32 node ids
    const int64_t gl = (8 * (int64_t)t.capacity + 255) / 256;
    k_tree_leaves<<<(unsigned)(gl < 8192 ? gl : 8192), 256, 0, s>>>(p, t, st, st, bbox ? 1 : 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // level 21 holds leaves only; levels 20 .. 0 in three-level steps
    for (int level = SFC_KEY_BITS - 3; level >= 0; level -= 3) {
        k_tree_up3<<<gnodes, 256, 0, s>>>(t, st, bbox ? 1 : 0, level);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int64_t gk = (8 * (int64_t)t.capacity + 255) / 256;
    k_tree_krec<<<(unsigned)(gk < 4096 ? gk : 4096), 256, 0, s>>>(t, st);
    return hipGetLastError();
}
