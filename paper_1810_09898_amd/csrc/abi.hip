// abi.hip -- the extern "C" boundary of libsfcngb: argument checks,
// workspace layout, and the order of launches of each call.
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "internal.h"

// Device scratch of sfc_sort_static: a file-scope array that every device
// the library runs on holds until the process ends.  Host code never uses
// the name `scratch` as an address: its device address is looked up once per
// device (sfc_ctx_create, with that device current) and kept in g_scratch.
static __device__ __align__(256) char scratch[SFC_STATIC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[MAX_DEVICES];      // device address of `scratch` on each device
hipError_t g_scratch_err[MAX_DEVICES];

// the address of `scratch` on the current device `dev` (looked up once)
void *scratch_resolve(int dev, hipError_t *err)
{
    if (dev < 0 || dev >= MAX_DEVICES) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev] && g_scratch_err[dev] == hipSuccess) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e == hipSuccess && ptr) g_scratch[dev] = ptr;
        else g_scratch_err[dev] = e != hipSuccess ? e : hipErrorInvalidSymbol;
    }
    *err = g_scratch_err[dev];
    return g_scratch[dev];
}
} // namespace

hipError_t launch_gather(hipStream_t s, const sfc_particles *in, sfc_particles *out,
                         const uint32_t *perm, uint32_t *perm_out);
hipError_t launch_density(hipStream_t s, const PartDev &p, const TreeDev &t, const GroupBufs &g,
                          SearchBufs &sb, const DensityArgs &a, DevStatus *st);
hipError_t launch_hydro(hipStream_t s, const PartDev &p, const TreeDev &t, const GroupBufs &g,
                        SearchBufs &sb, const HydroArgs &a, DevStatus *st);
hipError_t launch_verify(hipStream_t s, const PartDev &p, const TreeDev &t, const GroupBufs &g,
                         SearchBufs &sb, const sfc_verify &v, int t_cand, DevStatus *st);

struct sfc_ctx {
    hipStream_t stream;
    int device;
    int cu;
    int wclk_khz; // the device's constant clock (wall_clock64), kHz
    bool trace;   // schedule statistics of the group and member kernels
    char err[512];
    bool bound;
    sfc_dims dims;
    char *ws;
    size_t ws_bytes;
    DevStatus *st;
    SortBufs sb;
    TreeBufs tb;
    TreeDev td;
    GroupBufs gb;
    SearchBufs xb;  // the density pass (and every pass without kept supersets)
    SearchBufs xh;  // the hydro pass: == xb unless dims.keep_supersets
    uint32_t *scan_tmp;
    int tree_leaf; // n_leaf of the last tree, 0 = none
    int have_groups;
    int kept_d, kept_h; // t_cand of the kept density / hydro supersets, 0 = none
    bool capturing;
    void *scratch;  // device address of the static scratch on this device (or NULL)
    hipError_t scratch_err;
};

struct sfc_graph {
    hipGraph_t g;
    hipGraphExec_t e;
};

namespace {

int fail(sfc_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(c->err, sizeof(c->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

int hip_fail(sfc_ctx *c, hipError_t e, const char *where)
{
    return fail(c, SFC_EHIP, "%s: %s", where, hipGetErrorString(e));
}

// bump allocator over the workspace (or a size count when base is null)
struct Bump {
    char *base;
    size_t off;
    template <class T> T *take(size_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

int64_t node_capacity(const sfc_dims &d)
{
    return d.n + 22 * d.n / ((int64_t)d.n_leaf_min + 1) + d.n_boxes + 64;
}

int64_t sort_tiles(const sfc_dims &d) { return (d.n + 4095) / 4096; }

int64_t cand_capacity(const sfc_dims &d)
{
    const int64_t per = d.cand_per_particle > 0 ? d.cand_per_particle : 96;
    return per * d.n + 64 * (int64_t)d.t_cand_max;
}

// the sort's buffers (records, double-buffered keys, payloads and box ids,
// tile histograms) for n particles in nb boxes
SortBufs carve_sort(Bump &b, int64_t n, int64_t nb)
{
    SortBufs sb;
    const int64_t nt = (n + 4095) / 4096;
    sb.rec = b.take<PRec>(n);
    sb.key_a = b.take<uint64_t>(n);
    sb.key_b = b.take<uint64_t>(n);
    sb.val_a = b.take<uint32_t>(n);
    sb.val_b = b.take<uint32_t>(n);
    sb.box_a = b.take<uint32_t>(nb > 1 ? n : 1);
    sb.box_b = b.take<uint32_t>(nb > 1 ? n : 1);
    sb.hist = b.take<uint32_t>(2 * 256 * nt);
    sb.scan_tmp = nullptr;
    return sb;
}

bool dims_ok(const sfc_dims *d)
{
    return d && d->n >= 1 && d->n < ((int64_t)1 << 30) && d->n_boxes >= 1 &&
           d->n_boxes <= 65536 && d->n_boxes <= d->n && d->n_leaf_min >= 1 &&
           d->t_cand_max >= 64 && d->t_cand_max <= 8192 && d->t_cand_max % 64 == 0 &&
           d->cand_per_particle >= 0 && d->cand_per_particle <= 4096 &&
           (d->keep_supersets == 0 || d->keep_supersets == 1) &&
           node_capacity(*d) <= TREE_ITEM_NODE;
}

size_t layout(sfc_ctx *c, const sfc_dims &d, char *base)
{
    Bump b{base, 0};
    int64_t n = d.n, nb = d.n_boxes, cap = node_capacity(d);
    int64_t nt = sort_tiles(d);
    DevStatus *st = b.take<DevStatus>(1);
    SortBufs sb = carve_sort(b, n, nb);
    int64_t scan_n = n + 1;
    if (256 * nt > scan_n) scan_n = 256 * nt;
    uint32_t *scan_tmp = b.take<uint32_t>(scan_tmp_elems(scan_n));
    sb.scan_tmp = scan_tmp;
    TreeBufs tb;
    tb.lcp = b.take<int8_t>(n);
    tb.dlev = b.take<int8_t>(n);
    tb.cnt = b.take<uint32_t>(n + 1);
    tb.start = b.take<uint32_t>(n + 1);
    TreeDev td;
    td.info = b.take<int4>(cap);
    td.kids = b.take<int32_t>(8 * cap);
    td.lo = b.take<double4>(cap);
    td.hi = b.take<double4>(cap);
    td.box32 = b.take<float4>(2 * cap);
    td.nchild = b.take<int32_t>(cap);
    td.krec = b.take<float4>(16 * cap);
    td.box_root = b.take<int32_t>(nb + 1);
    td.capacity = (int32_t)cap;
    GroupBufs gb;
    gb.flag_scan = b.take<uint32_t>(n + 1);
    gb.act = b.take<int32_t>(n);
    gb.nxt = b.take<int32_t>(n);
    {
        int64_t ni[GROUP_LEVELS_MAX], sp[GROUP_LEVELS_MAX];
        const int L = group_levels(n, ni, sp);
        for (int l = 0; l < GROUP_LEVELS_MAX; l++) {
            gb.map[l] = l < L ? b.take<GMap>(ni[l]) : nullptr;
            gb.ent[l] = l < L ? b.take<int32_t>(ni[l]) : nullptr;
            gb.before[l] = l < L ? b.take<int32_t>(ni[l]) : nullptr;
        }
    }
    gb.goff = b.take<int32_t>(n + 1);
    gb.n_act = b.take<int32_t>(1);
    gb.n_groups = b.take<int32_t>(1);
    gb.box_T = b.take<int32_t>(nb);
    SearchBufs xb;
    xb.cand_cap = cand_capacity(d);
    xb.cand = b.take<int32_t>(xb.cand_cap);
    xb.sup = b.take<GSup>(n);
    xb.grp = b.take<int32_t>(n);
    xb.pa = b.take<float4>(n);
    xb.pb = b.take<float4>(n);
    xb.pc = b.take<float4>(n);
    xb.pos4 = b.take<float4>(n);
    xb.p64 = b.take<double4>(n);
    xb.dstate = b.take<double4>(n);
    xb.snap = nullptr;
    xb.drift = nullptr;
    xb.sel = nullptr;
    xb.dfr = b.take<int32_t>(n);
    xb.gmark = b.take<int32_t>(n);
    xb.glist = b.take<int32_t>(n);
    xb.cu_count = c ? c->cu : 0;
    SearchBufs xh = xb;
    if (d.keep_supersets) {
        // the hydro pass gets buffers of its own; snapshots and drift bounds
        xb.snap = b.take<double4>(n);
        xb.drift = b.take<unsigned long long>(4 + 3 * 512);
        xb.sel = b.take<int32_t>(n);
        xh.cand = b.take<int32_t>(xh.cand_cap);
        xh.sup = b.take<GSup>(n);
        xh.snap = b.take<double4>(n);
        xh.drift = b.take<unsigned long long>(4 + 3 * 512);
        xh.sel = xb.sel;
    }
    if (c && base) {
        c->st = st;
        c->sb = sb;
        c->tb = tb;
        c->td = td;
        c->gb = gb;
        c->xb = xb;
        c->xh = xh;
        c->scan_tmp = scan_tmp;
        c->kept_d = c->kept_h = 0;
    }
    return (b.off + 255) & ~(size_t)255;
}

int check_ctx(sfc_ctx *c)
{
    if (!c) return SFC_EINVAL;
    if (!c->bound) return fail(c, SFC_EWORKSPACE, "no workspace bound");
    return SFC_OK;
}

int check_particles(sfc_ctx *c, const sfc_particles *p, bool need_state)
{
    if (!p) return fail(c, SFC_EINVAL, "particles: NULL");
    if (p->n != c->dims.n || p->n_boxes != c->dims.n_boxes)
        return fail(c, SFC_EINVAL, "particles: n=%lld boxes=%d differ from the bound dims (%lld, %d)",
                    (long long)p->n, p->n_boxes, (long long)c->dims.n, c->dims.n_boxes);
    if (!p->box_off_host || !p->box_off || !p->box_L)
        return fail(c, SFC_EINVAL, "particles: box arrays missing");
    if (p->box_off_host[0] != 0 || p->box_off_host[p->n_boxes] != p->n)
        return fail(c, SFC_EINVAL, "particles: box_off must start at 0 and end at n");
    for (int b = 0; b < p->n_boxes; b++)
        if (p->box_off_host[b + 1] < p->box_off_host[b])
            return fail(c, SFC_EINVAL, "particles: box_off not monotone at %d", b);
    if (!p->x || !p->y || !p->z || !p->h || !p->m || !p->active)
        return fail(c, SFC_EINVAL, "particles: x, y, z, h, m and active are required");
    if (need_state && (!p->rho || !p->fgrad))
        return fail(c, SFC_EINVAL, "particles: rho and fgrad are required");
    return SFC_OK;
}

PartDev part_dev(const sfc_particles *p)
{
    PartDev d;
    d.n = p->n;
    d.nb = p->n_boxes;
    d.box_off = p->box_off;
    d.box_L = p->box_L;
    d.x = p->x;
    d.y = p->y;
    d.z = p->z;
    d.h = p->h;
    d.m = p->m;
    d.vx = p->vx;
    d.vy = p->vy;
    d.vz = p->vz;
    d.u = p->u;
    d.rho = p->rho;
    d.fgrad = p->fgrad;
    d.active = p->active;
    d.orig = p->orig;
    return d;
}

} // namespace

extern "C" {

int sfc_ctx_create(sfc_ctx **out, void *hip_stream)
{
    if (!out) return SFC_EINVAL;
    *out = nullptr;
    sfc_ctx *c = new (std::nothrow) sfc_ctx();
    if (!c) return SFC_EINVAL;
    memset(c, 0, sizeof(*c));
    c->stream = (hipStream_t)hip_stream;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->cu, hipDeviceAttributeMultiprocessorCount, c->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->wclk_khz, hipDeviceAttributeWallClockRate, c->device);
    if (e != hipSuccess) {
        delete c;
        return SFC_EHIP;
    }
    // the static scratch of sfc_sort_static on this device (its failure only
    // disables that call)
    c->scratch = scratch_resolve(c->device, &c->scratch_err);
    *out = c;
    return SFC_OK;
}

void sfc_ctx_destroy(sfc_ctx *ctx) { delete ctx; }

int sfc_ctx_set_trace(sfc_ctx *ctx, int on)
{
    if (!ctx || (on != 0 && on != 1)) return SFC_EINVAL;
    ctx->trace = on != 0;
    return SFC_OK;
}

int sfc_ctx_set_stream(sfc_ctx *ctx, void *hip_stream)
{
    if (!ctx) return SFC_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
    return SFC_OK;
}

const char *sfc_ctx_last_error(const sfc_ctx *ctx) { return ctx ? ctx->err : "no context"; }

int32_t sfc_ctx_cu_count(const sfc_ctx *ctx) { return ctx ? ctx->cu : 0; }

size_t sfc_workspace_bytes(const sfc_dims *dims)
{
    if (!dims_ok(dims)) return 0;
    return layout(nullptr, *dims, nullptr);
}

int sfc_workspace_bind(sfc_ctx *ctx, const sfc_dims *dims, void *ws, size_t ws_bytes)
{
    if (!ctx) return SFC_EINVAL;
    if (!dims_ok(dims)) return fail(ctx, SFC_EINVAL, "workspace: invalid dims");
    if (!ws) return fail(ctx, SFC_EINVAL, "workspace: NULL");
    if ((uintptr_t)ws % 256 != 0) return fail(ctx, SFC_EINVAL, "workspace: must be 256-byte aligned");
    size_t need = layout(nullptr, *dims, nullptr);
    if (ws_bytes < need)
        return fail(ctx, SFC_EWORKSPACE, "workspace: %zu bytes given, %zu needed", ws_bytes, need);
    ctx->dims = *dims;
    ctx->ws = (char *)ws;
    ctx->ws_bytes = ws_bytes;
    layout(ctx, *dims, (char *)ws);
    ctx->bound = true;
    ctx->tree_leaf = 0;
    ctx->have_groups = 0;
    ctx->kept_d = ctx->kept_h = 0;
    // a new workspace: the whole status block, the node count included
    hipError_t e = launch_fill_i32(ctx->stream, (int32_t *)ctx->st, 0,
                                   (int64_t)(sizeof(DevStatus) / sizeof(int32_t)));
    return e == hipSuccess ? SFC_OK : hip_fail(ctx, e, "status clear");
}

int sfc_status_clear(sfc_ctx *ctx)
{
    int r = check_ctx(ctx);
    if (r) return r;
    // flags and counters only: the node count of the current tree (which
    // the refits and walks read) and the sizes of the last grouping stay
    static_assert(offsetof(DevStatus, flags) == 0, "flags lead the status block");
    static_assert(offsetof(DevStatus, n_deferred) % 4 == 0 && offsetof(DevStatus, cand_top) % 4 == 0,
                  "counters are whole words");
    int32_t *base = (int32_t *)ctx->st;
    hipError_t e = launch_fill_i32(ctx->stream, base, 0, 1);
    if (e == hipSuccess)
        e = launch_fill_i32(ctx->stream, base + offsetof(DevStatus, n_deferred) / 4, 0,
                            (int64_t)((offsetof(DevStatus, cand_top) - offsetof(DevStatus, n_deferred)) / 4));
    return e == hipSuccess ? SFC_OK : hip_fail(ctx, e, "status clear");
}

int sfc_sort(sfc_ctx *ctx, const sfc_particles *in, sfc_particles *out, uint64_t *keys_out,
             uint32_t *perm_out)
{
    int r = check_ctx(ctx);
    if (r) return r;
    if ((r = check_particles(ctx, in, false))) return r;
    if (!out || !keys_out) return fail(ctx, SFC_EINVAL, "sort: out and keys_out are required");
    if (out->n != in->n || !out->x || !out->y || !out->z || !out->h || !out->m || !out->active)
        return fail(ctx, SFC_EINVAL, "sort: out must have n and x, y, z, h, m, active");
    if (out->x == in->x || out->h == in->h) return fail(ctx, SFC_EINVAL, "sort: in and out alias");
    if (in->orig && !out->orig) return fail(ctx, SFC_EINVAL, "sort: out->orig missing");
    hipError_t e = launch_keys(ctx->stream, in, ctx->sb);
    if (e != hipSuccess) return hip_fail(ctx, e, "sort keys");
    uint32_t *perm = nullptr;
    e = launch_radix_sort(ctx->stream, in->n, in->n_boxes, ctx->sb, keys_out, &perm);
    if (e != hipSuccess) return hip_fail(ctx, e, "radix sort");
    e = launch_gather(ctx->stream, in, out, perm, ctx->sb.rec, perm_out);
    if (e != hipSuccess) return hip_fail(ctx, e, "gather");
    ctx->tree_leaf = 0;
    ctx->have_groups = 0;
    ctx->kept_d = ctx->kept_h = 0;
    return SFC_OK;
}

int sfc_sort_static(sfc_ctx *ctx, const sfc_particles *in, sfc_particles *out, uint64_t *keys_out,
                    uint32_t *perm_out)
{
    if (!ctx) return SFC_EINVAL;
    if (!in) return fail(ctx, SFC_EINVAL, "sort_static: particles NULL");
    if (in->n < 1 || in->n > SFC_SORT_STATIC_MAX_N)
        return fail(ctx, SFC_EINVAL, "sort_static: n=%lld outside [1, %d] (the static scratch)",
                    (long long)in->n, SFC_SORT_STATIC_MAX_N);
    if (in->n_boxes < 1 || in->n_boxes > in->n || in->n_boxes > 65536)
        return fail(ctx, SFC_EINVAL, "sort_static: n_boxes=%d outside [1, min(n, 65536)]",
                    in->n_boxes);
    if (!in->box_off_host || !in->box_off || !in->box_L)
        return fail(ctx, SFC_EINVAL, "sort_static: box arrays missing");
    if (in->box_off_host[0] != 0 || in->box_off_host[in->n_boxes] != in->n)
        return fail(ctx, SFC_EINVAL, "sort_static: box_off must start at 0 and end at n");
    for (int b = 0; b < in->n_boxes; b++)
        if (in->box_off_host[b + 1] < in->box_off_host[b])
            return fail(ctx, SFC_EINVAL, "sort_static: box_off not monotone at %d", b);
    if (!in->x || !in->y || !in->z || !in->h || !in->m || !in->active)
        return fail(ctx, SFC_EINVAL, "sort_static: x, y, z, h, m and active are required");
    if (!out || !keys_out) return fail(ctx, SFC_EINVAL, "sort_static: out and keys_out are required");
    if (out->n != in->n || !out->x || !out->y || !out->z || !out->h || !out->m || !out->active)
        return fail(ctx, SFC_EINVAL, "sort_static: out must have n and x, y, z, h, m, active");
    if (out->x == in->x || out->h == in->h)
        return fail(ctx, SFC_EINVAL, "sort_static: in and out alias");
    if (in->orig && !out->orig) return fail(ctx, SFC_EINVAL, "sort_static: out->orig missing");
    if (!ctx->scratch)
        return hip_fail(ctx, ctx->scratch_err, "sort_static: no static scratch on this device");
    // the sort's buffers and its scan scratch, carved from the static array
    Bump b{(char *)ctx->scratch, 0};
    SortBufs sb = carve_sort(b, in->n, in->n_boxes);
    const int64_t nt = (in->n + 4095) / 4096;
    sb.scan_tmp = b.take<uint32_t>(scan_tmp_elems(256 * nt));
    if (b.off > (size_t)SFC_STATIC_SCRATCH_BYTES)
        return fail(ctx, SFC_EINVAL, "sort_static: %zu bytes of scratch needed, %zu held", b.off,
                    (size_t)SFC_STATIC_SCRATCH_BYTES);
    hipError_t e = launch_keys(ctx->stream, in, sb);
    if (e != hipSuccess) return hip_fail(ctx, e, "sort_static keys");
    uint32_t *perm = nullptr;
    e = launch_radix_sort(ctx->stream, in->n, in->n_boxes, sb, keys_out, &perm);
    if (e != hipSuccess) return hip_fail(ctx, e, "sort_static radix sort");
    e = launch_gather(ctx->stream, in, out, perm, sb.rec, perm_out);
    if (e != hipSuccess) return hip_fail(ctx, e, "sort_static gather");
    return SFC_OK;
}

int tree_build(sfc_ctx *ctx, const sfc_particles *p, const uint64_t *keys, int32_t n_leaf)
{
    int r = check_ctx(ctx);
    if (r) return r;
    if ((r = check_particles(ctx, p, false))) return r;
    if (!keys) return fail(ctx, SFC_EINVAL, "tree_build: keys NULL");
    if (n_leaf < ctx->dims.n_leaf_min || n_leaf > 4096)
        return fail(ctx, SFC_EINVAL, "tree_build: n_leaf %d outside [%d, 4096]", n_leaf,
                    ctx->dims.n_leaf_min);
    PartDev pd = part_dev(p);
    hipError_t e = launch_tree_build(ctx->stream, pd, keys, n_leaf, ctx->tb, ctx->td,
                                     ctx->scan_tmp, ctx->st);
    if (e != hipSuccess) return hip_fail(ctx, e, "tree_build");
    ctx->tree_leaf = n_leaf;
    ctx->have_groups = 0;
    ctx->kept_d = ctx->kept_h = 0;
    return SFC_OK;
}

int tree_refit_hmax(sfc_ctx *ctx, const sfc_particles *p)
{
    int r = check_ctx(ctx);
    if (r) return r;
    if ((r = check_particles(ctx, p, false))) return r;
    if (!ctx->tree_leaf) return fail(ctx, SFC_EORDER, "tree_refit_hmax: no tree");
    PartDev pd = part_dev(p);
    hipError_t e = launch_tree_refit(ctx->stream, pd, ctx->td, false, ctx->st, p->n);
    return e == hipSuccess ? SFC_OK : hip_fail(ctx, e, "tree_refit_hmax");
}

int tree_refit(sfc_ctx *ctx, const sfc_particles *p)
{
    int r = check_ctx(ctx);
    if (r) return r;
    if ((r = check_particles(ctx, p, false))) return r;
    if (!ctx->tree_leaf) return fail(ctx, SFC_EORDER, "tree_refit: no tree");
    PartDev pd = part_dev(p);
    hipError_t e = launch_tree_refit(ctx->stream, pd, ctx->td, true, ctx->st, p->n);
    return e == hipSuccess ? SFC_OK : hip_fail(ctx, e, "tree_refit");
}

static int check_group_params(sfc_ctx *ctx, const sfc_group_params *gp)
{
    if (gp->policy != SFC_POLICY_COUNT && gp->policy != SFC_POLICY_PAPER &&
        gp->policy != SFC_POLICY_TREE)
        return fail(ctx, SFC_EINVAL, "group params: bad policy %d", gp->policy);
    if (gp->policy == SFC_POLICY_TREE && (gp->level < 0 || gp->level > SFC_KEY_BITS))
        return fail(ctx, SFC_EINVAL, "group params: level %d outside [0, 21]", gp->level);
    if (gp->n_group_max < 1 || gp->n_group_max > SFC_WAVE_GROUP_MAX)
        return fail(ctx, SFC_EINVAL, "group params: n_group_max %d outside [1, 64]", gp->n_group_max);
    if (gp->policy == SFC_POLICY_PAPER && !(gp->f >= 0.0))
        return fail(ctx, SFC_EINVAL, "group params: f must be >= 0");
    return SFC_OK;
}

static int check_tile(sfc_ctx *ctx, int t_cand)
{
    if (t_cand < 64 || t_cand % 64 != 0 || t_cand > ctx->dims.t_cand_max)
        return fail(ctx, SFC_EINVAL, "t_cand %d must be a multiple of 64 in [64, %d]", t_cand,
                    ctx->dims.t_cand_max);
    return SFC_OK;
}

int group_ngb_search(sfc_ctx *ctx, const sfc_particles *p, const sfc_group_params *gp,
                     const sfc_group_params *gp_box, const sfc_verify *verify, int32_t t_cand)
{
    int r = check_ctx(ctx);
    if (r) return r;
    if ((r = check_particles(ctx, p, false))) return r;
    if (!ctx->tree_leaf) return fail(ctx, SFC_EORDER, "group_ngb_search: build the tree first");
    if (!gp && !gp_box) return fail(ctx, SFC_EINVAL, "group_ngb_search: no group parameters");
    if (gp && (r = check_group_params(ctx, gp))) return r;
    if (verify) {
        if ((r = check_tile(ctx, t_cand))) return r;
        if (verify->mode != 0 && verify->mode != 1)
            return fail(ctx, SFC_EINVAL, "verify: mode must be 0 or 1");
        if (!verify->count) return fail(ctx, SFC_EINVAL, "verify: count is required");
        if (verify->list && !verify->list_off)
            return fail(ctx, SFC_EINVAL, "verify: list needs list_off");
    }
    PartDev pd = part_dev(p);
    hipError_t e = launch_groups(ctx->stream, pd, gp_box ? nullptr : gp, gp_box, ctx->tb.dlev,
                                 ctx->gb, ctx->scan_tmp, ctx->st);
    if (e != hipSuccess) return hip_fail(ctx, e, "groups");
    ctx->have_groups = 1;
    ctx->kept_d = ctx->kept_h = 0;
    if (verify) {
        if (verify->mode == 1) {
            e = launch_tree_refit(ctx->stream, pd, ctx->td, false, ctx->st, p->n);
            if (e != hipSuccess) return hip_fail(ctx, e, "verify refit");
        }
        e = launch_verify(ctx->stream, pd, ctx->td, ctx->gb, ctx->xb, *verify, t_cand, ctx->st);
        if (e != hipSuccess) return hip_fail(ctx, e, "verify");
    }
    return SFC_OK;
}

int density(sfc_ctx *ctx, sfc_particles *p, const sfc_density_params *dp, sfc_density_out *out)
{
    int r = check_ctx(ctx);
    if (r) return r;
    if ((r = check_particles(ctx, p, true))) return r;
    if (!dp) return fail(ctx, SFC_EINVAL, "density: params NULL");
    if (!ctx->have_groups) return fail(ctx, SFC_EORDER, "density: run group_ngb_search first");
    if (dp->kernel != SFC_KERNEL_CUBIC && dp->kernel != SFC_KERNEL_WC6)
        return fail(ctx, SFC_EINVAL, "density: bad kernel %d", dp->kernel);
    if (dp->n_ngb < 1 || dp->dn < 0 || dp->max_iter < 1 || dp->max_iter > 1000)
        return fail(ctx, SFC_EINVAL, "density: n_ngb >= 1, dn >= 0, 1 <= max_iter <= 1000");
    if (!(dp->skin >= 1.0 && dp->skin <= 4.0))
        return fail(ctx, SFC_EINVAL, "density: skin must be in [1, 4]");
    if (dp->accum != SFC_ACCUM_F32 && dp->accum != SFC_ACCUM_F64)
        return fail(ctx, SFC_EINVAL, "density: bad accum");
    if ((r = check_tile(ctx, dp->t_cand))) return r;
    if (dp->reuse != 0 && dp->reuse != 1) return fail(ctx, SFC_EINVAL, "density: reuse must be 0 or 1");
    if (dp->reuse && ctx->kept_d == 0)
        return fail(ctx, SFC_EORDER, "density: reuse without kept supersets (dims.keep_supersets, "
                                     "a walking density call since group_ngb_search)");
    if (dp->reuse && ctx->kept_d != dp->t_cand)
        return fail(ctx, SFC_EINVAL, "density: reuse needs the kept t_cand %d", ctx->kept_d);
    DensityArgs a;
    a.dp = *dp;
    a.keep = ctx->dims.keep_supersets && !dp->reuse;
    a.trace = ctx->trace;
    if (out) a.out = *out;
    else memset(&a.out, 0, sizeof(a.out));
    PartDev pd = part_dev(p);
    hipError_t e = hipSuccess;
    if (dp->reuse) {
        // members that leave a kept superset walk the tree: its node boxes
        // must span the particles where they are now
        e = launch_tree_refit(ctx->stream, pd, ctx->td, true, ctx->st, p->n);
        if (e != hipSuccess) return hip_fail(ctx, e, "density refit");
    }
    e = launch_density(ctx->stream, pd, ctx->td, ctx->gb, ctx->xb, a, ctx->st);
    if (e != hipSuccess) return hip_fail(ctx, e, "density");
    if (a.keep) ctx->kept_d = dp->t_cand;
    return SFC_OK;
}

int hydro_force(sfc_ctx *ctx, const sfc_particles *p, const sfc_hydro_params *hp,
                sfc_hydro_out *out)
{
    int r = check_ctx(ctx);
    if (r) return r;
    if ((r = check_particles(ctx, p, true))) return r;
    if (!hp || !out) return fail(ctx, SFC_EINVAL, "hydro_force: params and out are required");
    if (!p->vx || !p->vy || !p->vz || !p->u)
        return fail(ctx, SFC_EINVAL, "hydro_force: vx, vy, vz, u are required");
    if (!out->ax || !out->ay || !out->az || !out->dudt || !out->vsigmax)
        return fail(ctx, SFC_EINVAL, "hydro_force: ax, ay, az, dudt, vsigmax are required");
    if (!ctx->have_groups) return fail(ctx, SFC_EORDER, "hydro_force: run group_ngb_search first");
    if (hp->kernel != SFC_KERNEL_CUBIC && hp->kernel != SFC_KERNEL_WC6)
        return fail(ctx, SFC_EINVAL, "hydro_force: bad kernel %d", hp->kernel);
    if (!(hp->gamma > 1.0) || !(hp->alpha >= 0.0))
        return fail(ctx, SFC_EINVAL, "hydro_force: gamma > 1 and alpha >= 0 required");
    if (hp->accum != SFC_ACCUM_F32 && hp->accum != SFC_ACCUM_F64)
        return fail(ctx, SFC_EINVAL, "hydro_force: bad accum");
    if ((r = check_tile(ctx, hp->t_cand))) return r;
    if (!(hp->skin >= 1.0 && hp->skin <= 4.0))
        return fail(ctx, SFC_EINVAL, "hydro_force: skin must be in [1, 4]");
    if (hp->physics != SFC_HYDRO_STANDARD && hp->physics != SFC_HYDRO_PRODUCTION)
        return fail(ctx, SFC_EINVAL, "hydro_force: bad physics %d", hp->physics);
    if (hp->physics == SFC_HYDRO_PRODUCTION &&
        (!hp->alpha_i || !(hp->alpha_u >= 0.0) || !(hp->alpha_min >= 0.0) ||
         !(hp->alpha_max >= hp->alpha_min) || !(hp->ell >= 0.0)))
        return fail(ctx, SFC_EINVAL,
                    "hydro_force: production physics needs alpha_i, alpha_u >= 0, "
                    "0 <= alpha_min <= alpha_max and ell >= 0");
    if (hp->reuse != 0 && hp->reuse != 1)
        return fail(ctx, SFC_EINVAL, "hydro_force: reuse must be 0 or 1");
    if (hp->reuse && ctx->kept_h == 0)
        return fail(ctx, SFC_EORDER, "hydro_force: reuse without kept supersets");
    if (hp->reuse && ctx->kept_h != hp->t_cand)
        return fail(ctx, SFC_EINVAL, "hydro_force: reuse needs the kept t_cand %d", ctx->kept_h);
    HydroArgs a;
    a.hp = *hp;
    a.out = *out;
    a.keep = ctx->dims.keep_supersets && !hp->reuse;
    a.trace = ctx->trace;
    PartDev pd = part_dev(p);
    // the hydro walks read every node's max h: refresh it from the current h
    // (and the boxes after a drift, for the members that walk alone)
    hipError_t e = launch_tree_refit(ctx->stream, pd, ctx->td, hp->reuse != 0, ctx->st, p->n);
    if (e != hipSuccess) return hip_fail(ctx, e, "hydro_force refit");
    e = launch_hydro(ctx->stream, pd, ctx->td, ctx->gb, ctx->xh, a, ctx->st);
    if (e != hipSuccess) return hip_fail(ctx, e, "hydro_force");
    if (a.keep) ctx->kept_h = hp->t_cand;
    return SFC_OK;
}

int sfc_status_read(sfc_ctx *ctx, sfc_status *out)
{
    int r = check_ctx(ctx);
    if (r) return r;
    if (!out) return fail(ctx, SFC_EINVAL, "status: out NULL");
    DevStatus s;
    hipError_t e = hipMemcpyAsync(&s, ctx->st, sizeof(s), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "status read");
    out->flags = s.flags;
    out->n_nodes = s.n_nodes;
    out->n_active = s.n_active;
    out->n_groups = s.n_groups;
    out->n_deferred = (int64_t)s.n_deferred;
    out->n_overflow = (int64_t)s.n_overflow;
    out->n_not_converged = (int64_t)s.n_not_converged;
    out->sum_cand = (int64_t)s.sum_cand;
    out->n_walks = (int64_t)s.n_walks;
    out->sum_iters = (int64_t)s.sum_iters;
    out->sum_tests = (int64_t)s.sum_tests;
    out->sum_pairs = (int64_t)s.sum_pairs;
    for (int k = 0; k < 2; k++) {
        // the eight per-XCD slots combined
        unsigned long long t0 = ~0ull, t1 = 0, n = 0;
        double sum = 0.0;
        for (int x = 0; x < 8; x++) {
            const unsigned long long *q = s.sched[k][x];
            if (!q[3]) continue;
            t0 = q[0] < t0 ? q[0] : t0;
            t1 = q[1] > t1 ? q[1] : t1;
            sum += (double)q[2];
            n += q[3];
        }
        const bool ok = n > 0 && t1 >= t0 && ctx->wclk_khz > 0;
        const double us = ok ? 1000.0 / (double)ctx->wclk_khz : 0.0; // microseconds per tick
        out->sched_units[k] = ok ? (int64_t)n : 0;
        out->sched_span_us[k] = ok ? (double)(t1 - t0) * us : 0.0;
        out->sched_tail_us[k] = ok ? ((double)t1 - sum / (double)n) * us : 0.0;
    }
    if (s.flags & (SFC_ST_LIST_OVERFLOW | SFC_ST_NODE_OVERFLOW | SFC_ST_GUARD))
        return fail(ctx, SFC_EOVERFLOW, "device capacity or loop limit exceeded (flags 0x%x)", s.flags);
    return SFC_OK;
}

int sfc_get_views(const sfc_ctx *ctx, sfc_views *out)
{
    if (!ctx || !out) return SFC_EINVAL;
    if (!ctx->bound) return SFC_EWORKSPACE;
    out->capacity = ctx->td.capacity;
    out->n_nodes = &ctx->st->n_nodes;
    out->info = (const int32_t *)ctx->td.info;
    out->lo = (const double *)ctx->td.lo;
    out->hi = (const double *)ctx->td.hi;
    out->box_root = ctx->td.box_root;
    out->act = ctx->gb.act;
    out->n_act = ctx->gb.n_act;
    out->goff = ctx->gb.goff;
    out->n_groups = ctx->gb.n_groups;
    return SFC_OK;
}

int sfc_graph_begin(sfc_ctx *ctx)
{
    if (!ctx) return SFC_EINVAL;
    if (!ctx->stream) return fail(ctx, SFC_EINVAL, "graph capture needs a non-null stream");
    hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(ctx, e, "begin capture");
    ctx->capturing = true;
    return SFC_OK;
}

int sfc_graph_end(sfc_ctx *ctx, sfc_graph **out)
{
    if (!ctx || !out) return SFC_EINVAL;
    *out = nullptr;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->stream, &g);
    ctx->capturing = false;
    if (e != hipSuccess) return hip_fail(ctx, e, "end capture");
    sfc_graph *sg = new (std::nothrow) sfc_graph();
    if (!sg) {
        (void)hipGraphDestroy(g);
        return fail(ctx, SFC_EINVAL, "graph: out of host memory");
    }
    sg->g = g;
    e = hipGraphInstantiate(&sg->e, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete sg;
        return hip_fail(ctx, e, "graph instantiate");
    }
    *out = sg;
    return SFC_OK;
}

int sfc_graph_launch(sfc_ctx *ctx, sfc_graph *g)
{
    if (!ctx || !g) return SFC_EINVAL;
    hipError_t e = hipGraphLaunch(g->e, ctx->stream);
    return e == hipSuccess ? SFC_OK : hip_fail(ctx, e, "graph launch");
}

void sfc_graph_destroy(sfc_graph *g)
{
    if (!g) return;
    (void)hipGraphExecDestroy(g->e);
    (void)hipGraphDestroy(g->g);
    delete g;
}

} // extern "C"
