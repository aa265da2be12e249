// search.hip -- grouped neighbour search, density and hydro force.
//
// One wavefront owns one group (groups are dealt to waves round-robin).  A
// group is a run of actives along the Hilbert curve (section
// "Implementation of Neighbour Recycling using a Space Filling Curve"):
//   1. walk: the 64 lanes test 64 consecutive pre-order nodes at once and
//      follow the stackless walk inside that window with ballot masks; the
//      particles of the opened leaves are tested against the group ball
//      (centre = first member, radius = R_g + skin*max h for density,
//      R_g + max(max h, h_j) for hydro) and compacted into an LDS list, in
//      ascending particle order: the group's candidate superset;
//   2. filter: lanes hold candidates, the loop runs over members; one FP64
//      test per (member, candidate) and one ballot give each member a 64-bit
//      neighbour mask per candidate chunk (kept in LDS);
//   3. density only: each member iterates its h on the superset while
//      h + |x_i - x_0| stays inside the walk radius;
//   4. sums: per member, the masks are compacted (mbcnt) into a FIFO of
//      neighbour indices; the k-th neighbour always lands on lane k mod 64,
//      so each lane accumulates a fixed subsequence in a fixed order and the
//      result does not depend on the group the particle was in.
// Members whose h outgrows the superset, and all members of a group whose
// superset overflows the LDS tile, finish alone in the same wave: one walk
// per h evaluation with the particle's own radius, neighbours streamed
// through the FIFO.
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
    T u = q < T(1) ? T(1) - q : T(0);
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

} // namespace

// --------------------------------------------------------------- kernel args
struct Geom {
    const double *x, *y, *z;
    double *h;
    const int64_t *box_off;
    const double *box_L;
    const int4 *info;
    const double4 *lo, *hi;
    const int32_t *box_root;
    int nb;
};
struct GroupArg {
    const int32_t *act, *goff, *n_groups;
    int T, gm;
};

namespace {

// ------------------------------------------------------------------ scheduling
// Workgroups are dealt to the 8 XCDs round-robin (block b on XCD b mod 8),
// and each XCD has its own L2.  Give each XCD one contiguous eighth of the
// groups (groups follow the Hilbert curve, so an eighth is a compact region
// of space): the waves on one XCD then share the tree nodes and particles
// they read.  Within an XCD the waves take the groups in a round-robin
// stride, so the groups in flight are neighbours.
struct GroupRange {
    int g, end, stride;
};
__device__ __forceinline__ GroupRange group_range(int G)
{
    const int W = (int)gridDim.x;
    GroupRange r;
    if (W < 8 || (W & 7)) {
        r.g = blockIdx.x;
        r.end = G;
        r.stride = W;
        return r;
    }
    const int xcd = blockIdx.x & 7;
    const int gx = (G + 7) >> 3;
    r.g = xcd * gx + (int)(blockIdx.x >> 3);
    r.end = min(G, (xcd + 1) * gx);
    r.stride = W >> 3;
    return r;
}

// ------------------------------------------------------------------ walk
struct Ball {
    double cx, cy, cz, L;
    double W2;     // density: squared walk radius
    double Rg, Hg; // hydro: node radius R_g + max(H_g, node hmax)
    int hydro;
};

__device__ __forceinline__ double axis_gap(double c, double lo, double hi, double L)
{
    double a = lo - c, b = c - hi;
    double d = fmax(fmax(a, b), 0.0);
    d = fmin(d, a + L);
    d = fmin(d, b + L);
    return d;
}

struct WalkLds {
    int *first; // [64]
    int *pref;  // [66]
};

// Leaves `vl` (lane mask) of the current window: flatten their particles and
// hand them to `visit` 64 at a time, ascending.
template <class V> __device__ __forceinline__ void emit_leaves(uint64_t vl, int4 inf, WalkLds wl, V &visit)
{
    const int lane = lane_id();
    bool isl = (vl >> lane) & 1ull;
    int c = isl ? inf.y : 0;
    int incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    const int total = uni(readlane_i(incl, 63));
    int r = mbcnt(vl);
    if (isl) {
        wl.first[r] = inf.x;
        wl.pref[r] = incl - c;
    }
    const int nl = popc64(vl);
    wave_lds_sync();
    for (int t0 = 0; t0 < total; t0 += 64) {
        int q = t0 + lane;
        bool valid = q < total;
        int j = 0;
        if (valid) {
            int lo = 0, hi = nl;
#pragma unroll
            for (int s = 0; s < 7; s++) { // nl <= 64: at most 6 halvings
                if (hi - lo > 1) {
                    int mid = (lo + hi) >> 1;
                    if (wl.pref[mid] <= q) lo = mid; else hi = mid;
                }
            }
            j = wl.first[lo] + (q - wl.pref[lo]);
        }
        visit(j, valid);
    }
    wave_lds_sync();
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
template <class V>
__device__ void walk(const Geom &g, int root, int root_end, const Ball &B, WalkLds wl, V &visit,
                     DevStatus *st)
{
    const int lane = lane_id();
    int k = uni(root);
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
            double4 lo = g.lo[node], hi = g.hi[node];
            double gx = axis_gap(B.cx, lo.x, hi.x, B.L);
            double gy = axis_gap(B.cy, lo.y, hi.y, B.L);
            double gz = axis_gap(B.cz, lo.z, hi.z, B.L);
            double d2 = gx * gx + gy * gy + gz * gz;
            double lim = B.hydro ? sq((B.Rg + fmax(B.Hg, lo.w)) * INFL) : B.W2;
            open = d2 < lim;
        }
        const int hide = (inr && !open) ? inf.z : -1;
        const int incl = wave_incl_max(hide);
        int excl = __shfl_up(incl, 1, 64);
        if (lane == 0) excl = -1;
        const bool on_walk = inr && excl <= node;
        const uint64_t vl = ballot(on_walk && open && (inf.w >> 8));
        const int far = uni(readlane_i(incl, 63));
        int nk = max(k + 64, far);
        if (vl) emit_leaves(vl, inf, wl, visit);
        k = uni(min(nk, root_end));
    }
}

// ------------------------------------------------------------------ LDS
struct GroupLds {
    int *cand;       // [T]
    uint64_t *masks; // [T/64 * gm]
    double *mx, *my, *mz, *mh; // [64]
    int *mi;         // [64]
    WalkLds wl;
    int *pend;       // [128]
};

__host__ __device__ constexpr size_t group_lds_bytes(int T, int gm)
{
    return (size_t)4 * T + (size_t)8 * (T / 64) * gm + 4 * 64 * 8 + 64 * 4 + (64 + 66 + 128) * 4;
}

__device__ __forceinline__ GroupLds carve(char *base, int T, int gm)
{
    GroupLds g;
    g.cand = (int *)base;
    g.masks = (uint64_t *)(base + 4 * T);
    g.mx = (double *)(g.masks + (T / 64) * gm);
    g.my = g.mx + 64;
    g.mz = g.my + 64;
    g.mh = g.mz + 64;
    g.mi = (int *)(g.mh + 64);
    g.wl.first = g.mi + 64;
    g.wl.pref = g.wl.first + 64;
    g.pend = g.wl.pref + 66;
    return g;
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

// candidate collection for a group ball; also records whether any kept
// candidate needed the periodic fold relative to the centre and the largest
// per-axis displacement of a kept candidate (lane-wise, see pair_wrap)
struct AppendCand {
    const double *x, *y, *z, *h;
    int *cand;
    int T;
    int n;
    bool over;
    bool folded;
    Ball B;
    double ext;
    __device__ bool stop() const { return over; }
    __device__ void operator()(int j, bool valid)
    {
        bool keep = false, fl = false;
        double e = 0.0;
        if (valid) {
            double rx = x[j] - B.cx, ry = y[j] - B.cy, rz = z[j] - B.cz;
            double dx = fold(rx, B.L), dy = fold(ry, B.L), dz = fold(rz, B.L);
            double r2 = __builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx));
            double lim = B.hydro ? sq((B.Rg + fmax(B.Hg, h[j])) * INFL) : B.W2;
            keep = r2 < lim;
            fl = (dx != rx) | (dy != ry) | (dz != rz);
            e = fmax(fabs(dx), fmax(fabs(dy), fabs(dz)));
        }
        if (keep) ext = fmax(ext, e);
        const uint64_t m = ballot(keep);
        if (ballot(keep && fl)) folded = true;
        const int cnt = popc64(m);
        if (n + cnt > T) {
            over = true;
            return;
        }
        if (keep) cand[n + mbcnt(m)] = j;
        n = uni(n + cnt);
    }
};

// FIFO of neighbour indices; the k-th pushed index is consumed by lane k%64
struct Fifo {
    int *buf; // [128]
    int np;
    template <class F> __device__ __forceinline__ void push(bool hit, int j, F &consume)
    {
        const uint64_t m = ballot(hit);
        if (hit) buf[np + mbcnt(m)] = j;
        np = uni(np + popc64(m));
        if (np >= 64) {
            wave_lds_sync();
            const int lane = lane_id();
            consume(buf[lane], true);
            const int rest = np - 64;
            int mv = lane < rest ? buf[64 + lane] : 0;
            wave_lds_sync();
            if (lane < rest) buf[lane] = mv;
            np = rest;
        }
    }
    template <class F> __device__ __forceinline__ void flush(F &consume)
    {
        wave_lds_sync();
        const int lane = lane_id();
        if (np > 0) {
            bool v = lane < np;
            consume(v ? buf[lane] : 0, v);
        }
        np = 0;
        wave_lds_sync();
    }
};

// ------------------------------------------------------------------ group set-up
struct GroupHead {
    int nm;          // members act[a .. a+nm)
    int i;           // this lane's member particle (lane < nm)
    bool mem;
    double xi, yi, zi, h;
    double cx, cy, cz, L;
    double d;        // |x_i - x_0|
    double R, H;     // max member distance, max member h
    bool mfold;      // some member needed the periodic fold
    double mext;     // largest per-axis |x_i - x_0| over members
    int root, root_end;
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

__device__ __forceinline__ GroupHead group_head(const Geom &geo, const GroupArg &ga, int g)
{
    GroupHead G;
    const int lane = lane_id();
    const int a = uni(ga.goff[g]);
    G.nm = min(uni(ga.goff[g + 1]) - a, 64);
    G.mem = lane < G.nm;
    G.i = G.mem ? ga.act[a + lane] : 0;
    const int i0 = uni(readlane_i(G.i, 0));
    const int b = geo.nb > 1 ? uni(box_of(geo.box_off, geo.nb, i0)) : 0;
    G.L = uni_d(geo.box_L[b]);
    G.root = uni(geo.box_root[b]);
    G.root_end = uni(geo.box_root[b + 1]);
    G.xi = G.yi = G.zi = G.h = 0.0;
    if (G.mem) {
        G.xi = geo.x[G.i];
        G.yi = geo.y[G.i];
        G.zi = geo.z[G.i];
        G.h = geo.h[G.i];
    }
    G.cx = uni_d(readlane_d(G.xi, 0));
    G.cy = uni_d(readlane_d(G.yi, 0));
    G.cz = uni_d(readlane_d(G.zi, 0));
    double rx = G.xi - G.cx, ry = G.yi - G.cy, rz = G.zi - G.cz;
    double dx = fold(rx, G.L), dy = fold(ry, G.L), dz = fold(rz, G.L);
    bool fl = G.mem && ((dx != rx) | (dy != ry) | (dz != rz));
    G.mfold = ballot(fl) != 0ull;
    G.mext = uni_d(wave_max_d(G.mem ? fmax(fabs(dx), fmax(fabs(dy), fabs(dz))) : 0.0));
    G.d = G.mem ? sqrt(__builtin_fma(dz, dz, __builtin_fma(dy, dy, dx * dx))) : 0.0;
    G.R = uni_d(wave_max_d(G.d));
    G.H = uni_d(wave_max_d(G.h));
    return G;
}

// filter pass: masks[ch*gm + m] for the members in `need`
//   mode 0: r2 < mh[m] (= h_m^2, density),  mode 1: j != i_m and r2 < max(h_m, h_j)^2
template <int MODE>
__device__ __forceinline__ void filter_pass(const Geom &geo, const GroupLds &S, int gm, int nc,
                                            uint64_t need, double L, bool wrap)
{
    const int lane = lane_id();
    const int nch = uni((nc + 63) >> 6);
    for (int ch = 0; ch < nch; ch++) {
        int slot = (ch << 6) + lane;
        bool v = slot < nc;
        int j = v ? S.cand[slot] : 0;
        double xj = geo.x[j], yj = geo.y[j], zj = geo.z[j];
        double hj = MODE == 1 ? geo.h[j] : 0.0;
        uint64_t mm = 0ull;
        uint64_t nd = need;
        while (nd) {
            const int m = ctz64(nd);
            nd &= nd - 1ull;
            double r2 = r2_of(xj, yj, zj, S.mx[m], S.my[m], S.mz[m], L, wrap);
            bool hit;
            if (MODE == 0) {
                hit = r2 < S.mh[m];
            } else {
                double hm = fmax(S.mh[m], hj);
                hit = (j != S.mi[m]) && (r2 < hm * hm);
            }
            mm = writelane_u64(mm, ballot(v && hit), m);
        }
        if ((need >> lane) & 1ull) S.masks[ch * gm + lane] = mm;
    }
    wave_lds_sync();
}

// stream the neighbours of member m (masks) through a FIFO into `consume`
template <class F>
__device__ __forceinline__ void consume_member(const GroupLds &S, int gm, int nc, int m, F &consume)
{
    const int lane = lane_id();
    const int nch = uni((nc + 63) >> 6);
    Fifo q{S.pend, 0};
    for (int ch = 0; ch < nch; ch++) {
        uint64_t M = S.masks[ch * gm + m];
        M = readlane_u64(M, 0);
        int slot = (ch << 6) + lane;
        bool hit = (M >> lane) & 1ull;
        int j = hit ? S.cand[slot] : 0;
        q.push(hit, j, consume);
    }
    q.flush(consume);
}

// counts |{j : r2 < h2}| over walked particles
struct CountVisit {
    const double *x, *y, *z;
    double xi, yi, zi, L, h2;
    int cnt;
    __device__ bool stop() const { return false; }
    __device__ void operator()(int j, bool valid)
    {
        bool hit = false;
        if (valid) hit = r2_of(x[j], y[j], z[j], xi, yi, zi, L, true) < h2;
        cnt = uni(cnt + popc64(ballot(hit)));
    }
};

// filter walked particles against one particle and push the neighbours
template <int MODE, class F> struct StreamVisit {
    const double *x, *y, *z, *h;
    double xi, yi, zi, L, hi;
    int i;
    Fifo q;
    F *consume;
    __device__ bool stop() const { return false; }
    __device__ void operator()(int j, bool valid)
    {
        bool hit = false;
        if (valid) {
            double r2 = r2_of(x[j], y[j], z[j], xi, yi, zi, L, true);
            if (MODE == 0) {
                hit = r2 < hi * hi;
            } else {
                double hm = fmax(hi, h[j]);
                hit = (j != i) && (r2 < hm * hm);
            }
        }
        q.push(hit, j, *consume);
    }
};

} // namespace

// ================================================================== density
struct DensK {
    Geom g;
    GroupArg ga;
    const float *m;
    float *rho, *fgrad;
    sfc_density_out out;
    DevStatus *st;
    int n_ngb, dn, max_iter, fixed_h;
    double skin;
};

namespace {

template <int KER, typename ACC> struct DensPair {
    const double *x, *y, *z;
    const float *m;
    double xi, yi, zi, L;
    bool wrap;
    ACC hinv;
    Kahan<ACC> sw, sd;
    __device__ void operator()(int j, bool valid)
    {
        if (!valid) return;
        double dxd = x[j] - xi, dyd = y[j] - yi, dzd = z[j] - zi;
        if (wrap) {
            dxd = fold(dxd, L);
            dyd = fold(dyd, L);
            dzd = fold(dzd, L);
        }
        ACC dx = (ACC)dxd, dy = (ACC)dyd, dz = (ACC)dzd;
        ACC r2 = mad(dz, dz, mad(dy, dy, dx * dx));
        ACC q = sqrt(r2) * hinv;
        ACC w, dw;
        kern_eval<KER, ACC>(q, w, dw);
        ACC mj = (ACC)m[j];
        sw.add(mj * w);
        sd.add(mj * mad(q, dw, ACC(3) * w));
    }
};

template <int KER, typename ACC>
__device__ __forceinline__ DensPair<KER, ACC> dens_pair(const DensK &k, double xi, double yi, double zi,
                                                        double h, double L, bool wrap)
{
    DensPair<KER, ACC> pp;
    pp.x = k.g.x;
    pp.y = k.g.y;
    pp.z = k.g.z;
    pp.m = k.m;
    pp.xi = xi;
    pp.yi = yi;
    pp.zi = zi;
    pp.L = L;
    pp.wrap = wrap;
    pp.hinv = (ACC)(1.0 / h);
    return pp;
}

template <int KER, typename ACC>
__device__ void dens_write(const DensK &k, int i, double h, int nn, int it, bool conv,
                           const DensPair<KER, ACC> &pp)
{
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
    atomicAdd(&k.st->sum_iters, (unsigned long long)it);
    if (!conv) atomicAdd(&k.st->n_not_converged, 1ull);
}

// one particle on its own: one walk per h evaluation, then the sums
template <int KER, typename ACC>
__device__ void dens_solo(const DensK &k, const GroupLds &S, int i, double h, double lo, double hi,
                          int it, double L, int root, int root_end)
{
    const double xi = uni_d(k.g.x[i]), yi = uni_d(k.g.y[i]), zi = uni_d(k.g.z[i]);
    int nn = 0;
    bool conv = false;
    for (int guard = 0; guard <= k.max_iter; guard++) {
        Ball B{xi, yi, zi, L, sq(h * INFL), 0.0, 0.0, 0};
        CountVisit cv{k.g.x, k.g.y, k.g.z, xi, yi, zi, L, h * h, 0};
        walk(k.g, root, root_end, B, S.wl, cv, k.st);
        if (lane_id() == 0) atomicAdd(&k.st->n_walks, 1ull);
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
    DensPair<KER, ACC> pp = dens_pair<KER, ACC>(k, xi, yi, zi, h, L, true);
    StreamVisit<0, DensPair<KER, ACC>> sv{k.g.x, k.g.y, k.g.z, k.g.h, xi, yi, zi, L, h, i,
                                          Fifo{S.pend, 0}, &pp};
    Ball B{xi, yi, zi, L, sq(h * INFL), 0.0, 0.0, 0};
    walk(k.g, root, root_end, B, S.wl, sv, k.st);
    sv.q.flush(pp);
    dens_write<KER, ACC>(k, i, h, nn, it, conv, pp);
}

} // namespace

template <int KER, typename ACC> __global__ __launch_bounds__(64) void k_density(DensK k)
{
    extern __shared__ __align__(16) char lds_raw[];
    const GroupLds S = carve(lds_raw, k.ga.T, k.ga.gm);
    const int lane = lane_id();
    const int G = uni(*k.ga.n_groups);
    const GroupRange gr = group_range(G);
    for (int g = gr.g; g < gr.end; g += gr.stride) {
        const GroupHead H = group_head(k.g, k.ga, g);
        const double cov = H.R + k.skin * H.H;
        Ball B{H.cx, H.cy, H.cz, H.L, sq(cov * INFL), 0.0, 0.0, 0};
        AppendCand ap{k.g.x, k.g.y, k.g.z, k.g.h, S.cand, k.ga.T, 0, false, false, B, 0.0};
        walk(k.g, H.root, H.root_end, B, S.wl, ap, k.st);
        if (lane == 0) {
            atomicAdd(&k.st->n_walks, 1ull);
            atomicAdd(&k.st->sum_cand, (unsigned long long)ap.n);
        }
        double h = H.h, lo = 0.0, hi = INFINITY;
        int it = 0, nn = 0;
        bool done = !H.mem, conv = false, solo = false;
        if (uni_b(ap.over)) {
            solo = H.mem;
            if (lane == 0) atomicAdd(&k.st->n_overflow, 1ull);
        } else {
            const int nc = uni(ap.n);
            const bool wrap = pair_wrap(uni_b(ap.folded), ap.ext, H.mfold, H.mext, H.L);
            const int nch = (nc + 63) >> 6;
            for (int pass = 0; pass <= k.max_iter; pass++) {
                if (!done && !solo && !(h + H.d <= cov)) solo = true;
                const uint64_t need = ballot(!done && !solo);
                if (!need) break;
                if ((need >> lane) & 1ull) {
                    S.mx[lane] = H.xi;
                    S.my[lane] = H.yi;
                    S.mz[lane] = H.zi;
                    S.mh[lane] = h * h;
                }
                wave_lds_sync();
                filter_pass<0>(k.g, S, k.ga.gm, nc, need, H.L, wrap);
                if ((need >> lane) & 1ull) {
                    int cnt = 0;
                    for (int ch = 0; ch < nch; ch++) cnt += popc64(S.masks[ch * k.ga.gm + lane]);
                    nn = cnt;
                    it++;
                    if (k.fixed_h || (cnt >= k.n_ngb - k.dn && cnt <= k.n_ngb + k.dn)) {
                        done = true;
                        conv = true;
                    } else if (it >= k.max_iter) {
                        done = true;
                    } else {
                        h = h_step(cnt, k.n_ngb, k.dn, h, lo, hi);
                    }
                }
                if (pass == k.max_iter) guard_hit(k.st);
            }
            uint64_t fin = ballot(done && H.mem);
            while (fin) {
                const int m = ctz64(fin);
                fin &= fin - 1ull;
                const double hm = uni_d(readlane_d(h, m));
                DensPair<KER, ACC> pp = dens_pair<KER, ACC>(k, uni_d(readlane_d(H.xi, m)),
                                                            uni_d(readlane_d(H.yi, m)),
                                                            uni_d(readlane_d(H.zi, m)), hm, H.L, wrap);
                consume_member(S, k.ga.gm, nc, m, pp);
                dens_write<KER, ACC>(k, uni(readlane_i(H.i, m)), hm, uni(readlane_i(nn, m)),
                                     uni(readlane_i(it, m)), ballot(conv && lane == m) != 0ull, pp);
            }
        }
        // members that left the superset finish alone, in this wave
        uint64_t rest = ballot(solo);
        if (rest && lane == 0) atomicAdd(&k.st->n_deferred, (unsigned long long)popc64(rest));
        while (rest) {
            const int m = ctz64(rest);
            rest &= rest - 1ull;
            dens_solo<KER, ACC>(k, S, uni(readlane_i(H.i, m)), uni_d(readlane_d(h, m)),
                                uni_d(readlane_d(lo, m)), uni_d(readlane_d(hi, m)),
                                uni(readlane_i(it, m)), H.L, H.root, H.root_end);
        }
    }
}

// ================================================================== hydro
struct HydroK {
    Geom g;
    GroupArg ga;
    const float *m, *vx, *vy, *vz, *u, *rho, *fgrad, *pf, *cs;
    sfc_hydro_out out;
    DevStatus *st;
    double gamma, alpha;
};

namespace {
template <int KER, typename ACC> struct HydroPair {
    const HydroK *k;
    double xi, yi, zi, L;
    bool wrap;
    ACC hinv, hinv4, vx, vy, vz, rho, pf, cs;
    Kahan<ACC> ax, ay, az, du;
    ACC vmax;
    __device__ void operator()(int j, bool valid)
    {
        if (!valid) return;
        constexpr ACC C = (ACC)knorm<KER>();
        double dxd = xi - k->g.x[j], dyd = yi - k->g.y[j], dzd = zi - k->g.z[j];
        if (wrap) {
            dxd = fold(dxd, L);
            dyd = fold(dyd, L);
            dzd = fold(dzd, L);
        }
        ACC dx = (ACC)dxd, dy = (ACC)dyd, dz = (ACC)dzd;
        ACC r2 = mad(dz, dz, mad(dy, dy, dx * dx));
        ACC r = sqrt(r2);
        ACC rinv = r > ACC(0) ? ACC(1) / r : ACC(0);
        ACC w, dwi, dwj;
        kern_eval<KER, ACC>(r * hinv, w, dwi);
        ACC hjinv = ACC(1) / (ACC)k->g.h[j];
        kern_eval<KER, ACC>(r * hjinv, w, dwj);
        ACC hj2 = hjinv * hjinv;
        ACC dWi = C * dwi * hinv4;
        ACC dWj = C * dwj * (hj2 * hj2);
        ACC dWb = ACC(0.5) * (dWi + dWj);
        ACC rhoj = (ACC)k->rho[j];
        ACC pfj, csj;
        if (sizeof(ACC) == 8) {
            double gm1 = k->gamma - 1.0;
            double uj = k->u[j];
            pfj = (ACC)(k->fgrad[j] * gm1 * uj / (double)k->rho[j]);
            csj = (ACC)sqrt(k->gamma * gm1 * uj);
        } else {
            pfj = (ACC)k->pf[j];
            csj = (ACC)k->cs[j];
        }
        ACC vdx = vx - (ACC)k->vx[j], vdy = vy - (ACC)k->vy[j], vdz = vz - (ACC)k->vz[j];
        ACC vr = mad(vdz, dz, mad(vdy, dy, vdx * dx));
        ACC wij = vr < ACC(0) ? vr * rinv : ACC(0);
        ACC vsig = cs + csj - ACC(3) * wij;
        ACC visc = -(ACC)k->alpha * vsig * wij / (rho + rhoj);
        ACC mj = (ACC)k->m[j];
        ACC fac = mj * (pf * dWi + pfj * dWj + visc * dWb);
        ACC fr = fac * rinv;
        ax.add(-fr * dx);
        ay.add(-fr * dy);
        az.add(-fr * dz);
        du.add(mj * (pf * dWi + ACC(0.5) * visc * dWb) * vr * rinv);
        vmax = vsig > vmax ? vsig : vmax;
    }
};

template <int KER, typename ACC>
__device__ __forceinline__ HydroPair<KER, ACC> hydro_pair(const HydroK &k, int i, double xi, double yi,
                                                          double zi, double h, double L, bool wrap)
{
    HydroPair<KER, ACC> hp;
    hp.k = &k;
    hp.xi = xi;
    hp.yi = yi;
    hp.zi = zi;
    hp.L = L;
    hp.wrap = wrap;
    double hinv = 1.0 / h;
    hp.hinv = (ACC)hinv;
    hp.hinv4 = (ACC)(hinv * hinv * hinv * hinv);
    hp.vx = (ACC)k.vx[i];
    hp.vy = (ACC)k.vy[i];
    hp.vz = (ACC)k.vz[i];
    hp.rho = (ACC)k.rho[i];
    double gm1 = k.gamma - 1.0;
    double u = k.u[i];
    hp.pf = (ACC)(k.fgrad[i] * gm1 * u / (double)k.rho[i]);
    hp.cs = (ACC)sqrt(k.gamma * gm1 * u);
    hp.vmax = ACC(0);
    return hp;
}

template <int KER, typename ACC>
__device__ void hydro_write(const HydroK &k, int i, const HydroPair<KER, ACC> &hp)
{
    double ax = (double)wave_sum_f_or_d(hp.ax.value());
    double ay = (double)wave_sum_f_or_d(hp.ay.value());
    double az = (double)wave_sum_f_or_d(hp.az.value());
    double du = (double)wave_sum_f_or_d(hp.du.value());
    ACC vm = hp.vmax;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        ACC t = __shfl_xor(vm, o, 64);
        vm = t > vm ? t : vm;
    }
    if (lane_id() != 0) return;
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

template <int KER, typename ACC>
__device__ void hydro_solo(const HydroK &k, const GroupLds &S, int i, double L, int root, int root_end)
{
    const double xi = uni_d(k.g.x[i]), yi = uni_d(k.g.y[i]), zi = uni_d(k.g.z[i]);
    const double h = uni_d(k.g.h[i]);
    HydroPair<KER, ACC> hp = hydro_pair<KER, ACC>(k, i, xi, yi, zi, h, L, true);
    StreamVisit<1, HydroPair<KER, ACC>> sv{k.g.x, k.g.y, k.g.z, k.g.h, xi, yi, zi, L, h, i,
                                           Fifo{S.pend, 0}, &hp};
    Ball B{xi, yi, zi, L, 0.0, 0.0, h, 1};
    walk(k.g, root, root_end, B, S.wl, sv, k.st);
    if (lane_id() == 0) atomicAdd(&k.st->n_walks, 1ull);
    sv.q.flush(hp);
    hydro_write<KER, ACC>(k, i, hp);
}
} // namespace

__global__ void k_hydro_prep(int64_t n, const float *__restrict__ rho,
                             const float *__restrict__ fgrad, const float *__restrict__ u,
                             double gamma, float *__restrict__ pf, float *__restrict__ cs)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double gm1 = gamma - 1.0;
    double uu = u[i];
    pf[i] = (float)(fgrad[i] * gm1 * uu / (double)rho[i]);
    cs[i] = (float)sqrt(gamma * gm1 * uu);
}

template <int KER, typename ACC> __global__ __launch_bounds__(64) void k_hydro(HydroK k)
{
    extern __shared__ __align__(16) char lds_raw[];
    const GroupLds S = carve(lds_raw, k.ga.T, k.ga.gm);
    const int lane = lane_id();
    const int G = uni(*k.ga.n_groups);
    const GroupRange gr = group_range(G);
    for (int g = gr.g; g < gr.end; g += gr.stride) {
        const GroupHead H = group_head(k.g, k.ga, g);
        Ball B{H.cx, H.cy, H.cz, H.L, 0.0, H.R, H.H, 1};
        AppendCand ap{k.g.x, k.g.y, k.g.z, k.g.h, S.cand, k.ga.T, 0, false, false, B, 0.0};
        walk(k.g, H.root, H.root_end, B, S.wl, ap, k.st);
        if (lane == 0) {
            atomicAdd(&k.st->n_walks, 1ull);
            atomicAdd(&k.st->sum_cand, (unsigned long long)ap.n);
        }
        const uint64_t need = ballot(H.mem);
        if (uni_b(ap.over)) {
            if (lane == 0) {
                atomicAdd(&k.st->n_overflow, 1ull);
                atomicAdd(&k.st->n_deferred, (unsigned long long)popc64(need));
            }
            uint64_t rest = need;
            while (rest) {
                const int m = ctz64(rest);
                rest &= rest - 1ull;
                hydro_solo<KER, ACC>(k, S, uni(readlane_i(H.i, m)), H.L, H.root, H.root_end);
            }
            continue;
        }
        const int nc = uni(ap.n);
        const bool wrap = pair_wrap(uni_b(ap.folded), ap.ext, H.mfold, H.mext, H.L);
        if (H.mem) {
            S.mx[lane] = H.xi;
            S.my[lane] = H.yi;
            S.mz[lane] = H.zi;
            S.mh[lane] = H.h;
            S.mi[lane] = H.i;
        }
        wave_lds_sync();
        filter_pass<1>(k.g, S, k.ga.gm, nc, need, H.L, wrap);
        uint64_t fin = need;
        while (fin) {
            const int m = ctz64(fin);
            fin &= fin - 1ull;
            const int im = uni(readlane_i(H.i, m));
            HydroPair<KER, ACC> hp = hydro_pair<KER, ACC>(
                k, im, uni_d(readlane_d(H.xi, m)), uni_d(readlane_d(H.yi, m)),
                uni_d(readlane_d(H.zi, m)), uni_d(readlane_d(H.h, m)), H.L, wrap);
            consume_member(S, k.ga.gm, nc, m, hp);
            hydro_write<KER, ACC>(k, im, hp);
        }
    }
}

// ================================================================== verify
struct VerK {
    Geom g;
    GroupArg ga;
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
    const double *x, *y, *z, *h;
    double xi, yi, zi, L, hi;
    int i, mode;
    VerifyAcc *va;
    __device__ bool stop() const { return false; }
    __device__ void operator()(int j, bool valid)
    {
        bool hit = false;
        if (valid) {
            double r2 = r2_of(x[j], y[j], z[j], xi, yi, zi, L, true);
            if (mode == 0) {
                hit = r2 < hi * hi;
            } else {
                double hm = fmax(hi, h[j]);
                hit = (j != i) && (r2 < hm * hm);
            }
        }
        (*va)(j, hit);
    }
};

__device__ void verify_solo(const VerK &k, const GroupLds &S, int i, double L, int root, int root_end)
{
    const double xi = uni_d(k.g.x[i]), yi = uni_d(k.g.y[i]), zi = uni_d(k.g.z[i]);
    const double h = uni_d(k.g.h[i]);
    VerifyAcc va = verify_init(k, i);
    VerVisit vv{k.g.x, k.g.y, k.g.z, k.g.h, xi, yi, zi, L, h, i, k.ver.mode, &va};
    Ball B = k.ver.mode == 0 ? Ball{xi, yi, zi, L, sq(h * INFL), 0.0, 0.0, 0}
                             : Ball{xi, yi, zi, L, 0.0, 0.0, h, 1};
    walk(k.g, root, root_end, B, S.wl, vv, k.st);
    verify_write(k, i, va);
}
} // namespace

__global__ __launch_bounds__(64) void k_verify(VerK k)
{
    extern __shared__ __align__(16) char lds_raw[];
    const GroupLds S = carve(lds_raw, k.ga.T, k.ga.gm);
    const int lane = lane_id();
    const int G = uni(*k.ga.n_groups);
    const int mode = k.ver.mode;
    const GroupRange gr = group_range(G);
    for (int g = gr.g; g < gr.end; g += gr.stride) {
        const GroupHead H = group_head(k.g, k.ga, g);
        const double cov = H.R + H.H;
        Ball B = mode == 0 ? Ball{H.cx, H.cy, H.cz, H.L, sq(cov * INFL), 0.0, 0.0, 0}
                           : Ball{H.cx, H.cy, H.cz, H.L, 0.0, H.R, H.H, 1};
        AppendCand ap{k.g.x, k.g.y, k.g.z, k.g.h, S.cand, k.ga.T, 0, false, false, B, 0.0};
        walk(k.g, H.root, H.root_end, B, S.wl, ap, k.st);
        if (lane == 0) {
            atomicAdd(&k.st->n_walks, 1ull);
            atomicAdd(&k.st->sum_cand, (unsigned long long)ap.n);
        }
        const uint64_t need = ballot(H.mem);
        if (uni_b(ap.over)) {
            if (lane == 0) atomicAdd(&k.st->n_overflow, 1ull);
            uint64_t rest = need;
            while (rest) {
                const int m = ctz64(rest);
                rest &= rest - 1ull;
                verify_solo(k, S, uni(readlane_i(H.i, m)), H.L, H.root, H.root_end);
            }
            continue;
        }
        const int nc = uni(ap.n);
        const bool wrap = pair_wrap(uni_b(ap.folded), ap.ext, H.mfold, H.mext, H.L);
        if (H.mem) {
            S.mx[lane] = H.xi;
            S.my[lane] = H.yi;
            S.mz[lane] = H.zi;
            S.mh[lane] = mode == 0 ? H.h * H.h : H.h;
            S.mi[lane] = H.i;
        }
        wave_lds_sync();
        if (mode == 0) filter_pass<0>(k.g, S, k.ga.gm, nc, need, H.L, wrap);
        else filter_pass<1>(k.g, S, k.ga.gm, nc, need, H.L, wrap);
        uint64_t fin = need;
        const int nch = (nc + 63) >> 6;
        while (fin) {
            const int m = ctz64(fin);
            fin &= fin - 1ull;
            const int im = uni(readlane_i(H.i, m));
            VerifyAcc va = verify_init(k, im);
            for (int ch = 0; ch < nch; ch++) {
                uint64_t M = readlane_u64(S.masks[ch * k.ga.gm + m], 0);
                bool hit = (M >> lane) & 1ull;
                va(hit ? S.cand[(ch << 6) + lane] : 0, hit);
            }
            verify_write(k, im, va);
        }
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
    g.box_root = t.box_root;
    g.nb = p.nb;
    return g;
}

GroupArg make_groups(const GroupBufs &gb, int T, int gm)
{
    GroupArg a;
    a.act = gb.act;
    a.goff = gb.goff;
    a.n_groups = gb.n_groups;
    a.T = T;
    a.gm = gm;
    return a;
}

// waves: as many as fit on the chip at once (a multiple of 8, one per
// workgroup), so that every wave is resident and keeps its XCD's groups
template <class Kern>
int64_t wave_count(Kern kern, size_t lds, int cu, int64_t max_groups)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 8;
    int64_t w = (int64_t)cu * per_cu;
    int64_t cap = ((max_groups + 7) / 8) * 8;
    if (cap < w) w = cap;
    w = (w / 8) * 8;
    return w < 8 ? 8 : w;
}

template <class Kern, class Arg>
hipError_t launch_waves(Kern kern, hipStream_t s, const Arg &a, size_t lds, int cu, int64_t max_groups)
{
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    kern<<<(unsigned)wave_count(kern, lds, cu, max_groups), 64, lds, s>>>(a);
    return hipGetLastError();
}
} // namespace

hipError_t launch_density(hipStream_t s, const PartDev &p, const TreeDev &t, const GroupBufs &g,
                          SearchBufs &sb, const DensityArgs &a, DevStatus *st, int gm)
{
    const sfc_density_params &dp = a.dp;
    DensK k;
    memset(&k, 0, sizeof(k));
    k.g = make_geom(p, t);
    k.ga = make_groups(g, dp.t_cand, gm);
    k.m = p.m;
    k.rho = p.rho;
    k.fgrad = p.fgrad;
    k.out = a.out;
    k.st = st;
    k.n_ngb = dp.n_ngb;
    k.dn = dp.dn;
    k.max_iter = dp.max_iter;
    k.fixed_h = dp.fixed_h;
    k.skin = dp.skin;
    const size_t lds = group_lds_bytes(dp.t_cand, gm);
    const int64_t n = p.n;
    if (dp.kernel == 0 && dp.accum == SFC_ACCUM_F32)
        return launch_waves(k_density<0, float>, s, k, lds, sb.cu_count, n);
    if (dp.kernel == 0) return launch_waves(k_density<0, double>, s, k, lds, sb.cu_count, n);
    if (dp.accum == SFC_ACCUM_F32) return launch_waves(k_density<1, float>, s, k, lds, sb.cu_count, n);
    return launch_waves(k_density<1, double>, s, k, lds, sb.cu_count, n);
}

hipError_t launch_hydro(hipStream_t s, const PartDev &p, const TreeDev &t, const GroupBufs &g,
                        SearchBufs &sb, const HydroArgs &a, DevStatus *st, int gm)
{
    const sfc_hydro_params &hp = a.hp;
    k_hydro_prep<<<(unsigned)((p.n + 255) / 256), 256, 0, s>>>(p.n, p.rho, p.fgrad, p.u, hp.gamma,
                                                               sb.pf, sb.cs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    HydroK k;
    memset(&k, 0, sizeof(k));
    k.g = make_geom(p, t);
    k.ga = make_groups(g, hp.t_cand, gm);
    k.m = p.m;
    k.vx = p.vx;
    k.vy = p.vy;
    k.vz = p.vz;
    k.u = p.u;
    k.rho = p.rho;
    k.fgrad = p.fgrad;
    k.pf = sb.pf;
    k.cs = sb.cs;
    k.out = a.out;
    k.st = st;
    k.gamma = hp.gamma;
    k.alpha = hp.alpha;
    const size_t lds = group_lds_bytes(hp.t_cand, gm);
    const int64_t n = p.n;
    if (hp.kernel == 0 && hp.accum == SFC_ACCUM_F32)
        return launch_waves(k_hydro<0, float>, s, k, lds, sb.cu_count, n);
    if (hp.kernel == 0) return launch_waves(k_hydro<0, double>, s, k, lds, sb.cu_count, n);
    if (hp.accum == SFC_ACCUM_F32) return launch_waves(k_hydro<1, float>, s, k, lds, sb.cu_count, n);
    return launch_waves(k_hydro<1, double>, s, k, lds, sb.cu_count, n);
}

hipError_t launch_verify(hipStream_t s, const PartDev &p, const TreeDev &t, const GroupBufs &g,
                         SearchBufs &sb, const sfc_verify &v, int t_cand, DevStatus *st, int gm)
{
    VerK k;
    memset(&k, 0, sizeof(k));
    k.g = make_geom(p, t);
    k.ga = make_groups(g, t_cand, gm);
    k.ver = v;
    k.orig = p.orig;
    k.st = st;
    return launch_waves(k_verify, s, k, group_lds_bytes(t_cand, gm), sb.cu_count, p.n);
}
