// sort.hip -- Peano-Hilbert keys, stable LSD radix sort of (key, index),
// gather of the particle arrays, and the device-wide exclusive scan used by
// every compaction in the library.
#include "internal.h"

// ------------------------------------------------------------------ keys
// Spread the low 21 bits of v to every third bit position (bit k -> 3k).
__device__ __forceinline__ uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// Hilbert index of cell (a0, a1, a2), 21 bits per axis: Skilling's
// transposition of the axes (AIP Conf. Proc. 707, 2004), written
// branch-free, then the three transposed words are bit-interleaved with
// axis 0 in the most significant position of every 3-bit digit.
__device__ __forceinline__ uint64_t hilbert_key63(uint32_t a0, uint32_t a1, uint32_t a2)
{
#pragma unroll
    for (int b = SFC_KEY_BITS - 1; b >= 1; --b) {
        const uint32_t Q = 1u << b, P = Q - 1u;
        // axis 0 against itself: invert low bits when its bit b is set
        a0 ^= P & (0u - ((a0 >> b) & 1u));
        // axis 1: invert a0's low bits if set, else exchange low bits with a0
        uint32_t s1 = 0u - ((a1 >> b) & 1u);
        uint32_t t1 = (a0 ^ a1) & P & ~s1;
        a0 ^= t1 ^ (P & s1);
        a1 ^= t1;
        uint32_t s2 = 0u - ((a2 >> b) & 1u);
        uint32_t t2 = (a0 ^ a2) & P & ~s2;
        a0 ^= t2 ^ (P & s2);
        a2 ^= t2;
    }
    // Gray code across the axes
    a1 ^= a0;
    a2 ^= a1;
    // bit k of t = parity of the bits of a2 above k
    uint32_t t = a2 >> 1;
    t ^= t >> 1;
    t ^= t >> 2;
    t ^= t >> 4;
    t ^= t >> 8;
    t ^= t >> 16;
    a0 ^= t;
    a1 ^= t;
    a2 ^= t;
    return (spread3(a0) << 2) | (spread3(a1) << 1) | spread3(a2);
}


// Keys, the sort payload (input index, with the active flag in bit 31: n <
// 2^30) and the particle's 64-byte record: the fields are read here once, in
// input order and coalesced, so that the gather after the sort fetches one
// record per particle instead of one cache line per field.
__global__ void k_keys(int64_t n, int nb, const int64_t *__restrict__ box_off,
                       const double *__restrict__ box_L, const sfc_particles in,
                       uint64_t *__restrict__ key, uint32_t *__restrict__ val,
                       uint32_t *__restrict__ boxid, PRec *__restrict__ rec)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = nb > 1 ? box_of(box_off, nb, i) : 0;
    double L = box_L[b];
    const double x = in.x[i], y = in.y[i], z = in.z[i];
    key[i] = hilbert_key63(key_cell(x, L), key_cell(y, L), key_cell(z, L));
    val[i] = (uint32_t)i | (in.active[i] ? 0x80000000u : 0u);
    if (boxid) boxid[i] = (uint32_t)b;
    PRec r;
    r.x = x;
    r.y = y;
    r.z = z;
    r.h = in.h[i];
    r.m = in.m[i];
    r.vx = in.vx ? in.vx[i] : 0.0f;
    r.vy = in.vy ? in.vy[i] : 0.0f;
    r.vz = in.vz ? in.vz[i] : 0.0f;
    r.u = in.u ? in.u[i] : 0.0f;
    r.rho = in.rho ? in.rho[i] : 0.0f;
    r.fgrad = in.fgrad ? in.fgrad[i] : 0.0f;
    r.orig = in.orig ? in.orig[i] : (uint32_t)i;
    rec[i] = r;
}

hipError_t launch_keys(hipStream_t s, const sfc_particles *in, SortBufs &b)
{
    int64_t n = in->n;
    int blocks = (int)((n + 255) / 256);
    k_keys<<<blocks, 256, 0, s>>>(n, in->n_boxes, in->box_off, in->box_L, *in, b.key_a, b.val_a,
                                  in->n_boxes > 1 ? b.box_a : nullptr, b.rec);
    return hipGetLastError();
}

// ------------------------------------------------------------------ scan
constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 8;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;

// exclusive scan of one 2048-element tile; tile total to sums[blockIdx]
__global__ void k_scan_tile(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                            int64_t n, uint32_t *__restrict__ sums)
{
    __shared__ uint32_t wtot[SC_THREADS / 64];
    int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
    uint32_t v[SC_ITEMS];
    uint32_t run = 0;
#pragma unroll
    for (int k = 0; k < SC_ITEMS; k++) {
        int64_t i = base + k;
        uint32_t a = i < n ? in[i] : 0u;
        v[k] = run;
        run += a;
    }
    // inclusive scan of per-thread totals within the wave
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) wtot[w] = inc;
    __syncthreads();
    uint32_t woff = 0;
    for (int k = 0; k < w; k++) woff += wtot[k];
    uint32_t excl = woff + inc - run;
#pragma unroll
    for (int k = 0; k < SC_ITEMS; k++) {
        int64_t i = base + k;
        if (i < n) out[i] = v[k] + excl;
    }
    if (threadIdx.x == SC_THREADS - 1 && sums) {
        uint32_t t = 0;
        for (int k = 0; k < SC_THREADS / 64; k++) t += wtot[k];
        sums[blockIdx.x] = t;
    }
}

__global__ void k_scan_add(uint32_t *__restrict__ out, int64_t n, const uint32_t *__restrict__ add)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += add[i / SC_TILE];
}

__global__ void k_scan_total(const uint32_t *__restrict__ in, const uint32_t *__restrict__ out,
                             int64_t n, uint32_t *__restrict__ total)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *total = n > 0 ? out[n - 1] + in[n - 1] : 0u;
}

size_t scan_tmp_elems(int64_t n)
{
    size_t t = 0;
    while (n > SC_TILE) {
        n = (n + SC_TILE - 1) / SC_TILE;
        t += 2 * (size_t)n;
    }
    return t + 2;
}

static hipError_t scan_rec(hipStream_t s, const uint32_t *in, uint32_t *out, int64_t n,
                           uint32_t *tmp)
{
    int64_t nblk = (n + SC_TILE - 1) / SC_TILE;
    if (nblk <= 1) {
        k_scan_tile<<<1, SC_THREADS, 0, s>>>(in, out, n, nullptr);
        return hipGetLastError();
    }
    uint32_t *sums = tmp, *ssum = tmp + nblk;
    k_scan_tile<<<(unsigned)nblk, SC_THREADS, 0, s>>>(in, out, n, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_rec(s, sums, ssum, nblk, tmp + 2 * nblk);
    if (e != hipSuccess) return e;
    k_scan_add<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(out, n, ssum);
    return hipGetLastError();
}

hipError_t launch_scan_excl_u32(hipStream_t s, const uint32_t *in, uint32_t *out, int64_t n,
                                uint32_t *tmp, uint32_t *total)
{
    if (n <= 0) return hipSuccess;
    hipError_t e = scan_rec(s, in, out, n, tmp);
    if (e != hipSuccess) return e;
    if (total) {
        k_scan_total<<<1, 64, 0, s>>>(in, out, n, total);
        e = hipGetLastError();
    }
    return e;
}

__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(hipStream_t s, int32_t *p, int32_t v, int64_t n)
{
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ radix sort
// 8-bit digits, tiles of 4096 keys (256 threads x 16 rounds).  Pass =
// per-tile digit histogram, one exclusive scan over the digit-major table,
// then a stable scatter in which every round of 256 keys is ranked with
// wave-level digit matching (eight ballots) and per-wave digit counters.
constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;

__device__ __forceinline__ uint32_t rs_digit(const uint64_t *key, const uint32_t *boxk,
                                             int64_t i, int shift)
{
    return boxk ? (boxk[i] >> shift) & 255u : (uint32_t)(key[i] >> shift) & 255u;
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint64_t *__restrict__ key,
                                                        const uint32_t *__restrict__ boxk,
                                                        int64_t n, int shift,
                                                        uint32_t *__restrict__ hist,
                                                        int ntiles)
{
    __shared__ uint32_t cnt[4][256];
    int t = threadIdx.x, w = t >> 6;
    for (int k = 0; k < 4; k++) cnt[k][t] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; r++) {
        int64_t i = base + r * RS_THREADS + t;
        if (i < n) atomicAdd(&cnt[w][rs_digit(key, boxk, i, shift)], 1u);
    }
    __syncthreads();
    hist[(int64_t)t * ntiles + blockIdx.x] = cnt[0][t] + cnt[1][t] + cnt[2][t] + cnt[3][t];
}

// Stable scatter of one tile: wave w owns the tile's keys [1024 w, 1024 w +
// 1024) and ranks them round by round (64 keys, eight ballots find the lanes
// with the same digit) against a wave-private running count per digit; the
// tile-local position of a key is then its digit's start in the tile + the
// counts of the earlier waves + its rank in the wave.  Keys go to LDS in
// that order and leave in it, so consecutive threads write consecutive
// addresses of a digit's run.
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(
    const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    const uint32_t *__restrict__ bin, uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
    uint32_t *__restrict__ bout, int64_t n, int shift, int box_pass,
    const uint32_t *__restrict__ offs, int ntiles)
{
    constexpr int PER_WAVE = RS_TILE / (RS_THREADS / 64); // 1024 keys
    constexpr int WR = PER_WAVE / 64;                     // 16 rounds
    __shared__ uint64_t lk[RS_TILE];
    __shared__ uint32_t lv[RS_TILE];
    __shared__ uint32_t lb[RS_TILE];
    __shared__ uint32_t cntw[RS_THREADS / 64][256];
    __shared__ uint32_t dstart[256];
    __shared__ uint32_t gbase[256];
    __shared__ uint32_t wsum[RS_THREADS / 64];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const int tile_n = (int)(n - base < RS_TILE ? n - base : RS_TILE);
    gbase[t] = offs[(int64_t)t * ntiles + blockIdx.x];
    for (int k = 0; k < RS_THREADS / 64; k++) cntw[k][t] = 0;
    __syncthreads();
    uint64_t kk[WR];
    uint32_t vv[WR], bb[WR], dd[WR], rk[WR];
#pragma unroll
    for (int r = 0; r < WR; r++) {
        const int li = w * PER_WAVE + r * 64 + lane;
        const bool valid = li < tile_n;
        kk[r] = valid ? kin[base + li] : 0ull;
        vv[r] = valid ? vin[base + li] : 0u;
        bb[r] = (valid && bin) ? bin[base + li] : 0u;
    }
#pragma unroll
    for (int r = 0; r < WR; r++) {
        const int li = w * PER_WAVE + r * 64 + lane;
        const bool valid = li < tile_n;
        const uint32_t d = box_pass ? (bb[r] >> shift) & 255u : (uint32_t)(kk[r] >> shift) & 255u;
        uint64_t peers = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = ballot(bit);
            peers &= bit ? m : ~m;
        }
        const int rank = mbcnt(peers);
        const uint32_t before = valid ? cntw[w][d] : 0u;
        wave_lds_sync();
        if (valid && rank == 0) cntw[w][d] = before + (uint32_t)popc64(peers);
        wave_lds_sync();
        dd[r] = d;
        rk[r] = before + (uint32_t)rank;
    }
    __syncthreads();
    // digit d = thread t: counts of the waves before each wave, the tile
    // total, and its exclusive scan over the digits
    uint32_t tot = 0;
    for (int k = 0; k < RS_THREADS / 64; k++) {
        const uint32_t c = cntw[k][t];
        cntw[k][t] = tot;
        tot += c;
    }
    uint32_t inc = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t woff = 0;
    for (int k = 0; k < w; k++) woff += wsum[k];
    dstart[t] = woff + inc - tot;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < WR; r++) {
        const int li = w * PER_WAVE + r * 64 + lane;
        if (li < tile_n) {
            const uint32_t lp = dstart[dd[r]] + cntw[w][dd[r]] + rk[r];
            lk[lp] = kk[r];
            lv[lp] = vv[r];
            lb[lp] = bb[r];
        }
    }
    __syncthreads();
    for (int j = t; j < tile_n; j += RS_THREADS) {
        const uint64_t k = lk[j];
        const uint32_t bx = lb[j];
        const uint32_t d = box_pass ? (bx >> shift) & 255u : (uint32_t)(k >> shift) & 255u;
        const uint32_t pos = gbase[d] + (uint32_t)j - dstart[d];
        kout[pos] = k;
        vout[pos] = lv[j];
        if (bout) bout[pos] = bx;
    }
}

hipError_t launch_radix_sort(hipStream_t s, int64_t n, int nb, SortBufs &b, uint64_t *keys_out,
                             uint32_t **perm_out)
{
    int ntiles = (int)((n + RS_TILE - 1) / RS_TILE);
    // digit passes: 8 over the key, then 1 or 2 over the box id (stable)
    struct Pass { int shift; int box; };
    Pass passes[10];
    int np = 0;
    for (int sh = 0; sh < 64; sh += 8) passes[np++] = {sh, 0};
    if (nb > 1) {
        passes[np++] = {0, 1};
        if (nb > 256) passes[np++] = {8, 1};
    }
    uint64_t *ka = b.key_a, *kb = b.key_b;
    uint32_t *va = b.val_a, *vb = b.val_b;
    uint32_t *ba = nb > 1 ? b.box_a : nullptr, *bbx = nb > 1 ? b.box_b : nullptr;
    for (int p = 0; p < np; p++) {
        bool last = p == np - 1;
        uint64_t *ko = last ? keys_out : kb;
        uint32_t *vo = vb;
        const uint32_t *digit_box = passes[p].box ? ba : nullptr;
        k_rs_hist<<<ntiles, RS_THREADS, 0, s>>>(ka, digit_box, n, passes[p].shift, b.hist,
                                                ntiles);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = launch_scan_excl_u32(s, b.hist, b.hist + (size_t)256 * ntiles, (int64_t)256 * ntiles,
                                 b.scan_tmp, nullptr);
        if (e != hipSuccess) return e;
        k_rs_scatter<<<ntiles, RS_THREADS, 0, s>>>(ka, va, ba, ko, vo, bbx, n, passes[p].shift,
                                                   passes[p].box,
                                                   b.hist + (size_t)256 * ntiles, ntiles);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (!last) {
            std::swap(ka, kb);
            std::swap(va, vb);
            std::swap(ba, bbx);
        } else {
            *perm_out = vo;
        }
    }
    return hipSuccess;
}

// ------------------------------------------------------------------ gather
// One record per output slot: the sorted order of every field, the active
// flag from the payload's bit 31 (written as 0 / 1), the input index.
__global__ void k_gather(int64_t n, const uint32_t *__restrict__ perm, const PRec *__restrict__ rec,
                         sfc_particles out, uint32_t has, uint32_t *__restrict__ perm_out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t v = perm[i];
    const uint32_t j = v & 0x7fffffffu;
    const PRec r = rec[j];
    out.x[i] = r.x;
    out.y[i] = r.y;
    out.z[i] = r.z;
    out.h[i] = r.h;
    out.m[i] = r.m;
    if (has & 1u) out.vx[i] = r.vx;
    if (has & 2u) out.vy[i] = r.vy;
    if (has & 4u) out.vz[i] = r.vz;
    if (has & 8u) out.u[i] = r.u;
    if (has & 16u) out.rho[i] = r.rho;
    if (has & 32u) out.fgrad[i] = r.fgrad;
    if (has & 64u) out.orig[i] = r.orig;
    out.active[i] = (uint8_t)(v >> 31);
    if (perm_out) perm_out[i] = j;
}

hipError_t launch_gather(hipStream_t s, const sfc_particles *in, sfc_particles *out,
                         const uint32_t *perm, const PRec *rec, uint32_t *perm_out)
{
    // a field is written when both sides have it (x, y, z, h, m and active
    // always do); orig is written whenever out has it
    const uint32_t has = (in->vx && out->vx ? 1u : 0u) | (in->vy && out->vy ? 2u : 0u) |
                         (in->vz && out->vz ? 4u : 0u) | (in->u && out->u ? 8u : 0u) |
                         (in->rho && out->rho ? 16u : 0u) | (in->fgrad && out->fgrad ? 32u : 0u) |
                         (out->orig ? 64u : 0u);
    int64_t n = in->n;
    k_gather<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, perm, rec, *out, has, perm_out);
    return hipGetLastError();
}
