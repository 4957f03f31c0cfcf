// S1: cell list and neighbour lists (the chaining mesh of Sec. 3.3 with one
// interaction list per step that every later pass reuses).
//
// 1. validate + reduce H (deterministic two-level reduction)
// 2. key = Morton code of the particle's cell; stable radix sort -> perm
// 3. gather sorted x, y, z, H into one double4 per particle; cell ranges
// 4. walk: a group of lanes per particle visits the cells of the hierarchy
//    level matched to its support and finds the j with r^2 < H_i^2 (the
//    gather set, self excluded), and among them the j with r^2 >= H_j^2: j
//    reaches i only through i's larger support, so the pair is an "extra"
//    of j. Hits go to a capped scratch row, with exact counts.
// 5. exclusive scans of both counts give every particle its output slots;
//    the scratch rows are compacted, and rows past the cap walked again
// 6. the extras, grouped by i, are transposed into rows per j, each row
//    ascending in i (placed by rank, so the atomic slot counters of the
//    scatter decide nothing). The lists, and every sum over them, are the
//    same bit for bit from run to run.
#include <math.h>

#include <algorithm>

#include "crk_internal.h"

namespace crk {
namespace {

__global__ __launch_bounds__(kBlock) void k_validate(const double *x, const double *y,
                                                     const double *z, const double *H, int64_t n,
                                                     double L, double *part /* [nblk][3] */,
                                                     int *flags /* [3] */) {
    __shared__ double smax[kBlock], smin[kBlock], ssum[kBlock];
    double hmax = 0.0, hmin = INFINITY, hsum = 0.0;
    int nf = 0, rg = 0, bh = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        double a = x[i], b = y[i], c = z[i], h = H[i];
        if (!isfinite(a) || !isfinite(b) || !isfinite(c) || !isfinite(h)) {
            nf = 1;
            continue;
        }
        if (a < 0.0 || a >= L || b < 0.0 || b >= L || c < 0.0 || c >= L) rg = 1;
        if (!(h > 0.0)) bh = 1;
        hmax = fmax(hmax, h);
        hmin = fmin(hmin, h);
        hsum += h;
    }
    smax[threadIdx.x] = hmax;
    smin[threadIdx.x] = hmin;
    ssum[threadIdx.x] = hsum;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
            ssum[threadIdx.x] += ssum[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x * 3 + 0] = smax[0];
        part[blockIdx.x * 3 + 1] = smin[0];
        part[blockIdx.x * 3 + 2] = ssum[0];
    }
    if (nf) atomicOr(&flags[0], 1);
    if (rg) atomicOr(&flags[1], 1);
    if (bh) atomicOr(&flags[2], 1);
}

// final reduction of the (at most 1024) block partials by one block, in a
// fixed tree order
__global__ __launch_bounds__(1024) void k_validate_final(const double *part, int nblk, double *out) {
    __shared__ double smax[1024], smin[1024], ssum[1024];
    const int t = threadIdx.x;
    smax[t] = t < nblk ? part[t * 3 + 0] : 0.0;
    smin[t] = t < nblk ? part[t * 3 + 1] : INFINITY;
    ssum[t] = t < nblk ? part[t * 3 + 2] : 0.0;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (t < s) {
            smax[t] = fmax(smax[t], smax[t + s]);
            smin[t] = fmin(smin[t], smin[t + s]);
            ssum[t] += ssum[t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = smax[0];
        out[1] = smin[0];
        out[2] = ssum[0];
    }
}

// Graph mode cannot stop on invalid input before the walk, so such a
// particle is moved to a fixed in-box point (the R3 low-discrepancy sequence
// of its index) with a vanishing support: every later access stays in
// bounds, and the step's status reports the error.
__device__ __forceinline__ bool invalid_particle(double x, double y, double z, double h, double L) {
    return !(x >= 0.0 && x < L && y >= 0.0 && y < L && z >= 0.0 && z < L && h > 0.0 && h < 0.5 * L);
}

__device__ __forceinline__ double4 stand_in(int64_t i, double L) {
    double t = (double)i;
    return make_double4(L * (t * 0.8191725133961645 - floor(t * 0.8191725133961645)),
                        L * (t * 0.6710436067037893 - floor(t * 0.6710436067037893)),
                        L * (t * 0.5497004779019703 - floor(t * 0.5497004779019703)), 1e-9 * L);
}

__device__ __forceinline__ int cell_of(double x, double inv_c, int nc) {
    int k = (int)floor(x * inv_c);
    return k < 0 ? 0 : (k >= nc ? nc - 1 : k);
}

// key = (box << 3 bits) | Morton code of the particle's finest cell; the box
// is found by bisection of the batch's particle offsets
__global__ __launch_bounds__(kBlock) void k_keys(const double *x, const double *y, const double *z,
                                                 int64_t n, double inv_c, int nc, int bits,
                                                 const int64_t *__restrict__ boff, int nboxes,
                                                 const double *H, double L, uint32_t *key, int32_t *val) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = nboxes - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (boff[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    double px = x[i], py = y[i], pz = z[i];
    if (H && invalid_particle(px, py, pz, H[i], L)) {
        double4 s = stand_in(i, L);
        px = s.x;
        py = s.y;
        pz = s.z;
    }
    uint32_t m = morton3(cell_of(px, inv_c, nc), cell_of(py, inv_c, nc), cell_of(pz, inv_c, nc));
    key[i] = ((uint32_t)lo << (3 * bits)) | m;
    val[i] = (int32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_gather_sorted(const double *x, const double *y,
                                                          const double *z, const double *H,
                                                          const int32_t *perm, int64_t n,
                                                          int stand_ins, double L, double4 *posH) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    int32_t i = perm[k];
    double4 p = make_double4(x[i], y[i], z[i], H[i]);
    if (stand_ins && invalid_particle(p.x, p.y, p.z, p.w, L)) p = stand_in(i, L);
    posH[k] = p;
}

// graph mode: the input checks of the eager build, as a status word
// (bit 0 non-finite, bit 1 outside [0, L), bit 2 H <= 0, bit 3 H >= L/2)
__global__ void k_graph_inputs(const double *res, const int *flags, double L, GraphStat *st) {
    int e = (flags[0] ? 1 : 0) | (flags[1] ? 2 : 0) | (flags[2] || !(res[1] > 0.0) ? 4 : 0);
    if (!flags[0] && !(res[0] < 0.5 * L)) e |= 8;
    st->input_error = e;
    st->overflow = 0;
    st->clear = 0;
}

// graph mode: lists longer than the recorded capacity empty every row (so
// that the fills below stay in bounds) and raise the overflow flag
__global__ void k_graph_cap(const int64_t *goff, const int64_t *eoff, int64_t n, int64_t gcap,
                            int64_t ecap, GraphStat *st) {
    int64_t G = goff[n], E = eoff[n];
    int o = (G > gcap || E > ecap) ? 1 : 0;
    st->overflow = o;
    st->clear = o;
    st->n_gather = o ? 0 : G;
    st->n_extra = o ? 0 : E;
}

__global__ __launch_bounds__(kBlock) void k_graph_clear(const GraphStat *st, int64_t n, int64_t *goff,
                                                        int64_t *eoff, int32_t *ng) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i > n || !st->clear) return;
    goff[i] = 0;
    eoff[i] = 0;
    if (i < n) ng[i] = 0;
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t *a, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) a[i] = v;
}

// zeros into two int32 arrays of n entries (16-byte aligned; b may be
// null), four entries per store, one launch for both
__global__ __launch_bounds__(kBlock) void k_zero2_i32(int32_t *a, int32_t *b, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x, n4 = n >> 2;
    const int4 z = make_int4(0, 0, 0, 0);
    if (t < n4) {
        ((int4 *)a)[t] = z;
        if (b) ((int4 *)b)[t] = z;
    } else if (t < n4 + (n & 3)) {
        a[4 * n4 + (t - n4)] = 0;
        if (b) b[4 * n4 + (t - n4)] = 0;
    }
}

// sorted-index range of every cell of every level (a level-k cell is the set
// of particles whose fine Morton code shifted right by 3k is its id)
__global__ __launch_bounds__(kBlock) void k_tables(const uint32_t *skey, int64_t n, Levels v,
                                                   int32_t *cbeg, int32_t *cend) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    uint32_t key = skey[k];
    uint32_t prev = k > 0 ? skey[k - 1] : 0u, next = k + 1 < n ? skey[k + 1] : 0u;
    const int64_t base = box_base(v, k);
    const uint32_t mort = key & (uint32_t)(((uint64_t)1 << (3 * v.bits)) - 1);
    for (int l = 0; l <= v.bits; l++) {
        // a cell of level l is identified by key >> 3l (box bits included)
        uint32_t id = key >> (3 * l);
        uint32_t loc = mort >> (3 * l);
        if (k == 0 || (prev >> (3 * l)) != id) cbeg[base + v.off[l] + loc] = (int32_t)k;
        if (k == n - 1 || (next >> (3 * l)) != id) cend[base + v.off[l] + loc] = (int32_t)(k + 1);
    }
}

// The cells of one particle's walk. CULL: the walked range lies within half
// a period of i, so every particle of an (unwrapped) cell has its nearest
// image in that cell's image: the separation is (x_i - x_j) + c with c in
// {-L, 0, L} fixed per cell, the same two roundings the minimum-image rule
// makes, and cells wholly outside the (slightly widened) support are
// skipped. Otherwise each separation takes the minimum-image rule.
template <int G, bool DIRECT, bool CULL>
__device__ __forceinline__ void walk_row(const double4 *__restrict__ posH, int64_t i, const double4 &pi,
                                         int l, int gshift, uint32_t below, const Levels &v,
                                         const int32_t *__restrict__ cb, const int32_t *__restrict__ ce_,
                                         int nck, int lx, int ly, int lz, int mx, int my, int mz,
                                         double cs, double Hc2, int cap, uint32_t *row,
                                         const int64_t *__restrict__ goff, int32_t *gidx,
                                         int32_t *rcnt, const int64_t *__restrict__ eoff,
                                         int32_t *efill, int32_t *etmp, int32_t &cg) {
    const double H2 = pi.w * pi.w;
    const double L = v.L;
    for (int a = 0; a < mz; a++) {
        const int kz = lz + a;
        uint32_t mzb = spread3(wrapc(kz, nck)) << 2;
        const double cz = kz < 0 ? L : (kz >= nck ? -L : 0.0);
        const double gz = CULL ? cell_gap(pi.z, kz, cs) : 0.0;
        const double gz2 = gz * gz;
        for (int b = 0; b < my; b++) {
            const int ky = ly + b;
            uint32_t myb = mzb | (spread3(wrapc(ky, nck)) << 1);
            const double cy = ky < 0 ? L : (ky >= nck ? -L : 0.0);
            const double gy = CULL ? cell_gap(pi.y, ky, cs) : 0.0;
            const double gzy = gz2 + gy * gy;
            if (CULL && gzy > Hc2) continue;
            for (int e = 0; e < mx; e++) {
                const int kx = lx + e;
                const double gx = CULL ? cell_gap(pi.x, kx, cs) : 0.0;
                if (CULL && gzy + gx * gx > Hc2) continue;
                const double cx = kx < 0 ? L : (kx >= nck ? -L : 0.0);
                uint32_t id = myb | spread3(wrapc(kx, nck));
                int jb = cb[id], je = ce_[id];
                for (int j0 = jb; j0 < je; j0 += G) {
                    int j = j0 + l;
                    bool hit = false, extra = false;
                    if (j < je) {
                        double4 pj = posH[j];
                        double dx, dy, dz;
                        if (CULL) {
                            dx = (pi.x - pj.x) + cx;
                            dy = (pi.y - pj.y) + cy;
                            dz = (pi.z - pj.z) + cz;
                        } else {
                            dx = min_image(pi.x - pj.x, v.L, v.hL);
                            dy = min_image(pi.y - pj.y, v.L, v.hL);
                            dz = min_image(pi.z - pj.z, v.L, v.hL);
                        }
                        double r2 = r2_exact(dx, dy, dz);
                        hit = r2 < H2 && (int64_t)j != i;
                        extra = hit && !(r2 < pj.w * pj.w);
                    }
                    uint32_t hm;
                    if (G == 1) {
                        hm = hit;
                    } else {
                        uint64_t mh = __ballot(hit);
                        hm = (uint32_t)((mh >> gshift) & ((G == 64) ? ~0ull : (((uint64_t)1 << G) - 1)));
                    }
                    if (hit) {
                        int pos = cg + (G == 1 ? 0 : __popc(hm & below));
                        if (DIRECT) {
                            gidx[goff[i] + pos] = j;
                            if (extra) etmp[atomicAdd(&efill[j], 1)] = (int32_t)i;
                        } else {
                            if (pos < cap) row[pos] = (uint32_t)j | (extra ? 0x80000000u : 0u);
                            if (extra) atomicAdd(&rcnt[j], 1);
                        }
                    }
                    cg += __popc(hm);
                }
            }
        }
    }
}

// Flattened form of the same walk. The cells of a wavefront's groups hold
// different numbers of particles, so a cell-by-cell loop keeps most lanes
// idle; here a group first lists its non-empty, non-skipped cells as ranges
// of sorted particles (in walk order, up to walk_ranges<G>() at a time, in
// LDS, each with the code of its periodic image shift) and then takes the
// concatenated candidates G at a time across cell boundaries. The candidate
// order, hence every row, is the same as the cell-by-cell walk's.
//
// The group first fills its axis tables (fill_axes); a listed cell then
// costs three table reads, and its range carries the one-byte code of its
// image shift (the 27 shift triples are a table of the block).

// cell ranges a group lists at a time: four steps of G cells, at most 64
template <int G>
__host__ __device__ constexpr int walk_ranges() {
    return 4 * G > 64 ? 64 : 4 * G;
}

// the 27 image shift triples (dx, dy, dz) by code cx + 3 cy + 9 cz
__device__ __forceinline__ void fill_shifts(double (*sh)[3], double L) {
    const int c = threadIdx.x;
    if (c < 27) {
        const int q[3] = {c % 3, (c / 3) % 3, c / 9};
#pragma unroll
        for (int a = 0; a < 3; a++) sh[c][a] = q[a] == 1 ? L : (q[a] == 2 ? -L : 0.0);
    }
}

template <int G, bool DIRECT, bool CULL>
__device__ __forceinline__ void walk_row_flat(const double4 *__restrict__ posH, int64_t i,
                                              const double4 &pi, int l, int gshift, uint32_t below,
                                              const Levels &v, const int32_t *__restrict__ cb,
                                              const int32_t *__restrict__ ce_, int nck, int lx, int ly,
                                              int lz, int mx, int my, int mz, double cs, double Hc2,
                                              int cap, uint32_t *row, const int64_t *__restrict__ goff,
                                              int32_t *gidx, int32_t *rcnt,
                                              const int64_t *__restrict__ eoff, int32_t *efill,
                                              int32_t *etmp, int32_t &cg, int32_t *sb, int32_t *sc,
                                              uint8_t *scode, AxisTab &tab, const double (*shifts)[3]) {
    constexpr int NR = walk_ranges<G>();
    const double H2 = pi.w * pi.w;
    const int ncell = mx * my * mz;
    // 1. axis tables
    fill_axes<G, CULL, false>(tab, pi, l, lx, ly, lz, mx, my, mz, nck, cs, v.L);
    const uint32_t dx_ = div16(mx), dy_ = div16(my);
    int c0 = 0;
    while (c0 < ncell) {
        // 2. list up to NR non-empty cells, G cells per step
        int nr = 0, cum = 0;
        while (c0 < ncell && nr + G <= NR) {
            const int cidx = c0 + l;
            int jb = 0, len = 0, code = 0;
            if (cidx < ncell) {
                const int t = (int)(((uint32_t)cidx * dx_) >> 16);
                const int e = cidx - t * mx;
                const int a = (int)(((uint32_t)t * dy_) >> 16);
                const int b = t - a * my;
                bool keep = true;
                if (CULL) keep = (tab.g2[2][a] + tab.g2[1][b]) + tab.g2[0][e] <= Hc2;
                if (keep) {
                    const uint32_t ix = tab.id[0][e], iy = tab.id[1][b], iz = tab.id[2][a];
                    const uint32_t id = (ix | iy | iz) & 0x3fffffffu;
                    code = (int)(ix >> 30) + 3 * (int)(iy >> 30) + 9 * (int)(iz >> 30);
                    jb = cb[id];
                    len = ce_[id] - jb;
                }
            }
            int tot;
            const int pre = group_excl_scan<G>(len, l, tot);
            const bool has = len > 0;
            const uint32_t hm = (uint32_t)((__ballot(has) >> gshift) & (((uint64_t)1 << G) - 1));
            if (has) {
                const int pos = nr + __popc(hm & below);
                sb[pos] = jb;
                sc[pos] = cum + pre;
                scode[pos] = (uint8_t)code;
            }
            nr += __popc(hm);
            cum += tot;
            c0 += G;
        }
        if (l == 0) sc[nr] = cum;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // 3. the listed candidates, G at a time
        int r = 0;
        for (int f0 = 0; f0 < cum; f0 += G) {
            const int f = f0 + l;
            bool hit = false, extra = false;
            int j = 0;
            if (f < cum) {
                while (sc[r + 1] <= f) r++;
                j = sb[r] + (f - sc[r]);
                const double4 pj = posH[j];
                double dx, dy, dz;
                if (CULL) {
                    const double *sh = shifts[scode[r]];
                    dx = (pi.x - pj.x) + sh[0];
                    dy = (pi.y - pj.y) + sh[1];
                    dz = (pi.z - pj.z) + sh[2];
                } else {
                    dx = min_image(pi.x - pj.x, v.L, v.hL);
                    dy = min_image(pi.y - pj.y, v.L, v.hL);
                    dz = min_image(pi.z - pj.z, v.L, v.hL);
                }
                const double r2 = r2_exact(dx, dy, dz);
                hit = r2 < H2 && (int64_t)j != i;
                extra = hit && !(r2 < pj.w * pj.w);
            }
            const uint32_t hm = (uint32_t)((__ballot(hit) >> gshift) & (((uint64_t)1 << G) - 1));
            if (hit) {
                const int pos = cg + __popc(hm & below);
                if (DIRECT) {
                    gidx[goff[i] + pos] = j;
                    if (extra) etmp[atomicAdd(&efill[j], 1)] = (int32_t)i;
                } else {
                    if (pos < cap) row[pos] = (uint32_t)j | (extra ? 0x80000000u : 0u);
                    if (extra) atomicAdd(&rcnt[j], 1);
                }
            }
            cg += __popc(hm);
        }
        // the list is rewritten by the next batch only after every lane read it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Single-pass walk of particle i by a group of G lanes of one wavefront:
// the group visits i's cells in order and takes each cell's particles G at a
// time (consecutive, so the loads coalesce). A ballot over the group orders
// the hits exactly as a serial walk would, so row i is the same list for
// every G. Row entries go to a per-particle scratch of `cap` slots, with bit
// 31 marking the pairs that are extras of j; the returned count covers every
// hit, so a row longer than cap is detected and walked again (DIRECT) into
// its final place.
// DIRECT = true is that second walk: it writes the gather row and the
// extras straight to their final places.
template <int G, bool DIRECT>
__device__ __forceinline__ int32_t walk_one(const double4 *__restrict__ posH, int64_t i, int l,
                                            const Levels &v, const int32_t *__restrict__ cbeg,
                                            const int32_t *__restrict__ cend, int cap, uint32_t *scratch,
                                            int32_t *rcnt, const int64_t *__restrict__ goff,
                                            int32_t *gidx, const int64_t *__restrict__ eoff,
                                            int32_t *efill, int32_t *etmp, int shift,
                                            const double (*s_shift)[3]) {
    const double4 pi = posH[i];
    const int lane = threadIdx.x & 63;
    const int gshift = lane - l;
    const uint32_t below = (l == 0) ? 0u : ((1u << l) - 1u);
    int32_t cg = 0;
    uint32_t *row = DIRECT ? nullptr : scratch + (size_t)i * cap;
    int k = level_for(pi.w * (double)(1 << shift), v);
    int nck = 1 << (v.bits - k);
    Grid g{v.L, v.hL, (double)nck / v.L, v.margin, nck};
    int lx, ly, lz, mx, my, mz;
    axis_range(pi.x, pi.w, g, lx, mx);
    axis_range(pi.y, pi.w, g, ly, my);
    axis_range(pi.z, pi.w, g, lz, mz);
    const int64_t base = box_base(v, i) + v.off[k];
    const int32_t *cb = cbeg + base, *ce_ = cend + base;
    // the support widened by twice the axis margin (far above any rounding)
    const double cs = v.L / (double)nck;
    const double Hc = pi.w + 2.0 * v.margin;
    const bool cull = 2.0 * (Hc + cs) < v.L;
    bool done = false;
    if constexpr (G >= 4) {
        // the flattened walk (narrower groups would need too much LDS for
        // their range lists, and walk cell by cell)
        if (mx <= kAxisCells && my <= kAxisCells && mz <= kAxisCells) {
            constexpr int NG = kBlock / G;
            constexpr int NR = walk_ranges<G>();
            __shared__ int32_t s_b[NG][NR], s_c[NG][NR + 1];
            __shared__ uint8_t s_code[NG][NR];
            __shared__ AxisTab s_ax[NG];
            const int grp = threadIdx.x / G;
            if (cull)
                walk_row_flat<G, DIRECT, true>(posH, i, pi, l, gshift, below, v, cb, ce_, nck, lx, ly, lz,
                                               mx, my, mz, cs, Hc * Hc, cap, row, goff, gidx, rcnt, eoff,
                                               efill, etmp, cg, s_b[grp], s_c[grp], s_code[grp], s_ax[grp],
                                               s_shift);
            else
                walk_row_flat<G, DIRECT, false>(posH, i, pi, l, gshift, below, v, cb, ce_, nck, lx, ly, lz,
                                                mx, my, mz, cs, INFINITY, cap, row, goff, gidx, rcnt, eoff,
                                                efill, etmp, cg, s_b[grp], s_c[grp], s_code[grp], s_ax[grp],
                                                s_shift);
            done = true;
        }
    }
    if (done) {
    } else if (cull) {
        walk_row<G, DIRECT, true>(posH, i, pi, l, gshift, below, v, cb, ce_, nck, lx, ly, lz, mx, my,
                                  mz, cs, Hc * Hc, cap, row, goff, gidx, rcnt, eoff, efill, etmp, cg);
    } else {
        walk_row<G, DIRECT, false>(posH, i, pi, l, gshift, below, v, cb, ce_, nck, lx, ly, lz, mx, my,
                                   mz, cs, INFINITY, cap, row, goff, gidx, rcnt, eoff, efill, etmp, cg);
    }
    return cg;
}

// First walk (DIRECT = false): one group per particle; ng[i] gets the full
// count. Second walk (DIRECT = true): a grid of any size whose groups take
// the particles that compaction listed in longs (rows past cap; longs[0]
// counts them, the list follows) in turn, so it costs nothing when no row
// is long.
template <int G, bool DIRECT>
__global__ __launch_bounds__(kBlock) void k_walk_scratch(const double4 *__restrict__ posH, int64_t n,
                                                         Levels v, const int32_t *__restrict__ cbeg,
                                                         const int32_t *__restrict__ cend, int cap,
                                                         uint32_t *scratch, int32_t *ng, int32_t *rcnt,
                                                         const int64_t *__restrict__ goff, int32_t *gidx,
                                                         const int64_t *__restrict__ eoff, int32_t *efill,
                                                         int32_t *etmp, int shift, int32_t *longs) {
    // the shift table first: every wave of the block is still running
    __shared__ double s_shift[27][3];
    fill_shifts(s_shift, v.L);
    __syncthreads();
    // the first walk maps blocks to XCDs in contiguous runs of particles; the
    // list of the second is short, so its blocks go round the XCDs in order
    const int64_t gid = (DIRECT ? (int64_t)blockIdx.x : xcd_block(blockIdx.x, gridDim.x)) * kBlock + threadIdx.x;
    const int l = (int)(gid % G);
    if constexpr (!DIRECT) {
        const int64_t i = gid / G;
        if (i >= n) return;   // whole groups leave together (G divides the block)
        const int32_t cg = walk_one<G, false>(posH, i, l, v, cbeg, cend, cap, scratch, rcnt, goff, gidx,
                                              eoff, efill, etmp, shift, s_shift);
        if (l == 0) ng[i] = cg;
    } else {
        const int64_t nl = longs[0];
        const int64_t stride = (int64_t)gridDim.x * (kBlock / G);
        for (int64_t t = gid / G; t < nl; t += stride) {
            const int64_t i = longs[1 + t];
            // a recorded step whose lists overflowed their capacities has
            // its counts cleared: then nothing is written
            if (ng[i] <= cap) continue;
            walk_one<G, true>(posH, i, l, v, cbeg, cend, cap, scratch, rcnt, goff, gidx, eoff, efill, etmp,
                              shift, s_shift);
        }
    }
}

// scratch rows -> gather rows, for rows that fit in cap (G lanes per row
// read and write consecutive slots; longer rows are listed for the second
// walk); each extra (j, i) goes to a slot of row j of the transposed lists
// (efill[j], which the offsets scan set to row j's start, hands out its
// places; slot order is fixed later by rank). A lane takes U entries of its row at
// a time: their loads, then the slot atomics of their extras, then the
// dependent stores, so the atomics' round trips overlap instead of
// following one another.
//
// With vnsum, each row's FP64 volume sum of eq. (vol) comes along: the
// group re-reads its row (in cache) and adds W(r_ij, H_i) over the self
// pair and every gather entry, the terms of the volume pass (same
// separations, square root and weight) in another order; n_i goes to
// vnsum[i] and (x_i, V_i = 1 / n_i) to posV[i]. The rows past cap get
// theirs from k_volume_longs after the second walk.
template <int G, int U>
__global__ __launch_bounds__(kBlock) void k_compact_rows(const uint32_t *__restrict__ scratch, int cap,
                                                         int64_t n, const int32_t *__restrict__ ng,
                                                         const int64_t *__restrict__ goff, int32_t *gidx,
                                                         int32_t *efill, int32_t *etmp, int32_t *longs,
                                                         const double4 *__restrict__ posH, Box box,
                                                         double *vnsum, double4 *posV) {
    int64_t gid = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const int l = (int)(gid % G);
    const int64_t i = gid / G;
    if (i >= n) return;
    const int cnt = ng[i];
    if (cnt > cap) {
        // walked again into place (the list order is immaterial)
        if (l == 0) longs[1 + atomicAdd(&longs[0], 1)] = (int32_t)i;
        return;
    }
    const uint32_t *row = scratch + (size_t)i * cap;
    const int64_t gw = goff[i];
    for (int k0 = l; k0 < cnt; k0 += G * U) {
        uint32_t w[U];
#pragma unroll
        for (int u = 0; u < U; u++) w[u] = k0 + u * G < cnt ? row[k0 + u * G] : 0u;
        bool ex[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int k = k0 + u * G;
            ex[u] = k < cnt && (w[u] & 0x80000000u);
            if (k < cnt) gidx[gw + k] = (int32_t)(w[u] & 0x7fffffffu);
        }
        // the returned places are used only after every atomic is issued
        // (efill[j] starts at row j's offset, so the atomic returns the place)
        int32_t at[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            at[u] = -1;
            if (ex[u]) at[u] = atomicAdd(&efill[(int32_t)(w[u] & 0x7fffffffu)], 1);
        }
#pragma unroll
        for (int u = 0; u < U; u++)
            if (at[u] >= 0) etmp[at[u]] = (int32_t)i;
    }
    if (vnsum) {
        const double4 pi = posH[i];
        const double invH = 1.0 / pi.w;
        const double cw = kW * invH * invH * invH;
        double s = l == 0 ? cw : 0.0;   // the self pair: W(0, H_i)
        // four partners' positions in flight at a time; the terms are added
        // in the order k = l, l + G, ... all the same
        constexpr int VB = 4;
        for (int k0 = l; k0 < cnt; k0 += VB * G) {
            double4 pj[VB];
#pragma unroll
            for (int u = 0; u < VB; u++)
                if (k0 + u * G < cnt) pj[u] = posH[row[k0 + u * G] & 0x7fffffffu];
#pragma unroll
            for (int u = 0; u < VB; u++) {
                if (k0 + u * G >= cnt) break;
                const double dx = pair_image(pi.x - pj[u].x, box), dy = pair_image(pi.y - pj[u].y, box),
                             dz = pair_image(pi.z - pj[u].z, box);
                const double q = sqrt_dist(dx * dx + dy * dy + dz * dz) * invH;
                s += kernel_w(q, cw);
            }
        }
#pragma unroll
        for (int m = G / 2; m >= 1; m >>= 1) s += __shfl_xor(s, m, G);
        if (l == 0) {
            vnsum[i] = s;
            posV[i] = make_double4(pi.x, pi.y, pi.z, 1.0 / s);
        }
    }
}

// The FP64 volume sums of the rows listed in longs (those over the scratch
// rows' cap, written into place by the second walk), as k_compact_rows
// forms them (with its G, lane l adds entries l, l + G, ... and the same
// reduction follows, so the sum is bit for bit the compaction's), over a
// grid of any size.
template <int G>
__global__ __launch_bounds__(kBlock) void k_volume_longs(const int32_t *__restrict__ longs,
                                                         const int32_t *__restrict__ ng, int cap,
                                                         const int64_t *__restrict__ goff,
                                                         const int32_t *__restrict__ gidx,
                                                         const double4 *__restrict__ posH, Box box,
                                                         double *vnsum, double4 *posV) {
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int l = (int)(gid % G);
    const int64_t nl = longs[0];
    const int64_t stride = (int64_t)gridDim.x * (kBlock / G);
    for (int64_t t = gid / G; t < nl; t += stride) {
        const int64_t i = longs[1 + t];
        if (ng[i] <= cap) continue;   // cleared by an overflowed recorded step
        const double4 pi = posH[i];
        const double invH = 1.0 / pi.w;
        const double cw = kW * invH * invH * invH;
        double s = l == 0 ? cw : 0.0;
        for (int64_t k = goff[i] + l; k < goff[i + 1]; k += G) {
            const double4 pj = posH[gidx[k]];
            const double dx = pair_image(pi.x - pj.x, box), dy = pair_image(pi.y - pj.y, box),
                         dz = pair_image(pi.z - pj.z, box);
            const double q = sqrt_dist(dx * dx + dy * dy + dz * dz) * invH;
            s += kernel_w(q, cw);
        }
#pragma unroll
        for (int m = G / 2; m >= 1; m >>= 1) s += __shfl_xor(s, m, G);
        if (l == 0) {
            vnsum[i] = s;
            posV[i] = make_double4(pi.x, pi.y, pi.z, 1.0 / s);
        }
    }
}

// Extras rows (per receiving particle j): the walk counts them per j, a
// scan gives the row offsets, the compaction and the second walk drop each
// (j, i) into some slot of row j (atomic slot counters), and here every
// entry moves to the place given by its rank in its row, so each row is
// ascending in i whatever order the slots were taken in. G lanes per row;
// entries of a row are distinct emitters, so the ranks are a permutation of
// the row's slots. A row of up to CAP entries is first staged in LDS (row
// stride CAP + 4 words, so the groups of a wavefront read different banks)
// and every rank is counted from there, four entries per read; longer rows
// count from global memory.
template <int G, int CAP>
__global__ __launch_bounds__(kBlock) void k_extra_rank(const int64_t *__restrict__ eoff,
                                                       const int32_t *__restrict__ tmp, int64_t n,
                                                       int32_t *out, int32_t *eb, int32_t *ee) {
    static_assert(CAP % 4 == 0, "rows are read four entries at a time");
    constexpr int S = CAP + 4;
    __shared__ __align__(16) int32_t srow[kBlock / G][S];
    int64_t gid = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const int l = (int)(gid % G);
    const int64_t j = gid / G;
    if (j >= n) return;
    const int64_t b = eoff[j];
    const int c = (int)(eoff[j + 1] - b);
    if (l == 0) {
        eb[j] = (int32_t)b;
        ee[j] = (int32_t)(b + c);
    }
    if (c <= CAP) {
        int32_t *sr = srow[threadIdx.x / G];
        // padded to a multiple of four with values above every index
        const int c4 = (c + 3) & ~3;
        for (int t = l; t < c4; t += G) sr[t] = t < c ? tmp[b + t] : INT32_MAX;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int4 *s4 = reinterpret_cast<const int4 *>(sr);
        for (int t = l; t < c; t += G) {
            const int32_t v = sr[t];
            int r = 0;
            for (int u = 0; u < c4 / 4; u++) {
                const int4 q = s4[u];
                r += (q.x < v) + (q.y < v) + (q.z < v) + (q.w < v);
            }
            out[b + r] = v;
        }
        return;
    }
    for (int t = l; t < c; t += G) {
        const int32_t v = tmp[b + t];
        int r = 0;
        for (int u = 0; u < c; u++) r += tmp[b + u] < v ? 1 : 0;
        out[b + r] = v;
    }
}

__global__ __launch_bounds__(kBlock) void k_set_H(double4 *posH, const double *H, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) posH[i].w = H[i];
}

__global__ __launch_bounds__(kBlock) void k_get_xyz(const double4 *posH, int64_t n, double *x,
                                                    double *y, double *z) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double4 p = posH[i];
    x[i] = p.x;
    y[i] = p.y;
    z[i] = p.z;
}

__global__ __launch_bounds__(kBlock) void k_permute(const int32_t *perm, const double *src,
                                                    double *dst, int64_t n, int ncomp, int to_sorted) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    int64_t o = perm[k];
    for (int c = 0; c < ncomp; c++) {
        if (to_sorted) dst[c * n + k] = src[c * n + o];
        else dst[c * n + o] = src[c * n + k];
    }
}

// row lengths of the exported sets: which 0 -> N_g (self + gather row),
// which 1 -> N_s (gather row + extras row)
__global__ __launch_bounds__(kBlock) void k_export_len(const int64_t *goff, const int32_t *eb,
                                                       const int32_t *ee, int64_t n, int which,
                                                       int64_t *len) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) len[i] = (goff[i + 1] - goff[i]) + (which == 0 ? 1 : (int64_t)(ee[i] - eb[i]));
    if (i == n) len[n] = 0;
}

__global__ __launch_bounds__(kBlock) void k_export_fill(const int64_t *goff, const int32_t *gidx,
                                                        const int32_t *eb, const int32_t *ee,
                                                        const int32_t *eidx, int64_t n, int which,
                                                        const int64_t *off, int32_t *idx) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int64_t o = off[i];
    if (which == 0) idx[o++] = (int32_t)i;
    for (int64_t k = goff[i]; k < goff[i + 1]; k++) idx[o++] = gidx[k];
    if (which == 1)
        for (int k = eb[i]; k < ee[i]; k++) idx[o++] = eidx[k];
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

// the reduced input checks of k_validate / k_validate_final, on the host
static crk_status read_checks(crk_ctx *c, const double *res, const int *flags, double *hmax,
                              double *hmin) {
    double *pin = (double *)c->pinned.p;
    CRK_HIP(c, hipMemcpyAsync(pin, res, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    CRK_HIP(c, hipMemcpyAsync(pin + 3, flags, 3 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    CRK_HIP(c, hipStreamSynchronize(c->stream));
    *hmax = pin[0];
    *hmin = pin[1];
    int *hf = (int *)(pin + 3);
    if (hf[0]) return set_err(c, CRK_ERR_NONFINITE, "non-finite position or H");
    if (hf[1]) return set_err(c, CRK_ERR_INVALID_ARG, "position outside [0, L)");
    if (hf[2] || !(*hmin > 0.0)) return set_err(c, CRK_ERR_SUPPORT, "H must be positive");
    return CRK_OK;
}

crk_status validate_inputs(crk_ctx *c, const double *x, const double *y, const double *z,
                           const double *H, int64_t n, double L, double *hmax, double *hmin) {
    int nblk = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 1024);
    CRK_TRY(ensure(c, c->red, (size_t)nblk * 3 * sizeof(double) + 64));
    double *part = (double *)c->red.p;
    int *flags = (int *)(part + (size_t)nblk * 3);
    CRK_TRY(ensure(c, c->misc, 256));
    double *res = (double *)c->misc.p;
    k_fill_i32<<<1, kBlock, 0, c->stream>>>(flags, 3, 0);
    k_validate<<<nblk, kBlock, 0, c->stream>>>(x, y, z, H, n, L, part, flags);
    k_validate_final<<<1, 1024, 0, c->stream>>>(part, nblk, res);
    CRK_HIP(c, hipGetLastError());
    return read_checks(c, res, flags, hmax, hmin);
}

Levels levels(const crk_ctx *c) {
    Levels v;
    v.L = c->L;
    v.hL = 0.5 * c->L;
    v.c0 = c->cell;
    v.margin = 1e-9 * c->L;
    v.bits = c->bits;
    for (int k = 0; k < 12; k++) v.off[k] = c->lvl_off[k];
    v.skey = (const uint32_t *)c->keyA.p;
    v.box_stride = c->ntab;
    return v;
}

// Neighbour lists for the current posH / cell tables.
static crk_status build_lists(crk_ctx *c) {
    int64_t n = c->n;
    Levels v = levels(c);
    CRK_TRY(ensure(c, c->ng, (size_t)n * sizeof(int32_t)));
    // goff[n + 1]: the longest gather row, for the next build's scratch rows
    CRK_TRY(ensure(c, c->goff, (size_t)(n + 2) * sizeof(int64_t)));
    CRK_TRY(ensure(c, c->ecnt, (size_t)n * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->efill, (size_t)n * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->eoff, (size_t)(n + 1) * sizeof(int64_t)));
    int32_t *ng = (int32_t *)c->ng.p;
    int64_t *goff = (int64_t *)c->goff.p;
    int32_t *ecnt = (int32_t *)c->ecnt.p, *efill = (int32_t *)c->efill.p;
    int64_t *eoff = (int64_t *)c->eoff.p;
    const double4 *posH = (const double4 *)c->posH.p;
    const int32_t *cbeg = (const int32_t *)c->cbeg.p, *cend = (const int32_t *)c->cend.p;
    // one walk into a capped scratch row per particle; exact counts come
    // with it, and the extras are counted per receiving particle
    const int cap = std::max(c->walk_cap, c->walk_cap_auto);
    CRK_TRY(ensure(c, c->scratch, (size_t)n * cap * sizeof(uint32_t)));
    uint32_t *scratch = (uint32_t *)c->scratch.p;
    // long rows: longs[0] counts them, their particles follow
    CRK_TRY(ensure(c, c->longs, (size_t)(n + 1) * sizeof(int32_t)));
    int32_t *longs = (int32_t *)c->longs.p;
    k_zero2_i32<<<nblocks((n >> 2) + (n & 3)), kBlock, 0, c->stream>>>(ecnt, nullptr, n);
    k_fill_i32<<<1, kBlock, 0, c->stream>>>(longs, 1, 0);
    {
        KTimer kt_(c, "k_walk");
        int G = c->G_walk;
#define L_WALK(GG) k_walk_scratch<GG, false><<<(unsigned)((n * GG + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(posH, n, v, cbeg, cend, cap, scratch, ng, ecnt, nullptr, nullptr, nullptr, nullptr, nullptr, c->walk_shift, longs)
        switch (G) {
            case 1: L_WALK(1); break;
            case 2: L_WALK(2); break;
            case 4: L_WALK(4); break;
            case 8: L_WALK(8); break;
            case 16: L_WALK(16); break;
            default: return set_err(c, CRK_ERR_INVALID_ARG, "walk lanes must be 1, 2, 4, 8 or 16");
        }
#undef L_WALK
    }
    CRK_HIP(c, hipGetLastError());
    // efill[j] = eoff[j]: the slot counters of the extras rows start at
    // their rows' offsets
    CRK_TRY(scan_counts2(c, ng, ecnt, n, goff, eoff, goff + n + 1, efill));
    int64_t G, E, longest = 0;
    GraphStat *gst = (GraphStat *)c->gstat.p;
    if (c->graph_mode) {
        // fixed capacities; the counts stay on the device
        G = c->gcap;
        E = c->ecap;
        k_graph_cap<<<1, 1, 0, c->stream>>>(goff, eoff, n, G, E, gst);
        k_graph_clear<<<nblocks(n + 1), kBlock, 0, c->stream>>>(gst, n, goff, eoff, ng);
        CRK_HIP(c, hipGetLastError());
    } else {
        int64_t *pin = (int64_t *)c->pinned.p;
        CRK_HIP(c, hipMemcpyAsync(pin, goff + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
        CRK_HIP(c, hipMemcpyAsync(pin + 1, eoff + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
        CRK_HIP(c, hipMemcpyAsync(pin + 2, goff + n + 1, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
        CRK_HIP(c, hipStreamSynchronize(c->stream));
        G = pin[0];
        E = pin[1];
        longest = pin[2];
    }
    if (E > INT32_MAX - 1) return set_err(c, CRK_ERR_INVALID_ARG, "more than 2^31 extra pairs");
    CRK_TRY(ensure(c, c->gidx, (size_t)(G > 0 ? G : 1) * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->etmp, (size_t)(E > 0 ? E : 1) * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->eidx, (size_t)(E > 0 ? E : 1) * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->eb, (size_t)n * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->ee, (size_t)n * sizeof(int32_t)));
    int32_t *etmp = (int32_t *)c->etmp.p, *eidx = (int32_t *)c->eidx.p;
    // the FP64 volumes of eq. (vol) come with the compaction when wanted
    const bool vol = c->vol_in_build != 0;
    double *vnsum = nullptr;
    double4 *posV = nullptr;
    if (vol) {
        CRK_TRY(ensure(c, c->vnsum, (size_t)n * sizeof(double)));
        CRK_TRY(ensure(c, c->posV, (size_t)n * sizeof(double4)));
        vnsum = (double *)c->vnsum.p;
        posV = (double4 *)c->posV.p;
    }
    const Box box{c->L, 1.0 / c->L};
    // (the long rows' volumes take the same lanes per row, so a row's sum
    // does not depend on which of the two kernels forms it)
    constexpr int GC = 16, UC = 8;
    {
        KTimer kt_(c, "k_compact_rows");
        k_compact_rows<GC, UC><<<(unsigned)((n * GC + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(
            scratch, cap, n, ng, goff, (int32_t *)c->gidx.p, efill, etmp, longs, posH, box, vnsum, posV);
    }
    {
        // the rows over the cap are few and long: 32 lanes each (the row is
        // the same list for any lane count), over the list the compaction made
        KTimer kt_(c, "k_walk_long");
        constexpr int GL = 32;
        const unsigned nb = (unsigned)std::min<int64_t>((n * GL + kBlock - 1) / kBlock, 4096);
        k_walk_scratch<GL, true><<<nb, kBlock, 0, c->stream>>>(
            posH, n, v, cbeg, cend, cap, nullptr, ng, nullptr, goff, (int32_t *)c->gidx.p, eoff, efill,
            etmp, c->walk_shift, longs);
    }
    CRK_HIP(c, hipGetLastError());
    if (vol) {
        const unsigned nb = (unsigned)std::min<int64_t>((n * GC + kBlock - 1) / kBlock, 1024);
        k_volume_longs<GC><<<nb, kBlock, 0, c->stream>>>(longs, ng, cap, goff, (const int32_t *)c->gidx.p,
                                                          posH, box, vnsum, posV);
        CRK_HIP(c, hipGetLastError());
    }
    // each extras row ascending in the emitting particle
    {
        KTimer kt_(c, "k_extra_rank");
        constexpr int GR = 8;
        k_extra_rank<GR, 128><<<(unsigned)((n * GR + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(
            eoff, etmp, n, eidx, (int32_t *)c->eb.p, (int32_t *)c->ee.p);
    }
    CRK_HIP(c, hipGetLastError());
    if (c->graph_mode) {
        // counts are on the device (crk_graph_replay reads them)
        c->ngather = c->nextra = c->npairs = -1;
    } else {
        c->ngather = G;
        c->nextra = E;
        c->npairs = G + E;
        c->walk_cap_auto = walk_cap_next((double)G, (double)n, longest);
    }
    c->built = 1;
    c->have_V = 0;
    c->vol_ready = vol ? 1 : 0;
    return CRK_OK;
}

// Steps 2-4 of the build for the geometry held in the context (box offsets
// already on the device). stand_ins: graph mode (see stand_in).
crk_status build_sorted(crk_ctx *c, const double *x, const double *y, const double *z,
                               const double *H, int32_t *perm, bool stand_ins, int64_t *n_pairs,
                               int32_t *n_cells) {
    const int64_t n = c->n;
    const int bits = c->bits;
    const int nboxes = (int)c->nboxes;
    int boxbits = 0;
    while ((1 << boxbits) < nboxes) boxbits++;
    int64_t ntot = c->ntab * nboxes;
    CRK_TRY(ensure(c, c->keyA, (size_t)n * sizeof(uint32_t)));
    CRK_TRY(ensure(c, c->perm, (size_t)n * sizeof(int32_t)));
    uint32_t *key = (uint32_t *)c->keyA.p;
    int32_t *pm = (int32_t *)c->perm.p;
    k_keys<<<nblocks(n), kBlock, 0, c->stream>>>(x, y, z, n, 1.0 / c->cell, c->nc, bits,
                                                  (const int64_t *)(c->graph_mode ? c->gboff.p : c->boff.p),
                                                  nboxes, stand_ins ? H : nullptr, c->L, key, pm);
    CRK_HIP(c, hipGetLastError());
    {
        KTimer kt_(c, "sort");
        CRK_TRY(radix_sort_pairs(c, key, pm, n, 3 * bits + boxbits));
    }
    // 3. sorted particles and the cell tables of every level of every box
    CRK_TRY(ensure(c, c->posH, (size_t)n * sizeof(double4)));
    CRK_TRY(ensure(c, c->cbeg, (size_t)ntot * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->cend, (size_t)ntot * sizeof(int32_t)));
    k_gather_sorted<<<nblocks(n), kBlock, 0, c->stream>>>(x, y, z, H, pm, n, stand_ins ? 1 : 0, c->L,
                                                           (double4 *)c->posH.p);
    k_zero2_i32<<<nblocks((ntot >> 2) + (ntot & 3)), kBlock, 0, c->stream>>>((int32_t *)c->cbeg.p,
                                                                             (int32_t *)c->cend.p, ntot);
    k_tables<<<nblocks(n), kBlock, 0, c->stream>>>(key, n, levels(c), (int32_t *)c->cbeg.p,
                                                    (int32_t *)c->cend.p);
    CRK_HIP(c, hipGetLastError());
    CRK_HIP(c, hipMemcpyAsync(perm, pm, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
    // 4. neighbour lists
    CRK_TRY(build_lists(c));
    if (n_pairs) *n_pairs = c->npairs;
    if (n_cells) *n_cells = c->nc;
    return CRK_OK;
}

}  // namespace crk

using namespace crk;

extern "C" {

crk_status crk_build_cells_batch(crk_ctx *c, int32_t nboxes, const int64_t *box_offsets, int64_t n,
                                 const double *x, const double *y, const double *z, const double *H,
                                 const crk_params *p, double cell_size, int32_t *perm,
                                 int64_t *n_pairs, int32_t *n_cells) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (n < 1 || !x || !y || !z || !H || !p || !perm || nboxes < 1 || !box_offsets)
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_build_cells: n < 1 or NULL argument");
    if (n > INT32_MAX / 2) return set_err(c, CRK_ERR_INVALID_ARG, "n too large");
    if (!(p->L > 0.0)) return set_err(c, CRK_ERR_INVALID_ARG, "L must be positive");
    if (box_offsets[0] != 0 || box_offsets[nboxes] != n)
        return set_err(c, CRK_ERR_INVALID_ARG, "box offsets must run from 0 to n");
    for (int b = 0; b < nboxes; b++)
        if (box_offsets[b + 1] < box_offsets[b])
            return set_err(c, CRK_ERR_INVALID_ARG, "box offsets must not decrease");
    CRK_HIP(c, hipSetDevice(c->device));
    const bool gm = c->graph_mode != 0;
    if (gm && (n != c->n || nboxes != c->nboxes || p->L != c->L || !c->built))
        return set_err(c, CRK_ERR_STATE, "graph mode needs the geometry of the last build");
    if (!gm) {
        c->built = 0;
        c->leaf_mode = 0;
        c->nc = 0;
        c->n = n;
        c->L = p->L;
        c->nboxes = nboxes;
    }
    c->have_V = 0;
    c->vol_ready = 0;
    // the FP64 volumes come with the lists unless the pure FP32 mode is asked
    // for (its volume pass sums in FP32)
    c->vol_in_build = p->precision != CRK_MIXED;
    // 1. validate and reduce H
    int nblk = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 1024);
    CRK_TRY(ensure(c, c->red, (size_t)nblk * 3 * sizeof(double) + 64));
    double *part = (double *)c->red.p;
    int *flags = (int *)(part + (size_t)nblk * 3);
    CRK_TRY(ensure(c, c->misc, 256));
    double *res = (double *)c->misc.p;
    k_fill_i32<<<1, kBlock, 0, c->stream>>>(flags, 3, 0);
    k_validate<<<nblk, kBlock, 0, c->stream>>>(x, y, z, H, n, p->L, part, flags);
    k_validate_final<<<1, 1024, 0, c->stream>>>(part, nblk, res);
    CRK_HIP(c, hipGetLastError());
    if (gm) {
        CRK_TRY(ensure(c, c->gstat, sizeof(GraphStat)));
        k_graph_inputs<<<1, 1, 0, c->stream>>>(res, flags, p->L, (GraphStat *)c->gstat.p);
        CRK_HIP(c, hipGetLastError());
        return build_sorted(c, x, y, z, H, perm, true, n_pairs, n_cells);
    }
    double hmax = 0.0, hmin = 0.0;
    CRK_TRY(read_checks(c, res, flags, &hmax, &hmin));
    if (!(hmax < 0.5 * p->L)) return set_err(c, CRK_ERR_SUPPORT, "max H %g >= L/2", hmax);
    // 2. Morton cell hierarchy: finest side near half the smallest support
    //    (or the requested side), at most 256 cells a side and at most about
    //    2^26 table entries over all boxes; box id above the Morton bits
    double cfine = cell_size > 0.0 ? cell_size : 0.5 * hmin;
    int bits = 0;
    while (bits < 8 && p->L / (double)(1 << bits) > cfine &&
           (double)nboxes * (double)((int64_t)1 << (3 * (bits + 1))) * 8.0 / 7.0 <= (double)(1 << 26))
        bits++;
    int boxbits = 0;
    while ((1 << boxbits) < nboxes) boxbits++;
    if (3 * bits + boxbits > 32) return set_err(c, CRK_ERR_INVALID_ARG, "too many boxes for the key width");
    c->bits = bits;
    c->nc = 1 << bits;
    c->cell = p->L / c->nc;
    int64_t off = 0;
    for (int k = 0; k <= bits; k++) {
        c->lvl_off[k] = off;
        int64_t m = (int64_t)1 << (bits - k);
        off += m * m * m;
    }
    c->ntab = off;
    CRK_TRY(ensure(c, c->boff, (size_t)(nboxes + 1) * sizeof(int64_t)));
    CRK_HIP(c, hipMemcpyAsync(c->boff.p, box_offsets, (size_t)(nboxes + 1) * sizeof(int64_t),
                              hipMemcpyHostToDevice, c->stream));
    return build_sorted(c, x, y, z, H, perm, false, n_pairs, n_cells);
}

crk_status crk_build_cells(crk_ctx *c, int64_t n, const double *x, const double *y, const double *z,
                           const double *H, const crk_params *p, double cell_size, int32_t *perm,
                           int64_t *n_pairs, int32_t *n_cells) {
    int64_t off[2] = {0, n};
    return crk_build_cells_batch(c, 1, off, n, x, y, z, H, p, cell_size, perm, n_pairs, n_cells);
}

crk_status crk_update_support(crk_ctx *c, const double *H_sorted, int64_t *n_pairs) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (!H_sorted) return set_err(c, CRK_ERR_INVALID_ARG, "H_sorted is NULL");
    if (c->nc == 0) return set_err(c, CRK_ERR_STATE, "crk_build_cells has not run");
    CRK_HIP(c, hipSetDevice(c->device));
    int64_t n = c->n;
    CRK_TRY(ensure(c, c->scanTmp, (size_t)n * 3 * sizeof(double)));
    double *xs = (double *)c->scanTmp.p;
    k_get_xyz<<<nblocks(n), kBlock, 0, c->stream>>>((const double4 *)c->posH.p, n, xs, xs + n,
                                                     xs + 2 * n);
    int nblk = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 1024);
    CRK_TRY(ensure(c, c->red, (size_t)nblk * 3 * sizeof(double) + 64));
    double *part = (double *)c->red.p;
    int *flags = (int *)(part + (size_t)nblk * 3);
    double *res = (double *)c->misc.p;
    k_fill_i32<<<1, kBlock, 0, c->stream>>>(flags, 3, 0);
    k_validate<<<nblk, kBlock, 0, c->stream>>>(xs, xs + n, xs + 2 * n, H_sorted, n, c->L, part, flags);
    k_validate_final<<<1, 1024, 0, c->stream>>>(part, nblk, res);
    double *pin = (double *)c->pinned.p;
    CRK_HIP(c, hipMemcpyAsync(pin, res, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    CRK_HIP(c, hipMemcpyAsync(pin + 3, flags, 3 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    CRK_HIP(c, hipStreamSynchronize(c->stream));
    int *hf = (int *)(pin + 3);
    if (hf[0]) return set_err(c, CRK_ERR_NONFINITE, "non-finite H");
    if (hf[2] || !(pin[1] > 0.0)) return set_err(c, CRK_ERR_SUPPORT, "H must be positive");
    if (!(pin[0] < 0.5 * c->L)) return set_err(c, CRK_ERR_SUPPORT, "max H %g >= L/2", pin[0]);
    k_set_H<<<nblocks(n), kBlock, 0, c->stream>>>((double4 *)c->posH.p, H_sorted, n);
    CRK_TRY(build_lists(c));
    if (n_pairs) *n_pairs = c->npairs;
    return CRK_OK;
}

crk_status crk_permute(crk_ctx *c, const double *src, double *dst, int32_t ncomp, int32_t to_sorted) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (!src || !dst || ncomp < 1) return set_err(c, CRK_ERR_INVALID_ARG, "crk_permute: bad argument");
    if (c->nc == 0 && !c->leaf_mode) return set_err(c, CRK_ERR_STATE, "crk_build_cells has not run");
    CRK_HIP(c, hipSetDevice(c->device));
    k_permute<<<nblocks(c->n), kBlock, 0, c->stream>>>((const int32_t *)c->perm.p, src, dst, c->n,
                                                        ncomp, to_sorted);
    CRK_HIP(c, hipGetLastError());
    return CRK_OK;
}

crk_status crk_export_neighbors(crk_ctx *c, int32_t which, int64_t *offsets, int32_t *idx,
                                int64_t cap, int64_t *total) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (!c->built) return set_err(c, CRK_ERR_STATE, "no neighbour lists");
    if (!offsets || !total || (which != 0 && which != 1))
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_export_neighbors: bad argument");
    CRK_HIP(c, hipSetDevice(c->device));
    int64_t n = c->n;
    *total = which == 0 ? c->ngather + n : c->npairs;
    k_export_len<<<nblocks(n + 1), kBlock, 0, c->stream>>>((const int64_t *)c->goff.p,
                                                            (const int32_t *)c->eb.p,
                                                            (const int32_t *)c->ee.p, n, which, offsets);
    CRK_TRY(scan_exclusive_i64(c, offsets, offsets, n + 1));
    if (idx) {
        if (cap < *total) return set_err(c, CRK_ERR_INVALID_ARG, "cap too small");
        k_export_fill<<<nblocks(n), kBlock, 0, c->stream>>>(
            (const int64_t *)c->goff.p, (const int32_t *)c->gidx.p, (const int32_t *)c->eb.p,
            (const int32_t *)c->ee.p, (const int32_t *)c->eidx.p, n, which, offsets, idx);
    }
    CRK_HIP(c, hipGetLastError());
    CRK_HIP(c, hipStreamSynchronize(c->stream));
    return CRK_OK;
}

}  // extern "C"
