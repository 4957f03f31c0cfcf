// Internal declarations of the CRKSPH neighbour-pass library (gfx950).
//
// Layout in HBM (all owned by the context, sized for the largest n seen):
//   posH   double4 [n]      sorted x, y, z, H (one 32-byte load per neighbour)
//   perm   int32   [n]      sorted k -> original index
//   skey   uint32  [n]      Morton code of each sorted particle's finest cell
//   cbeg/cend int32 [sum_k 8^(b-k)]  sorted-index range of every cell of every
//                           level k = 0..b of the Morton cell hierarchy (a
//                           level-k cell is an aligned block of 2^k fine cells
//                           a side, hence one contiguous range of particles)
//   goff   int64   [n+1]    gather rows: N_g(i) without i, in cell-walk order
//   gidx   int32   [sum ng]
//   eb/ee  int32   [n]      extras rows in eidx: {j : H_i <= |d| < H_j}, the
//   eidx   int32   [E]      partners that reach i only through their own larger
//                           support, ascending; N_s(i) = gather row ++ extras row
//                           (eoff [n+1] int64 holds the same row offsets)
//   recV   T       [n]      volumes in the pass precision
//   rec6   T4      [n]      {vx, vy, vz, V}            (velocity-gradient pass)
//   rec7   T4      [8][n]   packed per-particle records (derivative pass)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/crk.h"

namespace crk {

constexpr double kPi = 3.14159265358979323846;
// eq. (C4): W = kW H^-3 (1-q)^6 (1 + 6q + 35/3 q^2);
// grad_i W = kG H^-5 (1 + 5q) (1-q)^5 d  with kG = -1155 / (4 pi)
constexpr double kW = 495.0 / (32.0 * kPi);
constexpr double kG = -1155.0 / (4.0 * kPi);

constexpr int kBlock = 256;       // threads per block of every pair pass (4 wave64)

struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace crk

struct crk_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    // geometry of the last build: fine cells nc = 2^bits a side, levels 0..bits
    int64_t n = 0;
    double L = 1.0;
    int nc = 0;
    int bits = 0;
    double cell = 0.0;
    int64_t lvl_off[12] = {0};
    int64_t ntab = 0;        // table entries of one box
    int64_t nboxes = 1;
    int built = 0;          // lists valid
    int have_V = 0;         // recV valid (after crk_moments)
    // FP64 volumes summed by the build's compaction (vnsum, and V in posV.w)
    // for the current lists: wanted when the build's precision is not the
    // pure FP32 one, valid until the lists or the supports change
    int vol_in_build = 0, vol_ready = 0;
    int prec_V = -1;        // precision recV was written in
    int64_t npairs = 0;     // sum of |N_s(i)|
    int64_t ngather = 0;    // sum of ng (excludes self)
    int64_t nextra = 0;     // entries of eidx

    // workspace
    crk::Buf posH, perm, cbeg, cend, goff, gidx, ng, eb, ee, eidx;
    crk::Buf keyA, keyB, valA, valB, hist, scanTmp;
    crk::Buf recV, rec6, rec7, red, misc;
    crk::Buf flag, flist, tlist, fpos, tpos, rec6d, aux;   // adaptive-precision rows
    crk::Buf scratch;                                     // walk rows before compaction
    crk::Buf hnet_part, hnet_feat;                        // network gradients / features
    crk::Buf hs_list, hs_state, hs_pos, hs_iters, hs_pool;   // smoothing-length rounds
    crk::Buf ts_vs, ts_qr;                                   // time-step maxima per particle
    int ts_on = 0, ts_valid = 0;
    crk::Buf ce, ced;                                     // compatible-energy records (q, s)
    crk::Buf vstep;                                       // Verlet step: half-step state, evaluation outputs
    crk::Buf hs_rows, hs_rcnt, hs_R;                      // candidate rows (r^2)
    crk::Buf boff;                                        // batch box offsets
    crk::Buf sv, sm, su, srho;                            // sorted gas state (crk_step)
    crk::Buf gstat;                                       // device status of a graph step
    crk::Buf gboff;                                       // box offsets the graph was recorded with
    crk::Buf ecnt, efill, eoff, etmp;                     // extras rows: counts, slots, offsets, unordered rows
    crk::Buf vnsum;                                       // FP64 n_i of the build (vol_ready)
    crk::Buf longs;                                       // rows past the walk cap: count, then particles
    crk::Buf posV;                                        // sorted x, y, z and V (the moment pass reads both at once)
    // RCB leaf tiling (crk_build_leaves): keys, the three sorted lists (two
    // copies), sides, nodes, tables, boxes, interaction lists
    crk::Buf rq, rsk, rla, rlb, rside, rpnode, rscan, rnode, rtab, rbox, rpoff, rpart;
    int leaf_mode = 0;                                    // lists come from crk_build_leaves
    int64_t nleaves = 0, nleaf_pairs = 0;

    // graph mode (crk_graph_capture): the build keeps the geometry of the
    // last eager build, lists are bounded by fixed capacities, and no call
    // reads device values back on the host; `capturing` forbids workspace growth
    int graph_mode = 0;
    int capturing = 0;
    int64_t gcap = 0, ecap = 0;           // gather / extras capacity
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_prec = -1;
    struct Geo {
        int64_t n, ntab, nboxes, lvl_off[12];
        double L, cell;
        int nc, bits;
    } geo{};                              // geometry the graph was recorded with
    int G_hsolve = 16, hs_round = 12, hs_cap = 320;
    double hs_factor = 1.15;
    int64_t last_nflag = 0, last_ntouch = 0;
    crk::Buf pinned;        // small host-pinned readback area

    // per-pass tuning: lanes per particle (1..64)
    int G_vol = 4, G_mom = 1, G_grad = 4, G_der = 8;
    // volume, moment, velocity-gradient, derivative (and compatible)
    // passes: particles per wavefront of the balanced lane-group mapping
    // (4, 8, 16 or 32); 0 = the G_* lanes per particle above
    int P_vol = 0, P_mom = 0, P_grad = 0, P_der = 8;
    // neighbour walk: lanes per particle and scratch slots per row
    int G_walk = 8, walk_cap = 192;
    // scratch row slots the next walk uses at least: 2.5x the mean gather
    // row of the last eager build (a multiple of 64, at most 1024), so that
    // rows past the cap, walked twice, stay rare when supports hold many
    // more neighbours than the default cap
    int walk_cap_auto = 0;
    // walked level: the first whose cell side is at least 2^(walk_shift-1) H
    int walk_shift = 0;

    // per-kernel timing with HIP events on `stream` (crk_timing_*)
    int timing = 0;
    std::string timing_only;   // non-empty: only this kernel name is timed
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> ev_pend;
    std::map<std::string, std::pair<double, int64_t>> ev_total;
};

namespace crk {

crk_status set_err(crk_ctx *c, crk_status s, const char *fmt, ...);
crk_status hip_err(crk_ctx *c, hipError_t e, const char *what);
crk_status ensure(crk_ctx *c, Buf &b, size_t bytes);
void graph_release(crk_ctx *c);
// input checks of a build: non-finite values (CRK_ERR_NONFINITE), positions
// outside [0, L) (CRK_ERR_INVALID_ARG), H <= 0 (CRK_ERR_SUPPORT); *hmax and
// *hmin receive the extreme supports (synchronises the stream)
crk_status validate_inputs(crk_ctx *c, const double *x, const double *y, const double *z,
                           const double *H, int64_t n, double L, double *hmax, double *hmin);
// steps 2-4 of crk_build_cells_batch for the geometry held in the context
crk_status build_sorted(crk_ctx *c, const double *x, const double *y, const double *z,
                        const double *H, int32_t *perm, bool stand_ins, int64_t *n_pairs,
                        int32_t *n_cells);

// The compatible energy pass (crk_compatible_energy) for one kick, or, with
// du2, for two kicks that share the pair forces of one evaluation and start
// from the momenta pk and pk2 (a velocity-Verlet closing kick and the next
// opening kick): one pair loop, two sums. reuse: the arrays are those of the
// crk_derivatives call just made on this context (same state, same
// precision), whose packed records and FP64-row lists are used as they are.
crk_status compat_pass(crk_ctx *c, const crk_params *p, const double *v, const double *m,
                       const double *u, const double *rho, const double *V, const double *A,
                       const double *B, const double *gA, const double *gB, const double *gradv,
                       const double *dpdt, const double *pk, const double *pk2, double dt,
                       double *du, double *du2, bool reuse);

// Device status of a graph-mode step (written by the step's own kernels and
// read back by crk_graph_replay).
struct GraphStat {
    int64_t n_gather, n_extra;
    uint64_t n_singular;
    int64_t n_flag, n_touch;
    int32_t input_error, overflow, clear, state_error;
};

// Records a start/stop event pair around the launches in its scope when the
// context's timing is on; the pairs are read back by crk_timing_read.
struct KTimer {
    crk_ctx *c;
    const char *name;
    hipEvent_t a = nullptr, b = nullptr;
    KTimer(crk_ctx *ctx, const char *nm);
    ~KTimer();
};

// device-wide exclusive scan of n values (int64 in/out may alias)
crk_status scan_exclusive_i64(crk_ctx *c, const int64_t *in, int64_t *out, int64_t n);
// offsets of n rows from two int32 count arrays at once: oa[k] = sum of
// a[0..k) for k = 0..n (oa[n] the total), likewise ob from b (b and ob
// both null: a alone); with amax (device) also the largest entry of a (0
// when n = 0); with ob32 also ob[0..n) as int32 (the totals fit in 31 bits)
crk_status scan_counts2(crk_ctx *c, const int32_t *a, const int32_t *b, int64_t n, int64_t *oa,
                        int64_t *ob, int64_t *amax = nullptr, int32_t *ob32 = nullptr);
// stable LSD radix sort of (key, value) pairs on the low `bits` bits of the keys
crk_status radix_sort_pairs(crk_ctx *c, uint32_t *keys, int32_t *vals, int64_t n, int bits);

// grid index remap that gives each XCD a contiguous run of logical blocks:
// blocks are dispatched round-robin over the 8 XCDs, so block b runs on XCD
// b % 8; neighbouring particles then share that XCD's L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
    int64_t q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

// Minimum-image separation d = xi - xj in FP64 and r^2 = (dx dx + dy dy) + dz dz
// without contraction, so that neighbour decisions are reproducible bit for bit.
// (selects rather than branches: the wrapped value is d - L or d + L either way)
__device__ __forceinline__ double min_image(double d, double L, double hL) {
    const double up = d - L, dn = d + L;
    return d > hL ? up : (d < -hL ? dn : d);
}

__device__ __forceinline__ double r2_exact(double dx, double dy, double dz) {
#pragma clang fp contract(off)
    return (dx * dx + dy * dy) + dz * dz;
}

// ---- the FP64 volume sum of eq. (vol): shared by the volume pass and the
// build's compaction, which forms the same terms

// Square root of a squared distance x >= 0: Newton-Raphson refinement of the
// hardware reciprocal square root estimate y ~ 1/sqrt(x), as coupled
// iterations for s ~ sqrt(x) and h ~ 1/(2 sqrt(x)) (one coupled step, then
// two corrections of s by the residual x - s^2), the same steps the
// correctly rounded library square root takes for arguments of normal range.
// x is first raised to 2^-767, the bound below which the library rescales
// its argument: no distance of distinct particles comes near it, and at
// x = 0 the result (about 7e-116) leaves every kernel factor of the passes
// exactly as at 0.
__device__ __forceinline__ double sqrt_dist(double x) {
    x = fmax(x, 0x1p-767);
    const double y = __builtin_amdgcn_rsq(x);
    double s = x * y, h = 0.5 * y;
    const double r = fma(-h, s, 0.5);
    s = fma(s, r, s);
    h = fma(h, r, h);
    double d = fma(-s, s, x);
    s = fma(d, h, s);
    d = fma(-s, s, x);
    return fma(d, h, s);
}

struct Box {
    double L, invL;
};

// Minimum image of a listed pair: d - L rint(d / L), one fused rounding,
// so the value equals d, d - L or d + L exactly as the branch form gives;
// a listed pair has |d| < H < L/2 per component, far from the tie at L/2
// (neighbour decisions themselves use the branch form).
__device__ __forceinline__ double pair_image(double d, const Box &b) {
    return fma(-b.L, rint(d * b.invL), d);
}

// Wendland C4 weight of eq. (C4) at q = r/H with the prefactor cw = kW H^-3
template <typename T>
__device__ __forceinline__ T kernel_w(T q, T cw) {
    T s = q < (T)1 ? (T)1 - q : (T)0;
    T s2 = s * s;
    return cw * s2 * s2 * s2 * ((T)1 + q * ((T)6 + q * (T)(35.0 / 3.0)));
}


// Uniform periodic cell grid of side c = L / nc over the sorted particles.
struct Grid {
    double L, hL, inv_c, margin;
    int nc;
};

// cells along one axis overlapping [x - R, x + R], with a margin far above
// any rounding in the division; a range of nc or more cells is one period
__device__ __forceinline__ void axis_range(double x, double R, const Grid &g, int &lo, int &cnt) {
    int a = (int)floor((x - R - g.margin) * g.inv_c);
    int b = (int)floor((x + R + g.margin) * g.inv_c);
    cnt = b - a + 1;
    if (cnt >= g.nc) {
        a = 0;
        cnt = g.nc;
    }
    lo = a;
}

// Distance along one axis from p to the unwrapped cell k of side cs (0 when
// p is inside). Used to skip cells that lie wholly outside a support sphere;
// a walk only does so while its whole range stays within half a period of p
// (then the unwrapped cell is the nearest image of every particle in it).
__device__ __forceinline__ double cell_gap(double p, int k, double cs) {
    double lo = (double)k * cs, hi = lo + cs;
    return fmax(0.0, fmax(lo - p, p - hi));
}

// cell ranges a lane group lists in LDS at a time in the flattened walks
// (at most; flat_ranges<G>() is two steps of G cells, at least 8, so the
// lists of a 256-thread block stay near 16 KB whatever G)
constexpr int kRanges = 32;
template <int G>
__host__ __device__ constexpr int flat_ranges() {
    return 2 * G < 8 ? 8 : (2 * G > kRanges ? kRanges : 2 * G);
}

// exclusive prefix sum of x over a group of G lanes (total to every lane)
template <int G>
__device__ __forceinline__ int group_excl_scan(int x, int l, int &total) {
    int inc = x;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        int t = __shfl_up(inc, o, G);
        if (l >= o) inc += t;
    }
    total = __shfl(inc, G - 1, G);
    return inc - x;
}

// periodic cell index: every level has a power-of-two number of cells a
// side, so the wrap is a mask (two's complement keeps it right for a < 0)
__device__ __forceinline__ int wrapc(int a, int nc) { return a & (nc - 1); }


// Morton cell hierarchy: level k has nc >> k cells a side, side c0 2^k, and
// its table starts at off[k] in cbeg/cend (indexed by the level-k Morton id).
// Boxes of a batch share one sort: a particle's key is (box << 3 bits) |
// Morton code, and box b's tables start at b * box_stride.
struct Levels {
    double L, hL, c0, margin;
    int bits;
    int64_t off[12];
    const uint32_t *skey;   // sorted keys (box id in the bits above 3 * bits)
    int64_t box_stride;     // table entries per box
};

__device__ __forceinline__ int64_t box_base(const Levels &v, int64_t i) {
    return (int64_t)(v.skey[i] >> (3 * v.bits)) * v.box_stride;
}

__device__ __forceinline__ uint32_t spread3(uint32_t v) {   // 10 bits -> every third bit
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

// level whose cell side is at least R/2 (so at most five cells a side cover
// the support), capped at the single-cell level
__device__ __forceinline__ int level_for(double R, const Levels &v) {
    int k = 0;
    double c = v.c0;
    while (k < v.bits && c < 0.5 * R) {
        c *= 2.0;
        k++;
    }
    return k;
}

// scratch row slots for gather rows of g entries in all over n particles:
// 2.5 times the mean row, rounded up to a multiple of 64, at most 1024
__host__ __device__ inline int walk_cap_for(double g, double n) {
    const double m = n > 0.0 ? 2.5 * g / n : 0.0;
    const double c = 64.0 * std::ceil(m / 64.0);
    return (int)(c < 1024.0 ? c : 1024.0);
}

// The most slots per scratch row that still fit 2^33 slots (32 GiB) for n
// particles, a multiple of 64 and at most 1024.
inline int walk_cap_limit(double n) {
    const double c = n > 0.0 ? 64.0 * std::floor(8589934592.0 / n / 64.0) : 1024.0;
    return (int)(c < 1024.0 ? c : 1024.0);
}

// Slots of the next walk's scratch rows after a build with g gather pairs
// whose longest row held `longest`: room for that row and an eighth more
// (rounded up to 64) within walk_cap_limit, and never below walk_cap_for, so
// that rows of the next step are walked twice only where they grew past it.
inline int walk_cap_next(double g, double n, int64_t longest) {
    const double want = 64.0 * std::ceil(((double)longest + (double)longest / 8.0) / 64.0);
    const double lim = (double)walk_cap_limit(n);
    const int c = (int)(want < lim ? want : lim);
    const int f = walk_cap_for(g, n);
    return c > f ? c : f;
}

// Per-axis tables of a flattened walk. The walked cells form an
// mx x my x mz box, so the work per cell is separable: a group first
// tabulates, for the cells lo_a .. lo_a + m_a - 1 along each axis a, the
// Morton bits of the wrapped index (bits 0..29) with the axis's image shift
// code above them (bits 30..31: 0 none, 1 +L, 2 -L), the shift itself and
// the squared gap from the particle to the unwrapped cell; a listed cell
// then costs three table reads instead of three bit spreads and three gap
// evaluations. At most 6 cells a side: the walked level's side is at least
// half the radius, so a support spans at most 5 cell boundaries.
constexpr int kAxisCells = 8;
struct AxisTab {
    uint32_t id[3][kAxisCells];
    double g2[3][kAxisCells];
    double sh[3][kAxisCells];
};

// ceil(2^16 / m): (x * it) >> 16 is x / m rounded down for every x < 512 and
// m <= 8 (the error, below 512 / 2^16, stays under the 1/8 gap)
__device__ __forceinline__ uint32_t div16(int m) { return (uint32_t)((65536 + m - 1) / m); }

// fill the tables of one particle (G lanes of a group; SH: the shifts too);
// coordinates are selected as values (a selected reference would put pi in
// private memory)
template <int G, bool CULL, bool SH = true>
__device__ __forceinline__ void fill_axes(AxisTab &tab, const double4 &pi, int l, int lx, int ly, int lz,
                                          int mx, int my, int mz, int nck, double cs, double L) {
    const double px = pi.x, py = pi.y, pz = pi.z;
    for (int t = l; t < mx + my + mz; t += G) {
        int ax = 0, idx = t, k = lx + t;
        double p = px;
        if (t >= mx + my) {
            ax = 2;
            idx = t - mx - my;
            k = lz + idx;
            p = pz;
        } else if (t >= mx) {
            ax = 1;
            idx = t - mx;
            k = ly + idx;
            p = py;
        }
        uint32_t id = spread3(wrapc(k, nck)) << ax;
        double g2 = 0.0, sh = 0.0;
        if (CULL) {
            const int code = k < 0 ? 1 : (k >= nck ? 2 : 0);
            id |= (uint32_t)code << 30;
            sh = code == 1 ? L : (code == 2 ? -L : 0.0);
            const double g = cell_gap(p, k, cs);
            g2 = g * g;
        }
        tab.id[ax][idx] = id;
        tab.g2[ax][idx] = g2;
        if (SH) tab.sh[ax][idx] = sh;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Flattened walk of the cells that a sphere of radius R about particle i
// overlaps, by an aligned group of G lanes (4 <= G <= NR) of one wavefront.
// The group lists its cells as ranges of sorted particles in LDS (sb: first
// particle, sc[NR + 1]: offset in the concatenation, sx[3 NR]: the FP64
// image shift of the cell's particles; NR at a time), skipping cells wholly
// outside R when the range stays within half a period (then each listed
// cell carries the image shift of all its particles), and then takes the
// concatenated candidates G at a time across cell boundaries, so the loads
// of different cells overlap.
// visit(valid, r2) sees every batch on every lane (valid false past the
// end; r2 the exact FP64 minimum-image r^2 with i itself included) and
// returns true to stop the walk; its value must be the same on every lane
// of the group.
template <int G, int NR, typename Visit>
__device__ __forceinline__ void flat_candidates(const double4 *__restrict__ posH,
                                                const int32_t *__restrict__ cbeg,
                                                const int32_t *__restrict__ cend, const Levels &v,
                                                int64_t i, const double4 &pi, double R, int l,
                                                int32_t *sb, int32_t *sc, double *sx, AxisTab &tab,
                                                Visit &&visit) {
    static_assert(G >= 4 && G <= NR, "the flattened walk needs 4..NR lanes");
    const int gshift = (threadIdx.x & 63) - l;
    const uint64_t gmask = ((uint64_t)1 << G) - 1;
    const uint64_t below = ((uint64_t)1 << l) - 1;
    const int k = level_for(R, v);
    const int nck = 1 << (v.bits - k);
    Grid g{v.L, v.hL, (double)nck / v.L, v.margin, nck};
    int lx, ly, lz, mx, my, mz;
    axis_range(pi.x, R, g, lx, mx);
    axis_range(pi.y, R, g, ly, my);
    axis_range(pi.z, R, g, lz, mz);
    const int64_t base = box_base(v, i) + v.off[k];
    const int32_t *cb = cbeg + base, *ce = cend + base;
    const double cs = v.L / (double)nck;
    const double Rc = R + 2.0 * v.margin;   // far above any rounding of the gaps
    const bool cull = 2.0 * (Rc + cs) < v.L;
    const double Rc2 = Rc * Rc;
    const double L = v.L;
    const int ncell = mx * my * mz;
    if (cull)
        fill_axes<G, true>(tab, pi, l, lx, ly, lz, mx, my, mz, nck, cs, L);
    else
        fill_axes<G, false>(tab, pi, l, lx, ly, lz, mx, my, mz, nck, cs, L);
    const uint32_t dvx = div16(mx), dvy = div16(my);
    int c0 = 0;
    bool stop = false;
    while (c0 < ncell && !stop) {
        int nr = 0, cum = 0;
        while (c0 < ncell && nr + G <= NR) {
            const int cidx = c0 + l;
            int jb = 0, len = 0;
            double cx = 0.0, cy = 0.0, cz = 0.0;
            if (cidx < ncell) {
                const int t = (int)(((uint32_t)cidx * dvx) >> 16);
                const int e = cidx - t * mx;
                const int a = (int)(((uint32_t)t * dvy) >> 16);
                const int b = t - a * my;
                const bool keep = !cull || (tab.g2[2][a] + tab.g2[1][b]) + tab.g2[0][e] <= Rc2;
                if (keep) {
                    const uint32_t id = (tab.id[0][e] | tab.id[1][b] | tab.id[2][a]) & 0x3fffffffu;
                    cx = tab.sh[0][e];
                    cy = tab.sh[1][b];
                    cz = tab.sh[2][a];
                    jb = cb[id];
                    len = ce[id] - jb;
                }
            }
            int tot;
            const int pre = group_excl_scan<G>(len, l, tot);
            const bool has = len > 0;
            const uint64_t hm = (__ballot(has) >> gshift) & gmask;
            if (has) {
                const int p = nr + __popcll(hm & below);
                sb[p] = jb;
                sc[p] = cum + pre;
                sx[3 * p + 0] = cx;
                sx[3 * p + 1] = cy;
                sx[3 * p + 2] = cz;
            }
            nr += __popcll(hm);
            cum += tot;
            c0 += G;
        }
        if (l == 0) sc[nr] = cum;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        int r = 0;
        for (int f0 = 0; f0 < cum; f0 += G) {
            const int f = f0 + l;
            double r2 = 0.0;
            if (f < cum) {
                while (sc[r + 1] <= f) r++;
                const int j = sb[r] + (f - sc[r]);
                const double4 pj = posH[j];
                double dx, dy, dz;
                if (cull) {
                    dx = (pi.x - pj.x) + sx[3 * r + 0];
                    dy = (pi.y - pj.y) + sx[3 * r + 1];
                    dz = (pi.z - pj.z) + sx[3 * r + 2];
                } else {
                    dx = min_image(pi.x - pj.x, v.L, v.hL);
                    dy = min_image(pi.y - pj.y, v.L, v.hL);
                    dz = min_image(pi.z - pj.z, v.L, v.hL);
                }
                r2 = r2_exact(dx, dy, dz);
            }
            if (visit(f < cum, r2)) {
                stop = true;
                break;
            }
        }
        // the lists are rewritten by the next batch only after every lane read them
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}


// Walks every cell of the level chosen for radius R that overlaps the cube
// [x - R, x + R]^3 (periodic), calling f(j) for each particle j in them, in a
// fixed order: cells z-major, then y, then x; particles in sorted order.
template <typename F>
__device__ __forceinline__ void walk_cells(const Levels &v, const int32_t *__restrict__ cbeg,
                                           const int32_t *__restrict__ cend, int64_t i, double px,
                                           double py, double pz, double R, F &&f) {
    int k = level_for(R, v);
    int nck = 1 << (v.bits - k);
    Grid g{v.L, v.hL, (double)nck / v.L, v.margin, nck};
    int lx, ly, lz, mx, my, mz;
    axis_range(px, R, g, lx, mx);
    axis_range(py, R, g, ly, my);
    axis_range(pz, R, g, lz, mz);
    const int64_t base = box_base(v, i) + v.off[k];
    const int32_t *cb = cbeg + base, *ce = cend + base;
    for (int a = 0; a < mz; a++) {
        uint32_t mzb = spread3(wrapc(lz + a, nck)) << 2;
        for (int b = 0; b < my; b++) {
            uint32_t myb = mzb | (spread3(wrapc(ly + b, nck)) << 1);
            for (int e = 0; e < mx; e++) {
                uint32_t id = myb | spread3(wrapc(lx + e, nck));
                int jb = cb[id], je = ce[id];
                for (int j = jb; j < je; j++) f(j);
            }
        }
    }
}

// device address of the allocation-free training step's static scratch,
// taken once per device (the device current); called by crk_create
crk_status hnet_scratch_init(crk_ctx *c);

// geometry of the last build as seen by the walks (host side)
Levels levels(const crk_ctx *c);

// zero `words` 32-bit words on the context's stream with a kernel (not a
// memset node, so the call can sit inside a captured graph)
crk_status zero_async(crk_ctx *c, void *p, int64_t words);

}  // namespace crk

#define CRK_HIP(c, call)                                                   \
    do {                                                                   \
        hipError_t e_ = (call);                                            \
        if (e_ != hipSuccess) return crk::hip_err((c), e_, #call);         \
    } while (0)

#define CRK_TRY(expr)                                                      \
    do {                                                                   \
        crk_status s_ = (expr);                                            \
        if (s_ < 0) return s_;                                             \
    } while (0)
