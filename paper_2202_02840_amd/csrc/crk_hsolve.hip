// S3: smoothing-length iteration, eqs. (hi) and (thacker).
//
// Each particle's neighbour count depends only on its own H and the fixed
// positions, so every particle iterates on its own: a round launch takes up
// to R updates per listed particle, stopped particles are compacted out
// between rounds. Each particle keeps a candidate row (the distances of
// every j within a radius a little above H), so an update re-sums W from the
// row instead of walking the cells; a row is rebuilt when H leaves it, and a
// support whose row would overflow goes to a wide pass (a wavefront per
// particle, larger rows, cell walks as the last resort). FP64 throughout:
// the converged H is compared across implementations at 1e-6.
#include <math.h>

#include "crk_internal.h"

namespace crk {
namespace {

// wide-pass rows: kPoolCap slots each (or 8 cap), for at most kPoolBytes of
// rows per launch (262144 particles at 4096 slots)
constexpr int64_t kPoolBytes = (int64_t)8 << 30;
constexpr int kPoolCap = 4096;
// row slots per lane held in registers by the narrow pass (8 and 16 lanes)
constexpr int kRegSlots8 = 40;
constexpr int kRegSlots16 = 20;

// n_i(H) by a group of G lanes: the group walks i's cells together, lanes
// take a cell's particles G at a time, and the partial sums are combined
// with cross-lane shuffles (every lane ends with the same total).
template <int G>
__device__ __forceinline__ double nsum_group(const double4 *__restrict__ posH,
                                             const int32_t *__restrict__ cbeg,
                                             const int32_t *__restrict__ cend, const Levels &v,
                                             int64_t i, const double4 &pi, double H, int l) {
    const double H2 = H * H, invH = 1.0 / H;
    double s = 0.0;
    int k = level_for(H, v);
    int nck = 1 << (v.bits - k);
    Grid g{v.L, v.hL, (double)nck / v.L, v.margin, nck};
    int lx, ly, lz, mx, my, mz;
    axis_range(pi.x, H, g, lx, mx);
    axis_range(pi.y, H, g, ly, my);
    axis_range(pi.z, H, g, lz, mz);
    const int64_t base = box_base(v, i) + v.off[k];
    const int32_t *cb = cbeg + base, *ce = cend + base;
    for (int a = 0; a < mz; a++) {
        uint32_t mzb = spread3(wrapc(lz + a, nck)) << 2;
        for (int b = 0; b < my; b++) {
            uint32_t myb = mzb | (spread3(wrapc(ly + b, nck)) << 1);
            for (int e = 0; e < mx; e++) {
                uint32_t id = myb | spread3(wrapc(lx + e, nck));
                int je = ce[id];
                for (int j = cb[id] + l; j < je; j += G) {
                    double4 pj = posH[j];
                    double dx = min_image(pi.x - pj.x, v.L, v.hL);
                    double dy = min_image(pi.y - pj.y, v.L, v.hL);
                    double dz = min_image(pi.z - pj.z, v.L, v.hL);
                    double r2 = r2_exact(dx, dy, dz);
                    if (r2 < H2) {
                        double q = sqrt(r2) * invH;
                        double t = 1.0 - q, t2 = t * t;
                        s += t2 * t2 * t2 * (1.0 + q * (6.0 + q * (35.0 / 3.0)));
                    }
                }
            }
        }
    }
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) s += __shfl_xor(s, m, G);
    return kW * invH * invH * invH * s;
}

// Candidate row of particle i: the distance r of every j within R (self
// included; membership decided on the exact FP64 r^2), in cell-walk order,
// in a row of cap slots, by a group of G lanes (a ballot orders the hits).
// The square root is taken here once, not at every update. Returns the
// number of candidates, or a number above cap as soon as the row cannot hold
// them all (the walk stops there).
template <int G>
__device__ __forceinline__ int build_row(const double4 *__restrict__ posH,
                                         const int32_t *__restrict__ cbeg,
                                         const int32_t *__restrict__ cend, const Levels &v, int64_t i,
                                         const double4 &pi, double R, int cap, double *row, int l) {
    const double R2 = R * R;
    const int gshift = (threadIdx.x & 63) - l;
    const uint64_t below = (l == 0) ? 0ull : (((uint64_t)1 << l) - 1);
    int c = 0;
    int k = level_for(R, v);
    int nck = 1 << (v.bits - k);
    Grid g{v.L, v.hL, (double)nck / v.L, v.margin, nck};
    int lx, ly, lz, mx, my, mz;
    axis_range(pi.x, R, g, lx, mx);
    axis_range(pi.y, R, g, ly, my);
    axis_range(pi.z, R, g, lz, mz);
    const int64_t base = box_base(v, i) + v.off[k];
    const int32_t *cb = cbeg + base, *ce = cend + base;
    for (int a = 0; a < mz; a++) {
        uint32_t mzb = spread3(wrapc(lz + a, nck)) << 2;
        for (int b = 0; b < my; b++) {
            uint32_t myb = mzb | (spread3(wrapc(ly + b, nck)) << 1);
            for (int e = 0; e < mx; e++) {
                uint32_t id = myb | spread3(wrapc(lx + e, nck));
                int jb = cb[id], je = ce[id];
                for (int j0 = jb; j0 < je; j0 += G) {
                    int j = j0 + l;
                    bool hit = false;
                    double r2 = 0.0;
                    if (j < je) {
                        double4 pj = posH[j];
                        double dx = min_image(pi.x - pj.x, v.L, v.hL);
                        double dy = min_image(pi.y - pj.y, v.L, v.hL);
                        double dz = min_image(pi.z - pj.z, v.L, v.hL);
                        r2 = r2_exact(dx, dy, dz);
                        hit = r2 < R2;
                    }
                    // 64-bit masks: a group may be a whole wavefront
                    const uint64_t hm = (__ballot(hit) >> gshift) &
                                        ((G == 64) ? ~0ull : (((uint64_t)1 << G) - 1));
                    if (hit) {
                        int p = c + __popcll(hm & below);
                        if (p < cap) row[p] = sqrt(r2);
                    }
                    c += __popcll(hm);
                    if (c > cap) return c;   // the same for every lane of the group
                }
            }
        }
    }
    return c;
}

// The same row by the flattened walk (flat_candidates): the loads of
// different cells overlap. Candidate order differs from build_row; the rows
// hold the same set.
template <int G>
__device__ __forceinline__ int build_row_flat(const double4 *__restrict__ posH,
                                              const int32_t *__restrict__ cbeg,
                                              const int32_t *__restrict__ cend, const Levels &v,
                                              int64_t i, const double4 &pi, double R, int cap,
                                              double *row, int l, int32_t *sb, int32_t *sc,
                                              double *sx, AxisTab &tab) {
    const double R2 = R * R;
    const int gshift = (threadIdx.x & 63) - l;
    const uint64_t gmask = ((uint64_t)1 << G) - 1;
    const uint64_t below = ((uint64_t)1 << l) - 1;
    int c = 0;
    flat_candidates<G, flat_ranges<G>()>(posH, cbeg, cend, v, i, pi, R, l, sb, sc, sx, tab,
                                         [&](bool valid, double r2) {
        const bool hit = valid && r2 < R2;
        const uint64_t hm = (__ballot(hit) >> gshift) & gmask;
        if (hit) {
            const int p = c + __popcll(hm & below);
            if (p < cap) row[p] = sqrt(r2);
        }
        c += __popcll(hm);
        return c > cap;   // the same for every lane of the group
    });
    return c;
}

// Unnormalised C4 weight (1-q)^6 (1 + 6q + 35q^2/3), zero for q >= 1 without
// a branch (the clamp makes the first factor vanish)
__device__ __forceinline__ double w_c4(double q) {
    const double t = fmax(1.0 - q, 0.0), t2 = t * t;
    return t2 * t2 * t2 * (1.0 + q * (6.0 + q * (35.0 / 3.0)));
}

// n_i(H) from a candidate row of distances (valid while H <= the row's
// radius); rows that are not a multiple of 4G long finish one slot at a time
template <int G>
__device__ __forceinline__ double nsum_row(const double *__restrict__ row, int c, double H, int l) {
    const double invH = 1.0 / H;
    double s = 0.0;
    int k = l;
    for (; k + 3 * G < c; k += 4 * G) {
        const double r0 = row[k], r1 = row[k + G], r2 = row[k + 2 * G], r3 = row[k + 3 * G];
        s += (w_c4(r0 * invH) + w_c4(r1 * invH)) + (w_c4(r2 * invH) + w_c4(r3 * invH));
    }
    for (; k < c; k += G) s += w_c4(row[k] * invH);
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) s += __shfl_xor(s, m, G);
    return kW * invH * invH * invH * s;
}

// Delta = x^(1/3) for x > 0 (x = Nres / N lies between ~1e-6 and ~3): an FP32
// seed from the hardware log2/exp2, then one Newton step in FP64, which
// squares the seed's ~1e-7 relative error to ~1e-14; the step's divisor
// 3 y^2 needs only the seed's accuracy, so a hardware reciprocal serves.
__device__ __forceinline__ double cube_root(double x) {
    const double y = (double)__builtin_amdgcn_exp2f(__builtin_amdgcn_logf((float)x) * (1.0f / 3.0f));
    return y - (y * y * y - x) * __builtin_amdgcn_rcp(3.0 * y * y);
}

// Everything a round needs besides its list (kernel argument by value)
struct HsArgs {
    const double4 *posH;
    const int32_t *cbeg, *cend;
    Levels v;
    double Nres, inv_Nres, tol, f;
    int max_iter, cap;
    double *rows;   // n rows of cap slots (nullptr: no rows, every update walks)
    int32_t *rcnt;
    double *Rlist;
    double *H;
    int32_t *iters, *state;
};

// Takes updates of eq. (thacker) from H until stop or R updates; returns the
// state (0 running, 1 converged, 2 hit max_iter, 3 support reached L/2).
// NS(H) gives n_i(H) and is the only part that differs between passes.
template <typename NSum>
__device__ __forceinline__ int thacker_updates(const HsArgs &a, double &H, int &it, int R,
                                               double Rmax, bool stop_outside, NSum &&NS) {
    for (int r = 0; r < R; r++) {
        if (stop_outside && !(H <= Rmax)) return 0;   // a new row next round
        const double ns = NS(H);
        const double N = (4.0 * kPi / 3.0) * H * H * H * ns;
        const double x = a.Nres / N;   // Delta^3
        const double D = cube_root(x);
        const double lam = D < 1.0 ? 0.2 * (1.0 + D * D) : 0.2 * (1.0 + N * a.inv_Nres);
        const double Hn = H * (1.0 - lam + lam * D);
        it++;
        const bool done = fabs(Hn - H) <= a.tol * H;
        H = Hn;
        if (!(H < a.v.hL)) return 3;
        if (done) return 1;
        if (it >= a.max_iter) return 2;
    }
    return 0;
}

// A row at f H for particle i (which then serves every update with H <= f H
// without a cell walk); when f H holds more candidates than the row, a row
// just past H is tried (it still serves the updates that shrink H).
// (FLAT: the flattened walk, with the group's LDS lists sb, sc, sx and axis
// tables)
template <int G, bool FLAT = false>
__device__ __forceinline__ int make_row(const HsArgs &a, int64_t i, const double4 &pi, double H,
                                        int rcap, double *row, double &Rmax, int l,
                                        int32_t *sb = nullptr, int32_t *sc = nullptr,
                                        double *sx = nullptr, AxisTab *tab = nullptr) {
    auto build = [&](double R) {
        if constexpr (FLAT)
            return build_row_flat<G>(a.posH, a.cbeg, a.cend, a.v, i, pi, R, rcap, row, l, sb, sc, sx, *tab);
        else
            return build_row<G>(a.posH, a.cbeg, a.cend, a.v, i, pi, R, rcap, row, l);
    };
    Rmax = a.f * H;
    int c = build(Rmax);
    if (c > rcap && a.f > 1.02) {
        Rmax = 1.02 * H;
        c = build(Rmax);
    }
    return c;
}

// One round of list[k] with G lanes per particle (state 4: running, but its
// support holds more candidates than a row of cap slots).
//
// Narrow pass (pool == nullptr, defer set): rows of cap slots kept per
// particle across rounds. A particle never walks the cells here: when its
// row cannot be built it is handed to the wide pass (state 4), and when H
// leaves its row it stops for this round (the next round rebuilds the row),
// so no group holds up the launch with a long walk.
// Wide pass (pool set, 64 lanes): a row of pcap slots per listed particle,
// built at the start of every round in pool[k]; a support beyond even that
// row walks the cells at every update. A particle goes back to the narrow
// pass once its row fits cap slots.
// Neither (no rows, or the tail where a particle has a wavefront): rows kept
// as in the narrow pass, cell walks where a row does not serve.
template <int G>
__device__ __forceinline__ void round_body(const HsArgs &a, const int32_t *__restrict__ list,
                                           int64_t k, int l, int R, double *pool, int pcap,
                                           int defer) {
    const int64_t i = list[k];
    const double4 pi = a.posH[i];
    double H = a.H[i];
    int it = a.iters[i];
    int c, rcap;
    double Rmax;
    double *row;
    if (pool) {
        rcap = pcap;
        row = pool + (size_t)k * pcap;
        c = rcap + 1;
        Rmax = 0.0;
    } else {
        rcap = a.cap;
        row = a.rows ? a.rows + (size_t)i * a.cap : nullptr;
        c = a.rows ? a.rcnt[i] : a.cap + 1;
        Rmax = a.rows ? a.Rlist[i] : 0.0;
    }
    if (row && !(c <= rcap && H <= Rmax)) {
        c = make_row<G>(a, i, pi, H, rcap, row, Rmax, l);
        if (l == 0 && !pool) {
            a.rcnt[i] = c;
            a.Rlist[i] = Rmax;
        }
    }
    if (defer && c > rcap) {
        if (l == 0) a.state[i] = 4;
        return;
    }
    int st = thacker_updates(a, H, it, R, Rmax, defer != 0, [&](double h) {
        // the candidate row holds every j within Rmax, so it answers any h <= Rmax
        return (c <= rcap && h <= Rmax) ? nsum_row<G>(row, c, h, l)
                                        : nsum_group<G>(a.posH, a.cbeg, a.cend, a.v, i, pi, h, l);
    });
    // still running: the wide pass keeps a support that a narrow row cannot hold
    if (a.rows && st == 0 && c > a.cap) st = 4;
    if (l == 0) {
        a.H[i] = H;
        a.iters[i] = it;
        a.state[i] = st;
    }
}

// One lane's FP64 value from lane CTRL-selected within its DPP row (both
// 32-bit halves moved; every source lane lies in the row)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over an aligned group of G = 8 or 16 lanes; every lane ends with the
// same total (each step adds commuting pairs): swap neighbours, swap pairs,
// mirror the 8-lane halves, mirror the 16-lane row
template <int G>
__device__ __forceinline__ double group_sum(double s) {
    static_assert(G == 8 || G == 16, "DPP group sum covers 8 or 16 lanes");
    s += dpp_f64<0xB1>(s);   // quad_perm(1,0,3,2)
    s += dpp_f64<0x4E>(s);   // quad_perm(2,3,0,1)
    s += dpp_f64<0x141>(s);  // row_half_mirror
    if constexpr (G == 16) s += dpp_f64<0x140>(s);  // row_mirror
    return s;
}

// Narrow pass with the row held in registers: the round loads each
// particle's row once (slot s of lane l holds candidate s G + l, empty slots
// a distance of 2 Rmax, whose weight is zero) and every update sums from
// registers; the same hand-over rules as the narrow pass of round_body.
template <int G, int S>
__device__ __forceinline__ void narrow_body(const HsArgs &a, const int32_t *__restrict__ list,
                                            int64_t k, int l, int R) {
    const int64_t i = list[k];
    const double4 pi = a.posH[i];
    double H = a.H[i];
    int it = a.iters[i];
    int c = a.rcnt[i];
    double Rmax = a.Rlist[i];
    double *row = a.rows + (size_t)i * a.cap;
    if (!(c <= a.cap && H <= Rmax)) {
        constexpr int NR = flat_ranges<G>();
        __shared__ int32_t s_b[kBlock / G][NR], s_c[kBlock / G][NR + 1];
        __shared__ double s_x[kBlock / G][3 * NR];
        __shared__ AxisTab s_ax[kBlock / G];
        const int grp = (threadIdx.x & (kBlock - 1)) / G;
        c = make_row<G, true>(a, i, pi, H, a.cap, row, Rmax, l, s_b[grp], s_c[grp], s_x[grp], &s_ax[grp]);
        if (l == 0) {
            a.rcnt[i] = c;
            a.Rlist[i] = Rmax;
        }
    }
    if (c > a.cap) {
        if (l == 0) a.state[i] = 4;
        return;
    }
    double rr[S];
    const double pad = 2.0 * Rmax;
#pragma unroll
    for (int s = 0; s < S; s++) {
        const int q = s * G + l;
        rr[s] = q < c ? row[q] : pad;
    }
    const int st = thacker_updates(a, H, it, R, Rmax, true, [&](double h) {
        const double invH = 1.0 / h;
        double acc = 0.0;
#pragma unroll
        for (int s = 0; s < S; s++) {
            if (!__any(s * G < c)) break;
            acc += w_c4(rr[s] * invH);
        }
        return kW * invH * invH * invH * group_sum<G>(acc);
    });
    if (l == 0) {
        a.H[i] = H;
        a.iters[i] = it;
        a.state[i] = st;
    }
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_hsolve_round(HsArgs a, const int32_t *__restrict__ list,
                                                         int64_t m, int R, double *pool, int pcap,
                                                         int defer) {
    const int64_t gid = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const int64_t k = gid / G;
    if (k >= m) return;   // whole groups leave together
    round_body<G>(a, list, k, (int)(gid % G), R, pool, pcap, defer);
}

// One launch for both passes: the first nbw blocks (a multiple of 8, so the
// XCD of a narrow block is the one xcd_block assumes) take the wide list with
// a wavefront per particle and are dispatched first, since their particles
// are the slow ones; the other blocks take the narrow list with register
// rows. The two lists hold different particles.
template <int G, int S>
__global__ __launch_bounds__(kBlock) void k_hsolve_both(HsArgs a, const int32_t *__restrict__ ln,
                                                        int64_t mn, int Rn, const int32_t *__restrict__ lw,
                                                        int64_t mw, int Rw, int64_t nbw, double *pool,
                                                        int pcap) {
    if ((int64_t)blockIdx.x < nbw) {
        const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
        const int64_t k = gid / 64;
        if (k >= mw) return;
        round_body<64>(a, lw, k, (int)(gid % 64), Rw, pool, pcap, 0);
        return;
    }
    const int64_t gid = xcd_block(blockIdx.x - nbw, gridDim.x - nbw) * kBlock + threadIdx.x;
    const int64_t k = gid / G;
    if (k >= mn) return;
    narrow_body<G, S>(a, ln, k, (int)(gid % G), Rn);
}

__global__ __launch_bounds__(kBlock) void k_hs_init(int64_t n, int32_t *list, int32_t *iters, int32_t *state,
                                                    int32_t *rcnt, int cap) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    list[i] = (int32_t)i;
    iters[i] = 0;
    state[i] = 0;
    if (rcnt) rcnt[i] = cap + 1;   // no candidate row yet
}

// run[k]: 1 when list[k] runs on in the narrow pass, 1 << 32 when it runs on
// in the wide pass (one scan then counts both classes)
__global__ __launch_bounds__(kBlock) void k_hs_running(const int32_t *__restrict__ list, int64_t m,
                                                       const int32_t *__restrict__ state, int64_t *run) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < m) {
        const int s = state[list[k]];
        run[k] = s == 0 ? 1 : (s == 4 ? ((int64_t)1 << 32) : 0);
    }
    if (k == m) run[m] = 0;
}

// running particles to out: the narrow ones first, then the wide ones
__global__ __launch_bounds__(kBlock) void k_hs_compact(const int32_t *__restrict__ list, int64_t m,
                                                       const int64_t *__restrict__ pos, int32_t *out) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= m) return;
    const int64_t d = pos[k + 1] - pos[k];
    if (d == 1) out[pos[k] & 0xffffffff] = list[k];
    else if (d != 0) out[(pos[m] & 0xffffffff) + (pos[k] >> 32)] = list[k];
}

__global__ __launch_bounds__(kBlock) void k_hs_count(const int32_t *__restrict__ state, int64_t n,
                                                     unsigned long long *cnt) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    int s = state[i];
    if (s == 2) atomicAdd(&cnt[0], 1ull);
    if (s == 3) atomicAdd(&cnt[1], 1ull);
}

__global__ __launch_bounds__(kBlock) void k_set_H2(double4 *posH, const double *H, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) posH[i].w = H[i];
}

}  // namespace

// one round over list[0..m) with G lanes per particle
static crk_status hsolve_round(crk_ctx *c, const HsArgs &a, int G, const int32_t *list, int64_t m,
                               int R, double *pool, int pcap, int defer) {
    const unsigned nb = (unsigned)((m * G + kBlock - 1) / kBlock);
    switch (G) {
        case 1: k_hsolve_round<1><<<nb, kBlock, 0, c->stream>>>(a, list, m, R, pool, pcap, defer); break;
        case 2: k_hsolve_round<2><<<nb, kBlock, 0, c->stream>>>(a, list, m, R, pool, pcap, defer); break;
        case 4: k_hsolve_round<4><<<nb, kBlock, 0, c->stream>>>(a, list, m, R, pool, pcap, defer); break;
        case 8: k_hsolve_round<8><<<nb, kBlock, 0, c->stream>>>(a, list, m, R, pool, pcap, defer); break;
        case 16: k_hsolve_round<16><<<nb, kBlock, 0, c->stream>>>(a, list, m, R, pool, pcap, defer); break;
        case 32: k_hsolve_round<32><<<nb, kBlock, 0, c->stream>>>(a, list, m, R, pool, pcap, defer); break;
        case 64: k_hsolve_round<64><<<nb, kBlock, 0, c->stream>>>(a, list, m, R, pool, pcap, defer); break;
        default: return set_err(c, CRK_ERR_INVALID_ARG, "hsolve lanes must be a power of two <= 64");
    }
    CRK_HIP(c, hipGetLastError());
    return CRK_OK;
}

// both passes of a round in one launch (register rows of S slots for the
// narrow one); mw at most the pool's rows
template <int G, int S>
static crk_status hsolve_both(crk_ctx *c, const HsArgs &a, const int32_t *ln, int64_t mn, int Rn,
                              const int32_t *lw, int64_t mw, int Rw, double *pool, int pcap) {
    const int64_t nbw = (mw * 64 + kBlock - 1) / kBlock;
    const int64_t nbw8 = (nbw + 7) / 8 * 8;
    const int64_t nbn = (mn * G + kBlock - 1) / kBlock;
    k_hsolve_both<G, S><<<(unsigned)(nbw8 + nbn), kBlock, 0, c->stream>>>(a, ln, mn, Rn, lw, mw, Rw,
                                                                         nbw8, pool, pcap);
    CRK_HIP(c, hipGetLastError());
    return CRK_OK;
}
}  // namespace crk

using namespace crk;

extern "C" {

crk_status crk_hsolve(crk_ctx *c, double Nres, double tol, int32_t max_iter, double *H_inout,
                      int32_t *iters, int64_t *n_unconverged) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (!H_inout || max_iter < 1 || !(tol >= 0.0))
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_hsolve: bad argument");
    // the self term alone gives N = (4 pi / 3) * 495 / (32 pi) = 20.625
    if (!(Nres > 4.0 / 3.0 * kPi * kW))
        return set_err(c, CRK_ERR_INVALID_ARG, "Nres must exceed 20.625 (the self term alone)");
    if (c->nc == 0) return set_err(c, CRK_ERR_STATE, "crk_build_cells has not run");
    CRK_HIP(c, hipSetDevice(c->device));
    const int64_t n = c->n;
    Levels v = levels(c);
    CRK_TRY(ensure(c, c->hs_list, (size_t)2 * n * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->hs_state, (size_t)n * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->hs_pos, (size_t)(n + 1) * sizeof(int64_t)));
    CRK_TRY(ensure(c, c->hs_iters, (size_t)n * sizeof(int32_t)));
    int32_t *la = (int32_t *)c->hs_list.p, *lb = la + n;
    int32_t *state = (int32_t *)c->hs_state.p;
    int32_t *it = iters ? iters : (int32_t *)c->hs_iters.p;
    int64_t *pos = (int64_t *)c->hs_pos.p;
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    // candidate rows (positions do not move during the iteration); each
    // particle's first round builds its row
    const int cap = c->hs_cap;
    double *rows = nullptr;
    int32_t *rcnt = nullptr;
    double *Rl = nullptr;
    if (cap > 0) {
        CRK_TRY(ensure(c, c->hs_rows, (size_t)n * cap * sizeof(double)));
        CRK_TRY(ensure(c, c->hs_rcnt, (size_t)n * sizeof(int32_t)));
        CRK_TRY(ensure(c, c->hs_R, (size_t)n * sizeof(double)));
        rows = (double *)c->hs_rows.p;
        rcnt = (int32_t *)c->hs_rcnt.p;
        Rl = (double *)c->hs_R.p;
    }
    k_hs_init<<<nb, kBlock, 0, c->stream>>>(n, la, it, state, rcnt, cap);
    CRK_HIP(c, hipGetLastError());
    int64_t mn = n, mw = 0;   // narrow and wide particles still running
    const int pcap = kPoolCap < 8 * cap ? 8 * cap : kPoolCap;
    const int64_t prow = kPoolBytes / ((int64_t)pcap * (int64_t)sizeof(double));   // >= 2048
    const HsArgs a{(const double4 *)c->posH.p, (const int32_t *)c->cbeg.p, (const int32_t *)c->cend.p,
                   v, Nres, 1.0 / Nres, tol, c->hs_factor, max_iter, cap, rows, rcnt, Rl, H_inout, it,
                   state};
    int64_t *pin = (int64_t *)c->pinned.p + 24;
    const int G = c->G_hsolve;
    {
        KTimer kt_(c, "k_hsolve");
        while (mn + mw > 0) {
            // few particles left (the slowly contracting tail): give each one
            // more lanes so the device stays busy, and run longer rounds
            int Gr = G;
            while (Gr < 64 && mn * Gr < (int64_t)1 << 19) Gr *= 2;
            const int Rn = Gr > G ? 4 * c->hs_round : c->hs_round;
            // the wide pass runs longer rounds: its particles are few and slow
            const int Rw = 4 * c->hs_round;
            const int64_t mw0 = mw < prow ? mw : prow;   // wide particles in the first launch
            if (mw0 > 0) CRK_TRY(ensure(c, c->hs_pool, (size_t)mw0 * pcap * sizeof(double)));
            double *pool = (double *)c->hs_pool.p;
            const bool reg8 = rows && Gr == 8 && cap <= 8 * kRegSlots8;
            const bool reg16 = rows && Gr == 16 && cap <= 16 * kRegSlots16;
            if (mn > 0 && reg8)
                CRK_TRY((hsolve_both<8, kRegSlots8>(c, a, la, mn, Rn, la + mn, mw0, Rw, pool, pcap)));
            else if (mn > 0 && reg16)
                CRK_TRY((hsolve_both<16, kRegSlots16>(c, a, la, mn, Rn, la + mn, mw0, Rw, pool, pcap)));
            else {
                if (mn > 0) CRK_TRY(hsolve_round(c, a, Gr, la, mn, Rn, nullptr, 0, rows && Gr < 64));
                if (mw0 > 0) CRK_TRY(hsolve_round(c, a, 64, la + mn, mw0, Rw, pool, pcap, 0));
            }
            // wide particles beyond the pool: further launches reusing it
            for (int64_t w0 = mw0; w0 < mw; w0 += prow) {
                const int64_t mc = mw - w0 < prow ? mw - w0 : prow;
                CRK_TRY(hsolve_round(c, a, 64, la + mn + w0, mc, Rw, pool, pcap, 0));
            }
            const int64_t m = mn + mw;
            const unsigned mb = (unsigned)((m + 1 + kBlock - 1) / kBlock);
            k_hs_running<<<mb, kBlock, 0, c->stream>>>(la, m, state, pos);
            CRK_TRY(scan_exclusive_i64(c, pos, pos, m + 1));
            k_hs_compact<<<mb, kBlock, 0, c->stream>>>(la, m, pos, lb);
            CRK_HIP(c, hipGetLastError());
            CRK_HIP(c, hipMemcpyAsync(pin, pos + m, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
            CRK_HIP(c, hipStreamSynchronize(c->stream));
            mn = pin[0] & 0xffffffff;
            mw = pin[0] >> 32;
            int32_t *t = la;
            la = lb;
            lb = t;
        }
    }
    CRK_TRY(ensure(c, c->misc, 256));
    unsigned long long *cnt = (unsigned long long *)c->misc.p + 6;
    CRK_TRY(zero_async(c, cnt, 4));
    k_hs_count<<<nb, kBlock, 0, c->stream>>>(state, n, cnt);
    unsigned long long *pc = (unsigned long long *)c->pinned.p + 16;
    CRK_HIP(c, hipMemcpyAsync(pc, cnt, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
    CRK_HIP(c, hipStreamSynchronize(c->stream));
    if (n_unconverged) *n_unconverged = (int64_t)pc[0];
    if (pc[1]) return set_err(c, CRK_ERR_SUPPORT, "%llu supports reached L/2", pc[1]);
    // the lists no longer match the support radii
    c->built = 0;
    c->have_V = 0;
    c->vol_ready = 0;
    k_set_H2<<<nb, kBlock, 0, c->stream>>>((double4 *)c->posH.p, H_inout, n);
    CRK_HIP(c, hipGetLastError());
    if (pc[0]) return CRK_WARN_NOT_CONVERGED;
    return CRK_OK;
}

crk_status crk_set_hsolve(crk_ctx *c, int32_t lanes, int32_t round, int32_t cap, double factor) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (lanes < 0 || lanes > 64 || (lanes & (lanes - 1)))
        return set_err(c, CRK_ERR_INVALID_ARG, "hsolve lanes must be a power of two <= 64");
    if (round < 0 || cap < -1 || cap > 65536 || factor < 0.0)
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_set_hsolve: bad argument");
    if (lanes) c->G_hsolve = lanes;
    if (round) c->hs_round = round;
    if (cap) c->hs_cap = cap < 0 ? 0 : cap;
    if (factor > 0.0) c->hs_factor = factor;
    return CRK_OK;
}

}  // extern "C"
