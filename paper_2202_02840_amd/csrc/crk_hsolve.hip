// S3: smoothing-length iteration, eqs. (hi) and (thacker).
//
// Each particle's neighbour count depends only on its own H and the fixed
// positions, so every particle iterates on its own inside one launch: no host
// round trip per iteration. Each iteration re-walks the cells that the
// current support overlaps (the cell grid is fixed, the walk range follows H),
// so H may grow past the cell side. FP64 throughout: the converged H is
// compared across implementations at 1e-6.
#include <math.h>

#include "crk_internal.h"

namespace crk {
namespace {

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

// Candidate row of particle i: the exact FP64 r^2 of every j within R (self
// included), in cell-walk order, in a row of cap slots, by a group of G
// lanes (a ballot orders the hits). Returns the number of candidates, which
// exceeds cap when the row could not hold them all.
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
                        if (p < cap) row[p] = r2;
                    }
                    c += __popcll(hm);
                }
            }
        }
    }
    return c;
}

// n_i(H) from a candidate row (valid while H <= the row's radius)
template <int G>
__device__ __forceinline__ double nsum_row(const double *__restrict__ row, int c, double H, int l) {
    const double H2 = H * H, invH = 1.0 / H;
    double s = 0.0;
    // four loads in flight per lane: the row streams from memory, so the
    // latency, not the arithmetic, sets the pace
    int k = l;
    for (; k + 3 * G < c; k += 4 * G) {
        double r[4] = {row[k], row[k + G], row[k + 2 * G], row[k + 3 * G]};
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (r[u] < H2) {
                double q = sqrt(r[u]) * invH;
                double t = 1.0 - q, t2 = t * t;
                s += t2 * t2 * t2 * (1.0 + q * (6.0 + q * (35.0 / 3.0)));
            }
    }
    for (; k < c; k += G) {
        double r2 = row[k];
        if (r2 < H2) {
            double q = sqrt(r2) * invH;
            double t = 1.0 - q, t2 = t * t;
            s += t2 * t2 * t2 * (1.0 + q * (6.0 + q * (35.0 / 3.0)));
        }
    }
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) s += __shfl_xor(s, m, G);
    return kW * invH * invH * invH * s;
}

// One round: each listed particle takes up to R more updates of eq. (thacker)
// from its stored state. state[i]: 0 running, 1 converged, 2 hit max_iter,
// 3 support reached L/2.
template <int G>
__global__ __launch_bounds__(kBlock) void k_hsolve_round(const double4 *__restrict__ posH,
                                                         const int32_t *__restrict__ cbeg,
                                                         const int32_t *__restrict__ cend, Levels v,
                                                         const int32_t *__restrict__ list, int64_t m,
                                                         double Nres, double tol, int max_iter, int R,
                                                         double *rows, int32_t *rcnt, double *Rlist,
                                                         int cap, double f, double *H_io,
                                                         int32_t *iters, int32_t *state) {
    int64_t gid = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const int l = (int)(gid % G);
    const int64_t k = gid / G;
    if (k >= m) return;
    const int64_t i = list[k];
    const double4 pi = posH[i];
    double H = H_io[i];
    int it = iters[i];
    int st = 0;
    int c = rows ? rcnt[i] : cap + 1;
    double Rmax = rows ? Rlist[i] : 0.0;
    double *row = rows ? rows + (size_t)i * cap : nullptr;
    // a support that left its candidate row (or has none yet) gets a new
    // row at f H, which serves every later update with H <= f H without a
    // cell walk; when f H holds more candidates than the row, a row just
    // past H is tried (it still serves the updates that shrink H)
    if (rows && !(c <= cap && H <= Rmax)) {
        Rmax = f * H;
        c = build_row<G>(posH, cbeg, cend, v, i, pi, Rmax, cap, row, l);
        if (c > cap && f > 1.02) {
            Rmax = 1.02 * H;
            c = build_row<G>(posH, cbeg, cend, v, i, pi, Rmax, cap, row, l);
        }
        if (l == 0) {
            rcnt[i] = c;
            Rlist[i] = Rmax;
        }
    }
    for (int r = 0; r < R; r++) {
        // the candidate row holds every j within Rmax, so it answers any H <= Rmax
        double ns = (c <= cap && H <= Rmax) ? nsum_row<G>(row, c, H, l)
                                            : nsum_group<G>(posH, cbeg, cend, v, i, pi, H, l);
        double N = (4.0 * kPi / 3.0) * H * H * H * ns;
        double D = cbrt(Nres / N);
        double lam = D < 1.0 ? 0.2 * (1.0 + D * D) : 0.2 * (1.0 + 1.0 / (D * D * D));
        double Hn = H * (1.0 - lam + lam * D);
        it++;
        bool done = fabs(Hn - H) <= tol * H;
        H = Hn;
        if (!(H < v.hL)) { st = 3; break; }
        if (done) { st = 1; break; }
        if (it >= max_iter) { st = 2; break; }
    }
    if (l == 0) {
        H_io[i] = H;
        iters[i] = it;
        state[i] = st;
    }
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

// running[k] = 1 when list[k] is still running (for the compaction scan)
__global__ __launch_bounds__(kBlock) void k_hs_running(const int32_t *__restrict__ list, int64_t m,
                                                       const int32_t *__restrict__ state, int64_t *run) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < m) run[k] = state[list[k]] == 0;
    if (k == m) run[m] = 0;
}

__global__ __launch_bounds__(kBlock) void k_hs_compact(const int32_t *__restrict__ list, int64_t m,
                                                       const int64_t *__restrict__ pos, int32_t *out) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k < m && pos[k + 1] != pos[k]) out[pos[k]] = list[k];
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
    int64_t m = n;
    int64_t *pin = (int64_t *)c->pinned.p + 24;
    const int G = c->G_hsolve;
    {
        KTimer kt_(c, "k_hsolve");
        while (m > 0) {
            // few particles left (the slowly contracting tail): give each one
            // more lanes so the device stays busy, and run longer rounds
            int Gr = G;
            while (Gr < 64 && m * Gr < (int64_t)1 << 19) Gr *= 2;
            const int R = Gr > G ? 4 * c->hs_round : c->hs_round;
#define L_HS(GG) k_hsolve_round<GG><<<(unsigned)((m * GG + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>((const double4 *)c->posH.p, (const int32_t *)c->cbeg.p, (const int32_t *)c->cend.p, v, la, m, Nres, tol, max_iter, R, rows, rcnt, Rl, cap, c->hs_factor, H_inout, it, state)
            switch (Gr) {
                case 1: L_HS(1); break;
                case 2: L_HS(2); break;
                case 4: L_HS(4); break;
                case 8: L_HS(8); break;
                case 16: L_HS(16); break;
                case 32: L_HS(32); break;
                case 64: L_HS(64); break;
                default: return set_err(c, CRK_ERR_INVALID_ARG, "hsolve lanes must be a power of two <= 64");
            }
#undef L_HS
            const unsigned mb = (unsigned)((m + 1 + kBlock - 1) / kBlock);
            k_hs_running<<<mb, kBlock, 0, c->stream>>>(la, m, state, pos);
            CRK_TRY(scan_exclusive_i64(c, pos, pos, m + 1));
            k_hs_compact<<<mb, kBlock, 0, c->stream>>>(la, m, pos, lb);
            CRK_HIP(c, hipGetLastError());
            CRK_HIP(c, hipMemcpyAsync(pin, pos + m, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
            CRK_HIP(c, hipStreamSynchronize(c->stream));
            m = pin[0];
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
