// Alternative S1: recursive coordinate bisection (RCB) leaf tiling of the
// short-range solver (Sec. 3.3). The particles of each box are split by an
// RCB tree down to flat leaves of at most N_ppl particles (N_ppl in
// [128, 256] in the paper); each leaf gets one interaction list, the leaves
// whose boxes grown by the largest support of either leaf overlap its own,
// and the neighbour rows are found leaf pair by leaf pair with the partner
// leaf's particles staged in LDS. The result is the same gather and pair
// sets N_g, N_s as crk_build_cells (rows in tile order), in the leaf order.
//
// Tree. A coordinate is compared as the 32-bit fixed-point key
// q = floor(x / L 2^32) (ties by the original index). A node of more than
// `bucket` particles is split along the axis of largest key extent (lowest
// axis on a tie), its first floor(n/2) particles in key order going left;
// a leaf is the first node on a path with at most N_ppl particles; the
// buckets (<= bucket particles) below it order the leaf and let the walk
// skip partner particles in groups. Inside a bucket particles follow the x
// key.
//
// Build. Three copies of the particle list, sorted once by the x, y and z
// keys, are partitioned stably level by level (every node's split is then
// a prefix of its segment in the list of its axis): a flag per particle, a
// scan and a scatter per list and level. Node ranges follow from the box
// sizes alone (balanced halving), so the host lays them out; only the
// split axes depend on the data.
#include <math.h>

#include <algorithm>
#include <vector>

#include "crk_internal.h"

namespace crk {
namespace {

constexpr double kTwo32 = 4294967296.0;
constexpr int kLeafMax = 256;     // particles per leaf: one thread each
constexpr int kBucketsMax = 64;   // buckets per leaf

inline unsigned lblocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__device__ __forceinline__ uint32_t fixkey(double x, double L) {
    double q = floor(x / L * kTwo32);
    q = q < 0.0 ? 0.0 : (q > 4294967295.0 ? 4294967295.0 : q);
    return (uint32_t)q;
}

__global__ __launch_bounds__(kBlock) void k_rcb_keys(const double *x, const double *y, const double *z,
                                                     int64_t n, double L, uint32_t *q, uint32_t *sk,
                                                     int32_t *lv) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t a = fixkey(x[i], L), b = fixkey(y[i], L), c = fixkey(z[i], L);
    q[i] = a;
    q[n + i] = b;
    q[2 * n + i] = c;
    sk[i] = a;
    sk[n + i] = b;
    sk[2 * n + i] = c;
    lv[i] = lv[n + i] = lv[2 * n + i] = (int32_t)i;
}

// box id of each particle (box offsets) as a sort key
__global__ __launch_bounds__(kBlock) void k_box_keys(const int64_t *__restrict__ boff, int nboxes,
                                                     const int32_t *__restrict__ lv, int64_t n,
                                                     uint32_t *key) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int64_t i = lv[k];
    int lo = 0, hi = nboxes - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boff[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    key[k] = (uint32_t)lo;
}

// node of position p among the level's split nodes (begin-sorted, disjoint): -1 if none
__device__ __forceinline__ int node_of(int64_t p, const int32_t *__restrict__ nb,
                                       const int32_t *__restrict__ ns, int nnode) {
    int lo = 0, hi = nnode - 1;
    if (nnode == 0 || p < nb[0]) return -1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (nb[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return p < (int64_t)nb[lo] + ns[lo] ? lo : -1;
}

// split axis of every node: largest key extent, lowest axis on a tie
__global__ __launch_bounds__(kBlock) void k_rcb_axis(const int32_t *__restrict__ nb,
                                                     const int32_t *__restrict__ ns, int nnode,
                                                     const int32_t *__restrict__ lists,
                                                     const uint32_t *__restrict__ q, int64_t n,
                                                     int8_t *axis) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= nnode) return;
    const int64_t b = nb[k], e = b + ns[k];
    int best = 0;
    int64_t ext = -1;
    for (int a = 0; a < 3; a++) {
        const int32_t *la = lists + a * n;
        const int64_t x = (int64_t)q[a * n + la[e - 1]] - (int64_t)q[a * n + la[b]];
        if (x > ext) {
            ext = x;
            best = a;
        }
    }
    axis[k] = (int8_t)best;
}

// side of every particle of a split node (1: right half), read from the
// list of the node's axis; the node of every position for the moves
__global__ __launch_bounds__(kBlock) void k_rcb_flag(const int32_t *__restrict__ nb,
                                                     const int32_t *__restrict__ ns, int nnode,
                                                     const int8_t *__restrict__ axis,
                                                     const int32_t *__restrict__ lists, int64_t n,
                                                     int8_t *side, int32_t *pnode) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    const int k = node_of(p, nb, ns, nnode);
    pnode[p] = k;
    if (k < 0) return;
    const int32_t pid = lists[axis[k] * n + p];
    side[pid] = (p - nb[k]) >= (ns[k] >> 1) ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_rcb_sides(const int32_t *__restrict__ list,
                                                      const int32_t *__restrict__ pnode,
                                                      const int8_t *__restrict__ side, int64_t n,
                                                      int64_t *s) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p > n) return;
    s[p] = (p < n && pnode[p] >= 0) ? side[list[p]] : 0;
}

// stable partition of each split node's segment by side
__global__ __launch_bounds__(kBlock) void k_rcb_move(const int32_t *__restrict__ list,
                                                     const int32_t *__restrict__ pnode,
                                                     const int8_t *__restrict__ side,
                                                     const int64_t *__restrict__ s,
                                                     const int32_t *__restrict__ nb,
                                                     const int32_t *__restrict__ ns, int64_t n,
                                                     int32_t *out) {
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    const int32_t pid = list[p];
    const int k = pnode[p];
    if (k < 0) {
        out[p] = pid;
        return;
    }
    const int64_t b = nb[k];
    const int64_t right_before = s[p] - s[b];
    const int64_t to = side[pid] ? b + (ns[k] >> 1) + right_before : b + (p - b - right_before);
    out[to] = pid;
}

__global__ __launch_bounds__(kBlock) void k_leaf_gather(const double *x, const double *y, const double *z,
                                                        const double *H, const int32_t *perm,
                                                        int64_t n, double4 *posH) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int32_t i = perm[k];
    posH[k] = make_double4(x[i], y[i], z[i], H[i]);
}

// FP64 box (lo, hi) and largest support of every bucket: {lo.xyz, Hmax}, {hi.xyz, -}
__global__ __launch_bounds__(kBlock) void k_bucket_boxes(const double4 *__restrict__ posH,
                                                         const int32_t *__restrict__ boff, int nb,
                                                         double4 *blo, double4 *bhi) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= nb) return;
    double4 lo = make_double4(INFINITY, INFINITY, INFINITY, 0.0);
    double4 hi = make_double4(-INFINITY, -INFINITY, -INFINITY, 0.0);
    for (int32_t p = boff[k]; p < boff[k + 1]; p++) {
        const double4 q = posH[p];
        lo.x = fmin(lo.x, q.x);
        lo.y = fmin(lo.y, q.y);
        lo.z = fmin(lo.z, q.z);
        lo.w = fmax(lo.w, q.w);
        hi.x = fmax(hi.x, q.x);
        hi.y = fmax(hi.y, q.y);
        hi.z = fmax(hi.z, q.z);
    }
    blo[k] = lo;
    bhi[k] = hi;
}

// leaf boxes from their buckets
__global__ __launch_bounds__(kBlock) void k_leaf_boxes(const double4 *__restrict__ blo,
                                                       const double4 *__restrict__ bhi,
                                                       const int32_t *__restrict__ lbk, int nl,
                                                       double4 *llo, double4 *lhi) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= nl) return;
    double4 lo = make_double4(INFINITY, INFINITY, INFINITY, 0.0);
    double4 hi = make_double4(-INFINITY, -INFINITY, -INFINITY, 0.0);
    for (int32_t u = lbk[k]; u < lbk[k + 1]; u++) {
        const double4 a = blo[u], b = bhi[u];
        lo.x = fmin(lo.x, a.x);
        lo.y = fmin(lo.y, a.y);
        lo.z = fmin(lo.z, a.z);
        lo.w = fmax(lo.w, a.w);
        hi.x = fmax(hi.x, b.x);
        hi.y = fmax(hi.y, b.y);
        hi.z = fmax(hi.z, b.z);
    }
    llo[k] = lo;
    lhi[k] = hi;
}

// smallest periodic distance between two boxes (per axis the nearest of
// the three images of b), in a fixed order of roundings
__device__ __forceinline__ double box_gap(const double4 &la, const double4 &ha, const double4 &lb,
                                          const double4 &hb, double L) {
#pragma clang fp contract(off)
    const double al[3] = {la.x, la.y, la.z}, ah[3] = {ha.x, ha.y, ha.z};
    const double bl[3] = {lb.x, lb.y, lb.z}, bh[3] = {hb.x, hb.y, hb.z};
    const double sh[3] = {-L, 0.0, L};
    double g2 = 0.0;
    for (int a = 0; a < 3; a++) {
        double best = INFINITY;
        for (int t = 0; t < 3; t++) {
            const double g = fmax(0.0, fmax((bl[a] + sh[t]) - ah[a], al[a] - (bh[a] + sh[t])));
            best = fmin(best, g);
        }
        g2 = g2 + best * best;
    }
    return sqrt(g2);
}

// leaf interaction lists: leaves of the same box whose boxes come within
// max(Hmax_a, Hmax_b) (+ a margin far above rounding) of each other. FILL
// false counts, true writes the row (partners ascending).
template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_leaf_pairs(const double4 *__restrict__ llo,
                                                       const double4 *__restrict__ lhi,
                                                       const int32_t *__restrict__ lbox,
                                                       const int32_t *__restrict__ bleaf, int nl,
                                                       double L, double margin, int64_t *cnt,
                                                       const int64_t *__restrict__ off, int32_t *part) {
    const int a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= nl) return;
    const int box = lbox[a];
    const double4 la = llo[a], ha = lhi[a];
    int64_t c = 0, o = FILL ? off[a] : 0;
    for (int b = bleaf[box]; b < bleaf[box + 1]; b++) {
        const double4 lb = llo[b], hb = lhi[b];
        const double R = fmax(la.w, lb.w) + margin;
        if (box_gap(la, ha, lb, hb, L) < R) {
            if (FILL) part[o + c] = b;
            c++;
        }
    }
    if (!FILL) cnt[a] = c;
}

// Rows of one leaf: block per leaf A, thread t <-> particle A.begin + t.
// For each partner leaf B (A included) its particles and bucket boxes are
// staged in LDS; a wavefront skips a bucket none of its particles' supports
// (or the bucket's largest support) reaches, and tests the others' particles
// with the exact FP64 rule: d the minimum image of x_i - x_j (a per-pair
// image shift of the leaves when every pair of the two boxes is within half
// a period of it), r^2 = (dx dx + dy dy) + dz dz uncontracted, gather hit
// r^2 < H_i^2 (j != i), extra H_i^2 <= r^2 < H_j^2. Hits go to capped
// scratch rows with exact counts; DIRECT writes the rows of the particles
// whose counts passed a cap straight to their final places.
template <bool DIRECT>
__global__ __launch_bounds__(kBlock) void k_leaf_walk(const double4 *__restrict__ posH,
                                                      const int32_t *__restrict__ loff,
                                                      const int32_t *__restrict__ lbk,
                                                      const int32_t *__restrict__ bkoff,
                                                      const double4 *__restrict__ blo,
                                                      const double4 *__restrict__ bhi,
                                                      const double4 *__restrict__ llo,
                                                      const double4 *__restrict__ lhi,
                                                      const int64_t *__restrict__ poff,
                                                      const int32_t *__restrict__ part, double L,
                                                      double margin, int gcap, int xcap,
                                                      uint32_t *grow, uint32_t *xrow, int32_t *ng,
                                                      int32_t *ne, const int64_t *__restrict__ goff,
                                                      int32_t *gidx, const int64_t *__restrict__ eoff,
                                                      int32_t *eidx) {
    __shared__ double4 sp[kLeafMax];
    __shared__ double4 sbl[kBucketsMax], sbh[kBucketsMax];
    __shared__ int32_t sbo[kBucketsMax + 1];
    const int A = blockIdx.x;
    const int32_t a0 = loff[A], na = loff[A + 1] - a0;
    const int t = threadIdx.x;
    const bool act = t < na;
    const int64_t i = a0 + (act ? t : 0);
    const double4 pi = posH[i];
    const double Hi2 = pi.w * pi.w;
    const double hL = 0.5 * L;
    int32_t cg = 0, cx = 0;
    bool mine = act;
    if (DIRECT) mine = act && (ng[i] > gcap || ne[i] > xcap);
    const int64_t gw = DIRECT ? goff[i] : 0, ew = DIRECT ? eoff[i] : 0;
    uint32_t *gr = grow + (size_t)i * gcap, *xr = xrow + (size_t)i * xcap;
    const double4 la = llo[A], ha = lhi[A];
    for (int64_t q = poff[A]; q < poff[A + 1]; q++) {
        const int B = part[q];
        const int32_t b0 = loff[B], nbp = loff[B + 1] - b0;
        const int32_t u0 = lbk[B], nu = lbk[B + 1] - u0;
        __syncthreads();
        if (t < nbp) sp[t] = posH[b0 + t];
        if (t < nu) {
            sbl[t] = blo[u0 + t];
            sbh[t] = bhi[u0 + t];
            sbo[t] = bkoff[u0 + t] - b0;
        }
        if (t == 0) sbo[nu] = nbp;
        __syncthreads();
        // image shift of B per axis: when every separation of the two boxes
        // in that image lies within half a period (by a margin), the
        // minimum image of each pair is (x_i - x_j) + c
        const double4 lb = llo[B], hb = lhi[B];
        double c3[3];
        bool safe = true;
        {
            const double al[3] = {la.x, la.y, la.z}, ah[3] = {ha.x, ha.y, ha.z};
            const double bl[3] = {lb.x, lb.y, lb.z}, bh[3] = {hb.x, hb.y, hb.z};
            for (int x = 0; x < 3; x++) {
                bool found = false;
                for (int s = -1; s <= 1 && !found; s++) {
                    const double sh = s * L;   // image x_j + sh
                    const double dmin = al[x] - (bh[x] + sh), dmax = ah[x] - (bl[x] + sh);
                    if (dmin > -hL + margin && dmax < hL - margin) {
                        c3[x] = -sh;
                        found = true;
                    }
                }
                if (!found) {
                    c3[x] = 0.0;
                    safe = false;
                }
            }
        }
        for (int u = 0; u < nu; u++) {
            // bucket cull: distance from x_i to the bucket's box (nearest image)
            bool near = false;
            if (act) {
                const double4 bl = sbl[u], bh = sbh[u];
                const double R = fmax(pi.w, bl.w) + margin;
                double g2 = 0.0;
                const double pv[3] = {pi.x, pi.y, pi.z}, lo[3] = {bl.x, bl.y, bl.z},
                             hi[3] = {bh.x, bh.y, bh.z};
                for (int x = 0; x < 3; x++) {
                    double best = INFINITY;
                    for (int s = -1; s <= 1; s++) {
                        const double g = fmax(0.0, fmax((lo[x] + s * L) - pv[x], pv[x] - (hi[x] + s * L)));
                        best = fmin(best, g);
                    }
                    g2 += best * best;
                }
                near = g2 < R * R;
            }
            if (__ballot(near) == 0) continue;
            const int j0 = sbo[u], j1 = sbo[u + 1];
            for (int jj = j0; jj < j1; jj++) {
                const double4 pj = sp[jj];
                double dx, dy, dz;
                if (safe) {
                    dx = (pi.x - pj.x) + c3[0];
                    dy = (pi.y - pj.y) + c3[1];
                    dz = (pi.z - pj.z) + c3[2];
                } else {
                    dx = min_image(pi.x - pj.x, L, hL);
                    dy = min_image(pi.y - pj.y, L, hL);
                    dz = min_image(pi.z - pj.z, L, hL);
                }
                const double r2 = r2_exact(dx, dy, dz);
                const int32_t j = b0 + jj;
                const bool gat = r2 < Hi2 && (int64_t)j != i;
                const bool ext = !gat && r2 < pj.w * pj.w && (int64_t)j != i;
                if (mine && gat) {
                    if (DIRECT) gidx[gw + cg] = j;
                    else if (cg < gcap) gr[cg] = (uint32_t)j;
                    cg++;
                }
                if (mine && ext) {
                    if (DIRECT) eidx[ew + cx] = j;
                    else if (cx < xcap) xr[cx] = (uint32_t)j;
                    cx++;
                }
            }
        }
    }
    if (!DIRECT && act) {
        ng[i] = cg;
        ne[i] = cx;
    }
}

__global__ __launch_bounds__(kBlock) void k_count_i64(const int32_t *a, int64_t n, int64_t *o) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) o[i] = a[i];
    if (i == n) o[n] = 0;
}

// capped scratch rows -> CSR rows (rows past the cap are written by the DIRECT walk)
__global__ __launch_bounds__(kBlock) void k_leaf_copy(const uint32_t *__restrict__ rows, int cap,
                                                      const int32_t *__restrict__ cnt, int64_t n,
                                                      const int64_t *__restrict__ off, int32_t *idx) {
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int l = (int)(gid & 15);
    const int64_t i = gid >> 4;
    if (i >= n) return;
    const int c = cnt[i];
    if (c > cap) return;
    const uint32_t *r = rows + (size_t)i * cap;
    const int64_t o = off[i];
    for (int k = l; k < c; k += 16) idx[o + k] = (int32_t)r[k];
}

__global__ __launch_bounds__(kBlock) void k_rows_eb_ee(const int64_t *__restrict__ eoff, int64_t n,
                                                       int32_t *eb, int32_t *ee) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    eb[i] = (int32_t)eoff[i];
    ee[i] = (int32_t)eoff[i + 1];
}

__global__ __launch_bounds__(kBlock) void k_any_over(const int32_t *ng, const int32_t *ne, int64_t n,
                                                     int gcap, int xcap, int *flag) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n && (ng[i] > gcap || ne[i] > xcap)) atomicOr(flag, 1);
}

// Host layout of the trees: split nodes per level (begin-sorted), leaves
// and buckets in tree order, all from the box sizes.
struct Layout {
    std::vector<std::vector<int32_t>> nb, ns;   // per level: split nodes
    std::vector<int32_t> loff, boff, lbk, lbox, bleaf;
};

void lay_out(const int64_t *box_offsets, int nboxes, int nppl, int bucket, Layout &t) {
    t.loff.assign(1, 0);
    t.boff.assign(1, 0);
    t.lbk.assign(1, 0);
    t.lbox.clear();
    t.bleaf.assign(1, 0);
    t.nb.clear();
    t.ns.clear();
    struct Item { int64_t b, s; int lvl; bool in_leaf; };
    for (int bx = 0; bx < nboxes; bx++) {
        const int64_t b0 = box_offsets[bx], s0 = box_offsets[bx + 1] - b0;
        if (s0 > 0) {
            // depth-first in tree order; an explicit stack (right pushed first)
            std::vector<Item> st{{b0, s0, 0, false}};
            while (!st.empty()) {
                const Item it = st.back();
                st.pop_back();
                const bool leaf_here = !it.in_leaf && it.s <= nppl;
                if (it.s <= bucket) {
                    t.boff.push_back((int32_t)(it.b + it.s));
                    if (leaf_here) {
                        t.loff.push_back((int32_t)(it.b + it.s));
                        t.lbk.push_back((int32_t)(t.boff.size() - 1));
                        t.lbox.push_back(bx);
                    }
                } else {
                    if ((int)t.nb.size() <= it.lvl) {
                        t.nb.resize(it.lvl + 1);
                        t.ns.resize(it.lvl + 1);
                    }
                    t.nb[it.lvl].push_back((int32_t)it.b);
                    t.ns[it.lvl].push_back((int32_t)it.s);
                    const int64_t h = it.s / 2;
                    const bool il = it.in_leaf || leaf_here;
                    if (leaf_here) {
                        // a leaf closes after its last bucket: a marker item
                        st.push_back({it.b + it.s, -1, it.lvl, true});
                    }
                    st.push_back({it.b + h, it.s - h, it.lvl + 1, il});
                    st.push_back({it.b, h, it.lvl + 1, il});
                }
                // leaf markers (s = -1) close a leaf whose buckets are all out
                while (!st.empty() && st.back().s == -1) {
                    const Item mk = st.back();
                    st.pop_back();
                    t.loff.push_back((int32_t)mk.b);
                    t.lbk.push_back((int32_t)(t.boff.size() - 1));
                    t.lbox.push_back(bx);
                }
            }
        }
        t.bleaf.push_back((int32_t)(t.loff.size() - 1));
    }
    // split nodes of a level sorted by begin (depth-first order already is)
    for (size_t l = 0; l < t.nb.size(); l++) {
        std::vector<std::pair<int32_t, int32_t>> v;
        for (size_t k = 0; k < t.nb[l].size(); k++) v.push_back({t.nb[l][k], t.ns[l][k]});
        std::sort(v.begin(), v.end());
        for (size_t k = 0; k < v.size(); k++) {
            t.nb[l][k] = v[k].first;
            t.ns[l][k] = v[k].second;
        }
    }
}

}  // namespace
}  // namespace crk

using namespace crk;

extern "C" {

crk_status crk_build_leaves(crk_ctx *c, int32_t nboxes, const int64_t *box_offsets, int64_t n,
                            const double *x, const double *y, const double *z, const double *H,
                            const crk_params *p, int32_t nppl, int32_t bucket, int32_t *perm,
                            int64_t *n_pairs, int32_t *n_leaves, int32_t *leaf_offsets,
                            int64_t leaf_cap) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (n < 1 || !x || !y || !z || !H || !p || !perm || nboxes < 1 || !box_offsets)
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_build_leaves: n < 1 or NULL argument");
    if (n > INT32_MAX / 2) return set_err(c, CRK_ERR_INVALID_ARG, "n too large");
    if (nppl < 2 || nppl > kLeafMax || bucket < 4 || bucket > 64 || bucket > nppl)
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_build_leaves: need 4 <= bucket <= 64, bucket <= nppl <= 256");
    if (nppl / ((bucket + 1) / 2) + 1 > kBucketsMax)
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_build_leaves: nppl / bucket too large");
    if (!(p->L > 0.0)) return set_err(c, CRK_ERR_INVALID_ARG, "L must be positive");
    if (box_offsets[0] != 0 || box_offsets[nboxes] != n)
        return set_err(c, CRK_ERR_INVALID_ARG, "box offsets must run from 0 to n");
    for (int b = 0; b < nboxes; b++)
        if (box_offsets[b + 1] < box_offsets[b])
            return set_err(c, CRK_ERR_INVALID_ARG, "box offsets must not decrease");
    if (c->graph_mode) return set_err(c, CRK_ERR_STATE, "crk_build_leaves is not recorded in a graph");
    CRK_HIP(c, hipSetDevice(c->device));
    c->built = 0;
    c->have_V = 0;
    c->vol_ready = 0;
    c->leaf_mode = 0;
    c->nc = 0;   // no cell hierarchy: the calls that walk cells refuse
    c->n = n;
    c->L = p->L;
    c->nboxes = nboxes;
    const double L = p->L;
    const double margin = 1e-9 * L;

    // 1. validate (positions in [0, L), finite, 0 < H < L/2)
    CRK_TRY(ensure(c, c->misc, 256));
    {
        double hmax = 0.0, hmin = 0.0;
        CRK_TRY(validate_inputs(c, x, y, z, H, n, L, &hmax, &hmin));
        if (!(hmax < 0.5 * L)) return set_err(c, CRK_ERR_SUPPORT, "max H %g >= L/2", hmax);
    }

    // 2. keys, three sorted lists (within each box)
    Layout lay;
    lay_out(box_offsets, nboxes, nppl, bucket, lay);
    const int nl = (int)lay.loff.size() - 1, nbk = (int)lay.boff.size() - 1;
    CRK_TRY(ensure(c, c->rq, (size_t)3 * n * sizeof(uint32_t)));
    CRK_TRY(ensure(c, c->rsk, (size_t)3 * n * sizeof(uint32_t)));
    CRK_TRY(ensure(c, c->rla, (size_t)3 * n * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->rlb, (size_t)3 * n * sizeof(int32_t)));
    uint32_t *q = (uint32_t *)c->rq.p, *sk = (uint32_t *)c->rsk.p;
    int32_t *la = (int32_t *)c->rla.p, *lb = (int32_t *)c->rlb.p;
    {
        KTimer kt_(c, "rcb_sort");
        k_rcb_keys<<<lblocks(n), kBlock, 0, c->stream>>>(x, y, z, n, L, q, sk, la);
        CRK_HIP(c, hipGetLastError());
        int boxbits = 0;
        while ((1 << boxbits) < nboxes) boxbits++;
        if (boxbits > 0) {
            CRK_TRY(ensure(c, c->boff, (size_t)(nboxes + 1) * sizeof(int64_t)));
            CRK_HIP(c, hipMemcpyAsync(c->boff.p, box_offsets, (size_t)(nboxes + 1) * sizeof(int64_t),
                                      hipMemcpyHostToDevice, c->stream));
        }
        for (int a = 0; a < 3; a++) {
            CRK_TRY(radix_sort_pairs(c, sk + a * n, la + a * n, n, 32));
            if (boxbits > 0) {
                // then by box, stably: each box's particles in key order
                k_box_keys<<<lblocks(n), kBlock, 0, c->stream>>>((const int64_t *)c->boff.p, nboxes,
                                                                 la + a * n, n, sk + a * n);
                CRK_TRY(radix_sort_pairs(c, sk + a * n, la + a * n, n, boxbits));
            }
        }
    }

    // 3. levels: stable partition of the three lists by side
    CRK_TRY(ensure(c, c->rside, (size_t)n));
    CRK_TRY(ensure(c, c->rpnode, (size_t)n * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->rscan, (size_t)(n + 1) * sizeof(int64_t)));
    int8_t *side = (int8_t *)c->rside.p;
    int32_t *pnode = (int32_t *)c->rpnode.p;
    int64_t *sc = (int64_t *)c->rscan.p;
    // every level's split nodes in one table: begins, then sizes
    std::vector<int32_t> nodes;
    std::vector<size_t> lvoff{0};
    for (auto &v : lay.nb) lvoff.push_back(lvoff.back() + v.size());
    const size_t tot = lvoff.back();
    nodes.resize(2 * tot + 1);
    for (size_t lv = 0; lv < lay.nb.size(); lv++)
        for (size_t k = 0; k < lay.nb[lv].size(); k++) {
            nodes[lvoff[lv] + k] = lay.nb[lv][k];
            nodes[tot + lvoff[lv] + k] = lay.ns[lv][k];
        }
    size_t maxnodes = 1;
    for (auto &v : lay.nb) maxnodes = std::max(maxnodes, v.size());
    CRK_TRY(ensure(c, c->rnode, nodes.size() * sizeof(int32_t) + maxnodes));
    int32_t *dnodes = (int32_t *)c->rnode.p;
    int8_t *dax = (int8_t *)(dnodes + nodes.size());
    CRK_HIP(c, hipMemcpyAsync(dnodes, nodes.data(), nodes.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    CRK_HIP(c, hipStreamSynchronize(c->stream));   // the host table is not kept
    {
        KTimer kt_(c, "rcb_levels");
        for (size_t lv = 0; lv < lay.nb.size(); lv++) {
            const int nn = (int)lay.nb[lv].size();
            if (nn == 0) continue;
            const int32_t *dnb = dnodes + lvoff[lv], *dns = dnodes + tot + lvoff[lv];
            k_rcb_axis<<<lblocks(nn), kBlock, 0, c->stream>>>(dnb, dns, nn, la, q, n, dax);
            k_rcb_flag<<<lblocks(n), kBlock, 0, c->stream>>>(dnb, dns, nn, dax, la, n, side, pnode);
            for (int a = 0; a < 3; a++) {
                k_rcb_sides<<<lblocks(n + 1), kBlock, 0, c->stream>>>(la + a * n, pnode, side, n, sc);
                CRK_TRY(scan_exclusive_i64(c, sc, sc, n + 1));
                k_rcb_move<<<lblocks(n), kBlock, 0, c->stream>>>(la + a * n, pnode, side, sc, dnb, dns, n,
                                                                 lb + a * n);
            }
            CRK_HIP(c, hipGetLastError());
            std::swap(la, lb);
        }
    }
    // tree order: the x list
    CRK_TRY(ensure(c, c->perm, (size_t)n * sizeof(int32_t)));
    CRK_HIP(c, hipMemcpyAsync(c->perm.p, la, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
    CRK_HIP(c, hipMemcpyAsync(perm, la, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
    CRK_TRY(ensure(c, c->posH, (size_t)n * sizeof(double4)));
    double4 *posH = (double4 *)c->posH.p;
    k_leaf_gather<<<lblocks(n), kBlock, 0, c->stream>>>(x, y, z, H, la, n, posH);

    // 4. boxes, interaction lists
    CRK_TRY(ensure(c, c->rtab, (lay.loff.size() + lay.boff.size() + lay.lbk.size() + lay.lbox.size() +
                                lay.bleaf.size()) * sizeof(int32_t)));
    int32_t *dloff = (int32_t *)c->rtab.p, *dboff = dloff + lay.loff.size(),
            *dlbk = dboff + lay.boff.size(), *dlbox = dlbk + lay.lbk.size(), *dbleaf = dlbox + lay.lbox.size();
    CRK_HIP(c, hipMemcpyAsync(dloff, lay.loff.data(), lay.loff.size() * 4, hipMemcpyHostToDevice, c->stream));
    CRK_HIP(c, hipMemcpyAsync(dboff, lay.boff.data(), lay.boff.size() * 4, hipMemcpyHostToDevice, c->stream));
    CRK_HIP(c, hipMemcpyAsync(dlbk, lay.lbk.data(), lay.lbk.size() * 4, hipMemcpyHostToDevice, c->stream));
    CRK_HIP(c, hipMemcpyAsync(dlbox, lay.lbox.data(), lay.lbox.size() * 4, hipMemcpyHostToDevice, c->stream));
    CRK_HIP(c, hipMemcpyAsync(dbleaf, lay.bleaf.data(), lay.bleaf.size() * 4, hipMemcpyHostToDevice, c->stream));
    CRK_HIP(c, hipStreamSynchronize(c->stream));
    CRK_TRY(ensure(c, c->rbox, (size_t)(2 * nbk + 2 * nl) * sizeof(double4)));
    double4 *blo = (double4 *)c->rbox.p, *bhi = blo + nbk, *llo = bhi + nbk, *lhi = llo + nl;
    CRK_TRY(ensure(c, c->rpoff, (size_t)(nl + 1) * sizeof(int64_t)));
    int64_t *poff = (int64_t *)c->rpoff.p;
    int64_t npart = 0;
    {
        KTimer kt_(c, "rcb_lists");
        k_bucket_boxes<<<lblocks(nbk), kBlock, 0, c->stream>>>(posH, dboff, nbk, blo, bhi);
        k_leaf_boxes<<<lblocks(nl), kBlock, 0, c->stream>>>(blo, bhi, dlbk, nl, llo, lhi);
        k_leaf_pairs<false><<<lblocks(nl + 1), kBlock, 0, c->stream>>>(llo, lhi, dlbox, dbleaf, nl, L, margin, poff, nullptr, nullptr);
        k_count_i64<<<1, 1, 0, c->stream>>>(nullptr, 0, poff + nl);
        CRK_HIP(c, hipGetLastError());
        CRK_TRY(scan_exclusive_i64(c, poff, poff, nl + 1));
        int64_t *pin = (int64_t *)c->pinned.p + 48;
        CRK_HIP(c, hipMemcpyAsync(pin, poff + nl, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
        CRK_HIP(c, hipStreamSynchronize(c->stream));
        npart = pin[0];
        CRK_TRY(ensure(c, c->rpart, (size_t)std::max<int64_t>(npart, 1) * sizeof(int32_t)));
        k_leaf_pairs<true><<<lblocks(nl), kBlock, 0, c->stream>>>(llo, lhi, dlbox, dbleaf, nl, L, margin, nullptr, poff, (int32_t *)c->rpart.p);
        CRK_HIP(c, hipGetLastError());
    }
    const int32_t *part = (const int32_t *)c->rpart.p;

    // 5. rows: one tile walk into capped rows, scans, copies, a second walk
    //    for rows past a cap
    const int gcap = c->walk_cap, xcap = 64;
    CRK_TRY(ensure(c, c->scratch, (size_t)n * gcap * sizeof(uint32_t)));
    CRK_TRY(ensure(c, c->etmp, (size_t)n * xcap * sizeof(uint32_t)));
    CRK_TRY(ensure(c, c->ng, (size_t)n * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->ecnt, (size_t)n * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->goff, (size_t)(n + 1) * sizeof(int64_t)));
    CRK_TRY(ensure(c, c->eoff, (size_t)(n + 1) * sizeof(int64_t)));
    uint32_t *grow = (uint32_t *)c->scratch.p, *xrow = (uint32_t *)c->etmp.p;
    int32_t *ng = (int32_t *)c->ng.p, *ne = (int32_t *)c->ecnt.p;
    int64_t *goff = (int64_t *)c->goff.p, *eoff = (int64_t *)c->eoff.p;
    {
        KTimer kt_(c, "rcb_walk");
        k_leaf_walk<false><<<nl, kBlock, 0, c->stream>>>(posH, dloff, dlbk, dboff, blo, bhi, llo, lhi, poff,
                                                         part, L, margin, gcap, xcap, grow, xrow, ng, ne,
                                                         nullptr, nullptr, nullptr, nullptr);
        CRK_HIP(c, hipGetLastError());
    }
    CRK_TRY(scan_counts2(c, ng, ne, n, goff, eoff));
    int *over = (int *)c->misc.p + 8;
    CRK_TRY(zero_async(c, over, 1));
    k_any_over<<<lblocks(n), kBlock, 0, c->stream>>>(ng, ne, n, gcap, xcap, over);
    CRK_HIP(c, hipGetLastError());
    int64_t G = 0, E = 0;
    int ovr = 0;
    {
        int64_t *pin = (int64_t *)c->pinned.p + 52;
        CRK_HIP(c, hipMemcpyAsync(pin, goff + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
        CRK_HIP(c, hipMemcpyAsync(pin + 1, eoff + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
        CRK_HIP(c, hipMemcpyAsync(pin + 2, over, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        CRK_HIP(c, hipStreamSynchronize(c->stream));
        G = pin[0];
        E = pin[1];
        ovr = *(int *)(pin + 2);
    }
    if (E > INT32_MAX - 1) return set_err(c, CRK_ERR_INVALID_ARG, "more than 2^31 extra pairs");
    CRK_TRY(ensure(c, c->gidx, (size_t)std::max<int64_t>(G, 1) * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->eidx, (size_t)std::max<int64_t>(E, 1) * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->eb, (size_t)n * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->ee, (size_t)n * sizeof(int32_t)));
    {
        KTimer kt_(c, "rcb_copy");
        k_leaf_copy<<<lblocks(n * 16), kBlock, 0, c->stream>>>(grow, gcap, ng, n, goff, (int32_t *)c->gidx.p);
        k_leaf_copy<<<lblocks(n * 16), kBlock, 0, c->stream>>>(xrow, xcap, ne, n, eoff, (int32_t *)c->eidx.p);
        k_rows_eb_ee<<<lblocks(n), kBlock, 0, c->stream>>>(eoff, n, (int32_t *)c->eb.p, (int32_t *)c->ee.p);
        if (ovr)
            k_leaf_walk<true><<<nl, kBlock, 0, c->stream>>>(posH, dloff, dlbk, dboff, blo, bhi, llo, lhi, poff,
                                                            part, L, margin, gcap, xcap, grow, xrow, ng, ne,
                                                            goff, (int32_t *)c->gidx.p, eoff,
                                                            (int32_t *)c->eidx.p);
        CRK_HIP(c, hipGetLastError());
    }
    if (leaf_offsets) {
        if (leaf_cap < nl + 1) return set_err(c, CRK_ERR_INVALID_ARG, "leaf_offsets holds fewer than n_leaves + 1 values");
        CRK_HIP(c, hipMemcpyAsync(leaf_offsets, dloff, (size_t)(nl + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
    }
    CRK_HIP(c, hipStreamSynchronize(c->stream));
    c->ngather = G;
    c->nextra = E;
    c->npairs = G + E;
    c->built = 1;
    c->leaf_mode = 1;
    c->nleaves = nl;
    c->nleaf_pairs = npart;
    if (n_pairs) *n_pairs = c->npairs;
    if (n_leaves) *n_leaves = nl;
    return CRK_OK;
}

}  // extern "C"
