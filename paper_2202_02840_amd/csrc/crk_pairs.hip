// S2, S4, S5, S6, S7: the pair passes and the per-particle RK solve.
//
// Thread mapping. Every pair pass gives each particle i a group of G lanes
// (G in {1, 2, 4, 8, 16, 32, 64}, a divisor of the 64-wide wavefront). The
// lanes of a group stride over i's neighbour row, each keeping partial sums,
// and the group then reduces with cross-lane shuffles. G = 1 is one thread
// per particle; larger G trades a final reduction for balanced rows and
// coalesced loads of consecutive neighbours (rows follow the cell walk, and
// particles of a cell are contiguous after the sort). The best G per pass is
// chosen by the tuner; there is no MFMA here: each pass is a gather plus a
// reduction, not a dense contraction.
//
// Precision. T = double: every term and sum in FP64. T = float (CRK_MIXED):
// the separation d = x_i - x_j and its minimum image are formed in FP64 from
// the FP64 positions and only then rounded to FP32 (so close pairs keep their
// relative accuracy anywhere in the box); kernel values and pair terms are
// FP32 and every sum is a compensated (Kahan) FP32 sum whose high and low
// parts are combined in FP64 at the boundary.
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "crk_internal.h"

namespace crk {
namespace {

// ------------------------------------------------------------- arithmetic
template <typename T> struct Mth;
template <> struct Mth<float> {
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float exp(float x) { return __expf(x); }
};
template <> struct Mth<double> {
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double sqrt(double x) { return sqrt_dist(x); }
    static __device__ __forceinline__ double exp(double x) { return ::exp(x); }
};

// sum accumulator: plain FP64, or compensated FP32 (value = s - c)
template <typename T> struct Acc;
template <> struct Acc<double> {
    double s = 0.0;
    __device__ __forceinline__ void add(double x) { s += x; }
    __device__ __forceinline__ double value() const { return s; }
    __device__ __forceinline__ void merge_xor(int m, int w) { s += __shfl_xor(s, m, w); }
};
template <> struct Acc<float> {
    float s = 0.0f, c = 0.0f;
    __device__ __forceinline__ void add(float x) {
        float y = x - c;
        float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double value() const { return (double)s - (double)c; }
    // combine with the partner lane's (s, c): exact two-sum of the high parts
    __device__ __forceinline__ void merge_xor(int m, int w) {
        float s2 = __shfl_xor(s, m, w), c2 = __shfl_xor(c, m, w);
        float t = s + s2;
        float bp = t - s;
        float e = (s - (t - bp)) + (s2 - bp);
        s = t;
        c = c + c2 - e;
    }
};

template <typename T, int G, int K>
__device__ __forceinline__ void group_reduce(Acc<T> (&a)[K]) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1)
#pragma unroll
        for (int k = 0; k < K; k++) a[k].merge_xor(m, G);
}

// Fixed-point coordinate of x in [0, L): Q = floor(x 2^42 / L), kept as
// its high 32 bits q and its low 10 bits f (qinv = 2^42 / L; 2^42 fl(1 / L)
// is the same double)
struct Fixed {
    uint32_t q, f;
};
__device__ __forceinline__ Fixed fixed_q(double x, double qinv) {
    const double t = floor(x * qinv);
    const uint64_t Q = (uint64_t)(t < 4398046511103.0 ? t : 4398046511103.0);
    return Fixed{(uint32_t)(Q >> 10), (uint32_t)(Q & 1023u)};
}

// FP32 separation of two fixed-point coordinates: the 32-bit difference of
// the high parts wraps to the minimum image; the low parts add their
// difference at 2^-10 of the step (qs = L 2^-32), so d is within L 2^-42
// of the exact separation before the FP32 rounding
__device__ __forceinline__ float fixed_d(uint32_t qi, uint32_t fi, uint32_t qj, uint32_t fj, float qs) {
    return fmaf((float)((int32_t)fi - (int32_t)fj), qs * (1.0f / 1024.0f), (float)(int32_t)(qi - qj) * qs);
}

// the three low parts packed in one word (10 bits each)
__device__ __forceinline__ uint32_t pack_f(const Fixed &a, const Fixed &b, const Fixed &c) {
    return a.f | (b.f << 10) | (c.f << 20);
}
__device__ __forceinline__ uint32_t unpack_f(uint32_t w, int k) { return (w >> (10 * k)) & 1023u; }

// d = x_i - x_j of a listed pair: FP64 with the minimum image, or, for the
// FP32 passes, from the fixed-point coordinates, so that every FP32 pass
// (those reading positions and those reading packed records) sees the same
// d and the RK corrections cancel on the d they were built from
template <typename T>
__device__ __forceinline__ void separation(const double4 &pi, const double4 &pj, const Box &b,
                                           T &dx, T &dy, T &dz) {
    if constexpr (sizeof(T) == 4) {
        const double qinv = 4398046511104.0 * b.invL;
        const float qs = (float)(b.L * 2.3283064365386962890625e-10);
        const Fixed ix = fixed_q(pi.x, qinv), iy = fixed_q(pi.y, qinv), iz = fixed_q(pi.z, qinv);
        const Fixed jx = fixed_q(pj.x, qinv), jy = fixed_q(pj.y, qinv), jz = fixed_q(pj.z, qinv);
        dx = fixed_d(ix.q, ix.f, jx.q, jx.f, qs);
        dy = fixed_d(iy.q, iy.f, jy.q, jy.f, qs);
        dz = fixed_d(iz.q, iz.f, jz.q, jz.f, qs);
    } else {
        dx = (T)pair_image(pi.x - pj.x, b);
        dy = (T)pair_image(pi.y - pj.y, b);
        dz = (T)pair_image(pi.z - pj.z, b);
    }
}

// Wendland C4 with unit support, eq. (C4): with q = r/H and s = max(1 - q, 0),
//   W = kW H^-3 s^6 (1 + 6q + 35q^2/3),  grad_i W = kG H^-5 (1 + 5q) s^5 d.
template <typename T>
__device__ __forceinline__ void kernel_wg(T q, T cw, T cg, T &w, T &gf) {
    T s = q < (T)1 ? (T)1 - q : (T)0;
    T s2 = s * s;
    T s5 = s2 * s2 * s;
    w = cw * s5 * s * ((T)1 + q * ((T)6 + q * (T)(35.0 / 3.0)));
    gf = cg * ((T)1 + (T)5 * q) * s5;
}

// Wendland C4 radial factors with unit support, eq. (C4): s = max(1 - q, 0),
// pw = s^6 (1 + 6q + 35q^2/3), pg = (1 + 5q) s^5
template <typename T>
__device__ __forceinline__ void kfac(T q, T &pw, T &pg) {
    const T s = q < (T)1 ? (T)1 - q : (T)0;
    const T s2 = s * s;
    const T s5 = s2 * s2 * s;
    pw = s5 * s * ((T)1 + q * ((T)6 + q * (T)(35.0 / 3.0)));
    pg = ((T)1 + (T)5 * q) * s5;
}

__device__ __forceinline__ int64_t group_index(int G, int &lane) {
    int64_t gid = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    lane = (int)(gid % G);
    return gid / G;
}

// ------------------------------------------------------------- S2 volume
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_volume(const double4 *__restrict__ posH,
                                                   const int64_t *__restrict__ goff,
                                                   const int32_t *__restrict__ gidx, int64_t n, Box box,
                                                   double *nsum_out, double *V_out, T *recV,
                                                   double4 *posV) {
    int l;
    int64_t i = group_index(G, l);
    Acc<T> acc[1];
    if (i < n) {
        double4 pi = posH[i];
        T invH = (T)(1.0 / pi.w);
        T cw = (T)kW * invH * invH * invH;
        if (l == 0) acc[0].add(cw);            // self pair: W(0, H_i)
        int64_t b = goff[i];
        int cnt = (int)(goff[i + 1] - b);
        // the next neighbour index is fetched one step ahead
        int32_t jn = l < cnt ? gidx[b + l] : 0;
        for (int k = l; k < cnt; k += G) {
            const int32_t j = jn;
            if (k + G < cnt) jn = gidx[b + k + G];
            double4 pj = posH[j];
            T dx, dy, dz;
            separation(pi, pj, box, dx, dy, dz);
            T q = Mth<T>::sqrt(dx * dx + dy * dy + dz * dz) * invH;
            acc[0].add(kernel_w(q, cw));
        }
    }
    group_reduce<T, G, 1>(acc);
    if (i < n && l == 0) {
        double s = acc[0].value();
        if (nsum_out) nsum_out[i] = s;
        V_out[i] = 1.0 / s;
        recV[i] = (T)(1.0 / s);
        // the moment pass reads a partner's position and volume in one load
        posV[i] = make_double4(posH[i].x, posH[i].y, posH[i].z, 1.0 / s);
    }
}

// ------------------------------------------------------------- S4 moments
// The 40 outputs per particle (m0, m1[3], m2[6], gm0[3], gm1[9], gm2[18])
// come from 29 sums. With t = V_j W and u = V_j gf (grad_i W = gf d, the
// kernel being radial):
//   m0 = sum t, m1_a = sum t d_a, m2_ab = sum t d_a d_b, gm0_g = sum u d_g,
//   gm1_ag = Q2_ag + delta_ag m0,  gm2_abg = Q3_abg + delta_ag m1_b + delta_bg m1_a,
// with Q2_ag = sum u d_a d_g and Q3_abg = sum u d_a d_b d_g, both symmetric
// in their indices (6 and 10 distinct sums), since d/dx_i (d_a W) = delta W +
// d_a grad W. Same sums as the term-by-term form, grouped differently.
// index of the symmetric pair (a, b) among (0,0),(0,1),(0,2),(1,1),(1,2),(2,2),
// and of the sorted triple (a, b, c) among the ten triples in lexicographic order
__device__ constexpr int kSym2[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
__device__ constexpr int kSym3[3][3][3] = {{{0, 1, 2}, {1, 3, 4}, {2, 4, 5}}, {{1, 3, 4}, {3, 6, 7}, {4, 7, 8}}, {{2, 4, 5}, {4, 7, 8}, {5, 8, 9}}};

template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_moments(const double4 *__restrict__ posH,
                                                    const int64_t *__restrict__ goff,
                                                    const int32_t *__restrict__ gidx,
                                                    const double4 *__restrict__ posV, int64_t n, Box box,
                                                    double *m0, double *m1, double *m2, double *gm0,
                                                    double *gm1, double *gm2) {
    // sums: 0 m0 | 1-3 m1 | 4-9 m2 | 10-12 gm0 | 13-18 Q2 | 19-28 Q3
    int l;
    int64_t i = group_index(G, l);
    Acc<T> a[29];
    if (i < n) {
        double4 pi = posH[i];
        T invH = (T)(1.0 / pi.w);
        T invH2 = invH * invH;
        T cw = (T)kW * invH2 * invH;
        T cg = (T)kG * invH2 * invH2 * invH;
        if (l == 0) a[0].add((T)posV[i].w * cw);   // self pair: d = 0, so m0 only
        int64_t b = goff[i];
        int cnt = (int)(goff[i + 1] - b);
        int32_t jn = l < cnt ? gidx[b + l] : 0;
        for (int k = l; k < cnt; k += G) {
            const int32_t j = jn;
            if (k + G < cnt) jn = gidx[b + k + G];
            const double4 pj = posV[j];   // x, y, z and V
            T Vj = (T)pj.w;
            T d[3];
            separation(pi, pj, box, d[0], d[1], d[2]);
            T q = Mth<T>::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) * invH;
            T w, gf;
            kernel_wg(q, cw, cg, w, gf);
            const T t = Vj * w, u = Vj * gf;
            a[0].add(t);
            T dd[6];
#pragma unroll
            for (int x = 0; x < 3; x++) {
                a[1 + x].add(t * d[x]);
                a[10 + x].add(u * d[x]);
#pragma unroll
                for (int y = x; y < 3; y++) dd[kSym2[x][y]] = d[x] * d[y];
            }
#pragma unroll
            for (int e = 0; e < 6; e++) {
                a[4 + e].add(t * dd[e]);
                a[13 + e].add(u * dd[e]);
            }
#pragma unroll
            for (int x = 0; x < 3; x++)
#pragma unroll
                for (int y = x; y < 3; y++)
#pragma unroll
                    for (int z = y; z < 3; z++) a[19 + kSym3[x][y][z]].add(u * dd[kSym2[x][y]] * d[z]);
        }
    }
    group_reduce<T, G, 29>(a);
    if (i < n && l == 0) {
        const double p0 = a[0].value();
        double p1[3];
#pragma unroll
        for (int x = 0; x < 3; x++) p1[x] = a[1 + x].value();
        m0[i] = p0;
#pragma unroll
        for (int x = 0; x < 3; x++) {
            m1[x * n + i] = p1[x];
            gm0[x * n + i] = a[10 + x].value();
        }
#pragma unroll
        for (int e = 0; e < 6; e++) m2[e * n + i] = a[4 + e].value();
#pragma unroll
        for (int x = 0; x < 3; x++)
#pragma unroll
            for (int c = 0; c < 3; c++)
                gm1[(x * 3 + c) * n + i] = a[13 + kSym2[x][c]].value() + (x == c ? p0 : 0.0);
        int s = 0;
#pragma unroll
        for (int x = 0; x < 3; x++)
#pragma unroll
            for (int y = x; y < 3; y++, s++)
#pragma unroll
                for (int c = 0; c < 3; c++)
                    gm2[(s * 3 + c) * n + i] = a[19 + kSym3[x][y][c]].value() + (x == c ? p1[y] : 0.0) +
                                               (y == c ? p1[x] : 0.0);
    }
}

// ------------------------------------------------------------- S5 corrections
// Per particle, FP64. The constraints sum V W^R = 1 and sum V d W^R = 0 of
// eq. (RK) give B = -m2^{-1} m1 and A = 1/(m0 + B.m1); their gradients follow
// by differentiating the same constraints. m2 is inverted by its adjugate;
// det(m2) <= 1e-12 (tr m2 / 3)^3 selects normalised SPH (A = 1/m0, B = 0).
__global__ __launch_bounds__(kBlock) void k_corrections(int64_t n, const double *m0, const double *m1,
                                                        const double *m2, const double *gm0,
                                                        const double *gm1, const double *gm2,
                                                        double *A, double *B, double *gA, double *gB,
                                                        unsigned long long *nsing) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int sym[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    double M[3][3];
#pragma unroll
    for (int x = 0; x < 3; x++)
#pragma unroll
        for (int y = 0; y < 3; y++) M[x][y] = m2[sym[x][y] * n + i];
    double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                 M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                 M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
    double tr = (M[0][0] + M[1][1] + M[2][2]) / 3.0;
    double mm0 = m0[i];
    double mm1[3] = {m1[i], m1[n + i], m1[2 * n + i]};
    if (!(det > 1e-12 * tr * tr * tr)) {
        A[i] = 1.0 / mm0;
#pragma unroll
        for (int x = 0; x < 3; x++) {
            B[x * n + i] = 0.0;
            gA[x * n + i] = -gm0[x * n + i] / (mm0 * mm0);
        }
#pragma unroll
        for (int s = 0; s < 9; s++) gB[s * n + i] = 0.0;
        atomicAdd(nsing, 1ull);
        return;
    }
    double id = 1.0 / det;
    double Mi[3][3];
    Mi[0][0] = (M[1][1] * M[2][2] - M[1][2] * M[2][1]) * id;
    Mi[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) * id;
    Mi[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) * id;
    Mi[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) * id;
    Mi[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) * id;
    Mi[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) * id;
    Mi[1][0] = Mi[0][1];
    Mi[2][0] = Mi[0][2];
    Mi[2][1] = Mi[1][2];
    double Bv[3];
#pragma unroll
    for (int x = 0; x < 3; x++) Bv[x] = -(Mi[x][0] * mm1[0] + Mi[x][1] * mm1[1] + Mi[x][2] * mm1[2]);
    double Av = 1.0 / (mm0 + Bv[0] * mm1[0] + Bv[1] * mm1[1] + Bv[2] * mm1[2]);
    A[i] = Av;
#pragma unroll
    for (int x = 0; x < 3; x++) B[x * n + i] = Bv[x];
#pragma unroll
    for (int g = 0; g < 3; g++) {
        double r[3];
#pragma unroll
        for (int x = 0; x < 3; x++) {
            double s = gm1[(x * 3 + g) * n + i];
#pragma unroll
            for (int y = 0; y < 3; y++) s += gm2[(sym[x][y] * 3 + g) * n + i] * Bv[y];
            r[x] = s;
        }
        double dB[3];
#pragma unroll
        for (int x = 0; x < 3; x++) dB[x] = -(Mi[x][0] * r[0] + Mi[x][1] * r[1] + Mi[x][2] * r[2]);
        double s = gm0[g * n + i];
#pragma unroll
        for (int x = 0; x < 3; x++) s += dB[x] * mm1[x] + Bv[x] * gm1[(x * 3 + g) * n + i];
        gA[g * n + i] = -Av * Av * s;
#pragma unroll
        for (int x = 0; x < 3; x++) gB[(x * 3 + g) * n + i] = dB[x];
    }
}

// ------------------------------------------------------------- S6 grad v
// RK gradient template of eq. (gRK) for the ordered pair (i, j) with i's
// coefficients, c = 1 + B.d, (gradB^T d)_g = sum_a d_a dB_a/dx_g:
//   grad W^R_g = w (dA_g c + A ((gradB^T d)_g + B_g)) + A c gf d_g.
// The FP64 pass evaluates it term by term as written. It is linear in the
// kernel's radial factors w = kW H^-3 pw(q) and gf = kG H^-5 pg(q), so the
// FP32 pass groups it per particle:
//   grad W^R = pw (U + M d) + Ag c pg d,
//   U_g = kW H^-3 (dA_g + A B_g), M_ga = kW H^-3 (dA_g B_a + A dB_a/dx_g),
//   Ag = A kG H^-5,
// the same sum with fewer operations per pair (its rounding differs, which
// the FP32 pass's error budget absorbs; the FP64 pass keeps the order of
// the written form, whose rounding the ill-conditioned sets show).
template <typename T>
struct Coef {
    T A, B[3], gA[3], gB[9];
};

template <typename T>
__device__ __forceinline__ void rk_grad(const Coef<T> &k, const T d[3], T w, T gf, T out[3]) {
    T c = (T)1 + k.B[0] * d[0] + k.B[1] * d[1] + k.B[2] * d[2];
    T acg = k.A * c * gf;
#pragma unroll
    for (int g = 0; g < 3; g++) {
        T btd = d[0] * k.gB[0 * 3 + g] + d[1] * k.gB[1 * 3 + g] + d[2] * k.gB[2 * 3 + g];
        out[g] = w * (k.gA[g] * c + k.A * (btd + k.B[g])) + acg * d[g];
    }
}

// i = list[g] when a list is given (the FP64 rows of the adaptive mode),
// else i = g; rows with skip[i] set are left to another launch.
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_gradv(const double4 *__restrict__ posH,
                                                  const int64_t *__restrict__ goff,
                                                  const int32_t *__restrict__ gidx,
                                                  const typename std::conditional<sizeof(T) == 4, float4, double4>::type *__restrict__ rec6,
                                                  const double *__restrict__ A, const double *__restrict__ B,
                                                  const double *__restrict__ gA,
                                                  const double *__restrict__ gB, int64_t n, Box box,
                                                  const int32_t *__restrict__ list, int64_t nlist,
                                                  const int64_t *__restrict__ nlist_dev,
                                                  const int32_t *__restrict__ skip, double *gradv) {
    int l;
    int64_t g = group_index(G, l);
    if (nlist_dev) nlist = *nlist_dev;
    const int64_t gstride = (int64_t)gridDim.x * (kBlock / G);
    // a list launch may cover its rows with fewer groups than rows
    for (;; g += gstride) {
    int64_t i = -1;
    if (list) {
        if (g < nlist) i = list[g];
    } else if (g < n && !(skip && skip[g])) {
        i = g;
    }
    // FP64 sums of the pair terms (in the FP32 pass a conversion and an add
    // per term, cheaper than a compensated FP32 sum on this VALU, with FP64
    // vector adds at full rate)
    Acc<double> a[9];
    if (i >= 0) {
        const double4 pi = posH[i];
        // FP32 records are two 4-vectors (v, V) and the fixed-point position
        constexpr int S6 = sizeof(T) == 4 ? 2 : 1;
        auto ri = rec6[S6 * i];
        const T vi[3] = {ri.x, ri.y, ri.z};
        const int64_t b = goff[i];
        const int cnt = (int)(goff[i + 1] - b);
        if constexpr (sizeof(T) == 8) {
            // eq. (gRK) term by term
            const T invH = (T)(1.0 / pi.w);
            const T invH2 = invH * invH;
            const T cw = (T)kW * invH2 * invH;
            const T cg = (T)kG * invH2 * invH2 * invH;
            Coef<T> k;
            k.A = (T)A[i];
#pragma unroll
            for (int x = 0; x < 3; x++) {
                k.B[x] = (T)B[x * n + i];
                k.gA[x] = (T)gA[x * n + i];
            }
#pragma unroll
            for (int s = 0; s < 9; s++) k.gB[s] = (T)gB[s * n + i];
            int32_t jn = l < cnt ? gidx[b + l] : 0;
            for (int kk = l; kk < cnt; kk += G) {
                const int32_t j = jn;
                if (kk + G < cnt) jn = gidx[b + kk + G];
                const double4 pj = posH[j];
                auto rj = rec6[j];
                T d[3];
                separation(pi, pj, box, d[0], d[1], d[2]);
                const T q = Mth<T>::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) * invH;
                T w, gf;
                kernel_wg(q, cw, cg, w, gf);
                T G3[3];
                rk_grad(k, d, w, gf, G3);
                const T dv[3] = {(vi[0] - (T)rj.x) * rj.w, (vi[1] - (T)rj.y) * rj.w, (vi[2] - (T)rj.z) * rj.w};
#pragma unroll
                for (int x = 0; x < 3; x++)
#pragma unroll
                    for (int y = 0; y < 3; y++) a[x * 3 + y].add(-dv[x] * G3[y]);
            }
        } else {
            // the regrouped template: grad W^R_ij = pw (U + M d) + Ag c pg d
            const double ihd = 1.0 / pi.w, cwd = kW * ihd * ihd * ihd;
            const double Ad = A[i];
            double Bd[3], gAd[3];
#pragma unroll
            for (int x = 0; x < 3; x++) {
                Bd[x] = B[x * n + i];
                gAd[x] = gA[x * n + i];
            }
            T U[3], M[9], Bt[3];
#pragma unroll
            for (int g = 0; g < 3; g++) {
                Bt[g] = (T)Bd[g];
                U[g] = (T)(cwd * (gAd[g] + Ad * Bd[g]));
#pragma unroll
                for (int c = 0; c < 3; c++)
                    M[g * 3 + c] = (T)(cwd * (gAd[g] * Bd[c] + Ad * gB[(c * 3 + g) * n + i]));
            }
            const T Ag = (T)(Ad * kG * ihd * ihd * ihd * ihd * ihd);
            const T ih = (T)ihd;
            const auto qv = rec6[S6 * i + 1];
            const uint32_t qi[3] = {__float_as_uint(qv.x), __float_as_uint(qv.y), __float_as_uint(qv.z)};
            const uint32_t fi = __float_as_uint(qv.w);
            const T qs = (T)(box.L * 2.3283064365386962890625e-10);
            int32_t jn = l < cnt ? gidx[b + l] : 0;
            for (int kk = l; kk < cnt; kk += G) {
                const int32_t j = jn;
                if (kk + G < cnt) jn = gidx[b + kk + G];
                auto rj = rec6[S6 * j];
                const auto qj = rec6[S6 * j + 1];
                T d[3];
                // d from the fixed-point positions (as in the derivative pass)
                d[0] = fixed_d(qi[0], unpack_f(fi, 0), __float_as_uint(qj.x), unpack_f(__float_as_uint(qj.w), 0), qs);
                d[1] = fixed_d(qi[1], unpack_f(fi, 1), __float_as_uint(qj.y), unpack_f(__float_as_uint(qj.w), 1), qs);
                d[2] = fixed_d(qi[2], unpack_f(fi, 2), __float_as_uint(qj.z), unpack_f(__float_as_uint(qj.w), 2), qs);
                const T r = Mth<T>::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                T pw, pg;
                kfac(r * ih, pw, pg);
                const T kc = Ag * ((T)1 + (Bt[0] * d[0] + Bt[1] * d[1] + Bt[2] * d[2])) * pg;
                T G3[3];
#pragma unroll
                for (int g = 0; g < 3; g++)
                    G3[g] = pw * (U[g] + (M[g * 3 + 0] * d[0] + M[g * 3 + 1] * d[1] + M[g * 3 + 2] * d[2])) +
                            kc * d[g];
                // -V_j (v_i - v_j) (x) grad W^R_ij
                const T w[3] = {((T)rj.x - vi[0]) * (T)rj.w, ((T)rj.y - vi[1]) * (T)rj.w,
                                ((T)rj.z - vi[2]) * (T)rj.w};
#pragma unroll
                for (int x = 0; x < 3; x++)
#pragma unroll
                    for (int y = 0; y < 3; y++) a[x * 3 + y].add((double)(w[x] * G3[y]));
            }
        }
    }
    group_reduce<double, G, 9>(a);
    if (i >= 0 && l == 0)
#pragma unroll
        for (int s = 0; s < 9; s++) gradv[s * n + i] = a[s].value();
    if (!list || g + gstride >= nlist) break;
    }
}

// ------------------------------------------------------------- S7 derivatives
// The RK gradient template of eq. (gRK) for the ordered pair (i, j), with
// i's coefficients and c = 1 + B.d,
//   grad W^R_ij = w (gradA c + A ((gradB)^T d + B)) + A c gf d,
// is regrouped per particle so that a pair needs no per-particle prefactor.
// With the kernel's radial factors w = kW H^-3 pw(q) and gf = kG H^-5 pg(q),
//   grad W^R_ij = pw (U + M d) + Ag c pg d,
//   U_g = kW H^-3 (dA/dx_g + A B_g),  M_ga = kW H^-3 (dA/dx_g B_a + A dB_a/dx_g),
//   Ag = A kG H^-5.
// The limiter of eqs. (phi)-(phiad) and the projected velocity of eq.
// (hatvi) need the velocity gradient only through s = d^T (grad v) d (the
// projection (v_i - v_j - phi/2 (grad v_i + grad v_j) d + adot d).d is
// (v_i - v_j).d - phi/2 (s_i + s_j) + adot r^2), so only the symmetric part
// of grad v is kept. Same quantities as the term-by-term form, grouped
// differently.
//
// Packed per-particle record of the derivative and compatible passes, eight
// 4-vectors of data and one of padding (a 144-byte stride for FP32: with
// a power-of-two stride the partners' records of one step fall on few
// memory channels, which measured 1.5x slower):
//   0 {vx, vy, vz, Vs}      Vs = V a / sqrt(2), so Vs_i Vs_j = (a^2/2) V_i V_j
//   1 {P, rho, Clcs, ih}    Clcs = C_l c_s; ih = 1/H, negated for an FP64 row
//   2 {hA, he, Ag, B0}      hA = hh / a, he = hh^2 eps^2 (hh = H / n_h, eq. mu)
//   3 {B1, B2, U0, U1}
//   4 {U2, M00, M01, M02}   M row g (derivative direction), column a
//   5 {M10, M11, M12, M20}
//   6 {M21, M22, S0, S1}    S = (g00, g11, g22, g01 + g10, g02 + g20, g12 + g21)
//   7 {S2, S3, S4, S5}      of grad v (g_ab = dv_a/dx_b)
constexpr int kRec = 9;   // 4-vectors per record (the last one padding)

struct DerivPrm {
    double gamma, Cl, Cq, eps2, inv_nh, inv_a, adot, eta_c, inv_eta_f, vs_scale, inv_a5;
    // fixed-point positions of the FP32 records: Q = floor(x 2^42 / L)
    // (qinv = 2^42 / L; qs = L 2^-32, the step of Q's high 32 bits)
    double qinv, qs;
};

template <typename T>
struct Rec {
    T v[3], Vs, P, rho, Clcs, ih, hA, he, Ag, B[3], U[3], M[9], S[6];
    // FP32 records: the position in fixed point (the record's ninth
    // 4-vector): high parts q (q_i - q_j taken mod 2^32 is the minimum
    // image) and the packed low parts qf
    uint32_t q[3], qf;
};

// the record of one particle from FP64 state (P, rho, c_s given)
__device__ __forceinline__ void make_rec(double H, double vx, double vy, double vz, double Vi, double P,
                                         double rho, double cs, double A, const double B3[3],
                                         const double gA3[3], const double gB9[9], const double gv9[9],
                                         const DerivPrm &p, bool fp64_row, Rec<double> &r) {
    const double ih = 1.0 / H;
    const double ih2 = ih * ih;
    const double cw = kW * ih2 * ih;
    const double hh = H * p.inv_nh;
    r.v[0] = vx;
    r.v[1] = vy;
    r.v[2] = vz;
    r.Vs = Vi * p.vs_scale;
    r.P = P;
    r.rho = rho;
    r.Clcs = p.Cl * cs;
    r.ih = fp64_row ? -ih : ih;
    r.hA = hh * p.inv_a;
    r.he = hh * hh * p.eps2;
    r.Ag = A * kG * ih2 * ih2 * ih;
#pragma unroll
    for (int g = 0; g < 3; g++) {
        r.B[g] = B3[g];
        r.U[g] = cw * (gA3[g] + A * B3[g]);
#pragma unroll
        for (int a = 0; a < 3; a++) r.M[g * 3 + a] = cw * (gA3[g] * B3[a] + A * gB9[a * 3 + g]);
    }
    r.S[0] = gv9[0];
    r.S[1] = gv9[4];
    r.S[2] = gv9[8];
    r.S[3] = gv9[1] + gv9[3];
    r.S[4] = gv9[2] + gv9[6];
    r.S[5] = gv9[5] + gv9[7];
}

template <typename V4, typename T>
__device__ __forceinline__ void store_rec(V4 *o, const Rec<double> &r) {
    o[0] = V4{(T)r.v[0], (T)r.v[1], (T)r.v[2], (T)r.Vs};
    o[1] = V4{(T)r.P, (T)r.rho, (T)r.Clcs, (T)r.ih};
    o[2] = V4{(T)r.hA, (T)r.he, (T)r.Ag, (T)r.B[0]};
    o[3] = V4{(T)r.B[1], (T)r.B[2], (T)r.U[0], (T)r.U[1]};
    o[4] = V4{(T)r.U[2], (T)r.M[0], (T)r.M[1], (T)r.M[2]};
    o[5] = V4{(T)r.M[3], (T)r.M[4], (T)r.M[5], (T)r.M[6]};
    o[6] = V4{(T)r.M[7], (T)r.M[8], (T)r.S[0], (T)r.S[1]};
    o[7] = V4{(T)r.S[2], (T)r.S[3], (T)r.S[4], (T)r.S[5]};
    o[8] = V4{(T)0, (T)0, (T)0, (T)0};
}

template <typename V4, typename T>
__device__ __forceinline__ void load_rec(const V4 *__restrict__ rec, int64_t j, Rec<T> &s) {
    const V4 *o = rec + j * kRec;
    const V4 r0 = o[0], r1 = o[1], r2 = o[2], r3 = o[3], r4 = o[4], r5 = o[5], r6 = o[6], r7 = o[7];
    if constexpr (sizeof(T) == 4) {
        const V4 r8 = o[8];
        s.q[0] = __float_as_uint(r8.x);
        s.q[1] = __float_as_uint(r8.y);
        s.q[2] = __float_as_uint(r8.z);
        s.qf = __float_as_uint(r8.w);
    }
    s.v[0] = r0.x; s.v[1] = r0.y; s.v[2] = r0.z; s.Vs = r0.w;
    s.P = r1.x; s.rho = r1.y; s.Clcs = r1.z; s.ih = r1.w;
    s.hA = r2.x; s.he = r2.y; s.Ag = r2.z; s.B[0] = r2.w;
    s.B[1] = r3.x; s.B[2] = r3.y; s.U[0] = r3.z; s.U[1] = r3.w;
    s.U[2] = r4.x; s.M[0] = r4.y; s.M[1] = r4.z; s.M[2] = r4.w;
    s.M[3] = r5.x; s.M[4] = r5.y; s.M[5] = r5.z; s.M[6] = r5.w;
    s.M[7] = r6.x; s.M[8] = r6.y; s.S[0] = r6.z; s.S[1] = r6.w;
    s.S[2] = r7.x; s.S[3] = r7.y; s.S[4] = r7.z; s.S[5] = r7.w;
}

// P = (gamma - 1) rho u (eq. EOS) with rho = m / V unless given, and
// c_s = sqrt(gamma P / rho); flags a non-finite or non-positive state
__device__ __forceinline__ void gas_state(int64_t i, const double *v, const double *m, const double *u,
                                          const double *rho, const double *V, int64_t n, double gamma,
                                          double &r, double &P, double &cs, int *bad) {
    r = rho ? rho[i] : m[i] / V[i];
    P = (gamma - 1.0) * r * u[i];
    cs = sqrt(gamma * P / r);
    if (!isfinite(r) || !isfinite(P) || !isfinite(cs) || !isfinite(m[i]) || !isfinite(v[i]) ||
        !isfinite(v[n + i]) || !isfinite(v[2 * n + i]) || !(r > 0.0))
        atomicOr(bad, 1);
}

// Appends i to list when `take` (one atomic per wavefront; the list order
// is that of the arrivals, and every user treats the rows independently).
__device__ __forceinline__ void append_row(bool take, int64_t i, int32_t *list,
                                           unsigned long long *count) {
    const uint64_t m = __ballot(take);
    if (m == 0) return;
    const int lane = threadIdx.x & 63;
    const int lead = __ffsll((unsigned long long)m) - 1;
    unsigned long long base = 0;
    if (lane == lead) base = atomicAdd(count, (unsigned long long)__popcll(m));
    base = __shfl(base, lead, 64);
    if (take) list[base + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)i;
}

// Conditioning of particle i's RK template (see k_flag): 1 when it exceeds
// kappa_max, so that the row runs in FP64
__device__ __forceinline__ int kappa_flag(int64_t i, int64_t n, const double4 *__restrict__ posH,
                                          const double *A, const double *B, const double *gA,
                                          const double *gB, double kappa_max) {
    double H = posH[i].w;
    double b2 = 0.0, a2 = 0.0, g2 = 0.0;
#pragma unroll
    for (int x = 0; x < 3; x++) {
        b2 += B[x * n + i] * B[x * n + i];
        a2 += gA[x * n + i] * gA[x * n + i];
    }
#pragma unroll
    for (int q = 0; q < 9; q++) g2 += gB[q * n + i] * gB[q * n + i];
    double kap = 1.0 + sqrt(b2) * H + sqrt(g2) * H * H + sqrt(a2) * H / fabs(A[i]);
    return !(kap <= kappa_max);
}

template <typename V4, typename T>
__device__ __forceinline__ void pack8_one(int64_t i, int64_t n, const double4 *__restrict__ posH,
                                          const double *v, const double *m, const double *u,
                                          const double *rho, const double *V, const double *A,
                                          const double *B, const double *gA, const double *gB,
                                          const double *gv, const DerivPrm &p, bool fp64row,
                                          V4 *o, double4 *aux, int *bad) {
    double r, P, cs;
    gas_state(i, v, m, u, rho, V, n, p.gamma, r, P, cs, bad);
    double B3[3], gA3[3], gB9[9], gv9[9];
#pragma unroll
    for (int x = 0; x < 3; x++) {
        B3[x] = B[x * n + i];
        gA3[x] = gA[x * n + i];
    }
#pragma unroll
    for (int q = 0; q < 9; q++) {
        gB9[q] = gB[q * n + i];
        gv9[q] = gv[q * n + i];
    }
    Rec<double> rc;
    make_rec(posH[i].w, v[i], v[n + i], v[2 * n + i], V[i], P, r, cs, A[i], B3, gA3, gB9, gv9, p,
             fp64row, rc);
    store_rec<V4, T>(o, rc);
    if constexpr (sizeof(T) == 4) {
        const double4 x = posH[i];
        const Fixed fx = fixed_q(x.x, p.qinv), fy = fixed_q(x.y, p.qinv), fz = fixed_q(x.z, p.qinv);
        o[8] = V4{__uint_as_float(fx.q), __uint_as_float(fy.q), __uint_as_float(fz.q),
                  __uint_as_float(pack_f(fx, fy, fz))};
    }
    if (aux) aux[i] = make_double4(r, P, cs, 0.0);
}

template <typename V4, typename T>
__global__ __launch_bounds__(kBlock) void k_pack8(int64_t n, const double4 *__restrict__ posH,
                                                  const double *v, const double *m, const double *u,
                                                  const double *rho, const double *V, const double *A,
                                                  const double *B, const double *gA, const double *gB,
                                                  const double *gv, DerivPrm p, const int32_t *flag,
                                                  V4 *rec, double4 *aux, int *bad, double kappa_max,
                                                  int32_t *flag_out, int32_t *flist,
                                                  unsigned long long *nflag) {
    // FP32 records are assembled in LDS and leave as one contiguous run per
    // block (consecutive lanes, consecutive 16 bytes) instead of nine
    // 16-byte stores 144 bytes apart per lane
    constexpr bool STAGE = sizeof(T) == 4;
    __shared__ V4 s_rec[STAGE ? kBlock * kRec : 1];
    const int64_t b0 = (int64_t)blockIdx.x * kBlock;
    const int64_t i = b0 + threadIdx.x;
    // with flag_out the FP64 rows are decided here (as k_flag does), from
    // the corrections the record is made of
    int f = 0;
    if (i < n) {
        if (flag_out) {
            f = kappa_flag(i, n, posH, A, B, gA, gB, kappa_max);
            flag_out[i] = f;
        } else {
            f = flag && flag[i] != 0;
        }
        pack8_one<V4, T>(i, n, posH, v, m, u, rho, V, A, B, gA, gB, gv, p, f != 0,
                         STAGE ? s_rec + threadIdx.x * kRec : rec + i * kRec, aux, bad);
    }
    if (flag_out) append_row(f != 0, i, flist, nflag);
    if constexpr (STAGE) {
        __syncthreads();
        const int cnt = (int)((n - b0 < kBlock ? n - b0 : kBlock) * kRec);
        V4 *dst = rec + b0 * kRec;
        for (int k = threadIdx.x; k < cnt; k += kBlock) dst[k] = s_rec[k];
    }
}

// FP64 state of the adaptive mode's FP64 rows from the boundary arrays
struct Soa {
    const double *v, *V, *A, *B, *gA, *gB, *gv;
    const double4 *aux;   // {rho, P, c_s, -}
};

__device__ __forceinline__ void load_rec_soa(const Soa &s, const double4 *__restrict__ posH, int64_t n,
                                             int64_t j, const DerivPrm &p, Rec<double> &r) {
    double B3[3], gA3[3], gB9[9], gv9[9];
#pragma unroll
    for (int x = 0; x < 3; x++) {
        B3[x] = s.B[x * n + j];
        gA3[x] = s.gA[x * n + j];
    }
#pragma unroll
    for (int q = 0; q < 9; q++) {
        gB9[q] = s.gB[q * n + j];
        gv9[q] = s.gv[q * n + j];
    }
    const double4 a = s.aux[j];
    make_rec(posH[j].w, s.v[j], s.v[n + j], s.v[2 * n + j], s.V[j], a.y, a.x, a.z, s.A[j], B3, gA3,
             gB9, gv9, p, false, r);
}

template <typename T>
struct PairK {
    T Cq, eta_c, inv_eta_f, adot, inv_a, qs;
};

template <typename T>
__device__ __forceinline__ PairK<T> pair_k(const DerivPrm &p) {
    return PairK<T>{(T)p.Cq, (T)p.eta_c, (T)p.inv_eta_f, (T)p.adot, (T)p.inv_a, (T)p.qs};
}

// One ordered pair (i = a, j = b) of eqs. (mom) and (eng) with P -> P + Q:
//   FD = Vs_j (P_i + Q_i + P_j + Q_j) D,  D = grad W^R_ji - grad W^R_ij,
//   EP = Vs_j (P_j + Q_j) (v_j - v_i).D,
// so that m_i dv_i/dt = Vs_i sum FD and m_i du_i/dt = Vs_i a^-5 sum EP.
// With TS also the pair's time-step terms (Sec. 3.1): vs = the closing speed
// max(-w, 0), w = (xdot_ij + (adot/a) x_ij).x_ij / r, and qr = Q_i / rho_i.
template <typename T, bool TS>
__device__ __forceinline__ void pair_deriv(const Rec<T> &a, const Rec<T> &b, const T d[3],
                                           const PairK<T> &k, T FD[3], T &EP, T &vs, T &qr) {
    const T xx = d[0] * d[0], yy = d[1] * d[1], zz = d[2] * d[2];
    const T xy = d[0] * d[1], xz = d[0] * d[2], yz = d[1] * d[2];
    const T r2 = (xx + yy) + zz;
    const T r = Mth<T>::sqrt(r2);
    const T qi = r * fabs(a.ih), qj = r * fabs(b.ih);
    T pwi, pgi, pwj, pgj;
    kfac(qi, pwi, pgi);
    kfac(qj, pwj, pgj);
    // grad W^R_ij = pwi (U_i + M_i d) + ki d, grad W^R_ji = pwj (U_j - M_j d) - kj d
    const T ci = (T)1 + (a.B[0] * d[0] + a.B[1] * d[1] + a.B[2] * d[2]);
    const T cj = (T)1 - (b.B[0] * d[0] + b.B[1] * d[1] + b.B[2] * d[2]);
    const T kk = a.Ag * ci * pgi + b.Ag * cj * pgj;
    T D[3];
#pragma unroll
    for (int g = 0; g < 3; g++) {
        const T ei = a.U[g] + (a.M[g * 3 + 0] * d[0] + a.M[g * 3 + 1] * d[1] + a.M[g * 3 + 2] * d[2]);
        const T ej = b.U[g] - (b.M[g * 3 + 0] * d[0] + b.M[g * 3 + 1] * d[1] + b.M[g * 3 + 2] * d[2]);
        D[g] = (pwj * ej - pwi * ei) - kk * d[g];
    }
    // limiter, eqs. (phi)-(phiad), from s = d^T grad v d
    const T si = a.S[0] * xx + a.S[1] * yy + a.S[2] * zz + a.S[3] * xy + a.S[4] * xz + a.S[5] * yz;
    const T sj = b.S[0] * xx + b.S[1] * yy + b.S[2] * zz + b.S[3] * xy + b.S[4] * xz + b.S[5] * yz;
    const T vij[3] = {a.v[0] - b.v[0], a.v[1] - b.v[1], a.v[2] - b.v[2]};
    const T vd = vij[0] * d[0] + vij[1] * d[1] + vij[2] * d[2];
    const T prod = si * sj;
    const T ssum = si + sj;
    T phi = (T)0;
    if (prod > (T)0) {
        phi = (T)4 * prod * Mth<T>::rcp(ssum * ssum);
        phi = phi < (T)1 ? phi : (T)1;
        const T eta = qi < qj ? qi : qj;
        if (eta < k.eta_c) {
            const T x = (eta - k.eta_c) * k.inv_eta_f;
            phi *= Mth<T>::exp(-x * x);
        }
    }
    // projected velocity difference, eq. (hatvi), along d; eq. (mu), eq. (visc)
    const T ud = (vd - (T)0.5 * phi * ssum) + k.adot * r2;
    T Qi = (T)0, Qj = (T)0;
    if constexpr (TS) {
        const T w = (vd + k.adot * r2) * k.inv_a;
        vs = w < (T)0 ? -w * Mth<T>::rcp(r) : (T)0;
        qr = (T)0;
    }
    if (ud < (T)0) {
        const T mui = a.hA * ud * Mth<T>::rcp(r2 + a.he);
        const T muj = b.hA * ud * Mth<T>::rcp(r2 + b.he);
        const T qi_ = mui * (k.Cq * mui - a.Clcs);
        Qi = a.rho * qi_;
        Qj = b.rho * (muj * (k.Cq * muj - b.Clcs));
        if constexpr (TS) qr = qi_;
    }
    const T pqj = b.P + Qj;
    const T t = b.Vs * ((a.P + Qi) + pqj);
    FD[0] = t * D[0];
    FD[1] = t * D[1];
    FD[2] = t * D[2];
    EP = -(b.Vs * pqj) * (vij[0] * D[0] + vij[1] * D[1] + vij[2] * D[2]);
}

template <typename T>
__device__ __forceinline__ bool fp64_row(const Rec<T> &r) {
    return r.ih < (T)0;
}

// Balanced lane groups. Wave w owns the P particles [i0, i0 + np) and
// splits its 64 lanes among them in proportion to the lengths of their pair
// rows N_s(i) (gather row, then extras row): particle p gets a contiguous
// group of g_p >= 1 lanes, one plus its share of the other 64 - np lanes,
// so every group needs about the same number of steps and the wave's lanes
// stay busy whatever the rows' lengths. A lane keeps its particle's state
// in registers, strides over the row by g_p and sums its pairs in FP64;
// the groups' sums are reduced once at the end by a segmented scan across
// the lanes, and each group's last lane holds its particle's totals.
struct LaneGroup {
    int64_t i;   // particle of this lane
    int first;   // first entry of the row this lane takes
    int g;       // lanes of the group (the stride)
    int key;     // group id (particle offset in the wave)
    bool last;   // last lane of the group
};

// (eb == nullptr: gather rows only)
template <int P>
__device__ __forceinline__ LaneGroup lane_group(int64_t i0, int np, int lane,
                                                const int64_t *__restrict__ goff,
                                                const int32_t *__restrict__ eb,
                                                const int32_t *__restrict__ ee) {
    static_assert(P >= 1 && P <= 32, "at most 32 particles per wave");
    // row lengths and their inclusive prefix over the wave's particles
    const int len = lane < np ? (int)(goff[i0 + lane + 1] - goff[i0 + lane]) +
                                    (eb ? ee[i0 + lane] - eb[i0 + lane] : 0)
                              : 0;
    int cum = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(cum, o, 64);
        if (lane >= o) cum += t;
    }
    const int64_t S = __shfl(cum, 63, 64);
    // group start of particle p: p + floor((64 - np) * (prefix before p) / S),
    // increasing in p, 0 for p = 0
    const int spare = 64 - np;
    const int start = lane < np ? lane + (S > 0 ? (int)(((int64_t)spare * (cum - len)) / S) : 0) : 64;
    // this lane's particle: the last p with start_p <= lane
    int p = 0;
#pragma unroll
    for (int q = 1; q < P; q++) {
        const int sq = __shfl(start, q, 64);
        if (q < np && sq <= lane) p = q;
    }
    const int sp = __shfl(start, p, 64);
    const int sn = __shfl(start, p + 1 < np ? p + 1 : 63, 64);
    const int end = p + 1 < np ? sn : 64;
    LaneGroup lg;
    lg.i = i0 + p;
    lg.first = lane - sp;
    lg.g = end - sp;
    lg.key = p;
    lg.last = lane == end - 1;
    return lg;
}

// sum of x over the lanes of each group, left in the group's last lane
template <typename T, int K>
__device__ __forceinline__ void group_scan(int lane, int key, T (&x)[K]) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int ko = __shfl_up(key, o, 64);
        const bool take = lane >= o && ko == key;
#pragma unroll
        for (int k = 0; k < K; k++) {
            const T y = __shfl_up(x[k], o, 64);
            if (take) x[k] += y;
        }
    }
}

template <typename T>
__device__ __forceinline__ void group_scan_max(int lane, int key, T &x) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int ko = __shfl_up(key, o, 64);
        const T y = __shfl_up(x, o, 64);
        if (lane >= o && ko == key) x = x > y ? x : y;
    }
}

// first particle of this wave when every wave takes P particles
__device__ __forceinline__ int64_t wave_first(int P) {
    return (xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + (threadIdx.x >> 6)) * (int64_t)P;
}

// Derivative pass, balanced lane groups (P particles per wave). Pairs with
// an FP64-row flag on either side are left to k_deriv_fix.
template <typename T, int P, bool TS>
__global__ __launch_bounds__(kBlock) void k_deriv_bal(const double4 *__restrict__ posH,
                                                      const int64_t *__restrict__ goff,
                                                      const int32_t *__restrict__ gidx,
                                                      const int32_t *__restrict__ eb,
                                                      const int32_t *__restrict__ ee,
                                                      const int32_t *__restrict__ eidx,
                                                      const typename std::conditional<sizeof(T) == 4, float4, double4>::type *__restrict__ rec,
                                                      const double *__restrict__ m, int64_t n, Box box,
                                                      DerivPrm p, double *dpdt, double *dudt,
                                                      double *ts_vs = nullptr, double *ts_qr = nullptr) {
    const int64_t i0 = wave_first(P);
    if (i0 >= n) return;   // whole waves leave together
    const int lane = threadIdx.x & 63;
    const int np = (int)(n - i0 < P ? n - i0 : P);
    const LaneGroup lg = lane_group<P>(i0, np, lane, goff, eb, ee);
    const int64_t i = lg.i;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    T vs = (T)0, qr = (T)0;
    Rec<T> si;
    load_rec(rec, i, si);
    const double4 pi = posH[i];
    const PairK<T> pk = pair_k<T>(p);
    const int64_t gb = goff[i];
    const int ngi = (int)(goff[i + 1] - gb);
    const int ebi = eb[i];
    const int tot = fp64_row(si) ? 0 : ngi + (ee[i] - ebi);
    const int G = lg.g;
    int kk = lg.first;
    int32_t jn = kk < tot ? (kk < ngi ? gidx[gb + kk] : eidx[ebi + (kk - ngi)]) : 0;
    for (; kk < tot; kk += G) {
        const int32_t j = jn;
        const int kn = kk + G;
        if (kn < tot) jn = kn < ngi ? gidx[gb + kn] : eidx[ebi + (kn - ngi)];
        // the partner's position and record are loaded together and the
        // pair is evaluated before its FP64-row flag is looked at, so no
        // load waits on another
        Rec<T> sj;
        load_rec(rec, j, sj);
        T d[3];
        if constexpr (sizeof(T) == 4) {
            // FP32 pair terms: d from the fixed-point positions, whose
            // 32-bit difference wraps to the minimum image (error at most
            // L 2^-32 per component, then the FP32 rounding); the position
            // rides in the record, so no separate position load
#pragma unroll
            for (int x = 0; x < 3; x++) d[x] = fixed_d(si.q[x], unpack_f(si.qf, x), sj.q[x], unpack_f(sj.qf, x), pk.qs);
        } else {
            separation(pi, posH[j], box, d[0], d[1], d[2]);
        }
        T FD[3], EP, pvs, pqr;
        pair_deriv<T, TS>(si, sj, d, pk, FD, EP, pvs, pqr);
        if (!fp64_row(sj)) {
            a[0] += (double)FD[0];
            a[1] += (double)FD[1];
            a[2] += (double)FD[2];
            a[3] += (double)EP;
            if constexpr (TS) {
                vs = pvs > vs ? pvs : vs;
                qr = pqr > qr ? pqr : qr;
            }
        }
    }
    group_scan<double, 4>(lane, lg.key, a);
    if constexpr (TS) {
        group_scan_max<T>(lane, lg.key, vs);
        group_scan_max<T>(lane, lg.key, qr);
    }
    if (lg.last) {
        const double f = (double)si.Vs / m[i];
        dpdt[i] = a[0] * f;
        dpdt[n + i] = a[1] * f;
        dpdt[2 * n + i] = a[2] * f;
        dudt[i] = a[3] * f * p.inv_a5;
        if constexpr (TS) {
            ts_vs[i] = (double)vs;
            ts_qr[i] = (double)qr;
        }
    }
}

// Volume pass, balanced lane groups (gather rows only): n_i = W(0, H_i) +
// sum_j W(r, H_i), the self term taken by the group's first lane.
template <typename T, int P>
__global__ __launch_bounds__(kBlock) void k_volume_bal(const double4 *__restrict__ posH,
                                                       const int64_t *__restrict__ goff,
                                                       const int32_t *__restrict__ gidx, int64_t n,
                                                       Box box, double *nsum_out, double *V_out, T *recV,
                                                       double4 *posV) {
    const int64_t i0 = wave_first(P);
    if (i0 >= n) return;
    const int lane = threadIdx.x & 63;
    const int np = (int)(n - i0 < P ? n - i0 : P);
    const LaneGroup lg = lane_group<P>(i0, np, lane, goff, nullptr, nullptr);
    const int64_t i = lg.i;
    const double4 pi = posH[i];
    const T invH = (T)(1.0 / pi.w);
    const T cw = (T)kW * invH * invH * invH;
    double a[1] = {lg.first == 0 ? (double)cw : 0.0};
    const int64_t gb = goff[i];
    const int tot = (int)(goff[i + 1] - gb);
    const int G = lg.g;
    int kk = lg.first;
    int32_t jn = kk < tot ? gidx[gb + kk] : 0;
    for (; kk < tot; kk += G) {
        const int32_t j = jn;
        if (kk + G < tot) jn = gidx[gb + kk + G];
        const double4 pj = posH[j];
        T dx, dy, dz;
        separation(pi, pj, box, dx, dy, dz);
        const T q = Mth<T>::sqrt(dx * dx + dy * dy + dz * dz) * invH;
        a[0] += (double)kernel_w(q, cw);
    }
    group_scan<double, 1>(lane, lg.key, a);
    if (lg.last) {
        if (nsum_out) nsum_out[i] = a[0];
        V_out[i] = 1.0 / a[0];
        recV[i] = (T)(1.0 / a[0]);
        // the moment pass reads a partner's position and volume in one load
        posV[i] = make_double4(pi.x, pi.y, pi.z, 1.0 / a[0]);
    }
}

// Moment pass, balanced lane groups (gather rows only): the 29 sums of
// k_moments, assembled into the 40 outputs by the group's last lane.
template <typename T, int P>
__global__ __launch_bounds__(kBlock) void k_moments_bal(const double4 *__restrict__ posH,
                                                        const int64_t *__restrict__ goff,
                                                        const int32_t *__restrict__ gidx,
                                                        const double4 *__restrict__ posV, int64_t n, Box box,
                                                        double *m0, double *m1, double *m2, double *gm0,
                                                        double *gm1, double *gm2) {
    const int64_t i0 = wave_first(P);
    if (i0 >= n) return;
    const int lane = threadIdx.x & 63;
    const int np = (int)(n - i0 < P ? n - i0 : P);
    const LaneGroup lg = lane_group<P>(i0, np, lane, goff, nullptr, nullptr);
    const int64_t i = lg.i;
    // sums: 0 m0 | 1-3 m1 | 4-9 m2 | 10-12 gm0 | 13-18 Q2 | 19-28 Q3
    double a[29] = {};
    const double4 pi = posH[i];
    const T invH = (T)(1.0 / pi.w);
    const T invH2 = invH * invH;
    const T cw = (T)kW * invH2 * invH;
    const T cg = (T)kG * invH2 * invH2 * invH;
    if (lg.first == 0) a[0] = (double)((T)posV[i].w * cw);   // self pair: d = 0, so m0 only
    const int64_t gb = goff[i];
    const int tot = (int)(goff[i + 1] - gb);
    const int G = lg.g;
    int kk = lg.first;
    int32_t jn = kk < tot ? gidx[gb + kk] : 0;
    for (; kk < tot; kk += G) {
        const int32_t j = jn;
        if (kk + G < tot) jn = gidx[gb + kk + G];
        const double4 pj = posV[j];   // x, y, z and V
        const T Vj = (T)pj.w;
        T d[3];
        separation(pi, pj, box, d[0], d[1], d[2]);
        const T q = Mth<T>::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) * invH;
        T w, gf;
        kernel_wg(q, cw, cg, w, gf);
        const T t = Vj * w, u = Vj * gf;
        a[0] += (double)t;
        T dd[6];
#pragma unroll
        for (int x = 0; x < 3; x++) {
            a[1 + x] += (double)(t * d[x]);
            a[10 + x] += (double)(u * d[x]);
#pragma unroll
            for (int y = x; y < 3; y++) dd[kSym2[x][y]] = d[x] * d[y];
        }
#pragma unroll
        for (int e = 0; e < 6; e++) {
            a[4 + e] += (double)(t * dd[e]);
            a[13 + e] += (double)(u * dd[e]);
        }
#pragma unroll
        for (int x = 0; x < 3; x++)
#pragma unroll
            for (int y = x; y < 3; y++)
#pragma unroll
                for (int z = y; z < 3; z++) a[19 + kSym3[x][y][z]] += (double)(u * dd[kSym2[x][y]] * d[z]);
    }
    group_scan<double, 29>(lane, lg.key, a);
    if (lg.last) {
        const double p0 = a[0];
        const double p1[3] = {a[1], a[2], a[3]};
        m0[i] = p0;
#pragma unroll
        for (int x = 0; x < 3; x++) {
            m1[x * n + i] = p1[x];
            gm0[x * n + i] = a[10 + x];
        }
#pragma unroll
        for (int e = 0; e < 6; e++) m2[e * n + i] = a[4 + e];
#pragma unroll
        for (int x = 0; x < 3; x++)
#pragma unroll
            for (int c = 0; c < 3; c++) gm1[(x * 3 + c) * n + i] = a[13 + kSym2[x][c]] + (x == c ? p0 : 0.0);
        int s = 0;
#pragma unroll
        for (int x = 0; x < 3; x++)
#pragma unroll
            for (int y = x; y < 3; y++, s++)
#pragma unroll
                for (int c = 0; c < 3; c++)
                    gm2[(s * 3 + c) * n + i] = a[19 + kSym3[x][y][c]] + (x == c ? p1[y] : 0.0) +
                                               (y == c ? p1[x] : 0.0);
    }
}

// Velocity gradient, balanced lane groups (P particles per wave, gather
// rows only). i's RK template is regrouped once per lane as in the
// derivative pass: grad W^R_ij = pw (U + M d) + Ag c pg d. Rows with
// skip[i] set are left to the FP64 launch.
template <typename T, int P>
__global__ __launch_bounds__(kBlock) void k_gradv_bal(const double4 *__restrict__ posH,
                                                      const int64_t *__restrict__ goff,
                                                      const int32_t *__restrict__ gidx,
                                                      const typename std::conditional<sizeof(T) == 4, float4, double4>::type *__restrict__ rec6,
                                                      const double *__restrict__ A, const double *__restrict__ B,
                                                      const double *__restrict__ gA,
                                                      const double *__restrict__ gB, int64_t n, Box box,
                                                      const int32_t *__restrict__ skip, double *gradv) {
    const int64_t i0 = wave_first(P);
    if (i0 >= n) return;   // whole waves leave together
    const int lane = threadIdx.x & 63;
    const int np = (int)(n - i0 < P ? n - i0 : P);
    const LaneGroup lg = lane_group<P>(i0, np, lane, goff, nullptr, nullptr);
    const int64_t i = lg.i;
    const bool run = !(skip && skip[i]);
    // i's template
    const double4 pi = posH[i];
    const double ihd = 1.0 / pi.w, cwd = kW * ihd * ihd * ihd;
    const double Ad = A[i];
    double Bd[3], gAd[3];
#pragma unroll
    for (int x = 0; x < 3; x++) {
        Bd[x] = B[x * n + i];
        gAd[x] = gA[x * n + i];
    }
    T U[3], M[9], Bt[3];
#pragma unroll
    for (int g = 0; g < 3; g++) {
        Bt[g] = (T)Bd[g];
        U[g] = (T)(cwd * (gAd[g] + Ad * Bd[g]));
#pragma unroll
        for (int a = 0; a < 3; a++) M[g * 3 + a] = (T)(cwd * (gAd[g] * Bd[a] + Ad * gB[(a * 3 + g) * n + i]));
    }
    const T Ag = (T)(Ad * kG * ihd * ihd * ihd * ihd * ihd);
    const T ih = (T)ihd;
    constexpr int S6 = sizeof(T) == 4 ? 2 : 1;   // FP32 records: (v, V), position
    const auto ri = rec6[S6 * i];
    const T vi[3] = {(T)ri.x, (T)ri.y, (T)ri.z};
    double a[9] = {};
    const int64_t gb = goff[i];
    const int tot = run ? (int)(goff[i + 1] - gb) : 0;
    const int G = lg.g;
    int kk = lg.first;
    int32_t jn = kk < tot ? gidx[gb + kk] : 0;
    for (; kk < tot; kk += G) {
        const int32_t j = jn;
        if (kk + G < tot) jn = gidx[gb + kk + G];
        const double4 pj = posH[j];
        const auto rj = rec6[S6 * j];
        T d[3];
        separation(pi, pj, box, d[0], d[1], d[2]);
        const T r = Mth<T>::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        T pw, pg;
        kfac(r * ih, pw, pg);
        const T k = Ag * ((T)1 + (Bt[0] * d[0] + Bt[1] * d[1] + Bt[2] * d[2])) * pg;
        T Gr[3];
#pragma unroll
        for (int g = 0; g < 3; g++)
            Gr[g] = pw * (U[g] + (M[g * 3 + 0] * d[0] + M[g * 3 + 1] * d[1] + M[g * 3 + 2] * d[2])) + k * d[g];
        // -V_j (v_i - v_j) (x) grad W^R_ij
        const T w[3] = {((T)rj.x - vi[0]) * (T)rj.w, ((T)rj.y - vi[1]) * (T)rj.w, ((T)rj.z - vi[2]) * (T)rj.w};
#pragma unroll
        for (int x = 0; x < 3; x++)
#pragma unroll
            for (int y = 0; y < 3; y++) a[x * 3 + y] += (double)(w[x] * Gr[y]);
    }
    group_scan<double, 9>(lane, lg.key, a);
    if (lg.last && run)
#pragma unroll
        for (int q = 0; q < 9; q++) gradv[q * n + i] = a[q];
}

// Derivative pass, G lanes per particle striding over N_s(i) (the gather row,
// then the extras row), compensated sums reduced across the group.
template <typename T, int G, bool TS = false>
__global__ __launch_bounds__(kBlock) void k_deriv(const double4 *__restrict__ posH,
                                                  const int64_t *__restrict__ goff,
                                                  const int32_t *__restrict__ gidx,
                                                  const int32_t *__restrict__ eb,
                                                  const int32_t *__restrict__ ee,
                                                  const int32_t *__restrict__ eidx,
                                                  const typename std::conditional<sizeof(T) == 4, float4, double4>::type *__restrict__ rec,
                                                  const double *__restrict__ m, int64_t n, Box box,
                                                  DerivPrm p, double *dpdt, double *dudt,
                                                  double *ts_vs = nullptr, double *ts_qr = nullptr) {
    int l;
    int64_t i = group_index(G, l);
    Acc<T> a[4];
    T vs = (T)0, qr = (T)0;
    T Vsi = (T)0;
    if (i < n) {
        const double4 pi = posH[i];
        Rec<T> si;
        load_rec(rec, i, si);
        Vsi = si.Vs;
        const PairK<T> pk = pair_k<T>(p);
        const int64_t gb = goff[i];
        const int ngi = (int)(goff[i + 1] - gb);
        const int ebi = eb[i];
        const int tot = fp64_row(si) ? 0 : ngi + (ee[i] - ebi);
        int32_t jn = l < tot ? (l < ngi ? gidx[gb + l] : eidx[ebi + (l - ngi)]) : 0;
        for (int kk = l; kk < tot; kk += G) {
            const int32_t j = jn;
            const int kn = kk + G;
            if (kn < tot) jn = kn < ngi ? gidx[gb + kn] : eidx[ebi + (kn - ngi)];
            const double4 pj = posH[j];
            Rec<T> sj;
            load_rec(rec, j, sj);
            T d[3];
            separation(pi, pj, box, d[0], d[1], d[2]);
            T FD[3], EP, pvs, pqr;
            pair_deriv<T, TS>(si, sj, d, pk, FD, EP, pvs, pqr);
            if (!fp64_row(sj)) {
                a[0].add(FD[0]);
                a[1].add(FD[1]);
                a[2].add(FD[2]);
                a[3].add(EP);
                if constexpr (TS) {
                    vs = pvs > vs ? pvs : vs;
                    qr = pqr > qr ? pqr : qr;
                }
            }
        }
    }
    group_reduce<T, G, 4>(a);
    if constexpr (TS) {
#pragma unroll
        for (int o = G / 2; o >= 1; o >>= 1) {
            const T v2 = __shfl_xor(vs, o, G), q2 = __shfl_xor(qr, o, G);
            vs = v2 > vs ? v2 : vs;
            qr = q2 > qr ? q2 : qr;
        }
    }
    if (i < n && l == 0) {
        const double f = (double)Vsi / m[i];
        dpdt[i] = a[0].value() * f;
        dpdt[n + i] = a[1].value() * f;
        dpdt[2 * n + i] = a[2].value() * f;
        dudt[i] = a[3].value() * f * p.inv_a5;
        if constexpr (TS) {
            ts_vs[i] = (double)vs;
            ts_qr[i] = (double)qr;
        }
    }
}

// FP64 rows of the adaptive mode: for each listed particle, every pair when
// the particle itself is flagged, else only the pairs with a flagged
// partner; the FP64 sums are added to the outputs of the FP32 launch.
template <int G, bool TS = false>
__global__ __launch_bounds__(kBlock) void k_deriv_fix(const double4 *__restrict__ posH,
                                                      const int64_t *__restrict__ goff,
                                                      const int32_t *__restrict__ gidx,
                                                      const int32_t *__restrict__ eb,
                                                      const int32_t *__restrict__ ee,
                                                      const int32_t *__restrict__ eidx, Soa s,
                                                      const int32_t *__restrict__ flag,
                                                      const int32_t *__restrict__ list, int64_t nlist,
                                                      const int64_t *__restrict__ nlist_dev,
                                                      const double *__restrict__ m, int64_t n, Box box,
                                                      DerivPrm p, double *dpdt, double *dudt,
                                                      double *ts_vs = nullptr, double *ts_qr = nullptr) {
    int l;
    int64_t g = group_index(G, l);
    if (nlist_dev) nlist = *nlist_dev;
    const int64_t gstride = (int64_t)gridDim.x * (kBlock / G);
    for (; g < nlist; g += gstride) {
        const int64_t i = list[g];
        Acc<double> a[4];
        double vs = 0.0, qr = 0.0, Vsi = 0.0;
        if (i >= 0) {
            const double4 pi = posH[i];
            Rec<double> si;
            load_rec_soa(s, posH, n, i, p, si);
            Vsi = si.Vs;
            const PairK<double> pk = pair_k<double>(p);
            const bool all = flag[i] != 0;
            const int64_t gb = goff[i];
            const int ngi = (int)(goff[i + 1] - gb);
            const int ebi = eb[i];
            const int tot = ngi + (ee[i] - ebi);
            for (int kk = l; kk < tot; kk += G) {
                const int32_t j = kk < ngi ? gidx[gb + kk] : eidx[ebi + (kk - ngi)];
                if (!all && flag[j] == 0) continue;
                Rec<double> sj;
                load_rec_soa(s, posH, n, j, p, sj);
                double d[3];
                separation(pi, posH[j], box, d[0], d[1], d[2]);
                double FD[3], EP, pvs, pqr;
                pair_deriv<double, TS>(si, sj, d, pk, FD, EP, pvs, pqr);
                a[0].add(FD[0]);
                a[1].add(FD[1]);
                a[2].add(FD[2]);
                a[3].add(EP);
                if constexpr (TS) {
                    vs = fmax(vs, pvs);
                    qr = fmax(qr, pqr);
                }
            }
        }
        group_reduce<double, G, 4>(a);
        if constexpr (TS) {
#pragma unroll
            for (int o = G / 2; o >= 1; o >>= 1) {
                vs = fmax(vs, __shfl_xor(vs, o, G));
                qr = fmax(qr, __shfl_xor(qr, o, G));
            }
        }
        if (l == 0 && i >= 0) {
            const double f = Vsi / m[i];
            dpdt[i] += a[0].value() * f;
            dpdt[n + i] += a[1].value() * f;
            dpdt[2 * n + i] += a[2].value() * f;
            dudt[i] += a[3].value() * f * p.inv_a5;
            if constexpr (TS) {
                // the pairs the FP32 launch skipped: the maximum over both launches
                ts_vs[i] = fmax(ts_vs[i], vs);
                ts_qr[i] = fmax(ts_qr[i], qr);
            }
        }
    }
}

// Compatible energy update (eqs. compEng, compEng2, Eij, ptdt, fij): per
// particle q = p + p' = 2 p + dt dp/dt (p = a v, or the kick's start
// momenta pk when given; eq. ptdt) and the specific entropy s = P / rho^gamma,
// FP64, then rounded to the pass's type.
template <typename V4, typename T>
__global__ __launch_bounds__(kBlock) void k_pack_ce(int64_t n, const double *v, const double *pk,
                                                    const double *dpdt,
                                                    const double *m, const double *u,
                                                    const double *rho, const double *V, double gamma,
                                                    double a, double dt, V4 *ce, double4 *ced) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double r = rho ? rho[i] : m[i] / V[i];
    const double sp = (gamma - 1.0) * u[i] * pow(r, 1.0 - gamma);
    const double px = pk ? pk[i] : a * v[i];
    const double py = pk ? pk[n + i] : a * v[n + i];
    const double pz = pk ? pk[2 * n + i] : a * v[2 * n + i];
    const double qx = 2.0 * px + dt * dpdt[i];
    const double qy = 2.0 * py + dt * dpdt[n + i];
    const double qz = 2.0 * pz + dt * dpdt[2 * n + i];
    ce[i] = V4{(T)qx, (T)qy, (T)qz, (T)sp};
    if (ced) ced[i] = make_double4(qx, qy, qz, sp);
}

// One ordered pair of the compatible update: c = (q_j - q_i).F with F =
// m_i dp_ij/dt of eq. (mom) (here F / Vs_i, which has the same sign), so
// Delta E_ij = c / (2 a^4) and, from the four cases of eq. (fij), f_ij =
// s_j / (s_i + s_j) when Delta E_ij >= 0 and s_i / (s_i + s_j) otherwise;
// returns f_ij c.
template <typename T, typename V4>
__device__ __forceinline__ T compat_term(const V4 &ci, const V4 &cj, const T F[3]) {
    const T c = (cj.x - ci.x) * F[0] + (cj.y - ci.y) * F[1] + (cj.z - ci.z) * F[2];
    const T sh = c >= (T)0 ? cj.w : ci.w;
    return sh * Mth<T>::rcp(ci.w + cj.w) * c;
}

// Delta u_i = dt / (2 a^4 m_i) sum_j f_ij c_ij - dt (adot/a)(3(gamma-1)+2) u_i,
// balanced lane groups. With NK = 2 a second kick (records ce2, output du2)
// shares the pair forces. Pairs with an FP64-row flag on either side are
// left to k_compat_fix.
template <typename T, int P, int NK>
__global__ __launch_bounds__(kBlock) void k_compat_bal(const double4 *__restrict__ posH,
                                                       const int64_t *__restrict__ goff,
                                                       const int32_t *__restrict__ gidx,
                                                       const int32_t *__restrict__ eb,
                                                       const int32_t *__restrict__ ee,
                                                       const int32_t *__restrict__ eidx,
                                                       const typename std::conditional<sizeof(T) == 4, float4, double4>::type *__restrict__ rec,
                                                       const typename std::conditional<sizeof(T) == 4, float4, double4>::type *__restrict__ ce,
                                                       const typename std::conditional<sizeof(T) == 4, float4, double4>::type *__restrict__ ce2,
                                                       const double *__restrict__ m,
                                                       const double *__restrict__ u, int64_t n, Box box,
                                                       DerivPrm p, double scale, double cool, double *du,
                                                       double *du2) {
    using V4 = typename std::conditional<sizeof(T) == 4, float4, double4>::type;
    const int64_t i0 = wave_first(P);
    if (i0 >= n) return;
    const int lane = threadIdx.x & 63;
    const int np = (int)(n - i0 < P ? n - i0 : P);
    const LaneGroup lg = lane_group<P>(i0, np, lane, goff, eb, ee);
    const int64_t i = lg.i;
    double a[NK] = {};
    Rec<T> si;
    load_rec(rec, i, si);
    const double4 pi = posH[i];
    const V4 cei = ce[i];
    const V4 cei2 = NK == 2 ? ce2[i] : cei;
    const PairK<T> pk = pair_k<T>(p);
    const int64_t gb = goff[i];
    const int ngi = (int)(goff[i + 1] - gb);
    const int ebi = eb[i];
    const int tot = fp64_row(si) ? 0 : ngi + (ee[i] - ebi);
    const int G = lg.g;
    int kk = lg.first;
    int32_t jn = kk < tot ? (kk < ngi ? gidx[gb + kk] : eidx[ebi + (kk - ngi)]) : 0;
    for (; kk < tot; kk += G) {
        const int32_t j = jn;
        const int kn = kk + G;
        if (kn < tot) jn = kn < ngi ? gidx[gb + kn] : eidx[ebi + (kn - ngi)];
        const V4 cej = ce[j];
        const V4 cej2 = NK == 2 ? ce2[j] : cej;
        Rec<T> sj;
        load_rec(rec, j, sj);
        T d[3];
        if constexpr (sizeof(T) == 4) {
            // as in the derivative pass: d from the records' fixed-point positions
#pragma unroll
            for (int x = 0; x < 3; x++) d[x] = fixed_d(si.q[x], unpack_f(si.qf, x), sj.q[x], unpack_f(sj.qf, x), pk.qs);
        } else {
            separation(pi, posH[j], box, d[0], d[1], d[2]);
        }
        T FD[3], EP, vs, qr;
        pair_deriv<T, false>(si, sj, d, pk, FD, EP, vs, qr);
        if (!fp64_row(sj)) {
            a[0] += (double)compat_term<T>(cei, cej, FD);
            if constexpr (NK == 2) a[1] += (double)compat_term<T>(cei2, cej2, FD);
        }
    }
    group_scan<double, NK>(lane, lg.key, a);
    if (lg.last) {
        const double f = (double)si.Vs * scale / m[i];
        du[i] = a[0] * f - cool * u[i];
        if constexpr (NK == 2) du2[i] = a[1] * f - cool * u[i];
    }
}

// FP64 pairs of the adaptive mode (as k_deriv_fix): adds their share of
// the sum to the output(s) of k_compat_bal.
template <int G, int NK>
__global__ __launch_bounds__(kBlock) void k_compat_fix(const double4 *__restrict__ posH,
                                                       const int64_t *__restrict__ goff,
                                                       const int32_t *__restrict__ gidx,
                                                       const int32_t *__restrict__ eb,
                                                       const int32_t *__restrict__ ee,
                                                       const int32_t *__restrict__ eidx, Soa s,
                                                       const double4 *__restrict__ ced,
                                                       const double4 *__restrict__ ced2,
                                                       const int32_t *__restrict__ flag,
                                                       const int32_t *__restrict__ list, int64_t nlist,
                                                       const double *__restrict__ m, int64_t n, Box box,
                                                       DerivPrm p, double scale, double *du,
                                                       double *du2) {
    int l;
    int64_t g = group_index(G, l);
    const int64_t gstride = (int64_t)gridDim.x * (kBlock / G);
    for (; g < nlist; g += gstride) {
        const int64_t i = list[g];
        Acc<double> a[NK];
        double Vsi = 0.0;
        if (i >= 0) {
            const double4 pi = posH[i];
            Rec<double> si;
            load_rec_soa(s, posH, n, i, p, si);
            Vsi = si.Vs;
            const double4 cei = ced[i];
            const double4 cei2 = NK == 2 ? ced2[i] : cei;
            const PairK<double> pk = pair_k<double>(p);
            const bool all = flag[i] != 0;
            const int64_t gb = goff[i];
            const int ngi = (int)(goff[i + 1] - gb);
            const int ebi = eb[i];
            const int tot = ngi + (ee[i] - ebi);
            for (int kk = l; kk < tot; kk += G) {
                const int32_t j = kk < ngi ? gidx[gb + kk] : eidx[ebi + (kk - ngi)];
                if (!all && flag[j] == 0) continue;
                Rec<double> sj;
                load_rec_soa(s, posH, n, j, p, sj);
                double d[3];
                separation(pi, posH[j], box, d[0], d[1], d[2]);
                double FD[3], EP, pvs, pqr;
                pair_deriv<double, false>(si, sj, d, pk, FD, EP, pvs, pqr);
                a[0].add(compat_term<double>(cei, ced[j], FD));
                if constexpr (NK == 2) a[1].add(compat_term<double>(cei2, ced2[j], FD));
            }
        }
        group_reduce<double, G, NK>(a);
        if (l == 0 && i >= 0) {
            du[i] += a[0].value() * (Vsi * scale / m[i]);
            if constexpr (NK == 2) du2[i] += a[1].value() * (Vsi * scale / m[i]);
        }
    }
}

// Courant criterion (Sec. 3.1) per particle from the derivative pass's
// maxima: c_s from the gas state, c_sq = sqrt(zeta max Q/rho), |div u| =
// |Tr grad v + 3 adot|, h_hat = H / n_h; v_max = max(v_sig, c_s, c_sq,
// h_hat |div u| / a) and dt_hyd = C_CFL h_hat / v_max (time; the caller
// applies dy/dt).
__global__ __launch_bounds__(kBlock) void k_timestep(int64_t n, const double4 *__restrict__ posH,
                                                     const double *__restrict__ u,
                                                     const double *__restrict__ m,
                                                     const double *__restrict__ rho,
                                                     const double *__restrict__ V,
                                                     const double *__restrict__ gradv,
                                                     const double *__restrict__ tvs,
                                                     const double *__restrict__ tqr, double gamma,
                                                     double inv_nh, double a, double adot, double zeta,
                                                     double c_cfl, double *vsig, double *csq,
                                                     double *vmax, double *dt) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double r = rho ? rho[i] : m[i] / V[i];
    const double P = (gamma - 1.0) * r * u[i];
    const double cs = sqrt(gamma * P / r);
    const double cq = sqrt(zeta * tqr[i]);
    const double hh = posH[i].w * inv_nh;
    const double divu = fabs(gradv[i] + gradv[4 * n + i] + gradv[8 * n + i] + 3.0 * adot);
    const double vm = fmax(fmax(tvs[i], cs), fmax(cq, hh / a * divu));
    if (vsig) vsig[i] = tvs[i];
    if (csq) csq[i] = cq;
    vmax[i] = vm;
    if (dt) dt[i] = c_cfl * hh / vm;
}

// Conditioning of particle i's RK template: the pair terms of eq. (gRK)
// carry B.d, (gradB)^T d and gradA / A, which reach |B| H, |gradB| H^2 and
// |gradA| H / |A| relative to the O(1) part; their sum bounds how much a
// rounding of the terms is amplified in the (cancelling) row sums.
__global__ __launch_bounds__(kBlock) void k_flag(int64_t n, const double4 *__restrict__ posH,
                                                 const double *A, const double *B, const double *gA,
                                                 const double *gB, double kappa_max, int32_t *flag,
                                                 int32_t *flist, unsigned long long *nflag) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int f = 0;
    if (i < n) {
        f = kappa_flag(i, n, posH, A, B, gA, gB, kappa_max);
        flag[i] = f;
    }
    append_row(f != 0, i, flist, nflag);
}

// rows that need an FP64 launch in the derivative pass: the flagged
// particles and their partners (N_s is symmetric, so the partners of a
// flagged particle are exactly the particles with a flagged partner).
// Sixteen lanes per flagged particle, over a grid of any size; the count is
// *nf, where k_flag counted its appends.
__global__ __launch_bounds__(kBlock) void k_mark(const int32_t *__restrict__ flist,
                                                 const int64_t *__restrict__ nf,
                                                 const int64_t *__restrict__ goff,
                                                 const int32_t *__restrict__ gidx,
                                                 const int32_t *__restrict__ eb,
                                                 const int32_t *__restrict__ ee,
                                                 const int32_t *__restrict__ eidx, int32_t *mark) {
    constexpr int G = 16;
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int l = (int)(gid % G);
    const int64_t cnt = *nf;
    const int64_t stride = (int64_t)gridDim.x * (kBlock / G);
    for (int64_t k = gid / G; k < cnt; k += stride) {
        const int32_t i = flist[k];
        if (l == 0) mark[i] = 1;
        for (int64_t q = goff[i] + l; q < goff[i + 1]; q += G) mark[gidx[q]] = 1;
        for (int q = eb[i] + l; q < ee[i]; q += G) mark[eidx[q]] = 1;
    }
}

// marks a[0..n) and the flag counter cleared
__global__ __launch_bounds__(kBlock) void k_zero_marks(int32_t *a, int64_t n, int64_t *c0) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) a[i] = 0;
    if (i == 0) *c0 = 0;
}

__global__ __launch_bounds__(kBlock) void k_compact(int64_t n, const int64_t *__restrict__ pos,
                                                    int32_t *list) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n && pos[i + 1] != pos[i]) list[pos[i]] = (int32_t)i;
}

// FP32 velocity-gradient records: (v, V), then the 32-bit fixed-point
// position q = floor(x 2^32 / L) (the bits in the float slots)
__global__ __launch_bounds__(kBlock) void k_pack6_f(int64_t n, const double *v, const double *V,
                                                    const double4 *__restrict__ posH, double qinv,
                                                    float4 *rec) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    rec[2 * i] = make_float4((float)v[i], (float)v[n + i], (float)v[2 * n + i], (float)V[i]);
    const double4 x = posH[i];
    const Fixed fx = fixed_q(x.x, qinv), fy = fixed_q(x.y, qinv), fz = fixed_q(x.z, qinv);
    rec[2 * i + 1] = make_float4(__uint_as_float(fx.q), __uint_as_float(fy.q), __uint_as_float(fz.q),
                                 __uint_as_float(pack_f(fx, fy, fz)));
}
__global__ __launch_bounds__(kBlock) void k_pack6_d(int64_t n, const double *v, const double *V,
                                                    double4 *rec) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) rec[i] = make_double4(v[i], v[n + i], v[2 * n + i], V[i]);
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
inline unsigned gblocks(int64_t n, int G) { return (unsigned)((n * G + kBlock - 1) / kBlock); }
// list launches of graph mode do not know their row count on the host: a
// bounded grid loops over the rows (the flagged rows are a small fraction)
inline unsigned fix_blocks(int64_t rows, int G, bool graph) {
    unsigned b = gblocks(rows, G);
    return graph ? std::min(b, 2048u) : b;
}

#define CRK_DISPATCH_G(G, LAUNCH)                                                          \
    switch (G) {                                                                           \
        case 1: LAUNCH(1); break;                                                          \
        case 2: LAUNCH(2); break;                                                          \
        case 4: LAUNCH(4); break;                                                          \
        case 8: LAUNCH(8); break;                                                          \
        case 16: LAUNCH(16); break;                                                        \
        case 32: LAUNCH(32); break;                                                        \
        case 64: LAUNCH(64); break;                                                        \
        default: return set_err(c, CRK_ERR_INVALID_ARG, "lanes per particle must be a power of two <= 64"); \
    }

DerivPrm deriv_prm(const crk_params *p) {
    const double a = p->a;
    return DerivPrm{p->gamma, p->Cl, p->Cq, p->eps * p->eps, 1.0 / p->nh, 1.0 / a, p->adot,
                    p->eta_crit, 1.0 / p->eta_fold, a * sqrt(0.5), 1.0 / (a * a * a * a * a),
                    4398046511104.0 / p->L, p->L / 4294967296.0};
}

// balanced-lane derivative / compatible launches: particles per wave (4 .. 32)
#define CRK_DISPATCH_P(P, LAUNCH)                                                          \
    switch (P) {                                                                           \
        case 4: LAUNCH(4); break;                                                          \
        case 8: LAUNCH(8); break;                                                          \
        case 16: LAUNCH(16); break;                                                        \
        case 32: LAUNCH(32); break;                                                        \
        default: return set_err(c, CRK_ERR_INVALID_ARG, "particles per wave must be 4, 8, 16 or 32"); \
    }

inline unsigned pblocks(int64_t n, int P) {
    return (unsigned)(((n + P - 1) / P + kBlock / 64 - 1) / (kBlock / 64));
}

// volume then (optionally) moment pass in type T, with the lane mapping of
// the context (balanced groups of P particles per wave, or G lanes each)
// n_i and V_i of the volumes the build summed (vnsum, posV.w) into the
// caller's arrays
__global__ __launch_bounds__(kBlock) void k_volume_out(int64_t n, const double *__restrict__ vnsum,
                                                       const double4 *__restrict__ posV, double *nsum,
                                                       double *V) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    if (nsum) nsum[i] = vnsum[i];
    V[i] = posV[i].w;
}

template <typename T>
crk_status volume_moments(crk_ctx *c, const double4 *posH, const int64_t *goff, const int32_t *gidx,
                          int64_t n, Box box, double *nsum, double *V, T *rv, bool want_m, double *m0,
                          double *m1, double *m2, double *gm0, double *gm1, double *gm2) {
    const int Gv = c->G_vol, Gm = c->G_mom, Pv = c->P_vol, Pm = c->P_mom;
    CRK_TRY(ensure(c, c->posV, (size_t)n * sizeof(double4)));
    double4 *posV = (double4 *)c->posV.p;
    if (sizeof(T) == 8 && c->vol_ready) {
        // the build's compaction summed these FP64 volumes with the lists
        KTimer kt_(c, "k_volume");
        k_volume_out<<<nblocks(n), kBlock, 0, c->stream>>>(n, (const double *)c->vnsum.p, posV, nsum, V);
    } else {
        KTimer kt_(c, "k_volume");
        if (Pv > 0) {
#define L_VOL(PP) k_volume_bal<T, PP><<<pblocks(n, PP), kBlock, 0, c->stream>>>(posH, goff, gidx, n, box, nsum, V, rv, posV)
            CRK_DISPATCH_P(Pv, L_VOL);
#undef L_VOL
        } else {
#define L_VOL(GG) k_volume<T, GG><<<gblocks(n, GG), kBlock, 0, c->stream>>>(posH, goff, gidx, n, box, nsum, V, rv, posV)
            CRK_DISPATCH_G(Gv, L_VOL);
#undef L_VOL
        }
    }
    if (want_m) {
        KTimer kt_(c, "k_moments");
        if (Pm > 0) {
#define L_MOM(PP) k_moments_bal<T, PP><<<pblocks(n, PP), kBlock, 0, c->stream>>>(posH, goff, gidx, posV, n, box, m0, m1, m2, gm0, gm1, gm2)
            CRK_DISPATCH_P(Pm, L_MOM);
#undef L_MOM
        } else {
#define L_MOM(GG) k_moments<T, GG><<<gblocks(n, GG), kBlock, 0, c->stream>>>(posH, goff, gidx, posV, n, box, m0, m1, m2, gm0, gm1, gm2)
            CRK_DISPATCH_G(Gm, L_MOM);
#undef L_MOM
        }
    }
    CRK_HIP(c, hipGetLastError());
    return CRK_OK;
}

bool valid_prec(int p) { return p == CRK_FP64 || p == CRK_MIXED || p == CRK_MIXED_ADAPT; }

}  // namespace
}  // namespace crk

using namespace crk;

extern "C" {

// lanes per particle for each pass (tuning hook; 0 leaves a pass unchanged)
crk_status crk_set_walk(crk_ctx *c, int32_t lanes, int32_t cap, int32_t level_shift) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (lanes != 0 && lanes != 1 && lanes != 2 && lanes != 4 && lanes != 8 && lanes != 16)
        return set_err(c, CRK_ERR_INVALID_ARG, "walk lanes must be 1, 2, 4, 8 or 16");
    if (cap < 0 || cap > 65536) return set_err(c, CRK_ERR_INVALID_ARG, "walk cap out of range");
    if (level_shift < -1 || level_shift > 3)
        return set_err(c, CRK_ERR_INVALID_ARG, "walk level shift must be -1 (keep) or 0..3");
    if (lanes) c->G_walk = lanes;
    if (cap) c->walk_cap = cap;
    if (level_shift >= 0) c->walk_shift = level_shift;
    return CRK_OK;
}

crk_status crk_set_wave_mapping(crk_ctx *c, int32_t vol_ppw, int32_t mom_ppw, int32_t grad_ppw,
                                int32_t deriv_ppw) {
    if (!c) return CRK_ERR_INVALID_ARG;
    for (int p : {vol_ppw, mom_ppw, grad_ppw, deriv_ppw})
        if (p != -1 && p != 0 && p != 4 && p != 8 && p != 16 && p != 32)
            return set_err(c, CRK_ERR_INVALID_ARG, "particles per wave must be -1, 0, 4, 8, 16 or 32");
    if (vol_ppw >= 0) c->P_vol = vol_ppw;
    if (mom_ppw >= 0) c->P_mom = mom_ppw;
    if (grad_ppw >= 0) c->P_grad = grad_ppw;
    if (deriv_ppw >= 0) c->P_der = deriv_ppw;
    return CRK_OK;
}

crk_status crk_set_lanes(crk_ctx *c, int32_t g_vol, int32_t g_mom, int32_t g_grad, int32_t g_der) {
    if (!c) return CRK_ERR_INVALID_ARG;
    int gs[4] = {g_vol, g_mom, g_grad, g_der};
    for (int g : gs)
        if (g != 0 && (g < 1 || g > 64 || (g & (g - 1))))
            return set_err(c, CRK_ERR_INVALID_ARG, "lanes per particle must be a power of two <= 64");
    if (g_vol) c->G_vol = g_vol;
    if (g_mom) c->G_mom = g_mom;
    if (g_grad) c->G_grad = g_grad;
    if (g_der) c->G_der = g_der;
    return CRK_OK;
}

crk_status crk_moments(crk_ctx *c, const crk_params *p, double *nsum, double *V, double *m0,
                       double *m1, double *m2, double *gm0, double *gm1, double *gm2) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (!p || !V) return set_err(c, CRK_ERR_INVALID_ARG, "crk_moments: NULL argument");
    if (!valid_prec(p->precision)) return set_err(c, CRK_ERR_INVALID_ARG, "bad precision");
    if (!c->built) return set_err(c, CRK_ERR_STATE, "crk_build_cells has not run");
    bool want_m = m0 || m1 || m2 || gm0 || gm1 || gm2;
    if (want_m && !(m0 && m1 && m2 && gm0 && gm1 && gm2))
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_moments: give all moment outputs or none");
    CRK_HIP(c, hipSetDevice(c->device));
    int64_t n = c->n;
    Box box{c->L, 1.0 / c->L};
    const double4 *posH = (const double4 *)c->posH.p;
    const int64_t *goff = (const int64_t *)c->goff.p;
    const int32_t *gidx = (const int32_t *)c->gidx.p;
    bool f32 = p->precision == CRK_MIXED;
    CRK_TRY(ensure(c, c->recV, (size_t)n * (f32 ? 4 : 8)));
    if (f32) {
        float *rv = (float *)c->recV.p;
        CRK_TRY(volume_moments<float>(c, posH, goff, gidx, n, box, nsum, V, rv, want_m, m0, m1, m2, gm0, gm1, gm2));
    } else {
        double *rv = (double *)c->recV.p;
        CRK_TRY(volume_moments<double>(c, posH, goff, gidx, n, box, nsum, V, rv, want_m, m0, m1, m2, gm0, gm1, gm2));
    }
    CRK_HIP(c, hipGetLastError());
    c->have_V = 1;
    c->prec_V = p->precision;
    return CRK_OK;
}

crk_status crk_corrections(crk_ctx *c, int64_t n, const double *m0, const double *m1,
                           const double *m2, const double *gm0, const double *gm1, const double *gm2,
                           double *A, double *B, double *gA, double *gB, int64_t *n_singular) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (n < 1 || !m0 || !m1 || !m2 || !gm0 || !gm1 || !gm2 || !A || !B || !gA || !gB)
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_corrections: n < 1 or NULL argument");
    CRK_HIP(c, hipSetDevice(c->device));
    CRK_TRY(ensure(c, c->misc, 256));
    unsigned long long *cnt = (unsigned long long *)c->misc.p + 4;
    CRK_TRY(zero_async(c, cnt, 2));
    {
        KTimer kt_(c, "k_corrections");
        k_corrections<<<nblocks(n), kBlock, 0, c->stream>>>(n, m0, m1, m2, gm0, gm1, gm2, A, B, gA, gB, cnt);
    }
    CRK_HIP(c, hipGetLastError());
    if (n_singular) {
        unsigned long long *pin = (unsigned long long *)c->pinned.p + 8;
        CRK_HIP(c, hipMemcpyAsync(pin, cnt, sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
        CRK_HIP(c, hipStreamSynchronize(c->stream));
        *n_singular = (int64_t)pin[0];
        if (pin[0] > 0) return CRK_WARN_SINGULAR;
    }
    return CRK_OK;
}

// FP64 rows of the adaptive mode: flags the particles whose RK template is
// ill-conditioned (flist) and lists every particle with a flagged pair side
// (tlist), each list in no particular order. In graph mode the counts stay
// on the device.
struct AdaptRows {
    int32_t *flag = nullptr, *flist = nullptr, *tlist = nullptr;
    int64_t nflag = 0, ntouch = 0;
    const int64_t *nflag_dev = nullptr, *ntouch_dev = nullptr;
};

// fpos[n] counts the flagged rows (appended in any order: their fix is per
// row), the int32 words below it mark the touched rows, whose offsets tpos
// list them in ascending order (rows of neighbouring particles side by side
// share their partners' loads in the fix). First the buffers, the cleared
// marks and counter; the flagging follows (k_flag, or the record packing of
// the derivative call), then adapt_finish.
static crk_status adapt_prep(crk_ctx *c, AdaptRows &r) {
    const int64_t n = c->n;
    CRK_TRY(ensure(c, c->flag, (size_t)n * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->flist, (size_t)n * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->tlist, (size_t)n * sizeof(int32_t)));
    CRK_TRY(ensure(c, c->fpos, (size_t)(n + 1) * sizeof(int64_t)));
    CRK_TRY(ensure(c, c->tpos, (size_t)(n + 1) * sizeof(int64_t)));
    r.flag = (int32_t *)c->flag.p;
    r.flist = (int32_t *)c->flist.p;
    r.tlist = (int32_t *)c->tlist.p;
    int64_t *fpos = (int64_t *)c->fpos.p;
    k_zero_marks<<<nblocks(n), kBlock, 0, c->stream>>>((int32_t *)fpos, n, fpos + n);
    CRK_HIP(c, hipGetLastError());
    return CRK_OK;
}

// the flagged rows' partners marked and listed, and the counts
static crk_status adapt_finish(crk_ctx *c, bool gm, AdaptRows &r) {
    const int64_t n = c->n;
    const int64_t *goff = (const int64_t *)c->goff.p;
    const int32_t *gidx = (const int32_t *)c->gidx.p;
    const int32_t *eb = (const int32_t *)c->eb.p, *ee = (const int32_t *)c->ee.p,
                  *eidx = (const int32_t *)c->eidx.p;
    int64_t *fpos = (int64_t *)c->fpos.p, *tpos = (int64_t *)c->tpos.p;
    {
        KTimer kt_(c, "k_flag");
        int32_t *mark = (int32_t *)fpos;
        k_mark<<<(unsigned)std::min<int64_t>(nblocks(n * 16), 1024), kBlock, 0, c->stream>>>(
            r.flist, fpos + n, goff, gidx, eb, ee, eidx, mark);
        CRK_TRY(scan_counts2(c, mark, nullptr, n, tpos, nullptr));
        k_compact<<<nblocks(n), kBlock, 0, c->stream>>>(n, tpos, r.tlist);
    }
    CRK_HIP(c, hipGetLastError());
    if (gm) {
        // row counts stay on the device; the fix launches loop over them
        r.nflag_dev = fpos + n;
        r.ntouch_dev = tpos + n;
        r.nflag = r.ntouch = n;
        c->last_nflag = c->last_ntouch = -1;
    } else {
        int64_t *pin = (int64_t *)c->pinned.p + 40;
        CRK_HIP(c, hipMemcpyAsync(pin, fpos + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
        CRK_HIP(c, hipMemcpyAsync(pin + 1, tpos + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
        CRK_HIP(c, hipStreamSynchronize(c->stream));
        r.nflag = pin[0];
        r.ntouch = pin[1];
        c->last_nflag = r.nflag;
        c->last_ntouch = r.ntouch;
    }
    return CRK_OK;
}

// FP64 rows from the corrections given (k_flag), then adapt_finish
static crk_status adapt_rows(crk_ctx *c, const crk_params *p, const double *A, const double *B,
                             const double *gA, const double *gB, bool gm, AdaptRows &r) {
    const int64_t n = c->n;
    CRK_TRY(adapt_prep(c, r));
    {
        KTimer kt_(c, "k_flag");
        k_flag<<<nblocks(n), kBlock, 0, c->stream>>>(n, (const double4 *)c->posH.p, A, B, gA, gB,
                                                     p->kappa_max, r.flag, r.flist,
                                                     (unsigned long long *)((int64_t *)c->fpos.p + n));
    }
    CRK_HIP(c, hipGetLastError());
    return adapt_finish(c, gm, r);
}

crk_status crk_derivatives(crk_ctx *c, const crk_params *p, const double *v, const double *m,
                           const double *u, const double *rho, const double *V, const double *A,
                           const double *B, const double *gA, const double *gB, double *gradv,
                           double *dpdt, double *dudt) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (!p || !v || !m || !u || !V || !A || !B || !gA || !gB || !gradv || !dpdt || !dudt)
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_derivatives: NULL argument");
    if (!valid_prec(p->precision)) return set_err(c, CRK_ERR_INVALID_ARG, "bad precision");
    if (!(p->a > 0.0) || !(p->nh > 0.0) || !(p->eta_fold > 0.0) || !(p->gamma > 1.0))
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_derivatives: bad parameter");
    if (!c->built) return set_err(c, CRK_ERR_STATE, "crk_build_cells has not run");
    CRK_HIP(c, hipSetDevice(c->device));
    int64_t n = c->n;
    // time-step terms (crk_set_timestep): per-particle maxima kept for crk_timestep
    const bool ts = c->ts_on != 0;
    double *tvs = nullptr, *tqr = nullptr;
    if (ts) {
        CRK_TRY(ensure(c, c->ts_vs, (size_t)n * sizeof(double)));
        CRK_TRY(ensure(c, c->ts_qr, (size_t)n * sizeof(double)));
        tvs = (double *)c->ts_vs.p;
        tqr = (double *)c->ts_qr.p;
    }
    c->ts_valid = 0;
    Box box{c->L, 1.0 / c->L};
    const double4 *posH = (const double4 *)c->posH.p;
    const int64_t *goff = (const int64_t *)c->goff.p;
    const int32_t *gidx = (const int32_t *)c->gidx.p;
    const int32_t *eb = (const int32_t *)c->eb.p, *ee = (const int32_t *)c->ee.p,
                  *eidx = (const int32_t *)c->eidx.p;
    const bool f32 = p->precision != CRK_FP64;
    const bool adapt = p->precision == CRK_MIXED_ADAPT;
    const DerivPrm dp = deriv_prm(p);
    CRK_TRY(ensure(c, c->misc, 256));
    int *bad = (int *)c->misc.p + 2;
    CRK_TRY(zero_async(c, bad, 1));
    int Gg = c->G_grad, Gd = c->G_der, Pd = c->P_der, Pg = c->P_grad;

    // adaptive mode: FP64 rows for ill-conditioned RK templates, flagged by
    // the record packing (which reads the corrections anyway) after the FP32
    // velocity gradient has summed every row; the flagged rows' gradients
    // are then redone in FP64, and the FP32 passes never read the grad v
    // part of a flagged particle's record (its pairs are left to FP64)
    const bool gm = c->graph_mode != 0;
    AdaptRows ar;
    if (adapt) CRK_TRY(adapt_prep(c, ar));

    if (f32) {
        CRK_TRY(ensure(c, c->rec6, (size_t)n * 2 * sizeof(float4)));
        CRK_TRY(ensure(c, c->rec7, (size_t)n * kRec * sizeof(float4)));
        float4 *r6 = (float4 *)c->rec6.p, *r7 = (float4 *)c->rec7.p;
        double4 *r6d = nullptr, *aux = nullptr;
        if (adapt) {
            CRK_TRY(ensure(c, c->rec6d, (size_t)n * sizeof(double4)));
            CRK_TRY(ensure(c, c->aux, (size_t)n * sizeof(double4)));
            r6d = (double4 *)c->rec6d.p;
            aux = (double4 *)c->aux.p;
        }
        {
            KTimer kt_(c, "k_pack");
            k_pack6_f<<<nblocks(n), kBlock, 0, c->stream>>>(n, v, V, posH, dp.qinv, r6);
            if (adapt) k_pack6_d<<<nblocks(n), kBlock, 0, c->stream>>>(n, v, V, r6d);
        }
        {
            KTimer kt_(c, "k_gradv");
            if (Pg > 0) {
#define L_GV(PP) k_gradv_bal<float, PP><<<pblocks(n, PP), kBlock, 0, c->stream>>>(posH, goff, gidx, r6, A, B, gA, gB, n, box, nullptr, gradv)
                CRK_DISPATCH_P(Pg, L_GV);
#undef L_GV
            } else {
#define L_GV(GG) k_gradv<float, GG><<<gblocks(n, GG), kBlock, 0, c->stream>>>(posH, goff, gidx, r6, A, B, gA, gB, n, box, nullptr, 0, nullptr, nullptr, gradv)
                CRK_DISPATCH_G(Gg, L_GV);
#undef L_GV
            }
        }
        {
            KTimer kt_(c, "k_pack");
            if (adapt)
                k_pack8<float4, float><<<nblocks(n), kBlock, 0, c->stream>>>(
                    n, posH, v, m, u, rho, V, A, B, gA, gB, gradv, dp, nullptr, r7, aux, bad, p->kappa_max,
                    ar.flag, ar.flist, (unsigned long long *)((int64_t *)c->fpos.p + n));
            else
                k_pack8<float4, float><<<nblocks(n), kBlock, 0, c->stream>>>(
                    n, posH, v, m, u, rho, V, A, B, gA, gB, gradv, dp, nullptr, r7, aux, bad, 0.0, nullptr,
                    nullptr, nullptr);
        }
        if (adapt) CRK_TRY(adapt_finish(c, gm, ar));
        int32_t *flag = ar.flag, *flist = ar.flist, *tlist = ar.tlist;
        const int64_t nflag = ar.nflag, ntouch = ar.ntouch;
        const int64_t *nflag_dev = ar.nflag_dev, *ntouch_dev = ar.ntouch_dev;
        if (adapt && nflag > 0) {
#define L_GV(GG) k_gradv<double, GG><<<fix_blocks(nflag, GG, gm), kBlock, 0, c->stream>>>(posH, goff, gidx, r6d, A, B, gA, gB, n, box, flist, nflag, nflag_dev, nullptr, gradv)
            KTimer kt_(c, "k_gradv_fix");
            CRK_DISPATCH_G(Gg, L_GV);
#undef L_GV
        }
        {
            KTimer kt_(c, "k_deriv");
            if (Pd > 0) {
#define L_DER(PP) if (ts) k_deriv_bal<float, PP, true><<<pblocks(n, PP), kBlock, 0, c->stream>>>(posH, goff, gidx, eb, ee, eidx, r7, m, n, box, dp, dpdt, dudt, tvs, tqr); else k_deriv_bal<float, PP, false><<<pblocks(n, PP), kBlock, 0, c->stream>>>(posH, goff, gidx, eb, ee, eidx, r7, m, n, box, dp, dpdt, dudt)
                CRK_DISPATCH_P(Pd, L_DER);
#undef L_DER
            } else {
#define L_DER(GG) if (ts) k_deriv<float, GG, true><<<gblocks(n, GG), kBlock, 0, c->stream>>>(posH, goff, gidx, eb, ee, eidx, r7, m, n, box, dp, dpdt, dudt, tvs, tqr); else k_deriv<float, GG><<<gblocks(n, GG), kBlock, 0, c->stream>>>(posH, goff, gidx, eb, ee, eidx, r7, m, n, box, dp, dpdt, dudt)
                CRK_DISPATCH_G(Gd, L_DER);
#undef L_DER
            }
        }
        if (adapt && ntouch > 0) {
            Soa s{v, V, A, B, gA, gB, gradv, aux};
#define L_FIX(GG) if (ts) k_deriv_fix<GG, true><<<fix_blocks(ntouch, GG, gm), kBlock, 0, c->stream>>>(posH, goff, gidx, eb, ee, eidx, s, flag, tlist, ntouch, ntouch_dev, m, n, box, dp, dpdt, dudt, tvs, tqr); else k_deriv_fix<GG><<<fix_blocks(ntouch, GG, gm), kBlock, 0, c->stream>>>(posH, goff, gidx, eb, ee, eidx, s, flag, tlist, ntouch, ntouch_dev, m, n, box, dp, dpdt, dudt)
            KTimer kt_(c, "k_deriv_fix");
            CRK_DISPATCH_G(Gd, L_FIX);
#undef L_FIX
        }
    } else {
        CRK_TRY(ensure(c, c->rec6, (size_t)n * sizeof(double4)));
        CRK_TRY(ensure(c, c->rec7, (size_t)n * kRec * sizeof(double4)));
        double4 *r6 = (double4 *)c->rec6.p, *r7 = (double4 *)c->rec7.p;
        {
            KTimer kt_(c, "k_pack");
            k_pack6_d<<<nblocks(n), kBlock, 0, c->stream>>>(n, v, V, r6);
        }
        {
            KTimer kt_(c, "k_gradv");
            if (Pg > 0) {
#define L_GV(PP) k_gradv_bal<double, PP><<<pblocks(n, PP), kBlock, 0, c->stream>>>(posH, goff, gidx, r6, A, B, gA, gB, n, box, nullptr, gradv)
                CRK_DISPATCH_P(Pg, L_GV);
#undef L_GV
            } else {
#define L_GV(GG) k_gradv<double, GG><<<gblocks(n, GG), kBlock, 0, c->stream>>>(posH, goff, gidx, r6, A, B, gA, gB, n, box, nullptr, 0, nullptr, nullptr, gradv)
                CRK_DISPATCH_G(Gg, L_GV);
#undef L_GV
            }
        }
        {
            KTimer kt_(c, "k_pack");
            k_pack8<double4, double><<<nblocks(n), kBlock, 0, c->stream>>>(n, posH, v, m, u, rho, V, A, B, gA, gB, gradv, dp, nullptr, r7, nullptr, bad, 0.0, nullptr, nullptr, nullptr);
        }
        {
            KTimer kt_(c, "k_deriv");
            if (Pd > 0) {
#define L_DER(PP) if (ts) k_deriv_bal<double, PP, true><<<pblocks(n, PP), kBlock, 0, c->stream>>>(posH, goff, gidx, eb, ee, eidx, r7, m, n, box, dp, dpdt, dudt, tvs, tqr); else k_deriv_bal<double, PP, false><<<pblocks(n, PP), kBlock, 0, c->stream>>>(posH, goff, gidx, eb, ee, eidx, r7, m, n, box, dp, dpdt, dudt)
                CRK_DISPATCH_P(Pd, L_DER);
#undef L_DER
            } else {
#define L_DER(GG) if (ts) k_deriv<double, GG, true><<<gblocks(n, GG), kBlock, 0, c->stream>>>(posH, goff, gidx, eb, ee, eidx, r7, m, n, box, dp, dpdt, dudt, tvs, tqr); else k_deriv<double, GG><<<gblocks(n, GG), kBlock, 0, c->stream>>>(posH, goff, gidx, eb, ee, eidx, r7, m, n, box, dp, dpdt, dudt)
                CRK_DISPATCH_G(Gd, L_DER);
#undef L_DER
            }
        }
    }
    CRK_HIP(c, hipGetLastError());
    c->ts_valid = ts;
    if (gm) return CRK_OK;   // the graph's status kernel reads `bad`
    int *pin = (int *)c->pinned.p + 32;
    CRK_HIP(c, hipMemcpyAsync(pin, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    CRK_HIP(c, hipStreamSynchronize(c->stream));
    if (pin[0]) return set_err(c, CRK_ERR_NONFINITE, "non-finite or non-positive gas state");
    return CRK_OK;
}

crk_status crk_set_timestep(crk_ctx *c, int32_t on) {
    if (!c) return CRK_ERR_INVALID_ARG;
    c->ts_on = on != 0;
    return CRK_OK;
}

crk_status crk_timestep(crk_ctx *c, const crk_params *p, const double *u, const double *m,
                        const double *rho, const double *V, const double *gradv, double zeta,
                        double c_cfl, double *vsig, double *csq, double *vmax, double *dt_hyd) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (!p || !u || !m || !V || !gradv || !vmax)
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_timestep: NULL argument");
    if (!(zeta >= 0.0) || !(c_cfl > 0.0) || !(p->a > 0.0) || !(p->nh > 0.0) || !(p->gamma > 1.0))
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_timestep: bad parameter");
    if (!c->ts_valid)
        return set_err(c, CRK_ERR_STATE, "crk_timestep needs a crk_derivatives call made with crk_set_timestep on");
    CRK_HIP(c, hipSetDevice(c->device));
    k_timestep<<<nblocks(c->n), kBlock, 0, c->stream>>>(
        c->n, (const double4 *)c->posH.p, u, m, rho, V, gradv, (const double *)c->ts_vs.p,
        (const double *)c->ts_qr.p, p->gamma, 1.0 / p->nh, p->a, p->adot, zeta, c_cfl, vsig, csq, vmax,
        dt_hyd);
    CRK_HIP(c, hipGetLastError());
    return CRK_OK;
}

}  // extern "C"

crk_status crk::compat_pass(crk_ctx *c, const crk_params *p, const double *v, const double *m,
                            const double *u, const double *rho, const double *V, const double *A,
                            const double *B, const double *gA, const double *gB,
                            const double *gradv, const double *dpdt, const double *pk,
                            const double *pk2, double dt, double *du, double *du2, bool reuse) {
    if (!c) return CRK_ERR_INVALID_ARG;
    const bool two = du2 != nullptr;
    if (!p || !v || !m || !u || !V || !A || !B || !gA || !gB || !gradv || !dpdt || !du)
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_compatible_energy: NULL argument");
    if (!valid_prec(p->precision)) return set_err(c, CRK_ERR_INVALID_ARG, "bad precision");
    if (!(p->a > 0.0) || !(p->nh > 0.0) || !(p->eta_fold > 0.0) || !(p->gamma > 1.0) ||
        !isfinite(dt) || !isfinite(p->adot))
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_compatible_energy: bad parameter");
    if (!c->built) return set_err(c, CRK_ERR_STATE, "crk_build_cells has not run");
    if (c->capturing) return set_err(c, CRK_ERR_STATE, "crk_compatible_energy is not recorded in a graph");
    CRK_HIP(c, hipSetDevice(c->device));
    const int64_t n = c->n;
    Box box{c->L, 1.0 / c->L};
    const double4 *posH = (const double4 *)c->posH.p;
    const int64_t *goff = (const int64_t *)c->goff.p;
    const int32_t *gidx = (const int32_t *)c->gidx.p;
    const int32_t *eb = (const int32_t *)c->eb.p, *ee = (const int32_t *)c->ee.p,
                  *eidx = (const int32_t *)c->eidx.p;
    const bool f32 = p->precision != CRK_FP64;
    const bool adapt = p->precision == CRK_MIXED_ADAPT;
    const DerivPrm dp = deriv_prm(p);
    const double a4 = p->a * p->a * p->a * p->a;
    const double scale = dt / (2.0 * a4);
    const double cool = dt * (p->adot / p->a) * (3.0 * (p->gamma - 1.0) + 2.0);
    CRK_TRY(ensure(c, c->misc, 256));
    int *bad = (int *)c->misc.p + 2;
    CRK_TRY(zero_async(c, bad, 1));
    const int Gd = c->G_der, Pd = c->P_der > 0 ? c->P_der : 8;
    AdaptRows ar;
    // the records, FP64-row flags and lists of the derivative call just made
    // on this same state are reused when the caller says so (eager only)
    const bool keep = reuse && c->last_ntouch >= 0 && !c->graph_mode;
    if (adapt) {
        if (keep) {
            ar.flag = (int32_t *)c->flag.p;
            ar.tlist = (int32_t *)c->tlist.p;
            ar.ntouch = c->last_ntouch;
        } else {
            CRK_TRY(adapt_rows(c, p, A, B, gA, gB, false, ar));
        }
    }
    if (f32) {
        CRK_TRY(ensure(c, c->rec7, (size_t)n * kRec * sizeof(float4)));
        CRK_TRY(ensure(c, c->ce, (size_t)n * sizeof(float4) * (two ? 2 : 1)));
        float4 *r7 = (float4 *)c->rec7.p, *ce = (float4 *)c->ce.p;
        float4 *ce2 = two ? ce + n : nullptr;
        double4 *aux = nullptr, *ced = nullptr, *ced2 = nullptr;
        if (adapt) {
            CRK_TRY(ensure(c, c->aux, (size_t)n * sizeof(double4)));
            CRK_TRY(ensure(c, c->ced, (size_t)n * sizeof(double4) * (two ? 2 : 1)));
            aux = (double4 *)c->aux.p;
            ced = (double4 *)c->ced.p;
            ced2 = two ? ced + n : nullptr;
        }
        {
            KTimer kt_(c, "k_pack");
            if (!keep) k_pack8<float4, float><<<nblocks(n), kBlock, 0, c->stream>>>(n, posH, v, m, u, rho, V, A, B, gA, gB, gradv, dp, ar.flag, r7, aux, bad, 0.0, nullptr, nullptr, nullptr);
            k_pack_ce<float4, float><<<nblocks(n), kBlock, 0, c->stream>>>(n, v, pk, dpdt, m, u, rho, V, p->gamma, p->a, dt, ce, ced);
            if (two) k_pack_ce<float4, float><<<nblocks(n), kBlock, 0, c->stream>>>(n, v, pk2, dpdt, m, u, rho, V, p->gamma, p->a, dt, ce2, ced2);
        }
#define L_CE(PP) if (two) k_compat_bal<float, PP, 2><<<pblocks(n, PP), kBlock, 0, c->stream>>>(posH, goff, gidx, eb, ee, eidx, r7, ce, ce2, m, u, n, box, dp, scale, cool, du, du2); else k_compat_bal<float, PP, 1><<<pblocks(n, PP), kBlock, 0, c->stream>>>(posH, goff, gidx, eb, ee, eidx, r7, ce, nullptr, m, u, n, box, dp, scale, cool, du, nullptr)
        {
            KTimer kt_(c, "k_compat");
            CRK_DISPATCH_P(Pd, L_CE);
        }
#undef L_CE
        if (adapt && ar.ntouch > 0) {
            Soa s{v, V, A, B, gA, gB, gradv, aux};
#define L_CEF(GG) if (two) k_compat_fix<GG, 2><<<fix_blocks(ar.ntouch, GG, false), kBlock, 0, c->stream>>>(posH, goff, gidx, eb, ee, eidx, s, ced, ced2, ar.flag, ar.tlist, ar.ntouch, m, n, box, dp, scale, du, du2); else k_compat_fix<GG, 1><<<fix_blocks(ar.ntouch, GG, false), kBlock, 0, c->stream>>>(posH, goff, gidx, eb, ee, eidx, s, ced, nullptr, ar.flag, ar.tlist, ar.ntouch, m, n, box, dp, scale, du, nullptr)
            KTimer kt_(c, "k_compat_fix");
            CRK_DISPATCH_G(Gd, L_CEF);
#undef L_CEF
        }
    } else {
        CRK_TRY(ensure(c, c->rec7, (size_t)n * kRec * sizeof(double4)));
        CRK_TRY(ensure(c, c->ce, (size_t)n * sizeof(double4) * (two ? 2 : 1)));
        double4 *r7 = (double4 *)c->rec7.p, *ce = (double4 *)c->ce.p;
        double4 *ce2 = two ? ce + n : nullptr;
        {
            KTimer kt_(c, "k_pack");
            if (!keep) k_pack8<double4, double><<<nblocks(n), kBlock, 0, c->stream>>>(n, posH, v, m, u, rho, V, A, B, gA, gB, gradv, dp, nullptr, r7, nullptr, bad, 0.0, nullptr, nullptr, nullptr);
            k_pack_ce<double4, double><<<nblocks(n), kBlock, 0, c->stream>>>(n, v, pk, dpdt, m, u, rho, V, p->gamma, p->a, dt, ce, nullptr);
            if (two) k_pack_ce<double4, double><<<nblocks(n), kBlock, 0, c->stream>>>(n, v, pk2, dpdt, m, u, rho, V, p->gamma, p->a, dt, ce2, nullptr);
        }
#define L_CE(PP) if (two) k_compat_bal<double, PP, 2><<<pblocks(n, PP), kBlock, 0, c->stream>>>(posH, goff, gidx, eb, ee, eidx, r7, ce, ce2, m, u, n, box, dp, scale, cool, du, du2); else k_compat_bal<double, PP, 1><<<pblocks(n, PP), kBlock, 0, c->stream>>>(posH, goff, gidx, eb, ee, eidx, r7, ce, nullptr, m, u, n, box, dp, scale, cool, du, nullptr)
        {
            KTimer kt_(c, "k_compat");
            CRK_DISPATCH_P(Pd, L_CE);
        }
#undef L_CE
    }
    CRK_HIP(c, hipGetLastError());
    int *pin = (int *)c->pinned.p + 32;
    CRK_HIP(c, hipMemcpyAsync(pin, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    CRK_HIP(c, hipStreamSynchronize(c->stream));
    if (pin[0]) return set_err(c, CRK_ERR_NONFINITE, "non-finite or non-positive gas state");
    return CRK_OK;
}

extern "C" {

crk_status crk_compatible_energy(crk_ctx *c, const crk_params *p, const double *v, const double *m,
                                 const double *u, const double *rho, const double *V,
                                 const double *A, const double *B, const double *gA,
                                 const double *gB, const double *gradv, const double *dpdt,
                                 const double *pk, double dt, double *du) {
    return crk::compat_pass(c, p, v, m, u, rho, V, A, B, gA, gB, gradv, dpdt, pk, nullptr, dt, du,
                            nullptr, false);
}

crk_status crk_adaptive_rows(crk_ctx *c, int64_t *n_fp64_rows, int64_t *n_touched_rows) {
    if (!c || !n_fp64_rows || !n_touched_rows) return CRK_ERR_INVALID_ARG;
    *n_fp64_rows = c->last_nflag;
    *n_touched_rows = c->last_ntouch;
    return CRK_OK;
}

}  // extern "C"
