// S9: the smoothing-length network (not in the paper): an 8 -> 64 -> 64 -> 1
// MLP with exact-erf GELU, FP32, whose output ln(H_conv / H_prev) seeds the
// iteration of eqs. (hi), (thacker). Features, inference, training (forward,
// backward, Adam) are all kernels here.
//
// Parameter vector (4801 floats): W1 [64][8], b1 [64], W2 [64][64], b2 [64],
// w3 [64], b3. Every kernel stages it in LDS (19 KB) and reads it with
// wave-wide broadcasts; one thread evaluates one sample. The batch gradient
// is reduced deterministically: per-block partial sums in a fixed sample
// order, then a fixed-order sum over blocks (no float atomics).
#include <math.h>

#include "crk_internal.h"

namespace crk {
namespace {

constexpr int kIn = 8, kHid = 64;
constexpr int oW1 = 0, ob1 = oW1 + kHid * kIn, oW2 = ob1 + kHid, ob2 = oW2 + kHid * kHid,
              ow3 = ob2 + kHid, ob3 = ow3 + kHid, kNP = ob3 + 1;   // kNP = 4801
constexpr int kGradBlock = 64;                                      // samples per gradient block
constexpr int kAdamLanes = 8;                                       // lanes summing one parameter's partials

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * __expf(-0.5f * x * x);
}

__device__ __forceinline__ void load_theta(const float *__restrict__ th, float *s) {
    for (int e = threadIdx.x; e < kNP; e += blockDim.x) s[e] = th[e];
    __syncthreads();
}

// forward of one sample; keeps z1, a1, z2 when asked
template <bool KEEP>
__device__ __forceinline__ float mlp_forward(const float *__restrict__ s, const float f[kIn], float *z1k,
                                             float *a1k, float *z2k) {
    float a1[kHid];
#pragma unroll
    for (int j = 0; j < kHid; j++) {
        float z = s[ob1 + j];
#pragma unroll
        for (int q = 0; q < kIn; q++) z += s[oW1 + j * kIn + q] * f[q];
        if (KEEP) z1k[j] = z;
        a1[j] = gelu(z);
        if (KEEP) a1k[j] = a1[j];
    }
    float y = s[ob3];
    for (int k = 0; k < kHid; k++) {
        float z = s[ob2 + k];
#pragma unroll
        for (int j = 0; j < kHid; j++) z += s[oW2 + k * kHid + j] * a1[j];
        if (KEEP) z2k[k] = z;
        y += s[ow3 + k] * gelu(z);
    }
    return y;
}

__global__ __launch_bounds__(kBlock) void k_hnet_fwd(const float *__restrict__ theta,
                                                     const float *__restrict__ feat, int64_t nb,
                                                     float *y) {
    __shared__ float s[kNP];
    load_theta(theta, s);
    int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (b >= nb) return;
    float f[kIn];
#pragma unroll
    for (int q = 0; q < kIn; q++) f[q] = feat[q * nb + b];
    y[b] = mlp_forward<false>(s, f, nullptr, nullptr, nullptr);
}

// One block = kGradBlock samples. Phase 1: each thread runs its sample
// forward and backward (dL/dy = 2 (y - t) / B) and parks the per-sample
// factors in LDS. Phase 2: the block's threads sum the outer products of
// those factors over the block's samples in sample order and write one
// partial gradient row per block.
__global__ __launch_bounds__(kGradBlock) void k_hnet_grad(const float *__restrict__ theta,
                                                          const float *__restrict__ feat,
                                                          const float *__restrict__ target, int64_t nb,
                                                          float inv_b, float *partial, float *ploss) {
    __shared__ float s[kNP];
    __shared__ float sf[kGradBlock][kIn];
    __shared__ float sa1[kGradBlock][kHid + 1];
    __shared__ float sa2[kGradBlock][kHid + 1];
    __shared__ float sdz1[kGradBlock][kHid + 1];
    __shared__ float sdz2[kGradBlock][kHid + 1];
    __shared__ float sdy[kGradBlock];
    __shared__ float sl[kGradBlock];
    load_theta(theta, s);
    const int t = threadIdx.x;
    const int64_t b = (int64_t)blockIdx.x * kGradBlock + t;
    // z1 and z2 are parked in this sample's LDS rows of dz1 and dz2 (each is
    // overwritten by its gradient once read), so no per-thread array is
    // indexed at run time
    float f[kIn];
    bool act = b < nb;
#pragma unroll
    for (int q = 0; q < kIn; q++) f[q] = act ? feat[q * nb + b] : 0.0f;
    float y = mlp_forward<true>(s, f, sdz1[t], sa1[t], sdz2[t]);
    float r = act ? (y - target[b]) : 0.0f;
    float dy = 2.0f * r * inv_b;
    sl[t] = r * r;
    sdy[t] = dy;
#pragma unroll
    for (int q = 0; q < kIn; q++) sf[t][q] = f[q];
    float dz2[kHid];
#pragma unroll
    for (int k = 0; k < kHid; k++) {
        const float z2 = sdz2[t][k];
        dz2[k] = dy * s[ow3 + k] * gelu_d(z2);
        sdz2[t][k] = dz2[k];
        sa2[t][k] = gelu(z2);
    }
    for (int j = 0; j < kHid; j++) {
        float da = 0.0f;
#pragma unroll
        for (int k = 0; k < kHid; k++) da += s[oW2 + k * kHid + j] * dz2[k];
        sdz1[t][j] = da * gelu_d(sdz1[t][j]);
    }
    __syncthreads();
    float *out = partial + (int64_t)blockIdx.x * kNP;
    // dW2: each thread an 8 x 8 tile of rows k0.. and columns j0.., summed
    // over the samples in order (the same order as every other entry)
    static_assert(kGradBlock == 64 && kHid == 64, "one 8 x 8 tile of dW2 per thread");
    {
        const int k0 = (t / 8) * 8, j0 = (t % 8) * 8;
        float acc[8][8];
#pragma unroll
        for (int a = 0; a < 8; a++)
#pragma unroll
            for (int c = 0; c < 8; c++) acc[a][c] = 0.0f;
        for (int u = 0; u < kGradBlock; u++) {
            float dk[8], aj[8];
#pragma unroll
            for (int a = 0; a < 8; a++) {
                dk[a] = sdz2[u][k0 + a];
                aj[a] = sa1[u][j0 + a];
            }
#pragma unroll
            for (int a = 0; a < 8; a++)
#pragma unroll
                for (int c = 0; c < 8; c++) acc[a][c] += dk[a] * aj[c];
        }
#pragma unroll
        for (int a = 0; a < 8; a++)
#pragma unroll
            for (int c = 0; c < 8; c++) out[oW2 + (k0 + a) * kHid + j0 + c] = acc[a][c];
    }
    for (int e = t; e < kNP; e += kGradBlock) {
        if (e >= oW2 && e < ob2) continue;   // the tiles above
        float acc = 0.0f;
        if (e < ob1) {
            int j = e / kIn, q = e % kIn;
            for (int u = 0; u < kGradBlock; u++) acc += sdz1[u][j] * sf[u][q];
        } else if (e < oW2) {
            int j = e - ob1;
            for (int u = 0; u < kGradBlock; u++) acc += sdz1[u][j];
        } else if (e < ow3) {
            int k = e - ob2;
            for (int u = 0; u < kGradBlock; u++) acc += sdz2[u][k];
        } else if (e < ob3) {
            int k = e - ow3;
            for (int u = 0; u < kGradBlock; u++) acc += sdy[u] * sa2[u][k];
        } else {
            for (int u = 0; u < kGradBlock; u++) acc += sdy[u];
        }
        out[e] = acc;
    }
    if (t == 0) {
        float L = 0.0f;
        for (int u = 0; u < kGradBlock; u++) L += sl[u];
        ploss[blockIdx.x] = L;
    }
}

// fixed-order sum of the block partials (kAdamLanes lanes per parameter,
// lane c takes blocks c, c + kAdamLanes, ...; the lanes combine in a fixed
// butterfly), then one Adam step per parameter (bias-corrected, beta1 0.9,
// beta2 0.999, eps 1e-8)
__global__ __launch_bounds__(kBlock) void k_hnet_adam(const float *__restrict__ partial, int64_t nblk,
                                                      float *theta, float *m, float *v, float lr,
                                                      float bc1, float bc2, float *grad_out) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    const int e = t / kAdamLanes, c = t % kAdamLanes;
    if (e >= kNP) return;   // whole lane groups leave together
    float g = 0.0f;
    for (int64_t b = c; b < nblk; b += kAdamLanes) g += partial[b * kNP + e];
#pragma unroll
    for (int o = 1; o < kAdamLanes; o <<= 1) g += __shfl_xor(g, o, kAdamLanes);
    if (c != 0) return;
    if (grad_out) grad_out[e] = g;
    if (!theta) return;
    float mm = 0.9f * m[e] + 0.1f * g;
    float vv = 0.999f * v[e] + 0.001f * g * g;
    m[e] = mm;
    v[e] = vv;
    theta[e] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + 1e-8f);
}

__global__ void k_hnet_loss(const float *__restrict__ ploss, int64_t nblk, float inv_b, float *out) {
    if (threadIdx.x != 0) return;
    float L = 0.0f;
    for (int64_t b = 0; b < nblk; b++) L += ploss[b];
    out[0] = L * inv_b;
}

// Features at radius H (one walk over the support): kernel-weighted counts
// N_w(h) = (4 pi/3) h^3 sum W(r, h) at h = H, H/2, H/4 and raw counts within
// H and H/2 (self included), see crk.h for the eight definitions.
template <int G>
__global__ __launch_bounds__(kBlock) void k_hnet_features(const double4 *__restrict__ posH,
                                                          const int32_t *__restrict__ cbeg,
                                                          const int32_t *__restrict__ cend, Levels v,
                                                          int64_t n, const double *__restrict__ H,
                                                          double Nres, float *feat) {
    // G lanes per particle share a flattened walk of the support; the five
    // sums are combined across the group at the end
    const int64_t gid = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const int l = (int)(gid % G);
    const int64_t i = gid / G;
    if (i >= n) return;   // whole groups leave together
    const double4 pi = posH[i];
    const double h = H[i];
    double s1 = 0.0, s2 = 0.0, s4 = 0.0, c1 = 0.0, c2 = 0.0;
    const double h2 = h * h, ih = 1.0 / h;
    __shared__ int32_t s_b[kBlock / G][kRanges], s_c[kBlock / G][kRanges + 1], s_o[kBlock / G][kRanges];
    const int grp = threadIdx.x / G;
    flat_candidates<G>(posH, cbeg, cend, v, i, pi, h, l, s_b[grp], s_c[grp], s_o[grp],
                       [&](bool valid, double r2) {
        if (valid && r2 < h2) {
            double q = sqrt(r2) * ih;
            double w1 = 1.0 - q, w1_2 = w1 * w1;
            s1 += w1_2 * w1_2 * w1_2 * (1.0 + q * (6.0 + q * (35.0 / 3.0)));
            c1 += 1.0;
            if (r2 < 0.25 * h2) {
                double q2 = 2.0 * q, w2 = 1.0 - q2, w2_2 = w2 * w2;
                s2 += w2_2 * w2_2 * w2_2 * (1.0 + q2 * (6.0 + q2 * (35.0 / 3.0)));
                c2 += 1.0;
                if (r2 < 0.0625 * h2) {
                    double q4 = 4.0 * q, w4 = 1.0 - q4, w4_2 = w4 * w4;
                    s4 += w4_2 * w4_2 * w4_2 * (1.0 + q4 * (6.0 + q4 * (35.0 / 3.0)));
                }
            }
        }
        return false;
    });
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) {
        s1 += __shfl_xor(s1, m, G);
        s2 += __shfl_xor(s2, m, G);
        s4 += __shfl_xor(s4, m, G);
        c1 += __shfl_xor(c1, m, G);
        c2 += __shfl_xor(c2, m, G);
    }
    if (l != 0) return;
    // (4 pi/3) h^3 * kW h^-3 sum = (4 pi/3) kW sum, the same at every radius
    const double c = 4.0 / 3.0 * kPi * kW;
    double N1 = c * s1, N2 = c * s2, N4 = c * s4;
    feat[0 * n + i] = (float)log(N1 / Nres);
    feat[1 * n + i] = (float)(cbrt(Nres / N1) - 1.0);
    feat[2 * n + i] = (float)log(8.0 * N2 / Nres);
    feat[3 * n + i] = (float)log(64.0 * N4 / Nres);
    feat[4 * n + i] = (float)log(c1 / Nres);
    feat[5 * n + i] = (float)log(8.0 * c2 / Nres);
    feat[6 * n + i] = (float)log(h * cbrt((double)n) / v.L);
    feat[7 * n + i] = 1.0f;
}

// seed = H_prev exp(y), clamped to [H_prev / 8, 8 H_prev] and below L/2;
// a non-finite network output keeps H_prev
__global__ __launch_bounds__(kBlock) void k_hnet_seed(const double *__restrict__ Hprev,
                                                      const float *__restrict__ y, int64_t n,
                                                      double hmax, double *Hseed) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double h = Hprev[i];
    double o = (double)y[i];
    double s = isfinite(o) ? h * exp(o) : h;
    s = fmin(fmax(s, 0.125 * h), 8.0 * h);
    Hseed[i] = fmin(s, hmax);
}

__global__ __launch_bounds__(kBlock) void k_hnet_targets(const double *__restrict__ Hprev,
                                                         const double *__restrict__ Hconv, int64_t n,
                                                         float *t) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) t[i] = (float)log(Hconv[i] / Hprev[i]);
}

}  // namespace


}  // namespace crk

using namespace crk;

extern "C" {

crk_status crk_hnet_features(crk_ctx *c, double Nres, const double *H_sorted, float *feat) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (!H_sorted || !feat || !(Nres > 0.0)) return set_err(c, CRK_ERR_INVALID_ARG, "crk_hnet_features: bad argument");
    if (c->nc == 0) return set_err(c, CRK_ERR_STATE, "crk_build_cells has not run");
    CRK_HIP(c, hipSetDevice(c->device));
    int64_t n = c->n;
    {
        KTimer kt_(c, "k_hnet_features");
        constexpr int GF = 8;
        k_hnet_features<GF><<<(unsigned)((n * GF + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(
            (const double4 *)c->posH.p, (const int32_t *)c->cbeg.p, (const int32_t *)c->cend.p,
            levels(c), n, H_sorted, Nres, feat);
    }
    CRK_HIP(c, hipGetLastError());
    return CRK_OK;
}

crk_status crk_hnet_forward(crk_ctx *c, const float *theta, const float *feat, int64_t nb, float *y) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (!theta || !feat || !y || nb < 1) return set_err(c, CRK_ERR_INVALID_ARG, "crk_hnet_forward: bad argument");
    CRK_HIP(c, hipSetDevice(c->device));
    {
        KTimer kt_(c, "k_hnet_fwd");
        k_hnet_fwd<<<(unsigned)((nb + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(theta, feat, nb, y);
    }
    CRK_HIP(c, hipGetLastError());
    return CRK_OK;
}

crk_status crk_hnet_train_step(crk_ctx *c, float *theta, float *adam_m, float *adam_v, int64_t step,
                               float lr, const float *feat, const float *target, int64_t nb,
                               float *grad, float *loss) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (!feat || !target || nb < 1 || (theta && (!adam_m || !adam_v || step < 1)) || (!theta && !grad))
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_hnet_train_step: bad argument");
    CRK_HIP(c, hipSetDevice(c->device));
    int64_t nblk = (nb + kGradBlock - 1) / kGradBlock;
    CRK_TRY(ensure(c, c->hnet_part, (size_t)nblk * (kNP + 1) * sizeof(float) + 64));
    float *part = (float *)c->hnet_part.p;
    float *ploss = part + nblk * kNP;
    const float *th_in = theta;
    if (!theta) return set_err(c, CRK_ERR_INVALID_ARG, "theta is NULL");
    {
        KTimer kt_(c, "k_hnet_grad");
        k_hnet_grad<<<(unsigned)nblk, kGradBlock, 0, c->stream>>>(th_in, feat, target, nb, 1.0f / (float)nb,
                                                                   part, ploss);
    }
    float bc1 = 1.0f - powf(0.9f, (float)step), bc2 = 1.0f - powf(0.999f, (float)step);
    {
        KTimer kt_(c, "k_hnet_adam");
        k_hnet_adam<<<(kNP * kAdamLanes + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(
            part, nblk, lr > 0.0f ? theta : nullptr, adam_m, adam_v, lr, bc1, bc2, grad);
    }
    CRK_HIP(c, hipGetLastError());
    if (loss) {
        CRK_TRY(ensure(c, c->misc, 256));
        float *dl = (float *)c->misc.p + 48;
        k_hnet_loss<<<1, 64, 0, c->stream>>>(ploss, nblk, 1.0f / (float)nb, dl);
        float *pin = (float *)c->pinned.p + 256;
        CRK_HIP(c, hipMemcpyAsync(pin, dl, sizeof(float), hipMemcpyDeviceToHost, c->stream));
        CRK_HIP(c, hipStreamSynchronize(c->stream));
        *loss = pin[0];
    }
    return CRK_OK;
}

crk_status crk_hnet_targets(crk_ctx *c, int64_t n, const double *H_prev, const double *H_conv,
                            float *target) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (n < 1 || !H_prev || !H_conv || !target)
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_hnet_targets: bad argument");
    CRK_HIP(c, hipSetDevice(c->device));
    k_hnet_targets<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(H_prev, H_conv, n, target);
    CRK_HIP(c, hipGetLastError());
    return CRK_OK;
}

crk_status crk_hnet_seed(crk_ctx *c, const float *theta, double Nres, const double *H_prev, double *H_seed) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (!theta || !H_prev || !H_seed) return set_err(c, CRK_ERR_INVALID_ARG, "crk_hnet_seed: bad argument");
    if (c->nc == 0) return set_err(c, CRK_ERR_STATE, "crk_build_cells has not run");
    CRK_HIP(c, hipSetDevice(c->device));
    int64_t n = c->n;
    CRK_TRY(ensure(c, c->hnet_feat, (size_t)n * (kIn + 1) * sizeof(float)));
    float *feat = (float *)c->hnet_feat.p, *y = feat + (size_t)n * kIn;
    CRK_TRY(crk_hnet_features(c, Nres, H_prev, feat));
    CRK_TRY(crk_hnet_forward(c, theta, feat, n, y));
    k_hnet_seed<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(H_prev, y, n,
                                                                                  0.49 * c->L, H_seed);
    CRK_HIP(c, hipGetLastError());
    return CRK_OK;
}

}  // extern "C"
