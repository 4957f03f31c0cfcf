// S9: the smoothing-length network (not in the paper): an 8 -> 64 -> 64 -> 1
// MLP with exact-erf GELU, FP32, whose output ln(H_conv / H_prev) seeds the
// iteration of eqs. (hi), (thacker). Features, inference, training (forward,
// backward, Adam) are all kernels here.
//
// Parameter vector (4801 floats): W1 [64][8], b1 [64], W2 [64][64], b2 [64],
// w3 [64], b3. Every kernel stages it in LDS (19 KB). The dense products of
// the forward and backward passes run on the matrix cores (FP32 MFMA), 16
// samples per wavefront. The batch gradient is reduced deterministically:
// one partial row per 16-sample tile, then a fixed-order sum over the rows
// (no float atomics).
#include <math.h>

#include <mutex>

#include "crk_internal.h"

namespace crk {
namespace {

constexpr int kIn = 8, kHid = 64;
constexpr int oW1 = 0, ob1 = oW1 + kHid * kIn, oW2 = ob1 + kHid, ob2 = oW2 + kHid * kHid,
              ow3 = ob2 + kHid, ob3 = ow3 + kHid, kNP = ob3 + 1;   // kNP = 4801
constexpr int kAdamLanes = 32;                                      // lanes summing one parameter's partials

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * __expf(-0.5f * x * x);
}

__device__ __forceinline__ void load_theta(const float *__restrict__ th, float *s) {
    for (int e = threadIdx.x; e < kNP; e += blockDim.x) s[e] = th[e];
    __syncthreads();
}

// ---------------------------------------------------------------- matrix cores
// v_mfma_f32_16x16x4_f32: D[16x16] = A[16x4] B[4x16] + C with, for lane l,
// c = l % 16 and g = l / 16: A[c][g], B[g][c] and D[4g + r][c] (r = 0..3).
typedef float f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f4v mfma4(float a, float b, f4v c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Forward on the matrix cores, 16 samples (the columns) per wavefront step.
// Layer 1: Z1 = W1 F as four 16-row tiles over two k-steps. Layer 2: Z2 = W2
// A1, where the k-step (mt, r) takes the hidden units 16 mt + 4 g + r, i.e.
// the values each lane already holds in register r of tile mt (the sum over
// k runs in a permuted order, so no data moves between lanes); the matching
// W2 entries are per-lane constants. Output: each lane's share of w3.a2,
// then a sum over the four lane groups of a column.
__global__ __launch_bounds__(kBlock) void k_hnet_fwd(const float *__restrict__ theta,
                                                     const float *__restrict__ feat, int64_t nb,
                                                     float *y) {
    __shared__ float s[kNP];
    load_theta(theta, s);
    const int lane = threadIdx.x & 63;
    const int c = lane & 15, g = lane >> 4;
    float w1a[4][2], w2a[4][4][4], b1r[4][4], b2r[4][4], w3r[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
#pragma unroll
        for (int ks = 0; ks < 2; ks++) w1a[mt][ks] = s[oW1 + (16 * mt + c) * kIn + 4 * ks + g];
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int h = 16 * mt + 4 * g + r;   // the hidden unit of register r of tile mt
            b1r[mt][r] = s[ob1 + h];
            b2r[mt][r] = s[ob2 + h];
            w3r[mt][r] = s[ow3 + h];
#pragma unroll
            for (int m2 = 0; m2 < 4; m2++) w2a[m2][mt][r] = s[oW2 + (16 * m2 + c) * kHid + h];
        }
    }
    const float b3 = s[ob3];
    const int64_t wstep = (int64_t)gridDim.x * (kBlock / 64) * 16;
    for (int64_t t0 = ((int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) * 16; t0 < nb; t0 += wstep) {
        const int64_t smp = t0 + c;
        const bool act = smp < nb;
        f4v z1[4];
#pragma unroll
        for (int mt = 0; mt < 4; mt++) z1[mt] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < 2; ks++) {
            const float bf = act ? feat[(int64_t)(4 * ks + g) * nb + smp] : 0.0f;
#pragma unroll
            for (int mt = 0; mt < 4; mt++) z1[mt] = mfma4(w1a[mt][ks], bf, z1[mt]);
        }
        float a1[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; mt++)
#pragma unroll
            for (int r = 0; r < 4; r++) a1[mt][r] = gelu(z1[mt][r] + b1r[mt][r]);
        f4v z2[4];
#pragma unroll
        for (int m2 = 0; m2 < 4; m2++) z2[m2] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int mt = 0; mt < 4; mt++)
#pragma unroll
            for (int r = 0; r < 4; r++)
#pragma unroll
                for (int m2 = 0; m2 < 4; m2++) z2[m2] = mfma4(w2a[m2][mt][r], a1[mt][r], z2[m2]);
        float part = 0.0f;
#pragma unroll
        for (int m2 = 0; m2 < 4; m2++)
#pragma unroll
            for (int r = 0; r < 4; r++) part += w3r[m2][r] * gelu(z2[m2][r] + b2r[m2][r]);
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        if (g == 0 && act) y[smp] = part + b3;
    }
}

// Sum over the 16 lanes of a DPP row (every lane gets the total)
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float row_sum16(float x) {
    x += dpp_f32<0xB1>(x);    // quad_perm(1,0,3,2)
    x += dpp_f32<0x4E>(x);    // quad_perm(2,3,0,1)
    x += dpp_f32<0x141>(x);   // row_half_mirror
    x += dpp_f32<0x140>(x);   // row_mirror
    return x;
}

// Gradient on the matrix cores: a wavefront takes a tile of 16 samples (the
// columns; lane c = l % 16 is a sample, g = l / 16 picks four hidden units
// per register tile) and writes one partial gradient row. Forward as in
// k_hnet_fwd. Backward: dZ2 = dy w3 gelu'(z2) in the same layout; dA1 =
// W2^T dZ2 on the matrix cores with the permuted k order of the forward;
// dZ1 = dA1 gelu'(z1). Weight gradients are sums over the tile's samples,
// so the sample index becomes the k of the product: dZ2, A1 and dZ1 are
// transposed through LDS (row stride 17), and dW2 = dZ2 A1^T, db2 (a column
// of ones), dW1 = dZ1 F^T and db1 (F padded with a row of ones) run on the
// matrix cores; dw3 and db3 are row sums over the 16 sample lanes.
constexpr int kTS = 17;   // LDS row stride of the transposed 64 x 16 tiles
__global__ __launch_bounds__(kBlock) void k_hnet_grad(const float *__restrict__ theta,
                                                      const float *__restrict__ feat,
                                                      const float *__restrict__ target, int64_t nb,
                                                      float inv_b, float *partial, float *ploss) {
    __shared__ float s[kNP];
    __shared__ float tr[kBlock / 64][3][kHid * kTS];
    load_theta(theta, s);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c = lane & 15, g = lane >> 4;
    const int64_t tile = (int64_t)blockIdx.x * (kBlock / 64) + wv;
    if (tile * 16 >= nb) return;   // the whole wavefront: no samples left
    const int64_t smp = tile * 16 + c;
    const bool act = smp < nb;
    float *Ta1 = tr[wv][0], *Tdz2 = tr[wv][1], *Tdz1 = tr[wv][2];
    // forward
    f4v z1[4], z2[4];
#pragma unroll
    for (int mt = 0; mt < 4; mt++) z1[mt] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < 2; ks++) {
        const float bf = act ? feat[(int64_t)(4 * ks + g) * nb + smp] : 0.0f;
#pragma unroll
        for (int mt = 0; mt < 4; mt++) z1[mt] = mfma4(s[oW1 + (16 * mt + c) * kIn + 4 * ks + g], bf, z1[mt]);
    }
    float a1[4][4];
#pragma unroll
    for (int mt = 0; mt < 4; mt++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            z1[mt][r] += s[ob1 + 16 * mt + 4 * g + r];
            a1[mt][r] = gelu(z1[mt][r]);
        }
#pragma unroll
    for (int m2 = 0; m2 < 4; m2++) z2[m2] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int mt = 0; mt < 4; mt++)
#pragma unroll
        for (int r = 0; r < 4; r++)
#pragma unroll
            for (int m2 = 0; m2 < 4; m2++)
                z2[m2] = mfma4(s[oW2 + (16 * m2 + c) * kHid + 16 * mt + 4 * g + r], a1[mt][r], z2[m2]);
    float part = 0.0f;
#pragma unroll
    for (int m2 = 0; m2 < 4; m2++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            z2[m2][r] += s[ob2 + 16 * m2 + 4 * g + r];
            part += s[ow3 + 16 * m2 + 4 * g + r] * gelu(z2[m2][r]);
        }
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    const float res = act ? part + s[ob3] - target[smp] : 0.0f;
    const float dy = 2.0f * res * inv_b;
    float *out = partial + tile * kNP;
    // loss and db3: sums over the tile's samples
    const float lsum = row_sum16(res * res), dysum = row_sum16(dy);
    if (lane == 0) {
        ploss[tile] = lsum;
        out[ob3] = dysum;
    }
    // dZ2 (and dw3 from the same registers)
    float dz2[4][4];
#pragma unroll
    for (int m2 = 0; m2 < 4; m2++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int h = 16 * m2 + 4 * g + r;
            dz2[m2][r] = dy * s[ow3 + h] * gelu_d(z2[m2][r]);
            const float dw3 = row_sum16(dy * gelu(z2[m2][r]));
            if (c == 0) out[ow3 + h] = dw3;
            Tdz2[h * kTS + c] = dz2[m2][r];
        }
    // dA1 = W2^T dZ2, then dZ1
    f4v da1[4];
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
        da1[mt] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int m2 = 0; m2 < 4; m2++)
#pragma unroll
            for (int r = 0; r < 4; r++)
                da1[mt] = mfma4(s[oW2 + (16 * m2 + 4 * g + r) * kHid + 16 * mt + c], dz2[m2][r], da1[mt]);
    }
#pragma unroll
    for (int mt = 0; mt < 4; mt++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int h = 16 * mt + 4 * g + r;
            Ta1[h * kTS + c] = a1[mt][r];
            Tdz1[h * kTS + c] = da1[mt][r] * gelu_d(z1[mt][r]);
        }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // dW2 and db2: k = the tile's samples
    float fb[4];   // B of dW1: F[c][s] for c < 8, ones for c == 8 (db1), else 0
#pragma unroll
    for (int ks = 0; ks < 4; ks++) {
        const int64_t sk = tile * 16 + 4 * ks + g;
        fb[ks] = c < kIn ? (sk < nb ? feat[(int64_t)c * nb + sk] : 0.0f) : (c == kIn ? 1.0f : 0.0f);
    }
#pragma unroll
    for (int m2 = 0; m2 < 4; m2++) {
        float av[4];
#pragma unroll
        for (int ks = 0; ks < 4; ks++) av[ks] = Tdz2[(16 * m2 + c) * kTS + 4 * ks + g];
#pragma unroll
        for (int mt = 0; mt < 4; mt++) {
            f4v acc = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < 4; ks++) acc = mfma4(av[ks], Ta1[(16 * mt + c) * kTS + 4 * ks + g], acc);
#pragma unroll
            for (int r = 0; r < 4; r++) out[oW2 + (16 * m2 + 4 * g + r) * kHid + 16 * mt + c] = acc[r];
        }
        f4v acc = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < 4; ks++) acc = mfma4(av[ks], c == 0 ? 1.0f : 0.0f, acc);
        if (c == 0)
#pragma unroll
            for (int r = 0; r < 4; r++) out[ob2 + 16 * m2 + 4 * g + r] = acc[r];
    }
    // dW1 (columns 0..7) and db1 (column 8)
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
        f4v acc = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < 4; ks++) acc = mfma4(Tdz1[(16 * mt + c) * kTS + 4 * ks + g], fb[ks], acc);
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int h = 16 * mt + 4 * g + r;
            if (c < kIn) out[oW1 + h * kIn + c] = acc[r];
            else if (c == kIn) out[ob1 + h] = acc[r];
        }
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

// Features at radius H: kernel-weighted counts N_w(h) = (4 pi/3) h^3 sum
// W(r, h) at h = H, H/2, H/4 and raw counts within H and H/2 (self
// included), see crk.h for the eight definitions. G lanes per particle
// share the candidates and combine their five sums at the end. When the
// last build's gather rows are given and the particle's H is the support
// they were built with, the row is the candidate set (it holds every j with
// r < H, self aside); otherwise a flattened walk of the support.
template <int G>
__global__ __launch_bounds__(kBlock) void k_hnet_features(const double4 *__restrict__ posH,
                                                          const int32_t *__restrict__ cbeg,
                                                          const int32_t *__restrict__ cend, Levels v,
                                                          int64_t n, const double *__restrict__ H,
                                                          const int64_t *__restrict__ goff,
                                                          const int32_t *__restrict__ gidx,
                                                          double Nres, float *feat) {
    const int64_t gid = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    const int l = (int)(gid % G);
    const int64_t i = gid / G;
    if (i >= n) return;   // whole groups leave together
    const double4 pi = posH[i];
    const double h = H[i];
    double s1 = 0.0, s2 = 0.0, s4 = 0.0, c1 = 0.0, c2 = 0.0;
    const double h2 = h * h, ih = 1.0 / h;
    auto add = [&](double r2) {
        if (r2 < h2) {
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
    };
    constexpr int NR = flat_ranges<G>();
    __shared__ int32_t s_b[kBlock / G][NR], s_c[kBlock / G][NR + 1];
    __shared__ double s_x[kBlock / G][3 * NR];
    __shared__ AxisTab s_ax[kBlock / G];
    if (goff && h == pi.w) {
        if (l == 0) add(0.0);   // self
        for (int64_t k = goff[i] + l; k < goff[i + 1]; k += G) {
            const double4 pj = posH[gidx[k]];
            add(r2_exact(min_image(pi.x - pj.x, v.L, v.hL), min_image(pi.y - pj.y, v.L, v.hL),
                         min_image(pi.z - pj.z, v.L, v.hL)));
        }
    } else {
        const int grp = threadIdx.x / G;
        flat_candidates<G, NR>(posH, cbeg, cend, v, i, pi, h, l, s_b[grp], s_c[grp], s_x[grp], s_ax[grp],
                               [&](bool valid, double r2) {
                                   if (valid) add(r2);
                                   return false;
                               });
    }
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

// ---------------------------------------------------------------- allocation-free training step
// crk_hnet_train_step_noalloc keeps the partial gradient rows and losses of
// up to kStaticTiles 16-sample tiles in this file-scope device array instead
// of the context workspace. Each device holds its own copy (9.8 MB) until the
// process ends, and every call on that device shares it. Host code never
// passes the array's name to a kernel: it is a host-side stand-in there. The
// device address comes from hipGetSymbolAddress, taken once per device by
// hnet_scratch_init (called from crk_create with the device current).
constexpr int64_t kStaticTiles = 512;   // batches of up to 8192 samples
constexpr int64_t kStaticWords = kStaticTiles * (kNP + 1) + 64;
static __device__ __align__(256) float scratch[kStaticWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_dev[kMaxDevices] = {};
}  // namespace

crk_status hnet_scratch_init(crk_ctx *c) {
    if (c->device < 0 || c->device >= kMaxDevices)
        return set_err(c, CRK_ERR_INVALID_ARG, "device %d beyond the static scratch table", c->device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[c->device]) return CRK_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return set_err(c, CRK_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    }
    g_scratch_dev[c->device] = (float *)p;
    return CRK_OK;
}

static float *hnet_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_dev[device];
}

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
        // the gather rows serve the particles whose H is the one they were
        // built with (graph-mode lists are capacity-bound, so never those)
        const bool rows = c->built && !c->graph_mode;
        k_hnet_features<GF><<<(unsigned)((n * GF + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(
            (const double4 *)c->posH.p, (const int32_t *)c->cbeg.p, (const int32_t *)c->cend.p,
            levels(c), n, H_sorted, rows ? (const int64_t *)c->goff.p : nullptr,
            rows ? (const int32_t *)c->gidx.p : nullptr, Nres, feat);
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
        // 16 samples per wavefront step; enough blocks to fill the device, each
        // wavefront striding over the batch
        const int64_t tiles = (nb + 15) / 16;
        int64_t nbk = (tiles + kBlock / 64 - 1) / (kBlock / 64);
        if (nbk > 4096) nbk = 4096;
        k_hnet_fwd<<<(unsigned)nbk, kBlock, 0, c->stream>>>(theta, feat, nb, y);
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
    int64_t nblk = (nb + 15) / 16;   // one partial row per 16-sample tile
    CRK_TRY(ensure(c, c->hnet_part, (size_t)nblk * (kNP + 1) * sizeof(float) + 64));
    float *part = (float *)c->hnet_part.p;
    float *ploss = part + nblk * kNP;
    const float *th_in = theta;
    if (!theta) return set_err(c, CRK_ERR_INVALID_ARG, "theta is NULL");
    {
        KTimer kt_(c, "k_hnet_grad");
        k_hnet_grad<<<(unsigned)((nblk + kBlock / 64 - 1) / (kBlock / 64)), kBlock, 0, c->stream>>>(th_in, feat, target, nb, 1.0f / (float)nb,
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

crk_status crk_hnet_train_step_noalloc(crk_ctx *c, float *theta, float *adam_m, float *adam_v,
                                       int64_t step, float lr, const float *feat,
                                       const float *target, int64_t nb, float *grad, float *loss) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (!theta || !feat || !target || nb < 1 || (lr > 0.0f && (!adam_m || !adam_v || step < 1)))
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_hnet_train_step_noalloc: bad argument");
    if (nb > kStaticTiles * 16)
        return set_err(c, CRK_ERR_INVALID_ARG,
                       "crk_hnet_train_step_noalloc: %lld samples exceed the static scratch (at most %lld)",
                       (long long)nb, (long long)(kStaticTiles * 16));
    float *part = hnet_scratch(c->device);
    if (!part) return set_err(c, CRK_ERR_STATE, "static scratch address not set up for device %d", c->device);
    CRK_HIP(c, hipSetDevice(c->device));
    // the same kernels and partial layout as crk_hnet_train_step: every
    // partial row and loss of tiles 0 .. nblk-1 is written before it is read
    const int64_t nblk = (nb + 15) / 16;
    float *ploss = part + nblk * kNP;
    {
        KTimer kt_(c, "k_hnet_grad");
        k_hnet_grad<<<(unsigned)((nblk + kBlock / 64 - 1) / (kBlock / 64)), kBlock, 0, c->stream>>>(
            theta, feat, target, nb, 1.0f / (float)nb, part, ploss);
    }
    const float bc1 = 1.0f - powf(0.9f, (float)step), bc2 = 1.0f - powf(0.999f, (float)step);
    {
        KTimer kt_(c, "k_hnet_adam");
        k_hnet_adam<<<(kNP * kAdamLanes + kBlock - 1) / kBlock, kBlock, 0, c->stream>>>(
            part, nblk, lr > 0.0f ? theta : nullptr, adam_m, adam_v, lr, bc1, bc2, grad);
    }
    if (loss) k_hnet_loss<<<1, 64, 0, c->stream>>>(ploss, nblk, 1.0f / (float)nb, loss);
    CRK_HIP(c, hipGetLastError());
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
