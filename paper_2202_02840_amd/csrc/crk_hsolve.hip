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

__device__ __forceinline__ double nsum_walk(const double4 *__restrict__ posH, const int32_t *__restrict__ cbeg,
                                            const int32_t *__restrict__ cend, const Levels &v, double4 pi,
                                            double H) {
    const double H2 = H * H, invH = 1.0 / H;
    double s = 0.0;
    walk_cells(v, cbeg, cend, pi.x, pi.y, pi.z, H, [&](int j) {
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
    });
    return kW * invH * invH * invH * s;
}

__global__ __launch_bounds__(kBlock) void k_hsolve(const double4 *__restrict__ posH,
                                                   const int32_t *__restrict__ cbeg,
                                                   const int32_t *__restrict__ cend, Levels v, int64_t n,
                                                   double Nres, double tol, int max_iter, double *H_io,
                                                   int32_t *iters, unsigned long long *counters) {
    int64_t i = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    double4 pi = posH[i];
    double H = H_io[i];
    int it = 0;
    bool conv = false, support = false;
    while (it < max_iter) {
        double ns = nsum_walk(posH, cbeg, cend, v, pi, H);
        double N = (4.0 * kPi / 3.0) * H * H * H * ns;
        double D = cbrt(Nres / N);
        double lam = D < 1.0 ? 0.2 * (1.0 + D * D) : 0.2 * (1.0 + 1.0 / (D * D * D));
        double Hn = H * (1.0 - lam + lam * D);
        it++;
        bool done = fabs(Hn - H) <= tol * H;
        H = Hn;
        if (!(H < v.hL)) {
            support = true;
            break;
        }
        if (done) {
            conv = true;
            break;
        }
    }
    H_io[i] = H;
    if (iters) iters[i] = it;
    if (!conv) atomicAdd(&counters[0], 1ull);
    if (support) atomicAdd(&counters[1], 1ull);
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
    int64_t n = c->n;
    Levels v;
    v.L = c->L;
    v.hL = 0.5 * c->L;
    v.c0 = c->cell;
    v.margin = 1e-9 * c->L;
    v.bits = c->bits;
    for (int k = 0; k < 12; k++) v.off[k] = c->lvl_off[k];
    CRK_TRY(ensure(c, c->misc, 256));
    unsigned long long *cnt = (unsigned long long *)c->misc.p + 6;
    CRK_HIP(c, hipMemsetAsync(cnt, 0, 2 * sizeof(unsigned long long), c->stream));
    {
        KTimer kt_(c, "k_hsolve");
        k_hsolve<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>(
            (const double4 *)c->posH.p, (const int32_t *)c->cbeg.p, (const int32_t *)c->cend.p, v, n,
            Nres, tol, max_iter, H_inout, iters, cnt);
    }
    CRK_HIP(c, hipGetLastError());
    unsigned long long *pin = (unsigned long long *)c->pinned.p + 16;
    CRK_HIP(c, hipMemcpyAsync(pin, cnt, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
    CRK_HIP(c, hipStreamSynchronize(c->stream));
    if (n_unconverged) *n_unconverged = (int64_t)pin[0];
    if (pin[1]) return set_err(c, CRK_ERR_SUPPORT, "%llu supports reached L/2", pin[1]);
    // the lists no longer match the support radii
    c->built = 0;
    c->have_V = 0;
    k_set_H2<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>((double4 *)c->posH.p, H_inout, n);
    CRK_HIP(c, hipGetLastError());
    if (pin[0]) return CRK_WARN_NOT_CONVERGED;
    return CRK_OK;
}

}  // extern "C"
