// Velocity-Verlet hydro step, eq. (verletOP): half kick and drift from the
// derivatives of the start state, a predicted momentum and energy at the
// end of the step, one whole derivative evaluation there (the step of
// crk_step: build, volumes, moments, corrections, velocity gradient,
// derivatives), and the closing half kick. The time step dt is the paper's
// (dt/dy) Delta y; a and adot are held over the step.
//
// Also the hierarchical time-step levels of the time integrator (Sec. 3.1)
// from the Courant time and the hydrodynamic acceleration.
//
// The state stays in the caller's (original) particle order; the
// evaluation's outputs come back in cell-sorted order and the closing kick
// gathers them through the sort permutation. The elementwise kernels are
// HBM-bound; the evaluation is the step itself.
#include <math.h>

#include "crk_internal.h"

// the kicks and the drift are written operation by operation; no product is
// fused into the following sum (hipcc contracts by default)
#pragma clang fp contract(off)

namespace crk {
namespace {

constexpr int kVB = 256;

// p^1/2 = a v + dt/2 dp/dt(0), u^1/2 = u + dt/2 du/dt(0),
// x^1 = x + p^1/2 dt / a^2 wrapped into [0, L), p_p = p^1/2 + dt/2 dp/dt(0),
// u_p = u^1/2 + dt/2 du/dt(0); the products and sums are rounded one by one
// (no fused multiply-add, see the pragma above), so a drift reproduces
// x + p dt / a^2 exactly as written.
__global__ __launch_bounds__(kVB) void k_kick_drift(int64_t n, double a, double k, double c, double L,
                                                    double *x, double *y, double *z,
                                                    const double *__restrict__ v,
                                                    const double *__restrict__ u,
                                                    const double *__restrict__ dpdt,
                                                    const double *__restrict__ dudt,
                                                    double *__restrict__ ph, double *__restrict__ uh,
                                                    double *__restrict__ vp, double *__restrict__ up) {
    const int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x;
    if (i >= n) return;
    double *pos[3] = {x, y, z};
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const int64_t j = q * n + i;
        const double kd = k * dpdt[j];
        const double h = a * v[j] + kd;
        ph[j] = h;
        const double dx = h * c;
        double xn = pos[q][i] + dx;
        if (xn < 0.0) xn = xn + L;
        if (xn >= L) xn = xn - L;
        pos[q][i] = xn;
        vp[j] = (h + kd) / a;
    }
    const double kd = k * dudt[i];
    const double hu = u[i] + kd;
    uh[i] = hu;
    up[i] = hu + kd;
}

// p^1 = p^1/2 + dt/2 dp/dt(1), u^1 = u^1/2 + dt/2 du/dt(1) with the end
// derivatives in sorted order (perm: sorted -> original), or u^1 = u^1/2 +
// the compatible change sdc of the closing kick when given; the end
// derivatives are also returned in the original order for the next step.
__global__ __launch_bounds__(kVB) void k_kick_close(int64_t n, const int32_t *__restrict__ perm,
                                                    double a, double k,
                                                    const double *__restrict__ ph,
                                                    const double *__restrict__ uh,
                                                    const double *__restrict__ sdp,
                                                    const double *__restrict__ sdu,
                                                    const double *__restrict__ sdc, double *v,
                                                    double *u, double *dpdt, double *dudt) {
    const int64_t s = (int64_t)blockIdx.x * kVB + threadIdx.x;
    if (s >= n) return;
    const int64_t i = perm[s];
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const double d = sdp[q * n + s];
        const double p1 = ph[q * n + i] + k * d;
        v[q * n + i] = p1 / a;
        dpdt[q * n + i] = d;
    }
    const double du = sdu[s];
    u[i] = sdc ? uh[i] + sdc[s] : uh[i] + k * du;
    dudt[i] = du;
}

// the two kicks' start momenta in sorted order: p^1/2 (closing kick) and
// p^1 = p^1/2 + dt/2 dp/dt(1) (the next opening kick), the latter with the
// same operations as the closing kick itself
__global__ __launch_bounds__(kVB) void k_gather_kicks(int64_t n, const int32_t *__restrict__ perm,
                                                      double k, const double *__restrict__ ph,
                                                      const double *__restrict__ sdp,
                                                      double *__restrict__ phs,
                                                      double *__restrict__ p1s) {
    const int64_t s = (int64_t)blockIdx.x * kVB + threadIdx.x;
    if (s >= n) return;
    const int64_t i = perm[s];
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const double h = ph[q * n + i];
        phs[q * n + s] = h;
        p1s[q * n + s] = h + k * sdp[q * n + s];
    }
}

// the opening kick's energy change of the next step as a rate: dudt = du / k
__global__ __launch_bounds__(kVB) void k_rate(int64_t n, const int32_t *__restrict__ perm,
                                              double k, const double *__restrict__ sdu,
                                              double *dudt) {
    const int64_t s = (int64_t)blockIdx.x * kVB + threadIdx.x;
    if (s >= n) return;
    dudt[perm[s]] = sdu[s] / k;
}

// sorted derivatives -> original order
__global__ __launch_bounds__(kVB) void k_unsort_d(int64_t n, const int32_t *__restrict__ perm,
                                                  const double *__restrict__ sdp,
                                                  const double *__restrict__ sdu, double *dpdt,
                                                  double *dudt) {
    const int64_t s = (int64_t)blockIdx.x * kVB + threadIdx.x;
    if (s >= n) return;
    const int64_t i = perm[s];
#pragma unroll
    for (int q = 0; q < 3; q++) dpdt[q * n + i] = sdp[q * n + s];
    dudt[i] = sdu[s];
}

// dt_acc = sqrt(min(h_hat, r_soft) / |a_hyd|), a_hyd = dp/dt / a^2 (infinite
// when it vanishes), dt_min = min(dt_hyd, dt_acc), and the smallest level
// l >= 0 with dt_min > dt_sub / 2^l (l_max + 1, counted, when none is); the
// halvings of dt_sub are exact, as in the definition.
__global__ __launch_bounds__(kVB) void k_levels(int64_t n, const double4 *__restrict__ posH,
                                                const double *__restrict__ dt_hyd,
                                                const double *__restrict__ dpdt, double inv_nh,
                                                double inv_a2, double r_soft, double dt_sub,
                                                int l_max, double *dt_acc, double *dt_min,
                                                int32_t *level,
                                                unsigned long long *n_over) {
    const int64_t i = (int64_t)blockIdx.x * kVB + threadIdx.x;
    if (i >= n) return;
    const double hh = posH[i].w * inv_nh;
    const double gx = dpdt[i], gy = dpdt[n + i], gz = dpdt[2 * n + i];
    const double acc = sqrt(gx * gx + gy * gy + gz * gz) * inv_a2;
    const double ta = acc > 0.0 ? sqrt(fmin(hh, r_soft) / acc) : INFINITY;
    const double tm = fmin(dt_hyd[i], ta);
    int l = 0;
    double thr = dt_sub;
    while (l <= l_max && !(tm > thr)) {
        thr *= 0.5;
        l++;
    }
    if (dt_acc) dt_acc[i] = ta;
    if (dt_min) dt_min[i] = tm;
    level[i] = l;
    if (l > l_max) atomicAdd(n_over, 1ull);
}

inline unsigned vblocks(int64_t n) { return (unsigned)((n + kVB - 1) / kVB); }

// doubles per particle of the step's sorted outputs, in crk_step_io order
constexpr int kOutDoubles = 1 + 1 + 3 + 6 + 3 + 9 + 18 + 1 + 3 + 3 + 9 + 9 + 3 + 1;

// points the sorted outputs of the evaluation into the workspace
void carve(double *w, int64_t n, int32_t *perm, crk_step_io &io) {
    io.perm = perm;
    io.V = w;        w += n;
    io.m0 = w;       w += n;
    io.m1 = w;       w += 3 * n;
    io.m2 = w;       w += 6 * n;
    io.gm0 = w;      w += 3 * n;
    io.gm1 = w;      w += 9 * n;
    io.gm2 = w;      w += 18 * n;
    io.A = w;        w += n;
    io.B = w;        w += 3 * n;
    io.gA = w;       w += 3 * n;
    io.gB = w;       w += 9 * n;
    io.gradv = w;    w += 9 * n;
    io.dpdt = w;     w += 3 * n;
    io.dudt = w;
}

}  // namespace
}  // namespace crk

using namespace crk;

extern "C" {

// compatible change of half kicks of length k from the sorted momenta pks
// (NULL: a v of the evaluation) and, with dus2, pks2, with the pair forces of
// the evaluation just made by crk_step (its sorted state and outputs, and
// the records its derivative pass packed)
static crk_status compat_half(crk_ctx *c, const crk_params *p, const crk_step_io &sio,
                              const double *pks, const double *pks2, double k, double *dus,
                              double *dus2) {
    const double *sv = (const double *)c->sv.p, *sm = (const double *)c->sm.p,
                 *su = (const double *)c->su.p;
    const double *srho = sio.rho ? (const double *)c->srho.p : nullptr;
    return compat_pass(c, p, sv, sm, su, srho, sio.V, sio.A, sio.B, sio.gA, sio.gB, sio.gradv,
                       sio.dpdt, pks, pks2, k, dus, dus2, true);
}

crk_status crk_verlet_step(crk_ctx *c, int32_t nboxes, const int64_t *box_offsets, int64_t n,
                           const crk_verlet_io *io, const crk_params *p, double cell_size,
                           double dt, int32_t start_eval, int32_t energy, int64_t *n_pairs) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (!io || !p || !box_offsets || nboxes < 1 || n < 1 || !io->x || !io->y || !io->z || !io->H ||
        !io->v || !io->m || !io->u || !io->dpdt || !io->dudt)
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_verlet_step: bad argument");
    if (!isfinite(dt) || !(p->a > 0.0) || !(p->L > 0.0) || (energy != 0 && energy != 1) ||
        (energy == 1 && !(dt != 0.0)))
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_verlet_step: bad parameter");
    if (c->graph_mode || c->capturing)
        return set_err(c, CRK_ERR_STATE, "crk_verlet_step is not recorded in a graph");
    CRK_HIP(c, hipSetDevice(c->device));
    // workspace: p^1/2, u^1/2, p_p / a, u_p, the evaluation's outputs, then
    // sorted kick-start momenta and energy changes (compatible mode)
    const bool compat = energy == 1;
    const size_t nd = (size_t)(8 + kOutDoubles + 8) * n;
    CRK_TRY(ensure(c, c->vstep, nd * sizeof(double) + (size_t)n * sizeof(int32_t)));
    double *w = (double *)c->vstep.p;
    double *ph = w, *uh = w + 3 * n, *vp = w + 4 * n, *up = w + 7 * n;
    int32_t *perm = (int32_t *)(w + nd);
    crk_step_io sio{};
    carve(w + 8 * n, n, perm, sio);
    double *pks = w + (size_t)(8 + kOutDoubles) * n, *p1s = pks + 3 * n, *dus = p1s + 3 * n,
           *dus2 = dus + n;
    const double a = p->a, k = 0.5 * dt, cd = dt / (a * a);
    sio.H = io->H;
    sio.m = io->m;
    sio.rho = io->rho;
    if (start_eval) {
        sio.x = io->x;
        sio.y = io->y;
        sio.z = io->z;
        sio.v = io->v;
        sio.u = io->u;
        crk_status st = crk_step(c, nboxes, box_offsets, n, &sio, p, cell_size, nullptr, nullptr);
        if (st < 0) return st;
        {
            KTimer kt_(c, "k_verlet");
            k_unsort_d<<<vblocks(n), kVB, 0, c->stream>>>(n, perm, sio.dpdt, sio.dudt, io->dpdt, io->dudt);
            CRK_HIP(c, hipGetLastError());
        }
        if (compat) {
            // the first opening kick's compatible change, from p = a v
            CRK_TRY(compat_half(c, p, sio, nullptr, nullptr, k, dus, nullptr));
            k_rate<<<vblocks(n), kVB, 0, c->stream>>>(n, perm, k, dus, io->dudt);
            CRK_HIP(c, hipGetLastError());
        }
    }
    {
        KTimer kt_(c, "k_verlet");
        k_kick_drift<<<vblocks(n), kVB, 0, c->stream>>>(n, a, k, cd, p->L, io->x, io->y, io->z, io->v,
                                                         io->u, io->dpdt, io->dudt, ph, uh, vp, up);
        CRK_HIP(c, hipGetLastError());
    }
    sio.x = io->x;
    sio.y = io->y;
    sio.z = io->z;
    sio.v = vp;
    sio.u = up;
    crk_status st = crk_step(c, nboxes, box_offsets, n, &sio, p, cell_size, n_pairs, nullptr);
    if (st < 0) return st;
    if (compat) {
        // the closing kick (from p^1/2) and the next step's opening kick
        // (from p^1 = p^1/2 + dt/2 dp/dt(1)) share the end evaluation's pair
        // forces: one pass gives both changes
        {
            KTimer kt_(c, "k_verlet");
            k_gather_kicks<<<vblocks(n), kVB, 0, c->stream>>>(n, perm, k, ph, sio.dpdt, pks, p1s);
            CRK_HIP(c, hipGetLastError());
        }
        CRK_TRY(compat_half(c, p, sio, pks, p1s, k, dus, dus2));
    }
    {
        KTimer kt_(c, "k_verlet");
        k_kick_close<<<vblocks(n), kVB, 0, c->stream>>>(n, perm, a, k, ph, uh, sio.dpdt, sio.dudt,
                                                         compat ? dus : nullptr, io->v, io->u, io->dpdt,
                                                         io->dudt);
        CRK_HIP(c, hipGetLastError());
    }
    if (compat) {
        // the next opening kick's change, carried as a rate in dudt
        k_rate<<<vblocks(n), kVB, 0, c->stream>>>(n, perm, k, dus2, io->dudt);
        CRK_HIP(c, hipGetLastError());
    }
    CRK_HIP(c, hipStreamSynchronize(c->stream));
    return st;
}

crk_status crk_time_levels(crk_ctx *c, const crk_params *p, const double *dt_hyd,
                           const double *dpdt, double r_soft, double dt_sub, int32_t l_max,
                           double *dt_acc, double *dt_min, int32_t *level, int64_t *n_over) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (!p || !dt_hyd || !dpdt || !level)
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_time_levels: NULL argument");
    if (!(p->a > 0.0) || !(p->nh > 0.0) || !(r_soft > 0.0) || !(dt_sub > 0.0) ||
        !isfinite(dt_sub) || l_max < 0 || l_max > 60)
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_time_levels: bad parameter");
    if (!c->built) return set_err(c, CRK_ERR_STATE, "crk_build_cells has not run");
    CRK_HIP(c, hipSetDevice(c->device));
    CRK_TRY(ensure(c, c->misc, 256));
    unsigned long long *cnt = (unsigned long long *)c->misc.p + 12;
    CRK_HIP(c, hipMemsetAsync(cnt, 0, sizeof(*cnt), c->stream));
    const int64_t n = c->n;
    k_levels<<<vblocks(n), kVB, 0, c->stream>>>(n, (const double4 *)c->posH.p, dt_hyd, dpdt,
                                                 1.0 / p->nh, 1.0 / (p->a * p->a), r_soft, dt_sub,
                                                 l_max, dt_acc, dt_min, level, cnt);
    CRK_HIP(c, hipGetLastError());
    unsigned long long *pin = (unsigned long long *)c->pinned.p + 60;
    CRK_HIP(c, hipMemcpyAsync(pin, cnt, sizeof(*cnt), hipMemcpyDeviceToHost, c->stream));
    CRK_HIP(c, hipStreamSynchronize(c->stream));
    if (n_over) *n_over = (int64_t)*pin;
    return CRK_OK;
}

}  // extern "C"
