// Context, errors, workspace and parameter defaults of the C ABI.
#include <math.h>

#include <algorithm>
#include <cmath>
#include <stdarg.h>
#include <stdio.h>

#include <new>

#include <vector>

#include "crk_internal.h"

namespace crk {

crk_status set_err(crk_ctx *c, crk_status s, const char *fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

crk_status hip_err(crk_ctx *c, hipError_t e, const char *what) {
    return set_err(c, CRK_ERR_HIP, "%s failed: %s", what, hipGetErrorString(e));
}

crk_status ensure(crk_ctx *c, Buf &b, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (b.bytes >= bytes) return CRK_OK;
    if (c->capturing)
        return set_err(c, CRK_ERR_STATE, "workspace of %zu bytes needed while recording a graph", bytes);
    if (b.p) {
        graph_release(c);                     // a recorded graph holds the old address
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_err(c, e, "hipStreamSynchronize");
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes + bytes / 8;          // headroom against regrowth
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_err(c, CRK_ERR_WORKSPACE, "workspace allocation of %zu bytes failed: %s", want,
                       hipGetErrorString(e));
    }
    b.bytes = want;
    return CRK_OK;
}

__global__ void k_zero_words(uint32_t *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

crk_status zero_async(crk_ctx *c, void *p, int64_t words) {
    if (words <= 0) return CRK_OK;
    k_zero_words<<<(unsigned)((words + kBlock - 1) / kBlock), kBlock, 0, c->stream>>>((uint32_t *)p, words);
    CRK_HIP(c, hipGetLastError());
    return CRK_OK;
}

static hipEvent_t pool_get(crk_ctx *c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

KTimer::KTimer(crk_ctx *ctx, const char *nm) : c(ctx), name(nm) {
    if (!c->timing || c->capturing) return;
    if (!c->timing_only.empty() && c->timing_only != nm) return;
    a = pool_get(c);
    b = pool_get(c);
    if (a && b && hipEventRecord(a, c->stream) == hipSuccess) return;
    // no timing for this scope: the events go back to the pool
    if (a) c->ev_pool.push_back(a);
    if (b) c->ev_pool.push_back(b);
    a = b = nullptr;
}

KTimer::~KTimer() {
    if (!a || !b) return;
    if (hipEventRecord(b, c->stream) != hipSuccess) {
        c->ev_pool.push_back(a);
        c->ev_pool.push_back(b);
        return;
    }
    c->ev_pend.push_back({name, {a, b}});
}

static crk_status timing_flush(crk_ctx *c) {
    if (c->ev_pend.empty()) return CRK_OK;
    CRK_HIP(c, hipStreamSynchronize(c->stream));
    for (auto &p : c->ev_pend) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) {
            auto &t = c->ev_total[p.first];
            t.first += ms;
            t.second += 1;
        } else {
            (void)hipGetLastError();
        }
        c->ev_pool.push_back(p.second.first);
        c->ev_pool.push_back(p.second.second);
    }
    c->ev_pend.clear();
    return CRK_OK;
}

}  // namespace crk

extern "C" {

crk_status crk_timing_enable(crk_ctx *c, int32_t on) {
    if (!c) return CRK_ERR_INVALID_ARG;
    CRK_TRY(crk::timing_flush(c));
    c->timing = on ? 1 : 0;
    return CRK_OK;
}

crk_status crk_timing_only(crk_ctx *c, const char *kernel) {
    if (!c) return CRK_ERR_INVALID_ARG;
    CRK_TRY(crk::timing_flush(c));
    c->timing_only = kernel ? kernel : "";
    return CRK_OK;
}

crk_status crk_timing_reset(crk_ctx *c) {
    if (!c) return CRK_ERR_INVALID_ARG;
    CRK_TRY(crk::timing_flush(c));
    c->ev_total.clear();
    return CRK_OK;
}

crk_status crk_timing_read(crk_ctx *c, const char *kernel, double *total_ms, int64_t *launches) {
    if (!c || !kernel || !total_ms || !launches) return CRK_ERR_INVALID_ARG;
    CRK_TRY(crk::timing_flush(c));
    auto it = c->ev_total.find(kernel);
    if (it == c->ev_total.end()) {
        *total_ms = 0.0;
        *launches = 0;
    } else {
        *total_ms = it->second.first;
        *launches = it->second.second;
    }
    return CRK_OK;
}

const char *crk_version(void) { return "crk-mi355x 0.1 (gfx950)"; }

crk_status crk_params_default(crk_params *p, double Nres) {
    if (!p || !(Nres > 0.0)) return CRK_ERR_INVALID_ARG;
    double nh = cbrt(3.0 * Nres / (4.0 * crk::kPi));
    p->L = 1.0;
    p->gamma = 5.0 / 3.0;
    p->Cl = 2.0;
    p->Cq = 1.0;
    p->eps = 0.1;
    p->nh = nh;
    p->eta_crit = 1.0 / nh;
    p->eta_fold = 0.2 / nh;
    p->a = 1.0;
    p->adot = 0.0;
    p->kappa_max = 1000.0;
    p->precision = CRK_FP64;
    p->reserved = 0;
    return CRK_OK;
}

crk_status crk_create(crk_ctx **out, int device, void *hip_stream) {
    if (!out) return CRK_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return CRK_ERR_HIP;
    }
    if (device < 0 || device >= ndev) return CRK_ERR_INVALID_ARG;
    crk_ctx *c = new (std::nothrow) crk_ctx();
    if (!c) return CRK_ERR_WORKSPACE;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return CRK_ERR_HIP;
    }
    void *pin = nullptr;
    if (hipHostMalloc(&pin, 4096, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return CRK_ERR_WORKSPACE;
    }
    c->pinned.p = pin;
    c->pinned.bytes = 4096;
    if (crk::hnet_scratch_init(c) != CRK_OK) {
        (void)hipHostFree(pin);
        delete c;
        return CRK_ERR_HIP;
    }
    *out = c;
    return CRK_OK;
}

// every device workspace buffer of a context (freed by crk_destroy, summed
// by crk_workspace_bytes)
static std::vector<crk::Buf *> ctx_buffers(crk_ctx *c) {
    return {&c->posH, &c->perm,  &c->cbeg,  &c->cend, &c->goff, &c->gidx, &c->ng,
                       &c->eb,    &c->ee,   &c->eidx, &c->keyA,
                       &c->keyB, &c->valA,  &c->valB,  &c->hist, &c->scanTmp, &c->recV,
                       &c->rec6, &c->rec7,  &c->red,   &c->misc, &c->flag, &c->flist,
                       &c->tlist, &c->fpos, &c->tpos,  &c->rec6d, &c->aux, &c->scratch,
                       &c->hnet_part, &c->hnet_feat, &c->hs_list, &c->hs_state, &c->hs_pos,
                       &c->hs_iters, &c->hs_pool, &c->hs_rows, &c->hs_rcnt, &c->hs_R, &c->boff,
                       &c->sv, &c->sm, &c->su, &c->srho, &c->gstat, &c->gboff,
                       &c->ecnt, &c->efill, &c->eoff, &c->etmp, &c->vnsum, &c->longs, &c->posV, &c->rq, &c->rsk, &c->rla, &c->rlb, &c->rside,
                       &c->rpnode, &c->rscan, &c->rnode, &c->rtab, &c->rbox, &c->rpoff, &c->rpart, &c->ts_vs, &c->ts_qr, &c->ce, &c->ced, &c->vstep};
}

void crk_destroy(crk_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    const std::vector<crk::Buf *> all = ctx_buffers(c);
    crk::graph_release(c);
    for (crk::Buf *b : all)
        if (b->p) (void)hipFree(b->p);
    if (c->pinned.p) (void)hipHostFree(c->pinned.p);
    for (auto &p : c->ev_pend) {
        (void)hipEventDestroy(p.second.first);
        (void)hipEventDestroy(p.second.second);
    }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
}

const char *crk_last_error(const crk_ctx *c) { return c ? c->err.c_str() : "null context"; }

// Bytes one workspace buffer reaches for a request of b bytes (ensure():
// an eighth of headroom, 256 bytes at least).
static double held(double b) {
    if (b <= 0.0) b = 256.0;
    return b + std::floor(b / 8.0);
}

// Block-sum scratch of scan_exclusive_i64 for up to m values, and of
// scan_counts2 (two arrays' block sums and one's block maxima, then the
// scan of one of them).
static double scan_bytes(double m) {
    const double tile = 2048.0;
    double need = 0.0;
    for (double k = std::ceil(m / tile); k > 1.0; k = std::ceil(k / tile)) need += k;
    return (need + 3.0 * std::ceil(m / tile) + 16.0) * 8.0;
}

crk_status crk_workspace_estimate(const crk_ctx *c, int64_t n, int32_t nboxes,
                                  double pairs_per_particle, int32_t precision, int32_t uses,
                                  int64_t *bytes) {
    if (!bytes || n < 1 || nboxes < 1 || !(pairs_per_particle >= 0.0) ||
        (precision != CRK_FP64 && precision != CRK_MIXED && precision != CRK_MIXED_ADAPT))
        return CRK_ERR_INVALID_ARG;
    const double N = (double)n, P = N * pairs_per_particle;
    // the walk's row slots: the set cap, or the adaptive one, which follows
    // the mean row (gather rows are never longer than the pairs per
    // particle) and the longest row within walk_cap_limit
    const int walk_cap = std::max({c ? c->walk_cap : 192, crk::walk_cap_for(N * pairs_per_particle, N),
                                   crk::walk_cap_limit(N)}),
              hs_cap = c ? c->hs_cap : 320;
    double t = 0.0;
    // build (crk_build_cells, any use): checks, sort, tables, lists
    const double nblk = std::min(std::ceil(N / 256.0), 1024.0);
    t += held(nblk * 24.0 + 64.0) + held(256.0) + held((nboxes + 1) * 8.0);
    t += 2 * held(4.0 * N) + 2 * held(4.0 * N) + held(std::ceil(N / 2048.0) * 256.0 * 8.0);
    t += held(std::max(scan_bytes(N + 1.0), 24.0 * N));   // scans; crk_update_support's copies
    t += held(32.0 * N);
    // cell tables of every level: at most the finest level the size cap allows
    int bits = 0;
    while (bits < 8 && (double)nboxes * std::pow(8.0, bits + 1) * 8.0 / 7.0 <= (double)(1 << 26)) bits++;
    const double ntab = (std::pow(8.0, bits + 1) - 1.0) / 7.0 * nboxes;
    t += 2 * held(4.0 * ntab);
    t += held(4.0 * N) + held(8.0 * (N + 2.0)) + held(8.0 * (N + 1.0)) + 2 * held(4.0 * N);   // counts, offsets
    t += held(4.0 * N * walk_cap) + held(4.0 * (N + 1.0));                // walk rows, long rows
    t += held(4.0 * P) + 2 * held(4.0 * 0.5 * P) + 2 * held(4.0 * N);    // N_g rows, extras (E <= P/2)
    if (precision != CRK_MIXED) t += held(8.0 * N);                       // the build's FP64 volumes
    // passes
    const bool f64 = precision == CRK_FP64, adapt = precision == CRK_MIXED_ADAPT;
    t += held((precision == CRK_MIXED ? 4.0 : 8.0) * N) + held(32.0 * N);   // volumes; positions with V
    t += held(16.0 * N * (f64 ? 2 : 1)) + held(144.0 * N * (f64 ? 2 : 1));   // records
    if (adapt) t += 2 * held(32.0 * N) + 3 * held(4.0 * N) + 2 * held(8.0 * (N + 1.0));
    if (uses & CRK_WS_TIMESTEP) t += 2 * held(8.0 * N);
    if (uses & CRK_WS_COMPAT) t += held(32.0 * N * (f64 ? 2 : 1)) + (adapt ? held(64.0 * N) : 0.0);
    if (uses & CRK_WS_HSOLVE) {
        t += held(8.0 * N) + 2 * held(4.0 * N) + held(8.0 * (N + 1.0)) + held(8.0 * N * hs_cap) +
             held(4.0 * N) + held(8.0 * N);
        // rows of the particles whose candidates pass the cap: at most 8 GiB
        const double pcap = std::max(4096.0, 8.0 * hs_cap);
        t += held(std::min(N * pcap * 8.0, (double)(8LL << 30)));
    }
    if (uses & CRK_WS_HNET) t += held(36.0 * N) + held(std::ceil(N / 16.0) * 4802.0 * 4.0 + 64.0);
    if (uses & CRK_WS_VERLET) t += held((16.0 + 70.0) * 8.0 * N + 4.0 * N);
    if (uses & CRK_WS_GRAPH) {
        t += held(24.0 * N) + 3 * held(8.0 * N) + held((nboxes + 1) * 8.0) + held(64.0);
        // list capacities of the recorded step: 1.25 P + 1024 (default headroom)
        t += held(4.0 * (1.25 * P + 1024.0)) - held(4.0 * P);
        t += 2 * (held(4.0 * (0.625 * P + 1024.0)) - held(2.0 * P));
    }
    if (uses & CRK_WS_LEAVES) {
        // keys and lists, sides, node and leaf tables, boxes, leaf partners,
        // capped extras rows
        const double nl = std::ceil(N / 128.0) + nboxes;
        t += 4 * held(12.0 * N) + held(N) + held(4.0 * N) + held(8.0 * (N + 1.0));
        t += held(9.0 * N) + held(16.0 * (N / 8.0 + 2.0 * nl + nboxes + 1.0)) + held(64.0 * N / 8.0 + 64.0 * nl);
        t += held(8.0 * (nl + 1.0)) + held(4.0 * nl * std::min(nl, 4096.0)) + held(4.0 * N * 64.0);
    }
    *bytes = (int64_t)std::ceil(t);
    return CRK_OK;
}

crk_status crk_workspace_bytes(crk_ctx *c, int64_t *bytes) {
    if (!c || !bytes) return CRK_ERR_INVALID_ARG;
    int64_t t = 0;
    for (const crk::Buf *b : ctx_buffers(c)) t += (int64_t)b->bytes;
    *bytes = t;
    return CRK_OK;
}

}  // extern "C"
