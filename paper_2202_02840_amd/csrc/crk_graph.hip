// One whole step (S1 build, S2 volumes, S4 moments, S5 corrections, S6
// velocity gradient, S7 derivatives) behind one call, and the same step
// recorded once as a HIP graph and replayed.
//
// Every pass already covers all boxes of a batch in one launch (a particle's
// key carries its box), so the graph of a batch step is one launch per pass
// for all boxes. Recording needs a step without host round trips: in graph
// mode the build keeps the cell geometry of the last eager build, neighbour
// lists live in capacities fixed at capture time (an overflow empties the
// rows and is reported), the adaptive-precision fix launches loop over
// device-side row counts, and every count or error the eager calls would
// read back is gathered on the device into one status record.
#include <algorithm>

#include "crk_internal.h"

namespace crk {
namespace {

// gathers the counts and error words of a graph-mode step into its status
__global__ void k_graph_stat(GraphStat *st, const unsigned long long *n_singular, const int *bad,
                             const int64_t *nflag, const int64_t *ntouch) {
    st->n_singular = *n_singular;
    st->state_error = *bad ? 1 : 0;
    st->n_flag = nflag ? *nflag : 0;
    st->n_touch = ntouch ? *ntouch : 0;
}

crk_status check_io(crk_ctx *c, const crk_step_io *io) {
    if (!io || !io->x || !io->y || !io->z || !io->H || !io->v || !io->m || !io->u || !io->perm ||
        !io->V || !io->m0 || !io->m1 || !io->m2 || !io->gm0 || !io->gm1 || !io->gm2 || !io->A ||
        !io->B || !io->gA || !io->gB || !io->gradv || !io->dpdt || !io->dudt)
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_step: NULL pointer in the step arguments");
    return CRK_OK;
}

// the step's call sequence; in graph mode nothing in it waits on the device
crk_status step_run(crk_ctx *c, int32_t nboxes, const int64_t *box_offsets, int64_t n,
                    const crk_step_io *io, const crk_params *p, double cell_size, int64_t *n_pairs,
                    int64_t *n_singular) {
    const bool gm = c->graph_mode != 0;
    CRK_TRY(crk_build_cells_batch(c, nboxes, box_offsets, n, io->x, io->y, io->z, io->H, p, cell_size,
                                  io->perm, n_pairs, nullptr));
    CRK_TRY(crk_moments(c, p, nullptr, io->V, io->m0, io->m1, io->m2, io->gm0, io->gm1, io->gm2));
    crk_status sc = crk_corrections(c, n, io->m0, io->m1, io->m2, io->gm0, io->gm1, io->gm2, io->A,
                                    io->B, io->gA, io->gB, gm ? nullptr : n_singular);
    if (sc < 0) return sc;
    CRK_TRY(ensure(c, c->sv, (size_t)3 * n * sizeof(double)));
    CRK_TRY(ensure(c, c->sm, (size_t)n * sizeof(double)));
    CRK_TRY(ensure(c, c->su, (size_t)n * sizeof(double)));
    double *sv = (double *)c->sv.p, *sm = (double *)c->sm.p, *su = (double *)c->su.p;
    double *srho = nullptr;
    CRK_TRY(crk_permute(c, io->v, sv, 3, 1));
    CRK_TRY(crk_permute(c, io->m, sm, 1, 1));
    CRK_TRY(crk_permute(c, io->u, su, 1, 1));
    if (io->rho) {
        CRK_TRY(ensure(c, c->srho, (size_t)n * sizeof(double)));
        srho = (double *)c->srho.p;
        CRK_TRY(crk_permute(c, io->rho, srho, 1, 1));
    }
    CRK_TRY(crk_derivatives(c, p, sv, sm, su, srho, io->V, io->A, io->B, io->gA, io->gB, io->gradv,
                            io->dpdt, io->dudt));
    if (gm) {
        // the counters of crk_corrections and crk_derivatives live in `misc`
        const bool adapt = p->precision == CRK_MIXED_ADAPT;
        k_graph_stat<<<1, 1, 0, c->stream>>>(
            (GraphStat *)c->gstat.p, (const unsigned long long *)c->misc.p + 4, (const int *)c->misc.p + 2,
            adapt ? (const int64_t *)c->fpos.p + n : nullptr, adapt ? (const int64_t *)c->tpos.p + n : nullptr);
        CRK_HIP(c, hipGetLastError());
    }
    return sc;
}

crk_status step_args(crk_ctx *c, int32_t nboxes, const int64_t *box_offsets, int64_t n,
                     const crk_step_io *io, const crk_params *p) {
    if (!p || !box_offsets || nboxes < 1 || n < 1)
        return set_err(c, CRK_ERR_INVALID_ARG, "crk_step: bad argument");
    return check_io(c, io);
}

}  // namespace

void graph_release(crk_ctx *c) {
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    if (c->graph) {
        (void)hipGraphDestroy(c->graph);
        c->graph = nullptr;
    }
}

}  // namespace crk

using namespace crk;

extern "C" {

crk_status crk_step(crk_ctx *c, int32_t nboxes, const int64_t *box_offsets, int64_t n,
                    const crk_step_io *io, const crk_params *p, double cell_size, int64_t *n_pairs,
                    int64_t *n_singular) {
    if (!c) return CRK_ERR_INVALID_ARG;
    CRK_TRY(step_args(c, nboxes, box_offsets, n, io, p));
    if (c->graph_mode) return set_err(c, CRK_ERR_STATE, "a graph is being recorded");
    return step_run(c, nboxes, box_offsets, n, io, p, cell_size, n_pairs, n_singular);
}

crk_status crk_graph_capture(crk_ctx *c, int32_t nboxes, const int64_t *box_offsets, int64_t n,
                             const crk_step_io *io, const crk_params *p, double cell_size,
                             double headroom) {
    if (!c) return CRK_ERR_INVALID_ARG;
    CRK_TRY(step_args(c, nboxes, box_offsets, n, io, p));
    if (!(headroom >= 0.0 && headroom <= 16.0))
        return set_err(c, CRK_ERR_INVALID_ARG, "headroom must be in [0, 16]");
    if (c->graph_mode) return set_err(c, CRK_ERR_STATE, "a graph is being recorded");
    CRK_HIP(c, hipSetDevice(c->device));
    graph_release(c);
    // 1. eager step: checks the input on the host, fixes the cell geometry
    //    and measures the lists
    int64_t np = 0, ns = 0;
    crk_status st = step_run(c, nboxes, box_offsets, n, io, p, cell_size, &np, &ns);
    if (st < 0) return st;
    double g = (double)c->ngather * (1.0 + headroom) + 1024.0;
    double e = (double)c->nextra * (1.0 + headroom) + 1024.0;
    if (e > (double)(INT32_MAX - 1)) e = (double)(INT32_MAX - 1);
    if (g > 9.0e18) return set_err(c, CRK_ERR_INVALID_ARG, "gather capacity out of range");
    c->gcap = (int64_t)g;
    c->ecap = (int64_t)e;
    // the graph keeps its own copy of the box offsets (eager builds rewrite boff)
    CRK_TRY(ensure(c, c->gboff, (size_t)(nboxes + 1) * sizeof(int64_t)));
    CRK_HIP(c, hipMemcpyAsync(c->gboff.p, c->boff.p, (size_t)(nboxes + 1) * sizeof(int64_t),
                              hipMemcpyDeviceToDevice, c->stream));
    // 2. the graph-mode step once, eagerly: every workspace reaches the size
    //    the recorded step uses, so recording allocates nothing
    c->graph_mode = 1;
    st = step_run(c, nboxes, box_offsets, n, io, p, cell_size, nullptr, nullptr);
    if (st < 0) {
        c->graph_mode = 0;
        return st;
    }
    hipError_t he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) {
        c->graph_mode = 0;
        return hip_err(c, he, "hipStreamSynchronize");
    }
    GraphStat gs;
    he = hipMemcpy(&gs, c->gstat.p, sizeof gs, hipMemcpyDeviceToHost);
    if (he != hipSuccess || gs.overflow || gs.input_error || gs.state_error) {
        c->graph_mode = 0;
        if (he != hipSuccess) return hip_err(c, he, "hipMemcpy");
        return set_err(c, CRK_ERR_STATE, "graph-mode step disagrees with the eager step");
    }
    // 3. record on a stream of our own (the null stream cannot be captured)
    hipStream_t user = c->stream, rec = nullptr;
    he = hipStreamCreateWithFlags(&rec, hipStreamNonBlocking);
    if (he != hipSuccess) {
        c->graph_mode = 0;
        return hip_err(c, he, "hipStreamCreateWithFlags");
    }
    c->stream = rec;
    c->capturing = 1;
    he = hipStreamBeginCapture(rec, hipStreamCaptureModeThreadLocal);
    if (he == hipSuccess) {
        st = step_run(c, nboxes, box_offsets, n, io, p, cell_size, nullptr, nullptr);
        hipGraph_t gr = nullptr;
        hipError_t he2 = hipStreamEndCapture(rec, &gr);
        if (st >= 0 && he2 != hipSuccess) st = hip_err(c, he2, "hipStreamEndCapture");
        if (st >= 0) {
            c->graph = gr;
            he2 = hipGraphInstantiate(&c->gexec, gr, nullptr, nullptr, 0);
            if (he2 != hipSuccess) {
                c->gexec = nullptr;
                st = hip_err(c, he2, "hipGraphInstantiate");
            }
        } else if (gr) {
            (void)hipGraphDestroy(gr);
        }
    } else {
        st = hip_err(c, he, "hipStreamBeginCapture");
    }
    c->capturing = 0;
    c->stream = user;
    c->graph_mode = 0;
    (void)hipStreamDestroy(rec);
    if (st < 0) {
        graph_release(c);
        return st;
    }
    c->graph_prec = p->precision;
    c->geo.n = c->n;
    c->geo.ntab = c->ntab;
    c->geo.nboxes = c->nboxes;
    for (int k = 0; k < 12; k++) c->geo.lvl_off[k] = c->lvl_off[k];
    c->geo.L = c->L;
    c->geo.cell = c->cell;
    c->geo.nc = c->nc;
    c->geo.bits = c->bits;
    return CRK_OK;
}

crk_status crk_graph_replay(crk_ctx *c, crk_graph_status *out) {
    if (!c) return CRK_ERR_INVALID_ARG;
    if (!c->gexec) return set_err(c, CRK_ERR_STATE, "no recorded step (crk_graph_capture)");
    CRK_HIP(c, hipSetDevice(c->device));
    // the context now describes the replayed step
    c->n = c->geo.n;
    c->ntab = c->geo.ntab;
    c->nboxes = c->geo.nboxes;
    for (int k = 0; k < 12; k++) c->lvl_off[k] = c->geo.lvl_off[k];
    c->L = c->geo.L;
    c->cell = c->geo.cell;
    c->nc = c->geo.nc;
    c->bits = c->geo.bits;
    c->built = 1;
    c->have_V = 1;
    c->prec_V = c->graph_prec;
    CRK_HIP(c, hipGraphLaunch(c->gexec, c->stream));
    if (!out) return CRK_OK;
    GraphStat *pin = (GraphStat *)((char *)c->pinned.p + 3072);
    CRK_HIP(c, hipMemcpyAsync(pin, c->gstat.p, sizeof(GraphStat), hipMemcpyDeviceToHost, c->stream));
    CRK_HIP(c, hipStreamSynchronize(c->stream));
    GraphStat gs = *pin;
    out->n_pairs = gs.n_gather + gs.n_extra;
    out->n_singular = (int64_t)gs.n_singular;
    out->n_fp64_rows = gs.n_flag;
    out->n_touched_rows = gs.n_touch;
    out->input_error = gs.input_error;
    out->overflow = gs.overflow;
    out->state_error = gs.state_error;
    out->reserved = 0;
    c->ngather = gs.n_gather;
    c->nextra = gs.n_extra;
    c->npairs = out->n_pairs;
    c->last_nflag = gs.n_flag;
    c->last_ntouch = gs.n_touch;
    if (gs.input_error & 1) return set_err(c, CRK_ERR_NONFINITE, "non-finite position or H");
    if (gs.input_error & 2) return set_err(c, CRK_ERR_INVALID_ARG, "position outside [0, L)");
    if (gs.input_error & 12) return set_err(c, CRK_ERR_SUPPORT, "H <= 0 or H >= L/2");
    if (gs.overflow)
        return set_err(c, CRK_ERR_CAPACITY, "neighbour lists outgrew the recorded capacity");
    if (gs.state_error) return set_err(c, CRK_ERR_NONFINITE, "non-finite or non-positive gas state");
    return gs.n_singular ? CRK_WARN_SINGULAR : CRK_OK;
}

crk_status crk_graph_destroy(crk_ctx *c) {
    if (!c) return CRK_ERR_INVALID_ARG;
    CRK_HIP(c, hipSetDevice(c->device));
    CRK_HIP(c, hipStreamSynchronize(c->stream));
    graph_release(c);
    return CRK_OK;
}

}  // extern "C"
