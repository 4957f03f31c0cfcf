/*
 * crk.h — C ABI of the CRKSPH neighbour-pass library for AMD Instinct MI355X
 * (gfx950).
 *
 * The library evaluates the particle passes of the conservative
 * reproducing-kernel SPH hydro solver of Frontiere et al., "Simulating
 * Hydrodynamics in Cosmology with CRK-HACC" (Sec. 2.2 and Sec. 3.6):
 *
 *   crk_build_cells  cell list + neighbour lists (chaining mesh, Sec. 3.3;
 *                    one interaction list per step, reused by every pass)
 *   crk_moments      volumes, eq. (vol), and the kernel moments whose
 *                    constraints fix the RK kernel, eqs. (RK), (gRK)
 *   crk_corrections  RK coefficients A, B and their gradients
 *   crk_derivatives  RK velocity gradient, eq. (gradv), then the momentum and
 *                    energy derivatives, eqs. (mom), (eng), with the limited
 *                    Monaghan-Gingold viscosity, eqs. (visc)-(phiad)
 *   crk_hsolve       smoothing-length iteration, eqs. (hi), (thacker)
 *
 * Notation. H is the kernel support radius (the paper's h in eq. (C4):
 * W = 0 for |x| >= h). d = x_i - x_j is the minimum-image separation in a
 * periodic cube of side L. The gather set of i is N_g(i) = {j : |d| < H_i}
 * (i included); the pair set is N_s(i) = {j != i : |d| < max(H_i, H_j)}.
 *
 * Memory. Every array argument is a DEVICE pointer to a caller-owned,
 * contiguous buffer on the context's device. Vector fields are
 * component-major: a field with k components over n particles is k
 * consecutive arrays of n values ([k][n]). The library never allocates or
 * frees caller memory; it owns only the context workspace (sorted copies,
 * neighbour lists, packed per-particle records, scratch), which grows on
 * demand and is released by crk_destroy.
 *
 * Ordering. crk_build_cells sorts the particles by cell (Morton order of the
 * cells, ties by original index). Every per-particle array passed to or
 * returned by the later calls is in that sorted order; crk_permute moves
 * arrays between the original and the sorted order.
 *
 * Index conventions (fixed so results can be compared element by element):
 *   m2 and other symmetric 3x3 tensors: (xx, xy, xz, yy, yz, zz)
 *   gm1[a*3+g] = d m1^a / d x^g      gm2[s*3+g] = d m2^s / d x^g
 *   gB[a*3+g]  = d B^a  / d x^g      gradv[a*3+b] = d v^a / d x^b
 *
 * Errors and synchronisation. Every function returns a crk_status and throws
 * nothing across the ABI. On an error the outputs are unspecified and
 * crk_last_error() holds a message. Work is enqueued on the context's HIP
 * stream; functions that return a host value (a count) synchronise that
 * stream. A context is used by one host thread at a time.
 */
#ifndef CRK_H
#define CRK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CRK_OK = 0,
    CRK_WARN_SINGULAR = 1,      /* some m2 were singular; those particles use the SPH fallback */
    CRK_WARN_NOT_CONVERGED = 2, /* the smoothing-length iteration hit max_iter for some particles */
    CRK_ERR_INVALID_ARG = -1,   /* NULL pointer, n < 1, position outside [0, L), bad parameter */
    CRK_ERR_NONFINITE = -2,     /* NaN or Inf in positions, H, masses, energies or densities */
    CRK_ERR_SUPPORT = -3,       /* H <= 0 or max H >= L/2 (the minimum image would be ambiguous) */
    CRK_ERR_WORKSPACE = -4,     /* device allocation of the workspace failed */
    CRK_ERR_HIP = -5,           /* a HIP runtime call failed */
    CRK_ERR_STATE = -6,         /* called out of order (e.g. crk_moments before crk_build_cells) */
    CRK_ERR_CAPACITY = -7       /* a replayed step's lists outgrew the capacity recorded in the graph */
} crk_status;

/* Arithmetic of the pair passes. */
typedef enum {
    CRK_FP64 = 0,  /* every pair term and sum in FP64 */
    CRK_MIXED = 1, /* FP32 pair terms with compensated (Kahan) FP32 sums in every pair pass;
                      separations are formed in FP64 before rounding; the RK solve
                      (crk_corrections) and every boundary array stay FP64.
                      Accuracy depends on the conditioning of the RK solve: on jittered
                      lattices every output meets 1e-5 normwise against CRK_FP64, but on
                      clustered inputs with nearly singular m2 it does NOT. Measured on
                      a lognormal 128^3 box (sigma_ln_rho = 1.5), normwise against
                      CRK_FP64: A 3e-2, B 3e-1, grad A 3e-1, grad B 9e+2 (the FP32
                      moment sums of the few nearly singular particles), velocity
                      gradient 6e-1, dv/dt 3e-1, du/dt 2e-1. Use CRK_MIXED_ADAPT for
                      clustered inputs (all outputs within 1e-5 there). */
    CRK_MIXED_ADAPT = 2 /* volume and moment passes in FP64 (their sums feed the RK solve,
                      whose conditioning amplifies any rounding in them); velocity-gradient
                      and derivative passes as in CRK_MIXED, except the rows of particles
                      whose RK template is ill-conditioned, kappa_i = 1 + |B_i| H_i +
                      |gradB_i| H_i^2 + |gradA_i| H_i / |A_i| > kappa_max: their velocity
                      gradient and every derivative pair they take part in run in FP64 */
} crk_precision;

/*
 * Solver parameters (Sec. 2.2, Sec. 3.6).
 *   L                periodic box side
 *   gamma            adiabatic index of P = (gamma - 1) rho u, eq. (EOS)
 *   Cl, Cq, eps      viscosity constants of eqs. (visc), (mu): 2, 1, 0.1
 *   nh               particles per smoothing length; hh = H / nh in eq. (mu)
 *   eta_crit, eta_fold   limiter adjustment scales of eq. (phiad): 1/nh, 0.2/nh
 *   a, adot          scale factor and its rate (a = 1, adot = 0 without expansion)
 *   kappa_max        conditioning bound of CRK_MIXED_ADAPT (ignored otherwise)
 *   precision        a crk_precision value
 */
typedef struct {
    double L, gamma, Cl, Cq, eps, nh, eta_crit, eta_fold, a, adot, kappa_max;
    int32_t precision;
    int32_t reserved;
} crk_params;

typedef struct crk_ctx crk_ctx;

/* Fills *p with the defaults for a target neighbour count Nres: L = 1,
 * gamma = 5/3, (Cl, Cq, eps) = (2, 1, 0.1), nh = (3 Nres / (4 pi))^(1/3)
 * (n_h = 4 for N_res = 268, Sec. 3.6), eta_crit = 1/nh, eta_fold = 0.2/nh,
 * a = 1, adot = 0, kappa_max = 1000, precision CRK_FP64. Host memory. */
crk_status crk_params_default(crk_params *p, double Nres);

/* Creates a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream). *out receives the context. */
crk_status crk_create(crk_ctx **out, int device, void *hip_stream);
void crk_destroy(crk_ctx *ctx);
const char *crk_last_error(const crk_ctx *ctx);

/* Device memory the context's workspace holds now, in bytes (sorted copies,
 * neighbour lists, records, scratch; excluding the caller's arrays and a few
 * KB of pinned host memory). The workspace grows on demand with n and with
 * the neighbour counts of the data, so query it after a representative call
 * (e.g. a first step) to learn the footprint. *bytes is a host pointer. */
crk_status crk_workspace_bytes(crk_ctx *ctx, int64_t *bytes);

/* Which calls a context will make, for crk_workspace_estimate. Every use
 * includes the step itself (crk_build_cells, crk_moments, crk_corrections,
 * crk_derivatives). */
enum {
    CRK_WS_STEP = 0,
    CRK_WS_HSOLVE = 1,     /* crk_hsolve */
    CRK_WS_HNET = 2,       /* crk_hnet_features / forward / train_step / seed */
    CRK_WS_COMPAT = 4,     /* crk_compatible_energy */
    CRK_WS_VERLET = 8,     /* crk_verlet_step (add CRK_WS_COMPAT for its compatible mode) */
    CRK_WS_GRAPH = 16,     /* crk_step / crk_graph_capture, default headroom */
    CRK_WS_TIMESTEP = 32,  /* crk_set_timestep(1) */
    CRK_WS_LEAVES = 64     /* crk_build_leaves */
};

/* Upper bound, computed before any call, on the device bytes a context's
 * workspace reaches for calls on n particles in nboxes boxes with at most
 * pairs_per_particle ordered pairs (|N_s(i)|, averaged) per particle, in
 * the given crk_precision, for the calls named by `uses` (CRK_WS_* or'ed).
 * It bounds crk_workspace_bytes after those calls when the realised pair
 * count stays within n * pairs_per_particle. Parts that depend on data it
 * cannot see are taken at their caps: the cell tables at the finest level
 * the build allows, the h iteration's overflow rows at their 8 GiB limit,
 * the leaf partner lists at 4096 partners per leaf. ctx (may be NULL: the
 * default tuning) supplies the walk and h-iteration row capacities. Host
 * memory only; no device call. */
crk_status crk_workspace_estimate(const crk_ctx *ctx, int64_t n, int32_t nboxes,
                                  double pairs_per_particle, int32_t precision, int32_t uses,
                                  int64_t *bytes);

/*
 * S1: cell list and neighbour lists (chaining mesh, Sec. 3.3).
 * In:  n particles, x, y, z in [0, L) and support radii H (original order).
 *      cell_size <= 0 picks the cell side from the mean H.
 * Out: perm[n] (device, int32): perm[k] = original index of sorted particle k.
 *      *n_pairs (host, may be NULL): number of ordered pairs (i, j), j in N_s(i).
 *      *n_cells (host, may be NULL): cells per dimension.
 * The context keeps the sorted positions and H, the gather lists N_g and the
 * pair lists N_s; unless p->precision is CRK_MIXED also the FP64 volumes of
 * eq. (vol) over N_g, summed as the lists are placed (crk_moments hands
 * them out). Synchronises the stream. Errors: CRK_ERR_INVALID_ARG,
 * CRK_ERR_NONFINITE, CRK_ERR_SUPPORT, CRK_ERR_WORKSPACE, CRK_ERR_HIP.
 */
crk_status crk_build_cells(crk_ctx *ctx, int64_t n, const double *x, const double *y,
                           const double *z, const double *H, const crk_params *p,
                           double cell_size, int32_t *perm, int64_t *n_pairs, int32_t *n_cells);

/*
 * S1, alternative tiling: recursive coordinate bisection leaves (Sec. 3.3:
 * an RCB tree whose flat leaves hold N_ppl particles, one interaction list
 * per leaf from leaf boxes grown by the smoothing support). Each box of the
 * batch (box_offsets: HOST int64 [nboxes+1], 0 .. n; one box: {0, n}) is
 * split by its own tree: a node of more than `bucket` particles is halved
 * along the axis of largest extent of the 32-bit fixed-point coordinate
 * keys q = floor(x / L 2^32), its floor(n/2) smallest keys (ties by original
 * index) going left; a leaf is the first node on a path with at most
 * `nppl` particles (so leaves hold nppl/2 .. nppl particles when the box
 * holds more than nppl), and inside a leaf the buckets below it follow in
 * tree order, each in x-key order. Leaves a and b of one box interact when
 * the periodic distance of their bounding boxes is below max(Hmax_a, Hmax_b)
 * (+ 1e-9 L). The rows are found leaf pair by leaf pair with the partner
 * leaf's particles in LDS, by the exact FP64 test of crk_build_cells, so
 * N_g and N_s are the same sets; the sorted order is the leaf order.
 * Requires 4 <= bucket <= 64, bucket <= nppl <= 256 (and nppl / bucket
 * small enough for 64 buckets per leaf).
 * Out: perm[n] (device int32, sorted -> original), *n_pairs, *n_leaves
 * (host, may be NULL), leaf_offsets (device int32 [n_leaves+1] in sorted
 * positions, may be NULL; leaf_cap = its capacity).
 * After this call crk_moments, crk_corrections, crk_derivatives,
 * crk_compatible_energy, crk_permute and crk_export_neighbors work as after
 * crk_build_cells; the calls that walk the cell hierarchy (crk_hsolve,
 * crk_update_support, crk_hnet_features, crk_hnet_seed) return
 * CRK_ERR_STATE. Synchronises the stream. Errors as crk_build_cells.
 */
crk_status crk_build_leaves(crk_ctx *ctx, int32_t nboxes, const int64_t *box_offsets, int64_t n,
                            const double *x, const double *y, const double *z, const double *H,
                            const crk_params *p, int32_t nppl, int32_t bucket, int32_t *perm,
                            int64_t *n_pairs, int32_t *n_leaves, int32_t *leaf_offsets,
                            int64_t leaf_cap);

/*
 * S10: many independent periodic boxes (same L) in one build. Particles are
 * concatenated box by box: box b owns [box_offsets[b], box_offsets[b+1]) of
 * the n particles (box_offsets: HOST int64 [nboxes+1], 0 .. n). The sort
 * groups particles by (box, Morton cell), each box gets its own cell
 * hierarchy, and a particle only ever pairs with particles of its own box.
 * Every later call (moments, corrections, derivatives, h iteration, network)
 * then runs over all boxes in one launch per pass, on the concatenated
 * arrays in the sorted order. crk_build_cells is this call with one box.
 */
crk_status crk_build_cells_batch(crk_ctx *ctx, int32_t nboxes, const int64_t *box_offsets,
                                 int64_t n, const double *x, const double *y, const double *z,
                                 const double *H, const crk_params *p, double cell_size,
                                 int32_t *perm, int64_t *n_pairs, int32_t *n_cells);

/* Rebuilds the neighbour lists after a change of support radii with the
 * particles' positions unchanged. H_sorted[n]: new H in sorted order. */
crk_status crk_update_support(crk_ctx *ctx, const double *H_sorted, int64_t *n_pairs);

/* Moves ncomp arrays of n doubles between orders using the last build's
 * permutation: to_sorted != 0: dst[c][k] = src[c][perm[k]];
 * to_sorted == 0: dst[c][perm[k]] = src[c][k]. src and dst must not overlap. */
crk_status crk_permute(crk_ctx *ctx, const double *src, double *dst, int32_t ncomp,
                       int32_t to_sorted);

/*
 * S2 + S4: volume, eq. (vol), and kernel moments (sorted order, FP64 out).
 *   nsum[n] = n_i = sum_{j in N_g(i)} W(|d|, H_i) (self included),  V[n] = 1 / n_i
 *   m0[n] = sum V_j W,  m1[3][n] = sum V_j d W,  m2[6][n] = sum V_j d d^T W
 *   gm0[3][n], gm1[9][n], gm2[18][n]: their gradients in x_i with H_i and
 *   every V_j held fixed (d d / d x_i = I).
 * Any output pointer except V may be NULL when the call is only needed for the
 * volumes. The context also keeps V for the later passes. In FP64 and
 * adaptive precision the build (crk_build_cells, crk_update_support) has
 * already summed the FP64 volumes over its lists, and this call copies them
 * out; after crk_build_leaves, or in CRK_MIXED, it sums them itself.
 */
crk_status crk_moments(crk_ctx *ctx, const crk_params *p, double *nsum, double *V, double *m0,
                       double *m1, double *m2, double *gm0, double *gm1, double *gm2);

/*
 * S5: RK correction coefficients from the moments, always in FP64. With the
 * constraints sum V W^R = 1 and sum V d W^R = 0 of eq. (RK):
 *   B = -m2^{-1} m1,  A = 1 / (m0 + B.m1),
 *   dB/dx^g = -m2^{-1} (dm1/dx^g + (dm2/dx^g) B),
 *   dA/dx^g = -A^2 (dm0/dx^g + (dB/dx^g).m1 + B.dm1/dx^g).
 * When det(m2) <= 1e-12 (tr(m2)/3)^3 the particle falls back to normalised
 * SPH: A = 1/m0, B = 0, dA = -dm0/m0^2, dB = 0.
 * Out: A[n], B[3][n], gA[3][n], gB[9][n]; *n_singular (host, may be NULL:
 * then the call does not synchronise). Returns CRK_WARN_SINGULAR when
 * n_singular is requested and positive.
 */
crk_status crk_corrections(crk_ctx *ctx, int64_t n, const double *m0, const double *m1,
                           const double *m2, const double *gm0, const double *gm1,
                           const double *gm2, double *A, double *B, double *gA, double *gB,
                           int64_t *n_singular);

/*
 * S6 + S7: velocity gradient, then momentum and energy derivatives.
 *   gradv[9][n]: grad v_i = - sum_{j in N_g(i)} V_j (v_i - v_j) (x) grad W^R_ij, eq. (gradv)
 *   dpdt[3][n] : dp_i/dt = (1/m_i) sum_{j in N_s(i)} (a^2/2) V_i V_j (P_i+Q_i+P_j+Q_j)
 *                (grad W^R_ji - grad W^R_ij), eq. (mom); p = a v, so this is dv/dt at a = 1
 *   dudt[n]    : du_i/dt = (1/m_i) sum (1/(2a^2)) V_i V_j (P_j+Q_j) (xdot_j - xdot_i).
 *                (grad W^R_ji - grad W^R_ij), eq. (eng), xdot = v / a
 * with P = (gamma-1) rho u, Q from eqs. (visc), (mu) on the midpoint-projected
 * velocities of eq. (hatvi) and the limiter of eqs. (phi)-(phiad).
 * grad W^R_ij is eq. (gRK) with i's coefficients and H_i (zero for |d| >= H_i);
 * grad W^R_ji is the same with j's coefficients, H_j and d -> -d.
 * In: v[3][n] (peculiar velocity), m[n], u[n], rho[n] (NULL: rho = m / V), V[n],
 *     A, B, gA, gB as returned by crk_corrections.
 */
crk_status crk_derivatives(crk_ctx *ctx, const crk_params *p, const double *v, const double *m,
                           const double *u, const double *rho, const double *V, const double *A,
                           const double *B, const double *gA, const double *gB, double *gradv,
                           double *dpdt, double *dudt);

/*
 * Time-step terms of the Courant criterion (Sec. 3.1; an extension beyond
 * the pair passes). crk_set_timestep(ctx, 1) makes every later
 * crk_derivatives call (and a step recorded after it) also keep, per
 * particle, the largest closing speed over its pair set, max_j max(-w_ij, 0)
 * with w_ij = (xdot_ij + (adot/a) x_ij).x_ij / |x_ij| and xdot = v / a, and
 * the largest Q_i / rho_i over its pairs (Q_i the pair's viscous pressure of
 * eq. (visc)); 0 turns it off. crk_timestep then forms, in sorted order,
 *   c_s = sqrt(gamma P / rho), c_sq = sqrt(zeta max Q_i / rho_i),
 *   |div u| = |Tr grad v + 3 adot|, h_hat = H / n_h,
 *   v_max = max(v_sig, c_s, c_sq, h_hat |div u| / a),
 *   dt_hyd = C_CFL h_hat / v_max   (in time: the caller applies dy/dt),
 * with the paper's zeta = 4 and C_CFL = 0.25 passed in. u, m, rho (NULL:
 * rho = m/V), V and gradv are the arrays the derivative call used (gradv as
 * it returned). vsig, csq and dt_hyd may be NULL; vmax may not. The
 * acceleration criterion needs gravity and is not computed.
 * Errors: CRK_ERR_STATE when the last crk_derivatives ran without the terms.
 */
crk_status crk_set_timestep(crk_ctx *ctx, int32_t on);
crk_status crk_timestep(crk_ctx *ctx, const crk_params *p, const double *u, const double *m,
                        const double *rho, const double *V, const double *gradv, double zeta,
                        double c_cfl, double *vsig, double *csq, double *vmax, double *dt_hyd);

/*
 * Compatible energy update over one time step dt (eqs. compEng, compEng2,
 * Eij, ptdt, fij; an extension beyond the pair passes). After
 * crk_derivatives, with the same lists and the same state arrays (v, m, u,
 * rho, V, A, B, gA, gB, and gradv and dpdt as that call returned), writes
 * in sorted order
 *   du[i] = dt sum_{j in N_s(i)} f_ij c_ij / (2 a^4)
 *           - dt (adot/a)(3(gamma-1)+2) u_i,
 *   c_ij = (p_j + p'_j - p_i - p'_i).dp_ij/dt,  p = a v,  p' = p + dt dp/dt,
 * (p = pk instead when pk is not NULL: the momenta a kick starts from, as in
 * a velocity-Verlet half step, while the pair forces stay those of the
 * state v; [3][n] sorted),
 * where dp_ij/dt is the pair's term of eq. (mom) with P -> P+Q (recomputed
 * pair by pair, with the same limiter and viscosity as crk_derivatives) and
 * f_ij is the entropy partition of eq. (fij), s = P / rho^gamma: the pair's
 * energy Delta E_ij = m_i c_ij / (2 a^4) goes to i in the share s_j/(s_i+s_j)
 * when Delta E_ij >= 0 and s_i/(s_i+s_j) otherwise, so that f_ij + f_ji = 1
 * and sum_i m_i du_i plus the kinetic change sum_i m_i (|p'_i|^2 - |p_i|^2) /
 * (2 a^4) is the expansion term alone. The last term is the comoving
 * energy equation's expansion term over dt, with that equation's sign.
 * Precision as crk_derivatives (p->precision; the adaptive mode sums the
 * pairs of flagged rows in FP64). Every pointer is a DEVICE array; du[n] is
 * written. Synchronises the stream.
 * Errors: CRK_ERR_INVALID_ARG (NULL, bad parameter, non-finite dt),
 * CRK_ERR_STATE (no build, or called while a step is being recorded),
 * CRK_ERR_NONFINITE (non-finite or non-positive gas state).
 */
crk_status crk_compatible_energy(crk_ctx *ctx, const crk_params *p, const double *v,
                                 const double *m, const double *u, const double *rho,
                                 const double *V, const double *A, const double *B,
                                 const double *gA, const double *gB, const double *gradv,
                                 const double *dpdt, const double *pk, double dt, double *du);

/*
 * Hierarchical time-step levels of the time integrator (Sec. 3.1), per
 * particle in sorted order, from the Courant time dt_hyd (crk_timestep, in
 * time units) and dpdt of the derivative pass:
 *   dt_acc = sqrt(min(h_hat, r_soft) / |a_hyd|), a_hyd = dp/dt / a^2, the
 *            hydrodynamic part of the acceleration (gravity is not part of
 *            this library); infinite where it vanishes;
 *   dt_min = min(dt_hyd, dt_acc);
 *   level  = the smallest l >= 0 with dt_min > dt_sub / 2^l, where dt_sub is
 *            the subcycle length in time units; particles that need a level
 *            above l_max (0..60) get l_max + 1 and are counted in *n_over.
 * h_hat = H / n_h from the last build. dt_acc and dt_min may be NULL. Per
 * particle only: the paper's grouping of the levels by tree leaf and its
 * limiter between neighbouring leaves are not applied. Synchronises.
 * Errors: CRK_ERR_INVALID_ARG (NULL, r_soft or dt_sub not positive, l_max
 * out of range), CRK_ERR_STATE (no build).
 */
crk_status crk_time_levels(crk_ctx *ctx, const crk_params *p, const double *dt_hyd,
                           const double *dpdt, double r_soft, double dt_sub, int32_t l_max,
                           double *dt_acc, double *dt_min, int32_t *level, int64_t *n_over);

/*
 * One whole step: S1 build (all boxes of a batch), S2 volumes, S4 moments,
 * S5 corrections, S6 velocity gradient and S7 derivatives, i.e. the calls
 * crk_build_cells_batch, crk_moments, crk_corrections, crk_derivatives in
 * that order (Sec. 3.3: one interaction list per step, reused by every pass).
 * Inputs are in the original particle order, outputs in the sorted order;
 * every pointer is a caller-owned DEVICE array. rho may be NULL (rho = m/V);
 * every other member must be set.
 */
typedef struct {
    const double *x, *y, *z, *H; /* [n] positions in [0, L), support radii   */
    const double *v;             /* [3][n] peculiar velocity                  */
    const double *m, *u;         /* [n] masses, specific internal energies    */
    const double *rho;           /* [n] densities or NULL                     */
    int32_t *perm;               /* [n] sorted k -> original index            */
    double *V;                   /* [n] volumes                               */
    double *m0, *m1, *m2, *gm0, *gm1, *gm2; /* as crk_moments                 */
    double *A, *B, *gA, *gB;     /* as crk_corrections                        */
    double *gradv, *dpdt, *dudt; /* as crk_derivatives                        */
} crk_step_io;

/* The step, eagerly. box_offsets: HOST int64 [nboxes+1] as in
 * crk_build_cells_batch. *n_pairs, *n_singular: host, may be NULL.
 * Synchronises the stream. Returns CRK_WARN_SINGULAR as crk_corrections. */
crk_status crk_step(crk_ctx *ctx, int32_t nboxes, const int64_t *box_offsets, int64_t n,
                    const crk_step_io *io, const crk_params *p, double cell_size,
                    int64_t *n_pairs, int64_t *n_singular);

/*
 * Velocity-Verlet hydro step, eq. (verletOP) (an extension beyond the pair
 * passes). With p = a v, D = (dp/dt, du/dt) of crk_derivatives and the time
 * step dt = (dt/dy) Delta y (a and adot held over the step):
 *   p^1/2 = p + dt/2 dp/dt(0),   u^1/2 = u + dt/2 du/dt(0),
 *   x^1   = x + p^1/2 dt / a^2   (wrapped once into [0, L)),
 *   p_p   = p^1/2 + dt/2 dp/dt(0), u_p = u^1/2 + dt/2 du/dt(0),
 *   D(1)  = the whole step (crk_step) at (x^1, p_p / a, u_p) with H, m, rho,
 *   p^1   = p^1/2 + dt/2 dp/dt(1), u^1 = u^1/2 + dt/2 du/dt(1).
 * energy = 0 uses du/dt of eq. (eng) as above. energy = 1 takes each half
 * kick's energy change from the compatible update instead (as
 * crk_compatible_energy over dt/2, with the pair forces of the evaluation the
 * kick uses and the momenta the kick starts from): the closing kick from
 * p^1/2, and the next step's opening kick from p^1, whose change is returned
 * as the rate dudt = Delta u / (dt/2) (so the next step must use the same dt
 * for the balance to be exact); with start_eval the first opening kick's
 * change is computed the same way. Energy is then conserved to rounding
 * (adot = 0). dt must not be 0 in this mode.
 * Every array is a caller-owned DEVICE array in the caller's particle order;
 * x, y, z, v, u are advanced in place. dpdt/dudt hold D at the start state
 * on entry (start_eval = 0; with start_eval = 1 the library evaluates it
 * first) and D at the end state on return, ready for the next step. The
 * products and sums of the kicks and the drift are rounded one by one (no
 * fused multiply-add). box_offsets: HOST int64 [nboxes+1] as in
 * crk_build_cells_batch. *n_pairs (host, may be NULL): pairs of the end
 * evaluation. Synchronises the stream. Errors: those of crk_step (a particle
 * that moves more than L in one step fails its position check) and of
 * crk_compatible_energy (energy = 1), CRK_ERR_INVALID_ARG for a bad energy
 * mode or dt, and CRK_ERR_STATE while a step is being recorded. After an
 * error raised past the drift the state arrays are partly advanced and not
 * valid; restart from a saved state.
 */
typedef struct {
    double *x, *y, *z;    /* [n] in/out positions in [0, L)                    */
    const double *H;      /* [n] support radii, held over the step              */
    double *v;            /* [3][n] in/out peculiar velocity (p = a v)          */
    const double *m;      /* [n] masses                                         */
    double *u;            /* [n] in/out specific internal energies              */
    const double *rho;    /* [n] densities or NULL (rho = m / V at evaluation)  */
    double *dpdt, *dudt;  /* [3][n], [n] in/out: D at the start / at the end     */
} crk_verlet_io;

crk_status crk_verlet_step(crk_ctx *ctx, int32_t nboxes, const int64_t *box_offsets, int64_t n,
                           const crk_verlet_io *io, const crk_params *p, double cell_size,
                           double dt, int32_t start_eval, int32_t energy, int64_t *n_pairs);

/* Device-side status of a replayed step (filled by crk_graph_replay). */
typedef struct {
    int64_t n_pairs;        /* ordered pairs of the replayed lists           */
    int64_t n_singular;     /* particles on the singular-m2 fallback         */
    int64_t n_fp64_rows;    /* CRK_MIXED_ADAPT: particles over kappa_max     */
    int64_t n_touched_rows; /* CRK_MIXED_ADAPT: particles with an FP64 pair  */
    int32_t input_error;    /* bit 0 non-finite, 1 outside [0, L), 2 H <= 0, 3 H >= L/2 */
    int32_t overflow;       /* 1: lists outgrew the recorded capacity        */
    int32_t state_error;    /* 1: non-finite or non-positive gas state       */
    int32_t reserved;
} crk_graph_status;

/*
 * S10: record the step once as a HIP graph, then replay it.
 * crk_graph_capture runs the step eagerly (checks the input, fixes the cell
 * geometry: box layout, L and the finest cell side), sizes the neighbour
 * lists at (1 + headroom) times the measured counts plus 1024, runs the
 * graph form of the step once, and records it (on a stream of its own, so
 * the context's stream may be the null stream). The outputs then hold the
 * step's results. The graph keeps every pointer of *io and every value of *p
 * and box_offsets: a replay re-reads the same input arrays (update them in
 * place between replays) and rewrites the same outputs; n and the boxes are
 * fixed. crk_graph_replay launches the graph on the context's stream; with
 * st == NULL it returns at once (no synchronisation), else it waits, fills
 * *st and returns: CRK_ERR_NONFINITE / CRK_ERR_INVALID_ARG / CRK_ERR_SUPPORT
 * for invalid positions or H (the offending particles were moved to stand-in
 * points with a vanishing support, so the replay itself stays in bounds),
 * CRK_ERR_CAPACITY when the lists outgrew the capacity (every row was
 * emptied; capture again), CRK_ERR_NONFINITE for a bad gas state,
 * CRK_WARN_SINGULAR as crk_corrections. On any error the outputs are not
 * valid. A workspace reallocation by a later call (e.g. a larger build on
 * the same context) discards the graph (replay then gives CRK_ERR_STATE).
 * One recorded step per context; crk_graph_destroy releases it.
 */
crk_status crk_graph_capture(crk_ctx *ctx, int32_t nboxes, const int64_t *box_offsets, int64_t n,
                             const crk_step_io *io, const crk_params *p, double cell_size,
                             double headroom);
crk_status crk_graph_replay(crk_ctx *ctx, crk_graph_status *st);
crk_status crk_graph_destroy(crk_ctx *ctx);

/*
 * S3: smoothing-length iteration, eqs. (hi), (thacker). For each particle on
 * its own (its neighbour count depends only on its own H):
 *   N = (4 pi/3) H^3 sum_j W(|d|, H),  Delta = (Nres / N)^(1/3),
 *   lambda = 0.2 (1 + Delta^2) if Delta < 1 else 0.2 (1 + Delta^-3),
 *   H <- H (1 - lambda + lambda Delta),
 * until |H_new - H_old| <= tol H_old or max_iter updates.
 * H_inout[n] (sorted order): start values in, converged values out.
 * iters[n] (int32, may be NULL): updates taken. *n_unconverged (host, may be
 * NULL). Uses the positions and cells of the last crk_build_cells; call
 * crk_update_support afterwards to rebuild the lists for the new H.
 * Errors: CRK_ERR_SUPPORT if an iterate reaches L/2; CRK_ERR_INVALID_ARG if
 * Nres <= 20.625 (the self term alone gives N = (4 pi/3)(495/(32 pi))).
 * The iteration runs in rounds of a few updates per particle; particles that
 * have stopped are compacted out between rounds, so the time follows the
 * total number of updates rather than the slowest particle of a wavefront;
 * when few particles remain each gets more lanes (up to a wavefront).
 * Each update sums W over a candidate row (the distances of every j within
 * a radius above H, rebuilt when H leaves it). A particle whose row does not
 * fit its slots is moved to a wide pass with a wavefront per particle and
 * rows of max(4096, 8 cap) slots (as many particles per launch as 8 GiB of
 * rows hold; that pool, sized to the particles it serves, is part of the
 * context workspace).
 */
crk_status crk_hsolve(crk_ctx *ctx, double Nres, double tol, int32_t max_iter, double *H_inout,
                      int32_t *iters, int64_t *n_unconverged);

/*
 * S9: smoothing-length network (an addition to the paper's method: a learned
 * starting value for the iteration of eq. (thacker); the iteration alone
 * decides the converged H). An 8 -> 64 -> 64 -> 1 MLP, exact-erf GELU, FP32:
 *   z1 = W1 f + b1, a1 = gelu(z1), z2 = W2 a1 + b2, a2 = gelu(z2), y = w3.a2 + b3,
 * y = ln(H_conv / H_prev). theta[4801] (device, float) holds W1 [64][8]
 * (row-major), b1 [64], W2 [64][64], b2 [64], w3 [64], b3.
 * Features (crk_hnet_features), feat[8][n] float, sorted order, at radius
 * H = H_sorted[i], with N_w(h) = (4 pi/3) h^3 sum_{r<h} W(r, h) (eq. hi) and
 * n_raw(h) = #{j : r < h} (self included in both):
 *   f0 = ln(N_w(H)/Nres)   f1 = (Nres/N_w(H))^(1/3) - 1   f2 = ln(8 N_w(H/2)/Nres)
 *   f3 = ln(64 N_w(H/4)/Nres)   f4 = ln(n_raw(H)/Nres)   f5 = ln(8 n_raw(H/2)/Nres)
 *   f6 = ln(H n^(1/3) / L)      f7 = 1
 * A particle whose H_sorted[i] is the support of the last crk_build_cells /
 * crk_update_support (lists not made stale since) takes its candidates from
 * its gather row; any other walks the cells (same values up to summation
 * order).
 * crk_hnet_forward: y[nb] for feat[8][nb]. crk_hnet_train_step: one step of
 * mean-squared-error training on a batch (feat[8][nb], target[nb]): the batch
 * gradient (reduced in a fixed order, so deterministic) goes to grad[4801]
 * if non-NULL, and when lr > 0 one bias-corrected Adam step (0.9, 0.999,
 * 1e-8; step counts from 1) updates theta, adam_m, adam_v in place;
 * *loss (host, may be NULL: no synchronisation) receives the batch loss at
 * the incoming theta. crk_hnet_seed: H_seed = H_prev exp(y) on the last
 * build's particles, clamped to [H_prev/8, 8 H_prev] and below L/2 (a
 * non-finite y keeps H_prev); H_prev and H_seed are sorted-order doubles.
 */
crk_status crk_hnet_features(crk_ctx *ctx, double Nres, const double *H_sorted, float *feat);
crk_status crk_hnet_forward(crk_ctx *ctx, const float *theta, const float *feat, int64_t nb,
                            float *y);
crk_status crk_hnet_train_step(crk_ctx *ctx, float *theta, float *adam_m, float *adam_v,
                               int64_t step, float lr, const float *feat, const float *target,
                               int64_t nb, float *grad, float *loss);
crk_status crk_hnet_seed(crk_ctx *ctx, const float *theta, double Nres, const double *H_prev,
                         double *H_seed);
/*
 * Allocation-free variant of crk_hnet_train_step, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight training
 * loops, harnesses that forbid hipMalloc. Same kernels, same arguments and
 * results (bit-identical theta, adam_m, adam_v, grad and loss), except:
 *   - loss (may be NULL) is a DEVICE float[1], written on the stream (no
 *     synchronisation);
 *   - nb is at most 8192: the per-tile partial gradients live in a static
 *     device array of 9.8 MB that each GPU holds until the process ends, not
 *     in the context workspace; larger batches return CRK_ERR_INVALID_ARG;
 *   - the call never allocates or frees (no hipMalloc, hipFree or allocating
 *     library routine) and never synchronises.
 * Every call on one GPU shares that GPU's static array: calls that overlap on
 * one GPU (other streams or host threads) race and must be serialised by the
 * caller. Errors: CRK_ERR_INVALID_ARG (NULL theta/feat/target, nb < 1 or
 * above 8192, lr > 0 without adam_m/adam_v or with step < 1), CRK_ERR_STATE
 * (the array's device address was not set up by crk_create).
 */
crk_status crk_hnet_train_step_noalloc(crk_ctx *ctx, float *theta, float *adam_m, float *adam_v,
                                       int64_t step, float lr, const float *feat,
                                       const float *target, int64_t nb, float *grad, float *loss);
/* Training targets target[i] = ln(H_conv[i] / H_prev[i]) (float) for n particles. */
crk_status crk_hnet_targets(crk_ctx *ctx, int64_t n, const double *H_prev, const double *H_conv,
                            float *target);

/*
 * Neighbour lists of the last build, for checking: which = 0 gives N_g
 * (self included), which = 1 gives N_s. offsets[n+1] (device int64) and
 * idx[cap] (device int32, SORTED-order indices). Rows are not ordered.
 * *total (host) receives the number of entries; idx may be NULL to query it.
 */
crk_status crk_export_neighbors(crk_ctx *ctx, int32_t which, int64_t *offsets, int32_t *idx,
                                int64_t cap, int64_t *total);

/* Thread mapping of the volume, moment, velocity-gradient and derivative
 * (with the compatible-energy) passes: 4, 8, 16 or 32 particles per
 * wavefront (default 8 for the derivative pass, 0 for the others), whose
 * 64 lanes are split among them in proportion
 * to their row lengths (each lane strides over its particle's row; the
 * lanes of a particle are summed in FP64 at the end, so the wavefront's
 * lanes stay busy however uneven the rows are); 0: the lanes-per-particle
 * mapping of crk_set_lanes (the compatible pass then keeps 8); -1 keeps the
 * current value. Tuning only: results agree to rounding for every choice. */
crk_status crk_set_wave_mapping(crk_ctx *ctx, int32_t vol_ppw, int32_t mom_ppw, int32_t grad_ppw,
                                int32_t deriv_ppw);

/* Lanes per particle of the four pair passes (volume, moments, velocity
 * gradient, derivatives): each particle's neighbour row is split over a
 * group of g lanes of one wavefront, g a power of two in 1..64; 0 keeps the
 * current value. Tuning only: results agree to rounding for every g. */
crk_status crk_set_lanes(crk_ctx *ctx, int32_t g_vol, int32_t g_mom, int32_t g_grad,
                         int32_t g_der);

/* Tuning of crk_hsolve (results do not depend on it beyond rounding; 0 keeps
 * a value): lanes per particle (a power of two <= 64), updates per round, and
 * the candidate rows: every j within factor * H of i (membership decided on
 * the exact FP64 r^2), stored as FP64 distances in rows of cap slots, built
 * again whenever H leaves the row (cap = -1: no rows, every update walks the
 * cells). Defaults 16, 12, 320, 1.15 (12 updates per round measured 2-6%
 * faster than 8 on 128^3 and 256^3 clustered sets, and than 16 or more on
 * the smaller one). */
crk_status crk_set_hsolve(crk_ctx *ctx, int32_t lanes, int32_t round, int32_t cap,
                          double factor);

/* Neighbour walk of crk_build_cells / crk_update_support (tuning only: the
 * neighbour sets do not depend on it): lanes (1, 2, 4, 8 or 16) of a
 * wavefront share one particle's walk; each row is first written to a
 * scratch row of cap slots, and rows longer than cap are walked again into
 * place (0 keeps either value). After an eager build the next walk uses at
 * least 2.5 times that build's mean gather row and, where its longest gather
 * row was longer, that row plus an eighth, as far as n x slots stays within
 * 2^33 (multiples of 64, at most 1024 slots; so at 2^21 particles up to 8
 * GiB of rows, at 2^24 up to 32 GiB), so cap is a floor (default 192). level_shift s (0..3; -1 keeps) walks the
 * first hierarchy level whose cell side is at least 2^(s-1) H: larger cells
 * mean fewer cells and more candidates per particle. The order of a gather
 * row is the walk order, so it follows the walked level. */
crk_status crk_set_walk(crk_ctx *ctx, int32_t lanes, int32_t cap, int32_t level_shift);

/* Per-kernel timing (off by default). While enabled, every kernel launch of
 * the library is bracketed by a pair of HIP events recorded on the context's
 * stream (graph replays are not timed). crk_timing_read synchronises the
 * stream and returns the summed event time (ms) and the launch count for one
 * kernel name ("sort", "k_walk", "k_compact_rows", "k_walk_long",
 * "k_extra_rank", "k_volume", "k_moments", "k_corrections", "k_flag",
 * "k_pack", "k_gradv", "k_gradv_fix", "k_deriv", "k_deriv_fix", "k_hsolve",
 * ...); crk_timing_reset clears the sums. crk_timing_only limits the
 * events to one kernel name (NULL or "" times every kernel again), so a
 * caller can time one kernel inside a run without bracketing the others
 * (each pair of events costs a few microseconds of host and queue time). */
crk_status crk_timing_enable(crk_ctx *ctx, int32_t on);
crk_status crk_timing_only(crk_ctx *ctx, const char *kernel);
crk_status crk_timing_reset(crk_ctx *ctx);
crk_status crk_timing_read(crk_ctx *ctx, const char *kernel, double *total_ms, int64_t *launches);

/* Rows the last CRK_MIXED_ADAPT crk_derivatives call ran in FP64: particles
 * over kappa_max, and particles with such a partner (host values). */
crk_status crk_adaptive_rows(crk_ctx *ctx, int64_t *n_fp64_rows, int64_t *n_touched_rows);

/* Library version string. */
const char *crk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CRK_H */
