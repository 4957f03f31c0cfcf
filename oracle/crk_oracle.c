/*
 * CRKSPH neighbour passes: plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, obviously correct
 * reference that the GPU library is checked against. It shares no code,
 * header, table or helper with the GPU library, and the library never
 * links, loads or calls it. Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark use it.
 *
 * Every function is a direct evaluation of one equation of the paper
 * (Frontiere et al., "Simulating Hydrodynamics in Cosmology with CRK-HACC"):
 *   W, grad W .............. Wendland C4 kernel, eq. (C4), Sec. 2.2
 *   n_i, V_i ............... SPH number density and volume, eq. (vol)
 *   N_i, Thacker update .... eq. (hi), eq. (thacker), Sec. 3.6
 *   moments, A, B, dA, dB .. first-order RK kernel, eqs. (RK), (gRK); the
 *                            constraints sum V W^R = 1, sum V x W^R = 0
 *   grad v ................. eq. (gradv)
 *   dp/dt, du/dt ........... eqs. (mom), (eng) with P -> P + Q, eqs. (visc),
 *                            (mu), midpoint projection (hatvi), limiter
 *                            (phi), (phiVL), (rij), (phiad)
 *
 * Readings of points the paper leaves open (the support radius H is the
 * paper's h; the self pair is included in the gather sums; grad W^R_ji is
 * the gradient with respect to x_j; what is held fixed in grad m; the
 * singular-m2 fallback; the form of the van Leer limiter used when the
 * ratio r_ij is undefined) are stated at the functions that use them.
 *
 * Precision: FP64 throughout, built with -ffp-contract=off so every
 * expression rounds as written.
 *
 * Conventions: arrays are component-major, a vector field of n particles
 * is [3][n]. The symmetric m2 is stored (xx, xy, xz, yy, yz, zz).
 * gm1[a*3+g] = d m1^a / d x^g, gm2[s*3+g] = d m2^s / d x^g,
 * gB[a*3+g] = d B^a / d x^g, gradv[a*3+b] = d v^a / d x^b.
 * Separations are d = x_i - x_j (minimum image in a periodic box).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* threads the OpenMP loops of this oracle use */
int orc_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ */
/* Kernel, eq. (C4): W = 495/(32 pi H^3) (1-q)^6 (1 + 6q + 35q^2/3),   */
/* q = r/H, W = 0 for q >= 1.                                          */
/* ------------------------------------------------------------------ */
double orc_W(double r, double H)
{
    double q = r / H;
    if (q >= 1.0) return 0.0;
    double s = 1.0 - q;
    double s2 = s * s;
    double s6 = s2 * s2 * s2;
    return 495.0 / (32.0 * ORC_PI * H * H * H) * s6 * (1.0 + 6.0 * q + 35.0 / 3.0 * q * q);
}

/* dW/dr of eq. (C4). Differentiating (1-q)^6 (1 + 6q + 35q^2/3) in q gives
 * -(56/3) q (1 + 5q) (1-q)^5, so dW/dr = -(1155/(4 pi H^4)) q (1+5q) (1-q)^5. */
double orc_dWdr(double r, double H)
{
    double q = r / H;
    if (q >= 1.0) return 0.0;
    double s = 1.0 - q;
    double s5 = s * s * s * s * s;
    return -1155.0 / (4.0 * ORC_PI * H * H * H * H) * q * (1.0 + 5.0 * q) * s5;
}

/* grad_i W(|x_i - x_j|, H) = dW/dr * d / r. The factor q/r = 1/H removes
 * the 1/r, so the gradient is finite (zero) at r = 0. */
static void orc_gradW(const double d[3], double r, double H, double g[3])
{
    double q = r / H;
    if (q >= 1.0) { g[0] = g[1] = g[2] = 0.0; return; }
    double s = 1.0 - q;
    double s5 = s * s * s * s * s;
    double f = -1155.0 / (4.0 * ORC_PI * H * H * H * H * H) * (1.0 + 5.0 * q) * s5;
    g[0] = f * d[0];
    g[1] = f * d[1];
    g[2] = f * d[2];
}

/* vector form for tests: w[k] = W(r[k], H[k]), dwdr[k] = dW/dr */
void orc_kernel_eval(int64_t n, const double *r, const double *H, double *w, double *dwdr)
{
    for (int64_t k = 0; k < n; k++) {
        w[k] = orc_W(r[k], H[k]);
        dwdr[k] = orc_dWdr(r[k], H[k]);
    }
}

/* ------------------------------------------------------------------ */
/* Separation d = x_i - x_j. Periodic boxes use the minimum image: a    */
/* component beyond L/2 is shifted by one period. r^2 is summed as      */
/* (dx dx + dy dy) + dz dz, no fused multiply-add. Neighbour decisions  */
/* use exactly this value with a strict '<'.                           */
/* ------------------------------------------------------------------ */
static double orc_sep(const double *x, const double *y, const double *z, int64_t i, int64_t j,
                      double L, int periodic, double d[3])
{
    d[0] = x[i] - x[j];
    d[1] = y[i] - y[j];
    d[2] = z[i] - z[j];
    if (periodic) {
        double hL = 0.5 * L;
        for (int k = 0; k < 3; k++) {
            if (d[k] > hL) d[k] -= L;
            else if (d[k] < -hL) d[k] += L;
        }
    }
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

/* ------------------------------------------------------------------ */
/* Neighbour sets.                                                      */
/*   which = 0: gather set  N_g(i) = { j : r_ij < H_i }, self included   */
/*              (eq. (SPHdisc) and eq. (vol) sum over j with h_i).       */
/*   which = 1: pair set    N_s(i) = { j != i : r_ij < max(H_i, H_j) },  */
/*              every pair that appears in eq. (mom) for particle i.    */
/* Rows are ascending in j. Call with idx == NULL to get the offsets   */
/* and the total; then again with idx of that size.                    */
/* ------------------------------------------------------------------ */
int64_t orc_neighbors_brute(int64_t n, const double *x, const double *y, const double *z,
                            const double *H, double L, int periodic, int which,
                            int64_t *off, int32_t *idx)
{
    off[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t c = 0;
        for (int64_t j = 0; j < n; j++) {
            double d[3];
            double r2 = orc_sep(x, y, z, i, j, L, periodic, d);
            int in;
            if (which == 0) in = r2 < H[i] * H[i];
            else in = (j != i) && (r2 < H[i] * H[i] || r2 < H[j] * H[j]);
            if (in) {
                if (idx) idx[off[i] + c] = (int32_t)j;
                c++;
            }
        }
        off[i + 1] = off[i] + c;
    }
    return off[n];
}

/* Uniform periodic cell grid (a chaining mesh, Sec. 3.3) used to find the
 * same sets without the O(N^2) loop. The grid only restricts the candidate
 * j; every decision is the same r^2 < H^2 test as the brute-force path. */
typedef struct {
    int nc;                 /* cells per dimension */
    double c;               /* cell side */
    int64_t *start;         /* [nc^3 + 1] */
    int32_t *list;          /* particles, cell by cell, ascending index */
} orc_grid;

static int orc_cell_of(double x, double c, int nc)
{
    int k = (int)floor(x / c);
    if (k < 0) k = 0;
    if (k >= nc) k = nc - 1;
    return k;
}

static void orc_grid_build(orc_grid *g, int64_t n, const double *x, const double *y,
                           const double *z, const double *H, double L)
{
    /* cell side near the mean support radius, at most 128 cells a side;
     * the cell size only affects speed, never which pairs are found */
    double mean = 0.0;
    for (int64_t i = 0; i < n; i++) mean += H[i];
    mean /= (double)(n > 0 ? n : 1);
    int nc = (int)floor(L / mean);
    if (nc < 1) nc = 1;
    if (nc > 128) nc = 128;
    g->nc = nc;
    g->c = L / nc;
    int64_t ncell = (int64_t)nc * nc * nc;
    g->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    g->list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *cellof = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; i++) {
        int cx = orc_cell_of(x[i], g->c, nc), cy = orc_cell_of(y[i], g->c, nc),
            cz = orc_cell_of(z[i], g->c, nc);
        cellof[i] = ((int64_t)cz * nc + cy) * nc + cx;
        g->start[cellof[i] + 1]++;
    }
    for (int64_t k = 0; k < ncell; k++) g->start[k + 1] += g->start[k];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    memcpy(fill, g->start, sizeof(int64_t) * (size_t)ncell);
    for (int64_t i = 0; i < n; i++) g->list[fill[cellof[i]]++] = (int32_t)i;
    free(fill);
    free(cellof);
}

static void orc_grid_free(orc_grid *g)
{
    free(g->start);
    free(g->list);
}

/* Cell index range along one axis that holds every j within R of xi.
 * One extra cell on each side absorbs any rounding in the division; the
 * range is truncated to one full period. */
static void orc_axis_range(double xi, double R, const orc_grid *g, int *lo, int *cnt)
{
    int a = (int)floor((xi - R) / g->c) - 1;
    int b = (int)floor((xi + R) / g->c) + 1;
    int m = b - a + 1;
    if (m >= g->nc) { a = 0; m = g->nc; }
    *lo = a;
    *cnt = m;
}

static int orc_mod(int a, int n) { int r = a % n; return r < 0 ? r + n : r; }

/* Gather rows via the grid, each row sorted ascending. */
static int64_t orc_gather_grid(int64_t n, const double *x, const double *y, const double *z,
                               const double *H, double L, const orc_grid *g, int64_t *off,
                               int32_t **idx_out)
{
    int64_t *cnt = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    /* pass 1: counts */
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        int lx, ly, lz, mx, my, mz;
        orc_axis_range(x[i], H[i], g, &lx, &mx);
        orc_axis_range(y[i], H[i], g, &ly, &my);
        orc_axis_range(z[i], H[i], g, &lz, &mz);
        int64_t c = 0;
        for (int a = 0; a < mz; a++)
            for (int b = 0; b < my; b++)
                for (int e = 0; e < mx; e++) {
                    int64_t cell = ((int64_t)orc_mod(lz + a, g->nc) * g->nc + orc_mod(ly + b, g->nc)) * g->nc
                                   + orc_mod(lx + e, g->nc);
                    for (int64_t k = g->start[cell]; k < g->start[cell + 1]; k++) {
                        double d[3];
                        int64_t j = g->list[k];
                        if (orc_sep(x, y, z, i, j, L, 1, d) < H[i] * H[i]) c++;
                    }
                }
        cnt[i] = c;
    }
    off[0] = 0;
    for (int64_t i = 0; i < n; i++) off[i + 1] = off[i] + cnt[i];
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(off[n] > 0 ? off[n] : 1));
    /* pass 2: fill and sort each row */
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        int lx, ly, lz, mx, my, mz;
        orc_axis_range(x[i], H[i], g, &lx, &mx);
        orc_axis_range(y[i], H[i], g, &ly, &my);
        orc_axis_range(z[i], H[i], g, &lz, &mz);
        int64_t p = off[i];
        for (int a = 0; a < mz; a++)
            for (int b = 0; b < my; b++)
                for (int e = 0; e < mx; e++) {
                    int64_t cell = ((int64_t)orc_mod(lz + a, g->nc) * g->nc + orc_mod(ly + b, g->nc)) * g->nc
                                   + orc_mod(lx + e, g->nc);
                    for (int64_t k = g->start[cell]; k < g->start[cell + 1]; k++) {
                        double d[3];
                        int64_t j = g->list[k];
                        if (orc_sep(x, y, z, i, j, L, 1, d) < H[i] * H[i]) idx[p++] = (int32_t)j;
                    }
                }
        /* insertion sort of the row */
        for (int64_t s = off[i] + 1; s < off[i + 1]; s++) {
            int32_t v = idx[s];
            int64_t t = s - 1;
            while (t >= off[i] && idx[t] > v) { idx[t + 1] = idx[t]; t--; }
            idx[t + 1] = v;
        }
    }
    free(cnt);
    *idx_out = idx;
    return off[n];
}

/* Same sets as orc_neighbors_brute for a periodic box, found on a grid.
 * The pair set is the union of the gather row of i (without i) and the
 * transposed gather rows, { j : i in N_g(j) }, merged ascending. */
int64_t orc_neighbors_grid(int64_t n, const double *x, const double *y, const double *z,
                           const double *H, double L, int which, int64_t *off, int32_t *idx)
{
    orc_grid g;
    orc_grid_build(&g, n, x, y, z, H, L);
    int64_t *goff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *gidx = NULL;
    orc_gather_grid(n, x, y, z, H, L, &g, goff, &gidx);
    orc_grid_free(&g);
    if (which == 0) {
        memcpy(off, goff, sizeof(int64_t) * (size_t)(n + 1));
        if (idx) memcpy(idx, gidx, sizeof(int32_t) * (size_t)goff[n]);
        free(goff);
        free(gidx);
        return off[n];
    }
    /* transpose: T(j) collects every i != j with j in N_g(i), ascending i */
    int64_t *toff = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; i++)
        for (int64_t k = goff[i]; k < goff[i + 1]; k++)
            if (gidx[k] != i) toff[gidx[k] + 1]++;
    for (int64_t i = 0; i < n; i++) toff[i + 1] += toff[i];
    int32_t *tidx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(toff[n] > 0 ? toff[n] : 1));
    int64_t *tfill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    memcpy(tfill, toff, sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; i++)
        for (int64_t k = goff[i]; k < goff[i + 1]; k++)
            if (gidx[k] != i) tidx[tfill[gidx[k]]++] = (int32_t)i;
    free(tfill);
    /* merge the two ascending rows, dropping i itself and duplicates */
    off[0] = 0;
    for (int pass = 0; pass < 2; pass++) {
        for (int64_t i = 0; i < n; i++) {
            int64_t a = goff[i], ae = goff[i + 1], b = toff[i], be = toff[i + 1];
            int64_t c = 0;
            while (a < ae || b < be) {
                int32_t v;
                if (b >= be || (a < ae && gidx[a] < tidx[b])) v = gidx[a++];
                else if (a >= ae || tidx[b] < gidx[a]) v = tidx[b++];
                else { v = gidx[a++]; b++; }
                if (v == i) continue;
                if (pass == 1) idx[off[i] + c] = v;
                c++;
            }
            if (pass == 0) off[i + 1] = off[i] + c;
        }
        if (!idx) break;
    }
    free(goff);
    free(gidx);
    free(toff);
    free(tidx);
    return off[n];
}

/* ------------------------------------------------------------------ */
/* Volume, eq. (vol): n_i = sum_{j in N_g(i)} W(r_ij, H_i), V_i = 1/n_i; */
/* neighbour count, eq. (hi): N_i = (4 pi / 3) H_i^3 n_i.               */
/* Reading: the j = i term, W(0, H_i), is part of the sum.              */
/* ------------------------------------------------------------------ */
void orc_volume(int64_t n, const double *x, const double *y, const double *z, const double *H,
                double L, int periodic, const int64_t *goff, const int32_t *gidx,
                double *nsum, double *V, double *Ncount)
{
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t k = goff[i]; k < goff[i + 1]; k++) {
            double d[3];
            double r2 = orc_sep(x, y, z, i, gidx[k], L, periodic, d);
            s += orc_W(sqrt(r2), H[i]);
        }
        nsum[i] = s;
        V[i] = 1.0 / s;
        if (Ncount) Ncount[i] = 4.0 / 3.0 * ORC_PI * H[i] * H[i] * H[i] * s;
    }
}

/* n_i at an arbitrary support radius Hi, by scanning every particle
 * (tests and the h iteration on small sets). */
double orc_nsum_at(int64_t n, const double *x, const double *y, const double *z, double L,
                   int periodic, int64_t i, double Hi)
{
    double s = 0.0;
    for (int64_t j = 0; j < n; j++) {
        double d[3];
        double r2 = orc_sep(x, y, z, i, j, L, periodic, d);
        if (r2 < Hi * Hi) s += orc_W(sqrt(r2), Hi);
    }
    return s;
}

/* ------------------------------------------------------------------ */
/* Kernel moments over the gather set, with w = W(r_ij, H_i) and        */
/* g = grad_i W_ij:                                                     */
/*   m0 = sum V_j w,  m1^a = sum V_j d^a w,  m2^ab = sum V_j d^a d^b w,  */
/* and their gradients with respect to x_i, holding H_i and every V_j   */
/* fixed (d d^a / d x_i^g = delta_ag):                                  */
/*   dm0/dx^g    = sum V_j g^g                                         */
/*   dm1^a/dx^g  = sum V_j (delta_ag w + d^a g^g)                      */
/*   dm2^ab/dx^g = sum V_j (delta_ag d^b w + delta_bg d^a w + d^a d^b g^g) */
/* These are the sums the constraints of eq. (RK) are written in.       */
/* ------------------------------------------------------------------ */
static const int orc_sym[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

void orc_moments(int64_t n, const double *x, const double *y, const double *z, const double *H,
                 const double *V, double L, int periodic, const int64_t *goff, const int32_t *gidx,
                 double *m0, double *m1, double *m2, double *gm0, double *gm1, double *gm2)
{
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        double s0 = 0.0, s1[3] = {0}, s2[6] = {0}, sg0[3] = {0}, sg1[9] = {0}, sg2[18] = {0};
        for (int64_t k = goff[i]; k < goff[i + 1]; k++) {
            int64_t j = gidx[k];
            double d[3], g[3];
            double r2 = orc_sep(x, y, z, i, j, L, periodic, d);
            double r = sqrt(r2);
            double w = orc_W(r, H[i]);
            orc_gradW(d, r, H[i], g);
            double Vj = V[j];
            s0 += Vj * w;
            for (int a = 0; a < 3; a++) {
                s1[a] += Vj * d[a] * w;
                sg0[a] += Vj * g[a];
                for (int b = a; b < 3; b++) s2[orc_sym[a][b]] += Vj * d[a] * d[b] * w;
                for (int c = 0; c < 3; c++)
                    sg1[a * 3 + c] += Vj * ((a == c ? w : 0.0) + d[a] * g[c]);
            }
            for (int a = 0; a < 3; a++)
                for (int b = a; b < 3; b++)
                    for (int c = 0; c < 3; c++)
                        sg2[orc_sym[a][b] * 3 + c] +=
                            Vj * ((a == c ? d[b] * w : 0.0) + (b == c ? d[a] * w : 0.0) + d[a] * d[b] * g[c]);
        }
        m0[i] = s0;
        for (int a = 0; a < 3; a++) { m1[a * n + i] = s1[a]; gm0[a * n + i] = sg0[a]; }
        for (int s = 0; s < 6; s++) m2[s * n + i] = s2[s];
        for (int s = 0; s < 9; s++) gm1[s * n + i] = sg1[s];
        for (int s = 0; s < 18; s++) gm2[s * n + i] = sg2[s];
    }
}

/* ------------------------------------------------------------------ */
/* Correction coefficients of eq. (RK). The two constraints, written as */
/* particle sums, are  A (m0 + B.m1) = 1  and  A (m1 + m2 B) = 0, so    */
/*   B = -m2^{-1} m1,   A = 1 / (m0 + B.m1).                            */
/* Differentiating both identities in x_i^g:                            */
/*   dB/dx^g = -m2^{-1} (dm1/dx^g + (dm2/dx^g) B)                       */
/*   dA/dx^g = -A^2 (dm0/dx^g + (dB/dx^g).m1 + B.(dm1/dx^g)).           */
/* m2 is solved by a Cholesky factorisation. Reading for a singular m2  */
/* (coplanar or isolated particles, which the paper does not treat):    */
/* when the factorisation fails or det(m2) <= 1e-12 (tr m2 / 3)^3, fall */
/* back to normalised SPH, A = 1/m0, B = 0, dA = -dm0/m0^2, dB = 0.     */
/* Returns the number of particles that took the fallback.             */
/* ------------------------------------------------------------------ */
static int orc_chol3(const double M[3][3], double Lc[3][3])
{
    memset(Lc, 0, sizeof(double) * 9);
    for (int j = 0; j < 3; j++) {
        double s = M[j][j];
        for (int k = 0; k < j; k++) s -= Lc[j][k] * Lc[j][k];
        if (!(s > 0.0)) return 0;
        Lc[j][j] = sqrt(s);
        for (int i = j + 1; i < 3; i++) {
            double t = M[i][j];
            for (int k = 0; k < j; k++) t -= Lc[i][k] * Lc[j][k];
            Lc[i][j] = t / Lc[j][j];
        }
    }
    return 1;
}

static void orc_chol3_solve(const double Lc[3][3], const double b[3], double xo[3])
{
    double t[3];
    for (int i = 0; i < 3; i++) {
        double s = b[i];
        for (int k = 0; k < i; k++) s -= Lc[i][k] * t[k];
        t[i] = s / Lc[i][i];
    }
    for (int i = 2; i >= 0; i--) {
        double s = t[i];
        for (int k = i + 1; k < 3; k++) s -= Lc[k][i] * xo[k];
        xo[i] = s / Lc[i][i];
    }
}

int64_t orc_corrections(int64_t n, const double *m0, const double *m1, const double *m2,
                        const double *gm0, const double *gm1, const double *gm2,
                        double *A, double *B, double *gA, double *gB, int32_t *singular)
{
    int64_t nsing = 0;
    #pragma omp parallel for schedule(static) reduction(+ : nsing)
    for (int64_t i = 0; i < n; i++) {
        double M[3][3], Lc[3][3];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) M[a][b] = m2[orc_sym[a][b] * n + i];
        double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
                   - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
                   + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
        double tr = (M[0][0] + M[1][1] + M[2][2]) / 3.0;
        int ok = (det > 1e-12 * tr * tr * tr) && orc_chol3(M, Lc);
        double mm0 = m0[i];
        double mm1[3] = {m1[0 * n + i], m1[1 * n + i], m1[2 * n + i]};
        if (!ok) {
            A[i] = 1.0 / mm0;
            for (int a = 0; a < 3; a++) {
                B[a * n + i] = 0.0;
                gA[a * n + i] = -gm0[a * n + i] / (mm0 * mm0);
            }
            for (int s = 0; s < 9; s++) gB[s * n + i] = 0.0;
            if (singular) singular[i] = 1;
            nsing++;
            continue;
        }
        if (singular) singular[i] = 0;
        double Bv[3], rhs[3];
        orc_chol3_solve(Lc, mm1, Bv);
        for (int a = 0; a < 3; a++) Bv[a] = -Bv[a];
        double Av = 1.0 / (mm0 + (Bv[0] * mm1[0] + Bv[1] * mm1[1] + Bv[2] * mm1[2]));
        double dB[3][3]; /* dB[a][g] */
        for (int g = 0; g < 3; g++) {
            for (int a = 0; a < 3; a++) {
                double s = gm1[(a * 3 + g) * n + i];
                for (int b = 0; b < 3; b++) s += gm2[(orc_sym[a][b] * 3 + g) * n + i] * Bv[b];
                rhs[a] = s;
            }
            double sol[3];
            orc_chol3_solve(Lc, rhs, sol);
            for (int a = 0; a < 3; a++) dB[a][g] = -sol[a];
        }
        A[i] = Av;
        for (int a = 0; a < 3; a++) B[a * n + i] = Bv[a];
        for (int g = 0; g < 3; g++) {
            double s = gm0[g * n + i];
            for (int a = 0; a < 3; a++) s += dB[a][g] * mm1[a] + Bv[a] * gm1[(a * 3 + g) * n + i];
            gA[g * n + i] = -Av * Av * s;
        }
        for (int a = 0; a < 3; a++)
            for (int g = 0; g < 3; g++) gB[(a * 3 + g) * n + i] = dB[a][g];
    }
    return nsing;
}

/* ------------------------------------------------------------------ */
/* RK kernel, eq. (RK), and its gradient, eq. (gRK), for one ordered     */
/* pair, with the first particle's coefficients and support radius:      */
/*   W^R = A (1 + B.d) w                                                */
/*   grad W^R = gradA (1 + B.d) w + A ((gradB)^T d + B) w + A (1 + B.d) g */
/* where ((gradB)^T d)^g = sum_a d^a dB^a/dx^g. grad W^R_ji, used in      */
/* eq. (mom), is this template for particle j with d -> -d (the          */
/* gradient with respect to x_j).                                       */
/* ------------------------------------------------------------------ */
static void orc_rk(const double d[3], double r, double H, double Av, const double Bv[3],
                   const double gAv[3], const double gBv[9], double *WR, double GR[3])
{
    double w = orc_W(r, H), g[3];
    orc_gradW(d, r, H, g);
    double c = 1.0 + (Bv[0] * d[0] + Bv[1] * d[1] + Bv[2] * d[2]);
    if (WR) *WR = Av * c * w;
    for (int gg = 0; gg < 3; gg++) {
        double btd = d[0] * gBv[0 * 3 + gg] + d[1] * gBv[1 * 3 + gg] + d[2] * gBv[2 * 3 + gg];
        GR[gg] = gAv[gg] * c * w + Av * (btd + Bv[gg]) * w + Av * c * g[gg];
    }
}

static void orc_coeffs(int64_t n, int64_t i, const double *A, const double *B, const double *gA,
                       const double *gB, double *Av, double Bv[3], double gAv[3], double gBv[9])
{
    *Av = A[i];
    for (int a = 0; a < 3; a++) { Bv[a] = B[a * n + i]; gAv[a] = gA[a * n + i]; }
    for (int s = 0; s < 9; s++) gBv[s] = gB[s * n + i];
}

/* W^R_ij and grad W^R_ij (with i's coefficients and H_i) for a list of
 * ordered pairs; tests sum these to check the reproducing conditions. */
void orc_rk_pairs(int64_t n, const double *x, const double *y, const double *z, const double *H,
                  double L, int periodic, const double *A, const double *B, const double *gA,
                  const double *gB, int64_t npair, const int32_t *pi, const int32_t *pj,
                  double *WR, double *GR /* [3][npair] */, double *dout /* [3][npair] */)
{
    for (int64_t k = 0; k < npair; k++) {
        int64_t i = pi[k], j = pj[k];
        double d[3], Av, Bv[3], gAv[3], gBv[9], G[3];
        double r = sqrt(orc_sep(x, y, z, i, j, L, periodic, d));
        orc_coeffs(n, i, A, B, gA, gB, &Av, Bv, gAv, gBv);
        orc_rk(d, r, H[i], Av, Bv, gAv, gBv, &WR[k], G);
        for (int a = 0; a < 3; a++) { GR[a * npair + k] = G[a]; dout[a * npair + k] = d[a]; }
    }
}

/* ------------------------------------------------------------------ */
/* Velocity gradient, eq. (gradv):                                      */
/*   grad v_i^{ab} = - sum_{j in N_g(i)} V_j (v_i^a - v_j^a) (grad W^R_ij)^b */
/* ------------------------------------------------------------------ */
void orc_gradv(int64_t n, const double *x, const double *y, const double *z, const double *H,
               double L, int periodic, const double *v, const double *V, const double *A,
               const double *B, const double *gA, const double *gB, const int64_t *goff,
               const int32_t *gidx, double *gradv)
{
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        double Av, Bv[3], gAv[3], gBv[9], acc[9] = {0};
        orc_coeffs(n, i, A, B, gA, gB, &Av, Bv, gAv, gBv);
        for (int64_t k = goff[i]; k < goff[i + 1]; k++) {
            int64_t j = gidx[k];
            double d[3], G[3];
            double r = sqrt(orc_sep(x, y, z, i, j, L, periodic, d));
            orc_rk(d, r, H[i], Av, Bv, gAv, gBv, NULL, G);
            for (int a = 0; a < 3; a++) {
                double dv = v[a * n + i] - v[a * n + j];
                for (int b = 0; b < 3; b++) acc[a * 3 + b] -= V[j] * dv * G[b];
            }
        }
        for (int s = 0; s < 9; s++) gradv[s * n + i] = acc[s];
    }
}

/* ------------------------------------------------------------------ */
/* Limiter, eqs. (phi), (phiVL), (rij), (phiad).                        */
/* s_i = d.(grad v_i d) and s_j = d.(grad v_j d) are the numerator and  */
/* denominator of r_ij, with (grad v d)^a = sum_b grad v^{ab} d^b.       */
/* 4r/(1+r)^2 = 4 s_i s_j / (s_i + s_j)^2. Reading where r_ij is not     */
/* defined (s_j = 0) or is -1: use the second form, with phi_VL = 0     */
/* whenever s_i s_j <= 0; it agrees with the paper's max/min clamp      */
/* wherever r_ij is defined, and is symmetric under i <-> j.            */
/* phi_ad = exp(-((eta - eta_c)/eta_f)^2) for eta < eta_c, else 1, with  */
/* eta = min(r/H_i, r/H_j).                                             */
/* ------------------------------------------------------------------ */
double orc_limiter(double si, double sj, double eta, double eta_c, double eta_f)
{
    double vl;
    if (si * sj <= 0.0) vl = 0.0;
    else {
        double t = 4.0 * si * sj / ((si + sj) * (si + sj));
        vl = t < 1.0 ? t : 1.0;
    }
    double ad = 1.0;
    if (eta < eta_c) {
        double e = (eta - eta_c) / eta_f;
        ad = exp(-e * e);
    }
    return vl * ad;
}

/* Parameters of eqs. (EOS), (visc), (mu), (phiad), cosmology factors. */
typedef struct {
    double gamma, Cl, Cq, eps, nh, eta_c, eta_f, a, adot;
} orc_params;

/* ------------------------------------------------------------------ */
/* Momentum and energy derivatives, eqs. (mom) and (eng) with P -> P+Q. */
/* For every j in N_s(i):                                               */
/*   G_ij = grad W^R_ij (zero when r >= H_i), G_ji = grad W^R_ji (zero  */
/*   when r >= H_j), D = G_ji - G_ij;                                   */
/*   P = (gamma-1) rho u (eq. EOS), c_s = sqrt(gamma P / rho);          */
/*   phi from the limiter; projected velocities (eq. hatvi)             */
/*     u_hat = (v_i - phi/2 grad v_i d) - (v_j + phi/2 grad v_j d) + adot d */
/*   (the j side is v_j - phi/2 grad v_j x_ji with x_ji = -d, and the    */
/*   Hubble term is not projected);                                     */
/*   mu_k = min(0, (hh_k / a) (u_hat.d) / (r^2 + hh_k^2 eps^2)),         */
/*   hh_k = H_k / n_h, Q_k = rho_k (-Cl c_k mu_k + Cq mu_k^2), k = i, j; */
/*   F_i += (a^2/2) V_i V_j (P_i + Q_i + P_j + Q_j) D                    */
/*   E_i += (1/(2 a^2)) V_i V_j (P_j + Q_j) (xdot_j - xdot_i).D          */
/* with xdot = v / a (p = a v = a^2 xdot). Outputs dp_i/dt = F_i / m_i, */
/* du_i/dt = E_i / m_i, and the conditioning sums                       */
/*   SF_i = sum |(a^2/2) V_i V_j (P_i+Q_i+P_j+Q_j)| |D|,  SE_i = sum |E term|. */
/* rho == NULL means rho = m / V.                                       */
/* Time-step terms (Sec. 3.1, the signal velocity and viscous sound     */
/* speed of the Courant criterion), when VS / QR are non-NULL:          */
/*   w_ij = (xdot_ij + (adot/a) x_ij).x_ij / |x_ij|,                     */
/*   VS_i = max_j max(-w_ij, 0)  (the closing speed of approaching pairs),*/
/*   QR_i = max_j Q_i / rho_i    (Q_i of the pair, as above).            */
/* ------------------------------------------------------------------ */
/* The state every pair of N_s(i) reads (see orc_derivatives).         */
typedef struct {
    int64_t n;
    const double *x, *y, *z, *H;
    double L;
    int periodic;
    const double *v, *m, *u, *rho, *V, *A, *B, *gA, *gB, *gradv;
    orc_params p;
} orc_gas;

/* Particle i's own terms: RK coefficients, rho, P (eq. EOS), c_s.      */
typedef struct {
    int64_t i;
    double A, B[3], gA[3], gB[9], rho, P, c;
} orc_row;

static void orc_gas_init(orc_gas *g, int64_t n, const double *x, const double *y, const double *z,
                         const double *H, double L, int periodic, const double *v, const double *m,
                         const double *u, const double *rho, const double *V, const double *A,
                         const double *B, const double *gA, const double *gB, const double *gradv,
                         const double *prm)
{
    g->n = n; g->x = x; g->y = y; g->z = z; g->H = H; g->L = L; g->periodic = periodic;
    g->v = v; g->m = m; g->u = u; g->rho = rho; g->V = V;
    g->A = A; g->B = B; g->gA = gA; g->gB = gB; g->gradv = gradv;
    g->p.gamma = prm[0]; g->p.Cl = prm[1]; g->p.Cq = prm[2]; g->p.eps = prm[3]; g->p.nh = prm[4];
    g->p.eta_c = prm[5]; g->p.eta_f = prm[6]; g->p.a = prm[7]; g->p.adot = prm[8];
}

static void orc_row_init(const orc_gas *g, int64_t i, orc_row *ri)
{
    ri->i = i;
    orc_coeffs(g->n, i, g->A, g->B, g->gA, g->gB, &ri->A, ri->B, ri->gA, ri->gB);
    ri->rho = g->rho ? g->rho[i] : g->m[i] / g->V[i];
    ri->P = (g->p.gamma - 1.0) * ri->rho * g->u[i];
    ri->c = sqrt(g->p.gamma * ri->P / ri->rho);
}

/* The terms of one ordered pair (i, j), j in N_s(i):                   */
/*   F  = (a^2/2) V_i V_j (P_i+Q_i+P_j+Q_j) D  (= m_i dp_ij/dt, eq. mom),*/
/*   E  = (1/(2a^2)) V_i V_j (P_j+Q_j) (xdot_j - xdot_i).D  (eq. eng),   */
/*   sf = |(a^2/2) V_i V_j (P_i+Q_i+P_j+Q_j)| |D|,                        */
/*   w  = (xdot_ij + (adot/a) x_ij).x_ij / |x_ij|,  qr = Q_i / rho_i.     */
typedef struct {
    double F[3], E, sf, w, qr;
} orc_pair_terms;

static void orc_pair(const orc_gas *g, const orc_row *ri, int64_t j, orc_pair_terms *t)
{
    const int64_t n = g->n, i = ri->i;
    const double *v = g->v, *gradv = g->gradv, *H = g->H, *V = g->V;
    const orc_params p = g->p;
    double d[3], md[3], Gij[3] = {0, 0, 0}, Gji[3] = {0, 0, 0};
    double r2 = orc_sep(g->x, g->y, g->z, i, j, g->L, g->periodic, d);
    double r = sqrt(r2);
    md[0] = -d[0]; md[1] = -d[1]; md[2] = -d[2];
    if (r2 < H[i] * H[i]) orc_rk(d, r, H[i], ri->A, ri->B, ri->gA, ri->gB, NULL, Gij);
    if (r2 < H[j] * H[j]) {
        double Aj, Bj[3], gAj[3], gBj[9];
        orc_coeffs(n, j, g->A, g->B, g->gA, g->gB, &Aj, Bj, gAj, gBj);
        orc_rk(md, r, H[j], Aj, Bj, gAj, gBj, NULL, Gji);
    }
    double D[3] = {Gji[0] - Gij[0], Gji[1] - Gij[1], Gji[2] - Gij[2]};
    double rhoi = ri->rho, Pi = ri->P, ci = ri->c;
    double rhoj = g->rho ? g->rho[j] : g->m[j] / V[j];
    double Pj = (p.gamma - 1.0) * rhoj * g->u[j];
    double cj = sqrt(p.gamma * Pj / rhoj);
    /* limiter */
    double gvi_d[3], gvj_d[3];
    for (int a = 0; a < 3; a++) {
        gvi_d[a] = gradv[(a * 3 + 0) * n + i] * d[0] + gradv[(a * 3 + 1) * n + i] * d[1]
                 + gradv[(a * 3 + 2) * n + i] * d[2];
        gvj_d[a] = gradv[(a * 3 + 0) * n + j] * d[0] + gradv[(a * 3 + 1) * n + j] * d[1]
                 + gradv[(a * 3 + 2) * n + j] * d[2];
    }
    double si = d[0] * gvi_d[0] + d[1] * gvi_d[1] + d[2] * gvi_d[2];
    double sj = d[0] * gvj_d[0] + d[1] * gvj_d[1] + d[2] * gvj_d[2];
    double qi = r / H[i], qj = r / H[j];
    double eta = qi < qj ? qi : qj;
    double phi = orc_limiter(si, sj, eta, p.eta_c, p.eta_f);
    /* projected velocity difference, eq. (hatvi) */
    double uh[3];
    for (int a = 0; a < 3; a++)
        uh[a] = (v[a * n + i] - 0.5 * phi * gvi_d[a]) - (v[a * n + j] + 0.5 * phi * gvj_d[a])
                + p.adot * d[a];
    double ud = uh[0] * d[0] + uh[1] * d[1] + uh[2] * d[2];
    /* viscous pressures, eqs. (visc), (mu) */
    double hi = H[i] / p.nh, hj = H[j] / p.nh;
    double mui = (hi / p.a) * ud / (r2 + hi * hi * p.eps * p.eps);
    double muj = (hj / p.a) * ud / (r2 + hj * hj * p.eps * p.eps);
    if (mui > 0.0) mui = 0.0;
    if (muj > 0.0) muj = 0.0;
    double Qi = rhoi * (-p.Cl * ci * mui + p.Cq * mui * mui);
    double Qj = rhoj * (-p.Cl * cj * muj + p.Cq * muj * muj);
    /* eq. (mom), eq. (eng) */
    double fm = 0.5 * p.a * p.a * V[i] * V[j] * (Pi + Qi + Pj + Qj);
    double fe = 0.5 / (p.a * p.a) * V[i] * V[j] * (Pj + Qj);
    double xdd = ((v[0 * n + j] - v[0 * n + i]) * D[0] + (v[1 * n + j] - v[1 * n + i]) * D[1]
                  + (v[2 * n + j] - v[2 * n + i]) * D[2]) / p.a;
    for (int a = 0; a < 3; a++) t->F[a] = fm * D[a];
    t->E = fe * xdd;
    t->sf = fabs(fm) * sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    /* time-step terms */
    double xd[3];
    for (int a = 0; a < 3; a++)
        xd[a] = (v[a * n + i] - v[a * n + j]) / p.a + (p.adot / p.a) * d[a];
    t->w = (xd[0] * d[0] + xd[1] * d[1] + xd[2] * d[2]) / r;
    t->qr = Qi / rhoi;
}

void orc_derivatives(int64_t n, const double *x, const double *y, const double *z,
                     const double *H, double L, int periodic, const double *v, const double *m,
                     const double *u, const double *rho, const double *V, const double *A,
                     const double *B, const double *gA, const double *gB, const double *gradv,
                     const double *prm, const int64_t *soff, const int32_t *sidx,
                     double *dvdt, double *dudt, double *SF, double *SE, double *VS, double *QR)
{
    orc_gas g;
    orc_gas_init(&g, n, x, y, z, H, L, periodic, v, m, u, rho, V, A, B, gA, gB, gradv, prm);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        orc_row ri;
        orc_row_init(&g, i, &ri);
        double F[3] = {0, 0, 0}, E = 0.0, sf = 0.0, se = 0.0, vs = 0.0, qr = 0.0;
        for (int64_t k = soff[i]; k < soff[i + 1]; k++) {
            orc_pair_terms t;
            orc_pair(&g, &ri, sidx[k], &t);
            for (int a = 0; a < 3; a++) F[a] += t.F[a];
            E += t.E;
            sf += t.sf;
            se += fabs(t.E);
            if (-t.w > vs) vs = -t.w;
            if (t.qr > qr) qr = t.qr;
        }
        for (int a = 0; a < 3; a++) dvdt[a * n + i] = F[a] / m[i];
        dudt[i] = E / m[i];
        if (SF) SF[i] = sf;
        if (SE) SE[i] = se;
        if (VS) VS[i] = vs;
        if (QR) QR[i] = qr;
    }
}

/* ------------------------------------------------------------------ */
/* Compatible energy update over one time step dt, eqs. (compEng),      */
/* (compEng2), (Eij), (ptdt) and (fij), for every particle i:           */
/*   p = a v, p'_k = p_k + dt dp_k/dt (eq. ptdt; dp/dt as returned by    */
/*   orc_derivatives for the same state); when PK is given, p = PK is    */
/*   the momentum at the start of the kick instead (the pair forces stay */
/*   those of the state v: a kick that starts elsewhere, as in a         */
/*   velocity-Verlet half step);                                        */
/*   for every j in N_s(i): dp_ij/dt = F_ij / m_i, the pair's term of   */
/*   eq. (mom) with P -> P+Q, and                                       */
/*     c_ij = (p_j + p'_j - p_i - p'_i).dp_ij/dt;                       */
/*   Delta E_ij = m_i c_ij / (2 a^4): eq. (Eij) for any partition with  */
/*   f_ij + f_ji = 1, because m_i dp_ij/dt = -m_j dp_ji/dt;              */
/*   s = P / rho^gamma (thermal pressure of eq. EOS) and f_ij from the  */
/*   four cases of eq. (fij) on the sign of Delta E_ij;                 */
/*   Delta u_ij = f_ij c_ij / (2 a^4) (eq. compEng2);                    */
/*   Delta u_i = dt sum_j Delta u_ij - dt (adot/a) (3(gamma-1)+2) u_i.   */
/* The last term is the expansion term of the comoving energy equation  */
/* taken over dt, with that equation's sign.                            */
/* ------------------------------------------------------------------ */
void orc_compatible_energy(int64_t n, const double *x, const double *y, const double *z,
                           const double *H, double L, int periodic, const double *v,
                           const double *m, const double *u, const double *rho, const double *V,
                           const double *A, const double *B, const double *gA, const double *gB,
                           const double *gradv, const double *prm, const int64_t *soff,
                           const int32_t *sidx, const double *dpdt, const double *PK, double dt,
                           double *du)
{
    orc_gas g;
    orc_gas_init(&g, n, x, y, z, H, L, periodic, v, m, u, rho, V, A, B, gA, gB, gradv, prm);
    const double a = g.p.a, gam = g.p.gamma;
    const double a4 = a * a * a * a;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        orc_row ri;
        orc_row_init(&g, i, &ri);
        double s_i = ri.P / pow(ri.rho, gam);
        double pi[3], ppi[3];
        for (int c = 0; c < 3; c++) {
            pi[c] = PK ? PK[c * n + i] : a * v[c * n + i];
            ppi[c] = pi[c] + dt * dpdt[c * n + i];
        }
        double sum = 0.0;
        for (int64_t k = soff[i]; k < soff[i + 1]; k++) {
            int64_t j = sidx[k];
            orc_pair_terms t;
            orc_pair(&g, &ri, j, &t);
            double rhoj = rho ? rho[j] : m[j] / V[j];
            double s_j = (gam - 1.0) * rhoj * u[j] / pow(rhoj, gam);
            double cij = 0.0;
            for (int c = 0; c < 3; c++) {
                double pj = PK ? PK[c * n + j] : a * v[c * n + j];
                double ppj = pj + dt * dpdt[c * n + j];
                cij += (pj + ppj - pi[c] - ppi[c]) * (t.F[c] / m[i]);
            }
            double dE = m[i] * cij / (2.0 * a4);
            double smin = s_i < s_j ? s_i : s_j, smax = s_i < s_j ? s_j : s_i;
            double f;
            if ((dE >= 0.0 && s_i >= s_j) || (dE < 0.0 && s_i < s_j)) f = smin / (s_i + s_j);
            else f = smax / (s_i + s_j);
            sum += f * cij / (2.0 * a4);
        }
        du[i] = dt * sum - dt * (g.p.adot / a) * (3.0 * (gam - 1.0) + 2.0) * u[i];
    }
}

/* ------------------------------------------------------------------ */
/* Smoothing-length iteration, eqs. (hi) and (thacker): per particle,   */
/*   N_i = (4 pi/3) H^3 n_i(H),  Delta^3 = N_res / N_i,                 */
/*   lambda = 0.2 (1 + Delta^2) if Delta < 1, else 0.2 (1 + Delta^-3),  */
/*   H <- H (1 - lambda + lambda Delta),                                */
/* repeated until |H_new - H| <= tol H or max_iter updates. n_i(H) is  */
/* recomputed from the positions at every step (each particle's sum     */
/* depends only on its own H). Returns the number not converged.       */
/* ------------------------------------------------------------------ */
double orc_thacker_step(double H, double N, double Nres)
{
    double Delta = cbrt(Nres / N);
    double lam = Delta < 1.0 ? 0.2 * (1.0 + Delta * Delta) : 0.2 * (1.0 + 1.0 / (Delta * Delta * Delta));
    return H * (1.0 - lam + lam * Delta);
}

int64_t orc_hsolve(int64_t n, const double *x, const double *y, const double *z, double L,
                   int periodic, double Nres, double tol, int max_iter, double *H, int32_t *iters)
{
    orc_grid g;
    int use_grid = periodic && n > 4096;
    if (use_grid) orc_grid_build(&g, n, x, y, z, H, L);
    int64_t nfail = 0;
    #pragma omp parallel for schedule(dynamic, 16) reduction(+ : nfail)
    for (int64_t i = 0; i < n; i++) {
        double h = H[i];
        int it = 0, conv = 0;
        while (it < max_iter) {
            double s = 0.0;
            if (use_grid) {
                int lx, ly, lz, mx, my, mz;
                orc_axis_range(x[i], h, &g, &lx, &mx);
                orc_axis_range(y[i], h, &g, &ly, &my);
                orc_axis_range(z[i], h, &g, &lz, &mz);
                for (int a = 0; a < mz; a++)
                    for (int b = 0; b < my; b++)
                        for (int e = 0; e < mx; e++) {
                            int64_t cell = ((int64_t)orc_mod(lz + a, g.nc) * g.nc + orc_mod(ly + b, g.nc)) * g.nc
                                           + orc_mod(lx + e, g.nc);
                            for (int64_t k = g.start[cell]; k < g.start[cell + 1]; k++) {
                                double d[3];
                                double r2 = orc_sep(x, y, z, i, g.list[k], L, 1, d);
                                if (r2 < h * h) s += orc_W(sqrt(r2), h);
                            }
                        }
            } else {
                s = orc_nsum_at(n, x, y, z, L, periodic, i, h);
            }
            double N = 4.0 / 3.0 * ORC_PI * h * h * h * s;
            double hn = orc_thacker_step(h, N, Nres);
            it++;
            double dh = fabs(hn - h);
            double hold = h;
            h = hn;
            if (dh <= tol * hold) { conv = 1; break; }
        }
        H[i] = h;
        if (iters) iters[i] = it;
        if (!conv) nfail++;
    }
    if (use_grid) orc_grid_free(&g);
    return nfail;
}

/* ------------------------------------------------------------------ */
/* Input features of the smoothing-length network (not in the paper;   */
/* they feed a learned starting value for the iteration of eq. thacker).*/
/* From one pass over the support of radius H = H_i, with              */
/* N_w(h) = (4 pi / 3) h^3 sum_{r < h} W(r, h) (eq. hi, self included)  */
/* and n_raw(h) = #{j : r < h} (self included):                         */
/*   f0 = ln(N_w(H) / N_res)          f1 = (N_res / N_w(H))^(1/3) - 1   */
/*   f2 = ln(8 N_w(H/2) / N_res)      f3 = ln(64 N_w(H/4) / N_res)      */
/*   f4 = ln(n_raw(H) / N_res)        f5 = ln(8 n_raw(H/2) / N_res)     */
/*   f6 = ln(H N_tot^(1/3) / L)       f7 = 1                            */
/* feat is [8][n].                                                     */
/* ------------------------------------------------------------------ */
void orc_hnet_features(int64_t n, const double *x, const double *y, const double *z,
                       const double *H, double L, double Nres, double *feat)
{
    orc_grid g;
    int use_grid = n > 4096;
    if (use_grid) orc_grid_build(&g, n, x, y, z, H, L);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        double h = H[i];
        double s1 = 0.0, s2 = 0.0, s4 = 0.0, c1 = 0.0, c2 = 0.0;
        int64_t jb = 0, je = n;
        int lx = 0, ly = 0, lz = 0, mx = 1, my = 1, mz = 1;
        if (use_grid) {
            orc_axis_range(x[i], h, &g, &lx, &mx);
            orc_axis_range(y[i], h, &g, &ly, &my);
            orc_axis_range(z[i], h, &g, &lz, &mz);
        }
        for (int a = 0; a < mz; a++)
            for (int b = 0; b < my; b++)
                for (int e = 0; e < mx; e++) {
                    if (use_grid) {
                        int64_t cell = ((int64_t)orc_mod(lz + a, g.nc) * g.nc + orc_mod(ly + b, g.nc)) * g.nc
                                       + orc_mod(lx + e, g.nc);
                        jb = g.start[cell];
                        je = g.start[cell + 1];
                    }
                    for (int64_t k = jb; k < je; k++) {
                        int64_t j = use_grid ? g.list[k] : k;
                        double d[3];
                        double r2 = orc_sep(x, y, z, i, j, L, 1, d);
                        double r = sqrt(r2);
                        if (r2 < h * h) { s1 += orc_W(r, h); c1 += 1.0; }
                        if (r2 < 0.25 * h * h) { s2 += orc_W(r, 0.5 * h); c2 += 1.0; }
                        if (r2 < 0.0625 * h * h) s4 += orc_W(r, 0.25 * h);
                    }
                }
        double v = 4.0 / 3.0 * ORC_PI;
        double N1 = v * h * h * h * s1;
        double N2 = v * 0.125 * h * h * h * s2;
        double N4 = v * h * h * h / 64.0 * s4;
        feat[0 * n + i] = log(N1 / Nres);
        feat[1 * n + i] = cbrt(Nres / N1) - 1.0;
        feat[2 * n + i] = log(8.0 * N2 / Nres);
        feat[3 * n + i] = log(64.0 * N4 / Nres);
        feat[4 * n + i] = log(c1 / Nres);
        feat[5 * n + i] = log(8.0 * c2 / Nres);
        feat[6 * n + i] = log(h * cbrt((double)n) / L);
        feat[7 * n + i] = 1.0;
    }
    if (use_grid) orc_grid_free(&g);
}

/* ------------------------------------------------------------------ */
/* Evaluation for listed particles only (sampled checks on large sets). */
/* A fine periodic grid over all n particles (up to 256 cells a side)  */
/* restricts the candidates; every decision is the same r^2 test as     */
/* the brute-force path, so the rows are the same sets.                 */
/* ------------------------------------------------------------------ */
typedef struct {
    int nc;
    double c;
    int64_t *start;   /* [nc^3 + 1] */
    int32_t *list;    /* particles cell by cell */
    double *hmax;     /* [nc^3] largest H of each cell */
} orc_fgrid;

static void orc_fgrid_build(orc_fgrid *g, int64_t n, const double *x, const double *y,
                            const double *z, const double *H, double L)
{
    double mean = 0.0;
    for (int64_t i = 0; i < n; i++) mean += H[i];
    mean /= (double)(n > 0 ? n : 1);
    int nc = (int)floor(2.0 * L / mean);
    if (nc < 1) nc = 1;
    if (nc > 256) nc = 256;
    g->nc = nc;
    g->c = L / nc;
    int64_t ncell = (int64_t)nc * nc * nc;
    g->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    g->hmax = (double *)calloc((size_t)ncell, sizeof(double));
    g->list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *cellof = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; i++) {
        int cx = orc_cell_of(x[i], g->c, nc), cy = orc_cell_of(y[i], g->c, nc),
            cz = orc_cell_of(z[i], g->c, nc);
        cellof[i] = ((int64_t)cz * nc + cy) * nc + cx;
        g->start[cellof[i] + 1]++;
        if (H[i] > g->hmax[cellof[i]]) g->hmax[cellof[i]] = H[i];
    }
    for (int64_t k = 0; k < ncell; k++) g->start[k + 1] += g->start[k];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
    memcpy(fill, g->start, sizeof(int64_t) * (size_t)ncell);
    for (int64_t i = 0; i < n; i++) g->list[fill[cellof[i]]++] = (int32_t)i;
    free(fill);
    free(cellof);
}

static void orc_fgrid_free(orc_fgrid *g)
{
    free(g->start);
    free(g->list);
    free(g->hmax);
}

static void orc_faxis(double xi, double R, const orc_fgrid *g, int *lo, int *cnt)
{
    int a = (int)floor((xi - R) / g->c) - 1;
    int b = (int)floor((xi + R) / g->c) + 1;
    int m = b - a + 1;
    if (m >= g->nc) { a = 0; m = g->nc; }
    *lo = a;
    *cnt = m;
}

/* shortest periodic distance along one axis from xi to the cell of     */
/* (unwrapped) index k, 0 inside; used only to skip cells, with a whole */
/* extra cell of slack around the support                              */
static double orc_cell_gap(double xi, int k, const orc_fgrid *g, double L)
{
    double lo = k * g->c, hi = lo + g->c, best = INFINITY;
    for (int s = -1; s <= 1; s++) {
        double a = lo + s * L, b = hi + s * L;
        double d = xi < a ? a - xi : (xi > b ? xi - b : 0.0);
        if (d < best) best = d;
    }
    return best;
}

static int orc_cmp_i32(const void *a, const void *b)
{
    int32_t u = *(const int32_t *)a, v = *(const int32_t *)b;
    return (u > v) - (u < v);
}

/* One row for particle i: which 0 -> N_g(i) (i included), which 1 ->   */
/* N_s(i). Writes at most cap entries to row (if row != NULL) and       */
/* returns the row length; the row is ascending.                        */
static int64_t orc_row_one(int64_t i, const double *x, const double *y, const double *z,
                           const double *H, double L, int which, double Hall, const orc_fgrid *g,
                           int32_t *row, int64_t cap)
{
    double R = which == 0 ? H[i] : (H[i] > Hall ? H[i] : Hall);
    int lx, ly, lz, mx, my, mz;
    orc_faxis(x[i], R, g, &lx, &mx);
    orc_faxis(y[i], R, g, &ly, &my);
    orc_faxis(z[i], R, g, &lz, &mz);
    int64_t c = 0;
    for (int a = 0; a < mz; a++) {
        int kz = orc_mod(lz + a, g->nc);
        double gz = orc_cell_gap(z[i], kz, g, L);
        for (int b = 0; b < my; b++) {
            int ky = orc_mod(ly + b, g->nc);
            double gy = orc_cell_gap(y[i], ky, g, L);
            for (int e = 0; e < mx; e++) {
                int kx = orc_mod(lx + e, g->nc);
                int64_t cell = ((int64_t)kz * g->nc + ky) * g->nc + kx;
                if (which == 1) {
                    /* no j of this cell can reach i, nor i reach it */
                    double gx = orc_cell_gap(x[i], kx, g, L);
                    double reach = H[i] > g->hmax[cell] ? H[i] : g->hmax[cell];
                    reach += g->c;
                    if (gx * gx + gy * gy + gz * gz > reach * reach) continue;
                }
                for (int64_t k = g->start[cell]; k < g->start[cell + 1]; k++) {
                    int64_t j = g->list[k];
                    double d[3];
                    double r2 = orc_sep(x, y, z, i, j, L, 1, d);
                    int in = which == 0 ? r2 < H[i] * H[i]
                                        : (j != i && (r2 < H[i] * H[i] || r2 < H[j] * H[j]));
                    if (in) {
                        if (row && c < cap) row[c] = (int32_t)j;
                        c++;
                    }
                }
            }
        }
    }
    if (row && c <= cap) qsort(row, (size_t)c, sizeof(int32_t), orc_cmp_i32);
    return c;
}

/* Rows of N_g (which 0) or N_s (which 1) for the m particles in list,  */
/* over all n particles of a periodic box, ascending. off[m+1] always;  */
/* idx (cap entries) is filled when it holds the total. Returns the     */
/* total.                                                               */
int64_t orc_rows_for(int64_t n, const double *x, const double *y, const double *z,
                     const double *H, double L, int which, int64_t m, const int64_t *list,
                     int64_t *off, int32_t *idx, int64_t cap)
{
    orc_fgrid g;
    orc_fgrid_build(&g, n, x, y, z, H, L);
    double Hall = 0.0;
    for (int64_t i = 0; i < n; i++)
        if (H[i] > Hall) Hall = H[i];
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < m; t++)
        cnt[t] = orc_row_one(list[t], x, y, z, H, L, which, Hall, &g, NULL, 0);
    off[0] = 0;
    for (int64_t t = 0; t < m; t++) off[t + 1] = off[t] + cnt[t];
    if (idx && cap >= off[m]) {
        #pragma omp parallel for schedule(dynamic, 16)
        for (int64_t t = 0; t < m; t++)
            orc_row_one(list[t], x, y, z, H, L, which, Hall, &g, idx + off[t], cnt[t]);
    }
    free(cnt);
    orc_fgrid_free(&g);
    return off[m];
}

/* The iteration of orc_hsolve for the m listed particles only, over all */
/* n positions; H0 and H are [m] (start and result), iters [m].         */
int64_t orc_hsolve_for(int64_t n, const double *x, const double *y, const double *z, double L,
                       const double *Hgrid, double Nres, double tol, int max_iter, int64_t m,
                       const int64_t *list, const double *H0, double *H, int32_t *iters)
{
    orc_fgrid g;
    orc_fgrid_build(&g, n, x, y, z, Hgrid, L);
    int64_t nfail = 0;
    #pragma omp parallel for schedule(dynamic, 4) reduction(+ : nfail)
    for (int64_t t = 0; t < m; t++) {
        int64_t i = list[t];
        double h = H0[t];
        int it = 0, conv = 0;
        while (it < max_iter) {
            double s = 0.0;
            int lx, ly, lz, mx, my, mz;
            orc_faxis(x[i], h, &g, &lx, &mx);
            orc_faxis(y[i], h, &g, &ly, &my);
            orc_faxis(z[i], h, &g, &lz, &mz);
            for (int a = 0; a < mz; a++)
                for (int b = 0; b < my; b++)
                    for (int e = 0; e < mx; e++) {
                        int64_t cell = ((int64_t)orc_mod(lz + a, g.nc) * g.nc + orc_mod(ly + b, g.nc)) * g.nc
                                       + orc_mod(lx + e, g.nc);
                        for (int64_t k = g.start[cell]; k < g.start[cell + 1]; k++) {
                            double d[3];
                            double r2 = orc_sep(x, y, z, i, g.list[k], L, 1, d);
                            if (r2 < h * h) s += orc_W(sqrt(r2), h);
                        }
                    }
            double N = 4.0 / 3.0 * ORC_PI * h * h * h * s;
            double hn = orc_thacker_step(h, N, Nres);
            it++;
            double dh = fabs(hn - h);
            double hold = h;
            h = hn;
            if (dh <= tol * hold) { conv = 1; break; }
        }
        H[t] = h;
        if (iters) iters[t] = it;
        if (!conv) nfail++;
    }
    orc_fgrid_free(&g);
    return nfail;
}
