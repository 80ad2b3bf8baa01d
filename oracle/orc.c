/*
 * orc.c -- FP64 CPU oracle for monopole borehole acoustic FWI.
 *
 * TEST INFRASTRUCTURE ONLY (see orc.h).  Serial plain C, double precision.
 *
 * What is computed, and from which passage of the paper:
 *   - Eq. 2 (Method): velocity-stress monopole equations in (r, z) with the
 *     1/r terms, discretised on a staggered grid with second-order differences
 *     in space and leapfrog in time.  The radial divergence is taken in the
 *     conservative form (1/r) d(r v_r)/dr, which is what the averaged 1/r terms
 *     below give.  PML on the outer radius and both axial ends (complex
 *     frequency-shifted, auxiliary-variable form); symmetry on the axis
 *     (v_r = tau_rz = 0 at r = 0).
 *   - Source f added to the three normal stresses of the on-axis source cell.
 *   - Recorded pressure: the mean normal stress at on-axis receiver cells.
 *   - Eq. 1, 5: misfit and residual.
 *   - Eq. 6: adjoint equations, here the exact transpose of the discrete
 *     forward map (scatter form: every forward read becomes an adjoint write).
 *   - Eq. 7-8: zero-lag correlation of forward strain rates with adjoint stresses.
 *   - Eq. 3-4, 9-12: moduli, update, velocities.
 * Where the paper is silent (order, averaging, PML constants, source and
 * receiver conventions) the readings stated in the design notes are used.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define ORC_RC 1.0e-4 /* PML theoretical reflection coefficient */

/* ---------------------------------------------------------------------------
 * Grid, coefficients and state
 * ------------------------------------------------------------------------- */
typedef struct {
    int NR, NZ, nr, nz, pr, pz;
    double dr, dz, dt;
    /* PML profiles.  r at integer positions (R, S nodes) and half positions
     * (C, Z nodes); z at integer positions (C, R nodes) and half positions
     * (Z, S nodes).  on = 1 where the node lies inside the layer (x > 0). */
    double *ar_i, *br_i, *ar_h, *br_h;
    double *az_i, *bz_i, *az_h, *bz_h;
    char *onr_i, *onr_h, *onz_i, *onz_h;
    const double *lam, *mu, *rho;
} grid;

/* State: 14 arrays of NR*NZ. psi[] are the PML memory variables:
 *   A: R node, d/dr tau_rr      B: R node, d/dz tau_rz
 *   C: Z node, d/dr tau_rz      D: Z node, d/dz tau_zz
 *   E: C node, d/dr v_r         F: C node, d/dz v_z
 *   G: S node, d/dz v_r         H: S node, d/dr v_z                        */
typedef struct {
    double *vr, *vz, *trr, *ttt, *tzz, *trz;
    double *psi[8];
} state;

static void state_bind(state *s, double *mem, size_t n)
{
    s->vr = mem;
    s->vz = mem + n;
    s->trr = mem + 2 * n;
    s->ttt = mem + 3 * n;
    s->tzz = mem + 4 * n;
    s->trz = mem + 5 * n;
    for (int q = 0; q < 8; ++q) s->psi[q] = mem + (6 + q) * n;
}

/* CFS-PML coefficients for penetration x in (0,1]:
 *   d(x) = d0 x^2, alpha(x) = pi f0 (1 - x), kappa = 1,
 *   b = exp(-(d + alpha) dt), a = d (b - 1) / (d + alpha);
 * memory update psi <- b psi + a D, the difference D is then replaced by D + psi. */
static void pml_ab(double x, double d0, double f0, double dt, double *a, double *b, char *on)
{
    if (!(x > 0.0)) {
        *a = 0.0;
        *b = 1.0;
        *on = 0;
        return;
    }
    double d = d0 * x * x;
    double al = ORC_PI * f0 * (1.0 - x);
    *b = exp(-(d + al) * dt);
    *a = d * (*b - 1.0) / (d + al);
    *on = 1;
}

static int grid_init(grid *G, const orc_geom *g, const double *lam, const double *mu,
                     const double *rho)
{
    if (g->nr <= 1 || g->nz <= 1 || g->pr < 0 || g->pz < 0 || g->nt < 0) return -1;
    if (!(g->dr > 0) || !(g->dz > 0) || !(g->dt > 0)) return -1;
    G->nr = g->nr;
    G->nz = g->nz;
    G->pr = g->pr;
    G->pz = g->pz;
    G->NR = g->nr + g->pr;
    G->NZ = g->nz + 2 * g->pz;
    G->dr = g->dr;
    G->dz = g->dz;
    G->dt = g->dt;
    G->lam = lam;
    G->mu = mu;
    G->rho = rho;
    int NR = G->NR, NZ = G->NZ;
    G->ar_i = calloc(NR, sizeof(double));
    G->br_i = calloc(NR, sizeof(double));
    G->ar_h = calloc(NR, sizeof(double));
    G->br_h = calloc(NR, sizeof(double));
    G->az_i = calloc(NZ, sizeof(double));
    G->bz_i = calloc(NZ, sizeof(double));
    G->az_h = calloc(NZ, sizeof(double));
    G->bz_h = calloc(NZ, sizeof(double));
    G->onr_i = calloc(NR, 1);
    G->onr_h = calloc(NR, 1);
    G->onz_i = calloc(NZ, 1);
    G->onz_h = calloc(NZ, 1);
    double lnR = log(ORC_RC);
    double d0r = g->pr > 0 ? -3.0 * g->vmax * lnR / (2.0 * g->pr * g->dr) : 0.0;
    double d0z = g->pz > 0 ? -3.0 * g->vmax * lnR / (2.0 * g->pz * g->dz) : 0.0;
    for (int i = 0; i < NR; ++i) {
        double xi = 0.0, xh = 0.0;
        if (g->pr > 0) {
            xi = ((double)i - g->nr) / g->pr;
            xh = ((double)i + 0.5 - g->nr) / g->pr;
        }
        pml_ab(xi, d0r, g->f0, g->dt, &G->ar_i[i], &G->br_i[i], &G->onr_i[i]);
        pml_ab(xh, d0r, g->f0, g->dt, &G->ar_h[i], &G->br_h[i], &G->onr_h[i]);
    }
    for (int k = 0; k < NZ; ++k) {
        double xi = 0.0, xh = 0.0;
        if (g->pz > 0) {
            /* physical C rows are k in [pz, pz+nz); their cell faces span
             * [pz - 1/2, pz + nz - 1/2] in index units */
            double lo = g->pz - 0.5, hi = g->pz + g->nz - 0.5;
            double ui = k, uh = k + 0.5;
            if (ui < lo) xi = (lo - ui) / g->pz;
            if (ui > hi) xi = (ui - hi) / g->pz;
            if (uh < lo) xh = (lo - uh) / g->pz;
            if (uh > hi) xh = (uh - hi) / g->pz;
        }
        pml_ab(xi, d0z, g->f0, g->dt, &G->az_i[k], &G->bz_i[k], &G->onz_i[k]);
        pml_ab(xh, d0z, g->f0, g->dt, &G->az_h[k], &G->bz_h[k], &G->onz_h[k]);
    }
    return 0;
}

static void grid_free(grid *G)
{
    free(G->ar_i); free(G->br_i); free(G->ar_h); free(G->br_h);
    free(G->az_i); free(G->bz_i); free(G->az_h); free(G->bz_h);
    free(G->onr_i); free(G->onr_h); free(G->onz_i); free(G->onz_h);
}

#define IX(i, k) ((size_t)(i) * (size_t)NZ + (size_t)(k))

/* Medium averaging (reading: arithmetic density at velocity nodes, harmonic
 * rigidity at tau_rz nodes, zero if any neighbour is fluid). */
static double buoy_R(const grid *G, int i, int k)
{
    int NZ = G->NZ;
    return 2.0 / (G->rho[IX(i - 1, k)] + G->rho[IX(i, k)]);
}
static double buoy_Z(const grid *G, int i, int k)
{
    int NZ = G->NZ;
    int k1 = k + 1 < NZ ? k + 1 : NZ - 1;
    return 2.0 / (G->rho[IX(i, k)] + G->rho[IX(i, k1)]);
}
static double mu_S(const grid *G, int i, int k)
{
    int NZ = G->NZ;
    int k1 = k + 1 < NZ ? k + 1 : NZ - 1;
    double m1 = G->mu[IX(i - 1, k)], m2 = G->mu[IX(i, k)];
    double m3 = G->mu[IX(i - 1, k1)], m4 = G->mu[IX(i, k1)];
    if (!(m1 > 0 && m2 > 0 && m3 > 0 && m4 > 0)) return 0.0;
    return 4.0 / (1.0 / m1 + 1.0 / m2 + 1.0 / m3 + 1.0 / m4);
}

/* ---------------------------------------------------------------------------
 * One forward step (Eq. 2).  srcval is added to the three normal stresses of
 * C(0, src_k).  If eps != NULL the strain rates used for the stress update are
 * stored: eps[0..3] planes = e_rr', e_tt, e_zz' (C nodes), e_rz' (S nodes),
 * where ' marks the PML-modified difference.
 * ------------------------------------------------------------------------- */
/* One leapfrog step.  eps (nullable) receives the strain rates the stress
 * update used (4 N); dvb (nullable) receives d v^{n+1/2} / d b for v_r and v_z
 * (2 N: dt times the bracket the buoyancy multiplies). */
static void fwd_step(const grid *G, state *s, int src_k, double srcval, double *eps,
                     double *dvb)
{
    const int NR = G->NR, NZ = G->NZ;
    const double dr = G->dr, dz = G->dz, dt = G->dt;
    double *vr = s->vr, *vz = s->vz, *trr = s->trr, *ttt = s->ttt, *tzz = s->tzz, *trz = s->trz;
    double *pA = s->psi[0], *pB = s->psi[1], *pC = s->psi[2], *pD = s->psi[3];
    double *pE = s->psi[4], *pF = s->psi[5], *pG = s->psi[6], *pH = s->psi[7];
    size_t N = (size_t)NR * NZ;

    /* velocity: R nodes, i >= 1 */
    for (int i = 1; i < NR; ++i) {
        double ri = i * dr;
        for (int k = 0; k < NZ; ++k) {
            size_t c = IX(i, k), cm = IX(i - 1, k);
            double Dr = (trr[c] - trr[cm]) / dr;
            if (G->onr_i[i]) {
                pA[c] = G->br_i[i] * pA[c] + G->ar_i[i] * Dr;
                Dr += pA[c];
            }
            double trz_km = k > 0 ? trz[IX(i, k - 1)] : 0.0;
            double Dz = (trz[c] - trz_km) / dz;
            if (G->onz_i[k]) {
                pB[c] = G->bz_i[k] * pB[c] + G->az_i[k] * Dz;
                Dz += pB[c];
            }
            double hoop = ((trr[c] - ttt[c]) + (trr[cm] - ttt[cm])) / (2.0 * ri);
            vr[c] += dt * buoy_R(G, i, k) * (Dr + Dz + hoop);
            if (dvb) dvb[c] = dt * (Dr + Dz + hoop);
        }
    }
    /* velocity: Z nodes */
    for (int i = 0; i < NR; ++i) {
        double rh = (i + 0.5) * dr;
        for (int k = 0; k < NZ; ++k) {
            size_t c = IX(i, k);
            double trz_ip = i + 1 < NR ? trz[IX(i + 1, k)] : 0.0;
            double Dr = (trz_ip - trz[c]) / dr;
            if (G->onr_h[i]) {
                pC[c] = G->br_h[i] * pC[c] + G->ar_h[i] * Dr;
                Dr += pC[c];
            }
            double tzz_kp = k + 1 < NZ ? tzz[IX(i, k + 1)] : 0.0;
            double Dz = (tzz_kp - tzz[c]) / dz;
            if (G->onz_h[k]) {
                pD[c] = G->bz_h[k] * pD[c] + G->az_h[k] * Dz;
                Dz += pD[c];
            }
            double hoop = (trz_ip + trz[c]) / (2.0 * rh);
            vz[c] += dt * buoy_Z(G, i, k) * (Dr + Dz + hoop);
            if (dvb) dvb[N + c] = dt * (Dr + Dz + hoop);
        }
    }
    /* stress: C nodes */
    for (int i = 0; i < NR; ++i) {
        double rh = (i + 0.5) * dr;
        for (int k = 0; k < NZ; ++k) {
            size_t c = IX(i, k);
            double vr_ip = i + 1 < NR ? vr[IX(i + 1, k)] : 0.0;
            double err = (vr_ip - vr[c]) / dr;
            if (G->onr_h[i]) {
                pE[c] = G->br_h[i] * pE[c] + G->ar_h[i] * err;
                err += pE[c];
            }
            double ett = (vr_ip + vr[c]) / (2.0 * rh);
            double vz_km = k > 0 ? vz[IX(i, k - 1)] : 0.0;
            double ezz = (vz[c] - vz_km) / dz;
            if (G->onz_i[k]) {
                pF[c] = G->bz_i[k] * pF[c] + G->az_i[k] * ezz;
                ezz += pF[c];
            }
            double l = G->lam[c], m = G->mu[c];
            trr[c] += dt * ((l + 2.0 * m) * err + l * (ett + ezz));
            ttt[c] += dt * ((l + 2.0 * m) * ett + l * (err + ezz));
            tzz[c] += dt * ((l + 2.0 * m) * ezz + l * (err + ett));
            if (eps) {
                eps[c] = err;
                eps[N + c] = ett;
                eps[2 * N + c] = ezz;
            }
        }
    }
    /* source: f of Eq. 2 in the three normal stresses */
    {
        size_t c = IX(0, src_k);
        trr[c] += srcval;
        ttt[c] += srcval;
        tzz[c] += srcval;
    }
    /* stress: S nodes, i >= 1 */
    if (eps)
        for (int k = 0; k < NZ; ++k) eps[3 * N + IX(0, k)] = 0.0;
    for (int i = 1; i < NR; ++i) {
        for (int k = 0; k < NZ; ++k) {
            size_t c = IX(i, k);
            double vr_kp = k + 1 < NZ ? vr[IX(i, k + 1)] : 0.0;
            double ez = (vr_kp - vr[c]) / dz;
            if (G->onz_h[k]) {
                pG[c] = G->bz_h[k] * pG[c] + G->az_h[k] * ez;
                ez += pG[c];
            }
            double er = (vz[c] - vz[IX(i - 1, k)]) / dr;
            if (G->onr_i[i]) {
                pH[c] = G->br_i[i] * pH[c] + G->ar_i[i] * er;
                er += pH[c];
            }
            trz[c] += dt * mu_S(G, i, k) * (ez + er);
            if (eps) eps[3 * N + c] = ez + er;
        }
    }
}

/* ---------------------------------------------------------------------------
 * Exact transpose of fwd_step (without source), applied to the adjoint state a.
 * Order is the reverse of the forward: stress phase first, then velocity.
 * ------------------------------------------------------------------------- */
/* Transpose of one step, in two halves: the stress phase (after which a->vr,
 * a->vz hold dJ/dv^{n+1/2}) and the velocity phase. */
static void adj_stress_phase(const grid *G, state *a)
{
    const int NR = G->NR, NZ = G->NZ;
    const double dr = G->dr, dz = G->dz, dt = G->dt;
    double *avr = a->vr, *avz = a->vz, *atrr = a->trr, *attt = a->ttt, *atzz = a->tzz,
           *atrz = a->trz;
    double *qE = a->psi[4], *qF = a->psi[5], *qG = a->psi[6], *qH = a->psi[7];

    /* transpose of the stress phase: C nodes */
    for (int i = 0; i < NR; ++i) {
        double rh = (i + 0.5) * dr;
        for (int k = 0; k < NZ; ++k) {
            size_t c = IX(i, k);
            double l = G->lam[c], m = G->mu[c];
            double srr = (l + 2.0 * m) * atrr[c] + l * attt[c] + l * atzz[c];
            double stt = l * atrr[c] + (l + 2.0 * m) * attt[c] + l * atzz[c];
            double szz = l * atrr[c] + l * attt[c] + (l + 2.0 * m) * atzz[c];
            double g_err = dt * srr, g_ett = dt * stt, g_ezz = dt * szz;
            if (G->onr_h[i]) {
                double q = qE[c] + g_err;
                qE[c] = G->br_h[i] * q;
                g_err += G->ar_h[i] * q;
            }
            if (G->onz_i[k]) {
                double q = qF[c] + g_ezz;
                qF[c] = G->bz_i[k] * q;
                g_ezz += G->az_i[k] * q;
            }
            if (i + 1 < NR) avr[IX(i + 1, k)] += g_err / dr + g_ett / (2.0 * rh);
            avr[c] += -g_err / dr + g_ett / (2.0 * rh);
            avz[c] += g_ezz / dz;
            if (k > 0) avz[IX(i, k - 1)] -= g_ezz / dz;
        }
    }
    /* transpose of the stress phase: S nodes */
    for (int i = 1; i < NR; ++i) {
        for (int k = 0; k < NZ; ++k) {
            size_t c = IX(i, k);
            double g = dt * mu_S(G, i, k) * atrz[c];
            double g_ez = g, g_er = g;
            if (G->onz_h[k]) {
                double q = qG[c] + g;
                qG[c] = G->bz_h[k] * q;
                g_ez += G->az_h[k] * q;
            }
            if (G->onr_i[i]) {
                double q = qH[c] + g;
                qH[c] = G->br_i[i] * q;
                g_er += G->ar_i[i] * q;
            }
            if (k + 1 < NZ) avr[IX(i, k + 1)] += g_ez / dz;
            avr[c] -= g_ez / dz;
            avz[c] += g_er / dr;
            avz[IX(i - 1, k)] -= g_er / dr;
        }
    }
}

static void adj_velocity_phase(const grid *G, state *a)
{
    const int NR = G->NR, NZ = G->NZ;
    const double dr = G->dr, dz = G->dz, dt = G->dt;
    double *avr = a->vr, *avz = a->vz, *atrr = a->trr, *attt = a->ttt, *atzz = a->tzz,
           *atrz = a->trz;
    double *qA = a->psi[0], *qB = a->psi[1], *qC = a->psi[2], *qD = a->psi[3];

    /* transpose of the velocity phase: R nodes, i >= 1 */
    for (int i = 1; i < NR; ++i) {
        double ri = i * dr;
        for (int k = 0; k < NZ; ++k) {
            size_t c = IX(i, k), cm = IX(i - 1, k);
            double w = dt * buoy_R(G, i, k) * avr[c];
            double g_Dr = w, g_Dz = w;
            if (G->onr_i[i]) {
                double q = qA[c] + w;
                qA[c] = G->br_i[i] * q;
                g_Dr += G->ar_i[i] * q;
            }
            if (G->onz_i[k]) {
                double q = qB[c] + w;
                qB[c] = G->bz_i[k] * q;
                g_Dz += G->az_i[k] * q;
            }
            atrr[c] += g_Dr / dr;
            atrr[cm] -= g_Dr / dr;
            atrz[c] += g_Dz / dz;
            if (k > 0) atrz[IX(i, k - 1)] -= g_Dz / dz;
            double h = w / (2.0 * ri);
            atrr[c] += h;
            attt[c] -= h;
            atrr[cm] += h;
            attt[cm] -= h;
        }
    }
    /* transpose of the velocity phase: Z nodes */
    for (int i = 0; i < NR; ++i) {
        double rh = (i + 0.5) * dr;
        for (int k = 0; k < NZ; ++k) {
            size_t c = IX(i, k);
            double w = dt * buoy_Z(G, i, k) * avz[c];
            double g_Dr = w, g_Dz = w;
            if (G->onr_h[i]) {
                double q = qC[c] + w;
                qC[c] = G->br_h[i] * q;
                g_Dr += G->ar_h[i] * q;
            }
            if (G->onz_h[k]) {
                double q = qD[c] + w;
                qD[c] = G->bz_h[k] * q;
                g_Dz += G->az_h[k] * q;
            }
            if (i + 1 < NR) atrz[IX(i + 1, k)] += g_Dr / dr + w / (2.0 * rh);
            atrz[c] += -g_Dr / dr + w / (2.0 * rh);
            if (k + 1 < NZ) atzz[IX(i, k + 1)] += g_Dz / dz;
            atzz[c] -= g_Dz / dz;
        }
    }
}

static void adj_step(const grid *G, state *a)
{
    adj_stress_phase(G, a);
    adj_velocity_phase(G, a);
}

static double src_scale(const grid *G)
{
    /* point source spread over the on-axis cell, volume pi dr^2 dz */
    return G->dt / (ORC_PI * G->dr * G->dr * G->dz);
}

/* Source scale of the assembled step of the given order.
 *
 * A point source must inject its whole strength in the norm in which the
 * discrete divergence theorem holds.  With F = r v_r (even across the axis
 * once v_r is odd) and the radial divergence h r_{i+1/2} div_i = D_i =
 * c1 (F_{i+1} - F_i) + c2 (F_{i+2} - F_{i-1}), the sum over cells of
 * w_i D_i telescopes to the outer boundary only if, for every interior
 * node j, c1 (w_{j-1} - w_j) + c2 (w_{j-2} - w_{j+1}) = 0, and at the first
 * node (which also meets the mirror image F_{-1} = F_1)
 * c1 (w_0 - w_1) - c2 (w_0 + w_2) = 0.  With plain cell volumes (w = 1) the
 * first condition holds and the second leaves -2 c2 F_1: order 2 (c2 = 0)
 * conserves, order 4 does not.  Writing w_i = 1 + d_i, the interior
 * recurrence has the roots 1 and z = 13 -/+ 2 sqrt(42) for c1 = 9/8,
 * c2 = -1/24; the bounded solution is d_i = A z^i with z = 13 - 2 sqrt(42),
 * and the first-node condition gives A = 2 c2 / (c1 (1 - z) - c2 (1 + z^2))
 * = -1 / (7 + sqrt(42)).  The on-axis cell's weight is then
 * w_0 = 1 + A = sqrt(6/7): the mirrored fourth-order step sees that fraction
 * of the cell's volume, so the source is divided by it. */
static double src_scale_order(const grid *G, int order)
{
    if (order != 4) return src_scale(G);
    const double c1 = 9.0 / 8.0, c2 = -1.0 / 24.0;
    const double z = 13.0 - 2.0 * sqrt(42.0);
    const double w0 = 1.0 + 2.0 * c2 / (c1 * (1.0 - z) - c2 * (1.0 + z * z));
    return src_scale(G) / w0;
}

static int geom_ok(const orc_geom *g)
{
    int NZ = g->nz + 2 * g->pz;
    if (g->src_k < 0 || g->src_k >= NZ) return 0;
    for (int j = 0; j < g->nrec; ++j)
        if (g->rec_k[j] < 0 || g->rec_k[j] >= NZ) return 0;
    return 1;
}

/* ---------------------------------------------------------------------------
 * Public entry points
 * ------------------------------------------------------------------------- */
void orc_moduli(int64_t n, const double *vp, const double *vs, const double *rho, double *lam,
                double *mu)
{
    for (int64_t c = 0; c < n; ++c) {
        lam[c] = rho[c] * vp[c] * vp[c] - 2.0 * rho[c] * vs[c] * vs[c];
        mu[c] = rho[c] * vs[c] * vs[c];
    }
}

void orc_moduli_grad(int64_t n, const double *vp, const double *vs, const double *rho,
                     const double *glam, const double *gmu, double *gvp, double *gvs,
                     double *grho)
{
    for (int64_t c = 0; c < n; ++c) {
        /* lambda = rho vp^2 - 2 rho vs^2, mu = rho vs^2 */
        double dl_dvp = 2.0 * rho[c] * vp[c];
        double dl_dvs = -4.0 * rho[c] * vs[c];
        double dm_dvs = 2.0 * rho[c] * vs[c];
        gvp[c] = dl_dvp * glam[c];
        gvs[c] = dl_dvs * glam[c] + dm_dvs * gmu[c];
        if (grho) {
            double dl_drho = vp[c] * vp[c] - 2.0 * vs[c] * vs[c];
            double dm_drho = vs[c] * vs[c];
            grho[c] = dl_drho * glam[c] + dm_drho * gmu[c];
        }
    }
}

void orc_velocities(int64_t n, const double *lam, const double *mu, const double *rho,
                    double *vp, double *vs)
{
    for (int64_t c = 0; c < n; ++c) {
        vp[c] = sqrt((lam[c] + 2.0 * mu[c]) / rho[c]);
        vs[c] = sqrt(mu[c] / rho[c]);
    }
}

int64_t orc_state_len(const orc_geom *g)
{
    return (int64_t)14 * (g->nr + g->pr) * (g->nz + 2 * g->pz);
}

int orc_forward(const orc_geom *g, const double *lam, const double *mu, const double *rho,
                const double *wavelet, double *traces, double *final_state)
{
    grid G;
    if (grid_init(&G, g, lam, mu, rho) || !geom_ok(g)) return -1;
    int NZ = G.NZ;
    size_t N = (size_t)G.NR * G.NZ;
    double *mem = calloc(14 * N, sizeof(double));
    if (!mem) {
        grid_free(&G);
        return -1;
    }
    state s;
    state_bind(&s, mem, N);
    double sc = src_scale(&G);
    for (int n = 0; n < g->nt; ++n) {
        fwd_step(&G, &s, g->src_k, sc * wavelet[n], NULL, NULL);
        for (int j = 0; j < g->nrec; ++j) {
            size_t c = IX(0, g->rec_k[j]);
            traces[(size_t)j * g->nt + n] = (s.trr[c] + s.ttt[c] + s.tzz[c]) / 3.0;
        }
    }
    if (final_state) memcpy(final_state, mem, 14 * N * sizeof(double));
    free(mem);
    grid_free(&G);
    return 0;
}

double orc_misfit(int64_t n, const double *d, const double *dobs, double *resid)
{
    double J = 0.0;
    for (int64_t c = 0; c < n; ++c) {
        double r = d[c] - dobs[c];
        if (resid) resid[c] = r;
        J += 0.5 * r * r;
    }
    return J;
}

/* Rigidity at tau_rz nodes is the harmonic mean of the four adjacent C cells:
 * d muS / d mu_c = muS^2 / (4 mu_c^2) per occurrence of c among the four. */
static void fold_mu_s(const grid *G, const double *gmuS, double *gmu)
{
    const int NR = G->NR, NZ = G->NZ;
    for (int i = 1; i < NR; ++i)
        for (int k = 0; k < NZ; ++k) {
            double ms = mu_S(G, i, k);
            if (!(ms > 0)) continue;
            int k1 = k + 1 < NZ ? k + 1 : NZ - 1;
            size_t nb[4] = {IX(i - 1, k), IX(i, k), IX(i - 1, k1), IX(i, k1)};
            for (int q = 0; q < 4; ++q) {
                double mc = G->mu[nb[q]];
                gmu[nb[q]] += gmuS[IX(i, k)] * ms * ms / (4.0 * mc * mc);
            }
        }
}

static void inject_residual(const orc_geom *g, int NZ, state *a, const double *resid, int n)
{
    for (int j = 0; j < g->nrec; ++j) {
        size_t c = IX(0, g->rec_k[j]);
        double r3 = resid[(size_t)j * g->nt + n] / 3.0;
        a->trr[c] += r3;
        a->ttt[c] += r3;
        a->tzz[c] += r3;
    }
}

/* dJ/drho from dJ/db at the v_r and v_z nodes (gb: 2 N).  b_R = 2/(rho[i-1,k]
 * + rho[i,k]) and b_Z = 2/(rho[i,k] + rho[i,k1]): d b / d rho = -b^2/2 for
 * each of the two cells (k1 = k on the top row counts twice). */
static void rho_chain(const grid *Gp, const double *gb, double *grho)
{
    const grid G = *Gp;
    const int NR = G.NR, NZ = G.NZ;
    const size_t N = (size_t)NR * NZ;
    memset(grho, 0, N * sizeof(double));
    for (int i = 1; i < NR; ++i)
        for (int k = 0; k < NZ; ++k) {
            double b = buoy_R(&G, i, k), t = -0.5 * b * b * gb[IX(i, k)];
            grho[IX(i - 1, k)] += t;
            grho[IX(i, k)] += t;
        }
    for (int i = 0; i < NR; ++i)
        for (int k = 0; k < NZ; ++k) {
            int k1 = k + 1 < NZ ? k + 1 : NZ - 1;
            double b = buoy_Z(&G, i, k), t = -0.5 * b * b * gb[N + IX(i, k)];
            grho[IX(i, k)] += t;
            grho[IX(i, k1)] += t;
        }
}

int orc_gradient(const orc_geom *g, const double *lam, const double *mu, const double *rho,
                 const double *wavelet, const double *resid, int32_t seg, double *glam,
                 double *gmu, double *illum, double *grho, double *hl, double *hm)
{
    grid G;
    if (seg <= 0 || grid_init(&G, g, lam, mu, rho) || !geom_ok(g)) return -1;
    const int NR = G.NR, NZ = G.NZ, nt = g->nt;
    const double dt = G.dt;
    size_t N = (size_t)NR * NZ, SL = 14 * N;
    int nseg = (nt + seg - 1) / seg;
    double *ckpt = malloc((size_t)(nseg > 0 ? nseg : 1) * SL * sizeof(double));
    double *fmem = calloc(SL, sizeof(double));
    double *amem = calloc(SL, sizeof(double));
    double *eps = malloc((size_t)seg * 4 * N * sizeof(double));
    double *gmuS = calloc(N, sizeof(double));
    /* for the density: d v^{n+1/2} / d b per step of a segment, and
     * dJ/db at the v_r and v_z nodes */
    double *dvb = grho ? malloc((size_t)seg * 2 * N * sizeof(double)) : NULL;
    double *gb = grho ? calloc(2 * N, sizeof(double)) : NULL;
    if (!ckpt || !fmem || !amem || !eps || !gmuS || (grho && (!dvb || !gb))) {
        free(ckpt); free(fmem); free(amem); free(eps); free(gmuS); free(dvb); free(gb);
        grid_free(&G);
        return -1;
    }
    state s, a;
    state_bind(&s, fmem, N);
    state_bind(&a, amem, N);
    double sc = src_scale(&G);
    memset(glam, 0, N * sizeof(double));
    memset(gmu, 0, N * sizeof(double));
    memset(illum, 0, N * sizeof(double));
    if (hl) memset(hl, 0, N * sizeof(double));
    if (hm) memset(hm, 0, N * sizeof(double));

    /* forward pass: checkpoints every seg steps, illumination from v^{n+1/2} */
    for (int n = 0; n < nt; ++n) {
        if (n % seg == 0) memcpy(ckpt + (size_t)(n / seg) * SL, fmem, SL * sizeof(double));
        fwd_step(&G, &s, g->src_k, sc * wavelet[n], NULL, NULL);
        for (int i = 0; i < NR; ++i)
            for (int k = 0; k < NZ; ++k) {
                size_t c = IX(i, k);
                double vr_ip = i + 1 < NR ? s.vr[IX(i + 1, k)] : 0.0;
                double vz_km = k > 0 ? s.vz[IX(i, k - 1)] : 0.0;
                double ur = 0.5 * (s.vr[c] + vr_ip), uz = 0.5 * (vz_km + s.vz[c]);
                illum[c] += dt * (ur * ur + uz * uz);
                if (hl || hm) {
                    /* virtual sources: d(stress update)/d(modulus) applied to
                     * v^{n+1/2}, with the plain strain rates of the stencil */
                    double rh = (i + 0.5) * G.dr;
                    double err = (vr_ip - s.vr[c]) / G.dr, ett = (vr_ip + s.vr[c]) / (2.0 * rh);
                    double ezz = (s.vz[c] - vz_km) / G.dz, es = 0.0;
                    if (i >= 1) {
                        double vr_kp = k + 1 < NZ ? s.vr[IX(i, k + 1)] : 0.0;
                        es = (vr_kp - s.vr[c]) / G.dz + (s.vz[c] - s.vz[IX(i - 1, k)]) / G.dr;
                    }
                    double dv = err + ett + ezz;
                    if (hl) hl[c] += dt * dt * 3.0 * dv * dv;
                    if (hm) hm[c] += dt * dt * (4.0 * (err * err + ett * ett + ezz * ezz) + es * es);
                }
            }
    }

    /* reverse pass, one segment at a time */
    for (int j = nseg - 1; j >= 0; --j) {
        int n0 = j * seg, n1 = n0 + seg < nt ? n0 + seg : nt;
        memcpy(fmem, ckpt + (size_t)j * SL, SL * sizeof(double));
        for (int n = n0; n < n1; ++n)
            fwd_step(&G, &s, g->src_k, sc * wavelet[n], eps + (size_t)(n - n0) * 4 * N,
                     dvb ? dvb + (size_t)(n - n0) * 2 * N : NULL);
        for (int n = n1 - 1; n >= n0; --n) {
            inject_residual(g, NZ, &a, resid, n);
            const double *e = eps + (size_t)(n - n0) * 4 * N;
            /* Eq. 7 and Eq. 8, the adjoint stress being dJ/dtau^{n+1} */
            for (size_t c = 0; c < N; ++c) {
                double err = e[c], ett = e[N + c], ezz = e[2 * N + c];
                double sa = a.trr[c] + a.ttt[c] + a.tzz[c];
                glam[c] += dt * (err + ett + ezz) * sa;
                gmu[c] += dt * 2.0 * (err * a.trr[c] + ett * a.ttt[c] + ezz * a.tzz[c]);
                gmuS[c] += dt * e[3 * N + c] * a.trz[c];
            }
            adj_stress_phase(&G, &a);
            if (gb) {
                /* v^{n+1/2} = v^{n-1/2} + b dv/db: dJ/db += dJ/dv^{n+1/2} dv/db */
                const double *d = dvb + (size_t)(n - n0) * 2 * N;
                for (size_t c = 0; c < N; ++c) {
                    gb[c] += a.vr[c] * d[c];
                    gb[N + c] += a.vz[c] * d[N + c];
                }
            }
            adj_velocity_phase(&G, &a);
        }
    }
    if (grho) rho_chain(&G, gb, grho);
    fold_mu_s(&G, gmuS, gmu);
    free(ckpt); free(fmem); free(amem); free(eps); free(gmuS); free(dvb); free(gb);
    grid_free(&G);
    return 0;
}

int orc_source_adjoint(const orc_geom *g, const double *lam, const double *mu,
                       const double *rho, const double *resid, double *wadj)
{
    grid G;
    if (grid_init(&G, g, lam, mu, rho) || !geom_ok(g)) return -1;
    int NZ = G.NZ;
    size_t N = (size_t)G.NR * G.NZ;
    double *amem = calloc(14 * N, sizeof(double));
    if (!amem) {
        grid_free(&G);
        return -1;
    }
    state a;
    state_bind(&a, amem, N);
    double sc = src_scale(&G);
    size_t cs = IX(0, g->src_k);
    for (int n = g->nt - 1; n >= 0; --n) {
        inject_residual(g, NZ, &a, resid, n);
        wadj[n] = sc * (a.trr[cs] + a.ttt[cs] + a.tzz[cs]);
        adj_step(&G, &a);
    }
    free(amem);
    grid_free(&G);
    return 0;
}

int orc_propagate(const orc_geom *g, const double *lam, const double *mu, const double *rho,
                  double *st, int32_t nsteps)
{
    grid G;
    if (grid_init(&G, g, lam, mu, rho) || !geom_ok(g)) return -1;
    size_t N = (size_t)G.NR * G.NZ;
    state s;
    state_bind(&s, st, N);
    for (int n = 0; n < nsteps; ++n) fwd_step(&G, &s, g->src_k, 0.0, NULL, NULL);
    grid_free(&G);
    return 0;
}

int orc_propagate_adjoint(const orc_geom *g, const double *lam, const double *mu,
                          const double *rho, double *ast, int32_t nsteps)
{
    grid G;
    if (grid_init(&G, g, lam, mu, rho) || !geom_ok(g)) return -1;
    size_t N = (size_t)G.NR * G.NZ;
    state a;
    state_bind(&a, ast, N);
    for (int n = 0; n < nsteps; ++n) adj_step(&G, &a);
    grid_free(&G);
    return 0;
}

double orc_precondition(int64_t n, const double *illum, const uint8_t *mask, double eps,
                        double *g_lam, double *g_mu)
{
    double emax = 0.0, gpg = 0.0;
    for (int64_t c = 0; c < n; ++c)
        if (mask[c] && illum[c] > emax) emax = illum[c];
    for (int64_t c = 0; c < n; ++c) {
        if (!mask[c]) {
            g_lam[c] = 0.0;
            g_mu[c] = 0.0;
            continue;
        }
        double p = 1.0 / (illum[c] + eps * emax);
        double pl = p * g_lam[c], pm = p * g_mu[c];
        gpg += g_lam[c] * pl + g_mu[c] * pm;
        g_lam[c] = pl;
        g_mu[c] = pm;
    }
    return gpg;
}

double orc_line_search(double J0, double J1, double gpg, double alpha1)
{
    /* Model the misfit along the step m - a*Pg as a quadratic q(a) through
     * q(0) = J0 with q'(0) = -gpg and q(alpha1) = J1. */
    if (!(alpha1 > 0)) return 0.0;
    double slope = -gpg;
    double curv = (J1 - J0 - slope * alpha1) / (alpha1 * alpha1);
    if (curv > 0) {
        double a = -slope / (2.0 * curv);
        if (a < 0.1 * alpha1) a = 0.1 * alpha1;
        if (a > 3.0 * alpha1) a = 3.0 * alpha1;
        return a;
    }
    /* no interior minimum: keep the trial step if it helped, else halve it */
    return J1 <= J0 ? alpha1 : 0.5 * alpha1;
}

double orc_update(int64_t n, double *lam, double *mu, const double *rho, const double *g_lam,
                  const double *g_mu, const uint8_t *mask, double eta, double alpha_override,
                  double vp_min, double vp_max, double vs_min, double vs_max)
{
    double alpha = alpha_override;
    if (!(alpha > 0)) {
        double gl = 0, gm = 0, lm = 0, mm = 0;
        for (int64_t c = 0; c < n; ++c) {
            if (!mask[c]) continue;
            if (fabs(g_lam[c]) > gl) gl = fabs(g_lam[c]);
            if (fabs(g_mu[c]) > gm) gm = fabs(g_mu[c]);
            if (fabs(lam[c]) > lm) lm = fabs(lam[c]);
            if (fabs(mu[c]) > mm) mm = fabs(mu[c]);
        }
        double rl = lm > 0 ? gl / lm : 0, rm = mm > 0 ? gm / mm : 0;
        double r = rl > rm ? rl : rm;
        alpha = r > 0 ? eta / r : 0.0;
    }
    for (int64_t c = 0; c < n; ++c) {
        if (!mask[c]) continue;
        double l = lam[c] - alpha * g_lam[c];
        double m = mu[c] - alpha * g_mu[c];
        double r = rho[c];
        if (m < r * vs_min * vs_min) m = r * vs_min * vs_min;
        if (m > r * vs_max * vs_max) m = r * vs_max * vs_max;
        double p = l + 2.0 * m;
        if (p < r * vp_min * vp_min) p = r * vp_min * vp_min;
        if (p > r * vp_max * vp_max) p = r * vp_max * vp_max;
        lam[c] = p - 2.0 * m;
        mu[c] = m;
    }
    return alpha;
}

/* ---------------------------------------------------------------------------
 * Starting model (Introduction; Numerical Examples section, Fig. 3-4):
 * slowness-time coherence over the receiver array (the semblance analysis the
 * paper cites to Kimball and Marzetta), then velocities linear in radius from
 * the near-source values at the borehole wall to the far-source values 1 m
 * into the formation.
 * ------------------------------------------------------------------------- */

/* Trace m at the fractional sample position u, linear between samples, zero
 * outside the record. */
static double trace_at(const double *x, int32_t nt, double u)
{
    if (!(u >= 0.0) || u > (double)(nt - 1)) return 0.0;
    int32_t n = (int32_t)floor(u);
    if (n >= nt - 1) return x[nt - 1];
    double f = u - n;
    return (1.0 - f) * x[n] + f * x[n + 1];
}

void orc_semblance(int32_t nrec, int32_t nt, const double *traces, double dt,
                   const double *offset, int32_t np, double p0, double dp,
                   int32_t ntau, int32_t tau_stride, int32_t win, double *coh,
                   double *energy)
{
    for (int32_t j = 0; j < np; ++j) {
        double p = p0 + j * dp;
        for (int32_t i = 0; i < ntau; ++i) {
            int32_t n0 = i * tau_stride;
            double num = 0.0, den = 0.0;
            for (int32_t n = n0; n < n0 + win; ++n) {
                double stack = 0.0, energy = 0.0;
                for (int32_t m = 0; m < nrec; ++m) {
                    /* the arrival at receiver m comes p*offset_m later */
                    double v = trace_at(traces + (int64_t)m * nt, nt, n + p * offset[m] / dt);
                    stack += v;
                    energy += v * v;
                }
                num += stack * stack;
                den += energy;
            }
            coh[(int64_t)j * ntau + i] = den > 0.0 ? num / (nrec * den) : 0.0;
            if (energy) energy[(int64_t)j * ntau + i] = den;
        }
    }
}

void orc_starting_model(int32_t NR, int32_t NZ, double dr, double a, double dist,
                        const double *vp_wall, const double *vs_wall, const double *vp_far,
                        const double *vs_far, double vp_fluid, double *vp, double *vs)
{
    for (int32_t i = 0; i < NR; ++i) {
        double r = (i + 0.5) * dr;
        for (int32_t k = 0; k < NZ; ++k) {
            int64_t c = (int64_t)i * NZ + k;
            if (r < a) {
                vp[c] = vp_fluid;
                vs[c] = 0.0;
                continue;
            }
            double f = (r - a) / dist;
            if (f > 1.0) f = 1.0;
            vp[c] = vp_wall[k] + f * (vp_far[k] - vp_wall[k]);
            vs[c] = vs_wall[k] + f * (vs_far[k] - vs_wall[k]);
        }
    }
}

/* ===========================================================================
 * Assembled operators: the leapfrog step of Eq. 2 written as two sparse linear
 * maps over the 14-plane state, V (velocity update and its PML memories) then
 * S (stress update and its PML memories), for staggered differences of order
 * 2 or 4 in space.  The fourth-order scheme (the finite-difference scheme the
 * Method section cites is of this family; the order is a reading) replaces
 * every staggered difference and every two-point 1/r average by
 *     D f = [c1 (f(+1/2) - f(-1/2)) + c2 (f(+3/2) - f(-3/2))] / h,
 *     I f =  g1 (f(+1/2) + f(-1/2)) + g2 (f(+3/2) + f(-3/2)),
 * c1 = 9/8, c2 = -1/24, g1 = 9/16, g2 = -1/16 (order 2: 1, 0, 1/2, 0, which is
 * the hand-written step above).  D + I/r is then exactly the conservative
 * (1/r) d(r f)/dr of the wider stencil.  Values beyond the outer radius and
 * the axial ends are zero; across the axis the fields are mirrored: those at
 * half radial positions (normal stresses, v_z) are even, those at integer
 * positions (v_r, tau_rz) odd and zero on the axis.  Medium averaging, PML
 * and receivers are those of the second-order step; the on-axis source is
 * divided by the axis cell's weight in the norm of the discrete divergence
 * theorem (src_scale_order), which is 1 at order 2.
 *
 * Each row of V and S is assembled from the stencil as written; the adjoint is
 * the transpose of the assembled rows applied in scatter form, so it is exact
 * by construction.
 * ========================================================================= */
enum { P_VR = 0, P_VZ, P_TRR, P_TTT, P_TZZ, P_TRZ, P_PA, P_PB, P_PC, P_PD, P_PE, P_PF, P_PG,
       P_PH, P_N };

typedef struct {
    size_t n, cap;
    int64_t *col;
    double *val;
} lform;

typedef struct {
    size_t nrow, nnz, cap;
    size_t *ptr;
    int64_t *col;
    double *val;
} spm;

typedef struct {
    const grid *G;
    size_t N;
    double c1, c2, g1, g2;
} asm_ctx;

static int lf_push(lform *L, int64_t col, double v)
{
    if (v == 0.0) return 0;
    if (L->n == L->cap) {
        size_t nc = L->cap ? 2 * L->cap : 32;
        int64_t *c = realloc(L->col, nc * sizeof(int64_t));
        if (!c) return -1;
        L->col = c;
        double *w = realloc(L->val, nc * sizeof(double));
        if (!w) return -1;
        L->val = w;
        L->cap = nc;
    }
    L->col[L->n] = col;
    L->val[L->n] = v;
    ++L->n;
    return 0;
}

/* the value of plane p at radial row i, axial row k, with the axis mirror and
 * zero outside the grid */
static void lf_at(lform *L, const asm_ctx *A, int p, int i, int k, double v)
{
    const int NR = A->G->NR, NZ = A->G->NZ;
    if (k < 0 || k >= NZ) return;
    const int odd = (p == P_VR || p == P_TRZ);
    if (i < 0) {
        if (odd) {
            i = -i;
            v = -v;
        } else {
            i = -1 - i;
        }
    }
    if (odd && i == 0) return; /* zero on the axis */
    if (i >= NR) return;
    lf_push(L, (int64_t)p * (int64_t)A->N + (int64_t)IX(i, k), v);
}

/* D (scaled by s/h) and I (scaled by s) along r or z of plane p; lo is the
 * index of the input just below the output node */
static void lf_D(lform *L, const asm_ctx *A, int p, int radial, int i, int k, int lo, double s)
{
    const double h = radial ? A->G->dr : A->G->dz;
    const double w1 = A->c1 * s / h, w2 = A->c2 * s / h;
    if (radial) {
        lf_at(L, A, p, lo + 1, k, w1);
        lf_at(L, A, p, lo, k, -w1);
        lf_at(L, A, p, lo + 2, k, w2);
        lf_at(L, A, p, lo - 1, k, -w2);
    } else {
        lf_at(L, A, p, i, lo + 1, w1);
        lf_at(L, A, p, i, lo, -w1);
        lf_at(L, A, p, i, lo + 2, w2);
        lf_at(L, A, p, i, lo - 1, -w2);
    }
}
static void lf_I(lform *L, const asm_ctx *A, int p, int i, int k, int lo, double s)
{
    lf_at(L, A, p, lo + 1, k, A->g1 * s);
    lf_at(L, A, p, lo, k, A->g1 * s);
    lf_at(L, A, p, lo + 2, k, A->g2 * s);
    lf_at(L, A, p, lo - 1, k, A->g2 * s);
}

static void lf_scaled(lform *dst, const lform *src, double s)
{
    for (size_t q = 0; q < src->n; ++q) lf_push(dst, src->col[q], s * src->val[q]);
}

static int spm_row(spm *M, const lform *L)
{
    if (M->nnz + L->n > M->cap) {
        size_t nc = M->cap ? M->cap : 1024;
        while (nc < M->nnz + L->n) nc *= 2;
        int64_t *c = realloc(M->col, nc * sizeof(int64_t));
        if (!c) return -1;
        M->col = c;
        double *w = realloc(M->val, nc * sizeof(double));
        if (!w) return -1;
        M->val = w;
        M->cap = nc;
    }
    memcpy(M->col + M->nnz, L->col, L->n * sizeof(int64_t));
    memcpy(M->val + M->nnz, L->val, L->n * sizeof(double));
    M->nnz += L->n;
    M->ptr[++M->nrow] = M->nnz;
    return 0;
}

static void spm_free(spm *M)
{
    free(M->ptr);
    free(M->col);
    free(M->val);
}

/* y = M x (all rows) or y += M^T x */
static void spm_apply(const spm *M, const double *x, double *y)
{
    for (size_t r = 0; r < M->nrow; ++r) {
        double s = 0.0;
        for (size_t q = M->ptr[r]; q < M->ptr[r + 1]; ++q) s += M->val[q] * x[M->col[q]];
        y[r] = s;
    }
}
static void spm_apply_t(const spm *M, const double *x, double *y)
{
    for (size_t r = 0; r < M->nrow; ++r) {
        const double xr = x[r];
        if (xr == 0.0) continue;
        for (size_t q = M->ptr[r]; q < M->ptr[r + 1]; ++q) y[M->col[q]] += M->val[q] * xr;
    }
}

/* A derivative form D with its PML memory: with the memory on, the row of the
 * memory is psi' = b psi + a D and the derivative used is D + psi' =
 * (1 + a) D + b psi. */
static void pml_pair(const asm_ctx *A, const lform *D, int on, double a, double b, int64_t psi,
                     lform *eff, lform *psirow)
{
    if (on) {
        lf_scaled(eff, D, 1.0 + a);
        lf_push(eff, psi, b);
        lf_push(psirow, psi, b);
        lf_scaled(psirow, D, a);
    } else {
        lf_scaled(eff, D, 1.0);
        lf_push(psirow, psi, 1.0);
    }
    (void)A;
}

typedef struct {
    spm V, S, E; /* E: 4 N strain rows (e_rr', e_tt, e_zz', e_z' + e_r') over the state after V */
    spm B;       /* B: 2 N rows d v_r / d b_R, d v_z / d b_Z over the state before V */
    spm H;       /* H: 4 N plain strain rows (no PML stretching: e_rr, e_tt, e_zz,
                    e_z + e_r) over the state after V */
} asm_ops;

static void ops_free(asm_ops *O)
{
    spm_free(&O->V);
    spm_free(&O->S);
    spm_free(&O->E);
    spm_free(&O->B);
    spm_free(&O->H);
}

static int ops_build(const grid *G, int order, asm_ops *O)
{
    memset(O, 0, sizeof(*O));
    asm_ctx A;
    A.G = G;
    A.N = (size_t)G->NR * G->NZ;
    if (order == 2) {
        A.c1 = 1.0; A.c2 = 0.0; A.g1 = 0.5; A.g2 = 0.0;
    } else if (order == 4) {
        A.c1 = 9.0 / 8.0; A.c2 = -1.0 / 24.0; A.g1 = 9.0 / 16.0; A.g2 = -1.0 / 16.0;
    } else {
        return -1;
    }
    const int NR = G->NR, NZ = G->NZ;
    const size_t N = A.N;
    const double dt = G->dt, dr = G->dr;
    O->V.ptr = calloc(P_N * N + 1, sizeof(size_t));
    O->S.ptr = calloc(P_N * N + 1, sizeof(size_t));
    O->E.ptr = calloc(4 * N + 1, sizeof(size_t));
    O->B.ptr = calloc(2 * N + 1, sizeof(size_t));
    O->H.ptr = calloc(4 * N + 1, sizeof(size_t));
    if (!O->V.ptr || !O->S.ptr || !O->E.ptr || !O->B.ptr || !O->H.ptr) {
        ops_free(O);
        return -1;
    }
    /* rows of V and S in state order: plane-major, then (i, k); each plane's
     * rows are collected per node first (some nodes define several planes) */
    lform *rowV = calloc(P_N * N, sizeof(lform)), *rowS = calloc(P_N * N, sizeof(lform));
    lform *rowE = calloc(4 * N, sizeof(lform));
    lform *rowB = calloc(2 * N, sizeof(lform)), *rowH = calloc(4 * N, sizeof(lform));
    if (!rowV || !rowS || !rowE || !rowB || !rowH) {
        free(rowV); free(rowS); free(rowE); free(rowB); free(rowH);
        ops_free(O);
        return -1;
    }
#define ROW(R, p, c) (&(R)[(size_t)(p) * N + (c)])
#define COL(p, c) ((int64_t)(p) * (int64_t)N + (int64_t)(c))
    for (int i = 0; i < NR; ++i)
        for (int k = 0; k < NZ; ++k) {
            const size_t c = IX(i, k);
            lform t = {0};
            /* ---- V: v_r at R(i,k), i >= 1 */
            if (i >= 1) {
                lform Dr = {0}, Dz = {0}, vr = {0};
                lf_D(&Dr, &A, P_TRR, 1, i, k, i - 1, 1.0);
                lf_D(&Dz, &A, P_TRZ, 0, i, k, k - 1, 1.0);
                const double bR = buoy_R(G, i, k), ri = i * dr;
                lf_push(&vr, COL(P_VR, c), 1.0);
                lform eff = {0};
                pml_pair(&A, &Dr, G->onr_i[i], G->ar_i[i], G->br_i[i], COL(P_PA, c), &eff,
                         ROW(rowV, P_PA, c));
                pml_pair(&A, &Dz, G->onz_i[k], G->az_i[k], G->bz_i[k], COL(P_PB, c), &eff,
                         ROW(rowV, P_PB, c));
                lf_I(&eff, &A, P_TRR, i, k, i - 1, 1.0 / ri);
                lf_I(&eff, &A, P_TTT, i, k, i - 1, -1.0 / ri);
                lf_scaled(&vr, &eff, dt * bR);
                lf_scaled(ROW(rowB, 0, c), &eff, dt);
                *ROW(rowV, P_VR, c) = vr;
                free(Dr.col); free(Dr.val); free(Dz.col); free(Dz.val);
                free(eff.col); free(eff.val);
            } else {
                lf_push(ROW(rowV, P_VR, c), COL(P_VR, c), 1.0);
                lf_push(ROW(rowV, P_PA, c), COL(P_PA, c), 1.0);
                lf_push(ROW(rowV, P_PB, c), COL(P_PB, c), 1.0);
            }
            /* ---- V: v_z at Z(i,k) */
            {
                lform Dr = {0}, Dz = {0}, vz = {0}, eff = {0};
                lf_D(&Dr, &A, P_TRZ, 1, i, k, i, 1.0);
                lf_D(&Dz, &A, P_TZZ, 0, i, k, k, 1.0);
                const double bZ = buoy_Z(G, i, k), rh = (i + 0.5) * dr;
                lf_push(&vz, COL(P_VZ, c), 1.0);
                pml_pair(&A, &Dr, G->onr_h[i], G->ar_h[i], G->br_h[i], COL(P_PC, c), &eff,
                         ROW(rowV, P_PC, c));
                pml_pair(&A, &Dz, G->onz_h[k], G->az_h[k], G->bz_h[k], COL(P_PD, c), &eff,
                         ROW(rowV, P_PD, c));
                lf_I(&eff, &A, P_TRZ, i, k, i, 1.0 / rh);
                lf_scaled(&vz, &eff, dt * bZ);
                lf_scaled(ROW(rowB, 1, c), &eff, dt);
                *ROW(rowV, P_VZ, c) = vz;
                free(Dr.col); free(Dr.val); free(Dz.col); free(Dz.val);
                free(eff.col); free(eff.val);
            }
            /* V leaves the stresses and their memories alone */
            for (int p = P_TRR; p <= P_TRZ; ++p) lf_push(ROW(rowV, p, c), COL(p, c), 1.0);
            for (int p = P_PE; p <= P_PH; ++p) lf_push(ROW(rowV, p, c), COL(p, c), 1.0);

            /* ---- S: normal stresses at C(i,k) */
            {
                lform Dr = {0}, Dz = {0}, err = {0}, ett = {0}, ezz = {0};
                lf_D(&Dr, &A, P_VR, 1, i, k, i, 1.0);
                lf_D(&Dz, &A, P_VZ, 0, i, k, k - 1, 1.0);
                lf_scaled(ROW(rowH, 0, c), &Dr, 1.0);
                lf_scaled(ROW(rowH, 2, c), &Dz, 1.0);
                const double rh = (i + 0.5) * dr;
                pml_pair(&A, &Dr, G->onr_h[i], G->ar_h[i], G->br_h[i], COL(P_PE, c), &err,
                         ROW(rowS, P_PE, c));
                pml_pair(&A, &Dz, G->onz_i[k], G->az_i[k], G->bz_i[k], COL(P_PF, c), &ezz,
                         ROW(rowS, P_PF, c));
                lf_I(&ett, &A, P_VR, i, k, i, 1.0 / rh);
                const double l = G->lam[c], m = G->mu[c];
                const double wr[3] = {l + 2.0 * m, l, l}, wt[3] = {l, l + 2.0 * m, l},
                             wz[3] = {l, l, l + 2.0 * m};
                const int pl[3] = {P_TRR, P_TTT, P_TZZ};
                for (int q = 0; q < 3; ++q) {
                    lform *R = ROW(rowS, pl[q], c);
                    lf_push(R, COL(pl[q], c), 1.0);
                    lf_scaled(R, &err, dt * wr[q]);
                    lf_scaled(R, &ett, dt * wt[q]);
                    lf_scaled(R, &ezz, dt * wz[q]);
                }
                lf_scaled(ROW(rowE, 0, c), &err, 1.0);
                lf_scaled(ROW(rowE, 1, c), &ett, 1.0);
                lf_scaled(ROW(rowH, 1, c), &ett, 1.0);
                lf_scaled(ROW(rowE, 2, c), &ezz, 1.0);
                free(Dr.col); free(Dr.val); free(Dz.col); free(Dz.val);
                free(err.col); free(err.val); free(ett.col); free(ett.val);
                free(ezz.col); free(ezz.val);
            }
            /* ---- S: tau_rz at S(i,k), i >= 1 */
            if (i >= 1) {
                lform Dz = {0}, Dr = {0}, es = {0};
                lf_D(&Dz, &A, P_VR, 0, i, k, k, 1.0);
                lf_D(&Dr, &A, P_VZ, 1, i, k, i - 1, 1.0);
                lf_scaled(ROW(rowH, 3, c), &Dz, 1.0);
                lf_scaled(ROW(rowH, 3, c), &Dr, 1.0);
                pml_pair(&A, &Dz, G->onz_h[k], G->az_h[k], G->bz_h[k], COL(P_PG, c), &es,
                         ROW(rowS, P_PG, c));
                pml_pair(&A, &Dr, G->onr_i[i], G->ar_i[i], G->br_i[i], COL(P_PH, c), &es,
                         ROW(rowS, P_PH, c));
                lform *R = ROW(rowS, P_TRZ, c);
                lf_push(R, COL(P_TRZ, c), 1.0);
                lf_scaled(R, &es, dt * mu_S(G, i, k));
                lf_scaled(ROW(rowE, 3, c), &es, 1.0);
                free(Dz.col); free(Dz.val); free(Dr.col); free(Dr.val);
                free(es.col); free(es.val);
            } else {
                lf_push(ROW(rowS, P_TRZ, c), COL(P_TRZ, c), 1.0);
                lf_push(ROW(rowS, P_PG, c), COL(P_PG, c), 1.0);
                lf_push(ROW(rowS, P_PH, c), COL(P_PH, c), 1.0);
            }
            /* S leaves the velocities and their memories alone */
            for (int p = P_VR; p <= P_VZ; ++p) lf_push(ROW(rowS, p, c), COL(p, c), 1.0);
            for (int p = P_PA; p <= P_PD; ++p) lf_push(ROW(rowS, p, c), COL(p, c), 1.0);
            (void)t;
        }
    int rc = 0;
    for (size_t r = 0; r < P_N * N && !rc; ++r) rc |= spm_row(&O->V, &rowV[r]);
    for (size_t r = 0; r < P_N * N && !rc; ++r) rc |= spm_row(&O->S, &rowS[r]);
    for (size_t r = 0; r < 4 * N && !rc; ++r) rc |= spm_row(&O->E, &rowE[r]);
    for (size_t r = 0; r < 2 * N && !rc; ++r) rc |= spm_row(&O->B, &rowB[r]);
    for (size_t r = 0; r < 4 * N && !rc; ++r) rc |= spm_row(&O->H, &rowH[r]);
    for (size_t r = 0; r < P_N * N; ++r) {
        free(rowV[r].col); free(rowV[r].val); free(rowS[r].col); free(rowS[r].val);
    }
    for (size_t r = 0; r < 4 * N; ++r) {
        free(rowE[r].col); free(rowE[r].val); free(rowH[r].col); free(rowH[r].val);
    }
    for (size_t r = 0; r < 2 * N; ++r) {
        free(rowB[r].col); free(rowB[r].val);
    }
    free(rowV); free(rowS); free(rowE); free(rowB); free(rowH);
#undef ROW
#undef COL
    if (rc) ops_free(O);
    return rc;
}

/* one step s <- S (V s) plus the source; eps (nullable, 4 N) receives the
 * strain rates the stress update used */
static void asm_step(const asm_ops *O, size_t N, int NZ, double *s, double *tmp, int src_k,
                     double srcval, double *eps)
{
    spm_apply(&O->V, s, tmp);
    if (eps) spm_apply(&O->E, tmp, eps);
    spm_apply(&O->S, tmp, s);
    size_t c = IX(0, src_k);
    s[P_TRR * N + c] += srcval;
    s[P_TTT * N + c] += srcval;
    s[P_TZZ * N + c] += srcval;
}

/* the transpose of asm_step without the source: a <- V^T (S^T a) */
static void asm_step_t(const asm_ops *O, size_t N, double *a, double *tmp)
{
    memset(tmp, 0, P_N * N * sizeof(double));
    spm_apply_t(&O->S, a, tmp);
    memset(a, 0, P_N * N * sizeof(double));
    spm_apply_t(&O->V, tmp, a);
}

int orc_forward_asm(const orc_geom *g, int32_t order, const double *lam, const double *mu,
                    const double *rho, const double *wavelet, double *traces,
                    double *final_state)
{
    grid G;
    if (grid_init(&G, g, lam, mu, rho) || !geom_ok(g)) return -1;
    asm_ops O;
    if (ops_build(&G, order, &O)) {
        grid_free(&G);
        return -1;
    }
    const int NZ = G.NZ;
    const size_t N = (size_t)G.NR * G.NZ;
    double *s = calloc(P_N * N, sizeof(double)), *tmp = calloc(P_N * N, sizeof(double));
    int rc = (!s || !tmp) ? -1 : 0;
    const double sc = src_scale_order(&G, order);
    for (int n = 0; n < g->nt && !rc; ++n) {
        asm_step(&O, N, NZ, s, tmp, g->src_k, sc * wavelet[n], NULL);
        for (int j = 0; j < g->nrec; ++j) {
            size_t c = IX(0, g->rec_k[j]);
            traces[(size_t)j * g->nt + n] = (s[P_TRR * N + c] + s[P_TTT * N + c] +
                                             s[P_TZZ * N + c]) / 3.0;
        }
    }
    if (!rc && final_state) memcpy(final_state, s, P_N * N * sizeof(double));
    free(s); free(tmp);
    ops_free(&O);
    grid_free(&G);
    return rc;
}

int orc_propagate_asm(const orc_geom *g, int32_t order, const double *lam, const double *mu,
                      const double *rho, double *st, int32_t nsteps, int32_t adjoint)
{
    grid G;
    if (grid_init(&G, g, lam, mu, rho) || !geom_ok(g)) return -1;
    asm_ops O;
    if (ops_build(&G, order, &O)) {
        grid_free(&G);
        return -1;
    }
    const int NZ = G.NZ;
    const size_t N = (size_t)G.NR * G.NZ;
    double *tmp = calloc(P_N * N, sizeof(double));
    if (!tmp) {
        ops_free(&O);
        grid_free(&G);
        return -1;
    }
    for (int n = 0; n < nsteps; ++n) {
        if (adjoint)
            asm_step_t(&O, N, st, tmp);
        else
            asm_step(&O, N, NZ, st, tmp, g->src_k, 0.0, NULL);
    }
    free(tmp);
    ops_free(&O);
    grid_free(&G);
    return 0;
}

int orc_gradient_asm(const orc_geom *g, int32_t order, const double *lam, const double *mu,
                     const double *rho, const double *wavelet, const double *resid,
                     int32_t seg, double *glam, double *gmu, double *illum, double *grho,
                     double *hl, double *hm)
{
    grid G;
    if (seg <= 0 || grid_init(&G, g, lam, mu, rho) || !geom_ok(g)) return -1;
    asm_ops O;
    if (ops_build(&G, order, &O)) {
        grid_free(&G);
        return -1;
    }
    const int NR = G.NR, NZ = G.NZ, nt = g->nt;
    const double dt = G.dt;
    const size_t N = (size_t)NR * NZ, SL = P_N * N;
    const int nseg = (nt + seg - 1) / seg;
    double *ckpt = malloc((size_t)(nseg > 0 ? nseg : 1) * SL * sizeof(double));
    double *s = calloc(SL, sizeof(double)), *a = calloc(SL, sizeof(double));
    double *tmp = calloc(SL, sizeof(double));
    double *eps = malloc((size_t)seg * 4 * N * sizeof(double));
    double *gmuS = calloc(N, sizeof(double));
    /* density: d v^{n+1/2} / d b per step of a segment (B applied to the state
     * before the step) and dJ/db at the v_r and v_z nodes; pseudo-Hessian: the
     * plain strain rates of v^{n+1/2} */
    double *dvb = grho ? malloc((size_t)seg * 2 * N * sizeof(double)) : NULL;
    double *gb = grho ? calloc(2 * N, sizeof(double)) : NULL;
    double *hp = (hl || hm) ? malloc(4 * N * sizeof(double)) : NULL;
    if (!ckpt || !s || !a || !tmp || !eps || !gmuS || (grho && (!dvb || !gb)) ||
        ((hl || hm) && !hp)) {
        free(ckpt); free(s); free(a); free(tmp); free(eps); free(gmuS);
        free(dvb); free(gb); free(hp);
        ops_free(&O);
        grid_free(&G);
        return -1;
    }
    const double sc = src_scale_order(&G, order);
    memset(glam, 0, N * sizeof(double));
    memset(gmu, 0, N * sizeof(double));
    memset(illum, 0, N * sizeof(double));
    if (hl) memset(hl, 0, N * sizeof(double));
    if (hm) memset(hm, 0, N * sizeof(double));
    /* forward pass: checkpoints, illumination from v^{n+1/2} averaged to C nodes */
    for (int n = 0; n < nt; ++n) {
        if (n % seg == 0) memcpy(ckpt + (size_t)(n / seg) * SL, s, SL * sizeof(double));
        asm_step(&O, N, NZ, s, tmp, g->src_k, sc * wavelet[n], NULL);
        if (hp) {
            /* virtual sources: d(stress update)/d(modulus) applied to v^{n+1/2},
             * with the plain strain rates of the stencil (the stress update
             * leaves v alone, so H may read the state after the whole step) */
            spm_apply(&O.H, s, hp);
            for (size_t c = 0; c < N; ++c) {
                double err = hp[c], ett = hp[N + c], ezz = hp[2 * N + c], es = hp[3 * N + c];
                double dv = err + ett + ezz;
                if (hl) hl[c] += dt * dt * 3.0 * dv * dv;
                if (hm) hm[c] += dt * dt * (4.0 * (err * err + ett * ett + ezz * ezz) + es * es);
            }
        }
        const double *vr = s + P_VR * N, *vz = s + P_VZ * N;
        for (int i = 0; i < NR; ++i)
            for (int k = 0; k < NZ; ++k) {
                size_t c = IX(i, k);
                double vr_ip = i + 1 < NR ? vr[IX(i + 1, k)] : 0.0;
                double vz_km = k > 0 ? vz[IX(i, k - 1)] : 0.0;
                double ur = 0.5 * (vr[c] + vr_ip), uz = 0.5 * (vz_km + vz[c]);
                illum[c] += dt * (ur * ur + uz * uz);
            }
    }
    /* reverse pass, one segment at a time */
    for (int j = nseg - 1; j >= 0; --j) {
        int n0 = j * seg, n1 = n0 + seg < nt ? n0 + seg : nt;
        memcpy(s, ckpt + (size_t)j * SL, SL * sizeof(double));
        for (int n = n0; n < n1; ++n) {
            if (dvb) spm_apply(&O.B, s, dvb + (size_t)(n - n0) * 2 * N);
            asm_step(&O, N, NZ, s, tmp, g->src_k, sc * wavelet[n], eps + (size_t)(n - n0) * 4 * N);
        }
        for (int n = n1 - 1; n >= n0; --n) {
            for (int q = 0; q < g->nrec; ++q) {
                size_t c = IX(0, g->rec_k[q]);
                double r3 = resid[(size_t)q * nt + n] / 3.0;
                a[P_TRR * N + c] += r3;
                a[P_TTT * N + c] += r3;
                a[P_TZZ * N + c] += r3;
            }
            const double *e = eps + (size_t)(n - n0) * 4 * N;
            /* Eq. 7 and Eq. 8 with the strain rates of this scheme */
            for (size_t c = 0; c < N; ++c) {
                double err = e[c], ett = e[N + c], ezz = e[2 * N + c];
                double atr = a[P_TRR * N + c], att = a[P_TTT * N + c], atz = a[P_TZZ * N + c];
                double sa = atr + att + atz;
                glam[c] += dt * (err + ett + ezz) * sa;
                gmu[c] += dt * 2.0 * (err * atr + ett * att + ezz * atz);
                gmuS[c] += dt * e[3 * N + c] * a[P_TRZ * N + c];
            }
            asm_step_t(&O, N, a, tmp);
            if (gb) {
                /* tmp now holds S^T a: at the velocity rows, dJ/dv^{n+1/2};
                 * v^{n+1/2} = v^{n-1/2} + b dv/db gives dJ/db += that times dv/db */
                const double *d = dvb + (size_t)(n - n0) * 2 * N;
                for (size_t c = 0; c < N; ++c) {
                    gb[c] += tmp[P_VR * N + c] * d[c];
                    gb[N + c] += tmp[P_VZ * N + c] * d[N + c];
                }
            }
        }
    }
    if (grho) rho_chain(&G, gb, grho);
    fold_mu_s(&G, gmuS, gmu);
    free(ckpt); free(s); free(a); free(tmp); free(eps); free(gmuS);
    free(dvb); free(gb); free(hp);
    ops_free(&O);
    grid_free(&G);
    return 0;
}
