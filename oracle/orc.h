/*
 * orc.h -- FP64 CPU oracle for monopole borehole acoustic FWI
 *          (Tang, Cheng, Li & Fang, "Borehole acoustic full-waveform inversion").
 *
 * TEST INFRASTRUCTURE.  This library exists only to check the HIP path.  It is
 * loaded by the tests, by the smoke check and by the CPU-baseline leg of the
 * benchmark, never by the product path.  It shares no code, header, table or
 * constant with the HIP library: everything here is written from the paper's
 * equations and from the discretisation readings listed in the design notes.
 *
 * Plain, serial, double precision.  No blocking, no fusion, no reordering
 * beyond what the equations state.
 *
 * Grid (one shot).  NR = nr + pr radial rows i, NZ = nz + 2*pz axial columns k,
 * k contiguous in memory, index i*NZ + k.  Node families (staggered, Method
 * section, Eq. 2):
 *   C (i,k) at (r = (i+1/2)dr, z = k dz)      tau_rr, tau_tt, tau_zz, lambda, mu, rho
 *   R (i,k) at (r = i dr,      z = k dz)      v_r        (v_r = 0 on the axis, i = 0)
 *   Z (i,k) at (r = (i+1/2)dr, z = (k+1/2)dz) v_z
 *   S (i,k) at (r = i dr,      z = (k+1/2)dz) tau_rz     (tau_rz = 0 on the axis)
 * Every field read outside [0,NR) x [0,NZ) is zero.
 *
 * Parity status of each entry point is stated in its comment.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

typedef struct {
    int32_t nr, nz, pr, pz;   /* physical cells, PML widths (outer r, both z ends) */
    double dr, dz, dt;        /* metres, seconds */
    int32_t nt;               /* time steps */
    double f0;                /* Hz: PML frequency shift alpha_max = pi*f0 */
    double vmax;              /* m/s: PML damping reference velocity (fixed per shot) */
    int32_t src_k;            /* C row of the on-axis source, padded-grid index */
    int32_t nrec;             /* on-axis receivers */
    const int32_t *rec_k;     /* their C rows, padded-grid index */
} orc_geom;

/* Eq. 3-4: lambda = rho Vp^2 - 2 rho Vs^2, mu = rho Vs^2.  Pinned by closed form. */
void orc_moduli(int64_t n, const double *vp, const double *vs, const double *rho,
                double *lam, double *mu);
/* Chain rule of Eq. 3-4: dJ/dVp = 2 rho Vp dJ/dlambda,
 * dJ/dVs = -4 rho Vs dJ/dlambda + 2 rho Vs dJ/dmu, and (grho nullable) the
 * moduli's share of dJ/drho at fixed velocities,
 * (Vp^2 - 2 Vs^2) dJ/dlambda + Vs^2 dJ/dmu.  Pinned by central differences
 * of the misfit in velocity space. */
void orc_moduli_grad(int64_t n, const double *vp, const double *vs, const double *rho,
                     const double *glam, const double *gmu, double *gvp, double *gvs,
                     double *grho);
/* Eq. 11-12: Vp = sqrt((lambda+2mu)/rho), Vs = sqrt(mu/rho). */
void orc_velocities(int64_t n, const double *lam, const double *mu, const double *rho,
                    double *vp, double *vs);

/* Eq. 2 forward modelling; traces[j*nt + n] = mean normal stress at receiver j
 * after step n (time (n+1) dt).  final_state (nullable) receives the full state
 * (orc_state_len doubles) after the last step.  Returns 0 or -1 on bad input. */
int orc_forward(const orc_geom *g, const double *lam, const double *mu, const double *rho,
                const double *wavelet, double *traces, double *final_state);

/* Eq. 1 and 5: resid = d - dobs, returns J = 0.5 * sum(resid^2). */
double orc_misfit(int64_t n, const double *d, const double *dobs, double *resid);

/* Eq. 6-8 by the exact transpose of the discrete forward, driven by resid
 * (= dJ/dtraces, [nrec][nt]).  Checkpoints every `seg` steps, recomputes each
 * segment storing the strain rates it used, correlates them with the adjoint
 * stresses.  Outputs (NR*NZ each, overwritten): glam = dJ/dlambda,
 * gmu = dJ/dmu (the tau_rz-node harmonic-mean chain rule included; cells with
 * mu <= 0 get only their own-node term), illum = sum_n dt |v|^2 at C nodes,
 * grho (nullable) = dJ/drho through the buoyancies of the velocity update
 * (density held fixed by the paper, inverted jointly as an extension);
 * hl, hm (nullable) = the virtual-source pseudo-Hessian diagonal: with the
 * plain strain rates of v^{n+1/2} at C cells, hl = sum_n 3 dt^2 (div v)^2
 * and hm = sum_n dt^2 (4 (e_rr^2 + e_tt^2 + e_zz^2) + (e_z + e_r)^2), the
 * last term that of the tau_rz node with the cell's index (i >= 1).
 * Pinned by brute-force central differences and by dot-product tests. */
int orc_gradient(const orc_geom *g, const double *lam, const double *mu, const double *rho,
                 const double *wavelet, const double *resid, int32_t seg,
                 double *glam, double *gmu, double *illum, double *grho, double *hl,
                 double *hm);

/* Transpose of the map wavelet -> traces for a fixed model: wadj[n] =
 * d<traces, resid>/d wavelet[n].  Used by the source-to-trace dot-product test. */
int orc_source_adjoint(const orc_geom *g, const double *lam, const double *mu,
                       const double *rho, const double *resid, double *wadj);

/* Full state vector: 14 arrays of NR*NZ doubles in this order:
 * vr vz trr ttt tzz trz psiA..psiH (memory variables of the PML, see orc.c).
 * propagate: nsteps source-free forward steps in place.
 * propagate_adjoint: the exact transpose of propagate, in place.          */
int64_t orc_state_len(const orc_geom *g);
int orc_propagate(const orc_geom *g, const double *lam, const double *mu, const double *rho,
                  double *state, int32_t nsteps);
int orc_propagate_adjoint(const orc_geom *g, const double *lam, const double *mu,
                          const double *rho, double *astate, int32_t nsteps);

/* Diagonal preconditioner (reading of the Numerical Examples section and
 * Fig. 6): P = 1 / (E + eps * max_{mask} E); g <- P*g on mask cells, 0 elsewhere.
 * Returns sum over mask cells of g.(P g) (both parameters): minus the slope of
 * the misfit along the preconditioned descent step. */
double orc_precondition(int64_t n, const double *illum, const uint8_t *mask, double eps,
                        double *g_lam, double *g_mu);

/* Step length of the parabolic line search (reading of Eq. 9-10, whose alpha
 * the paper leaves as a free choice): the quadratic through J0 (slope -gpg) at
 * 0 and J1 at the trial step alpha1; its minimiser clamped to
 * [alpha1/10, 3 alpha1] when the quadratic is convex, else alpha1 when
 * J1 <= J0 and alpha1/2 otherwise; 0 when alpha1 <= 0.  Pinned by exact
 * quadratics and by each branch. */
double orc_line_search(double J0, double J1, double gpg, double alpha1);

/* Eq. 9-10 with one alpha chosen so that the largest change relative to the
 * largest modulus is eta (alpha_override > 0 uses that alpha instead), then a
 * velocity box clip.  Only mask cells change.  Returns alpha. */
/* Semblance (slowness-time coherence) of an on-axis receiver array, the
 * analysis the paper builds its starting models from (Introduction; Fig. 4).
 * traces[m*nt + n]: receiver m at sample n; offset[m]: its axial distance
 * from the array's first receiver (m); slownesses p0 + j dp (s/m),
 * j < np; windows of win samples starting at sample i*tau_stride, i < ntau.
 * coh[j*ntau + i] = sum_n (sum_m x_m(n + p off_m/dt))^2 /
 *                   (nrec sum_n sum_m x_m(n + p off_m/dt)^2),
 * traces interpolated linearly between samples and zero outside the record;
 * 0 where the window holds no energy.  energy (nullable) receives the
 * denominator sum_n sum_m x^2.  Pinned by plane waves (coherence 1 at their
 * slowness) and by the formation velocities of modelled data. */
void orc_semblance(int32_t nrec, int32_t nt, const double *traces, double dt,
                   const double *offset, int32_t np, double p0, double dp,
                   int32_t ntau, int32_t tau_stride, int32_t win, double *coh,
                   double *energy);

/* Starting model (Numerical Examples section): per axial row k, formation
 * velocities vp_wall/vs_wall at the borehole wall r = a and vp_far/vs_far at
 * r = a + dist, linear in r between and constant beyond; cells with
 * r = (i + 1/2) dr < a are fluid (vp_fluid, vs = 0).  NR x NZ outputs. */
void orc_starting_model(int32_t NR, int32_t NZ, double dr, double a, double dist,
                        const double *vp_wall, const double *vs_wall, const double *vp_far,
                        const double *vs_far, double vp_fluid, double *vp, double *vs);

double orc_update(int64_t n, double *lam, double *mu, const double *rho,
                  const double *g_lam, const double *g_mu, const uint8_t *mask,
                  double eta, double alpha_override,
                  double vp_min, double vp_max, double vs_min, double vs_max);

/* The step of Eq. 2 assembled as sparse rows (velocity phase, then stress
 * phase) for staggered differences of order 2 or 4 in space, the adjoint as
 * the transpose of the assembled rows.  order 2 is the scheme of
 * orc_forward/orc_gradient written another way (a cross-check of either);
 * order 4 uses D f = [9/8 (f(+1/2) - f(-1/2)) - 1/24 (f(+3/2) - f(-3/2))] / h
 * and I f = 9/16 (f(+1/2) + f(-1/2)) - 1/16 (f(+3/2) + f(-3/2)) for every
 * difference and 1/r average, with the fields mirrored across the axis (even
 * at half radial positions, odd and zero on the axis at integer ones).
 * Same arguments and outputs as orc_forward, orc_propagate(_adjoint) and
 * orc_gradient.  The density gradient takes dv/db per step from rows of its
 * own (the velocity rows without the buoyancy); the pseudo-Hessian takes the
 * plain strain rates of v^{n+1/2} from rows without the PML stretching.
 * Pinned: order 2 against the hand-written step (all outputs), order 4 by
 * closed forms, convergence, dot products, central differences (moduli and
 * density) and the pseudo-Hessian by differencing one step. */
int orc_forward_asm(const orc_geom *g, int32_t order, const double *lam, const double *mu,
                    const double *rho, const double *wavelet, double *traces,
                    double *final_state);
int orc_propagate_asm(const orc_geom *g, int32_t order, const double *lam, const double *mu,
                      const double *rho, double *st, int32_t nsteps, int32_t adjoint);
int orc_gradient_asm(const orc_geom *g, int32_t order, const double *lam, const double *mu,
                     const double *rho, const double *wavelet, const double *resid,
                     int32_t seg, double *glam, double *gmu, double *illum, double *grho,
                     double *hl, double *hm);

#endif
