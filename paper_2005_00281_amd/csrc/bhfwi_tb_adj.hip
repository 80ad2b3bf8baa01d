// bhfwi_tb_adj.hip -- temporally blocked adjoint step (Eq. 6 as the exact
// transpose of the discrete forward) fused with the zero-lag correlation of
// Eq. 7-8 and the illumination.
//
// Same tiling as the forward kernel: a workgroup of W wave64 owns TRE - 2T
// radial by 64 - 2T axial cells, loads them with a T-cell halo, and runs T
// reverse steps n_hi, n_hi - 1, ... with the adjoint state, the medium
// coefficients, the PML recursions and the gradient sums of its cells in
// registers.  Per step:
//   A  inject the residual at the receivers; drivers of the transposed stress
//      update at C and S nodes (sigma = C a_tau, plus the PML recursions)
//      -> LDS; stage the stored v^{n+1/2} of the tile in LDS;
//   B  correlate; transposed stress update into a_v at R and Z nodes, then
//      the transposed velocity update products -> LDS;
//   C  gather the products into a_tau.
// Only values needed by the radial neighbour rows (other waves) go through
// LDS; the axial neighbours are lanes of the same wave and are read with DPP
// wavefront shifts, which keeps the LDS footprint at 8 planes.
// The gradient and illumination sums stay in registers for the T steps and
// are added to the accumulators once per launch (owned cells only).  As in
// the forward kernel the step loop has no per-cell branches: zero
// coefficients keep cells outside the grid and the axis nodes inert, and rows
// that have fallen out of the correct region are skipped (whole-wave
// branches).  From two rows per thread the values a lane wrote to LDS are
// read back from there instead of being held across the barriers, which
// keeps the PML-free kernel within 64 registers without spills.
//
// Optional outputs, selected by the bits of X (extensions of the paper, which
// holds the density fixed and gives the preconditioner only as diagonal):
//
// X & 1 adds the density correlation.  The velocity update is v^{n+1/2} = v^{n-1/2} + b dv_n with
// buoyancy b, so dJ/db = sum_n a_v^n dv_n with a_v^n the adjoint velocity
// after the transposed stress update of step n.  Summed by parts, with
// a_v^{nt} = 0 and v^{-1/2} = 0, b dJ/db = sum_n (a_v^n - a_v^{n+1}) v^{n+1/2},
// and a_v^n - a_v^{n+1} is exactly the phase-B increment of a_v (the
// transposed velocity update leaves a_v unchanged).  The kernel accumulates
// that increment times the stored v^{n+1/2} at the R and Z nodes, so no
// history beyond the velocities already kept is needed.
//
// X & 4 records the transpose of the source injection: at each step the sum
// of the three adjoint normal stresses of the on-axis source cell, which is
// dJ/dtau^{n+1} there, times the source scale gives dJ/dw[n], the gradient
// with respect to the source wavelet (the transpose of wavelet -> traces).
//
// X & 2 adds the virtual-source pseudo-Hessian diagonal: with the strain
// rates of v^{n+1/2}, H_lambda += 3 dt^2 (e_rr + e_tt + e_zz)^2 (the lambda
// derivative of the three normal-stress updates) and H_mu += dt^2 (4 (e_rr^2 +
// e_tt^2 + e_zz^2) + (e_z + e_r)^2), the last term that of the tau_rz node with
// the cell's index.
#pragma once
#include "bhfwi_internal.h"
#include "bhfwi_tb_fwd.hip"

namespace bhfwi {

template <int T, int TRE, int W, int PM, int X>
__global__ void __launch_bounds__(64 * W, (W >= 16 && (TRE == W || (PM == 0 && TRE <= 2 * W))) ? 8 : 1)
k_adj_tb(const ShotDev* __restrict__ shots, const int4* __restrict__ work, int nwork, int map,
         int n_hi, int nsteps, const float* __restrict__ lam, const float* __restrict__ mu,
         const float* __restrict__ rho, const int* __restrict__ rec_k,
         const float* __restrict__ resid, const float* __restrict__ pml_r,
         const float* __restrict__ pml_z, const float* __restrict__ ain,
         float* __restrict__ aout, const float* __restrict__ hist_hi, long long hist_stride,
         float* __restrict__ acc, float* __restrict__ acc_rho, float* __restrict__ acc_h,
         float* __restrict__ wgrad, long long cells_total)
{
    static_assert(TRE % W == 0 && TRE > 2 * T && 64 > 2 * T, "tile too small for the halo");
    constexpr bool RHO = (X & 1) != 0, HES = (X & 2) != 0, WAV = (X & 4) != 0;
    constexpr int RPT = TRE / W;
    // LDSE: the values this lane wrote to LDS are read back from there rather
    // than held in registers across the barriers (fewer live registers: no
    // spills at two rows per thread and 64 VGPRs)
    constexpr bool LDSE = RPT >= 2;
    constexpr int LDW = (TRE + 2) * 64;
    enum { ERR = 0, ETT, ER, UR, HR, ZR, HVR, HVZ, NPL };
    __shared__ float L[NPL][LDW];
    __shared__ float Lres[T][64];  // residual/3 of this lane's receiver, per step

    const int wg = xcd_chunk(blockIdx.x, nwork, map);
    if (wg >= nwork) return;
    const int4 wk = work[wg];
    const ShotDev& S = shots[wk.x];
    // steps n_hi - t, t = t0 .. nsteps-1, that this shot runs (n < nt)
    const int t0 = max(0, n_hi - (S.nt - 1));
    if (t0 >= nsteps) return;  // uniform over the workgroup

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int NR = S.NR, NZ = S.NZ, nr = S.nr, pz = S.pz;
    const long long cells = (long long)NR * NZ;
    const int k = wk.y - T + lane;
    const bool kin = (k >= 0) && (k < NZ);
    const bool lown = lane >= T && lane < 64 - T;
    const bool zp = kin && (k < pz || k >= NZ - pz);
    const int kc = kin ? k : 0;
    const int kk = zp ? (k < pz ? k : k - (NZ - 2 * pz)) : 0;
    const int k1 = min(kc + 1, NZ - 1);
    const float dt = S.dt, idr = S.inv_dr, idz = S.inv_dz, dr = S.dr;
    const int ihi = wk.z - T + TRE - 1;
    const int klo = wk.y - T, khi = wk.y - T + 63;
    // PM = 0: the launch holds only tiles clear of every PML layer
    const bool tile_pr = PM != 0 && ihi >= nr;                        // reaches the radial layer
    const bool tile_pz = PM != 0 && ((klo < pz) || (khi >= NZ - pz));  // reaches an axial layer
    const bool tile_pml = tile_pr || tile_pz;

    const float* __restrict__ Ai = ain + S.ast_off;
    float* __restrict__ Ao = aout + S.ast_off;
    const long long LR = S.psir_len, LZ = S.psiz_len;
    const long long oPR = 6 * cells, oPZ = oPR + 5 * LR;
    const float* __restrict__ prt = pml_r + S.pml_r_off;
    const float* __restrict__ pzt = pml_z + S.pml_z_off;

    if (wave == 0) {
#pragma unroll
        for (int f = 0; f < NPL; ++f) {
            L[f][lane] = 0.f;
            L[f][(TRE + 1) * 64 + lane] = 0.f;
        }
    }

    float avr[RPT], avz[RPT], trr[RPT], ttt[RPT], tzz[RPT], trz[RPT];
    float dl[RPT], d2m[RPT], dbR[RPT], dbZ[RPT], dmuS[RPT];
    float rR[RPT], rZ[RPT], rRm[RPT];  // 1/(2r) at R, C and the R node below
    float mrow[RPT];                   // 1 on rows i >= 1 of the grid, 0 elsewhere
    // PML: A-bar, B-bar, C-bar, D-bar (velocity side), Phi recursions (stress side)
    float qA[RPT], qB[RPT], qC[RPT], qD[RPT], pTr[RPT], pRr[RPT], pTz[RPT], pZz[RPT], pG[RPT],
        pH[RPT];
    float a_ri[RPT], b_ri[RPT], a_rh[RPT], b_rh[RPT];
    float gl[RPT], gm[RPT], gs[RPT], ge[RPT];
    float gR[RPT], gZ[RPT];  // density correlation (X & 1)
    float hL[RPT], hM[RPT];  // pseudo-Hessian diagonal (X & 2)
    float a_zi = 0.f, b_zi = 1.f, a_zh = 0.f, b_zh = 1.f;
    if (zp) {
        a_zi = pzt[k];
        b_zi = pzt[NZ + k];
        a_zh = pzt[2 * NZ + k];
        b_zh = pzt[3 * NZ + k];
    }

#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int e = wave + W * j;
        const int i = wk.z - T + e;  // uniform
        const bool iin = i >= 0 && i < NR;
        const bool in = kin && iin;
        const bool up = in && i >= 1;
        const long long c = (long long)(iin ? i : 0) * NZ + kc;
        avr[j] = up ? Ai[c] : 0.f;
        avz[j] = in ? Ai[cells + c] : 0.f;
        trr[j] = in ? Ai[2 * cells + c] : 0.f;
        ttt[j] = in ? Ai[3 * cells + c] : 0.f;
        tzz[j] = in ? Ai[4 * cells + c] : 0.f;
        trz[j] = up ? Ai[5 * cells + c] : 0.f;
        const long long m = S.model_off + (long long)(iin ? i : 0) * S.model_ld;
        const long long mm = m - S.model_ld;
        const float r0 = in ? rho[m + kc] : 1.f;
        const float r_kp = in ? rho[m + k1] : 1.f;
        const float r_im = up ? rho[mm + kc] : 1.f;
        const float m0 = in ? mu[m + kc] : 0.f;
        const float m_kp = in ? mu[m + k1] : 0.f;
        const float m_im = up ? mu[mm + kc] : 0.f;
        const float m_imkp = up ? mu[mm + k1] : 0.f;
        dl[j] = in ? dt * lam[m + kc] : 0.f;
        d2m[j] = dt * 2.0f * m0;
        dbR[j] = up ? dt * 2.0f * rcp(r_im + r0) : 0.f;
        dbZ[j] = in ? dt * 2.0f * rcp(r0 + r_kp) : 0.f;
        dmuS[j] = up ? dt * mu_harm(m_im, m0, m_imkp, m_kp) : 0.f;
        rR[j] = wave_uniform((iin && i >= 1) ? 0.5f * rcp(i * dr) : 0.f);
        rRm[j] = wave_uniform((iin && i >= 1) ? 0.5f * rcp((i - 0.5f) * dr) : 0.f);
        rZ[j] = wave_uniform(iin ? 0.5f * rcp((i + 0.5f) * dr) : 0.f);
        mrow[j] = wave_uniform((iin && i >= 1) ? 1.f : 0.f);
        qA[j] = qB[j] = qC[j] = qD[j] = 0.f;
        pTr[j] = pRr[j] = pTz[j] = pZz[j] = pG[j] = pH[j] = 0.f;
        a_ri[j] = a_rh[j] = 0.f;
        b_ri[j] = b_rh[j] = 1.f;
        gl[j] = gm[j] = gs[j] = ge[j] = 0.f;
        gR[j] = gZ[j] = hL[j] = hM[j] = 0.f;
        if (tile_pml) {
            if (iin && i >= nr) {
                a_ri[j] = prt[i];
                b_ri[j] = prt[NR + i];
                a_rh[j] = prt[2 * NR + i];
                b_rh[j] = prt[3 * NR + i];
                if (kin) {
                    const long long q = oPR + (long long)(i - nr) * NZ + kc;
                    qA[j] = Ai[q];
                    qC[j] = Ai[q + LR];
                    pTr[j] = Ai[q + 2 * LR];
                    pRr[j] = Ai[q + 3 * LR];
                    pH[j] = Ai[q + 4 * LR];
                }
            }
            if (in && zp) {
                const long long q = oPZ + (long long)i * (2 * pz) + kk;
                qB[j] = Ai[q];
                qD[j] = Ai[q + LZ];
                pTz[j] = Ai[q + 2 * LZ];
                pZz[j] = Ai[q + 3 * LZ];
                pG[j] = Ai[q + 4 * LZ];
            }
        }
        a_ri[j] = wave_uniform(a_ri[j]);
        b_ri[j] = wave_uniform(b_ri[j]);
        a_rh[j] = wave_uniform(a_rh[j]);
        b_rh[j] = wave_uniform(b_rh[j]);
    }

    // the residual of every step of this launch at this lane's receiver (if
    // the lane's axial row holds one), staged once
    if (wave == 0) {
        float rsum[T];
#pragma unroll
        for (int t = 0; t < T; ++t) rsum[t] = 0.f;
        for (int r = 0; r < S.nrec; ++r)
            if (kin && rec_k[S.rec_off + r] == k) {
#pragma unroll
                for (int t = 0; t < T; ++t)
                    if (t >= t0 && t < nsteps)
                        rsum[t] += resid[S.trace_off + (long long)r * S.nt + (n_hi - t)];
            }
#pragma unroll
        for (int t = 0; t < T; ++t) Lres[t][lane] = rsum[t] * (1.0f / 3.0f);
    }
    // stored v^{n+1/2} of the first step; later steps are fetched one step ahead.
    // The correlation of the owned cells reads it on the owned tile and one
    // cell around it only (rows T-1 .. TRE-T, lanes T-1 .. 64-T).
    float hvr[RPT], hvz[RPT];
    const bool hlane = kin && lane >= T - 1 && lane <= 64 - T;
    auto fetch_hist = [&](int t) {
        const float* __restrict__ vrh = hist_hi - (long long)t * hist_stride + S.cell_off;
        const float* __restrict__ vzh = vrh + cells_total;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int e = wave + W * j;
            const int i = wk.z - T + e;
            const bool in = hlane && e >= T - 1 && e <= TRE - T && i >= 0 && i < NR;
            const long long c = (long long)(in ? i : 0) * NZ + kc;
            hvr[j] = in ? vrh[c] : 0.f;
            hvz[j] = in ? vzh[c] : 0.f;
        }
    };
    fetch_hist(t0);
    __syncthreads();

    // Rows that have left the correct region (the halo shrinks one row per
    // step) are skipped; what they last left in LDS is read only by rows that
    // are themselves outside the correct region after this step.
    auto live = [&](int e, int t) { return e >= t && e < TRE - t; };

    // The step loop in three PML forms besides the plain one: radial and
    // axial memories, radial only, axial only.  A tile that does not reach a
    // layer has zero coefficients for it everywhere, so leaving that layer's
    // terms out changes nothing; most PML tiles reach the radial layer only.
    auto steps = [&](auto PRC, auto PZC) {
        constexpr bool PR = decltype(PRC)::value != 0, PZ = decltype(PZC)::value != 0;
        for (int t = t0; t < nsteps; ++t) {
            float Err_[RPT], Ett_[RPT], Ezz_[RPT], Ez_[RPT], Er_[RPT];
            // ---- A: residual, drivers, stage the stored velocities
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const int e = wave + W * j;
                const int i = wk.z - T + e;
                const int x = (e + 1) * 64 + lane;
                L[HVR][x] = hvr[j];
                L[HVZ][x] = hvz[j];
                if (!live(e, t)) continue;  // uniform
                if (i == 0) {  // uniform
                    const float v = Lres[t][lane];
                    trr[j] += v;
                    ttt[j] += v;
                    tzz[j] += v;
                }
                const float sa = trr[j] + ttt[j] + tzz[j];
                if constexpr (WAV) {
                    // the tile that owns row 0 and the source cell's lane
                    if (i == 0 && lown && k == S.src_k)
                        wgrad[S.wave_off + (n_hi - t)] = S.src_scale * sa;
                }
                float Err = dl[j] * sa + d2m[j] * trr[j];
                const float Ett = dl[j] * sa + d2m[j] * ttt[j];
                float Ezz = dl[j] * sa + d2m[j] * tzz[j];
                float Ez = dmuS[j] * trz[j];
                float Er = Ez;
                // a (lambda Phi_T + 2 mu Phi_R); dl, d2m, dmuS carry a factor dt
                if constexpr (PR) {
                    pTr[j] = dt * sa + b_rh[j] * pTr[j];
                    pRr[j] = dt * trr[j] + b_rh[j] * pRr[j];
                    pH[j] = dt * trz[j] + b_ri[j] * pH[j];
                    const float idt = 1.0f / dt;
                    Err += a_rh[j] * idt * (dl[j] * pTr[j] + d2m[j] * pRr[j]);
                    Er += a_ri[j] * idt * dmuS[j] * pH[j];
                }
                if constexpr (PZ) {
                    pTz[j] = dt * sa + b_zi * pTz[j];
                    pZz[j] = dt * tzz[j] + b_zi * pZz[j];
                    pG[j] = dt * trz[j] + b_zh * pG[j];
                    const float idt = 1.0f / dt;
                    Ezz += a_zi * idt * (dl[j] * pTz[j] + d2m[j] * pZz[j]);
                    Ez += a_zh * idt * dmuS[j] * pG[j];
                }
                L[ERR][x] = Err;
                L[ETT][x] = Ett;
                L[ER][x] = Er;
                Err_[j] = Err;
                Ett_[j] = Ett;
                Ezz_[j] = Ezz;
                Ez_[j] = Ez;
                Er_[j] = Er;
            }
            __syncthreads();
            // fetch the next step's stored velocities now; this step's own
            // values are read back from LDS (LDSE) or kept in registers
            float vr0_[RPT], vz0_[RPT];
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                vr0_[j] = LDSE ? 0.f : hvr[j];
                vz0_[j] = LDSE ? 0.f : hvz[j];
            }
            if (t + 1 < nsteps) fetch_hist(t + 1);
            // ---- B: correlation, transposed updates of a_v
            float U_[RPT], H_[RPT], DzR_[RPT], DzZ_[RPT], ZS_[RPT];
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                if (!live(wave + W * j, t)) continue;  // uniform
                const int x = (wave + W * j + 1) * 64 + lane;
                // Eq. 7-8 with the strain rates of v^{n+1/2} and dJ/dtau^{n+1}
                const float vr0 = LDSE ? L[HVR][x] : vr0_[j], vr1 = L[HVR][x + 64];
                const float vz0 = LDSE ? L[HVZ][x] : vz0_[j];
                const float vz_km = from_lane_below(vz0), vr_kp = from_lane_above(vr0);
                const float vz_im = L[HVZ][x - 64];
                const float err = (vr1 - vr0) * idr;
                const float ett = (vr1 + vr0) * rZ[j];
                const float ezz = (vz0 - vz_km) * idz;
                const float ez = (vr_kp - vr0) * idz;
                const float er = (vz0 - vz_im) * idr;
                // the sums leave out the factors dt (g_lambda, g_muS), 2 dt
                // (g_mu) and dt/4 (illumination), applied once at write-back
                const float sa = trr[j] + ttt[j] + tzz[j];
                gl[j] = fmaf(err + ett + ezz, sa, gl[j]);
                gm[j] = fmaf(err, trr[j], fmaf(ett, ttt[j], fmaf(ezz, tzz[j], gm[j])));
                gs[j] = fmaf(ez + er, trz[j], gs[j]);
                if constexpr (PR) {
                    const float idt = 1.0f / dt;
                    gl[j] += idt * (a_rh[j] * err * pTr[j]);
                    gm[j] += idt * (a_rh[j] * err * pRr[j]);
                    gs[j] += idt * (a_ri[j] * er * pH[j]);
                }
                if constexpr (PZ) {
                    const float idt = 1.0f / dt;
                    gl[j] += idt * (a_zi * ezz * pTz[j]);
                    gm[j] += idt * (a_zi * ezz * pZz[j]);
                    gs[j] += idt * (a_zh * ez * pG[j]);
                }
                if constexpr (HES) {
                    const float dv = err + ett + ezz, es = mrow[j] * (ez + er);
                    hL[j] += 3.0f * dv * dv;
                    hM[j] += 4.0f * (err * err + ett * ett + ezz * ezz) + es * es;
                }
                const float ur = vr0 + vr1, uz = vz_km + vz0;  // twice the C-node means
                ge[j] = fmaf(ur, ur, fmaf(uz, uz, ge[j]));
                // transposed stress update into a_v, then the transposed velocity update
                // with two or more rows per thread the drivers this lane
                // wrote to LDS are read back instead of being held in registers
                const float Err0 = LDSE ? L[ERR][x] : Err_[j];
                const float Ett0 = LDSE ? L[ETT][x] : Ett_[j];
                const float Er0 = LDSE ? L[ER][x] : Er_[j];
                const float dar =
                    mrow[j] * ((L[ERR][x - 64] - Err0) * idr + L[ETT][x - 64] * rRm[j] +
                               Ett0 * rZ[j] + (from_lane_below(Ez_[j]) - Ez_[j]) * idz);
                const float daz = (Ezz_[j] - from_lane_above(Ezz_[j])) * idz +
                                  (Er0 - L[ER][x + 64]) * idr;
                avr[j] += dar;
                avz[j] += daz;
                if constexpr (RHO) {
                    gR[j] += dar * vr0;
                    gZ[j] += daz * vz0;
                }
                const float W1 = dbR[j] * avr[j];
                float aDr = W1, aDzR = W1;
                const float W2 = dbZ[j] * avz[j];
                float aDrZ = W2, aDzZ = W2;
                if constexpr (PR) {
                    float q = qA[j] + W1;
                    qA[j] = b_ri[j] * q;
                    aDr += a_ri[j] * q;
                    q = qC[j] + W2;
                    qC[j] = b_rh[j] * q;
                    aDrZ += a_rh[j] * q;
                }
                if constexpr (PZ) {
                    float q = qB[j] + W1;
                    qB[j] = b_zi * q;
                    aDzR += a_zi * q;
                    q = qD[j] + W2;
                    qD[j] = b_zh * q;
                    aDzZ += a_zh * q;
                }
                U_[j] = aDr * idr;
                H_[j] = W1 * rR[j];
                DzR_[j] = aDzR;
                DzZ_[j] = aDzZ;
                ZS_[j] = -aDrZ * idr + W2 * rZ[j];
                L[UR][x] = U_[j];
                L[HR][x] = H_[j];
                L[ZR][x] = aDrZ * idr + W2 * rZ[j];
                if constexpr (LDSE) {
                    // the parts of the gather that stay within this wave are
                    // applied now, so that only LDS crosses the barrier
                    tzz[j] += (from_lane_below(DzZ_[j]) - DzZ_[j]) * idz;
                    trz[j] += mrow[j] * ((DzR_[j] - from_lane_above(DzR_[j])) * idz + ZS_[j]);
                }
            }
            __syncthreads();
            // ---- C: transposed velocity update gathered into a_tau
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                if (!live(wave + W * j, t)) continue;  // uniform
                const int x = (wave + W * j + 1) * 64 + lane;
                const float h0 = LDSE ? L[HR][x] : H_[j], h1 = L[HR][x + 64];
                trr[j] += (LDSE ? L[UR][x] : U_[j]) + h0 - L[UR][x + 64] + h1;
                ttt[j] -= h0 + h1;
                if constexpr (LDSE) {
                    trz[j] += mrow[j] * L[ZR][x - 64];
                } else {
                    tzz[j] += (from_lane_below(DzZ_[j]) - DzZ_[j]) * idz;
                    trz[j] += mrow[j] * ((DzR_[j] - from_lane_above(DzR_[j])) * idz + ZS_[j] +
                                         L[ZR][x - 64]);
                }
            }
        }
    };
    if constexpr (X == 0) {
        if (tile_pr && tile_pz)
            steps(IntC<1>{}, IntC<1>{});
        else if (tile_pr)
            steps(IntC<1>{}, IntC<0>{});
        else if (tile_pz)
            steps(IntC<0>{}, IntC<1>{});
        else
            steps(IntC<0>{}, IntC<0>{});
    } else {  // the extra outputs' registers leave no room for three PML loops
        if (tile_pml)
            steps(IntC<1>{}, IntC<1>{});
        else
            steps(IntC<0>{}, IntC<0>{});
    }

    // ---- write back the owned tile and add the correlation sums
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int e = wave + W * j;
        const int i = wk.z - T + e;
        const bool in = kin && i >= 0 && i < NR;
        if (!(in && lown && e >= T && e < TRE - T)) continue;
        const long long c = (long long)i * NZ + k;
        if (i >= 1) {
            Ao[c] = avr[j];
            Ao[5 * cells + c] = trz[j];
        }
        Ao[cells + c] = avz[j];
        Ao[2 * cells + c] = trr[j];
        Ao[3 * cells + c] = ttt[j];
        Ao[4 * cells + c] = tzz[j];
        if (tile_pml) {
            if (i >= nr) {
                const long long q = oPR + (long long)(i - nr) * NZ + k;
                Ao[q] = qA[j];
                Ao[q + LR] = qC[j];
                Ao[q + 2 * LR] = pTr[j];
                Ao[q + 3 * LR] = pRr[j];
                Ao[q + 4 * LR] = pH[j];
            }
            if (zp) {
                const long long q = oPZ + (long long)i * (2 * pz) + kk;
                Ao[q] = qB[j];
                Ao[q + LZ] = qD[j];
                Ao[q + 2 * LZ] = pTz[j];
                Ao[q + 3 * LZ] = pZz[j];
                Ao[q + 4 * LZ] = pG[j];
            }
        }
        float* g = acc + S.cell_off + c;
        g[0] += dt * gl[j];
        g[cells_total] += (2.0f * dt) * gm[j];
        if (i >= 1) g[2 * cells_total] += dt * gs[j];
        g[3 * cells_total] += (0.25f * dt) * ge[j];
        if constexpr (RHO) {
            float* gr = acc_rho + S.cell_off + c;
            if (i >= 1) gr[0] += gR[j];
            gr[cells_total] += gZ[j];
        }
        if constexpr (HES) {
            float* h = acc_h + S.cell_off + c;
            h[0] += dt * dt * hL[j];
            h[cells_total] += dt * dt * hM[j];
        }
    }
}

}  // namespace bhfwi
