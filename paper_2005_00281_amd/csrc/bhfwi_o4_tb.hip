// bhfwi_o4_tb.hip -- temporally blocked fourth-order steps: the forward (the
// Eq. 2 step with the four-point staggered differences and 1/r averages of
// the one-step kernels in bhfwi_o4.hip) and its exact adjoint with the
// correlation of Eq. 7-8.
//
// The tiling is that of the second-order time blocks: a workgroup of W wave64
// owns TRE - 2H radial by 64 - 2H axial cells and loads them with an H-cell
// halo, lane = axial row, wave w holding rows w, w + W, ... (a row index is
// uniform over a wave).  Each half step of the fourth-order scheme reaches
// one and a half cells on either side, so a full step needs three: H = 3T.
// The fields, medium coefficients and PML memories stay in registers for the
// T steps; the radial neighbours at -2 .. +2 rows come from LDS planes with
// two zeroed guard rows on each side, the axial ones from DPP wavefront
// shifts (two shifts for the second neighbour).
//
// Across the axis the fields are mirrored (even at half radial positions:
// normal stresses and v_z; odd and zero on the axis at integer ones: v_r,
// tau_rz).  In the forward a row whose stencil reaches below the axis reads
// the image row instead, with the field's sign (per-row constant rows and
// signs), so the rows below the axis in a window at the axis are never read;
// the adjoint's treatment is described with its kernel.
//
// As in the second-order kernels the step loop has no per-cell branches,
// rows that have left the correct region are skipped, and tiles that reach a
// PML layer run the memories of the layers they reach only.
#pragma once
#include "bhfwi_internal.h"
#include "bhfwi_kernels.hip"
#include "bhfwi_tb_fwd.hip"
#include "bhfwi_o4.hip"

namespace bhfwi {
namespace o4 {

__device__ inline float from_lane_below2(float v) { return from_lane_below(from_lane_below(v)); }
__device__ inline float from_lane_above2(float v) { return from_lane_above(from_lane_above(v)); }

template <int T, int TRE, int W, int PM>
__global__ void __launch_bounds__(64 * W, (W >= 16 && PM == 0 && TRE <= 2 * W) ? 8 : 1)
k_fwd4_tb(const ShotDev* __restrict__ shots, const int4* __restrict__ work, int nwork, int map,
          int n0, int nsteps, const float* __restrict__ lam, const float* __restrict__ mu,
          const float* __restrict__ rho, const float* __restrict__ wavelet,
          const int* __restrict__ rec_k, const float* __restrict__ pml_r,
          const float* __restrict__ pml_z, const float* __restrict__ sin,
          float* __restrict__ sout, float* __restrict__ traces, float* __restrict__ hist,
          long long hist_stride, long long cells_total)
{
    constexpr int H = 3 * T;  // halo
    constexpr int RPT = TRE / W;
    constexpr int GR = 2;  // guard rows on each side of the LDS planes
    constexpr int LDW = (TRE + 2 * GR) * 64;
    static_assert(TRE % W == 0 && TRE > 2 * H && 64 > 2 * H, "tile too small for the halo");
    enum { TRR = 0, TTT, TRZ, VR, VZ, NPL };
    __shared__ float L[NPL][LDW];
    __shared__ float Lwav[T];

    const int wg = xcd_chunk(blockIdx.x, nwork, map);
    if (wg >= nwork) return;
    const int4 wk = work[wg];
    const ShotDev& S = shots[wk.x];
    const int ns = min(nsteps, S.nt - n0);
    if (ns <= 0) return;  // uniform over the workgroup

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int NR = S.NR, NZ = S.NZ, nr = S.nr, pz = S.pz;
    const long long cells = (long long)NR * NZ;
    const int k = wk.y - H + lane;
    const bool kin = (k >= 0) && (k < NZ);
    const bool lown = lane >= H && lane < 64 - H;
    const bool zp = kin && (k < pz || k >= NZ - pz);
    const int kc = kin ? k : 0;
    const int kk = zp ? (k < pz ? k : k - (NZ - 2 * pz)) : 0;
    const int k1 = min(kc + 1, NZ - 1);
    const float dt = S.dt, idr = S.inv_dr, idz = S.inv_dz, dr = S.dr;
    const int ihi = wk.z - H + TRE - 1;
    const int klo = wk.y - H, khi = wk.y - H + 63;
    const bool tile_pr = PM != 0 && ihi >= nr;
    const bool tile_pz = PM != 0 && ((klo < pz) || (khi >= NZ - pz));
    const bool tile_pml = tile_pr || tile_pz;

    const float* __restrict__ Fi = sin + S.fst_off;
    float* __restrict__ Fo = sout + S.fst_off;
    const long long LR = S.psir_len, LZ = S.psiz_len;
    const long long oPR = 6 * cells, oPZ = oPR + 4 * LR;
    const float* __restrict__ prt = pml_r + S.pml_r_off;
    const float* __restrict__ pzt = pml_z + S.pml_z_off;

    if (wave == 0) {
#pragma unroll
        for (int f = 0; f < NPL; ++f)
#pragma unroll
            for (int gq = 0; gq < GR; ++gq) {
                L[f][gq * 64 + lane] = 0.f;
                L[f][(TRE + GR + gq) * 64 + lane] = 0.f;
            }
        if (lane < T) Lwav[lane] = lane < ns ? wavelet[S.wave_off + n0 + lane] : 0.f;
    }
    int rj = -1;  // receiver recorded by this lane's axial row (first match)
    if (traces && wk.z == 0)
        for (int r = S.nrec - 1; r >= 0; --r)
            if (kin && rec_k[S.rec_off + r] == k) rj = r;

    float vr[RPT], vz[RPT], trr[RPT], ttt[RPT], tzz[RPT], trz[RPT];
    float cl[RPT], c2m[RPT], dbR[RPT], dbZ[RPT], dmuS[RPT], srcw[RPT];
    float iR[RPT], iZ[RPT];  // 1/r at R and C/Z nodes (0 on the axis / outside)
    // LDS rows of the -1 and -2 neighbours of even fields, of the -1
    // neighbour of odd fields and its sign (the image below the axis)
    int em1[RPT], em2[RPT], om1[RPT];
    float os1[RPT];
    float pA[RPT], pB[RPT], pC[RPT], pD[RPT], pE[RPT], pF[RPT], pG[RPT], pH[RPT];
    float a_ri[RPT], b_ri[RPT], a_rh[RPT], b_rh[RPT];
    float a_zi = 0.f, b_zi = 1.f, a_zh = 0.f, b_zh = 1.f;
    if (zp) {
        a_zi = pzt[k];
        b_zi = pzt[NZ + k];
        a_zh = pzt[2 * NZ + k];
        b_zh = pzt[3 * NZ + k];
    }

    // window row of grid row ii, clamped into the planes (rows past the
    // guards belong to cells whose results are discarded)
    auto slot = [&](int ii) { return min(max(ii - (wk.z - H), -GR), TRE + GR - 1); };
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int e = wave + W * j;
        const int i = wk.z - H + e;  // uniform
        const bool iin = i >= 0 && i < NR;
        const bool in = kin && iin;
        const long long c = (long long)(iin ? i : 0) * NZ + kc;
        vr[j] = in ? Fi[c] : 0.f;
        vz[j] = in ? Fi[cells + c] : 0.f;
        trr[j] = in ? Fi[2 * cells + c] : 0.f;
        ttt[j] = in ? Fi[3 * cells + c] : 0.f;
        tzz[j] = in ? Fi[4 * cells + c] : 0.f;
        trz[j] = in ? Fi[5 * cells + c] : 0.f;
        const long long m = S.model_off + (long long)(iin ? i : 0) * S.model_ld;
        const long long mm = m - S.model_ld;
        const bool up = in && i >= 1;
        const float r0 = in ? rho[m + kc] : 1.f;
        const float r_kp = in ? rho[m + k1] : 1.f;
        const float r_im = up ? rho[mm + kc] : 1.f;
        const float m0 = in ? mu[m + kc] : 0.f;
        const float m_kp = in ? mu[m + k1] : 0.f;
        const float m_im = up ? mu[mm + kc] : 0.f;
        const float m_imkp = up ? mu[mm + k1] : 0.f;
        cl[j] = in ? dt * lam[m + kc] : 0.f;
        c2m[j] = dt * 2.0f * m0;
        dbR[j] = up ? dt * 2.0f * rcp(r_im + r0) : 0.f;
        dbZ[j] = in ? dt * 2.0f * rcp(r0 + r_kp) : 0.f;
        dmuS[j] = up ? dt * mu_harm(m_im, m0, m_imkp, m_kp) : 0.f;
        srcw[j] = (in && i == 0 && k == S.src_k) ? AXIS_SRC * S.src_scale : 0.f;
        iR[j] = wave_uniform((iin && i >= 1) ? rcp(i * dr) : 0.f);
        iZ[j] = wave_uniform(iin ? rcp((i + 0.5f) * dr) : 0.f);
        // even fields: grid row -1 - x mirrors row x; odd: -x mirrors x, negated
        em1[j] = __builtin_amdgcn_readfirstlane(slot(i - 1 >= 0 ? i - 1 : -i));
        em2[j] = __builtin_amdgcn_readfirstlane(slot(i - 2 >= 0 ? i - 2 : 1 - i));
        om1[j] = __builtin_amdgcn_readfirstlane(slot(i - 1 >= 0 ? i - 1 : 1 - i));
        os1[j] = wave_uniform(i - 1 >= 0 ? 1.f : -1.f);
        pA[j] = pB[j] = pC[j] = pD[j] = pE[j] = pF[j] = pG[j] = pH[j] = 0.f;
        a_ri[j] = a_rh[j] = 0.f;
        b_ri[j] = b_rh[j] = 1.f;
        if (tile_pml) {
            if (iin && i >= nr) {
                a_ri[j] = prt[i];
                b_ri[j] = prt[NR + i];
                a_rh[j] = prt[2 * NR + i];
                b_rh[j] = prt[3 * NR + i];
                if (kin) {
                    const long long q = oPR + (long long)(i - nr) * NZ + kc;
                    pA[j] = Fi[q];
                    pC[j] = Fi[q + LR];
                    pE[j] = Fi[q + 2 * LR];
                    pH[j] = Fi[q + 3 * LR];
                }
            }
            if (in && zp) {
                const long long q = oPZ + (long long)i * (2 * pz) + kk;
                pB[j] = Fi[q];
                pD[j] = Fi[q + LZ];
                pF[j] = Fi[q + 2 * LZ];
                pG[j] = Fi[q + 3 * LZ];
            }
        }
        a_ri[j] = wave_uniform(a_ri[j]);
        b_ri[j] = wave_uniform(b_ri[j]);
        a_rh[j] = wave_uniform(a_rh[j]);
        b_rh[j] = wave_uniform(b_rh[j]);
        const int x = (e + GR) * 64 + lane;
        L[TRR][x] = trr[j];
        L[TTT][x] = ttt[j];
        L[TRZ][x] = trz[j];
    }
    unsigned hoff[RPT];  // byte offset of this lane's cell in each row of a history plane
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int i = wk.z - H + wave + W * j;
        hoff[j] = (unsigned)(max(i, 0) * NZ + kc) * 4u;
    }
    __syncthreads();

    // the correct region shrinks three rows per step on each side
    auto live = [&](int e, int t) { return e >= 3 * t && e < TRE - 3 * t; };
    auto at = [&](int f, int row) { return L[f][row * 64 + lane]; };  // row: plane row

    auto steps = [&](auto PRC, auto PZC) {
        constexpr bool PR = decltype(PRC)::value != 0, PZ = decltype(PZC)::value != 0;
        for (int t = 0; t < ns; ++t) {
            const int n = n0 + t;
            const float wv = Lwav[t];
            char* const hvr_t =
                hist ? reinterpret_cast<char*>(hist + (long long)t * hist_stride + S.cell_off)
                     : nullptr;
            char* const hvz_t = hist ? hvr_t + 4 * cells_total : nullptr;
            // ---- velocities (R and Z nodes) from the stresses
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const int e = wave + W * j;
                if (!live(e, t)) continue;  // uniform
                const int p = e + GR;
                const float trr_m1 = at(TRR, em1[j] + GR), trr_m2 = at(TRR, em2[j] + GR);
                const float ttt_m1 = at(TTT, em1[j] + GR), ttt_m2 = at(TTT, em2[j] + GR);
                const float trr_p1 = at(TRR, p + 1), ttt_p1 = at(TTT, p + 1);
                const float trz_m1 = os1[j] * at(TRZ, om1[j] + GR);
                const float trz_p1 = at(TRZ, p + 1), trz_p2 = at(TRZ, p + 2);
                const float trz_km = from_lane_below(trz[j]), trz_km2 = from_lane_below2(trz[j]);
                const float trz_kp = from_lane_above(trz[j]);
                const float tzz_kp = from_lane_above(tzz[j]), tzz_kp2 = from_lane_above2(tzz[j]);
                const float tzz_km = from_lane_below(tzz[j]);
                float Dr = (C1 * (trr[j] - trr_m1) + C2 * (trr_p1 - trr_m2)) * idr;
                float Dz = (C1 * (trz[j] - trz_km) + C2 * (trz_kp - trz_km2)) * idz;
                const float hoop = (G1 * ((trr[j] - ttt[j]) + (trr_m1 - ttt_m1)) +
                                    G2 * ((trr_p1 - ttt_p1) + (trr_m2 - ttt_m2))) * iR[j];
                float Dr2 = (C1 * (trz_p1 - trz[j]) + C2 * (trz_p2 - trz_m1)) * idr;
                float Dz2 = (C1 * (tzz_kp - tzz[j]) + C2 * (tzz_kp2 - tzz_km)) * idz;
                const float hoop2 = (G1 * (trz_p1 + trz[j]) + G2 * (trz_p2 + trz_m1)) * iZ[j];
                if constexpr (PR) {
                    pA[j] = b_ri[j] * pA[j] + a_ri[j] * Dr;
                    Dr += pA[j];
                    pC[j] = b_rh[j] * pC[j] + a_rh[j] * Dr2;
                    Dr2 += pC[j];
                }
                if constexpr (PZ) {
                    pB[j] = b_zi * pB[j] + a_zi * Dz;
                    Dz += pB[j];
                    pD[j] = b_zh * pD[j] + a_zh * Dz2;
                    Dz2 += pD[j];
                }
                vr[j] += dbR[j] * (Dr + Dz + hoop);
                vz[j] += dbZ[j] * (Dr2 + Dz2 + hoop2);
                L[VR][p * 64 + lane] = vr[j];
                L[VZ][p * 64 + lane] = vz[j];
            }
            __syncthreads();
            // ---- stresses (C and S nodes) from the new velocities
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const int e = wave + W * j;
                if (!live(e, t)) continue;  // uniform
                const int p = e + GR;
                const float vr_m1 = os1[j] * at(VR, om1[j] + GR);
                const float vr_p1 = at(VR, p + 1), vr_p2 = at(VR, p + 2);
                const float vz_m1 = at(VZ, em1[j] + GR), vz_m2 = at(VZ, em2[j] + GR);
                const float vz_p1 = at(VZ, p + 1);
                const float vz_km = from_lane_below(vz[j]), vz_km2 = from_lane_below2(vz[j]);
                const float vz_kp = from_lane_above(vz[j]);
                const float vr_kp = from_lane_above(vr[j]), vr_kp2 = from_lane_above2(vr[j]);
                const float vr_km = from_lane_below(vr[j]);
                float err = (C1 * (vr_p1 - vr[j]) + C2 * (vr_p2 - vr_m1)) * idr;
                const float ett = (G1 * (vr_p1 + vr[j]) + G2 * (vr_p2 + vr_m1)) * iZ[j];
                float ezz = (C1 * (vz[j] - vz_km) + C2 * (vz_kp - vz_km2)) * idz;
                float ez = (C1 * (vr_kp - vr[j]) + C2 * (vr_kp2 - vr_km)) * idz;
                float er = (C1 * (vz[j] - vz_m1) + C2 * (vz_p1 - vz_m2)) * idr;
                if constexpr (PR) {
                    pE[j] = b_rh[j] * pE[j] + a_rh[j] * err;
                    err += pE[j];
                    pH[j] = b_ri[j] * pH[j] + a_ri[j] * er;
                    er += pH[j];
                }
                if constexpr (PZ) {
                    pF[j] = b_zi * pF[j] + a_zi * ezz;
                    ezz += pF[j];
                    pG[j] = b_zh * pG[j] + a_zh * ez;
                    ez += pG[j];
                }
                const float ltr = cl[j] * (err + ett + ezz) + srcw[j] * wv;
                trr[j] += ltr + c2m[j] * err;
                ttt[j] += ltr + c2m[j] * ett;
                tzz[j] += ltr + c2m[j] * ezz;
                trz[j] += dmuS[j] * (ez + er);
                L[TRR][p * 64 + lane] = trr[j];
                L[TTT][p * 64 + lane] = ttt[j];
                L[TRZ][p * 64 + lane] = trz[j];
                const int i = wk.z - H + e;
                const bool own = kin && lown && e >= H && e < TRE - H && i < NR;
                if (hist && own) {
                    *reinterpret_cast<float*>(hvr_t + hoff[j]) = vr[j];
                    *reinterpret_cast<float*>(hvz_t + hoff[j]) = vz[j];
                }
                if (i == 0 && own && rj >= 0)
                    traces[S.trace_off + (long long)rj * S.nt + n] =
                        (trr[j] + ttt[j] + tzz[j]) * (1.0f / 3.0f);
            }
            __syncthreads();
        }
    };
    if (tile_pr && tile_pz)
        steps(IntC<1>{}, IntC<1>{});
    else if (tile_pr)
        steps(IntC<1>{}, IntC<0>{});
    else if (tile_pz)
        steps(IntC<0>{}, IntC<1>{});
    else
        steps(IntC<0>{}, IntC<0>{});

    // ---- write back the owned tile
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int e = wave + W * j;
        const int i = wk.z - H + e;
        const bool in = kin && i >= 0 && i < NR;
        if (!(in && lown && e >= H && e < TRE - H)) continue;
        const long long c = (long long)i * NZ + k;
        if (i >= 1) {
            Fo[c] = vr[j];
            Fo[5 * cells + c] = trz[j];
        }
        Fo[cells + c] = vz[j];
        Fo[2 * cells + c] = trr[j];
        Fo[3 * cells + c] = ttt[j];
        Fo[4 * cells + c] = tzz[j];
        if (tile_pml) {
            if (i >= nr) {
                const long long q = oPR + (long long)(i - nr) * NZ + k;
                Fo[q] = pA[j];
                Fo[q + LR] = pC[j];
                Fo[q + 2 * LR] = pE[j];
                Fo[q + 3 * LR] = pH[j];
            }
            if (zp) {
                const long long q = oPZ + (long long)i * (2 * pz) + kk;
                Fo[q] = pB[j];
                Fo[q + LZ] = pD[j];
                Fo[q + 2 * LZ] = pF[j];
                Fo[q + 3 * LZ] = pG[j];
            }
        }
    }
}


// ---------------------------------------------------------------------------
// Temporally blocked fourth-order adjoint step fused with the correlation of
// Eq. 7-8 (the transpose of k_fwd4_tb, as k_adj4 is of k_fwd4), on the same
// tiling with a three-cell halo per step.  Per reverse step:
//   A  residual injection, the drivers of the transposed stress update
//      (Err, Ett, Ezz at C nodes, Ez = Er at S nodes, with the stress-side
//      PML recursions) and the stored v^{n+1/2} -> LDS (Ett as Ett / r);
//   B  Eq. 7-8 with the fourth-order strain rates of v^{n+1/2} (the mirror
//      images read as in the forward); the adjoint velocities gather the
//      drivers with the transposed four-point stencils; the products of the
//      transposed velocity update (with the velocity-side PML) -> LDS;
//   C  the adjoint stresses gather the products.
// A transposed gather reads zero at rows below the axis (their drivers and
// products vanish: zero coefficients), and the reads the forward stencils
// made through the mirror are added back to their image rows 0 and 1 with
// the field's parity: per-row factors f0 = [i = 0], f1 = [i = 1].  X selects
// the extra outputs of the second-order adjoint: bit 0 the density
// correlation (the adjoint velocity increments of phase B times the stored
// v^{n+1/2}, into acc_rho), bit 1 the virtual-source pseudo-Hessian (the
// plain fourth-order strain rates of v^{n+1/2}, into acc_h).
// ---------------------------------------------------------------------------
template <int T, int TRE, int W, int PM, int X>
__global__ void __launch_bounds__(64 * W, 1)
k_adj4_tb(const ShotDev* __restrict__ shots, const int4* __restrict__ work, int nwork, int map,
          int n_hi, int nsteps, const float* __restrict__ lam, const float* __restrict__ mu,
          const float* __restrict__ rho, const int* __restrict__ rec_k,
          const float* __restrict__ resid, const float* __restrict__ pml_r,
          const float* __restrict__ pml_z, const float* __restrict__ ain,
          float* __restrict__ aout, const float* __restrict__ hist_hi, long long hist_stride,
          float* __restrict__ acc, float* __restrict__ acc_rho, float* __restrict__ acc_h,
          long long cells_total)
{
    constexpr bool RHO = (X & 1) != 0, HES = (X & 2) != 0;
    constexpr int H = 3 * T;
    constexpr int RPT = TRE / W;
    constexpr int GR = 2;
    constexpr int LDW = (TRE + 2 * GR) * 64;
    static_assert(TRE % W == 0 && TRE > 2 * H && 64 > 2 * H, "tile too small for the halo");
    enum { ERR = 0, ETQ, ER, HVR, HVZ, UR, HR, ZR, ZH, NPL };
    __shared__ float L[NPL][LDW];
    __shared__ float Lres[T][64];

    const int wg = xcd_chunk(blockIdx.x, nwork, map);
    if (wg >= nwork) return;
    const int4 wk = work[wg];
    const ShotDev& S = shots[wk.x];
    const int t0 = max(0, n_hi - (S.nt - 1));
    if (t0 >= nsteps) return;  // uniform over the workgroup

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int NR = S.NR, NZ = S.NZ, nr = S.nr, pz = S.pz;
    const long long cells = (long long)NR * NZ;
    const int k = wk.y - H + lane;
    const bool kin = (k >= 0) && (k < NZ);
    const bool lown = lane >= H && lane < 64 - H;
    const bool zp = kin && (k < pz || k >= NZ - pz);
    const int kc = kin ? k : 0;
    const int kk = zp ? (k < pz ? k : k - (NZ - 2 * pz)) : 0;
    const int k1 = min(kc + 1, NZ - 1);
    const float dt = S.dt, idr = S.inv_dr, idz = S.inv_dz, dr = S.dr;
    const float idt = 1.0f / dt;
    const int ihi = wk.z - H + TRE - 1;
    const int klo = wk.y - H, khi = wk.y - H + 63;
    const bool tile_pr = PM != 0 && ihi >= nr;
    const bool tile_pz = PM != 0 && ((klo < pz) || (khi >= NZ - pz));
    const bool tile_pml = tile_pr || tile_pz;

    const float* __restrict__ Ai = ain + S.ast_off;
    float* __restrict__ Ao = aout + S.ast_off;
    const long long LR = S.psir_len, LZ = S.psiz_len;
    const long long oPR = 6 * cells, oPZ = oPR + 5 * LR;
    const float* __restrict__ prt = pml_r + S.pml_r_off;
    const float* __restrict__ pzt = pml_z + S.pml_z_off;

    if (wave == 0) {
#pragma unroll
        for (int f = 0; f < NPL; ++f)
#pragma unroll
            for (int gq = 0; gq < GR; ++gq) {
                L[f][gq * 64 + lane] = 0.f;
                L[f][(TRE + GR + gq) * 64 + lane] = 0.f;
            }
    }

    float avr[RPT], avz[RPT], trr[RPT], ttt[RPT], tzz[RPT], trz[RPT];
    float dl[RPT], d2m[RPT], dbR[RPT], dbZ[RPT], dmuS[RPT];
    float iR[RPT], iZ[RPT], mrow[RPT], f0[RPT], f1[RPT];
    int em1[RPT], em2[RPT], om1[RPT];
    float os1[RPT];
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
    auto slot = [&](int ii) { return min(max(ii - (wk.z - H), -GR), TRE + GR - 1); };

#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int e = wave + W * j;
        const int i = wk.z - H + e;  // uniform
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
        iR[j] = wave_uniform((iin && i >= 1) ? rcp(i * dr) : 0.f);
        iZ[j] = wave_uniform(iin ? rcp((i + 0.5f) * dr) : 0.f);
        mrow[j] = wave_uniform((iin && i >= 1) ? 1.f : 0.f);
        f0[j] = wave_uniform(i == 0 ? 1.f : 0.f);
        f1[j] = wave_uniform(i == 1 ? 1.f : 0.f);
        em1[j] = __builtin_amdgcn_readfirstlane(slot(i - 1 >= 0 ? i - 1 : -i));
        em2[j] = __builtin_amdgcn_readfirstlane(slot(i - 2 >= 0 ? i - 2 : 1 - i));
        om1[j] = __builtin_amdgcn_readfirstlane(slot(i - 1 >= 0 ? i - 1 : 1 - i));
        os1[j] = wave_uniform(i - 1 >= 0 ? 1.f : -1.f);
        a_ri[j] = a_rh[j] = 0.f;
        b_ri[j] = b_rh[j] = 1.f;
        gl[j] = gm[j] = gs[j] = ge[j] = 0.f;
        gR[j] = gZ[j] = hL[j] = hM[j] = 0.f;
        if (tile_pr && iin && i >= nr) {
            a_ri[j] = prt[i];
            b_ri[j] = prt[NR + i];
            a_rh[j] = prt[2 * NR + i];
            b_rh[j] = prt[3 * NR + i];
        }
        a_ri[j] = wave_uniform(a_ri[j]);
        b_ri[j] = wave_uniform(b_ri[j]);
        a_rh[j] = wave_uniform(a_rh[j]);
        b_rh[j] = wave_uniform(b_rh[j]);
    }

    if (wave == 0) {  // residual / 3 at this lane's receivers, per step
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
    // stored v^{n+1/2}; the correlation of the owned cells reads it two rows
    // and two lanes around the owned tile
    float hvr[RPT], hvz[RPT];
    const bool hlane = kin && lane >= H - 2 && lane < 64 - H + 2;
    auto fetch_hist = [&](int t) {
        const float* __restrict__ vrh = hist_hi - (long long)t * hist_stride + S.cell_off;
        const float* __restrict__ vzh = vrh + cells_total;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int e = wave + W * j;
            const int i = wk.z - H + e;
            const bool in = hlane && e >= H - 2 && e < TRE - H + 2 && i >= 0 && i < NR;
            const long long c = (long long)(in ? i : 0) * NZ + kc;
            hvr[j] = in ? vrh[c] : 0.f;
            hvz[j] = in ? vzh[c] : 0.f;
        }
    };
    fetch_hist(t0);
    __syncthreads();

    auto live = [&](int e, int t) { return e >= 3 * t && e < TRE - 3 * t; };
    auto at = [&](int f, int row) { return L[f][row * 64 + lane]; };

    // The PML memories live inside the loop form that updates them: a form
    // without the axial (radial) layer neither loads nor keeps the axial
    // (radial) memories, which every cell of such a tile lacks.
    auto steps = [&](auto PRC, auto PZC) {
        constexpr bool PR = decltype(PRC)::value != 0, PZ = decltype(PZC)::value != 0;
        float qA[RPT], qC[RPT], pTr[RPT], pRr[RPT], pH[RPT];  // radial layer
        float qB[RPT], qD[RPT], pTz[RPT], pZz[RPT], pG[RPT];  // axial layers
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int i = wk.z - H + wave + W * j;
            const bool iin = i >= 0 && i < NR;
            qA[j] = qC[j] = pTr[j] = pRr[j] = pH[j] = 0.f;
            qB[j] = qD[j] = pTz[j] = pZz[j] = pG[j] = 0.f;
            if (PR && kin && iin && i >= nr) {
                const long long q = oPR + (long long)(i - nr) * NZ + kc;
                qA[j] = Ai[q];
                qC[j] = Ai[q + LR];
                pTr[j] = Ai[q + 2 * LR];
                pRr[j] = Ai[q + 3 * LR];
                pH[j] = Ai[q + 4 * LR];
            }
            if (PZ && kin && iin && zp) {
                const long long q = oPZ + (long long)i * (2 * pz) + kk;
                qB[j] = Ai[q];
                qD[j] = Ai[q + LZ];
                pTz[j] = Ai[q + 2 * LZ];
                pZz[j] = Ai[q + 3 * LZ];
                pG[j] = Ai[q + 4 * LZ];
            }
        }
        for (int t = t0; t < nsteps; ++t) {
            // the values phase A writes to LDS (drivers, stored velocities) are
            // read back from there in phase B rather than held in registers
            float Ezz_[RPT], Ez_[RPT];
            // ---- A: residual, drivers, stored velocities -> LDS
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const int e = wave + W * j;
                const int i = wk.z - H + e;
                const int p = e + GR;
                L[HVR][p * 64 + lane] = hvr[j];
                L[HVZ][p * 64 + lane] = hvz[j];
                if (!live(e, t)) continue;  // uniform
                if (i == 0) {  // uniform
                    const float v = Lres[t][lane];
                    trr[j] += v;
                    ttt[j] += v;
                    tzz[j] += v;
                }
                const float sa = trr[j] + ttt[j] + tzz[j];
                float Err = dl[j] * sa + d2m[j] * trr[j];
                const float Ett = dl[j] * sa + d2m[j] * ttt[j];
                float Ezz = dl[j] * sa + d2m[j] * tzz[j];
                float Ez = dmuS[j] * trz[j];
                float Er = Ez;
                if constexpr (PR) {
                    pTr[j] = dt * sa + b_rh[j] * pTr[j];
                    pRr[j] = dt * trr[j] + b_rh[j] * pRr[j];
                    pH[j] = dt * trz[j] + b_ri[j] * pH[j];
                    Err += a_rh[j] * idt * (dl[j] * pTr[j] + d2m[j] * pRr[j]);
                    Er += a_ri[j] * idt * dmuS[j] * pH[j];
                }
                if constexpr (PZ) {
                    pTz[j] = dt * sa + b_zi * pTz[j];
                    pZz[j] = dt * tzz[j] + b_zi * pZz[j];
                    pG[j] = dt * trz[j] + b_zh * pG[j];
                    Ezz += a_zi * idt * (dl[j] * pTz[j] + d2m[j] * pZz[j]);
                    Ez += a_zh * idt * dmuS[j] * pG[j];
                }
                const float Q = Ett * iZ[j];
                L[ERR][p * 64 + lane] = Err;
                L[ETQ][p * 64 + lane] = Q;
                L[ER][p * 64 + lane] = Er;
                Ezz_[j] = Ezz;
                Ez_[j] = Ez;
            }
            __syncthreads();
            if (t + 1 < nsteps) fetch_hist(t + 1);
            // ---- B: Eq. 7-8, adjoint velocities, products of the transposed velocity update
            float DZR_[RPT], DZZ_[RPT];
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const int e = wave + W * j;
                if (!live(e, t)) continue;  // uniform
                const int p = e + GR;
                // strain rates of the stored v^{n+1/2} (mirror images as in the forward)
                const float vr0 = at(HVR, p), vz0 = at(HVZ, p);
                const float sa = trr[j] + ttt[j] + tzz[j];  // phase C has not run yet
                const float vr_p1 = at(HVR, p + 1), vr_p2 = at(HVR, p + 2);
                const float vr_m1 = os1[j] * at(HVR, om1[j] + GR);
                const float vz_p1 = at(HVZ, p + 1), vz_m1 = at(HVZ, em1[j] + GR);
                const float vz_m2 = at(HVZ, em2[j] + GR);
                const float vz_km = from_lane_below(vz0), vz_km2 = from_lane_below2(vz0);
                const float vz_kp = from_lane_above(vz0);
                const float vr_kp = from_lane_above(vr0), vr_kp2 = from_lane_above2(vr0);
                const float vr_km = from_lane_below(vr0);
                const float err = (C1 * (vr_p1 - vr0) + C2 * (vr_p2 - vr_m1)) * idr;
                const float ett = (G1 * (vr_p1 + vr0) + G2 * (vr_p2 + vr_m1)) * iZ[j];
                const float ezz = (C1 * (vz0 - vz_km) + C2 * (vz_kp - vz_km2)) * idz;
                const float ez = (C1 * (vr_kp - vr0) + C2 * (vr_kp2 - vr_km)) * idz;
                const float er = (C1 * (vz0 - vz_m1) + C2 * (vz_p1 - vz_m2)) * idr;
                // the sums leave out dt (g_lambda, g_muS), 2 dt (g_mu), dt/4 (illumination)
                gl[j] = fmaf(err + ett + ezz, sa, gl[j]);
                gm[j] = fmaf(err, trr[j], fmaf(ett, ttt[j], fmaf(ezz, tzz[j], gm[j])));
                gs[j] = fmaf(ez + er, trz[j], gs[j]);
                if constexpr (PR) {
                    gl[j] += idt * (a_rh[j] * err * pTr[j]);
                    gm[j] += idt * (a_rh[j] * err * pRr[j]);
                    gs[j] += idt * (a_ri[j] * er * pH[j]);
                }
                if constexpr (PZ) {
                    gl[j] += idt * (a_zi * ezz * pTz[j]);
                    gm[j] += idt * (a_zi * ezz * pZz[j]);
                    gs[j] += idt * (a_zh * ez * pG[j]);
                }
                const float ur = vr0 + vr_p1, uz = vz_km + vz0;  // twice the C-node means
                ge[j] = fmaf(ur, ur, fmaf(uz, uz, ge[j]));
                if constexpr (HES) {  // dt^2 applied at write-back
                    const float dv = err + ett + ezz, es = mrow[j] * (ez + er);
                    hL[j] += 3.0f * dv * dv;
                    hM[j] += 4.0f * (err * err + ett * ett + ezz * ezz) + es * es;
                }
                // a_v_r at R(i): the stress update read v_r through e_rr (radial
                // "hi" stencil), e_tt (I / r) and e_z (axial "hi" stencil)
                const float E_m1 = at(ERR, p - 1), E_m2 = at(ERR, p - 2), E_p1 = at(ERR, p + 1);
                const float Q_m1 = at(ETQ, p - 1), Q_m2 = at(ETQ, p - 2), Q_p1 = at(ETQ, p + 1);
                const float Err0 = at(ERR, p), Q0 = at(ETQ, p);
                const float dEr = C1 * (E_m1 - Err0) + C2 * (E_m2 - E_p1) + f1[j] * C2 * E_m1;
                const float it = G1 * (Q_m1 + Q0) + G2 * (Q_m2 + Q_p1) - f1[j] * G2 * Q_m1;
                const float Ez_m1 = from_lane_below(Ez_[j]), Ez_m2 = from_lane_below2(Ez_[j]);
                const float Ez_p1 = from_lane_above(Ez_[j]);
                const float dEz = C1 * (Ez_m1 - Ez_[j]) + C2 * (Ez_m2 - Ez_p1);
                const float dar = mrow[j] * (dEr * idr + it + dEz * idz);
                avr[j] += dar;
                // a_v_z at Z(i): read through e_zz (axial "lo") and e_r (radial "lo")
                const float R_p1 = at(ER, p + 1), R_p2 = at(ER, p + 2), R_m1 = at(ER, p - 1);
                const float Er0 = at(ER, p);
                const float dRr = C1 * (Er0 - R_p1) + C2 * (R_m1 - R_p2) -
                                  f0[j] * (C1 * Er0 + C2 * R_p1) - f1[j] * C2 * R_m1;
                const float Zz_p1 = from_lane_above(Ezz_[j]), Zz_p2 = from_lane_above2(Ezz_[j]);
                const float Zz_m1 = from_lane_below(Ezz_[j]);
                const float dZz = C1 * (Ezz_[j] - Zz_p1) + C2 * (Zz_m1 - Zz_p2);
                const float daz = dZz * idz + dRr * idr;
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
                L[UR][p * 64 + lane] = aDr;
                L[HR][p * 64 + lane] = W1 * iR[j];
                L[ZR][p * 64 + lane] = aDrZ;
                L[ZH][p * 64 + lane] = W2 * iZ[j];
                DZR_[j] = aDzR;
                DZZ_[j] = aDzZ;
            }
            __syncthreads();
            // ---- C: the adjoint stresses gather the products
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const int e = wave + W * j;
                if (!live(e, t)) continue;  // uniform
                const int p = e + GR;
                // C node: v_r read tau_rr, tau_tt (radial "lo", D and I), v_z
                // read tau_zz (axial "hi")
                const float U0 = at(UR, p), U_p1 = at(UR, p + 1), U_p2 = at(UR, p + 2);
                const float U_m1 = at(UR, p - 1);
                const float H0 = at(HR, p), H_p1 = at(HR, p + 1), H_p2 = at(HR, p + 2);
                const float H_m1 = at(HR, p - 1);
                const float dU = C1 * (U0 - U_p1) + C2 * (U_m1 - U_p2) -
                                 f0[j] * (C1 * U0 + C2 * U_p1) - f1[j] * C2 * U_m1;
                const float hI = G1 * (H0 + H_p1) + G2 * (H_m1 + H_p2) +
                                 f0[j] * (G1 * H0 + G2 * H_p1) + f1[j] * G2 * H_m1;
                const float D_m1 = from_lane_below(DZZ_[j]), D_m2 = from_lane_below2(DZZ_[j]);
                const float D_p1 = from_lane_above(DZZ_[j]);
                trr[j] += dU * idr + hI;
                ttt[j] -= hI;
                tzz[j] += (C1 * (D_m1 - DZZ_[j]) + C2 * (D_m2 - D_p1)) * idz;
                // S node: v_r read tau_rz (axial "lo"), v_z read it (radial "hi", D and I)
                const float Z_m1 = at(ZR, p - 1), Z_m2 = at(ZR, p - 2), Z_p1 = at(ZR, p + 1);
                const float Zh_m1 = at(ZH, p - 1), Zh_m2 = at(ZH, p - 2), Zh_p1 = at(ZH, p + 1);
                const float Z0 = at(ZR, p), Zh0 = at(ZH, p);
                const float dZr = C1 * (Z_m1 - Z0) + C2 * (Z_m2 - Z_p1) + f1[j] * C2 * Z_m1;
                const float zI = G1 * (Zh_m1 + Zh0) + G2 * (Zh_m2 + Zh_p1) - f1[j] * G2 * Zh_m1;
                const float R_p1 = from_lane_above(DZR_[j]), R_p2 = from_lane_above2(DZR_[j]);
                const float R_m1 = from_lane_below(DZR_[j]);
                const float dZ = C1 * (DZR_[j] - R_p1) + C2 * (R_m1 - R_p2);
                trz[j] += mrow[j] * (dZ * idz + dZr * idr + zI);
            }
        }
        // the owned tile's PML memories
        if constexpr (PR || PZ) {
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const int e = wave + W * j;
                const int i = wk.z - H + e;
                if (!(kin && i >= 0 && i < NR && lown && e >= H && e < TRE - H)) continue;
                if (PR && i >= nr) {
                    const long long q = oPR + (long long)(i - nr) * NZ + k;
                    Ao[q] = qA[j];
                    Ao[q + LR] = qC[j];
                    Ao[q + 2 * LR] = pTr[j];
                    Ao[q + 3 * LR] = pRr[j];
                    Ao[q + 4 * LR] = pH[j];
                }
                if (PZ && zp) {
                    const long long q = oPZ + (long long)i * (2 * pz) + kk;
                    Ao[q] = qB[j];
                    Ao[q + LZ] = qD[j];
                    Ao[q + 2 * LZ] = pTz[j];
                    Ao[q + 3 * LZ] = pZz[j];
                    Ao[q + 4 * LZ] = pG[j];
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
    } else {  // the extra sums leave registers for two loop forms only
        if (tile_pml)
            steps(IntC<1>{}, IntC<1>{});
        else
            steps(IntC<0>{}, IntC<0>{});
    }

    // ---- write back the owned tile and add the correlation sums
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int e = wave + W * j;
        const int i = wk.z - H + e;
        const bool in = kin && i >= 0 && i < NR;
        if (!(in && lown && e >= H && e < TRE - H)) continue;
        const long long c = (long long)i * NZ + k;
        if (i >= 1) {
            Ao[c] = avr[j];
            Ao[5 * cells + c] = trz[j];
        }
        Ao[cells + c] = avz[j];
        Ao[2 * cells + c] = trr[j];
        Ao[3 * cells + c] = ttt[j];
        Ao[4 * cells + c] = tzz[j];
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

}  // namespace o4
}  // namespace bhfwi
