// bhfwi_o4_tb.hip -- temporally blocked fourth-order forward step (the Eq. 2
// step with the four-point staggered differences and 1/r averages of the
// one-step kernels in bhfwi_o4.hip).
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
// tau_rz).  A row whose stencil reaches below the axis reads the image row
// instead, with the field's sign; the rows and signs are per-row constants.
// Rows below the axis in the window (tiles at the axis) are never read.
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

}  // namespace o4
}  // namespace bhfwi
